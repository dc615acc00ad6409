// Momentum projection of the loops (appendix A.2, contraction kernels, and
// the Fourier step of appendix A.3): the colour-traced Dirac outer products are formed per site,
// C(x)[b][a] = sum_r sum_c v_{r,bc}(x) w*_{r,ac}(x) for ultra-local
// insertions, and for the one-derivative insertions (the covariant-derivative
// kernel of appendix A.2) in each direction mu
//   D_mu(x)[b][a] = 1/4 sum_r sum_c [(nabla_mu v)_{bc} w*_{ac} - v_{bc} (nabla_mu w)*_{ac}],
//   nabla_mu f(x) = U_mu(x) f(x + mu) - U_mu(x - mu)^dag f(x - mu)
// (the symmetric left-right derivative of the bilinear w^dag Gamma D_mu v
// attributed to x, time-boundary phase included).  Then they are transformed
// over the spatial coordinates of each time slice,
//   C_p(t) = sum_{x in t} e^{i p.x} C(x),  p = 2 pi (nx/Lx, ny/Ly, nz/Lz),
// for every integer n with |n|^2 <= p2max.  The transform is separable, so it
// runs as three direct one-dimensional transforms (x, then y, then z) over
// the 2N+1 needed components per direction (N = floor(sqrt(p2max))), each a
// fixed-order sum, followed by the selection of the momenta inside the
// sphere.  Phases come from FP64 tables of e^{2 pi i k / L}, k = n x mod L.
#include <cmath>

#include "runtime.h"

namespace {

constexpr int kBlock = 256;

// Cf[e][s], e = 4 b + a, s = x + Lx (y + Ly (z + Lz t)) (canonical order)
__global__ __launch_bounds__(kBlock) void k_outer_sites(const double2 *ve, const double2 *vo, const double2 *we,
                                                        const double2 *wo, Geo g, long V, int nrhs, double2 *Cf)
{
    const long s = (long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= V) return;
    const int x = (int)(s % g.L[0]);
    const long q = s / g.L[0];
    const int y = (int)(q % g.L[1]);
    const long q2 = q / g.L[1];
    const int z = (int)(q2 % g.L[2]);
    const int t = (int)(q2 / g.L[2]);
    const int p = (x + y + z + t) & 1;
    const size_t i = (size_t)(s >> 1);
    const double2 *v = p ? vo : ve, *w = p ? wo : we;
    cx<double> C[16];
#pragma unroll
    for (int e = 0; e < 16; e++) C[e] = {0, 0};
    for (int r = 0; r < nrhs; r++) {
        cx<double> a[12], b[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double2 va = v[(size_t)(r * 12 + k) * g.hs + i], vb = w[(size_t)(r * 12 + k) * g.hs + i];
            a[k] = {va.x, va.y};
            b[k] = {vb.x, vb.y};
        }
#pragma unroll
        for (int sb = 0; sb < 4; sb++)
#pragma unroll
            for (int sa = 0; sa < 4; sa++)
#pragma unroll
                for (int c = 0; c < 3; c++) cmac_conj(C[sb * 4 + sa], b[sa * 3 + c], a[sb * 3 + c]);
    }
#pragma unroll
    for (int e = 0; e < 16; e++) Cf[(size_t)e * V + s] = make_double2(C[e].r, C[e].i);
}

// D_mu(x); Cf[mu][e][s] with e = 4 b + a.
// Block order: block b runs on XCD b % 8 (round-robin dispatch).  XCD k owns
// the contiguous range of site blocks [k per, (k + 1) per) and takes them in
// order, the four directions of one site block as four consecutive blocks, so
// that the directions read the site's 12-RHS fields (4.6 KB per site) while
// they are in that XCD's L2 instead of streaming them from memory once per
// direction.  Blocks past the last site block exit.
__global__ __launch_bounds__(kBlock) void k_outer_deriv_sites(const double2 *ve, const double2 *vo, const double2 *we,
                                                              const double2 *wo, const double2 *l0, const double2 *l1,
                                                              Geo g, long V, int nrhs, int per, double2 *Cf)
{
    const int m = (int)(blockIdx.x >> 3);
    const int mu = m & 3;
    const long sblk = (long)(blockIdx.x & 7) * per + (m >> 2);
    const long s = sblk * kBlock + threadIdx.x;
    if (s >= V) return;
    int c4[4];
    c4[0] = (int)(s % g.L[0]);
    const long q = s / g.L[0];
    c4[1] = (int)(q % g.L[1]);
    const long q2 = q / g.L[1];
    c4[2] = (int)(q2 % g.L[2]);
    c4[3] = (int)(q2 / g.L[2]);
    const int p = (c4[0] + c4[1] + c4[2] + c4[3]) & 1;
    const size_t i = (size_t)(s >> 1);
    const size_t vh = (size_t)g.vh, hs = (size_t)g.hs;  // link and spinor plane strides
    int cf[4] = {c4[0], c4[1], c4[2], c4[3]}, cb[4] = {c4[0], c4[1], c4[2], c4[3]};
    cf[mu] = cf[mu] + 1 == g.L[mu] ? 0 : cf[mu] + 1;
    cb[mu] = cb[mu] == 0 ? g.L[mu] - 1 : cb[mu] - 1;
    const size_t jf = (size_t)eo_index(g, cf[0], cf[1], cf[2], cf[3]);
    const size_t jb = (size_t)eo_index(g, cb[0], cb[1], cb[2], cb[3]);
    // links[p][d][9][vh]: d = mu forward U_mu(x), d = 4 + mu backward U_mu(x - mu)^dag (phases included)
    const double2 *lk = p ? l1 : l0;
    cx<double> Uf[9], Ub[9];
#pragma unroll
    for (int e = 0; e < 9; e++) {
        const double2 a = lk[((size_t)mu * 9 + e) * vh + i], b = lk[((size_t)(4 + mu) * 9 + e) * vh + i];
        Uf[e] = {a.x, a.y};
        Ub[e] = {b.x, b.y};
    }
    const double2 *vs = p ? vo : ve, *vn = p ? ve : vo, *ws = p ? wo : we, *wn = p ? we : wo;
    cx<double> C[16];
#pragma unroll
    for (int e = 0; e < 16; e++) C[e] = {0, 0};
    // nabla f at x for spin a of field f (other-parity neighbours)
    auto nabla = [&](const double2 *f, size_t base, int a, cx<double> out[3]) {
        cx<double> ff[3], fb[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double2 x1 = f[(base + a * 3 + c) * hs + jf], x2 = f[(base + a * 3 + c) * hs + jb];
            ff[c] = {x1.x, x1.y};
            fb[c] = {x2.x, x2.y};
        }
#pragma unroll
        for (int r = 0; r < 3; r++) {
            cx<double> acc = {0, 0}, accb = {0, 0};
#pragma unroll
            for (int c = 0; c < 3; c++) {
                cmac(acc, Uf[3 * r + c], ff[c]);
                cmac(accb, Ub[3 * r + c], fb[c]);
            }
            out[r] = {acc.r - accb.r, acc.i - accb.i};
        }
    };
    for (int r = 0; r < nrhs; r++) {
        const size_t base = (size_t)r * 12;
        cx<double> wx[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double2 a = ws[(base + k) * hs + i];
            wx[k] = {a.x, a.y};
        }
#pragma unroll
        for (int sb = 0; sb < 4; sb++) {
            cx<double> gv[3];
            nabla(vn, base, sb, gv);
#pragma unroll
            for (int sa = 0; sa < 4; sa++)
#pragma unroll
                for (int c = 0; c < 3; c++) cmac_conj(C[sb * 4 + sa], wx[sa * 3 + c], gv[c]);
        }
        cx<double> vx[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double2 a = vs[(base + k) * hs + i];
            vx[k] = {a.x, a.y};
        }
#pragma unroll
        for (int sa = 0; sa < 4; sa++) {
            cx<double> gw[3];
            nabla(wn, base, sa, gw);
#pragma unroll
            for (int c = 0; c < 3; c++) gw[c] = {-gw[c].r, -gw[c].i};
#pragma unroll
            for (int sb = 0; sb < 4; sb++)
#pragma unroll
                for (int c = 0; c < 3; c++) cmac_conj(C[sb * 4 + sa], gw[c], vx[sb * 3 + c]);
        }
    }
#pragma unroll
    for (int e = 0; e < 16; e++) Cf[((size_t)mu * 16 + e) * V + s] = make_double2(0.25 * C[e].r, 0.25 * C[e].i);
}

// One direction of the transform: in [outer][n][inner] -> out[outer][W][inner]
// with out[o][j][k] = sum_m ph[j][m] in[o][m][k] (fixed order in m).
__global__ __launch_bounds__(kBlock) void k_dft_dim(const double2 *in, double2 *out, const double2 *ph, long outer,
                                                    int n, int W, long inner)
{
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    const long total = outer * W * inner;
    if (idx >= total) return;
    const long k = idx % inner;
    const long rest = idx / inner;
    const int j = (int)(rest % W);
    const long o = rest / W;
    const double2 *src = in + (o * n) * inner + k;
    const double2 *f = ph + (long)j * n;
    cx<double> acc = {0, 0};
    for (int m = 0; m < n; m++) {
        const double2 a = f[m], b = src[(long)m * inner];
        cmac(acc, cx<double>{a.x, a.y}, cx<double>{b.x, b.y});
    }
    out[idx] = make_double2(acc.r, acc.i);
}

// The first direction (inner = 1: the transformed index is the fastest):
// one thread per row in[o][0..n) forms all W outputs out[o][j], up to kDftJ
// at a time, so the row is read once (8 consecutive complex per unrolled
// batch, one 128-byte line per lane) and the phases, the same for every lane,
// come through scalar loads.  Every output is the same fixed-order sum over m
// as in k_dft_dim.
constexpr int kDftJ = 8;

__global__ __launch_bounds__(kBlock) void k_dft_rows(const double2 *in, double2 *out, const double2 *ph, long outer,
                                                     int n, int W)
{
    const long o = (long)blockIdx.x * kBlock + threadIdx.x;
    if (o >= outer) return;
    const double2 *row = in + o * n;
    double2 *dst = out + o * W;
    for (int j0 = 0; j0 < W; j0 += kDftJ) {
        cx<double> acc[kDftJ];
#pragma unroll
        for (int jj = 0; jj < kDftJ; jj++) acc[jj] = {0, 0};
#pragma unroll 8
        for (int m = 0; m < n; m++) {
            const double2 b = row[m];
#pragma unroll
            for (int jj = 0; jj < kDftJ; jj++)
                if (j0 + jj < W) {
                    const double2 a = ph[(long)(j0 + jj) * n + m];
                    cmac(acc[jj], cx<double>{a.x, a.y}, cx<double>{b.x, b.y});
                }
        }
#pragma unroll
        for (int jj = 0; jj < kDftJ; jj++)
            if (j0 + jj < W) dst[j0 + jj] = make_double2(acc[jj].r, acc[jj].i);
    }
}

// out[m][blk][t][e] = T[16 blk + e][t][nz + N][ny + N][nx + N] for the listed momenta
__global__ void k_pick_momenta(const double2 *T, const int *mom, int n_mom, int nblk, int Lt, int W, int N,
                               double2 *out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_mom * nblk * Lt * 16) return;
    const int e = idx % 16, t = (idx / 16) % Lt, blk = (idx / (16 * Lt)) % nblk, m = idx / (16 * Lt * nblk);
    const int nx = mom[3 * m] + N, ny = mom[3 * m + 1] + N, nz = mom[3 * m + 2] + N;
    out[idx] = T[((((size_t)(16 * blk + e) * Lt + t) * W + nz) * W + ny) * W + nx];
}

// e^{2 pi i (j - N) x / L} for j < W, x < L, reduced mod L in integers
std::vector<double2> phase_table(int L, int N)
{
    const int W = 2 * N + 1;
    std::vector<double2> ph((size_t)W * L);
    for (int j = 0; j < W; j++)
        for (int x = 0; x < L; x++) {
            const long k = (((long)(j - N) * x) % L + L) % L;
            const double a = 2.0 * M_PI * (double)k / (double)L;
            ph[(size_t)j * L + x] = make_double2(std::cos(a), std::sin(a));
        }
    return ph;
}

}  // namespace

std::vector<Momentum> momenta_list(int p2max)
{
    std::vector<Momentum> out;
    if (p2max < 0) return out;
    int N = 0;
    while ((N + 1) * (N + 1) <= p2max) N++;
    for (int n2 = 0; n2 <= p2max; n2++)
        for (int nx = -N; nx <= N; nx++)
            for (int ny = -N; ny <= N; ny++)
                for (int nz = -N; nz <= N; nz++)
                    if (nx * nx + ny * ny + nz * nz == n2) out.push_back(Momentum{{nx, ny, nz}});
    return out;
}

void check_momenta(tm_ctx *c, int p2max)
{
    TM_REQUIRE(p2max >= 0, "p2max must be >= 0");
    int N = 0;
    while ((N + 1) * (N + 1) <= p2max) N++;
    for (int mu = 0; mu < 3; mu++)
        TM_REQUIRE(2 * N < c->geo.L[mu], "momentum components must stay below L/2 in every spatial direction");
}

namespace {

// Fourier sums of per-site components Cf[ncomp][V] (ncomp = 16 nblk) over each
// time slice for the listed momenta -> host out[n_mom][nblk][Lt][16]
void project_components(tm_ctx *c, const double2 *Cf, int nblk, const std::vector<Momentum> &mom,
                        std::vector<cx<double>> &out, hipStream_t s)
{
    const Geo &g = c->geo;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const long ncomp = 16L * nblk;
    int N = 0;
    for (const auto &m : mom)
        for (int d = 0; d < 3; d++) N = std::max(N, std::abs(m.n[d]));
    const int W = 2 * N + 1;
    // phase tables for x, y, z
    std::vector<double2> px = phase_table(Lx, N), py = phase_table(Ly, N), pz = phase_table(Lz, N);
    double2 *dph = (double2 *)ws_get(c, "mom_ph", sizeof(double2) * (size_t)W * (Lx + Ly + Lz));
    upload(dph, px.data(), sizeof(double2) * px.size(), s);
    upload(dph + px.size(), py.data(), sizeof(double2) * py.size(), s);
    upload(dph + px.size() + py.size(), pz.data(), sizeof(double2) * pz.size(), s);
    // x: [ncomp Lt Lz Ly][Lx][1] -> [ncomp Lt Lz Ly][W][1]
    const long o1 = ncomp * Lt * Lz * Ly;
    double2 *T1 = (double2 *)ws_get(c, "mom_t1", sizeof(double2) * o1 * W);
    hipLaunchKernelGGL(k_dft_rows, dim3((unsigned)((o1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, Cf, T1,
                       (const double2 *)dph, o1, Lx, W);
    // y: [ncomp Lt Lz][Ly][W] -> [ncomp Lt Lz][W][W]
    const long o2 = ncomp * Lt * Lz;
    double2 *T2 = (double2 *)ws_get(c, "mom_t2", sizeof(double2) * o2 * W * W);
    const long n2 = o2 * W * W;
    hipLaunchKernelGGL(k_dft_dim, dim3((unsigned)((n2 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const double2 *)T1, T2, (const double2 *)(dph + px.size()), o2, Ly, W, (long)W);
    // z: [ncomp Lt][Lz][W W] -> [ncomp Lt][W][W W]
    const long o3 = ncomp * Lt;
    double2 *T3 = (double2 *)ws_get(c, "mom_t3", sizeof(double2) * o3 * W * W * W);
    const long n3 = o3 * W * W * W;
    hipLaunchKernelGGL(k_dft_dim, dim3((unsigned)((n3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const double2 *)T2, T3, (const double2 *)(dph + px.size() + py.size()), o3, Lz, W,
                       (long)W * W);
    TM_HIP(hipGetLastError());
    const int n_mom = (int)mom.size();
    std::vector<int> ml(3 * n_mom);
    for (int m = 0; m < n_mom; m++)
        for (int d = 0; d < 3; d++) ml[3 * m + d] = mom[m].n[d];
    int *dm = (int *)ws_get(c, "mom_list", sizeof(int) * 3 * n_mom);
    upload(dm, ml.data(), sizeof(int) * ml.size(), s);
    const int n_out = n_mom * nblk * Lt * 16;
    double2 *dout = (double2 *)ws_get(c, "mom_out", sizeof(double2) * n_out);
    hipLaunchKernelGGL(k_pick_momenta, dim3((n_out + 255) / 256), dim3(256), 0, s, (const double2 *)T3,
                       (const int *)dm, n_mom, nblk, Lt, W, N, dout);
    TM_HIP(hipGetLastError());
    out.resize((size_t)n_out);
    download(c, out.data(), dout, sizeof(double2) * out.size(), s);
}

}  // namespace

void outer_momenta_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                        const std::vector<Momentum> &mom, std::vector<cx<double>> &out, hipStream_t s)
{
    const long V = c->V;
    double2 *Cf = (double2 *)ws_get(c, "mom_cf", sizeof(double2) * 16 * V);
    hipLaunchKernelGGL(k_outer_sites, dim3((unsigned)((V + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const double2 *)ve, (const double2 *)vo, (const double2 *)we, (const double2 *)wo, c->geo, V,
                       nrhs, Cf);
    TM_HIP(hipGetLastError());
    project_components(c, Cf, 1, mom, out, s);
}

void outer_deriv_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                      const std::vector<Momentum> &mom, std::vector<cx<double>> &out, hipStream_t s)
{
    TM_REQUIRE(c->have_gauge, "no gauge field set");
    const long V = c->V;
    double2 *Cf = (double2 *)ws_get(c, "mom_cfd", sizeof(double2) * 64 * V);
    const long nsb = (V + kBlock - 1) / kBlock;
    const long per = (nsb + 7) / 8;  // site blocks per XCD
    TM_REQUIRE(32 * per <= 0x7fffffffL, "lattice too large for the derivative contraction grid");
    hipLaunchKernelGGL(k_outer_deriv_sites, dim3((unsigned)(32 * per)), dim3(kBlock), 0, s, (const double2 *)ve,
                       (const double2 *)vo, (const double2 *)we, (const double2 *)wo, (const double2 *)c->links64[0],
                       (const double2 *)c->links64[1], c->geo, V, nrhs, (int)per, Cf);
    TM_HIP(hipGetLastError());
    project_components(c, Cf, 4, mom, out, s);
}
