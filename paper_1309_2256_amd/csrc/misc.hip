// Layout conversion, gauge ingest, Z4 noise and the loop contraction kernel.
#include "tm_internal.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ long lex_site(const Geo &g, int x, int y, int z, int t)
{
    return x + (long)g.L[0] * (y + (long)g.L[1] * (z + (long)g.L[2] * t));
}

// ---------------------------------------------------------------- pack / unpack

// The canonical field stores the 12 complex of a site contiguously, the half
// layout one plane per component: a block stages its 256 sites' 3072
// complex in LDS (row stride 13 to spread the banks), so that the global
// reads and the plane writes are both coalesced.
constexpr int kPackRow = 13;

__device__ __forceinline__ int site_parity(const Geo &g, long s)
{
    int q = (int)(s / g.L[0]);
    int x = (int)(s - (long)q * g.L[0]);
    int y = q % g.L[1];
    int q2 = q / g.L[1];
    int z = q2 % g.L[2];
    int t = q2 / g.L[2];
    return (x + y + z + t) & 1;
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_pack(S *even, S *odd, const double2 *full, Geo g, long V,
                                                 const double *scale)
{
    __shared__ double2 buf[kBlock * kPackRow];
    const long s0 = (long)blockIdx.x * kBlock;
    const int r = blockIdx.y;
    const int ns = (int)(V - s0 < kBlock ? V - s0 : kBlock);  // sites of this block
    const double2 *src = full + ((size_t)r * V + s0) * 12;
    for (int e = threadIdx.x; e < 12 * ns; e += kBlock) buf[(e / 12) * kPackRow + e % 12] = src[e];
    __syncthreads();
    if ((int)threadIdx.x >= ns) return;
    const long s = s0 + threadIdx.x;
    const int i = (int)(s >> 1);
    S *dst = site_parity(g, s) ? odd : even;
    const double sc = scale ? scale[r] : 1.0;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double2 v = buf[threadIdx.x * kPackRow + k];
        stT<double>(dst, (size_t)(r * 12 + k) * g.hs + i, cx<double>{sc * v.x, sc * v.y});
    }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_unpack(double2 *full, const S *even, const S *odd, Geo g, long V)
{
    __shared__ double2 buf[kBlock * kPackRow];
    const long s0 = (long)blockIdx.x * kBlock;
    const int r = blockIdx.y;
    const int ns = (int)(V - s0 < kBlock ? V - s0 : kBlock);
    if ((int)threadIdx.x < ns) {
        const long s = s0 + threadIdx.x;
        const int i = (int)(s >> 1);
        const S *src = site_parity(g, s) ? odd : even;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const cx<double> v = ldT<double>(src, (size_t)(r * 12 + k) * g.hs + i);
            buf[threadIdx.x * kPackRow + k] = make_double2(v.r, v.i);
        }
    }
    __syncthreads();
    double2 *dst = full + ((size_t)r * V + s0) * 12;
    for (int e = threadIdx.x; e < 12 * ns; e += kBlock) dst[e] = buf[(e / 12) * kPackRow + e % 12];
}

// ---------------------------------------------------------------- gauge

// links[p][d][k][i]: d < 4 forward U_d(x), d >= 4 backward U_{d-4}(x - e)^dag,
// times the time-boundary phase on hops that cross t = Lt-1 <-> 0
__global__ __launch_bounds__(kBlock) void k_gauge_ingest(double2 *l0, double2 *l1, const double2 *U, Geo g,
                                                         long V, int t_bc)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    const int p = blockIdx.y;
    double2 *dst = p ? l1 : l0;
    int x, y, z, t;
    eo_coords(g, p, i, x, y, z, t);
    const long s = lex_site(g, x, y, z, t);
    for (int mu = 0; mu < 4; mu++) {
        double ph = (mu == 3 && t == g.L[3] - 1) ? (double)t_bc : 1.0;
        for (int k = 0; k < 9; k++) {
            double2 u = U[((size_t)mu * V + s) * 9 + k];
            dst[(size_t)(mu * 9 + k) * g.vh + i] = make_double2(ph * u.x, ph * u.y);
        }
        int c[4] = {x, y, z, t};
        c[mu] = (c[mu] == 0) ? g.L[mu] - 1 : c[mu] - 1;
        const long sb = lex_site(g, c[0], c[1], c[2], c[3]);
        double phb = (mu == 3 && t == 0) ? (double)t_bc : 1.0;
        for (int row = 0; row < 3; row++)
            for (int col = 0; col < 3; col++) {
                // (U^dag)[row][col] = conj(U[col][row])
                double2 u = U[((size_t)mu * V + sb) * 9 + 3 * col + row];
                dst[(size_t)((4 + mu) * 9 + 3 * row + col) * g.vh + i] = make_double2(phb * u.x, -phb * u.y);
            }
    }
}

// Deviation of each link from SU(3): max over entries of |U U^dag - 1| and
// |det U - 1|; per-block maxima, then one block takes the maximum of those.
__global__ __launch_bounds__(kBlock) void k_su3_dev(const double2 *U, long nlinks, double *part)
{
    const long l = (long)blockIdx.x * kBlock + threadIdx.x;
    double dev = 0;
    if (l < nlinks) {
        cx<double> u[9];
        for (int k = 0; k < 9; k++) {
            const double2 v = U[l * 9 + k];
            u[k] = {v.x, v.y};
        }
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                cx<double> acc{a == b ? -1.0 : 0.0, 0.0};
                for (int k = 0; k < 3; k++) cmac(acc, u[3 * a + k], conjg(u[3 * b + k]));
                dev = fmax(dev, fmax(fabs(acc.r), fabs(acc.i)));
            }
        const cx<double> det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                               u[2] * (u[3] * u[7] - u[4] * u[6]);
        dev = fmax(dev, fmax(fabs(det.r - 1.0), fabs(det.i)));
        if (dev != dev) dev = INFINITY;  // NaN entries count as far off
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = dev;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_max_finish(const double *part, long n, double *out)
{
    double m = 0;
    for (long k = threadIdx.x; k < n; k += kBlock) m = fmax(m, part[k]);
    __shared__ double red[kBlock];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// out[d][k][i] = binary16(in[d][k][i]) for the first two rows (k < 6) of
// every link, d < 8, i < vh
__global__ __launch_bounds__(kBlock) void k_d2h_rows(h2 *out, const double2 *in, long vh)
{
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 48 * vh) return;
    const long i = idx % vh, dk = idx / vh;
    const long d = dk / 6, k = dk % 6;
    const double2 v = in[(d * 9 + k) * vh + i];
    out[idx] = h2{(_Float16)v.x, (_Float16)v.y};
}

// the same rows kept in FP64
__global__ __launch_bounds__(kBlock) void k_d2d_rows(double2 *out, const double2 *in, long vh)
{
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 48 * vh) return;
    const long i = idx % vh, dk = idx / vh;
    const long d = dk / 6, k = dk % 6;
    out[idx] = in[(d * 9 + k) * vh + i];
}

// 8-parameter FP64 links (appendix A.1; the paper stores 8 real numbers per
// link and recomputes the full matrix in the kernel).  Of U = [[a1 a2 a3],
// [b1 b2 b3], [c1 c2 c3]] in SU(3) the form keeps the complex a2, a3, b1 and
// the phases of a1 and c1: |a1| and |c1| follow from the unit first row and
// first column, and the 2x2 block from conj(U) = cofactor matrix (U^-1 = U^dag,
// det U = 1), a linear system in (b2, b3) and in (c2, c3) with determinant
// n = |a2|^2 + |a3|^2.  |c1|^2 = n - |b1|^2 loses accuracy when |c1| << |b1|;
// such links are stored as W = -(rows 1, 3, 2 of U) (again special unitary,
// its first-column entries below a1 being -c1, -b1), flagged by adding 8 to
// the stored phase of W's c1, and the kernel swaps and negates the rows back.
// The boundary factor folded into the stored links (f = -1 makes det = -1) is
// removed here and restored by the kernel on the links that cross the
// boundary.  Layout [8 directions][4][vh] double2: a2, a3, b1, (arg a1, arg c1
// [+ 8]).  part[block] = smallest n of the block.
__global__ __launch_bounds__(kBlock) void k_d2r8(double2 *out, const double2 *in, Geo g, int p, int t_bc,
                                                 double *part)
{
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    const long vh = g.vh;
    double nmin = INFINITY;
    if (idx < 8 * vh) {
        const long i = idx % vh, d = idx / vh;
        int x, y, z, t;
        eo_coords(g, p, (int)i, x, y, z, t);
        const bool cross = (d == 3 && t == g.L[3] - 1) || (d == 7 && t == 0);
        const double f = cross ? (double)t_bc : 1.0;
        cx<double> u[9];
        for (int k = 0; k < 9; k++) {
            const double2 v = in[(d * 9 + k) * vh + i];
            u[k] = {f * v.x, f * v.y};
        }
        const bool swap = u[6].r * u[6].r + u[6].i * u[6].i < u[3].r * u[3].r + u[3].i * u[3].i;
        if (swap) {
            for (int k = 0; k < 3; k++) {
                const cx<double> r1 = u[3 + k], r2 = u[6 + k];
                u[k] = {-u[k].r, -u[k].i};
                u[3 + k] = {-r2.r, -r2.i};
                u[6 + k] = {-r1.r, -r1.i};
            }
        }
        double2 *o = out + d * 4 * vh + i;
        o[0] = make_double2(u[1].r, u[1].i);
        o[vh] = make_double2(u[2].r, u[2].i);
        o[2 * vh] = make_double2(u[3].r, u[3].i);
        o[3 * vh] = make_double2(atan2(u[0].i, u[0].r), atan2(u[6].i, u[6].r) + (swap ? 8.0 : 0.0));
        nmin = u[1].r * u[1].r + u[1].i * u[1].i + u[2].r * u[2].r + u[2].i * u[2].i;
        if (nmin != nmin) nmin = 0;  // NaN entries: the form is not used
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = nmin;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_min_finish(const double *part, long n, double *out)
{
    double m = INFINITY;
    for (long k = threadIdx.x; k < n; k += kBlock) m = fmin(m, part[k]);
    __shared__ double red[kBlock];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// and rounded once to FP32
__global__ __launch_bounds__(kBlock) void k_d2f_rows(float2 *out, const double2 *in, long vh)
{
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 48 * vh) return;
    const long i = idx % vh, dk = idx / vh;
    const long d = dk / 6, k = dk % 6;
    const double2 v = in[(d * 9 + k) * vh + i];
    out[idx] = make_float2((float)v.x, (float)v.y);
}

__global__ __launch_bounds__(kBlock) void k_d2f(float2 *out, const double2 *in, size_t n)
{
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        double2 v = in[e];
        out[e] = make_float2((float)v.x, (float)v.y);  // round to nearest even
    }
}

// one rounding FP64 -> binary16 (not through FP32)
__global__ __launch_bounds__(kBlock) void k_d2h(h2 *out, const double2 *in, size_t n)
{
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        double2 v = in[e];
        h2 o;
        o.x = (_Float16)v.x;
        o.y = (_Float16)v.y;
        out[e] = o;
    }
}

// ---------------------------------------------------------------- noise

// SplitMix64 (Steele, Lea & Flood 2014): output c of the stream seeded with
// `seed` is the finaliser applied to seed + (c + 1) * golden-gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Z4 noise number r: entry (site s, spin a, colour c) is i^k, k = top two bits
// of output ((r*V + s)*4 + a)*3 + c.  dilution = 1 writes 12 right-hand sides,
// source d = 3a + c holding only that component.
// RHS j = q * nsc + d (nsc = 12 with spin-colour dilution, else 1): the noise
// restricted to spin-colour component d (when diluted) and, with time
// dilution (t_period > 0), to the slices t = o_first + q (mod t_period).
__global__ __launch_bounds__(kBlock) void k_noise(double2 *even, double2 *odd, Geo g, long V, uint64_t seed,
                                                  long r, int dilution, int t_period, int o_first, int n_off)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    const int p = blockIdx.y;
    double2 *dst = p ? odd : even;
    int x, y, z, t;
    eo_coords(g, p, i, x, y, z, t);
    const long s = lex_site(g, x, y, z, t);
    double2 eta[12];
    for (int k = 0; k < 12; k++) {
        uint64_t cnt = (uint64_t)((r * V + s) * 12 + k);
        unsigned q = (unsigned)(splitmix64_at(seed, cnt) >> 62);
        // i^q
        eta[k] = q == 0 ? make_double2(1, 0) : q == 1 ? make_double2(0, 1) : q == 2 ? make_double2(-1, 0)
                                                                                   : make_double2(0, -1);
    }
    const int nsc = dilution ? 12 : 1;
    for (int q = 0; q < n_off; q++) {
        const bool on = t_period == 0 || t % t_period == o_first + q;
        for (int d = 0; d < nsc; d++)
            for (int k = 0; k < 12; k++) {
                const bool keep = on && (!dilution || k == d);
                dst[(size_t)((q * nsc + d) * 12 + k) * g.hs + i] = keep ? eta[k] : make_double2(0, 0);
            }
    }
}

// ---------------------------------------------------------------- contraction

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Per time slice and block: C[b][a] = sum_{x, rhs, colour} v_{b c}(x) conj(w_{a c}(x)),
// both parities, FP64; partial[t][blk][32].
template <typename S>
// time slices t = t0 + dt * blockIdx.y
__global__ __launch_bounds__(kBlock) void k_outer(const S *ve, const S *vo, const S *we, const S *wo, Geo g,
                                                  int nrhs, int t0, int dt, double *part)
{
    const int t = t0 + dt * (int)blockIdx.y;
    const int il = blockIdx.x * kBlock + threadIdx.x;
    cx<double> C[16];
#pragma unroll
    for (int k = 0; k < 16; k++) C[k] = {0, 0};
    if (il < g.vsh) {
        const int i = t * g.vsh + il;
        for (int p = 0; p < 2; p++) {
            const S *v = p ? vo : ve;
            const S *w = p ? wo : we;
            for (int r = 0; r < nrhs; r++) {
                cx<double> a[12], b[12];
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    a[k] = ldT<double>(v, (size_t)(r * 12 + k) * g.hs + i);
                    b[k] = ldT<double>(w, (size_t)(r * 12 + k) * g.hs + i);
                }
#pragma unroll
                for (int sb = 0; sb < 4; sb++)
#pragma unroll
                    for (int sa = 0; sa < 4; sa++)
#pragma unroll
                        for (int c = 0; c < 3; c++) cmac_conj(C[sb * 4 + sa], b[sa * 3 + c], a[sb * 3 + c]);
            }
        }
    }
    __shared__ double red[kBlock / 64][32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        double re = wave_sum(C[k].r), im = wave_sum(C[k].i);
        if (lane == 0) {
            red[wv][2 * k] = re;
            red[wv][2 * k + 1] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        double s = 0;
        for (int k = 0; k < kBlock / 64; k++) s += red[k][threadIdx.x];
        part[((size_t)t * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = s;
    }
}

// slices not visited by k_outer (t != t0 mod dt, or t < t0) are zero
__global__ void k_outer_finish(const double *part, int nblk, int t0, int dt, double *out)
{
    const int t = blockIdx.x;
    const int j = threadIdx.x;  // 32 values
    double s = 0;
    if (t >= t0 && (t - t0) % dt == 0)
        for (int b = 0; b < nblk; b++) s += part[((size_t)t * nblk + b) * 32 + j];
    out[(size_t)t * 32 + j] = s;
}

template <typename F>
void dispatch_prec(int prec, F &&f)
{
    switch (prec) {
    case TM_F64: f((double2 *)nullptr); break;
    case TM_F32: f((float2 *)nullptr); break;
    case TM_F16: f((h2 *)nullptr); break;
    case TM_BF16: f((b2 *)nullptr); break;
    default: throw TmError{TM_ERR_ARG, "bad precision"};
    }
}

}  // namespace

void launch_pack(tm_ctx *c, void *even, void *odd, const double *full, int nrhs, int prec,
                 const double *dscale, hipStream_t s)
{
    dim3 grid((unsigned)((c->V + kBlock - 1) / kBlock), nrhs);
    account(c, (double)c->V * 12 * nrhs * (16 + prec_bytes(prec)), 0.0);
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_pack<S>, grid, dim3(kBlock), 0, s, (S *)even, (S *)odd, (const double2 *)full,
                           c->geo, c->V, dscale);
    });
    TM_HIP(hipGetLastError());
}

void launch_unpack(tm_ctx *c, double *full, const void *even, const void *odd, int nrhs, int prec,
                   hipStream_t s)
{
    dim3 grid((unsigned)((c->V + kBlock - 1) / kBlock), nrhs);
    account(c, (double)c->V * 12 * nrhs * (16 + prec_bytes(prec)), 0.0);
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_unpack<S>, grid, dim3(kBlock), 0, s, (double2 *)full, (const S *)even,
                           (const S *)odd, c->geo, c->V);
    });
    TM_HIP(hipGetLastError());
}

void launch_gauge_ingest(tm_ctx *c, const double *U, hipStream_t s)
{
    dim3 grid((c->geo.vh + kBlock - 1) / kBlock, 2);
    hipLaunchKernelGGL(k_gauge_ingest, grid, dim3(kBlock), 0, s, (double2 *)c->links64[0],
                       (double2 *)c->links64[1], (const double2 *)U, c->geo, c->V, c->t_bc);
    TM_HIP(hipGetLastError());
}

double gauge_su3_deviation(tm_ctx *c, const double *U, hipStream_t s)
{
    const long nl = 4 * c->V;
    const long nb = (nl + kBlock - 1) / kBlock;
    double *part = (double *)ws_get(c, "su3_part", sizeof(double) * (nb + 1));
    hipLaunchKernelGGL(k_su3_dev, dim3((unsigned)nb), dim3(kBlock), 0, s, (const double2 *)U, nl, part + 1);
    TM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(kBlock), 0, s, (const double *)(part + 1), nb, part);
    TM_HIP(hipGetLastError());
    double dev = 0;
    TM_HIP(hipMemcpyAsync(&dev, part, sizeof(double), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    return dev;
}

void launch_links_to_f32(tm_ctx *c, hipStream_t s)
{
    size_t n = (size_t)72 * c->geo.vh;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_d2f, dim3(2048), dim3(kBlock), 0, s, (float2 *)c->links32[p],
                           (const double2 *)c->links64[p], n);
    TM_HIP(hipGetLastError());
}

void launch_links_to_r12(tm_ctx *c, hipStream_t s)
{
    const long n = 48L * c->geo.vh;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_d2h_rows, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           (h2 *)c->links12[p], (const double2 *)c->links64[p], (long)c->geo.vh);
    TM_HIP(hipGetLastError());
}

double launch_links_to_r8d(tm_ctx *c, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TM_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        throw TmError{TM_ERR_UNSUPPORTED, "8-parameter links are built on first use outside graph capture"};
    const long n = 8L * c->geo.vh;
    const long nb = (n + kBlock - 1) / kBlock;
    double *part = (double *)ws_get(c, "r8_part", sizeof(double) * (2 * nb + 1));
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_d2r8, dim3((unsigned)nb), dim3(kBlock), 0, s, (double2 *)c->links8d[p],
                           (const double2 *)c->links64[p], c->geo, p, c->t_bc, part + 1 + p * nb);
    TM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(kBlock), 0, s, (const double *)(part + 1), 2 * nb, part);
    TM_HIP(hipGetLastError());
    double nmin = 0;
    TM_HIP(hipMemcpyAsync(&nmin, part, sizeof(double), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    return nmin;
}

void launch_links_to_r12d(tm_ctx *c, hipStream_t s)
{
    const long n = 48L * c->geo.vh;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_d2d_rows, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           (double2 *)c->links12d[p], (const double2 *)c->links64[p], (long)c->geo.vh);
    TM_HIP(hipGetLastError());
}

void launch_links_to_r12f(tm_ctx *c, hipStream_t s)
{
    const long n = 48L * c->geo.vh;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_d2f_rows, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           (float2 *)c->links12f[p], (const double2 *)c->links64[p], (long)c->geo.vh);
    TM_HIP(hipGetLastError());
}

void launch_links_to_f16(tm_ctx *c, hipStream_t s)
{
    size_t n = (size_t)72 * c->geo.vh;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_d2h, dim3(2048), dim3(kBlock), 0, s, (h2 *)c->links16[p],
                           (const double2 *)c->links64[p], n);
    TM_HIP(hipGetLastError());
}

void launch_noise(tm_ctx *c, void *even, void *odd, uint64_t seed, long r, int dilution, hipStream_t s,
                  int t_period, int o_first, int n_off)
{
    dim3 grid((c->geo.vh + kBlock - 1) / kBlock, 2);
    hipLaunchKernelGGL(k_noise, grid, dim3(kBlock), 0, s, (double2 *)even, (double2 *)odd, c->geo, c->V, seed,
                       r, dilution, t_period, o_first, n_off);
    TM_HIP(hipGetLastError());
}

void launch_outer_slices(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                         double *dev_out, hipStream_t s, int t0, int dt)
{
    const int nblk = (c->geo.vsh + kBlock - 1) / kBlock;
    const int Lt = c->geo.L[3];
    TM_REQUIRE(t0 >= 0 && t0 < Lt && dt >= 1, "bad time-slice selection");
    const int n_t = (Lt - t0 + dt - 1) / dt;
    double *part = (double *)ws_get(c, "outer_part", sizeof(double) * 32 * nblk * Lt);
    hipLaunchKernelGGL(k_outer<double2>, dim3(nblk, n_t), dim3(kBlock), 0, s, (const double2 *)ve,
                       (const double2 *)vo, (const double2 *)we, (const double2 *)wo, c->geo, nrhs, t0, dt, part);
    hipLaunchKernelGGL(k_outer_finish, dim3(Lt), dim3(32), 0, s, (const double *)part, nblk, t0, dt, dev_out);
    TM_HIP(hipGetLastError());
}
