// Learned preconditioner: a gauge-covariant parallel-transport convolution
// network (PTC, the layer form of Lehner and Wettig, arXiv:2302.05419) with
// one input channel, nc hidden channels and one output channel over the nine
// paths {identity, the eight nearest-neighbour hops}:
//   phi_c = sum_k W1[k][c] T_k psi,   N(psi) = sum_{k,c} W2[k][c] T_k phi_c,
// W[k][c] a 4x4 complex spin matrix.  Both layers are linear and every T_k
// commutes with spin matrices, so the device evaluates the collapsed form
//   N(psi) = sum_k T_k u_k,   u_k = sum_k' A[k][k'] T_k' psi,
//   A[k][k'] = sum_c W2[k][c] W1[k'][c]                               (*)
// in two passes over the lattice (k_ptc_mix forms the nine u_k of one
// parity, k_ptc_gather transports them back), and trains through (*): the
// loss gradient with respect to A is a colour-traced outer product summed
// over the lattice,
//   dl/dA[k][k'] = sum_x (T_k^dag delta)(x) (T_k' psi)(x)^dag,
//   delta = 2 (N(psi) - e) / |e|^2,   T_k^dag = T_(k+4 mod 8) (reversed hop),
// and the chain rule through (*) gives
//   dl/dW2[k][c] = sum_k' dl/dA[k][k'] W1[k'][c]^dag,
//   dl/dW1[k'][c] = sum_k W2[k][c]^dag dl/dA[k][k'],
// with complex gradients G = dl/dRe w + i dl/dIm w.  Fields are half-lattice
// FP32 (or BF16 for stored training pairs); links are the FP32 even-odd
// copies of the Dslash (direction d = k - 1, backward links pre-conjugated,
// boundary phase folded in).  Weight updates use Adam (Kingma and Ba 2015)
// in FP64 in one block.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "runtime.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxNc = 64;
constexpr int kGradBlocks = 240;  // site blocks of the gradient reduction
constexpr int kKG = 3;            // paths k per thread of k_ptc_mix

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// half-site index of the neighbour of (x, y, z, t) in direction d (d < 4:
// +mu, else -mu, mu = d & 3), periodic wrap
__device__ __forceinline__ int nb_index(const Geo &g, int x, int y, int z, int t, int d)
{
    const int mu = d & 3, step = d < 4 ? 1 : -1;
    int c[4] = {x, y, z, t};
    c[mu] += step;
    if (c[mu] == g.L[mu]) c[mu] = 0;
    if (c[mu] < 0) c[mu] = g.L[mu] - 1;
    return eo_index(g, c[0], c[1], c[2], c[3]);
}

// f -> W f on each of the four spins (W row-major 3x3)
__device__ __forceinline__ void colour_mul(cx<float> out[12], const cx<float> W[9], const cx<float> f[12])
{
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int r = 0; r < 3; r++) {
            cx<float> acc = {0, 0};
#pragma unroll
            for (int c = 0; c < 3; c++) cmac(acc, W[3 * r + c], f[3 * a + c]);
            out[3 * a + r] = acc;
        }
}

// (T_k f)(i) on output parity p: identity from the same parity, else the link
// of direction k - 1 at i times f at the neighbour (other parity)
template <typename S>
__device__ __forceinline__ void transport_at(cx<float> out[12], int k, const S *same, const S *other,
                                             const float2 *links, const Geo &g, int i, int x, int y, int z,
                                             int t)
{
    const size_t vh = (size_t)g.vh, hs = (size_t)g.hs;  // link and field plane strides
    if (k == 0) {
#pragma unroll
        for (int e = 0; e < 12; e++) out[e] = ldT<float>(same, e * hs + i);
        return;
    }
    const int d = k - 1;
    const int j = nb_index(g, x, y, z, t, d);
    cx<float> W[9], f[12];
#pragma unroll
    for (int e = 0; e < 9; e++) {
        const float2 w = links[((size_t)d * 9 + e) * vh + i];
        W[e] = {w.x, w.y};
    }
#pragma unroll
    for (int e = 0; e < 12; e++) f[e] = ldT<float>(other, e * hs + j);
    colour_mul(out, W, f);
}

// u_k (parity p) = sum_k' A[k][k'] T_k' in, for kKG consecutive k per thread.
// grid (site blocks, nrhs, 3); u layout [9][nrhs][12][hs].
template <typename S>
__global__ __launch_bounds__(kBlock) void k_ptc_mix(const S *in_same, const S *in_other, const float2 *links,
                                                    const float2 *__restrict__ A, float2 *u, Geo g, int p,
                                                    int nrhs)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    const int r = blockIdx.y, k0 = blockIdx.z * kKG;
    const size_t fs = (size_t)12 * g.hs;
    const S *same = in_same + r * fs, *other = in_other + r * fs;
    int x, y, z, t;
    eo_coords(g, p, i, x, y, z, t);
    cx<float> acc[kKG][12];
#pragma unroll
    for (int kk = 0; kk < kKG; kk++)
#pragma unroll
        for (int e = 0; e < 12; e++) acc[kk][e] = {0, 0};
#pragma unroll 1
    for (int kp = 0; kp < 9; kp++) {
        cx<float> gv[12];
        transport_at<S>(gv, kp, same, other, links, g, i, x, y, z, t);
#pragma unroll
        for (int kk = 0; kk < kKG; kk++) {
            const float2 *Sm = A + ((k0 + kk) * 9 + kp) * 16;
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const float2 w = Sm[4 * a + b];
                    const cx<float> wc = {w.x, w.y};
#pragma unroll
                    for (int c = 0; c < 3; c++) cmac(acc[kk][3 * a + c], wc, gv[3 * b + c]);
                }
        }
    }
    const size_t hs = (size_t)g.hs;
#pragma unroll
    for (int kk = 0; kk < kKG; kk++) {
        float2 *uo = u + ((size_t)(k0 + kk) * nrhs + r) * fs;
#pragma unroll
        for (int e = 0; e < 12; e++) uo[e * hs + i] = make_float2(acc[kk][e].r, acc[kk][e].i);
    }
}

// ---------------------------------------------------------------- matrix cores
// The spin mixing u = A G at one site, A the 36x36 complex block matrix
// A[(k,a)][(k',b)] = A[k][k'][a][b] and G[(k',b)][c] = (T_k' psi)_{b c}, as a
// real product on v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation)
// with real and imaginary parts interleaved: row 2i+ri, column 2j+rj of the
// real A is Re A_ij (ri = rj), -Im A_ij (ri = 0, rj = 1), Im A_ij (ri = 1,
// rj = 0); row 2j+rj of the real G holds Re / Im G_j.  72 x 72 padded to 5
// row tiles of 16 and 3 K steps of 32.  One wave takes 16 sites (the MFMA
// columns) and one colour c at a time.  Operand lanes: A[i][k] in lane
// (i = l % 16, g = l / 16) at k = 8g + j; B[k][n] in lane (n = l % 16, g) at
// k = 8g + j; D[i][n] in lane (n, g) at i = 4g + v (v = 0..3).  So lane
// (n, g) at K step q holds path k' = 4q + g of site n (8 values: 4 spins,
// re/im), and its D of row tile t holds complex rows 8t + 2g, 8t + 2g + 1.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMT = 5, kKS = 3;  // row tiles, K steps

// frag[(t * kKS + q) * 64 + lane] = the A operand of row tile t, K step q
__global__ void k_ptc_afrag(const float2 *A, bf16x8 *frag)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kMT * kKS * 64) return;
    const int lane = idx % 64, tq = idx / 64, t = tq / kKS, q = tq % kKS;
    const int R = 16 * t + lane % 16, i = R / 2, ri = R % 2;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int K = 32 * q + 8 * (lane / 16) + j, jj = K / 2, rj = K % 2;
        float a = 0.f;
        if (i < 36 && jj < 36) {
            const float2 w = A[((i / 4) * 9 + jj / 4) * 16 + 4 * (i % 4) + jj % 4];
            a = ri == rj ? w.x : (ri == 0 ? -w.y : w.y);
        }
        v[j] = (__bf16)a;
    }
    frag[idx] = v;
}

// u_k (parity p) for all nine k on the matrix cores; block of 4 waves = 64
// sites, grid (site blocks of 64, nrhs).  u layout [9][nrhs][12][hs].
template <typename S>
__global__ __launch_bounds__(kBlock, 2) void k_ptc_mix_mfma(const S *in_same, const S *in_other,
                                                            const float2 *links, const bf16x8 *frag, float2 *u,
                                                            Geo g, int p, int nrhs)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane % 16, grp = lane / 16;
    const int i_raw = blockIdx.x * 64 + w * 16 + n;
    const bool valid = i_raw < g.vh;
    const int i = valid ? i_raw : g.vh - 1;
    const int r = blockIdx.y;
    const size_t fs = (size_t)12 * g.hs, hs = (size_t)g.hs;
    const S *same = in_same + r * fs, *other = in_other + r * fs;
    int x, y, z, t;
    eo_coords(g, p, i, x, y, z, t);
    // B operands: the transports of this lane's paths, per colour
    bf16x8 bq[3][kKS];
#pragma unroll
    for (int q = 0; q < kKS; q++) {
        const int kp = 4 * q + grp;
        cx<float> gv[12];
        if (kp <= 8) {
            transport_at<S>(gv, kp, same, other, links, g, i, x, y, z, t);
        } else {
#pragma unroll
            for (int e = 0; e < 12; e++) gv[e] = {0.f, 0.f};
        }
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int b = 0; b < 4; b++) {
                bq[c][q][2 * b] = (__bf16)gv[3 * b + c].r;
                bq[c][q][2 * b + 1] = (__bf16)gv[3 * b + c].i;
            }
    }
    bf16x8 af[kMT][kKS];
#pragma unroll
    for (int tt = 0; tt < kMT; tt++)
#pragma unroll
        for (int q = 0; q < kKS; q++) af[tt][q] = frag[(tt * kKS + q) * 64 + lane];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        f32x4 acc[kMT];
#pragma unroll
        for (int tt = 0; tt < kMT; tt++) acc[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kKS; q++)
#pragma unroll
            for (int tt = 0; tt < kMT; tt++)
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[tt][q], bq[c][q], acc[tt], 0, 0, 0);
        if (valid) {
#pragma unroll
            for (int tt = 0; tt < kMT; tt++)
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const int cr = 8 * tt + 2 * grp + e, k = cr / 4, a = cr % 4;
                    if (k < 9)
                        u[(((size_t)k * nrhs + r) * 12 + 3 * a + c) * hs + i] =
                            make_float2(acc[tt][2 * e], acc[tt][2 * e + 1]);
                }
        }
    }
}

// out (parity p) = u_0 + sum_{k >= 1} T_k u_k; u_same / u_other: the u
// fields of parity p / 1 - p.  grid (site blocks, nrhs).
template <typename SO>
__global__ __launch_bounds__(kBlock) void k_ptc_gather(const float2 *u_same, const float2 *u_other,
                                                       const float2 *links, SO *out, Geo g, int p, int nrhs)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    const int r = blockIdx.y;
    const size_t fs = (size_t)12 * g.hs, hs = (size_t)g.hs;
    int x, y, z, t;
    eo_coords(g, p, i, x, y, z, t);
    cx<float> acc[12];
    const float2 *u0 = u_same + (size_t)r * fs;
#pragma unroll
    for (int e = 0; e < 12; e++) {
        const float2 v = u0[e * hs + i];
        acc[e] = {v.x, v.y};
    }
#pragma unroll 1
    for (int k = 1; k < 9; k++) {
        cx<float> tv[12];
        const float2 *uk = u_other + ((size_t)k * nrhs + r) * fs;
        transport_at<float2>(tv, k, uk, uk, links, g, i, x, y, z, t);
#pragma unroll
        for (int e = 0; e < 12; e++) acc[e] = acc[e] + tv[e];
    }
    SO *o = out + (size_t)r * fs;
#pragma unroll
    for (int e = 0; e < 12; e++) stT<float>(o, e * hs + i, acc[e]);
}

// delta = 2 (out - e) / (nrhs |e_b|^2) for sample b, partial |out - e|^2
// per block, over the vh valid sites of each plane (stride hs; the pad
// sites of delta are not written).  grid (blocks, nrhs); part [nrhs][nblk].
template <typename SE>
__global__ __launch_bounds__(kBlock) void k_ptc_delta(const float2 *out, const SE *e, const double *en2,
                                                      float2 *delta, double *part, int vh, int hs, int nblk)
{
    const int r = blockIdx.y;
    const size_t base = (size_t)r * 12 * hs;
    const float sc = (float)(2.0 / (gridDim.y * en2[r]));
    double acc = 0;
    for (int q = 0; q < 12; q++)
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < vh; i += gridDim.x * kBlock) {
            const size_t k = base + (size_t)q * hs + i;
            const float2 o = out[k];
            const cx<float> ev = ldT<float>(e, k);
            const float dr = o.x - ev.r, di = o.y - ev.i;
            acc += (double)dr * dr + (double)di * di;
            delta[k] = make_float2(sc * dr, sc * di);
        }
    __shared__ double red[kBlock / 64];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int w = 0; w < kBlock / 64; w++) s += red[w];
        part[(size_t)r * nblk + blockIdx.x] = s;
    }
}

// loss += sum_b (sum of partials of both parities of sample b) / |e_b|^2 / nrhs
__global__ void k_ptc_loss_finish(const double *part0, const double *part1, const double *en2, int nblk,
                                  int nrhs, double *loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double l = 0;
    for (int r = 0; r < nrhs; r++) {
        double s = 0;
        for (int b = 0; b < nblk; b++) s += part0[(size_t)r * nblk + b];
        for (int b = 0; b < nblk; b++) s += part1[(size_t)r * nblk + b];
        l += s / en2[r];
    }
    *loss = l / nrhs;
}

// Residual loss: w -= r (r in the pair-store precision), partial |w|^2 per
// block, over the vh valid sites of each plane (stride hs).  grid (blocks,
// nrhs); part [nrhs][nblk].
template <typename SR>
__global__ __launch_bounds__(kBlock) void k_ptc_resid(float2 *w, const SR *r, double *part, int vh, int hs, int nblk)
{
    const size_t base = (size_t)blockIdx.y * 12 * hs;
    double acc = 0;
    for (int q = 0; q < 12; q++)
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < vh; i += gridDim.x * kBlock) {
            const size_t k = base + (size_t)q * hs + i;
            const float2 o = w[k];
            const cx<float> rv = ldT<float>(r, k);
            const float dr = o.x - rv.r, di = o.y - rv.i;
            acc += (double)dr * dr + (double)di * di;
            w[k] = make_float2(dr, di);
        }
    __shared__ double red[kBlock / 64];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int ww = 0; ww < kBlock / 64; ww++) s += red[ww];
        part[(size_t)blockIdx.y * nblk + blockIdx.x] = s;
    }
}

// v *= 2 / (nrhs |r_b|^2) for sample b = blockIdx.y
__global__ __launch_bounds__(kBlock) void k_ptc_scale(float2 *v, const double *rn2, size_t n)
{
    const size_t base = (size_t)blockIdx.y * n;
    const float sc = (float)(2.0 / (gridDim.y * rn2[blockIdx.y]));
    for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (size_t)gridDim.x * kBlock) {
        const float2 o = v[base + k];
        v[base + k] = make_float2(sc * o.x, sc * o.y);
    }
}

// Partial dl/dA[k][k'] on parity p: sum over the block's sites (grid-stride)
// and all samples of (T_kbar delta)(x) (T_k' in)(x)^dag, colour traced, FP64.
// grid (kGradBlocks, 81); part [81][kGradBlocks][32].
template <typename S>
__global__ __launch_bounds__(kBlock) void k_ptc_grad(const S *in_same, const S *in_other, const float2 *dl_same,
                                                     const float2 *dl_other, const float2 *links, Geo g, int p,
                                                     int nrhs, double *part)
{
    const int pair = blockIdx.y, k = pair / 9, kp = pair % 9;
    const int kbar = k == 0 ? 0 : (k <= 4 ? k + 4 : k - 4);
    const size_t fs = (size_t)12 * g.hs;
    double acc[32];
#pragma unroll
    for (int q = 0; q < 32; q++) acc[q] = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.vh; i += gridDim.x * kBlock) {
        int x, y, z, t;
        eo_coords(g, p, i, x, y, z, t);
#pragma unroll 1
        for (int r = 0; r < nrhs; r++) {
            cx<float> gv[12], hv[12];
            transport_at<S>(gv, kp, in_same + r * fs, in_other + r * fs, links, g, i, x, y, z, t);
            transport_at<float2>(hv, kbar, dl_same + r * fs, dl_other + r * fs, links, g, i, x, y, z, t);
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    double re = acc[2 * (4 * a + b)], im = acc[2 * (4 * a + b) + 1];
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        // h_a conj(g_b)
                        const double hr = hv[3 * a + c].r, hi = hv[3 * a + c].i;
                        const double gr = gv[3 * b + c].r, gi = gv[3 * b + c].i;
                        re = fma(hr, gr, re);
                        re = fma(hi, gi, re);
                        im = fma(hi, gr, im);
                        im = fma(-hr, gi, im);
                    }
                    acc[2 * (4 * a + b)] = re;
                    acc[2 * (4 * a + b) + 1] = im;
                }
        }
    }
    __shared__ double red[kBlock / 64][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 32; q++) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[w][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        double s = 0;
        for (int ww = 0; ww < kBlock / 64; ww++) s += red[ww][threadIdx.x];
        part[((size_t)pair * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = s;
    }
}

// dl/dA [81][16] complex from the partials of both parities, fixed order
__global__ void k_ptc_grad_finish(const double *part0, const double *part1, int nblk, double2 *GA)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // pair * 16 + element
    if (idx >= 81 * 16) return;
    const int pair = idx / 16, el = idx % 16;
    double re = 0, im = 0;
    for (int b = 0; b < nblk; b++) {
        re += part0[((size_t)pair * nblk + b) * 32 + 2 * el];
        im += part0[((size_t)pair * nblk + b) * 32 + 2 * el + 1];
    }
    for (int b = 0; b < nblk; b++) {
        re += part1[((size_t)pair * nblk + b) * 32 + 2 * el];
        im += part1[((size_t)pair * nblk + b) * 32 + 2 * el + 1];
    }
    GA[idx] = make_double2(re, im);
}

struct AdamArgs {
    double lr, b1, b2, eps;
    long step;  // 1-based step number of this update
};

__device__ __forceinline__ cx<double> ldc(const double2 *p, int k)
{
    const double2 v = p[k];
    return {v.x, v.y};
}

// mode 0: gradients only (G1, G2 from GA); mode 1: gradients then one Adam
// step on W1, W2; mode 2: neither.  Every mode ends by recomputing A (FP32)
// from the weights.  One block; W, G, M1/V1, M2/V2: [9][nc][16].
__global__ __launch_bounds__(kBlock) void k_ptc_update(int mode, int nc, const double2 *GA, double2 *W1,
                                                       double2 *W2, double2 *G1, double2 *G2, double2 *M1,
                                                       double2 *V1, double2 *M2, double2 *V2, AdamArgs ad,
                                                       float2 *A)
{
    const int nw = 9 * nc * 16;
    if (mode <= 1) {
        for (int idx = threadIdx.x; idx < nw; idx += blockDim.x) {
            const int kc = idx / 16, el = idx % 16, a = el / 4, b = el % 4;
            const int kk = kc / nc, c = kc % nc;
            // G2[k][c] = sum_k' GA[k][k'] W1[k'][c]^dag:   (a,b) += GA[a][e] conj(W1[b][e])
            cx<double> g2 = {0, 0};
            for (int kp = 0; kp < 9; kp++)
                for (int e = 0; e < 4; e++)
                    cmac_conj(g2, ldc(W1, (kp * nc + c) * 16 + 4 * b + e), ldc(GA, (kk * 9 + kp) * 16 + 4 * a + e));
            // G1[k'][c] = sum_k W2[k][c]^dag GA[k][k']:   (a,b) += conj(W2[e][a]) GA[e][b]  (here k' = kk)
            cx<double> g1 = {0, 0};
            for (int k = 0; k < 9; k++)
                for (int e = 0; e < 4; e++)
                    cmac_conj(g1, ldc(W2, (k * nc + c) * 16 + 4 * e + a), ldc(GA, (k * 9 + kk) * 16 + 4 * e + b));
            G1[idx] = make_double2(g1.r, g1.i);
            G2[idx] = make_double2(g2.r, g2.i);
        }
        __syncthreads();
    }
    if (mode == 1) {
        const double c1 = 1.0 - pow(ad.b1, (double)ad.step), c2 = 1.0 - pow(ad.b2, (double)ad.step);
        for (int idx = threadIdx.x; idx < 2 * nw; idx += blockDim.x) {
            const int w = idx / nw, k = idx % nw;
            double2 *W = w ? W2 : W1, *M = w ? M2 : M1, *Vv = w ? V2 : V1;
            const double2 gg = (w ? G2 : G1)[k];
            double2 m = M[k], v = Vv[k], x = W[k];
            m.x = ad.b1 * m.x + (1 - ad.b1) * gg.x;
            m.y = ad.b1 * m.y + (1 - ad.b1) * gg.y;
            v.x = ad.b2 * v.x + (1 - ad.b2) * gg.x * gg.x;
            v.y = ad.b2 * v.y + (1 - ad.b2) * gg.y * gg.y;
            x.x -= ad.lr * (m.x / c1) / (sqrt(v.x / c2) + ad.eps);
            x.y -= ad.lr * (m.y / c1) / (sqrt(v.y / c2) + ad.eps);
            M[k] = m;
            Vv[k] = v;
            W[k] = x;
        }
        __syncthreads();
    }
    // A[k][k'] = sum_c W2[k][c] W1[k'][c]
    for (int idx = threadIdx.x; idx < 81 * 16; idx += blockDim.x) {
        const int pair = idx / 16, el = idx % 16, a = el / 4, b = el % 4;
        const int k = pair / 9, kp = pair % 9;
        cx<double> s = {0, 0};
        for (int c = 0; c < nc; c++)
            for (int e = 0; e < 4; e++)
                cmac(s, ldc(W2, (k * nc + c) * 16 + 4 * a + e), ldc(W1, (kp * nc + c) * 16 + 4 * e + b));
        A[idx] = make_float2((float)s.r, (float)s.i);
    }
}

// ---------------------------------------------------------------- host side

int site_blocks(const tm_ctx *c) { return (c->geo.vh + kBlock - 1) / kBlock; }

size_t wbytes(int nc) { return sizeof(double2) * 9 * nc * 16; }

double2 *wbuf(tm_ctx *c, const char *name) { return (double2 *)ws_get(c, name, wbytes(kMaxNc)); }

void run_update(tm_ctx *c, int mode, const AdamArgs &ad, hipStream_t s)
{
    hipLaunchKernelGGL(k_ptc_update, dim3(1), dim3(kBlock), 0, s, mode, c->ptc_nc,
                       (const double2 *)ws_get(c, "ptc_GA", sizeof(double2) * 81 * 16), wbuf(c, "ptc_W1"),
                       wbuf(c, "ptc_W2"), wbuf(c, "ptc_G1"), wbuf(c, "ptc_G2"), wbuf(c, "ptc_M1"), wbuf(c, "ptc_V1"),
                       wbuf(c, "ptc_M2"), wbuf(c, "ptc_V2"), ad, (float2 *)ws_get(c, "ptc_A", sizeof(float2) * 81 * 16));
    TM_HIP(hipGetLastError());
    // BF16 operand fragments of A for the matrix-core spin mixing
    hipLaunchKernelGGL(k_ptc_afrag, dim3((kMT * kKS * 64 + 255) / 256), dim3(256), 0, s,
                       (const float2 *)ws_get(c, "ptc_A", sizeof(float2) * 81 * 16),
                       (bf16x8 *)ws_get(c, "ptc_Afrag", sizeof(bf16x8) * kMT * kKS * 64));
    TM_HIP(hipGetLastError());
}

// N(in) for nrhs fields given as FP32-or-BF16 halves (S) -> FP32 halves
template <typename S>
void forward_t(tm_ctx *c, const void *in_e, const void *in_o, float2 *out_e, float2 *out_o, int nrhs, hipStream_t s)
{
    ensure_links32(c, s);
    const size_t fl = (size_t)12 * c->geo.hs * nrhs;
    float2 *u[2] = {(float2 *)ws_get(c, "ptc_u0", sizeof(float2) * 9 * fl),
                    (float2 *)ws_get(c, "ptc_u1", sizeof(float2) * 9 * fl)};
    const float2 *A = (const float2 *)ws_get(c, "ptc_A", sizeof(float2) * 81 * 16);
    const S *in[2] = {(const S *)in_e, (const S *)in_o};
    if (c->ptc_arith == TM_BF16) {
        const bf16x8 *frag = (const bf16x8 *)ws_get(c, "ptc_Afrag", sizeof(bf16x8) * kMT * kKS * 64);
        dim3 gm((c->geo.vh + 63) / 64, nrhs);
        for (int p = 0; p < 2; p++) {
            hipLaunchKernelGGL(k_ptc_mix_mfma<S>, gm, dim3(kBlock), 0, s, in[p], in[1 - p],
                               (const float2 *)c->links32[p], frag, u[p], c->geo, p, nrhs);
            TM_HIP(hipGetLastError());
        }
    } else {
        dim3 gm(site_blocks(c), nrhs, 9 / kKG);
        for (int p = 0; p < 2; p++) {
            hipLaunchKernelGGL(k_ptc_mix<S>, gm, dim3(kBlock), 0, s, in[p], in[1 - p], (const float2 *)c->links32[p],
                               A, u[p], c->geo, p, nrhs);
            TM_HIP(hipGetLastError());
        }
    }
    float2 *out[2] = {out_e, out_o};
    dim3 gg(site_blocks(c), nrhs);
    for (int p = 0; p < 2; p++) {
        hipLaunchKernelGGL(k_ptc_gather<float2>, gg, dim3(kBlock), 0, s, (const float2 *)u[p],
                           (const float2 *)u[1 - p], (const float2 *)c->links32[p], out[p], c->geo, p, nrhs);
        TM_HIP(hipGetLastError());
    }
}

void forward(tm_ctx *c, int in_prec, const void *in_e, const void *in_o, float2 *out_e, float2 *out_o, int nrhs,
             hipStream_t s)
{
    if (in_prec == TM_BF16)
        forward_t<b2>(c, in_e, in_o, out_e, out_o, nrhs, s);
    else
        forward_t<float2>(c, in_e, in_o, out_e, out_o, nrhs, s);
}

// loss (device scalar) and dl/dA of the batch mean for nrhs pairs (r, e)
// given as halves in precision prec; en2: device |e_b|^2
// LossKind::error: l = |N(r) - e|^2 / |e|^2, en2 = |e|^2;
// LossKind::residual: l = |M N(r) - r|^2 / |r|^2 with M = M(epsp) in FP32
// (the Dslash of the FP32 solver), en2 = |r|^2, e unused:
//   w = M out - r,  dl/d(conj out) = M^dag w / |r|^2
enum class LossKind { error = 0, residual = 1 };

template <typename S>
void loss_grad_t(tm_ctx *c, LossKind kind, double epsp, const void *r_e, const void *r_o, const void *e_e,
                 const void *e_o, const double *en2, int nrhs, double *loss, hipStream_t s)
{
    const size_t fl = (size_t)12 * c->geo.hs * nrhs;
    float2 *out[2] = {(float2 *)ws_get(c, "ptc_out0", sizeof(float2) * fl),
                      (float2 *)ws_get(c, "ptc_out1", sizeof(float2) * fl)};
    forward_t<S>(c, r_e, r_o, out[0], out[1], nrhs, s);
    const int nbd = 256;
    double *part[2] = {(double *)ws_get(c, "ptc_lpart0", sizeof(double) * nbd * nrhs),
                       (double *)ws_get(c, "ptc_lpart1", sizeof(double) * nbd * nrhs)};
    float2 *dl[2] = {(float2 *)ws_get(c, "ptc_dl0", sizeof(float2) * fl),
                     (float2 *)ws_get(c, "ptc_dl1", sizeof(float2) * fl)};
    if (kind == LossKind::error) {
        const S *ee[2] = {(const S *)e_e, (const S *)e_o};
        for (int p = 0; p < 2; p++) {
            hipLaunchKernelGGL(k_ptc_delta<S>, dim3(nbd, nrhs), dim3(kBlock), 0, s, (const float2 *)out[p], ee[p],
                               en2, dl[p], part[p], c->geo.vh, c->geo.hs, nbd);
            TM_HIP(hipGetLastError());
        }
    } else {
        float2 *w[2] = {(float2 *)ws_get(c, "ptc_w0", sizeof(float2) * fl),
                        (float2 *)ws_get(c, "ptc_w1", sizeof(float2) * fl)};
        const double k = c->kappa;
        // w = M out (per parity: R(eps) out_p - kappa Hop out_{1-p}), then w -= r
        for (int p = 0; p < 2; p++)
            op_dslash(c, w[p], out[1 - p], out[p], nrhs, TM_F32, p, 0, sd_scalar(-k), sd_twist(epsp), s);
        const S *rr[2] = {(const S *)r_e, (const S *)r_o};
        for (int p = 0; p < 2; p++) {
            hipLaunchKernelGGL(k_ptc_resid<S>, dim3(nbd, nrhs), dim3(kBlock), 0, s, w[p], rr[p], part[p],
                               c->geo.vh, c->geo.hs, nbd);
            TM_HIP(hipGetLastError());
        }
        // dl = M^dag w = R(-eps) w_p - kappa Hop^dag w_{1-p}, scaled by 2 / (n |r|^2)
        for (int p = 0; p < 2; p++)
            op_dslash(c, dl[p], w[1 - p], w[p], nrhs, TM_F32, p, 1, sd_scalar(-k), sd_twist(-epsp), s);
        for (int p = 0; p < 2; p++) {
            hipLaunchKernelGGL(k_ptc_scale, dim3(nbd, nrhs), dim3(kBlock), 0, s, dl[p], en2, (size_t)12 * c->geo.hs);
            TM_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_ptc_loss_finish, dim3(1), dim3(64), 0, s, (const double *)part[0], (const double *)part[1],
                       en2, nbd, nrhs, loss);
    TM_HIP(hipGetLastError());
    double *gp[2] = {(double *)ws_get(c, "ptc_gpart0", sizeof(double) * 81 * kGradBlocks * 32),
                     (double *)ws_get(c, "ptc_gpart1", sizeof(double) * 81 * kGradBlocks * 32)};
    const S *rr[2] = {(const S *)r_e, (const S *)r_o};
    const int nb = std::min(kGradBlocks, site_blocks(c));
    for (int p = 0; p < 2; p++) {
        hipLaunchKernelGGL(k_ptc_grad<S>, dim3(nb, 81), dim3(kBlock), 0, s, rr[p], rr[1 - p], (const float2 *)dl[p],
                           (const float2 *)dl[1 - p], (const float2 *)c->links32[p], c->geo, p, nrhs, gp[p]);
        TM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ptc_grad_finish, dim3((81 * 16 + 255) / 256), dim3(256), 0, s, (const double *)gp[0],
                       (const double *)gp[1], nb, (double2 *)ws_get(c, "ptc_GA", sizeof(double2) * 81 * 16));
    TM_HIP(hipGetLastError());
}

void loss_grad(tm_ctx *c, LossKind kind, double epsp, int prec, const void *r_e, const void *r_o, const void *e_e,
               const void *e_o, const double *en2, int nrhs, double *loss, hipStream_t s)
{
    if (prec == TM_BF16)
        loss_grad_t<b2>(c, kind, epsp, r_e, r_o, e_e, e_o, en2, nrhs, loss, s);
    else
        loss_grad_t<float2>(c, kind, epsp, r_e, r_o, e_e, e_o, en2, nrhs, loss, s);
}

LossKind loss_kind(int loss)
{
    TM_REQUIRE(loss == TM_PTC_LOSS_ERROR || loss == TM_PTC_LOSS_RESIDUAL,
               "loss must be TM_PTC_LOSS_ERROR or TM_PTC_LOSS_RESIDUAL");
    return loss == TM_PTC_LOSS_ERROR ? LossKind::error : LossKind::residual;
}

template <typename F>
int guard(tm_ctx *c, F &&f)
{
    if (!c) return TM_ERR_ARG;
    try {
        c->err.clear();
        TM_HIP(hipSetDevice(c->device));
        return f();
    } catch (const TmError &e) {
        c->err = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        c->err = "host allocation failed";
        return TM_ERR_OOM;
    } catch (...) {
        c->err = "unexpected internal error";
        return TM_ERR_HIP;
    }
}

hipStream_t hs(tm_stream s) { return (hipStream_t)s; }

uint64_t splitmix(uint64_t &state)
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void reset_adam(tm_ctx *c, hipStream_t s)
{
    for (const char *n : {"ptc_M1", "ptc_V1", "ptc_M2", "ptc_V2"})
        TM_HIP(hipMemsetAsync(wbuf(c, n), 0, wbytes(kMaxNc), s));
    c->ptc_step = 0;
}

// store layout: [parity][capacity][12][hs] of the store precision
size_t store_half_bytes(const tm_ctx *c) { return prec_bytes(c->ptc_store) * 12 * (size_t)c->geo.hs; }

}  // namespace

// out = N(in) on FP32 half fields (used by the flexible GMRES)
void ptc_apply_halves(tm_ctx *c, const void *in_e, const void *in_o, void *out_e, void *out_o, int nrhs,
                      hipStream_t s)
{
    TM_REQUIRE(c->ptc_nc > 0, "no network weights set");
    forward(c, TM_F32, in_e, in_o, (float2 *)out_e, (float2 *)out_o, nrhs, s);
}

extern "C" int tm_ptc_set_weights(tm_ctx *c, int nc, const double *W1, const double *W2)
{
    return guard(c, [&]() {
        TM_REQUIRE(W1 && W2, "null pointer");
        TM_REQUIRE(nc >= 1 && nc <= kMaxNc, "nc must be in [1, 64]");
        for (size_t k = 0; k < (size_t)2 * 9 * nc * 16; k++)
            TM_REQUIRE(std::isfinite(W1[k]) && std::isfinite(W2[k]), "non-finite weight");
        hipStream_t s = nullptr;
        c->ptc_nc = nc;
        upload(wbuf(c, "ptc_W1"), W1, wbytes(nc), s);
        upload(wbuf(c, "ptc_W2"), W2, wbytes(nc), s);
        reset_adam(c, s);
        run_update(c, 2, AdamArgs{}, s);
        TM_HIP(hipStreamSynchronize(s));
        return TM_OK;
    });
}

extern "C" int tm_ptc_set_arith(tm_ctx *c, int prec)
{
    return guard(c, [&]() {
        TM_REQUIRE(prec == TM_F32 || prec == TM_BF16, "network arithmetic must be TM_F32 or TM_BF16");
        c->ptc_arith = prec;
        return TM_OK;
    });
}

extern "C" int tm_ptc_get_weights(tm_ctx *c, int nc, double *W1, double *W2)
{
    return guard(c, [&]() {
        TM_REQUIRE(W1 && W2, "null pointer");
        TM_REQUIRE(c->ptc_nc > 0, "no network weights set");
        TM_REQUIRE(nc == c->ptc_nc, "nc differs from the stored weights");
        download(c, W1, wbuf(c, "ptc_W1"), wbytes(nc), nullptr);
        download(c, W2, wbuf(c, "ptc_W2"), wbytes(nc), nullptr);
        return TM_OK;
    });
}

extern "C" int tm_ptc_init_hopping(tm_ctx *c, int nc, int mu_sign, uint64_t seed, double noise)
{
    return guard(c, [&]() {
        TM_REQUIRE(nc >= 9 && nc <= kMaxNc, "nc must be in [9, 64]");
        TM_REQUIRE(mu_sign == 1 || mu_sign == -1, "mu_sign must be +1 or -1");
        TM_REQUIRE(noise >= 0 && std::isfinite(noise), "noise must be >= 0");
        // spin matrices: B = R^-1 (diagonal), P_k = -kappa (1 -+ gamma_mu) of the
        // hop of path k (forward: 1 - gamma, backward: 1 + gamma)
        const double epsp = eps_of(c, mu_sign), den = 1.0 + epsp * epsp;
        using M4 = cx<double>[4][4];
        M4 B{};
        for (int a = 0; a < 4; a++) B[a][a] = {1.0 / den, (a < 2 ? -epsp : epsp) / den};
        auto mul = [](const M4 &X, const M4 &Y, M4 &Z) {
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cx<double> s{0, 0};
                    for (int e = 0; e < 4; e++) s = s + X[a][e] * Y[e][b];
                    Z[a][b] = s;
                }
        };
        M4 P[9]{}, BPB[9]{};
        for (int k = 1; k < 9; k++) {
            const int mu = (k - 1) & 3;
            const double sg = k <= 4 ? -1.0 : 1.0;
            cx<double> G[4][4];
            gamma_n(1 << mu, G);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++)
                    P[k][a][b] = cx<double>{-c->kappa * ((a == b ? 1.0 : 0.0) + sg * G[a][b].r),
                                            -c->kappa * sg * G[a][b].i};
            M4 t;
            mul(B, P[k], t);
            mul(t, B, BPB[k]);
        }
        // A[0][0] = B, A[0][k'] = -B P_k' B, A[k][k'] = B P_k B P_k' B (k, k' >= 1);
        // channel c < 9 carries column k' = c: W1[k'][c] = delta_{k' c} 1, W2[k][c] = A[k][c]
        std::vector<cx<double>> W1((size_t)9 * nc * 16, cx<double>{0, 0}), W2(W1.size(), cx<double>{0, 0});
        uint64_t st = seed;
        for (int kp = 0; kp < 9; kp++)
            for (int ch = 0; ch < nc; ch++)
                for (int el = 0; el < 16; el++) {
                    cx<double> &w = W1[((size_t)kp * nc + ch) * 16 + el];
                    if (ch < 9) {
                        if (ch == kp && el % 5 == 0) w = {1.0, 0.0};
                    } else {
                        const double u1 = (splitmix(st) >> 11) * 0x1.0p-53, u2 = (splitmix(st) >> 11) * 0x1.0p-53;
                        w = {noise * (2 * u1 - 1), noise * (2 * u2 - 1)};
                    }
                }
        for (int k = 0; k < 9; k++)
            for (int ch = 0; ch < 9; ch++) {
                M4 Akk{};
                if (k == 0 && ch == 0) {
                    memcpy(Akk, B, sizeof(M4));
                } else if (k == 0) {
                    for (int a = 0; a < 4; a++)
                        for (int b = 0; b < 4; b++) Akk[a][b] = cx<double>{-BPB[ch][a][b].r, -BPB[ch][a][b].i};
                } else if (ch >= 1) {
                    M4 t;
                    mul(BPB[k], P[ch], t);
                    mul(t, B, Akk);
                }
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) W2[((size_t)k * nc + ch) * 16 + 4 * a + b] = Akk[a][b];
            }
        return tm_ptc_set_weights(c, nc, (const double *)W1.data(), (const double *)W2.data());
    });
}

extern "C" int tm_ptc_apply(tm_ctx *c, double *out, const double *in, int nrhs, tm_stream stream)
{
    return guard(c, [&]() {
        TM_REQUIRE(out && in && out != in, "bad pointer");
        TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        TM_REQUIRE(c->ptc_nc > 0, "no network weights set");
        hipStream_t s = hs(stream);
        const size_t hb = field_bytes(c, TM_F32, nrhs);
        void *ie = ws_get(c, "pa_ie", hb), *io = ws_get(c, "pa_io", hb);
        void *oe = ws_get(c, "pa_oe", hb), *oo = ws_get(c, "pa_oo", hb);
        launch_pack(c, ie, io, in, nrhs, TM_F32, nullptr, s);
        forward(c, TM_F32, ie, io, (float2 *)oe, (float2 *)oo, nrhs, s);
        launch_unpack(c, out, oe, oo, nrhs, TM_F32, s);
        return TM_OK;
    });
}

extern "C" int tm_ptc_loss_grad(tm_ctx *c, int loss_kind_, int mu_sign, const double *r, const double *e,
                                int npairs, double *loss, double *G1, double *G2, tm_stream stream)
{
    return guard(c, [&]() {
        const LossKind kind = loss_kind(loss_kind_);
        TM_REQUIRE(r && loss && (e || kind == LossKind::residual), "null pointer");
        TM_REQUIRE(npairs >= 1, "npairs must be >= 1");
        TM_REQUIRE(mu_sign == 1 || mu_sign == -1, "mu_sign must be +1 or -1");
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        TM_REQUIRE(c->ptc_nc > 0, "no network weights set");
        hipStream_t s = hs(stream);
        const size_t hb = field_bytes(c, TM_F32, npairs);
        void *re = ws_get(c, "pl_re", hb), *ro = ws_get(c, "pl_ro", hb);
        void *ee = nullptr, *eo = nullptr;
        launch_pack(c, re, ro, r, npairs, TM_F32, nullptr, s);
        if (kind == LossKind::error) {
            ee = ws_get(c, "pl_ee", hb);
            eo = ws_get(c, "pl_eo", hb);
            launch_pack(c, ee, eo, e, npairs, TM_F32, nullptr, s);
        }
        // |e|^2 (error loss) or |r|^2 (residual loss) of the FP32 fields the loss uses
        const void *ne = kind == LossKind::error ? ee : re, *no = kind == LossKind::error ? eo : ro;
        double *en2 = (double *)ws_get(c, "pl_en2", sizeof(double) * npairs);
        std::vector<double> a = norms_host(c, ne, TM_F32, npairs, s), b = norms_host(c, no, TM_F32, npairs, s);
        for (int k = 0; k < npairs; k++) {
            a[k] += b[k];
            TM_REQUIRE(a[k] > 0, "zero field in a pair");
        }
        upload(en2, a.data(), sizeof(double) * npairs, s);
        double *dl = (double *)ws_get(c, "pl_loss", sizeof(double));
        loss_grad(c, kind, eps_of(c, mu_sign), TM_F32, re, ro, ee, eo, en2, npairs, dl, s);
        run_update(c, 0, AdamArgs{}, s);
        download(c, loss, dl, sizeof(double), s);
        const int nc = c->ptc_nc;
        if (G1) download(c, G1, wbuf(c, "ptc_G1"), wbytes(nc), s);
        if (G2) download(c, G2, wbuf(c, "ptc_G2"), wbytes(nc), s);
        return TM_OK;
    });
}

extern "C" int tm_ptc_pairs_reserve(tm_ctx *c, int capacity, int store_prec)
{
    return guard(c, [&]() {
        TM_REQUIRE(capacity >= 1, "capacity must be >= 1");
        TM_REQUIRE(store_prec == TM_F32 || store_prec == TM_BF16, "store precision must be TM_F32 or TM_BF16");
        c->ptc_store = store_prec;
        c->ptc_cap = capacity;
        c->ptc_n = 0;
        const size_t one = store_half_bytes(c);
        ws_get(c, "ptc_pairs_r", 2 * one * capacity);
        ws_get(c, "ptc_pairs_e", 2 * one * capacity);
        ws_get(c, "ptc_pairs_en2", sizeof(double) * capacity);
        ws_get(c, "ptc_pairs_rn2", sizeof(double) * capacity);
        return TM_OK;
    });
}

namespace {

// append n pairs given as FP64 half fields (r_e, r_o, e_e, e_o; [n][12][hs]
// each) to the store, converted to its precision; pairs with r = 0 or
// e = 0 in the stored precision are dropped when skip_zero, else an error.
// Returns the number appended.
int store_pairs(tm_ctx *c, const void *r_e, const void *r_o, const void *e_e, const void *e_o, int n, bool skip_zero,
                hipStream_t s)
{
    const size_t one = store_half_bytes(c), cap = (size_t)c->ptc_cap;
    const size_t in1 = field_bytes(c, TM_F64, 1);
    char *R = (char *)ws_get(c, "ptc_pairs_r", 2 * one * cap), *E = (char *)ws_get(c, "ptc_pairs_e", 2 * one * cap);
    double *en2 = (double *)ws_get(c, "ptc_pairs_en2", sizeof(double) * cap);
    double *rn2 = (double *)ws_get(c, "ptc_pairs_rn2", sizeof(double) * cap);
    int added = 0;
    for (int k = 0; k < n; k++) {
        TM_REQUIRE(c->ptc_n + 1 <= c->ptc_cap, "pair store capacity exceeded");
        const size_t at = one * c->ptc_n;
        launch_copy_convert(c, R + at, c->ptc_store, (const char *)r_e + k * in1, TM_F64, 1, nullptr, s);
        launch_copy_convert(c, R + one * cap + at, c->ptc_store, (const char *)r_o + k * in1, TM_F64, 1, nullptr, s);
        launch_copy_convert(c, E + at, c->ptc_store, (const char *)e_e + k * in1, TM_F64, 1, nullptr, s);
        launch_copy_convert(c, E + one * cap + at, c->ptc_store, (const char *)e_o + k * in1, TM_F64, 1, nullptr, s);
        const double ne = norms_host(c, E + at, c->ptc_store, 1, s)[0] +
                          norms_host(c, E + one * cap + at, c->ptc_store, 1, s)[0];
        const double nr = norms_host(c, R + at, c->ptc_store, 1, s)[0] +
                          norms_host(c, R + one * cap + at, c->ptc_store, 1, s)[0];
        const bool ok = ne > 0 && nr > 0 && std::isfinite(ne) && std::isfinite(nr);
        if (!ok) {
            TM_REQUIRE(skip_zero, "r = 0, e = 0 or non-finite in a pair");
            continue;
        }
        upload(en2 + c->ptc_n, &ne, sizeof(double), s);
        upload(rn2 + c->ptc_n, &nr, sizeof(double), s);
        c->ptc_n++;
        added++;
    }
    return added;
}

}  // namespace

extern "C" int tm_ptc_pairs_add(tm_ctx *c, const double *r, const double *e, int n, tm_stream stream)
{
    return guard(c, [&]() {
        TM_REQUIRE(r && e, "null pointer");
        TM_REQUIRE(n >= 1, "n must be >= 1");
        TM_REQUIRE(c->ptc_cap > 0, "no pair store reserved");
        TM_REQUIRE(c->ptc_n + n <= c->ptc_cap, "pair store capacity exceeded");
        hipStream_t s = hs(stream);
        const size_t hb = field_bytes(c, TM_F64, n);
        void *re = ws_get(c, "pp_re", hb), *ro = ws_get(c, "pp_ro", hb);
        void *ee = ws_get(c, "pp_ee", hb), *eo = ws_get(c, "pp_eo", hb);
        launch_pack(c, re, ro, r, n, TM_F64, nullptr, s);
        launch_pack(c, ee, eo, e, n, TM_F64, nullptr, s);
        store_pairs(c, re, ro, ee, eo, n, false, s);
        return TM_OK;
    });
}

extern "C" int tm_ptc_pairs_from_solve(tm_ctx *c, const double *b, int nrhs, const tm_solve_params *p,
                                       const int *iters, int n_iters, int *added, tm_stream stream)
{
    return guard(c, [&]() {
        TM_REQUIRE(b && p && iters, "null pointer");
        TM_REQUIRE(nrhs >= 1 && n_iters >= 1, "nrhs and n_iters must be >= 1");
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        TM_REQUIRE(c->ptc_cap > 0, "no pair store reserved");
        for (int j = 0; j < n_iters; j++) TM_REQUIRE(iters[j] >= 1, "iteration counts must be >= 1");
        TM_REQUIRE(p->solver == TM_CG_F64 || p->solver == TM_CG_MIXED, "pairs come from TM_CG_F64 or TM_CG_MIXED");
        hipStream_t s = hs(stream);
        const size_t hb = field_bytes(c, TM_F64, nrhs);
        void *be = ws_get(c, "pp_be", hb), *bo = ws_get(c, "pp_bo", hb);
        void *se = ws_get(c, "pp_se", hb), *so = ws_get(c, "pp_so", hb);
        void *xe = ws_get(c, "pp_xe", hb), *xo = ws_get(c, "pp_xo", hb);
        void *re = ws_get(c, "pp_re", hb), *ro = ws_get(c, "pp_ro", hb);
        launch_pack(c, be, bo, b, nrhs, TM_F64, nullptr, s);
        // x* to the solver's tolerance
        SolveOut full = solve_halves(c, se, so, be, bo, nrhs, *p, s);
        TM_REQUIRE(full.status == TM_OK, "the reference solve did not converge");
        const double epsp = eps_of(c, p->mu_sign), k = c->kappa;
        int n_add = 0;
        for (int j = 0; j < n_iters; j++) {
            tm_solve_params pk = *p;
            pk.maxiter = iters[j];
            SolveOut it = solve_halves(c, xe, xo, be, bo, nrhs, pk, s);
            TM_REQUIRE(it.status == TM_OK || it.status == TM_ERR_NOCONV, "NaN/Inf in an iterate");
            // r = b - M x with all 18 link parameters; e = x* - x (in place in x)
            for (int par = 0; par < 2; par++)
                op_dslash(c, par ? ro : re, par ? xe : xo, par ? xo : xe, nrhs, TM_F64, par, 0, sd_scalar(-k),
                          sd_twist(epsp), s, true);
            launch_axpby_host(c, re, be, TM_F64, nrhs, 1.0, -1.0, s);
            launch_axpby_host(c, ro, bo, TM_F64, nrhs, 1.0, -1.0, s);
            launch_axpby_host(c, xe, se, TM_F64, nrhs, 1.0, -1.0, s);
            launch_axpby_host(c, xo, so, TM_F64, nrhs, 1.0, -1.0, s);
            n_add += store_pairs(c, re, ro, xe, xo, nrhs, true, s);
        }
        if (added) *added = n_add;
        return TM_OK;
    });
}

extern "C" int tm_ptc_train(tm_ctx *c, const tm_ptc_train_params *p, tm_ptc_train_stats *stats, double *loss_per_step,
                            tm_stream stream)
{
    return guard(c, [&]() {
        TM_REQUIRE(p, "null pointer");
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        TM_REQUIRE(c->ptc_nc > 0, "no network weights set");
        TM_REQUIRE(p->epochs >= 1, "epochs must be >= 1");
        TM_REQUIRE(p->batch >= 1 && p->batch <= c->ptc_n, "batch must be in [1, stored pairs]");
        TM_REQUIRE(p->lr > 0 && p->beta1 >= 0 && p->beta1 < 1 && p->beta2 >= 0 && p->beta2 < 1 && p->adam_eps > 0,
                   "bad Adam parameters");
        const LossKind kind = loss_kind(p->loss);
        TM_REQUIRE(p->mu_sign == 1 || p->mu_sign == -1, "mu_sign must be +1 or -1");
        hipStream_t s = hs(stream);
        const double t0 = now_s();
        const int nb = c->ptc_n / p->batch, steps = nb * p->epochs;
        const size_t one = store_half_bytes(c), cap = (size_t)c->ptc_cap;
        const char *R = (const char *)ws_get(c, "ptc_pairs_r", 2 * one * cap);
        const char *E = (const char *)ws_get(c, "ptc_pairs_e", 2 * one * cap);
        const double *en2 = (const double *)ws_get(
            c, kind == LossKind::error ? "ptc_pairs_en2" : "ptc_pairs_rn2", sizeof(double) * cap);
        double *hist = (double *)ws_get(c, "ptc_hist", sizeof(double) * steps);
        std::vector<int> order(nb);
        uint64_t st = p->seed;
        int step = 0;
        for (int ep = 0; ep < p->epochs; ep++) {
            for (int k = 0; k < nb; k++) order[k] = k;
            for (int k = nb - 1; k > 0; k--) std::swap(order[k], order[splitmix(st) % (uint64_t)(k + 1)]);
            for (int k = 0; k < nb; k++, step++) {
                const size_t b0 = (size_t)order[k] * p->batch;
                loss_grad(c, kind, eps_of(c, p->mu_sign), c->ptc_store, R + one * b0, R + one * (cap + b0),
                          E + one * b0, E + one * (cap + b0), en2 + b0, p->batch, hist + step, s);
                AdamArgs ad{p->lr, p->beta1, p->beta2, p->adam_eps, ++c->ptc_step};
                run_update(c, 1, ad, s);
            }
        }
        std::vector<double> h(steps);
        download(c, h.data(), hist, sizeof(double) * steps, s);
        for (double v : h) TM_REQUIRE(std::isfinite(v), "non-finite training loss");
        if (loss_per_step) memcpy(loss_per_step, h.data(), sizeof(double) * steps);
        if (stats) {
            *stats = tm_ptc_train_stats{};
            stats->steps = steps;
            double f = 0, l = 0;
            for (int k = 0; k < nb; k++) f += h[k];
            for (int k = steps - nb; k < steps; k++) l += h[k];
            stats->loss_first = f / nb;
            stats->loss_last = l / nb;
            stats->seconds = now_s() - t0;
        }
        return TM_OK;
    });
}
