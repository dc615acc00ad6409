// Vector kernels of the solvers: spin-diagonal scaling, precision conversion,
// axpy forms and per-right-hand-side norms.  Reductions are deterministic:
// each block writes one FP64 partial per right-hand side (fixed grid, fixed
// wave-then-LDS tree) and a single block per right-hand side sums the
// partials in a fixed order.  Products are formed in the arithmetic precision
// and accumulated in FP64.
#include "cg_device.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxPart = 1024;

using cgdev::block_sum;
using cgdev::sum_partials;
static_assert(kBlock == cgdev::kThreads, "block sums assume 256 threads");

template <typename S>
__global__ __launch_bounds__(kBlock) void k_spin_diag(S *out, const S *in, int hs, cx<float> fu,
                                                      cx<float> fl, cx<double> du, cx<double> dl)
{
    using T = typename StoreTraits<S>::real;
    const size_t n = (size_t)12 * hs;
    const size_t base = (size_t)blockIdx.y * n;
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        const int k = (int)(e / hs);
        cx<T> f;
        if (sizeof(T) == 8) {
            cx<double> d = k < 6 ? du : dl;
            f = {(T)d.r, (T)d.i};
        } else {
            cx<float> d = k < 6 ? fu : fl;
            f = {(T)d.r, (T)d.i};
        }
        stT<T>(out, base + e, f * ldT<T>(in, base + e));
    }
}

template <typename SO, typename SI>
__global__ __launch_bounds__(kBlock) void k_convert(SO *out, const SI *in, size_t n, const double *scale)
{
    const size_t base = (size_t)blockIdx.y * n;
    const double sc = scale ? scale[blockIdx.y] : 1.0;
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        cx<double> v = ldT<double>(in, base + e);
        stT<double>(out, base + e, sc * v);
    }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_axpby(S *y, const S *x, size_t n, double a, double b)
{
    using T = typename StoreTraits<S>::real;
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        cx<T> xv = ldT<T>(x, e), yv = ldT<T>(y, e);
        stT<T>(y, e, (T)a * xv + (T)b * yv);
    }
}

// out = a x + b y with a separate output (the same arithmetic as k_axpby)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_axpby_to(S *out, const S *x, const S *y, size_t n, double a, double b)
{
    using T = typename StoreTraits<S>::real;
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        cx<T> xv = ldT<T>(x, e), yv = ldT<T>(y, e);
        stT<T>(out, e, (T)a * xv + (T)b * yv);
    }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_zero(S *y, size_t n)
{
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock)
        stT<double>(y, e, cx<double>{0.0, 0.0});
}

// y[r] += a[r] * x[r] with per-rhs device scalars (x may be a lower precision)
template <typename SY, typename SX>
__global__ __launch_bounds__(kBlock) void k_axpy_dev(SY *y, const SX *x, size_t n, const double *a)
{
    using T = typename StoreTraits<SY>::real;
    const size_t base = (size_t)blockIdx.y * n;
    const T av = (T)a[blockIdx.y];
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
        const size_t k = base + e;
        stT<T>(y, k, ldT<T>(y, k) + av * ldT<T>(x, k));
    }
}

// partial |v|^2 of right-hand side blockIdx.y over the vh valid sites of
// each of its 12 planes (the pad sites of a plane are skipped)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_partial_norm2(const S *v, int vh, int hs, double *part, int nblk)
{
    using T = typename StoreTraits<S>::real;
    const size_t base = (size_t)blockIdx.y * 12 * hs;
    double acc = 0;
    for (int k = 0; k < 12; k++)
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < vh; i += gridDim.x * kBlock) {
            cx<T> a = ldT<T>(v, base + (size_t)k * hs + i);
            acc += (double)(a.r * a.r + a.i * a.i);
        }
    double s = block_sum(acc);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * nblk + blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_finish_sum(const double *part, int nblk, double *out)
{
    double s = sum_partials(part, nblk, blockIdx.x);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// part layout: [rhs][nblk] (one slot)
__global__ __launch_bounds__(kBlock) void k_finish_alpha(CGScalars *sc, const double *part, int nblk)
{
    cgdev::finish_alpha(sc, part, nblk, blockIdx.x);
}

// part layout: [slot 0: |r|^2 for all rhs][slot 1: |rho|^2 for all rhs]
__global__ __launch_bounds__(kBlock) void k_finish_beta(CGScalars *sc, const double *part, int nblk,
                                                        int nrhs, double delta)
{
    cgdev::finish_beta(sc, part, nblk, nrhs, delta, blockIdx.x);
}

// x += alpha p; p = r + beta p  (the solution update of this iteration folded
// into the search-direction update; both use the p that produced q)
template <typename S, typename XS>
__global__ __launch_bounds__(kBlock) void k_update_px(S *p, const S *rv, XS *x, size_t n, const CGScalars *sc)
{
    cgdev::update_px(p, rv, x, n, sc, blockIdx.y, (size_t)blockIdx.x * kBlock + threadIdx.x, n,
                     (size_t)gridDim.x * kBlock);
}

// Several lattices per launch (a batch iteration).  Scalar kernels: block b
// is right-hand side b - rstart[i] of lattice i.  Update: lattice i owns
// blocks [ustart[i], ustart[i+1]) laid out as its single launch's
// (gx[i] x nrhs) grid, so every element sees the same thread-stride loop.
constexpr int kTailInst = 8;
template <typename S, typename XS>
struct TailArgs {
    CGScalars *sc[kTailInst];
    const double *part[kTailInst];
    S *p[kTailInst];
    const S *r[kTailInst];
    XS *x[kTailInst];
    size_t n[kTailInst];
    double delta[kTailInst];
    int nblk[kTailInst], nrhs[kTailInst], gx[kTailInst];
    int rstart[kTailInst + 1], ustart[kTailInst + 1];
    int ninst;
};
static_assert(sizeof(TailArgs<double2, double2>) <= 4096, "kernel arguments exceed 4 KiB");

__device__ __forceinline__ int tail_inst(const int *start, int n, int b)
{
    int i = 0;
    while (i + 1 < n && b >= start[i + 1]) i++;
    return i;
}

template <typename S, typename XS>
__global__ __launch_bounds__(kBlock) void k_finish_alpha_multi(const TailArgs<S, XS> a)
{
    const int i = tail_inst(a.rstart, a.ninst, blockIdx.x);
    cgdev::finish_alpha(a.sc[i], a.part[i], a.nblk[i], blockIdx.x - a.rstart[i]);
}

template <typename S, typename XS>
__global__ __launch_bounds__(kBlock) void k_finish_beta_multi(const TailArgs<S, XS> a)
{
    const int i = tail_inst(a.rstart, a.ninst, blockIdx.x);
    cgdev::finish_beta(a.sc[i], a.part[i], a.nblk[i], a.nrhs[i], a.delta[i], blockIdx.x - a.rstart[i]);
}

template <typename S, typename XS>
__global__ __launch_bounds__(kBlock) void k_update_px_multi(const TailArgs<S, XS> a)
{
    const int i = tail_inst(a.ustart, a.ninst, blockIdx.x);
    const int local = blockIdx.x - a.ustart[i], gx = a.gx[i];
    const int r = local / gx, bx = local - r * gx;
    cgdev::update_px(a.p[i], a.r[i], a.x[i], a.n[i], a.sc[i], r, (size_t)bx * kBlock + threadIdx.x, a.n[i],
                     (size_t)gx * kBlock);
}

// complex elements of one right-hand side of a half field, pads included
size_t half_elems(tm_ctx *c) { return (size_t)12 * c->geo.hs; }

int grid_for(size_t n)
{
    size_t g = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
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

void launch_spin_diag(tm_ctx *c, void *out, const void *in, int prec, int nrhs, SpinDiag d, hipStream_t s)
{
    size_t n = half_elems(c);
    dim3 grid(grid_for(n), nrhs);
    cx<float> fu{(float)d.u.r, (float)d.u.i}, fl{(float)d.l.r, (float)d.l.i};
    account(c, 2.0 * n * nrhs * prec_bytes(prec), 6.0 * n * nrhs);
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_spin_diag<S>, grid, dim3(kBlock), 0, s, (S *)out, (const S *)in, c->geo.hs, fu,
                           fl, d.u, d.l);
    });
    TM_HIP(hipGetLastError());
}

void launch_copy_convert(tm_ctx *c, void *out, int out_prec, const void *in, int in_prec, int nrhs,
                         const double *dscale, hipStream_t s)
{
    size_t n = half_elems(c);
    dim3 grid(grid_for(n), nrhs);
    account(c, (double)n * nrhs * (prec_bytes(in_prec) + prec_bytes(out_prec)), dscale ? 2.0 * n * nrhs : 0.0);
    dispatch_prec(out_prec, [&](auto *to) {
        using SO = std::remove_pointer_t<decltype(to)>;
        dispatch_prec(in_prec, [&](auto *ti) {
            using SI = std::remove_pointer_t<decltype(ti)>;
            hipLaunchKernelGGL((k_convert<SO, SI>), grid, dim3(kBlock), 0, s, (SO *)out, (const SI *)in, n,
                               dscale);
        });
    });
    TM_HIP(hipGetLastError());
}

void launch_axpby_host(tm_ctx *c, void *y, const void *x, int prec, int nrhs, double a, double b,
                       hipStream_t s)
{
    size_t n = half_elems(c) * nrhs;
    account(c, 3.0 * n * prec_bytes(prec), 6.0 * n);
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_axpby<S>, dim3(grid_for(n)), dim3(kBlock), 0, s, (S *)y, (const S *)x, n, a, b);
    });
    TM_HIP(hipGetLastError());
}

void launch_axpby_to_host(tm_ctx *c, void *out, const void *x, const void *y, int prec, int nrhs, double a,
                          double b, hipStream_t s)
{
    size_t n = half_elems(c) * nrhs;
    account(c, 3.0 * n * prec_bytes(prec), 6.0 * n);
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_axpby_to<S>, dim3(grid_for(n)), dim3(kBlock), 0, s, (S *)out, (const S *)x,
                           (const S *)y, n, a, b);
    });
    TM_HIP(hipGetLastError());
}

template <typename S, typename XS>
static TailArgs<S, XS> tail_args(const std::vector<CgTail> &t, size_t i0, size_t i1, bool beta)
{
    TailArgs<S, XS> a{};
    a.ninst = (int)(i1 - i0);
    a.rstart[0] = a.ustart[0] = 0;
    for (size_t k = i0; k < i1; k++) {
        const int j = (int)(k - i0);
        const CgTail &q = t[k];
        a.sc[j] = q.sc;
        a.part[j] = beta ? q.partb : q.partq;
        a.p[j] = (S *)q.p;
        a.r[j] = (const S *)q.r;
        a.x[j] = (XS *)q.x;
        a.n[j] = half_elems(q.c);
        a.delta[j] = q.delta;
        a.nblk[j] = q.nblk;
        a.nrhs[j] = q.nrhs;
        a.gx[j] = grid_for(a.n[j]);
        a.rstart[j + 1] = a.rstart[j] + q.nrhs;
        a.ustart[j + 1] = a.ustart[j] + a.gx[j] * q.nrhs;
    }
    return a;
}

template <typename F>
static void dispatch_tail(int prec, int xprec, F &&f)
{
    if (prec == TM_F64) {
        TM_REQUIRE(xprec == TM_F64, "FP64 CG needs an FP64 solution vector");
        f((double2 *)nullptr, (double2 *)nullptr);
        return;
    }
    TM_REQUIRE(xprec == TM_F32, "low-precision CG accumulates in FP32");
    dispatch_prec(prec, [&](auto *tag) { f(tag, (float2 *)nullptr); });
}

void cg_finish_alpha_multi(const std::vector<CgTail> &t, hipStream_t s)
{
    for (size_t i0 = 0; i0 < t.size(); i0 += kTailInst) {
        const size_t i1 = std::min(t.size(), i0 + kTailInst);
        const TailArgs<double2, double2> a = tail_args<double2, double2>(t, i0, i1, false);
        hipLaunchKernelGGL((k_finish_alpha_multi<double2, double2>), dim3(a.rstart[a.ninst]), dim3(kBlock), 0, s,
                           a);
        TM_HIP(hipGetLastError());
    }
}

void cg_tail_multi(const std::vector<CgTail> &t, int prec, int xprec, hipStream_t s)
{
    for (size_t i0 = 0; i0 < t.size(); i0 += kTailInst) {
        const size_t i1 = std::min(t.size(), i0 + kTailInst);
        dispatch_tail(prec, xprec, [&](auto *ts, auto *tx) {
            using S = std::remove_pointer_t<decltype(ts)>;
            using XS = std::remove_pointer_t<decltype(tx)>;
            const TailArgs<S, XS> a = tail_args<S, XS>(t, i0, i1, true);
            hipLaunchKernelGGL((k_finish_beta_multi<S, XS>), dim3(a.rstart[a.ninst]), dim3(kBlock), 0, s, a);
            TM_HIP(hipGetLastError());
            hipLaunchKernelGGL((k_update_px_multi<S, XS>), dim3(a.ustart[a.ninst]), dim3(kBlock), 0, s, a);
            TM_HIP(hipGetLastError());
        });
        for (size_t k = i0; k < i1; k++) {
            const size_t n = half_elems(t[k].c);
            account(t[k].c, (double)n * t[k].nrhs * (3 * prec_bytes(prec) + 2 * prec_bytes(xprec)),
                    8.0 * n * t[k].nrhs);
        }
    }
}

// partial-sum blocks of the vector norms (a few per CU, at most kMaxPart)
static int reduce_blocks(tm_ctx *c)
{
    // one site per thread: its 12 planes, 12 elements
    size_t n = c->geo.vh;
    size_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kMaxPart) g = kMaxPart;
    return (int)g;
}

static void partial_norm2(tm_ctx *c, const void *v, int prec, int nrhs, double *part, int nblk, hipStream_t s)
{
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_partial_norm2<S>, dim3(nblk, nrhs), dim3(kBlock), 0, s, (const S *)v, c->geo.vh,
                           c->geo.hs, part, nblk);
    });
    TM_HIP(hipGetLastError());
}

void launch_norm2(tm_ctx *c, const void *v, int prec, int nrhs, double *dev_out, hipStream_t s)
{
    int nblk = reduce_blocks(c);
    account(c, (double)half_elems(c) * nrhs * prec_bytes(prec), 4.0 * half_elems(c) * nrhs);
    double *part = (double *)ws_get(c, "norm_part", sizeof(double) * nblk * nrhs);
    partial_norm2(c, v, prec, nrhs, part, nblk, s);
    hipLaunchKernelGGL(k_finish_sum, dim3(nrhs), dim3(kBlock), 0, s, (const double *)part, nblk, dev_out);
    TM_HIP(hipGetLastError());
}

void cg_finish_alpha(tm_ctx *c, CGScalars *sc, const double *part, int nblk, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_alpha, dim3(nrhs), dim3(kBlock), 0, s, sc, part, nblk);
    TM_HIP(hipGetLastError());
}

void cg_finish_beta(tm_ctx *c, CGScalars *sc, const double *part, int nblk, int nrhs, double delta,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_beta, dim3(nrhs), dim3(kBlock), 0, s, sc, part, nblk, nrhs, delta);
    TM_HIP(hipGetLastError());
}

void launch_zero(tm_ctx *c, void *y, int prec, int nrhs, hipStream_t s)
{
    size_t n = half_elems(c) * nrhs;
    account(c, (double)n * prec_bytes(prec), 0.0);
    dispatch_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_zero<S>, dim3(grid_for(n)), dim3(kBlock), 0, s, (S *)y, n);
    });
    TM_HIP(hipGetLastError());
}

void launch_axpy_dev(tm_ctx *c, void *y, int yprec, const void *x, int xprec, int nrhs, const double *a_dev,
                     hipStream_t s)
{
    size_t n = half_elems(c);
    dim3 grid(grid_for(n), nrhs);
    account(c, (double)n * nrhs * (2 * prec_bytes(yprec) + prec_bytes(xprec)), 4.0 * n * nrhs);
    dispatch_prec(yprec, [&](auto *ty) {
        using SY = std::remove_pointer_t<decltype(ty)>;
        dispatch_prec(xprec, [&](auto *tx) {
            using SX = std::remove_pointer_t<decltype(tx)>;
            hipLaunchKernelGGL((k_axpy_dev<SY, SX>), grid, dim3(kBlock), 0, s, (SY *)y, (const SX *)x, n, a_dev);
        });
    });
    TM_HIP(hipGetLastError());
}

void cg_update_px(tm_ctx *c, void *p, const void *r, void *x, int prec, int xprec, int nrhs, const CGScalars *sc,
                  hipStream_t s)
{
    size_t n = half_elems(c);
    dim3 grid(grid_for(n), nrhs);
    // reads p, r, x; writes p, x; x += alpha p and p = r + beta p
    account(c, (double)n * nrhs * (3 * prec_bytes(prec) + 2 * prec_bytes(xprec)), 8.0 * n * nrhs);
    if (prec == TM_F64) {
        TM_REQUIRE(xprec == TM_F64, "FP64 CG needs an FP64 solution vector");
        hipLaunchKernelGGL((k_update_px<double2, double2>), grid, dim3(kBlock), 0, s, (double2 *)p,
                           (const double2 *)r, (double2 *)x, n, sc);
    } else {
        TM_REQUIRE(xprec == TM_F32, "low-precision CG accumulates in FP32");
        dispatch_prec(prec, [&](auto *tag) {
            using S = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((k_update_px<S, float2>), grid, dim3(kBlock), 0, s, (S *)p, (const S *)r,
                               (float2 *)x, n, sc);
        });
    }
    TM_HIP(hipGetLastError());
}
