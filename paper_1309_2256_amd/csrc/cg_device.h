// Device parts of the CG scalar updates and the search-direction update,
// shared by the stand-alone kernels (blas.hip) and the persistent batch
// kernel (dslash.hip) so that both perform the same operations in the same
// order: a right-hand side solved in a batch follows its single solve bit
// for bit.  Every function here is called by all threads of a 256-thread
// block (the sums use the block's LDS and barriers).
//
// The block partial sums and the CG scalars are small arrays that blocks on
// different XCDs write within one launch of the persistent kernel (several
// writers share a cache line).  They are read and written with device-scope
// atomic loads and stores, which do not depend on the state of a
// non-coherent L2 copy of the line; the data fields themselves are never
// shared between writers at line granularity.
#pragma once

#include "tm_internal.h"

namespace cgdev {

constexpr int kThreads = 256;

template <typename V>
__device__ __forceinline__ V ld_coh(const V *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ void st_coh(V *p, V v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// sum over the block; result valid in thread 0
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[kThreads / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kThreads / 64; k++) s += red[k];
    }
    __syncthreads();
    return s;
}

// sum_b part[idx * nblk + b]: thread-strided partial sums, then the block
// tree; result valid in thread 0
__device__ __forceinline__ double sum_partials(const double *part, int nblk, int idx)
{
    double acc = 0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) acc += ld_coh(part + (size_t)idx * nblk + b);
    return block_sum(acc);
}

__device__ __forceinline__ bool finite(double v) { return v == v && v - v == 0; }

// alpha = |r|^2 / |q|^2 of right-hand side r; part layout [rhs][nblk]
__device__ __forceinline__ void finish_alpha(CGScalars *sc, const double *part, int nblk, int r)
{
    const double qq = sum_partials(part, nblk, r);
    if (threadIdx.x == 0) {
        CGScalars &s = sc[r];
        const double rr = ld_coh(&s.rr);
        const int active = ld_coh(&s.active);
        st_coh(&s.qq, qq);
        if (!finite(qq) || !finite(rr)) st_coh(&s.bad, 1);
        st_coh(&s.alpha, (active && qq > 0 && finite(qq)) ? rr / qq : 0.0);
    }
}

// beta, the new |r|^2 and |rho|^2 and the convergence / reliable-update
// flags of right-hand side r.  part layout: [slot 0: |r|^2 for all rhs]
// [slot 1: |rho|^2 for all rhs].  With reliable updates (delta > 0) slot 1
// is not used: the Schur residual rho -= alpha q has
// |rho'|^2 = |rho|^2 - 2 alpha <r, p> + alpha^2 |q|^2 = |rho|^2 - alpha |r|^2
// (CG: <r, p> = |r|^2, alpha = |r|^2 / |q|^2), a recurrence whose rounding
// stays far below the delta^2 |rho_ref|^2 it is compared with between two
// updates (each update resets it to the FP64 true residual).
__device__ __forceinline__ void finish_beta(CGScalars *sc, const double *part, int nblk, int nrhs, double delta,
                                            int r)
{
    const double rr = sum_partials(part, nblk, r);
    double rho2 = delta > 0 ? 0.0 : sum_partials(part, nblk, nrhs + r);
    if (threadIdx.x == 0) {
        CGScalars &s = sc[r];
        const int active = ld_coh(&s.active);
        const double rr_old = ld_coh(&s.rr), rho2_old = ld_coh(&s.rho2), target2 = ld_coh(&s.target2);
        if (delta > 0) rho2 = active ? fmax(rho2_old - ld_coh(&s.alpha) * rr_old, 0.0) : rho2_old;
        if (!finite(rr) || !finite(rho2)) st_coh(&s.bad, 1);
        if (active) {
            st_coh(&s.beta, (rr_old > 0) ? rr / rr_old : 0.0);
            st_coh(&s.rr, rr);
            st_coh(&s.rho2, rho2);
            st_coh(&s.iters, ld_coh(&s.iters) + 1);
            if (delta > 0) {
                // reliable-update solver: converged estimate or residual fallen
                // by delta since the last update -> request an update
                if (rho2 <= target2 || rho2 < delta * delta * ld_coh(&s.rho2_ref)) st_coh(&s.want_update, 1);
            } else if (rho2 <= target2) {
                st_coh(&s.active, 0);
            }
        } else {
            st_coh(&s.beta, 0.0);
        }
    }
}

// x += alpha p; p = r + beta p for elements [e0, e1) of right-hand side r
// (n complex per right-hand side), with the element stride `step` between a
// thread's elements (the solution update of this iteration folded into the
// search-direction update; both use the p that produced q).  Elementwise:
// any split of the range gives the same result.
template <typename S, typename XS>
__device__ __forceinline__ void update_px(S *p, const S *rv, XS *x, size_t n, const CGScalars *sc, int r,
                                          size_t e0, size_t e1, size_t step)
{
    using T = typename StoreTraits<S>::real;
    using TX = typename StoreTraits<XS>::real;
    const int active = ld_coh(&sc[r].active);
    const double alpha = ld_coh(&sc[r].alpha);
    if (!active && alpha == 0.0) return;
    const T b = active ? (T)ld_coh(&sc[r].beta) : (T)0;
    const TX ax = (TX)alpha;
    const bool upd_p = active != 0;
    const size_t base = (size_t)r * n;
    for (size_t e = e0; e < e1; e += step) {
        const size_t k = base + e;
        cx<T> pv = ldT<T>(p, k);
        cx<TX> xv = ldT<TX>(x, k);
        stT<TX>(x, k, xv + ax * cx<TX>{(TX)pv.r, (TX)pv.i});
        if (upd_p) stT<T>(p, k, ldT<T>(rv, k) + b * pv);
    }
}

}  // namespace cgdev
