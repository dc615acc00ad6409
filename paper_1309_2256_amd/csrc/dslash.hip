// Even-odd twisted-mass hopping kernel for gfx950.
//
// One thread per output half-site and R right-hand sides; each thread loads
// each of its 8 links once and reuses it for its R spinors.  Per direction the
// neighbour 4-spinor is projected to a 2-spinor with (1 -+ gamma_mu) (chiral
// basis, appendix A.1 operator), multiplied by the colour link, and
// reconstructed into the accumulator; the epilogue applies the spin-diagonal
// local terms (twist R = 1 + i eps gamma5, its inverse, gamma5, -kappa) so that
// the fused forms R^-1 H and R x - H y of the Schur operator (eq. A.2) cost no
// extra memory pass.
//
// Memory layout (all coalesced over the half-site index i):
//   spinors  [rhs][spin*3 + colour][vh]
//   links    [direction 0..7][row*3 + col][vh] for the output parity; the
//            backward links are stored conjugated and the antiperiodic
//            boundary phase is folded in, so the kernel has no branch on it.
#include "tm_internal.h"

namespace {

constexpr int kBlock = 256;
// resident waves per SIMD requested from the compiler (bounds the registers
// per lane to 512 / waves): one FP64 right-hand side needs ~180 registers,
// one or two FP32-arithmetic right-hand sides fit in 128
template <typename T, int R>
constexpr int waves_for() { return sizeof(T) == 8 ? 2 : 4; }

template <typename T>
struct DParams {
    void *out;
    const void *in;
    const void *own;
    const void *links;
    Geo g;
    int p;          // output parity
    int nrhs;
    cx<T> own_u, own_l, hop_u, hop_l, in_u, in_l;
    int has_own, has_in;
};

// (w0, w1) = i sigma_k (v0, v1) for k = 0, 1, 2 (sigma_1, sigma_2, sigma_3)
template <int K, typename T>
__device__ __forceinline__ void isigma(cx<T> v0, cx<T> v1, cx<T> &w0, cx<T> &w1)
{
    if (K == 0) {            // i sigma_1 = [[0, i], [i, 0]]
        w0 = times_i(v1);
        w1 = times_i(v0);
    } else if (K == 1) {     // i sigma_2 = [[0, 1], [-1, 0]]
        w0 = v1;
        w1 = cx<T>{-v0.r, -v0.i};
    } else {                 // i sigma_3 = [[i, 0], [0, -i]]
        w0 = times_i(v0);
        w1 = cx<T>{v1.i, -v1.r};
    }
}

// acc += (1 - S gamma_MU) (W (x) 1) psi  for S = +1 or -1, using the
// half-spinor form: h = P psi (2 spins), w = W h, lower spins rebuilt from w.
// Spatial gamma_k = [[0, -i s_k], [i s_k, 0]]:  h = u + S i s_k l,
//   lower = -S i s_k h.   gamma_4 = [[0, 1], [1, 0]]:  h = u - S l, lower = -S h.
template <int MU, int S, typename T>
__device__ __forceinline__ void hop_dir(cx<T> acc[12], const cx<T> W[9], const cx<T> psi[12])
{
    const T s = (T)S;
    cx<T> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (MU == 3) {
            h0[c] = psi[c] - s * psi[6 + c];
            h1[c] = psi[3 + c] - s * psi[9 + c];
        } else {
            cx<T> a, b;
            isigma<MU>(psi[6 + c], psi[9 + c], a, b);
            h0[c] = psi[c] + s * a;
            h1[c] = psi[3 + c] + s * b;
        }
    }
    cx<T> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        cx<T> a = {0, 0}, b = {0, 0};
#pragma unroll
        for (int c = 0; c < 3; c++) {
            cmac(a, W[3 * r + c], h0[c]);
            cmac(b, W[3 * r + c], h1[c]);
        }
        w0[r] = a;
        w1[r] = b;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc[c] = acc[c] + w0[c];
        acc[3 + c] = acc[3 + c] + w1[c];
        if (MU == 3) {
            acc[6 + c] = acc[6 + c] - s * w0[c];
            acc[9 + c] = acc[9 + c] - s * w1[c];
        } else {
            cx<T> a, b;
            isigma<MU>(w0[c], w1[c], a, b);
            acc[6 + c] = acc[6 + c] - s * a;
            acc[9 + c] = acc[9 + c] - s * b;
        }
    }
}

// ---------------------------------------------------------------- buffer I/O
// Raw buffer loads/stores: the 128-bit resource descriptor (base, byte range)
// lives in SGPRs, each lane supplies a 32-bit byte offset and the component
// stride is a scalar offset, so a neighbour costs one VGPR of address state.
using rsrc_t = __amdgpu_buffer_rsrc_t;
// the builtins' own (GCC-style) vector types; values are moved in and out by
// bit_cast to plain structs (element access on these vectors lowers to a
// single-dword load with this compiler)
typedef unsigned v2u __attribute__((__vector_size__(2 * sizeof(unsigned))));
typedef unsigned v4u __attribute__((__vector_size__(4 * sizeof(unsigned))));
// descriptor word 3 for raw (untyped) access on gfx9-class parts
constexpr int kRsrcFlags = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, size_t bytes)
{
    const unsigned n = bytes >= 0xffffffffull ? 0xffffffffu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, kRsrcFlags);
}

template <typename S>
struct BufIO;
struct F2 {
    float x, y;
};
struct D2 {
    double x, y;
};
template <>
struct BufIO<double2> {
    template <typename T>
    __device__ __forceinline__ static cx<T> ld(rsrc_t r, int voff, int soff)
    {
        D2 v = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        return {(T)v.x, (T)v.y};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        D2 v{(double)c.r, (double)c.i};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, v), r, voff, soff, 0);
    }
};
template <>
struct BufIO<float2> {
    template <typename T>
    __device__ __forceinline__ static cx<T> ld(rsrc_t r, int voff, int soff)
    {
        F2 v = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
        return {(T)v.x, (T)v.y};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        F2 v{(float)c.r, (float)c.i};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, 0);
    }
};
template <>
struct BufIO<h2> {
    template <typename T>
    __device__ __forceinline__ static cx<T> ld(rsrc_t r, int voff, int soff)
    {
        unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        h2 h = __builtin_bit_cast(h2, v);
        return {(T)(float)h.x, (T)(float)h.y};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        h2 h;
        h.x = (_Float16)(float)c.r;
        h.y = (_Float16)(float)c.i;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, h), r, voff, soff, 0);
    }
};
template <>
struct BufIO<b2> {
    template <typename T>
    __device__ __forceinline__ static cx<T> ld(rsrc_t r, int voff, int soff)
    {
        unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        return {(T)__builtin_bit_cast(float, v << 16), (T)__builtin_bit_cast(float, v & 0xffff0000u)};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        unsigned v = (unsigned)f32_to_bf16((float)c.r) | ((unsigned)f32_to_bf16((float)c.i) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, 0);
    }
};

template <typename LS, typename T>
__device__ __forceinline__ void load_link(cx<T> W[9], rsrc_t lr, int vbytes, int voff)
{
#pragma unroll
    for (int k = 0; k < 9; k++) W[k] = BufIO<LS>::template ld<T>(lr, voff, k * vbytes);
}

template <typename SS, typename T>
__device__ __forceinline__ void load_spinor(cx<T> psi[12], rsrc_t sr, int vbytes, int voff, const DParams<T> &a)
{
#pragma unroll
    for (int k = 0; k < 12; k++) psi[k] = BufIO<SS>::template ld<T>(sr, voff, k * vbytes);
    if (a.has_in) {
#pragma unroll
        for (int k = 0; k < 6; k++) psi[k] = a.in_u * psi[k];
#pragma unroll
        for (int k = 6; k < 12; k++) psi[k] = a.in_l * psi[k];
    }
}

template <int MU, int S, typename SS, typename LS, typename T, int R>
__device__ __forceinline__ void do_dir(cx<T> acc[R][12], const DParams<T> &a, const rsrc_t *sr, int dir, int j,
                                       int i)
{
    const LS *lbase = (const LS *)a.links + (size_t)dir * 9 * a.g.vh;
    const rsrc_t lr = make_rsrc(lbase, (size_t)9 * a.g.vh * sizeof(LS));
    cx<T> W[9];
    load_link<LS>(W, lr, a.g.vh * (int)sizeof(LS), i * (int)sizeof(LS));
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        cx<T> psi[12];
        load_spinor<SS>(psi, sr[rr], a.g.vh * (int)sizeof(SS), j * (int)sizeof(SS), a);
        hop_dir<MU, S>(acc[rr], W, psi);
    }
    // keep the loads of one direction from being hoisted above the previous
    // direction's arithmetic: bounds the live registers to one direction
    __builtin_amdgcn_sched_barrier(0);
}

template <typename SS, typename LS, typename T, int R, int DAG>
__global__ __launch_bounds__(kBlock, (waves_for<T, R>())) void k_dslash(DParams<T> a)
{
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int i = b * kBlock + threadIdx.x;
    if (i >= a.g.vh) return;
    const int r0 = blockIdx.y * R;
    const size_t fbytes = (size_t)12 * a.g.vh * sizeof(SS);  // one right-hand side
    rsrc_t sr[R];
#pragma unroll
    for (int rr = 0; rr < R; rr++) sr[rr] = make_rsrc((const char *)a.in + (r0 + rr) * fbytes, fbytes);

    int x, y, z, t;
    eo_coords(a.g, a.p, i, x, y, z, t);

    cx<T> acc[R][12];
#pragma unroll
    for (int rr = 0; rr < R; rr++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[rr][k] = {0, 0};

    // forward hops use (1 - gamma) for H and (1 + gamma) for H^dag
    constexpr int SF = DAG ? -1 : 1;
    constexpr int SB = -SF;
    // One direction per iteration; the loop is kept rolled so that the loads
    // of a direction are consumed before the next direction's are issued
    // (the switch is uniform across the wavefront).
#pragma unroll 1
    for (int d = 0; d < 8; d++) {
        const int mu = d & 3, step = d < 4 ? 1 : -1;
        int c[4] = {x, y, z, t};
        c[mu] += step;
        if (c[mu] == a.g.L[mu]) c[mu] = 0;
        if (c[mu] < 0) c[mu] = a.g.L[mu] - 1;
        const int j = eo_index(a.g, c[0], c[1], c[2], c[3]);
        switch (d) {
        case 0: do_dir<0, SF, SS, LS, T, R>(acc, a, sr, 0, j, i); break;
        case 1: do_dir<1, SF, SS, LS, T, R>(acc, a, sr, 1, j, i); break;
        case 2: do_dir<2, SF, SS, LS, T, R>(acc, a, sr, 2, j, i); break;
        case 3: do_dir<3, SF, SS, LS, T, R>(acc, a, sr, 3, j, i); break;
        case 4: do_dir<0, SB, SS, LS, T, R>(acc, a, sr, 4, j, i); break;
        case 5: do_dir<1, SB, SS, LS, T, R>(acc, a, sr, 5, j, i); break;
        case 6: do_dir<2, SB, SS, LS, T, R>(acc, a, sr, 6, j, i); break;
        default: do_dir<3, SB, SS, LS, T, R>(acc, a, sr, 7, j, i); break;
        }
    }

    const int vb = a.g.vh * (int)sizeof(SS), vo = i * (int)sizeof(SS);
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        const rsrc_t outr = make_rsrc((char *)a.out + (r0 + rr) * fbytes, fbytes);
        const rsrc_t ownr = make_rsrc((const char *)a.own + (r0 + rr) * fbytes, fbytes);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<T> v = (k < 6 ? a.hop_u : a.hop_l) * acc[rr][k];
            if (a.has_own) {
                cx<T> o = BufIO<SS>::template ld<T>(ownr, vo, k * vb);
                v = v + (k < 6 ? a.own_u : a.own_l) * o;
            }
            BufIO<SS>::template st<T>(outr, vo, k * vb, v);
        }
    }
}

template <typename T>
cx<T> cvt(cx<double> v)
{
    return cx<T>{(T)v.r, (T)v.i};
}

template <typename SS, typename LS, typename T, int R>
void launch_t(tm_ctx *c, const DslashCall &dc, hipStream_t s)
{
    DParams<T> a;
    a.out = dc.out;
    a.in = dc.in;
    a.own = dc.own;
    a.links = (std::is_same<LS, double2>::value ? c->links64 : c->links32)[dc.out_parity];
    a.g = c->geo;
    a.p = dc.out_parity;
    a.nrhs = dc.nrhs;
    a.own_u = cvt<T>(dc.d_own.u);
    a.own_l = cvt<T>(dc.d_own.l);
    a.hop_u = cvt<T>(dc.d_hop.u);
    a.hop_l = cvt<T>(dc.d_hop.l);
    a.in_u = cvt<T>(dc.d_in.u);
    a.in_l = cvt<T>(dc.d_in.l);
    a.has_own = dc.has_own ? 1 : 0;
    a.has_in = dc.has_in ? 1 : 0;
    dim3 grid((c->geo.vh + kBlock - 1) / kBlock, dc.nrhs / R);
    if (dc.dag)
        hipLaunchKernelGGL((k_dslash<SS, LS, T, R, 1>), grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_dslash<SS, LS, T, R, 0>), grid, dim3(kBlock), 0, s, a);
    TM_HIP(hipGetLastError());
}

template <typename SS, typename LS, typename T>
void launch_rhs(tm_ctx *c, const DslashCall &dc, hipStream_t s)
{
    // right-hand sides per thread: reuse each loaded link for two spinors
    const int n = dc.nrhs;
    if constexpr (std::is_same<T, double>::value) {
        launch_t<SS, LS, T, 1>(c, dc, s);
    } else {
        if (n % 2 == 0)
            launch_t<SS, LS, T, 2>(c, dc, s);
        else
            launch_t<SS, LS, T, 1>(c, dc, s);
    }
}

}  // namespace

void launch_dslash(tm_ctx *c, const DslashCall &dc, hipStream_t s)
{
    TM_REQUIRE(c->have_gauge, "no gauge field set");
    switch (dc.spinor_prec) {
    case TM_F64: launch_rhs<double2, double2, double>(c, dc, s); break;
    case TM_F32: ensure_links32(c, s); launch_rhs<float2, float2, float>(c, dc, s); break;
    case TM_F16: ensure_links32(c, s); launch_rhs<h2, float2, float>(c, dc, s); break;
    case TM_BF16: ensure_links32(c, s); launch_rhs<b2, float2, float>(c, dc, s); break;
    default: throw TmError{TM_ERR_ARG, "bad spinor precision"};
    }
}
