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
//   spinors  [rhs][spin*3 + colour][hs] (hs >= vh, the padded plane stride)
//   links    [direction 0..7][row*3 + col][vh] for the output parity; the
//            backward links are stored conjugated and the antiperiodic
//            boundary phase is folded in, so the kernel has no branch on it.
#include <cstdlib>
#include <cstring>

#include "cg_device.h"

namespace {

constexpr int kBlock = 256;
// resident waves per SIMD requested from the compiler (bounds the registers
// per lane to 512 / waves): one FP64 right-hand side fits in ~150 registers,
// two in 256; one or two FP32-arithmetic right-hand sides fit in 128
template <typename T, int R>
constexpr int waves_for() { return sizeof(T) == 8 ? (R == 1 ? 3 : 2) : (R <= 2 ? 4 : R == 3 ? 3 : 2); }

// 16-byte aligned so that an array of records keeps every complex field
// naturally aligned
template <typename T>
struct alignas(16) DParams {
    void *out;
    const void *in;
    const void *own;
    const void *links;
    Geo g;
    int p;          // output parity
    int nrhs;
    int ngroups;    // nrhs / R right-hand-side groups
    cx<T> own_u, own_l, hop_u, hop_l;
    // +1, passed at run time so that the +-1 factors of the spin projection
    // stay FMAs (which take the FP16 inputs directly) instead of being folded
    // into adds that need separate conversions
    T one;
    // fused epilogues: partial sums [quantity][rhs][site block]
    void *r;        // EPI_CG: normal residual, updated in place
    void *rho;      // EPI_CG: Schur residual, updated in place
    const CGScalars *sc;
    double *part;
    int nblk;       // site blocks
    int nb_t;       // site blocks per time slice (tiled traversal) or 0
    int t_bc;       // time-boundary factor (rebuilds the third row of 12-parameter links)
};

// Block -> (site block, right-hand-side group).  Hardware dispatches
// workgroup b to XCD b % 8.  Tiled traversal (when each time slice is a
// whole number of site blocks and of 8-block spatial chunks): XCD k owns the
// k-th eighth of every time slice and walks t slowest, so a site's t +- 1
// neighbours were loaded about eight site blocks earlier / later on the same
// XCD (its L2), z +- 1 two blocks away; the right-hand-side groups sharing a
// site block (and its links) are adjacent.  Otherwise: contiguous chunks of
// the natural order per XCD.
__device__ __forceinline__ int map_block(int b, int nblk_hw, int ngroups, int nb_t, int &grp)
{
    if (nb_t) {
        const int k = b & 7, m = b >> 3;
        grp = m % ngroups;
        const int m2 = m / ngroups, w = nb_t >> 3;
        const int t = m2 / w;
        return t * nb_t + k * w + (m2 - t * w);
    }
    const int lb = xcd_block(b, nblk_hw);
    grp = lb % ngroups;
    return lb / ngroups;
}

// A stored complex value as loaded: components in the storage type (FP16
// stays FP16 so that the projection below folds the conversion into a
// mixed-precision FMA), converted to T where they are combined.
template <typename L>
struct rawc {
    L r, i;
};

// h = u + S*l, h = u + S*i*l and h = u - S*i*l in arithmetic type T, each real
// part one FMA on the raw stored components
template <typename T, typename L>
__device__ __forceinline__ cx<T> p_add(rawc<L> u, rawc<L> l, T s)
{
    return {fma(s, (T)l.r, (T)u.r), fma(s, (T)l.i, (T)u.i)};
}
template <typename T, typename L>
__device__ __forceinline__ cx<T> p_addi(rawc<L> u, rawc<L> l, T s)
{
    return {fma(-s, (T)l.i, (T)u.r), fma(s, (T)l.r, (T)u.i)};
}

// acc += (1 - S gamma_MU) (W (x) 1) psi  for S = +1 or -1 in the half-spinor
// form: h = P psi (two spins), w = W h, the lower spins rebuilt from w.
// gamma_k = [[0, -i s_k], [i s_k, 0]]:  h = u + S (i s_k) l,  lower = -S (i s_k) w
// gamma_4 = [[0, 1], [1, 0]]:           h = u - S l,          lower = -S w
// with i s_1 = [[0, i], [i, 0]], i s_2 = [[0, 1], [-1, 0]], i s_3 = [[i, 0], [0, -i]].
// psi[3*spin + colour]; u = spins 0, 1 and l = spins 2, 3.
// acc += a * b for a link entry kept as stored binary16 (the conversion folds
// into mixed-precision FMAs) or already converted
template <typename T>
__device__ __forceinline__ void lmac(cx<T> &acc, cx<T> a, cx<T> b) { cmac(acc, a, b); }
template <typename T>
__device__ __forceinline__ void lmac(cx<T> &acc, rawc<_Float16> a, cx<T> b)
{
    acc.r = fma((T)a.r, b.r, acc.r);
    acc.r = fma(-(T)a.i, b.i, acc.r);
    acc.i = fma((T)a.r, b.i, acc.i);
    acc.i = fma((T)a.i, b.r, acc.i);
}

template <int MU, int S, typename T, typename L, typename WT>
__device__ __forceinline__ void hop_dir(cx<T> acc[12], const WT W[9], const rawc<L> psi[12], T one)
{
    const T s = (T)S * one;
    cx<T> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const rawc<L> u0 = psi[c], u1 = psi[3 + c], l0 = psi[6 + c], l1 = psi[9 + c];
        if (MU == 0) {          // h0 = u0 + S i l1, h1 = u1 + S i l0
            h0[c] = p_addi(u0, l1, s);
            h1[c] = p_addi(u1, l0, s);
        } else if (MU == 1) {   // h0 = u0 + S l1,   h1 = u1 - S l0
            h0[c] = p_add(u0, l1, s);
            h1[c] = p_add(u1, l0, -s);
        } else if (MU == 2) {   // h0 = u0 + S i l0, h1 = u1 - S i l1
            h0[c] = p_addi(u0, l0, s);
            h1[c] = p_addi(u1, l1, -s);
        } else {                // h0 = u0 - S l0,   h1 = u1 - S l1
            h0[c] = p_add(u0, l0, -s);
            h1[c] = p_add(u1, l1, -s);
        }
    }
    cx<T> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        cx<T> a = {0, 0}, b = {0, 0};
#pragma unroll
        for (int c = 0; c < 3; c++) {
            lmac(a, W[3 * r + c], h0[c]);
            lmac(b, W[3 * r + c], h1[c]);
        }
        w0[r] = a;
        w1[r] = b;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc[c].r += w0[c].r;
        acc[c].i += w0[c].i;
        acc[3 + c].r += w1[c].r;
        acc[3 + c].i += w1[c].i;
        cx<T> &l0 = acc[6 + c], &l1 = acc[9 + c];
        // explicit FMAs: the rounding must not depend on what the compiler
        // contracts in a given instantiation (results are bit-identical for
        // every right-hand-side tile)
        if (MU == 0) {          // lower = -S (i w1, i w0)
            l0.r = fma(s, w1[c].i, l0.r); l0.i = fma(-s, w1[c].r, l0.i);
            l1.r = fma(s, w0[c].i, l1.r); l1.i = fma(-s, w0[c].r, l1.i);
        } else if (MU == 1) {   // lower = -S (w1, -w0)
            l0.r = fma(-s, w1[c].r, l0.r); l0.i = fma(-s, w1[c].i, l0.i);
            l1.r = fma(s, w0[c].r, l1.r); l1.i = fma(s, w0[c].i, l1.i);
        } else if (MU == 2) {   // lower = -S (i w0, -i w1)
            l0.r = fma(s, w0[c].i, l0.r); l0.i = fma(-s, w0[c].r, l0.i);
            l1.r = fma(-s, w1[c].i, l1.r); l1.i = fma(s, w1[c].r, l1.i);
        } else {                // lower = -S (w0, w1)
            l0.r = fma(-s, w0[c].r, l0.r); l0.i = fma(-s, w0[c].i, l0.i);
            l1.r = fma(-s, w1[c].r, l1.r); l1.i = fma(-s, w1[c].i, l1.i);
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
// cache-policy operand of the output stores: non-temporal (streaming) hint,
// outputs are not re-read by this launch.  Links are loaded with the default
// policy: the right-hand-side groups of a site block (adjacent workgroups on
// one XCD) read them again, and a streaming hint on them raised the fetched
// bytes by a quarter.
constexpr int kNT = 2;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, size_t bytes)
{
    const unsigned n = bytes >= 0xffffffffull ? 0xffffffffu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, kRsrcFlags);
}

template <typename S>
struct BufIO;
// component type of a raw load
template <typename S>
struct RawT {
    using L = float;
};
template <>
struct RawT<double2> {
    using L = double;
};
template <>
struct RawT<h2> {
    using L = _Float16;
};
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
    __device__ __forceinline__ static cx<T> ldlink(rsrc_t r, int voff, int soff)
    {
        D2 v = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        return {(T)v.x, (T)v.y};
    }
    __device__ __forceinline__ static rawc<double> ldraw(rsrc_t r, int voff, int soff)
    {
        D2 v = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        return {v.x, v.y};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        D2 v{(double)c.r, (double)c.i};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, v), r, voff, soff, kNT);
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
    __device__ __forceinline__ static cx<T> ldlink(rsrc_t r, int voff, int soff)
    {
        F2 v = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
        return {(T)v.x, (T)v.y};
    }
    __device__ __forceinline__ static rawc<float> ldraw(rsrc_t r, int voff, int soff)
    {
        F2 v = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
        return {v.x, v.y};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        F2 v{(float)c.r, (float)c.i};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, kNT);
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
    __device__ __forceinline__ static rawc<_Float16> ldraw(rsrc_t r, int voff, int soff)
    {
        h2 h = __builtin_bit_cast(h2, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
        return {h.x, h.y};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        h2 h;
        h.x = (_Float16)(float)c.r;
        h.y = (_Float16)(float)c.i;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, h), r, voff, soff, kNT);
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
    __device__ __forceinline__ static rawc<float> ldraw(rsrc_t r, int voff, int soff)
    {
        unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        return {__builtin_bit_cast(float, v << 16), __builtin_bit_cast(float, v & 0xffff0000u)};
    }
    template <typename T>
    __device__ __forceinline__ static void st(rsrc_t r, int voff, int soff, cx<T> c)
    {
        unsigned v = (unsigned)f32_to_bf16((float)c.r) | ((unsigned)f32_to_bf16((float)c.i) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, kNT);
    }
};

// link entry as held in registers: binary16 links stay binary16 (converted
// inside the FMAs), FP32/FP64 links and rebuilt 12-parameter links in the
// arithmetic type
template <typename LS, typename T>
struct LinkEl {
    using type = cx<T>;
};
template <typename T>
struct LinkEl<h2, T> {
    using type = rawc<_Float16>;
};

template <typename LS, typename T>
__device__ __forceinline__ void load_link(typename LinkEl<LS, T>::type W[9], rsrc_t lr, int vbytes, int voff)
{
#pragma unroll
    for (int k = 0; k < 9; k++) {
        if constexpr (std::is_same<LS, h2>::value)
            W[k] = BufIO<h2>::ldraw(lr, voff, k * vbytes);
        else
            W[k] = BufIO<LS>::template ldlink<T>(lr, voff, k * vbytes);
    }
}

template <typename SS>
__device__ __forceinline__ void load_spinor(rawc<typename RawT<SS>::L> psi[12], rsrc_t sr, int vbytes, int voff)
{
#pragma unroll
    for (int k = 0; k < 12; k++) psi[k] = BufIO<SS>::ldraw(sr, voff, k * vbytes);
}

// 12-parameter link (appendix A.1, link reconstruction): the first two rows in
// binary16, [8 directions][6][vh]; the third row of a special unitary matrix
// is the complex conjugate of the cross product of the first two.  The stored
// rows carry the time-boundary factor f = +-1, which cancels in the cross
// product (f^2 = 1), so the rebuilt row is multiplied by f again on links
// that cross the boundary.
template <typename RS, typename T>
__device__ __forceinline__ void load_link12(cx<T> W[9], rsrc_t lr, int vbytes, int voff, bool cross, T tbc)
{
#pragma unroll
    for (int k = 0; k < 6; k++) {
        if constexpr (std::is_same<RS, h2>::value) {
            const rawc<_Float16> w = BufIO<h2>::ldraw(lr, voff, k * vbytes);
            W[k] = {(T)w.r, (T)w.i};
        } else {
            W[k] = BufIO<RS>::template ldlink<T>(lr, voff, k * vbytes);
        }
    }
    // conj(a b - c d) for each entry of row0 x row1
    auto cr = [](cx<T> a, cx<T> b, cx<T> c, cx<T> d) {
        T re = a.r * b.r;
        re = fma(-a.i, b.i, re);
        re = fma(-c.r, d.r, re);
        re = fma(c.i, d.i, re);
        T im = a.r * b.i;
        im = fma(a.i, b.r, im);
        im = fma(-c.r, d.i, im);
        im = fma(-c.i, d.r, im);
        return cx<T>{re, -im};
    };
    W[6] = cr(W[1], W[5], W[2], W[4]);
    W[7] = cr(W[2], W[3], W[0], W[5]);
    W[8] = cr(W[0], W[4], W[1], W[3]);
    if (cross) {
#pragma unroll
        for (int k = 6; k < 9; k++) W[k] = {tbc * W[k].r, tbc * W[k].i};
    }
}

// 8-parameter FP64 link (appendix A.1; stored form in misc.hip): |a1| and
// |c1| from the unit first row and column, their phases from the stored
// angles, the 2x2 block from the cofactor relations conj(U) = cof(U):
//   b2 = -(conj(a1) a2 b1 + conj(c1) conj(a3)) / n,  b3 = (conj(a2) conj(c1) - conj(a1) a3 b1) / n,
//   c2 = (conj(a3) conj(b1) - conj(a1) a2 c1) / n,   c3 = -(conj(a2) conj(b1) + conj(a1) a3 c1) / n,
// n = |a2|^2 + |a3|^2; rows swapped and negated back for links stored that
// way (phase flag), then the time-boundary factor on crossing links
template <typename T>
__device__ __forceinline__ void load_link8(cx<T> W[9], rsrc_t lr, int vbytes, int voff, bool cross, T tbc)
{
    const cx<T> a2 = BufIO<double2>::template ldlink<T>(lr, voff, 0);
    const cx<T> a3 = BufIO<double2>::template ldlink<T>(lr, voff, vbytes);
    const cx<T> b1 = BufIO<double2>::template ldlink<T>(lr, voff, 2 * vbytes);
    const cx<T> ph = BufIO<double2>::template ldlink<T>(lr, voff, 3 * vbytes);
    const bool swap = ph.i > (T)4;
    const T tc = swap ? ph.i - (T)8 : ph.i;
    const T n = a2.r * a2.r + a2.i * a2.i + a3.r * a3.r + a3.i * a3.i;
    const T ra = sqrt((T)1 - n), rc = sqrt(fmax(n - (b1.r * b1.r + b1.i * b1.i), (T)0));
    T sa, ca, sc, cc;
    sincos(ph.r, &sa, &ca);
    sincos(tc, &sc, &cc);
    const cx<T> a1 = {ra * ca, ra * sa}, c1 = {rc * cc, rc * sc};
    const T inv = (T)1 / n;
    const cx<T> ab = conjg(a1) * b1, ac = conjg(a1) * c1;
    const cx<T> a2c = conjg(a2), a3c = conjg(a3), b1c = conjg(b1), c1c = conjg(c1);
    const cx<T> b2 = (ab * a2 + c1c * a3c) * cx<T>{-inv, 0};
    const cx<T> b3 = (a2c * c1c - ab * a3) * cx<T>{inv, 0};
    const cx<T> c2 = (a3c * b1c - ac * a2) * cx<T>{inv, 0};
    const cx<T> c3 = (a2c * b1c + ac * a3) * cx<T>{-inv, 0};
    const cx<T> m[9] = {a1, a2, a3, b1, b2, b3, c1, c2, c3};
    const T g = (swap ? (T)-1 : (T)1) * (cross ? tbc : (T)1);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        W[k] = {g * m[k].r, g * m[k].i};
        const cx<T> r1 = swap ? m[6 + k] : m[3 + k], r2 = swap ? m[3 + k] : m[6 + k];
        W[3 + k] = {g * r1.r, g * r1.i};
        W[6 + k] = {g * r2.r, g * r2.i};
    }
}

// ------------------------------------------------ FP16 spinors, binary16 links
// Packed form of the hop for IEEE binary16 spinors and links: the spin
// projection h = u + a l (a = +-1, +-i) is one packed binary16 add per
// complex value, producing h in the two arrangements the colour product
// needs, conj(h) = (h.r, -h.i) and swap(h) = (h.i, h.r); each complex
// multiply-add of the 3x3 link product is then two v_dot2_f32_f16
//   Re(w h) += w.r h.r - w.i h.i = dot2(w, conj h),
//   Im(w h) += w.r h.i + w.i h.r = dot2(w, swap h),
// whose binary16 products are exact and whose sums are FP32.  Relative to
// the FP32 projection this rounds h once to binary16 (the storage precision
// of its inputs); all accumulation stays FP32.
typedef _Float16 hv2 __attribute__((ext_vector_type(2)));

// h = u + SG l (I = false) or u + SG i l (I = true), as (conj h, swap h):
// each one v_pk_add_f16 whose operand selection (op_sel: which half of each
// source feeds the low result, op_sel_hi: the high result) and negation
// modifiers (neg_lo, neg_hi: negate that source's value in the low / high
// result) form the arrangement, written out so that no separate swap or
// sign instruction is generated.  With u = (ur, ui), l = (lr, li):
//   real, SG > 0:  conj = (ur + lr, -ui - li)   swap = (ui + li, ur + lr)
//   real, SG < 0:  conj = (ur - lr, -ui + li)   swap = (ui - li, ur - lr)
//   i,    SG > 0:  conj = (ur - li, -ui - lr)   swap = (ui + lr, ur - li)
//   i,    SG < 0:  conj = (ur + li, -ui + lr)   swap = (ui - lr, ur + li)
template <bool I, int SG>
__device__ __forceinline__ void proj2(hv2 u, hv2 l, hv2 &hc, hv2 &hs)
{
    if constexpr (!I && SG > 0) {
        asm("v_pk_add_f16 %0, %1, %2 neg_hi:[1,1]" : "=v"(hc) : "v"(u), "v"(l));
        asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,1] op_sel_hi:[0,0]" : "=v"(hs) : "v"(u), "v"(l));
    } else if constexpr (!I) {
        asm("v_pk_add_f16 %0, %1, %2 neg_lo:[0,1] neg_hi:[1,0]" : "=v"(hc) : "v"(u), "v"(l));
        asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[0,1]"
            : "=v"(hs) : "v"(u), "v"(l));
    } else if constexpr (SG > 0) {
        asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[1,1]"
            : "=v"(hc) : "v"(u), "v"(l));
        asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1] neg_hi:[0,1]" : "=v"(hs) : "v"(u), "v"(l));
    } else {
        asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0] neg_hi:[1,0]" : "=v"(hc) : "v"(u), "v"(l));
        asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1]" : "=v"(hs) : "v"(u), "v"(l));
    }
}

// a.lo b.lo + a.hi b.hi (binary16 products, FP32 sum) with no accumulator
// input: the first term of a chain, without a register cleared to zero
__device__ __forceinline__ float dot2_first(hv2 a, hv2 b)
{
    float d;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

template <int MU, int S>
__device__ __forceinline__ void hop_dir_h(cx<float> acc[12], const hv2 W[9], const hv2 psi[12])
{
    hv2 c0[3], s0[3], c1[3], s1[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const hv2 u0 = psi[c], u1 = psi[3 + c], l0 = psi[6 + c], l1 = psi[9 + c];
        if (MU == 0) {          // h0 = u0 + S i l1, h1 = u1 + S i l0
            proj2<true, S>(u0, l1, c0[c], s0[c]);
            proj2<true, S>(u1, l0, c1[c], s1[c]);
        } else if (MU == 1) {   // h0 = u0 + S l1,   h1 = u1 - S l0
            proj2<false, S>(u0, l1, c0[c], s0[c]);
            proj2<false, -S>(u1, l0, c1[c], s1[c]);
        } else if (MU == 2) {   // h0 = u0 + S i l0, h1 = u1 - S i l1
            proj2<true, S>(u0, l0, c0[c], s0[c]);
            proj2<true, -S>(u1, l1, c1[c], s1[c]);
        } else {                // h0 = u0 - S l0,   h1 = u1 - S l1
            proj2<false, -S>(u0, l0, c0[c], s0[c]);
            proj2<false, -S>(u1, l1, c1[c], s1[c]);
        }
    }
    cx<float> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        float ar = dot2_first(W[3 * r], c0[0]), ai = dot2_first(W[3 * r], s0[0]);
        float br = dot2_first(W[3 * r], c1[0]), bi = dot2_first(W[3 * r], s1[0]);
#pragma unroll
        for (int c = 1; c < 3; c++) {
            ar = __builtin_amdgcn_fdot2(W[3 * r + c], c0[c], ar, false);
            ai = __builtin_amdgcn_fdot2(W[3 * r + c], s0[c], ai, false);
            br = __builtin_amdgcn_fdot2(W[3 * r + c], c1[c], br, false);
            bi = __builtin_amdgcn_fdot2(W[3 * r + c], s1[c], bi, false);
        }
        w0[r] = {ar, ai};
        w1[r] = {br, bi};
    }
    constexpr float s = (float)S;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc[c].r += w0[c].r;
        acc[c].i += w0[c].i;
        acc[3 + c].r += w1[c].r;
        acc[3 + c].i += w1[c].i;
        cx<float> &l0 = acc[6 + c], &l1 = acc[9 + c];
        if (MU == 0) {          // lower = -S (i w1, i w0)
            l0.r += s * w1[c].i; l0.i -= s * w1[c].r;
            l1.r += s * w0[c].i; l1.i -= s * w0[c].r;
        } else if (MU == 1) {   // lower = -S (w1, -w0)
            l0.r -= s * w1[c].r; l0.i -= s * w1[c].i;
            l1.r += s * w0[c].r; l1.i += s * w0[c].i;
        } else if (MU == 2) {   // lower = -S (i w0, -i w1)
            l0.r += s * w0[c].i; l0.i -= s * w0[c].r;
            l1.r -= s * w1[c].i; l1.i += s * w1[c].r;
        } else {                // lower = -S (w0, w1)
            l0.r -= s * w0[c].r; l0.i -= s * w0[c].i;
            l1.r -= s * w1[c].r; l1.i -= s * w1[c].i;
        }
    }
}

__device__ __forceinline__ hv2 ld_hv2(rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(hv2, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// binary16 link as nine packed entries; the 12-parameter form rebuilds the
// third row conj(row0 x row1) with dot2 products (exact binary16 products,
// FP32 sums) rounded once to binary16, times the time-boundary factor on
// links that cross the boundary
template <bool REC>
__device__ __forceinline__ void load_link_h(hv2 W[9], rsrc_t lr, int vbytes, int voff, bool cross, float tbc)
{
    if constexpr (!REC) {
#pragma unroll
        for (int k = 0; k < 9; k++) W[k] = ld_hv2(lr, voff, k * vbytes);
    } else {
#pragma unroll
        for (int k = 0; k < 6; k++) W[k] = ld_hv2(lr, voff, k * vbytes);
        // conj(a b - c d): Re(a b) = dot2(a, conj b), Im(a b) = dot2(a, swap b)
        auto cr = [](hv2 a, hv2 b, hv2 c, hv2 d) {
            const hv2 nc = -c;
            const float re = __builtin_amdgcn_fdot2(nc, hv2{d.x, -d.y}, dot2_first(a, hv2{b.x, -b.y}), false);
            const float im = __builtin_amdgcn_fdot2(nc, hv2{d.y, d.x}, dot2_first(a, hv2{b.y, b.x}), false);
            return hv2{(_Float16)re, (_Float16)(-im)};
        };
        W[6] = cr(W[1], W[5], W[2], W[4]);
        W[7] = cr(W[2], W[3], W[0], W[5]);
        W[8] = cr(W[0], W[4], W[1], W[3]);
        if (cross) {
            const _Float16 f = (_Float16)tbc;
#pragma unroll
            for (int k = 6; k < 9; k++) W[k] = W[k] * f;
        }
    }
}

template <int MU, int S, typename SS, typename LS, typename T, int R>
__device__ __forceinline__ void do_dir(cx<T> acc[R][12], const DParams<T> &a, const rsrc_t *sr, int dir, int j,
                                       int i, int t)
{
    if constexpr (std::is_same<SS, h2>::value && (std::is_same<LS, L12>::value || std::is_same<LS, h2>::value)) {
        constexpr bool REC = std::is_same<LS, L12>::value;
        constexpr int NP = REC ? 6 : 9;
        const h2 *lbase = (const h2 *)a.links + (size_t)dir * NP * a.g.vh;
        const rsrc_t lr = make_rsrc(lbase, (size_t)NP * a.g.vh * sizeof(h2));
        const bool bnd = MU == 3 && (dir < 4 ? t == a.g.L[3] - 1 : t == 0);
        hv2 W[9];
        load_link_h<REC>(W, lr, a.g.vh * (int)sizeof(h2), i * (int)sizeof(h2), bnd, (float)a.t_bc);
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            hv2 psi[12];
#pragma unroll
            for (int k = 0; k < 12; k++) psi[k] = ld_hv2(sr[rr], j * (int)sizeof(h2), k * a.g.hs * (int)sizeof(h2));
            hop_dir_h<MU, S>(reinterpret_cast<cx<float> *>(acc[rr]), W, psi);
        }
        __builtin_amdgcn_sched_barrier(0);
        return;
    }
    typename LinkEl<LS, T>::type W[9];
    if constexpr (std::is_same<LS, L8D>::value) {
        const double2 *lbase = (const double2 *)a.links + (size_t)dir * 4 * a.g.vh;
        const rsrc_t lr = make_rsrc(lbase, (size_t)4 * a.g.vh * sizeof(double2));
        const bool bnd = MU == 3 && (dir < 4 ? t == a.g.L[3] - 1 : t == 0);
        load_link8<T>(W, lr, a.g.vh * (int)sizeof(double2), i * (int)sizeof(double2), bnd, (T)a.t_bc);
    } else if constexpr (std::is_same<LS, L12>::value || std::is_same<LS, L12D>::value ||
                         std::is_same<LS, L12F>::value) {
        using RS = std::conditional_t<std::is_same<LS, L12>::value, h2,
                                      std::conditional_t<std::is_same<LS, L12D>::value, double2, float2>>;
        const RS *lbase = (const RS *)a.links + (size_t)dir * 6 * a.g.vh;
        const rsrc_t lr = make_rsrc(lbase, (size_t)6 * a.g.vh * sizeof(RS));
        const bool bnd = MU == 3 && (dir < 4 ? t == a.g.L[3] - 1 : t == 0);
        load_link12<RS, T>(W, lr, a.g.vh * (int)sizeof(RS), i * (int)sizeof(RS), bnd, (T)a.t_bc);
    } else {
        const LS *lbase = (const LS *)a.links + (size_t)dir * 9 * a.g.vh;
        const rsrc_t lr = make_rsrc(lbase, (size_t)9 * a.g.vh * sizeof(LS));
        load_link<LS, T>(W, lr, a.g.vh * (int)sizeof(LS), i * (int)sizeof(LS));
    }
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        rawc<typename RawT<SS>::L> psi[12];
        load_spinor<SS>(psi, sr[rr], a.g.hs * (int)sizeof(SS), j * (int)sizeof(SS));
        hop_dir<MU, S>(acc[rr], W, psi, a.one);
    }
    // keep the loads of one direction from being hoisted above the previous
    // direction's arithmetic: bounds the live registers to one direction
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// value as stored in precision SS (what later kernels will read)
template <typename SS, typename T>
__device__ __forceinline__ cx<T> stored(cx<T> v)
{
    if constexpr (std::is_same<SS, double2>::value) {
        return v;
    } else if constexpr (std::is_same<SS, float2>::value) {
        return {(T)(float)v.r, (T)(float)v.i};
    } else if constexpr (std::is_same<SS, h2>::value) {
        return {(T)(float)(_Float16)(float)v.r, (T)(float)(_Float16)(float)v.i};
    } else {
        return {(T)bf16_to_f32(f32_to_bf16((float)v.r)), (T)bf16_to_f32(f32_to_bf16((float)v.i))};
    }
}

template <typename T>
__device__ __forceinline__ double norm2c(cx<T> v)
{
    return (double)(v.r * v.r + v.i * v.i);
}

// Epilogue forms:
//   EPI_STORE  out = D_hop Hop[in] (+ D_own own)
//   EPI_NORM   as EPI_STORE, plus per-block partial |out|^2 per right-hand side
//   EPI_CG     s = D_hop Hop[in] + D_own q (own = q); then r -= alpha s,
//              rho -= alpha q in place (s is never stored), partial |r|^2 and
//              |rho|^2 -- the last half of Ahat^dag q fused with the CG updates;
//              rho = null: r only (the solver follows |rho|^2 by recurrence)
enum { EPI_STORE = 0, EPI_NORM = 1, EPI_CG = 2 };

// Block order: see map_block.
// One block of the launch: bhw is the block's index within its instance's
// range of nhw blocks (that range starts at a multiple of 8, so bhw % 8 is
// still the XCD).
template <typename SS, typename LS, typename T, int R, int DAG, int OWN, int EPI>
__device__ __forceinline__ void dslash_block(const DParams<T> &a, int bhw, int nhw)
{
    int grp;
    const int sblk = map_block(bhw, nhw, a.ngroups, a.nb_t, grp);
    const int r0 = grp * R;
    const int i_raw = sblk * kBlock + threadIdx.x;
    const bool valid = i_raw < a.g.vh;
    if (EPI == EPI_STORE && !valid) return;
    const int i = valid ? i_raw : a.g.vh - 1;  // idle lanes join the block reduction
    const size_t fbytes = (size_t)12 * a.g.hs * sizeof(SS);  // one right-hand side
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
        case 0: do_dir<0, SF, SS, LS, T, R>(acc, a, sr, 0, j, i, t); break;
        case 1: do_dir<1, SF, SS, LS, T, R>(acc, a, sr, 1, j, i, t); break;
        case 2: do_dir<2, SF, SS, LS, T, R>(acc, a, sr, 2, j, i, t); break;
        case 3: do_dir<3, SF, SS, LS, T, R>(acc, a, sr, 3, j, i, t); break;
        case 4: do_dir<0, SB, SS, LS, T, R>(acc, a, sr, 4, j, i, t); break;
        case 5: do_dir<1, SB, SS, LS, T, R>(acc, a, sr, 5, j, i, t); break;
        case 6: do_dir<2, SB, SS, LS, T, R>(acc, a, sr, 6, j, i, t); break;
        default: do_dir<3, SB, SS, LS, T, R>(acc, a, sr, 7, j, i, t); break;
        }
    }

    const int vb = a.g.hs * (int)sizeof(SS), vo = i * (int)sizeof(SS);
    constexpr int NQ = EPI == EPI_CG ? 2 : 1;
    double nrm[R][NQ];
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        const rsrc_t outr = make_rsrc((char *)a.out + (r0 + rr) * fbytes, fbytes);
        const rsrc_t ownr = make_rsrc((const char *)a.own + (r0 + rr) * fbytes, fbytes);
        const rsrc_t rr_r = make_rsrc((char *)a.r + (r0 + rr) * fbytes, fbytes);
        const rsrc_t rho_r = make_rsrc((char *)a.rho + (r0 + rr) * fbytes, fbytes);
        T alpha = 0;
        if constexpr (EPI == EPI_CG) alpha = (T)cgdev::ld_coh(&a.sc[r0 + rr].alpha);
#pragma unroll
        for (int q = 0; q < NQ; q++) nrm[rr][q] = 0;
        // all loads of this right-hand side first, then arithmetic and
        // stores: the stores may alias the loaded fields as far as the
        // compiler knows, so interleaving them would serialise the loads
        cx<T> o[12], rl[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            o[k] = {0, 0};
            if (OWN) o[k] = BufIO<SS>::template ld<T>(ownr, vo, k * vb);
            if constexpr (EPI == EPI_CG) rl[k] = BufIO<SS>::template ld<T>(rr_r, vo, k * vb);
        }
        const bool track_rho = EPI == EPI_CG && a.rho != nullptr;  // uniform
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<T> v = (k < 6 ? a.hop_u : a.hop_l) * acc[rr][k];
            if (OWN) v = v + (k < 6 ? a.own_u : a.own_l) * o[k];
            if constexpr (EPI == EPI_CG) {
                const cx<T> rv = rl[k] - alpha * v;
                if (valid) {
                    BufIO<SS>::template st<T>(rr_r, vo, k * vb, rv);
                    nrm[rr][0] += norm2c(stored<SS>(rv));
                }
            } else {
                if (valid) {
                    BufIO<SS>::template st<T>(outr, vo, k * vb, v);
                    if constexpr (EPI == EPI_NORM) nrm[rr][0] += norm2c(stored<SS>(v));
                }
            }
        }
        if (track_rho) {
            cx<T> hl[12];
#pragma unroll
            for (int k = 0; k < 12; k++) hl[k] = BufIO<SS>::template ld<T>(rho_r, vo, k * vb);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<T> hv = hl[k] - alpha * o[k];
                if (valid) {
                    BufIO<SS>::template st<T>(rho_r, vo, k * vb, hv);
                    nrm[rr][1] += norm2c(stored<SS>(hv));
                }
            }
        }
    }
    if constexpr (EPI != EPI_STORE) {
        // deterministic block reduction: wave shuffles, then the 4 waves in order
        __shared__ double red[kBlock / 64][R * NQ];
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                double v = wave_sum(nrm[rr][q]);
                if (lane == 0) red[w][rr * NQ + q] = v;
            }
        __syncthreads();
        if (threadIdx.x < R * NQ) {
            const int rr = threadIdx.x / NQ, q = threadIdx.x % NQ;
            double s = 0;
#pragma unroll
            for (int k = 0; k < kBlock / 64; k++) s += red[k][threadIdx.x];
            cgdev::st_coh(a.part + ((size_t)q * a.nrhs + r0 + rr) * a.nblk + sblk, s);
        }
    }
}

template <typename SS, typename LS, typename T, int R, int DAG, int OWN, int EPI>
__global__ __launch_bounds__(kBlock, (waves_for<T, R>())) void k_dslash(DParams<T> a)
{
    dslash_block<SS, LS, T, R, DAG, OWN, EPI>(a, blockIdx.x, gridDim.x);
}

// Several lattices in one launch: instance i owns hardware blocks
// [start[i], start[i+1]) (padded to multiples of 8; padding blocks exit).
// The records travel in the kernel-argument segment, like the single form's
// parameters: uniform, read-only scalar loads that the compiler may repeat
// after the epilogue's stores without going through the vector caches.
template <typename T>
struct MultiArgs {
    DParams<T> p[kMultiInst];
    int start[kMultiInst + 1];
    int n;
};
static_assert(sizeof(MultiArgs<double>) <= 4096, "kernel arguments exceed 4 KiB");

template <typename SS, typename LS, typename T, int R, int DAG, int OWN, int EPI>
__global__ __launch_bounds__(kBlock, (waves_for<T, R>())) void k_dslash_multi(const MultiArgs<T> m)
{
    int i = 0;
    while (i + 1 < m.n && (int)blockIdx.x >= m.start[i + 1]) i++;
    const int local = (int)blockIdx.x - m.start[i];
    const int nreal = m.p[i].nblk * m.p[i].ngroups;
    if (local >= nreal) return;
    dslash_block<SS, LS, T, R, DAG, OWN, EPI>(m.p[i], local, nreal);
}

// ---------------------------------------------------------------- persistent batch
// One launch runs `iters` CG iterations of every instance of a batch: the
// four half-Dslash stages, the CG scalars and the vector update, separated
// by grid-wide barriers.  The grid is sized so that every block is resident
// (cooperative launch).  Each Dslash stage walks the virtual blocks of all
// instances (the same (instance, site block, RHS group) decomposition and
// XCD mapping as the multi-instance kernel: the grid is a multiple of 8, so
// virtual block v runs on XCD v % 8); the scalar stages give one
// (instance, right-hand side) to a block and run the code of the
// stand-alone scalar kernels, so every instance follows its single solve
// bit for bit.  Per iteration:
//   S1 | S2 | S3 + alpha | S4 | beta | update |
// (alpha is summed while the third stage runs: that stage does not read it).

// Barrier state in device memory (zeroed before each launch), one 128-byte
// line per word: arrivals of the blocks with blockIdx % 8 == j, arrivals of
// the eight groups, the generation published to group j, the failure flag.
constexpr int kBarLine = 32;  // unsigned words per line
constexpr int kBarWords = 18 * kBarLine;
__device__ __forceinline__ unsigned *bar_cnt(unsigned *b, int j) { return b + j * kBarLine; }
__device__ __forceinline__ unsigned *bar_top(unsigned *b) { return b + 8 * kBarLine; }
__device__ __forceinline__ unsigned *bar_gen(unsigned *b, int j) { return b + (9 + j) * kBarLine; }
__device__ __forceinline__ unsigned *bar_fail(unsigned *b) { return b + 17 * kBarLine; }

// Launch parameters, kept in device memory (read-only during the launch):
// the stages index them with the instance number, which a kernel-argument
// block would have to copy to per-lane scratch memory.
template <typename T>
struct PersistArgs {
    DParams<T> st[4][kPersistInst];  // the stage forms of each instance
    void *x[kPersistInst];           // solution accumulator (FP32)
    CGScalars *sc[kPersistInst];
    double delta[kPersistInst];
    int start[kPersistInst + 1];     // virtual Dslash blocks, multiples of 8
    int ustart[kPersistInst + 1];    // update work items (right-hand side x chunk)
    int uchunks[kPersistInst];       // chunks per right-hand side
    int fstart[kPersistInst + 1];    // scalar work items (right-hand sides)
    int n;
    unsigned *bar;                   // kBarWords words
};

constexpr int kUpdChunk = 8 * kBlock;  // elements per update work item

// Grid-wide barrier with a bounded wait, in two levels (the blocks of each
// of the eight residue classes of blockIdx, then the eight classes) so that
// no address takes more than G/8 arrivals or pollers.  Returns false (in
// every thread) when this or another block gave up; the caller then leaves
// the kernel.
__device__ __forceinline__ bool grid_sync(unsigned *bar, unsigned long long spin_limit)
{
    __shared__ int ok;
    // every wave waits until its own stores have reached the L2 (the
    // workgroup barrier alone does not wait for other waves' stores); the
    // release below then writes this L2's dirty lines back once per block
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int j = blockIdx.x & 7;
        const unsigned per = gridDim.x >> 3;  // the grid is a multiple of 8
        // release this block's results to the other XCDs (L2 write-back)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // the generation is read before arriving (acquire: the arrival below
        // cannot be performed first), so it cannot have advanced yet
        const unsigned g = __hip_atomic_load(bar_gen(bar, j), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        if (__hip_atomic_fetch_add(bar_cnt(bar, j), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == per) {
            // the class's counter is reset before the class arrives above (a
            // block of the class may arrive at the next barrier as soon as
            // the generation moves)
            __hip_atomic_store(bar_cnt(bar, j), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            if (__hip_atomic_fetch_add(bar_top(bar), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == 8) {
                __hip_atomic_store(bar_top(bar), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                for (int k = 0; k < 8; k++)
                    __hip_atomic_fetch_add(bar_gen(bar, k), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // poll about every 0.5 us, the failure flag every 32nd poll
        unsigned long long n = 0;
        while (__hip_atomic_load(bar_gen(bar, j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
            if (++n > spin_limit ||
                ((n & 31) == 0 && __hip_atomic_load(bar_fail(bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(bar_fail(bar), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(20);
        }
        if (__hip_atomic_load(bar_fail(bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) good = 0;
        // acquire the other blocks' results (invalidate this CU's L1 and
        // the stale L2 lines)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// One Dslash stage over the virtual blocks of all instances; stage index k.
template <typename SS, typename LS, typename T, int R, int DAG, int OWN, int EPI>
__device__ __forceinline__ void persist_stage(const PersistArgs<T> &a, int k)
{
    const int total = a.start[a.n];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        int i = 0;
        while (i + 1 < a.n && vb >= a.start[i + 1]) i++;
        const DParams<T> &p = a.st[k][i];
        const int local = vb - a.start[i];
        const int nreal = p.nblk * p.ngroups;
        if (local >= nreal) continue;
        dslash_block<SS, LS, T, R, DAG, OWN, EPI>(p, local, nreal);
        // the block reduction of the next virtual block reuses the LDS
        if constexpr (EPI != EPI_STORE) __syncthreads();
    }
}

// The CG scalars of one right-hand side per block: alpha from the partial
// sums of stage 2 (BETA = false) or beta and the flags from those of stage 4.
template <typename T, bool BETA>
__device__ __forceinline__ void persist_scalars(const PersistArgs<T> &a)
{
    const int total = a.fstart[a.n];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        int i = 0;
        while (i + 1 < a.n && w >= a.fstart[i + 1]) i++;
        const int r = w - a.fstart[i];
        if constexpr (BETA) {
            const DParams<T> &p = a.st[3][i];
            cgdev::finish_beta(a.sc[i], p.part, p.nblk, p.nrhs, a.delta[i], r);
        } else {
            const DParams<T> &p = a.st[1][i];
            cgdev::finish_alpha(a.sc[i], p.part, p.nblk, r);
        }
    }
}

template <typename SS, typename T>
__device__ __forceinline__ void persist_update(const PersistArgs<T> &a)
{
    const int total = a.ustart[a.n];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        int i = 0;
        while (i + 1 < a.n && w >= a.ustart[i + 1]) i++;
        const int local = w - a.ustart[i];
        const int r = local / a.uchunks[i], ch = local - r * a.uchunks[i];
        const DParams<T> &p0 = a.st[0][i];  // stage 1 reads p
        const DParams<T> &p3 = a.st[3][i];  // stage 4 updates r
        const size_t n = (size_t)12 * p0.g.hs;
        const size_t e0 = (size_t)ch * kUpdChunk, e1 = e0 + kUpdChunk < n ? e0 + kUpdChunk : n;
        cgdev::update_px((SS *)p0.in, (const SS *)p3.r, (float2 *)a.x[i], n, a.sc[i], r, e0 + threadIdx.x, e1,
                         (size_t)kBlock);
    }
}

template <typename SS, typename LS, typename T, int R>
__global__ __launch_bounds__(kBlock, (waves_for<T, R>())) void k_batch_persist(const PersistArgs<T> *__restrict__ pa,
                                                                             int iters,
                                                                             unsigned long long spin_limit)
{
    const PersistArgs<T> &a = *pa;
    for (int it = 0; it < iters; it++) {
        persist_stage<SS, LS, T, R, 0, 0, EPI_STORE>(a, 0);  // t = R_oo^-1 H_oe p
        if (!grid_sync(a.bar, spin_limit)) return;
        persist_stage<SS, LS, T, R, 0, 1, EPI_NORM>(a, 1);   // q = R_ee p - H_eo t, |q|^2 partials
        if (!grid_sync(a.bar, spin_limit)) return;
        persist_stage<SS, LS, T, R, 1, 0, EPI_STORE>(a, 2);  // t = R_oo^-1 H_oe^dag q
        persist_scalars<T, false>(a);                       // alpha
        if (!grid_sync(a.bar, spin_limit)) return;
        persist_stage<SS, LS, T, R, 0, 1, EPI_CG>(a, 3);     // r -= alpha Ahat^dag q, partials
        if (!grid_sync(a.bar, spin_limit)) return;
        persist_scalars<T, true>(a);                        // beta, flags
        if (!grid_sync(a.bar, spin_limit)) return;
        persist_update<SS, T>(a);                           // x += alpha p, p = r + beta p
        if (it + 1 < iters && !grid_sync(a.bar, spin_limit)) return;
    }
}

template <typename T>
cx<T> cvt(cx<double> v)
{
    return cx<T>{(T)v.r, (T)v.i};
}

template <typename SS, typename LS, typename T, int R, int DAG, int OWN>
void launch_epi(const DslashCall &dc, dim3 grid, hipStream_t s, const DParams<T> &a)
{
    switch (dc.epi) {
    case EPI_NORM: hipLaunchKernelGGL((k_dslash<SS, LS, T, R, DAG, OWN, EPI_NORM>), grid, dim3(kBlock), 0, s, a); break;
    case EPI_CG:
        if constexpr (OWN == 1)
            hipLaunchKernelGGL((k_dslash<SS, LS, T, R, DAG, OWN, EPI_CG>), grid, dim3(kBlock), 0, s, a);
        else
            throw TmError{TM_ERR_ARG, "fused CG epilogue needs the own-site term"};
        break;
    default: hipLaunchKernelGGL((k_dslash<SS, LS, T, R, DAG, OWN, EPI_STORE>), grid, dim3(kBlock), 0, s, a);
    }
}

template <typename SS, typename LS, typename T, int R>
DParams<T> fill_params(tm_ctx *c, const DslashCall &dc)
{
    DParams<T> a;
    a.out = dc.out;
    a.in = dc.in;
    a.own = dc.own;
    a.links = (std::is_same<LS, double2>::value ? c->links64
               : std::is_same<LS, h2>::value     ? c->links16
               : std::is_same<LS, L12>::value    ? c->links12
               : std::is_same<LS, L12D>::value   ? c->links12d
               : std::is_same<LS, L12F>::value   ? c->links12f
               : std::is_same<LS, L8D>::value    ? c->links8d
                                                 : c->links32)[dc.out_parity];
    a.g = c->geo;
    a.p = dc.out_parity;
    a.nrhs = dc.nrhs;
    a.ngroups = dc.nrhs / R;
    a.own_u = cvt<T>(dc.d_own.u);
    a.own_l = cvt<T>(dc.d_own.l);
    a.hop_u = cvt<T>(dc.d_hop.u);
    a.hop_l = cvt<T>(dc.d_hop.l);
    a.one = (T)1;
    a.r = dc.r;
    a.rho = dc.rho;
    a.sc = dc.sc;
    a.part = dc.part;
    a.nblk = dslash_site_blocks(c);
    a.nb_t = (c->geo.vsh % kBlock == 0 && (c->geo.vsh / kBlock) % 8 == 0) ? c->geo.vsh / kBlock : 0;
    a.t_bc = c->t_bc;
    return a;
}

template <typename SS, typename LS, typename T, int R>
void launch_t(tm_ctx *c, const DslashCall &dc, hipStream_t s)
{
    const DParams<T> a = fill_params<SS, LS, T, R>(c, dc);
    dim3 grid((unsigned)(a.nblk * a.ngroups));
    // separate kernels per projector placement and per presence of the
    // own-site term (the x - H y forms read one more field)
    if (dc.dag) {
        if (dc.has_own)
            launch_epi<SS, LS, T, R, 1, 1>(dc, grid, s, a);
        else
            launch_epi<SS, LS, T, R, 1, 0>(dc, grid, s, a);
    } else {
        if (dc.has_own)
            launch_epi<SS, LS, T, R, 0, 1>(dc, grid, s, a);
        else
            launch_epi<SS, LS, T, R, 0, 0>(dc, grid, s, a);
    }
    TM_HIP(hipGetLastError());
}

// Right-hand sides per thread that fit the register budget: FP32 arithmetic
// 1..3 (4 or more exceed 3 resident waves and spill), FP64 1..2; the packed
// binary16 form (FP16 spinors, binary16 links) keeps its spinors in half the
// registers and also tries 4 (at 2 waves per SIMD)
template <typename SS, typename LS, typename T>
constexpr int max_tile()
{
    if constexpr (sizeof(T) == 8) return 2;
    if constexpr (std::is_same<SS, h2>::value && (std::is_same<LS, L12>::value || std::is_same<LS, h2>::value))
        return 4;
    return 3;
}

template <typename SS, typename LS, typename T>
void launch_r(tm_ctx *c, const DslashCall &dc, int R, hipStream_t s)
{
    if constexpr (max_tile<SS, LS, T>() >= 4) {
        if (R == 4) {
            launch_t<SS, LS, T, 4>(c, dc, s);
            return;
        }
    }
    if (R == 3) {
        if constexpr (max_tile<SS, LS, T>() >= 3) {
            launch_t<SS, LS, T, 3>(c, dc, s);
            return;
        }
    }
    if (R >= 2)
        launch_t<SS, LS, T, 2>(c, dc, s);
    else
        launch_t<SS, LS, T, 1>(c, dc, s);
}

// Right-hand sides per thread (each loaded link serves R spinors).  The first
// side-effect-free launch for a (precision, nrhs) pair times every tile that
// divides nrhs and keeps the fastest; results are bit-identical across tiles.
template <typename SS, typename LS, typename T>
void launch_rhs(tm_ctx *c, const DslashCall &dc, hipStream_t s)
{
    const int n = dc.nrhs;
    // tiles are tuned per (spinor precision, link storage, operator form, nrhs):
    // the fused epilogues favour other tiles than the plain store
    const int lcode = std::is_same<LS, h2>::value    ? 1
                      : std::is_same<LS, L12>::value ? 2
                      : std::is_same<LS, L12D>::value ? 3
                      : std::is_same<LS, L12F>::value ? 4
                      : std::is_same<LS, L8D>::value  ? 5
                                                      : 0;
    const int form = dc.dag + 2 * (dc.has_own ? 1 : 0) + 4 * dc.epi;
    const auto key = std::make_pair(dc.spinor_prec + 8 * lcode + 32 * form, n);
    auto it = c->rhs_tile.find(key);
    if (it != c->rhs_tile.end()) {
        launch_r<SS, LS, T>(c, dc, it->second, s);
        return;
    }
    const int def = sizeof(T) == 8 ? 1 : (n % 2 == 0 ? 2 : 1);
    if (c->no_alloc) {  // allocation-free call: no timing launches, no events
        launch_r<SS, LS, T>(c, dc, def, s);
        return;
    }
    int fixed = 0;
    if (const char *e = getenv("TM_DSLASH_RHS_TILE")) fixed = atoi(e);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TM_HIP(hipStreamIsCapturing(s, &cs));
    // timing launches must leave the caller's fields as they were: the output
    // distinct from both inputs, and the in-place CG update of the fused form
    // redirected to scratch fields (its block partials are rewritten by the
    // real launch that follows)
    DslashCall tc = dc;
    const bool repeatable = dc.epi == EPI_CG || (dc.out != dc.in && dc.out != dc.own);
    if (fixed > 0 && fixed <= max_tile<SS, LS, T>() && n % fixed == 0) {
        c->rhs_tile[key] = fixed;
    } else if (!repeatable || cs != hipStreamCaptureStatusNone || n == 1) {
        launch_r<SS, LS, T>(c, dc, def, s);  // tune on a later plain launch
        return;
    } else {
        if (dc.epi == EPI_CG) {  // not capturing here: allocation is allowed
            const size_t fb = (size_t)prec_bytes(dc.spinor_prec) * 12 * c->geo.hs * n;
            tc.r = ws_get(c, "tune_r", fb);
            tc.rho = dc.rho ? ws_get(c, "tune_rho", fb) : nullptr;
        }
        hipEvent_t e0, e1;
        TM_HIP(hipEventCreate(&e0));
        TM_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        int bestR = def;
        for (int R = 1; R <= max_tile<SS, LS, T>(); R++) {
            if (n % R) continue;
            launch_r<SS, LS, T>(c, tc, R, s);  // warm
            TM_HIP(hipEventRecord(e0, s));
            // enough launches that tiles a few percent apart are ranked reliably
            for (int k = 0; k < 6; k++) launch_r<SS, LS, T>(c, tc, R, s);
            TM_HIP(hipEventRecord(e1, s));
            TM_HIP(hipEventSynchronize(e1));
            float ms = 0;
            TM_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bestR = R;
            }
        }
        TM_HIP(hipEventDestroy(e0));
        TM_HIP(hipEventDestroy(e1));
        c->rhs_tile[key] = bestR;
    }
    launch_r<SS, LS, T>(c, dc, c->rhs_tile[key], s);
}

template <typename SS, typename LS, typename T, int R>
void multi_fill(MultiDslash &m, const std::vector<tm_ctx *> &cs, const std::vector<DslashCall> &dcs)
{
    m.args.clear();
    m.grid.clear();
    for (size_t c0 = 0; c0 < cs.size(); c0 += kMultiInst) {
        MultiArgs<T> a{};
        const size_t c1 = std::min(cs.size(), c0 + kMultiInst);
        a.n = (int)(c1 - c0);
        a.start[0] = 0;
        for (size_t k = c0; k < c1; k++) {
            TM_REQUIRE(dcs[k].nrhs % R == 0, "RHS tile must divide every instance's nrhs");
            const int j = (int)(k - c0);
            a.p[j] = fill_params<SS, LS, T, R>(cs[k], dcs[k]);
            const int nb = a.p[j].nblk * a.p[j].ngroups;
            a.start[j + 1] = a.start[j] + (nb + 7) / 8 * 8;
        }
        const unsigned char *raw = reinterpret_cast<const unsigned char *>(&a);
        m.args.emplace_back(raw, raw + sizeof(a));
        m.grid.push_back(a.start[a.n]);
    }
}

template <typename SS, typename LS, typename T, int R>
void multi_go(const MultiDslash &m, hipStream_t s)
{
    for (size_t c = 0; c < m.args.size(); c++) {
        TM_REQUIRE(m.args[c].size() == sizeof(MultiArgs<T>), "multi-instance arguments of another precision");
        MultiArgs<T> a;
        std::memcpy(&a, m.args[c].data(), sizeof(a));
        dim3 g(m.grid[c]), b(kBlock);
        // the four stage forms of a CG iteration on the Schur normal equations
        if (m.dag == 0 && m.own == 0 && m.epi == EPI_STORE)
            hipLaunchKernelGGL((k_dslash_multi<SS, LS, T, R, 0, 0, EPI_STORE>), g, b, 0, s, a);
        else if (m.dag == 1 && m.own == 0 && m.epi == EPI_STORE)
            hipLaunchKernelGGL((k_dslash_multi<SS, LS, T, R, 1, 0, EPI_STORE>), g, b, 0, s, a);
        else if (m.dag == 0 && m.own == 1 && m.epi == EPI_NORM)
            hipLaunchKernelGGL((k_dslash_multi<SS, LS, T, R, 0, 1, EPI_NORM>), g, b, 0, s, a);
        else if (m.dag == 0 && m.own == 1 && m.epi == EPI_CG)
            hipLaunchKernelGGL((k_dslash_multi<SS, LS, T, R, 0, 1, EPI_CG>), g, b, 0, s, a);
        else
            throw TmError{TM_ERR_UNSUPPORTED, "multi-instance Dslash form not instantiated"};
        TM_HIP(hipGetLastError());
    }
}

template <typename F>
void multi_dispatch(int prec, bool recon12, bool recon8, int R, F &&f)
{
    auto byR = [&](auto *tag) {
        using P3 = std::remove_pointer_t<decltype(tag)>;
        if constexpr (std::is_same<typename P3::T, double>::value) {
            TM_REQUIRE(R == 1, "FP64 uses one right-hand side per thread");
            f.template operator()<typename P3::SS, typename P3::LS, typename P3::T, 1>();
        } else {
            if (R == 3)
                f.template operator()<typename P3::SS, typename P3::LS, typename P3::T, 3>();
            else if (R == 2)
                f.template operator()<typename P3::SS, typename P3::LS, typename P3::T, 2>();
            else
                f.template operator()<typename P3::SS, typename P3::LS, typename P3::T, 1>();
        }
    };
    struct PD { using SS = double2; using LS = double2; using T = double; };
    struct PD12 { using SS = double2; using LS = L12D; using T = double; };
    struct PD8 { using SS = double2; using LS = L8D; using T = double; };
    struct PF { using SS = float2; using LS = float2; using T = float; };
    struct PF12 { using SS = float2; using LS = L12F; using T = float; };
    struct PH { using SS = h2; using LS = h2; using T = float; };
    struct PB { using SS = b2; using LS = h2; using T = float; };
    struct PH12 { using SS = h2; using LS = L12; using T = float; };
    struct PB12 { using SS = b2; using LS = L12; using T = float; };
    switch (prec) {
    case TM_F64:
        if (recon8)
            byR((PD8 *)nullptr);
        else
            recon12 ? byR((PD12 *)nullptr) : byR((PD *)nullptr);
        break;
    case TM_F32: recon12 ? byR((PF12 *)nullptr) : byR((PF *)nullptr); break;
    case TM_F16: recon12 ? byR((PH12 *)nullptr) : byR((PH *)nullptr); break;
    case TM_BF16: recon12 ? byR((PB12 *)nullptr) : byR((PB *)nullptr); break;
    default: throw TmError{TM_ERR_ARG, "bad precision"};
    }
}

template <typename SS, typename LS, typename T, int R>
void persist_fill(PersistBatch &pb, const std::vector<PersistInst> &v, hipStream_t s)
{
    if constexpr (sizeof(T) == 8) {
        throw TmError{TM_ERR_UNSUPPORTED, "the persistent batch kernel takes FP32-arithmetic solvers"};
    } else {
    PersistArgs<T> a{};
    a.n = (int)v.size();
    for (int k = 0; k < a.n; k++) {
        for (int st = 0; st < 4; st++) {
            TM_REQUIRE(v[k].st[st].nrhs % R == 0, "RHS tile must divide every instance's nrhs");
            a.st[st][k] = fill_params<SS, LS, T, R>(v[k].c, v[k].st[st]);
        }
        const int nb = a.st[0][k].nblk * a.st[0][k].ngroups;
        a.start[k + 1] = a.start[k] + (nb + 7) / 8 * 8;
        const size_t n = (size_t)12 * v[k].c->geo.hs;
        a.uchunks[k] = (int)((n + kUpdChunk - 1) / kUpdChunk);
        a.ustart[k + 1] = a.ustart[k] + a.uchunks[k] * v[k].st[0].nrhs;
        a.fstart[k + 1] = a.fstart[k] + v[k].st[0].nrhs;
        a.x[k] = v[k].x;
        a.sc[k] = v[k].sc;
        a.delta[k] = v[k].delta;
    }
    pb.work = std::max(a.start[a.n], a.ustart[a.n]);
    pb.sync_bytes = sizeof(unsigned) * kBarWords;
    pb.bar = ws_get(v[0].c, "persist_sync", pb.sync_bytes);
    a.bar = (unsigned *)pb.bar;
    pb.args_bytes = sizeof(a);
    // the table is rewritten only when no launch that reads it is in flight
    TM_HIP(hipStreamSynchronize(s));
    pb.dev_args = ws_get(v[0].c, "persist_args", sizeof(a));
    TM_HIP(hipMemcpy(pb.dev_args, &a, sizeof(a), hipMemcpyHostToDevice));
    // co-resident blocks of this instantiation: the grid of the cooperative launch
    int per_cu = 0, ncu = 0;
    TM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persist<SS, LS, T, R>, kBlock, 0));
    TM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, v[0].c->device));
    if (pb.blocks_per_cu > 0) per_cu = std::min(per_cu, pb.blocks_per_cu);
    const int cap = per_cu * ncu / 8 * 8;
    TM_REQUIRE(cap >= 8, "the persistent batch kernel does not fit the device");
    pb.grid = std::min(cap, (pb.work + 7) / 8 * 8);
    }
}

template <typename SS, typename LS, typename T, int R>
bool persist_go(const PersistBatch &pb, hipStream_t s)
{
    if constexpr (sizeof(T) == 8) {
        return false;
    } else {
    TM_REQUIRE(pb.args_bytes == sizeof(PersistArgs<T>), "persistent batch arguments of another precision");
    const PersistArgs<T> *pa = (const PersistArgs<T> *)pb.dev_args;
    int iters = pb.iters;
    unsigned long long spin = pb.spin_limit;
    void *kargs[] = {&pa, &iters, &spin};
    if (hipLaunchCooperativeKernel((const void *)k_batch_persist<SS, LS, T, R>, dim3(pb.grid), dim3(kBlock), kargs,
                                   0, s) != hipSuccess) {
        (void)hipGetLastError();  // refused (e.g. the grid cannot be co-resident): nothing was launched
        return false;
    }
    return true;
    }
}

}  // namespace

void multi_dslash_prepare(MultiDslash &m, const std::vector<tm_ctx *> &cs, const std::vector<DslashCall> &dcs, int R,
                          hipStream_t s)
{
    TM_REQUIRE(!cs.empty() && cs.size() == dcs.size(), "bad multi-instance call");
    for (tm_ctx *c : cs)
        if (dcs[0].spinor_prec == TM_F16 || dcs[0].spinor_prec == TM_BF16)
            if (c->half_links_f32)
                throw TmError{TM_ERR_UNSUPPORTED, "batches read binary16 links for FP16/BF16 spinors"};
    m.prec = dcs[0].spinor_prec;
    m.dag = dcs[0].dag;
    m.own = dcs[0].has_own ? 1 : 0;
    m.epi = dcs[0].epi;
    m.R = R;
    m.n = (int)cs.size();
    m.recon8 = false;
    for (size_t k = 0; k < cs.size(); k++) {
        TM_REQUIRE(dcs[k].spinor_prec == m.prec && dcs[k].dag == m.dag && (dcs[k].has_own ? 1 : 0) == m.own &&
                       dcs[k].epi == m.epi,
                   "multi-instance calls must share precision and operator form");
        TM_REQUIRE(cs[k]->have_gauge, "no gauge field set");
        TM_REQUIRE(recon12_ok(cs[k], m.prec) == recon12_ok(cs[0], m.prec),
                   "multi-instance calls must share the link format");
        if (m.prec == TM_F32) {
            if (recon12_ok(cs[k], m.prec))
                ensure_links12f(cs[k], s);
            else
                ensure_links32(cs[k], s);
        }
        if (m.prec == TM_F64) {
            const bool r8 = recon8_wanted(cs[k]) && ensure_links8d(cs[k], s);
            TM_REQUIRE(k == 0 || r8 == m.recon8, "multi-instance calls must share the link format");
            m.recon8 = r8;
            if (!r8 && recon12_ok(cs[k], m.prec)) ensure_links12d(cs[k], s);
        }
        if (m.prec == TM_F16 || m.prec == TM_BF16) {
            if (recon12_ok(cs[k], m.prec))
                ensure_links12(cs[k], s);
            else
                ensure_links16(cs[k], s);
        }
    }
    m.recon12 = recon12_ok(cs[0], m.prec);
    multi_dispatch(m.prec, m.recon12, m.recon8, R,
                   [&]<typename SS, typename LS, typename T, int RR>() { multi_fill<SS, LS, T, RR>(m, cs, dcs); });
}

void multi_dslash_launch(const MultiDslash &m, hipStream_t s)
{
    multi_dispatch(m.prec, m.recon12, m.recon8, m.R,
                   [&]<typename SS, typename LS, typename T, int RR>() { multi_go<SS, LS, T, RR>(m, s); });
}

bool persist_supported(int device)
{
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return coop != 0;
}

void persist_prepare(PersistBatch &pb, const std::vector<PersistInst> &v, int R, hipStream_t s)
{
    TM_REQUIRE(!v.empty() && (int)v.size() <= kPersistInst, "persistent batch: 1 to 4 instances");
    const int prec = v[0].st[0].spinor_prec;
    TM_REQUIRE(prec != TM_F64, "the persistent batch kernel takes FP32-arithmetic solvers");
    tm_ctx *c0 = v[0].c;
    bool recon8 = false;
    for (const auto &q : v) {
        // the link copies the stage forms read (the same choice as the
        // multi-instance launches of the same stages)
        MultiDslash m;
        std::vector<tm_ctx *> cs(1, q.c);
        for (int st = 0; st < 4; st++) {
            TM_REQUIRE(q.st[st].spinor_prec == prec, "batched solves share precision");
            multi_dslash_prepare(m, cs, std::vector<DslashCall>(1, q.st[st]), R, s);
        }
        TM_REQUIRE(recon12_ok(q.c, prec) == recon12_ok(c0, prec), "batched instances must share the link format");
        if (&q == &v[0]) recon8 = m.recon8;
        TM_REQUIRE(m.recon8 == recon8, "batched instances must share the link format");
    }
    pb.prec = prec;
    pb.R = R;
    pb.recon12 = recon12_ok(c0, prec);
    pb.recon8 = recon8;
    multi_dispatch(pb.prec, pb.recon12, pb.recon8, R,
                   [&]<typename SS, typename LS, typename T, int RR>() { persist_fill<SS, LS, T, RR>(pb, v, s); });
}

bool persist_launch(PersistBatch &pb, int iters, unsigned long long spin_limit, hipStream_t s)
{
    TM_REQUIRE(iters >= 1, "iters must be >= 1");
    pb.iters = iters;
    pb.spin_limit = spin_limit;
    // the barrier state starts at zero (a launch that gave up may have left
    // it set)
    TM_HIP(hipMemsetAsync(pb.bar, 0, pb.sync_bytes, s));
    bool ok = false;
    multi_dispatch(pb.prec, pb.recon12, pb.recon8, pb.R,
                   [&]<typename SS, typename LS, typename T, int RR>() { ok = persist_go<SS, LS, T, RR>(pb, s); });
    return ok;
}

bool persist_failed(const PersistBatch &pb, hipStream_t s)
{
    unsigned fail = 0;
    TM_HIP(hipMemcpyAsync(&fail, (const unsigned *)pb.bar + 17 * kBarLine, sizeof(fail), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    return fail != 0;
}

int dslash_site_blocks(tm_ctx *c) { return (c->geo.vh + kBlock - 1) / kBlock; }

void dslash_cost(tm_ctx *c, const DslashCall &dc, double &bytes, double &flops)
{
    const double sites = (double)c->geo.vh, n = dc.nrhs;
    const double sb = 12.0 * prec_bytes(dc.spinor_prec);  // one half-site spinor
    // link entries per site (8 directions) and bytes per complex entry
    double lb;
    const int par = recon12_ok(c, dc.spinor_prec) && !dc.links18 ? 6 : 9;
    switch (dc.spinor_prec) {
    case TM_F64: lb = !dc.links18 && recon8_wanted(c) && c->links8_usable ? 64.0 : 16.0 * par; break;
    case TM_F32: lb = 8.0 * par; break;
    default: lb = c->half_links_f32 ? 8.0 * 9 : 4.0 * par; break;
    }
    double per = 2 * sb;  // input once, output once
    double fl = 1320 + 72;
    if (dc.has_own) {
        per += sb;
        fl += 96;
    }
    if (dc.epi == 1) fl += 48;
    if (dc.epi == 2) {
        per += sb;  // r read; the output is r itself (written once)
        fl += 96;
        if (dc.rho) {
            per += 2 * sb;
            fl += 96;
        }
    }
    bytes = sites * (n * per + 8 * lb);
    flops = sites * n * fl;
}

void launch_dslash(tm_ctx *c, const DslashCall &dc, hipStream_t s)
{
    TM_REQUIRE(c->have_gauge, "no gauge field set");
    {
        double b, f;
        dslash_cost(c, dc, b, f);
        account(c, b, f);
    }
    switch (dc.spinor_prec) {
    // FP64 (the plain solver and the reliable updates): 12-parameter FP64
    // links in the context's format, the third row rebuilt exactly up to rounding
    case TM_F64:
        if (!dc.links18 && recon8_wanted(c) && ensure_links8d(c, s)) {
            launch_rhs<double2, L8D, double>(c, dc, s);
        } else if (recon12_ok(c, TM_F64) && !dc.links18) {
            ensure_links12d(c, s);
            launch_rhs<double2, L12D, double>(c, dc, s);
        } else {
            launch_rhs<double2, double2, double>(c, dc, s);
        }
        break;
    case TM_F32:
        if (recon12_ok(c, TM_F32)) {
            ensure_links12f(c, s);
            launch_rhs<float2, L12F, float>(c, dc, s);
        } else {
            ensure_links32(c, s);
            launch_rhs<float2, float2, float>(c, dc, s);
        }
        break;
    // FP16/BF16 spinors: binary16 links in the context's format (all 18
    // parameters or 12 with the third row rebuilt; the solvers' choice)
    // unless the caller asked for the FP32 copy
    case TM_F16:
        if (c->half_links_f32) {
            ensure_links32(c, s);
            launch_rhs<h2, float2, float>(c, dc, s);
        } else if (recon12_ok(c, TM_F16)) {
            ensure_links12(c, s);
            launch_rhs<h2, L12, float>(c, dc, s);
        } else {
            ensure_links16(c, s);
            launch_rhs<h2, h2, float>(c, dc, s);
        }
        break;
    case TM_BF16:
        if (c->half_links_f32) {
            ensure_links32(c, s);
            launch_rhs<b2, float2, float>(c, dc, s);
        } else if (recon12_ok(c, TM_BF16)) {
            ensure_links12(c, s);
            launch_rhs<b2, L12, float>(c, dc, s);
        } else {
            ensure_links16(c, s);
            launch_rhs<b2, h2, float>(c, dc, s);
        }
        break;
    default: throw TmError{TM_ERR_ARG, "bad spinor precision"};
    }
}
