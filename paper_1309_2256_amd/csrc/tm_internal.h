// Internal definitions of the gfx950 twisted-mass library: complex arithmetic,
// storage precisions, lattice geometry, the context and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "tm.h"

// ---------------------------------------------------------------- errors

struct TmError {
    int status;
    std::string msg;
};

#define TM_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw TmError{TM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define TM_REQUIRE(cond, msg)                                 \
    do {                                                      \
        if (!(cond)) throw TmError{TM_ERR_ARG, (msg)};        \
    } while (0)

// ---------------------------------------------------------------- complex

template <typename T>
struct cx {
    T r, i;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> cmk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
// a * i
template <typename T>
__host__ __device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.r, -a.i}; }
// acc += a * b
template <typename T>
__host__ __device__ __forceinline__ void cmac(cx<T> &acc, cx<T> a, cx<T> b)
{
    acc.r = fma(a.r, b.r, acc.r);
    acc.r = fma(-a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i);
    acc.i = fma(a.i, b.r, acc.i);
}
// acc += conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ void cmac_conj(cx<T> &acc, cx<T> a, cx<T> b)
{
    acc.r = fma(a.r, b.r, acc.r);
    acc.r = fma(a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i);
    acc.i = fma(-a.i, b.r, acc.i);
}

// ---------------------------------------------------------------- storage types

// IEEE binary16 pair and bfloat16 pair, 4 bytes per complex value.
// tag types of the 12-parameter link formats (Dslash template argument):
// binary16 rows and FP64 rows
struct L12 {};
struct L12D {};
struct L12F {};
// 8-parameter FP64 links (appendix A.1): [8 directions][4][vh] double2
struct L8D {};

struct alignas(4) h2 {
    _Float16 x, y;
};
struct alignas(4) b2 {
    uint16_t x, y;
};

__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t v)
{
    union { uint32_t u; float f; } c;
    c.u = ((uint32_t)v) << 16;
    return c.f;
}
// round to nearest even; NaN stays NaN
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    union { uint32_t u; float f; } c;
    c.f = f;
    if ((c.u & 0x7f800000u) == 0x7f800000u && (c.u & 0x007fffffu)) return (uint16_t)((c.u >> 16) | 0x40);
    uint32_t lsb = (c.u >> 16) & 1u;
    c.u += 0x7fffu + lsb;
    return (uint16_t)(c.u >> 16);
}

template <typename S>
struct StoreTraits;
template <>
struct StoreTraits<double2> {
    using real = double;
    __device__ __forceinline__ static cx<double> ld(const double2 *p, size_t k)
    {
        double2 v = p[k];
        return {v.x, v.y};
    }
    __device__ __forceinline__ static void st(double2 *p, size_t k, cx<double> v) { p[k] = make_double2(v.r, v.i); }
};
template <>
struct StoreTraits<float2> {
    using real = float;
    __device__ __forceinline__ static cx<float> ld(const float2 *p, size_t k)
    {
        float2 v = p[k];
        return {v.x, v.y};
    }
    __device__ __forceinline__ static void st(float2 *p, size_t k, cx<float> v) { p[k] = make_float2(v.r, v.i); }
};
template <>
struct StoreTraits<h2> {
    using real = float;
    __device__ __forceinline__ static cx<float> ld(const h2 *p, size_t k)
    {
        h2 v = p[k];
        return {(float)v.x, (float)v.y};
    }
    __device__ __forceinline__ static void st(h2 *p, size_t k, cx<float> v)
    {
        h2 o;
        o.x = (_Float16)v.r;
        o.y = (_Float16)v.i;
        p[k] = o;
    }
};
template <>
struct StoreTraits<b2> {
    using real = float;
    __device__ __forceinline__ static cx<float> ld(const b2 *p, size_t k)
    {
        b2 v = p[k];
        return {bf16_to_f32(v.x), bf16_to_f32(v.y)};
    }
    __device__ __forceinline__ static void st(b2 *p, size_t k, cx<float> v)
    {
        b2 o;
        o.x = f32_to_bf16(v.r);
        o.y = f32_to_bf16(v.i);
        p[k] = o;
    }
};

// load a complex of storage S converted to arithmetic type T
template <typename T, typename S>
__device__ __forceinline__ cx<T> ldT(const S *p, size_t k)
{
    auto v = StoreTraits<S>::ld(p, k);
    return {(T)v.r, (T)v.i};
}
template <typename T, typename S>
__device__ __forceinline__ void stT(S *p, size_t k, cx<T> v)
{
    if constexpr (std::is_same<S, h2>::value && std::is_same<T, double>::value) {
        // one rounding FP64 -> binary16 (not through FP32, whose rounding
        // could move a value onto a binary16 tie)
        h2 o;
        o.x = (_Float16)v.r;
        o.y = (_Float16)v.i;
        p[k] = o;
    } else {
        using R = typename StoreTraits<S>::real;
        StoreTraits<S>::st(p, k, cx<R>{(R)v.r, (R)v.i});
    }
}

static inline size_t prec_bytes(int prec)
{
    switch (prec) {
    case TM_F64: return 16;
    case TM_F32: return 8;
    case TM_F16: return 4;
    case TM_BF16: return 4;
    }
    return 0;
}

// ---------------------------------------------------------------- geometry

// Lattice geometry for kernels (passed by value).  Half-site index i of parity
// p is s >> 1 with s = x + Lx*(y + Ly*(z + Lz*t)); the row q = y + Ly*(z + Lz*t)
// gives i = (x >> 1) + (Lx/2) * q.
struct Geo {
    int L[4];
    int lxh;   // Lx / 2
    int vh;    // V / 2
    int vsh;   // half-sites per time slice, Lx*Ly*Lz / 2
    int hs;    // plane stride of half-site fields (sites), see half_stride
};

// Half-site fields are stored [rhs][spin*3 + colour][hs] with hs >= vh; the
// hs - vh pad sites at the end of every plane are never read for a result
// (their contents are unspecified).  hs is vh rounded up to an odd multiple
// of 32 sites: with a power-of-two plane stride the 12 planes of a site (and
// the right-hand sides of a thread) fall on the same cache sets and memory
// channels, and the neighbour gathers of the hopping kernel lose ~7% of
// their bandwidth to the conflicts.
inline int half_stride(int vh)
{
    int q = (vh + 31) / 32;
    if (q % 2 == 0) q++;
    return 32 * q;
}

__device__ __forceinline__ void eo_coords(const Geo &g, int p, int i, int &x, int &y, int &z, int &t)
{
    int q = i / g.lxh;
    int xh = i - q * g.lxh;
    y = q % g.L[1];
    int q2 = q / g.L[1];
    z = q2 % g.L[2];
    t = q2 / g.L[2];
    x = 2 * xh + ((p ^ (y + z + t)) & 1);
}

__device__ __forceinline__ int eo_index(const Geo &g, int x, int y, int z, int t)
{
    return (x >> 1) + g.lxh * (y + g.L[1] * (z + g.L[2] * t));
}

// Logical block index with contiguous chunks of blocks on each of the 8 XCDs:
// hardware dispatches consecutive workgroups round-robin over the XCDs, so
// block b runs on XCD b % 8; mapping it to chunk (b % 8) keeps lattice
// neighbours (nearby half-site indices) inside one XCD's L2.
__host__ __device__ __forceinline__ int xcd_block(int b, int nblk)
{
    // XCD k receives hardware blocks k, k+8, ...: base + (k < rem) of them
    int base = nblk >> 3, rem = nblk & 7;
    int k = b & 7, m = b >> 3;
    return k * base + (k < rem ? k : rem) + m;
}

// ---------------------------------------------------------------- context

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct tm_ctx {
    int device = 0;
    tm_lattice lat{};
    Geo geo{};
    long V = 0;
    double kappa = 0, eps = 0;
    int t_bc = -1;
    // internal links per parity of the output site: [8 directions][9][vh]
    // direction d < 4: U_d(x) (forward hop); d >= 4: U_{d-4}(x - d)^dag
    // (backward hop), boundary phase folded in
    void *links64[2] = {nullptr, nullptr};
    void *links32[2] = {nullptr, nullptr};
    void *links16[2] = {nullptr, nullptr};  // IEEE binary16 copy (FP16/BF16 spinors)
    // binary16 12-parameter copy: the first two rows, [8 directions][6][vh]
    void *links12[2] = {nullptr, nullptr};
    // FP64 and FP32 12-parameter copies, same layout
    void *links12d[2] = {nullptr, nullptr};
    void *links12f[2] = {nullptr, nullptr};
    // FP64 8-parameter copy (a2, a3, b1 or -c1, phases; see misc.hip), [8][4][vh]
    void *links8d[2] = {nullptr, nullptr};
    bool have_gauge = false;
    bool have_links32 = false;
    bool have_links16 = false;
    bool have_links12 = false;
    bool have_links12d = false;
    bool have_links12f = false;
    bool have_links8d = false;
    // the 8-parameter copy was built and every link's first row has
    // |a2|^2 + |a3|^2 >= kRecon8MinN (the reconstruction divides by it)
    bool links8_usable = false;
    // binary16 link format of the FP16/BF16-spinor kernels: 18 or 12
    // parameters (12 reads a third fewer link bytes; measured no slower at 12
    // RHS and 9-24% faster at 1-4 RHS per call)
    int link_recon = 12;
    // largest deviation of the gauge field from SU(3) measured at ingest,
    // max over links of max(|U U^dag - 1|, |det U - 1|) entrywise; the
    // 12-parameter format of a precision is used only while this stays
    // below that precision's rounding scale (recon12_ok)
    double su3_dev = 0;
    // FP16/BF16-spinor Dslash launches read the FP32 links instead of the
    // binary16 copy (set by tm_dslash for link_prec = TM_F32)
    bool half_links_f32 = false;
    // links of the FP16/BF16-spinor kernels when no call overrides them
    // (tm_set_half_spinor_links): false = binary16 copy, true = FP32 (18)
    bool half_links_f32_default = false;
    std::map<std::string, DevBuf> ws;
    // autotuned right-hand sides per Dslash thread, keyed by (precision, nrhs)
    std::map<std::pair<int, int>, int> rhs_tile;
    std::string err;
    hipStream_t stream = nullptr;  // stream of the current loop-driver call
    // pinned host staging for scalar read-back
    void *host_pinned = nullptr;
    size_t host_pinned_bytes = 0;
    void *host_up = nullptr;  // pinned slots of asynchronous uploads (host_upload_slot)
    size_t host_up_bytes = 0;
    // learned preconditioner (ptc.hip): channel count (0 = no weights),
    // Adam step counter, training-pair store (capacity, count, precision)
    int ptc_nc = 0;
    // network arithmetic: TM_F32 (VALU, FP32 weights) or TM_BF16 (spin mixing
    // on the matrix cores, BF16 weights and activations, FP32 accumulation)
    int ptc_arith = TM_F32;
    long ptc_step = 0;
    int ptc_cap = 0, ptc_n = 0, ptc_store = TM_F32;
    // algorithmic work of the kernels launched on this context so far
    // (compulsory device-memory bytes and flops by the conventions of tm.h);
    // acct_pause > 0 while launches are recorded into a graph that is
    // accounted per replay instead
    double acct_bytes = 0, acct_flops = 0;
    int acct_pause = 0;
    // set for the duration of an allocation-free call: ws_get refuses to
    // allocate and the Dslash tile tuner is not run
    bool no_alloc = false;
};

// 12-parameter links for kernels of spinor precision prec: the format asks
// for 12 (or 8, which the FP64 kernels alone read, the others taking 12)
// and the links are special unitary to that precision's rounding (the third
// row is rebuilt from the first two assuming U in SU(3))
inline bool recon12_ok(const tm_ctx *c, int prec)
{
    if (c->link_recon != 12 && c->link_recon != 8) return false;
    const double lim = prec == TM_F64 ? 1e-12 : prec == TM_F32 ? 1e-6 : 1e-3;
    return c->su3_dev <= lim;
}

// smallest |a2|^2 + |a3|^2 (over the links) with which the 8-parameter form
// is used; fields with a link closer to diagonal (unit links) keep 12
constexpr double kRecon8MinN = 1e-10;

// the FP64 kernels read 8-parameter links: asked for, special unitary to
// FP64 rounding; links8_usable is settled when the copy is built
inline bool recon8_wanted(const tm_ctx *c) { return c->link_recon == 8 && c->su3_dev <= 1e-12; }

inline void account(tm_ctx *c, double bytes, double flops)
{
    if (c->acct_pause) return;
    c->acct_bytes += bytes;
    c->acct_flops += flops;
}

void *ws_get(tm_ctx *c, const std::string &name, size_t bytes);
void *host_stage(tm_ctx *c, size_t bytes);
// Pinned staging slot `slot` (< kUpSlots) of `bytes` for an asynchronous
// upload on stream s.  A slot's previous copy must have completed before it
// is reused (the callers synchronise the stream in between).
constexpr int kUpSlots = 4;
void *host_upload_slot(tm_ctx *c, int slot, size_t bytes, hipStream_t s);
void ensure_links32(tm_ctx *c, hipStream_t s);
void ensure_links16(tm_ctx *c, hipStream_t s);
void ensure_links12(tm_ctx *c, hipStream_t s);
void ensure_links12d(tm_ctx *c, hipStream_t s);
// builds the 8-parameter copy if needed; true when the FP64 kernels use it
bool ensure_links8d(tm_ctx *c, hipStream_t s);
void ensure_links12f(tm_ctx *c, hipStream_t s);

// ---------------------------------------------------------------- dslash

// spin-diagonal operator: diag(u, u, l, l) in the chiral basis (R(eps),
// R^-1, gamma5 and their products are all of this form)
struct SpinDiag {
    cx<double> u, l;
};

static inline SpinDiag sd_scalar(double a) { return {{a, 0}, {a, 0}}; }
static inline SpinDiag sd_mul(SpinDiag a, SpinDiag b) { return {a.u * b.u, a.l * b.l}; }
static inline SpinDiag sd_twist(double eps)  // R = 1 + i eps gamma5
{
    return {{1.0, eps}, {1.0, -eps}};
}
static inline SpinDiag sd_twist_inv(double eps)  // R^-1 = (1 - i eps gamma5)/(1 + eps^2)
{
    double d = 1.0 / (1.0 + eps * eps);
    return {{d, -eps * d}, {d, eps * d}};
}
static inline SpinDiag sd_gamma5() { return {{1.0, 0}, {-1.0, 0}}; }

// out(x) = D_own own(x) + D_hop (Hop[in])(x),
// x over the half sites of parity out_parity; Hop is the hopping sum without
// the -kappa factor (fold it into D_hop).  dag selects the adjoint projector
// placement ((1+gamma) forward, (1-gamma) backward), i.e. Hop^dag.
struct DslashCall {
    void *out;
    const void *in;
    const void *own;  // may be null when D_own = 0
    int nrhs;
    int out_parity;
    int dag;
    int spinor_prec;  // TM_F64 with FP64 links, else FP32 links
    SpinDiag d_own, d_hop;
    bool has_own;
    // fused epilogue (0 store, 1 store + partial |out|^2, 2 CG update of r and
    // rho with partial |r|^2, |rho|^2; see dslash.hip)
    int epi = 0;
    void *r = nullptr, *rho = nullptr;
    const struct CGScalars *sc = nullptr;
    double *part = nullptr;  // [quantity][nrhs][dslash_site_blocks]
    // FP64 only: read all 18 parameters of the FP64 links whatever the
    // format (the exact operator for reliable updates and true residuals)
    bool links18 = false;
};

void launch_dslash(tm_ctx *c, const DslashCall &dc, hipStream_t s);
int dslash_site_blocks(tm_ctx *c);
// algorithmic bytes (each field and link read once, each output written
// once) and flops (1320 per site and RHS for the hopping term, 72 for its
// spin-diagonal coefficient, 96 for the own-site term, 48 per fused norm or
// update) of one launch of dc on this context's link format
void dslash_cost(tm_ctx *c, const DslashCall &dc, double &bytes, double &flops);

// One launch over several contexts (lattices), one DslashCall each; all
// share precision and operator form; R right-hand sides per thread divides
// every nrhs.  prepare() builds the launch arguments on the host;
// launch() is one kernel launch per chunk of instances (capturable).
struct MultiDslash {
    // per chunk of at most kMultiInst instances: the kernel-argument block
    // (instance records + block offsets) and the grid it covers
    std::vector<std::vector<unsigned char>> args;
    std::vector<int> grid;
    int prec = 0, dag = 0, own = 0, epi = 0, R = 1, n = 0;
    bool recon12 = false;  // links in the 12-parameter format
    bool recon8 = false;   // FP64 links in the 8-parameter format
};
constexpr int kMultiInst = 16;  // instances per launch (kernel-argument space)
void multi_dslash_prepare(MultiDslash &m, const std::vector<tm_ctx *> &cs, const std::vector<DslashCall> &dcs, int R,
                          hipStream_t s);
void multi_dslash_launch(const MultiDslash &m, hipStream_t s);

// Persistent batch: `iters` CG iterations of up to kPersistInst instances in
// one cooperative launch (grid barriers between the stages, bounded waits);
// solvers with FP32 arithmetic (FP32, FP16 or BF16 storage) only.
constexpr int kPersistInst = 4;
struct PersistInst {
    tm_ctx *c = nullptr;
    DslashCall st[4];       // the four stage forms of one CG iteration
    void *x = nullptr;      // solution accumulator of the update
    CGScalars *sc = nullptr;
    double delta = 0;       // reliable-update threshold (0: none)
};
struct PersistBatch {
    void *dev_args = nullptr;          // launch parameters (device, owned by the first context)
    size_t args_bytes = 0, sync_bytes = 0;
    int grid = 0, work = 0, iters = 0;
    int blocks_per_cu = 0;             // cap on resident blocks per CU (0: as many as fit)
    int prec = 0, R = 1;
    bool recon12 = false, recon8 = false;
    void *bar = nullptr;               // barrier state (device)
    unsigned long long spin_limit = 0;
};
bool persist_supported(int device);
void persist_prepare(PersistBatch &pb, const std::vector<PersistInst> &v, int R, hipStream_t s);
// false if the runtime refused the cooperative launch (nothing launched)
bool persist_launch(PersistBatch &pb, int iters, unsigned long long spin_limit, hipStream_t s);
// reads the barrier state (synchronises the stream): true if a wait gave up
bool persist_failed(const PersistBatch &pb, hipStream_t s);

// ---------------------------------------------------------------- blas

// All vectors: half layout [nrhs][12][hs] of the given precision.
// Per-RHS scalars live in device memory (double).
void launch_spin_diag(tm_ctx *c, void *out, const void *in, int prec, int nrhs, SpinDiag d,
                      hipStream_t s);
void launch_copy_convert(tm_ctx *c, void *out, int out_prec, const void *in, int in_prec, int nrhs,
                         const double *dscale /* device per-rhs or null */, hipStream_t s);
// y = a*x + b*y with host scalars (same prec)
void launch_axpby_host(tm_ctx *c, void *y, const void *x, int prec, int nrhs, double a, double b,
                       hipStream_t s);
// out = a x + b y (x, y, out distinct or out == y)
void launch_axpby_to_host(tm_ctx *c, void *out, const void *x, const void *y, int prec, int nrhs, double a,
                          double b, hipStream_t s);
void launch_zero(tm_ctx *c, void *y, int prec, int nrhs, hipStream_t s);
// y[r] += a_dev[r] * x[r]
void launch_axpy_dev(tm_ctx *c, void *y, int yprec, const void *x, int xprec, int nrhs, const double *a_dev,
                     hipStream_t s);
// per-rhs |v|^2 into dev_out[nrhs] (device doubles), deterministic
void launch_norm2(tm_ctx *c, const void *v, int prec, int nrhs, double *dev_out, hipStream_t s);

// CG building blocks (blas.hip; the iteration itself is in runtime.hip)
struct CGScalars {
    double rr;       // |r|^2 (normal residual)
    double qq;       // |Ahat p|^2
    double alpha, beta;
    double rho2;     // |rho|^2, iterated Schur residual
    double rho2_ref; // |rho|^2 at the last reliable update
    double target2;  // (tol |b|)^2 in the units of the vectors
    double sigma;    // scale of the low-precision vectors (MIXED/LOW)
    int active;
    int iters;
    int want_update; // reliable update requested
    int bad;         // NaN/Inf seen
};

void cg_finish_alpha(tm_ctx *c, CGScalars *sc, const double *part, int nblk, int nrhs, hipStream_t s);
void cg_finish_beta(tm_ctx *c, CGScalars *sc, const double *part, int nblk, int nrhs, double delta,
                    hipStream_t s);
// x += alpha p; p = r + beta p
void cg_update_px(tm_ctx *c, void *p, const void *r, void *x, int prec, int xprec, int nrhs, const CGScalars *sc,
                  hipStream_t s);

// The same scalar and vector steps for several lattices in one launch each
// (a batch's iteration): per lattice its context, CG scalars, partial sums
// and fields; all share prec and xprec.  Bit-identical to the per-lattice
// launches (the same device code per right-hand side and element).
struct CgTail {
    tm_ctx *c;
    CGScalars *sc;
    const double *partq;  // |q|^2 partials (alpha)
    const double *partb;  // |r|^2 (and |rho|^2) partials (beta)
    int nblk;             // partial-sum blocks
    int nrhs;
    double delta;
    void *p;
    const void *r;
    void *x;
};
void cg_finish_alpha_multi(const std::vector<CgTail> &t, hipStream_t s);
void cg_tail_multi(const std::vector<CgTail> &t, int prec, int xprec, hipStream_t s);  // beta, then x and p

// ---------------------------------------------------------------- misc kernels

void launch_pack(tm_ctx *c, void *even, void *odd, const double *full, int nrhs, int prec,
                 const double *dscale, hipStream_t s);
void launch_unpack(tm_ctx *c, double *full, const void *even, const void *odd, int nrhs, int prec,
                   hipStream_t s);
void launch_gauge_ingest(tm_ctx *c, const double *U, hipStream_t s);
// max over the 4V links of the canonical field U (device) of
// max(|U U^dag - 1|, |det U - 1|) entrywise; synchronises s
double gauge_su3_deviation(tm_ctx *c, const double *U, hipStream_t s);
void launch_links_to_f32(tm_ctx *c, hipStream_t s);
void launch_links_to_f16(tm_ctx *c, hipStream_t s);
// first two rows of every link, rounded once to binary16: [8][6][vh] per parity
void launch_links_to_r12(tm_ctx *c, hipStream_t s);
// first two rows of every link in FP64: [8][6][vh] per parity
void launch_links_to_r12d(tm_ctx *c, hipStream_t s);
// builds links8d for both parities; returns the smallest |a2|^2 + |a3|^2
double launch_links_to_r8d(tm_ctx *c, hipStream_t s);
// first two rows of every link rounded once to FP32: [8][6][vh] per parity
void launch_links_to_r12f(tm_ctx *c, hipStream_t s);
// Z4 noise for noise index r into FP64 half fields: n_off x (12 with
// spin-colour dilution, else 1) RHS; with t_period > 0 RHS group q keeps the
// slices t = o_first + q (mod t_period) only (time dilution, coherent when
// t_period < Lt)
void launch_noise(tm_ctx *c, void *even, void *odd, uint64_t seed, long r, int dilution, hipStream_t s,
                  int t_period = 0, int o_first = 0, int n_off = 1);
// per time slice 4x4 colour-traced outer products C[b][a](t) = sum_x sum_c v_{bc} w*_{ac}
// accumulated over nrhs pairs and both parities, FP64; out device [Lt][16] complex.
// Only the slices t0, t0 + dt, ... are computed; the others are zero.
void launch_outer_slices(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo,
                         int nrhs, double *dev_out /* [Lt][16][2] */, hipStream_t s, int t0 = 0, int dt = 1);
