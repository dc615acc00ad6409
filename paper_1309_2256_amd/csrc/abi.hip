// C-ABI entry points (declared in include/tm.h).  Every function validates its
// arguments before launching, converts internal errors to tm_status codes and
// records a message retrievable with tm_last_error.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "runtime.h"

// ---------------------------------------------------------------- context helpers

void *ws_get(tm_ctx *c, const std::string &name, size_t bytes)
{
    if (c->no_alloc) {
        auto it = c->ws.find(name);
        if (it != c->ws.end() && it->second.p && it->second.bytes >= bytes) return it->second.p;
        throw TmError{TM_ERR_UNSUPPORTED, "the allocation-free call would allocate " + std::to_string(bytes) +
                                              " bytes of device memory (" + name +
                                              "); one allocating call with the same precisions builds it"};
    }
    DevBuf &b = c->ws[name];
    if (b.p && b.bytes >= bytes) return b.p;
    if (b.p) {
        TM_HIP(hipDeviceSynchronize());
        TM_HIP(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        throw TmError{TM_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed (" + name + ")"};
    }
    b.p = p;
    b.bytes = bytes;
    return p;
}

void *host_stage(tm_ctx *c, size_t bytes)
{
    if (c->host_pinned && c->host_pinned_bytes >= bytes) return c->host_pinned;
    if (c->host_pinned) TM_HIP(hipHostFree(c->host_pinned));
    c->host_pinned = nullptr;
    size_t n = bytes < 4096 ? 4096 : bytes;
    TM_HIP(hipHostMalloc(&c->host_pinned, n, hipHostMallocDefault));
    c->host_pinned_bytes = n;
    return c->host_pinned;
}

void *host_upload_slot(tm_ctx *c, int slot, size_t bytes, hipStream_t s)
{
    TM_REQUIRE(slot >= 0 && slot < kUpSlots, "bad upload slot");
    const size_t per = (bytes + 255) / 256 * 256;
    if (!c->host_up || c->host_up_bytes < per * kUpSlots) {
        if (c->host_up) {
            TM_HIP(hipStreamSynchronize(s));  // copies from the old slots have completed
            TM_HIP(hipHostFree(c->host_up));
        }
        c->host_up = nullptr;
        const size_t n = std::max<size_t>(per, 1024) * kUpSlots;
        TM_HIP(hipHostMalloc(&c->host_up, n, hipHostMallocDefault));
        c->host_up_bytes = n;
    }
    return (char *)c->host_up + (size_t)slot * (c->host_up_bytes / kUpSlots);
}

void ensure_links32(tm_ctx *c, hipStream_t s)
{
    if (c->have_links32) return;
    for (int p = 0; p < 2; p++)
        if (!c->links32[p]) c->links32[p] = ws_get(c, p ? "links32_1" : "links32_0", (size_t)72 * c->geo.vh * 8);
    launch_links_to_f32(c, s);
    c->have_links32 = true;
}

void ensure_links16(tm_ctx *c, hipStream_t s)
{
    if (c->have_links16) return;
    for (int p = 0; p < 2; p++)
        if (!c->links16[p]) c->links16[p] = ws_get(c, p ? "links16_1" : "links16_0", (size_t)72 * c->geo.vh * 4);
    launch_links_to_f16(c, s);
    c->have_links16 = true;
}

void ensure_links12(tm_ctx *c, hipStream_t s)
{
    if (c->have_links12) return;
    for (int p = 0; p < 2; p++)
        if (!c->links12[p]) c->links12[p] = ws_get(c, p ? "links12_1" : "links12_0", (size_t)48 * c->geo.vh * 4);
    launch_links_to_r12(c, s);
    c->have_links12 = true;
}

void ensure_links12d(tm_ctx *c, hipStream_t s)
{
    if (c->have_links12d) return;
    for (int p = 0; p < 2; p++)
        if (!c->links12d[p]) c->links12d[p] = ws_get(c, p ? "links12d_1" : "links12d_0", (size_t)48 * c->geo.vh * 16);
    launch_links_to_r12d(c, s);
    c->have_links12d = true;
}

bool ensure_links8d(tm_ctx *c, hipStream_t s)
{
    if (!recon8_wanted(c)) return false;
    if (c->have_links8d) return c->links8_usable;
    for (int p = 0; p < 2; p++)
        if (!c->links8d[p]) c->links8d[p] = ws_get(c, p ? "links8d_1" : "links8d_0", (size_t)32 * c->geo.vh * 16);
    c->links8_usable = launch_links_to_r8d(c, s) >= kRecon8MinN;
    c->have_links8d = true;
    return c->links8_usable;
}

void ensure_links12f(tm_ctx *c, hipStream_t s)
{
    if (c->have_links12f) return;
    for (int p = 0; p < 2; p++)
        if (!c->links12f[p]) c->links12f[p] = ws_get(c, p ? "links12f_1" : "links12f_0", (size_t)48 * c->geo.vh * 8);
    launch_links_to_r12f(c, s);
    c->have_links12f = true;
}

namespace {

template <typename F>
int guarded(tm_ctx *c, F &&f)
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

size_t half_bytes(tm_ctx *c, int prec, int nrhs) { return prec_bytes(prec) * 12 * (size_t)c->geo.hs * nrhs; }

bool valid_prec(int p) { return p == TM_F64 || p == TM_F32 || p == TM_F16 || p == TM_BF16; }

}  // namespace

// ---------------------------------------------------------------- lifecycle

extern "C" int tm_create(tm_ctx **out, const tm_lattice *lat, int device)
{
    if (!out || !lat) return TM_ERR_ARG;
    *out = nullptr;
    long V = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (lat->L[mu] < 2 || (lat->L[mu] & 1)) return TM_ERR_ARG;
        V *= lat->L[mu];
    }
    if (V / 2 > (1L << 30)) return TM_ERR_ARG;
    // the kernels address one right-hand side of a half field with 32-bit
    // byte offsets (FP64: 12 complex of 16 bytes per half-site)
    if ((long)half_stride((int)(V / 2)) * 12L * 16L > 0x7fffffffL) return TM_ERR_UNSUPPORTED;
    if (!std::isfinite(lat->kappa) || !std::isfinite(lat->two_kappa_mu)) return TM_ERR_ARG;
    if (lat->t_bc != 1 && lat->t_bc != -1) return TM_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TM_ERR_HIP;
    // device address of the allocation-free entry points' scratch (once per device)
    if (noalloc_setup(device) != TM_OK) return TM_ERR_HIP;
    tm_ctx *c = new (std::nothrow) tm_ctx();
    if (!c) return TM_ERR_OOM;
    c->device = device;
    c->lat = *lat;
    for (int mu = 0; mu < 4; mu++) c->geo.L[mu] = lat->L[mu];
    c->V = V;
    c->geo.lxh = lat->L[0] / 2;
    c->geo.vh = (int)(V / 2);
    c->geo.vsh = lat->L[0] * lat->L[1] * lat->L[2] / 2;
    c->geo.hs = half_stride(c->geo.vh);
    c->kappa = lat->kappa;
    c->eps = lat->two_kappa_mu;
    c->t_bc = lat->t_bc;
    *out = c;
    return TM_OK;
}

extern "C" void tm_destroy(tm_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->ws)
        if (kv.second.p) (void)hipFree(kv.second.p);
    for (int p = 0; p < 2; p++)
        if (c->links64[p]) (void)hipFree(c->links64[p]);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    if (c->host_up) (void)hipHostFree(c->host_up);
    delete c;
}

extern "C" const char *tm_last_error(const tm_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" int tm_half_stride(const tm_ctx *c) { return c ? c->geo.hs : 0; }

extern "C" int tm_set_gauge(tm_ctx *c, const double *U, tm_stream stream)
{
    return guarded(c, [&]() {
        TM_REQUIRE(U != nullptr, "null gauge field");
        for (int p = 0; p < 2; p++)
            if (!c->links64[p]) {
                void *q = nullptr;
                if (hipMalloc(&q, (size_t)72 * c->geo.vh * 16) != hipSuccess) {
                    (void)hipGetLastError();
                    throw TmError{TM_ERR_OOM, "link allocation failed"};
                }
                c->links64[p] = q;
            }
        launch_gauge_ingest(c, U, hs(stream));
        c->su3_dev = gauge_su3_deviation(c, U, hs(stream));
        c->have_gauge = true;
        c->have_links32 = false;
        c->have_links16 = false;
        c->have_links12 = false;
        c->have_links12d = false;
        c->have_links8d = false;
        c->links8_usable = false;
        c->have_links12f = false;
        return TM_OK;
    });
}

// ---------------------------------------------------------------- dslash

extern "C" int tm_set_half_spinor_links(tm_ctx *c, int link_prec)
{
    return guarded(c, [&]() {
        TM_REQUIRE(link_prec == TM_F16 || link_prec == TM_F32, "link precision must be TM_F16 or TM_F32");
        c->half_links_f32_default = link_prec == TM_F32;
        c->half_links_f32 = c->half_links_f32_default;
        return TM_OK;
    });
}

extern "C" int tm_set_link_format(tm_ctx *c, int params)
{
    return guarded(c, [&]() {
        TM_REQUIRE(params == 18 || params == 12 || params == 8, "link format must be 18, 12 or 8 parameters");
        c->link_recon = params;
        return TM_OK;
    });
}

namespace {

// Body of tm_dslash and tm_dslash_noalloc.  tmp(name, bytes) supplies the
// intermediate half fields; every one is requested before the first launch,
// so a request that cannot be met fails before anything is enqueued.
template <typename Tmp>
int dslash_body(tm_ctx *c, void *out, const void *in, int nrhs, int kind, int mu_sign, int spinor_prec,
                int link_prec, tm_stream stream, Tmp &&tmp)
{
    TM_REQUIRE(out && in && out != in, "out and in must be distinct non-null pointers");
    TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    TM_REQUIRE(mu_sign == 1 || mu_sign == -1, "mu_sign must be +1 or -1");
    TM_REQUIRE(valid_prec(spinor_prec), "bad spinor precision");
    TM_REQUIRE(c->have_gauge, "no gauge field set");
    if (spinor_prec == TM_F64)
        TM_REQUIRE(link_prec == TM_F64, "FP64 spinors need FP64 links");
    else if (spinor_prec == TM_F32)
        TM_REQUIRE(link_prec == TM_F32, "FP32 spinors use FP32 links");
    else
        TM_REQUIRE(link_prec == TM_F32 || link_prec == TM_F16, "FP16/BF16 spinors use FP16 or FP32 links");
    // the link copy for this call only (solvers use the binary16 copy)
    struct LinkChoice {
        tm_ctx *c;
        ~LinkChoice() { c->half_links_f32 = c->half_links_f32_default; }
    } restore{c};
    c->half_links_f32 = link_prec == TM_F32;
    hipStream_t s = hs(stream);
    const double epsp = eps_of(c, mu_sign), k = c->kappa;
    switch (kind) {
    case TM_HOP_EO:
    case TM_HOP_OE:
        op_dslash(c, out, in, nullptr, nrhs, spinor_prec, kind == TM_HOP_OE, 0, sd_scalar(-k), sd_scalar(0), s);
        break;
    case TM_RINV_HOP_OE:
    case TM_RINV_HOP_EO:
        op_dslash(c, out, in, nullptr, nrhs, spinor_prec, kind == TM_RINV_HOP_OE, 0,
                  sd_mul(sd_scalar(-k), sd_twist_inv(epsp)), sd_scalar(0), s);
        break;
    case TM_SCHUR:
        op_schur(c, out, in, tmp("d_tmp", half_bytes(c, spinor_prec, nrhs)), nrhs, spinor_prec, epsp, s);
        break;
    case TM_SCHUR_DAG:
        op_schur_dag(c, out, in, tmp("d_tmp", half_bytes(c, spinor_prec, nrhs)), nrhs, spinor_prec, epsp, s);
        break;
    case TM_NORMAL: {
        void *t = tmp("d_tmp", half_bytes(c, spinor_prec, nrhs));
        void *mid = tmp("d_mid", half_bytes(c, spinor_prec, nrhs));
        op_schur(c, mid, in, t, nrhs, spinor_prec, epsp, s);
        op_schur_dag(c, out, mid, t, nrhs, spinor_prec, epsp, s);
        break;
    }
    case TM_FULL:
    case TM_FULL_DAG: {
        TM_REQUIRE(spinor_prec == TM_F64, "full-lattice kinds take canonical FP64 spinors");
        const size_t b = half_bytes(c, TM_F64, nrhs);
        void *ie = tmp("d_ie", b), *io = tmp("d_io", b);
        void *oe = tmp("d_oe", b), *oo = tmp("d_oo", b);
        launch_pack(c, ie, io, (const double *)in, nrhs, TM_F64, nullptr, s);
        const int dag = kind == TM_FULL_DAG;
        // M = R(eps) + H;  M^dag = R(-eps) + H^dag
        const SpinDiag tw = sd_twist(dag ? -epsp : epsp);
        op_dslash(c, oe, io, ie, nrhs, TM_F64, 0, dag, sd_scalar(-k), tw, s);
        op_dslash(c, oo, ie, io, nrhs, TM_F64, 1, dag, sd_scalar(-k), tw, s);
        launch_unpack(c, (double *)out, oe, oo, nrhs, TM_F64, s);
        break;
    }
    default: throw TmError{TM_ERR_ARG, "unknown dslash kind"};
    }
    return TM_OK;
}

}  // namespace

extern "C" int tm_dslash(tm_ctx *c, void *out, const void *in, int nrhs, int kind, int mu_sign, int spinor_prec,
                         int link_prec, tm_stream stream)
{
    return guarded(c, [&]() {
        return dslash_body(c, out, in, nrhs, kind, mu_sign, spinor_prec, link_prec, stream,
                           [&](const char *name, size_t bytes) { return ws_get(c, name, bytes); });
    });
}

extern "C" int tm_dslash_noalloc(tm_ctx *c, void *out, const void *in, int nrhs, int kind, int mu_sign,
                                 int spinor_prec, int link_prec, tm_stream stream)
{
    return guarded(c, [&]() {
        char *base = (char *)noalloc_scratch(c->device);
        if (!base) throw TmError{TM_ERR_HIP, "device scratch not set up for this device"};
        struct NoAlloc {
            tm_ctx *c;
            ~NoAlloc() { c->no_alloc = false; }
        } guard{c};
        c->no_alloc = true;
        size_t used = 0;
        // consecutive 256-byte aligned pieces of the scratch array
        auto take = [&](const char *name, size_t bytes) -> void * {
            const size_t at = used;
            used += (bytes + 255) / 256 * 256;
            if (used > kNoallocScratchBytes)
                throw TmError{TM_ERR_UNSUPPORTED,
                              std::string("tm_dslash_noalloc: the intermediate fields of this kind need more than the ") +
                                  std::to_string(kNoallocScratchBytes) + " bytes of device scratch (" + name + ")"};
            return base + at;
        };
        return dslash_body(c, out, in, nrhs, kind, mu_sign, spinor_prec, link_prec, stream, take);
    });
}

// ---------------------------------------------------------------- layout

extern "C" int tm_pack(tm_ctx *c, void *even, void *odd, const double *full, int nrhs, int prec,
                       const double *scale_host, tm_stream stream)
{
    return guarded(c, [&]() {
        TM_REQUIRE(even && odd && full, "null pointer");
        TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        TM_REQUIRE(valid_prec(prec), "bad precision");
        double *ds = nullptr;
        if (scale_host) {
            ds = (double *)ws_get(c, "pack_scale", sizeof(double) * nrhs);
            TM_HIP(hipMemcpyAsync(ds, scale_host, sizeof(double) * nrhs, hipMemcpyHostToDevice, hs(stream)));
            TM_HIP(hipStreamSynchronize(hs(stream)));
        }
        launch_pack(c, even, odd, full, nrhs, prec, ds, hs(stream));
        return TM_OK;
    });
}

extern "C" int tm_unpack(tm_ctx *c, double *full, const void *even, const void *odd, int nrhs, int prec,
                         tm_stream stream)
{
    return guarded(c, [&]() {
        TM_REQUIRE(even && odd && full, "null pointer");
        TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        TM_REQUIRE(valid_prec(prec), "bad precision");
        launch_unpack(c, full, even, odd, nrhs, prec, hs(stream));
        return TM_OK;
    });
}

// ---------------------------------------------------------------- solve

extern "C" int tm_solve(tm_ctx *c, double *x, const double *b, int nrhs, const tm_solve_params *p,
                        tm_solve_stats *stats, tm_stream stream)
{
    return guarded(c, [&]() {
        const auto t0 = std::chrono::steady_clock::now();
        TM_REQUIRE(x && b && p, "null pointer");
        TM_REQUIRE(x != b, "x and b must differ");
        TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        hipStream_t s = hs(stream);
        const double b0 = c->acct_bytes, f0 = c->acct_flops;
        const size_t hb = half_bytes(c, TM_F64, nrhs);
        void *be = ws_get(c, "a_be", hb), *bo = ws_get(c, "a_bo", hb);
        void *xe = ws_get(c, "a_xe", hb), *xo = ws_get(c, "a_xo", hb);
        launch_pack(c, be, bo, b, nrhs, TM_F64, nullptr, s);
        SolveOut r = solve_halves(c, xe, xo, be, bo, nrhs, *p, s);
        launch_unpack(c, x, xe, xo, nrhs, TM_F64, s);
        TM_HIP(hipStreamSynchronize(s));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats)
            for (int i = 0; i < nrhs; i++) {
                stats[i] = r.st[i];
                stats[i].seconds = secs;
                stats[i].bytes = (c->acct_bytes - b0) / nrhs;
                stats[i].flops = (c->acct_flops - f0) / nrhs;
            }
        if (r.status == TM_ERR_NOCONV) c->err = "a right-hand side missed the tolerance within maxiter";
        if (r.status == TM_ERR_NAN) c->err = "NaN/Inf in the solution";
        return r.status;
    });
}

// ---------------------------------------------------------------- noise and loops

extern "C" int tm_noise(tm_ctx *c, double *out, uint64_t seed, long r, int dilution, tm_stream stream)
{
    return guarded(c, [&]() {
        TM_REQUIRE(out != nullptr, "null pointer");
        TM_REQUIRE(r >= 0, "noise index must be >= 0");
        TM_REQUIRE(dilution == TM_DIL_NONE || dilution == TM_DIL_SPIN_COLOUR, "bad dilution");
        const int nrhs = dilution ? 12 : 1;
        const size_t hb = half_bytes(c, TM_F64, nrhs);
        void *ee = ws_get(c, "n_e", hb), *eo = ws_get(c, "n_o", hb);
        launch_noise(c, ee, eo, seed, r, dilution, hs(stream));
        launch_unpack(c, out, ee, eo, nrhs, TM_F64, hs(stream));
        return TM_OK;
    });
}

extern "C" int tm_loops(tm_ctx *c, const tm_loop_params *p, double *loops, double *per_noise, tm_loop_stats *stats,
                        tm_stream stream)
{
    return guarded(c, [&]() {
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        int st = run_loops(c, p, loops, per_noise, stats, hs(stream));
        TM_HIP(hipStreamSynchronize(hs(stream)));
        if (st == TM_ERR_NOCONV) c->err = "a high-precision solve missed its tolerance";
        return st;
    });
}

namespace {

// tm_contract and tm_contract_momentum: mom = null for p = 0 per time slice
int contract_fields(tm_ctx *c, const double *eta, const double *s_, int nrhs, int estimators, int mu_sign,
                    int derivative, double *out, tm_stream stream, const std::vector<Momentum> *mom)
{
    TM_REQUIRE(s_ && out, "null pointer");
    TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    TM_REQUIRE(estimators > 0 && (estimators & ~(TM_EST_STD | TM_EST_ONE_END | TM_EST_GEN_ONE_END)) == 0,
               "contractions accept TM_EST_STD, TM_EST_ONE_END and TM_EST_GEN_ONE_END");
    TM_REQUIRE(!(estimators & TM_EST_STD) || eta, "STD needs eta");
    TM_REQUIRE(mu_sign == 1 || mu_sign == -1, "mu_sign must be +1 or -1");
    TM_REQUIRE(derivative == 0 || derivative == 1, "derivative must be 0 or 1");
    TM_REQUIRE(c->have_gauge || !(derivative || (estimators & TM_EST_GEN_ONE_END)),
               "derivative insertions and GEN_ONE_END need the gauge field");
    hipStream_t s = hs(stream);
    const size_t hb = half_bytes(c, TM_F64, nrhs);
    void *se = ws_get(c, "c_se", hb), *so = ws_get(c, "c_so", hb);
    launch_pack(c, se, so, s_, nrhs, TM_F64, nullptr, s);
    void *ee = se, *eo = so;
    if (estimators & TM_EST_STD) {
        ee = ws_get(c, "c_ee", hb);
        eo = ws_get(c, "c_eo", hb);
        launch_pack(c, ee, eo, eta, nrhs, TM_F64, nullptr, s);
    }
    c->stream = s;
    contract_noise(c, estimators, derivative, ee, eo, se, so, nrhs, eps_of(c, mu_sign), (cx<double> *)out, mom);
    TM_HIP(hipStreamSynchronize(s));
    return TM_OK;
}

}  // namespace

extern "C" int tm_contract(tm_ctx *c, const double *eta, const double *s_, int nrhs, int estimators, int mu_sign,
                           double *out, tm_stream stream)
{
    return guarded(c, [&]() { return contract_fields(c, eta, s_, nrhs, estimators, mu_sign, 0, out, stream, nullptr); });
}

extern "C" int tm_momenta(int p2max, int *count, int *list)
{
    if (p2max < 0 || !count) return TM_ERR_ARG;
    const std::vector<Momentum> m = momenta_list(p2max);
    if (list) {
        if (*count < (int)m.size()) return TM_ERR_ARG;
        for (size_t k = 0; k < m.size(); k++)
            for (int d = 0; d < 3; d++) list[3 * k + d] = m[k].n[d];
    }
    *count = (int)m.size();
    return TM_OK;
}

extern "C" int tm_contract_momentum(tm_ctx *c, const double *eta, const double *s_, int nrhs, int estimators,
                                    int mu_sign, int derivative, int p2max, double *out, tm_stream stream)
{
    return guarded(c, [&]() {
        check_momenta(c, p2max);
        const std::vector<Momentum> mom = momenta_list(p2max);
        return contract_fields(c, eta, s_, nrhs, estimators, mu_sign, derivative, out, stream, &mom);
    });
}

extern "C" int tm_loops_momentum(tm_ctx *c, const tm_loop_params *p, int p2max, double *loops, double *per_noise,
                                 tm_loop_stats *stats, tm_stream stream)
{
    return guarded(c, [&]() {
        TM_REQUIRE(c->have_gauge, "no gauge field set");
        check_momenta(c, p2max);
        const std::vector<Momentum> mom = momenta_list(p2max);
        int st = run_loops(c, p, loops, per_noise, stats, hs(stream), &mom);
        TM_HIP(hipStreamSynchronize(hs(stream)));
        if (st == TM_ERR_NOCONV) c->err = "a high-precision solve missed its tolerance";
        return st;
    });
}
