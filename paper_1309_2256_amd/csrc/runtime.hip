// Host runtime: operators on half-lattice fields, CG solvers on the even-odd
// normal equations (plain FP64, mixed precision with reliable updates, and the
// truncated low-precision solve of the Truncated Solver Method), and the
// disconnected-loop driver.
#include <chrono>
#include <cmath>
#include <cstring>

#include "runtime.h"

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

void upload(void *dev, const void *host, size_t bytes, hipStream_t s)
{
    TM_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s));
    TM_HIP(hipStreamSynchronize(s));
}

// upload without waiting, through pinned slot `slot` of the context (see
// host_upload_slot: the slot is reused only after a stream synchronisation)
static void upload_async(tm_ctx *c, int slot, void *dev, const void *host, size_t bytes, hipStream_t s)
{
    void *st = host_upload_slot(c, slot, bytes, s);
    memcpy(st, host, bytes);
    TM_HIP(hipMemcpyAsync(dev, st, bytes, hipMemcpyHostToDevice, s));
}

void download(tm_ctx *c, void *host, const void *dev, size_t bytes, hipStream_t s)
{
    void *stage = host_stage(c, bytes);
    TM_HIP(hipMemcpyAsync(stage, dev, bytes, hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    memcpy(host, stage, bytes);
}

std::vector<double> norms_host(tm_ctx *c, const void *v, int prec, int nrhs, hipStream_t s)
{
    double *d = (double *)ws_get(c, "norms_out", sizeof(double) * nrhs);
    launch_norm2(c, v, prec, nrhs, d, s);
    std::vector<double> h(nrhs);
    download(c, h.data(), d, sizeof(double) * nrhs, s);
    return h;
}

size_t field_bytes(tm_ctx *c, int prec, int nrhs) { return prec_bytes(prec) * 12 * (size_t)c->geo.hs * nrhs; }

void copy_field(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    TM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
}

namespace {

// chiral-basis Dirac matrices gamma_1..gamma_4 (x, y, z, t)
const cx<double> kGamma[4][4][4] = {
    {{{0, 0}, {0, 0}, {0, 0}, {0, -1}}, {{0, 0}, {0, 0}, {0, -1}, {0, 0}},
     {{0, 0}, {0, 1}, {0, 0}, {0, 0}}, {{0, 1}, {0, 0}, {0, 0}, {0, 0}}},
    {{{0, 0}, {0, 0}, {0, 0}, {-1, 0}}, {{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}}, {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},
    {{{0, 0}, {0, 0}, {0, -1}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}, {0, 1}},
     {{0, 1}, {0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {0, -1}, {0, 0}, {0, 0}}},
    {{{0, 0}, {0, 0}, {1, 0}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}, {1, 0}},
     {{1, 0}, {0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {1, 0}, {0, 0}, {0, 0}}},
};

}  // namespace

// Gamma_n = gamma_1^n0 gamma_2^n1 gamma_3^n2 gamma_4^n3
void gamma_n(int n, cx<double> G[4][4])
{
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) G[a][b] = {a == b ? 1.0 : 0.0, 0.0};
    for (int mu = 0; mu < 4; mu++) {
        if (!((n >> mu) & 1)) continue;
        cx<double> T[4][4];
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                cx<double> acc{0, 0};
                for (int k = 0; k < 4; k++) acc = acc + G[a][k] * kGamma[mu][k][b];
                T[a][b] = acc;
            }
        memcpy(G, T, sizeof(T));
    }
}

hipStream_t s_of(tm_ctx *c) { return c->stream; }

double eps_of(tm_ctx *c, int mu_sign) { return mu_sign >= 0 ? c->eps : -c->eps; }

void op_dslash(tm_ctx *c, void *out, const void *in, const void *own, int nrhs, int prec, int out_par, int dag,
               SpinDiag dhop, SpinDiag down, hipStream_t s, bool links18)
{
    DslashCall dc{};
    dc.links18 = links18;
    dc.out = out;
    dc.in = in;
    dc.own = own;
    dc.nrhs = nrhs;
    dc.out_parity = out_par;
    dc.dag = dag;
    dc.spinor_prec = prec;
    dc.d_own = down;
    dc.d_hop = dhop;
    dc.has_own = own != nullptr;
    launch_dslash(c, dc, s);
}

// Ahat x = R x - H_eo R^-1 H_oe x, with H = -kappa Hop
void op_schur(tm_ctx *c, void *out, const void *in, void *tmp, int nrhs, int prec, double epsp, hipStream_t s,
              bool links18)
{
    const double k = c->kappa;
    op_dslash(c, tmp, in, nullptr, nrhs, prec, 1, 0, sd_mul(sd_scalar(-k), sd_twist_inv(epsp)), sd_scalar(0), s,
              links18);
    op_dslash(c, out, tmp, in, nrhs, prec, 0, 0, sd_scalar(k), sd_twist(epsp), s, links18);
}

// Ahat^dag x = gamma5 Ahat(-eps) gamma5 x
//            = R(-eps) x - gamma5 H_eo t,  t = R^-1(-eps) H_oe gamma5 x = R^-1(-eps) gamma5 H^dag_oe x
void op_schur_dag(tm_ctx *c, void *out, const void *in, void *tmp, int nrhs, int prec, double epsp,
                  hipStream_t s)
{
    const double k = c->kappa;
    op_dslash(c, tmp, in, nullptr, nrhs, prec, 1, 1,
              sd_mul(sd_scalar(-k), sd_mul(sd_twist_inv(-epsp), sd_gamma5())), sd_scalar(0), s);
    op_dslash(c, out, tmp, in, nrhs, prec, 0, 0, sd_mul(sd_scalar(k), sd_gamma5()), sd_twist(-epsp), s);
}

void op_bh_power(tm_ctx *c, void *se, void *so, int nrhs, double epsp, int kpow, hipStream_t s)
{
    size_t bytes = field_bytes(c, TM_F64, nrhs);
    void *te = ws_get(c, "bh_e", bytes), *to = ws_get(c, "bh_o", bytes);
    SpinDiag d = sd_mul(sd_scalar(-c->kappa), sd_twist_inv(epsp));
    for (int i = 0; i < kpow; i++) {
        op_dslash(c, to, se, nullptr, nrhs, TM_F64, 1, 0, d, sd_scalar(0), s);
        op_dslash(c, te, so, nullptr, nrhs, TM_F64, 0, 0, d, sd_scalar(0), s);
        copy_field(se, te, bytes, s);
        copy_field(so, to, bytes, s);
    }
}

// ---------------------------------------------------------------- CG

namespace {

// One CG iteration on the Schur normal equations for one instance, as four
// half-Dslash launches with fused epilogues plus three small kernels:
//   t = R^-1 H p;  q = R p - H t   (+ partial |q|^2)          D1, D2
//   alpha = rr / |q|^2                                          finish
//   t = R^-1(-eps) g5 H^dag q;  s = R(-eps) q + kappa g5 H t,  D3, D4
//     r -= alpha s, rho -= alpha q (+ partial |r|^2, |rho|^2)
//   beta, convergence / update flags                            finish
//   x += alpha p, p = r + beta p                                update
DslashCall stage_call(tm_ctx *c, const CGWork &w, double epsp, int stage)
{
    const double k = c->kappa;
    DslashCall dc{};
    dc.nrhs = w.nrhs;
    dc.spinor_prec = w.prec;
    switch (stage) {
    case 1:
        dc.out = w.tmp;
        dc.in = w.p;
        dc.out_parity = 1;
        dc.d_hop = sd_mul(sd_scalar(-k), sd_twist_inv(epsp));
        dc.d_own = sd_scalar(0);
        break;
    case 2:
        dc.out = w.q;
        dc.in = w.tmp;
        dc.own = w.p;
        dc.has_own = true;
        dc.d_own = sd_twist(epsp);
        dc.d_hop = sd_scalar(k);
        dc.epi = 1;
        dc.part = w.partq;
        break;
    case 3:
        dc.out = w.tmp;
        dc.in = w.q;
        dc.out_parity = 1;
        dc.dag = 1;
        dc.d_hop = sd_mul(sd_scalar(-k), sd_mul(sd_twist_inv(-epsp), sd_gamma5()));
        dc.d_own = sd_scalar(0);
        break;
    default:
        dc.in = w.tmp;
        dc.own = w.q;
        dc.has_own = true;
        dc.d_own = sd_twist(-epsp);
        dc.d_hop = sd_mul(sd_scalar(k), sd_gamma5());
        dc.epi = 2;
        dc.r = w.r;
        dc.rho = w.rho_vec ? w.rho : nullptr;
        dc.sc = w.dsc;
        dc.part = w.partb;
        break;
    }
    return dc;
}

}  // namespace

void Solver::init(tm_ctx *ctx, void *xe_, void *xo_, const void *be_, const void *bo_, int nrhs_,
                  const tm_solve_params &par, hipStream_t s)
{
    t0 = now_s();
    c = ctx;
    xe = xe_;
    xo = xo_;
    be = be_;
    bo = bo_;
    nrhs = nrhs_;
    p = par;
    TM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    TM_REQUIRE(p.tol > 0 && std::isfinite(p.tol), "tol must be > 0");
    TM_REQUIRE(p.maxiter > 0, "maxiter must be > 0");
    TM_REQUIRE(p.solver >= TM_CG_F64 && p.solver <= TM_CG_LOW, "unknown solver");
    TM_REQUIRE(p.mu_sign == 1 || p.mu_sign == -1, "mu_sign must be +1 or -1");
    lp = p.solver == TM_CG_F64 ? TM_F64 : p.inner_prec;
    TM_REQUIRE(lp == TM_F64 || lp == TM_F32 || lp == TM_F16 || lp == TM_BF16, "bad inner precision");
    TM_REQUIRE(p.solver == TM_CG_F64 || lp != TM_F64, "MIXED/LOW need a FP32/FP16/BF16 inner precision");
    check_every = p.check_every > 0 ? p.check_every : 8;
    delta = p.solver == TM_CG_MIXED ? (p.delta > 0 ? p.delta : 0.1) : 0.0;
    epsp = eps_of(c, p.mu_sign);
    nsb = dslash_site_blocks(c);
    total = since_check = 0;
    done = false;
    const size_t f64 = field_bytes(c, TM_F64, nrhs);
    bh = ws_get(c, "s_bh", f64);
    t64 = ws_get(c, "s_t64", f64);
    rho64 = ws_get(c, "s_rho64", f64);
    r64 = ws_get(c, "s_r64", f64);
    q64 = ws_get(c, "s_q64", f64);

    bn2 = norms_host(c, be, TM_F64, nrhs, s);
    {
        std::vector<double> bo2 = norms_host(c, bo, TM_F64, nrhs, s);
        for (int r = 0; r < nrhs; r++) bn2[r] += bo2[r];
    }
    for (int r = 0; r < nrhs; r++)
        if (!std::isfinite(bn2[r])) throw TmError{TM_ERR_NAN, "NaN/Inf in the source"};

    // bhat_e = b_e - H_eo R_oo^-1 b_o
    launch_spin_diag(c, t64, bo, TM_F64, nrhs, sd_twist_inv(epsp), s);
    op_dslash(c, bh, t64, be, nrhs, TM_F64, 0, 0, sd_scalar(c->kappa), sd_scalar(1.0), s, true);

    hsc.assign(nrhs, CGScalars{});
    n_rel.assign(nrhs, 0);
    iter_res.assign(nrhs, 0.0);
    sigma.assign(nrhs, 1.0);
    w = CGWork{};
    w.nrhs = nrhs;
    w.prec = lp;
    // with reliable updates |rho|^2 follows a scalar recurrence between
    // updates; plain and truncated solves keep the vector (the recurrence
    // would lose the residual below ~1e-7 of its start to cancellation)
    w.rho_vec = p.solver != TM_CG_MIXED;
    w.dsc = (CGScalars *)ws_get(c, "s_sc", sizeof(CGScalars) * nrhs);
    w.partq = (double *)ws_get(c, "s_partq", sizeof(double) * nsb * nrhs);
    w.partb = (double *)ws_get(c, "s_partb", sizeof(double) * nsb * nrhs * 2);
    dscale = (double *)ws_get(c, "s_scale", sizeof(double) * nrhs);
    launch_zero(c, xe, TM_F64, nrhs, s);
    copy_field(rho64, bh, f64, s);
    if (lp == TM_F64) {
        w.x = xe;
        w.xprec = TM_F64;
        w.rho = rho64;
        w.r = r64;
        w.q = q64;
        w.tmp = t64;
        w.p = ws_get(c, "s_p64", f64);
        op_schur_dag(c, r64, rho64, t64, nrhs, TM_F64, epsp, s);
        copy_field(w.p, r64, f64, s);
        std::vector<double> rr = norms_host(c, r64, TM_F64, nrhs, s);
        std::vector<double> rho2 = norms_host(c, rho64, TM_F64, nrhs, s);
        for (int r = 0; r < nrhs; r++) {
            CGScalars &q = hsc[r];
            q.rr = rr[r];
            q.rho2 = rho2[r];
            q.rho2_ref = rho2[r];
            q.target2 = p.tol * p.tol * bn2[r];
            q.sigma = 1.0;
            q.active = rho2[r] > q.target2 ? 1 : 0;
            iter_res[r] = std::sqrt(rho2[r] / bn2[r]);
        }
        upload(w.dsc, hsc.data(), sizeof(CGScalars) * nrhs, s);
    } else {
        // low-precision vectors scaled to unit RMS per element
        const size_t fl = field_bytes(c, lp, nrhs);
        w.x = ws_get(c, "s_y32", field_bytes(c, TM_F32, nrhs));
        w.xprec = TM_F32;
        w.rho = ws_get(c, "s_rho_lo", fl);
        w.r = ws_get(c, "s_r_lo", fl);
        w.q = ws_get(c, "s_q_lo", fl);
        w.p = ws_get(c, "s_p_lo", fl);
        w.tmp = ws_get(c, "s_t_lo", fl);
        restart(true, s);
    }
    bool any = false;
    for (auto &q : hsc) any |= q.active != 0;
    done = !any;
}

// (re)start the low-precision iteration from the FP64 residual rho64:
// r = Ahat^dag rho, new per-RHS scales, p rescaled (kept otherwise)
void Solver::restart(bool first, hipStream_t s, bool reactivate)
{
    const double nel = 12.0 * c->geo.vh;
    const size_t fl = field_bytes(c, lp, nrhs);
    std::vector<double> hscale(nrhs), sig_new(nrhs);
    std::vector<double> nrho = norms_host(c, rho64, TM_F64, nrhs, s);
    auto unit_scale = [&](double n2) {
        const double v = n2 > 0 ? std::sqrt(nel / n2) : 1.0;
        return std::isfinite(v) ? v : 1.0;
    };
    if (first) {
        // r = Ahat^dag rho in FP64, both scaled to unit RMS of r
        op_schur_dag(c, r64, rho64, t64, nrhs, TM_F64, epsp, s);
        std::vector<double> nr = norms_host(c, r64, TM_F64, nrhs, s);
        for (int r = 0; r < nrhs; r++) sig_new[r] = unit_scale(nr[r]);
        for (int r = 0; r < nrhs; r++) hscale[r] = sig_new[r];
        upload(dscale, hscale.data(), sizeof(double) * nrhs, s);
        launch_copy_convert(c, w.r, lp, r64, TM_F64, nrhs, dscale, s);
        launch_copy_convert(c, w.rho, lp, rho64, TM_F64, nrhs, dscale, s);
        copy_field(w.p, w.r, fl, s);
    } else {
        // the true residual rho (FP64) enters the low-precision iteration at
        // unit RMS; r = Ahat^dag rho is formed at the iteration's precision
        // (the FP64 part of the update is the residual itself), then both
        // are rescaled to unit RMS of r and p follows the new scale
        // the scale uploads go through pinned slots without waiting: slot 0
        // follows the norms_host synchronisation after accumulate's copy,
        // slots 1-3 are each used once between two synchronisations
        std::vector<double> srho(nrhs);
        for (int r = 0; r < nrhs; r++) srho[r] = unit_scale(nrho[r]);
        upload_async(c, 1, dscale, srho.data(), sizeof(double) * nrhs, s);
        launch_copy_convert(c, w.rho, lp, rho64, TM_F64, nrhs, dscale, s);
        op_schur_dag(c, w.r, w.rho, w.tmp, nrhs, lp, epsp, s);
        std::vector<double> nrl = norms_host(c, w.r, lp, nrhs, s);
        for (int r = 0; r < nrhs; r++) sig_new[r] = unit_scale(nrl[r] / (srho[r] * srho[r]));
        for (int r = 0; r < nrhs; r++) hscale[r] = sig_new[r] / srho[r];
        upload_async(c, 2, dscale, hscale.data(), sizeof(double) * nrhs, s);
        launch_copy_convert(c, w.r, lp, w.r, lp, nrhs, dscale, s);
        upload_async(c, 3, dscale, sig_new.data(), sizeof(double) * nrhs, s);
        launch_copy_convert(c, w.rho, lp, rho64, TM_F64, nrhs, dscale, s);
        for (int r = 0; r < nrhs; r++) hscale[r] = sig_new[r] / sigma[r];
        upload_async(c, 0, dscale, hscale.data(), sizeof(double) * nrhs, s);
        launch_copy_convert(c, w.p, lp, w.p, lp, nrhs, dscale, s);
    }
    launch_zero(c, w.x, TM_F32, nrhs, s);
    std::vector<double> rr = norms_host(c, w.r, lp, nrhs, s);
    std::vector<double> rho2 = norms_host(c, w.rho, lp, nrhs, s);
    if (!first) download(c, hsc.data(), w.dsc, sizeof(CGScalars) * nrhs, s);
    for (int r = 0; r < nrhs; r++) {
        CGScalars &q = hsc[r];
        if (first) {
            memset(&q, 0, sizeof(q));
            q.active = 1;
        }
        q.rr = rr[r];
        q.rho2 = rho2[r];
        q.rho2_ref = rho2[r];
        q.target2 = p.tol * p.tol * bn2[r] * sig_new[r] * sig_new[r];
        q.sigma = sig_new[r];
        q.want_update = 0;
        if (reactivate) q.active = 1;
        if (nrho[r] <= p.tol * p.tol * bn2[r]) q.active = 0;  // converged on the true FP64 residual
        iter_res[r] = std::sqrt(nrho[r] / bn2[r]);
    }
    sigma = sig_new;
    upload(w.dsc, hsc.data(), sizeof(CGScalars) * nrhs, s);
}

// x_hi += y / sigma
void Solver::accumulate(hipStream_t s)
{
    std::vector<double> hscale(nrhs);
    for (int r = 0; r < nrhs; r++) hscale[r] = 1.0 / sigma[r];
    // slot 0; every caller synchronises (a norm download) before the next
    // use of the slot
    upload_async(c, 0, dscale, hscale.data(), sizeof(double) * nrhs, s);
    launch_axpy_dev(c, xe, TM_F64, w.x, TM_F32, nrhs, dscale, s);
}

void Solver::iteration_tail(hipStream_t s)
{
    cg_finish_beta(c, w.dsc, w.partb, nsb, nrhs, delta, s);
    cg_update_px(c, w.p, w.r, w.x, w.prec, w.xprec, nrhs, w.dsc, s);
}

void Solver::iteration(hipStream_t s)
{
    launch_dslash(c, stage_call(c, w, epsp, 1), s);
    launch_dslash(c, stage_call(c, w, epsp, 2), s);
    cg_finish_alpha(c, w.dsc, w.partq, nsb, nrhs, s);
    launch_dslash(c, stage_call(c, w, epsp, 3), s);
    launch_dslash(c, stage_call(c, w, epsp, 4), s);
    iteration_tail(s);
}

DslashCall Solver::stage(int k) const { return stage_call(c, w, epsp, k); }

void Solver::iter_cost(double &bytes, double &flops) const
{
    bytes = flops = 0;
    for (int k = 1; k <= 4; k++) {
        double b, f;
        dslash_cost(c, stage(k), b, f);
        bytes += b;
        flops += f;
    }
    const double n = 12.0 * c->geo.vh * nrhs;
    bytes += n * (3 * prec_bytes(w.prec) + 2 * prec_bytes(w.xprec));
    flops += 8.0 * n;
}

void Solver::count_iteration()
{
    total++;
    since_check++;
}

bool Solver::due() const { return since_check >= check_every || total >= p.maxiter; }

// host check after a group of iterations: NaN, convergence, reliable update
void Solver::check(hipStream_t s)
{
    since_check = 0;
    download(c, hsc.data(), w.dsc, sizeof(CGScalars) * nrhs, s);
    bool any_active = false, any_update = false, any_bad = false;
    for (auto &q : hsc) {
        any_active |= q.active != 0;
        any_update |= (q.active && q.want_update);
        any_bad |= q.bad != 0;
    }
    if (any_bad) throw TmError{TM_ERR_NAN, "NaN/Inf in a solver reduction"};
    const bool out_of_iters = total >= p.maxiter;
    if (lp == TM_F64) {
        for (int r = 0; r < nrhs; r++) iter_res[r] = std::sqrt(hsc[r].rho2 / bn2[r]);
        done = !any_active || out_of_iters;
        return;
    }
    if (p.solver == TM_CG_LOW) {
        if (!any_active || out_of_iters) {
            for (int r = 0; r < nrhs; r++) iter_res[r] = std::sqrt(hsc[r].rho2 / bn2[r]) / hsc[r].sigma;
            accumulate(s);
            done = true;
            if (out_of_iters) return;
            // the truncation criterion holds for the true residual: the FP64
            // Schur residual of the accumulated solution (equal to the
            // full-system residual after odd reconstruction); right-hand
            // sides still above tol continue from it, as after a reliable
            // update
            op_schur(c, q64, xe, t64, nrhs, TM_F64, epsp, s, true);
            launch_axpby_to_host(c, rho64, q64, bh, TM_F64, nrhs, -1.0, 1.0, s);  // rho = bh - Ahat x
            std::vector<double> nrho = norms_host(c, rho64, TM_F64, nrhs, s);
            bool again = false;
            for (int r = 0; r < nrhs; r++) again |= nrho[r] > p.tol * p.tol * bn2[r];
            if (again) {
                restart(false, s, true);
                bool any = false;
                for (auto &q : hsc) any |= q.active != 0;
                done = !any;
            }
        }
        return;
    }
    if (!any_update && !out_of_iters) return;
    // reliable update: FP64 true residual of the accumulated solution
    accumulate(s);
    op_schur(c, q64, xe, t64, nrhs, TM_F64, epsp, s, true);
    launch_axpby_to_host(c, rho64, q64, bh, TM_F64, nrhs, -1.0, 1.0, s);  // rho = bh - Ahat x
    for (int r = 0; r < nrhs; r++)
        if (hsc[r].active) n_rel[r]++;
    restart(false, s);
    bool any = false;
    for (auto &q : hsc) any |= q.active != 0;
    done = !any || out_of_iters;
}

SolveOut Solver::finalize(hipStream_t s)
{
    const double kap = c->kappa;
    // odd reconstruction psi_o = R^-1 (b_o - H_oe psi_e)
    op_dslash(c, xo, xe, bo, nrhs, TM_F64, 1, 0, sd_mul(sd_scalar(kap), sd_twist_inv(epsp)), sd_twist_inv(epsp), s,
              true);
    // true residual b - M x, both parities, with the exact (18-parameter) links
    op_dslash(c, rho64, xo, xe, nrhs, TM_F64, 0, 0, sd_scalar(-kap), sd_twist(epsp), s, true);
    launch_axpby_host(c, rho64, be, TM_F64, nrhs, -1.0, 1.0, s);
    op_dslash(c, t64, xe, xo, nrhs, TM_F64, 1, 0, sd_scalar(-kap), sd_twist(epsp), s, true);
    launch_axpby_host(c, t64, bo, TM_F64, nrhs, -1.0, 1.0, s);
    std::vector<double> re = norms_host(c, rho64, TM_F64, nrhs, s);
    std::vector<double> ro = norms_host(c, t64, TM_F64, nrhs, s);
    download(c, hsc.data(), w.dsc, sizeof(CGScalars) * nrhs, s);
    const double t1 = now_s();
    SolveOut out;
    out.st.assign(nrhs, tm_solve_stats{});
    for (int r = 0; r < nrhs; r++) {
        tm_solve_stats &st = out.st[r];
        st.iters = hsc[r].iters;
        st.n_reliable = n_rel[r];
        st.true_rel_res = bn2[r] > 0 ? std::sqrt((re[r] + ro[r]) / bn2[r]) : 0.0;
        st.iter_rel_res = iter_res[r];
        st.converged = st.true_rel_res <= p.tol ? 1 : 0;
        st.seconds = t1 - t0;
        if (!std::isfinite(st.true_rel_res)) out.status = TM_ERR_NAN;
        if (!st.converged && p.solver != TM_CG_LOW && out.status == TM_OK) out.status = TM_ERR_NOCONV;
    }
    return out;
}

SolveOut solve_halves(tm_ctx *c, void *xe, void *xo, const void *be, const void *bo, int nrhs,
                      const tm_solve_params &p, hipStream_t s)
{
    if (p.solver == TM_FGMRES || p.solver == TM_FGMRES_PTC) return fgmres_halves(c, xe, xo, be, bo, nrhs, p, s);
    Solver S;
    S.init(c, xe, xo, be, bo, nrhs, p, s);
    while (!S.done) {
        S.iteration(s);
        S.count_iteration();
        if (S.due()) S.check(s);
    }
    return S.finalize(s);
}

// ---------------------------------------------------------------- loops

void outer_slices_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                       std::vector<cx<double>> &out, hipStream_t s, int t0, int dt)
{
    const int Lt = c->geo.L[3];
    double *d = (double *)ws_get(c, "outer_out", sizeof(double) * 32 * Lt);
    launch_outer_slices(c, ve, vo, we, wo, nrhs, d, s, t0, dt);
    out.resize((size_t)16 * Lt);
    download(c, out.data(), d, sizeof(double) * 32 * Lt, s);
}

void loops_from_outer(tm_ctx *c, const cx<double> *C, GammaForm form, cx<double> coef, cx<double> *out)
{
    const int Lt = c->geo.L[3];
    cx<double> g5[4][4];
    gamma_n(15, g5);
    for (int n = 0; n < 16; n++) {
        cx<double> G[4][4], X[4][4];
        gamma_n(n, G);
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                if (form == G_PLAIN) {
                    X[a][b] = G[a][b];
                } else {
                    cx<double> acc{0, 0};
                    for (int k = 0; k < 4; k++) acc = acc + g5[a][k] * G[k][b];
                    X[a][b] = acc;
                }
            }
        if (form == G_G5_BOTH) {
            cx<double> Y[4][4];
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cx<double> acc{0, 0};
                    for (int k = 0; k < 4; k++) acc = acc + X[a][k] * g5[k][b];
                    Y[a][b] = acc;
                }
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) X[a][b] = Y[a][b];
        }
        for (int t = 0; t < Lt; t++) {
            cx<double> acc{0, 0};
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) acc = acc + X[a][b] * C[(size_t)t * 16 + b * 4 + a];
            out[(size_t)n * Lt + t] = coef * acc;
        }
    }
}

// Per site, tr[Gamma_n (B + (BH)^2 B)] is gauge independent when every L_mu >= 3
// (only back-and-forth hop pairs return to the site); in the chiral basis
// with b0 = 1/(1+eps^2), b1 = i eps/(1+eps^2) ... it is non-zero only for
// Gamma = 1 and Gamma = gamma5:
//   n = 0:  12/(1+eps^2) - 384 kappa^2 eps^2/(1+eps^2)^3
//   n = 15: -12 i eps/(1+eps^2) - 192 i kappa^2 eps (1-eps^2)/(1+eps^2)^3
void hpe_exact_part(tm_ctx *c, double e, cx<double> *out)
{
    const int Lt = c->geo.L[3];
    const double Vs = (double)c->geo.L[0] * c->geo.L[1] * c->geo.L[2];
    const double k2 = c->kappa * c->kappa, d = 1.0 + e * e;
    cx<double> c0{Vs * (12.0 / d - 384.0 * k2 * e * e / (d * d * d)), 0.0};
    cx<double> c15{0.0, Vs * (-12.0 * e / d - 192.0 * k2 * e * (1.0 - e * e) / (d * d * d))};
    for (int n = 0; n < 16; n++)
        for (int t = 0; t < Lt; t++) out[(size_t)n * Lt + t] = n == 0 ? c0 : n == 15 ? c15 : cx<double>{0, 0};
}

void op_wilson(tm_ctx *c, void *oe, void *oo, const void *fe, const void *fo, int nrhs, hipStream_t s)
{
    const double k = c->kappa;
    op_dslash(c, oe, fo, fe, nrhs, TM_F64, 0, 0, sd_scalar(-k), sd_scalar(1), s);
    op_dslash(c, oo, fe, fo, nrhs, TM_F64, 1, 0, sd_scalar(-k), sd_scalar(1), s);
}

void contract_noise(tm_ctx *c, int estimators, int derivative, const void *ee, const void *eo, const void *se,
                    const void *so, int nrhs, double epsp, cx<double> *dst, const std::vector<Momentum> *mom,
                    const TimeDil *td)
{
    const int Lt = c->geo.L[3];
    const size_t per_ins = (size_t)16 * Lt;  // one block of 16 insertions
    const int n_ins = n_insertions(derivative);
    const int n_mom = mom ? (int)mom->size() : 1;
    const size_t per_m = (size_t)Lt * n_ins;
    const size_t per = per_m * n_mom;
    const size_t f64 = field_bytes(c, TM_F64, nrhs);
    static const std::vector<Momentum> zero{Momentum{{0, 0, 0}}};
    std::vector<cx<double>> C;
    // outer products of (right v, left w), then the Gamma insertions per momentum;
    // slice_ok: w is the time-diluted source itself, so group q of a
    // time-diluted batch contributes on its source slices only
    auto outer_loops = [&](const void *ve, const void *vo, const void *we, const void *wo, GammaForm form,
                           cx<double> coef, bool deriv, cx<double> *out, bool slice_ok = false) {
        if (!mom && slice_ok && td && td->period > 0) {
            const size_t grp = field_bytes(c, TM_F64, td->nsc);
            std::vector<cx<double>> acc((size_t)16 * Lt, cx<double>{0, 0});
            for (int q = 0; q < td->n_off; q++) {
                outer_slices_host(c, (const char *)ve + q * grp, (const char *)vo + q * grp,
                                  (const char *)we + q * grp, (const char *)wo + q * grp, td->nsc, C, s_of(c),
                                  td->o_first + q, td->period);
                for (size_t j = 0; j < acc.size(); j++) acc[j] = acc[j] + C[j];
            }
            loops_from_outer(c, acc.data(), form, coef, out);
        } else if (mom) {
            outer_momenta_host(c, ve, vo, we, wo, nrhs, *mom, C, s_of(c));
            for (int m = 0; m < n_mom; m++) loops_from_outer(c, C.data() + per_ins * m, form, coef, out + per_m * m);
        } else {
            outer_slices_host(c, ve, vo, we, wo, nrhs, C, s_of(c));
            loops_from_outer(c, C.data(), form, coef, out);
        }
        if (!deriv) return;
        // D_mu blocks [n_mom][4][Lt][16]; per time slice = the zero momentum
        outer_deriv_host(c, ve, vo, we, wo, nrhs, mom ? *mom : zero, C, s_of(c));
        for (int m = 0; m < n_mom; m++)
            for (int mu = 0; mu < 4; mu++)
                loops_from_outer(c, C.data() + per_ins * (4 * m + mu), form, coef,
                                 out + per_m * m + per_ins * (1 + mu));
    };
    int k = 0;
    if (estimators & TM_EST_STD)
        outer_loops(se, so, ee, eo, G_PLAIN, cx<double>{1, 0}, derivative, dst + per * k++, true);
    if (estimators & TM_EST_ONE_END)
        outer_loops(se, so, se, so, G_G5_LEFT, cx<double>{0, 2.0 * epsp}, derivative, dst + per * k++);
    if (estimators & TM_EST_HPE) {
        void *he = ws_get(c, "l_h_e", f64), *ho = ws_get(c, "l_h_o", f64);
        copy_field(he, se, f64, s_of(c));
        copy_field(ho, so, f64, s_of(c));
        op_bh_power(c, he, ho, nrhs, epsp, 4, s_of(c));
        outer_loops(he, ho, ee, eo, G_PLAIN, cx<double>{1, 0}, false, dst + per * k++, true);
    }
    if (estimators & TM_EST_GEN_ONE_END) {
        // 2 s^dag gamma5 X gamma5 D_W s (eq. loopStD): right field D_W s, left s
        void *we = ws_get(c, "l_w_e", f64), *wo = ws_get(c, "l_w_o", f64);
        op_wilson(c, we, wo, se, so, nrhs, s_of(c));
        outer_loops(we, wo, se, so, G_G5_BOTH, cx<double>{2, 0}, derivative, dst + per * k++);
    }
}

int run_loops(tm_ctx *c, const tm_loop_params *p, double *loops, double *per_noise, tm_loop_stats *stats,
              hipStream_t s, const std::vector<Momentum> *mom)
{
    const double t0 = now_s();
    TM_REQUIRE(p != nullptr && loops != nullptr, "null argument");
    TM_REQUIRE(p->n_hp >= 0 && p->n_lp >= 0 && p->n_hp + p->n_lp >= 1, "need at least one noise vector");
    TM_REQUIRE(p->estimators > 0 && p->estimators < 16, "bad estimator mask");
    TM_REQUIRE(p->derivative == 0 || p->derivative == 1, "derivative must be 0 or 1");
    TM_REQUIRE(!(p->derivative && (p->estimators & TM_EST_HPE)),
               "HPE takes ultra-local insertions only (derivative = 0)");
    TM_REQUIRE(p->dilution == TM_DIL_NONE || p->dilution == TM_DIL_SPIN_COLOUR, "bad dilution");
    TM_REQUIRE(p->mu_sign == 1 || p->mu_sign == -1, "mu_sign must be +1 or -1");
    TM_REQUIRE(p->noise_offset >= 0, "noise_offset must be >= 0");
    if (p->estimators & TM_EST_HPE)
        for (int mu = 0; mu < 4; mu++)
            TM_REQUIRE(c->geo.L[mu] >= 4, "HPE needs every L_mu >= 4");
    const int Lt = c->geo.L[3];
    TM_REQUIRE(p->t_period >= 0 && p->t_period <= Lt && (p->t_period == 0 || Lt % p->t_period == 0),
               "t_period must be 0 or a divisor of Lt");
    const int nsc = p->dilution == TM_DIL_SPIN_COLOUR ? 12 : 1;
    // time dilution: t_period offsets per noise, solved in batches of up to 12 RHS
    const int n_offsets = p->t_period > 0 ? p->t_period : 1;
    const int per_batch = p->t_period > 0 ? std::max(1, std::min(n_offsets, 12 / nsc)) : 1;
    const int nrhs = per_batch * nsc;
    const int n_noise = p->n_hp + p->n_lp;
    const double epsp = eps_of(c, p->mu_sign);
    int n_est = 0;
    int est_ids[4];
    for (int b = 0; b < 4; b++)
        if (p->estimators & (1 << b)) est_ids[n_est++] = 1 << b;
    const size_t f64 = field_bytes(c, TM_F64, nrhs);
    void *ee = ws_get(c, "l_eta_e", f64), *eo = ws_get(c, "l_eta_o", f64);
    void *se = ws_get(c, "l_s_e", f64), *so = ws_get(c, "l_s_o", f64);
    // per estimator: [n_mom][n_ins][Lt] (one momentum, p = 0, without mom)
    const size_t per = (size_t)n_insertions(p->derivative) * Lt * (mom ? mom->size() : 1);
    // per-noise loops [noise][prec 0 hp, 1 lp][est][per]
    std::vector<cx<double>> pn((size_t)n_noise * 2 * n_est * per, cx<double>{0, 0});
    tm_loop_stats st{};
    int status = TM_OK;
    c->stream = s;

    std::vector<cx<double>> part(n_est * per);
    // per-noise loops summed over the time-dilution batches of the noise
    auto contract = [&](int noise, int slot, int nr, const TimeDil *td) {
        contract_noise(c, p->estimators, p->derivative, ee, eo, se, so, nr, epsp, part.data(), mom, td);
        cx<double> *dst = &pn[((size_t)noise * 2 + slot) * n_est * per];
        for (size_t j = 0; j < part.size(); j++) dst[j] = dst[j] + part[j];
    };

    for (int k = 0; k < n_noise; k++) {
        const long r = (long)p->noise_offset + k;
        for (int o = 0; o < n_offsets; o += per_batch) {
            const int n_off = std::min(per_batch, n_offsets - o);
            const int nr = n_off * nsc;
            const TimeDil td{p->t_period, o, n_off, nsc};
            launch_noise(c, ee, eo, p->seed, r, p->dilution, s, p->t_period, o, n_off);
            if (k < p->n_hp) {
                tm_solve_params hp = p->hp;
                hp.mu_sign = p->mu_sign;
                SolveOut so_ = solve_halves(c, se, so, ee, eo, nr, hp, s);
                for (auto &q : so_.st) {
                    st.n_solves_hp++;
                    st.iters_hp += q.iters;
                    st.max_res_hp = std::max(st.max_res_hp, q.true_rel_res);
                }
                if (so_.status != TM_OK && status == TM_OK) status = so_.status;
                contract(k, 0, nr, &td);
            }
            if (p->n_lp > 0) {
                tm_solve_params lp = p->lp;
                lp.mu_sign = p->mu_sign;
                SolveOut so_ = solve_halves(c, se, so, ee, eo, nr, lp, s);
                for (auto &q : so_.st) {
                    st.n_solves_lp++;
                    st.iters_lp += q.iters;
                    st.max_res_lp = std::max(st.max_res_lp, q.true_rel_res);
                }
                if (so_.status == TM_ERR_NAN) status = TM_ERR_NAN;
                contract(k, 1, nr, &td);
            }
        }
    }

    // TSM combination (eq. estiTSM) or the plain mean, per estimator
    // the exact HPE part is the same at every site: it enters p = 0 only
    // (the first 16 Lt entries; momenta_list puts (0,0,0) first)
    std::vector<cx<double>> ex(per, cx<double>{0, 0});
    if (p->estimators & TM_EST_HPE) hpe_exact_part(c, epsp, ex.data());
    for (int k = 0; k < n_est; k++) {
        cx<double> *dst = (cx<double> *)loops + (size_t)k * per;
        for (size_t j = 0; j < per; j++) {
            cx<double> acc{0, 0};
            if (p->n_lp == 0) {
                for (int r = 0; r < p->n_hp; r++) acc = acc + pn[(((size_t)r * 2 + 0) * n_est + k) * per + j];
                acc = (1.0 / p->n_hp) * acc;
            } else {
                cx<double> corr{0, 0}, lpm{0, 0};
                for (int r = 0; r < p->n_hp; r++)
                    corr = corr + pn[(((size_t)r * 2 + 0) * n_est + k) * per + j] -
                           pn[(((size_t)r * 2 + 1) * n_est + k) * per + j];
                for (int r = p->n_hp; r < n_noise; r++) lpm = lpm + pn[(((size_t)r * 2 + 1) * n_est + k) * per + j];
                if (p->n_hp > 0) acc = (1.0 / p->n_hp) * corr;
                acc = acc + (1.0 / p->n_lp) * lpm;
            }
            if (est_ids[k] == TM_EST_HPE) acc = acc + ex[j];
            dst[j] = acc;
        }
    }
    if (per_noise) memcpy(per_noise, pn.data(), pn.size() * sizeof(cx<double>));
    st.seconds = now_s() - t0;
    if (stats) *stats = st;
    return status;
}
