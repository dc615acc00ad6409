// Uneven batches: several lattices (contexts) solved together.  A group of
// `check_every` CG iterations of all instances is one launch of the
// persistent batch kernel (up to four instances: the four half-Dslash
// stages, the CG scalars and the vector update of every iteration, with grid
// barriers between the stages; see dslash.hip).  Otherwise every iteration
// is four multi-instance half-Dslash launches (all lattices in one grid)
// plus per-instance scalar and vector kernels, the group captured once into
// a HIP graph and replayed.  Either way the host reads the convergence
// scalars only between groups.  Reliable updates and convergence decisions
// are per instance, with the same cadence as a single solve, so each
// instance follows exactly the arithmetic of its own solve.
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <new>

#include "runtime.h"

struct tm_batch {
    std::vector<tm_ctx *> ctx;
    int device = 0;
    std::string err;
    hipStream_t stream = nullptr;  // own stream (graph capture needs a non-null stream)
    MultiDslash md[4];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int> graph_set;  // instances captured in the current graph
    int graph_iters = 0, graph_R = 0;
    std::map<std::vector<int>, int> tuned_R;  // (prec, nrhs...) -> RHS per thread
    PersistBatch pb;
    std::vector<int> pb_set;  // instances of the prepared persistent launch
    // launch form per (precision, nrhs...): 1 persistent kernel, 0 graph;
    // untuned keys time one group of each form and keep the faster (their
    // results are bit-identical)
    std::map<std::vector<int>, int> tuned_form;
    std::map<std::vector<int>, float> form_ms[2];
    hipEvent_t ev[2] = {nullptr, nullptr};
    // switches (environment): TM_BATCH_PERSIST=1 / 0 forces the persistent
    // kernel / the graph of multi-instance launches (default: timed choice),
    // TM_BATCH_EAGER=1 replays the graph's iterations without capture,
    // TM_BATCH_SINGLE=1 uses per-instance launches; TM_BATCH_SPIN_LIMIT sets
    // the persistent kernel's barrier wait bound in polls (each at least
    // ~0.5 us: the default gives up after 0.5 s or more, far beyond any stage)
    int persist = -1;  // -1 timed choice, 1 persistent, 0 graph
    bool eager = false, single_launches = false;
    unsigned long long spin_limit = 1ull << 20;
};

namespace {

void drop_graph(tm_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_set.clear();
    b->pb_set.clear();
}

template <typename F>
int bguard(tm_batch *b, F &&f)
{
    if (!b) return TM_ERR_ARG;
    try {
        b->err.clear();
        TM_HIP(hipSetDevice(b->device));
        return f();
    } catch (const TmError &e) {
        b->err = e.msg;
        drop_graph(b);
        return e.status;
    } catch (const std::bad_alloc &) {
        b->err = "host allocation failed";
        drop_graph(b);
        return TM_ERR_OOM;
    } catch (...) {
        b->err = "unexpected internal error";
        drop_graph(b);
        return TM_ERR_HIP;
    }
}

void prepare_stages(tm_batch *b, std::vector<Solver> &S, const std::vector<int> &set, int R)
{
    std::vector<tm_ctx *> cs;
    for (int i : set) cs.push_back(S[i].c);
    for (int k = 0; k < 4; k++) {
        std::vector<DslashCall> dcs;
        for (int i : set) dcs.push_back(S[i].stage(k + 1));
        multi_dslash_prepare(b->md[k], cs, dcs, R, b->stream);
    }
}

void launch_iteration(tm_batch *b, std::vector<Solver> &S, const std::vector<int> &set)
{
    hipStream_t s = b->stream;
    if (b->single_launches) {
        for (int i : set) S[i].iteration(s);
        return;
    }
    std::vector<CgTail> t;
    for (int i : set)
        t.push_back(CgTail{S[i].c, S[i].w.dsc, S[i].w.partq, S[i].w.partb, S[i].nsb, S[i].nrhs, S[i].delta, S[i].w.p,
                           S[i].w.r, S[i].w.x});
    multi_dslash_launch(b->md[0], s);
    multi_dslash_launch(b->md[1], s);
    cg_finish_alpha_multi(t, s);
    multi_dslash_launch(b->md[2], s);
    multi_dslash_launch(b->md[3], s);
    cg_tail_multi(t, S[set[0]].w.prec, S[set[0]].w.xprec, s);
}

// right-hand sides per Dslash thread for the batch: the fastest (timed on the
// side-effect-free first stage) among the tiles that divide every nrhs
int choose_R(tm_batch *b, std::vector<Solver> &S, const std::vector<int> &set)
{
    const int prec = S[set[0]].lp;
    if (prec == TM_F64) return 1;
    if (const char *e = getenv("TM_BATCH_RHS_TILE")) {  // fixed tile, if it divides every nrhs
        const int R = atoi(e);
        bool ok = R >= 1 && R <= 3;
        for (int i : set) ok = ok && S[i].nrhs % R == 0;
        if (ok) return R;
    }
    std::vector<int> key{prec};
    for (int i : set) key.push_back(S[i].nrhs);
    auto it = b->tuned_R.find(key);
    if (it != b->tuned_R.end()) return it->second;
    hipEvent_t e0, e1;
    TM_HIP(hipEventCreate(&e0));
    TM_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bestR = 1;
    for (int R : {1, 2, 3}) {
        bool ok = true;
        for (int i : set) ok &= S[i].nrhs % R == 0;
        if (!ok) continue;
        prepare_stages(b, S, set, R);
        multi_dslash_launch(b->md[0], b->stream);
        TM_HIP(hipEventRecord(e0, b->stream));
        multi_dslash_launch(b->md[0], b->stream);
        multi_dslash_launch(b->md[0], b->stream);
        TM_HIP(hipEventRecord(e1, b->stream));
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
    b->tuned_R[key] = bestR;
    return bestR;
}

void build_graph(tm_batch *b, std::vector<Solver> &S, const std::vector<int> &set, int iters)
{
    drop_graph(b);
    const int R = b->single_launches ? 1 : choose_R(b, S, set);
    if (!b->single_launches) prepare_stages(b, S, set, R);
    TM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    try {
        for (int k = 0; k < iters; k++) launch_iteration(b, S, set);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    TM_HIP(hipStreamEndCapture(b->stream, &b->graph));
    TM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_set = set;
    b->graph_iters = iters;
    b->graph_R = R;
}

// the persistent kernel runs the FP32-arithmetic solvers (FP32, FP16 or
// BF16 storage); plain FP64 batches take the graph path
bool persist_usable(tm_batch *b, const std::vector<Solver> &S, const std::vector<int> &set)
{
    return b->persist != 0 && !b->eager && !b->single_launches && (int)set.size() <= kPersistInst &&
           S[set[0]].lp != TM_F64 && persist_supported(b->device);
}

std::vector<int> form_key(const std::vector<Solver> &S, const std::vector<int> &set)
{
    std::vector<int> key{S[set[0]].lp};
    for (int i : set) key.push_back(S[i].nrhs);
    return key;
}

// K iterations of the instances in `set` as one persistent launch; false
// (nothing run) if the runtime refuses the cooperative launch.  `timed`:
// record the start event after the set-up, right before the launch.
bool run_persist(tm_batch *b, std::vector<Solver> &S, const std::vector<int> &set, int K, bool timed)
{
    if (b->pb_set != set) {
        const int R = choose_R(b, S, set);
        std::vector<PersistInst> v;
        for (int i : set) {
            PersistInst q;
            q.c = S[i].c;
            for (int k = 0; k < 4; k++) q.st[k] = S[i].stage(k + 1);
            q.x = S[i].w.x;
            q.sc = S[i].w.dsc;
            q.delta = S[i].delta;
            v.push_back(q);
        }
        persist_prepare(b->pb, v, R, b->stream);
        b->pb_set = set;
    }
    if (timed) TM_HIP(hipEventRecord(b->ev[0], b->stream));
    if (!persist_launch(b->pb, K, b->spin_limit, b->stream)) return false;
    if (persist_failed(b->pb, b->stream))
        throw TmError{TM_ERR_HIP, "persistent batch kernel: a grid barrier wait exceeded its limit"};
    return true;
}

// Run all solvers to completion.
void run_batch(tm_batch *b, std::vector<Solver> &S)
{
    const int K = S[0].check_every;
    for (auto &x : S) TM_REQUIRE(x.check_every == K && x.lp == S[0].lp, "batched solves share precision and cadence");
    while (true) {
        std::vector<int> set;
        for (int i = 0; i < (int)S.size(); i++)
            if (!S[i].done) set.push_back(i);
        if (set.empty()) break;
        int room = K;
        for (int i : set) room = std::min(room, S[i].p.maxiter - S[i].total);
        if (room < K) {
            // the last iterations before maxiter: single-instance launches
            for (int i : set) {
                S[i].iteration(b->stream);
                S[i].count_iteration();
                if (S[i].due()) S[i].check(b->stream);
            }
            continue;
        }
        // the grouped iterations are accounted per instance below, not per
        // recorded launch (a graph is recorded once and replayed)
        for (int i : set) S[i].c->acct_pause++;
        try {
            // launch form: forced, tuned, or (untuned) the one not timed yet
            const std::vector<int> key = form_key(S, set);
            int form = 0;
            bool timing = false;
            if (persist_usable(b, S, set)) {
                auto it = b->tuned_form.find(key);
                if (b->persist == 1) {
                    form = 1;
                } else if (it != b->tuned_form.end()) {
                    form = it->second;
                } else {
                    form = b->form_ms[1].count(key) ? 0 : 1;
                    timing = true;
                }
            }
            bool ran = false;
            if (form == 1) {
                ran = run_persist(b, S, set, K, timing);
                if (!ran) b->persist = 0;  // refused: the graph path from now on
            }
            if (!ran && b->eager) {
                if (!b->single_launches) prepare_stages(b, S, set, choose_R(b, S, set));
                for (int k = 0; k < K; k++) launch_iteration(b, S, set);
            } else if (!ran) {
                if (b->graph_set != set || b->graph_iters != K) build_graph(b, S, set, K);
                if (timing) TM_HIP(hipEventRecord(b->ev[0], b->stream));  // graph set-up not timed
                TM_HIP(hipGraphLaunch(b->exec, b->stream));
            }
            if (timing && ran == (form == 1)) {
                TM_HIP(hipEventRecord(b->ev[1], b->stream));
                TM_HIP(hipEventSynchronize(b->ev[1]));
                float ms = 0;
                TM_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
                b->form_ms[form][key] = ms;
                if (b->form_ms[0].count(key) && b->form_ms[1].count(key))
                    b->tuned_form[key] = b->form_ms[1][key] < b->form_ms[0][key] ? 1 : 0;
            }
        } catch (...) {
            for (int i : set) S[i].c->acct_pause--;
            throw;
        }
        for (int i : set) {
            S[i].c->acct_pause--;
            double ib, ifl;
            S[i].iter_cost(ib, ifl);
            account(S[i].c, K * ib, K * ifl);
        }
        for (int i : set) {
            for (int k = 0; k < K; k++) S[i].count_iteration();
            S[i].check(b->stream);
        }
    }
    drop_graph(b);
}

}  // namespace

extern "C" int tm_batch_create(tm_batch **out, tm_ctx *const *ctxs, int n)
{
    if (!out || !ctxs || n < 1) return TM_ERR_ARG;
    *out = nullptr;
    for (int i = 0; i < n; i++) {
        if (!ctxs[i]) return TM_ERR_ARG;
        if (ctxs[i]->device != ctxs[0]->device) return TM_ERR_ARG;
        for (int j = 0; j < i; j++)
            if (ctxs[j] == ctxs[i]) return TM_ERR_ARG;  // instances need their own work buffers
    }
    tm_batch *b = new (std::nothrow) tm_batch();
    if (!b) return TM_ERR_OOM;
    b->ctx.assign(ctxs, ctxs + n);
    b->device = ctxs[0]->device;
    if (const char *e = getenv("TM_BATCH_PERSIST")) b->persist = atoi(e) != 0 ? 1 : 0;
    if (const char *e = getenv("TM_BATCH_SPIN_LIMIT")) b->spin_limit = strtoull(e, nullptr, 10);
    if (const char *e = getenv("TM_BATCH_BLOCKS_PER_CU")) b->pb.blocks_per_cu = atoi(e);
    if (const char *e = getenv("TM_BATCH_EAGER")) b->eager = atoi(e) != 0;
    if (const char *e = getenv("TM_BATCH_SINGLE")) b->single_launches = atoi(e) != 0;
    int st = bguard(b, [&]() {
        TM_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        TM_HIP(hipEventCreate(&b->ev[0]));
        TM_HIP(hipEventCreate(&b->ev[1]));
        return TM_OK;
    });
    if (st != TM_OK) {
        tm_batch_destroy(b);
        return st;
    }
    *out = b;
    return TM_OK;
}

extern "C" void tm_batch_destroy(tm_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    drop_graph(b);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

extern "C" const char *tm_batch_last_error(const tm_batch *b) { return b ? b->err.c_str() : "null batch"; }

extern "C" int tm_batch_solve(tm_batch *b, double *const *x, const double *const *src, const int *nrhs,
                              const tm_solve_params *p, tm_solve_stats *const *stats, tm_stream stream)
{
    return bguard(b, [&]() {
        const int n = (int)b->ctx.size();
        TM_REQUIRE(x && src && nrhs && p, "null pointer");
        for (int i = 0; i < n; i++) {
            TM_REQUIRE(x[i] && src[i] && x[i] != src[i], "bad solution/source pointer");
            TM_REQUIRE(nrhs[i] >= 1, "nrhs must be >= 1");
            TM_REQUIRE(b->ctx[i]->have_gauge, "no gauge field set");
        }
        TM_HIP(hipStreamSynchronize((hipStream_t)stream));
        hipStream_t s = b->stream;
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<Solver> S(n);
        std::vector<void *> xe(n), xo(n);
        std::vector<double> b0(n), f0(n);
        for (int i = 0; i < n; i++) {
            b0[i] = b->ctx[i]->acct_bytes;
            f0[i] = b->ctx[i]->acct_flops;
        }
        for (int i = 0; i < n; i++) {
            tm_ctx *c = b->ctx[i];
            const size_t hb = field_bytes(c, TM_F64, nrhs[i]);
            void *be = ws_get(c, "a_be", hb), *bo = ws_get(c, "a_bo", hb);
            xe[i] = ws_get(c, "a_xe", hb);
            xo[i] = ws_get(c, "a_xo", hb);
            launch_pack(c, be, bo, src[i], nrhs[i], TM_F64, nullptr, s);
            S[i].init(c, xe[i], xo[i], be, bo, nrhs[i], *p, s);
        }
        run_batch(b, S);
        int status = TM_OK;
        for (int i = 0; i < n; i++) {
            SolveOut r = S[i].finalize(s);
            launch_unpack(b->ctx[i], x[i], xe[i], xo[i], nrhs[i], TM_F64, s);
            TM_HIP(hipStreamSynchronize(s));
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (stats && stats[i])
                for (int k = 0; k < nrhs[i]; k++) {
                    stats[i][k] = r.st[k];
                    stats[i][k].seconds = secs;
                    stats[i][k].bytes = (b->ctx[i]->acct_bytes - b0[i]) / nrhs[i];
                    stats[i][k].flops = (b->ctx[i]->acct_flops - f0[i]) / nrhs[i];
                }
            if (r.status != TM_OK && status == TM_OK) status = r.status;
        }
        if (status == TM_ERR_NOCONV) b->err = "a right-hand side missed the tolerance within maxiter";
        return status;
    });
}

extern "C" int tm_batch_loops(tm_batch *b, const tm_loop_params *p, double *const *loops, tm_loop_stats *stats,
                              tm_stream stream)
{
    return bguard(b, [&]() {
        const int n = (int)b->ctx.size();
        TM_REQUIRE(p && loops, "null pointer");
        for (int i = 0; i < n; i++) {
            TM_REQUIRE(loops[i], "null loop output");
            TM_REQUIRE(p[i].n_hp >= 1 && p[i].n_lp == 0, "batched loops take high-precision noises only (n_lp = 0)");
            TM_REQUIRE(p[i].estimators > 0 && p[i].estimators < 16, "bad estimator mask");
            TM_REQUIRE(p[i].derivative == 0 || p[i].derivative == 1, "derivative must be 0 or 1");
            TM_REQUIRE(p[i].t_period == 0, "batched loops take volume sources (t_period = 0)");
            TM_REQUIRE(!(p[i].derivative && (p[i].estimators & TM_EST_HPE)),
                       "HPE takes ultra-local insertions only (derivative = 0)");
            TM_REQUIRE(p[i].dilution == TM_DIL_NONE || p[i].dilution == TM_DIL_SPIN_COLOUR, "bad dilution");
            TM_REQUIRE(p[i].mu_sign == 1 || p[i].mu_sign == -1, "mu_sign must be +1 or -1");
            TM_REQUIRE(p[i].noise_offset >= 0, "noise_offset must be >= 0");
            TM_REQUIRE(b->ctx[i]->have_gauge, "no gauge field set");
            if (p[i].estimators & TM_EST_HPE)
                for (int mu = 0; mu < 4; mu++) TM_REQUIRE(b->ctx[i]->geo.L[mu] >= 4, "HPE needs every L_mu >= 4");
        }
        TM_HIP(hipStreamSynchronize((hipStream_t)stream));
        hipStream_t s = b->stream;
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<Solver> S(n);
        std::vector<int> per_noise(n), nr(n);
        std::vector<void *> ee(n), eo(n), se(n), so(n);
        for (int i = 0; i < n; i++) {
            tm_ctx *c = b->ctx[i];
            c->stream = s;
            per_noise[i] = p[i].dilution == TM_DIL_SPIN_COLOUR ? 12 : 1;
            nr[i] = per_noise[i] * p[i].n_hp;
            const size_t one = field_bytes(c, TM_F64, per_noise[i]);
            ee[i] = ws_get(c, "b_eta_e", one * p[i].n_hp);
            eo[i] = ws_get(c, "b_eta_o", one * p[i].n_hp);
            se[i] = ws_get(c, "b_s_e", one * p[i].n_hp);
            so[i] = ws_get(c, "b_s_o", one * p[i].n_hp);
            for (int k = 0; k < p[i].n_hp; k++)
                launch_noise(c, (char *)ee[i] + one * k, (char *)eo[i] + one * k, p[i].seed,
                             (long)p[i].noise_offset + k, p[i].dilution, s);
            tm_solve_params hp = p[i].hp;
            hp.mu_sign = p[i].mu_sign;
            S[i].init(c, se[i], so[i], ee[i], eo[i], nr[i], hp, s);
        }
        run_batch(b, S);
        int status = TM_OK;
        for (int i = 0; i < n; i++) {
            tm_ctx *c = b->ctx[i];
            SolveOut r = S[i].finalize(s);
            if (r.status != TM_OK && status == TM_OK) status = r.status;
            const int Lt = c->geo.L[3];
            const size_t per = (size_t)n_insertions(p[i].derivative) * Lt;
            int n_est = 0, hpe_slot = -1;
            for (int k = 0; k < 4; k++)
                if ((p[i].estimators >> k) & 1) {
                    if ((1 << k) == TM_EST_HPE) hpe_slot = n_est;
                    n_est++;
                }
            const double epsp = eps_of(c, p[i].mu_sign);
            const size_t one = field_bytes(c, TM_F64, per_noise[i]);
            std::vector<cx<double>> acc(n_est * per, cx<double>{0, 0}), one_loop(n_est * per);
            for (int k = 0; k < p[i].n_hp; k++) {
                contract_noise(c, p[i].estimators, p[i].derivative, (char *)ee[i] + one * k, (char *)eo[i] + one * k,
                               (char *)se[i] + one * k, (char *)so[i] + one * k, per_noise[i], epsp, one_loop.data());
                for (size_t j = 0; j < acc.size(); j++) acc[j] = acc[j] + one_loop[j];
            }
            std::vector<cx<double>> ex(per);
            if (p[i].estimators & TM_EST_HPE) hpe_exact_part(c, epsp, ex.data());
            cx<double> *dst = (cx<double> *)loops[i];
            for (int k = 0; k < n_est; k++) {
                const bool hpe = k == hpe_slot;
                for (size_t j = 0; j < per; j++)
                    dst[k * per + j] = (1.0 / p[i].n_hp) * acc[k * per + j] + (hpe ? ex[j] : cx<double>{0, 0});
            }
            if (stats) {
                tm_loop_stats &q = stats[i];
                q = tm_loop_stats{};
                for (auto &x : r.st) {
                    q.n_solves_hp++;
                    q.iters_hp += x.iters;
                    q.max_res_hp = std::max(q.max_res_hp, x.true_rel_res);
                }
                q.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            }
        }
        TM_HIP(hipStreamSynchronize(s));
        if (status == TM_ERR_NOCONV) b->err = "a high-precision solve missed its tolerance";
        return status;
    });
}
