// Host runtime of the library: operators on half-lattice fields, the CG
// solvers and the loop driver.  Used by the C-ABI layer (abi.hip).
#pragma once

#include "tm_internal.h"

// eps' = mu_sign * eps
double eps_of(tm_ctx *c, int mu_sign);

// device scratch of the allocation-free entry points (noalloc.hip): bytes
// per device; setup looks the array's address up on `device` (once per
// device, TM_OK or TM_ERR_HIP); scratch returns it (null before setup)
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
int noalloc_setup(int device);
void *noalloc_scratch(int device);

// host helpers: wall clock; synchronous upload; download through the pinned
// stage (synchronises s); per-RHS |v|^2 on the host; bytes of a half field;
// asynchronous device copy
double now_s();
void upload(void *dev, const void *host, size_t bytes, hipStream_t s);
void download(tm_ctx *c, void *host, const void *dev, size_t bytes, hipStream_t s);
std::vector<double> norms_host(tm_ctx *c, const void *v, int prec, int nrhs, hipStream_t s);
size_t field_bytes(tm_ctx *c, int prec, int nrhs);
void copy_field(void *dst, const void *src, size_t bytes, hipStream_t s);
// chiral-basis Gamma_n = gamma_1^n0 gamma_2^n1 gamma_3^n2 gamma_4^n3
void gamma_n(int n, cx<double> G[4][4]);

// learned preconditioner out = N(in) on FP32 half fields (ptc.hip)
void ptc_apply_halves(tm_ctx *c, const void *in_e, const void *in_o, void *out_e, void *out_o, int nrhs,
                      hipStream_t s);

// out = D_hop Hop[in] (+ D_own own) on output parity out_par (see DslashCall)
void op_dslash(tm_ctx *c, void *out, const void *in, const void *own, int nrhs, int prec, int out_par,
               int dag, SpinDiag dhop, SpinDiag down, hipStream_t s, bool links18 = false);

// half-layout operators; tmp is an odd-parity scratch field of nrhs in prec
// (links18: FP64 with all 18 link parameters, the exact operator)
void op_schur(tm_ctx *c, void *out, const void *in, void *tmp, int nrhs, int prec, double epsp, hipStream_t s,
              bool links18 = false);
void op_schur_dag(tm_ctx *c, void *out, const void *in, void *tmp, int nrhs, int prec, double epsp,
                  hipStream_t s);
// (B H)^k on a full field given as halves (ping-pong in place), FP64
void op_bh_power(tm_ctx *c, void *se, void *so, int nrhs, double epsp, int k, hipStream_t s);

struct SolveOut {
    std::vector<tm_solve_stats> st;
    int status = TM_OK;
};

// CG work vectors of one solve (see runtime.hip)
struct CGWork {
    int nrhs = 0, prec = 0;
    void *q = nullptr, *p = nullptr, *r = nullptr, *rho = nullptr, *tmp = nullptr;
    void *x = nullptr;  // solution accumulator: FP64 (plain) or FP32 (low precision)
    int xprec = 0;
    CGScalars *dsc = nullptr;
    double *partq = nullptr, *partb = nullptr;
    bool rho_vec = true;  // the fused update also updates the vector rho
};

// State of one solve of M x = b on FP64 half fields: init, then iterations
// (each followed by count_iteration, and check when due), then finalize.
// The batched driver runs several of these with shared launches.
struct Solver {
    tm_ctx *c = nullptr;
    tm_solve_params p{};
    int nrhs = 0, lp = 0, check_every = 8, nsb = 0, total = 0, since_check = 0;
    bool done = false;
    double delta = 0, epsp = 0, t0 = 0;
    void *xe = nullptr, *xo = nullptr;
    const void *be = nullptr, *bo = nullptr;
    void *bh = nullptr, *t64 = nullptr, *rho64 = nullptr, *r64 = nullptr, *q64 = nullptr;
    double *dscale = nullptr;
    CGWork w{};
    std::vector<double> bn2, sigma, iter_res;
    std::vector<int> n_rel;
    std::vector<CGScalars> hsc;

    void init(tm_ctx *c, void *xe, void *xo, const void *be, const void *bo, int nrhs, const tm_solve_params &p,
              hipStream_t s);
    void iteration(hipStream_t s);       // one iteration, single-instance launches
    DslashCall stage(int k) const;       // the k-th (1..4) half-Dslash of an iteration
    void iteration_tail(hipStream_t s);  // finish_beta + x/p update
    // algorithmic bytes and flops of one iteration (the four half-Dslash
    // stages and the x/p update), as accounted by single-instance launches
    void iter_cost(double &bytes, double &flops) const;
    void count_iteration();
    bool due() const;
    void check(hipStream_t s);
    SolveOut finalize(hipStream_t s);

  private:
    // reactivate: right-hand sides whose true residual is above tol iterate
    // again (truncated solves); otherwise activity is kept
    void restart(bool first, hipStream_t s, bool reactivate = false);
    void accumulate(hipStream_t s);
};

// Restarted (flexible) GMRES on the full system (fgmres.hip)
SolveOut fgmres_halves(tm_ctx *c, void *xe, void *xo, const void *be, const void *bo, int nrhs,
                       const tm_solve_params &p, hipStream_t s);

// Solve M(mu_sign) x = b with b, x given as FP64 half fields (even, odd).
SolveOut solve_halves(tm_ctx *c, void *xe, void *xo, const void *be, const void *bo, int nrhs,
                      const tm_solve_params &p, hipStream_t s);

// Colour-traced Dirac outer products per time slice, C[t][b][a] = sum v_b w_a^*,
// FP64 halves -> host [Lt][16] complex
void outer_slices_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                       std::vector<cx<double>> &out, hipStream_t s, int t0 = 0, int dt = 1);
// Spin matrix inserted for Gamma_n: Gamma_n, gamma5 Gamma_n (one-end) or
// gamma5 Gamma_n gamma5 (generalised one-end)
enum GammaForm { G_PLAIN = 0, G_G5_LEFT = 1, G_G5_BOTH = 2 };
// Loops from outer products: L_n(t) = coef * sum_ab G[a][b] C[t][b][a] with
// G from GammaForm; C [Lt][16], out [16][Lt]
void loops_from_outer(tm_ctx *c, const cx<double> *C, GammaForm form, cx<double> coef, cx<double> *out);

// insertions per estimator: the 16 ultra-local Gamma_n, with derivative also
// the 4 x 16 one-derivative insertions (index 16 (1 + mu) + n)
inline int n_insertions(int derivative) { return derivative ? 80 : 16; }

// spatial momentum p = 2 pi (n_x / L_x, n_y / L_y, n_z / L_z)
struct Momentum {
    int n[3];
};
// all n with |n|^2 <= p2max, by |n|^2 then lexicographically; (0,0,0) first
std::vector<Momentum> momenta_list(int p2max);
// every |n_i| must stay below L_i / 2 (distinct momenta on the lattice)
void check_momenta(tm_ctx *c, int p2max);
// momentum-projected outer products, out [n_mom][Lt][16] (momentum.hip)
void outer_momenta_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                        const std::vector<Momentum> &mom, std::vector<cx<double>> &out, hipStream_t s);
// one-derivative outer products D_mu, out [n_mom][4 mu][Lt][16] (momentum.hip)
void outer_deriv_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                      const std::vector<Momentum> &mom, std::vector<cx<double>> &out, hipStream_t s);
// D_W f = f + H f (no twist) on FP64 half fields
void op_wilson(tm_ctx *c, void *oe, void *oo, const void *fe, const void *fo, int nrhs, hipStream_t s);
// exactly known part of the hopping expansion for ultra-local insertions
void hpe_exact_part(tm_ctx *c, double epsp, cx<double> *out /* [16][Lt] */);

// per-noise loops of one noise vector's sources (ee, eo) and solutions (se,
// so), estimators in mask order, into dst [n_est][n_ins][Lt], or with mom
// [n_est][n_mom][n_ins][Lt] (n_ins = n_insertions(derivative)); uses
// c->stream.  HPE takes ultra-local insertions only.
// Time-diluted sources of one solve batch: RHS group q (nsc RHS each) has its
// source on the slices t = o_first + q (mod period); the ultra-local STD and
// HPE contractions of group q then only visit those slices (the
// single-time-slice contraction), the source being zero elsewhere.
struct TimeDil {
    int period, o_first, n_off, nsc;
};
void contract_noise(tm_ctx *c, int estimators, int derivative, const void *ee, const void *eo, const void *se,
                    const void *so, int nrhs, double epsp, cx<double> *dst,
                    const std::vector<Momentum> *mom = nullptr, const TimeDil *td = nullptr);
hipStream_t s_of(tm_ctx *c);

// loops [n_est][n_ins][Lt] (mom = null) or [n_est][n_mom][n_ins][Lt]
int run_loops(tm_ctx *c, const tm_loop_params *p, double *loops, double *per_noise, tm_loop_stats *stats,
              hipStream_t s, const std::vector<Momentum> *mom = nullptr);
