// Host runtime of the library: operators on half-lattice fields, the CG
// solvers and the loop driver.  Used by the C-ABI layer (abi.hip).
#pragma once

#include "tm_internal.h"

// eps' = mu_sign * eps
double eps_of(tm_ctx *c, int mu_sign);

// out = D_hop Hop[in] (+ D_own own) on output parity out_par (see DslashCall)
void op_dslash(tm_ctx *c, void *out, const void *in, const void *own, int nrhs, int prec, int out_par,
               int dag, SpinDiag dhop, SpinDiag down, hipStream_t s);

// half-layout operators; tmp is an odd-parity scratch field of nrhs in prec
void op_schur(tm_ctx *c, void *out, const void *in, void *tmp, int nrhs, int prec, double epsp, hipStream_t s);
void op_schur_dag(tm_ctx *c, void *out, const void *in, void *tmp, int nrhs, int prec, double epsp,
                  hipStream_t s);
// (B H)^k on a full field given as halves (ping-pong in place), FP64
void op_bh_power(tm_ctx *c, void *se, void *so, int nrhs, double epsp, int k, hipStream_t s);

struct SolveOut {
    std::vector<tm_solve_stats> st;
    int status = TM_OK;
};

// Solve M(mu_sign) x = b with b, x given as FP64 half fields (even, odd).
SolveOut solve_halves(tm_ctx *c, void *xe, void *xo, const void *be, const void *bo, int nrhs,
                      const tm_solve_params &p, hipStream_t s);

// Colour-traced Dirac outer products per time slice, C[t][b][a] = sum v_b w_a^*,
// FP64 halves -> host [Lt][16] complex
void outer_slices_host(tm_ctx *c, const void *ve, const void *vo, const void *we, const void *wo, int nrhs,
                       std::vector<cx<double>> &out, hipStream_t s);
// Loops from outer products: L_n(t) = coef * sum_ab G[a][b] C[t][b][a] with
// G = Gamma_n (pre = false) or gamma5 Gamma_n (pre = true); out [16][Lt]
void loops_from_outer(tm_ctx *c, const std::vector<cx<double>> &C, bool g5pre, cx<double> coef,
                      cx<double> *out);
// exactly known part of the hopping expansion for ultra-local insertions
void hpe_exact_part(tm_ctx *c, double epsp, cx<double> *out /* [16][Lt] */);

int run_loops(tm_ctx *c, const tm_loop_params *p, double *loops, double *per_noise, tm_loop_stats *stats,
              hipStream_t s);
