/*
 * FP64 CPU oracle - test infrastructure only (see oracle.c).
 * All arrays are canonical-layout complex doubles passed as interleaved
 * double pointers; L = {Lx, Ly, Lz, Lt}; t_bc = -1 antiperiodic in t, +1 periodic.
 */
#ifndef TM_ORACLE_H
#define TM_ORACLE_H
#include <stdint.h>

void or_site_parity(const int L[4], int *par_out);
void or_neighbours(const int L[4], long *nb_out);
void or_gamma(int n, double *out);
void or_twist(const int L[4], double eps, int which, const double *in, double *out);
void or_hop(const int L[4], double kappa, int t_bc, const double *U, const double *in,
            double *out, int adj);
void or_apply_M(const int L[4], double kappa, double eps, int t_bc, const double *U,
                const double *in, double *out, int adj);
void or_schur(const int L[4], double kappa, double eps, int t_bc, const double *U,
              const double *in, double *out, int adj, int form);
void or_source_prep(const int L[4], double kappa, double eps, int t_bc, const double *U,
                    const double *b, double *bhat, int form);
void or_reconstruct(const int L[4], double kappa, double eps, int t_bc, const double *U,
                    const double *b, const double *xe, double *full);
double or_cgnr(const int L[4], double kappa, double eps, int t_bc, const double *U,
               const double *b, double *x_full, double tol, int maxiter, int form,
               int *iters_out);
double or_cgnr_iterations(const int L[4], double kappa, double eps, int t_bc,
                          const double *U, const double *b, int niter);
uint64_t or_splitmix64(uint64_t seed, uint64_t c);
void or_noise_z4(const int L[4], uint64_t seed, long r, double *out);
void or_contract_std(const int L[4], const double *eta, const double *s, double *out);
void or_contract_oneend(const int L[4], double eps, const double *s, double *out);
void or_bh_power(const int L[4], double kappa, double eps, int t_bc, const double *U,
                 const double *in, double *out, int k);
void or_hpe_exact(const int L[4], double kappa, double eps, int t_bc, const double *U,
                  double *out);
void or_schur_at(const int L[4], double kappa, double eps, int t_bc, const double *U,
                 const double *x, const long *sites, long nsites, double *out);
void or_transport(const int L[4], int t_bc, const double *U, int k, const double *in, double *out,
                  int adj);
void or_ptc_forward(const int L[4], int t_bc, const double *U, int nc, const double *W1,
                    const double *W2, const double *in, double *out);
void or_ptc_at(const int L[4], int t_bc, const double *U, int nc, const double *W1, const double *W2,
               const double *in, const long *sites, long nsites, double *out);
double or_ptc_loss_grad(const int L[4], int t_bc, const double *U, int nc, const double *W1,
                        const double *W2, const double *in, const double *e, double *G1,
                        double *G2);
double or_ptc_res_loss_grad(const int L[4], double kappa, double eps, int t_bc, const double *U, int nc,
                            const double *W1, const double *W2, const double *in, double *G1, double *G2);
void or_set_threads(int n);
int or_get_threads(void);
#endif
