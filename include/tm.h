/*
 * tm.h -- C-ABI of the MI355X (gfx950) twisted-mass solve and disconnected-loop
 * library.
 *
 * The library computes the data-parallel hot path of the stochastic
 * disconnected-quark-loop method of Alexandrou et al. (arXiv:1309.2256):
 * Z4 noise sources (sec. II.A), even-odd preconditioned twisted-mass
 * inversions by CG on the normal equations (sec. II.B and appendix A.1),
 * the Truncated Solver Method (sec. II.B, eq. estiTSM), the one-end trick
 * (sec. II.C, eq. loopVv), spin-colour dilution (sec. II.D) and the Hopping
 * Parameter Expansion (sec. II.E, eqs. HPE and loopHPE1), with the loops at
 * every time slice from volume sources.
 *
 * Operator (kappa normalisation; eps = 2 kappa mu, sec. II.E):
 *   M(+-mu) = R(+-eps) + H,  R(eps) = 1 + i eps gamma5,  B = R^-1,
 *   (H psi)(x) = -kappa sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                               +(1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *   chiral gamma basis: gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *   gamma_4 = [[0,1],[1,0]], gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1,1,-1,-1).
 *   Gamma_n = gamma1^n0 gamma2^n1 gamma3^n2 gamma4^n3 for n = n0+2n1+4n2+8n3.
 *   Fermion boundary: periodic in space; in time per tm_lattice.t_bc.
 * Even-odd system (appendix A.1, eq. A.2, "asymmetric"):
 *   Ahat = R_ee - H_eo R_oo^-1 H_oe,  bhat_e = b_e - H_eo R_oo^-1 b_o,
 *   psi_o = R_oo^-1 (b_o - H_oe psi_e).
 *
 * LAYOUTS
 *   Canonical (every full-lattice FP64 argument):
 *     site s = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2 (0 = even);
 *     spinor field  psi[rhs][s][spin 4][colour 3]   complex double (re, im);
 *     gauge field   U[mu 4][s][row 3][col 3]        complex double, U_mu(x)
 *                   on the link x -> x+mu; the boundary phase is NOT in U.
 *   Half-lattice (tm_dslash's HOP/SCHUR kinds, tm_pack/tm_unpack):
 *     one parity p, half-site index i = s >> 1 over the sites of parity p
 *     (unique because Lx is even), structure of arrays:
 *     element (rhs r, spin a, colour c, half-site i) at complex offset
 *     (r*12 + 3*a + c) * HS + i, each complex stored as (re, im) pairs of
 *     the precision given (double, float, IEEE binary16, bfloat16).
 *     HS = tm_half_stride(ctx) >= V/2 is V/2 rounded up to an odd multiple
 *     of 32; the HS - V/2 pad entries of each (r, a, c) plane are never read
 *     for a result and the library leaves their contents unspecified.  A
 *     half field of nrhs right-hand sides takes 12 * HS * nrhs complex.
 *
 * OWNERSHIP AND STREAMS
 *   Every pointer argument is owned by the caller; the library never frees
 *   or retains it past the call.  Device pointers must be on the context's
 *   device.  The library owns its own work buffers (allocated on first use,
 *   freed by tm_destroy).  All device work is enqueued on the stream given
 *   (0 = the null stream); tm_solve and tm_loops synchronise that stream
 *   before returning (they read convergence data), tm_dslash/tm_pack/
 *   tm_unpack/tm_set_gauge do not.
 *
 * ERRORS
 *   Every call returns a tm_status.  Arguments are validated before any
 *   launch; on failure tm_last_error(ctx) gives a message.  No C++ exception
 *   crosses this boundary.  A context is used by one host thread at a time.
 */
#ifndef TM_H
#define TM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tm_ctx tm_ctx;
typedef void *tm_stream; /* hipStream_t */

typedef enum {
    TM_OK = 0,
    TM_ERR_ARG = -1,         /* invalid argument (nothing was launched) */
    TM_ERR_HIP = -2,         /* a HIP runtime call failed */
    TM_ERR_OOM = -3,         /* device allocation failed */
    TM_ERR_NOCONV = -4,      /* a solve reached maxiter; x holds the last iterate */
    TM_ERR_NAN = -5,         /* NaN/Inf met in a solver reduction */
    TM_ERR_UNSUPPORTED = -6  /* valid request that the library does not implement   */
} tm_status;

typedef enum { TM_F64 = 0, TM_F32 = 1, TM_F16 = 2, TM_BF16 = 3 } tm_prec;

typedef struct {
    int L[4];            /* Lx, Ly, Lz, Lt: all even, Lx >= 2 */
    double kappa;        /* hopping parameter */
    double two_kappa_mu; /* eps = 2 kappa mu (twisted mass, kappa normalised) */
    int t_bc;            /* -1 antiperiodic in time (default), +1 periodic */
} tm_lattice;

/* Create a context on HIP device `device` for the given lattice.
 * Returns TM_ERR_ARG for odd or non-positive extents, TM_ERR_UNSUPPORTED when
 * one FP64 right-hand side of a half field (HS x 12 x 16 bytes) exceeds
 * 2^31 - 1 bytes (the kernels' 32-bit offsets; V <= 22369600 sites, e.g.
 * 48^3 x 96 fits, 64^3 x 128 does not). */
int tm_create(tm_ctx **ctx, const tm_lattice *lat, int device);

/* Destroy a context and free every buffer it owns.  NULL is ignored. */
void tm_destroy(tm_ctx *ctx);

/* Message for the last failing call on ctx ("" if none). */
const char *tm_last_error(const tm_ctx *ctx);

/* Plane stride HS of the half-lattice layout (see LAYOUTS): V/2 rounded up
 * to an odd multiple of 32 half-sites, so that the 12 planes of a field do
 * not sit a power of two apart in memory.  0 for a null context. */
int tm_half_stride(const tm_ctx *ctx);

/* Upload the gauge field.  U: device pointer, canonical [4][V][3][3] complex
 * double.  Builds the internal even-odd link layout (forward links and
 * pre-conjugated backward links per site, boundary phase folded in) in FP64,
 * and the FP32 and IEEE binary16 copies on first use by a kernel that reads
 * them (each rounded once from FP64, to nearest even).  Measures how far the
 * links are from SU(3) (max over links of |U U^dag - 1| and |det U - 1|,
 * entrywise) and synchronises the stream for that.  U is not retained. */
int tm_set_gauge(tm_ctx *ctx, const double *U, tm_stream stream);

/* Link format of the Dslash kernels (FP64 links for FP64 spinors, FP32 for
 * FP32, binary16 for FP16/BF16 unless tm_dslash asks for FP32 links; every
 * solve):
 *   18  all nine complex entries per link;
 *   12  (default) the first two rows only (appendix A.1, 12-parameter
 *       reconstruction): the third row of the special unitary link is
 *       rebuilt in the kernel as the complex conjugate of the cross product of
 *       the first two, times the time-boundary factor on links that cross
 *       t = Lt-1 <-> 0.  Used by the kernels of a precision only while the
 *       field's measured distance from SU(3) (tm_set_gauge) stays below that
 *       precision's rounding scale (FP64 1e-12, FP32 1e-6, binary16 1e-3);
 *       otherwise those kernels read all 18.  Reliable-update residuals and
 *       the final true residual of every solve always use all 18 FP64
 *       parameters.
 *   8   the FP64 kernels (plain solves, HPE, D_W, odd reconstruction) read
 *       8 real parameters per link (appendix A.1, 8-parameter
 *       reconstruction): a2, a3, b1 of U = [[a1,a2,a3],[b1,b2,b3],
 *       [c1,c2,c3]] and the phases of a1 and c1; |a1|, |c1| follow from
 *       the unit first row and column and the 2x2 block from the cofactor
 *       relations of a special unitary matrix (links with |c1| < |b1| are
 *       stored with their lower rows exchanged and negated, flagged in the
 *       stored phase).  The FP32/FP16/BF16 kernels read the 12-parameter
 *       form.  Used only while the field is special unitary to 1e-12 and
 *       every link has |a2|^2 + |a3|^2 >= 1e-10 (the reconstruction divides
 *       by it; exactly diagonal links such as a unit field keep 12).  The
 *       reconstructed links agree with the stored ones to ~1e-13.
 * FP16/BF16 spinors with FP32 links (tm_dslash, link_prec TM_F32) keep all
 * 18.  Returns TM_ERR_ARG for other values. */
int tm_set_link_format(tm_ctx *ctx, int params);

/* Links read by the FP16/BF16-spinor kernels of the solvers (TM_CG_MIXED and
 * TM_CG_LOW with FP16/BF16 storage) and of tm_dslash calls that do not ask
 * otherwise: TM_F16 (default) the binary16 copy in the tm_set_link_format
 * format, TM_F32 the FP32 copy with all 18 parameters (the FP32-link /
 * FP16-spinor operator).  Batches (tm_batch_*) take TM_F16 only
 * (TM_ERR_UNSUPPORTED otherwise).  TM_ERR_ARG for other values. */
int tm_set_half_spinor_links(tm_ctx *ctx, int link_prec);

/* Operator kinds of tm_dslash. */
typedef enum {
    TM_HOP_EO = 0,      /* out_e = H_eo in_o                     (half layout)  */
    TM_HOP_OE = 1,      /* out_o = H_oe in_e                     (half layout)  */
    TM_RINV_HOP_OE = 2, /* out_o = R_oo^-1 H_oe in_e             (half layout)  */
    TM_SCHUR = 3,       /* out_e = Ahat in_e                     (half layout)  */
    TM_SCHUR_DAG = 4,   /* out_e = Ahat^dag in_e = g5 Ahat(-mu) g5 in_e         */
    TM_NORMAL = 5,      /* out_e = Ahat^dag Ahat in_e            (half layout)  */
    TM_FULL = 6,        /* out = M in, canonical full FP64 spinors              */
    TM_FULL_DAG = 7,    /* out = M^dag in, canonical full FP64 spinors          */
    TM_RINV_HOP_EO = 8  /* out_e = R_ee^-1 H_eo in_o             (half layout)  */
} tm_dslash_kind;

/* Apply the operator of `kind` to nrhs right-hand sides.
 *   in, out     device pointers; half layout in spinor_prec for the half
 *               kinds, canonical FP64 for TM_FULL/TM_FULL_DAG (spinor_prec
 *               and link_prec must then be TM_F64).  in != out.
 *   mu_sign     +1: M_u (twist +eps), -1: M_d (twist -eps), sec. II.C.
 *   spinor_prec TM_F64 (link_prec TM_F64), TM_F32 (link_prec TM_F32), or
 *               TM_F16/TM_BF16 (link_prec TM_F16, the solvers' choice, or
 *               TM_F32); FP32/FP16/BF16 storage is computed in FP32.
 * Enqueued on `stream`; does not synchronise. */
int tm_dslash(tm_ctx *ctx, void *out, const void *in, int nrhs, int kind, int mu_sign,
              int spinor_prec, int link_prec, tm_stream stream);

/* tm_dslash without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, operator and results as tm_dslash (the same
 * kernels; the right-hand-side tile is the tuned one when tm_dslash already
 * tuned this case, else the default, bit-identical either way).  The
 * intermediate fields of TM_SCHUR, TM_SCHUR_DAG (one half field of nrhs in
 * spinor_prec), TM_NORMAL (two) and TM_FULL/TM_FULL_DAG (four FP64 half
 * fields), each rounded up to 256 bytes, come from one 64 MiB device array
 * per device that the library holds until the process ends; larger requests
 * return TM_ERR_UNSUPPORTED before anything is launched.  The link copy the
 * call reads must already exist (built by an earlier allocating call with the
 * same precisions, e.g. tm_dslash); otherwise TM_ERR_UNSUPPORTED.  Calls on
 * one device share the array: calls that overlap in time on that device
 * (other streams, other contexts, other host threads) race and must be
 * serialised by the caller.  Enqueued on `stream`; does not synchronise. */
int tm_dslash_noalloc(tm_ctx *ctx, void *out, const void *in, int nrhs, int kind, int mu_sign,
                      int spinor_prec, int link_prec, tm_stream stream);

/* Canonical full FP64 spinors [nrhs][V][4][3] -> two half-layout fields
 * (even, odd) in precision `prec`, each element multiplied by scale[r]
 * (scale may be NULL = 1).  Conversions round to nearest even. */
int tm_pack(tm_ctx *ctx, void *even, void *odd, const double *full, int nrhs, int prec,
            const double *scale_host, tm_stream stream);
/* Inverse of tm_pack (exact for FP64). */
int tm_unpack(tm_ctx *ctx, double *full, const void *even, const void *odd, int nrhs,
              int prec, tm_stream stream);

/* Solver schemes. */
typedef enum {
    TM_CG_F64 = 0,   /* plain FP64 CGNR on the even-odd system */
    TM_CG_MIXED = 1, /* CGNR with FP32 arithmetic and inner_prec storage, FP64
                        reliable updates (true residual recomputed in FP64);
                        FP16/BF16 storage reads binary16 links, FP32 storage
                        FP32 links */
    TM_CG_LOW = 2,   /* truncated low-precision CGNR (TSM low-precision solve):
                        inner_prec storage, FP32 arithmetic; when the iterated
                        residual meets tol the FP64 true residual is formed and
                        right-hand sides still above tol continue from it, so
                        the exit criterion holds for |b - M x| / |b| */
    TM_FGMRES = 3,   /* restarted GMRES(m) on the full system M x = b in FP64
                        (no preconditioner); the reference for TM_FGMRES_PTC */
    TM_FGMRES_PTC = 4 /* flexible GMRES(m) (Saad 1993) in FP64, right-
                        preconditioned by the parallel-transport network of
                        tm_ptc_* evaluated in FP32 (weights must be set) */
} tm_solver;

typedef struct {
    double tol;       /* target |b - M x| / |b| per right-hand side (> 0)        */
    int maxiter;      /* iteration cap (CG iterations, > 0)                      */
    int solver;       /* tm_solver                                               */
    int inner_prec;   /* TM_F32, TM_F16 or TM_BF16 storage (MIXED, LOW)          */
    double delta;     /* reliable-update trigger: update when the iterated Schur
                         residual falls below delta x its value at the last
                         update (MIXED; 0 selects 0.1)                           */
    int mu_sign;      /* +1 u flavour, -1 d flavour                              */
    int check_every;  /* CG: iterations between host convergence checks (0 = 8);
                         FGMRES: restart length m (0 = 16, at most 32)           */
} tm_solve_params;

typedef struct {
    int iters;            /* CG iterations (FGMRES: Arnoldi steps)              */
    int n_reliable;       /* reliable updates performed (FGMRES: restarts)      */
    int converged;        /* 1 when |b - M x| <= tol |b| at exit                 */
    int fallback;         /* TM_FGMRES_PTC: 1 when a restart cycle failed to halve
                             the residual and the plain mixed CG (FP16 storage,
                             FP64 reliable updates) finished the solve from the
                             current x; iters then adds its CG iterations        */
    double true_rel_res;  /* |b - M x| / |b| recomputed in FP64 at exit         */
    double iter_rel_res;  /* the solver's own (iterated) residual at exit       */
    double seconds;       /* wall time of the whole call                        */
    double bytes;         /* algorithmic device-memory bytes of the call's
                             kernels (every field and link read once and every
                             output written once per launch), this RHS's share
                             (the call's total / nrhs)                           */
    double flops;         /* the call's floating-point work / nrhs: per site
                             and RHS 1320 for the hopping term of a half-Dslash,
                             72 for its spin-diagonal coefficient, 96 for an
                             own-site term, 48 per fused norm or vector update;
                             vector kernels by their arithmetic (a complex
                             multiply 6, an add 2)                               */
} tm_solve_stats;

/* Solve M(mu_sign) x = b for nrhs right-hand sides at once.
 *   x, b   device, canonical full FP64 [nrhs][V][4][3]; x is output only.
 *   stats  host array of nrhs entries (may be NULL).
 * Returns TM_ERR_NOCONV if any right-hand side missed tol within maxiter
 * (x then holds the last iterates), TM_ERR_NAN on NaN/Inf. */
int tm_solve(tm_ctx *ctx, double *x, const double *b, int nrhs, const tm_solve_params *p,
             tm_solve_stats *stats, tm_stream stream);

/* Z4 noise vector number r (sec. II.A: entries from {1, i, -1, -i}) as
 * canonical full FP64 spinors; entry (site s, spin a, colour c) is i^k with k
 * the top two bits of SplitMix64 output ((r*V + s)*4 + a)*3 + c of the stream
 * seeded with `seed` (Steele, Lea & Flood 2014: output n is the finaliser of
 * seed + (n+1)*0x9e3779b97f4a7c15).  dilution = TM_DIL_SPIN_COLOUR writes
 * 12 sources, source d = 3a + c keeping only that component (sec. II.D).
 *   out  device, [1 or 12][V][4][3] complex double. */
int tm_noise(tm_ctx *ctx, double *out, uint64_t seed, long r, int dilution, tm_stream stream);

/* Loop estimators (bit mask). */
enum {
    TM_EST_STD = 1,     /* sum_x eta^dag Gamma_n s            (eq. loopSt)       */
    TM_EST_ONE_END = 2, /* 2 i eps sum_x s^dag gamma5 Gamma_n s  (eq. loopVv);
                           estimates Tr_t(Gamma M_d^-1) - Tr_t(Gamma M_u^-1)
                           for s = M_u^-1 eta (mu_sign = +1)                    */
    TM_EST_HPE = 4,     /* exact part + sum_x eta^dag Gamma_n (BH)^4 s (eqs. HPE,
                           loopHPE1); requires every L_mu >= 4; ultra-local
                           insertions only                                      */
    TM_EST_GEN_ONE_END = 8 /* 2 sum_x s^dag gamma5 Gamma_n gamma5 D_W s, D_W = 1 + H
                           (eq. loopStD, generalised one-end trick); estimates
                           Tr_t(Gamma M_u^-1) + Tr_t(Gamma M_d^-1)             */
};

/* Insertions per estimator.  derivative = 0: the 16 ultra-local Gamma_n.
 * derivative = 1: also the one-derivative insertions of appendix A.2 (the
 * covariant-derivative kernel), n_ins = 80, insertion 16 (1 + mu) + n for
 * direction mu = 0..3 (x, y, z, t): the bilinear w^dag Gamma_n D_mu v with
 * the symmetric left-right covariant derivative attributed to site x,
 *   1/4 [w^dag(x) G U_mu(x) v(x+mu) - w^dag(x) G U_mu(x-mu)^dag v(x-mu)
 *        - w^dag(x+mu) U_mu(x)^dag G v(x) + w^dag(x-mu) U_mu(x-mu) G v(x)],
 * time-boundary phase on links that cross t = Lt-1 <-> 0; (w, v, G) = (eta,
 * s, Gamma_n) for STD, (s, s, gamma5 Gamma_n) times 2 i eps for ONE_END,
 * (s, D_W s, gamma5 Gamma_n gamma5) times 2 for GEN_ONE_END. */

typedef enum { TM_DIL_NONE = 0, TM_DIL_SPIN_COLOUR = 1 } tm_dilution;

typedef struct {
    uint64_t seed;        /* Z4 noise stream seed                                 */
    int n_hp;             /* noises 0..n_hp-1 get high-precision solves           */
    int n_lp;             /* noises n_hp..n_hp+n_lp-1 get low-precision solves only;
                             noises 0..n_hp-1 also get a low-precision solve when
                             n_lp > 0 (TSM, eq. estiTSM).  n_lp = 0: plain HP.   */
    int noise_offset;     /* index of the first noise vector (resume support)     */
    int dilution;         /* tm_dilution                                          */
    int estimators;       /* TM_EST_* mask                                        */
    int mu_sign;          /* flavour inverted: +1 u, -1 d                         */
    int derivative;       /* 0: 16 ultra-local insertions; 1: also one-derivative
                             (80 insertions); not with TM_EST_HPE              */
    int t_period;         /* 0: volume sources.  P > 0 (a divisor of Lt): time
                             dilution with coherent sources (sec. II.D): each
                             noise (and spin-colour component) is split into P
                             sources, source o on the slices t = o (mod P), all
                             solved (in batches of up to 12 RHS) and summed;
                             P = Lt is plain time dilution.  The ultra-local
                             STD and HPE contractions visit only each source's
                             own slices (the single-time-slice contraction).  */
    tm_solve_params hp;   /* high-precision solve parameters                      */
    tm_solve_params lp;   /* low-precision solve parameters (n_lp > 0)            */
} tm_loop_params;

typedef struct {
    int n_solves_hp, n_solves_lp;
    int iters_hp, iters_lp;      /* summed CG iterations                          */
    double max_res_hp, max_res_lp; /* worst true relative residual               */
    double seconds;
} tm_loop_stats;

/* Estimate the disconnected loops L_n(t) for the 16 Gamma_n at every time
 * slice t from Z4 noise (volume sources, or time-diluted, see t_period).  Noise vector r has entries i^k, k the top two
 * bits of SplitMix64 output ((r*V + s)*4 + spin)*3 + colour of `seed`.
 *   loops      host, [n_est][n_ins][Lt] complex double, estimators in mask
 *              order (STD, ONE_END, HPE, GEN_ONE_END); the TSM combination
 *              (or plain mean).
 *   per_noise  host or NULL: [n_noise][2][n_est][n_ins][Lt] complex double,
 *              index 0 = high precision, 1 = low precision (zero when absent),
 *              n_noise = n_hp + n_lp.  The HPE entries hold only the
 *              stochastic part; its exact part is added to `loops` once.
 *   stats      host or NULL.
 * Returns TM_ERR_NOCONV when a high-precision solve missed its tolerance. */
int tm_loops(tm_ctx *ctx, const tm_loop_params *p, double *loops, double *per_noise,
             tm_loop_stats *stats, tm_stream stream);

/* Contract given full FP64 spinors (device, canonical, nrhs each) into
 * per-time-slice loops of the 16 ultra-local insertions for the estimators in
 * `estimators` (STD uses eta and s, ONE_END and GEN_ONE_END use s only and
 * GEN_ONE_END the gauge field; HPE is not accepted here).  Sums over the nrhs
 * pairs.  out: host [n_est][16][Lt] complex double. */
int tm_contract(tm_ctx *ctx, const double *eta, const double *s, int nrhs, int estimators,
                int mu_sign, double *out, tm_stream stream);

/* ---------------------------------------------------------------- momenta
 * Momentum projection of the loops (appendix A.2, contraction kernels, and
 * the Fourier step of appendix A.3): L_n(t, p) = sum_{x in t} e^{+i p.x} [loop density at x],
 * p = 2 pi (n_x / L_x, n_y / L_y, n_z / L_z), x = (x, y, z) in 0 .. L - 1,
 * for every integer vector n with |n|^2 <= p2max (the paper's cut-off in p^2,
 * in units of (2 pi / L)^2).  Momentum order: |n|^2 ascending, then n_x, n_y,
 * n_z ascending; (0, 0, 0) is first.  Every |n_i| must stay below L_i / 2. */

/* Momenta for p2max: *count receives their number; list (may be NULL)
 * receives [count][3] integers n and must hold *count entries on input. */
int tm_momenta(int p2max, int *count, int *list);

/* As tm_contract, momentum resolved and with the insertions of `derivative`
 * (0 or 1, see the insertion list above): out host [n_est][n_mom][n_ins][Lt]
 * complex double.  p2max = 0 gives the per-time-slice sums. */
int tm_contract_momentum(tm_ctx *ctx, const double *eta, const double *s, int nrhs, int estimators, int mu_sign,
                         int derivative, int p2max, double *out, tm_stream stream);

/* As tm_loops, momentum resolved: loops host [n_est][n_mom][n_ins][Lt];
 * per_noise host [n_noise][2][n_est][n_mom][n_ins][Lt] or NULL.  The exact
 * HPE part (the same at every site) enters p = 0 only. */
int tm_loops_momentum(tm_ctx *ctx, const tm_loop_params *p, int p2max, double *loops, double *per_noise,
                      tm_loop_stats *stats, tm_stream stream);

/* ---------------------------------------------------------------- batches
 * Uneven batches: several lattices (one context each, gauge set, same
 * device, distinct contexts) advanced together.  Each CG iteration of all
 * instances is one launch per half-Dslash stage over every lattice, and a
 * group of check_every iterations is captured once as a HIP graph and
 * replayed; per-RHS scalars stay on the device between groups.  Reliable
 * updates and convergence are decided per instance with the cadence of
 * tm_solve, so each instance gets the result of its own tm_solve bit for bit.
 * The batch owns a private HIP stream; calls synchronise the given stream on
 * entry and return after all work is complete. */
typedef struct tm_batch tm_batch;

/* ctxs: n >= 1 distinct contexts on one device (not retained beyond
 * tm_batch_destroy; they must outlive the batch). */
int tm_batch_create(tm_batch **batch, tm_ctx *const *ctxs, int n);
void tm_batch_destroy(tm_batch *batch);
const char *tm_batch_last_error(const tm_batch *batch);

/* Solve M_i(mu_sign) x_i = b_i for every instance i, nrhs[i] right-hand sides
 * each (canonical full FP64 device arrays).  One parameter set for all
 * instances (same solver, precision and check cadence).  stats[i]: host array
 * of nrhs[i] entries or NULL (stats itself may be NULL). */
int tm_batch_solve(tm_batch *batch, double *const *x, const double *const *b, const int *nrhs,
                   const tm_solve_params *p, tm_solve_stats *const *stats, tm_stream stream);

/* Per-instance loops (sec. II, as tm_loops) with p[i].n_hp noise vectors of
 * high-precision solves each (n_lp must be 0), all instances' sources solved
 * in one batch; p[i].hp must agree across instances in solver, inner_prec and
 * check_every; volume sources only (t_period = 0).  loops[i]: host
 * [n_est_i][n_ins_i][Lt_i] complex double; stats:
 * host array of n entries or NULL. */
int tm_batch_loops(tm_batch *batch, const tm_loop_params *p, double *const *loops,
                   tm_loop_stats *stats, tm_stream stream);

/* ---------------------------------------------------------------- learned preconditioner
 * A gauge-covariant parallel-transport convolution network (PTC, in the form
 * of Lehner and Wettig, arXiv:2302.05419) that approximates M^-1 and serves as
 * the right preconditioner of TM_FGMRES_PTC.  It is an addition to the 2013
 * method, acting on full-lattice fields.
 *   Paths: k = 0 identity; k = 1..4 (T_k f)(x) = U_mu(x) f(x+mu), mu = k-1;
 *   k = 5..8 (T_k f)(x) = U_mu(x-mu)^dag f(x-mu), mu = k-5; the time boundary
 *   phase of tm_lattice.t_bc multiplies hops across t = Lt-1 <-> 0.
 *   Two linear layers, one input channel, nc hidden channels, one output:
 *     phi_c = sum_k W1[k][c] T_k psi,   N(psi) = sum_{k,c} W2[k][c] T_k phi_c,
 *   W1, W2: host [9][nc][4][4] complex double, spin matrices (row-major)
 *   acting on the spin index only (gauge covariance allows no colour mixing).
 *   Loss of a pair (r, e): |N(r) - e|^2 / |e|^2; gradients are complex
 *   numbers dl/dRe(w) + i dl/dIm(w).
 * The device evaluates the collapsed form N = sum_k T_k sum_k' A[k][k'] T_k'
 * with A[k][k'] = sum_c W2[k][c] W1[k'][c] (exact: both layers are linear and
 * T_k commutes with spin matrices), transports in FP32, gradient sums in FP64. */

/* Arithmetic of the network's forward pass (tm_ptc_apply, the FGMRES
 * preconditioner, the training forward): TM_F32 (default; FP32 weights and
 * fields on the vector units) or TM_BF16 (the spin mixing u_k = sum_k'
 * A[k][k'] T_k' psi on the matrix cores, v_mfma_f32_16x16x32_bf16: A and the
 * transported fields rounded to bfloat16, FP32 accumulation; transports and
 * the gather stay FP32).  Gradients are FP32/FP64 either way.  TM_ERR_ARG for
 * other values. */
int tm_ptc_set_arith(tm_ctx *ctx, int prec);

/* Set / read the weights (1 <= nc <= 64). */
int tm_ptc_set_weights(tm_ctx *ctx, int nc, const double *W1, const double *W2);
int tm_ptc_get_weights(tm_ctx *ctx, int nc, double *W1, double *W2);
/* Weights of the hopping expansion of M^-1 to second order,
 * N = B - B H B + B H B H B with B = R(mu_sign eps)^-1 (sec. II.E), using
 * channels 0..8 (nc >= 9); the other entries of W1 get uniform values in
 * [-noise, noise] from SplitMix64(seed). */
int tm_ptc_init_hopping(tm_ctx *ctx, int nc, int mu_sign, uint64_t seed, double noise);
/* out = N(in): device canonical full FP64 [nrhs][V][4][3], computed in FP32. */
int tm_ptc_apply(tm_ctx *ctx, double *out, const double *in, int nrhs, tm_stream stream);
/* Training losses of a pair (r, e), r a residual and e = M^-1 r its error:
 *   TM_PTC_LOSS_ERROR     |N(r) - e|^2 / |e|^2
 *   TM_PTC_LOSS_RESIDUAL  |M N(r) - r|^2 / |r|^2 with M = M(mu_sign) (e unused): how far
 *                         M N is from the identity on r, what a right
 *                         preconditioner is judged by.  On the device M is the
 *                         FP32 even-odd operator and the gradient is carried
 *                         back through M^dag. */
enum { TM_PTC_LOSS_ERROR = 0, TM_PTC_LOSS_RESIDUAL = 1 };

/* Mean loss of kind `loss_kind` over npairs pairs (r[i], e[i]) (device
 * canonical full FP64; e may be NULL for TM_PTC_LOSS_RESIDUAL) and its
 * gradient; G1, G2: host [9][nc][4][4] complex double (may be NULL). */
int tm_ptc_loss_grad(tm_ctx *ctx, int loss_kind, int mu_sign, const double *r, const double *e, int npairs,
                     double *loss, double *G1, double *G2, tm_stream stream);
/* Training-pair store owned by the context: reserve room for `capacity`
 * pairs held in store_prec (TM_F32 or TM_BF16, round to nearest even); this
 * drops stored pairs.  tm_ptc_pairs_add appends n pairs (device canonical
 * full FP64 r, e; TM_ERR_ARG beyond capacity or for e = 0). */
int tm_ptc_pairs_reserve(tm_ctx *ctx, int capacity, int store_prec);
int tm_ptc_pairs_add(tm_ctx *ctx, const double *r, const double *e, int n, tm_stream stream);
/* Pairs from the solver's own iterates: solves M(p->mu_sign) x = b for the
 * nrhs right-hand sides b (device canonical full FP64) with p (TM_CG_F64 or
 * TM_CG_MIXED) to its tolerance for x*, then again from x = 0 with maxiter =
 * iters[j] for the iterates x_j (the solver is deterministic, so x_j is its
 * own iterate after iters[j] iterations), and appends the pairs
 * (r_j, e_j) = (b - M x_j, x* - x_j), r_j with all 18 FP64 link parameters,
 * to the pair store (at most nrhs * n_iters; pairs whose r or e rounds to
 * zero in the store precision are dropped).  *added (may be NULL) receives the
 * number appended.  TM_ERR_ARG beyond capacity or if the reference solve
 * does not converge. */
int tm_ptc_pairs_from_solve(tm_ctx *ctx, const double *b, int nrhs, const tm_solve_params *p, const int *iters,
                            int n_iters, int *added, tm_stream stream);

typedef struct {
    int epochs;        /* passes over the stored pairs (>= 1)                      */
    int batch;         /* pairs per optimiser step (1 <= batch <= stored pairs)    */
    double lr;         /* Adam step size (Kingma and Ba 2015)                      */
    double beta1, beta2, adam_eps; /* Adam moments and denominator guard            */
    uint64_t seed;     /* order of the batches within each epoch                   */
    int loss;          /* TM_PTC_LOSS_ERROR or TM_PTC_LOSS_RESIDUAL                */
    int mu_sign;       /* flavour of M in the residual loss (+1 u, -1 d)           */
} tm_ptc_train_params;

typedef struct {
    int steps;         /* optimiser steps taken                                    */
    int reserved;
    double loss_first; /* mean batch loss over the first epoch                     */
    double loss_last;  /* mean batch loss over the last epoch                      */
    double seconds;
} tm_ptc_train_stats;

/* Train the weights by Adam on the stored pairs: each epoch visits the
 * floor(n / batch) consecutive batches in an order drawn from `seed`; a step
 * minimises the batch mean of the loss of kind p->loss.  loss_per_step: host array of
 * epochs * floor(n / batch) doubles (loss of each batch before its step) or
 * NULL.  The weights start from the current ones (set or initialised). */
int tm_ptc_train(tm_ctx *ctx, const tm_ptc_train_params *p, tm_ptc_train_stats *stats, double *loss_per_step,
                 tm_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TM_H */
