"""FP64 CPU oracle for the twisted-mass disconnected-loop hot path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the HIP path; the only common inputs come from the seeded generators
in ``synth`` (gauge links), and the Z4 noise is re-derived here from the
published SplitMix64 definition.

Layouts are canonical numpy complex128 arrays:
  links   U[mu, site, row, col]   shape (4, V, 3, 3)
  spinor  psi[site, spin, colour] shape (V, 4, 3)
  loops   L[n, t]                  shape (16, Lt),  n the Gamma index
with site = x + Lx*(y + Ly*(z + Lz*t)).

The arithmetic lives in oracle.c (plain C, OpenMP over sites); this module
marshals arguments and writes out the estimator formulas of the paper:
  * stochastic estimate of M^-1 and the standard loop (section II.A, eqs.
    estiM and loopSt),
  * the Truncated Solver Method combination (section II.B, eq. estiTSM),
  * the one-end trick (section II.C, eq. loopVv) and its generalised form
    (eq. loopStD),
  * the Hopping Parameter Expansion (section II.E, eqs. HPE and loopHPE1),
  * one-derivative insertions (the covariant-derivative contraction of
    appendix A.2) and the momentum projection (the Fourier step of appendix A.3).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_c_int4 = ctypes.c_int * 4
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_gamma.argtypes = [ctypes.c_int, dp]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_twist.argtypes = [_c_int4, ctypes.c_double, ctypes.c_int, dp, dp]
        L.or_hop.argtypes = [_c_int4, ctypes.c_double, ctypes.c_int, dp, dp, dp, ctypes.c_int]
        L.or_apply_M.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 dp, dp, dp, ctypes.c_int]
        L.or_schur.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               dp, dp, dp, ctypes.c_int, ctypes.c_int]
        L.or_source_prep.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     dp, dp, dp, ctypes.c_int]
        L.or_reconstruct.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     dp, dp, dp, dp]
        L.or_cgnr.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                              dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int)]
        L.or_cgnr.restype = ctypes.c_double
        L.or_cgnr_iterations.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, dp, dp, ctypes.c_int]
        L.or_cgnr_iterations.restype = ctypes.c_double
        L.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_noise_z4.argtypes = [_c_int4, ctypes.c_uint64, ctypes.c_long, dp]
        L.or_contract_std.argtypes = [_c_int4, dp, dp, dp]
        L.or_contract_oneend.argtypes = [_c_int4, ctypes.c_double, dp, dp]
        L.or_bh_power.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  dp, dp, dp, ctypes.c_int]
        L.or_hpe_exact.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   dp, dp]
        L.or_schur_at.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  dp, dp, ctypes.POINTER(ctypes.c_long), ctypes.c_long, dp]
        L.or_transport.argtypes = [_c_int4, ctypes.c_int, dp, ctypes.c_int, dp, dp, ctypes.c_int]
        L.or_ptc_forward.argtypes = [_c_int4, ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp]
        L.or_ptc_at.argtypes = [_c_int4, ctypes.c_int, dp, ctypes.c_int, dp, dp, dp,
                                ctypes.POINTER(ctypes.c_long), ctypes.c_long, dp]
        L.or_ptc_loss_grad.argtypes = [_c_int4, ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp, dp,
                                       dp]
        L.or_ptc_loss_grad.restype = ctypes.c_double
        L.or_ptc_res_loss_grad.argtypes = [_c_int4, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                                           ctypes.c_int, dp, dp, dp, dp, dp]
        L.or_ptc_res_loss_grad.restype = ctypes.c_double
        L.or_site_parity.argtypes = [_c_int4, ctypes.POINTER(ctypes.c_int)]
        L.or_neighbours.argtypes = [_c_int4, ctypes.POINTER(ctypes.c_long)]
        _lib = L
    return _lib


def _p(a):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _L(L):
    return _c_int4(*[int(v) for v in L])


def volume(L):
    return int(np.prod(L))


def _cvec(x, shape):
    a = np.ascontiguousarray(x, dtype=np.complex128)
    assert a.shape == tuple(shape), (a.shape, shape)
    return a


def _spinor(L, x):
    return _cvec(x, (volume(L), 4, 3))


def _links(L, U):
    return _cvec(U, (4, volume(L), 3, 3))


# ---------------------------------------------------------------- geometry

def site_parity(L):
    out = np.zeros(volume(L), dtype=np.intc)
    lib().or_site_parity(_L(L), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def neighbours(L):
    """nb[s, 2*mu + 0] = s + mu, nb[s, 2*mu + 1] = s - mu (periodic wrap)."""
    out = np.zeros((volume(L), 8), dtype=np.int_)
    lib().or_neighbours(_L(L), out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    return out


def gamma(n):
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().or_gamma(int(n), _p(out))
    return out


# ---------------------------------------------------------------- operators

def twist(L, eps, psi, which=0):
    """which: 0 R, 1 R^dag, 2 R^-1, 3 (R^-1)^dag with R = 1 + i eps gamma5."""
    psi = _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_twist(_L(L), float(eps), int(which), _p(psi), _p(out))
    return out


def hop(L, kappa, t_bc, U, psi, adj=False):
    U, psi = _links(L, U), _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_hop(_L(L), float(kappa), int(t_bc), _p(U), _p(psi), _p(out), int(adj))
    return out


def apply_M(L, kappa, eps, t_bc, U, psi, adj=False):
    U, psi = _links(L, U), _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_apply_M(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(psi), _p(out),
                     int(adj))
    return out


def schur(L, kappa, eps, t_bc, U, psi, adj=False, form=0):
    """Even-site Schur complement applied to the even part of a full vector."""
    U, psi = _links(L, U), _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_schur(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(psi), _p(out),
                   int(adj), int(form))
    return out


def schur_at(L, kappa, eps, t_bc, U, psi, sites):
    """(Ahat psi)(s) for the even sites s in `sites` -> (n, 4, 3); for large lattices."""
    U, psi = _links(L, U), _spinor(L, psi)
    sites = np.ascontiguousarray(sites, dtype=np.int_)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    lib().or_schur_at(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(psi),
                      sites.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(sites), _p(out))
    return out


def source_prep(L, kappa, eps, t_bc, U, b, form=0):
    U, b = _links(L, U), _spinor(L, b)
    out = np.empty_like(b)
    lib().or_source_prep(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(b), _p(out),
                         int(form))
    return out


def reconstruct(L, kappa, eps, t_bc, U, b, xe):
    U, b, xe = _links(L, U), _spinor(L, b), _spinor(L, xe)
    out = np.empty_like(b)
    lib().or_reconstruct(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(b), _p(xe),
                         _p(out))
    return out


def cgnr(L, kappa, eps, t_bc, U, b, tol, maxiter=100000, form=0):
    """Solve M x = b; returns (x, iterations, true relative residual)."""
    U, b = _links(L, U), _spinor(L, b)
    x = np.empty_like(b)
    it = ctypes.c_int(0)
    res = lib().or_cgnr(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(b), _p(x),
                        float(tol), int(maxiter), int(form), ctypes.byref(it))
    return x, it.value, res


def cgnr_iterations(L, kappa, eps, t_bc, U, b, niter):
    U, b = _links(L, U), _spinor(L, b)
    return lib().or_cgnr_iterations(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(b),
                                    int(niter))


def bh_power(L, kappa, eps, t_bc, U, psi, k=4):
    U, psi = _links(L, U), _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_bh_power(_L(L), float(kappa), float(eps), int(t_bc), _p(U), _p(psi), _p(out),
                      int(k))
    return out


# ---------------------------------------------------------------- noise

def splitmix64(seed, c):
    return int(lib().or_splitmix64(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.c_uint64(c)))


def noise_z4(L, seed, r):
    out = np.empty((volume(L), 4, 3), dtype=np.complex128)
    lib().or_noise_z4(_L(L), ctypes.c_uint64(seed & (2**64 - 1)), int(r), _p(out))
    return out


def dilute_spin_colour(eta):
    """Spin-colour dilution: 12 sources, number d = 3*spin + colour keeps only
    that component of eta (section II.D)."""
    out = np.zeros((12,) + eta.shape, dtype=np.complex128)
    for a in range(4):
        for c in range(3):
            out[3 * a + c, :, a, c] = eta[:, a, c]
    return out


def dilute_time(L, etas, period):
    """Time dilution with coherent sources (section II.D): every source is
    split into `period` sources, number o keeping the slices t = o (mod
    period); period = Lt gives one slice per source."""
    t = np.arange(volume(L)) // (L[0] * L[1] * L[2])
    out = []
    for e in etas:
        for o in range(period):
            m = np.array(e, dtype=np.complex128, copy=True)
            m[t % period != o] = 0
            out.append(m)
    return out


def noise_sources(L, seed, r, dilution=False, t_period=0):
    """The sources of noise vector r: spin-colour and/or time diluted."""
    eta = noise_z4(L, seed, r)
    etas = list(dilute_spin_colour(eta)) if dilution else [eta]
    return dilute_time(L, etas, t_period) if t_period else etas


# ---------------------------------------------------------------- contractions

def contract_std(L, eta, s):
    """sum_{x in t} eta^dag Gamma_n s  ->  (16, Lt)"""
    out = np.zeros((16, L[3]), dtype=np.complex128)
    lib().or_contract_std(_L(L), _p(_spinor(L, eta)), _p(_spinor(L, s)), _p(out))
    return out


def contract_oneend(L, eps, s):
    """2 i eps sum_{x in t} s^dag gamma5 Gamma_n s  ->  (16, Lt)"""
    out = np.zeros((16, L[3]), dtype=np.complex128)
    lib().or_contract_oneend(_L(L), float(eps), _p(_spinor(L, s)), _p(out))
    return out


def hpe_exact(L, kappa, eps, t_bc, U):
    """sum_{x in t} tr[Gamma_n (B + (BH)^2 B)_xx]  ->  (16, Lt)"""
    out = np.zeros((16, L[3]), dtype=np.complex128)
    lib().or_hpe_exact(_L(L), float(kappa), float(eps), int(t_bc), _p(_links(L, U)),
                       _p(out))
    return out


# ---------------------------------------------------------------- estimators

EST_STD, EST_ONE_END, EST_HPE, EST_GEN_ONE_END = 1, 2, 4, 8
EST_ALL_ORDER = (EST_STD, EST_ONE_END, EST_HPE, EST_GEN_ONE_END)


def wilson(L, kappa, t_bc, U, psi):
    """D_W psi = (1 + H) psi: the operator M without its twisted-mass term."""
    return apply_M(L, kappa, 0.0, t_bc, U, psi)


def g5_field(psi):
    return np.einsum("ab,...bc->...ac", gamma(15), psi)


def contract_gen(L, kappa, t_bc, U, s):
    """2 sum_{x in t} s^dag gamma5 Gamma_n gamma5 D_W s (eq. loopStD) -> (16, Lt),
    written as 2 (gamma5 s)^dag Gamma_n (gamma5 D_W s) (gamma5 is Hermitian)."""
    s = _spinor(L, s)
    return 2.0 * contract_std(L, g5_field(s), g5_field(wilson(L, kappa, t_bc, U, s)))


def _nbr(L, sites, mu, step):
    """Site index of x + step * mu_hat for each site x in `sites` (periodic)."""
    c = [sites % L[0], (sites // L[0]) % L[1], (sites // (L[0] * L[1])) % L[2],
         sites // (L[0] * L[1] * L[2])]
    c[mu] = (c[mu] + step) % L[mu]
    return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))


def _phased_links(L, t_bc, U):
    """U_mu(x) with the fermion time-boundary factor on links from t = Lt-1 to 0."""
    U = _links(L, U).copy()
    t = _site_coords(L)[3]
    U[3, t == L[3] - 1] *= t_bc
    return U


def derivative_outer(L, t_bc, U, left, right, sites=None):
    """Spin matrices P_mu(x)[a][b] of the one-derivative bilinear with the
    symmetric left-right covariant derivative attributed to site x,
      left^dag G D_mu right (x) = sum_ab G[a][b] P_mu(x)[a][b],
      P_mu = 1/4 [ l(x)^* U_mu(x) r(x+mu) - l(x)^* U_mu(x-mu)^dag r(x-mu)
                   - l(x+mu)^* U_mu(x)^dag r(x) + l(x-mu)^* U_mu(x-mu) r(x) ]
    with colour contracted through the link in each term -> (4, n_sites, 4, 4)
    for the given sites (default: all, in site order)."""
    Uph = _phased_links(L, t_bc, U)
    l, r = _spinor(L, left), _spinor(L, right)
    x = np.arange(volume(L)) if sites is None else np.asarray(sites)
    out = np.zeros((4, len(x), 4, 4), dtype=np.complex128)

    def mv(W, f):          # colour matrix W(x) times f(x) on each spin: [b][c] = sum_d W_cd f_bd
        return f @ W.transpose(0, 2, 1)

    def outer(w, v):       # [a][b] = sum_c w*_{ac} v_{bc}
        return w.conj() @ v.transpose(0, 2, 1)

    for mu in range(4):
        xf, xb = _nbr(L, x, mu, 1), _nbr(L, x, mu, -1)
        Uf = Uph[mu][x]                                 # U_mu(x)
        Ubd = Uph[mu][xb].conj().transpose(0, 2, 1)     # U_mu(x - mu)^dag
        # l^dag(x+mu) U_mu(x)^dag = (U_mu(x) l(x+mu))^dag, and likewise backwards
        t1 = outer(l[x], mv(Uf, r[xf]))
        t2 = outer(l[x], mv(Ubd, r[xb]))
        t3 = outer(mv(Uf, l[xf]), r[x])
        t4 = outer(mv(Ubd, l[xb]), r[x])
        out[mu] = 0.25 * (t1 - t2 - t3 + t4)
    return out


def _gammas(form):
    g5 = gamma(15)
    Gs = [gamma(n) for n in range(16)]
    if form == "g5":
        Gs = [g5 @ G for G in Gs]
    elif form == "g5g5":
        Gs = [g5 @ G @ g5 for G in Gs]
    return np.array(Gs)


def insertion_densities(L, kappa, eps, t_bc, U, eta, s, estimator, derivative=False, sites=None):
    """Per-site loop densities of one (source, solution) pair -> (n_ins, V)
    (or (n_ins, n_sites) at the given sites),
    n_ins = 16 ultra-local Gamma_n, then (derivative) 16 per direction mu:
      STD      eta^dag X s                       (eq. loopSt)
      ONE_END  2 i eps s^dag gamma5 X s          (eq. loopVv)
      GEN      2 s^dag gamma5 X gamma5 D_W s     (eq. loopStD)
      HPE      eta^dag X (BH)^4 s                (eq. loopHPE1, ultra-local only)."""
    if estimator == EST_STD:
        left, right, form, coef = eta, s, "", 1.0
    elif estimator == EST_ONE_END:
        left, right, form, coef = s, s, "g5", 2j * eps
    elif estimator == EST_GEN_ONE_END:
        left, right, form, coef = s, wilson(L, kappa, t_bc, U, s), "g5g5", 2.0
    elif estimator == EST_HPE:
        assert not derivative, "HPE takes ultra-local insertions only"
        left, right, form, coef = eta, bh_power(L, kappa, eps, t_bc, U, s, 4), "", 1.0
    else:
        raise ValueError(estimator)
    Gs = _gammas(form)
    l, r = _spinor(L, left), _spinor(L, right)
    x = np.arange(volume(L)) if sites is None else np.asarray(sites)
    local = np.einsum("nab,xab->nx", Gs, l[x].conj() @ r[x].transpose(0, 2, 1))
    if not derivative:
        return coef * local
    P = derivative_outer(L, t_bc, U, l, r, x)
    der = np.einsum("nab,mxab->mnx", Gs, P).reshape(64, -1)
    return coef * np.concatenate([local, der])


def slice_sums(L, dens):
    """sum over each time slice (t is the slowest site index) -> (..., Lt)."""
    return dens.reshape(dens.shape[:-1] + (L[3], -1)).sum(axis=-1)


def loops_for_solution(L, kappa, eps, t_bc, U, etas, sols, estimators, derivative=False):
    """Per-noise loops from the sources of one noise vector (one entry per
    dilution component) and their solutions.  Returns {estimator: (n_ins, Lt)}.

    STD:     sum_d eta_d^dag Gamma s_d                  (eq. loopSt)
    ONE_END: 2 i eps sum_d s_d^dag gamma5 Gamma s_d     (eq. loopVv, lhs)
    HPE:     sum_d eta_d^dag Gamma (BH)^4 s_d           (eq. loopHPE1); the
             exactly known part is added once per estimate, not per noise.
    GEN:     2 sum_d s_d^dag gamma5 Gamma gamma5 D_W s_d (eq. loopStD)
    With derivative the one-derivative insertions follow the 16 local ones.
    """
    out = {}
    if estimators & EST_STD:
        out[EST_STD] = sum(contract_std(L, e, s) for e, s in zip(etas, sols))
    if estimators & EST_ONE_END:
        out[EST_ONE_END] = sum(contract_oneend(L, eps, s) for s in sols)
    if estimators & EST_HPE:
        assert not derivative, "HPE takes ultra-local insertions only"
        out[EST_HPE] = sum(contract_std(L, e, bh_power(L, kappa, eps, t_bc, U, s, 4))
                           for e, s in zip(etas, sols))
    if estimators & EST_GEN_ONE_END:
        out[EST_GEN_ONE_END] = sum(contract_gen(L, kappa, t_bc, U, s) for s in sols)
    if derivative:
        for e in (EST_STD, EST_ONE_END, EST_GEN_ONE_END):
            if estimators & e:
                der = sum(slice_sums(L, insertion_densities(L, kappa, eps, t_bc, U, et, s, e, True)[16:])
                          for et, s in zip(etas, sols))
                out[e] = np.concatenate([out[e], der])
    return out


# ---------------------------------------------------------------- momenta

def momenta(p2max):
    """Integer vectors n with |n|^2 <= p2max, ordered by |n|^2, then n_x,
    n_y, n_z ascending ((0, 0, 0) first) -> (n_mom, 3)."""
    n = int(np.floor(np.sqrt(p2max)))
    out = []
    for n2 in range(p2max + 1):
        for nx in range(-n, n + 1):
            for ny in range(-n, n + 1):
                for nz in range(-n, n + 1):
                    if nx * nx + ny * ny + nz * nz == n2:
                        out.append((nx, ny, nz))
    return np.array(out, dtype=int).reshape(-1, 3)


def _site_coords(L):
    s = np.arange(volume(L))
    return (s % L[0], (s // L[0]) % L[1], (s // (L[0] * L[1])) % L[2], s // (L[0] * L[1] * L[2]))


def _bilinear(L, left, right, G):
    """Per-site left(x)^dag G right(x) summed over spin and colour -> (V,)."""
    left, right = _spinor(L, left), _spinor(L, right)
    return np.einsum("xac,ab,xbc->x", left.conj(), G, right)


def project_momenta(L, dens, moms, slices=None):
    """sum_{x in t} e^{+i p.x} dens[..., x], p = 2 pi n / L -> (..., n_mom, Lt).
    With `slices`, dens holds the sites of those time slices only (in site
    order) and the other slices stay zero."""
    Vs = L[0] * L[1] * L[2]
    ts = list(range(L[3])) if slices is None else list(slices)
    sites = np.concatenate([np.arange(t * Vs, (t + 1) * Vs) for t in ts])
    x, y, z = sites % L[0], (sites // L[0]) % L[1], (sites // (L[0] * L[1])) % L[2]
    out = np.zeros(dens.shape[:-1] + (len(moms), L[3]), dtype=np.complex128)
    for m, (nx, ny, nz) in enumerate(moms):
        ph = np.exp(2j * np.pi * (nx * x / L[0] + ny * y / L[1] + nz * z / L[2]))
        # one row of Vs sites per listed time slice
        out[..., m, ts] = (dens * ph).reshape(dens.shape[:-1] + (len(ts), Vs)).sum(axis=-1)
    return out


def slice_sites(L, slices):
    """Site indices of the given time slices, in site order."""
    Vs = L[0] * L[1] * L[2]
    return np.concatenate([np.arange(t * Vs, (t + 1) * Vs) for t in slices])


def contract_momentum(L, eps, eta, s, estimators, moms):
    """Momentum-resolved loops of given fields (no solve):
    STD: sum_{x in t} e^{ip.x} eta^dag Gamma_n s;  ONE_END: 2 i eps sum e^{ip.x}
    s^dag gamma5 Gamma_n s.  Returns {estimator: (n_mom, 16, Lt)}."""
    g5 = gamma(15)
    out = {}
    if estimators & EST_STD:
        d = np.stack([_bilinear(L, eta, s, gamma(n)) for n in range(16)])
        out[EST_STD] = np.transpose(project_momenta(L, d, moms), (1, 0, 2))
    if estimators & EST_ONE_END:
        d = np.stack([_bilinear(L, s, s, g5 @ gamma(n)) for n in range(16)]) * (2j * eps)
        out[EST_ONE_END] = np.transpose(project_momenta(L, d, moms), (1, 0, 2))
    return out


def contract_insertions(L, kappa, eps, t_bc, U, eta, s, estimators, derivative, moms,
                        slices=None):
    """Momentum-resolved loops of given fields for any estimators and
    insertions -> {estimator: (n_mom, n_ins, Lt)}; with `slices` only those
    time slices are evaluated (the others are zero)."""
    out = {}
    sites = None if slices is None else slice_sites(L, slices)
    for e in EST_ALL_ORDER:
        if estimators & e:
            d = insertion_densities(L, kappa, eps, t_bc, U, eta, s, e, derivative, sites)
            out[e] = np.transpose(project_momenta(L, d, moms, slices), (1, 0, 2))
    return out


def loops_momentum_for_solution(L, kappa, eps, t_bc, U, etas, sols, estimators, moms,
                                derivative=False):
    """As loops_for_solution, momentum resolved: {estimator: (n_mom, n_ins, Lt)}."""
    out = {}
    for e, s in zip(etas, sols):
        part = contract_insertions(L, kappa, eps, t_bc, U, e, s, estimators, derivative, moms)
        for k, v in part.items():
            out[k] = out.get(k, 0) + v
    return out


def loops_momentum(L, kappa, eps, t_bc, U, seed, n_noise, tol, estimators, moms, dilution=False,
                   derivative=False, t_period=0):
    """As loops, momentum resolved ({estimator: (n_mom, 16, Lt)}).  The exact
    HPE part is the same at every site of a slice, so its Fourier sum over the
    slice vanishes for p != 0 and it enters p = 0 only."""
    per_noise = []
    for r in range(n_noise):
        etas = noise_sources(L, seed, r, dilution, t_period)
        sols, _, _ = solve_sources(L, kappa, eps, t_bc, U, etas, tol)
        per_noise.append(loops_momentum_for_solution(L, kappa, eps, t_bc, U, etas, sols,
                                                     estimators, moms, derivative))
    mean = {e: sum(p[e] for p in per_noise) / n_noise for e in per_noise[0]}
    if estimators & EST_HPE:
        assert tuple(moms[0]) == (0, 0, 0)
        mean[EST_HPE] = mean[EST_HPE].copy()
        mean[EST_HPE][0] += hpe_exact(L, kappa, eps, t_bc, U)
    return mean, per_noise


def tsm_combine(hp_loops, lp_of_hp_loops, lp_only_loops):
    """Truncated Solver Method (eq. estiTSM), applied to any loop functional:
       (1/N_HP) sum_{r<=N_HP} [L(s_HP,r) - L(s_LP,r)] + (1/N_LP) sum_{r>N_HP} L(s_LP,r).
    With no LP-only noises the plain estimate (1/N_HP) sum L(s_HP,r) is
    returned; with no HP noises, the (biased) LP mean."""
    n_hp, n_lp = len(hp_loops), len(lp_only_loops)
    if n_lp == 0:
        return sum(hp_loops) / n_hp
    if n_hp == 0:
        return sum(lp_only_loops) / n_lp
    corr = sum(h - l for h, l in zip(hp_loops, lp_of_hp_loops)) / n_hp
    return corr + sum(lp_only_loops) / n_lp


def solve_sources(L, kappa, eps, t_bc, U, srcs, tol, maxiter=100000):
    sols, its, res = [], [], []
    for b in srcs:
        x, it, r = cgnr(L, kappa, eps, t_bc, U, b, tol, maxiter)
        sols.append(x)
        its.append(it)
        res.append(r)
    return sols, its, res


def loops(L, kappa, eps, t_bc, U, seed, n_noise, tol, estimators, dilution=False,
          noise_offset=0, derivative=False, t_period=0):
    """Plain stochastic loop estimate from n_noise Z4 noise vectors solved to
    tol (mean over noises, eq. estiM / loopSt / loopVv / loopHPE1 / loopStD).
    Returns ({estimator: (n_ins, Lt)}, per_noise list of {estimator: (n_ins, Lt)}),
    n_ins = 16, or 80 with the one-derivative insertions."""
    per_noise = []
    for r in range(noise_offset, noise_offset + n_noise):
        etas = noise_sources(L, seed, r, dilution, t_period)
        sols, _, _ = solve_sources(L, kappa, eps, t_bc, U, etas, tol)
        per_noise.append(loops_for_solution(L, kappa, eps, t_bc, U, etas, sols, estimators,
                                            derivative))
    mean = {e: sum(p[e] for p in per_noise) / n_noise for e in per_noise[0]}
    if estimators & EST_HPE:
        mean[EST_HPE] = mean[EST_HPE] + hpe_exact(L, kappa, eps, t_bc, U)
    return mean, per_noise


# ---------------------------------------------------------------- learned preconditioner

def transport(L, t_bc, U, k, psi, adj=False):
    """Path k: 0 identity, 1..4 hop in +mu, 5..8 hop in -mu (parallel transported)."""
    U, psi = _links(L, U), _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_transport(_L(L), int(t_bc), _p(U), int(k), _p(psi), _p(out), int(adj))
    return out


def _weights(W, nc):
    W = np.ascontiguousarray(W, dtype=np.complex128)
    assert W.shape == (9, nc, 4, 4), W.shape
    return W


def ptc_forward(L, t_bc, U, W1, W2, psi):
    """Two linear parallel-transport layers 1 -> nc -> 1 (weights [9][nc][4][4])."""
    nc = W1.shape[1]
    W1, W2 = _weights(W1, nc), _weights(W2, nc)
    U, psi = _links(L, U), _spinor(L, psi)
    out = np.empty_like(psi)
    lib().or_ptc_forward(_L(L), int(t_bc), _p(U), nc, _p(W1), _p(W2), _p(psi), _p(out))
    return out


def ptc_at(L, t_bc, U, W1, W2, psi, sites):
    """N(psi) at the given sites only (site by site from the definition) -> (n, 4, 3)."""
    nc = W1.shape[1]
    W1, W2 = _weights(W1, nc), _weights(W2, nc)
    U, psi = _links(L, U), _spinor(L, psi)
    sites = np.ascontiguousarray(sites, dtype=np.int_)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    lib().or_ptc_at(_L(L), int(t_bc), _p(U), nc, _p(W1), _p(W2), _p(psi),
                    sites.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(sites), _p(out))
    return out


def ptc_loss_grad(L, t_bc, U, W1, W2, rs, es):
    """Mean over pairs of |N(r) - e|^2 / |e|^2 and its gradient (complex
    dl/dRe w + i dl/dIm w) for W1 and W2."""
    nc = W1.shape[1]
    W1, W2 = _weights(W1, nc), _weights(W2, nc)
    U = _links(L, U)
    G1 = np.zeros_like(W1)
    G2 = np.zeros_like(W2)
    loss = 0.0
    for r, e in zip(rs, es):
        loss += lib().or_ptc_loss_grad(_L(L), int(t_bc), _p(U), nc, _p(W1), _p(W2),
                                       _p(_spinor(L, r)), _p(_spinor(L, e)), _p(G1), _p(G2))
    n = len(rs)
    return loss / n, G1 / n, G2 / n


def ptc_res_loss_grad(L, kappa, eps, t_bc, U, W1, W2, rs):
    """Mean over residuals of |M N(r) - r|^2 / |r|^2 and its gradient (complex
    dl/dRe w + i dl/dIm w) for W1 and W2."""
    nc = W1.shape[1]
    W1, W2 = _weights(W1, nc), _weights(W2, nc)
    U = _links(L, U)
    G1 = np.zeros_like(W1)
    G2 = np.zeros_like(W2)
    loss = 0.0
    for r in rs:
        loss += lib().or_ptc_res_loss_grad(_L(L), float(kappa), float(eps), int(t_bc), _p(U), nc, _p(W1),
                                           _p(W2), _p(_spinor(L, r)), _p(G1), _p(G2))
    n = len(rs)
    return loss / n, G1 / n, G2 / n


def set_threads(n):
    """OpenMP threads of the oracle (timing of the CPU baseline)."""
    lib().or_set_threads(int(n))


def get_threads():
    return lib().or_get_threads()
