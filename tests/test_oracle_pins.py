"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each checks it against
something independent of its code -- a closed form (free-field spectrum and
traces, the hopping-expansion constants), an identity of the method
(gamma5-hermiticity, M^dag M = D_W^dag D_W + eps^2, the one-end identity,
the hopping expansion, gauge covariance), a dense brute-force computation
(LU inverse on tiny lattices), published generator outputs, or statistics of
the estimators.
"""
import os

import numpy as np
import pytest

import oracle as O
import synth as S

G5 = np.diag([1, 1, -1, -1]).astype(complex)
HERE = os.path.dirname(os.path.abspath(__file__))


def dense(f, L):
    """Dense matrix of a linear map on spinor fields, column by column."""
    V = int(np.prod(L))
    n = 12 * V
    D = np.zeros((n, n), dtype=complex)
    for i in range(n):
        e = np.zeros(n, dtype=complex)
        e[i] = 1
        D[:, i] = f(e.reshape(V, 4, 3)).ravel()
    return D


def slice_traces(L, A):
    """Tr_t(Gamma_n A) = sum_{x in t} tr[(Gamma_n (x) 1_c) A_xx] for a dense A."""
    V, Lt = int(np.prod(L)), L[3]
    out = np.zeros((16, Lt), dtype=complex)
    blocks = np.array([A[12 * x:12 * x + 12, 12 * x:12 * x + 12] for x in range(V)])
    for n in range(16):
        Gc = np.kron(O.gamma(n), np.eye(3))
        per_site = np.einsum("ij,xji->x", Gc, blocks)
        out[n] = per_site.reshape(Lt, -1).sum(1)
    return out


def g5(psi):
    return np.einsum("ab,...bc->...ac", G5, psi)


def momenta(L, t_bc):
    ps = []
    for nx in range(L[0]):
        for ny in range(L[1]):
            for nz in range(L[2]):
                for nt in range(L[3]):
                    pt = (2 * nt + (1 if t_bc == -1 else 0)) * np.pi / L[3]
                    ps.append([2 * np.pi * nx / L[0], 2 * np.pi * ny / L[1],
                               2 * np.pi * nz / L[2], pt])
    return np.array(ps)


# ---------------------------------------------------------------- gamma algebra

def test_gamma_algebra():
    g = [O.gamma(1 << mu) for mu in range(4)]
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * np.eye(4) * (m == n), atol=0)
    assert np.array_equal(O.gamma(0), np.eye(4))
    assert np.allclose(O.gamma(15), G5, atol=0)  # gamma5 = g1 g2 g3 g4 is diag(1,1,-1,-1)
    for m in range(16):
        for n in range(16):
            tr = np.trace(O.gamma(m).conj().T @ O.gamma(n))
            assert abs(tr - 4 * (m == n)) < 1e-14
    # chiral basis: gamma_4 couples upper and lower spin pairs
    assert np.allclose(O.gamma(8), np.block([[np.zeros((2, 2)), np.eye(2)],
                                             [np.eye(2), np.zeros((2, 2))]]))


# ---------------------------------------------------------------- free field

@pytest.mark.parametrize("t_bc", [-1, +1])
def test_free_field_singular_values(t_bc):
    """U = 1: singular values of M are sqrt(A^2 + eps^2 + sum_mu (2 kappa sin p_mu)^2),
    A = 1 - 2 kappa sum_mu cos p_mu, each 12-fold; p_t odd multiples of pi/Lt
    for antiperiodic time."""
    L, kappa, eps = (4, 2, 2, 4), 0.13, 0.05
    M = dense(lambda v: O.apply_M(L, kappa, eps, t_bc, S.unit_links(L), v), L)
    sv = np.sort(np.linalg.svd(M, compute_uv=False))
    p = momenta(L, t_bc)
    A = 1 - 2 * kappa * np.cos(p).sum(1)
    ex = np.sqrt(A ** 2 + eps ** 2 + 4 * kappa ** 2 * (np.sin(p) ** 2).sum(1))
    assert np.abs(sv - np.sort(np.repeat(ex, 12))).max() < 1e-13


def test_free_field_slice_traces_full_dilution():
    """Every unit source solved by the oracle CG and contracted with the standard
    estimator gives Tr_t(Gamma_n M^-1) exactly; for U = 1 that is
    (12/Lt) sum_p A/den for n=0, -(12 i eps/Lt) sum_p 1/den for gamma5, 0 else."""
    L, kappa, eps = (2, 2, 2, 4), 0.125, 0.1
    U = S.unit_links(L)
    V = int(np.prod(L))
    tot = np.zeros((16, L[3]), dtype=complex)
    for i in range(12 * V):
        e = np.zeros((V, 4, 3), dtype=complex)
        e.reshape(-1)[i] = 1
        x, _, res = O.cgnr(L, kappa, eps, -1, U, e, 1e-13)
        assert res < 1e-12
        tot += O.contract_std(L, e, x)
    p = momenta(L, -1)
    A = 1 - 2 * kappa * np.cos(p).sum(1)
    den = A ** 2 + eps ** 2 + 4 * kappa ** 2 * (np.sin(p) ** 2).sum(1)
    ex0 = 12.0 / L[3] * (A / den).sum()
    ex15 = -12j * eps / L[3] * (1 / den).sum()
    assert np.abs(tot[0] - ex0).max() < 1e-10
    assert np.abs(tot[15] - ex15).max() < 1e-10
    assert np.abs(tot[1:15]).max() < 1e-10


# ---------------------------------------------------------------- operator identities

@pytest.fixture(scope="module")
def small():
    L = (4, 2, 2, 4)
    return dict(L=L, kappa=0.124, eps=0.07, U=S.gauge_links(L, 0.4, 11))


def test_adjoint_and_gamma5_hermiticity(small):
    L, kappa, eps, U = small["L"], small["kappa"], small["eps"], small["U"]
    v, w = S.random_spinor(L, 1), S.random_spinor(L, 2)
    # the adjoint apply is the adjoint: <v, M w> = <M^dag v, w>
    Mw = O.apply_M(L, kappa, eps, -1, U, w)
    Mdv = O.apply_M(L, kappa, eps, -1, U, v, adj=True)
    assert abs(np.vdot(v, Mw) - np.vdot(Mdv, w)) < 1e-12
    # M(mu)^dag = gamma5 M(-mu) gamma5
    assert np.abs(Mdv - g5(O.apply_M(L, kappa, -eps, -1, U, g5(v)))).max() < 1e-14
    par = O.site_parity(L)
    ve, we = v.copy(), w.copy()
    ve[par == 1] = 0
    we[par == 1] = 0
    for form in (0, 1):
        Aw = O.schur(L, kappa, eps, -1, U, we, form=form)
        Adv = O.schur(L, kappa, eps, -1, U, ve, adj=True, form=form)
        assert abs(np.vdot(ve, Aw) - np.vdot(Adv, we)) < 1e-12
        assert np.abs(Aw[par == 1]).max() == 0
    # asymmetric Schur complement: Ahat(mu)^dag = gamma5 Ahat(-mu) gamma5
    Adv = O.schur(L, kappa, eps, -1, U, ve, adj=True)
    assert np.abs(Adv - g5(O.schur(L, kappa, -eps, -1, U, g5(ve)))).max() < 1e-14


def test_normal_operator_identity(small):
    """M^dag M = D_W^dag D_W + eps^2 (twist and Wilson operator anticommute
    up to the mass term), so sigma_min(M) >= eps."""
    L, kappa, eps, U = small["L"], small["kappa"], small["eps"], small["U"]
    v = S.random_spinor(L, 3)
    MdM = O.apply_M(L, kappa, eps, -1, U, O.apply_M(L, kappa, eps, -1, U, v), adj=True)
    DdD = O.apply_M(L, kappa, 0.0, -1, U, O.apply_M(L, kappa, 0.0, -1, U, v), adj=True)
    assert np.abs(MdM - DdD - eps ** 2 * v).max() < 1e-13


def test_gauge_covariance(small):
    L, kappa, eps, U = small["L"], small["kappa"], small["eps"], small["U"]
    V = int(np.prod(L))
    g = S.random_su3(V, 99)
    Ug = S.gauge_transform(L, U, g)
    psi = S.random_spinor(L, 4)
    gpsi = np.einsum("xab,xsb->xsa", g, psi)
    lhs = O.apply_M(L, kappa, eps, -1, Ug, gpsi)
    rhs = np.einsum("xab,xsb->xsa", g, O.apply_M(L, kappa, eps, -1, U, psi))
    assert np.abs(lhs - rhs).max() < 1e-13
    # per-noise loops: rotated noise through the rotated field gives the same loop
    eta = O.noise_z4(L, 5, 0)
    geta = np.einsum("xab,xsb->xsa", g, eta)
    s, _, _ = O.cgnr(L, kappa, eps, -1, U, eta, 1e-12)
    sg, _, _ = O.cgnr(L, kappa, eps, -1, Ug, geta, 1e-12)
    l1 = O.loops_for_solution(L, kappa, eps, -1, U, [eta], [s], 7)
    l2 = O.loops_for_solution(L, kappa, eps, -1, Ug, [geta], [sg], 7)
    for e in l1:
        assert np.abs(l1[e] - l2[e]).max() < 1e-9 * max(1, np.abs(l1[e]).max())
    assert np.abs(O.hpe_exact(L, kappa, eps, -1, U) - O.hpe_exact(L, kappa, eps, -1, Ug)).max() \
        < 1e-12


# ---------------------------------------------------------------- EO and the solver

def test_eo_solver_against_lu(small):
    """CG on the Schur normal equations, odd reconstruction, and the reported
    residual: x equals the dense LU solution, and the true full-system
    residual is below tol."""
    L, kappa, eps, U = small["L"], small["kappa"], small["eps"], small["U"]
    b = S.random_spinor(L, 6)
    M = dense(lambda v: O.apply_M(L, kappa, eps, -1, U, v), L)
    x_lu = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    for form in (0, 1):
        x, it, res = O.cgnr(L, kappa, eps, -1, U, b, 1e-12, form=form)
        assert it > 0 and res < 1e-12
        true_res = np.linalg.norm(b.ravel() - M @ x.ravel()) / np.linalg.norm(b)
        assert abs(true_res - res) < 1e-14
        assert np.abs(x - x_lu).max() < 1e-9
    # odd reconstruction from the exact even part solves the odd rows exactly
    par = O.site_parity(L)
    xe = x_lu.copy()
    xe[par == 1] = 0
    full = O.reconstruct(L, kappa, eps, -1, U, b, xe)
    assert np.abs(full - x_lu).max() < 1e-12
    # Schur residual of the exact even part is zero
    bh = O.source_prep(L, kappa, eps, -1, U, b)
    assert np.abs(bh - O.schur(L, kappa, eps, -1, U, xe)).max() < 1e-12


def test_maxiter_bounds_cg(small):
    L, kappa, eps, U = small["L"], small["kappa"], small["eps"], small["U"]
    b = S.random_spinor(L, 7)
    x, it, res = O.cgnr(L, kappa, eps, -1, U, b, 1e-14, maxiter=3)
    assert it == 3 and res > 1e-6


# ---------------------------------------------------------------- dense brute force

@pytest.fixture(scope="module")
def dense2():
    """2^4 lattice, random links: dense M, M_d and their inverses."""
    L, kappa, eps = (2, 2, 2, 2), 0.124, 0.05
    U = S.gauge_links(L, 0.5, 21)
    M = dense(lambda v: O.apply_M(L, kappa, eps, -1, U, v), L)
    Md = dense(lambda v: O.apply_M(L, kappa, -eps, -1, U, v), L)
    return dict(L=L, kappa=kappa, eps=eps, U=U, M=M, Mi=np.linalg.inv(M), Mdi=np.linalg.inv(Md))


def full_dilution_solutions(d, tol=1e-13):
    L, V = d["L"], int(np.prod(d["L"]))
    etas, sols = [], []
    for i in range(12 * V):
        e = np.zeros((V, 4, 3), dtype=complex)
        e.reshape(-1)[i] = 1
        x, _, res = O.cgnr(L, d["kappa"], d["eps"], -1, d["U"], e, tol)
        assert res < 10 * tol
        etas.append(e)
        sols.append(x)
    return etas, sols


def test_dense_traces_full_dilution(dense2):
    """Standard, one-end and HPE estimators with full dilution equal their dense
    traces: Tr_t(Gamma M^-1), Tr_t(Gamma M_d^-1) - Tr_t(Gamma M_u^-1) (the one-end
    identity, eq. loopVv, per time slice and for every Gamma), and again
    Tr_t(Gamma M^-1) for the hopping expansion (its exact part computed by the
    oracle's path sum, valid also with L = 2)."""
    d = dense2
    L, kappa, eps, U = d["L"], d["kappa"], d["eps"], d["U"]
    etas, sols = full_dilution_solutions(d)
    est = O.loops_for_solution(L, kappa, eps, -1, U, etas, sols, 7)
    ex_u = slice_traces(L, d["Mi"])
    ex_d = slice_traces(L, d["Mdi"])
    assert np.abs(est[O.EST_STD] - ex_u).max() < 1e-10
    assert np.abs(est[O.EST_ONE_END] - (ex_d - ex_u)).max() < 1e-10
    hpe = est[O.EST_HPE] + O.hpe_exact(L, kappa, eps, -1, U)
    assert np.abs(hpe - ex_u).max() < 1e-10


# ---------------------------------------------------------------- hopping expansion

def test_hpe_expansion_and_exact_part():
    """M^-1 = B - BHB + (BH)^2 B - (BH)^3 B + (BH)^4 M^-1 (eq. HPE); odd powers
    have no diagonal on a bipartite (all-even) lattice; the exact part from the
    path sum equals the diagonal of B + (BH)^2 B from unit vectors, and for all
    L >= 3 the closed forms
      tr B = 12/(1+eps^2),  tr g5 B = -12 i eps/(1+eps^2),
      tr (BH)^2 B = -384 kappa^2 eps^2/(1+eps^2)^3,
      tr g5 (BH)^2 B = -192 i kappa^2 eps (1-eps^2)/(1+eps^2)^3  per site."""
    L, kappa, eps = (4, 4, 2, 4), 0.124, 0.07
    U = S.gauge_links(L, 0.4, 31)
    H = dense(lambda v: O.hop(L, kappa, -1, U, v), L)
    B = dense(lambda v: O.twist(L, eps, v, 2), L)
    M = dense(lambda v: O.apply_M(L, kappa, eps, -1, U, v), L)
    Mi = np.linalg.inv(M)
    BH = B @ H
    BH2 = BH @ BH
    rhs = B - BH @ B + BH2 @ B - BH2 @ BH @ B + BH2 @ BH2 @ Mi
    assert np.abs(rhs - Mi).max() < 1e-13
    assert np.abs(np.diag(BH @ B)).max() < 1e-15
    assert np.abs(np.diag(BH2 @ BH @ B)).max() < 1e-15
    ex = slice_traces(L, B + BH2 @ B)
    he = O.hpe_exact(L, kappa, eps, -1, U)
    assert np.abs(he - ex).max() < 1e-12
    # closed form on a lattice with every L >= 3 (only back-and-forth paths)
    L3 = (4, 4, 4, 4)
    U3 = S.gauge_links(L3, 0.4, 32)
    he3 = O.hpe_exact(L3, kappa, eps, -1, U3)
    Vs = 64
    e2 = eps * eps
    c0 = Vs * (12 / (1 + e2) - 384 * kappa ** 2 * e2 / (1 + e2) ** 3)
    c15 = Vs * (-12j * eps / (1 + e2) - 192j * kappa ** 2 * eps * (1 - e2) / (1 + e2) ** 3)
    assert np.abs(he3[0] - c0).max() < 1e-12 * abs(c0)
    assert np.abs(he3[15] - c15).max() < 1e-12 * abs(c15)
    assert np.abs(he3[1:15]).max() < 1e-13


# ---------------------------------------------------------------- noise

def test_splitmix64_published_outputs():
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if ln.strip() and not ln.startswith("#")]
    for c, v in rows:
        assert O.splitmix64(0, int(c)) == int(v, 16)


def test_z4_noise_properties():
    """Entries in {1, i, -1, -i}; eq. eq1 (mean -> 0) and eq. eq2
    (eta eta^dag -> 1) at rate 1/sqrt(N)."""
    L = (2, 2, 2, 2)
    N = 2000
    etas = np.array([O.noise_z4(L, 77, r).ravel() for r in range(N)])
    assert np.all(np.isin(np.round(etas, 12), [1, 1j, -1, -1j]))
    mean = etas.mean(0)
    assert np.abs(mean).max() < 5 / np.sqrt(N)
    C = etas.T @ etas.conj() / N
    assert np.allclose(np.diag(C), 1)
    off = C - np.eye(C.shape[0])
    assert np.abs(off).max() < 5 / np.sqrt(N)
    # different seeds and noise indices give different vectors
    assert not np.array_equal(O.noise_z4(L, 77, 0), O.noise_z4(L, 78, 0))
    assert not np.array_equal(O.noise_z4(L, 77, 0), O.noise_z4(L, 77, 1))


# ---------------------------------------------------------------- TSM

def test_tsm_reduces_to_plain_and_is_unbiased(dense2):
    """With LP tolerance equal to HP tolerance the TSM estimate equals the plain
    one; with truncated LP solves its mean over many independent estimates
    equals the exact trace (eq. estiTSM)."""
    d = dense2
    L, kappa, eps, U = d["L"], d["kappa"], d["eps"], d["U"]
    ex = slice_traces(L, d["Mi"])
    est = O.EST_STD

    def one(seed, n_hp, n_lp, lp_tol, hp_tol=1e-12):
        etas = [O.noise_z4(L, seed, r) for r in range(n_hp + n_lp)]
        lp = [O.cgnr(L, kappa, eps, -1, U, e, lp_tol)[0] for e in etas]
        hp = [O.cgnr(L, kappa, eps, -1, U, e, hp_tol)[0] for e in etas[:n_hp]]
        lfun = lambda e, s: O.contract_std(L, e, s)  # noqa: E731
        return O.tsm_combine([lfun(e, s) for e, s in zip(etas, hp)],
                             [lfun(e, s) for e, s in zip(etas, lp)],
                             [lfun(e, s) for e, s in zip(etas[n_hp:], lp[n_hp:])])

    t = one(5, 2, 6, 1e-12)
    etas = [O.noise_z4(L, 5, r) for r in range(8)]
    # noises 2..7 are LP-only; with exact LP the correction vanishes
    plain_lp = sum(O.contract_std(L, e, O.cgnr(L, kappa, eps, -1, U, e, 1e-12)[0])
                   for e in etas[2:]) / 6
    assert np.abs(t - plain_lp).max() < 1e-9
    K = 300
    samples = np.array([one(1000 + k, 2, 6, 3e-1) for k in range(K)])
    m = samples.mean(0)
    se = samples.std(0) / np.sqrt(K)
    z = np.abs(m - ex) / np.maximum(se, 1e-12)
    assert np.max(z[se > 1e-12]) < 5
    assert np.abs(m - ex)[se <= 1e-12].max(initial=0) < 1e-9
    # the uncorrected LP mean is detectably biased at this truncation
    lp_only = np.array([O.contract_std(L, O.noise_z4(L, 5000 + k, 0),
                                       O.cgnr(L, kappa, eps, -1, U, O.noise_z4(L, 5000 + k, 0),
                                              3e-1)[0]) for k in range(K)])
    assert np.max(np.abs(lp_only.mean(0) - ex) / (lp_only.std(0) / np.sqrt(K) + 1e-30)) > 5


# ---------------------------------------------------------------- learned preconditioner

def _rand_weights(rng, nc, scale=0.3):
    return scale * (rng.standard_normal((9, nc, 4, 4)) + 1j * rng.standard_normal((9, nc, 4, 4)))


def test_transport_adjoints_and_equivariance():
    L = (4, 2, 2, 4)
    U = S.gauge_links(L, 0.5, 51)
    f, g = S.random_spinor(L, 52), S.random_spinor(L, 53)
    for k in range(9):
        Tg = O.transport(L, -1, U, k, g)
        Tdf = O.transport(L, -1, U, k, f, adj=True)
        assert abs(np.vdot(f, Tg) - np.vdot(Tdf, g)) < 1e-12
    for mu in range(4):  # the adjoint of a +mu hop is the -mu hop
        assert np.abs(O.transport(L, -1, U, 1 + mu, f, adj=True) - O.transport(L, -1, U, 5 + mu, f)).max() < 1e-15
    # gauge equivariance of the network: N[U^g](g phi) = g N[U](phi)
    rng = np.random.default_rng(54)
    W1, W2 = _rand_weights(rng, 12), _rand_weights(rng, 12)
    gm = S.random_su3(int(np.prod(L)), 55)
    Ug = S.gauge_transform(L, U, gm)
    rot = lambda v: np.einsum("xab,xsb->xsa", gm, v)  # noqa: E731
    lhs = O.ptc_forward(L, -1, Ug, W1, W2, rot(f))
    rhs = rot(O.ptc_forward(L, -1, U, W1, W2, f))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_ptc_special_weights():
    """Identity weights give the identity map; first-layer weights
    -kappa (1 -+ gamma_mu) on the +-mu paths give the hopping term H."""
    L, kappa = (4, 2, 2, 4), 0.13
    U = S.gauge_links(L, 0.5, 56)
    f = S.random_spinor(L, 57)
    nc = 12
    W1 = np.zeros((9, nc, 4, 4), dtype=complex)
    W2 = np.zeros((9, nc, 4, 4), dtype=complex)
    W1[0, 0] = np.eye(4)
    W2[0, 0] = np.eye(4)
    assert np.abs(O.ptc_forward(L, -1, U, W1, W2, f) - f).max() < 1e-15
    W1[0, 0] = 0
    for mu in range(4):
        g = O.gamma(1 << mu)
        W1[1 + mu, 0] = -kappa * (np.eye(4) - g)
        W1[5 + mu, 0] = -kappa * (np.eye(4) + g)
    assert np.abs(O.ptc_forward(L, -1, U, W1, W2, f) - O.hop(L, kappa, -1, U, f)).max() < 1e-14


def test_ptc_gradient_finite_differences():
    L = (2, 2, 2, 4)
    U = S.gauge_links(L, 0.5, 58)
    rng = np.random.default_rng(59)
    nc = 3
    W1, W2 = _rand_weights(rng, nc), _rand_weights(rng, nc)
    rs = [S.random_spinor(L, 60 + i) for i in range(2)]
    es = [S.random_spinor(L, 70 + i) for i in range(2)]
    loss, G1, G2 = O.ptc_loss_grad(L, -1, U, W1, W2, rs, es)
    h = 1e-6
    for W, G in ((W1, G1), (W2, G2)):
        for idx in [(0, 0, 0, 0), (3, 1, 2, 1), (8, 2, 3, 3), (5, 0, 1, 2)]:
            for part in (1, 1j):
                Wp, Wm = W.copy(), W.copy()
                Wp[idx] += h * part
                Wm[idx] -= h * part
                lp = O.ptc_loss_grad(L, -1, U, Wp if W is W1 else W1, Wp if W is W2 else W2, rs, es)[0]
                lm = O.ptc_loss_grad(L, -1, U, Wm if W is W1 else W1, Wm if W is W2 else W2, rs, es)[0]
                fd = (lp - lm) / (2 * h)
                an = G[idx].real if part == 1 else G[idx].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (idx, part, fd, an)


def test_ptc_residual_loss_gradient_finite_differences():
    """Residual loss |M N(r) - r|^2 / |r|^2: the analytic gradient (delta =
    2 M^dag w / |r|^2 propagated back through the network) against central
    differences of the loss, both signs of the twist."""
    L = (2, 2, 2, 4)
    U = S.gauge_links(L, 0.5, 61)
    rng = np.random.default_rng(62)
    nc = 3
    W1, W2 = _rand_weights(rng, nc), _rand_weights(rng, nc)
    rs = [S.random_spinor(L, 63 + i) for i in range(2)]
    h = 1e-6
    for eps in (0.05, -0.05):
        loss, G1, G2 = O.ptc_res_loss_grad(L, 0.13, eps, -1, U, W1, W2, rs)
        for W, G in ((W1, G1), (W2, G2)):
            for idx in [(0, 0, 0, 0), (3, 1, 2, 1), (8, 2, 3, 3), (6, 0, 1, 2)]:
                for part in (1, 1j):
                    Wp, Wm = W.copy(), W.copy()
                    Wp[idx] += h * part
                    Wm[idx] -= h * part
                    lp = O.ptc_res_loss_grad(L, 0.13, eps, -1, U, Wp if W is W1 else W1,
                                             Wp if W is W2 else W2, rs)[0]
                    lm = O.ptc_res_loss_grad(L, 0.13, eps, -1, U, Wm if W is W1 else W1,
                                             Wm if W is W2 else W2, rs)[0]
                    fd = (lp - lm) / (2 * h)
                    an = G[idx].real if part == 1 else G[idx].imag
                    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (eps, idx, part, fd, an)


def test_ptc_residual_loss_special_cases():
    """N = 0 gives loss 1 (w = -r); N = R^-1 on a field with H = 0 (kappa = 0)
    is the exact inverse, loss 0 and zero gradient; the residual loss of a
    pair equals |M (N r - e)|^2 / |r|^2 for e = M^-1 r, tying it to the error
    loss's quantity N r - e."""
    L = (2, 2, 2, 4)
    U = S.gauge_links(L, 0.5, 64)
    r = S.random_spinor(L, 65)
    nc = 2
    W1 = np.zeros((9, nc, 4, 4), dtype=complex)
    W2 = np.zeros((9, nc, 4, 4), dtype=complex)
    loss, G1, G2 = O.ptc_res_loss_grad(L, 0.13, 0.05, -1, U, W1, W2, [r])
    assert abs(loss - 1.0) < 1e-14
    eps = 0.05
    Rinv = np.diag([1 / (1 + 1j * eps)] * 2 + [1 / (1 - 1j * eps)] * 2)
    W1[0, 0] = np.eye(4)
    W2[0, 0] = Rinv
    loss, G1, G2 = O.ptc_res_loss_grad(L, 0.0, eps, -1, U, W1, W2, [r])
    assert loss < 1e-28 and np.abs(G1).max() < 1e-14 and np.abs(G2).max() < 1e-14
    rng = np.random.default_rng(66)
    W1, W2 = _rand_weights(rng, 3), _rand_weights(rng, 3)
    e, _, _ = O.cgnr(L, 0.13, eps, -1, U, r, 1e-13)
    d = O.ptc_forward(L, -1, U, W1, W2, r) - e
    ref = np.linalg.norm(O.apply_M(L, 0.13, eps, -1, U, d)) ** 2 / np.linalg.norm(r) ** 2
    loss, _, _ = O.ptc_res_loss_grad(L, 0.13, eps, -1, U, W1, W2, [r])
    assert abs(loss - ref) <= 1e-10 * ref


def test_ptc_at_equals_whole_lattice_forward():
    """The site-by-site evaluation (used at 32^3x64) agrees with the
    layer-by-layer whole-lattice evaluation, both boundary conditions."""
    L = (4, 2, 4, 6)
    U = S.gauge_links(L, 0.5, 80)
    rng = np.random.default_rng(81)
    W1, W2 = _rand_weights(rng, 4), _rand_weights(rng, 4)
    f = S.random_spinor(L, 82)
    sites = np.arange(0, int(np.prod(L)), 5)
    for t_bc in (-1, 1):
        full = O.ptc_forward(L, t_bc, U, W1, W2, f)
        at = O.ptc_at(L, t_bc, U, W1, W2, f, sites)
        assert np.abs(at - full[sites]).max() <= 1e-14 * np.abs(full).max()


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 2, 6)])
def test_schur_at_equals_whole_lattice_schur(L):
    """The site-by-site Schur operator (the reference of the full-size sampled
    checks) equals the whole-lattice Schur complement, built from the masked
    full operator, at every even site: both boundary conditions, both signs
    of the twist, a ragged lattice whose extents differ per direction.  Every
    second hop of the site-wise form crosses the time boundary somewhere on
    these lattices."""
    U = S.gauge_links(L, 0.5, 90)
    f = S.random_spinor(L, 91)
    even = np.where(O.site_parity(L) == 0)[0]
    for t_bc in (-1, 1):
        for eps in (0.037, -0.037):
            whole = O.schur(L, 0.124, eps, t_bc, U, f)
            at = O.schur_at(L, 0.124, eps, t_bc, U, f, even)
            assert np.abs(at - whole[even]).max() <= 1e-14 * np.abs(whole).max()


def test_schur_at_reads_even_sites_only():
    """The site-wise form sees only the even half of its argument, like the
    Schur complement: odd entries of the input change nothing."""
    L = (4, 4, 2, 6)
    U = S.gauge_links(L, 0.5, 92)
    f = S.random_spinor(L, 93)
    g = f.copy()
    odd = O.site_parity(L) == 1
    g[odd] = S.random_spinor(L, 94)[odd]
    even = np.where(~odd)[0]
    a = O.schur_at(L, 0.124, 0.02, -1, U, f, even)
    b = O.schur_at(L, 0.124, 0.02, -1, U, g, even)
    assert np.array_equal(a, b)


def test_momentum_projection_pins():
    """Momentum-resolved contraction: p = 0 equals the per-slice C oracle;
    shifting both fields by a spatial vector a multiplies L(t, p) by
    e^{+i p.a}; the momentum list has the lattice-point counts of the
    sphere |n|^2 <= 9 (1, 6, 12, 8, 6, 24, 24, 0, 12, 30 per shell)."""
    L, eps = (6, 4, 4, 4), 0.07
    moms = O.momenta(2)
    assert tuple(moms[0]) == (0, 0, 0) and len(moms) == 19
    shells = np.bincount((O.momenta(9) ** 2).sum(axis=1), minlength=10)
    assert shells.tolist() == [1, 6, 12, 8, 6, 24, 24, 0, 12, 30]
    eta, s = S.random_spinor(L, 90), S.random_spinor(L, 91)
    out = O.contract_momentum(L, eps, eta, s, O.EST_STD | O.EST_ONE_END, moms)
    assert np.abs(out[O.EST_STD][0] - O.contract_std(L, eta, s)).max() < 1e-12
    assert np.abs(out[O.EST_ONE_END][0] - O.contract_oneend(L, eps, s)).max() < 1e-12
    # translate by a = (1, 2, 3): field(x) -> field(x - a)
    a = (1, 2, 3)
    x, y, z, t = O._site_coords(L)
    src = (((x - a[0]) % L[0]) + L[0] * (((y - a[1]) % L[1]) + L[1] * (((z - a[2]) % L[2]) + L[2] * t)))
    out2 = O.contract_momentum(L, eps, eta[src], s[src], O.EST_STD, moms)[O.EST_STD]
    ph = np.exp(2j * np.pi * (moms[:, 0] * a[0] / L[0] + moms[:, 1] * a[1] / L[1] + moms[:, 2] * a[2] / L[2]))
    assert np.abs(out2 - ph[:, None, None] * out[O.EST_STD]).max() < 1e-11


def test_loops_momentum_zero_momentum_is_loops():
    """The p = 0 block of the momentum-resolved estimate equals the per-slice
    estimate for every estimator, the exact HPE part included; for p != 0 the
    HPE block is the pure stochastic part."""
    L, kappa, eps = (4, 4, 4, 4), 0.124, 0.01
    U = S.gauge_links(L, 0.3, 7)
    est = O.EST_STD | O.EST_ONE_END | O.EST_HPE
    moms = O.momenta(1)
    mm, pn = O.loops_momentum(L, kappa, eps, -1, U, 11, 1, 1e-13, est, moms)
    ref, _ = O.loops(L, kappa, eps, -1, U, 11, 1, 1e-13, est)
    for e in (O.EST_STD, O.EST_ONE_END, O.EST_HPE):
        assert np.abs(mm[e][0] - ref[e]).max() < 1e-10 * np.abs(ref[e]).max()
    assert np.abs(mm[O.EST_HPE][1:] - pn[0][O.EST_HPE][1:]).max() == 0


# ---------------------------------------------------------------- generalised one-end, derivatives

def unit_source_loops(L, kappa, eps, t_bc, U, Sinv, estimator, derivative):
    """Full dilution: every unit source j with solution column j of a dense
    inverse, contracted by the oracle's estimator and summed -> (n_ins, Lt)."""
    V = int(np.prod(L))
    tot = 0
    for j in range(12 * V):
        e = np.zeros((V, 4, 3), dtype=complex)
        e.reshape(-1)[j] = 1
        sol = Sinv[:, j].reshape(V, 4, 3)
        tot = tot + O.slice_sums(L, O.insertion_densities(L, kappa, eps, t_bc, U, e, sol,
                                                          estimator, derivative))
    return tot


@pytest.fixture(scope="module")
def dense4():
    """4x2x2x4 lattice, random links: dense M(+mu), M(-mu) and their inverses."""
    L, kappa, eps = (4, 2, 2, 4), 0.124, 0.09
    U = S.gauge_links(L, 0.5, 23)
    Mu = dense(lambda v: O.apply_M(L, kappa, eps, -1, U, v), L)
    Md = dense(lambda v: O.apply_M(L, kappa, -eps, -1, U, v), L)
    return dict(L=L, kappa=kappa, eps=eps, U=U, Mui=np.linalg.inv(Mu), Mdi=np.linalg.inv(Md))


def test_generalised_one_end_local_dense(dense2):
    """eq. loopStD with full dilution equals Tr_t(Gamma M_u^-1) + Tr_t(Gamma M_d^-1)
    for all 16 Gamma (dense LU traces), through the per-slice C contraction."""
    d = dense2
    L, kappa, eps, U = d["L"], d["kappa"], d["eps"], d["U"]
    V = int(np.prod(L))
    tot = 0
    for j in range(12 * V):
        tot = tot + O.contract_gen(L, kappa, -1, U, d["Mi"][:, j].reshape(V, 4, 3))
    want = slice_traces(L, d["Mi"]) + slice_traces(L, d["Mdi"])
    assert np.abs(tot - want).max() < 1e-11


def test_derivative_free_field_closed_form():
    """U = 1: the one-derivative STD loop with full dilution equals
    (V_s / V) sum_p i sin(p_mu) tr[Gamma_n S(p)], S(p) the inverse of
    A + i sum_nu gamma_nu 2 kappa sin p_nu + i eps gamma5 (times 1 in colour),
    p_t = (2n + 1) pi / Lt; all 16 x 4 insertions at every time slice."""
    L, kappa, eps = (4, 2, 2, 4), 0.124, 0.1
    U = S.unit_links(L)
    V, Lt = int(np.prod(L)), L[3]
    Si = np.linalg.inv(dense(lambda v: O.apply_M(L, kappa, eps, -1, U, v), L))
    got = unit_source_loops(L, kappa, eps, -1, U, Si, O.EST_STD, True)[16:].reshape(4, 16, Lt)
    gam = [O.gamma(n) for n in (1, 2, 4, 8)]      # gamma_x, gamma_y, gamma_z, gamma_t
    want = np.zeros((4, 16), dtype=complex)
    for p in momenta(L, -1):
        A = 1 - 2 * kappa * np.cos(p).sum()
        Mp = A * np.eye(4) + 1j * eps * G5
        for nu in range(4):
            Mp = Mp + 2j * kappa * np.sin(p[nu]) * gam[nu]
        Sp = np.linalg.inv(Mp)
        for mu in range(4):
            for n in range(16):
                want[mu, n] += 1j * np.sin(p[mu]) * 3 * np.trace(O.gamma(n) @ Sp)
    want *= (V // Lt) / V
    assert np.abs(want).max() > 1e-2
    assert np.abs(got - want[:, :, None]).max() < 1e-12
    # the ultra-local block is the plain per-slice contraction
    loc = unit_source_loops(L, kappa, eps, -1, U, Si, O.EST_STD, False)
    assert np.abs(loc - sum(O.contract_std(L, np.eye(12 * V)[j].reshape(V, 4, 3),
                                           Si[:, j].reshape(V, 4, 3))
                            for j in range(12 * V))).max() < 1e-12


def test_derivative_dense_operator_form(dense4):
    """Random links: the one-derivative STD loop with full dilution equals
    (1/4) Tr_t[Gamma (nabla_mu M^-1 + M^-1 nabla_mu)], nabla_mu = T_{+mu} - T_{-mu}
    built densely from the parallel transports (the bilinear's operator form:
    the right-derivative terms give Gamma nabla, the left-derivative terms
    nabla Gamma, both restricted to the slice by cyclicity)."""
    d = dense4
    L, kappa, eps, U = d["L"], d["kappa"], d["eps"], d["U"]
    got = unit_source_loops(L, kappa, eps, -1, U, d["Mui"], O.EST_STD, True)[16:]
    for mu in range(4):
        nab = dense(lambda v: O.transport(L, -1, U, 1 + mu, v) - O.transport(L, -1, U, 5 + mu, v), L)
        K = nab @ d["Mui"] + d["Mui"] @ nab
        want = 0.25 * slice_traces(L, K)
        assert np.abs(got[16 * mu:16 * mu + 16] - want).max() < 1e-12, mu


def test_derivative_and_local_estimator_identities(dense4):
    """For every one of the 80 insertions X (local and one-derivative), with
    full dilution of s = M_u^-1 eta:  GEN = Tr(M_u^-1 X) + Tr(M_d^-1 X)
    (eq. loopStD) and ONE_END = Tr(M_d^-1 X) - Tr(M_u^-1 X) (eq. loopVv),
    the traces being the STD estimator on M_u^-1 and M_d^-1 columns."""
    d = dense4
    L, kappa, eps, U = d["L"], d["kappa"], d["eps"], d["U"]
    tu = unit_source_loops(L, kappa, eps, -1, U, d["Mui"], O.EST_STD, True)
    td = unit_source_loops(L, kappa, -eps, -1, U, d["Mdi"], O.EST_STD, True)
    gen = unit_source_loops(L, kappa, eps, -1, U, d["Mui"], O.EST_GEN_ONE_END, True)
    one = unit_source_loops(L, kappa, eps, -1, U, d["Mui"], O.EST_ONE_END, True)
    scale = np.abs(tu).max()
    assert np.abs(gen - (tu + td)).max() < 1e-11 * scale
    assert np.abs(one - (td - tu)).max() < 1e-11 * scale
    assert np.abs(tu[16:]).max() > 1e-3 * scale       # the derivative block is not trivially zero


# ---------------------------------------------------------------- time dilution

@pytest.mark.parametrize("period", [1, 2, 4])
def test_time_dilution_dense_formula(dense4, period):
    """Coherent time dilution (sec. II.D): per noise, the STD and HPE loops at
    slice t equal sum_{x in t} sum_{y: t_y = t (mod P)} eta(x)^dag Gamma K(x, y)
    eta(y) with K = M^-1 and (BH)^4 M^-1 as dense matrices; P = 1 is the
    volume-source estimate."""
    d = dense4
    L, kappa, eps, U = d["L"], d["kappa"], d["eps"], d["U"]
    V, Lt = int(np.prod(L)), L[3]
    etas = O.noise_sources(L, 77, 3, False, period)
    assert len(etas) == period
    assert np.abs(sum(etas) - O.noise_z4(L, 77, 3)).max() == 0
    sols = [(d["Mui"] @ e.ravel()).reshape(V, 4, 3) for e in etas]
    got = O.loops_for_solution(L, kappa, eps, -1, U, etas, sols, O.EST_STD | O.EST_HPE)
    BH4 = dense(lambda v: O.bh_power(L, kappa, eps, -1, U, v, 4), L)
    eta = O.noise_z4(L, 77, 3).ravel()
    tsite = np.repeat(np.arange(V) // (V // Lt), 12)
    same = (tsite[:, None] % period) == (tsite[None, :] % period)
    for e, K in ((O.EST_STD, d["Mui"]), (O.EST_HPE, BH4 @ d["Mui"])):
        Km = np.where(same, K, 0)
        y = Km @ eta
        want = np.zeros((16, Lt), dtype=complex)
        for n in range(16):
            Gc = np.kron(np.eye(V), np.kron(O.gamma(n), np.eye(3)))
            dens = (eta.conj() * (Gc @ y)).reshape(V, 12).sum(1)
            want[n] = dens.reshape(Lt, -1).sum(1)
        assert np.abs(got[e] - want).max() < 1e-12, e


def test_site_restricted_evaluation_matches_whole_lattice():
    """Evaluating the densities at a subset of time slices (used at full
    lattice size) gives the whole-lattice values on those slices."""
    L, kappa, eps = (4, 4, 2, 6), 0.124, 0.05
    U = S.gauge_links(L, 0.4, 31)
    eta, s = S.random_spinor(L, 32), S.random_spinor(L, 33)
    moms = O.momenta(1)
    full = O.contract_insertions(L, kappa, eps, -1, U, eta, s, 1 | 2 | 8, True, moms)
    part = O.contract_insertions(L, kappa, eps, -1, U, eta, s, 1 | 2 | 8, True, moms,
                                 slices=[0, 3, 5])
    for e in full:
        assert np.abs(part[e][..., [0, 3, 5]] - full[e][..., [0, 3, 5]]).max() < 1e-13
        assert np.abs(part[e][..., [1, 2, 4]]).max() == 0
