"""Learned preconditioner and flexible GMRES through the C-ABI.

The device network evaluates the collapsed two-layer form in FP32 (FP64
gradient sums); the oracle evaluates the layers one after the other in FP64
and differentiates them by reverse mode.  Bars: forward 2e-5 and gradients
1e-4 normwise relative (FP32 rounding, unit 6e-8, over ~10^3 accumulated
products per output); the hopping-expansion weights against the oracle's own
operators; training must lower the loss; FGMRES solutions are judged by the
true residual recomputed by the oracle, like the CG solves.
"""
import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1309_2256_amd as P  # noqa: E402

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rand_weights(rng, nc, scale=0.3):
    return scale * (rng.standard_normal((9, nc, 4, 4)) + 1j * rng.standard_normal((9, nc, 4, 4)))


def make_ctx(L, kappa, eps, seed, eps_links=0.3):
    U = S.gauge_links(L, eps_links, seed)
    ctx = P.Context(L, kappa, eps)
    ctx.set_gauge(cuda(U))
    return ctx, U


LATTICES = [(4, 4, 4, 8), (6, 4, 4, 6), (16, 16, 16, 32)]


@pytest.mark.parametrize("L", LATTICES, ids=["L0", "ragged", "c2"])
def test_ptc_forward_matches_oracle(L):
    ctx, U = make_ctx(L, 0.124, 0.01, 301)
    rng = np.random.default_rng(302)
    nc = 12
    W1, W2 = rand_weights(rng, nc), rand_weights(rng, nc)
    ctx.ptc_set_weights(W1, W2)
    n = 2
    psi = S.random_spinor(L, 303, n)
    out = torch.zeros_like(cuda(psi))
    ctx.ptc_apply(out, cuda(psi), n)
    got = host(out)
    for r in range(n):
        ref = O.ptc_forward(L, -1, U, W1, W2, psi[r])
        assert rel(got[r], ref) < 2e-5, (L, r, rel(got[r], ref))
    # weights round trip
    G1, G2 = ctx.ptc_get_weights(nc)
    assert np.array_equal(G1, W1) and np.array_equal(G2, W2)
    ctx.close()


def test_ptc_loss_gradient_matches_oracle():
    L = (4, 4, 4, 8)
    ctx, U = make_ctx(L, 0.124, 0.01, 311)
    rng = np.random.default_rng(312)
    for nc in (3, 12):
        W1, W2 = rand_weights(rng, nc), rand_weights(rng, nc)
        ctx.ptc_set_weights(W1, W2)
        rs = S.random_spinor(L, 313, 3)
        es = S.random_spinor(L, 314, 3)
        loss, G1, G2 = ctx.ptc_loss_grad(cuda(rs), cuda(es), 3, nc)
        rl, R1, R2 = O.ptc_loss_grad(L, -1, U, W1, W2, list(rs), list(es))
        assert abs(loss - rl) <= 1e-5 * rl, (nc, loss, rl)
        assert rel(G1, R1) < 1e-4, (nc, rel(G1, R1))
        assert rel(G2, R2) < 1e-4, (nc, rel(G2, R2))
    ctx.close()


@pytest.mark.parametrize("mu_sign", [1, -1])
def test_ptc_hopping_initialisation(mu_sign):
    """N = B - B H B + B H B H B with the oracle's own B = R^-1 and H."""
    L, kappa, eps = (4, 4, 4, 8), 0.124, 0.05
    ctx, U = make_ctx(L, kappa, eps, 321)
    ctx.ptc_init_hopping(nc=12, mu_sign=mu_sign, seed=5, noise=0.01)
    f = S.random_spinor(L, 322, 1)
    out = torch.zeros_like(cuda(f))
    ctx.ptc_apply(out, cuda(f), 1)
    e = mu_sign * eps
    B = lambda v: O.twist(L, e, v, which=2)  # noqa: E731
    H = lambda v: O.hop(L, kappa, -1, U, v)  # noqa: E731
    Bf = B(f[0])
    ref = Bf - B(H(Bf)) + B(H(B(H(Bf))))
    assert rel(host(out)[0], ref) < 2e-5
    ctx.close()


def make_pairs(ctx, L, n, seed, tol=1e-7):
    """(r, e) = (eta, M^-1 eta) for Gaussian eta, mixed CG solves."""
    eta = cuda(S.random_spinor(L, seed, n))
    x = torch.zeros_like(eta)
    ctx.solve(x, eta, n, P.solve_params(tol=tol, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16))
    return eta, x


@pytest.mark.parametrize("store", [P.TM_F32, P.TM_BF16], ids=["f32", "bf16"])
def test_ptc_training_lowers_loss(store):
    cfg = S.CONFIGS["c4a"]
    L = cfg["L"]
    ctx, U = make_ctx(L, cfg["kappa"], cfg["two_kappa_mu"], cfg["seed"], cfg["eps_links"])
    r, e = make_pairs(ctx, L, 24, 331)
    rv, ev = make_pairs(ctx, L, 4, 332)
    ctx.ptc_pairs_reserve(24, store)
    ctx.ptc_pairs_add(r[:12], e[:12], 12)
    ctx.ptc_pairs_add(r[12:], e[12:], 12)
    with pytest.raises(P.TMError):
        ctx.ptc_pairs_add(r[:1], e[:1], 1)  # beyond capacity
    ctx.ptc_init_hopping(nc=12, mu_sign=1, seed=7, noise=1e-3)
    l0 = ctx.ptc_loss_grad(rv, ev, 4, 12)[0]
    st, hist = ctx.ptc_train(epochs=4, batch=4, lr=1e-3, seed=9, n_pairs=24)
    assert st.steps == 24 and np.all(np.isfinite(hist))
    assert st.loss_last < st.loss_first, (st.loss_first, st.loss_last)
    l1 = ctx.ptc_loss_grad(rv, ev, 4, 12)[0]  # held-out pairs
    assert l1 < l0, (l0, l1)
    ctx.close()


@pytest.mark.parametrize("mu_sign", [1, -1])
def test_fgmres_converges(mu_sign):
    cfg = S.CONFIGS["c4a"]
    L = cfg["L"]
    ctx, U = make_ctx(L, cfg["kappa"], cfg["two_kappa_mu"], cfg["seed"], cfg["eps_links"])
    n = 3
    b = S.random_spinor(L, 341, n)
    bt = cuda(b)
    its = {}
    for solver in (P.TM_FGMRES, P.TM_FGMRES_PTC):
        if solver == P.TM_FGMRES_PTC:
            ctx.ptc_init_hopping(nc=12, mu_sign=mu_sign)
        x = torch.zeros_like(bt)
        p = P.solve_params(tol=1e-9, solver=solver, mu_sign=mu_sign, check_every=16, maxiter=20000)
        _, stats = ctx.solve(x, bt, n, p)
        xh = host(x)
        for r in range(n):
            res = np.linalg.norm(b[r] - O.apply_M(L, cfg["kappa"], mu_sign * cfg["two_kappa_mu"], -1, U, xh[r]))
            res /= np.linalg.norm(b[r])
            assert res <= 1e-9, (solver, r, res)
            assert stats[r].converged == 1 and stats[r].true_rel_res <= 1e-9
        its[solver] = max(s.iters for s in stats)
    # the second-order hopping preconditioner cuts the Arnoldi steps
    assert its[P.TM_FGMRES_PTC] < its[P.TM_FGMRES], its
    ctx.close()


def test_fgmres_argument_checks():
    L = (4, 4, 4, 8)
    ctx, U = make_ctx(L, 0.124, 0.01, 351)
    b = cuda(S.random_spinor(L, 352, 1))
    x = torch.zeros_like(b)
    with pytest.raises(P.TMError) as ei:
        ctx.solve(x, b, 1, P.solve_params(solver=P.TM_FGMRES_PTC))  # no weights
    assert ei.value.status == P.TM_ERR_ARG
    with pytest.raises(P.TMError) as ei:
        ctx.solve(x, b, 1, P.solve_params(solver=P.TM_FGMRES, check_every=33))
    assert ei.value.status == P.TM_ERR_ARG
    with pytest.raises(P.TMError) as ei:
        ctx.ptc_pairs_add(b, b, 1)  # no store reserved
    assert ei.value.status == P.TM_ERR_ARG
    # maxiter reached: NOCONV with the residual reported
    st, stats = ctx.solve(x, b, 1, P.solve_params(solver=P.TM_FGMRES, maxiter=3, check_every=16),
                          allow_noconv=True)
    assert st == P.TM_ERR_NOCONV and stats[0].converged == 0 and stats[0].iters == 3
    ctx.close()


@pytest.fixture(scope="module")
def c5():
    cfg = S.CONFIGS["c5"]
    L = cfg["L"]
    U = S.gauge_links(L, cfg["eps_links"], cfg["seed"])
    ctx = P.Context(L, cfg["kappa"], cfg["two_kappa_mu"])
    ctx.set_gauge(cuda(U))
    yield dict(L=L, cfg=cfg, U=U, ctx=ctx)
    ctx.close()


def test_c5_ptc_forward_sampled_sites(c5):
    """32^3x64 (the FGMRES workload): the network at 64 sampled sites against
    the oracle's site-by-site evaluation of the two layers."""
    L, U, ctx = c5["L"], c5["U"], c5["ctx"]
    rng = np.random.default_rng(361)
    W1, W2 = rand_weights(rng, 12), rand_weights(rng, 12)
    ctx.ptc_set_weights(W1, W2)
    f = S.random_spinor(L, 362, 1)
    out = torch.zeros_like(cuda(f))
    ctx.ptc_apply(out, cuda(f), 1)
    got = host(out)[0]
    V = int(np.prod(L))
    sites = np.sort(rng.choice(V, 64, replace=False))
    sites[:2] = [0, V - 1]
    ref = O.ptc_at(L, -1, U, W1, W2, f[0], sites)
    assert rel(got[sites], ref) < 2e-5


def test_c5_fgmres_network_true_residual(c5):
    """32^3x64: FGMRES(16) with the network (hopping-expansion weights) to
    1e-9; the oracle recomputes |b - M x| / |b| in FP64 on the host."""
    L, U, ctx, cfg = c5["L"], c5["U"], c5["ctx"], c5["cfg"]
    ctx.ptc_init_hopping(nc=12, mu_sign=1)
    b = S.random_spinor(L, 363, 1)
    x = torch.zeros_like(cuda(b))
    _, st = ctx.solve(x, cuda(b), 1, P.solve_params(tol=1e-9, solver=P.TM_FGMRES_PTC, check_every=16,
                                                     maxiter=3000))
    xh = host(x)[0]
    res = np.linalg.norm(b[0] - O.apply_M(L, cfg["kappa"], cfg["two_kappa_mu"], -1, U, xh)) / np.linalg.norm(b[0])
    assert res <= 1e-9 and st[0].converged == 1, (res, st[0].iters)
