"""Learning the preconditioner from the solver's own iterates.

* The residual loss |M N(r) - r|^2 / |r|^2 and its gradient (carried back
  through M^dag on the device in FP32) against the FP64 oracle, both flavours.
* Pairs from solver iterates: the stored pairs (b - M x_k, x* - x_k) give the
  oracle's loss over pairs rebuilt on the host from the same iterates.
* The mixed-CG fallback of the network-preconditioned FGMRES: with weights
  that do not precondition, a stalled restart cycle hands the solve to mixed
  CG, whose result meets the tolerance by the oracle's residual.
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


def make_ctx(name):
    cfg = S.CONFIGS[name]
    U = S.gauge_links(cfg["L"], cfg["eps_links"], cfg["seed"])
    ctx = P.Context(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"])
    ctx.set_gauge(cuda(U))
    return ctx, cfg, U


@pytest.mark.parametrize("mu_sign", [1, -1])
def test_residual_loss_gradient_matches_oracle(mu_sign):
    """FP32 device evaluation (network, M, M^dag) against the FP64 oracle:
    loss within 1e-5 and gradients within 1e-4 normwise relative."""
    L, kappa, eps = (4, 4, 4, 8), 0.124, 0.01
    U = S.gauge_links(L, 0.3, 371)
    ctx = P.Context(L, kappa, eps)
    try:
        ctx.set_gauge(cuda(U))
        rng = np.random.default_rng(372)
        for nc in (3, 12):
            W1, W2 = rand_weights(rng, nc), rand_weights(rng, nc)
            ctx.ptc_set_weights(W1, W2)
            rs = S.random_spinor(L, 373, 3)
            loss, G1, G2 = ctx.ptc_loss_grad(cuda(rs), None, 3, nc, loss_kind=P.TM_PTC_LOSS_RESIDUAL,
                                             mu_sign=mu_sign)
            rl, R1, R2 = O.ptc_res_loss_grad(L, kappa, mu_sign * eps, -1, U, W1, W2, list(rs))
            assert abs(loss - rl) <= 1e-5 * rl, (nc, loss, rl)
            assert rel(G1, R1) < 1e-4, (nc, rel(G1, R1))
            assert rel(G2, R2) < 1e-4, (nc, rel(G2, R2))
    finally:
        ctx.close()


def test_pairs_from_solver_iterates():
    """tm_ptc_pairs_from_solve stores (b - M x_k, x* - x_k) for the solver's
    iterates x_k; the first training step's loss over all stored pairs equals
    the oracle's error loss over the pairs rebuilt on the host from the same
    iterates (tm_solve with maxiter = k, deterministic)."""
    ctx, cfg, U = make_ctx("c4a")
    try:
        L = cfg["L"]
        rng = np.random.default_rng(381)
        W1, W2 = rand_weights(rng, 4), rand_weights(rng, 4)
        ctx.ptc_set_weights(W1, W2)
        n, iters = 2, [3, 7, 12]
        b = S.random_spinor(L, 382, n)
        params = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
        ctx.ptc_pairs_reserve(n * len(iters), P.TM_F32)
        added = ctx.ptc_pairs_from_solve(cuda(b), n, params, iters)
        assert added == n * len(iters)
        xs = torch.zeros_like(cuda(b))
        ctx.solve(xs, cuda(b), n, params)
        xstar = host(xs)
        rs, es = [], []
        kappa, eps = cfg["kappa"], cfg["two_kappa_mu"]
        for k in iters:
            xk = torch.zeros_like(cuda(b))
            ctx.solve(xk, cuda(b), n, P.solve_params(tol=1e-9, maxiter=k, solver=P.TM_CG_MIXED,
                                                      inner_prec=P.TM_F16), allow_noconv=True)
            xkh = host(xk)
            for r in range(n):
                rs.append(b[r] - O.apply_M(L, kappa, eps, -1, U, xkh[r]))
                es.append(xstar[r] - xkh[r])
        ref, _, _ = O.ptc_loss_grad(L, -1, U, W1, W2, rs, es)
        st, hist = ctx.ptc_train(epochs=1, batch=n * len(iters), lr=1e-12, seed=1, n_pairs=n * len(iters))
        assert abs(hist[0] - ref) <= 1e-4 * ref, (hist[0], ref)
        with pytest.raises(P.TMError):  # store full
            ctx.ptc_pairs_from_solve(cuda(b), n, params, [5])
    finally:
        ctx.close()


def test_fgmres_falls_back_to_mixed_cg():
    """Weights that do not precondition M: a restart cycle fails to halve
    the residual, mixed CG finishes the solve, the oracle's residual meets
    the tolerance and the stats say so."""
    ctx, cfg, U = make_ctx("c4a")
    try:
        L = cfg["L"]
        rng = np.random.default_rng(391)
        W = rand_weights(rng, 12, scale=0.05)
        ctx.ptc_set_weights(W, W)
        b = S.random_spinor(L, 392, 2)
        x = torch.zeros_like(cuda(b))
        _, st = ctx.solve(x, cuda(b), 2, P.solve_params(tol=1e-9, solver=P.TM_FGMRES_PTC, check_every=16,
                                                         maxiter=2000))
        xh = host(x)
        for r in range(2):
            res = np.linalg.norm(b[r] - O.apply_M(L, cfg["kappa"], cfg["two_kappa_mu"], -1, U, xh[r]))
            res /= np.linalg.norm(b[r])
            assert res <= 1e-9 and st[r].converged == 1, (r, res)
            assert st[r].fallback == 1
    finally:
        ctx.close()


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 4, 6)])
def test_bf16_matrix_core_forward_matches_oracle(L):
    """Spin mixing on the matrix cores (BF16 weights and transported fields,
    FP32 accumulation): against the FP64 oracle within 1e-2 normwise (each
    product carries two roundings to 8 significand bits, 2^-8 relative,
    summed over 72 real terms of mixed sign); the FP32 path of the same
    weights stays at 2e-5."""
    U = S.gauge_links(L, 0.3, 401)
    ctx = P.Context(L, 0.124, 0.01)
    try:
        ctx.set_gauge(cuda(U))
        rng = np.random.default_rng(402)
        W1, W2 = rand_weights(rng, 12), rand_weights(rng, 12)
        ctx.ptc_set_weights(W1, W2)
        f = S.random_spinor(L, 403, 2)
        ref = [O.ptc_forward(L, -1, U, W1, W2, f[r]) for r in range(2)]
        for arith, bound in ((P.TM_BF16, 1e-2), (P.TM_F32, 2e-5)):
            ctx.ptc_set_arith(arith)
            out = torch.zeros_like(cuda(f))
            ctx.ptc_apply(out, cuda(f), 2)
            got = host(out)
            for r in range(2):
                assert rel(got[r], ref[r]) < bound, (arith, r, rel(got[r], ref[r]))
    finally:
        ctx.close()


def test_bf16_network_fgmres_converges():
    """FGMRES(16) with the BF16 matrix-core network (hopping-expansion
    weights) reaches 1e-9 by the oracle's residual: the flexible method
    absorbs the BF16 preconditioner."""
    ctx, cfg, U = make_ctx("c4a")
    try:
        L = cfg["L"]
        ctx.ptc_init_hopping(nc=12, mu_sign=1)
        ctx.ptc_set_arith(P.TM_BF16)
        b = S.random_spinor(L, 411, 2)
        x = torch.zeros_like(cuda(b))
        _, st = ctx.solve(x, cuda(b), 2, P.solve_params(tol=1e-9, solver=P.TM_FGMRES_PTC, check_every=16,
                                                         maxiter=4000))
        xh = host(x)
        for r in range(2):
            res = np.linalg.norm(b[r] - O.apply_M(L, cfg["kappa"], cfg["two_kappa_mu"], -1, U, xh[r]))
            assert res / np.linalg.norm(b[r]) <= 1e-9 and st[r].converged == 1
    finally:
        ctx.close()


def test_trained_network_beats_hopping_start():
    """What training gains: the network trained with the residual loss on
    pairs from the mixed CG's own iterates needs fewer FGMRES(16) steps on
    held-out right-hand sides than its analytic start, the second-order
    hopping expansion (8^3x16, the uneven-batch physics; the steps are the
    same for every held-out source to within one)."""
    ctx, cfg, U = make_ctx("c4a")
    try:
        L = cfg["L"]
        ctx.ptc_init_hopping(nc=12, mu_sign=1, seed=3, noise=1e-3)
        fg = P.solve_params(tol=1e-9, solver=P.TM_FGMRES_PTC, check_every=16, maxiter=4000)
        held = cuda(S.random_spinor(L, 421, 2))

        def steps():
            x = torch.zeros_like(held)
            _, st = ctx.solve(x, held, 2, fg)
            assert all(s.converged == 1 and s.fallback == 0 for s in st)
            return max(s.iters for s in st)

        start = steps()
        train = cuda(S.random_spinor(L, 422, 8))
        mixed = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
        ctx.ptc_pairs_reserve(32, P.TM_F32)
        n = ctx.ptc_pairs_from_solve(train, 8, mixed, [4, 8, 16, 32])
        assert n == 32
        st, hist = ctx.ptc_train(epochs=10, batch=8, lr=1e-3, seed=5, n_pairs=n, loss=P.TM_PTC_LOSS_RESIDUAL,
                                 mu_sign=1)
        assert st.loss_last < st.loss_first
        trained = steps()
        assert trained < start, (start, trained)
    finally:
        ctx.close()
