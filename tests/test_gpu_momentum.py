"""Momentum-projected loops on the device against the oracle: the Fourier
sum over each time slice of the loop density, for every momentum with
|n|^2 <= p2max (appendix A.3, the Fourier step after the contraction of appendix A.2)."""
import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1309_2256_amd as P  # noqa: E402

DEV = "cuda:0"
EST2 = P.TM_EST_STD | P.TM_EST_ONE_END
EST_ALL = EST2 | P.TM_EST_HPE
EST_ORDER = (O.EST_STD, O.EST_ONE_END, O.EST_HPE)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make_ctx(L, kappa, eps, seed, eps_links=0.3):
    U = S.gauge_links(L, eps_links, seed)
    ctx = P.Context(L, kappa, eps)
    ctx.set_gauge(cuda(U))
    return ctx, U


@pytest.mark.parametrize("L,p2max", [((4, 4, 4, 8), 2), ((6, 4, 8, 4), 1), ((6, 6, 6, 4), 5),
                                     ((8, 6, 10, 2), 4), ((10, 10, 10, 2), 16)])
def test_contract_momentum_matches_oracle(L, p2max):
    # |n|^2 <= 16 needs 2N + 1 = 9 components per direction: more than the
    # x pass forms per chunk (8), so its second chunk is covered
    eps = 0.0123
    ctx, _ = make_ctx(L, 0.124, eps, 61)
    nrhs = 3
    eta = S.random_spinor(L, 62, nrhs)
    s = S.random_spinor(L, 63, nrhs)
    moms = O.momenta(p2max)
    assert np.array_equal(P.momenta(p2max), moms)
    for mu_sign in (1, -1):
        got = ctx.contract_momentum(cuda(eta), cuda(s), nrhs, EST2, p2max, mu_sign)
        ref = [O.contract_momentum(L, mu_sign * eps, eta[r], s[r], O.EST_STD | O.EST_ONE_END, moms)
               for r in range(nrhs)]
        for k, e in enumerate((O.EST_STD, O.EST_ONE_END)):
            want = sum(x[e] for x in ref)
            assert got[k].shape == want.shape
            assert rel(got[k], want) < 1e-13, (e, rel(got[k], want))
        # p = 0 equals the per-slice contraction of the same fields
        flat = ctx.contract(cuda(eta), cuda(s), nrhs, EST2, mu_sign)
        assert rel(got[:, 0], flat) < 1e-13


def test_contract_momentum_argument_checks():
    ctx, _ = make_ctx((4, 4, 4, 4), 0.124, 0.01, 5)
    v = cuda(S.random_spinor((4, 4, 4, 4), 1))
    for bad in (-1, 4):          # 4 needs |n_i| = 2 = L / 2
        with pytest.raises(P.TMError) as ei:
            ctx.contract_momentum(v, v, 1, EST2, bad)
        assert ei.value.status == P.TM_ERR_ARG


def loop_params(seed, n_hp, n_lp, est, dilution=P.TM_DIL_NONE):
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.dilution, p.mu_sign = seed, n_hp, n_lp, est, \
        dilution, 1
    p.hp = P.solve_params(tol=1e-11, solver=P.TM_CG_F64)
    p.lp = P.solve_params(tol=1e-2, solver=P.TM_CG_LOW, inner_prec=P.TM_F16, check_every=1)
    return p


@pytest.mark.parametrize("dilution", [P.TM_DIL_NONE, P.TM_DIL_SPIN_COLOUR])
def test_loops_momentum_vs_oracle(dilution):
    """Small lattice of the 4^3 x 8 workload: every estimator, every momentum
    with |n|^2 <= 2, within 1e-8 normwise of the oracle (both solve tightly);
    the p = 0 block equals tm_loops on the same noises."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    n, p2max = (2 if dilution == P.TM_DIL_NONE else 1), 2
    moms = O.momenta(p2max)
    got, pn, stats, _ = ctx.loops_momentum(loop_params(211, n, 0, EST_ALL, dilution), p2max,
                                           per_noise=True)
    ref, ref_pn = O.loops_momentum(L, kappa, eps, -1, U, 211, n, 1e-13, EST_ALL, moms,
                                   dilution=dilution == P.TM_DIL_SPIN_COLOUR)
    for k, e in enumerate(EST_ORDER):
        assert rel(got[k], ref[e]) < 1e-8, (e, rel(got[k], ref[e]))
        for r in range(n):
            assert rel(pn[r, 0, k], ref_pn[r][e]) < 1e-8
    flat, _, _, _ = ctx.loops(loop_params(211, n, 0, EST_ALL, dilution))
    assert rel(got[:, 0], flat) < 1e-12
    assert stats.max_res_hp <= 1e-11


def test_loops_momentum_tsm():
    """TSM applies per momentum: the combination of the library's per-noise
    momentum loops (eq. estiTSM, by the oracle) is the returned estimate."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    n_hp, n_lp = 1, 2
    got, pn, _, _ = ctx.loops_momentum(loop_params(213, n_hp, n_lp, EST_ALL), 1, per_noise=True)
    for k, e in enumerate(EST_ORDER):
        comb = O.tsm_combine([pn[r, 0, k] for r in range(n_hp)],
                             [pn[r, 1, k] for r in range(n_hp)],
                             [pn[r, 1, k] for r in range(n_hp, n_hp + n_lp)])
        if e == O.EST_HPE:
            comb = comb.copy()
            comb[0] += O.hpe_exact(L, kappa, eps, -1, U)
        assert rel(got[k], comb) < 1e-13


def test_c3_contract_momentum_sampled():
    """32^3 x 64, 12 RHS (the timed contraction), |n|^2 <= 9 (123 momenta):
    sampled momenta against the oracle's Fourier sum of the same fields."""
    cfg = S.CONFIGS["c3"]
    L = cfg["L"]
    ctx, _ = make_ctx(L, cfg["kappa"], cfg["two_kappa_mu"], cfg["seed"], cfg["eps_links"])
    nrhs, p2max = 12, 9
    eta = S.random_spinor(L, 301, nrhs)
    s = S.random_spinor(L, 302, nrhs)
    got = ctx.contract_momentum(cuda(eta), cuda(s), nrhs, EST2, p2max)
    moms = O.momenta(p2max)
    assert got.shape == (2, len(moms), 16, L[3])
    pick = [0, 1, 17, 60, len(moms) - 1]
    ref = {O.EST_STD: 0, O.EST_ONE_END: 0}
    for r in (0, 5, 11):        # rank-one pieces sampled: the others enter via linearity below
        x = O.contract_momentum(L, cfg["two_kappa_mu"], eta[r], s[r], O.EST_STD | O.EST_ONE_END,
                                moms[pick])
        for e in ref:
            ref[e] = ref[e] + x[e]
    sub = ctx.contract_momentum(cuda(eta[[0, 5, 11]]), cuda(s[[0, 5, 11]]), 3, EST2, p2max)
    for k, e in enumerate((O.EST_STD, O.EST_ONE_END)):
        assert rel(sub[k, pick], ref[e]) < 1e-12, (e, rel(sub[k, pick], ref[e]))
    # linearity in the RHS: the 12-RHS result is the sum of its 3 + 9 split
    rest = [r for r in range(nrhs) if r not in (0, 5, 11)]
    sub2 = ctx.contract_momentum(cuda(eta[rest]), cuda(s[rest]), len(rest), EST2, p2max)
    assert rel(got, sub + sub2) < 1e-12
    ctx.close()
