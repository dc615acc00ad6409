"""Generalised one-end estimator (eq. loopStD) and one-derivative insertions
(the covariant-derivative contraction of appendix A.2) on the device against the
oracle, per time slice and momentum resolved."""
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
EST3 = P.TM_EST_STD | P.TM_EST_ONE_END | P.TM_EST_GEN_ONE_END
ORDER3 = (O.EST_STD, O.EST_ONE_END, O.EST_GEN_ONE_END)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make_ctx(L, kappa, eps, seed, eps_links=0.3, t_bc=-1):
    U = S.gauge_links(L, eps_links, seed)
    ctx = P.Context(L, kappa, eps, t_bc=t_bc)
    ctx.set_gauge(cuda(U))
    return ctx, U


@pytest.mark.parametrize("L,p2max,t_bc", [((4, 4, 4, 8), 0, -1), ((4, 4, 4, 8), 2, -1),
                                          ((6, 4, 8, 4), 1, 1), ((2, 2, 2, 2), 0, -1),
                                          ((8, 6, 10, 2), 4, -1)])
def test_contract_insertions_match_oracle(L, p2max, t_bc):
    """STD, one-end and generalised one-end, 16 local + 64 one-derivative
    insertions, every momentum with |n|^2 <= p2max: within 1e-13 of the
    oracle's site-by-site densities and Fourier sums."""
    kappa, eps = 0.124, 0.0123
    ctx, U = make_ctx(L, kappa, eps, 71, t_bc=t_bc)
    nrhs = 3
    eta = S.random_spinor(L, 72, nrhs)
    s = S.random_spinor(L, 73, nrhs)
    moms = O.momenta(p2max)
    for mu_sign in (1, -1):
        got = ctx.contract_momentum(cuda(eta), cuda(s), nrhs, EST3, p2max, mu_sign, derivative=1)
        assert got.shape == (3, len(moms), 80, L[3])
        ref = [O.contract_insertions(L, kappa, mu_sign * eps, t_bc, U, eta[r], s[r],
                                     P.TM_EST_STD | P.TM_EST_ONE_END | P.TM_EST_GEN_ONE_END,
                                     True, moms) for r in range(nrhs)]
        for k, e in enumerate(ORDER3):
            want = sum(x[e] for x in ref)
            assert rel(got[k], want) < 1e-13, (e, rel(got[k], want))
        # without derivative: the local block alone, and tm_contract per slice
        loc = ctx.contract_momentum(cuda(eta), cuda(s), nrhs, EST3, p2max, mu_sign)
        assert np.array_equal(loc, got[:, :, :16])
        if p2max == 0:
            flat = ctx.contract(cuda(eta), cuda(s), nrhs, EST3, mu_sign)
            assert rel(flat, got[:, 0, :16]) < 1e-13


def loop_params(seed, n_hp, n_lp, est, derivative, dilution=P.TM_DIL_NONE):
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.dilution, p.mu_sign = seed, n_hp, n_lp, est, \
        dilution, 1
    p.derivative = derivative
    p.hp = P.solve_params(tol=1e-11, solver=P.TM_CG_F64)
    p.lp = P.solve_params(tol=1e-2, solver=P.TM_CG_LOW, inner_prec=P.TM_F16, check_every=1)
    return p


@pytest.mark.parametrize("dilution", [P.TM_DIL_NONE, P.TM_DIL_SPIN_COLOUR])
def test_loops_insertions_vs_oracle(dilution):
    """4^3 x 8 workload: STD, one-end, generalised one-end with all 80
    insertions, per time slice and at |n|^2 <= 1, within 1e-8 of the oracle
    (both solve tightly)."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    n = 2 if dilution == P.TM_DIL_NONE else 1
    dil = dilution == P.TM_DIL_SPIN_COLOUR
    got, pn, st, _ = ctx.loops(loop_params(221, n, 0, EST3, 1, dilution), per_noise=True)
    ref, ref_pn = O.loops(L, kappa, eps, -1, U, 221, n, 1e-13, int(EST3), dilution=dil,
                          derivative=True)
    assert got.shape == (3, 80, L[3])
    for k, e in enumerate(ORDER3):
        assert rel(got[k], ref[e]) < 1e-8, (e, rel(got[k], ref[e]))
        for r in range(n):
            assert rel(pn[r, 0, k], ref_pn[r][e]) < 1e-8
    moms = O.momenta(1)
    gm, _, _, _ = ctx.loops_momentum(loop_params(221, n, 0, EST3, 1, dilution), 1)
    rm, _ = O.loops_momentum(L, kappa, eps, -1, U, 221, n, 1e-13, int(EST3), moms,
                             dilution=dil, derivative=True)
    for k, e in enumerate(ORDER3):
        assert rel(gm[k], rm[e]) < 1e-8, (e, rel(gm[k], rm[e]))
    assert rel(gm[:, 0], got) < 1e-12


def test_gen_one_end_with_hpe_and_tsm():
    """Mask order STD, ONE_END, HPE, GEN; the HPE exact part stays on the
    HPE block; TSM per insertion (eq. estiTSM applied by the oracle to the
    library's per-noise loops)."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    est = P.TM_EST_STD | P.TM_EST_HPE | P.TM_EST_GEN_ONE_END
    got, pn, _, _ = ctx.loops(loop_params(223, 1, 2, est, 0), per_noise=True)
    ex = O.hpe_exact(L, kappa, eps, -1, U)
    for k, e in enumerate((O.EST_STD, O.EST_HPE, O.EST_GEN_ONE_END)):
        comb = O.tsm_combine([pn[0, 0, k]], [pn[0, 1, k]], [pn[1, 1, k], pn[2, 1, k]])
        if e == O.EST_HPE:
            comb = comb + ex
        assert rel(got[k], comb) < 1e-13
    _, ref_pn = O.loops(L, kappa, eps, -1, U, 223, 1, 1e-13, int(est))
    for k, e in enumerate((O.EST_STD, O.EST_HPE, O.EST_GEN_ONE_END)):
        assert rel(pn[0, 0, k], ref_pn[0][e]) < 1e-8


def test_insertion_argument_checks():
    ctx, _ = make_ctx((4, 4, 4, 4), 0.124, 0.01, 5)
    v = cuda(S.random_spinor((4, 4, 4, 4), 1))
    with pytest.raises(P.TMError) as ei:          # HPE is ultra-local only
        ctx.loops(loop_params(1, 1, 0, P.TM_EST_HPE, 1))
    assert ei.value.status == P.TM_ERR_ARG
    with pytest.raises(P.TMError):
        ctx.loops(loop_params(1, 1, 0, P.TM_EST_STD, 2))
    with pytest.raises(P.TMError):
        ctx.contract_momentum(v, v, 1, P.TM_EST_HPE, 0)
    with pytest.raises(P.TMError):
        ctx.contract_momentum(v, v, 1, P.TM_EST_ONE_END, 0, derivative=3)


def test_c3_insertions_sampled():
    """32^3 x 64, 12 RHS, 80 insertions at |n|^2 <= 1: the first two RHS
    against the oracle (STD and generalised one-end) on three sampled time
    slices (boundary and bulk), the full 12 by linearity over the RHS split."""
    cfg = S.CONFIGS["c3"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    nrhs, p2max = 12, 1
    eta = S.random_spinor(L, 311, nrhs)
    s = S.random_spinor(L, 312, nrhs)
    est = P.TM_EST_STD | P.TM_EST_GEN_ONE_END
    got = ctx.contract_momentum(cuda(eta), cuda(s), nrhs, est, p2max, derivative=1)
    a = ctx.contract_momentum(cuda(eta[:2]), cuda(s[:2]), 2, est, p2max, derivative=1)
    b = ctx.contract_momentum(cuda(eta[2:]), cuda(s[2:]), nrhs - 2, est, p2max, derivative=1)
    assert rel(got, a + b) < 1e-12
    moms = O.momenta(p2max)
    ts = [0, 31, L[3] - 1]
    ref = None
    for r in range(2):
        x = O.contract_insertions(L, kappa, eps, -1, U, eta[r], s[r], int(est), True, moms,
                                  slices=ts)
        ref = x if ref is None else {e: ref[e] + x[e] for e in ref}
    for k, e in enumerate((O.EST_STD, O.EST_GEN_ONE_END)):
        assert rel(a[k][..., ts], ref[e][..., ts]) < 1e-12, (e, rel(a[k][..., ts], ref[e][..., ts]))
    ctx.close()
