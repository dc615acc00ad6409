"""Time dilution with coherent sources (sec. II.D) and the single-time-slice
contraction on the device against the oracle."""
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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def c1():
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    U = S.gauge_links(L, cfg["eps_links"], cfg["seed"])
    ctx = P.Context(L, kappa, eps)
    ctx.set_gauge(cuda(U))
    yield dict(L=L, kappa=kappa, eps=eps, U=U, ctx=ctx)
    ctx.close()


def loop_params(seed, n_hp, n_lp, est, period, dilution=P.TM_DIL_NONE, derivative=0):
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.dilution, p.mu_sign = seed, n_hp, n_lp, est, \
        dilution, 1
    p.t_period, p.derivative = period, derivative
    p.hp = P.solve_params(tol=1e-11, solver=P.TM_CG_F64)
    p.lp = P.solve_params(tol=1e-2, solver=P.TM_CG_LOW, inner_prec=P.TM_F16, check_every=1)
    return p


@pytest.mark.parametrize("period,dilution", [(2, P.TM_DIL_NONE), (8, P.TM_DIL_NONE),
                                             (4, P.TM_DIL_SPIN_COLOUR), (1, P.TM_DIL_NONE)])
def test_time_dilution_vs_oracle(c1, period, dilution):
    """STD, one-end and HPE loops from coherent (P < Lt) and plain (P = Lt)
    time-diluted sources within 1e-8 of the oracle; the solve count is
    P x (12 or 1) per noise, in batches of up to 12 RHS."""
    L, kappa, eps, U, ctx = c1["L"], c1["kappa"], c1["eps"], c1["U"], c1["ctx"]
    est = P.TM_EST_STD | P.TM_EST_ONE_END | P.TM_EST_HPE
    n = 1
    got, pn, st, _ = ctx.loops(loop_params(231, n, 0, est, period, dilution), per_noise=True)
    dil = dilution == P.TM_DIL_SPIN_COLOUR
    ref, ref_pn = O.loops(L, kappa, eps, -1, U, 231, n, 1e-13, int(est), dilution=dil,
                          t_period=period)
    for k, e in enumerate((O.EST_STD, O.EST_ONE_END, O.EST_HPE)):
        assert rel(got[k], ref[e]) < 1e-8, (e, rel(got[k], ref[e]))
    assert st.n_solves_hp == n * period * (12 if dil else 1)
    assert st.max_res_hp <= 1e-11


def test_time_dilution_with_derivative_momentum_and_tsm(c1):
    """Time-diluted sources with derivative insertions and momenta (these
    contractions visit every slice) and with TSM: the library's per-noise
    HP loops against the oracle, the combination against eq. estiTSM."""
    L, kappa, eps, U, ctx = c1["L"], c1["kappa"], c1["eps"], c1["U"], c1["ctx"]
    est = P.TM_EST_STD | P.TM_EST_GEN_ONE_END
    got, pn, _, _ = ctx.loops_momentum(loop_params(233, 1, 1, est, 4, derivative=1), 1,
                                       per_noise=True)
    moms = O.momenta(1)
    ref, ref_pn = O.loops_momentum(L, kappa, eps, -1, U, 233, 1, 1e-13, int(est), moms,
                                   derivative=True, t_period=4)
    for k, e in enumerate((O.EST_STD, O.EST_GEN_ONE_END)):
        assert rel(pn[0, 0, k], ref_pn[0][e]) < 1e-8, (e, rel(pn[0, 0, k], ref_pn[0][e]))
        comb = O.tsm_combine([pn[0, 0, k]], [pn[0, 1, k]], [pn[1, 1, k]])
        assert rel(got[k], comb) < 1e-13


def test_single_slice_contraction_support(c1):
    """With plain time dilution the per-noise STD loop of one source lives on
    its own slice: for P = Lt every slice is reached exactly once, and the
    sum equals the per-slice oracle value."""
    L, kappa, eps, U, ctx = c1["L"], c1["kappa"], c1["eps"], c1["U"], c1["ctx"]
    got, _, st, _ = ctx.loops(loop_params(235, 1, 0, P.TM_EST_STD, L[3]))
    ref, _ = O.loops(L, kappa, eps, -1, U, 235, 1, 1e-13, O.EST_STD, t_period=L[3])
    assert rel(got[0], ref[O.EST_STD]) < 1e-8
    assert got.shape == (1, 16, L[3]) and st.n_solves_hp == L[3]


def test_time_dilution_argument_checks(c1):
    ctx = c1["ctx"]
    for bad in (3, -1, 16):                       # Lt = 8: 3 does not divide, 16 > Lt
        with pytest.raises(P.TMError) as ei:
            ctx.loops(loop_params(1, 1, 0, P.TM_EST_STD, bad))
        assert ei.value.status == P.TM_ERR_ARG
