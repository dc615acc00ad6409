"""The benchmark configurations against the FP64 oracle, at their full sizes.

c2 (16^3x32, TSM + HPE): the high-precision loops of the first noises against
the oracle's own solves; the FP16- and FP32-storage truncated solves meet
the 1e-2 criterion by the oracle's residual and their loops are the oracle's
contraction of those solutions; the TSM combination is eq. estiTSM of the
per-noise loops.

c3 (32^3x64, the chosen scheme): one Z4 noise x 12 spin-colour dilutions
solved together with FP16-storage mixed CG; the oracle recomputes all twelve
residuals and contracts the one-end loop of the twelve solutions.

c4 (uneven batch, 8^3x16 / 12^3x24 / 16^3x32): every instance's solutions
meet 1e-9 by the oracle's residual and the batched loops of the two larger
lattices are the oracle's contraction of those solutions.

Several results are correct for a solve (any x within tolerance), so solver
parity is the oracle's residual, and loop parity is either the oracle's
contraction of the library's own solutions (1e-12) or, for exact solves, the
oracle's own loops (1e-8 normwise).
"""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def residual(cfg, U, x, b, mu_sign=1):
    Mx = O.apply_M(cfg["L"], cfg["kappa"], mu_sign * cfg["two_kappa_mu"], -1, U, x)
    return np.linalg.norm(b - Mx) / np.linalg.norm(b)


def context(name):
    cfg = S.CONFIGS[name]
    U = S.gauge_links(cfg["L"], cfg["eps_links"], cfg["seed"])
    ctx = P.Context(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"])
    ctx.set_gauge(cuda(U))
    return ctx, cfg, U


# ---------------------------------------------------------------- c2

@pytest.fixture(scope="module")
def c2():
    ctx, cfg, U = context("c2")
    yield ctx, cfg, U
    ctx.close()


@pytest.mark.parametrize("lprec", [P.TM_F16, P.TM_F32])
def test_c2_tsm_hpe(c2, lprec):
    """16^3x32 with the configuration's physics: 2 noises get high- and
    low-precision solves, 3 more low-precision only; STD and HPE loops."""
    ctx, cfg, U = c2
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    seed, n_hp, n_lp = S.NOISE_SEEDS["c2"], 2, 3
    est = P.TM_EST_STD | P.TM_EST_HPE
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.mu_sign = seed, n_hp, n_lp, est, 1
    # the high-precision leg tightened to 1e-11 so that loops can be compared
    # with the oracle's own solves (loop error ~ condition x residual)
    p.hp = P.solve_params(tol=1e-11, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    p.lp = P.solve_params(tol=1e-2, solver=P.TM_CG_LOW, inner_prec=lprec)
    loops, pn, stats, st = ctx.loops(p, per_noise=True)
    assert st == P.TM_OK and stats.n_solves_hp == n_hp and stats.n_solves_lp == n_hp + n_lp
    assert stats.max_res_hp <= 1e-11 and stats.max_res_lp <= 1e-2

    # HP loops against the oracle's loops of its own solves (normwise 1e-8)
    _, ref_pn = O.loops(L, kappa, eps, -1, U, seed, n_hp, 1e-13, O.EST_STD | O.EST_HPE)
    for r in range(n_hp):
        assert rel(pn[r, 0, 0], ref_pn[r][O.EST_STD]) < 1e-8
        assert rel(pn[r, 0, 1], ref_pn[r][O.EST_HPE]) < 1e-8

    # LP solves: the same truncated solve through tm_solve (the loop driver
    # solves each source alone with the same parameters, so the solutions
    # are the ones its loops contract); the oracle's residual meets 1e-2 and
    # the oracle's contraction of them gives the per-noise LP loops
    V = int(np.prod(L))
    x = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device=DEV)
    for r in range(n_hp + n_lp):
        eta = O.noise_z4(L, seed, r)
        _, sst = ctx.solve(x, cuda(eta[None]), 1, p.lp, allow_noconv=True)
        xs = host(x)[0]
        res = residual(cfg, U, xs, eta)
        assert res <= 1e-2, (r, res)
        assert abs(sst[0].true_rel_res - res) <= 1e-6 * res
        assert rel(pn[r, 1, 0], O.contract_std(L, eta, xs)) < 1e-12
        bh4 = O.bh_power(L, kappa, eps, -1, U, xs, 4)
        assert rel(pn[r, 1, 1], O.contract_std(L, eta, bh4)) < 1e-12

    # eq. estiTSM on the per-noise loops, plus the exact HPE part once
    for k, e in enumerate((O.EST_STD, O.EST_HPE)):
        comb = O.tsm_combine([pn[r, 0, k] for r in range(n_hp)],
                             [pn[r, 1, k] for r in range(n_hp)],
                             [pn[r, 1, k] for r in range(n_hp, n_hp + n_lp)])
        if e == O.EST_HPE:
            comb = comb + O.hpe_exact(L, kappa, eps, -1, U)
        assert rel(loops[k], comb) < 1e-13


# ---------------------------------------------------------------- c3

def test_c3_chosen_12rhs_solve_and_oneend_loops():
    """32^3x64: the benchmark step.  One Z4 noise (seed 203) x 12 spin-colour
    dilutions through tm_solve with the chosen scheme (FP16 storage, FP32
    arithmetic, FP64 reliable updates, 12 RHS per Dslash); all 12 residuals
    recomputed by the oracle; the one-end loops of tm_loops with the same
    scheme equal the oracle's contraction of those 12 solutions."""
    ctx, cfg, U = context("c3")
    L, eps = cfg["L"], cfg["two_kappa_mu"]
    V = int(np.prod(L))
    seed = S.NOISE_SEEDS["c3"]
    chosen = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    eta = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=DEV)
    ctx.noise(eta, seed, 0, P.TM_DIL_SPIN_COLOUR)
    x = torch.zeros_like(eta)
    st, stats = ctx.solve(x, eta, 12, chosen)
    assert st == P.TM_OK
    xs, es = host(x), host(eta)
    assert np.array_equal(es, O.dilute_spin_colour(O.noise_z4(L, seed, 0)))
    for d in range(12):
        res = residual(cfg, U, xs[d], es[d])
        assert res <= 1e-9, (d, res)
        assert abs(stats[d].true_rel_res - res) <= 1e-3 * res
        assert stats[d].bytes > 0 and stats[d].flops > 0
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.mu_sign = seed, 1, 0, P.TM_EST_ONE_END, 1
    p.dilution, p.hp = P.TM_DIL_SPIN_COLOUR, chosen
    loops, _, lst, lstatus = ctx.loops(p)
    assert lstatus == P.TM_OK and lst.max_res_hp <= 1e-9
    ref = sum(O.contract_oneend(L, eps, xs[d]) for d in range(12))
    assert rel(loops[0], ref) < 1e-12
    ctx.close()


# ---------------------------------------------------------------- c4

def test_c4_batch_solutions_and_loops_against_oracle():
    """Uneven batch 8^3x16 / 12^3x24 / 16^3x32 with 4 / 2 / 1 noises x 12
    dilutions: every solution of the batched solve meets 1e-9 by the oracle's
    residual, and the batched loops of 12^3x24 and 16^3x32 (STD and one-end)
    are the oracle's contraction of those solutions (the batch's loop driver
    solves the same sources with the same parameters in the same batch)."""
    names, n_noise = ("c4a", "c4b", "c4c"), (4, 2, 1)
    made = [context(n) for n in names]
    ctxs = [m[0] for m in made]
    hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    est = P.TM_EST_STD | P.TM_EST_ONE_END
    plist, srcs = [], []
    for k, ((ctx, cfg, U), nn) in enumerate(zip(made, n_noise)):
        p = P.tm_loop_params()
        p.seed, p.n_hp, p.n_lp, p.estimators, p.mu_sign = 1040 + k, nn, 0, est, 1
        p.dilution, p.hp = P.TM_DIL_SPIN_COLOUR, hp
        plist.append(p)
        srcs.append(np.concatenate([O.dilute_spin_colour(O.noise_z4(cfg["L"], 1040 + k, r))
                                    for r in range(nn)]))
    batch = P.Batch(ctxs)
    xs = [torch.zeros(s.shape, dtype=torch.complex128, device=DEV) for s in srcs]
    st, stats = batch.solve(xs, [cuda(s) for s in srcs], [len(s) for s in srcs], hp)
    assert st == P.TM_OK
    loops, lstats, lst = batch.loops(plist)
    assert lst == P.TM_OK
    for i, ((ctx, cfg, U), nn) in enumerate(zip(made, n_noise)):
        sol = host(xs[i])
        for d in range(len(srcs[i])):
            assert residual(cfg, U, sol[d], srcs[i][d]) <= 1e-9, (names[i], d)
        if i == 0:
            continue  # 8^3x16 loops: test_gpu_batch compares them with the oracle's loops
        L, eps = cfg["L"], cfg["two_kappa_mu"]
        ref_std = sum(O.contract_std(L, srcs[i][d], sol[d]) for d in range(len(sol))) / nn
        ref_1e = sum(O.contract_oneend(L, eps, sol[d]) for d in range(len(sol))) / nn
        assert rel(loops[i][0], ref_std) < 1e-12, names[i]
        assert rel(loops[i][1], ref_1e) < 1e-12, names[i]
    batch.close()
    for c in ctxs:
        c.close()
