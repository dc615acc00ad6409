"""Uneven batches (three lattices; each group of CG iterations one launch of
the persistent batch kernel or a graph of multi-instance launches, timed
once each and the faster kept; beyond four lattices, and for FP64, the
graph).

Each instance of a batch must reproduce its own single-lattice solve bit for
bit (same arithmetic, same reliable-update cadence); residuals are also
recomputed by the FP64 oracle, and the per-instance loops are checked
against the oracle and against the single-lattice loop driver.  The
persistent kernel's barrier waits are bounded: with a spin limit of zero
the launch gives up, the call reports it, and the device stays usable.
"""
import os

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
C4 = ("c4a", "c4b", "c4c")
NRHS = {"c4a": 48, "c4b": 24, "c4c": 12}


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def inst():
    out = []
    for name in C4:
        cfg = S.CONFIGS[name]
        U = S.gauge_links(cfg["L"], cfg["eps_links"], cfg["seed"])
        ctx = P.Context(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"])
        ctx.set_gauge(cuda(U))
        out.append(dict(name=name, cfg=cfg, U=U, ctx=ctx))
    yield out
    for d in out:
        d["ctx"].close()


def sources(d, n, seed):
    return S.random_spinor(d["cfg"]["L"], seed, n)


@pytest.mark.parametrize("solver,prec", [(P.TM_CG_MIXED, P.TM_F16), (P.TM_CG_F64, P.TM_F32)])
def test_batch_solve_matches_single_bit_for_bit(inst, solver, prec):
    params = P.solve_params(tol=1e-9, solver=solver, inner_prec=prec)
    bs = [cuda(sources(d, NRHS[d["name"]], 300 + k)) for k, d in enumerate(inst)]
    xs = [torch.zeros_like(b) for b in bs]
    batch = P.Batch([d["ctx"] for d in inst])
    st, bstats = batch.solve(xs, bs, [NRHS[d["name"]] for d in inst], params)
    batch.close()
    for k, d in enumerate(inst):
        n = NRHS[d["name"]]
        x1 = torch.zeros_like(bs[k])
        _, sstats = d["ctx"].solve(x1, bs[k], n, params)
        assert torch.equal(xs[k], x1), d["name"]
        assert [s.iters for s in bstats[k]] == [s.iters for s in sstats]
        assert max(s.true_rel_res for s in bstats[k]) <= 1e-9
        # the oracle recomputes the residual of a few right-hand sides
        cfg, U = d["cfg"], d["U"]
        xh, bh = host(xs[k]), host(bs[k])
        for r in (0, n - 1):
            res = np.linalg.norm(bh[r] - O.apply_M(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"], -1, U,
                                                   xh[r])) / np.linalg.norm(bh[r])
            assert res <= 1e-9, (d["name"], r, res)


def loop_params(seed, n_hp, est, hp):
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.dilution, p.mu_sign = seed, n_hp, 0, est, \
        P.TM_DIL_SPIN_COLOUR, 1
    p.hp = hp
    return p


def test_batch_loops(inst):
    """c4: 4 / 2 / 1 noise vectors x 12 spin-colour dilutions (48 / 24 / 12
    RHS) in one batch, mixed FP16 CG to 1e-9; per-instance loops against the
    single-lattice driver (1e-7 normwise: the solves differ only in reliable-
    update timing) and, for the 8^3x16 lattice, against the oracle."""
    hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    est = P.TM_EST_STD | P.TM_EST_ONE_END | P.TM_EST_HPE
    plist = [loop_params(1040 + k, NRHS[d["name"]] // 12, est, hp) for k, d in enumerate(inst)]
    batch = P.Batch([d["ctx"] for d in inst])
    outs, stats, st = batch.loops(plist)
    batch.close()
    for k, d in enumerate(inst):
        assert stats[k].max_res_hp <= 1e-9 and stats[k].n_solves_hp == NRHS[d["name"]]
        single, _, sst, _ = d["ctx"].loops(plist[k])
        for e in range(3):
            err = np.abs(outs[k][e] - single[e]).max() / np.abs(single[e]).max()
            assert err < 1e-7, (d["name"], e, err)
    # oracle, first lattice, first noise only
    d = inst[0]
    cfg = d["cfg"]
    p1 = loop_params(1040, 1, est, hp)
    batch = P.Batch([d["ctx"]])
    outs1, _, _ = batch.loops([p1])
    batch.close()
    ref, _ = O.loops(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"], -1, d["U"], 1040, 1, 1e-12, 7,
                     dilution=True)
    for e, key in enumerate((O.EST_STD, O.EST_ONE_END, O.EST_HPE)):
        err = np.abs(outs1[0][e] - ref[key]).max() / np.abs(ref[key]).max()
        assert err < 1e-7, (key, err)


def test_batch_loops_insertions_and_gen(inst):
    """Batched loops with the generalised one-end estimator and one-derivative
    insertions (80 per estimator) and the HPE in mask order STD, HPE, GEN:
    each instance against the single-lattice driver; time dilution is
    rejected for batches."""
    hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    est = P.TM_EST_STD | P.TM_EST_GEN_ONE_END
    plist = [loop_params(1050 + k, 1, est, hp) for k, d in enumerate(inst)]
    for p in plist:
        p.derivative = 1
    batch = P.Batch([d["ctx"] for d in inst])
    outs, stats, _ = batch.loops(plist)
    for k, d in enumerate(inst):
        assert outs[k].shape == (2, 80, d["cfg"]["L"][3])
        single, _, _, _ = d["ctx"].loops(plist[k])
        for e in range(2):
            err = np.abs(outs[k][e] - single[e]).max() / np.abs(single[e]).max()
            assert err < 1e-7, (d["name"], e, err)
    est3 = P.TM_EST_STD | P.TM_EST_HPE | P.TM_EST_GEN_ONE_END
    plist = [loop_params(1060 + k, 1, est3, hp) for k, d in enumerate(inst)]
    outs, _, _ = batch.loops(plist)
    for k, d in enumerate(inst):
        single, _, _, _ = d["ctx"].loops(plist[k])
        for e in range(3):
            err = np.abs(outs[k][e] - single[e]).max() / np.abs(single[e]).max()
            assert err < 1e-7, (d["name"], e, err)
    bad = [loop_params(1, 1, P.TM_EST_STD, hp) for _ in inst]
    bad[0].t_period = 2
    with pytest.raises(P.TMError) as ei:
        batch.loops(bad)
    assert ei.value.status == P.TM_ERR_ARG
    batch.close()


def test_batch_argument_checks(inst):
    import ctypes
    arr = (ctypes.c_void_p * 2)(inst[0]["ctx"].h, inst[0]["ctx"].h)
    h = ctypes.c_void_p()
    assert P.tm_batch_create(ctypes.byref(h), arr, 2) == P.TM_ERR_ARG
    batch = P.Batch([d["ctx"] for d in inst])
    hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    bad = [loop_params(1, 1, P.TM_EST_STD, hp) for _ in inst]
    bad[1].n_lp = 2
    with pytest.raises(P.TMError) as ei:
        batch.loops(bad)
    assert ei.value.status == P.TM_ERR_ARG
    batch.close()


def batch_solve_env(inst, names, params, env, seed0):
    """Batch solve of the listed instances with environment switches set
    while the batch is created; returns (sources, solutions, stats)."""
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        batch = P.Batch([inst[n]["ctx"] for n in names])
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    try:
        bs = [cuda(sources(inst[n], inst[n]["nrhs"], seed0 + k)) for k, n in enumerate(names)]
        xs = [torch.zeros_like(b) for b in bs]
        st, stats = batch.solve(xs, bs, [inst[n]["nrhs"] for n in names], params)
    finally:
        batch.close()
    return bs, xs, stats


@pytest.fixture(scope="module")
def five():
    """Five lattices: the three c4 ones and two more small ones."""
    out = {}
    specs = [(n, S.CONFIGS[n]["L"], S.CONFIGS[n]["kappa"], S.CONFIGS[n]["two_kappa_mu"],
              S.CONFIGS[n]["eps_links"], S.CONFIGS[n]["seed"], NRHS[n] // 4) for n in C4]
    specs += [("e1", (4, 4, 4, 8), 0.124, 0.01, 0.3, 1101, 6), ("e2", (6, 4, 4, 6), 0.124, 0.005, 0.2, 1102, 3)]
    for name, L, kappa, eps, el, seed, n in specs:
        U = S.gauge_links(L, el, seed)
        ctx = P.Context(L, kappa, eps)
        ctx.set_gauge(cuda(U))
        out[name] = dict(name=name, cfg=dict(L=L), ctx=ctx, nrhs=n)
    yield out
    for d in out.values():
        d["ctx"].close()


def test_graph_path_beyond_four_lattices_matches_persistent(five):
    """Five lattices take the graph of multi-instance launches; on three, the
    persistent kernel (forced), the graph (forced) and the timed choice give
    the same solutions: all bit-identical to the single-lattice solves."""
    params = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    names5 = ["c4a", "c4b", "c4c", "e1", "e2"]
    bs, xs, _ = batch_solve_env(five, names5, params, {}, 700)
    _, xs_p, _ = batch_solve_env(five, names5[:3], params, {"TM_BATCH_PERSIST": "1"}, 700)
    _, xs_g, _ = batch_solve_env(five, names5[:3], params, {"TM_BATCH_PERSIST": "0"}, 700)
    _, xs_t, _ = batch_solve_env(five, names5[:3], params, {}, 700)
    for k, n in enumerate(names5):
        x1 = torch.zeros_like(bs[k])
        five[n]["ctx"].solve(x1, bs[k], five[n]["nrhs"], params)
        assert torch.equal(xs[k], x1), n
        if k < 3:
            assert torch.equal(xs_p[k], x1) and torch.equal(xs_g[k], x1) and torch.equal(xs_t[k], x1), n


def test_ten_lattices_match_single_solves():
    """Ten small lattices in one batch: the multi-lattice scalar and update
    launches take at most eight lattices each, so an iteration issues two of
    each; every solution equals its single-lattice solve bit for bit, in the
    FP16 mixed and the plain FP64 solver."""
    shapes = [(4, 4, 4, 8), (6, 4, 4, 6), (4, 4, 6, 4), (4, 6, 4, 4), (6, 6, 4, 4)]
    inst = {}
    try:
        for k in range(10):
            L = shapes[k % len(shapes)]
            U = S.gauge_links(L, 0.2 + 0.02 * k, 1200 + k)
            ctx = P.Context(L, 0.124, 0.004 + 0.001 * k)
            ctx.set_gauge(cuda(U))
            inst["t%d" % k] = dict(name="t%d" % k, cfg=dict(L=L), ctx=ctx, nrhs=1 + k % 3)
        names = sorted(inst)
        for solver, prec in ((P.TM_CG_MIXED, P.TM_F16), (P.TM_CG_F64, P.TM_F32)):
            params = P.solve_params(tol=1e-9, solver=solver, inner_prec=prec)
            bs, xs, stats = batch_solve_env(inst, names, params, {}, 1300)
            for k, n in enumerate(names):
                x1 = torch.zeros_like(bs[k])
                inst[n]["ctx"].solve(x1, bs[k], inst[n]["nrhs"], params)
                assert torch.equal(xs[k], x1), (solver, n)
                assert all(st.converged == 1 for st in stats[k]), (solver, n)
    finally:
        for d in inst.values():
            d["ctx"].close()


def test_persistent_barrier_wait_is_bounded(five):
    """A spin limit of zero makes the persistent kernel's barrier waits give
    up at once: every block leaves the kernel, the call fails with
    TM_ERR_HIP and says why, and the next batch on the same contexts solves
    normally."""
    params = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    names = ["c4a", "c4b", "c4c"]
    with pytest.raises(P.TMError) as ei:
        batch_solve_env(five, names, params, {"TM_BATCH_SPIN_LIMIT": "0", "TM_BATCH_PERSIST": "1"}, 710)
    assert ei.value.status == P.TM_ERR_HIP and "barrier" in str(ei.value)
    bs, xs, stats = batch_solve_env(five, names, params, {}, 710)
    for k, n in enumerate(names):
        x1 = torch.zeros_like(bs[k])
        five[n]["ctx"].solve(x1, bs[k], five[n]["nrhs"], params)
        assert torch.equal(xs[k], x1), n
        assert all(s.converged == 1 for s in stats[k])
