"""8-parameter FP64 links (appendix A.1, the paper's 8-parameter
reconstruction) against the FP64 oracle.

The FP64 kernels rebuild each link from a2, a3, b1 and the phases of a1 and
c1; the operator they apply must agree with the oracle's exact operator to
1e-13 for every kind, both time boundary conditions, near-identity and
generic fields (the lower rows of about half the links are stored exchanged),
and solves must meet their tolerance by the oracle's residual.  Fields with
exactly diagonal links (the unit field) cannot use the form and keep 12
parameters.
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


def mask_parity(L, v, p):
    w = v.copy()
    w[..., O.site_parity(L) != p, :, :] = 0
    return w


def half_buf(ctx, prec, nrhs):
    return torch.zeros(ctx.half_numel(prec, nrhs), dtype=torch.uint8, device=DEV)


def operator_cases(L, kappa, eps, t_bc, U, v, nrhs):
    ve = [mask_parity(L, v[r], 0) for r in range(nrhs)]
    return [
        (P.TM_HOP_OE, 1, lambda r: mask_parity(L, O.hop(L, kappa, t_bc, U, ve[r]), 1)),
        (P.TM_SCHUR, 0, lambda r: O.schur(L, kappa, eps, t_bc, U, ve[r])),
        (P.TM_SCHUR_DAG, 0, lambda r: O.schur(L, kappa, eps, t_bc, U, ve[r], adj=True)),
        (P.TM_NORMAL, 0, lambda r: O.schur(L, kappa, eps, t_bc, U,
                                           O.schur(L, kappa, eps, t_bc, U, ve[r]), adj=True)),
    ]


@pytest.mark.parametrize("t_bc", [-1, 1])
@pytest.mark.parametrize("L,eps_links", [((4, 4, 2, 6), 0.3), ((6, 4, 4, 6), 0.05), ((4, 4, 4, 8), 2.0)])
def test_link_format_8_parameters_fp64(L, eps_links, t_bc):
    kappa, eps = 0.124, 0.0123
    U = S.gauge_links(L, eps_links, 23)
    ctx = P.Context(L, kappa, eps, t_bc=t_bc)
    try:
        ctx.set_gauge(cuda(U))
        nrhs = 2
        v = S.random_spinor(L, 11, nrhs)
        prec = P.TM_F64
        e, o = half_buf(ctx, prec, nrhs), half_buf(ctx, prec, nrhs)
        ctx.pack(e, o, cuda(v), nrhs, prec)
        outs = {}
        for fmt in (8, 18):
            ctx.set_link_format(fmt)
            for kind, par, ref in operator_cases(L, kappa, eps, t_bc, U, v, nrhs):
                outh = half_buf(ctx, prec, nrhs)
                ctx.dslash(outh, e, nrhs, kind, 1, prec, P.TM_F64)
                full = torch.zeros((nrhs,) + v.shape[1:], dtype=torch.complex128, device=DEV)
                if par == 0:
                    ctx.unpack(full, outh, half_buf(ctx, prec, nrhs), nrhs, prec)
                else:
                    ctx.unpack(full, half_buf(ctx, prec, nrhs), outh, nrhs, prec)
                outs[(fmt, kind)] = host(full)
                for r in range(nrhs):
                    assert rel(outs[(fmt, kind)][r], ref(r)) < 1e-13, (fmt, kind, r)
        for kind, _, _ in operator_cases(L, kappa, eps, t_bc, U, v, nrhs):
            # the rebuilt links differ from the stored ones by rounding only
            d = rel(outs[(8, kind)], outs[(18, kind)])
            assert 0 < d < 1e-13, (kind, d)
        # full-lattice operator (canonical FP64 in and out)
        ctx.set_link_format(8)
        x = torch.empty_like(cuda(v))
        ctx.dslash(x, cuda(v), nrhs, P.TM_FULL, 1, P.TM_F64)
        got = host(x)
        for r in range(nrhs):
            assert rel(got[r], O.apply_M(L, kappa, eps, t_bc, U, v[r])) < 1e-13
    finally:
        ctx.close()


def test_unit_links_keep_12_parameters():
    """Exactly diagonal links (n = 0) cannot be rebuilt from 8 parameters:
    the FP64 kernels keep the 12-parameter form and stay exact."""
    L, kappa, eps = (4, 4, 4, 8), 0.124, 0.0123
    U = S.unit_links(L)
    ctx = P.Context(L, kappa, eps)
    try:
        ctx.set_gauge(cuda(U))
        ctx.set_link_format(8)
        v = S.random_spinor(L, 12, 1)
        x = torch.empty_like(cuda(v))
        ctx.dslash(x, cuda(v), 1, P.TM_FULL, 1, P.TM_F64)
        assert rel(host(x)[0], O.apply_M(L, kappa, eps, -1, U, v[0])) < 1e-13
    finally:
        ctx.close()


@pytest.mark.parametrize("solver", [P.TM_CG_F64, P.TM_CG_MIXED])
def test_solves_with_8_parameter_links(solver):
    """Plain FP64 CG reads the 8-parameter links throughout; mixed CG its
    reliable updates (all 18 parameters) and FP16 inner solves (12): both
    meet the tolerance by the oracle's residual."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    U = S.gauge_links(L, cfg["eps_links"], cfg["seed"])
    ctx = P.Context(L, kappa, eps)
    try:
        ctx.set_gauge(cuda(U))
        ctx.set_link_format(8)
        b = S.random_spinor(L, 13, 2)
        x = torch.zeros_like(cuda(b))
        _, stats = ctx.solve(x, cuda(b), 2, P.solve_params(tol=1e-10, solver=solver,
                                                           inner_prec=P.TM_F16))
        xs = host(x)
        for r in range(2):
            Mx = O.apply_M(L, kappa, eps, -1, U, xs[r])
            res = np.linalg.norm(b[r] - Mx) / np.linalg.norm(b[r])
            assert res <= 1.05e-10, (r, res)
            assert stats[r].converged == 1
    finally:
        ctx.close()


def test_batch_with_8_parameter_links_matches_single():
    """The multi-instance FP64 Dslash reads the same 8-parameter links: a
    batch of two lattices equals their single solves bit for bit."""
    insts = []
    try:
        for name in ("c4a", "c4b"):
            cfg = S.CONFIGS[name]
            U = S.gauge_links(cfg["L"], cfg["eps_links"], cfg["seed"])
            ctx = P.Context(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"])
            ctx.set_gauge(cuda(U))
            ctx.set_link_format(8)
            insts.append((cfg, ctx))
        params = P.solve_params(tol=1e-9, solver=P.TM_CG_F64)
        bs = [cuda(S.random_spinor(cfg["L"], 40 + k, 2)) for k, (cfg, _) in enumerate(insts)]
        xs = [torch.zeros_like(b) for b in bs]
        batch = P.Batch([c for _, c in insts])
        try:
            batch.solve(xs, bs, [2, 2], params)
        finally:
            batch.close()
        for (cfg, ctx), b, xb in zip(insts, bs, xs):
            x1 = torch.zeros_like(b)
            ctx.solve(x1, b, 2, params)
            assert np.array_equal(host(xb), host(x1))
    finally:
        for _, c in insts:
            c.close()
