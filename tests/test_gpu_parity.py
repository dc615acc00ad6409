"""GPU parity: the HIP library through its C-ABI against the FP64 CPU oracle.

Bars: integer/layout work bit-exact (pack/unpack, Z4 noise); FP64 operators
within 1e-13 normwise; FP32/FP16/BF16 operators within their storage
rounding; solves judged by the true residual recomputed by the oracle (any x
meeting the tolerance is correct); loops within 1e-8 normwise of the oracle
for high-precision solves.
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
G5 = np.array([1, 1, -1, -1], dtype=float)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make_ctx(L, kappa, eps, seed, eps_links=0.3, t_bc=-1):
    U = S.gauge_links(L, eps_links, seed)
    ctx = P.Context(L, kappa, eps, t_bc=t_bc)
    ctx.set_gauge(cuda(U))
    return ctx, U


def half_buf(ctx, prec, nrhs):
    return torch.zeros(ctx.half_numel(prec, nrhs), dtype=torch.uint8, device=DEV)


def to_half_numpy(full, L):
    """Reference of the half layout's valid sites: even/odd [nrhs][12][V/2]
    from canonical (the library's planes have stride hs >= V/2)."""
    V = int(np.prod(L))
    par = O.site_parity(L)
    s = np.arange(V)
    f = full.reshape(full.shape[0], V, 12)
    out = []
    for p in (0, 1):
        h = np.zeros((full.shape[0], 12, V // 2), dtype=complex)
        h[:, :, s[par == p] >> 1] = f[:, par == p, :].transpose(0, 2, 1)
        out.append(h)
    return out


def valid(ctx, t, nrhs):
    """Valid half-sites of every plane of a half field given as bytes (the
    pad sites at the end of each plane of stride hs are unspecified)."""
    return t.view(nrhs, 12, ctx.hs, -1)[:, :, :ctx.vh]


def mask_parity(L, v, p):
    w = v.copy()
    w[..., O.site_parity(L) != p, :, :] = 0
    return w


def bf16_round(x):
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


LATS = [(4, 4, 4, 8), (6, 4, 4, 6), (2, 2, 2, 2), (16, 16, 16, 32)]


# ---------------------------------------------------------------- layout, noise

@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 2, 6)])
def test_pack_unpack_layout_bit_exact(L):
    ctx, _ = make_ctx(L, 0.124, 0.01, 5)
    nrhs = 3
    full = S.random_spinor(L, 7, nrhs)
    fe, fo = to_half_numpy(full, L)
    dfull = cuda(full)
    vh, hs = ctx.vh, ctx.hs
    # the plane stride: vh rounded up to an odd multiple of 32 half-sites
    assert hs >= vh and hs % 32 == 0 and (hs // 32) % 2 == 1 and hs - vh < 64
    for prec in (P.TM_F64, P.TM_F32, P.TM_F16, P.TM_BF16):
        e, o = half_buf(ctx, prec, nrhs), half_buf(ctx, prec, nrhs)
        assert e.numel() == P.PREC_BYTES[prec] * 12 * hs * nrhs
        ctx.pack(e, o, dfull, nrhs, prec)
        if prec == P.TM_F64:
            he = host(e).view(np.complex128).reshape(nrhs, 12, hs)[:, :, :vh]
            ho = host(o).view(np.complex128).reshape(nrhs, 12, hs)[:, :, :vh]
            assert np.array_equal(he, fe) and np.array_equal(ho, fo)
            back = torch.zeros_like(dfull)
            ctx.unpack(back, e, o, nrhs, prec)
            assert np.array_equal(host(back), full)
        else:
            for got, ref in ((host(e), fe), (host(o), fo)):
                # valid sites of every plane (re, im pairs of 2 or 4 bytes)
                got = got.reshape(nrhs, 12, hs, -1)[:, :, :vh].copy()
                if prec == P.TM_F32:
                    g = got.view(np.float32)
                    r = ref.view(np.float64).astype(np.float32)
                elif prec == P.TM_F16:
                    g = got.view(np.float16)
                    r = ref.view(np.float64).astype(np.float16)
                else:
                    g = got.view(np.uint16).astype(np.uint32) << 16
                    g = g.view(np.float32)
                    r = bf16_round(ref.view(np.float64).astype(np.float32))
                assert np.array_equal(g.reshape(-1), r.reshape(-1)), prec


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 2, 6)])
def test_noise_bit_exact(L):
    ctx, _ = make_ctx(L, 0.124, 0.01, 5)
    V = int(np.prod(L))
    for seed, r in ((201, 0), (201, 3), (2 ** 63 + 12345, 7)):
        out = torch.zeros((V, 4, 3), dtype=torch.complex128, device=DEV)
        ctx.noise(out, seed, r)
        assert np.array_equal(host(out), O.noise_z4(L, seed, r))
        out12 = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=DEV)
        ctx.noise(out12, seed, r, P.TM_DIL_SPIN_COLOUR)
        assert np.array_equal(host(out12), O.dilute_spin_colour(O.noise_z4(L, seed, r)))


# ---------------------------------------------------------------- operators

@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("mu_sign", [1, -1])
def test_full_operator_fp64(L, mu_sign):
    kappa, eps = 0.124, 0.0123
    ctx, U = make_ctx(L, kappa, eps, 11)
    nrhs = 2
    v = S.random_spinor(L, 3, nrhs)
    dv = cuda(v)
    for kind, adj in ((P.TM_FULL, False), (P.TM_FULL_DAG, True)):
        out = torch.zeros_like(dv)
        ctx.dslash(out, dv, nrhs, kind, mu_sign)
        got = host(out)
        for r in range(nrhs):
            ref = O.apply_M(L, kappa, mu_sign * eps, -1, U, v[r], adj=adj)
            assert rel(got[r], ref) < 1e-13, (kind, r)


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 4, 6), (2, 2, 2, 2)])
def test_periodic_time_boundary(L):
    kappa, eps = 0.124, 0.02
    ctx, U = make_ctx(L, kappa, eps, 12, t_bc=1)
    v = S.random_spinor(L, 4)
    out = torch.zeros((1,) + v.shape, dtype=torch.complex128, device=DEV)
    ctx.dslash(out, cuda(v[None]), 1, P.TM_FULL, 1)
    assert rel(host(out)[0], O.apply_M(L, kappa, eps, 1, U, v)) < 1e-13


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 4, 6)])
def test_half_kinds_fp64(L):
    kappa, eps = 0.124, 0.0123
    ctx, U = make_ctx(L, kappa, eps, 13)
    nrhs = 2
    v = S.random_spinor(L, 5, nrhs)
    dv = cuda(v)
    e, o = half_buf(ctx, P.TM_F64, nrhs), half_buf(ctx, P.TM_F64, nrhs)
    ctx.pack(e, o, dv, nrhs, P.TM_F64)
    outh = half_buf(ctx, P.TM_F64, nrhs)
    zero = half_buf(ctx, P.TM_F64, nrhs)
    full = torch.zeros_like(dv)

    def run(kind, inp, out_parity, mu_sign=1):
        ctx.dslash(outh, inp, nrhs, kind, mu_sign)
        if out_parity == 0:
            ctx.unpack(full, outh, zero, nrhs, P.TM_F64)
        else:
            ctx.unpack(full, zero, outh, nrhs, P.TM_F64)
        return host(full)

    for r in range(nrhs):
        ve, vo = mask_parity(L, v[r], 0), mask_parity(L, v[r], 1)
        cases = [
            (P.TM_HOP_EO, o, 0, mask_parity(L, O.hop(L, kappa, -1, U, vo), 0)),
            (P.TM_HOP_OE, e, 1, mask_parity(L, O.hop(L, kappa, -1, U, ve), 1)),
            (P.TM_RINV_HOP_OE, e, 1,
             mask_parity(L, O.twist(L, eps, O.hop(L, kappa, -1, U, ve), 2), 1)),
            (P.TM_RINV_HOP_EO, o, 0,
             mask_parity(L, O.twist(L, eps, O.hop(L, kappa, -1, U, vo), 2), 0)),
            (P.TM_SCHUR, e, 0, O.schur(L, kappa, eps, -1, U, ve)),
            (P.TM_SCHUR_DAG, e, 0, O.schur(L, kappa, eps, -1, U, ve, adj=True)),
            (P.TM_NORMAL, e, 0, O.schur(L, kappa, eps, -1, U,
                                        O.schur(L, kappa, eps, -1, U, ve), adj=True)),
        ]
        for kind, inp, par, ref in cases:
            got = run(kind, inp, par)[r]
            assert rel(got, ref) < 1e-13, (kind, r)
    # the d flavour
    ve = mask_parity(L, v[0], 0)
    got = run(P.TM_SCHUR, e, 0, mu_sign=-1)[0]
    assert rel(got, O.schur(L, kappa, -eps, -1, U, ve)) < 1e-13


@pytest.mark.parametrize("prec,links,bound", [(P.TM_F32, P.TM_F32, 2e-6), (P.TM_F16, P.TM_F32, 4e-3),
                                               (P.TM_F16, P.TM_F16, 4e-3), (P.TM_BF16, P.TM_F32, 3e-2),
                                               (P.TM_BF16, P.TM_F16, 3e-2)])
@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 4, 6)])
def test_schur_low_precision(prec, links, bound, L):
    """FP32 or binary16 links with FP32/FP16/BF16 spinor storage, FP32
    arithmetic: error against the FP64 oracle is at the storage rounding
    level (binary16 links add 2^-11 relative per entry); several right-hand
    sides per thread give bit-identical results to 1 per call."""
    kappa, eps = 0.124, 0.0123
    ctx, U = make_ctx(L, kappa, eps, 14)
    nrhs = 4
    v = S.random_spinor(L, 6, nrhs)
    e, o = half_buf(ctx, prec, nrhs), half_buf(ctx, prec, nrhs)
    ctx.pack(e, o, cuda(v), nrhs, prec)
    for kind, adj in ((P.TM_SCHUR, False), (P.TM_SCHUR_DAG, True)):
        outh = half_buf(ctx, prec, nrhs)
        ctx.dslash(outh, e, nrhs, kind, 1, prec, links)
        # same storage precision back to canonical FP64
        full = torch.zeros((nrhs,) + v.shape[1:], dtype=torch.complex128, device=DEV)
        ctx.unpack(full, outh, half_buf(ctx, prec, nrhs), nrhs, prec)
        got = host(full)
        for r in range(nrhs):
            ref = O.schur(L, kappa, eps, -1, U, mask_parity(L, v[r], 0), adj=adj)
            assert rel(got[r], ref) < bound, (kind, r, rel(got[r], ref))
        # batched (2 per thread) == one right-hand side at a time, bit for bit
        nb = ctx.half_numel(prec, 1)
        for r in range(nrhs):
            one = half_buf(ctx, prec, 1)
            ctx.dslash(one, e[r * nb:(r + 1) * nb], 1, kind, 1, prec, links)
            assert torch.equal(valid(ctx, one, 1), valid(ctx, outh[r * nb:(r + 1) * nb], 1)), (kind, r)
    # odd nrhs takes the one-per-thread path
    odd = half_buf(ctx, prec, 3)
    ctx.dslash(odd, e[:3 * ctx.half_numel(prec, 1)], 3, P.TM_SCHUR, 1, prec, links)
    ctx.dslash(outh, e, nrhs, P.TM_SCHUR, 1, prec, links)
    assert torch.equal(valid(ctx, odd, 3), valid(ctx, outh[:3 * ctx.half_numel(prec, 1)], 3))


@pytest.mark.parametrize("prec,bound", [(P.TM_F16, 4e-3), (P.TM_BF16, 3e-2), (P.TM_F32, 2e-6)])
@pytest.mark.parametrize("t_bc", [-1, 1])
@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 2, 6)])
def test_link_format_12_parameters(prec, bound, t_bc, L):
    """12-parameter binary16 (FP16/BF16 spinors) or FP32 links (third row rebuilt in the kernel, boundary
    factor restored on the links that cross t = Lt-1 <-> 0): every operator
    kind against the FP64 oracle at the storage rounding level, for both time
    boundary conditions; RHS tiles bit-identical; the rebuilt operator
    differs from the 18-parameter one only at the binary16 level."""
    kappa, eps = 0.124, 0.0123
    ctx, U = make_ctx(L, kappa, eps, 17, t_bc=t_bc)
    nrhs = 2
    v = S.random_spinor(L, 8, nrhs)
    e, o = half_buf(ctx, prec, nrhs), half_buf(ctx, prec, nrhs)
    ctx.pack(e, o, cuda(v), nrhs, prec)
    ve = [mask_parity(L, v[r], 0) for r in range(nrhs)]
    vo = [mask_parity(L, v[r], 1) for r in range(nrhs)]
    cases = [
        (P.TM_HOP_OE, e, 1, lambda r: mask_parity(L, O.hop(L, kappa, t_bc, U, ve[r]), 1)),
        (P.TM_HOP_EO, o, 0, lambda r: mask_parity(L, O.hop(L, kappa, t_bc, U, vo[r]), 0)),
        (P.TM_SCHUR, e, 0, lambda r: O.schur(L, kappa, eps, t_bc, U, ve[r])),
        (P.TM_SCHUR_DAG, e, 0, lambda r: O.schur(L, kappa, eps, t_bc, U, ve[r], adj=True)),
    ]
    outs = {}
    lprec = P.TM_F32 if prec == P.TM_F32 else P.TM_F16
    for fmt in (12, 18):
        ctx.set_link_format(fmt)
        for kind, inp, par, ref in cases:
            outh = half_buf(ctx, prec, nrhs)
            ctx.dslash(outh, inp, nrhs, kind, 1, prec, lprec)
            full = torch.zeros((nrhs,) + v.shape[1:], dtype=torch.complex128, device=DEV)
            if par == 0:
                ctx.unpack(full, outh, half_buf(ctx, prec, nrhs), nrhs, prec)
            else:
                ctx.unpack(full, half_buf(ctx, prec, nrhs), outh, nrhs, prec)
            got = host(full)
            outs[(fmt, kind)] = got
            for r in range(nrhs):
                assert rel(got[r], ref(r)) < bound, (fmt, kind, r, rel(got[r], ref(r)))
            if fmt == 12:
                nb = ctx.half_numel(prec, 1)
                one = half_buf(ctx, prec, 1)
                ctx.dslash(one, inp[nb:2 * nb], 1, kind, 1, prec, lprec)
                assert torch.equal(valid(ctx, one, 1), valid(ctx, outh[nb:2 * nb], 1)), kind
    for kind, _, _, _ in cases:
        assert 0 < rel(outs[(12, kind)], outs[(18, kind)]) < bound
    with pytest.raises(P.TMError):  # 18, 12 and 8 (FP64 kernels) only
        ctx.set_link_format(7)


@pytest.mark.parametrize("t_bc", [-1, 1])
def test_link_format_12_parameters_fp64(t_bc):
    """FP64 kernels with 12-parameter FP64 links (the plain solver and the
    reliable updates): every operator kind within 1e-13 of the oracle for
    both time boundary conditions, and within 1e-14 of the 18-parameter
    result (the rebuilt third row differs only by rounding)."""
    L, kappa, eps = (4, 4, 2, 6), 0.124, 0.0123
    ctx, U = make_ctx(L, kappa, eps, 19, t_bc=t_bc)
    nrhs = 2
    v = S.random_spinor(L, 9, nrhs)
    prec = P.TM_F64
    e, o = half_buf(ctx, prec, nrhs), half_buf(ctx, prec, nrhs)
    ctx.pack(e, o, cuda(v), nrhs, prec)
    ve = [mask_parity(L, v[r], 0) for r in range(nrhs)]
    cases = [
        (P.TM_HOP_OE, e, 1, lambda r: mask_parity(L, O.hop(L, kappa, t_bc, U, ve[r]), 1)),
        (P.TM_SCHUR, e, 0, lambda r: O.schur(L, kappa, eps, t_bc, U, ve[r])),
        (P.TM_SCHUR_DAG, e, 0, lambda r: O.schur(L, kappa, eps, t_bc, U, ve[r], adj=True)),
        (P.TM_NORMAL, e, 0, lambda r: O.schur(L, kappa, eps, t_bc, U,
                                              O.schur(L, kappa, eps, t_bc, U, ve[r]), adj=True)),
    ]
    outs = {}
    for fmt in (12, 18):
        ctx.set_link_format(fmt)
        for kind, inp, par, ref in cases:
            outh = half_buf(ctx, prec, nrhs)
            ctx.dslash(outh, inp, nrhs, kind, 1, prec, P.TM_F64)
            full = torch.zeros((nrhs,) + v.shape[1:], dtype=torch.complex128, device=DEV)
            if par == 0:
                ctx.unpack(full, outh, half_buf(ctx, prec, nrhs), nrhs, prec)
            else:
                ctx.unpack(full, half_buf(ctx, prec, nrhs), outh, nrhs, prec)
            outs[(fmt, kind)] = host(full)
            for r in range(nrhs):
                assert rel(outs[(fmt, kind)][r], ref(r)) < 1e-13, (fmt, kind, r)
    for kind, _, _, _ in cases:
        assert rel(outs[(12, kind)], outs[(18, kind)]) < 1e-14


def test_dslash_rejects_bad_arguments():
    L = (4, 4, 4, 8)
    ctx, _ = make_ctx(L, 0.124, 0.01, 5)
    a, b = half_buf(ctx, P.TM_F64, 1), half_buf(ctx, P.TM_F64, 1)
    for args in ((a, b, 0, P.TM_SCHUR, 1, P.TM_F64, P.TM_F64),
                 (a, b, 1, 99, 1, P.TM_F64, P.TM_F64),
                 (a, b, 1, P.TM_SCHUR, 0, P.TM_F64, P.TM_F64),
                 (a, b, 1, P.TM_SCHUR, 1, P.TM_F16, P.TM_F64),
                 (a, a, 1, P.TM_SCHUR, 1, P.TM_F64, P.TM_F64)):
        st = P.tm_dslash(ctx.h, P.binding._ptr(args[0]), P.binding._ptr(args[1]), *args[2:], None)
        assert st == P.TM_ERR_ARG


# ---------------------------------------------------------------- solvers

def oracle_residual(L, kappa, eps, U, x, b):
    return np.linalg.norm(b - O.apply_M(L, kappa, eps, -1, U, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("mu_sign", [1, -1])
def test_solve_fp64(mu_sign):
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    nrhs = 2
    b = S.random_spinor(L, 21, nrhs)
    x = torch.zeros_like(cuda(b))
    st, stats = ctx.solve(x, cuda(b), nrhs, P.solve_params(tol=1e-10, mu_sign=mu_sign))
    xs = host(x)
    for r in range(nrhs):
        res = oracle_residual(L, kappa, mu_sign * eps, U, xs[r], b[r])
        assert res <= 1e-10, res
        assert abs(stats[r].true_rel_res - res) <= 1e-3 * res + 1e-15
        assert stats[r].converged == 1 and stats[r].iters > 0


@pytest.mark.parametrize("prec,fmt", [(P.TM_F32, 18), (P.TM_F16, 18), (P.TM_BF16, 18),
                                      (P.TM_F16, 12), (P.TM_BF16, 12)])
def test_solve_mixed_reliable_updates(prec, fmt):
    L, kappa, eps = (8, 8, 8, 8), 0.124, 0.005
    ctx, U = make_ctx(L, kappa, eps, 31, 0.3)
    ctx.set_link_format(fmt)
    nrhs = 2
    b = S.random_spinor(L, 22, nrhs)
    x = torch.zeros_like(cuda(b))
    st, stats = ctx.solve(x, cuda(b), nrhs, P.solve_params(
        tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=prec))
    xs = host(x)
    for r in range(nrhs):
        res = oracle_residual(L, kappa, eps, U, xs[r], b[r])
        assert res <= 1e-9, (prec, res)
        assert stats[r].n_reliable >= 1


@pytest.mark.parametrize("prec", [P.TM_F32, P.TM_F16])
def test_solve_truncated_low_precision(prec):
    L, kappa, eps = (8, 8, 8, 8), 0.124, 0.005
    ctx, U = make_ctx(L, kappa, eps, 32, 0.3)
    b = S.random_spinor(L, 23, 1)
    x = torch.zeros_like(cuda(b))
    st, stats = ctx.solve(x, cuda(b), 1, P.solve_params(
        tol=1e-2, solver=P.TM_CG_LOW, inner_prec=prec, check_every=1))
    res = oracle_residual(L, kappa, eps, U, host(x)[0], b[0])
    assert abs(stats[0].true_rel_res - res) <= 1e-6 * res
    assert stats[0].iter_rel_res <= 1e-2
    assert res < 3e-2


@pytest.mark.parametrize("solver", [P.TM_CG_F64, P.TM_CG_MIXED])
def test_solve_links_off_su3(solver):
    """Links perturbed off SU(3) by ~1e-7 (as a field stored in single
    precision would be): the FP64 kernels fall back to all 18 parameters and
    the reported true residual is the oracle's residual for that very field;
    the solve converges to it."""
    L, kappa, eps = (4, 4, 4, 8), 0.124, 0.01
    U = S.gauge_links(L, 0.3, 34)
    rng = np.random.default_rng(35)
    U = U + 1e-7 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    ctx = P.Context(L, kappa, eps)
    ctx.set_gauge(cuda(U))
    b = S.random_spinor(L, 36, 1)
    x = torch.zeros_like(cuda(b))
    st, stats = ctx.solve(x, cuda(b), 1, P.solve_params(tol=1e-10, solver=solver,
                                                        inner_prec=P.TM_F16))
    res = oracle_residual(L, kappa, eps, U, host(x)[0], b[0])
    assert res <= 1e-10 and stats[0].converged == 1
    assert abs(stats[0].true_rel_res - res) <= 1e-3 * res
    # the FP64 Schur operator itself is the oracle's for the perturbed field
    v = S.random_spinor(L, 37, 1)
    e, o = half_buf(ctx, P.TM_F64, 1), half_buf(ctx, P.TM_F64, 1)
    ctx.pack(e, o, cuda(v), 1, P.TM_F64)
    out = half_buf(ctx, P.TM_F64, 1)
    ctx.dslash(out, e, 1, P.TM_SCHUR, 1, P.TM_F64)
    full = torch.zeros_like(cuda(v))
    ctx.unpack(full, out, half_buf(ctx, P.TM_F64, 1), 1, P.TM_F64)
    ref = O.schur(L, kappa, eps, -1, U, v[0])
    par = O.site_parity(L)
    assert rel(host(full)[0][par == 0], ref[par == 0]) < 1e-13


def test_solve_stats_count_work():
    """tm_solve_stats.bytes / flops: per right-hand side, at least the four
    half-Dslash launches of every CG iteration (1392 flops per site and RHS
    each, input + output + links) and within a small factor of that."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    vh = int(np.prod(L)) // 2
    for nrhs in (1, 3):
        b = S.random_spinor(L, 38, nrhs)
        x = torch.zeros_like(cuda(b))
        _, stats = ctx.solve(x, cuda(b), nrhs, P.solve_params(tol=1e-10))
        it = stats[0].iters
        lo_f = 4 * it * vh * 1392
        lo_b = 4 * it * vh * (2 * 192 + 8 * 6 * 16 / nrhs)
        assert lo_f <= stats[0].flops <= 2.0 * lo_f, (stats[0].flops, lo_f)
        assert lo_b <= stats[0].bytes <= 3.0 * lo_b, (stats[0].bytes, lo_b)


def test_solve_failure_paths():
    L = (4, 4, 4, 8)
    ctx, U = make_ctx(L, 0.124, 0.01, 33)
    b = S.random_spinor(L, 24, 1)
    x = torch.zeros_like(cuda(b))
    st, stats = ctx.solve(x, cuda(b), 1, P.solve_params(tol=1e-12, maxiter=2), allow_noconv=True)
    assert st == P.TM_ERR_NOCONV and stats[0].iters == 2 and stats[0].converged == 0
    bn = b.copy()
    bn[0, 3, 1, 2] = np.nan
    with pytest.raises(P.TMError) as ei:
        ctx.solve(x, cuda(bn), 1, P.solve_params(tol=1e-9))
    assert ei.value.status == P.TM_ERR_NAN
    with pytest.raises(P.TMError) as ei:
        ctx.solve(x, cuda(b), 1, P.solve_params(tol=-1.0))
    assert ei.value.status == P.TM_ERR_ARG
    with pytest.raises(P.TMError) as ei:
        ctx.solve(x, cuda(b), 1, P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED,
                                                inner_prec=P.TM_F64))
    assert ei.value.status == P.TM_ERR_ARG


# ---------------------------------------------------------------- contraction and loops

def test_contract_matches_oracle():
    L = (4, 4, 4, 8)
    eps = 0.0123
    ctx, _ = make_ctx(L, 0.124, eps, 41)
    nrhs = 3
    eta = S.random_spinor(L, 42, nrhs)
    s = S.random_spinor(L, 43, nrhs)
    for mu_sign in (1, -1):
        got = ctx.contract(cuda(eta), cuda(s), nrhs, P.TM_EST_STD | P.TM_EST_ONE_END, mu_sign)
        ref_std = sum(O.contract_std(L, eta[r], s[r]) for r in range(nrhs))
        ref_1e = sum(O.contract_oneend(L, mu_sign * eps, s[r]) for r in range(nrhs))
        assert rel(got[0], ref_std) < 1e-13
        assert rel(got[1], ref_1e) < 1e-13


EST_ALL = P.TM_EST_STD | P.TM_EST_ONE_END | P.TM_EST_HPE
EST_ORDER = (O.EST_STD, O.EST_ONE_END, O.EST_HPE)


def loop_params(seed, n_hp, n_lp, est, dilution=P.TM_DIL_NONE, hp_tol=1e-11, lp=None,
                mu_sign=1):
    p = P.tm_loop_params()
    p.seed, p.n_hp, p.n_lp, p.estimators, p.dilution, p.mu_sign = seed, n_hp, n_lp, est, \
        dilution, mu_sign
    p.hp = P.solve_params(tol=hp_tol, solver=P.TM_CG_F64)
    p.lp = lp if lp is not None else P.solve_params(tol=1e-2, solver=P.TM_CG_LOW,
                                                    inner_prec=P.TM_F16, check_every=1)
    return p


@pytest.mark.parametrize("dilution", [P.TM_DIL_NONE, P.TM_DIL_SPIN_COLOUR])
@pytest.mark.parametrize("mu_sign", [1, -1])
def test_loops_plain_vs_oracle(dilution, mu_sign):
    """c1 workload: loops at every time slice for the 16 Gamma, all three
    estimators, within 1e-8 normwise of the oracle (both solve tightly)."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    n = 2 if dilution == P.TM_DIL_NONE else 1
    loops, pn, stats, st = ctx.loops(loop_params(201, n, 0, EST_ALL, dilution, mu_sign=mu_sign),
                                     per_noise=True)
    ref, ref_pn = O.loops(L, kappa, mu_sign * eps, -1, U, 201, n, 1e-13, EST_ALL,
                          dilution=dilution == P.TM_DIL_SPIN_COLOUR)
    for k, e in enumerate(EST_ORDER):
        assert rel(loops[k], ref[e]) < 1e-8, (e, rel(loops[k], ref[e]))
        for r in range(n):
            assert rel(pn[r, 0, k], ref_pn[r][e]) < 1e-8
    assert stats.max_res_hp <= 1e-11 and stats.n_solves_hp == n * (12 if dilution else 1)


def test_loops_tsm_combination():
    """TSM: the combined estimate equals eq. estiTSM applied (by the oracle) to
    the library's own per-noise loops; the HP loops match the oracle's; the LP
    solves meet their truncation criterion."""
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    n_hp, n_lp = 2, 3
    loops, pn, stats, st = ctx.loops(loop_params(201, n_hp, n_lp, EST_ALL), per_noise=True)
    for k, e in enumerate(EST_ORDER):
        comb = O.tsm_combine([pn[r, 0, k] for r in range(n_hp)],
                             [pn[r, 1, k] for r in range(n_hp)],
                             [pn[r, 1, k] for r in range(n_hp, n_hp + n_lp)])
        if e == O.EST_HPE:
            comb = comb + O.hpe_exact(L, kappa, eps, -1, U)
        assert rel(loops[k], comb) < 1e-13
    _, ref_pn = O.loops(L, kappa, eps, -1, U, 201, n_hp, 1e-13, EST_ALL)
    for r in range(n_hp):
        for k, e in enumerate(EST_ORDER):
            assert rel(pn[r, 0, k], ref_pn[r][e]) < 1e-8
    assert stats.n_solves_lp == n_hp + n_lp and stats.max_res_lp < 3e-2
    # LP loops are contractions of valid LP solutions: close to HP at the 1e-2 level
    for r in range(n_hp):
        assert rel(pn[r, 1, 0], pn[r, 0, 0]) < 0.2


def test_loops_lp_equal_hp_is_plain():
    cfg = S.CONFIGS["c1"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    ctx, U = make_ctx(L, kappa, eps, cfg["seed"], cfg["eps_links"])
    lp = P.solve_params(tol=1e-11, solver=P.TM_CG_F64)
    loops, pn, stats, st = ctx.loops(loop_params(201, 1, 2, P.TM_EST_STD, lp=lp), per_noise=True)
    plain = (pn[1, 1, 0] + pn[2, 1, 0]) / 2
    assert rel(loops[0], plain) < 1e-9


def test_loops_argument_checks():
    ctx, _ = make_ctx((2, 2, 2, 2), 0.124, 0.01, 5)
    with pytest.raises(P.TMError) as ei:   # HPE needs every extent >= 4
        ctx.loops(loop_params(1, 1, 0, P.TM_EST_HPE))
    assert ei.value.status == P.TM_ERR_ARG
    with pytest.raises(P.TMError):
        ctx.loops(loop_params(1, 0, 0, P.TM_EST_STD))


# ---------------------------------------------------------------- full-size sampled

@pytest.fixture(scope="module")
def c3():
    cfg = S.CONFIGS["c3"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    U = S.gauge_links(L, cfg["eps_links"], cfg["seed"])
    ctx = P.Context(L, kappa, eps)
    ctx.set_gauge(cuda(U))
    yield dict(L=L, kappa=kappa, eps=eps, U=U, ctx=ctx)
    ctx.close()


def boundary_sample(L, even, rng, n):
    """n even sites: random ones plus sites on every face of the lattice
    (t = 0 and t = Lt - 1, where the hops cross the time boundary, and x, y,
    z = 0 and L - 1), so that every wrap-around of both hops is exercised."""
    V = int(np.prod(L))
    s = np.arange(V)
    c = [s % L[0], (s // L[0]) % L[1], (s // (L[0] * L[1])) % L[2], s // (L[0] * L[1] * L[2])]
    par_even = np.zeros(V, dtype=bool)
    par_even[even] = True
    faces = []
    for mu in (3, 0, 1, 2):
        for v in (0, L[mu] - 1):
            cand = np.where(par_even & (c[mu] == v))[0]
            faces.extend(rng.choice(cand, 4, replace=False))
    rest = np.setdiff1d(even, faces)
    pick = np.concatenate([faces, rng.choice(rest, n - len(faces), replace=False)])
    pick = np.sort(pick)
    t = pick // (L[0] * L[1] * L[2])
    assert (t == 0).any() and (t == L[3] - 1).any()
    return pick


def test_c3_schur_sampled_sites(c3):
    """32^3 x 64: the FP64 1-RHS and the 12-RHS FP16-storage Schur operator
    (the benchmarked launch) at 96 sampled even sites against the oracle
    evaluated site by site; the 12-RHS call equals 12 single calls bit for bit."""
    L, kappa, eps, U, ctx = c3["L"], c3["kappa"], c3["eps"], c3["U"], c3["ctx"]
    V = int(np.prod(L))
    rng = np.random.default_rng(5)
    par = O.site_parity(L)
    even = np.where(par == 0)[0]
    sites = boundary_sample(L, even, rng, 96)
    nrhs = 12
    v = (rng.standard_normal((nrhs, V, 4, 3)) + 1j * rng.standard_normal((nrhs, V, 4, 3)))
    dv = cuda(v)
    for prec, bound, n in ((P.TM_F64, 1e-13, 1), (P.TM_F16, 4e-3, nrhs)):
        e, o = half_buf(ctx, prec, n), half_buf(ctx, prec, n)
        ctx.pack(e, o, dv[:n], n, prec)
        outh = half_buf(ctx, prec, n)
        ctx.dslash(outh, e, n, P.TM_SCHUR, 1, prec)
        full = torch.zeros((n, V, 4, 3), dtype=torch.complex128, device=DEV)
        ctx.unpack(full, outh, half_buf(ctx, prec, n), n, prec)
        got = host(full)
        for r in range(0, n, 5):
            ref = O.schur_at(L, kappa, eps, -1, U, v[r], sites)
            err = np.abs(got[r][sites] - ref).max() / np.abs(ref).max()
            assert err < bound, (prec, r, err)
        if n > 1:
            nb = ctx.half_numel(prec, 1)
            one = half_buf(ctx, prec, 1)
            for r in (0, 7, 11):
                ctx.dslash(one, e[r * nb:(r + 1) * nb], 1, P.TM_SCHUR, 1, prec)
                assert torch.equal(valid(ctx, one, 1), valid(ctx, outh[r * nb:(r + 1) * nb], 1))
        del e, o, outh, full


def test_c3_mixed_solve_true_residual(c3):
    """32^3 x 64, one Z4 source solved with FP16-storage mixed CG to 1e-9; the
    oracle recomputes |eta - M x| / |eta| in FP64 on the host."""
    L, kappa, eps, U, ctx = c3["L"], c3["kappa"], c3["eps"], c3["U"], c3["ctx"]
    eta = O.noise_z4(L, 203, 0)
    x = torch.zeros((1,) + eta.shape, dtype=torch.complex128, device=DEV)
    st, stats = ctx.solve(x, cuda(eta[None]), 1, P.solve_params(
        tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16))
    res = oracle_residual(L, kappa, eps, U, host(x)[0], eta)
    assert res <= 1e-9 and abs(stats[0].true_rel_res - res) <= 1e-3 * res
