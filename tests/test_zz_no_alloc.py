"""tm_dslash_noalloc against tm_dslash: the same operator from the device
scratch array instead of context workspace.

Both entry points run the same kernels, so outputs are compared bit for bit
(on the valid half-sites; the pad sites of the half layout are unspecified),
on two calls in a row with the second on fewer right-hand sides (the scratch
keeps the first call's contents), for the kinds with intermediate fields
(Schur complement, its adjoint, the normal operator, the full operator) and
one without.  Requests beyond the scratch size and calls whose link copy was
never built are refused before any launch.
"""
import numpy as np
import pytest

import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1309_2256_amd as P  # noqa: E402

DEV = "cuda:0"
L = (16, 16, 16, 32)
KAPPA, EPS = 0.124, 0.0028


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(L, KAPPA, EPS)
    c.set_gauge(cuda(S.gauge_links(L, 0.2, 102)))
    yield c
    c.close()


def valid_sites(c, t, nrhs):
    """The valid half-sites of every plane of a half field given as bytes
    (the hs - vh pad sites at the end of each plane are unspecified)."""
    return t.view(nrhs, 12, c.hs, -1)[:, :, :c.vh]


def half_input(c, prec, nrhs, seed):
    full = cuda(S.random_spinor(L, seed, nrhs))
    e = torch.zeros(c.half_numel(prec, nrhs), dtype=torch.uint8, device=DEV)
    o = torch.zeros_like(e)
    c.pack(e, o, full, nrhs, prec)
    return e


HALF_KINDS = [P.TM_SCHUR, P.TM_SCHUR_DAG, P.TM_NORMAL, P.TM_RINV_HOP_OE]


@pytest.mark.parametrize("prec", [P.TM_F64, P.TM_F32, P.TM_F16])
@pytest.mark.parametrize("kind", HALF_KINDS)
def test_half_kinds_match_tm_dslash(ctx, kind, prec):
    # the normal operator's two FP64 fields of 3 right-hand sides exceed the scratch
    first = 2 if prec == P.TM_F64 else 3
    for call, (nrhs, mu) in enumerate([(first, 1), (1, -1)]):  # second call smaller
        inp = half_input(ctx, prec, nrhs, 300 + call)
        ref = torch.empty_like(inp)
        out = torch.full_like(inp, 0x7f)
        ctx.dslash(ref, inp, nrhs, kind, mu, prec)
        ctx.dslash_noalloc(out, inp, nrhs, kind, mu, prec)
        torch.cuda.synchronize()
        assert torch.equal(valid_sites(ctx, out, nrhs), valid_sites(ctx, ref, nrhs)), (kind, prec, nrhs)


def test_full_kinds_match_tm_dslash(ctx):
    # one FP64 right-hand side of the full operator takes 4 x 12.6 MB of scratch
    for call, kind in enumerate([P.TM_FULL, P.TM_FULL_DAG]):
        inp = cuda(S.random_spinor(L, 400 + call, 1))
        ref = torch.empty_like(inp)
        out = torch.full_like(inp, float("nan"))
        ctx.dslash(ref, inp, 1, kind, 1, P.TM_F64)
        ctx.dslash_noalloc(out, inp, 1, kind, 1, P.TM_F64)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), kind


def test_oversize_request_is_refused(ctx):
    nrhs = 3  # FP64 full operator: 4 x 3 x 12.6 MB > 64 MiB
    inp = cuda(S.random_spinor(L, 500, nrhs))
    out = torch.zeros_like(inp)
    with pytest.raises(P.TMError) as e:
        ctx.dslash_noalloc(out, inp, nrhs, P.TM_FULL, 1, P.TM_F64)
    assert e.value.status == P.TM_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert not out.any()  # nothing was launched


def test_missing_link_copy_is_refused():
    c = P.Context((8, 8, 8, 16), KAPPA, EPS)
    try:
        c.set_gauge(cuda(S.gauge_links((8, 8, 8, 16), 0.3, 7)))
        inp = half_input(c, P.TM_F16, 1, 600)
        out = torch.zeros_like(inp)
        with pytest.raises(P.TMError) as e:
            c.dslash_noalloc(out, inp, 1, P.TM_RINV_HOP_OE, 1, P.TM_F16)
        assert e.value.status == P.TM_ERR_UNSUPPORTED
        ref = torch.empty_like(inp)
        c.dslash(ref, inp, 1, P.TM_RINV_HOP_OE, 1, P.TM_F16)  # builds the copy
        c.dslash_noalloc(out, inp, 1, P.TM_RINV_HOP_OE, 1, P.TM_F16)
        torch.cuda.synchronize()
        assert torch.equal(valid_sites(c, out, 1), valid_sites(c, ref, 1))
    finally:
        c.close()
