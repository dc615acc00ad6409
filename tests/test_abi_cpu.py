"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/tm.h, and validates arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(tm_\w+)\s*\(", src,
                                 flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tm_create", "tm_destroy", "tm_last_error", "tm_set_gauge", "tm_dslash",
              "tm_solve", "tm_loops", "tm_pack", "tm_unpack", "tm_noise", "tm_contract"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    import paper_1309_2256_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(P.EXPORTED) == set(declared_functions())


def test_binding_struct_sizes_match_header():
    """ctypes mirrors of the parameter structs have the C layout sizes."""
    import paper_1309_2256_amd as P
    assert ctypes.sizeof(P.tm_lattice) == 4 * 4 + 8 + 8 + 4 + 4  # padded to 8
    assert ctypes.sizeof(P.tm_solve_params) == 8 + 4 + 4 + 4 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(P.tm_solve_stats) == 4 * 4 + 5 * 8
    assert ctypes.sizeof(P.tm_loop_params) == 8 + 8 * 4 + 2 * ctypes.sizeof(P.tm_solve_params)


@pytest.mark.parametrize("L", [(3, 4, 4, 4), (4, 4, 4, 5), (0, 4, 4, 4), (4, 4, -2, 4)])
def test_create_rejects_bad_lattices(L):
    import paper_1309_2256_amd as P
    lat = P.tm_lattice((ctypes.c_int * 4)(*L), 0.124, 0.01, -1)
    h = ctypes.c_void_p()
    assert P.tm_create(ctypes.byref(h), ctypes.byref(lat), 0) == P.TM_ERR_ARG
    assert not h.value


@pytest.mark.parametrize("L,ok", [((64, 64, 64, 128), False), ((48, 48, 48, 96), True)])
def test_create_guards_32bit_field_offsets(L, ok):
    """A geometry whose FP64 half field of one right-hand side exceeds 2^31 - 1
    bytes is refused before any device call (the kernels use 32-bit byte
    offsets); one that fits passes the guard (and then needs a device)."""
    import paper_1309_2256_amd as P
    lat = P.tm_lattice((ctypes.c_int * 4)(*L), 0.124, 0.01, -1)
    h = ctypes.c_void_p()
    st = P.tm_create(ctypes.byref(h), ctypes.byref(lat), 0)
    if ok:
        assert st != P.TM_ERR_UNSUPPORTED
        if st == P.TM_OK:
            P.tm_destroy(h)
    else:
        assert st == P.TM_ERR_UNSUPPORTED and not h.value


def test_create_rejects_bad_bc_and_nulls():
    import paper_1309_2256_amd as P
    lat = P.tm_lattice((ctypes.c_int * 4)(4, 4, 4, 4), 0.124, 0.01, 0)
    h = ctypes.c_void_p()
    assert P.tm_create(ctypes.byref(h), ctypes.byref(lat), 0) == P.TM_ERR_ARG
    assert P.tm_create(None, ctypes.byref(lat), 0) == P.TM_ERR_ARG
    assert P.tm_create(ctypes.byref(h), None, 0) == P.TM_ERR_ARG
    # calls on a null context fail cleanly
    assert P.tm_dslash(None, None, None, 1, 0, 1, 0, 0, None) == P.TM_ERR_ARG
    assert P.tm_last_error(None) == b"null context"
    assert P.tm_half_stride(None) == 0
    P.tm_destroy(None)


def test_ptc_structs_and_null_context():
    import paper_1309_2256_amd as P
    assert ctypes.sizeof(P.tm_ptc_train_params) == 4 + 4 + 4 * 8 + 8 + 4 + 4
    assert ctypes.sizeof(P.tm_ptc_train_stats) == 4 + 4 + 3 * 8
    assert P.tm_ptc_set_weights(None, 12, None, None) == P.TM_ERR_ARG
    assert P.tm_ptc_init_hopping(None, 12, 1, 0, 0.0) == P.TM_ERR_ARG
    assert P.tm_ptc_apply(None, None, None, 1, None) == P.TM_ERR_ARG
    assert P.tm_ptc_pairs_reserve(None, 1, P.TM_F32) == P.TM_ERR_ARG
    assert P.tm_ptc_train(None, None, None, None, None) == P.TM_ERR_ARG


@pytest.mark.parametrize("p2max", [0, 1, 2, 3, 4, 9, 12])
def test_momentum_list_matches_oracle(p2max):
    """tm_momenta is host logic: same vectors, same order as the oracle's
    enumeration, and argument errors come back as TM_ERR_ARG."""
    import numpy as np
    import oracle as O
    import paper_1309_2256_amd as P
    assert np.array_equal(P.momenta(p2max), O.momenta(p2max))
    n = ctypes.c_int(0)
    assert P.tm_momenta(-1, ctypes.byref(n), None) == P.TM_ERR_ARG
    assert P.tm_momenta(p2max, None, None) == P.TM_ERR_ARG
    small = (ctypes.c_int * 3)()
    n.value = 0
    if p2max > 0:
        assert P.tm_momenta(p2max, ctypes.byref(n), small) == P.TM_ERR_ARG


def test_momentum_calls_on_null_context():
    import paper_1309_2256_amd as P
    assert P.tm_contract_momentum(None, None, None, 1, 1, 1, 0, 0, None, None) == P.TM_ERR_ARG
    assert P.tm_loops_momentum(None, None, 0, None, None, None, None) == P.TM_ERR_ARG


def test_link_format_and_loop_entry_points_on_null_context():
    import paper_1309_2256_amd as P
    assert P.tm_set_link_format(None, 12) == P.TM_ERR_ARG
    assert P.tm_loops(None, None, None, None, None, None) == P.TM_ERR_ARG
    assert P.tm_loops_momentum(None, None, 0, None, None, None, None) == P.TM_ERR_ARG
    assert ctypes.sizeof(P.tm_loop_params) == 8 + 8 * 4 + 2 * ctypes.sizeof(P.tm_solve_params)
    p = P.tm_loop_params()
    assert p.derivative == 0 and p.t_period == 0     # zero-initialised: local, volume sources
