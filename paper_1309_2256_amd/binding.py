"""ctypes binding of the C-ABI in include/tm.h (argument marshalling only).

Every function here forwards to libtm.so, the gfx950 HIP library built from
csrc/; there is no fallback path: importing this module raises if the
library is missing.  Device buffers are passed as torch tensors (their
data_ptr()) and the work is enqueued on torch's current HIP stream unless a
stream handle is given.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libtm.so is not built (run paper_1309_2256_amd/build.py or "
                      "__graft_entry__.build()); there is no non-HIP fallback")

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants (tm.h)
TM_OK, TM_ERR_ARG, TM_ERR_HIP, TM_ERR_OOM, TM_ERR_NOCONV, TM_ERR_NAN, TM_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
TM_F64, TM_F32, TM_F16, TM_BF16 = 0, 1, 2, 3
(TM_HOP_EO, TM_HOP_OE, TM_RINV_HOP_OE, TM_SCHUR, TM_SCHUR_DAG, TM_NORMAL, TM_FULL, TM_FULL_DAG,
 TM_RINV_HOP_EO) = range(9)
TM_CG_F64, TM_CG_MIXED, TM_CG_LOW, TM_FGMRES, TM_FGMRES_PTC = 0, 1, 2, 3, 4
TM_EST_STD, TM_EST_ONE_END, TM_EST_HPE, TM_EST_GEN_ONE_END = 1, 2, 4, 8
TM_DIL_NONE, TM_DIL_SPIN_COLOUR = 0, 1
TM_PTC_LOSS_ERROR, TM_PTC_LOSS_RESIDUAL = 0, 1

STATUS_NAMES = {0: "TM_OK", -1: "TM_ERR_ARG", -2: "TM_ERR_HIP", -3: "TM_ERR_OOM",
                -4: "TM_ERR_NOCONV", -5: "TM_ERR_NAN", -6: "TM_ERR_UNSUPPORTED"}
PREC_BYTES = {TM_F64: 16, TM_F32: 8, TM_F16: 4, TM_BF16: 4}


class tm_lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("kappa", ctypes.c_double),
                ("two_kappa_mu", ctypes.c_double), ("t_bc", ctypes.c_int)]


class tm_solve_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("solver", ctypes.c_int),
                ("inner_prec", ctypes.c_int), ("delta", ctypes.c_double),
                ("mu_sign", ctypes.c_int), ("check_every", ctypes.c_int)]


class tm_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("n_reliable", ctypes.c_int), ("converged", ctypes.c_int),
                ("fallback", ctypes.c_int), ("true_rel_res", ctypes.c_double),
                ("iter_rel_res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class tm_loop_params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_hp", ctypes.c_int), ("n_lp", ctypes.c_int),
                ("noise_offset", ctypes.c_int), ("dilution", ctypes.c_int),
                ("estimators", ctypes.c_int), ("mu_sign", ctypes.c_int), ("derivative", ctypes.c_int),
                ("t_period", ctypes.c_int),
                ("hp", tm_solve_params), ("lp", tm_solve_params)]


class tm_loop_stats(ctypes.Structure):
    _fields_ = [("n_solves_hp", ctypes.c_int), ("n_solves_lp", ctypes.c_int),
                ("iters_hp", ctypes.c_int), ("iters_lp", ctypes.c_int),
                ("max_res_hp", ctypes.c_double), ("max_res_lp", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class tm_ptc_train_params(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("adam_eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("loss", ctypes.c_int), ("mu_sign", ctypes.c_int)]


class tm_ptc_train_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("reserved", ctypes.c_int), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("seconds", ctypes.c_double)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "tm_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(tm_lattice), ctypes.c_int]),
    "tm_destroy": (None, [_vp]),
    "tm_last_error": (ctypes.c_char_p, [_vp]),
    "tm_half_stride": (ctypes.c_int, [_vp]),
    "tm_set_gauge": (ctypes.c_int, [_vp, _vp, _vp]),
    "tm_dslash": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, _vp]),
    "tm_dslash_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, _vp]),
    "tm_set_link_format": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tm_set_half_spinor_links": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tm_pack": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _dp, _vp]),
    "tm_unpack": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "tm_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(tm_solve_params),
                                ctypes.POINTER(tm_solve_stats), _vp]),
    "tm_loops": (ctypes.c_int, [_vp, ctypes.POINTER(tm_loop_params), _dp, _dp,
                                ctypes.POINTER(tm_loop_stats), _vp]),
    "tm_noise": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, ctypes.c_long, ctypes.c_int, _vp]),
    "tm_contract": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                   _vp]),
    "tm_momenta": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]),
    "tm_contract_momentum": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, _dp, _vp]),
    "tm_loops_momentum": (ctypes.c_int, [_vp, ctypes.POINTER(tm_loop_params), ctypes.c_int, _dp, _dp,
                                         ctypes.POINTER(tm_loop_stats), _vp]),
    "tm_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int]),
    "tm_batch_destroy": (None, [_vp]),
    "tm_batch_last_error": (ctypes.c_char_p, [_vp]),
    "tm_batch_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(tm_solve_params),
                                      ctypes.POINTER(ctypes.POINTER(tm_solve_stats)), _vp]),
    "tm_batch_loops": (ctypes.c_int, [_vp, ctypes.POINTER(tm_loop_params), ctypes.POINTER(_dp),
                                      ctypes.POINTER(tm_loop_stats), _vp]),
    "tm_ptc_set_weights": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "tm_ptc_get_weights": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "tm_ptc_set_arith": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tm_ptc_init_hopping": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                           ctypes.c_double]),
    "tm_ptc_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "tm_ptc_loss_grad": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _dp, _dp,
                                        _dp, _vp]),
    "tm_ptc_pairs_reserve": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "tm_ptc_pairs_add": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "tm_ptc_pairs_from_solve": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(tm_solve_params),
                                               ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int), _vp]),
    "tm_ptc_train": (ctypes.c_int, [_vp, ctypes.POINTER(tm_ptc_train_params),
                                    ctypes.POINTER(tm_ptc_train_stats), _dp, _vp]),
}
EXPORTED = tuple(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class TMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def solve_params(tol=1e-9, maxiter=100000, solver=TM_CG_F64, inner_prec=TM_F32, delta=0.1,
                 mu_sign=1, check_every=8):
    return tm_solve_params(tol, maxiter, solver, inner_prec, delta, mu_sign, check_every)


class Context:
    """One library context (lattice + gauge field) on one HIP device."""

    def __init__(self, L, kappa, two_kappa_mu, t_bc=-1, device=0):
        self.L = tuple(int(v) for v in L)
        self.V = int(np.prod(self.L))
        self.vh = self.V // 2
        lat = tm_lattice((ctypes.c_int * 4)(*self.L), kappa, two_kappa_mu, t_bc)
        h = ctypes.c_void_p()
        st = tm_create(ctypes.byref(h), ctypes.byref(lat), device)
        if st != TM_OK:
            raise TMError(st, "tm_create failed")
        self.h = h
        # plane stride of the half-lattice layout (>= vh, padded)
        self.hs = int(tm_half_stride(h))

    def close(self):
        if getattr(self, "h", None):
            tm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != TM_OK and st not in allow:
            raise TMError(st, tm_last_error(self.h).decode())
        return st

    def half_numel(self, prec, nrhs=1):
        """Bytes of a half-lattice field of nrhs right-hand sides ([nrhs][12][hs],
        the last hs - vh sites of every plane are padding)."""
        return PREC_BYTES[prec] * 12 * self.hs * nrhs

    def set_gauge(self, U, stream=None):
        self._check(tm_set_gauge(self.h, _ptr(U), _stream(stream)))

    def set_half_spinor_links(self, link_prec):
        """Links of the FP16/BF16-spinor solver kernels: TM_F16 (binary16) or TM_F32."""
        self._check(tm_set_half_spinor_links(self.h, link_prec))

    def set_link_format(self, params):
        """Binary16 links of the FP16/BF16-spinor kernels: 18 or 12 parameters."""
        self._check(tm_set_link_format(self.h, params))

    def dslash(self, out, inp, nrhs, kind, mu_sign=1, spinor_prec=TM_F64, link_prec=None,
               stream=None):
        if link_prec is None:  # the solvers' choice for each spinor precision
            link_prec = {TM_F64: TM_F64, TM_F32: TM_F32}.get(spinor_prec, TM_F16)
        self._check(tm_dslash(self.h, _ptr(out), _ptr(inp), nrhs, kind, mu_sign, spinor_prec,
                              link_prec, _stream(stream)))

    def dslash_noalloc(self, out, inp, nrhs, kind, mu_sign=1, spinor_prec=TM_F64, link_prec=None,
                       stream=None):
        if link_prec is None:
            link_prec = {TM_F64: TM_F64, TM_F32: TM_F32}.get(spinor_prec, TM_F16)
        self._check(tm_dslash_noalloc(self.h, _ptr(out), _ptr(inp), nrhs, kind, mu_sign,
                                      spinor_prec, link_prec, _stream(stream)))

    def pack(self, even, odd, full, nrhs, prec, scale=None, stream=None):
        sc = None
        if scale is not None:
            arr = (ctypes.c_double * nrhs)(*scale)
            sc = ctypes.cast(arr, _dp)
        self._check(tm_pack(self.h, _ptr(even), _ptr(odd), _ptr(full), nrhs, prec, sc,
                            _stream(stream)))

    def unpack(self, full, even, odd, nrhs, prec, stream=None):
        self._check(tm_unpack(self.h, _ptr(full), _ptr(even), _ptr(odd), nrhs, prec,
                              _stream(stream)))

    def solve(self, x, b, nrhs, params, stream=None, allow_noconv=False):
        stats = (tm_solve_stats * nrhs)()
        st = tm_solve(self.h, _ptr(x), _ptr(b), nrhs, ctypes.byref(params), stats,
                      _stream(stream))
        self._check(st, allow=(TM_ERR_NOCONV,) if allow_noconv else ())
        return st, list(stats)

    def loops(self, params, per_noise=False, stream=None, allow_noconv=False):
        n_est = bin(params.estimators).count("1")
        Lt = self.L[3]
        n_ins = n_insertions(params.derivative)
        out = np.zeros((n_est, n_ins, Lt), dtype=np.complex128)
        n_noise = params.n_hp + params.n_lp
        pn = np.zeros((n_noise, 2, n_est, n_ins, Lt), dtype=np.complex128) if per_noise else None
        stats = tm_loop_stats()
        st = tm_loops(self.h, ctypes.byref(params), out.ctypes.data_as(_dp),
                      pn.ctypes.data_as(_dp) if pn is not None else None, ctypes.byref(stats),
                      _stream(stream))
        self._check(st, allow=(TM_ERR_NOCONV,) if allow_noconv else ())
        return out, pn, stats, st

    def noise(self, out, seed, r, dilution=TM_DIL_NONE, stream=None):
        self._check(tm_noise(self.h, _ptr(out), ctypes.c_uint64(seed), r, dilution,
                             _stream(stream)))

    # ------------------------------------------------------------ learned preconditioner
    def ptc_set_weights(self, W1, W2):
        W1 = np.ascontiguousarray(W1, dtype=np.complex128)
        W2 = np.ascontiguousarray(W2, dtype=np.complex128)
        assert W1.shape == W2.shape and W1.shape[0] == 9 and W1.shape[2:] == (4, 4), W1.shape
        self._check(tm_ptc_set_weights(self.h, W1.shape[1], W1.ctypes.data_as(_dp),
                                       W2.ctypes.data_as(_dp)))

    def ptc_set_arith(self, prec):
        """Network forward arithmetic: TM_F32 (vector units) or TM_BF16 (matrix cores)."""
        self._check(tm_ptc_set_arith(self.h, prec))

    def ptc_get_weights(self, nc):
        W1 = np.zeros((9, nc, 4, 4), dtype=np.complex128)
        W2 = np.zeros_like(W1)
        self._check(tm_ptc_get_weights(self.h, nc, W1.ctypes.data_as(_dp), W2.ctypes.data_as(_dp)))
        return W1, W2

    def ptc_init_hopping(self, nc=12, mu_sign=1, seed=0, noise=0.0):
        self._check(tm_ptc_init_hopping(self.h, nc, mu_sign, ctypes.c_uint64(seed), noise))

    def ptc_apply(self, out, inp, nrhs, stream=None):
        self._check(tm_ptc_apply(self.h, _ptr(out), _ptr(inp), nrhs, _stream(stream)))

    def ptc_loss_grad(self, r, e, npairs, nc, loss_kind=TM_PTC_LOSS_ERROR, mu_sign=1, stream=None):
        loss = ctypes.c_double()
        G1 = np.zeros((9, nc, 4, 4), dtype=np.complex128)
        G2 = np.zeros_like(G1)
        self._check(tm_ptc_loss_grad(self.h, loss_kind, mu_sign, _ptr(r),
                                     _ptr(e) if e is not None else None, npairs, ctypes.byref(loss),
                                     G1.ctypes.data_as(_dp), G2.ctypes.data_as(_dp), _stream(stream)))
        return loss.value, G1, G2

    def ptc_pairs_reserve(self, capacity, store_prec=TM_F32):
        self._check(tm_ptc_pairs_reserve(self.h, capacity, store_prec))

    def ptc_pairs_add(self, r, e, n, stream=None):
        self._check(tm_ptc_pairs_add(self.h, _ptr(r), _ptr(e), n, _stream(stream)))

    def ptc_pairs_from_solve(self, b, nrhs, params, iters, stream=None):
        it = (ctypes.c_int * len(iters))(*iters)
        added = ctypes.c_int(0)
        self._check(tm_ptc_pairs_from_solve(self.h, _ptr(b), nrhs, ctypes.byref(params), it, len(iters),
                                            ctypes.byref(added), _stream(stream)))
        return added.value

    def ptc_train(self, epochs, batch, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-12, seed=0,
                  n_pairs=None, loss=TM_PTC_LOSS_ERROR, mu_sign=1, stream=None):
        p = tm_ptc_train_params(epochs, batch, lr, beta1, beta2, adam_eps, ctypes.c_uint64(seed), loss,
                                mu_sign)
        st = tm_ptc_train_stats()
        hist = None
        if n_pairs is not None:
            hist = np.zeros(epochs * (n_pairs // batch))
        self._check(tm_ptc_train(self.h, ctypes.byref(p), ctypes.byref(st),
                                 hist.ctypes.data_as(_dp) if hist is not None else None, _stream(stream)))
        return st, hist

    def contract_momentum(self, eta, s, nrhs, estimators, p2max, mu_sign=1, derivative=0,
                          stream=None):
        n_est = bin(estimators).count("1")
        n_mom = len(momenta(p2max))
        out = np.zeros((n_est, n_mom, n_insertions(derivative), self.L[3]), dtype=np.complex128)
        self._check(tm_contract_momentum(self.h, _ptr(eta), _ptr(s), nrhs, estimators, mu_sign,
                                         derivative, p2max, out.ctypes.data_as(_dp),
                                         _stream(stream)))
        return out

    def loops_momentum(self, params, p2max, per_noise=False, stream=None, allow_noconv=False):
        n_est = bin(params.estimators).count("1")
        n_mom = len(momenta(p2max))
        Lt = self.L[3]
        n_ins = n_insertions(params.derivative)
        out = np.zeros((n_est, n_mom, n_ins, Lt), dtype=np.complex128)
        n_noise = params.n_hp + params.n_lp
        pn = (np.zeros((n_noise, 2, n_est, n_mom, n_ins, Lt), dtype=np.complex128)
              if per_noise else None)
        stats = tm_loop_stats()
        st = tm_loops_momentum(self.h, ctypes.byref(params), p2max, out.ctypes.data_as(_dp),
                               pn.ctypes.data_as(_dp) if pn is not None else None,
                               ctypes.byref(stats), _stream(stream))
        self._check(st, allow=(TM_ERR_NOCONV,) if allow_noconv else ())
        return out, pn, stats, st

    def contract(self, eta, s, nrhs, estimators, mu_sign=1, stream=None):
        n_est = bin(estimators).count("1")
        out = np.zeros((n_est, 16, self.L[3]), dtype=np.complex128)
        self._check(tm_contract(self.h, _ptr(eta), _ptr(s), nrhs, estimators, mu_sign,
                                out.ctypes.data_as(_dp), _stream(stream)))
        return out


def n_insertions(derivative):
    """Insertions per estimator: 16 ultra-local, 80 with one-derivative ones."""
    return 80 if derivative else 16


def momenta(p2max):
    """Integer momentum vectors n (p = 2 pi n / L) with |n|^2 <= p2max, in the
    library's order -> (n_mom, 3) int array."""
    n = ctypes.c_int(0)
    if tm_momenta(p2max, ctypes.byref(n), None) != TM_OK:
        raise TMError(TM_ERR_ARG, "p2max must be >= 0")
    out = np.zeros((n.value, 3), dtype=np.int32)
    st = tm_momenta(p2max, ctypes.byref(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if st != TM_OK:
        raise TMError(st, "tm_momenta failed")
    return out


class Batch:
    """Several contexts (lattices) solved together (tm_batch_*)."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        arr = (_vp * len(self.contexts))(*[c.h for c in self.contexts])
        h = ctypes.c_void_p()
        st = tm_batch_create(ctypes.byref(h), arr, len(self.contexts))
        if st != TM_OK:
            raise TMError(st, "tm_batch_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            tm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != TM_OK and st not in allow:
            raise TMError(st, tm_batch_last_error(self.h).decode())
        return st

    def solve(self, xs, bs, nrhs, params, stream=None, allow_noconv=False):
        n = len(self.contexts)
        xa = (_vp * n)(*[x.data_ptr() for x in xs])
        ba = (_vp * n)(*[b.data_ptr() for b in bs])
        na = (ctypes.c_int * n)(*nrhs)
        stats = [(tm_solve_stats * k)() for k in nrhs]
        sp = (ctypes.POINTER(tm_solve_stats) * n)(*[ctypes.cast(s, ctypes.POINTER(tm_solve_stats))
                                                    for s in stats])
        st = tm_batch_solve(self.h, xa, ba, na, ctypes.byref(params), sp, _stream(stream))
        self._check(st, allow=(TM_ERR_NOCONV,) if allow_noconv else ())
        return st, [list(s) for s in stats]

    def loops(self, params_list, stream=None, allow_noconv=False):
        n = len(self.contexts)
        pa = (tm_loop_params * n)(*params_list)
        outs = []
        for c, p in zip(self.contexts, params_list):
            outs.append(np.zeros((bin(p.estimators).count("1"), n_insertions(p.derivative), c.L[3]),
                                 dtype=np.complex128))
        la = (_dp * n)(*[o.ctypes.data_as(_dp) for o in outs])
        stats = (tm_loop_stats * n)()
        st = tm_batch_loops(self.h, pa, la, stats, _stream(stream))
        self._check(st, allow=(TM_ERR_NOCONV,) if allow_noconv else ())
        return outs, list(stats), st
