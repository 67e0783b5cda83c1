"""Python binding of libftcc.so (argument marshalling only).

Every function here converts numpy arrays to host pointers and calls the C ABI
declared in include/ftcc.h; all arithmetic runs in the library's HIP kernels.
The library is loaded from this package directory; if it is missing the import
fails with an error telling how to build it (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libftcc.so")

_lib = None

OK, EINVAL, ESTATE, ENOMEM, EDEVICE, ENOCONV, ENONFINITE, EDIVERGE = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {EINVAL: "EINVAL", ESTATE: "ESTATE", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
          ENOCONV: "ENOCONV", ENONFINITE: "ENONFINITE", EDIVERGE: "EDIVERGE"}


class FTCCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("n_tau", ctypes.c_int), ("nodes_per_panel", ctypes.c_int), ("propagator", ctypes.c_int),
                ("occ_thresh", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("checkpoint", ctypes.c_int), ("diis_depth", ctypes.c_int), ("mem_cap_bytes", ctypes.c_size_t),
                ("spin_orbital", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.POINTER(ctypes.c_long)


def library():
    """Load libftcc.so once (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2004_01729_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "ftcc_default_options": (None, [ctypes.POINTER(Options)]),
        "ftcc_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(Options)]),
        "ftcc_destroy": (ctypes.c_int, [ctypes.c_void_p]),
        "ftcc_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
        "ftcc_set_allocator": (ctypes.c_int, [ctypes.c_void_p, ALLOC_FN, FREE_FN, ctypes.c_void_p]),
        "ftcc_set_hamiltonian": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _D, _D, _D]),
        "ftcc_set_momentum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I]),
        "ftcc_solve_amplitudes": (ctypes.c_int, [ctypes.c_void_p, _D, _D, _I, _I]),
        "ftcc_grand_potential": (ctypes.c_int, [ctypes.c_void_p, _D, _D]),
        "ftcc_get_amplitudes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _D, _D]),
        "ftcc_lambda": (ctypes.c_int, [ctypes.c_void_p, _I, _I]),
        "ftcc_get_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]),
        "ftcc_response": (ctypes.c_int, [ctypes.c_void_p, _D, _D, _D, _D, ctypes.POINTER(_D), ctypes.POINTER(_D), _D]),
        "ftcc_response_noalloc": (ctypes.c_int, [ctypes.c_void_p, _D, _D]),
        "ftcc_eval_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              _D, _D, _D, _D, _D]),
        "ftcc_time_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _D, _D]),
        "ftcc_stats": (ctypes.c_int, [ctypes.c_void_p, _L, _L, _D, _D]),
        "ftcc_find_mu": (ctypes.c_int, [ctypes.c_void_p, _D, _D, _D, ctypes.c_double, ctypes.c_int, _D, _I, _I]),
        "ftcc_kernel_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _D, _D, _L]),
        "ftcc_plan_info": (ctypes.c_int, [ctypes.c_void_p, _L, _L, _D, _I]),
        "ftcc_two_body_density": (ctypes.c_int, [ctypes.c_void_p, _D]),
        "ftcc_last_error": (ctypes.c_char_p, []),
        "ftcc_abi_version": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the C header declares (used by the CPU-side load test)."""
    return ["ftcc_default_options", "ftcc_create", "ftcc_destroy", "ftcc_set_stream", "ftcc_set_allocator",
            "ftcc_set_momentum", "ftcc_set_hamiltonian",
            "ftcc_solve_amplitudes", "ftcc_grand_potential", "ftcc_get_amplitudes", "ftcc_lambda",
            "ftcc_get_lambda", "ftcc_response", "ftcc_response_noalloc", "ftcc_find_mu", "ftcc_eval_residual", "ftcc_time_residual",
            "ftcc_stats", "ftcc_plan_info",
            "ftcc_kernel_profile", "ftcc_two_body_density",
            "ftcc_last_error", "ftcc_abi_version"]


def _ptr(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _check(rc, lib=None, allow=()):
    if rc != OK and rc not in allow:
        lib = lib or library()
        raise FTCCError(rc, lib.ftcc_last_error().decode())
    return rc


def default_options(**kw):
    o = Options()
    library().ftcc_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Context:
    """One ftcc_ctx: n_instances problems solved together on one GPU."""

    def __init__(self, n_instances=1, device=0, **options):
        self.lib = library()
        self.opt = default_options(**options)
        self.B = int(n_instances)
        self._h = ctypes.c_void_p()
        _check(self.lib.ftcc_create(ctypes.byref(self._h), int(device), self.B, ctypes.byref(self.opt)))
        self.sizes = {}

    def close(self):
        if self._h:
            self.lib.ftcc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream_ptr):
        _check(self.lib.ftcc_set_stream(self._h, ctypes.c_void_p(stream_ptr)))

    def set_allocator(self, alloc, free):
        """Python callables alloc(nbytes) -> device address (int, 0 on failure) and
        free(address); called from the library for its bulk device buffers."""
        def _a(nbytes, _user):
            try:
                return int(alloc(int(nbytes))) or None
            except Exception:
                return None

        def _f(ptr, _user):
            free(int(ptr))
        # keep the C thunks alive as long as the context
        self._alloc_thunks = (ALLOC_FN(_a), FREE_FN(_f))
        _check(self.lib.ftcc_set_allocator(self._h, self._alloc_thunks[0], self._alloc_thunks[1], None))

    def set_hamiltonian(self, inst, h, eri, eps):
        h = _f64(h)
        n = h.shape[0]
        eri = _f64(eri, (n, n, n, n))
        eps = _f64(eps, (n,))
        _check(self.lib.ftcc_set_hamiltonian(self._h, int(inst), n, _ptr(h), _ptr(eri), _ptr(eps)))
        self.sizes[int(inst)] = n

    def set_momentum(self, inst, labels, modulus):
        """Integer momentum labels (n x dims) and per-component modulus (0 = none)."""
        lab = np.ascontiguousarray(np.asarray(labels), dtype=np.int32)
        if lab.ndim == 1:
            lab = lab.reshape(-1, 1)
        mod = np.ascontiguousarray(np.asarray(modulus), dtype=np.int32).reshape(-1)
        if mod.size != lab.shape[1]:
            raise ValueError("modulus needs one entry per label component")
        _check(self.lib.ftcc_set_momentum(self._h, int(inst), lab.shape[0], lab.shape[1], lab.ctypes.data_as(_I),
                                          mod.ctypes.data_as(_I)))

    def solve(self, mu, beta, raise_on_status=True):
        mu = _f64(np.broadcast_to(np.asarray(mu, float), (self.B,)))
        beta = _f64(np.broadcast_to(np.asarray(beta, float), (self.B,)))
        its = np.zeros(self.B, dtype=np.int32)
        st = np.zeros(self.B, dtype=np.int32)
        rc = self.lib.ftcc_solve_amplitudes(self._h, _ptr(mu), _ptr(beta), its.ctypes.data_as(_I),
                                           st.ctypes.data_as(_I))
        _check(rc, allow=() if raise_on_status else (ENOCONV, ENONFINITE, EDIVERGE))
        return its, st

    def grand_potential(self):
        om = np.zeros(self.B)
        parts = np.zeros((self.B, 3))
        _check(self.lib.ftcc_grand_potential(self._h, _ptr(om), _ptr(parts)))
        return om, parts

    def _size(self, inst):
        if int(inst) not in self.sizes:
            raise FTCCError(EINVAL, f"instance {inst} has no Hamiltonian")
        return self.sizes[int(inst)]

    def amplitudes(self, inst, node):
        n = self._size(inst)
        t1 = np.zeros((n, n))
        t2 = np.zeros((n, n, n, n))
        _check(self.lib.ftcc_get_amplitudes(self._h, int(inst), int(node), _ptr(t1), _ptr(t2)))
        return t1, t2

    def lam(self, raise_on_status=True):
        its = np.zeros(self.B, dtype=np.int32)
        st = np.zeros(self.B, dtype=np.int32)
        rc = self.lib.ftcc_lambda(self._h, its.ctypes.data_as(_I), st.ctypes.data_as(_I))
        _check(rc, allow=() if raise_on_status else (ENOCONV, ENONFINITE, EDIVERGE))
        return its, st

    def get_lambda(self, inst, node, tilde=True):
        """[lambda1, lambda2, lambda-tilde1, lambda-tilde2] of one node (the last two None
        unless `tilde`)."""
        n = self._size(inst)
        out = [np.zeros((n, n)), np.zeros((n,) * 4)]
        out += [np.zeros((n, n)), np.zeros((n,) * 4)] if tilde else [None, None]
        nul = ctypes.cast(None, _D)
        _check(self.lib.ftcc_get_lambda(self._h, int(inst), int(node),
                                        *[nul if a is None else _ptr(a) for a in out]))
        return out

    def response(self, want_mu=True, want_beta=True, want_h=True, deri_dtheta=None, dh_dtheta=None,
                 want_eps=False):
        """dOmega/dmu, dbeta, dh (list of n_i x n_i arrays), dOmega/deps (list of length-n_i
        arrays, when want_eps) and the optional theta direction."""
        B = self.B
        sizes = [self.sizes[i] for i in range(B)]
        n = max(sizes)
        dmu = np.zeros(B) if want_mu else None
        dbeta = np.zeros(B) if want_beta else None
        dh_flat = np.zeros(sum(k * k for k in sizes)) if want_h else None
        deps_flat = np.zeros(sum(sizes)) if want_eps else None
        dth = None
        keep = []
        p_deri = p_dh = None
        if deri_dtheta is not None or dh_dtheta is not None:
            dth = np.zeros(B)
            if deri_dtheta is not None:
                arrs = [None if a is None else _f64(a, (sizes[i],) * 4) for i, a in enumerate(deri_dtheta)]
                keep += arrs
                p_deri = (_D * B)(*[ctypes.cast(None, _D) if a is None else _ptr(a) for a in arrs])
            if dh_dtheta is not None:
                arrs = [None if a is None else _f64(a, (sizes[i],) * 2) for i, a in enumerate(dh_dtheta)]
                keep += arrs
                p_dh = (_D * B)(*[ctypes.cast(None, _D) if a is None else _ptr(a) for a in arrs])
        nul = ctypes.cast(None, _D)
        _check(self.lib.ftcc_response(self._h, _ptr(dmu) if dmu is not None else nul,
                                      _ptr(dbeta) if dbeta is not None else nul,
                                      _ptr(dh_flat) if dh_flat is not None else nul,
                                      _ptr(deps_flat) if deps_flat is not None else nul,
                                      p_deri, p_dh, _ptr(dth) if dth is not None else nul))
        dh = None
        if dh_flat is not None:
            dh, off = [], 0
            for k in sizes:
                dh.append(dh_flat[off:off + k * k].reshape(k, k))
                off += k * k
        deps = None
        if deps_flat is not None:
            deps, off = [], 0
            for k in sizes:
                deps.append(deps_flat[off:off + k].copy())
                off += k
        return dict(mu=dmu, beta=dbeta, h=dh, eps=deps, theta=dth)

    def response_noalloc(self, want_mu=True, want_beta=True):
        """dOmega/dmu and dOmega/dbeta through the allocation-free entry point."""
        nul = ctypes.cast(None, _D)
        dmu = np.zeros(self.B) if want_mu else None
        dbeta = np.zeros(self.B) if want_beta else None
        _check(self.lib.ftcc_response_noalloc(self._h, _ptr(dmu) if dmu is not None else nul,
                                              _ptr(dbeta) if dbeta is not None else nul))
        return dict(mu=dmu, beta=dbeta)

    def two_body_density(self):
        """Gamma_pqrs = dOmega/d<pq|rs> of every instance (list of n_i^4 arrays)."""
        sizes = [self.sizes[i] for i in range(self.B)]
        flat = np.zeros(sum(k ** 4 for k in sizes))
        _check(self.lib.ftcc_two_body_density(self._h, _ptr(flat)))
        out, off = [], 0
        for k in sizes:
            out.append(flat[off:off + k ** 4].reshape(k, k, k, k))
            off += k ** 4
        return out

    def find_mu(self, n_target, mu0, beta, tol=1e-10, max_iter=40, raise_on_status=True):
        """mu of every instance with -dOmega/dmu = n_target; returns (mu, N, iters, status)."""
        B = self.B
        nt = _f64(np.broadcast_to(np.asarray(n_target, float), (B,)))
        mu = _f64(np.array(np.broadcast_to(np.asarray(mu0, float), (B,))))
        beta = _f64(np.broadcast_to(np.asarray(beta, float), (B,)))
        n_out = np.zeros(B)
        its = np.zeros(B, dtype=np.int32)
        st = np.zeros(B, dtype=np.int32)
        rc = self.lib.ftcc_find_mu(self._h, _ptr(nt), _ptr(mu), _ptr(beta), float(tol), int(max_iter), _ptr(n_out),
                                   its.ctypes.data_as(_I), st.ctypes.data_as(_I))
        _check(rc, allow=() if raise_on_status else (ENOCONV, ENONFINITE, EDIVERGE))
        return mu, n_out, its, st

    def eval_residual(self, inst, mu, beta, t1, t2):
        n = self._size(inst)
        t1 = _f64(t1, (n, n))
        t2 = _f64(t2, (n, n, n, n))
        S1 = np.zeros((n, n))
        S2 = np.zeros((n, n, n, n))
        E = np.zeros(1)
        _check(self.lib.ftcc_eval_residual(self._h, int(inst), float(mu), float(beta), _ptr(t1), _ptr(t2),
                                           _ptr(S1), _ptr(S2), _ptr(E)))
        return S1, S2, float(E[0])

    def time_residual(self, reps):
        sec = np.zeros(1)
        fl = np.zeros(1)
        _check(self.lib.ftcc_time_residual(self._h, int(reps), _ptr(sec), _ptr(fl)))
        return float(sec[0]), float(fl[0])

    def plan_info(self):
        """Kernel dispatches of one forward / backward pass of the slot program, the
        algorithmic bytes of one forward pass, and the nodes per instance it evaluates."""
        df = ctypes.c_long()
        db = ctypes.c_long()
        by = ctypes.c_double()
        sl = ctypes.c_int()
        _check(self.lib.ftcc_plan_info(self._h, ctypes.byref(df), ctypes.byref(db), ctypes.byref(by),
                                       ctypes.byref(sl)))
        return dict(dispatches_forward=df.value, dispatches_backward=db.value, bytes_forward=by.value,
                    slots=sl.value)

    def kernel_profile(self, enable):
        """Totals of the dominant GEMM kernel since the previous call; then enable/disable."""
        fl = ctypes.c_double()
        sec = ctypes.c_double()
        nl = ctypes.c_long()
        _check(self.lib.ftcc_kernel_profile(self._h, int(enable), ctypes.byref(fl), ctypes.byref(sec),
                                            ctypes.byref(nl)))
        return dict(flops=fl.value, seconds=sec.value, launches=nl.value)

    def stats(self):
        r = ctypes.c_long()
        v = ctypes.c_long()
        ts = ctypes.c_double()
        tl = ctypes.c_double()
        _check(self.lib.ftcc_stats(self._h, ctypes.byref(r), ctypes.byref(v), ctypes.byref(ts), ctypes.byref(tl)))
        return dict(resid_evals=r.value, vjp_evals=v.value, solve_seconds=ts.value, lambda_seconds=tl.value)
