"""ctypes binding of libexacc.so (the C ABI in include/exacc.h).

Argument marshalling only: every step of the iteration runs in the HIP
library.  Inputs may be numpy arrays (host) or torch CUDA tensors (device);
PyTorch is used only for device memory and streams.  Loading fails loudly when
the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libexacc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "exacc.h")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_NOMEM, ERR_DEVICE, ERR_DIVERGED, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("diis_size", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("level_shift", ctypes.c_double),
        ("fp64_final_iters", ctypes.c_int),
        ("mixed_switch_tol", ctypes.c_double),
        ("inputs_on_device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("ladder_chunk_pairs", ctypes.c_long),
        ("timing", ctypes.c_int),
        ("doubles_only", ctypes.c_int),
        ("cc2", ctypes.c_int),
        ("triples_occ_block", ctypes.c_int),
        ("ladder_defect_correction", ctypes.c_int),
        ("graph_residual", ctypes.c_int),
        ("ladder_group_nvir", ctypes.c_int),
    ]


_lib = None


def load():
    """Load libexacc.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("libexacc.so is not built; run __graft_entry__.build() "
                           "(python -m paper_2103_08473_amd.build)")
    L = ctypes.CDLL(LIBPATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    L.exacc_ccsd_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.exacc_ccsd_default_opts.restype = None
    L.exacc_ccsd_memory_estimate.argtypes = [I, I, I, ctypes.POINTER(Opts)]
    L.exacc_ccsd_memory_estimate.restype = S
    L.exacc_ccsd_create.argtypes = [ctypes.POINTER(P), I, I, I, P, P, ctypes.POINTER(Opts)]
    L.exacc_ccsd_iterate.argtypes = [P, I, ip, dp, ip]
    L.exacc_ccsd_energy.argtypes = [P, dp, dp]
    L.exacc_ccsd_get_amplitudes.argtypes = [P, P, P, I]
    L.exacc_ccsd_set_amplitudes.argtypes = [P, P, P, I]
    L.exacc_ccsd_residual.argtypes = [P, P, P, I]
    L.exacc_ccsd_triples.argtypes = [P, dp, dp, dp]
    L.exacc_ccsd_lambda_iterate.argtypes = [P, I, ip, dp, ip]
    L.exacc_ccsd_lambda_residual.argtypes = [P, P, P, I]
    L.exacc_ccsd_get_lambda.argtypes = [P, P, P, I]
    L.exacc_ccsd_set_lambda.argtypes = [P, P, P, I]
    L.exacc_ccsd_density.argtypes = [P, P, I]
    L.exacc_df_factors.argtypes = [I, I, I, P, P, P, P, I, P, ip]
    L.exacc_df_factors_noalloc.argtypes = [I, I, I, P, P, P, P, P, ip]
    L.exacc_ccsd_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_char_p), dp, ip, I]
    L.exacc_ccsd_phase.argtypes = [P, ip, ip]
    L.exacc_ccsd_phase.restype = I
    L.exacc_ladder_flops.argtypes = [I, I, I]
    L.exacc_ladder_flops.restype = D
    L.exacc_ccsd_destroy.argtypes = [P]
    L.exacc_status_string.argtypes = [I]
    L.exacc_status_string.restype = ctypes.c_char_p
    L.exacc_last_error.argtypes = []
    L.exacc_last_error.restype = ctypes.c_char_p
    for f in ("exacc_ccsd_create", "exacc_ccsd_iterate", "exacc_ccsd_energy",
              "exacc_ccsd_get_amplitudes", "exacc_ccsd_set_amplitudes", "exacc_ccsd_residual",
              "exacc_ccsd_triples", "exacc_ccsd_lambda_iterate", "exacc_ccsd_lambda_residual",
              "exacc_ccsd_get_lambda", "exacc_ccsd_set_lambda", "exacc_ccsd_density",
              "exacc_df_factors", "exacc_df_factors_noalloc",
              "exacc_ccsd_stage_times", "exacc_ccsd_destroy"):
        getattr(L, f).restype = I
    _lib = L
    return L


def declared_symbols():
    """Function names declared in include/exacc.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(exacc_[a-z0-9_]+)\s*\(", text)))


class ExaccError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("exacc status %d: %s" % (status, msg))
        self.status = status


def _check(status, allow=(OK,)):
    if status not in allow:
        L = load()
        raise ExaccError(status, "%s (%s)" % (L.exacc_status_string(status).decode(),
                                            L.exacc_last_error().decode()))
    return status


def default_opts(**kw):
    o = Opts()
    load().exacc_ccsd_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def memory_estimate(nocc, nvir, naux, **kw):
    o = default_opts(**kw)
    return int(load().exacc_ccsd_memory_estimate(nocc, nvir, naux, ctypes.byref(o)))


def ladder_flops(nocc, nvir, naux):
    return float(load().exacc_ladder_flops(nocc, nvir, naux))


def df_factors(C, J, V, stream=None):
    """DF factors B[P][p][q] from spinor coefficients C [nao][n], AO three-index integrals
    J [naux][nao][nao] and the metric V [naux][naux] (exacc_df_factors).  numpy inputs give
    a numpy result (host pointers); torch CUDA tensors (complex128 C, J; float64 V) give a
    torch CUDA tensor.  Returns (B, Newton-Schulz step count)."""
    L = load()
    it = ctypes.c_int(0)
    if _is_torch(C):
        import torch
        nao, n = C.shape
        X = J.shape[0]
        B = torch.empty((X, n, n), dtype=torch.complex128, device=C.device)
        _check(L.exacc_df_factors(nao, n, X, C.data_ptr(), J.data_ptr(), V.data_ptr(), B.data_ptr(),
                                  1, stream, ctypes.byref(it)))
        return B, it.value
    c, pc = _host_c128(C)
    j, pj = _host_c128(J)
    v = np.ascontiguousarray(V, dtype=np.float64)
    nao, n = c.shape
    X = j.shape[0]
    B = np.zeros((X, n, n), np.complex128)
    _check(L.exacc_df_factors(nao, n, X, pc, pj, v.ctypes.data, B.ctypes.data, 0, None, ctypes.byref(it)))
    return B, it.value


def df_factors_noalloc(C, J, V, B, stream=None):
    """exacc_df_factors_noalloc on torch CUDA tensors: C complex128 [nao][n], J complex128
    [naux][nao][nao], V float64 [naux][naux] and the caller's output B complex128
    [naux][n][n] (written in place).  No device memory is allocated by the call.
    Returns the Newton-Schulz step count."""
    L = load()
    it = ctypes.c_int(0)
    nao, n = C.shape
    X = J.shape[0]
    assert tuple(B.shape) == (X, n, n) and tuple(V.shape) == (X, X) and tuple(J.shape) == (X, nao, nao)
    for t in (C, J, V, B):
        assert t.is_cuda and t.is_contiguous()
    _check(L.exacc_df_factors_noalloc(nao, n, X, C.data_ptr(), J.data_ptr(), V.data_ptr(),
                                      B.data_ptr(), stream, ctypes.byref(it)))
    return it.value


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _host_c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data


class CCSD:
    """One CCSD solve resident on the GPU (wraps an exacc_ccsd_t handle).

    eps : float64 [n], B : complex128 [naux, n, n]; numpy (host) or torch CUDA
    tensors (device; then torch.complex128 / torch.float64, contiguous).
    """

    def __init__(self, eps, B, nocc, **opts):
        L = load()
        self.L = L
        naux, n, n2 = B.shape
        assert n == n2 and eps.shape[0] == n
        self.nocc, self.nvir, self.naux = nocc, n - nocc, naux
        on_dev = _is_torch(B)
        if "stream" in opts and opts["stream"] is not None and not isinstance(opts["stream"], int):
            opts["stream"] = opts["stream"].cuda_stream
        self.opts = default_opts(inputs_on_device=1 if on_dev else 0, **opts)
        if on_dev:
            eptr, bptr = eps.data_ptr(), B.data_ptr()
            keep = (eps, B)
        else:
            e = np.ascontiguousarray(eps, dtype=np.float64)
            b = np.ascontiguousarray(B, dtype=np.complex128)
            eptr, bptr = e.ctypes.data, b.ctypes.data
            keep = (e, b)
        h = ctypes.c_void_p()
        st = L.exacc_ccsd_create(ctypes.byref(h), nocc, self.nvir, naux, eptr, bptr,
                                 ctypes.byref(self.opts))
        del keep
        _check(st)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.exacc_ccsd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def iterate(self, max_steps=1):
        """Returns (status, steps_done, residual, converged)."""
        steps, conv = ctypes.c_int(), ctypes.c_int()
        res = ctypes.c_double()
        st = self.L.exacc_ccsd_iterate(self.h, max_steps, ctypes.byref(steps), ctypes.byref(res),
                                       ctypes.byref(conv))
        _check(st, allow=(OK, NOT_CONVERGED, ERR_DIVERGED))
        return st, steps.value, res.value, bool(conv.value)

    def energy(self):
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(self.L.exacc_ccsd_energy(self.h, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def amplitudes(self):
        o, v = self.nocc, self.nvir
        t1 = np.zeros((o, v), np.complex128)
        t2 = np.zeros((o, o, v, v), np.complex128)
        _check(self.L.exacc_ccsd_get_amplitudes(self.h, t1.ctypes.data, t2.ctypes.data, 0))
        return t1, t2

    def set_amplitudes(self, t1, t2):
        if _is_torch(t1):
            _check(self.L.exacc_ccsd_set_amplitudes(self.h, t1.data_ptr(), t2.data_ptr(), 1))
            return
        a, pa = _host_c128(t1)
        b, pb = _host_c128(t2)
        _check(self.L.exacc_ccsd_set_amplitudes(self.h, pa, pb, 0))

    def residual(self, s1=None, s2=None):
        """S1 [o,v], S2 [o,o,v,v] of eq. CC_general at the current amplitudes.
        With torch CUDA output tensors s1/s2 given, fills them on the device."""
        if s1 is not None and _is_torch(s1):
            _check(self.L.exacc_ccsd_residual(self.h, s1.data_ptr(),
                                              s2.data_ptr() if s2 is not None else None, 1))
            return s1, s2
        o, v = self.nocc, self.nvir
        r1 = np.zeros((o, v), np.complex128)
        r2 = np.zeros((o, o, v, v), np.complex128)
        _check(self.L.exacc_ccsd_residual(self.h, r1.ctypes.data, r2.ctypes.data, 0))
        return r1, r2

    def triples(self):
        """(E(+T), E((T)), E(-T)) at the current amplitudes (App. C), FP64, Hartree."""
        e4, e5, ey = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(self.L.exacc_ccsd_triples(self.h, ctypes.byref(e4), ctypes.byref(e5), ctypes.byref(ey)))
        return e4.value, e5.value, ey.value

    # ---- Lambda equations (App. D) and the one-body density (App. E)
    def lambda_iterate(self, max_steps=1):
        """Lambda steps at the current amplitudes; returns (status, steps_done, residual,
        converged)."""
        steps, conv = ctypes.c_int(), ctypes.c_int()
        res = ctypes.c_double()
        st = self.L.exacc_ccsd_lambda_iterate(self.h, max_steps, ctypes.byref(steps),
                                              ctypes.byref(res), ctypes.byref(conv))
        _check(st, allow=(OK, NOT_CONVERGED, ERR_DIVERGED))
        return st, steps.value, res.value, bool(conv.value)

    def lambda_solve(self, max_iter=None):
        """Iterate the Lambda equations until converged; returns (converged, history of
        ||Delta lambda||)."""
        max_iter = self.opts.max_iter if max_iter is None else max_iter
        hist = []
        conv = False
        for _ in range(max_iter):
            st, _, r, conv = self.lambda_iterate(1)
            hist.append(r)
            if st == ERR_DIVERGED or conv:
                break
        return conv, hist

    def lambda_residual(self):
        """R1 [o,v], R2 [o,o,v,v] of the Lambda equations at the current lambda."""
        o, v = self.nocc, self.nvir
        r1 = np.zeros((o, v), np.complex128)
        r2 = np.zeros((o, o, v, v), np.complex128)
        _check(self.L.exacc_ccsd_lambda_residual(self.h, r1.ctypes.data, r2.ctypes.data, 0))
        return r1, r2

    def get_lambda(self):
        o, v = self.nocc, self.nvir
        l1 = np.zeros((o, v), np.complex128)
        l2 = np.zeros((o, o, v, v), np.complex128)
        _check(self.L.exacc_ccsd_get_lambda(self.h, l1.ctypes.data, l2.ctypes.data, 0))
        return l1, l2

    def set_lambda(self, l1, l2):
        a, pa = _host_c128(l1)
        b, pb = _host_c128(l2)
        _check(self.L.exacc_ccsd_set_lambda(self.h, pa, pb, 0))

    def density(self):
        """Correlation one-body density gamma[p, q] = <{q+ p}> [n, n] (App. E)."""
        n = self.nocc + self.nvir
        g = np.zeros((n, n), np.complex128)
        _check(self.L.exacc_ccsd_density(self.h, g.ctypes.data, 0))
        return g

    def phase(self):
        """(precision of the next step: 1 low precision, 2 FP64 with the defect-corrected
        low-precision ladder, 0 FP64; full FP64 iterations since the last phase change)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(self.L.exacc_ccsd_phase(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def stage_times(self, reset=False):
        n = ctypes.c_int(64)
        names = (ctypes.c_char_p * 64)()
        ms = (ctypes.c_double * 64)()
        _check(self.L.exacc_ccsd_stage_times(self.h, names, ms, ctypes.byref(n), int(reset)))
        return {names[i].decode(): ms[i] for i in range(min(n.value, 64))}

    def solve(self, max_iter=None, callback=None):
        """Iterate one step at a time until converged; returns (energy, converged, history)."""
        max_iter = self.opts.max_iter if max_iter is None else max_iter
        hist = []
        conv = False
        for it in range(1, max_iter + 1):
            st, _, r, conv = self.iterate(1)
            E = self.energy()
            hist.append((it, E, r))
            if callback:
                callback(it, E, r)
            if st == ERR_DIVERGED or conv:
                break
        return hist[-1][1] if hist else 0j, conv, hist
