"""Thin ctypes binding of the C ABI in include/afq.h.

Argument marshalling only: every step of the walker step runs in the HIP
library.  Host arrays are numpy arrays (float64 / complex128, C-contiguous);
device arrays are torch tensors on the context's device (passed by
data_ptr()).  If libafq.so is missing the import fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libafq.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = range(6)
EXP_KRYLOV, EXP_TAYLOR, EXP_BLOCK_KRYLOV, EXP_CHEBYSHEV = 0, 1, 2, 3
PROP_SPLIT2, PROP_SPLIT1, PROP_TAYLOR, PROP_CN = 0, 1, 2, 3
FB_START, FB_HALF = 0, 1
PREC_FP64, PREC_MIXED, PREC_MIXED_FAST, PREC_MIXED_ENERGY = 0, 1, 2, 3
SCHED_AUTO, SCHED_SERIAL, SCHED_STREAMS, SCHED_GRAPH = 0, 1, 2, 3
_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "ENUMERIC"}

EXPORTED = (
    "afq_create", "afq_destroy", "afq_last_error", "afq_init_hamiltonian", "afq_init_trial",
    "afq_init_walkers", "afq_propagate_batch", "afq_local_energy_batch",
    "afq_local_energy_adjoint", "afq_force_bias_adjoint", "afq_get_walkers",
    "afq_set_walkers", "afq_fill_fields", "afq_get_counters", "afq_profile",
    "afq_profile_read", "afq_sync", "afq_autotune", "afq_get_e0",
    "afq_local_energy_batch_noalloc", "afq_stats_time_average", "afq_stats_kappa",
    "afq_stats_blocking", "afq_tau_fit", "afq_init_trial_spin_orbital",
)
FIT_QUADRATIC, FIT_PURE_SQUARE, FIT_LINEAR = 0, 1, 2
PHASES = ("fields", "force_bias", "opbuild", "onebody", "exponential", "overlap", "weight", "qr",
          "exchange", "energy", "coulomb", "pop_control")


class AfqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class PropParams(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("exp_method", ctypes.c_int32),
        ("exp_order", ctypes.c_int32),
        ("reorth_every", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_steps", ctypes.c_int32),
        ("energy_every", ctypes.c_int32),
        ("e0", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("step0", ctypes.c_uint64),
        ("fields", ctypes.c_void_p),
        ("energies_out", ctypes.c_void_p),
        ("schedule", ctypes.c_int32),
        ("e0_window", ctypes.c_int32),
        ("pop_every", ctypes.c_int32),
        ("propagator", ctypes.c_int32),
        ("force_bias_at", ctypes.c_int32),
    ]


def load_library(path: str = _LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run __graft_entry__.build() "
                          "or python paper_2403_02542_amd/build_lib.py")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, u64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "afq_create": (i32, [ctypes.POINTER(P), ctypes.c_int, P]),
        "afq_destroy": (None, [P]),
        "afq_last_error": (ctypes.c_char_p, [P]),
        "afq_init_hamiltonian": (i32, [P, i64, i64, P, P, d, ctypes.c_int, ctypes.POINTER(i32)]),
        "afq_init_trial": (i32, [P, i32, i64, i64, P, ctypes.c_int]),
        "afq_init_trial_spin_orbital": (i32, [P, i32, i64, P, ctypes.c_int]),
        "afq_init_walkers": (i32, [P, i32, i64, P, ctypes.c_int]),
        "afq_propagate_batch": (i32, [P, ctypes.POINTER(i32), i32, ctypes.POINTER(PropParams)]),
        "afq_local_energy_batch": (i32, [P, i32, i32, P, P, ctypes.c_int]),
        "afq_local_energy_adjoint": (i32, [P, i32, P, P, P, ctypes.c_int]),
        "afq_force_bias_adjoint": (i32, [P, i32, P, P, ctypes.c_int]),
        "afq_get_walkers": (i32, [P, i32, P, P, P, P, ctypes.c_int]),
        "afq_set_walkers": (i32, [P, i32, P, P, ctypes.c_int]),
        "afq_fill_fields": (i32, [P, u64, u64, u64, i64, i64, P]),
        "afq_get_counters": (i32, [P, i32, ctypes.POINTER(i64), i32]),
        "afq_get_e0": (i32, [P, i32, ctypes.POINTER(d)]),
        "afq_local_energy_batch_noalloc": (i32, [P, i32, P, P]),
        "afq_profile": (i32, [P, ctypes.c_int]),
        "afq_profile_read": (i32, [P, ctypes.POINTER(d), ctypes.POINTER(i64), ctypes.c_int]),
        "afq_sync": (i32, [P]),
        "afq_autotune": (i32, [P, ctypes.POINTER(i32), i32, i32]),
        "afq_stats_time_average": (i32, [P, P, i64, i64, ctypes.POINTER(d)]),
        "afq_stats_kappa": (i32, [P, i64, d, ctypes.POINTER(d)]),
        "afq_stats_blocking": (i32, [P, i64, ctypes.POINTER(d), i32, ctypes.POINTER(i32)]),
        "afq_tau_fit": (i32, [P, P, P, i32, i32, ctypes.POINTER(d), ctypes.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _arg(x, dtype):
    """(pointer, is_device, keepalive) of a numpy array or torch tensor."""
    if x is None:
        return None, 0, None
    if _is_torch(x):
        import torch
        want = {np.float64: torch.float64, np.complex128: torch.complex128,
                np.int32: torch.int32}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"expected a contiguous {want} tensor")
        return x.data_ptr(), int(x.is_cuda), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, 0, a


def _stat_check(code):
    if code != OK:
        raise AfqError(code, "invalid statistics input")


def stats_time_average(w, e, n_eq=0):
    """(E_bar, sigma_E^2, N) of afq_stats_time_average."""
    wa = np.ascontiguousarray(w, dtype=np.float64)
    ea = np.ascontiguousarray(e, dtype=np.float64)
    if wa.shape != ea.shape:
        raise ValueError("w and e differ in length")
    out = (ctypes.c_double * 3)()
    _stat_check(lib().afq_stats_time_average(wa.ctypes.data, ea.ctypes.data, len(ea), int(n_eq),
                                             out))
    return out[0], out[1], int(out[2])


def stats_kappa(e, c=5.0):
    """dict(acf=kappa, window=M, block=kappa, level=l) of afq_stats_kappa."""
    ea = np.ascontiguousarray(e, dtype=np.float64)
    out = (ctypes.c_double * 4)()
    _stat_check(lib().afq_stats_kappa(ea.ctypes.data, len(ea), float(c), out))
    return {"acf": out[0], "window": int(out[1]), "block": out[2], "level": int(out[3])}


def stats_blocking(e):
    """[(n_l, se_l, se_err_l)] of afq_stats_blocking."""
    ea = np.ascontiguousarray(e, dtype=np.float64)
    cap = 64
    buf = (ctypes.c_double * (3 * cap))()
    nl = ctypes.c_int32()
    _stat_check(lib().afq_stats_blocking(ea.ctypes.data, len(ea), buf, cap, ctypes.byref(nl)))
    return [(int(buf[3 * l]), buf[3 * l + 1], buf[3 * l + 2]) for l in range(min(nl.value, cap))]


def tau_fit(tau, e, sigma=None, form=FIT_QUADRATIC):
    """((E0, alpha, beta), err_E0, sigma_x) of afq_tau_fit."""
    ta = np.ascontiguousarray(tau, dtype=np.float64)
    ea = np.ascontiguousarray(e, dtype=np.float64)
    sa = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.float64)
    coef = (ctypes.c_double * 3)()
    err = (ctypes.c_double * 2)()
    _stat_check(lib().afq_tau_fit(ta.ctypes.data, ea.ctypes.data,
                                  None if sa is None else sa.ctypes.data, len(ta), int(form),
                                  coef, err))
    return (coef[0], coef[1], coef[2]), err[0], err[1]


class Context:
    """One library context (afq_create) on one HIP device."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = lib()
        self._h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        self._check(self._lib.afq_create(ctypes.byref(self._h), int(device), s))
        self.dims = {}

    def _check(self, code):
        if code != OK:
            msg = ""
            if getattr(self, "_h", None):
                m = self._lib.afq_last_error(self._h)
                msg = m.decode() if m else ""
            raise AfqError(code, msg)

    def close(self):
        if self._h:
            self._lib.afq_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- set-up
    def init_hamiltonian(self, h, L, e_core: float = 0.0) -> int:
        hp, hd, hk = _arg(h, np.float64)
        lp, ld, lk = _arg(L, np.float64)
        if hd != ld:
            raise ValueError("h and L must both be host arrays or both device tensors")
        M = h.shape[0]
        sid = ctypes.c_int32()
        self._check(self._lib.afq_init_hamiltonian(self._h, M, L.shape[0], hp, lp,
                                                   float(e_core), hd, ctypes.byref(sid)))
        self.dims[sid.value] = {"M": M, "G": L.shape[0]}
        if hd:
            self.dims[sid.value]["src"] = ((h.data_ptr(), h._version), (L.data_ptr(), L._version))
        return sid.value

    def init_trial(self, sys_id: int, psi_t, n_beta=None):
        """Closed shell (n_beta None): psi_t is M x N, both spins.  Open shell:
        psi_t is M x (N_alpha + N_beta), the alpha orbitals then the beta
        ones, with N_alpha != N_beta; the library then works in 2M spin
        orbitals (walkers 2M x (N_alpha + N_beta))."""
        p, dev, keep = _arg(psi_t, np.float64)
        cols = psi_t.shape[1]
        if n_beta is None:
            n_alpha = n_beta = cols
        else:
            n_alpha = cols - n_beta
            if n_alpha == n_beta:
                raise ValueError("equal N_alpha and N_beta with separate orbitals: embed the "
                                 "system in spin orbitals and use init_trial_spin_orbital")
        self._check(self._lib.afq_init_trial(self._h, sys_id, n_alpha, n_beta, p, dev))
        self.dims[sys_id]["N"] = cols
        if n_alpha != n_beta:
            self.dims[sys_id]["M"] *= 2

    def init_trial_spin_orbital(self, sys_id: int, psi_t):
        """One determinant of spin orbitals (spin factor 1); the system's
        basis must be spin orbitals."""
        p, dev, keep = _arg(psi_t, np.float64)
        N = psi_t.shape[1]
        self._check(self._lib.afq_init_trial_spin_orbital(self._h, sys_id, N, p, dev))
        self.dims[sys_id]["N"] = N

    def init_walkers(self, sys_id: int, n_walkers: int, phi0=None):
        p, dev, keep = _arg(phi0, np.complex128)
        self._check(self._lib.afq_init_walkers(self._h, sys_id, n_walkers, p, dev))
        self.dims[sys_id]["W"] = n_walkers

    # --------------------------------------------------------------- stepping
    def propagate_batch(self, sys_ids, *, tau, n_steps, exp_method=EXP_KRYLOV, exp_order=6,
                        reorth_every=1, precision=PREC_FP64, energy_every=1, e0=None, seed=0,
                        step0=0, fields=None, energies_out=None, schedule=SCHED_AUTO,
                        e0_window=0, pop_every=0, propagator=0, force_bias_at=0):
        ids = [sys_ids] if isinstance(sys_ids, int) else list(sys_ids)
        arr = (ctypes.c_int32 * len(ids))(*ids)
        fp, fdev, fk = _arg(fields, np.float64)
        ep, edev, ek = _arg(energies_out, np.float64)
        if fields is not None and not fdev:
            raise ValueError("fields must be a device tensor")
        if energies_out is not None and not edev:
            raise ValueError("energies_out must be a device tensor")
        prm = PropParams(float(tau), int(exp_method), int(exp_order), int(reorth_every),
                         int(precision), int(n_steps), int(energy_every),
                         math.nan if e0 is None else float(e0), int(seed), int(step0), fp, ep,
                         int(schedule), int(e0_window), int(pop_every), int(propagator),
                         int(force_bias_at))
        self._check(self._lib.afq_propagate_batch(self._h, arr, len(ids), ctypes.byref(prm)))

    def autotune(self, sys_ids, reps: int = 3, **_ignored):
        """Measure and keep the fastest tile shapes of the listed systems."""
        ids = [sys_ids] if isinstance(sys_ids, int) else list(sys_ids)
        arr = (ctypes.c_int32 * len(ids))(*ids)
        self._check(self._lib.afq_autotune(self._h, arr, len(ids), int(reps)))

    def local_energy_batch(self, sys_id: int, eloc_out=None, ell_out=None, precision=PREC_FP64):
        W, G = self.dims[sys_id]["W"], self.dims[sys_id]["G"]
        host = eloc_out is None or not _is_torch(eloc_out)
        if eloc_out is None:
            eloc_out = np.empty(W, dtype=np.complex128)
            if ell_out is True:
                ell_out = np.empty((W, G), dtype=np.complex128)
        ep, edev, _ = _arg(eloc_out, np.complex128)
        lp, ldev, _ = _arg(ell_out if ell_out is not True else None, np.complex128)
        self._check(self._lib.afq_local_energy_batch(self._h, sys_id, int(precision), ep, lp,
                                                     edev))
        if host:
            return (eloc_out, ell_out) if ell_out is not None else eloc_out
        return eloc_out

    def local_energy_batch_noalloc(self, sys_id: int, eloc_out, ell_out=None):
        """FP64 local energies into device tensors, with no device allocation."""
        ep, edev, _ = _arg(eloc_out, np.complex128)
        lp, ldev, _ = _arg(ell_out, np.complex128)
        if not edev or (ell_out is not None and not ldev):
            raise ValueError("the allocation-free local energy writes device tensors")
        self._check(self._lib.afq_local_energy_batch_noalloc(self._h, sys_id, ep, lp))

    def get_walkers(self, sys_id: int):
        d = self.dims[sys_id]
        W, M, N = d["W"], d["M"], d["N"]
        phi = np.empty((W, M, N), dtype=np.complex128)
        wt = np.empty(W)
        lo = np.empty(W, dtype=np.complex128)
        al = np.empty(W, dtype=np.int32)
        self._check(self._lib.afq_get_walkers(self._h, sys_id, phi.ctypes.data, wt.ctypes.data,
                                              lo.ctypes.data, al.ctypes.data, 0))
        return {"phi": phi, "weight": wt, "log_ovlp": lo, "alive": al}

    def set_walkers(self, sys_id: int, phi=None, weight=None):
        p, pdev, pk = _arg(phi, np.complex128)
        w, wdev, wk = _arg(weight, np.float64)
        dev = pdev if phi is not None else wdev
        self._check(self._lib.afq_set_walkers(self._h, sys_id, p, w, dev))

    def fill_fields(self, seed: int, sys_id: int, step: int, out):
        p, dev, _ = _arg(out, np.float64)
        if not dev:
            raise ValueError("fill_fields writes device memory")
        self._check(self._lib.afq_fill_fields(self._h, seed, sys_id, step, out.shape[0],
                                              out.shape[1], p))

    def get_counters(self, sys_id: int):
        out = (ctypes.c_int64 * 5)()
        self._check(self._lib.afq_get_counters(self._h, sys_id, out, 5))
        return {"not_frozen": out[0], "capped_f": out[1], "krylov_breakdowns": out[2],
                "frozen": out[3], "weighted": out[4]}

    def get_e0(self, sys_id: int) -> float:
        v = ctypes.c_double()
        self._check(self._lib.afq_get_e0(self._h, sys_id, ctypes.byref(v)))
        return v.value

    def local_energy_adjoint(self, sys_id: int, dE_dEL, grad_h, grad_L):
        a, adev, _ = _arg(dE_dEL, np.float64)
        h, hdev, _ = _arg(grad_h, np.float64)
        g, gdev, _ = _arg(grad_L, np.float64)
        self._check(self._lib.afq_local_energy_adjoint(self._h, sys_id, a, h, g, hdev))

    def force_bias_adjoint(self, sys_id: int, d_ell, grad_L):
        a, adev, _ = _arg(d_ell, np.complex128)
        g, gdev, _ = _arg(grad_L, np.float64)
        self._check(self._lib.afq_force_bias_adjoint(self._h, sys_id, a, g, gdev))

    def profile(self, enable: bool):
        self._check(self._lib.afq_profile(self._h, int(bool(enable))))

    def profile_read(self):
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._check(self._lib.afq_profile_read(self._h, ms, cnt, n))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(PHASES)}

    def sync(self):
        self._check(self._lib.afq_sync(self._h))
