"""Thin ctypes binding of ``libscivr.so`` (the C ABI in include/scivr.h).

Only argument marshalling lives here: every step of the method runs in the
library's HIP kernels.  Streams may be given as a ``torch.cuda.Stream``, a
raw ``hipStream_t`` integer, or None (the legacy default stream); device
pointers may be given as torch tensors (their ``data_ptr``) or integers.

The library must have been built (``python -m paper_1312_4698_amd.build``);
importing this module on a machine without it raises immediately, there is no
fallback path.

PyTorch ships its own HIP runtime beside the system one the library links.
When torch tensors or streams are passed in, initialise torch's GPU runtime
(``torch.cuda.init()`` or any torch GPU call) before the first library call:
the two runtimes share the device in that order.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .inputs import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscivr.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOGOOD, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
KERNEL_KINDS = ("sample", "trajectory", "fourier", "reduce", "flow")
F_MAX = 32

_STATUS = {EINVAL: "SCIVR_EINVAL", ENOMEM: "SCIVR_ENOMEM", EDEVICE: "SCIVR_EDEVICE", ESTATE: "SCIVR_ESTATE",
           ENOGOOD: "SCIVR_ENOGOOD", EUNSUPPORTED: "SCIVR_EUNSUPPORTED"}

# Every symbol the header declares.
EXPORTED = (
    "scivr_abi_version", "scivr_create", "scivr_destroy", "scivr_last_error", "scivr_sample_husimi",
    "scivr_set_initial", "scivr_propagate", "scivr_set_stop_flagged", "scivr_accumulate_spectrum", "scivr_accumulate_spectrum_fft",
    "scivr_accumulate_spectrum_fft_noalloc", "scivr_accumulate_spectrum_full", "scivr_read_lags",
    "scivr_read_spectrum", "scivr_read_totals", "scivr_set_references", "scivr_read_spectrum_ref",
    "scivr_reset_spectrum", "scivr_batch_info", "scivr_read_initial", "scivr_read_state",
    "scivr_read_amplitudes", "scivr_read_contributions", "scivr_timing_enable", "scivr_kernel_times",
    "scivr_flow_create", "scivr_flow_destroy", "scivr_flow_param_count", "scivr_flow_set_params",
    "scivr_flow_get_params", "scivr_flow_train", "scivr_flow_train_on_batch", "scivr_flow_loss_grad",
    "scivr_flow_log_density", "scivr_flow_sample",
)


class ScivrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [
        ("F", ctypes.c_int32),
        ("k_harm", ctypes.c_void_p),
        ("morse_D", ctypes.c_void_p),
        ("morse_a", ctypes.c_void_p),
        ("lam", ctypes.c_void_p),
        ("gamma", ctypes.c_void_p),
        ("p_eq", ctypes.c_void_p),
        ("q_eq", ctypes.c_void_p),
        ("dt", ctypes.c_double),
        ("n_steps", ctypes.c_int32),
        ("e_min", ctypes.c_double),
        ("e_max", ctypes.c_double),
        ("n_energies", ctypes.c_int32),
        ("det_tol", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_traj", ctypes.c_int64),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1312_4698_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    v = ctypes.c_void_p
    i32, i64, u64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sigs = {
        "scivr_abi_version": (i32, []),
        "scivr_create": (i32, [ctypes.POINTER(_Problem), i32, ctypes.POINTER(v)]),
        "scivr_destroy": (None, [v]),
        "scivr_last_error": (ctypes.c_char_p, [v]),
        "scivr_sample_husimi": (i32, [v, u64, u64, i64, v]),
        "scivr_set_initial": (i32, [v, i64, v, v, v, i32, v]),
        "scivr_propagate": (i32, [v, i32, i32, v]),
        "scivr_accumulate_spectrum": (i32, [v, v]),
        "scivr_accumulate_spectrum_fft": (i32, [v, v]),
        "scivr_accumulate_spectrum_fft_noalloc": (i32, [v, v]),
        "scivr_accumulate_spectrum_full": (i32, [v, v]),
        "scivr_read_lags": (i32, [v, v]),
        "scivr_read_totals": (i32, [v, v, ctypes.POINTER(d), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "scivr_read_spectrum": (i32, [v, v, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "scivr_read_spectrum_ref": (i32, [v, i32, v, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "scivr_set_references": (i32, [v, i32, v, v]),
        "scivr_set_stop_flagged": (i32, [v, i32]),
        "scivr_reset_spectrum": (i32, [v, v]),
        "scivr_batch_info": (i32, [v, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "scivr_read_initial": (i32, [v, v, v, v]),
        "scivr_read_state": (i32, [v, v, v, v, v, v, v, v, v]),
        "scivr_read_amplitudes": (i32, [v, i64, i64, v]),
        "scivr_read_contributions": (i32, [v, v]),
        "scivr_timing_enable": (i32, [v, i32]),
        "scivr_kernel_times": (i32, [v, v, v]),
        "scivr_flow_create": (i32, [v, i32, i32, u64, ctypes.POINTER(v)]),
        "scivr_flow_destroy": (None, [v]),
        "scivr_flow_param_count": (i64, [v]),
        "scivr_flow_set_params": (i32, [v, v, i64, i32, v]),
        "scivr_flow_get_params": (i32, [v, v, i64]),
        "scivr_flow_train": (i32, [v, i64, v, v, v, i32, i32, i32, ctypes.c_float, v, ctypes.POINTER(d)]),
        "scivr_flow_train_on_batch": (i32, [v, i32, i32, ctypes.c_float, v, ctypes.POINTER(d)]),
        "scivr_flow_loss_grad": (i32, [v, i64, v, v, v, i32, ctypes.POINTER(d), v]),
        "scivr_flow_log_density": (i32, [v, i64, v, v, i32, i32, v, v]),
        "scivr_flow_sample": (i32, [v, u64, u64, i64, d, d, ctypes.POINTER(d), ctypes.POINTER(i32), v]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)  # torch.cuda.Stream


def _dptr(x) -> int:
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """One problem and its device buffers (``scivr_ctx``)."""

    def __init__(self, prob: Problem, max_traj: int, device: int = 0):
        lib = load()
        self.prob = prob
        self.F = int(prob.F)
        self.max_traj = int(max_traj)
        self._keep = [np.ascontiguousarray(np.asarray(getattr(prob, nm), dtype=np.float64))
                      for nm in ("k_harm", "morse_D", "morse_a", "lam", "gamma", "p_eq", "q_eq")]
        s = _Problem()
        s.F = self.F
        (s.k_harm, s.morse_D, s.morse_a, s.lam, s.gamma, s.p_eq, s.q_eq) = [a.ctypes.data for a in self._keep]
        s.dt = float(prob.dt)
        s.n_steps = int(prob.n_steps)
        s.e_min = float(prob.e_min)
        s.e_max = float(prob.e_max)
        s.n_energies = int(prob.n_energies)
        s.det_tol = float(prob.det_tol)
        s.check_every = int(prob.check_every)
        s.precision = int(prob.precision)
        s.max_traj = self.max_traj
        self._struct = s
        h = ctypes.c_void_p()
        st = lib.scivr_create(ctypes.byref(s), int(device), ctypes.byref(h))
        if st != OK:
            raise ScivrError(st, "scivr_create failed")
        self._h = h
        self._lib = lib

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None):
            self._lib.scivr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int, allow=()):
        if st != OK and st not in allow:
            raise ScivrError(st, self._lib.scivr_last_error(self._h).decode())
        return st

    # -- the method --
    def sample_husimi(self, seed: int, n_traj: int, first_index: int = 0, stream=None):
        self._check(self._lib.scivr_sample_husimi(self._h, int(seed), int(first_index), int(n_traj),
                                                  _stream(stream)))

    def set_initial(self, p0, q0, log_density, stream=None):
        """Initial conditions [F][n] from numpy (host) or torch tensors on the GPU (device)."""
        if isinstance(p0, np.ndarray):
            p0 = np.ascontiguousarray(p0, dtype=np.float64)
            q0 = np.ascontiguousarray(q0, dtype=np.float64)
            lr = np.ascontiguousarray(log_density, dtype=np.float64)
            n = lr.shape[0]
            assert p0.shape == (self.F, n) and q0.shape == (self.F, n)
            self._check(self._lib.scivr_set_initial(self._h, n, _np_ptr(p0), _np_ptr(q0), _np_ptr(lr), MEM_HOST,
                                                    _stream(stream)))
        else:
            n = int(log_density.shape[0])
            assert tuple(p0.shape) == (self.F, n) and p0.is_contiguous() and q0.is_contiguous()
            self._check(self._lib.scivr_set_initial(self._h, n, _dptr(p0), _dptr(q0), _dptr(log_density),
                                                    MEM_DEVICE, _stream(stream)))

    def propagate(self, step_begin: int = 0, step_end: Optional[int] = None, stream=None):
        if step_end is None:
            step_end = self.prob.n_steps
        self._check(self._lib.scivr_propagate(self._h, int(step_begin), int(step_end), _stream(stream)))

    def accumulate(self, stream=None):
        self._check(self._lib.scivr_accumulate_spectrum(self._h, _stream(stream)))

    def accumulate_fft(self, stream=None):
        """The batch's spectrum by the exact FFT-autocorrelation form (``scivr_accumulate_spectrum_fft``)."""
        self._check(self._lib.scivr_accumulate_spectrum_fft(self._h, _stream(stream)))

    def accumulate_fft_noalloc(self, stream=None):
        """The same, with the library's static scratch (``scivr_accumulate_spectrum_fft_noalloc``)."""
        self._check(self._lib.scivr_accumulate_spectrum_fft_noalloc(self._h, _stream(stream)))

    def accumulate_full(self, stream=None):
        """The batch's spectrum by the double-time form of Eq. (9) (``scivr_accumulate_spectrum_full``)."""
        self._check(self._lib.scivr_accumulate_spectrum_full(self._h, _stream(stream)))

    def read_lags(self):
        """Lag sums R_j(tau) [n][n_steps + 1] (complex) of the last double-time accumulation."""
        n, _ = self.batch_info()
        R = np.zeros((n, self.prob.n_steps + 1, 2))
        self._check(self._lib.scivr_read_lags(self._h, _np_ptr(R)))
        return R[..., 0] + 1j * R[..., 1]

    def read_spectrum(self, ref: int = 0):
        """(I [K], n_good, n_total) of reference state `ref` (0: the problem's chi); I is zero when n_good == 0."""
        I = np.zeros(self.prob.n_energies)
        ng = ctypes.c_int64()
        nt = ctypes.c_int64()
        if ref == 0:
            st = self._lib.scivr_read_spectrum(self._h, _np_ptr(I), ctypes.byref(ng), ctypes.byref(nt))
        else:
            st = self._lib.scivr_read_spectrum_ref(self._h, int(ref), _np_ptr(I), ctypes.byref(ng), ctypes.byref(nt))
        self._check(st, allow=(ENOGOOD,))
        return I, int(ng.value), int(nt.value)

    def set_stop_flagged(self, enable: bool = True):
        """Stop integrating trajectories once the stability monitor flags them (F > 16)."""
        self._check(self._lib.scivr_set_stop_flagged(self._h, 1 if enable else 0))

    def set_references(self, p_eq, q_eq):
        """Further reference states [n_extra][F] of the problem's widths, fed by every later batch."""
        p = np.ascontiguousarray(np.reshape(p_eq, (-1, self.F)), dtype=np.float64)
        q = np.ascontiguousarray(np.reshape(q_eq, (-1, self.F)), dtype=np.float64)
        self._check(self._lib.scivr_set_references(self._h, p.shape[0], _np_ptr(p), _np_ptr(q)))

    def read_totals(self):
        """Raw running sums: (total [K], good weight G, n_good, n_total)."""
        tot = np.zeros(self.prob.n_energies)
        gw = ctypes.c_double()
        ng = ctypes.c_int64()
        nt = ctypes.c_int64()
        self._check(self._lib.scivr_read_totals(self._h, _np_ptr(tot), ctypes.byref(gw), ctypes.byref(ng),
                                                ctypes.byref(nt)))
        return tot, float(gw.value), int(ng.value), int(nt.value)

    def reset_spectrum(self, stream=None):
        self._check(self._lib.scivr_reset_spectrum(self._h, _stream(stream)))

    def run(self, seed: int, n_traj: int, first_index: int = 0, stream=None):
        """Sample, propagate and accumulate one batch."""
        self.sample_husimi(seed, n_traj, first_index, stream)
        self.propagate(0, self.prob.n_steps, stream)
        self.accumulate(stream)

    # -- inspection --
    def batch_info(self):
        n = ctypes.c_int64()
        s = ctypes.c_int32()
        self._check(self._lib.scivr_batch_info(self._h, ctypes.byref(n), ctypes.byref(s)))
        return int(n.value), int(s.value)

    def read_initial(self):
        n, _ = self.batch_info()
        p0 = np.zeros((self.F, n))
        q0 = np.zeros((self.F, n))
        lr = np.zeros(n)
        self._check(self._lib.scivr_read_initial(self._h, _np_ptr(p0), _np_ptr(q0), _np_ptr(lr)))
        return p0, q0, lr

    def read_state(self, want_M: bool = True):
        """Final state of the batch; without want_M the monodromy matrices are not copied."""
        n, _ = self.batch_info()
        F = self.F
        out = dict(p=np.zeros((F, n)), q=np.zeros((F, n)), S=np.zeros(n), phi=np.zeros(n),
                   M=np.zeros((n, 2 * F, 2 * F)) if want_M else None, good=np.zeros(n, dtype=np.uint8),
                   detM=np.zeros(n), maxdev=np.zeros(n))
        self._check(self._lib.scivr_read_state(self._h, *[_np_ptr(out[k]) for k in
                                                          ("p", "q", "S", "phi", "M", "good", "detM", "maxdev")]))
        return out

    def read_amplitudes(self, j0: int, count: int):
        nt = self.prob.n_steps + 1
        a = np.zeros((count, nt, 2))
        self._check(self._lib.scivr_read_amplitudes(self._h, int(j0), int(count), _np_ptr(a)))
        return a[..., 0] + 1j * a[..., 1]

    def read_contributions(self):
        n, _ = self.batch_info()
        c = np.zeros(n)
        self._check(self._lib.scivr_read_contributions(self._h, _np_ptr(c)))
        return c

    def timing(self, on: bool = True):
        self._check(self._lib.scivr_timing_enable(self._h, 1 if on else 0))

    def kernel_times(self):
        """{kind: (launches, total ms)} since timing was enabled or last read."""
        cnt = np.zeros(len(KERNEL_KINDS), dtype=np.int64)
        ms = np.zeros(len(KERNEL_KINDS))
        self._check(self._lib.scivr_kernel_times(self._h, _np_ptr(cnt), _np_ptr(ms)))
        return {k: (int(cnt[i]), float(ms[i])) for i, k in enumerate(KERNEL_KINDS)}


class Flow:
    """Learned importance-sampling proposal bound to one context (``scivr_flow``)."""

    def __init__(self, ctx: Context, n_layers: int = 4, width: int = 128, seed: int = 0):
        self.ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        st = self._lib.scivr_flow_create(ctx._h, int(n_layers), int(width), int(seed), ctypes.byref(h))
        if st != OK:
            raise ScivrError(st, self._lib.scivr_last_error(ctx._h).decode())
        self._h = h
        self.n_layers, self.width = int(n_layers), int(width)
        self.n_params = int(self._lib.scivr_flow_param_count(h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.scivr_flow_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        return self.ctx._check(st)

    @staticmethod
    def _points(p0, q0, c=None):
        p0 = np.ascontiguousarray(p0, dtype=np.float64)
        q0 = np.ascontiguousarray(q0, dtype=np.float64)
        assert p0.shape == q0.shape and p0.ndim == 2
        cc = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        return p0, q0, cc

    def set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32)
        assert a.size == self.n_params
        self._check(self._lib.scivr_flow_set_params(self._h, _np_ptr(a), a.size, MEM_HOST, None))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(self._lib.scivr_flow_get_params(self._h, _np_ptr(a), a.size))
        return a

    def train(self, p0, q0, c, epochs: int, batch: int, lr: float, stream=None) -> float:
        p0, q0, c = self._points(p0, q0, c)
        loss = ctypes.c_double()
        self._check(self._lib.scivr_flow_train(self._h, p0.shape[1], _np_ptr(p0), _np_ptr(q0), _np_ptr(c), MEM_HOST,
                                               int(epochs), int(batch), float(lr), _stream(stream),
                                               ctypes.byref(loss)))
        return float(loss.value)

    def train_on_batch(self, epochs: int, batch: int, lr: float, stream=None) -> float:
        loss = ctypes.c_double()
        self._check(self._lib.scivr_flow_train_on_batch(self._h, int(epochs), int(batch), float(lr), _stream(stream),
                                                        ctypes.byref(loss)))
        return float(loss.value)

    def loss_grad(self, p0, q0, c):
        p0, q0, c = self._points(p0, q0, c)
        loss = ctypes.c_double()
        g = np.zeros(self.n_params, dtype=np.float32)
        self._check(self._lib.scivr_flow_loss_grad(self._h, p0.shape[1], _np_ptr(p0), _np_ptr(q0), _np_ptr(c),
                                                   MEM_HOST, ctypes.byref(loss), _np_ptr(g)))
        return float(loss.value), g

    def log_density(self, p0, q0, bf16: bool = False):
        """(log q [n], u [n][2F]) of the flow alone."""
        p0, q0, _ = self._points(p0, q0)
        n = p0.shape[1]
        lq = np.zeros(n)
        u = np.zeros((n, 2 * self.ctx.F), dtype=np.float32)
        self._check(self._lib.scivr_flow_log_density(self._h, n, _np_ptr(p0), _np_ptr(q0), MEM_HOST,
                                                     1 if bf16 else 0, _np_ptr(lq), _np_ptr(u)))
        return lq, u

    def sample(self, seed: int, n_traj: int, first_index: int = 0, alpha: float = 0.1, min_ess_frac: float = 0.1,
               stream=None):
        """Fill the context's batch from the mixture; returns (ess_frac, used_flow)."""
        ess = ctypes.c_double()
        used = ctypes.c_int32()
        self._check(self._lib.scivr_flow_sample(self._h, int(seed), int(first_index), int(n_traj), float(alpha),
                                                float(min_ess_frac), ctypes.byref(ess), ctypes.byref(used),
                                                _stream(stream)))
        return float(ess.value), bool(used.value)


def abi_version() -> int:
    return int(load().scivr_abi_version())
