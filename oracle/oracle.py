"""ctypes front end of the plain FP64 CPU oracle (``scivr_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports
this module.  It takes plain numpy arrays (the problem definition and the
initial conditions) and shares no code with the HIP library.

The functions here marshal arguments to the C files, which hold the method's
arithmetic and cite the paper's equations, with one exception: good_weight,
the importance-weighted good count of reading R15 (a few lines of numpy,
documented where it is defined).  precision_probe.c (same library) holds the
binary128 and long-double checks of what the stability monitor measures;
ta_full.c the double-time form of Eq. (9) without the separable approximation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scivr_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "precision_probe.c"), os.path.join(_HERE, "ta_full.c")]
_LIB = os.environ.get("SCIVR_ORACLE_SO") or os.path.join(_HERE, "libscivr_oracle.so")

# Offsets of the scalar part of the per-trajectory state (after p and q).
ST_S, ST_THETA, ST_RPREV, ST_PHI, ST_GOOD, ST_DETM, ST_MAXDEV, ST_STEP, ST_NSCALAR = range(9)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               "-std=gnu11", "-Wall", "-o", tmp, *_SRCS, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


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
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        d = ctypes.c_void_p
        lib.orc_state_size.restype = ctypes.c_int64
        lib.orc_state_size.argtypes = [ctypes.c_int32]
        lib.orc_potential.argtypes = [P, d, d, d, d]
        lib.orc_det_real.restype = ctypes.c_double
        lib.orc_det_real.argtypes = [ctypes.c_int32, d]
        lib.orc_det_complex.argtypes = [ctypes.c_int32, d, d, d, d]
        lib.orc_overlap.argtypes = [P, d, d, d, d]
        lib.orc_prefactor_matrix.argtypes = [P, d, d, d]
        lib.orc_yoshida_coefficients.argtypes = [d, d]
        lib.orc_traj_init.argtypes = [P, d, d, d, d]
        lib.orc_traj_advance.restype = ctypes.c_int
        lib.orc_traj_advance.argtypes = [P, d, ctypes.c_int32, d]
        lib.orc_energy_grid.argtypes = [P, d]
        lib.orc_philox4x64_10.argtypes = [d, d, d]
        lib.orc_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, d]
        lib.orc_sample_husimi.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, d, d, d]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run.argtypes = [P, ctypes.c_int64, d, d, d, d, ctypes.POINTER(ctypes.c_int64), d, d, d,
                                ctypes.c_int32]
        lib.orc_normalise.argtypes = [P, d, ctypes.c_int64, d]
        lib.orc_ta_full_run.restype = ctypes.c_int
        lib.orc_ta_full_run.argtypes = [P, ctypes.c_int64, d, d, d, d, ctypes.POINTER(ctypes.c_int64), d, d]
        lib.orc_monitor_probe.restype = ctypes.c_int
        lib.orc_monitor_probe.argtypes = [P, d, d, ctypes.c_int32, ctypes.c_int32, d]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleProblem:
    """Holds the C struct and keeps the arrays it points to alive."""

    def __init__(self, prob):
        self.prob = prob
        F = int(prob.F)
        self.F = F
        self._arrs = [np.ascontiguousarray(np.asarray(getattr(prob, nm), dtype=np.float64))
                      for nm in ("k_harm", "morse_D", "morse_a", "lam", "gamma", "p_eq", "q_eq")]
        s = _Problem()
        s.F = F
        (s.k_harm, s.morse_D, s.morse_a, s.lam, s.gamma, s.p_eq, s.q_eq) = [a.ctypes.data for a in self._arrs]
        s.dt = float(prob.dt)
        s.n_steps = int(prob.n_steps)
        s.e_min = float(prob.e_min)
        s.e_max = float(prob.e_max)
        s.n_energies = int(prob.n_energies)
        s.det_tol = float(prob.det_tol)
        s.check_every = int(prob.check_every)
        self.struct = s

    @property
    def ref(self):
        return ctypes.byref(self.struct)


def _op(prob) -> OracleProblem:
    return prob if isinstance(prob, OracleProblem) else OracleProblem(prob)


def state_size(F: int) -> int:
    return int(_load().orc_state_size(F))


def potential(prob, q):
    """V, gradient and Hessian at q."""
    op = _op(prob)
    F = op.F
    q = np.ascontiguousarray(q, dtype=np.float64)
    V = np.zeros(1)
    g = np.zeros(F)
    H = np.zeros((F, F))
    _load().orc_potential(op.ref, _ptr(q), _ptr(V), _ptr(g), _ptr(H))
    return float(V[0]), g, H


def det_real(a):
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    return float(_load().orc_det_real(a.shape[0], _ptr(a)))


def det_complex(a):
    re = np.ascontiguousarray(np.real(a), dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(a), dtype=np.float64).copy()
    dr = np.zeros(1)
    di = np.zeros(1)
    _load().orc_det_complex(re.shape[0], _ptr(re), _ptr(im), _ptr(dr), _ptr(di))
    return complex(dr[0], di[0])


def overlap(prob, p, q):
    """<chi|p,q> for the problem's reference state."""
    op = _op(prob)
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    re = np.zeros(1)
    im = np.zeros(1)
    _load().orc_overlap(op.ref, _ptr(p), _ptr(q), _ptr(re), _ptr(im))
    return complex(re[0], im[0])


def prefactor_matrix(prob, M):
    op = _op(prob)
    F = op.F
    M = np.ascontiguousarray(M, dtype=np.float64)
    re = np.zeros((F, F))
    im = np.zeros((F, F))
    _load().orc_prefactor_matrix(op.ref, _ptr(M), _ptr(re), _ptr(im))
    return re + 1j * im


def yoshida_coefficients():
    d = np.zeros(4)
    c = np.zeros(3)
    _load().orc_yoshida_coefficients(_ptr(d), _ptr(c))
    return d, c


@dataclass
class TrajState:
    """Decoded per-trajectory oracle state."""

    p: np.ndarray
    q: np.ndarray
    S: float
    theta: float
    rprev: float
    phi: float
    good: bool
    detM: float
    maxdev: float
    step: int
    M: np.ndarray

    @staticmethod
    def decode(st: np.ndarray, F: int) -> "TrajState":
        b = 2 * F
        return TrajState(p=st[:F].copy(), q=st[F:b].copy(), S=float(st[b + ST_S]), theta=float(st[b + ST_THETA]),
                         rprev=float(st[b + ST_RPREV]), phi=float(st[b + ST_PHI]), good=bool(st[b + ST_GOOD]),
                         detM=float(st[b + ST_DETM]), maxdev=float(st[b + ST_MAXDEV]), step=int(st[b + ST_STEP]),
                         M=st[b + ST_NSCALAR:].reshape(2 * F, 2 * F).copy())


class Trajectory:
    """A single oracle trajectory that can be advanced step by step."""

    def __init__(self, prob, p0, q0):
        self.op = _op(prob)
        F = self.op.F
        self.st = np.zeros(state_size(F))
        amp0 = np.zeros(2)
        _load().orc_traj_init(self.op.ref, _ptr(np.ascontiguousarray(p0, dtype=np.float64)),
                              _ptr(np.ascontiguousarray(q0, dtype=np.float64)), _ptr(self.st), _ptr(amp0))
        self.amp0 = complex(amp0[0], amp0[1])

    def advance(self, n: int) -> np.ndarray:
        amps = np.zeros(2 * n)
        rc = _load().orc_traj_advance(self.op.ref, _ptr(self.st), int(n), _ptr(amps))
        if rc != 0:
            raise MemoryError("oracle trajectory advance failed")
        return amps[0::2] + 1j * amps[1::2]

    @property
    def state(self) -> TrajState:
        return TrajState.decode(self.st, self.op.F)


def energy_grid(prob) -> np.ndarray:
    op = _op(prob)
    E = np.zeros(op.struct.n_energies)
    _load().orc_energy_grid(op.ref, _ptr(E))
    return E


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed: int, index: int, count: int) -> np.ndarray:
    out = np.zeros(count)
    _load().orc_normals(ctypes.c_uint64(seed), ctypes.c_uint64(index), int(count), _ptr(out))
    return out


def sample_husimi(prob, seed: int, n: int, first_index: int = 0):
    """Husimi samples: (p0 [F][n], q0 [F][n], logrho [n])."""
    op = _op(prob)
    F = op.F
    p0 = np.zeros((F, n))
    q0 = np.zeros((F, n))
    lr = np.zeros(n)
    _load().orc_sample_husimi(op.ref, ctypes.c_uint64(seed), ctypes.c_uint64(first_index), int(n),
                              _ptr(p0), _ptr(q0), _ptr(lr))
    return p0, q0, lr


@dataclass
class RunResult:
    spec_sum: np.ndarray
    n_good: int
    n_total: int
    spectrum: np.ndarray
    final_state: Optional[np.ndarray]
    contrib: Optional[np.ndarray]
    amps: Optional[np.ndarray]
    F: int
    good_weight: float = 0.0

    def state(self, j: int) -> TrajState:
        return TrajState.decode(self.final_state[j], self.F)


def run(prob, p0, q0, logrho, *, want_state: bool = True, want_contrib: bool = True,
        want_amps: bool = False, n_threads: int = 0) -> RunResult:
    """Run the whole estimator over the given initial conditions."""
    op = _op(prob)
    F = op.F
    K = op.struct.n_energies
    p0 = np.ascontiguousarray(p0, dtype=np.float64)
    q0 = np.ascontiguousarray(q0, dtype=np.float64)
    logrho = np.ascontiguousarray(logrho, dtype=np.float64)
    n = int(logrho.shape[0])
    assert p0.shape == (F, n) and q0.shape == (F, n)
    nt = op.struct.n_steps + 1
    spec = np.zeros(K)
    ng = ctypes.c_int64(0)
    fs = np.zeros((n, state_size(F)))  # always kept: the good flags enter the normalisation
    cb = np.zeros(n) if want_contrib else None
    am = np.zeros((n, nt, 2)) if want_amps else None
    rc = _load().orc_run(op.ref, n, _ptr(p0), _ptr(q0), _ptr(logrho), _ptr(spec), ctypes.byref(ng),
                         _ptr(fs), _ptr(cb), _ptr(am), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle run failed to allocate")
    good = fs[:, 2 * F + ST_GOOD] != 0.0
    gw = good_weight(prob, p0, q0, logrho, good)
    I = np.zeros(K)
    _load().orc_normalise(op.ref, _ptr(spec), ng.value, _ptr(I))
    if ng.value > 0:
        I *= ng.value / gw
    amps = None if am is None else am[..., 0] + 1j * am[..., 1]
    return RunResult(spec_sum=spec, n_good=int(ng.value), n_total=n, spectrum=I,
                     final_state=fs if want_state else None, contrib=cb, amps=amps, F=F, good_weight=gw)


def good_weight(prob, p0, q0, logrho, good) -> float:
    """Sum over good trajectories of r_j = Husimi density / sampling density.

    Eq. (11) divides by n_good, the number of good trajectories among points
    drawn from the Husimi density, i.e. a Monte Carlo count of the good part
    of that density.  Drawn from another density rho (the learned proposal),
    the same count is estimated by sum_j good_j H(z_j) / rho(z_j); for Husimi
    points every ratio is 1 and the sum is n_good.
    """
    g = np.asarray(prob.gamma, dtype=np.float64)[:, None]
    xi2 = g * (np.asarray(q0) - np.asarray(prob.q_eq)[:, None]) ** 2
    eta2 = (np.asarray(p0) - np.asarray(prob.p_eq)[:, None]) ** 2 / g
    F = len(prob.gamma)
    log_h = -F * np.log(2.0 * np.pi) - 0.5 * np.sum(xi2 + eta2, axis=0)
    r = np.exp(log_h - np.asarray(logrho, dtype=np.float64))
    return float(np.sum(r[np.asarray(good, dtype=bool)]))


def monitor_probe(prob, p0, q0, n_steps: int, every: int) -> dict:
    """What the stability monitor measures along one trajectory (precision_probe.c).

    Every `every` steps: ||M||_F of the FP64 trajectory, |det(M)^2 - 1| of its
    M by FP64 elimination (the monitor) and by binary128 elimination of the
    same stored matrix, |det^2 - 1| of M integrated in long double from the
    same point, and ||M^T J M - J||_F / ||M||_F^2 of the FP64 M."""
    op = _op(prob)
    rows = n_steps // every
    out = np.zeros((rows, 5))
    rc = _load().orc_monitor_probe(op.ref, _ptr(np.ascontiguousarray(p0, dtype=np.float64)),
                                   _ptr(np.ascontiguousarray(q0, dtype=np.float64)), int(n_steps), int(every),
                                   _ptr(out))
    if rc != 0:
        raise MemoryError("monitor probe failed to allocate")
    return {"step": every * np.arange(1, rows + 1), "normM": out[:, 0], "dev_fp64": out[:, 1],
            "dev_same_M_q": out[:, 2], "dev_longdouble": out[:, 3], "defect": out[:, 4]}


@dataclass
class FullResult:
    spectrum: np.ndarray
    spec_sum: np.ndarray
    n_good: int
    good: np.ndarray
    lags: Optional[np.ndarray]


def run_full(prob, p0, q0, logrho, want_lags: bool = False) -> FullResult:
    """The double-time estimator of Eq. (9) with each segment's Herman-Kluk
    prefactor (ta_full.c), normalised as Eq. (11) (good count of reading R15)."""
    op = _op(prob)
    F, K, ns = op.F, op.struct.n_energies, op.struct.n_steps
    p0 = np.ascontiguousarray(p0, dtype=np.float64)
    q0 = np.ascontiguousarray(q0, dtype=np.float64)
    logrho = np.ascontiguousarray(logrho, dtype=np.float64)
    n = int(logrho.shape[0])
    spec = np.zeros(K)
    ng = ctypes.c_int64(0)
    good = np.zeros(n)
    lags = np.zeros((n, ns + 1, 2)) if want_lags else None
    rc = _load().orc_ta_full_run(op.ref, n, _ptr(p0), _ptr(q0), _ptr(logrho), _ptr(spec), ctypes.byref(ng),
                                 _ptr(good), _ptr(lags))
    if rc != 0:
        raise MemoryError("full-form oracle failed to allocate")
    g = good != 0
    gw = good_weight(prob, p0, q0, logrho, g)
    I = np.zeros(K)
    if ng.value > 0:
        _load().orc_normalise(op.ref, _ptr(spec), ng.value, _ptr(I))
        I *= ng.value / gw
    return FullResult(spectrum=I, spec_sum=spec, n_good=int(ng.value), good=g,
                      lags=None if lags is None else lags[..., 0] + 1j * lags[..., 1])
