"""Seeded synthetic problem definitions (potential parameters and run settings).

This module only builds the *inputs* of the TA-SC-IVR power-spectrum method:
the potential-energy surface, the reference coherent state, the time grid
and the energy grid.  It holds none of the method's arithmetic (no sampling,
no integration, no prefactor, no Fourier sum); both the HIP library and the
CPU oracle receive the arrays it returns.

The potential family stands in for the paper's fitted molecular surfaces
(Results section, and its uncoupled-Morse control in the speed-up-versus-F
discussion): in mass-weighted normal coordinates (atomic units, hbar = 1)

    V(q) = sum_i [ k_i q_i^2 / 2 + D_i (1 - exp(-a_i q_i))^2 ]
           + sum_{i<j} lambda_ij q_i^2 q_j^2

with harmonic frequencies omega_i drawn uniformly in [1500, 4000] cm^-1,
Morse anharmonicity x_e = omega/(4 D) = 0.02 and omega = a sqrt(2 D), and
lambda_ij = eps_ij (omega_i omega_j)^(3/2), eps_ij uniform in [0, 0.01].
The quadratic term k_i is zero for that family; it exists so that exactly
harmonic and mixed problems can be posed for closed-form checks.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

CM1_PER_HARTREE = 219474.63
HARTREE_PER_CM1 = 1.0 / CM1_PER_HARTREE

PRECISION_FP64 = 0
PRECISION_MIXED = 1


@dataclasses.dataclass
class Problem:
    """A complete problem statement: potential, reference state, grids.

    Arrays are float64, length F (``lam`` is F x F symmetric with a zero
    diagonal).  ``omega`` is informational (the harmonic frequencies used to
    build the potential); the method itself reads k, D, a, lam, gamma,
    p_eq and q_eq.
    """

    F: int
    k_harm: np.ndarray
    morse_D: np.ndarray
    morse_a: np.ndarray
    lam: np.ndarray
    gamma: np.ndarray
    p_eq: np.ndarray
    q_eq: np.ndarray
    dt: float
    n_steps: int
    e_min: float
    e_max: float
    n_energies: int
    det_tol: float = 1e-6
    check_every: int = 1
    precision: int = PRECISION_FP64
    omega: Optional[np.ndarray] = None
    name: str = ""

    def __post_init__(self):
        F = int(self.F)
        for nm in ("k_harm", "morse_D", "morse_a", "gamma", "p_eq", "q_eq"):
            arr = np.ascontiguousarray(np.asarray(getattr(self, nm), dtype=np.float64).reshape(F))
            setattr(self, nm, arr)
        lam = np.ascontiguousarray(np.asarray(self.lam, dtype=np.float64).reshape(F, F))
        self.lam = lam
        if self.omega is not None:
            self.omega = np.ascontiguousarray(np.asarray(self.omega, dtype=np.float64).reshape(F))

    @property
    def n_times(self) -> int:
        return self.n_steps + 1

    @property
    def total_time(self) -> float:
        return self.n_steps * self.dt

    def energies(self) -> np.ndarray:
        """The equally spaced energy axis E_1 = e_min ... E_k = e_max."""
        return np.linspace(self.e_min, self.e_max, self.n_energies)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def morse_params(omega: np.ndarray, x_e: float = 0.02):
    """Morse D and a such that omega = a sqrt(2 D) and x_e = omega / (4 D)."""
    omega = np.asarray(omega, dtype=np.float64)
    D = omega / (4.0 * x_e)
    a = np.sqrt(2.0 * x_e * omega)
    return D, a


def coupling_matrix(omega: np.ndarray, eps_upper: np.ndarray) -> np.ndarray:
    """Symmetric lambda with lambda_ij = eps_ij (omega_i omega_j)^(3/2), zero diagonal.

    ``eps_upper`` lists eps_ij for i < j in lexicographic order.
    """
    F = len(omega)
    lam = np.zeros((F, F))
    n = 0
    for i in range(F):
        for j in range(i + 1, F):
            v = eps_upper[n] * (omega[i] * omega[j]) ** 1.5
            lam[i, j] = v
            lam[j, i] = v
            n += 1
    return lam


def morse_quartic(F: int, seed_pot: Optional[int] = None, *, n_steps: int = 2048, dt: float = 10.0,
                  e_min: float = 0.0, e_max: float = 0.05, n_energies: int = 512,
                  x_e: float = 0.02, eps_max: float = 0.01,
                  omega_cm1=(1500.0, 4000.0), p_eq=None, q_eq=None,
                  precision: int = PRECISION_FP64, det_tol: float = 1e-6,
                  check_every: int = 1, name: str = "") -> Problem:
    """The seeded Morse + quartic-coupling family.

    numpy.random.default_rng(seed_pot) draws omega_i ~ U[1500, 4000] cm^-1
    (F draws, converted to hartree), then eps_ij ~ U[0, eps_max] for i < j in
    lexicographic order.  gamma = omega; the reference state sits at
    (p_eq, q_eq) = (0, 0) unless given.
    """
    if seed_pot is None:
        seed_pot = F
    rng = np.random.default_rng(seed_pot)
    omega = rng.uniform(omega_cm1[0], omega_cm1[1], size=F) * HARTREE_PER_CM1
    eps = rng.uniform(0.0, eps_max, size=F * (F - 1) // 2)
    D, a = morse_params(omega, x_e)
    lam = coupling_matrix(omega, eps)
    z = np.zeros(F)
    return Problem(F=F, k_harm=z.copy(), morse_D=D, morse_a=a, lam=lam, gamma=omega.copy(),
                   p_eq=z.copy() if p_eq is None else p_eq, q_eq=z.copy() if q_eq is None else q_eq,
                   dt=dt, n_steps=n_steps, e_min=e_min, e_max=e_max, n_energies=n_energies,
                   det_tol=det_tol, check_every=check_every, precision=precision,
                   omega=omega, name=name or f"morse_quartic_F{F}_seed{seed_pot}")


def harmonic(omega_cm1, *, gamma=None, n_steps: int = 1024, dt: float = 10.0,
             e_min: float = 0.0, e_max: float = 0.05, n_energies: int = 512,
             p_eq=None, q_eq=None, name: str = "harmonic") -> Problem:
    """Uncoupled harmonic oscillators V = sum_i omega_i^2 q_i^2 / 2."""
    omega = np.atleast_1d(np.asarray(omega_cm1, dtype=np.float64)) * HARTREE_PER_CM1
    F = len(omega)
    z = np.zeros(F)
    return Problem(F=F, k_harm=omega ** 2, morse_D=z.copy(), morse_a=np.ones(F), lam=np.zeros((F, F)),
                   gamma=omega.copy() if gamma is None else gamma,
                   p_eq=z.copy() if p_eq is None else p_eq, q_eq=z.copy() if q_eq is None else q_eq,
                   dt=dt, n_steps=n_steps, e_min=e_min, e_max=e_max, n_energies=n_energies,
                   omega=omega, name=name)


def uncoupled_morse(omega_cm1, *, x_e: float = 0.02, n_steps: int = 2048, dt: float = 10.0,
                    e_min: float = 0.0, e_max: float = 0.05, n_energies: int = 512,
                    p_eq=None, q_eq=None, name: str = "uncoupled_morse") -> Problem:
    """Independent Morse oscillators (the paper's synthetic control)."""
    omega = np.atleast_1d(np.asarray(omega_cm1, dtype=np.float64)) * HARTREE_PER_CM1
    F = len(omega)
    D, a = morse_params(omega, x_e)
    z = np.zeros(F)
    return Problem(F=F, k_harm=z.copy(), morse_D=D, morse_a=a, lam=np.zeros((F, F)), gamma=omega.copy(),
                   p_eq=z.copy() if p_eq is None else p_eq, q_eq=z.copy() if q_eq is None else q_eq,
                   dt=dt, n_steps=n_steps, e_min=e_min, e_max=e_max, n_energies=n_energies,
                   omega=omega, name=name)


# The workloads: sizes, grids and precision of each run (F=30 FP64 is the reference of the F=30 mixed run).
WORKLOADS = {
    "F2_fp64": dict(F=2, n_traj=1024, n_steps=2048, dt=10.0, e_min=0.0, e_max=0.05, n_energies=512,
                    precision=PRECISION_FP64),
    "F6_fp64": dict(F=6, n_traj=65536, n_steps=4096, dt=10.0, e_min=0.0, e_max=0.1, n_energies=2048,
                    precision=PRECISION_FP64),
    "F9_mixed": dict(F=9, n_traj=262144, n_steps=4096, dt=10.0, e_min=0.0, e_max=0.1, n_energies=2048,
                     precision=PRECISION_MIXED),
    "F9_fp64": dict(F=9, n_traj=262144, n_steps=4096, dt=10.0, e_min=0.0, e_max=0.1, n_energies=2048,
                    precision=PRECISION_FP64),
    "F30_mixed": dict(F=30, n_traj=131072, n_steps=8192, dt=10.0, e_min=0.0, e_max=0.2, n_energies=4096,
                      precision=PRECISION_MIXED),
    "F30_fp64": dict(F=30, n_traj=131072, n_steps=8192, dt=10.0, e_min=0.0, e_max=0.2, n_energies=4096,
                     precision=PRECISION_FP64),
}


def workload(name: str, **override):
    """Problem and trajectory count of a named workload (seed_pot = F)."""
    cfg = dict(WORKLOADS[name])
    cfg.update(override)
    n_traj = cfg.pop("n_traj")
    F = cfg.pop("F")
    seed_pot = cfg.pop("seed_pot", F)
    prob = morse_quartic(F, seed_pot, name=name, **cfg)
    return prob, n_traj


__all__ = [
    "Problem", "morse_params", "coupling_matrix", "morse_quartic", "harmonic", "uncoupled_morse",
    "WORKLOADS", "workload", "CM1_PER_HARTREE", "HARTREE_PER_CM1", "PRECISION_FP64", "PRECISION_MIXED",
]
