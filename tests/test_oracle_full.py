"""Pins of the double-time estimator of Eq. (9) without the separable
approximation (oracle/ta_full.c): each segment [t1, t2] of a trajectory
carries the Herman-Kluk prefactor of the trajectory started at (p(t1), q(t1)).

* Harmonic modes with gamma = omega: the segment's prefactor is the pure phase
  exp(-i sum omega (t2 - t1) / 2) = exp(i (phi(t2) - phi(t1))), so Eq. (9)
  reduces exactly to the separable form.
* Harmonic mode with gamma = 2 omega (a squeezed reference state): Herman-Kluk
  is exact for quadratic Hamiltonians, so Eq. (9) gives the exact spectrum,
  sum_n |<n|chi>|^2 times the Dirichlet window, with only even n present:
  |<0|chi>|^2 = 2 sqrt(gamma omega)/(gamma + omega) = 2 sqrt(2)/3 and
  |<2m|chi>|^2 = |<0|chi>|^2 tanh(r)^(2m) (2m)! / (4^m m!^2), tanh r = 1/3.
  The separable form drops |C| >= 1 and misses the total intensity.
* Zero lag: C(t, t) = 1, so R_j(0) = (1/2) sum_c |<chi|z_c>|^2.
* Uncoupled Morse: the separable approximation shifts the zero-point peak by
  several cm^-1 (0.26 % at omega = 3000 cm^-1); Eq. (9) removes the shift.
"""
import math

import numpy as np

from paper_1312_4698_amd import inputs
from tests import _helpers as h


def test_full_reduces_to_separable_when_gamma_is_omega(oracle_mod):
    O = oracle_mod
    prob = inputs.harmonic([2000.0, 3100.0], n_steps=256, dt=10.0, e_max=0.05, n_energies=200)
    p0, q0, lr = O.sample_husimi(prob, 3, 24)
    rf, rs = O.run_full(prob, p0, q0, lr), O.run(prob, p0, q0, lr)
    assert rf.n_good == rs.n_good == 24
    assert np.max(np.abs(rf.spectrum - rs.spectrum)) < 1e-9 * np.max(rs.spectrum)


def _per_trajectory_integrals(prob, lags, lr):
    """Energy integral of each trajectory's term of the full estimator (mean = the estimate)."""
    E = prob.energies()
    tau = np.arange(prob.n_steps + 1)
    ph = np.exp(1j * np.outer(tau, E) * prob.dt)  # [tau][k]
    s = 2.0 * np.real(lags @ ph)                  # [j][k]
    w = np.exp(-lr - prob.F * np.log(2 * np.pi))
    dE = E[1] - E[0]
    return w * s.sum(axis=1) * dE * prob.dt ** 2 / (2 * np.pi * prob.total_time)


def test_full_is_exact_for_a_squeezed_harmonic_reference(oracle_mod):
    O = oracle_mod
    om_cm = 3000.0
    om = om_cm * inputs.HARTREE_PER_CM1
    prob = inputs.harmonic([om_cm], gamma=np.array([2 * om]), n_steps=512, dt=10.0, e_max=0.06, n_energies=300)
    p0, q0, lr = O.sample_husimi(prob, 5, 800)
    rf = O.run_full(prob, p0, q0, lr, want_lags=True)
    rs = O.run(prob, p0, q0, lr)
    E = prob.energies()
    P0 = 2 * math.sqrt(2) / 3
    probs = [(n, P0 * (1 / 3) ** n * math.factorial(n) / (2 ** n * math.factorial(n // 2) ** 2)) for n in (0, 2, 4)]
    ref = sum(P * h.dirichlet_power(E, [om * (n + 0.5)], prob.dt, prob.n_steps)[:, 0] for n, P in probs)
    ref_int = np.trapezoid(ref, E)
    c = _per_trajectory_integrals(prob, rf.lags, lr)
    se = c.std() / math.sqrt(len(c))
    assert abs(c.mean() - np.sum(rf.spectrum) * (E[1] - E[0])) < 1e-9 * abs(c.mean())
    assert abs(c.mean() - np.sum(ref) * (E[1] - E[0])) < 4 * se, (c.mean(), ref_int, se)
    # the separable form loses the prefactor's modulus: on the same trajectories its
    # total is low by far more than the paired difference's standard error
    cs = rs.contrib * (E[1] - E[0]) * prob.dt ** 2 / (2 * np.pi * prob.total_time)
    d = c - cs
    assert d.mean() > 8 * d.std() / math.sqrt(len(d)), (d.mean(), d.std())
    # the n = 2 line at 5 omega / 2 with its squeezed-state weight
    k0, k2 = int(np.argmin(np.abs(E - 0.5 * om))), int(np.argmin(np.abs(E - 2.5 * om)))
    assert abs(rf.spectrum[k2] / rf.spectrum[k0] - ref[k2] / ref[k0]) < 0.15 * ref[k2] / ref[k0]
    assert np.max(np.abs(rf.spectrum - ref)) < 0.05 * np.max(ref)


def test_zero_lag_is_half_the_summed_squared_overlaps(oracle_mod):
    O = oracle_mod
    prob = inputs.morse_quartic(3, 3, n_steps=64, n_energies=64, e_max=0.06)
    p0, q0, lr = O.sample_husimi(prob, 9, 4)
    rf = O.run_full(prob, p0, q0, lr, want_lags=True)
    for j in range(4):
        tr = O.Trajectory(prob, p0[:, j], q0[:, j])
        ov = [abs(O.overlap(prob, tr.state.p, tr.state.q)) ** 2]
        for _ in range(prob.n_steps):
            tr.advance(1)
            ov.append(abs(O.overlap(prob, tr.state.p, tr.state.q)) ** 2)
        assert abs(rf.lags[j, 0] - 0.5 * sum(ov)) < 1e-12 * sum(ov)


def test_full_removes_the_separable_zero_point_shift_for_morse(oracle_mod):
    O = oracle_mod
    om_cm = 3000.0
    om = om_cm * inputs.HARTREE_PER_CM1
    e0 = h.morse_level(om, 0.02, 0)
    prob = inputs.uncoupled_morse([om_cm], n_steps=512, dt=10.0, e_min=e0 - 3e-4, e_max=e0 + 3e-4, n_energies=241)
    p0, q0, lr = O.sample_husimi(prob, 5, 200)
    E = prob.energies()

    def peak(I):
        k = int(np.argmax(I))
        y0, y1, y2 = I[k - 1], I[k], I[k + 1]
        return E[k] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * (E[1] - E[0])

    sep = h.cm(peak(O.run(prob, p0, q0, lr, want_state=False).spectrum) - e0)
    full = h.cm(peak(O.run_full(prob, p0, q0, lr).spectrum) - e0)
    assert sep > 2.5, sep
    assert abs(full) < 2.0, full
