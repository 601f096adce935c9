"""Several reference states on one trajectory batch (the paper's "different
coherent state combinations" in Results and discussion), on the oracle.

One batch is drawn from the Husimi density of chi_0; the spectrum of another
coherent state chi_m of the same widths comes from the same trajectories with
chi_m in the overlaps <chi_m|z_t>, the same weights w_j = 1/((2 pi)^F rho(z_j))
and the good count estimated with chi_m's Husimi density, sum_j good_j
H_m(z_j)/rho(z_j) (reading R15).  For uncoupled harmonic modes with
gamma = omega the spectrum of a displaced chi is known in closed form: the
levels sum_i omega_i (n_i + 1/2) with Poisson weights of mean |alpha_i|^2 =
(gamma_i q_eq,i^2 + p_eq,i^2 / gamma_i) / 2, each broadened by the Dirichlet
window of the finite time sum."""
import math

import numpy as np

from paper_1312_4698_amd import inputs
from tests import _helpers as h


def _poisson_spectrum(prob, om, p_eq, q_eq, E):
    alpha2 = 0.5 * (prob.gamma * q_eq ** 2 + p_eq ** 2 / prob.gamma)
    ref = np.zeros_like(E)
    for n0 in range(12):
        for n1 in range(12):
            En = om[0] * (n0 + 0.5) + om[1] * (n1 + 0.5)
            wgt = h.poisson(n0, alpha2[0]) * h.poisson(n1, alpha2[1])
            ref += wgt * h.dirichlet_power(E, [En], prob.dt, prob.n_steps)[:, 0]
    return ref


def test_several_references_from_one_husimi_batch(oracle_mod):
    O = oracle_mod
    om_cm = np.array([2000.0, 3100.0])
    om = om_cm * inputs.HARTREE_PER_CM1
    sg = np.sqrt(om)
    prob0 = inputs.harmonic(om_cm, n_steps=1024, dt=10.0, e_min=0.0, e_max=0.06, n_energies=300)
    p0, q0, lr = O.sample_husimi(prob0, 17, 6000)  # one batch around chi_0 at the origin
    E = prob0.energies()
    refs = [(np.zeros(2), np.zeros(2)),                  # chi_0 itself: the exact ground state
            (sg * np.array([0.8, 0.0]), np.zeros(2)),    # displaced in momentum
            (np.zeros(2), np.array([0.0, 0.7]) / sg),    # displaced in position
            (sg * np.array([0.5, 0.4]), np.array([0.3, -0.3]) / sg)]
    for m, (pe, qe) in enumerate(refs):
        prob = prob0.replace(p_eq=pe, q_eq=qe)
        r = O.run(prob, p0, q0, lr, want_state=False)
        ref = _poisson_spectrum(prob, om, pe, qe, E)
        # the good count is chi_m's Husimi mass of the batch
        assert r.good_weight == O.good_weight(prob, p0, q0, lr, np.ones(p0.shape[1], bool))
        if m == 0:
            assert r.good_weight == r.n_good
            assert np.abs(r.spectrum - ref).max() < 1e-3 * ref.max()
            continue
        # the total intensity within its standard error from per-trajectory contributions
        dE = E[1] - E[0]
        scale = prob.dt ** 2 / (2 * math.pi * prob.total_time) * dE
        c = r.contrib * r.n_good / r.good_weight
        total, se = scale * c.mean(), scale * c.std() / math.sqrt(len(c))
        assert abs(total - ref.sum() * dE) < 4 * se + 5e-3, (m, total, ref.sum() * dE, se)
        assert np.abs(r.spectrum - ref).max() < 0.1 * ref.max(), m
        # the fundamentals appear at the harmonic levels
        for n0, n1 in ((1, 0), (0, 1)):
            En = om[0] * (n0 + 0.5) + om[1] * (n1 + 0.5)
            if _poisson_spectrum(prob, om, pe, qe, np.array([En]))[0] < 0.1 * ref.max():
                continue
            ep, _ = h.fine_peak(O, prob, p0[:, :2000], q0[:, :2000], lr[:2000], En, half=1e-4, n=101)
            assert abs(h.cm(ep - En)) < 3.0, (m, n0, n1, h.cm(ep), h.cm(En))
