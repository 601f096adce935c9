"""Continuity of the prefactor branch at F = 30 over the F = 30 workload's
length (8192 steps of 10 au), on the oracle.

At F = 30, dt sum(gamma) is about 3.8 rad, more than pi, so the step of the
principal argument is kept small only by the harmonic predictor
exp(i dt sum gamma) (the continuous branch of sqrt(det A) in Eq. (5), reading
R8).  An aliased step would shift phi by pi and flip the amplitude's sign.
Checks, along Husimi trajectories of the workload's potential:
  * every step's increment of the tracked argument stays below pi / 2 in
    magnitude (a margin of a factor 2 from the branch ambiguity);
  * phi at checkpoints converges as the step shrinks (dt, dt / 2, dt / 4)
    while the trajectory is good on all three and ||M||_F <= 1e5: the
    differences keep the fourth-order ratio of about 16, which a pi jump in
    any run would break.  (Beyond ||M|| ~ 1e5 the three runs separate by
    chaos, and the ratio no longer says anything about the branch.)
"""
import math

import numpy as np
import pytest

from paper_1312_4698_amd import inputs

pytestmark = pytest.mark.slow


def test_branch_steps_stay_small_at_f30(oracle_mod):
    O = oracle_mod
    prob, _ = inputs.workload("F30_fp64")
    p0, q0, _ = O.sample_husimi(prob, 303, 2)
    assert prob.dt * prob.gamma.sum() > math.pi  # the regime where only the predictor keeps steps small
    for j in range(2):
        tr = O.Trajectory(prob, p0[:, j], q0[:, j])
        theta = tr.state.theta
        worst = 0.0
        for _ in range(prob.n_steps):
            tr.advance(1)
            th = tr.state.theta
            worst = max(worst, abs(th - theta))
            theta = th
        assert worst < math.pi / 2, worst


def test_branch_agrees_under_step_halving_at_f30(oracle_mod):
    O = oracle_mod
    prob, _ = inputs.workload("F30_fp64")
    p0, q0, _ = O.sample_husimi(prob, 303, 3)
    T, every = prob.n_steps * prob.dt, 512 * prob.dt
    compared = 0
    for j in range(3):
        runs = []
        for dt in (10.0, 5.0, 2.5):
            pr = prob.replace(dt=dt, n_steps=int(round(T / dt)))
            tr = O.Trajectory(pr, p0[:, j], q0[:, j])
            pts = []
            for _ in range(int(T / every)):
                tr.advance(int(round(every / dt)))
                s = tr.state
                # compared while good and before the tangent map has grown so
                # large that chaos, not the step, sets the differences
                ok = s.good and np.linalg.norm(s.M) <= 1e5
                pts.append((s.phi, ok))
                if not ok:
                    break
            runs.append(pts)
        for (a, ga), (b, gb), (c, gc) in zip(*runs):
            if not (ga and gb and gc):
                break
            # fourth-order convergence: (a - b) / (b - c) ~ 16; an aliased step
            # (a pi jump of phi in one of the runs) cannot keep that ratio
            assert abs(b - c) < 0.5, (j, b, c)
            assert abs(b - c) < max(abs(a - b) / 6, 1e-6), (j, a, b, c)
            compared += 1
    assert compared >= 8, compared
