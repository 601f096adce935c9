"""The error of the separable prefactor approximation (after Eq. (9)),
measured with the double-time form of Eq. (9) on the GPU against exact
levels.

* Uncoupled Morse (3000 cm^-1, x_e = 0.02), reference state displaced in
  momentum so that levels 0, 1 and 2 carry weight: exact levels
  omega (n + 1/2) - omega x_e (n + 1/2)^2.
* Two coupled Morse modes (quartic coupling, the F = 2 workload's family with
  eps up to 0.05): eigenvalues of a sinc-DVR diagonalisation.
Both forms run on the same Husimi points; peak positions are refined on a fine
energy grid by the parabola through the maximum and its neighbours.  The
numbers are printed; the assertions are the physics pins' tolerances.
"""
import math
import sys

import numpy as np
import pytest

from paper_1312_4698_amd import inputs
from tests import _helpers as h

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scivr():
    from paper_1312_4698_amd import scivr as S
    S.load()
    return S


def _both(S, prob, seed, n):
    out = []
    for full in (False, True):
        ctx = S.Context(prob, max_traj=n)
        ctx.sample_husimi(seed, n)
        ctx.propagate()
        if full:
            ctx.accumulate_full()
        else:
            ctx.accumulate()
        out.append(ctx.read_spectrum()[0])
        ctx.close()
    return out


def _peak_near(E, I, e0, half):
    m = np.abs(E - e0) <= half
    idx = np.flatnonzero(m)
    k = idx[int(np.argmax(I[m]))]
    y0, y1, y2 = I[k - 1], I[k], I[k + 1]
    return E[k] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * (E[1] - E[0])


def test_separable_error_uncoupled_morse(scivr):
    om_cm = 3000.0
    om = om_cm * inputs.HARTREE_PER_CM1
    levels = [h.morse_level(om, 0.02, n) for n in range(3)]
    prob = inputs.uncoupled_morse([om_cm], n_steps=4096, dt=10.0, e_min=levels[0] - 4e-3, e_max=levels[2] + 4e-3,
                                  n_energies=12288, p_eq=np.array([1.5 * math.sqrt(om)]))
    Is, If = _both(scivr, prob, 5, 1024)
    E = prob.energies()
    rows = []
    for n, ex in enumerate(levels):
        es, ef = _peak_near(E, Is, ex, 2e-4), _peak_near(E, If, ex, 2e-4)
        rows.append((n, h.cm(ex), h.cm(es - ex), h.cm(ef - ex)))
        _say(f"[separable] Morse level {n}: exact {h.cm(ex):.2f} cm^-1, separable {h.cm(es - ex):+.2f}, "
             f"Eq. (9) {h.cm(ef - ex):+.2f}")
    assert rows[0][2] > 2.5 and abs(rows[0][3]) < 2.0
    for n, ex, ds, df in rows:
        assert abs(df) < 5e-3 * ex and abs(ds) < 5e-3 * ex


def test_separable_error_coupled_f2(scivr):
    base = inputs.morse_quartic(2, 2)
    prob = inputs.morse_quartic(2, 2, eps_max=0.05, n_steps=4096, e_min=0.0, e_max=0.05, n_energies=8192,
                                p_eq=np.sqrt(base.gamma))
    w, c2 = h.sinc_dvr_2d(prob, npts=48)
    Is, If = _both(scivr, prob, 7, 1024)
    E = prob.energies()
    res = 2 * math.pi / (prob.n_steps * prob.dt)
    strong = [n for n in range(len(w)) if c2[n] > 0.02 and w[n] < 0.05]
    tested = 0
    for n in strong:
        others = [m for m in strong if m != n]
        if others and min(abs(w[m] - w[n]) for m in others) < 4 * res:
            continue
        es, ef = _peak_near(E, Is, w[n], 2e-4), _peak_near(E, If, w[n], 2e-4)
        _say(f"[separable] F=2 level {n}: DVR {h.cm(w[n]):.2f} cm^-1, separable {h.cm(es - w[n]):+.2f}, "
             f"Eq. (9) {h.cm(ef - w[n]):+.2f}")
        assert abs(es - w[n]) / w[n] < 5e-3 and abs(ef - w[n]) / w[n] < 5e-3
        tested += 1
    assert tested >= 2
