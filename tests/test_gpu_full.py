"""The double-time form of Eq. (9) on the GPU (scivr_accumulate_spectrum_full)
against the oracle's (oracle/ta_full.c), through the C ABI.

Both sides run every segment [c1, c2] of every trajectory with its own
tangent map, prefactor branch and action, on the same Husimi points.  The lag
sums R_j(tau) and the spectrum agree to 1e-9 for trajectories whose
monodromy stays moderate; the physics checks repeat the oracle pins on the
GPU: the gamma = omega harmonic case reduces to the separable form, and the
uncoupled Morse zero-point peak loses the separable approximation's shift.
"""
import sys

import numpy as np
import pytest

from paper_1312_4698_amd import inputs
from tests import _helpers as h
from tests import _parity

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scivr():
    from paper_1312_4698_amd import scivr as S
    S.load()
    return S


def _gpu_full(S, prob, p0, q0, lr):
    ctx = S.Context(prob, max_traj=lr.shape[0])
    ctx.set_initial(p0, q0, lr)
    ctx.propagate()
    ctx.accumulate_full()
    I, ng, nt = ctx.read_spectrum()
    R = ctx.read_lags()
    st = ctx.read_state()
    ctx.close()
    return I, ng, R, st


@pytest.mark.parametrize("F,n,ns,K,emax", [
    (1, 40, 200, 150, 0.03),   # W = 64 groups per wave; several splits per trajectory
    (2, 20, 96, 120, 0.05),    # ragged last round (97 samples over 32-segment rounds)
    (3, 12, 64, 100, 0.06),
    (6, 6, 40, 80, 0.1),
    (9, 4, 30, 64, 0.1),
    (12, 3, 21, 48, 0.15),     # two waves per SIMD with a spill; rounds of 5 segments
    (16, 2, 19, 48, 0.2),      # one wave per SIMD; 4 groups, lag rings of 8 with a partial last
])
def test_full_form_matches_oracle(scivr, oracle_mod, F, n, ns, K, emax):
    O = oracle_mod
    _say(f"[full] F={F} n={n} steps={ns} K={K}")
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=emax)
    p0, q0, lr = O.sample_husimi(prob, 60 + F, n)
    I, ng, R, st = _gpu_full(scivr, prob, p0, q0, lr)
    ora = O.run_full(prob, p0, q0, lr, want_lags=True)
    sep = O.run(prob, p0, q0, lr)
    assert ng == ora.n_good
    strict = 0
    for j in range(n):
        mo = np.linalg.norm(_parity.scaled_monodromy(prob, sep.state(j).M))
        if mo > _parity.M_NORM_CAP:
            continue
        scale = max(np.max(np.abs(ora.lags[j])), 1e-300)
        err = np.max(np.abs(R[j] - ora.lags[j])) / scale
        assert err < 1e-9, (j, err)
        strict += 1
    _say(f"[full] lags at 1e-9 for {strict} of {n} trajectories")
    assert strict >= n // 2
    assert np.max(np.abs(I - ora.spectrum)) <= 1e-9 * np.max(np.abs(ora.spectrum))


def test_full_form_reduces_to_separable_for_gamma_omega_harmonic(scivr, oracle_mod):
    O = oracle_mod
    _say("[full] harmonic gamma = omega")
    prob = inputs.harmonic([2000.0, 3100.0], n_steps=256, dt=10.0, e_max=0.05, n_energies=200)
    p0, q0, lr = O.sample_husimi(prob, 3, 64)
    If, ngf, _, _ = _gpu_full(scivr, prob, p0, q0, lr)
    ctx = scivr.Context(prob, max_traj=64)
    ctx.set_initial(p0, q0, lr)
    ctx.propagate()
    ctx.accumulate()
    Is, ngs, _ = ctx.read_spectrum()
    ctx.close()
    assert ngf == ngs == 64
    assert np.max(np.abs(If - Is)) < 1e-9 * np.max(Is)


def test_full_form_removes_the_morse_zero_point_shift(scivr, oracle_mod):
    """Uncoupled Morse at 3000 cm^-1: the separable form puts the zero-point
    peak several cm^-1 above the exact level; Eq. (9) within 2 cm^-1."""
    O = oracle_mod
    om_cm = 3000.0
    om = om_cm * inputs.HARTREE_PER_CM1
    e0 = h.morse_level(om, 0.02, 0)
    prob = inputs.uncoupled_morse([om_cm], n_steps=512, dt=10.0, e_min=e0 - 3e-4, e_max=e0 + 3e-4, n_energies=241)
    _say("[full] Morse zero-point")
    p0, q0, lr = O.sample_husimi(prob, 5, 400)
    If, _, _, _ = _gpu_full(scivr, prob, p0, q0, lr)
    ctx = scivr.Context(prob, max_traj=400)
    ctx.set_initial(p0, q0, lr)
    ctx.propagate()
    ctx.accumulate()
    Is, _, _ = ctx.read_spectrum()
    ctx.close()
    E = prob.energies()

    def peak(I):
        k = int(np.argmax(I))
        y0, y1, y2 = I[k - 1], I[k], I[k + 1]
        return E[k] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * (E[1] - E[0])

    sep, full = h.cm(peak(Is) - e0), h.cm(peak(If) - e0)
    _say(f"[full] Morse ZPE: separable {sep:+.2f} cm^-1, Eq. (9) {full:+.2f} cm^-1")
    assert sep > 2.5 and abs(full) < 2.0


@pytest.mark.parametrize("F,n,ns,K,emax", [(3, 12, 64, 100, 0.06), (9, 4, 30, 64, 0.1)])
def test_full_form_reference_states_match_oracle(scivr, oracle_mod, F, n, ns, K, emax):
    """Several reference states with the double-time form (one pass per
    state): each state's spectrum equals the oracle's double-time form with
    that state as chi on the same points, its good count being the state's
    Husimi mass of the batch; the lag sums read back are chi's."""
    O = oracle_mod
    _say(f"[full] reference states F={F} n={n} steps={ns}")
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=emax)
    rng = np.random.default_rng(70 + F)
    sg = np.sqrt(prob.gamma)
    pe = rng.uniform(-0.6, 0.6, (2, F)) * sg
    qe = rng.uniform(-0.6, 0.6, (2, F)) / sg
    p0, q0, lr = O.sample_husimi(prob, 60 + F, n)
    ctx = scivr.Context(prob, max_traj=n)
    ctx.set_references(pe, qe)
    ctx.set_initial(p0, q0, lr)
    ctx.propagate()
    ctx.accumulate_full()
    spectra = [ctx.read_spectrum(m) for m in range(3)]
    R = ctx.read_lags()
    ctx.close()
    I0, ng0, R0, _ = _gpu_full(scivr, prob, p0, q0, lr)
    assert np.array_equal(spectra[0][0], I0) and spectra[0][1] == ng0
    assert np.array_equal(R, R0)
    for m in (1, 2):
        pm = prob.replace(p_eq=pe[m - 1], q_eq=qe[m - 1])
        ora = O.run_full(pm, p0, q0, lr)
        I, ng, nt = spectra[m]
        assert ng == ora.n_good and nt == n
        err = np.max(np.abs(I - ora.spectrum)) / np.max(np.abs(ora.spectrum))
        _say(f"[full] reference {m}: max rel diff {err:.2e}")
        assert err < 1e-9, (m, err)


def test_full_form_rejects_what_it_does_not_cover(scivr):
    _say("[full] unsupported forms")
    pm = inputs.morse_quartic(2, 2, n_steps=16, n_energies=16, precision=inputs.PRECISION_MIXED)
    ctx = scivr.Context(pm, max_traj=8)
    ctx.sample_husimi(1, 8)
    ctx.propagate()
    with pytest.raises(scivr.ScivrError, match="EUNSUPPORTED"):
        ctx.accumulate_full()
    ctx.close()
    p2 = inputs.morse_quartic(2, 2, n_steps=16, n_energies=16)
    ctx = scivr.Context(p2, max_traj=8)
    ctx.sample_husimi(1, 8)
    with pytest.raises(scivr.ScivrError, match="ESTATE"):
        ctx.accumulate_full()          # nothing propagated
    ctx.propagate()
    ctx.accumulate()
    with pytest.raises(scivr.ScivrError, match="ESTATE"):
        ctx.read_lags()                # the batch went through the separable form
    ctx.close()
