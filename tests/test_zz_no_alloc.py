"""The no-allocation FFT accumulation (scivr_accumulate_spectrum_fft_noalloc)
against the allocating one (scivr_accumulate_spectrum_fft) through the C ABI.

Both run the same kernels in the same order, the first on the context's own
scratch and the second on the library's static per-device scratch, so their
spectra are identical bit for bit.  Two calls in a row, the second on a
smaller batch with a shorter sequence, show that what the first call left in
the shared scratch does not leak into the second.
"""
import sys

import numpy as np
import pytest

from paper_1312_4698_amd import inputs

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
    ctx = S.Context(prob, max_traj=n)
    out = []
    for noalloc in (False, True):
        ctx.reset_spectrum()
        ctx.sample_husimi(seed, n)
        ctx.propagate(0, prob.n_steps)
        if noalloc:
            ctx.accumulate_fft_noalloc()
        else:
            ctx.accumulate_fft()
        out.append(ctx.read_spectrum())
    ctx.close()
    return out


@pytest.mark.parametrize("precision", [inputs.PRECISION_FP64, inputs.PRECISION_MIXED])
def test_noalloc_fft_matches_allocating_form_twice(scivr, precision):
    cases = [
        # F, n, steps, K, e_max: the second call is smaller in every size
        (9, 700, 1000, 300, 0.1),   # L = 2048
        (3, 130, 200, 90, 0.06),    # L = 512
    ]
    for F, n, ns, K, emax in cases:
        _say(f"[noalloc] precision={precision} F={F} n={n} steps={ns} K={K}")
        prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=emax, precision=precision)
        (Ia, nga, nta), (Ib, ngb, ntb) = _both(scivr, prob, 17 + F, n)
        assert nga == ngb and nta == ntb == n
        assert np.all(np.isfinite(Ia)) and np.max(Ia) > 0
        assert np.array_equal(Ia, Ib), np.max(np.abs(Ia - Ib)) / np.max(Ia)


def test_noalloc_fft_with_reference_states(scivr):
    """Several reference states pass through the static scratch one after
    another: every state's spectrum equals the allocating form's bit for bit."""
    F, n, ns, K = 6, 300, 400, 128
    _say(f"[noalloc] three reference states F={F} n={n} steps={ns}")
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=0.1)
    rng = np.random.default_rng(23)
    sg = np.sqrt(prob.gamma)
    pe = rng.uniform(-0.8, 0.8, (2, F)) * sg
    qe = rng.uniform(-0.8, 0.8, (2, F)) / sg
    ctx = scivr.Context(prob, max_traj=n)
    ctx.set_references(pe, qe)
    out = []
    for noalloc in (False, True):
        ctx.reset_spectrum()
        ctx.sample_husimi(31, n)
        ctx.propagate(0, prob.n_steps)
        if noalloc:
            ctx.accumulate_fft_noalloc()
        else:
            ctx.accumulate_fft()
        out.append([ctx.read_spectrum(m) for m in range(3)])
    ctx.close()
    for m in range(3):
        (Ia, nga, _), (Ib, ngb, _) = out[0][m], out[1][m]
        assert nga == ngb and np.max(Ia) > 0
        assert np.array_equal(Ia, Ib), (m, np.max(np.abs(Ia - Ib)) / np.max(Ia))


def test_noalloc_fft_rejects_sequences_beyond_its_scratch(scivr):
    _say("[noalloc] 4097 steps")
    prob = inputs.morse_quartic(2, 2, n_steps=4097, n_energies=64)
    ctx = scivr.Context(prob, max_traj=8)
    ctx.sample_husimi(1, 8)
    ctx.propagate(0, prob.n_steps)
    with pytest.raises(scivr.ScivrError, match="EUNSUPPORTED"):
        ctx.accumulate_fft_noalloc()
    ctx.close()
