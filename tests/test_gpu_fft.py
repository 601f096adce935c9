"""The FFT-autocorrelation form of the Fourier accumulation against the GEMM
form and the oracle.

Both forms compute sum_j w_j |sum_c amp_jc e^{i E_k c dt}|^2 of the same
batch; the FFT form goes through the trajectories' autocorrelations, so the
two agree to rounding.  Cases cover a sequence length L well above
2 (n_t - 1), L exactly 2 (n_t - 1) (the folded lag L/2 taken directly), a single
step, the longest sequence the form takes, and the mixed form's FP16 planes.
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


def _spectrum(S, prob, seed, n, fft):
    ctx = S.Context(prob, max_traj=n)
    ctx.sample_husimi(seed, n)
    ctx.propagate(0, prob.n_steps)
    if fft:
        ctx.accumulate_fft()
    else:
        ctx.accumulate()
    I, ng, nt = ctx.read_spectrum()
    return ctx, I, ng, nt


@pytest.mark.parametrize("F,n,ns,K,emax", [
    (2, 300, 300, 257, 0.05),    # L = 1024 > 2 (n_t - 1)
    (2, 257, 512, 130, 0.05),    # L = 1024 = 2 (n_t - 1): folded lag
    (3, 65, 1, 40, 0.06),        # one step
    (9, 140, 200, 129, 0.1),     # L = 512 > 400
    (9, 70, 256, 100, 0.1),      # L = 512 = 2 (n_t - 1)
    (17, 40, 150, 100, 0.15),    # amplitudes of the one-wave-per-trajectory kernel
    (30, 24, 128, 128, 0.2),     # L = 256 = 2 (n_t - 1)
])
def test_fft_form_matches_gemm_form(scivr, F, n, ns, K, emax):
    _say(f"[fft] F={F} n={n} steps={ns} K={K}")
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=emax)
    c1, Ig, ngg, ntg = _spectrum(scivr, prob, 7, n, fft=False)
    c2, If, ngf, ntf = _spectrum(scivr, prob, 7, n, fft=True)
    assert ngg == ngf and ntg == ntf == n
    rel = np.max(np.abs(If - Ig)) / np.max(np.abs(Ig))
    _say(f"[fft] max rel diff vs GEMM {rel:.2e}")
    assert rel < 1e-11
    c1.close()
    c2.close()


def test_fft_form_matches_oracle(scivr, oracle_mod):
    O = oracle_mod
    prob = inputs.morse_quartic(4, 4, n_steps=320, n_energies=200, e_max=0.08)
    n = 120
    ctx, I, ng, _ = _spectrum(scivr, prob, 13, n, fft=True)
    p0, q0, lr = O.sample_husimi(prob, 13, n)
    ora = O.run(prob, p0, q0, lr)
    assert ng == ora.n_good
    rel = np.max(np.abs(I - ora.spectrum)) / np.max(ora.spectrum)
    _say(f"[fft] F=4 vs oracle {rel:.2e}")
    assert rel < 1e-9
    ctx.close()


def test_fft_form_longest_sequence(scivr):
    # 4096 steps: L = 8192 = 2 (n_t - 1), the whole sequence in 128 KB of LDS
    prob = inputs.morse_quartic(2, 2, n_steps=4096, n_energies=256, e_max=0.05)
    n = 96
    c1, Ig, _, _ = _spectrum(scivr, prob, 3, n, fft=False)
    c2, If, _, _ = _spectrum(scivr, prob, 3, n, fft=True)
    rel = np.max(np.abs(If - Ig)) / np.max(np.abs(Ig))
    _say(f"[fft] 4096 steps: max rel diff vs GEMM {rel:.2e}")
    assert rel < 1e-11
    c1.close()
    c2.close()


@pytest.mark.parametrize("F,n", [(9, 140), (30, 24)])
def test_fft_form_mixed_precision(scivr, F, n):
    prob = inputs.morse_quartic(F, F, n_steps=256, n_energies=160, e_max=0.1 if F < 17 else 0.2,
                                precision=inputs.PRECISION_MIXED)
    c1, Ig, _, _ = _spectrum(scivr, prob, 5, n, fft=False)
    c2, If, _, _ = _spectrum(scivr, prob, 5, n, fft=True)
    rel = np.max(np.abs(If - Ig)) / np.max(np.abs(Ig))
    _say(f"[fft] mixed: max rel diff vs the FP16 GEMM {rel:.2e}")
    # the FFT form reads the same FP16 hi/lo amplitudes and works in FP64; the
    # GEMM multiplies them on FP16 matrix cores with FP32 accumulation
    assert rel < 1e-4
    c1.close()
    c2.close()


def test_fft_form_state_errors(scivr):
    S = scivr
    prob = inputs.morse_quartic(3, 3, n_steps=40, n_energies=16)
    ctx = S.Context(prob, max_traj=30)
    with pytest.raises(S.ScivrError) as e:
        ctx.accumulate_fft()                      # nothing propagated
    assert e.value.status == S.ESTATE
    ctx.sample_husimi(1, 30)
    ctx.propagate(0, 40)
    ctx.accumulate_fft()
    with pytest.raises(S.ScivrError) as e:
        ctx.accumulate_fft()                      # twice
    assert e.value.status == S.ESTATE
    with pytest.raises(S.ScivrError) as e:
        ctx.read_contributions()                  # the FFT form yields none
    assert e.value.status == S.ESTATE
    fl = S.Flow(ctx, 2, 8, seed=1)
    with pytest.raises(S.ScivrError) as e:
        fl.train_on_batch(epochs=1, batch=10, lr=1e-3)
    assert e.value.status == S.ESTATE
    fl.close()
    ctx.close()
    long_prob = inputs.morse_quartic(2, 2, n_steps=4097, n_energies=16)
    c2 = S.Context(long_prob, max_traj=2)
    c2.sample_husimi(1, 2)
    c2.propagate(0, 4097)
    with pytest.raises(S.ScivrError) as e:
        c2.accumulate_fft()                       # L would be 16384
    assert e.value.status == S.EUNSUPPORTED
    c2.close()


def test_fft_form_adds_into_the_running_totals(scivr):
    # two batches, the first by the GEMM and the second by the FFT form, give
    # the estimate of two GEMM batches
    prob = inputs.morse_quartic(3, 3, n_steps=256, n_energies=100, e_max=0.06)
    n = 80
    ref = scivr.Context(prob, max_traj=n)
    mix = scivr.Context(prob, max_traj=n)
    for b, first in enumerate((0, n)):
        for ctx, fft in ((ref, False), (mix, b == 1)):
            ctx.sample_husimi(17, n, first)
            ctx.propagate(0, prob.n_steps)
            if fft:
                ctx.accumulate_fft()
            else:
                ctx.accumulate()
    Ir, ngr, ntr = ref.read_spectrum()
    Im, ngm, ntm = mix.read_spectrum()
    assert ntr == ntm == 2 * n and ngr == ngm
    assert np.max(np.abs(Im - Ir)) < 1e-11 * np.max(np.abs(Ir))
    ref.close()
    mix.close()
