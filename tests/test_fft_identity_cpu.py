"""The identity behind the FFT-autocorrelation form of the Fourier step, on
the CPU with numpy (no GPU code involved).

For sequences a_j of n_t samples and weights w_j,

    sum_j w_j |sum_c a_jc e^{i E c dt}|^2 = C(0) + 2 Re sum_{tau=1}^{n_t-1} C(tau) e^{i E tau dt}

with C(tau) = sum_j w_j sum_c a_j[c + tau] conj(a_j[c]), and C(tau) for
tau < n_t is the inverse DFT of sum_j w_j |DFT_L(a_j)|^2 for a zero-padded
length L >= 2 (n_t - 1), except tau = L/2 when L = 2 (n_t - 1), where the
lags +-L/2 share one bin.  The GPU form follows exactly these steps.
"""
import numpy as np
import pytest


def _direct(a, w, E, dt):
    nt = a.shape[1]
    ph = np.exp(1j * np.outer(np.arange(nt), E) * dt)
    A = a @ ph
    return (w[:, None] * np.abs(A) ** 2).sum(axis=0)


def _via_fft(a, w, E, dt, fold_fix=True):
    n, nt = a.shape
    lg = max(3, int(np.ceil(np.log2(2 * (nt - 1)))) if nt > 1 else 3)
    L = 1 << lg
    X = np.fft.fft(a, n=L, axis=1)
    S = (w[:, None] * np.abs(X) ** 2).sum(axis=0)
    C = np.fft.ifft(S)[:nt]
    if fold_fix and L == 2 * (nt - 1):
        C[L // 2] = (w * a[:, L // 2] * np.conj(a[:, 0])).sum()
    tau = np.arange(1, nt)
    return C[0].real + 2.0 * (C[1:, None] * np.exp(1j * np.outer(tau, E) * dt)).real.sum(axis=0)


@pytest.mark.parametrize("nt", [2, 5, 301, 513, 257])
def test_autocorrelation_form_equals_direct_sum(nt):
    rng = np.random.default_rng(nt)
    n = 7
    a = rng.normal(size=(n, nt)) + 1j * rng.normal(size=(n, nt))
    w = rng.uniform(0.1, 2.0, size=n)
    dt = 10.0
    E = np.linspace(0.0, 0.1, 97)
    d = _direct(a, w, E, dt)
    f = _via_fft(a, w, E, dt)
    assert np.max(np.abs(f - d)) <= 1e-11 * np.max(np.abs(d))


def test_folded_lag_needs_its_direct_sum():
    # with L = 2 (n_t - 1) the circular bin L/2 holds C(L/2) + C(-L/2): using it
    # as C(L/2) is wrong by a visible amount, which the direct sum removes
    rng = np.random.default_rng(1)
    nt = 513
    a = rng.normal(size=(3, nt)) + 1j * rng.normal(size=(3, nt))
    w = np.ones(3)
    E = np.linspace(0.0, 0.1, 50)
    d = _direct(a, w, E, 10.0)
    wrong = _via_fft(a, w, E, 10.0, fold_fix=False)
    right = _via_fft(a, w, E, 10.0, fold_fix=True)
    assert np.max(np.abs(right - d)) <= 1e-11 * np.max(np.abs(d))
    assert np.max(np.abs(wrong - d)) > 1e-6 * np.max(np.abs(d))
