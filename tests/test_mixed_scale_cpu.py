"""The mixed form's amplitude scale and FP16 hi/lo split, restated on the host.

The trajectory kernels scale each trajectory's amplitudes by the power of two
2^e with e = floor(-log2 |<chi|z_0>|) + 3, so the scaled start lies in (4, 8],
and store each FP32 component as an FP16 pair hi = fp16(x), lo = fp16(x - hi);
the spectrum's weight carries 4^-e.  For a Husimi draw the overlap is
|<chi|z_0>| = exp(-sum(xi^2 + eta^2) / 4) (the Husimi density of the reference
state, Eq. (3) and the sampling section), so at F = 30 a typical start needs
e ~ 22 and the far tail of the chi-square(60) draw e > 40.  These checks push
typical and tail draws through the same rule and bound the stored amplitude's
relative error by 2^-21; the rule that clamped e at 12 fails it.
"""
import numpy as np
from scipy import stats


def _scale_exponent(ex0, clamp=None):
    e = np.floor(-ex0 / np.log(2.0)).astype(np.int64) + 3
    if clamp is not None:
        e = np.clip(np.floor(-ex0 / np.log(2.0)).astype(np.int64), 0, clamp)
    return e


def _store(x32):
    hi = x32.astype(np.float16)
    lo = (x32 - hi.astype(np.float32)).astype(np.float16)
    return hi.astype(np.float64) + lo.astype(np.float64)


def _stored_relative_error(ex, phase, e):
    mag = np.ldexp(np.exp(ex), e)
    re = (mag * np.cos(phase)).astype(np.float32)
    im = (mag * np.sin(phase)).astype(np.float32)
    got = _store(re) + 1j * _store(im)
    want = mag * np.exp(1j * phase)
    return np.abs(got - want) / np.abs(want)


def _draws(F, n, seed):
    rng = np.random.default_rng(seed)
    chi2 = (rng.standard_normal((n, 2 * F)) ** 2).sum(axis=1)
    # the far tail as well: quantiles out to 1 - 1e-12 of chi-square(2F)
    tail = stats.chi2.isf(np.logspace(-3, -12, 64), 2 * F)
    return -0.25 * np.concatenate([chi2, tail]), rng


def test_scaled_start_lies_in_4_8():
    ex0, _ = _draws(30, 20000, 1)
    e = _scale_exponent(ex0)
    start = np.ldexp(np.exp(ex0), e)
    assert np.all(start > 4.0 * (1 - 1e-12)) and np.all(start <= 8.0 * (1 + 1e-12))


def test_typical_and_tail_draws_keep_22_bits_at_f30():
    for F in (9, 30):
        ex0, rng = _draws(F, 20000, F)
        phase = rng.uniform(-np.pi, np.pi, ex0.size)
        e = _scale_exponent(ex0)
        err = _stored_relative_error(ex0, phase, e)
        assert err.max() < 2.0 ** -21, (F, err.max())
        # the overlap may grow 2^12-fold along the trajectory and still fit FP16
        grown = _stored_relative_error(ex0 + 12 * np.log(2.0), phase, e)
        assert np.all(np.isfinite(grown)) and grown.max() < 2.0 ** -21


def test_clamped_rule_loses_bits_in_the_f30_tail():
    ex0, rng = _draws(30, 20000, 30)
    phase = rng.uniform(-np.pi, np.pi, ex0.size)
    err = _stored_relative_error(ex0, phase, _scale_exponent(ex0, clamp=12))
    assert err.max() > 2.0 ** -12
