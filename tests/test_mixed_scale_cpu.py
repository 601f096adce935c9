"""The mixed form's amplitude scale and FP16 hi/lo split, restated on the host.

The trajectory kernels scale each trajectory's amplitudes by the power of two
2^e with e = min(floor(-log2 |<chi|z_0>|) + 3, 15), and store each FP32
component as an FP16 pair hi = fp16(x), lo = fp16(x - hi); the spectrum's
weight carries 4^-e.  For a Husimi draw the overlap is
|<chi|z_0>| = exp(-sum(xi^2 + eta^2) / 4) (the Husimi density of the reference
state, Eq. (3) and the sampling section).  Checks:
  * below the cap the scaled start lies in (4, 8] and the stored amplitude
    keeps about 22 bits (relative error < 2^-21) for F = 9 and F = 30 draws;
  * the cap makes overflow impossible: |<chi|z_t>| <= 1, so a scaled
    amplitude never exceeds 2^15 < 65504, however much the overlap grows along
    the trajectory (a point drawn far out whose trajectory passes near chi);
    without the cap such growth overflows FP16 and the hi/lo pair turns into
    inf - inf;
  * above the cap (most F = 30 draws) the low part goes subnormal: the
    typical draw keeps about 18 bits, draws above 2^-30 (about 97 %) at least
    9, and only draws below 2^-39 (a chi-square(60) tail under 5e-4) leave
    FP16's range.  The draws contribute comparably to the estimate, so this
    costs the spectrum about 2e-4 in relative magnitude and nothing in the
    phases that place the peaks.
"""
import numpy as np
from scipy import stats

CAP = 15


def _scale_exponent(ex0, cap=CAP):
    e = np.floor(-ex0 / np.log(2.0)) + 3
    if cap is not None:
        e = np.minimum(e, cap)
    return e.astype(np.int64)


def _store(x32):
    with np.errstate(over="ignore", invalid="ignore"):
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


def test_scaled_start_below_the_cap_lies_in_4_8():
    ex0, _ = _draws(30, 20000, 1)
    e = _scale_exponent(ex0)
    start = np.ldexp(np.exp(ex0), e)
    free = _scale_exponent(ex0, cap=None) <= CAP
    assert free.any() and (~free).any()
    assert np.all(start[free] > 4.0 * (1 - 1e-12)) and np.all(start[free] <= 8.0 * (1 + 1e-12))
    assert np.all(start[~free] <= 4.0)


def test_draws_below_the_cap_keep_22_bits():
    for F in (9, 30):
        ex0, rng = _draws(F, 20000, F)
        phase = rng.uniform(-np.pi, np.pi, ex0.size)
        free = _scale_exponent(ex0, cap=None) <= CAP
        err = _stored_relative_error(ex0[free], phase[free], _scale_exponent(ex0[free]))
        assert err.max() < 2.0 ** -21, (F, err.max())
    # at F = 9 nearly every draw is below the cap
    ex0, _ = _draws(9, 20000, 9)
    assert np.mean(_scale_exponent(ex0, cap=None) <= CAP) > 0.98


def test_no_overflow_whatever_the_overlap_grows_to():
    for F in (9, 30):
        ex0, rng = _draws(F, 20000, F + 1)
        phase = rng.uniform(-np.pi, np.pi, ex0.size)
        e = _scale_exponent(ex0)
        # the largest possible later amplitude: |<chi|z_t>| = 1
        err = _stored_relative_error(np.zeros_like(ex0), phase, e)
        assert np.all(np.isfinite(err)) and err.max() < 2.0 ** -21
        # without the cap, a draw far out whose trajectory comes near chi overflows
        e_free = _scale_exponent(ex0, cap=None)
        bad = _stored_relative_error(np.zeros_like(ex0), phase, e_free)
        assert not np.all(np.isfinite(bad) & (bad < 1e-3))


def test_capped_f30_draws_keep_most_bits():
    ex0, rng = _draws(30, 20000, 31)
    phase = rng.uniform(-np.pi, np.pi, ex0.size)
    err = _stored_relative_error(ex0, phase, _scale_exponent(ex0))
    depth = -ex0 / np.log(2.0)  # -log2 |<chi|z_0>|
    rand = np.arange(ex0.size) < 20000
    # the typical draw (depth 20 to 25) keeps about 18 bits
    typical = (depth >= 20) & (depth < 25)
    assert np.median(err[typical]) < 2.0 ** -17
    # draws shallower than 2^-30 (about 97 % of them) keep at least 9 bits
    shallow = depth < 30
    assert np.mean(shallow[rand]) > 0.95 and err[shallow].max() < 2.0 ** -9
    # only draws deeper than 2^-39 leave FP16's range
    assert np.mean(depth[rand] >= 39) < 5e-4
