"""Edge cases and error paths of the C ABI on the GPU.

Degenerate sizes (one trajectory, one time step, two energies, ragged tails
around every tile size), the largest F in both precision forms, device-memory
initial conditions, and the state machine of the batch calls (every misuse is
an error status, never a device fault).
"""
import sys

import numpy as np
import pytest

from paper_1312_4698_amd import inputs
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


@pytest.mark.parametrize("F,n,ns,K", [
    (2, 1, 1, 2),        # one trajectory, one step, two energies
    (3, 1, 37, 2),
    (5, 129, 33, 129),   # one past a GEMM tile in trajectories and energies
    (9, 127, 31, 127),   # one short of a tile; a time count not a multiple of the MFMA depth
    (16, 65, 20, 3),     # largest F of the small-F kernel, four trajectories per wave + tail
    (17, 1, 5, 2),       # smallest F of the one-wave kernel
])
def test_degenerate_sizes_match_oracle(scivr, oracle_mod, F, n, ns, K):
    O = oracle_mod
    _say(f"[edge] F={F} n={n} steps={ns} K={K}")
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=0.1)
    ctx = scivr.Context(prob, max_traj=n)
    ctx.run(seed=3, n_traj=n)
    I, ng, nt = ctx.read_spectrum()
    st = ctx.read_state()
    p0, q0, lr = O.sample_husimi(prob, 3, n)
    ora = O.run(prob, p0, q0, lr)
    compared, worst, fails = _parity.compare_states(prob, st, ora)
    assert not fails, fails[:3]
    assert nt == n and ng == ora.n_good
    assert np.max(np.abs(I - ora.spectrum)) <= 1e-9 * max(np.max(np.abs(ora.spectrum)), 1e-300)
    ctx.close()


@pytest.mark.parametrize("precision", [inputs.PRECISION_FP64, inputs.PRECISION_MIXED])
def test_largest_f_both_forms(scivr, oracle_mod, precision):
    O = oracle_mod
    F, n, ns = 32, 20, 60
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=64, e_max=0.25, precision=precision)
    ctx = scivr.Context(prob, max_traj=n)
    ctx.run(seed=8, n_traj=n)
    I, ng, _ = ctx.read_spectrum()
    st = ctx.read_state()
    p0, q0, lr = O.sample_husimi(prob, 8, n)
    ora = O.run(prob, p0, q0, lr)
    tol = _parity.STATE_TOL if precision == inputs.PRECISION_FP64 else 1e-4
    compared, worst, fails = _parity.compare_states(prob, st, ora, tol=tol)
    _say(f"[edge] F=32 precision={precision} compared={compared} worst={worst:.2e}")
    assert not fails and compared >= n // 2
    rel = np.max(np.abs(I - ora.spectrum)) / np.max(ora.spectrum)
    assert rel < (1e-9 if precision == inputs.PRECISION_FP64 else 2e-2)
    ctx.close()


def test_device_initial_conditions(scivr, oracle_mod):
    import torch
    O = oracle_mod
    prob = inputs.morse_quartic(4, 4, n_steps=100, n_energies=80)
    n = 90
    p0, q0, lr = O.sample_husimi(prob, 21, n)
    dev = torch.device("cuda", 0)
    tp, tq, tl = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (p0, q0, lr))
    stream = torch.cuda.current_stream()
    ctx = scivr.Context(prob, max_traj=n)
    ctx.set_initial(tp, tq, tl, stream=stream)
    ctx.propagate(stream=stream)
    ctx.accumulate(stream=stream)
    I, ng, _ = ctx.read_spectrum()
    ora = O.run(prob, p0, q0, lr)
    assert ng == ora.n_good
    assert np.max(np.abs(I - ora.spectrum)) <= 1e-9 * np.max(ora.spectrum)
    rp, rq, rl = ctx.read_initial()
    assert np.array_equal(rp, p0) and np.array_equal(rq, q0) and np.array_equal(rl, lr)
    ctx.close()


def test_batch_state_machine_errors(scivr):
    S = scivr
    prob = inputs.morse_quartic(3, 3, n_steps=20, n_energies=16)
    ctx = S.Context(prob, max_traj=50)
    with pytest.raises(S.ScivrError) as e:
        ctx.propagate(0, 20)                  # no initial conditions
    assert e.value.status == S.ESTATE
    with pytest.raises(S.ScivrError) as e:
        ctx.sample_husimi(1, 51)              # beyond the batch capacity
    assert e.value.status == S.EINVAL
    ctx.sample_husimi(1, 50)
    with pytest.raises(S.ScivrError) as e:
        ctx.accumulate()                      # not propagated
    assert e.value.status == S.ESTATE
    with pytest.raises(S.ScivrError) as e:
        ctx.propagate(5, 10)                  # does not continue from step 0
    assert e.value.status == S.ESTATE
    with pytest.raises(S.ScivrError) as e:
        ctx.propagate(0, 21)                  # past n_steps
    assert e.value.status == S.EINVAL
    ctx.propagate(0, 7)
    ctx.propagate(7, 20)
    with pytest.raises(S.ScivrError) as e:
        ctx.read_contributions()              # not accumulated yet
    assert e.value.status == S.ESTATE
    ctx.accumulate()
    with pytest.raises(S.ScivrError) as e:
        ctx.accumulate()                      # twice
    assert e.value.status == S.ESTATE
    I, ng, nt = ctx.read_spectrum()
    assert nt == 50 and ng > 0
    # a fresh context with nothing accumulated reports ENOGOOD through a zero spectrum
    c2 = S.Context(prob, max_traj=4)
    I0, ng0, nt0 = c2.read_spectrum()
    assert ng0 == 0 and nt0 == 0 and not np.any(I0)
    c2.close()
    ctx.close()


def test_flow_misuse_errors(scivr):
    S = scivr
    prob = inputs.morse_quartic(3, 3, n_steps=20, n_energies=16)
    ctx = S.Context(prob, max_traj=40)
    fl = S.Flow(ctx, 2, 8, seed=1)
    with pytest.raises(S.ScivrError) as e:
        fl.train_on_batch(epochs=1, batch=10, lr=1e-3)    # nothing accumulated
    assert e.value.status == S.ESTATE
    with pytest.raises(S.ScivrError) as e:
        fl.sample(seed=1, n_traj=41)                      # beyond the capacity
    assert e.value.status == S.EINVAL
    with pytest.raises(S.ScivrError) as e:
        fl.sample(seed=1, n_traj=10, alpha=1.5)
    assert e.value.status == S.EINVAL
    with pytest.raises(AssertionError):
        fl.set_params(np.zeros(fl.n_params + 1))
    fl.close()
    ctx.close()


@pytest.mark.parametrize("precision", [inputs.PRECISION_FP64, inputs.PRECISION_MIXED])
def test_amplitudes_zero_from_the_flagging_step(scivr, precision):
    """F = 9 finishes amplitudes in batches of eight time samples.  A
    trajectory flagged at step s must have non-zero amplitudes before sample s
    and zeros from it on, wherever s falls in a batch.  The flagging steps come
    from propagating one step per call and reading the sticky flag after each;
    the single-call run must give bit-identical amplitudes."""
    S = scivr
    ns, n = 800, 70
    # a tolerance at the median of the largest |det(M)^2 - 1| over 800 steps,
    # so trajectories turn bad at scattered steps
    prob = inputs.morse_quartic(9, 9, n_steps=ns, n_energies=64, e_max=0.1, det_tol=3e-13, precision=precision)
    c1 = S.Context(prob, max_traj=n)
    c1.sample_husimi(21, n)
    first_bad = np.full(n, -1)
    for s in range(ns):
        c1.propagate(s, s + 1)
        g = c1.read_state()["good"]
        first_bad[(g == 0) & (first_bad < 0)] = s + 1
    a1 = c1.read_amplitudes(0, n)
    c2 = S.Context(prob, max_traj=n)
    c2.sample_husimi(21, n)
    c2.propagate(0, ns)
    a2 = c2.read_amplitudes(0, n)
    assert np.array_equal(a1, a2)
    mag = np.abs(a2)
    # FP16 planes can underflow to an exact zero where the overlap has decayed,
    # so only the FP64 form checks that the samples before the flag are non-zero
    exact = precision == inputs.PRECISION_FP64
    mid = 0
    for j in range(n):
        if first_bad[j] < 0:
            assert not exact or np.all(mag[j] > 0), j
        else:
            fb = first_bad[j]
            assert np.all(mag[j, fb:] == 0), (j, fb)
            assert not exact or np.all(mag[j, :fb] > 0), (j, fb)
            mid += fb % 8 != 0
    _say(f"[flag step] {precision}: {np.sum(first_bad >= 0)} of {n} flagged, {mid} inside a batch of eight")
    assert mid >= 3
    c1.close()
    c2.close()
