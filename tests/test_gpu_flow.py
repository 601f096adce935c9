"""The learned importance-sampling proposal on the GPU against the flow oracle.

FP32 training path: density pass, loss and gradient, Adam steps.  BF16
inference path (sampling): within the tolerance BF16 rounding explains, and
self-consistent (the density the sampler reports is the density of the points
it returns).  Sampler: alpha = 1 is the Husimi sampler bit for bit; the
component choice and the normal draws match the oracle's Philox streams.
Estimator: importance weights and the weighted good count reproduce the
Husimi spectrum (exactly for the harmonic case, within Monte Carlo error for
an anharmonic one).
"""
import math
import sys

import numpy as np
import pytest

from oracle import flow_oracle as FO
from paper_1312_4698_amd import inputs, peaks

pytestmark = pytest.mark.gpu
CM = inputs.CM1_PER_HARTREE


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scivr():
    from paper_1312_4698_amd import scivr as S
    S.load()
    return S


def _params(F, H, L, seed, scale_out=0.3):
    rng = np.random.default_rng(seed)
    p = np.zeros(FO.param_count(F, H, L))
    for lp in FO.unpack(p, F, H, L):
        lp["W1"][:] = rng.normal(size=lp["W1"].shape) / math.sqrt(F)
        lp["b1"][:] = rng.normal(size=lp["b1"].shape) * 0.1
        lp["W2"][:] = rng.normal(size=lp["W2"].shape) / math.sqrt(H)
        lp["b2"][:] = rng.normal(size=lp["b2"].shape) * 0.1
        lp["W3"][:] = rng.normal(size=lp["W3"].shape) * scale_out / math.sqrt(H)
        lp["b3"][:] = rng.normal(size=lp["b3"].shape) * scale_out
    return p.astype(np.float32).astype(np.float64)  # the GPU holds FP32 parameters


def test_flow_init_is_identity(scivr, oracle_mod):
    prob = inputs.morse_quartic(9, 9, n_steps=8, n_energies=8)
    ctx = scivr.Context(prob, max_traj=1000)
    fl = scivr.Flow(ctx, 4, 128, seed=3)
    assert fl.n_params == FO.param_count(9, 128, 4) == 80456
    p = fl.get_params().astype(np.float64)
    lps = FO.unpack(p, 9, 128, 4)
    for lp in lps:
        assert not np.any(lp["W3"]) and not np.any(lp["b3"]) and not np.any(lp["b1"]) and not np.any(lp["b2"])
    w2 = np.concatenate([lp["W2"].ravel() for lp in lps])
    assert abs(w2.mean()) < 0.01 and abs(w2.std() * math.sqrt(128) - 1.0) < 0.02
    p0, q0, lr = oracle_mod.sample_husimi(prob, 4, 1000)
    for bf16 in (False, True):
        lq, u = fl.log_density(p0, q0, bf16=bf16)
        assert np.max(np.abs(lq - lr)) < 1e-4
        x = FO.whiten(prob, p0, q0)
        assert np.max(np.abs(u - x)) < 1e-5 * max(1.0, np.abs(x).max())
    fl.close()
    ctx.close()


@pytest.mark.parametrize("F,H", [(3, 16), (9, 128), (30, 256)])
def test_flow_density_matches_oracle(scivr, oracle_mod, F, H):
    L = 4
    prob = inputs.morse_quartic(F, F, n_steps=8, n_energies=8)
    n = 1500
    ctx = scivr.Context(prob, max_traj=n)
    fl = scivr.Flow(ctx, L, H, seed=1)
    params = _params(F, H, L, 20 + F)
    fl.set_params(params)
    p0, q0, _ = oracle_mod.sample_husimi(prob, 9, n)
    x = FO.whiten(prob, p0, q0)
    u_o, lq_o = FO.density(params, F, H, L, x)
    lq, u = fl.log_density(p0, q0)
    err_l = np.max(np.abs(lq - lq_o))
    err_u = np.max(np.abs(u - u_o))
    _say(f"[flow F={F} H={H}] fp32 density: |dlogq| {err_l:.2e}, |du| {err_u:.2e}")
    assert err_l < 2e-4 * max(1.0, np.abs(lq_o).max()) and err_u < 1e-4 * max(1.0, np.abs(u_o).max())
    lq16, u16 = fl.log_density(p0, q0, bf16=True)
    e16 = np.abs(lq16 - lq_o)
    _say(f"[flow F={F} H={H}] bf16 density: max |dlogq| {e16.max():.3e}, median {np.median(e16):.3e}")
    # BF16 keeps 8 bits (relative 4e-3 per rounding); log q sums F L log-scales whose
    # rounding errors add up like a random walk
    walk = math.sqrt(F * L)
    assert np.median(e16) < 0.006 * walk and e16.max() < 0.06 * walk
    fl.close()
    ctx.close()


@pytest.mark.parametrize("F,H,n", [
    (3, 16, 700), (9, 128, 2000), (30, 256, 1500),
    (3, 16, 40000),  # 512-row weight-gradient partials with a ragged last one; 64-row GEMM tiles
])
def test_flow_gradient_matches_oracle(scivr, oracle_mod, F, H, n):
    L = 4
    prob = inputs.morse_quartic(F, F, n_steps=8, n_energies=8)
    ctx = scivr.Context(prob, max_traj=n)
    fl = scivr.Flow(ctx, L, H, seed=1)
    params = _params(F, H, L, 40 + F, scale_out=0.5)
    fl.set_params(params)
    p0, q0, _ = oracle_mod.sample_husimi(prob, 11, n)
    c = np.random.default_rng(12).exponential(size=n)
    c[::7] = 0.0
    loss, g = fl.loss_grad(p0, q0, c)
    x = FO.whiten(prob, p0, q0)
    loss_o, g_o = FO.loss_and_grad(params, F, H, L, x, c)
    gm = np.abs(g_o).max()
    err = np.abs(g - g_o).max()
    _say(f"[flow F={F} H={H}] loss {loss:.6f} vs {loss_o:.6f}; |dgrad| {err:.2e} of max {gm:.2e}")
    assert abs(loss - loss_o) < 1e-5 * max(1.0, abs(loss_o))
    assert err < 2e-4 * gm
    fl.close()
    ctx.close()


def test_flow_adam_steps_match_oracle(scivr, oracle_mod):
    F, H, L, n = 3, 16, 4, 800
    prob = inputs.morse_quartic(F, F, n_steps=8, n_energies=8)
    ctx = scivr.Context(prob, max_traj=n)
    fl = scivr.Flow(ctx, L, H, seed=1)
    params = _params(F, H, L, 60, scale_out=0.4)
    fl.set_params(params)
    p0, q0, _ = oracle_mod.sample_husimi(prob, 13, n)
    c = np.random.default_rng(14).exponential(size=n)
    lr = 1e-3
    x = FO.whiten(prob, p0, q0)
    # one full-batch step: for every parameter whose gradient is not tiny, the
    # first Adam step is -lr sign(g) on both sides
    _, g_o = FO.loss_and_grad(params, F, H, L, x, c)
    fl.train(p0, q0, c, epochs=1, batch=n, lr=lr)
    p1 = fl.get_params().astype(np.float64)
    p1_o, _, _ = FO.train(params, F, H, L, x, c, epochs=1, batch=n, lr=lr)
    big = np.abs(g_o) > 1e-3 * np.abs(g_o).max()
    assert np.max(np.abs(p1 - p1_o)[big]) < 1e-6
    assert np.max(np.abs(p1 - p1_o)) < 2.0 * lr
    # six more steps over two mini-batches per epoch: the losses follow the oracle's
    fl.set_params(params)
    loss_g = fl.train(p0, q0, c, epochs=3, batch=n // 2, lr=lr)
    _, _, losses = FO.train(params, F, H, L, x, c, epochs=3, batch=n // 2, lr=lr)
    _say(f"[flow adam] last mini-batch loss gpu {loss_g:.6f} oracle {losses[-1]:.6f}")
    assert abs(loss_g - losses[-1]) < 1e-3 * max(1.0, abs(losses[-1]))
    fl.close()
    ctx.close()


def test_flow_sample_alpha_one_is_husimi(scivr):
    prob = inputs.morse_quartic(6, 6, n_steps=8, n_energies=8)
    n = 777
    ctx = scivr.Context(prob, max_traj=n)
    ctx.sample_husimi(seed=5, n_traj=n, first_index=100)
    ref = ctx.read_initial()
    fl = scivr.Flow(ctx, 4, 32, seed=2)
    fl.set_params(_params(6, 32, 4, 70))
    ess, used = fl.sample(seed=5, n_traj=n, first_index=100, alpha=1.0)
    got = ctx.read_initial()
    assert used and ess == pytest.approx(1.0, abs=1e-12)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    fl.close()
    ctx.close()


def test_flow_sample_matches_oracle_sampler(scivr, oracle_mod):
    F, H, L, n, alpha = 4, 32, 4, 1200, 0.3
    prob = inputs.morse_quartic(F, F, n_steps=8, n_energies=8)
    ctx = scivr.Context(prob, max_traj=n)
    fl = scivr.Flow(ctx, L, H, seed=2)
    params = _params(F, H, L, 80, scale_out=0.4)
    fl.set_params(params)
    ess, used = fl.sample(seed=17, n_traj=n, first_index=3, alpha=alpha, min_ess_frac=0.0)
    p0, q0, lr = ctx.read_initial()
    p0o, q0o, lro, from_n, xo = FO.sample(prob, params, H, L, seed=17, first_index=3, n=n, alpha=alpha)
    x = FO.whiten(prob, p0, q0)
    same = np.all(np.abs(x - xo) < 1e-12, axis=1)
    # the component choice is the oracle's: normal draws identical, flow images close
    assert np.array_equal(same | ~from_n, np.ones(n, dtype=bool))
    assert np.all(same[from_n])
    dx = np.abs(x - xo)[~from_n].max()
    _say(f"[flow sample] {from_n.sum()} normal, {(~from_n).sum()} flow points; max |dx| flow {dx:.3e}; ess {ess:.3f}")
    assert dx < 0.05
    # the reported density is the mixture density of the returned points (BF16 networks)
    _, lq_o = FO.density(params, F, H, L, x)
    mix_o = FO.mixture_log_density(x, lq_o, alpha)
    assert np.median(np.abs(lr - mix_o)) < 0.03 and np.abs(lr - mix_o).max() < 0.3
    # the reported ESS, which decides the fallback, is the pilot draw's: the
    # mixture's points at indices disjoint from the batch's; drawn as a batch of
    # their own, they give that ESS back from their returned densities
    fl.sample(seed=17, n_traj=min(n, 4096), first_index=3 + (1 << 62), alpha=alpha, min_ess_frac=0.0)
    pp, qp, lrp = ctx.read_initial()
    ess_pilot = FO.ess_fraction(FO.whiten(prob, pp, qp), lrp)
    _say(f"[flow sample] pilot ess {ess:.6f}, recomputed {ess_pilot:.6f}")
    assert ess == pytest.approx(ess_pilot, rel=1e-9)
    fl.close()
    ctx.close()


def test_flow_ess_fallback_to_husimi(scivr):
    # a flow that moves everything far away: with alpha = 0 the ratios collapse,
    # the ESS test fails and the batch is the Husimi draw
    F, H, L, n = 2, 8, 2, 500
    prob = inputs.morse_quartic(F, F, n_steps=8, n_energies=8)
    ctx = scivr.Context(prob, max_traj=n)
    fl = scivr.Flow(ctx, L, H, seed=2)
    p = np.zeros(FO.param_count(F, H, L))
    for lp in FO.unpack(p, F, H, L):
        lp["b3"][F:] = 6.0   # t = 6: shift every transformed coordinate by 6
    fl.set_params(p)
    ess, used = fl.sample(seed=1, n_traj=n, alpha=0.0, min_ess_frac=0.1)
    assert not used and ess < 0.1
    got = ctx.read_initial()
    ctx.sample_husimi(seed=1, n_traj=n)
    ref = ctx.read_initial()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    fl.close()
    ctx.close()


def test_weighted_good_count_harmonic_proposal(scivr, oracle_mod):
    # non-Husimi points through set_initial: GPU matches the oracle, and both the
    # Husimi spectrum, thanks to the importance-weighted good count
    O = oracle_mod
    prob = inputs.harmonic([2000.0, 3100.0], n_steps=1024, dt=10.0, e_min=0.0, e_max=0.05, n_energies=400)
    F = prob.F
    rng = np.random.default_rng(8)
    sc, mu = 1.4, 0.3
    n = 200
    x = mu + sc * rng.normal(size=(2 * F, n))
    sg = np.sqrt(prob.gamma)[:, None]
    q1 = prob.q_eq[:, None] + x[:F] / sg
    p1 = prob.p_eq[:, None] + x[F:] * sg
    lr1 = -F * np.log(2 * np.pi) - 2 * F * np.log(sc) - 0.5 * np.sum((x - mu) ** 2, axis=0) / sc ** 2
    ctx = scivr.Context(prob, max_traj=n)
    ctx.set_initial(p1, q1, lr1)
    ctx.propagate()
    ctx.accumulate()
    I, ng, _ = ctx.read_spectrum()
    ora = O.run(prob, p1, q1, lr1)
    assert np.max(np.abs(I - ora.spectrum)) < 1e-9 * ora.spectrum.max()
    ctx.sample_husimi(seed=5, n_traj=64)
    ctx.reset_spectrum()
    ctx.propagate()
    ctx.accumulate()
    Ih, _, _ = ctx.read_spectrum()
    assert np.max(np.abs(I - Ih)) < 2e-3 * Ih.max()
    ctx.close()


def test_learned_proposal_spectrum_matches_plain(scivr):
    # F=2 Morse + coupling: train on one Husimi batch's contributions, sample
    # from the mixture, and compare with a large plain run
    prob = inputs.morse_quartic(2, 2, n_steps=1024, n_energies=512, e_max=0.05)
    n_plain, n = 32768, 8192
    ctx = scivr.Context(prob, max_traj=n_plain)
    ctx.run(seed=1, n_traj=n_plain)
    I_plain, _, _ = ctx.read_spectrum()
    fl = scivr.Flow(ctx, 4, 64, seed=7)
    ctx.reset_spectrum()
    ctx.run(seed=2, n_traj=n)
    loss = fl.train_on_batch(epochs=30, batch=2048, lr=2e-3)
    ctx.reset_spectrum()
    ess, used = fl.sample(seed=3, n_traj=n, alpha=0.1)
    ctx.propagate()
    ctx.accumulate()
    I_l, ng, nt = ctx.read_spectrum()
    T, E = prob.total_time, prob.energies()
    pr, pl = peaks.find_peaks(E, I_plain, T), peaks.find_peaks(E, I_l, T)
    worst, missing = peaks.peak_errors(pr, pl, tol=20 / CM)
    rel = np.max(np.abs(I_l - I_plain)) / I_plain.max()
    _say(f"[flow F=2] loss {loss:.4f} ess {ess:.3f} used {used} good {ng}/{nt}; peaks {len(pr)} "
         f"worst {worst * CM:.3f} cm^-1; max rel diff {rel:.3e}")
    assert used and ess > 0.1
    assert missing == 0 and worst * CM < 1.0
    assert rel < 0.05
    fl.close()
    ctx.close()


def _ratio_estimate(prob, ctx):
    """Integrated spectrum of the last batch as the ratio estimator
    sum_j c_j / sum_j good_j r_j (r_j = Husimi density / sampling density),
    with its delta-method standard error."""
    c = ctx.read_contributions()
    p0, q0, lr = ctx.read_initial()
    good = ctx.read_state()["good"].astype(bool)
    g = np.asarray(prob.gamma)[:, None]
    log_h = (-len(prob.gamma) * np.log(2.0 * np.pi)
             - 0.5 * np.sum(g * (q0 - np.asarray(prob.q_eq)[:, None]) ** 2
                            + (p0 - np.asarray(prob.p_eq)[:, None]) ** 2 / g, axis=0))
    r = np.where(good, np.exp(log_h - lr), 0.0)
    x = c.sum() / r.sum()
    n = len(c)
    se = np.std(c - x * r) / (np.sqrt(n) * r.mean())
    return x, se


def test_mixed_learned_pipeline_at_f30(scivr):
    """The F = 30 form end to end at reduced length: mixed-precision batch,
    a width-256 flow trained on its contributions, a mixture batch, and its
    spectrum.  Two independent Monte Carlo estimates are compared where their
    statistics are known: the integrated spectrum, within five standard errors."""
    prob = inputs.morse_quartic(30, 30, n_steps=200, n_energies=256, e_max=0.25,
                                precision=inputs.PRECISION_MIXED)
    n = 4096
    ctx = scivr.Context(prob, max_traj=n)
    ctx.run(seed=5, n_traj=n)
    I_h, ng_h, _ = ctx.read_spectrum()
    x_h, se_h = _ratio_estimate(prob, ctx)
    fl = scivr.Flow(ctx, 4, 256, seed=9)
    assert fl.n_params == 356592
    loss = fl.train_on_batch(epochs=5, batch=1024, lr=1e-3)
    ctx.reset_spectrum()
    ess, used = fl.sample(seed=6, n_traj=n, alpha=0.1)
    ctx.propagate()
    ctx.accumulate()
    I_l, ng_l, nt = ctx.read_spectrum()
    x_l, se_l = _ratio_estimate(prob, ctx)
    z = (x_l - x_h) / np.hypot(se_h, se_l)
    # the spectrum sums to the ratio estimate times one constant in both batches
    k_h, k_l = I_h.sum() / x_h, I_l.sum() / x_l
    rel = np.max(np.abs(I_l - I_h)) / I_h.max()
    _say(f"[flow F=30] loss {loss:.3f} ess {ess:.3f} used {used} good {ng_h}/{ng_l}; "
         f"integrated {x_h:.4e}+-{se_h:.1e} vs {x_l:.4e}+-{se_l:.1e} (z {z:.2f}); max rel diff {rel:.3e}")
    assert np.isfinite(loss) and used and ess > 0.1
    assert ng_l > 0.5 * nt and np.all(np.isfinite(I_l))
    assert abs(k_l / k_h - 1.0) < 1e-9
    assert abs(z) < 5.0
    assert rel < 0.3
    fl.close()
    ctx.close()
