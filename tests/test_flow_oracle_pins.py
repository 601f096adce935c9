"""Pins of the flow oracle (learned importance-sampling proposal) against
what the mathematics fixes: identity at a zero output layer, exact inversion,
the log-determinant against a finite-difference Jacobian, normalisation by
quadrature, the gradient against finite differences, Adam's closed-form first
steps, recovery of a known target density and unbiasedness of the mixture
weights.
"""
import math

import numpy as np
import pytest

from oracle import flow_oracle as FO
from paper_1312_4698_amd import inputs


def _params(F, H, L, seed, scale_out=0.3, scale_in=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(FO.param_count(F, H, L))
    for lp in FO.unpack(p, F, H, L):
        lp["W1"][:] = rng.normal(size=lp["W1"].shape) * scale_in / math.sqrt(F)
        lp["b1"][:] = rng.normal(size=lp["b1"].shape) * 0.1
        lp["W2"][:] = rng.normal(size=lp["W2"].shape) * scale_in / math.sqrt(H)
        lp["b2"][:] = rng.normal(size=lp["b2"].shape) * 0.1
        lp["W3"][:] = rng.normal(size=lp["W3"].shape) * scale_out / math.sqrt(H)
        lp["b3"][:] = rng.normal(size=lp["b3"].shape) * scale_out
    return p


def test_param_count_matches_layout():
    # 4 layers of 9 -> 128 -> 128 -> 18: about 80 k parameters
    assert FO.param_count(9, 128, 4) == 4 * (9 * 128 + 128 + 128 * 128 + 128 + 18 * 128 + 18) == 80456


def test_zero_output_layer_is_identity():
    F, H, L = 3, 16, 4
    p = _params(F, H, L, 1)
    for lp in FO.unpack(p, F, H, L):
        lp["W3"][:] = 0.0
        lp["b3"][:] = 0.0
    u = np.random.default_rng(2).normal(size=(50, 2 * F))
    x, lq = FO.generate(p, F, H, L, u)
    assert np.array_equal(x, u)
    ref = -F * math.log(2 * math.pi) - 0.5 * np.sum(u * u, axis=1)
    assert np.allclose(lq, ref, rtol=0, atol=1e-13)
    z, lq2 = FO.density(p, F, H, L, u)
    assert np.array_equal(z, u) and np.allclose(lq2, ref, rtol=0, atol=1e-13)


def test_density_inverts_generation():
    F, H, L = 4, 12, 4
    p = _params(F, H, L, 3, scale_out=0.6)
    u = np.random.default_rng(4).normal(size=(200, 2 * F))
    x, lq = FO.generate(p, F, H, L, u)
    assert np.max(np.abs(x - u)) > 0.1  # the map is not trivial
    z, lq2 = FO.density(p, F, H, L, x)
    assert np.max(np.abs(z - u)) < 1e-12
    assert np.max(np.abs(lq - lq2)) < 1e-12


def test_log_determinant_against_fd_jacobian():
    F, H, L = 2, 10, 4
    p = _params(F, H, L, 5, scale_out=0.8)
    rng = np.random.default_rng(6)
    h = 1e-6
    for _ in range(5):
        u = rng.normal(size=(1, 2 * F))
        J = np.zeros((2 * F, 2 * F))
        for k in range(2 * F):
            e = np.zeros((1, 2 * F))
            e[0, k] = h
            J[:, k] = (FO.generate(p, F, H, L, u + e)[0][0] - FO.generate(p, F, H, L, u - e)[0][0]) / (2 * h)
        _, lq = FO.generate(p, F, H, L, u)
        lnN = -F * math.log(2 * math.pi) - 0.5 * float(np.sum(u * u))
        logdet = lnN - lq[0]  # generation: log q = log N(u) - log|det dx/du|
        assert abs(logdet - math.log(abs(np.linalg.det(J)))) < 1e-7


def test_density_normalised_by_quadrature():
    F, H, L = 1, 8, 4
    p = _params(F, H, L, 7, scale_out=0.5)
    g = np.linspace(-9.0, 9.0, 721)
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel()], axis=1)
    _, lq = FO.density(p, F, H, L, x)
    dx = g[1] - g[0]
    total = np.exp(lq).sum() * dx * dx
    assert abs(total - 1.0) < 1e-5


def test_gradient_against_finite_differences():
    F, H, L = 2, 6, 4
    p = _params(F, H, L, 8, scale_out=0.5)
    rng = np.random.default_rng(9)
    x = rng.normal(size=(24, 2 * F)) * 1.3
    c = rng.exponential(size=24)
    c[3] = 0.0
    loss, grad = FO.loss_and_grad(p, F, H, L, x, c)
    _, lq = FO.density(p, F, H, L, x)
    assert abs(loss + np.dot(c, lq) / c.sum()) < 1e-12
    eps = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        pp = p.copy()
        pp[i] += eps
        lp = FO.loss_and_grad(pp, F, H, L, x, c)[0]
        pp[i] -= 2 * eps
        lm = FO.loss_and_grad(pp, F, H, L, x, c)[0]
        fd[i] = (lp - lm) / (2 * eps)
    assert np.max(np.abs(fd - grad)) < 1e-7 * max(1.0, np.max(np.abs(grad)))


def test_zero_weights_give_zero_gradient():
    F, H, L = 2, 4, 2
    p = _params(F, H, L, 10)
    loss, grad = FO.loss_and_grad(p, F, H, L, np.ones((5, 4)), np.zeros(5))
    assert loss == 0.0 and not np.any(grad)


def test_adam_first_steps_closed_form():
    # with a constant gradient g, every bias-corrected Adam step is -lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, 0.0, -20.0])
    a = FO.Adam(g.size)
    p = np.zeros(g.size)
    lr = 0.01
    for k in range(1, 4):
        p = a.step(p, g, lr)
        expect = -k * lr * g / (np.abs(g) + FO.ADAM_EPS)
        assert np.allclose(p, expect, rtol=1e-12, atol=1e-15)


def test_weighted_mle_recovers_gaussian_target():
    # points from N(0, I) weighted by N(x; mu, diag sd^2) / N(x; 0, I): the ideal
    # density is that Gaussian; after training the flow's mean and spread follow it.
    F, H, L = 1, 16, 4
    rng = np.random.default_rng(11)
    mu = np.array([0.5, -0.3])
    sd = np.array([0.7, 1.2])
    x = rng.normal(size=(4000, 2))
    logt = -np.sum(np.log(sd)) - 0.5 * np.sum(((x - mu) / sd) ** 2, axis=1)
    c = np.exp(logt + 0.5 * np.sum(x * x, axis=1))
    p0 = _params(F, H, L, 12)
    for lp in FO.unpack(p0, F, H, L):
        lp["W3"][:] = 0.0
        lp["b3"][:] = 0.0
    p, _, losses = FO.train(p0, F, H, L, x, c, epochs=300, batch=4000, lr=1e-2)
    assert losses[-1] < losses[0] - 0.05
    u = rng.normal(size=(20000, 2))
    xs, _ = FO.generate(p, F, H, L, u)
    assert np.all(np.abs(xs.mean(axis=0) - mu) < 0.08)
    assert np.all(np.abs(xs.std(axis=0) - sd) < 0.1)


def test_alpha_one_reproduces_husimi_sampler(oracle_mod):
    O = oracle_mod
    prob = inputs.morse_quartic(3, 3, n_steps=10, n_energies=8)
    F, H, L = 3, 8, 4
    p = _params(F, H, L, 13)
    p0, q0, lr, fromN, _ = FO.sample(prob, p, H, L, seed=21, first_index=5, n=40, alpha=1.0)
    hp, hq, hl = O.sample_husimi(prob, 21, 40, first_index=5)
    assert fromN.all()
    assert np.allclose(p0, hp, rtol=1e-15, atol=1e-15) and np.allclose(q0, hq, rtol=1e-15, atol=1e-15)
    assert np.allclose(lr, hl, rtol=0, atol=1e-12)


def test_mixture_weights_unbiased():
    # E over the mixture of N(x) / density(x) is 1 (importance weights of the
    # Husimi target); the selection frequency is alpha.
    prob = inputs.morse_quartic(2, 2, n_steps=10, n_energies=8)
    F, H, L = 2, 8, 4
    p = _params(F, H, L, 14, scale_out=0.4)
    n = 4000
    _, _, lr, fromN, x = FO.sample(prob, p, H, L, seed=3, first_index=0, n=n, alpha=0.3)
    r = np.exp(FO.log_normal(x) - lr)
    se = r.std() / math.sqrt(n)
    assert abs(r.mean() - 1.0) < 4 * se + 1e-3
    assert abs(fromN.mean() - 0.3) < 4 * math.sqrt(0.21 / n)
    assert 0.0 < FO.ess_fraction(x, lr) <= 1.0
