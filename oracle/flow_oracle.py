"""Plain FP64 numpy oracle of the learned importance-sampling proposal.

TEST INFRASTRUCTURE ONLY: the test-suite and the benchmark's CPU leg are the
only callers; the product path never imports this module, and it shares no
code with the HIP library.

The proposal is not part of the paper.  The paper samples initial phase-space
points from the Husimi distribution of the reference state and weights each
trajectory by the inverse of that density (the Monte Carlo average that
follows Eq. (11)); any other sampling density q keeps the estimator unbiased
if the weight becomes 1 / ((2 pi)^F q(z)).  Here q is an affine-coupling
normalising flow, written out in the plainest form:

Coordinates.  x = (xi_1..xi_F, eta_1..eta_F) with xi_i = sqrt(gamma_i)
(q_i - q_eq,i) and eta_i = (p_i - p_eq,i) / sqrt(gamma_i); the Husimi
density is the standard normal in x, and the map (p, q) -> x has unit
Jacobian, so densities in x are densities in (p, q).

Layers.  Layer l conditions on one half of x and transforms the other:
even l: condition on xi, transform eta; odd l: condition on eta, transform
xi.  Its network is a two-hidden-layer tanh MLP a -> (s_raw, t) of width H;
s = C tanh(s_raw / C) with C = 2 (a soft clamp of the log-scale).

Generation (u -> x), layers 0..L-1 in order: b <- b * exp(s(a)) + t(a);
log q(x) = log N(u) - sum over layers of sum_i s_i.
Density (x -> u), layers L-1..0: b <- (b - t(a)) * exp(-s(a)); the same
log q(x) = log N(u) - sum s.

Training is weighted maximum likelihood: given points x_j drawn from a
density r and their contributions c_j = w_j sum_k |A_jk|^2 (w_j = 1 /
((2 pi)^F r(x_j)), so c_j is proportional to the ideal density divided by
r), minimise L = - sum_j c_j log q(x_j) / sum_j c_j over contiguous
mini-batches of the data in order, with Adam (beta1 0.9, beta2 0.999,
eps 1e-8, bias-corrected).  A batch with sum c = 0 is skipped.

Sampling uses the defensive mixture alpha N(x) + (1 - alpha) q(x): point j
draws 2F normals exactly as the Husimi sampler does (Philox4x64-10, key
(seed, 0), counter (index, block, 0, 0), Box-Muller; xi_i from normal 2i,
eta_i from normal 2i + 1) and one uniform from counter (index, 0, 1, 0);
if that uniform is below alpha the point is the normal vector itself,
otherwise its image under the flow.

Parameter layout (one flat array): per layer W1 [H][F], b1 [H], W2 [H][H],
b2 [H], W3 [2F][H], b3 [2F]; rows of W3 0..F-1 give s_raw, F..2F-1 give t.

Parity pinned in tests/test_flow_oracle_pins.py: identity at zero output
layer, exact inversion, log-determinant against a finite-difference
Jacobian, normalisation by quadrature, gradient against finite differences,
the first Adam step in closed form, and recovery of a known target density.
"""
from __future__ import annotations

import math

import numpy as np

S_CLAMP = 2.0
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
LOG_2PI = math.log(2.0 * math.pi)


def layer_size(F: int, H: int) -> int:
    return H * F + H + H * H + H + 2 * F * H + 2 * F


def param_count(F: int, H: int, L: int) -> int:
    return L * layer_size(F, H)


def unpack(params, F: int, H: int, L: int):
    """Views W1, b1, W2, b2, W3, b3 of every layer into the flat array."""
    params = np.asarray(params, dtype=np.float64)
    assert params.size == param_count(F, H, L)
    out = []
    off = 0
    for _ in range(L):
        d = {}
        for name, shape in (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (2 * F, H)),
                            ("b3", (2 * F,))):
            size = int(np.prod(shape))
            d[name] = params[off:off + size].reshape(shape)
            off += size
        out.append(d)
    return out


def halves(F: int, layer: int):
    """(conditioning indices, transformed indices) of layer `layer`."""
    xi = np.arange(F)
    eta = np.arange(F, 2 * F)
    return (xi, eta) if layer % 2 == 0 else (eta, xi)


def net(lp, a):
    """The layer network on rows a [n][F]: returns s, t and the hidden activations."""
    h1 = np.tanh(a @ lp["W1"].T + lp["b1"])
    h2 = np.tanh(h1 @ lp["W2"].T + lp["b2"])
    o = h2 @ lp["W3"].T + lp["b3"]
    F = a.shape[1]
    s = S_CLAMP * np.tanh(o[:, :F] / S_CLAMP)
    t = o[:, F:]
    return s, t, h1, h2


def log_normal(u):
    """log N(u; 0, I) per row."""
    D = u.shape[1]
    return -0.5 * D * LOG_2PI - 0.5 * np.sum(u * u, axis=1)


def generate(params, F: int, H: int, L: int, u):
    """u [n][2F] -> (x [n][2F], log q(x) [n])."""
    lps = unpack(params, F, H, L)
    x = np.array(u, dtype=np.float64, copy=True)
    sum_s = np.zeros(x.shape[0])
    for l in range(L):
        ci, ti = halves(F, l)
        s, t, _, _ = net(lps[l], x[:, ci])
        x[:, ti] = x[:, ti] * np.exp(s) + t
        sum_s += s.sum(axis=1)
    return x, log_normal(u) - sum_s


def density(params, F: int, H: int, L: int, x):
    """x [n][2F] -> (u [n][2F], log q(x) [n])."""
    lps = unpack(params, F, H, L)
    z = np.array(x, dtype=np.float64, copy=True)
    sum_s = np.zeros(z.shape[0])
    for l in reversed(range(L)):
        ci, ti = halves(F, l)
        s, t, _, _ = net(lps[l], z[:, ci])
        z[:, ti] = (z[:, ti] - t) * np.exp(-s)
        sum_s += s.sum(axis=1)
    return z, log_normal(z) - sum_s


def loss_and_grad(params, F: int, H: int, L: int, x, c):
    """Weighted negative log-likelihood L = -sum c_j log q(x_j) / sum c_j and dL/dparams.

    Reverse-mode differentiation of the density pass written out by hand.
    Returns (L, grad); (0, zeros) if sum c = 0.
    """
    params = np.asarray(params, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    csum = c.sum()
    grad = np.zeros_like(params)
    if csum == 0.0:
        return 0.0, grad
    m = -c / csum                           # dL / d log q_j
    lps = unpack(params, F, H, L)
    gps = unpack(grad, F, H, L)             # views into grad
    # forward (density direction), keeping what the backward pass needs
    z = x.copy()
    saved = [None] * L
    sum_s = np.zeros(z.shape[0])
    for l in reversed(range(L)):
        ci, ti = halves(F, l)
        a = z[:, ci].copy()
        s, t, h1, h2 = net(lps[l], a)
        b = (z[:, ti] - t) * np.exp(-s)
        z[:, ti] = b
        sum_s += s.sum(axis=1)
        saved[l] = (a, s, h1, h2, b)
    u = z
    logq = log_normal(u) - sum_s
    loss = float(np.dot(m, logq))
    # backward: g = dL/dz, starting from log N(u) = -|u|^2 / 2 + const
    g = -u * m[:, None]
    for l in range(L):
        ci, ti = halves(F, l)
        a, s, h1, h2, b = saved[l]
        lp, gp = lps[l], gps[l]
        g_b = g[:, ti]
        e = np.exp(-s)
        g_bin = g_b * e                            # d/d(b before this inverse step)
        g_t = -g_b * e
        g_s = -g_b * b - m[:, None]                # through b and through -sum s
        g_sraw = g_s * (1.0 - (s / S_CLAMP) ** 2)
        g_o = np.concatenate([g_sraw, g_t], axis=1)
        gp["W3"] += g_o.T @ h2
        gp["b3"] += g_o.sum(axis=0)
        g_p2 = (g_o @ lp["W3"]) * (1.0 - h2 * h2)
        gp["W2"] += g_p2.T @ h1
        gp["b2"] += g_p2.sum(axis=0)
        g_p1 = (g_p2 @ lp["W2"]) * (1.0 - h1 * h1)
        gp["W1"] += g_p1.T @ a
        gp["b1"] += g_p1.sum(axis=0)
        g_a = g[:, ci] + g_p1 @ lp["W1"]
        g = np.empty_like(g)
        g[:, ci] = g_a
        g[:, ti] = g_bin
    return loss, grad


class Adam:
    """Adam with bias correction; the state is (m, v, t)."""

    def __init__(self, n: int):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0

    def step(self, params, grad, lr: float):
        self.t += 1
        self.m = ADAM_B1 * self.m + (1.0 - ADAM_B1) * grad
        self.v = ADAM_B2 * self.v + (1.0 - ADAM_B2) * grad * grad
        mh = self.m / (1.0 - ADAM_B1 ** self.t)
        vh = self.v / (1.0 - ADAM_B2 ** self.t)
        return params - lr * mh / (np.sqrt(vh) + ADAM_EPS)


def train(params, F: int, H: int, L: int, x, c, epochs: int, batch: int, lr: float, adam: Adam = None):
    """Contiguous mini-batches [b*batch, (b+1)*batch) of the data in order, every epoch.
    Returns (params, adam, losses)."""
    params = np.array(params, dtype=np.float64, copy=True)
    adam = adam or Adam(params.size)
    n = x.shape[0]
    losses = []
    for _ in range(epochs):
        for b0 in range(0, n, batch):
            xb, cb = x[b0:b0 + batch], c[b0:b0 + batch]
            if cb.sum() == 0.0:
                continue
            loss, grad = loss_and_grad(params, F, H, L, xb, cb)
            params = adam.step(params, grad, lr)
            losses.append(loss)
    return params, adam, losses


def whiten(prob, p0, q0):
    """(p0 [F][n], q0 [F][n]) -> x [n][2F]."""
    sg = np.sqrt(np.asarray(prob.gamma, dtype=np.float64))[:, None]
    xi = sg * (np.asarray(q0) - np.asarray(prob.q_eq)[:, None])
    eta = (np.asarray(p0) - np.asarray(prob.p_eq)[:, None]) / sg
    return np.concatenate([xi, eta], axis=0).T.copy()


def unwhiten(prob, x):
    """x [n][2F] -> (p0 [F][n], q0 [F][n])."""
    F = len(prob.gamma)
    sg = np.sqrt(np.asarray(prob.gamma, dtype=np.float64))[:, None]
    q0 = np.asarray(prob.q_eq)[:, None] + x[:, :F].T / sg
    p0 = np.asarray(prob.p_eq)[:, None] + x[:, F:].T * sg
    return p0, q0


def mixture_log_density(x, logq, alpha: float):
    """log(alpha N(x) + (1 - alpha) q(x))."""
    ln = log_normal(x)
    if alpha >= 1.0:
        return ln
    if alpha <= 0.0:
        return np.array(logq, dtype=np.float64)
    return np.logaddexp(math.log(alpha) + ln, math.log1p(-alpha) + logq)


def draw(seed: int, first_index: int, n: int, F: int):
    """Normals u [n][2F] and selection uniforms v [n] of points first_index..first_index+n-1."""
    from oracle import oracle as O  # Philox4x64-10 and Box-Muller of the C oracle
    u = np.zeros((n, 2 * F))
    v = np.zeros(n)
    for j in range(n):
        z = O.normals(seed, first_index + j, 2 * F)
        u[j, :F] = z[0::2]
        u[j, F:] = z[1::2]
        r = O.philox4x64_10([first_index + j, 0, 1, 0], [seed, 0])
        v[j] = ((int(r[0]) >> 11) + 0.5) * (1.0 / 9007199254740992.0)
    return u, v


def sample(prob, params, H: int, L: int, seed: int, first_index: int, n: int, alpha: float):
    """Mixture samples: (p0 [F][n], q0 [F][n], log density [n], from_normal [n] bool, x [n][2F])."""
    F = len(prob.gamma)
    u, v = draw(seed, first_index, n, F)
    xf, _ = generate(params, F, H, L, u)
    from_normal = v < alpha
    x = np.where(from_normal[:, None], u, xf)
    _, logq = density(params, F, H, L, x)
    lr = mixture_log_density(x, logq, alpha)
    p0, q0 = unwhiten(prob, x)
    return p0, q0, lr, from_normal, x


def ess_fraction(x, log_density):
    """ESS / n of the ratios N(x_j) / density(x_j)."""
    r = np.exp(log_normal(x) - np.asarray(log_density))
    return float(r.sum() ** 2 / (r.size * np.sum(r * r)))
