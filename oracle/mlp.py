"""Learned control-variate level: a small MLP g that predicts the fine-level
quadratic form z^T p_n(A_hat) z from the cheap moments mu_0..mu_c of the same
probe (a project addition, not in the paper; it is the control-variate idea
of Section 5.4 with a learned instead of a linear map, used as one more
multilevel term in the sense of Section 2.3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

Network: x in R^{F} -> h1 = tanh(W1 x + b1) (H) -> h2 = tanh(W2 h1 + b2) (H)
-> out = w3 . h2 + b3.  Loss over a batch of N samples:
L = (1/N) sum_i (out_i - y_i)^2.  Gradients are derived by hand
(tanh' = 1 - tanh^2).  Optimiser: Adam (Kingma & Ba 2015) with bias
correction.

The library's g corrects the cheap truncation q_c = sum_{j<=c} c_j mu_j in
two stages on the standardised residual t = ((q - q_c)/mu_0 - ybar)/ysd:
inputs u_f = (mu_f/mu_0 - xmean_f)/xsd_f (f >= 1; ``standardize``), a
linear least-squares fit beta of t on u (``linear_stage``; the linear
control variate of Section 5.4), and the network on t - u.beta:
    g = q_c + mu_0 (ybar + ysd (u.beta + out(u))).
``fit_affine`` builds the affine stages from training moments and
``composite_g`` evaluates g (FP64, or with the inference's bfloat16
roundings of inputs, weights and hidden activations).

Estimator (unbiased for any fixed g): with disjoint probe sets S0 (cheap
degree, M0 probes) and S1 (fine degree, M1 probes), both disjoint from the
pilot that trained g,
    Gamma = (1/M0) sum_{S0} g(x) + (1/M1) sum_{S1} (q - g(x)),
    Var   = s0^2 / M0 + s1^2 / M1.
More generally g is one more level of the multilevel chain (Section 2.3,
eq. eqn:telescope): with S(l) the truncation of the fine interpolant to
degree l (eq. def:qlevels), except S(n_cheap) = g and S(-1) = 0, the level
variables S(l_k) - S(l_{k-1}) over independent probe sets telescope to
S(n_fine) = q (``chain_value``, ``learned_ml_estimate``), and
``learned_terms`` gives the pilot table on which the level-selection
programme of Theorem thm:levels places g among the Chebyshev levels.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Params:
    W1: np.ndarray  # [H, F]
    b1: np.ndarray  # [H]
    W2: np.ndarray  # [H, H]
    b2: np.ndarray  # [H]
    w3: np.ndarray  # [H]
    b3: float

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2, self.w3,
                               [self.b3]])

    @staticmethod
    def from_flat(v: np.ndarray, F: int, H: int) -> "Params":
        v = np.asarray(v, dtype=np.float64)
        o = 0
        W1 = v[o:o + H * F].reshape(H, F); o += H * F
        b1 = v[o:o + H]; o += H
        W2 = v[o:o + H * H].reshape(H, H); o += H * H
        b2 = v[o:o + H]; o += H
        w3 = v[o:o + H]; o += H
        return Params(W1.copy(), b1.copy(), W2.copy(), b2.copy(), w3.copy(), float(v[o]))


def standardize(Xraw: np.ndarray):
    """Column means and unbiased standard deviations of the raw inputs
    (rows = training probes); column 0 (mu_0 / mu_0 = 1) and constant
    columns get standard deviation 0, which maps them to 0."""
    Xraw = np.asarray(Xraw, dtype=np.float64)
    mean = Xraw.mean(axis=0)
    sd = Xraw.std(axis=0, ddof=1) if Xraw.shape[0] > 1 else np.zeros(Xraw.shape[1])
    mean[0], sd[0] = 0.0, 0.0
    sd = np.where(sd > 0.0, sd, 0.0)
    return mean, sd


def standardized(Xraw: np.ndarray, mean: np.ndarray, sd: np.ndarray) -> np.ndarray:
    Xraw = np.asarray(Xraw, dtype=np.float64)
    U = np.zeros_like(Xraw)
    ok = sd > 0.0
    U[:, ok] = (Xraw[:, ok] - mean[ok]) / sd[ok]
    return U


def linear_stage(U: np.ndarray, t: np.ndarray, ridge_rel: float = 1e-12) -> np.ndarray:
    """beta minimising |t - U beta|^2 over the inputs f >= 1 (beta_0 = 0),
    from the normal equations with a ridge of ridge_rel * trace / K on the
    diagonal (K = number of inputs), which leaves well-posed fits unchanged
    to rounding and makes constant (all-zero) inputs get beta = 0."""
    U = np.asarray(U, dtype=np.float64)[:, 1:]
    t = np.asarray(t, dtype=np.float64)
    K = U.shape[1]
    beta = np.zeros(K + 1)
    if K == 0:
        return beta
    G = U.T @ U
    G[np.diag_indices(K)] += ridge_rel * np.trace(G) / K + 1e-300
    beta[1:] = np.linalg.solve(G, U.T @ t)
    return beta


def n_params(F: int, H: int) -> int:
    return H * F + H + H * H + H + H + 1


def glorot_init(F: int, H: int, rng: np.random.Generator) -> Params:
    """Glorot-uniform weights, zero biases."""
    def u(fan_in, fan_out, shape):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=shape)
    return Params(u(F, H, (H, F)), np.zeros(H), u(H, H, (H, H)), np.zeros(H),
                  u(H, 1, (H,)), 0.0)


def forward(p: Params, X: np.ndarray):
    """Outputs [N] and the cached activations."""
    h1 = np.tanh(X @ p.W1.T + p.b1)
    h2 = np.tanh(h1 @ p.W2.T + p.b2)
    out = h2 @ p.w3 + p.b3
    return out, (h1, h2)


def loss_and_grad(p: Params, X: np.ndarray, y: np.ndarray):
    """Mean squared error and its gradient (same layout as Params.flat)."""
    N = X.shape[0]
    out, (h1, h2) = forward(p, X)
    r = out - y
    L = float(np.mean(r ** 2))
    g_out = 2.0 * r / N                          # dL/dout  [N]
    g_w3 = h2.T @ g_out                          # [H]
    g_b3 = float(np.sum(g_out))
    g_h2 = np.outer(g_out, p.w3)                 # [N, H]
    g_a2 = g_h2 * (1.0 - h2 ** 2)                # through tanh
    g_W2 = g_a2.T @ h1                           # [H, H]
    g_b2 = np.sum(g_a2, axis=0)
    g_h1 = g_a2 @ p.W2                           # [N, H]
    g_a1 = g_h1 * (1.0 - h1 ** 2)
    g_W1 = g_a1.T @ X                            # [H, F]
    g_b1 = np.sum(g_a1, axis=0)
    grad = Params(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)
    return L, grad.flat()


@dataclasses.dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_step(theta: np.ndarray, grad: np.ndarray, st: AdamState, lr=1e-3, b1=0.9,
              b2=0.999, eps=1e-8) -> np.ndarray:
    st.t += 1
    st.m = b1 * st.m + (1 - b1) * grad
    st.v = b2 * st.v + (1 - b2) * grad ** 2
    mhat = st.m / (1 - b1 ** st.t)
    vhat = st.v / (1 - b2 ** st.t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)


def train(p: Params, X: np.ndarray, y: np.ndarray, epochs: int, lr: float = 1e-3):
    """Full-batch Adam; returns trained params and the loss history."""
    F, H = X.shape[1], p.b1.size
    theta = p.flat()
    st = AdamState(np.zeros_like(theta), np.zeros_like(theta))
    hist = []
    for _ in range(epochs):
        L, g = loss_and_grad(Params.from_flat(theta, F, H), X, y)
        hist.append(L)
        theta = adam_step(theta, g, st, lr)
    return Params.from_flat(theta, F, H), hist


def learned_estimate(g_s0: np.ndarray, q_s1: np.ndarray, g_s1: np.ndarray):
    """(Gamma, Var) of the two-term estimator from per-probe values."""
    M0, M1 = len(g_s0), len(q_s1)
    d1 = q_s1 - g_s1
    val = float(np.mean(g_s0) + np.mean(d1))
    var = float(np.var(g_s0, ddof=1) / M0 + np.var(d1, ddof=1) / M1)
    return val, var


# ---- the library's composite g and the learned multilevel chain -------------

def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits, round to nearest, ties to even)
    through float32, returned as float64: the rounding the inference applies
    to its inputs, weights and hidden activations."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


@dataclasses.dataclass
class Affine:
    """Target and input standardisation and the linear stage of g."""
    ybar: float
    ysd: float
    xmean: np.ndarray  # [F]
    xsd: np.ndarray    # [F]
    lin: np.ndarray    # [F], lin[0] = 0


def fit_affine(mu: np.ndarray, c: np.ndarray, F: int) -> Affine:
    """The affine stages from the training probes' moments mu [N, n+1] and
    the fine interpolant's coefficients c [n+1]: t = (q - q_c)/mu_0
    standardised by its mean and unbiased standard deviation, inputs
    mu_f/mu_0 standardised by ``standardize``, and the linear fit of the
    standardised t on them (``linear_stage``)."""
    mu = np.asarray(mu, dtype=np.float64)
    r = (mu @ c - mu[:, :F] @ c[:F]) / mu[:, 0]
    ybar, ysd = float(r.mean()), float(r.std(ddof=1))
    Xraw = mu[:, :F] / mu[:, :1]
    xm, xs = standardize(Xraw)
    lin = linear_stage(standardized(Xraw, xm, xs), (r - ybar) / ysd)
    return Affine(ybar, ysd, xm, xs, lin)


def composite_g(mu: np.ndarray, c: np.ndarray, F: int, aff: Affine, p: Params,
                bf16: bool = True) -> np.ndarray:
    """g = q_c + mu_0 (ybar + ysd (u.beta + out(u))) per row of mu, with
    q_c = sum_{j<F} c_j mu_j and u the standardised inputs.  With bf16 the
    network's inputs, weights and hidden activations are rounded to bfloat16
    as the inference does (the affine parts stay FP64)."""
    mu = np.asarray(mu, dtype=np.float64)
    u = standardized(mu[:, :F] / mu[:, :1], aff.xmean[:F], aff.xsd[:F])
    lin = u @ aff.lin[:F]
    if bf16:
        r = bf16_round
        x = r(u)
        h1 = r(np.tanh(x @ r(p.W1).T + r(p.b1)))
        h2 = r(np.tanh(h1 @ r(p.W2).T + r(p.b2)))
        out = h2 @ r(p.w3) + float(r(p.b3))
    else:
        out, _ = forward(p, u)
    qc = mu[:, :F] @ c[:F]
    return qc + mu[:, 0] * (aff.ybar + aff.ysd * (lin + out))


def chain_value(mu: np.ndarray, c: np.ndarray, level: int, n_cheap: int,
                g: np.ndarray) -> np.ndarray:
    """S(l) per row: the truncation sum_{j<=l} c_j mu_j of the fine
    interpolant (eq. def:qlevels), except S(n_cheap) = g and S(-1) = 0."""
    mu = np.asarray(mu, dtype=np.float64)
    if level < 0:
        return np.zeros(mu.shape[0])
    if level == n_cheap:
        return np.asarray(g, dtype=np.float64)
    return mu[:, :level + 1] @ c[:level + 1]


def learned_ml_estimate(level_values):
    """(Gamma, Var) of the multilevel estimator (eq. eqn:multiEstimator) from
    the per-probe level variables S(l_k) - S(l_{k-1}) of each level."""
    val = float(sum(np.mean(q) for q in level_values))
    var = float(sum(np.var(q, ddof=1) / len(q) for q in level_values))
    return val, var


def learned_terms(mu: np.ndarray, c: np.ndarray, n_cheap: int, g: np.ndarray) -> np.ndarray:
    """Per-probe terms whose prefix sums are the chain values S(0..n), the
    pilot table on which the level-selection programme (Theorem thm:levels)
    decides where g enters the chain."""
    mu = np.asarray(mu, dtype=np.float64)
    n = mu.shape[1] - 1
    S = np.stack([chain_value(mu, c, l, n_cheap, g) for l in range(n + 1)], axis=1)
    return np.diff(np.concatenate([np.zeros((mu.shape[0], 1)), S], axis=1), axis=1)
