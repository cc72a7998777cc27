"""FP64 oracle of the learned proposal: scene encoding, network, Gaussian NLL, backward pass, Adam
and the Gaussian parameter draws.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: it checks the HIP proposal kernels and is
never called by the product path.

The paper samples controller parameters without a learned prior and names better-guided sampling
and warm starts from offline encodings as future work (Sect. V). The proposal implemented here is
that extension: a network maps an encoding of the planning problem to a diagonal Gaussian over the
controller parameters theta, and is trained on the plain planner's best samples theta*.

Definitions (all in FP64 unless a quantisation step says otherwise):

Encoding e (72 values) of a problem (z0, goal, a_prev, points, T), in the vehicle frame at z0
(the planner is invariant under rigid motions of the whole scene, so the encoding is too):
  e[0:4]   = [v0 / dv, a_prev[0], a_prev[1], T / 100]
  e[4:8]   = [xi_g / dxi, eta_g / deta, wrap(phi_g - phi0) / dphi, v_g / dv]
  e[8:72]  = 16 blocks [xi_j / d_cap, eta_j / d_cap, vxi_j / dv, veta_j / dv] for the 16 points
             nearest to (x0, y0) at the sampling time, ascending distance, lower index first on
             equal distance; missing points (P < 16) are the block [100 / d_cap, 0, 0, 0].
  (dxi, deta, dphi, dv, d_cap are the planner's feature normalisers of eq. (3) / Table II.)

Network: h1 = relu(W1 q(e) + b1), h2 = relu(W2 q(h1) + b2), y = W3 q(h2) + b3 with widths
72 -> 256 -> 256 -> 2 n_theta; mu = y[:n_theta], s = log sigma = y[n_theta:]. q() rounds to
bfloat16 (round to nearest, ties to even) and is applied to every matrix-product operand
(weights, activations and back-propagated gradients), matching a BF16 matrix-core pipeline with
wide accumulation; biases, sums and the loss stay wide. ``quant=False`` drops every q().

Loss over a batch of B labelled problems: L = (1/B) sum_b sum_k [ (theta*_bk - mu_bk)^2
exp(-2 s_bk) / 2 + s_bk ] (the Gaussian negative log-likelihood without its constant).

Adam (Kingma and Ba, 2015) with bias correction: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Gaussian draws: theta_k = mu_k + exp(s_k) z_k with z from the Box-Muller transform (Box and
Muller, 1958) of two uniforms u = (m + 1/2) 2^-23 (m the top 23 bits of a Philox4x32-10 word, so
that u is an exact binary32 value):
parameter k of sample i uses block (k >> 2, i, 1, inst) under key = seed, words (0, 1) for
k & 3 in {0, 1} and words (2, 3) for k & 3 in {2, 3}; z = sqrt(-2 ln u_a) cos(2 pi u_b) for even
k, the sine for odd k.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

ENC_DIM = 72
N_NEAR = 16
HIDDEN = 256
FAR = 100.0


# ------------------------------------------------------------------------------------------------
# bfloat16 rounding
# ------------------------------------------------------------------------------------------------
def bf16(x) -> np.ndarray:
    """Round every value to the nearest bfloat16 (8 significant bits, ties to even), returned as
    float64. Values below the smallest normal bfloat16 keep the subnormal spacing 2^-133."""
    x = np.asarray(x, np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    _, e = np.frexp(x[nz])                      # x = f 2^e, 0.5 <= |f| < 1
    step = np.ldexp(1.0, np.maximum(e, -125) - 8)
    out[nz] = np.round(x[nz] / step) * step     # numpy rounds halves to even
    out[~nz] = x[~nz]
    return out


def q(x, quant: bool):
    return bf16(x) if quant else np.asarray(x, np.float64)


# ------------------------------------------------------------------------------------------------
# Encoding
# ------------------------------------------------------------------------------------------------
def wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def nearest(z0, points, n=N_NEAR) -> np.ndarray:
    """Indices of the n points nearest to (x0, y0), ascending distance, lower index on ties."""
    pts = np.asarray(points, np.float64).reshape(-1, 4)
    d2 = (pts[:, 0] - z0[0]) ** 2 + (pts[:, 1] - z0[1]) ** 2
    order = np.lexsort((np.arange(len(pts)), d2))
    return order[:n]


def encode(norms: dict, z0, goal, a_prev, points, T: int, idx=None) -> np.ndarray:
    """The 72-value encoding of one problem. `idx` overrides the nearest-point selection (used to
    evaluate the encoding at another implementation's choice among near-equal distances)."""
    z0 = np.asarray(z0, np.float64)
    goal = np.asarray(goal, np.float64)
    pts = np.asarray(points, np.float64).reshape(-1, 4)
    c, s = math.cos(z0[2]), math.sin(z0[2])
    dxi, deta, dphi, dv, dcap = (norms[k] for k in ("norm_xi", "norm_eta", "norm_phi", "norm_v",
                                                    "d_cap"))
    e = np.empty(ENC_DIM)
    e[0:4] = [z0[3] / dv, a_prev[0], a_prev[1], T / 100.0]
    gx, gy = goal[0] - z0[0], goal[1] - z0[1]
    e[4:8] = [(c * gx + s * gy) / dxi, (-s * gx + c * gy) / deta, wrap(goal[2] - z0[2]) / dphi,
              goal[3] / dv]
    if idx is None:
        idx = nearest(z0, pts)
    for j in range(N_NEAR):
        b = 8 + 4 * j
        if j < len(idx):
            p = pts[idx[j]]
            dx, dy = p[0] - z0[0], p[1] - z0[1]
            e[b:b + 4] = [(c * dx + s * dy) / dcap, (-s * dx + c * dy) / dcap,
                          (c * p[2] + s * p[3]) / dv, (-s * p[2] + c * p[3]) / dv]
        else:
            e[b:b + 4] = [FAR / dcap, 0.0, 0.0, 0.0]
    return e


# ------------------------------------------------------------------------------------------------
# Network, loss, gradients
# ------------------------------------------------------------------------------------------------
def forward(params: dict, X, quant: bool = True) -> dict:
    """Forward pass for a batch X [B][72]; returns every intermediate (pre-activations a1, a2,
    activations h1, h2, output y, and the quantised operands)."""
    X = np.asarray(X, np.float64)
    W1, W2, W3 = (q(params[k], quant) for k in ("W1", "W2", "W3"))
    x_q = q(X, quant)
    a1 = x_q @ W1.T + params["b1"]
    h1 = np.maximum(a1, 0.0)
    h1_q = q(h1, quant)
    a2 = h1_q @ W2.T + params["b2"]
    h2 = np.maximum(a2, 0.0)
    h2_q = q(h2, quant)
    y = h2_q @ W3.T + params["b3"]
    return dict(x_q=x_q, a1=a1, h1=h1, h1_q=h1_q, a2=a2, h2=h2, h2_q=h2_q, y=y)


def nll(y, theta_star) -> tuple:
    """Mean Gaussian NLL over the batch and its gradient with respect to y = [mu, s]."""
    y = np.asarray(y, np.float64)
    t = np.asarray(theta_star, np.float64)
    B, n2 = y.shape
    nt = n2 // 2
    mu, s = y[:, :nt], y[:, nt:]
    r = t - mu
    w = np.exp(-2.0 * s)
    L = float(np.sum(0.5 * r * r * w + s)) / B
    dy = np.empty_like(y)
    dy[:, :nt] = -r * w / B
    dy[:, nt:] = (1.0 - r * r * w) / B
    return L, dy


def backward(params: dict, cache: dict, dy, quant: bool = True) -> dict:
    """Gradients of the loss with respect to every parameter, given dL/dy."""
    dy = np.asarray(dy, np.float64)
    W2, W3 = q(params["W2"], quant), q(params["W3"], quant)
    dy_q = q(dy, quant)
    g = {"W3": dy_q.T @ cache["h2_q"], "b3": dy.sum(0)}
    dh2 = dy_q @ W3
    da2 = dh2 * (cache["a2"] > 0)
    da2_q = q(da2, quant)
    g["W2"] = da2_q.T @ cache["h1_q"]
    g["b2"] = da2.sum(0)
    dh1 = da2_q @ W2
    da1 = dh1 * (cache["a1"] > 0)
    da1_q = q(da1, quant)
    g["W1"] = da1_q.T @ cache["x_q"]
    g["b1"] = da1.sum(0)
    return g


def adam(params: dict, grads: dict, m: dict, v: dict, t: int, lr: float, beta1: float = 0.9,
         beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam step (step number t >= 1), in place on params, m and v."""
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for k in params:
        g = np.asarray(grads[k], np.float64)
        m[k] = beta1 * m[k] + (1.0 - beta1) * g
        v[k] = beta2 * v[k] + (1.0 - beta2) * g * g
        params[k] = params[k] - lr * (m[k] / c1) / (np.sqrt(v[k] / c2) + eps)


def init_params(n_theta: int, seed: int, enc_dim: int = ENC_DIM, hidden: int = HIDDEN,
                log_sigma0: float = math.log(1.0 / math.sqrt(3.0))) -> dict:
    """A seeded starting point: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero hidden
    biases, output biases mu = 0 and s = log of the uniform(-1, 1) standard deviation."""
    rng = np.random.default_rng([int(seed), 0x9A0])
    u = lambda shape, fan: rng.uniform(-1.0, 1.0, shape) / math.sqrt(fan)  # noqa: E731
    p = {"W1": u((hidden, enc_dim), enc_dim), "b1": np.zeros(hidden),
         "W2": u((hidden, hidden), hidden), "b2": np.zeros(hidden),
         "W3": u((2 * n_theta, hidden), hidden) * 0.1,
         "b3": np.concatenate([np.zeros(n_theta), np.full(n_theta, log_sigma0)])}
    # values the device holds exactly (float32)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


# ------------------------------------------------------------------------------------------------
# Gaussian parameter draws
# ------------------------------------------------------------------------------------------------
def normals(seed: int, inst: int, i0: int, n: int, n_theta: int) -> np.ndarray:
    """Standard normal draws z[n][n_theta] of samples i0..i0+n-1 (stream 1, Box-Muller)."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty((n, n_theta))
    for r in range(n):
        for b in range((n_theta + 3) // 4):
            w = philox((b, i0 + r, 1, inst), key)
            for k in range(4 * b, min(4 * b + 4, n_theta)):
                pa = 2 * ((k & 3) >> 1)
                ua = ((w[pa] >> 9) + 0.5) * 2.0 ** -23
                ub = ((w[pa + 1] >> 9) + 0.5) * 2.0 ** -23
                rad = math.sqrt(-2.0 * math.log(ua))
                ang = 2.0 * math.pi * ub
                out[r, k] = rad * (math.cos(ang) if k % 2 == 0 else math.sin(ang))
    return out


def sample(mu, log_sigma, seed: int, inst: int, i0: int, n: int) -> np.ndarray:
    """theta[n][n_theta] = mu + exp(log_sigma) z."""
    mu = np.asarray(mu, np.float64)
    z = normals(seed, inst, i0, n, len(mu))
    return mu[None, :] + np.exp(np.asarray(log_sigma, np.float64))[None, :] * z


# ------------------------------------------------------------------------------------------------
# Flat parameter vector: W1 [256][72], b1, W2 [256][256], b2, W3 [2 n_theta][256], b3
# ------------------------------------------------------------------------------------------------
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], np.float64).ravel() for k in ORDER])


def unflatten(vec, n_theta: int, enc_dim: int = ENC_DIM, hidden: int = HIDDEN) -> dict:
    shapes = {"W1": (hidden, enc_dim), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (2 * n_theta, hidden), "b3": (2 * n_theta,)}
    vec = np.asarray(vec, np.float64)
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = vec[o:o + n].reshape(shapes[k]).copy()
        o += n
    assert o == len(vec), (o, len(vec))
    return out
