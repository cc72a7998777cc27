"""Pins of the proposal oracle (oracle/proposal.py) against independent definitions: torch's own
bfloat16 conversion and autograd, torch.optim.Adam, brute-force sorting, hand-computed encodings,
finite differences and the normal distribution."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import proposal as P

NORMS = dict(norm_xi=30.0, norm_eta=3.5, norm_phi=2.0 * math.pi, norm_v=120.0 / 3.6, d_cap=20.0)


# ------------------------------------------------------------------------------------------------
# bfloat16 rounding
# ------------------------------------------------------------------------------------------------
def test_bf16_matches_torch_conversion_of_float32():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.standard_normal(1000)]).astype(np.float32)
    # exact halfway cases (low 16 bits 0x8000) exercise ties-to-even in both directions
    bits = x.view(np.uint32)
    ties = ((bits[:4000] & 0xFFFF0000) | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, -2.5, 3.0e38])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = P.bf16(x.astype(np.float64))
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])


def test_bf16_idempotent_and_monotone():
    rng = np.random.default_rng(1)
    x = np.sort(rng.standard_normal(5000))
    q = P.bf16(x)
    assert np.array_equal(P.bf16(q), q)
    assert np.all(np.diff(q) >= 0)
    assert np.all(np.abs(q - x) <= np.abs(x) * 2.0 ** -8)


# ------------------------------------------------------------------------------------------------
# Encoding
# ------------------------------------------------------------------------------------------------
def test_nearest_against_brute_force_with_ties():
    rng = np.random.default_rng(2)
    pts = np.zeros((300, 4))
    pts[:, :2] = rng.integers(-20, 20, (300, 2))     # many exactly equal distances
    z0 = np.array([0.5, -0.5, 0.3, 1.0])
    idx = P.nearest(z0, pts)
    d2 = [((p[0] - z0[0]) ** 2 + (p[1] - z0[1]) ** 2, i) for i, p in enumerate(pts)]
    assert list(idx) == [i for _, i in sorted(d2)[:16]]


def test_encoding_hand_computed():
    # heading pi/2: body axis xi points along +y, eta along -x
    z0 = np.array([1.0, 2.0, math.pi / 2, 3.0])
    goal = np.array([1.0, 12.0, -math.pi / 2, 2.0])
    pts = np.array([[4.0, 2.0, 0.0, 5.0],     # 3 m to the right (world +x): xi 0, eta -3
                    [1.0, 0.0, 1.0, 0.0]])    # 2 m behind: xi -2, eta 0
    e = P.encode(NORMS, z0, goal, [0.25, -0.5], pts, 50)
    dv = 120.0 / 3.6
    assert np.allclose(e[:4], [3.0 / dv, 0.25, -0.5, 0.5], atol=1e-15)
    assert np.allclose(e[4:8], [10.0 / 30.0, 0.0, -0.5, 2.0 / dv], atol=1e-15)
    # nearest first: the point behind (2 m), then the one to the side (3 m)
    assert np.allclose(e[8:12], [-2.0 / 20.0, 0.0, 0.0, -1.0 / dv], atol=1e-15)
    assert np.allclose(e[12:16], [0.0, -3.0 / 20.0, 5.0 / dv, 0.0], atol=1e-15)
    assert np.allclose(e[16:], np.tile([100.0 / 20.0, 0, 0, 0], 14))


def test_encoding_rigid_motion_invariance():
    rng = np.random.default_rng(3)
    z0 = np.array([0.0, 0.0, 0.4, 7.0])
    goal = np.array([30.0, -10.0, 2.0, 0.0])
    pts = np.column_stack([rng.uniform(-30, 30, (100, 2)), rng.uniform(-5, 5, (100, 2))])
    e0 = P.encode(NORMS, z0, goal, [0.1, 0.2], pts, 40)
    a, tx, ty = 1.1, 12.0, -40.0
    c, s = math.cos(a), math.sin(a)
    R = np.array([[c, -s], [s, c]])
    z1 = np.array([*(R @ z0[:2] + [tx, ty]), P.wrap(z0[2] + a), z0[3]])
    g1 = np.array([*(R @ goal[:2] + [tx, ty]), P.wrap(goal[2] + a), goal[3]])
    p1 = np.column_stack([pts[:, :2] @ R.T + [tx, ty], pts[:, 2:] @ R.T])
    e1 = P.encode(NORMS, z1, g1, [0.1, 0.2], p1, 40)
    assert np.allclose(e0, e1, atol=1e-12)


# ------------------------------------------------------------------------------------------------
# Network, loss, gradients
# ------------------------------------------------------------------------------------------------
def small_params(rng, enc=7, hidden=5, nt=3):
    return {"W1": rng.standard_normal((hidden, enc)) * 0.5, "b1": rng.standard_normal(hidden) * 0.1,
            "W2": rng.standard_normal((hidden, hidden)) * 0.5, "b2": rng.standard_normal(hidden) * 0.1,
            "W3": rng.standard_normal((2 * nt, hidden)) * 0.5,
            "b3": rng.standard_normal(2 * nt) * 0.1}


def loss_of(params, X, T, quant=False):
    return P.nll(P.forward(params, X, quant)["y"], T)[0]


def test_forward_and_gradients_against_torch_autograd():
    rng = np.random.default_rng(4)
    nt = 1410
    params = P.init_params(nt, 0)
    params = {k: v + rng.standard_normal(v.shape) * 0.01 for k, v in params.items()}
    X = rng.standard_normal((6, P.ENC_DIM))
    T = rng.uniform(-1, 1, (6, nt))
    cache = P.forward(params, X, quant=False)
    L, dy = P.nll(cache["y"], T)
    g = P.backward(params, cache, dy, quant=False)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in params.items()}
    x = torch.tensor(X)
    h1 = torch.relu(x @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    y = h2 @ tp["W3"].T + tp["b3"]
    mu, s = y[:, :nt], y[:, nt:]
    dist = torch.distributions.Normal(mu, torch.exp(s))
    Lt = -(dist.log_prob(torch.tensor(T)) + 0.5 * math.log(2 * math.pi)).sum() / 6
    Lt.backward()
    assert np.allclose(cache["y"], y.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(L - Lt.item()) <= 1e-10 * abs(L)
    for k in params:
        assert np.allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-12), k


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(5)
    params = small_params(rng)
    X = rng.standard_normal((4, 7))
    T = rng.uniform(-1, 1, (4, 3))
    cache = P.forward(params, X, quant=False)
    g = P.backward(params, cache, P.nll(cache["y"], T)[1], quant=False)
    h = 1e-6
    for k in params:
        fd = np.zeros_like(params[k])
        for ix in np.ndindex(params[k].shape):
            p1 = {kk: vv.copy() for kk, vv in params.items()}
            p2 = {kk: vv.copy() for kk, vv in params.items()}
            p1[k][ix] += h
            p2[k][ix] -= h
            fd[ix] = (loss_of(p1, X, T) - loss_of(p2, X, T)) / (2 * h)
        assert np.allclose(g[k], fd, rtol=1e-5, atol=1e-7), k


def test_nll_closed_forms():
    T = np.array([[0.3, -0.7]])
    L, dy = P.nll(np.array([[0.3, -0.7, 0.0, 0.0]]), T)
    assert L == 0.0 and np.array_equal(dy, [[0.0, 0.0, 1.0, 1.0]])
    # r = 1, sigma = 2: 0.5 * 1 / 4 + log 2 per parameter; d/dmu = -1/4, d/ds = 1 - 1/4
    L, dy = P.nll(np.array([[0.0, 0.0, math.log(2.0), math.log(2.0)]]), np.array([[1.0, -1.0]]))
    assert abs(L - 2 * (0.125 + math.log(2.0))) < 1e-15
    assert np.allclose(dy, [[-0.25, 0.25, 0.75, 0.75]], atol=1e-15)


def test_quantised_pass_close_to_wide_pass():
    """The bfloat16 operand rounding perturbs outputs by about the bfloat16 unit roundoff (2^-8)
    relative; gradients a little more, since ReLU masks of pre-activations near zero can flip."""
    rng = np.random.default_rng(6)
    params = P.init_params(1410, 1)
    X = rng.standard_normal((16, P.ENC_DIM))
    T = rng.uniform(-1, 1, (16, 1410))
    cw, cq = P.forward(params, X, False), P.forward(params, X, True)
    rel = np.linalg.norm(cq["y"] - cw["y"]) / np.linalg.norm(cw["y"])
    assert 0 < rel < 2.0 ** -6
    gw = P.backward(params, cw, P.nll(cw["y"], T)[1], False)
    gq = P.backward(params, cq, P.nll(cq["y"], T)[1], True)
    for k in gw:
        rel = np.linalg.norm(gq[k] - gw[k]) / np.linalg.norm(gw[k])
        assert rel < 0.1, (k, rel)
    # with every operand already a bfloat16 value and ReLU outputs exact, rounding is the identity
    p2 = {k: P.bf16(v) for k, v in params.items()}
    p2["W2"][:] = 0.0
    p2["W3"] = P.bf16(p2["W3"])
    X2 = P.bf16(X)
    a = P.forward(p2, X2, True)
    b = P.forward(p2, X2, False)
    assert np.array_equal(a["a2"], b["a2"])


def test_adam_against_torch_optim():
    rng = np.random.default_rng(7)
    params = small_params(rng)
    m = {k: np.zeros_like(v) for k, v in params.items()}
    v = {k: np.zeros_like(x) for k, x in params.items()}
    tp = {k: torch.tensor(x, dtype=torch.float64, requires_grad=True) for k, x in params.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        grads = {k: rng.standard_normal(x.shape) for k, x in params.items()}
        P.adam(params, grads, m, v, t, 3e-3)
        opt.zero_grad()
        for k in tp:
            tp[k].grad = torch.tensor(grads[k])
        opt.step()
        for k in params:
            assert np.allclose(params[k], tp[k].detach().numpy(), rtol=1e-13, atol=1e-15), (t, k)


# ------------------------------------------------------------------------------------------------
# Gaussian draws
# ------------------------------------------------------------------------------------------------
def test_normals_distribution():
    from scipy import stats
    z = P.normals(0xDEADBEEF, 3, 0, 40, 1410)
    flat = z.ravel()
    assert abs(flat.mean()) < 0.02 and abs(flat.std() - 1.0) < 0.02
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    # the two normals of one Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z[:, 0::4].ravel(), z[:, 1::4].ravel())[0, 1]) < 0.03
    # samples and parameters are independent streams: no two rows equal
    assert len({tuple(r[:8]) for r in z}) == 40


def test_normals_use_stream_one_words():
    """Parameter 4b+r of sample i is built from block (b, i, 1, inst) only."""
    seed, inst = 0x1234_5678_9ABC, 9
    z = P.normals(seed, inst, 5, 1, 8)[0]
    w = oracle.philox((1, 5, 1, inst), (seed & 0xFFFFFFFF, seed >> 32))
    ua, ub = ((w[2] >> 9) + 0.5) / 2 ** 23, ((w[3] >> 9) + 0.5) / 2 ** 23
    r = math.sqrt(-2 * math.log(ua))
    assert z[6] == pytest.approx(r * math.cos(2 * math.pi * ub), abs=1e-15)
    assert z[7] == pytest.approx(r * math.sin(2 * math.pi * ub), abs=1e-15)
    assert z[6] ** 2 + z[7] ** 2 == pytest.approx(-2 * math.log(ua), rel=1e-13)


def test_sample_moments():
    mu = np.linspace(-2, 2, 1410)
    ls = np.linspace(-3, 0.5, 1410)
    th = P.sample(mu, ls, 77, 0, 0, 200)
    zs = (th - mu) / np.exp(ls)
    assert abs(zs.mean()) < 0.01 and abs(zs.std() - 1.0) < 0.01
