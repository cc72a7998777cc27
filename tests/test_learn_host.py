"""Host logic of the learned proposal's evaluation: the canonical form of a network's parameters
that the elite-Gaussian bound fits its Gaussians in."""
import numpy as np

from paper_1904_06680_amd.learn import canonical


def _forward(th, x):
    """Plain numpy forward pass of the 8-32-32-2 tanh MLP in the flat layout (W_l row-major,
    then b_l), written from the layout's definition."""
    w1, b1 = th[:256].reshape(32, 8), th[256:288]
    w2, b2 = th[288:1312].reshape(32, 32), th[1312:1344]
    wo, bo = th[1344:1408].reshape(2, 32), th[1408:1410]
    return np.tanh(wo @ np.tanh(w2 @ np.tanh(w1 @ x + b1) + b2) + bo)


def _scramble(th, rng):
    """The same function with its hidden units permuted and a random subset sign-flipped."""
    th = th.copy()
    w1, b1 = th[:256].reshape(32, 8), th[256:288]
    w2, b2 = th[288:1312].reshape(32, 32), th[1312:1344]
    wo = th[1344:1408].reshape(2, 32)
    p, s = rng.permutation(32), rng.choice([-1.0, 1.0], 32)
    w1n, b1n = (w1 * s[:, None])[p], (b1 * s)[p]
    w2n = (w2 * s[None, :])[:, p]
    q, r = rng.permutation(32), rng.choice([-1.0, 1.0], 32)
    w2n, b2n = (w2n * r[:, None])[q], (b2 * r)[q]
    won = (wo * r[None, :])[:, q]
    return np.concatenate([w1n.ravel(), b1n, w2n.ravel(), b2n, won.ravel(), th[1408:]])


def test_canonical_form_keeps_the_function_and_removes_the_symmetries():
    rng = np.random.default_rng(0)
    th = rng.uniform(-1, 1, (6, 1410))
    c = canonical(th)
    for i in range(len(th)):
        for _ in range(3):
            x = rng.normal(size=8)
            assert np.allclose(_forward(th[i], x), _forward(c[i], x), atol=1e-12)
        twin = _scramble(th[i], rng)
        assert not np.array_equal(twin, th[i])
        assert np.array_equal(canonical(twin[None])[0], c[i])        # same canonical form
    assert np.array_equal(canonical(c), c)                          # idempotent
    assert (c[:, 256:288] >= 0).all() and (np.diff(c[:, 256:288], axis=1) >= 0).all()
    assert (c[:, 1312:1344] >= 0).all() and (np.diff(c[:, 1312:1344], axis=1) >= 0).all()
