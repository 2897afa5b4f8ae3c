"""Pins of the CPU reference of the policy network: bfloat16 rounding against
hand-picked values, the backward formulas against float64 central finite
differences of the exact (unrounded) network."""
import numpy as np

from oracle import mlp_ref as R


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0,
                  1.0 + 2 ** -8 + 2 ** -20], dtype=np.float32)
    want = [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 0.0, 1.0 + 2 ** -7]
    assert list(R.bf16(x)) == want


def _params(rng, nin, nout):
    P = np.zeros(R.NPARAMS)
    W1 = np.zeros((R.IN, R.H)); W1[:nin] = rng.normal(0, 0.3, (nin, R.H))
    W3 = np.zeros((R.H, R.OUT)); W3[:, :nout] = rng.normal(0, 0.1, (R.H, nout))
    P[R.oW1:R.oB1] = W1.ravel()
    P[R.oB1:R.oW2] = rng.normal(0, 0.1, R.H)
    P[R.oW2:R.oB2] = rng.normal(0, 0.1, R.H * R.H)
    P[R.oB2:R.oW3] = rng.normal(0, 0.1, R.H)
    P[R.oW3:R.oB3] = W3.ravel()
    P[R.oB3:R.oB3 + nout] = rng.normal(0, 0.1, nout)
    return P


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    nin, nout, n = 22, 2, 9
    P = _params(rng, nin, nout)
    X = np.zeros((n, R.IN)); X[:, :nin] = rng.normal(0, 1, (n, nin))
    dY = rng.normal(0, 1, (n, nout))
    g, dX = R.backward(P, X, dY, nout, rounded=False)

    def L(P_, X_):
        y, _, _ = R.forward(P_, X_, nout, rounded=False)
        return float((y * dY).sum())

    eps = 1e-6
    idx = np.concatenate([rng.integers(R.oW1, R.oW1 + nin * R.H, 12),
                          rng.integers(R.oB1, R.oW2, 6), rng.integers(R.oW2, R.oB2, 12),
                          rng.integers(R.oB2, R.oW3, 6),
                          [R.oW3 + c * R.OUT + o for c in (3, 77) for o in range(nout)],
                          [R.oB3, R.oB3 + 1]])
    for j in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[j] += eps
        Pm[j] -= eps
        fd = (L(Pp, X) - L(Pm, X)) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])
    for r in range(3):
        for k in range(0, nin, 5):
            Xp, Xm = X.copy(), X.copy()
            Xp[r, k] += eps
            Xm[r, k] -= eps
            fd = (L(P, Xp) - L(P, Xm)) / (2 * eps)
            assert abs(fd - dX[r, k]) <= 1e-6 * max(1.0, abs(fd))


def test_relu_blocks_gradient_and_padding_stays_zero():
    rng = np.random.default_rng(1)
    P = _params(rng, 5, 1)
    P[R.oB1:R.oW2] = -100.0  # every first-layer unit off
    X = np.zeros((4, R.IN)); X[:, :5] = rng.normal(0, 1, (4, 5))
    g, dX = R.backward(P, X, np.ones((4, 1)), 1, rounded=False)
    assert np.all(g[R.oW1:R.oB2] == 0) and np.all(dX == 0)  # W1, b1, W2
    assert np.all(g[R.oW1 + 5 * R.H:R.oB1] == 0)
