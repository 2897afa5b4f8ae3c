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


def _representable_params(rng, nin, nout):
    """Integer weights and biases, sparse enough that every value the network
    rounds (weights, hidden activations, dZ2, dZ1) is an integer of magnitude
    below 256, hence exactly a bfloat16: W1 in {-1, 0, 1}; W2 and W3 with at
    most three nonzero entries (+-1) in every row and column (sums of
    permutation matrices)."""
    P = np.zeros(R.NPARAMS)
    W1 = np.zeros((R.IN, R.H)); W1[:nin] = rng.integers(-1, 2, (nin, R.H))
    W2 = np.zeros((R.H, R.H))
    for s in (1, 1, -1):
        W2[np.arange(R.H), rng.permutation(R.H)] += s
    W3 = np.zeros((R.H, R.OUT))
    for o in range(nout):
        W3[rng.choice(R.H, 3, replace=False), o] = rng.choice([-1.0, 1.0], 3)
    P[R.oW1:R.oB1] = W1.ravel()
    P[R.oB1:R.oW2] = rng.integers(-2, 3, R.H)
    P[R.oW2:R.oB2] = W2.ravel()
    P[R.oB2:R.oW3] = rng.integers(-2, 3, R.H)
    P[R.oW3:R.oB3] = W3.ravel()
    P[R.oB3:R.oB3 + nout] = rng.integers(-2, 3, nout)
    return P


def test_rounded_equals_exact_when_every_value_is_a_bfloat16():
    """With integer weights, inputs and output gradients chosen so that every
    value the rounded network rounds is exactly representable, the rounded
    forward and backward equal the exact (finite-difference-pinned) network
    bit for bit.  A dropped or extra term, a wrong layer, a transposed
    operand or a scale error in the rounded variant breaks the equality."""
    rng = np.random.default_rng(3)
    for nin, nout in ((22, 2), (32, 2), (7, 1)):
        P = _representable_params(rng, nin, nout)
        X = np.zeros((48, R.IN))
        X[:, :nin] = rng.integers(-3, 4, (48, nin))
        dY = rng.integers(-3, 4, (48, nout)).astype(np.float64)
        ye, h1, h2 = R.forward(P, X, nout, rounded=False)
        assert np.abs(h1).max() < 256 and np.abs(h2).max() < 256
        assert np.all(R.bf16(h1) == h1) and np.all(R.bf16(h2) == h2)
        yr, _, _ = R.forward(P, X, nout, rounded=True)
        assert np.array_equal(yr, ye)
        ge, dXe = R.backward(P, X, dY, nout, rounded=False)
        gr, dXr = R.backward(P, X, dY, nout, rounded=True)
        assert np.array_equal(gr, ge) and np.array_equal(dXr, dXe)
        assert np.any(h2 > 0) and np.any(ge != 0)
