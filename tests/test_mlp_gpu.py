"""The policy network's forward, backward and Adam kernels against the CPU
reference (same bfloat16 rounding points), and a training smoke test.

Floating point: the device sums in fp32 in matrix-core order, the reference in
float64; the products' inputs are identical bf16 values, so the results agree
to a few fp32 ulps except where a pre-rounding difference flips one bf16
rounding (one bf16 ulp, 2^-8 relative, of one activation).  The tolerances
below (1e-2 relative in norm, 3e-2 of the largest magnitude elementwise) cover
a few such flips and fail on any layout, transposition or indexing error,
which moves whole rows or columns.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fsp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_4973_amd import fsp as F
    F.lib()
    return F


def rand_x(rng, n, nin):
    X = np.zeros((n, R.IN), dtype=np.float32)
    X[:, :nin] = rng.normal(0, 1, (n, nin))
    xt = torch.from_numpy(X).to(torch.bfloat16)
    return xt.cuda(), xt.float().numpy().astype(np.float64)


def close(got, want, rel=1e-2, elem=3e-2):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    scale = max(np.abs(want).max(), 1e-12)
    assert np.abs(got - want).max() <= elem * scale, np.abs(got - want).max() / scale
    assert np.linalg.norm(got - want) <= rel * max(np.linalg.norm(want), 1e-12)


@pytest.mark.parametrize("n,nin,nout", [(1, 22, 2), (77, 22, 2), (1000, 22, 2), (4099, 32, 16),
                                        (513, 5, 1)])
def test_forward_matches_reference(fsp, n, nin, nout):
    rng = np.random.default_rng(n + nin)
    m = fsp.Model(nin, nout, seed=7)
    P = m.params().astype(np.float64)
    x, X = rand_x(rng, n, nin)
    y = m.forward(x).cpu().numpy()
    want, _, _ = R.forward(P, X, nout)
    close(y, want)


@pytest.mark.parametrize("n,nin,nout", [(64, 22, 2), (1000, 22, 2), (3001, 32, 16)])
def test_backward_matches_reference(fsp, n, nin, nout):
    rng = np.random.default_rng(10 * n + nout)
    m = fsp.Model(nin, nout, seed=3)
    P = m.params().astype(np.float64)
    x, X = rand_x(rng, n, nin)
    dy = rng.normal(0, 1, (n, nout)).astype(np.float32)
    dx = m.backward(x, torch.from_numpy(dy).cuda(), want_dx=True)
    torch.cuda.synchronize()
    g = m.grads()
    gw, dxw = R.backward(P, X, dy.astype(np.float64), nout)
    for a, b in ((R.oW1, R.oB1), (R.oB1, R.oW2), (R.oW2, R.oB2), (R.oB2, R.oW3),
                 (R.oW3, R.oB3), (R.oB3, R.NPARAMS)):
        close(g[a:b], gw[a:b])
    close(dx.cpu().numpy(), dxw)


def test_backward_accumulates(fsp):
    rng = np.random.default_rng(5)
    m = fsp.Model(22, 2, seed=1)
    x, _ = rand_x(rng, 300, 22)
    dy = torch.from_numpy(rng.normal(0, 1, (300, 2)).astype(np.float32)).cuda()
    m.backward(x, dy)
    g1 = m.grads()
    m.backward(x, dy, accumulate=True)
    g2 = m.grads()
    assert np.allclose(g2, 2 * g1, rtol=1e-6, atol=1e-7)


def test_adam_step_matches_cpu_update(fsp):
    rng = np.random.default_rng(6)
    m = fsp.Model(22, 2, seed=2)
    P0 = m.params().astype(np.float64)
    x, _ = rand_x(rng, 500, 22)
    dy = torch.from_numpy(rng.normal(0, 1, (500, 2)).astype(np.float32)).cuda()
    m.backward(x, dy)
    g = m.grads().astype(np.float64)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    m.adam_step(lr, b1, b2, eps)
    torch.cuda.synchronize()
    P1 = m.params().astype(np.float64)
    mom, vel = (1 - b1) * g, (1 - b2) * g * g
    want = P0 - lr * (mom / (1 - b1)) / (np.sqrt(vel / (1 - b2)) + eps)
    live = P0 != 0  # padded rows/columns are zero and must stay zero
    live[R.oB1:R.oW2] = live[R.oB2:R.oW3] = True
    live[R.oB3:R.oB3 + 2] = True
    assert np.allclose(P1[live], want[live], rtol=1e-5, atol=1e-7)
    assert np.all(P1[~live] == 0)


def test_training_reduces_the_loss(fsp):
    rng = np.random.default_rng(7)
    n = 4096
    x, X = rand_x(rng, n, 22)
    t = np.zeros((n, 2), np.float32)
    t[:, 0] = (X[:, :4] ** 2).sum(1) / 4 - 0.5 * X[:, 5]
    t[:, 1] = (X[:, 0] + X[:, 1] > 0).astype(np.float32)
    tt = torch.from_numpy(t).cuda()
    m = fsp.Model(22, 2, seed=11)
    losses = [m.train_step(x, tt, 3e-3) for _ in range(300)]
    assert losses[-1] < 0.25 * losses[0], (losses[0], losses[-1])
