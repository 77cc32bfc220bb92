"""Pins of the FP64 CNN oracle (the learned segment proposer): finite differences,
an independent torch-autograd (CPU, FP64) formulation, BF16 rounding, Adam."""
import numpy as np
import pytest

from oracle import cnn

torch = pytest.importorskip("torch")


def _data(n=4, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, 32, 32))
    lab = rng.integers(0, 4, n)
    return x, lab


def test_sizes():
    assert cnn.N_PARAMS == 28097
    assert cnn.macs_per_sample() == 3391488


def test_finite_differences():
    p = cnn.Params.init(3)
    x, lab = _data(3, 1)
    _, g, _ = cnn.loss_and_grad(p, x, lab)
    theta = p.flat()
    rng = np.random.default_rng(7)
    # coordinates from every tensor: conv weights, biases, readout
    idx = list(rng.choice(288, 3)) + list(288 + rng.choice(9216 * 3, 6)) + list(range(28064, 28097, 5))
    for k in idx:
        h = 1e-6 * max(1.0, abs(theta[k]))
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp = cnn.loss_and_grad(cnn.Params.from_flat(tp), x, lab)[0]
        lm = cnn.loss_and_grad(cnn.Params.from_flat(tm), x, lab)[0]
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9), k


def _torch_net(p, x, lab):
    import torch.nn.functional as F
    t = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)  # noqa: E731
    w = [t(a) for a in p.w]
    b = [t(a) for a in p.b]
    wl, bl = t(p.wl), t(np.array([p.bl]))
    h = torch.tensor(x, dtype=torch.float64)[:, None]
    for i in range(4):
        h = F.relu(F.conv2d(h, w[i], b[i], stride=cnn.STRIDES[i], padding=1))
    q = F.avg_pool2d(h, 2)                               # [N, C, 2, 2]: (by, bx) quadrants
    feat = q.permute(0, 2, 3, 1).reshape(h.shape[0], 4, cnn.CH)   # child = 2 by + bx
    logits = feat @ wl + bl
    loss = F.cross_entropy(logits, torch.tensor(lab))
    loss.backward()
    g = np.concatenate([a.grad.numpy().ravel() for a in w] + [a.grad.numpy().ravel() for a in b]
                       + [wl.grad.numpy(), bl.grad.numpy()])
    return float(loss), g, logits.detach().numpy()


def test_matches_torch_autograd():
    p = cnn.Params.init(5)
    p.b = [np.random.default_rng(i).normal(0, 0.1, cnn.CH) for i in range(4)]
    x, lab = _data(5, 2)
    l, g, prob = cnn.loss_and_grad(p, x, lab)
    tl, tg, tlog = _torch_net(p, x, lab)
    assert l == pytest.approx(tl, rel=1e-12)
    np.testing.assert_allclose(g, tg, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(prob, cnn.softmax(tlog), rtol=1e-12)
    np.testing.assert_allclose(prob.sum(axis=1), 1.0, rtol=1e-14)


def test_bf16_round_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000) * 10 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16_round(x), want)


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tt = torch.tensor(theta, requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-3)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        theta, m, v = cnn.adam_step(theta, m, v, g, step, 1e-3)
        tt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, tt.detach().numpy(), rtol=1e-12)


def test_quadrant_order():
    """Child c = bx + 2 by reads rows 2by..2by+1 and columns 2bx..2bx+1 of the 4x4 map."""
    a = np.zeros((1, 1, 4, 4))
    a[0, 0, 0:2, 2:4] = 1.0           # upper-x half, lower-y half -> child 1
    f = cnn.quadrant_pool(a)
    assert f[0, :, 0].tolist() == [0.0, 1.0, 0.0, 0.0]
