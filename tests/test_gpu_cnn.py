"""GPU CNN (BF16 weights/activations, FP32 accumulation) against the FP64 oracle fed the same
BF16-rounded weights, inputs and stored activations."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import cnn as ocnn  # noqa: E402


def uwb():
    import paper_1709_02549_amd as m
    return m


def _params(seed):
    p = ocnn.Params.init(seed)
    rng = np.random.default_rng(seed + 100)
    p.b = [rng.normal(0, 0.05, ocnn.CH) for _ in range(4)]
    p.bl = 0.1
    # the GPU computes with BF16 copies of the FP32 masters: give the oracle the same numbers
    flat32 = p.flat().astype(np.float32)
    return flat32, ocnn.Params.from_flat(ocnn.bf16_round(flat32))


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, 32, 32)) ** 4          # peaky, like normalised energy images
    xb = ocnn.bf16_round(x)
    return torch.tensor(xb, dtype=torch.float32, device="cuda").to(torch.bfloat16), xb, rng.integers(0, 4, n)


@pytest.mark.parametrize("n", [1, 37, 256])
def test_forward_matches_oracle(n):
    flat, p = _params(1)
    net = uwb().CNN(256, flat)
    xg, xb, _ = _inputs(n, 2)
    pg = net.forward(xg).cpu().numpy()
    logits, _ = ocnn.forward(p, xb, act_round=ocnn.bf16_round)
    po = ocnn.softmax(logits)
    np.testing.assert_allclose(pg.sum(axis=1), 1.0, rtol=1e-6)
    assert np.max(np.abs(pg - po)) <= 1e-2
    assert np.mean(np.abs(pg - po)) <= 2e-3
    net.close()


def _abs_gradient(p, xb, lab):
    """Every gradient element's sum of the magnitudes of the terms it adds up: the oracle's backward pass run on
    |weights|, |activations| and |upstream gradients|, with every ReLU whose input lies within 2^-6 of its
    layer's largest pre-activation of zero counted as open (its mask can differ between the two sides).  A
    stored BF16 activation differs between the GPU and the FP64 oracle by at most one BF16 ulp (2^-7 of it)
    when the two sides' sums round to neighbouring BF16 values; each term of a gradient element inherits such
    a relative difference from every rounded activation on its path, so |g_gpu - g_oracle| is bounded by a
    few 2^-7 times this sum."""
    logits, (a, pre, feat) = ocnn.forward(p, xb, act_round=ocnn.bf16_round)
    n = logits.shape[0]
    prob = ocnn.softmax(logits)
    dlog = prob.copy()
    dlog[np.arange(n), lab] -= 1.0
    dlog = np.abs(dlog) / n
    dwl = np.einsum("nc,nck->k", dlog, np.abs(feat))
    dbl = float(dlog.sum())
    dfeat = dlog[:, :, None] * np.abs(p.wl)[None, None, :]
    da = np.zeros_like(a[-1])
    for c in range(4):
        bx, by = c & 1, c >> 1
        da[:, :, 2 * by:2 * by + 2, 2 * bx:2 * bx + 2] += dfeat[:, c, :, None, None] / 4.0
    dw, db = [None] * 4, [None] * 4
    for i in reversed(range(4)):
        z = pre[i]
        open_ = z > -2.0 ** -6 * np.abs(z).max()
        dz = da * open_
        dx, dw[i], db[i] = ocnn.conv_backward(np.abs(a[i]), np.abs(p.w[i]), ocnn.STRIDES[i], dz)
        da = dx
    return ocnn.Params(dw, db, dwl, dbl).flat()


def test_gradients_match_oracle():
    """Element by element: |g_gpu - g_oracle| <= 4 * 2^-7 * (the element's sum of term magnitudes); per tensor:
    L2 relative error <= 1e-2."""
    flat, p = _params(3)
    net = uwb().CNN(64, flat)
    xg, xb, lab = _inputs(64, 4)
    g, loss = net.gradients(xg, torch.tensor(lab, dtype=torch.int32, device="cuda"))
    g = g.cpu().numpy().astype(np.float64)
    lo, go, _ = ocnn.loss_and_grad(p, xb, lab, act_round=ocnn.bf16_round)
    assert float(loss.cpu()) == pytest.approx(lo, rel=2e-3)
    ga = _abs_gradient(p, xb, lab)
    assert np.all(ga >= np.abs(go) * (1 - 1e-12))          # the magnitude sum bounds the gradient itself
    ratio = np.abs(g - go) / np.maximum(ga, 1e-300)
    print(f"gradient error / magnitude sum: max {ratio.max():.3e}, 99.9th percentile "
          f"{np.percentile(ratio, 99.9):.3e} (bound {4 * 2.0 ** -7:.3e})")
    assert ratio.max() <= 4 * 2.0 ** -7
    bounds = [0, 288, 288 + 9216, 288 + 2 * 9216, 288 + 3 * 9216, 288 + 3 * 9216 + 128, 28097]
    rels = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        rels.append(np.linalg.norm(g[a:b] - go[a:b]) / max(np.linalg.norm(go[a:b]), 1e-30))
    print("per-tensor L2 relative errors:", " ".join(f"{r:.2e}" for r in rels))
    assert max(rels) <= 1e-2, rels
    net.close()


def _task(n, seed):
    """Label = quadrant of the brightest pixel of a noisy image with one bright blob."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 0.3, (n, 32, 32))
    yy, xx = np.mgrid[0:32, 0:32]
    lab = rng.integers(0, 4, n)
    for i in range(n):
        cx = 4 + 16 * (lab[i] & 1) + rng.integers(0, 8)
        cy = 4 + 16 * (lab[i] >> 1) + rng.integers(0, 8)
        x[i] += np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / 8.0)
    x /= x.max(axis=(1, 2), keepdims=True)
    return (torch.tensor(x, dtype=torch.float32, device="cuda").to(torch.bfloat16),
            torch.tensor(lab, dtype=torch.int32, device="cuda"))


def test_training_learns_and_is_deterministic_and_resumable():
    flat, _ = _params(7)
    xs, ls = _task(512, 8)
    a = uwb().CNN(128, flat)
    losses = []
    for step in range(60):
        k = (step * 128) % 512
        losses.append(float(a.train_step(xs[k:k + 128], ls[k:k + 128], 3e-3).cpu()))
        if step == 29:
            ckpt = a.get_state()
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:5])
    probs = a.forward(xs[:128]).cpu().numpy()
    acc = np.mean(np.argmax(probs, 1) == ls[:128].cpu().numpy())
    assert acc >= 0.8
    # same run again: bitwise identical losses
    b = uwb().CNN(128, flat)
    again = [float(b.train_step(xs[(s * 128) % 512:(s * 128) % 512 + 128], ls[(s * 128) % 512:(s * 128) % 512 + 128],
                                3e-3).cpu()) for s in range(60)]
    assert again == losses
    # resume from step 30 in a fresh handle: bitwise identical continuation
    c = uwb().CNN(128, flat)
    c.set_state(ckpt)
    cont = [float(c.train_step(xs[(s * 128) % 512:(s * 128) % 512 + 128], ls[(s * 128) % 512:(s * 128) % 512 + 128],
                               3e-3).cpu()) for s in range(30, 60)]
    assert cont == losses[30:]
    assert np.array_equal(c.get_state()["theta"], a.get_state()["theta"])
    for h in (a, b, c):
        h.close()


def test_first_adam_step_moves_each_weight_against_its_gradient():
    """Step 1 of Adam moves every weight by lr * g / (|g| + eps): the sign must oppose the oracle's gradient."""
    flat, p = _params(9)
    net = uwb().CNN(32, flat)
    xg, xb, lab = _inputs(32, 10)
    net.train_step(xg, torch.tensor(lab, dtype=torch.int32, device="cuda"), 1e-3)
    th = net.get_state()["theta"].astype(np.float64)
    _, go, _ = ocnn.loss_and_grad(p, xb, lab, act_round=ocnn.bf16_round)
    d = th - flat.astype(np.float64)
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert np.mean(np.sign(d[big]) == -np.sign(go[big])) > 0.99
    assert np.allclose(np.abs(d[big]), 1e-3, rtol=1e-2)
    net.close()


def test_masked_labels_drop_out_of_loss_and_gradient():
    """A label outside 0..3 removes its sample; the mean still divides by the whole batch."""
    flat, p = _params(5)
    net = uwb().CNN(16, flat)
    xg, xb, lab = _inputs(16, 6)
    lab = lab.copy()
    lab[[2, 7, 11]] = [-1, 4, -7]
    keep = np.array([i not in (2, 7, 11) for i in range(16)])
    g, loss = net.gradients(xg, torch.tensor(lab, dtype=torch.int32, device="cuda"))
    lo, go, _ = ocnn.loss_and_grad(p, xb[keep], lab[keep], act_round=ocnn.bf16_round)
    scale = keep.sum() / 16.0
    assert float(loss.cpu()) == pytest.approx(lo * scale, rel=2e-3)
    g = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - go * scale) / np.linalg.norm(go * scale)
    assert rel <= 2e-2
    net.close()
