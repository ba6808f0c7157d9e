"""Pins of the CNN oracle (oracle/cnn.py) against library routines and finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import cnn


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-20, 100), [0.0, -0.0, 1e30, -3.0, 65504.0]])
    x = x.astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(x), want)


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(9, 11, 3))
    w = rng.normal(size=(3, 3, 3, 5))
    b = rng.normal(size=5)
    y = cnn.conv3x3(x, w, b)
    for o in range(5):
        ref = b[o] + sum(scipy.signal.correlate(x[:, :, c], w[:, :, c, o], mode="same") for c in range(3))
        assert np.allclose(y[:, :, o], ref, atol=1e-12)


def _loss(x, p, label, mask, pw):
    z3 = cnn.forward(x, p, emulate_bf16=False)[-1]
    return cnn.loss_and_grad_logits(z3, label, mask, pw)[0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    H, W = 6, 7
    x = rng.normal(size=(H, W, 4))
    p = {k: v.astype(np.float64) + rng.normal(0, 0.05, size=v.shape) for k, v in cnn.init_params(3).items()}
    label = (rng.random((H, W)) < 0.3).astype(np.float64)
    mask = (rng.random((H, W)) < 0.8).astype(np.float64)
    pw = 4.0
    cache = cnn.forward(x, p, emulate_bf16=False)
    _, dz3 = cnn.loss_and_grad_logits(cache[-1], label, mask, pw)
    g = cnn.backward(x, p, cache, dz3, emulate_bf16=False)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = _loss(x, p, label, mask, pw)
            flat[idx] = old - eps
            lm = _loss(x, p, label, mask, pw)
            flat[idx] = old
            num = (lp - lm) / (2 * eps)
            assert abs(num - g[k].reshape(-1)[idx]) <= 1e-6 + 1e-5 * abs(num), (k, idx, num, g[k].reshape(-1)[idx])


def test_bce_gradient_closed_form():
    z = np.linspace(-8, 8, 33).reshape(3, 11, 1)
    y = (np.arange(33) % 3 == 0).reshape(3, 11).astype(float)
    m = np.ones((3, 11))
    l0, g = cnn.loss_and_grad_logits(z, y, m, 2.5)
    h = 1e-6
    lp, _ = cnn.loss_and_grad_logits(z + h * np.eye(33)[5].reshape(3, 11, 1), y, m, 2.5)
    assert abs((lp - l0) / h - g.reshape(-1)[5]) < 1e-5
    # the loss at z = 0 is log 2 per pixel times the weights
    l, _ = cnn.loss_and_grad_logits(np.zeros((1, 2, 1)), np.array([[1.0, 0.0]]), np.ones((1, 2)), 3.0)
    assert abs(l - (3.0 + 1.0) * np.log(2.0) / 2) < 1e-12


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    p = {"w": rng.normal(size=(3, 4))}
    t_p = torch.tensor(p["w"], requires_grad=True)
    opt = torch.optim.Adam([t_p], lr=1e-2)
    m, v = {"w": np.zeros((3, 4))}, {"w": np.zeros((3, 4))}
    for t in range(1, 6):
        g = {"w": rng.normal(size=(3, 4))}
        p = cnn.adam_step(p, m, v, g, t, lr=1e-2)
        t_p.grad = torch.tensor(g["w"])
        opt.step()
    assert np.allclose(p["w"], t_p.detach().numpy(), rtol=1e-10, atol=1e-12)


def test_features_definitions():
    grey = np.zeros((5, 6), np.uint8)
    grey[:, 3:] = 255                       # a vertical dark-to-light step
    disp = np.full((3, 6), 10.0)
    valid = np.ones((3, 6), bool)
    valid[0, 0] = False
    f = np.array([10.0, 13.0, 100.0])
    feat = cnn.features(grey, disp, valid, f)
    assert feat.shape == (3, 6, 4)
    assert np.allclose(feat[1, :, 0], grey[2] / 255.0)
    assert np.isclose(feat[1, 3, 1], 4 * 255 / 1020.0) and np.isclose(feat[1, 3, 2], 0.0)   # G_x = 1020, G_y = 0
    assert feat[0, 0, 3] == -4.0 and feat[0, 1, 3] == 0.0 and feat[1, 1, 3] == -1.0 and feat[2, 1, 3] == -4.0
