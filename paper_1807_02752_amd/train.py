"""Training of the candidate-pruning network on the GPU by the library's own kernels.

Labels come from the plain method: ld_detect with lane curves, then ld_cnn_labels marks the
band pixels near the detected curves.  A step is ld_vdisp on the minibatch (road profile and
bands) and ld_cnn_train_step (forward, loss, backward, fixed-order gradient reduction, Adam).
The host only orders minibatches and passes pointers; the initial weights are drawn here
with numpy and handed to the library.
"""
from __future__ import annotations

import numpy as np

from . import ld

N_PARAMS = ld.LD_CNN_PARAMS
_SHAPES = [((3, 3, 4, 16), 36), ((16,), 0), ((3, 3, 16, 16), 144), ((16,), 0), ((3, 3, 16, 1), 144), ((1,), 0)]


def init_params(seed: int = 0, out_bias: float = -2.0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero hidden biases, output bias out_bias
    (starts the marking probability low, as markings are a few percent of the pixels)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in _SHAPES:
        if fan_in:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), size=shape).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    parts[-1][:] = out_bias
    v = np.concatenate(parts).astype(np.float32)
    assert v.size == N_PARAMS
    return v


def make_labels(net: ld.Cnn, greys, disps, d_max: int, fmt: int, batch: int, radius=2.0, radius_per_disp=0.139):
    """Device labels (N x n_bands x 16 x W) from the plain detections of every frame."""
    import torch
    N, H, W = greys.shape
    nb = net.config.n_bands
    det = ld.Detector(W, H, batch, fmt, d_max)
    lanes = det.lanes_buffer()
    curves = torch.empty((batch, ld.LD_MAX_LANES, H), dtype=torch.float32, device="cuda")
    labels = torch.empty((N, nb, 16, W), dtype=torch.uint8, device="cuda")
    for s in range(0, N, batch):
        n = min(batch, N - s)
        det.set_active(n)
        det.detect(greys[s:s + n], disps[s:s + n], lanes, curves_out=curves)
        net.labels(det, lanes, curves, labels[s:s + n], radius, radius_per_disp)
    det.sync()
    det.close()
    return labels


def train(greys, disps, d_max: int, *, steps: int, batch: int = 16, lr: float = 3e-3, pos_weight: float = 4.0,
          seed: int = 0, n_bands: int = 1, fmt: int = ld.LD_DISP_F32, params=None, **cnn_config):
    """Train on device-resident frames greys/disps (torch uint8 / disparity tensors [N, H, W]).
    Minibatches are consecutive runs of `batch` frames, visited in a seeded random order each
    epoch.  Returns (network, per-step losses as a numpy array)."""
    import torch
    N, H, W = greys.shape
    assert N >= batch
    net = ld.Cnn(init_params(seed) if params is None else params, n_bands=n_bands, max_batch=batch, max_width=W,
                 **cnn_config)
    labels = make_labels(net, greys, disps, d_max, fmt, batch)
    det = ld.Detector(W, H, batch, fmt, d_max)
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda")
    inv_norm = 1.0 / float(batch * n_bands * 16 * W)
    rng = np.random.default_rng(seed + 1)
    starts = np.arange(0, N - batch + 1, batch)
    order = []
    for step in range(steps):
        if not order:
            order = list(rng.permutation(starts))
        s = int(order.pop())
        g, d = greys[s:s + batch], disps[s:s + batch]
        det.vdisp(d)
        net.train_step(det, g, d, labels[s:s + batch], pos_weight, inv_norm, lr, losses[step:step + 1])
    det.sync()
    det.close()
    return net, losses.cpu().numpy()
