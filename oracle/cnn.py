"""fp64 numpy oracle of the learned start proposer (not part of the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).  It restates the
network, its loss and its gradients with plain array operations, so the GPU's
forward and backward kernels can be compared against it, and it is itself
pinned by finite differences (round=False).

Network (NHWC; input at a quarter of the frame resolution):
  x0 = [ (cur4 - ref4) / 32, (cur4 - 128) / 64 ]      cur4, ref4: 4x4 box means
  L1 conv 3x3 stride 1, 2 -> 16, ReLU
  L2 conv 3x3 stride 2, 16 -> 32, ReLU
  L3 conv 3x3 stride 2, 32 -> 32, ReLU      (one pixel per 16x16 block)
  L4 conv 3x3 stride 1, 32 -> 3             head (u, v, o)
All convolutions pad by 1.  Start vector = 8 (u, v) rounded; orientation
vertical when o > 0.

Loss per block, averaged over blocks (target t = FS motion vector / 8):
  huber(u - tx) + huber(v - ty) + 0.25 * bce(o, |ty| > |tx|)
  huber(d) = d^2 / 2 for |d| <= 1, |d| - 1/2 otherwise; bce(o, y) = softplus(o) - y o.

Storage precision of the GPU path, mirrored here when round=True: the input,
the weights used by the convolutions, every post-ReLU activation and every
activation gradient that feeds a convolution are rounded to bfloat16 (nearest
even); products and sums are exact here (fp64) and fp32 on the GPU.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(2, 16, 1, True), (16, 32, 2, True), (32, 32, 2, True), (32, 3, 1, False)]  # cin, cout, stride, relu
BCE_WEIGHT = 0.25
MV_SCALE = 8.0


def bf16(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def param_shapes():
    out = []
    for cin, cout, _, _ in LAYERS:
        out.append(((3, 3, cin, cout), (cout,)))
    return out


def num_params():
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unflatten(flat):
    """Flat fp32 parameter vector (the GPU's order: per layer W[ky][kx][ci][co] then b[co])."""
    flat = np.asarray(flat, dtype=np.float64)
    ps, i = [], 0
    for ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        ps.append((flat[i:i + nw].reshape(ws), flat[i + nw:i + nw + nb].reshape(bs)))
        i += nw + nb
    assert i == len(flat)
    return ps


def flatten(ps):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ps])


def downdiff(cur, ref, round_=True):
    """x0 [H/4, W/4, 2] from uint8 frames [H, W]."""
    H, W = cur.shape
    c = cur.astype(np.float64).reshape(H // 4, 4, W // 4, 4).mean(axis=(1, 3))
    r = ref.astype(np.float64).reshape(H // 4, 4, W // 4, 4).mean(axis=(1, 3))
    x = np.stack([(c - r) / 32.0, (c - 128.0) / 64.0], axis=-1)
    return bf16(x) if round_ else x


def _pad(x):
    return np.pad(x, ((1, 1), (1, 1), (0, 0)))


def out_size(n, stride):
    return (n - 1) // stride + 1


def conv(x, w, b, stride):
    """out[y, x, co] = b[co] + sum_{ky, kx, ci} in[y*s + ky - 1, x*s + kx - 1, ci] w[ky, kx, ci, co]."""
    H, W, _ = x.shape
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = _pad(x)
    out = np.zeros((Ho, Wo, w.shape[3])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            out += patch @ w[ky, kx]
    return out


def conv_grads(x, w, g, stride):
    """Gradients of conv with respect to its input, weights and bias, given the
    output gradient g [Ho, Wo, Cout] (the transpose of `conv`, written out)."""
    H, W, _ = x.shape
    Ho, Wo = g.shape[:2]
    xp = _pad(x)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(ky, ky + stride * (Ho - 1) + 1, stride), slice(kx, kx + stride * (Wo - 1) + 1, stride))
            patch = xp[sl[0], sl[1], :]
            dw[ky, kx] = np.einsum("hwi,hwo->io", patch, g)
            dxp[sl[0], sl[1], :] += g @ w[ky, kx].T
    db = g.sum(axis=(0, 1))
    return dxp[1:-1, 1:-1, :], dw, db


def forward(x0, ps, round_=True):
    """Returns (head [H/16, W/16, 3], activations [x0, x1, x2, x3])."""
    acts = [x0]
    x = x0
    for li, ((w, b), (_, _, s, relu)) in enumerate(zip(ps, LAYERS)):
        wq = bf16(w) if round_ else w
        z = conv(x, wq, b, s)
        if relu:
            z = np.maximum(z, 0.0)
            z = bf16(z) if round_ else z
            acts.append(z)
        x = z
    return x, acts


def loss_and_dhead(head, target_mv):
    """Mean loss over blocks and its gradient with respect to the head."""
    t = np.asarray(target_mv, dtype=np.float64) / MV_SCALE
    n = int(np.prod(head.shape[:-1]))  # every block of every pair
    d = head[..., :2] - t
    a = np.abs(d)
    hub = np.where(a <= 1.0, 0.5 * d * d, a - 0.5)
    dhub = np.clip(d, -1.0, 1.0)
    lab = (np.abs(t[..., 1]) > np.abs(t[..., 0])).astype(np.float64)
    o = head[..., 2]
    bce = np.logaddexp(0.0, o) - lab * o
    sig = 1.0 / (1.0 + np.exp(-o))
    loss = (hub.sum() + BCE_WEIGHT * bce.sum()) / n
    dh = np.zeros_like(head)
    dh[..., :2] = dhub / n
    dh[..., 2] = BCE_WEIGHT * (sig - lab) / n
    return loss, dh


def backward(acts, ps, dhead, round_=True):
    """Parameter gradients [(dW, db)] for the head gradient dhead."""
    grads = [None] * len(LAYERS)
    g = bf16(dhead) if round_ else dhead
    for li in range(len(LAYERS) - 1, -1, -1):
        w, _ = ps[li]
        wq = bf16(w) if round_ else w
        _, _, s, _ = LAYERS[li]
        x = acts[li]
        dx, dw, db = conv_grads(x, wq, g, s)
        grads[li] = (dw, db)
        if li > 0:
            # ReLU of the previous layer: its stored output decides the mask.
            dx = dx * (acts[li] > 0)
            g = bf16(dx) if round_ else dx
    return grads


def decode(head, R):
    """Start vectors and orientations from the head (the GPU's rule)."""
    s = np.rint(head[..., :2] * MV_SCALE)
    s = np.clip(s, -R, R).astype(np.int16)
    o = (head[..., 2] > 0).astype(np.uint8)
    return s, o


def init_params(seed):
    """He-normal weights, zero biases (the test's own initialisation)."""
    rng = np.random.default_rng(seed)
    ps = []
    for cin, cout, _, _ in LAYERS:
        std = np.sqrt(2.0 / (9 * cin))
        ps.append((rng.normal(0.0, std, (3, 3, cin, cout)), np.zeros(cout)))
    return ps
