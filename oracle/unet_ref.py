"""FP64 CPU reference of the learned coarse stepper's network -- TEST
INFRASTRUCTURE ONLY (see oracle/__init__.py for who may import it).

The same 4-level 3x3-convolution U-Net the GPU kernels run, written with
plain PyTorch CPU operations in float64: conv2d (zero padding 1), 2x2 average
pooling, nearest 2x upsampling, channel concatenation [upsampled, skip],
ReLU, and the front-weighted squared-error loss on the head's first two
channels.  Gradients come from autograd.  It shares no code with the GPU path.

Parameters: dict name -> (W, b) with W[tap][cout][cin], tap = 3*(dy+1) +
(dx+1), matching the kernels' layout.  Tensors are NHWC numpy arrays.
"""
from __future__ import annotations

import numpy as np
import torch

LAYERS = [("e0a", 32, 32, True), ("e0b", 32, 32, True),
          ("e1a", 32, 64, True), ("e1b", 64, 64, True),
          ("e2a", 64, 128, True), ("e2b", 128, 128, True),
          ("b3a", 128, 128, True), ("b3b", 128, 128, True),
          ("d2a", 256, 128, True), ("d2b", 128, 128, True),
          ("d1a", 192, 64, True), ("d1b", 64, 64, True),
          ("d0a", 96, 32, True), ("d0b", 32, 32, True),
          ("head", 32, 32, False)]


def _w(W):
    """[9][cout][cin] -> conv2d weight [cout][cin][3][3]."""
    W = torch.as_tensor(np.asarray(W), dtype=torch.float64)
    return W.reshape(3, 3, W.shape[1], W.shape[2]).permute(2, 3, 0, 1).contiguous()


def conv(x, W, b, relu):
    """x: [N, C, H, W] float64 tensor."""
    y = torch.nn.functional.conv2d(x, W, b, padding=1)
    return torch.relu(y) if relu else y


def forward(params, x_nhwc, requires_grad=False):
    """Returns (head [N, H, W, 32] tensor, dict of leaf parameter tensors)."""
    leaves = {}
    for name, cin, cout, _ in LAYERS:
        W, b = params[name]
        w = _w(W).requires_grad_(requires_grad)
        bb = torch.as_tensor(np.asarray(b), dtype=torch.float64).clone().requires_grad_(requires_grad)
        leaves[name] = (w, bb)
    relu = {n: r for n, _, _, r in LAYERS}
    f = lambda n, t: conv(t, leaves[n][0], leaves[n][1], relu[n])
    pool = lambda t: torch.nn.functional.avg_pool2d(t, 2)
    up = lambda t: torch.nn.functional.interpolate(t, scale_factor=2, mode="nearest")
    x = torch.as_tensor(np.asarray(x_nhwc), dtype=torch.float64).permute(0, 3, 1, 2)
    e0 = f("e0b", f("e0a", x))
    e1 = f("e1b", f("e1a", pool(e0)))
    e2 = f("e2b", f("e2a", pool(e1)))
    b3 = f("b3b", f("b3a", pool(e2)))
    d2 = f("d2b", f("d2a", torch.cat([up(b3), e2], 1)))
    d1 = f("d1b", f("d1a", torch.cat([up(d2), e1], 1)))
    d0 = f("d0b", f("d0a", torch.cat([up(d1), e0], 1)))
    head = f("head", d0)
    return head.permute(0, 2, 3, 1), leaves


def loss(head_nhwc, u, v, ut, vt, su, sv, theta, front_w):
    """Mean over pixels of w (|h0 - su (ut - u)|^2 + |h1 - sv (vt - v)|^2),
    w = 1 + front_w where u or ut (not both) is >= theta.  u, v, ut, vt:
    [N, H, W] numpy arrays."""
    t = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)
    u, v, ut, vt = t(u), t(v), t(ut), t(vt)
    w = 1.0 + front_w * ((u >= theta) != (ut >= theta)).to(torch.float64)
    eu = head_nhwc[..., 0] - su * (ut - u)
    ev = head_nhwc[..., 1] - sv * (vt - v)
    return (w * (eu * eu + ev * ev)).mean()


def conv_grads(x_nhwc, W, b, gy_nhwc):
    """Single convolution (no ReLU): returns (y, dx, dW[9][cout][cin], db) for
    the output gradient gy, all float64 numpy (NHWC for y, dx)."""
    x = torch.as_tensor(np.asarray(x_nhwc), dtype=torch.float64).permute(0, 3, 1, 2)
    x.requires_grad_(True)
    w = _w(W).requires_grad_(True)
    bb = torch.as_tensor(np.asarray(b), dtype=torch.float64).clone().requires_grad_(True)
    y = torch.nn.functional.conv2d(x, w, bb, padding=1)
    gy = torch.as_tensor(np.asarray(gy_nhwc), dtype=torch.float64).permute(0, 3, 1, 2)
    y.backward(gy)
    dW = w.grad.permute(2, 3, 0, 1).reshape(9, w.shape[0], w.shape[1])
    return (y.detach().permute(0, 2, 3, 1).numpy(), x.grad.permute(0, 2, 3, 1).numpy(),
            dW.numpy(), bb.grad.numpy())
