"""Pins of the FP64 reference network against independent computations: the
3x3 convolution against explicit loops, its gradients against central finite
differences, and the whole network's gradient along a random direction."""
import numpy as np
import torch

from oracle import unet_ref


def _loops_conv(x, W, b):
    """Explicit-loop 3x3 convolution, zero padding, NHWC, W[tap][cout][cin]."""
    N, H, Wd, C = x.shape
    cout = W.shape[1]
    y = np.zeros((N, H, Wd, cout))
    for n in range(N):
        for yy in range(H):
            for xx in range(Wd):
                acc = b.copy()
                for tap in range(9):
                    sy, sx = yy + tap // 3 - 1, xx + tap % 3 - 1
                    if 0 <= sy < H and 0 <= sx < Wd:
                        acc = acc + W[tap] @ x[n, sy, sx]
                y[n, yy, xx] = acc
    return y


def test_conv_matches_explicit_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 7, 3))
    W = rng.standard_normal((9, 4, 3))
    b = rng.standard_normal(4)
    y, _, _, _ = unet_ref.conv_grads(x, W, b, np.zeros((2, 5, 7, 4)))
    assert np.allclose(y, _loops_conv(x, W, b), rtol=1e-12, atol=1e-12)


def test_conv_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 4, 6, 3))
    W = rng.standard_normal((9, 2, 3))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((1, 4, 6, 2))
    _, dx, dW, db = unet_ref.conv_grads(x, W, b, gy)
    f = lambda xx, WW, bb: float((_loops_conv(xx, WW, bb) * gy).sum())
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 3, 5, 2), (0, 2, 3, 1)]:
        e = np.zeros_like(x); e[idx] = h
        assert abs((f(x + e, W, b) - f(x - e, W, b)) / (2 * h) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0), (4, 1, 2), (8, 0, 1)]:
        e = np.zeros_like(W); e[idx] = h
        assert abs((f(x, W + e, b) - f(x, W - e, b)) / (2 * h) - dW[idx]) < 1e-6
    assert np.allclose(db, gy.sum(axis=(0, 1, 2)))


def _params(seed):
    rng = np.random.default_rng(seed)
    return {n: (rng.standard_normal((9, co, ci)) * np.sqrt(2.0 / (9 * ci)),
                rng.standard_normal(co) * 0.1) for n, ci, co, _ in unet_ref.LAYERS}


def test_network_gradient_matches_directional_difference():
    rng = np.random.default_rng(2)
    P = _params(3)
    x = rng.standard_normal((1, 16, 16, 32))
    u, v, ut, vt = (rng.random((1, 16, 16)) for _ in range(4))
    head, leaves = unet_ref.forward(P, x, requires_grad=True)
    L = unet_ref.loss(head, u, v, ut, vt, 1.0, 4.0, 0.5, 3.0)
    L.backward()
    dirs = {n: rng.standard_normal((9, co, ci)) for n, ci, co, _ in unet_ref.LAYERS}
    # d/dt L(W + t D) = sum <grad, D>
    g = sum(float((leaves[n][0].grad.permute(2, 3, 0, 1).reshape(9, co, ci).numpy() *
                   dirs[n]).sum()) for n, ci, co, _ in unet_ref.LAYERS)
    h = 1e-6
    def L_at(t):
        Q = {n: (P[n][0] + t * dirs[n], P[n][1]) for n in P}
        hd, _ = unet_ref.forward(Q, x)
        return float(unet_ref.loss(hd, u, v, ut, vt, 1.0, 4.0, 0.5, 3.0))
    fd = (L_at(h) - L_at(-h)) / (2 * h)
    assert abs(fd - g) < 1e-5 * max(1.0, abs(g))


def test_pool_and_upsample_conventions():
    x = torch.arange(16, dtype=torch.float64).reshape(1, 1, 4, 4)
    p = torch.nn.functional.avg_pool2d(x, 2)
    assert p[0, 0, 0, 0] == (0 + 1 + 4 + 5) / 4
    u = torch.nn.functional.interpolate(p, scale_factor=2, mode="nearest")
    assert u[0, 0, 1, 1] == p[0, 0, 0, 0] and u[0, 0, 2, 3] == p[0, 0, 1, 1]


def test_loss_on_a_hand_computed_two_pixel_case():
    """loss on one image of 1 x 2 pixels, worked by hand: su = 2, sv = 8,
    theta = 0.5, front weight 4.
      pixel 0: u 0.2 -> ut 0.6 crosses theta: weight 5; targets su*0.4 =
               0.8, sv*0.2 = 1.6; head (0.5, 1.0): 5 * (0.09 + 0.36) = 2.25
      pixel 1: u 0.7 -> ut 0.7 stays above: weight 1; targets 0, sv*0.05 =
               0.4; head (0.1, 0.4): 1 * (0.01 + 0) = 0.01
      mean over the two pixels: 1.13"""
    head = torch.zeros((1, 1, 2, 32), dtype=torch.float64)
    head[0, 0, 0, 0], head[0, 0, 0, 1] = 0.5, 1.0
    head[0, 0, 1, 0], head[0, 0, 1, 1] = 0.1, 0.4
    head[0, 0, :, 2:] = 7.0                   # channels past the first two play no part
    u = np.array([[[0.2, 0.7]]])
    ut = np.array([[[0.6, 0.7]]])
    v = np.array([[[0.1, 0.0]]])
    vt = np.array([[[0.3, 0.05]]])
    L = unet_ref.loss(head, u, v, ut, vt, su=2.0, sv=8.0, theta=0.5, front_w=4.0)
    assert abs(float(L) - 1.13) < 1e-12
    # both cells above or both below theta: no front weight
    L2 = unet_ref.loss(head, u, v, np.array([[[0.3, 0.9]]]), vt, su=2.0, sv=8.0, theta=0.5,
                       front_w=4.0)
    e0 = (0.5 - 2.0 * 0.1) ** 2 + (1.0 - 8.0 * 0.2) ** 2
    e1 = (0.1 - 2.0 * 0.2) ** 2 + (0.4 - 8.0 * 0.05) ** 2
    assert abs(float(L2) - (e0 + e1) / 2) < 1e-12
