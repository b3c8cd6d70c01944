"""Learned coarse stepper: a 3x3-convolution U-Net that advances the
Oregonator state by K plain steps at once, trained and run on the GPU with
the library's own kernels (rdc_nn_*), with the plain forward-Euler stepper of
Sec. 2 (Eq. (1)) as data source, reference check and fallback.

Network (4 levels, 32-64-128-128 channels, NHWC bf16 activations, fp32
accumulation and fp32 master weights):

    x0 = (su u, sv v, sp phi, 0...)            32 ch
    e0 = conv(conv(x0))                        32      H
    e1 = conv(conv(pool(e0)))                  64      H/2
    e2 = conv(conv(pool(e1)))                  128     H/4
    b3 = conv(conv(pool(e2)))                  128     H/8
    d2 = conv(conv([up(b3), e2]))              128     H/4
    d1 = conv(conv([up(d2), e1]))              64      H/2
    d0 = conv(conv([up(d1), e0]))              32      H
    head = conv(d0) (no ReLU; channels 0, 1 used)
    (u, v)_K = (u, v) + (head0 / su, head1 / sv)

This module only sequences kernel launches and holds torch-allocated
buffers; every arithmetic step runs in librdc's HIP kernels.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import inputs, rdc

LAYERS = [("e0a", 32, 32, True), ("e0b", 32, 32, True),
          ("e1a", 32, 64, True), ("e1b", 64, 64, True),
          ("e2a", 64, 128, True), ("e2b", 128, 128, True),
          ("b3a", 128, 128, True), ("b3b", 128, 128, True),
          ("d2a", 256, 128, True), ("d2b", 128, 128, True),
          ("d1a", 192, 64, True), ("d1b", 64, 64, True),
          ("d0a", 96, 32, True), ("d0b", 32, 32, True),
          ("head", 32, 32, False)]
IN_C = 32
HEAD_C = 32
SU, SV, SP = 1.0, 4.0, 5.0          # input / increment scales of u, v, phi
THETA = 0.5


def _ptr(t) -> int:
    return t.data_ptr()


class UNet:
    """Parameters (fp32 masters, bf16 copies, gradients, Adam moments) in
    flat device tensors, with per-layer views."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.offsets: Dict[str, Tuple[int, int, int]] = {}   # name -> (w_off, b_off, w_size)
        off = 0
        for name, cin, cout, _ in LAYERS:
            nw = 9 * cout * cin
            self.offsets[name] = (off, off + nw, nw)
            off += nw + cout
        self.nparams = off
        rng = np.random.default_rng(seed)
        host = np.zeros(off, dtype=np.float32)
        for name, cin, cout, _ in LAYERS:
            wo, bo, nw = self.offsets[name]
            std = np.sqrt(2.0 / (9 * cin))
            w = (rng.standard_normal((9, cout, cin)) * std).astype(np.float32)
            if name == "head":
                w *= 0.01
                w[:, 2:, :] = 0.0          # only the (u, v) increments are read
            host[wo:wo + nw] = w.ravel()
        self.p = torch.from_numpy(host).to(self.device)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.pb = torch.empty(off, dtype=torch.bfloat16, device=self.device)
        self.wd = {n: torch.empty(9 * cout * cin, dtype=torch.bfloat16, device=self.device)
                   for n, cin, cout, _ in LAYERS}
        self.t = 0
        self.sync_bf16()

    # -- parameter views
    def w_ptr(self, name, bf16=True):
        wo, _, _ = self.offsets[name]
        base = self.pb if bf16 else self.p
        return _ptr(base) + wo * base.element_size()

    def b_ptr(self, name):
        _, bo, _ = self.offsets[name]
        return _ptr(self.p) + bo * 4

    def gw_ptr(self, name):
        return _ptr(self.g) + self.offsets[name][0] * 4

    def gb_ptr(self, name):
        return _ptr(self.g) + self.offsets[name][1] * 4

    def sync_bf16(self):
        """bf16 copies of the masters (forward) and the flipped, transposed
        copies (input-gradient convolutions)."""
        s = self.stream.cuda_stream
        rdc.nn("to_bf16", _ptr(self.p), _ptr(self.pb), self.nparams, s)
        for name, cin, cout, _ in LAYERS:
            rdc.nn("dgrad_weights", self.w_ptr(name, bf16=False), _ptr(self.wd[name]), cout, cin, s)

    def get(self, name) -> Tuple[np.ndarray, np.ndarray]:
        wo, bo, nw = self.offsets[name]
        cin, cout = [(ci, co) for n, ci, co, _ in LAYERS if n == name][0]
        h = self.p.cpu().numpy()
        return h[wo:wo + nw].reshape(9, cout, cin).copy(), h[bo:bo + cout].copy()

    def set_all(self, params: Dict[str, Tuple[np.ndarray, np.ndarray]]) -> None:
        h = self.p.cpu().numpy()
        for name, (W, b) in params.items():
            wo, bo, nw = self.offsets[name]
            h[wo:wo + nw] = np.asarray(W, np.float32).ravel()
            h[bo:bo + len(b)] = np.asarray(b, np.float32)
        self.p.copy_(self.torch.from_numpy(h))
        self.sync_bf16()

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, clip=1.0):
        self.t += 1
        lr_t = lr * np.sqrt(1 - b2 ** self.t) / (1 - b1 ** self.t)
        rdc.nn("adam", _ptr(self.p), _ptr(self.g), _ptr(self.m), _ptr(self.v), self.nparams,
               float(lr_t), b1, b2, eps, clip, self.stream.cuda_stream)
        self.sync_bf16()


class Workspace:
    """Activation and gradient buffers for N images of H x W (H a multiple of
    8 and W of 256, so the coarsest level is still a whole number of 32-pixel
    row segments)."""

    def __init__(self, net: UNet, N: int, H: int, W: int, train: bool = True):
        torch = net.torch
        if H % 8 or W % 256 or H < 8:
            raise ValueError("H must be a multiple of 8 and W of 256")
        self.net, self.N, self.H, self.W = net, N, H, W
        bf = lambda h, w, c: torch.zeros((N, h, w, c), dtype=torch.bfloat16, device=net.device)
        H1, W1, H2, W2, H3, W3 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8
        self.shape = {0: (H, W), 1: (H1, W1), 2: (H2, W2), 3: (H3, W3)}
        a = {}
        a["x0"] = bf(H, W, IN_C); a["e0a"] = bf(H, W, 32); a["c0"] = bf(H, W, 96)
        a["d0a"] = bf(H, W, 32); a["d0b"] = bf(H, W, 32); a["head"] = bf(H, W, HEAD_C)
        a["p1"] = bf(H1, W1, 32); a["e1a"] = bf(H1, W1, 64); a["c1"] = bf(H1, W1, 192)
        a["d1a"] = bf(H1, W1, 64); a["d1b"] = bf(H1, W1, 64)
        a["p2"] = bf(H2, W2, 64); a["e2a"] = bf(H2, W2, 128); a["c2"] = bf(H2, W2, 256)
        a["d2a"] = bf(H2, W2, 128); a["d2b"] = bf(H2, W2, 128)
        a["p3"] = bf(H3, W3, 128); a["b3a"] = bf(H3, W3, 128); a["b3b"] = bf(H3, W3, 128)
        self.a = a
        self.g = {k: torch.zeros_like(v) for k, v in a.items() if k != "x0"} if train else {}
        if train:
            need = max(rdc.load().rdc_nn_wgrad_scratch_floats(N, *self._hw(name), cin, cout)
                       for name, cin, cout, _ in LAYERS)
            self.scratch = torch.empty(int(need), dtype=torch.float32, device=net.device)
            self.partial = torch.empty(rdc.load().rdc_nn_loss_blocks(N * H * W) + 1,
                                       dtype=torch.float32, device=net.device)

    def _hw(self, name):
        lvl = {"e0": 0, "d0": 0, "he": 0, "e1": 1, "d1": 1, "e2": 2, "d2": 2, "b3": 3}[name[:2]]
        return self.shape[lvl]

    # (tensor name, channel offset, channel count) -> (address, pixel stride)
    def at(self, buf, name, off=0):
        t = buf[name]
        return _ptr(t) + off * 2, t.shape[-1]


def conv_flops(name: str, ws: "Workspace") -> int:
    """Multiply-adds x 2 of forward convolution `name` over the workspace."""
    cin, cout = [(ci, co) for n, ci, co, _ in LAYERS if n == name][0]
    H, W = ws._hw(name)
    return 2 * 9 * cin * cout * H * W * ws.N


UP_PREFIX = {"d2a": 128, "d1a": 128, "d0a": 64}   # upsampled channels of a decoder's input


def conv_bytes(name: str, ws: "Workspace") -> int:
    """HBM bytes one launch of convolution `name` must move in the inference
    form (forward_planes): its input read once (the first layer: the three
    fp32 stepper planes; a decoder: the skip channels at full resolution and
    the upsampled prefix at the coarse level), its output written once, and
    its bf16 weights."""
    cin, cout = [(ci, co) for n, ci, co, _ in LAYERS if n == name][0]
    H, W = ws._hw(name)
    px = ws.N * H * W
    if name == "e0a":
        x = px * 12
    elif name in UP_PREFIX:
        up = UP_PREFIX[name]
        x = px * (cin - up) * 2 + (px // 4) * up * 2
    else:
        x = px * cin * 2
    return x + px * cout * 2 + 9 * cin * cout * 2


def _conv(net, ws, name, src, dst, relu=True, store=None, events=None):
    """Forward convolution `name` from (addr, ld) src to (addr, ld) dst;
    with `events` (a dict), HIP events around the launch on the net's stream
    are appended to events[name]."""
    cin, cout = [(ci, co) for n, ci, co, _ in LAYERS if n == name][0]
    H, W = ws._hw(name)
    if events is not None:
        e0 = net.torch.cuda.Event(enable_timing=True)
        e1 = net.torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
    rdc.nn("conv3x3", src[0], src[1], net.w_ptr(name), net.b_ptr(name), dst[0], dst[1], ws.N,
           H, W, cin, cout, store or cout, 1 if relu else 0, net.stream.cuda_stream)
    if events is not None:
        e1.record(net.stream)
        events.setdefault(name, []).append((e0, e1))


def forward(net: UNet, ws: Workspace, events=None) -> None:
    """Runs the network on ws.a['x0'] (filled by prep), leaving ws.a['head'].
    `events`: see _conv."""
    A, s = ws.a, net.stream.cuda_stream
    at = lambda n, o=0: ws.at(A, n, o)

    def conv(name, src, dst, relu=True):
        _conv(net, ws, name, src, dst, relu=relu, events=events)

    N = ws.N
    (H, W), (H1, W1), (H2, W2), (H3, W3) = (ws.shape[i] for i in range(4))
    conv("e0a", at("x0"), at("e0a"))
    conv("e0b", at("e0a"), at("c0", 64))
    rdc.nn("pool2", *at("c0", 64), *at("p1"), N, H1, W1, 32, s)
    conv("e1a", at("p1"), at("e1a"))
    conv("e1b", at("e1a"), at("c1", 128))
    rdc.nn("pool2", *at("c1", 128), *at("p2"), N, H2, W2, 64, s)
    conv("e2a", at("p2"), at("e2a"))
    conv("e2b", at("e2a"), at("c2", 128))
    rdc.nn("pool2", *at("c2", 128), *at("p3"), N, H3, W3, 128, s)
    conv("b3a", at("p3"), at("b3a"))
    conv("b3b", at("b3a"), at("b3b"))
    rdc.nn("up2", *at("b3b"), *at("c2"), N, H2, W2, 128, s)
    conv("d2a", at("c2"), at("d2a"))
    conv("d2b", at("d2a"), at("d2b"))
    rdc.nn("up2", *at("d2b"), *at("c1"), N, H1, W1, 128, s)
    conv("d1a", at("c1"), at("d1a"))
    conv("d1b", at("d1a"), at("d1b"))
    rdc.nn("up2", *at("d1b"), *at("c0"), N, H, W, 64, s)
    conv("d0a", at("c0"), at("d0a"))
    conv("d0b", at("d0a"), at("d0b"))
    conv("head", at("d0b"), at("head"), relu=False)


def forward_planes(net: UNet, ws: Workspace, u, v, phi, pitch, plane_stride,
                   events=None, predict=None) -> None:
    """Inference form of prep + forward, leaving the same ws.a['head'] bit for
    bit: the first layer builds its input from the stepper planes while
    loading them (no x0), and each decoder layer reads the upsampled half of
    its concatenation straight from the coarser level (no up2 writes).  The
    concatenation buffers then hold only their skip channels, so training
    (whose backward pass reads them whole) uses prep + forward.  With
    `predict` = (uo, vo, params) the head's launch also applies the
    prediction (as `apply` would) and leaves ws.a['head'] untouched."""
    A, s = ws.a, net.stream.cuda_stream
    at = lambda n, o=0: ws.at(A, n, o)
    N = ws.N
    (H, W), (H1, W1), (H2, W2), _ = (ws.shape[i] for i in range(4))

    def timed(name, launch):
        if events is not None:
            e0 = net.torch.cuda.Event(enable_timing=True)
            e1 = net.torch.cuda.Event(enable_timing=True)
            e0.record(net.stream)
        launch()
        if events is not None:
            e1.record(net.stream)
            events.setdefault(name, []).append((e0, e1))

    def conv(name, src, dst, relu=True):
        _conv(net, ws, name, src, dst, relu=relu, events=events)

    def up_conv(name, skip, low, up_c, dst, h, w):
        cin, cout = [(ci, co) for n, ci, co, _ in LAYERS if n == name][0]
        timed(name, lambda: rdc.nn("conv3x3_up", skip[0], skip[1], low[0], low[1], up_c,
                                   net.w_ptr(name), net.b_ptr(name), dst[0], dst[1], N, h, w,
                                   cin, cout, cout, s))

    timed("e0a", lambda: rdc.nn("conv3x3_planes", u, v, phi, pitch, plane_stride, SU, SV, SP,
                                net.w_ptr("e0a"), net.b_ptr("e0a"), *at("e0a"), N, H, W, IN_C,
                                32, 32, s))
    conv("e0b", at("e0a"), at("c0", 64))
    rdc.nn("pool2", *at("c0", 64), *at("p1"), N, H1, W1, 32, s)
    conv("e1a", at("p1"), at("e1a"))
    conv("e1b", at("e1a"), at("c1", 128))
    rdc.nn("pool2", *at("c1", 128), *at("p2"), N, H2, W2, 64, s)
    conv("e2a", at("p2"), at("e2a"))
    conv("e2b", at("e2a"), at("c2", 128))
    rdc.nn("pool2", *at("c2", 128), *at("p3"), N, H2 // 2, W2 // 2, 128, s)
    conv("b3a", at("p3"), at("b3a"))
    conv("b3b", at("b3a"), at("b3b"))
    up_conv("d2a", at("c2"), at("b3b"), UP_PREFIX["d2a"], at("d2a"), H2, W2)
    conv("d2b", at("d2a"), at("d2b"))
    up_conv("d1a", at("c1"), at("d2b"), UP_PREFIX["d1a"], at("d1a"), H1, W1)
    conv("d1b", at("d1a"), at("d1b"))
    up_conv("d0a", at("c0"), at("d1b"), UP_PREFIX["d0a"], at("d0a"), H, W)
    conv("d0b", at("d0a"), at("d0b"))
    if predict is None:
        conv("head", at("d0b"), at("head"), relu=False)
    else:
        uo, vo, params = predict
        timed("head", lambda: rdc.nn("conv3x3_apply", *at("d0b"), net.w_ptr("head"),
                                     net.b_ptr("head"), u, v, phi, pitch, plane_stride, uo, vo,
                                     N, H, W, 32, SU, SV, float(params["f"]),
                                     euler_safe_c(params), s))


def _layer_bwd(net, ws, name, x, gy, gx=None):
    """Gradients of layer `name`: x = its input (addr, ld), gy = output
    gradient (addr, ld) (already through the ReLU adjoint).  Writes dW, db
    into net.g and, if gx is given, the input gradient there."""
    cin, cout = [(ci, co) for n, ci, co, _ in LAYERS if n == name][0]
    H, W = ws._hw(name)
    s = net.stream.cuda_stream
    rdc.nn("conv3x3_wgrad", x[0], x[1], gy[0], gy[1], _ptr(ws.scratch), net.gw_ptr(name),
           net.gb_ptr(name), ws.N, H, W, cin, cout, s)
    if gx is not None:
        rdc.nn("conv3x3", gy[0], gy[1], _ptr(net.wd[name]), None, gx[0], gx[1], ws.N, H, W,
               cout, cin, cin, 0, s)


def backward(net: UNet, ws: Workspace) -> None:
    """Back-propagates ws.g['head'] (from the loss) into net.g."""
    A, G, s = ws.a, ws.g, net.stream.cuda_stream
    a = lambda n, o=0: ws.at(A, n, o)
    g = lambda n, o=0: ws.at(G, n, o)
    N = ws.N
    (H, W), (H1, W1), (H2, W2), (H3, W3) = (ws.shape[i] for i in range(4))
    P = lambda lv: N * ws.shape[lv][0] * ws.shape[lv][1]

    def relu_bwd(gname, goff, yname, yoff, c, lvl):
        rdc.nn("relu_bwd", *g(gname, goff), *a(yname, yoff), P(lvl), c, s)

    _layer_bwd(net, ws, "head", a("d0b"), g("head"), g("d0b"))
    relu_bwd("d0b", 0, "d0b", 0, 32, 0)
    _layer_bwd(net, ws, "d0b", a("d0a"), g("d0b"), g("d0a"))
    relu_bwd("d0a", 0, "d0a", 0, 32, 0)
    _layer_bwd(net, ws, "d0a", a("c0"), g("d0a"), g("c0"))
    rdc.nn("up2_bwd", *g("c0"), *g("d1b"), N, H1, W1, 64, s)
    relu_bwd("d1b", 0, "d1b", 0, 64, 1)
    _layer_bwd(net, ws, "d1b", a("d1a"), g("d1b"), g("d1a"))
    relu_bwd("d1a", 0, "d1a", 0, 64, 1)
    _layer_bwd(net, ws, "d1a", a("c1"), g("d1a"), g("c1"))
    rdc.nn("up2_bwd", *g("c1"), *g("d2b"), N, H2, W2, 128, s)
    relu_bwd("d2b", 0, "d2b", 0, 128, 2)
    _layer_bwd(net, ws, "d2b", a("d2a"), g("d2b"), g("d2a"))
    relu_bwd("d2a", 0, "d2a", 0, 128, 2)
    _layer_bwd(net, ws, "d2a", a("c2"), g("d2a"), g("c2"))
    rdc.nn("up2_bwd", *g("c2"), *g("b3b"), N, H3, W3, 128, s)
    relu_bwd("b3b", 0, "b3b", 0, 128, 3)
    _layer_bwd(net, ws, "b3b", a("b3a"), g("b3b"), g("b3a"))
    relu_bwd("b3a", 0, "b3a", 0, 128, 3)
    _layer_bwd(net, ws, "b3a", a("p3"), g("b3a"), g("p3"))
    rdc.nn("pool2_bwd", *g("p3"), *g("c2", 128), N, H3, W3, 128, 1, s)
    relu_bwd("c2", 128, "c2", 128, 128, 2)
    _layer_bwd(net, ws, "e2b", a("e2a"), g("c2", 128), g("e2a"))
    relu_bwd("e2a", 0, "e2a", 0, 128, 2)
    _layer_bwd(net, ws, "e2a", a("p2"), g("e2a"), g("p2"))
    rdc.nn("pool2_bwd", *g("p2"), *g("c1", 128), N, H2, W2, 64, 1, s)
    relu_bwd("c1", 128, "c1", 128, 64, 1)
    _layer_bwd(net, ws, "e1b", a("e1a"), g("c1", 128), g("e1a"))
    relu_bwd("e1a", 0, "e1a", 0, 64, 1)
    _layer_bwd(net, ws, "e1a", a("p1"), g("e1a"), g("p1"))
    rdc.nn("pool2_bwd", *g("p1"), *g("c0", 64), N, H1, W1, 32, 1, s)
    relu_bwd("c0", 64, "c0", 64, 32, 0)
    _layer_bwd(net, ws, "e0b", a("e0a"), g("c0", 64), g("e0a"))
    relu_bwd("e0a", 0, "e0a", 0, 32, 0)
    _layer_bwd(net, ws, "e0a", a("x0"), g("e0a"))


def prep(net: UNet, ws: Workspace, u_addr, v_addr, phi_addr, pitch, plane_stride):
    rdc.nn("prep", u_addr, v_addr, phi_addr, pitch, plane_stride, _ptr(ws.a["x0"]), IN_C, ws.N,
           ws.H, ws.W, SU, SV, SP, net.stream.cuda_stream)


def loss_and_grad(net: UNet, ws: Workspace, u, v, ut, vt, pitch, plane_stride,
                  front_w: float = 4.0) -> float:
    """Writes d loss / d head into ws.g['head']; returns the loss (syncs)."""
    rdc.nn("loss", u, v, ut, vt, pitch, plane_stride, _ptr(ws.a["head"]), HEAD_C,
           _ptr(ws.g["head"]), HEAD_C, ws.N, ws.H, ws.W, SU, SV, THETA, front_w,
           _ptr(ws.partial), net.stream.cuda_stream)
    return float(ws.partial[-1].item())


def euler_safe_c(params, margin: float = 0.1) -> float:
    """Largest f v + phi the network's output may carry: one forward-Euler
    step of Eq. (1) from any u >= 0 stays above the reaction term's pole at
    u = -q iff dt (f v + phi) / eps < 8 q; `margin` leaves room for the
    diffusion term."""
    return (1.0 - margin) * 8.0 * params["q"] * params["eps"] / params["dt"]


def apply(net: UNet, ws: Workspace, u, v, phi, uo, vo, pitch, plane_stride, params):
    """(uo, vo) = (u, v) + the head's increments, projected onto the states
    the plain stepper can continue from (0 <= u <= 1, f v + phi <= cmax)."""
    rdc.nn("apply", u, v, phi, _ptr(ws.a["head"]), HEAD_C, pitch, plane_stride, uo, vo, ws.N,
           ws.H, ws.W, SU, SV, float(params["f"]), euler_safe_c(params), net.stream.cuda_stream)


# ----------------------------------------------------------------- training data and loop

def training_batch_sims(n: int, count: int, seed: int, steps: int) -> List[inputs.Workload]:
    """Random circuit maps (channels on phi=0.2, diodes and AND junctions)
    with input disks over the first `steps` steps, the earliest candidates
    kept first (waves are under way once the burn-in ends)."""
    return [inputs.circuit(n=n, seed=seed + i, steps=steps, ndisks=max(4, (n // 128) ** 2),
                           tile=128, disk_order="time") for i in range(count)]


class Trainer:
    """Trains the network on pairs (state at t, state at t + K) that the
    plain stepper generates on the fly from random circuits.

    With `pushforward` p > 0, a fraction p of the iterations (once a previous
    pair of the same circuits exists) replaces the input S_t by the network's
    own prediction of it from S_(t-K) (no gradient through that prediction),
    keeping the plain S_(t+K) as the target: the network learns to correct
    the kind of error it makes, which is what accumulates between the plain
    stepper's checks."""

    def __init__(self, net: UNet, n: int = 256, batch: int = 8, K: int = 50, burn_in: int = 1000,
                 seed: int = 100, pushforward: float = 0.0):
        import torch
        self.net, self.n, self.batch, self.K, self.burn_in = net, n, batch, K, burn_in
        self.seed = seed
        self.pushforward = float(pushforward)
        self.rng = np.random.default_rng(seed)
        self.ws = Workspace(net, batch, n, n, train=True)
        self.pitch = rdc.pitch_for(n)
        self.plane = self.pitch * n
        self.u_in = torch.empty(batch * self.plane, dtype=torch.float32, device=net.device)
        self.v_in = torch.empty_like(self.u_in)
        # S_(t-K) of the current circuits and a spare pair, for pushforward
        self.u_prev, self.v_prev, self.u_next, self.v_next = (
            torch.empty_like(self.u_in) for _ in range(4))
        self.prev_ok = False
        self.round = 0
        self.dropped_batches = 0      # batches with a non-finite plain grid (never trained on)
        self.skipped_iters = 0        # iterations whose loss was not finite (no update made)
        self._new_sims()

    def _new_sims(self):
        horizon = self.burn_in + 40 * self.K
        wls = training_batch_sims(self.n, self.batch, self.seed + 1000 * self.round, horizon)
        self.round += 1
        self.wls = wls
        self.sims = rdc.BatchSim([(w.nx, w.ny, w.params) for w in wls])
        for i, w in enumerate(wls):
            self.sims.set_phi(i, w.phi)
        self.now = 0
        self.sched = sorted((s.step, i, s.cx, s.cy, s.r) for i, w in enumerate(wls)
                            for s in w.stimuli)
        self._advance(self.burn_in)

    def _advance(self, n):
        end = self.now + n
        while self.now < end:
            pend = [t for t in self.sched if self.now <= t[0] < end]
            nxt = pend[0][0] if pend else end
            if nxt > self.now:
                self.sims.step(nxt - self.now)
                self.now = nxt
            if pend:
                self.sims.stimulate([(i, cx, cy, r) for (t, i, cx, cy, r) in self.sched
                                     if t == self.now])
                self.sched = [x for x in self.sched if x[0] != self.now]

    def pair(self):
        """Copies the current states to (u_in, v_in), advances K plain steps;
        returns device addresses (u, v, phi, u_target, v_target).  Pairs come
        from finite plain trajectories only: a batch in which any grid has
        set its non-finite flag (a stiff circuit whose refractory tail left
        the Euler scheme's stable range) is dropped and a fresh one drawn."""
        while True:
            if self.now + self.K > self.burn_in + 40 * self.K:
                self.sims.close()
                self._new_sims()
                self.prev_ok = False
            u, v = self.sims.current()
            s = self.net.stream.cuda_stream
            nb = 4 * self.batch * self.plane
            rdc.rdc_copy(_ptr(self.u_in), _ptr(u), nb, s)
            rdc.rdc_copy(_ptr(self.v_in), _ptr(v), nb, s)
            self._advance(self.K)
            if not self.sims.nonfinite():
                break
            self.dropped_batches += 1
            self.now = self.burn_in + 40 * self.K          # draw a fresh batch
        ut, vt = self.sims.current()
        return (_ptr(self.u_in), _ptr(self.v_in), _ptr(self.sims.planes[4]), _ptr(ut), _ptr(vt))

    def step(self, lr: float = 1e-3) -> float:
        u, v, phi, ut, vt = self.pair()          # (u, v) = plain S_t, (ut, vt) = S_(t+K)
        if self.pushforward > 0:
            s = self.net.stream.cuda_stream
            nb = 4 * self.batch * self.plane
            if self.prev_ok and self.rng.random() < self.pushforward:
                # training input := the network's prediction of S_t from S_(t-K)
                # (the inference form; the training forward below rewrites
                # every buffer it reads)
                rdc.rdc_copy(_ptr(self.u_next), u, nb, s)          # keep the plain S_t
                rdc.rdc_copy(_ptr(self.v_next), v, nb, s)
                forward_planes(self.net, self.ws, _ptr(self.u_prev), _ptr(self.v_prev), phi,
                               self.pitch, self.plane,
                               predict=(u, v, self.wls[0].params))
                self.u_prev, self.u_next = self.u_next, self.u_prev
                self.v_prev, self.v_next = self.v_next, self.v_prev
            else:
                rdc.rdc_copy(_ptr(self.u_prev), u, nb, s)
                rdc.rdc_copy(_ptr(self.v_prev), v, nb, s)
            self.prev_ok = True
        prep(self.net, self.ws, u, v, phi, self.pitch, self.plane)
        forward(self.net, self.ws)
        L = loss_and_grad(self.net, self.ws, u, v, ut, vt, self.pitch, self.plane)
        if not np.isfinite(L):
            self.skipped_iters += 1               # keep the weights finite
            return L
        backward(self.net, self.ws)
        self.net.adam(lr=lr)
        return L

    def close(self):
        self.sims.close()


def train(net: UNet, iters: int, n: int = 256, batch: int = 8, K: int = 50, lr: float = 1e-3,
          seed: int = 100, log_every: int = 0, pushforward: float = 0.0) -> List[float]:
    tr = Trainer(net, n=n, batch=batch, K=K, seed=seed, pushforward=pushforward)
    losses = []
    t0 = time.time()
    for it in range(iters):
        lr_it = lr * (0.1 ** (it / max(1, iters)))          # smooth decay to lr/10
        losses.append(tr.step(lr_it))
        if log_every and (it + 1) % log_every == 0:
            print("  iter %d loss %.5f (%.1f s)" % (it + 1, np.mean(losses[-log_every:]),
                                                      time.time() - t0), flush=True)
    tr.close()
    return losses


# ----------------------------------------------------------------- inference with fallback

class CoarseStepper:
    """Advances one FP32 grid K plain steps at a time with the network, under
    the plain stepper's supervision (predictor, checked by the plain stepper):

      * a checkpoint always holds a state the plain stepper produced: the
        start, the plain result of every passed check, the end of every plain
        window;
      * every `check_every`-th network step (the first one included) is also
        computed by the plain stepper from the same input.  The check passes
        if the two fronts (u >= theta) differ by more than one cell in at most
        `max_bad` cells and the plain result is one the plain stepper can
        continue (no NaN, u above the reaction term's pole at -q, f v + phi
        within the Euler bound 8 q eps / dt less the margin of
        euler_safe_c -- plain trajectories of the workloads stay below it,
        while states the network has pushed off them can exceed it and
        later diverge); the run then continues from the plain result, which
        becomes the checkpoint;
      * a failed check discards everything since the checkpoint: the grid is
        reset to it and the plain stepper replays the steps (and stimuli)
        since then, and the next `cooldown` windows run plainly before the
        network is tried again (its next step is checked).  So a network that
        never passes leaves exactly the plain stepper's trajectory;
      * stimuli land on their exact step: a window that would cross one is
        cut short with plain steps.

    `track=True` adds a third grid stepped plainly in lock-step (not part of
    the method: a measurement of its front error after every window)."""

    def __init__(self, net: UNet, nx: int, ny: int, params, phi, K: int = 50,
                 check_every: int = 10, theta: float = 0.5, max_bad: int = 0, cooldown: int = 1,
                 track: bool = False):
        import torch
        if nx % 256 or ny % 8:
            raise ValueError("the coarse stepper needs nx % 256 == 0 and ny % 8 == 0")
        self.net, self.K, self.check_every = net, K, check_every
        self.theta, self.max_bad, self.cooldown = theta, max_bad, cooldown
        self.params = dict(params)
        self.ulo = -float(params["q"])
        self.cmax_valid = euler_safe_c(params)
        self.sim = rdc.Sim(nx, ny, params, "fp32")
        self.verify_sim = rdc.Sim(nx, ny, params, "fp32")
        self.ref = rdc.Sim(nx, ny, params, "fp32") if track else None
        for s in (self.sim, self.verify_sim, self.ref):
            if s is not None:
                s.set_phi(phi)
        shape = self.sim.autotune()
        for s in (self.verify_sim, self.ref):
            if s is not None:
                s.set_block(shape["T"])
                s.set_tile_rows(shape["rows"])
        self.nx, self.ny, self.pitch = nx, ny, self.sim.pitch
        self.plane = ny * self.pitch
        self.ws = Workspace(net, 1, ny, nx, train=False)
        self.count = torch.zeros(1, dtype=torch.int32, device=net.device)
        self.ckpt = [torch.empty(self.plane, dtype=torch.float32, device=net.device)
                     for _ in range(2)]
        self.ckpt_t = None
        self.log: List[Tuple[int, list]] = []       # stimuli since the checkpoint
        self.now = 0
        # network_steps + plain_steps = steps of the final trajectory;
        # replayed_steps and discarded_network_steps are work redone or lost
        # after failed checks.
        self.stats = dict(network_steps=0, plain_steps=0, replayed_steps=0,
                          discarded_network_steps=0, checks=0, failed_checks=0, windows=0,
                          tracked_windows=0, windows_off=0, max_cells_off=0)
        self._pending = 0          # network steps since the checkpoint
        self._since_check = None
        self._cool = 0

    # -- state
    def write(self, u, v):
        for s in (self.sim, self.ref):
            if s is not None:
                s.write(u, v)
        self.ckpt_t = None

    def stimulate(self, disks):
        disks = [tuple(d) for d in disks]
        for s in (self.sim, self.ref):
            if s is not None:
                s.stimulate(disks)
        if self.ckpt_t is not None:
            self.log.append((self.now, disks))

    def current(self, allow_nonfinite: bool = False):
        return self.sim.current(allow_nonfinite)

    def read(self):
        return self.sim.read()

    # -- pieces
    def _copy(self, du, dv, su, sv):
        s = self.net.stream.cuda_stream
        nb = 4 * self.plane
        rdc.rdc_copy(du.data_ptr(), su.data_ptr(), nb, s)
        rdc.rdc_copy(dv.data_ptr(), sv.data_ptr(), nb, s)

    def _copy_state(self, dst: "rdc.Sim", src: "rdc.Sim"):
        du, dv = dst.current(allow_nonfinite=True)
        su, sv = src.current(allow_nonfinite=True)
        self._copy(du, dv, su, sv)

    def _checkpoint(self):
        u, v = self.sim.current(allow_nonfinite=True)
        self._copy(self.ckpt[0], self.ckpt[1], u, v)
        self.ckpt_t = self.now
        self.log = []
        self._pending = 0

    def _rollback_and_replay(self, until: int):
        """Reset the grid to the checkpoint and replay plainly to `until`."""
        u, v = self.sim.current(allow_nonfinite=True)
        self._copy(u, v, self.ckpt[0], self.ckpt[1])
        t = self.ckpt_t
        for when, disks in self.log:
            self.sim.step(when - t)
            t = when
            self.sim.stimulate(disks)
        self.sim.step(until - t)
        st = self.stats
        st["replayed_steps"] += until - self.ckpt_t
        st["network_steps"] -= self._pending
        st["plain_steps"] += self._pending
        st["discarded_network_steps"] += self._pending

    def _network_step(self):
        u, v = self.sim.current(allow_nonfinite=True)
        forward_planes(self.net, self.ws, u.data_ptr(), v.data_ptr(),
                       self.sim.planes[4].data_ptr(), self.pitch, self.plane,
                       predict=(u.data_ptr(), v.data_ptr(), self.params))

    def _cells_off(self, a: "rdc.Sim", b: "rdc.Sim") -> int:
        """Cells whose fronts differ by more than one cell between a and b."""
        self.count.zero_()
        ua = a.current(allow_nonfinite=True)[0]
        ub = b.current(allow_nonfinite=True)[0]
        rdc.nn("front_check", ua.data_ptr(), ub.data_ptr(), self.pitch,
               self.nx, self.ny, self.theta, self.count.data_ptr(), self.net.stream.cuda_stream)
        return int(self.count.item())

    def _invalid(self, a: "rdc.Sim") -> int:
        """Cells of a's state the plain stepper cannot be trusted to continue."""
        self.count.zero_()
        u, v = a.current(allow_nonfinite=True)
        rdc.nn("state_check", u.data_ptr(), v.data_ptr(), a.planes[4].data_ptr(), self.pitch,
               self.nx, self.ny, self.ulo, 1.5, float(self.params["f"]), self.cmax_valid,
               self.count.data_ptr(), self.net.stream.cuda_stream)
        return int(self.count.item())

    def _plain(self, n: int):
        if n > 0:
            self.sim.step(n)
            if self.ref is not None:
                self.ref.step(n)
            self.now += n
            self.stats["plain_steps"] += n

    def _window(self):
        K, st = self.K, self.stats
        st["windows"] += 1
        if self.ckpt_t is None:
            self._checkpoint()
        if self._cool > 0:
            self._cool -= 1
            self._plain(K)
            if self._pending == 0:
                self._checkpoint()
        else:
            checked = self._since_check is None or self._since_check >= self.check_every - 1
            if checked:
                self._copy_state(self.verify_sim, self.sim)
                self.verify_sim.step(K)
                self._network_step()
                st["checks"] += 1
                if (self._cells_off(self.verify_sim, self.sim) > self.max_bad
                        or self._invalid(self.verify_sim) > 0):
                    st["failed_checks"] += 1
                    self._rollback_and_replay(self.now + K)
                    self._cool = self.cooldown
                    self._since_check = None
                else:
                    self._copy_state(self.sim, self.verify_sim)
                    self._since_check = 0
                st["plain_steps"] += K
                self.now += K
                self._checkpoint()
            else:
                self._network_step()
                st["network_steps"] += K
                self._pending += K
                self._since_check += 1
                self.now += K
            if self.ref is not None:
                self.ref.step(K)
        if self.ref is not None:
            off = self._cells_off(self.ref, self.sim)
            st["tracked_windows"] += 1
            st["windows_off"] += int(off > 0)
            st["max_cells_off"] = max(st["max_cells_off"], off)

    def advance_to(self, until: int, stimuli=()):
        """Advance to step index `until`, applying (step, cx, cy, r)
        stimuli right before the step that leaves their step index."""
        groups = {}
        for s in stimuli:
            t = (s.step, s.cx, s.cy, s.r) if hasattr(s, "step") else tuple(s)
            groups.setdefault(int(t[0]), []).append(t[1:])
        for when in sorted(groups) + [until]:
            if when < self.now or when > until:
                continue
            while self.now + self.K <= when:
                self._window()
            self._plain(when - self.now)
            if when in groups:
                self.stimulate(groups[when])
            if when == until:
                break

    def close(self):
        for s in (self.sim, self.verify_sim, self.ref):
            if s is not None:
                s.close()
