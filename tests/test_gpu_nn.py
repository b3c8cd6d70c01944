"""The learned coarse stepper's kernels on the GPU, through the C ABI, against
the FP64 CPU network reference (oracle/unet_ref.py) and plain definitions.

Operands are rounded to bfloat16 on the host first, so the reference sees
exactly the values the kernels see; what remains is fp32 accumulation and
the final bf16 rounding of an output (half an ulp: 2^-8 relative).  The
tolerances below are those two terms, with the accumulation term scaled by
the sum of |terms| of each output (the same contraction on |x| and |w|).
"""
import numpy as np
import pytest

from oracle import unet_ref
from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu

HALF_ULP = 2.0 ** -8


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _bf(torch, a):
    """Host array -> (device bf16 tensor, float64 copy of the rounded values)."""
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.cuda(), t.double().numpy()


def _host(t):
    return t.double().cpu().numpy()


def _sync(torch):
    torch.cuda.synchronize()


def _stream(torch):
    return torch.cuda.current_stream().cuda_stream


CONV_CASES = [  # cin, cout, N, H, W, relu, bias, cout_store, ldx extra channels
    (16, 32, 1, 3, 32, 1, 1, 32, 0),
    (32, 32, 2, 5, 96, 1, 1, 32, 16),
    (32, 64, 1, 7, 64, 0, 1, 64, 0),
    (64, 128, 2, 4, 64, 1, 0, 128, 0),
    (128, 128, 1, 6, 32, 1, 1, 128, 32),
    (256, 128, 1, 3, 64, 1, 1, 128, 0),
    (192, 64, 1, 5, 32, 1, 1, 64, 0),
    (96, 32, 2, 3, 64, 1, 1, 32, 0),
    (32, 96, 1, 4, 32, 0, 0, 96, 0),
    (128, 256, 1, 2, 32, 0, 0, 256, 0),
    (64, 192, 1, 3, 32, 0, 0, 192, 0),
    (32, 32, 1, 4, 64, 0, 1, 4, 0),
    (64, 64, 2, 5, 64, 1, 1, 64, 8),      # weights of both chunks resident in LDS
    (64, 32, 1, 9, 96, 1, 1, 32, 0),      # 32 outputs, two resident chunks
]


@pytest.mark.parametrize("cin,cout,N,H,W,relu,bias,store,extra", CONV_CASES)
def test_conv3x3_forward(torch, cin, cout, N, H, W, relu, bias, store, extra):
    rng = np.random.default_rng(cin * 1000 + cout + H)
    ldx = cin + extra
    x, xr = _bf(torch, rng.standard_normal((N, H, W, ldx)))
    w, wr = _bf(torch, rng.standard_normal((9, cout, cin)) / np.sqrt(9 * cin))
    b = rng.standard_normal(cout).astype(np.float32)
    bd = torch.as_tensor(b).cuda()
    ldy = max(store, 4) + 4
    y = torch.full((N, H, W, ldy), 7.0, dtype=torch.bfloat16, device="cuda")
    rdc.nn("conv3x3", x.data_ptr(), ldx, w.data_ptr(), bd.data_ptr() if bias else None,
           y.data_ptr(), ldy, N, H, W, cin, cout, store, relu, _stream(torch))
    _sync(torch)
    bb = b.astype(np.float64) if bias else np.zeros(cout)
    ref, _, _, _ = unet_ref.conv_grads(xr[..., :cin], wr, bb, np.zeros((N, H, W, cout)))
    mag, _, _, _ = unet_ref.conv_grads(np.abs(xr[..., :cin]), np.abs(wr), np.abs(bb),
                                       np.zeros((N, H, W, cout)))
    if relu:
        ref = np.maximum(ref, 0.0)
    got = _host(y)
    s = max(store, 4)
    err = np.abs(got[..., :store] - ref[..., :store])
    tol = HALF_ULP * np.abs(ref[..., :store]) + 2.0 ** -18 * mag[..., :store]
    assert (err <= tol).all(), float((err - tol).max())
    assert (got[..., s:] == 7.0).all()          # channels past cout_store untouched


@pytest.mark.parametrize("cin,cout,N,H,W", [(32, 32, 2, 5, 64), (96, 32, 1, 4, 32),
                                            (256, 128, 1, 3, 32), (192, 64, 1, 3, 64)])
def test_dgrad_is_the_input_gradient(torch, cin, cout, N, H, W):
    rng = np.random.default_rng(cin + 7 * cout)
    wm = (rng.standard_normal((9, cout, cin)) / np.sqrt(9 * cin)).astype(np.float32)
    wmd = torch.as_tensor(wm).cuda()
    wd = torch.empty(9 * cout * cin, dtype=torch.bfloat16, device="cuda")
    rdc.nn("dgrad_weights", wmd.data_ptr(), wd.data_ptr(), cout, cin, _stream(torch))
    gy, gyr = _bf(torch, rng.standard_normal((N, H, W, cout)))
    gx = torch.empty((N, H, W, cin), dtype=torch.bfloat16, device="cuda")
    rdc.nn("conv3x3", gy.data_ptr(), cout, wd.data_ptr(), None, gx.data_ptr(), cin, N, H, W,
           cout, cin, cin, 0, _stream(torch))
    _sync(torch)
    wr = torch.as_tensor(wm).to(torch.bfloat16).double().numpy()
    x0 = np.zeros((N, H, W, cin))
    _, ref, _, _ = unet_ref.conv_grads(x0, wr, np.zeros(cout), gyr)
    _, mag, _, _ = unet_ref.conv_grads(x0, np.abs(wr), np.zeros(cout), np.abs(gyr))
    err = np.abs(_host(gx) - ref)
    assert (err <= HALF_ULP * np.abs(ref) + 2.0 ** -18 * mag).all()


@pytest.mark.parametrize("cin,cout,N,H,W,ldx", [(32, 32, 2, 40, 64, 32), (64, 128, 1, 9, 96, 80),
                                                (128, 128, 3, 3, 32, 128),
                                                (256, 128, 1, 5, 32, 256)])
def test_wgrad_and_bias_grad(torch, cin, cout, N, H, W, ldx):
    rng = np.random.default_rng(cin * 3 + cout + H)
    x, xr = _bf(torch, rng.standard_normal((N, H, W, ldx)))
    gy, gyr = _bf(torch, rng.standard_normal((N, H, W, cout)))
    need = rdc.load().rdc_nn_wgrad_scratch_floats(N, H, W, cin, cout)
    scratch = torch.empty(int(need), dtype=torch.float32, device="cuda")
    grads, gbs = [], []
    for rep in range(3):
        g = torch.full((9 * cout * cin,), 3.0, dtype=torch.float32, device="cuda")
        gb = torch.full((cout,), 3.0, dtype=torch.float32, device="cuda")
        rdc.nn("conv3x3_wgrad", x.data_ptr(), ldx, gy.data_ptr(), cout, scratch.data_ptr(),
               g.data_ptr(), gb.data_ptr() if rep < 2 else None, N, H, W, cin, cout,
               _stream(torch))
        grads.append(g)
        gbs.append(gb)
    _sync(torch)
    assert torch.equal(grads[0], grads[1]) and torch.equal(grads[0], grads[2])  # deterministic
    assert torch.equal(gbs[0], gbs[1]) and bool((gbs[2] == 3.0).all())
    gb = gbs[0]
    w0 = np.zeros((9, cout, cin))
    _, _, ref, rb = unet_ref.conv_grads(xr[..., :cin], w0, np.zeros(cout), gyr)
    _, _, mag, mb = unet_ref.conv_grads(np.abs(xr[..., :cin]), w0, np.zeros(cout), np.abs(gyr))
    got = grads[0].double().cpu().numpy().reshape(9, cout, cin)
    assert (np.abs(got - ref) <= 2.0 ** -14 * mag + 1e-30).all()
    assert (np.abs(gb.double().cpu().numpy() - rb) <= 2.0 ** -14 * mb).all()


@pytest.mark.parametrize("c,o_pool,o_acc,o_relu", [(48, 16, 8, 4), (48, 4, 12, 8), (44, 16, 8, 8)])
def test_relu_pool_upsample_and_adjoints(torch, c, o_pool, o_acc, o_relu):
    """Channel slices at 16-byte offsets and c % 8 == 0 take the 16-byte
    kernels, the others the scalar ones; both must give the same values."""
    rng = np.random.default_rng(5)
    N, H, W, ld = 2, 6, 64, 64
    s = _stream(torch)
    a, ar = _bf(torch, rng.standard_normal((N, H, W, ld)))
    # pool
    p = torch.zeros((N, H // 2, W // 2, c), dtype=torch.bfloat16, device="cuda")
    rdc.nn("pool2", a.data_ptr() + o_pool * 2, ld, p.data_ptr(), c, N, H // 2, W // 2, c, s)
    ap = ar[..., o_pool:o_pool + c]
    pref = 0.25 * (ap[:, 0::2, 0::2] + ap[:, 0::2, 1::2] + ap[:, 1::2, 0::2] + ap[:, 1::2, 1::2])
    # pool adjoint, accumulating into a channel slice
    g, gr = _bf(torch, rng.standard_normal((N, H // 2, W // 2, c)))
    acc, accr = _bf(torch, rng.standard_normal((N, H, W, ld)))
    rdc.nn("pool2_bwd", g.data_ptr(), c, acc.data_ptr() + o_acc * 2, ld, N, H // 2, W // 2, c, 1, s)
    up_g = np.repeat(np.repeat(gr, 2, axis=1), 2, axis=2)
    accref = accr.copy()
    accref[..., o_acc:o_acc + c] += 0.25 * up_g
    # upsample and its adjoint
    u = torch.zeros((N, H, W, c), dtype=torch.bfloat16, device="cuda")
    rdc.nn("up2", g.data_ptr(), c, u.data_ptr(), c, N, H, W, c, s)
    gu = torch.zeros((N, H // 2, W // 2, c), dtype=torch.bfloat16, device="cuda")
    rdc.nn("up2_bwd", a.data_ptr(), ld, gu.data_ptr(), c, N, H // 2, W // 2, c, s)
    guref = (ar[:, 0::2, 0::2] + ar[:, 0::2, 1::2] + ar[:, 1::2, 0::2] + ar[:, 1::2, 1::2])[..., :c]
    # relu adjoint on a slice
    y, yr = _bf(torch, rng.standard_normal((N, H, W, ld)))
    gg, ggr = _bf(torch, rng.standard_normal((N, H, W, ld)))
    rdc.nn("relu_bwd", gg.data_ptr() + o_relu * 2, ld, y.data_ptr() + o_relu * 2, ld, N * H * W,
           c, s)
    rref = ggr.copy()
    rref[..., o_relu:o_relu + c] = np.where(yr[..., o_relu:o_relu + c] > 0,
                                          ggr[..., o_relu:o_relu + c], 0.0)
    _sync(torch)
    for got, ref in ((p, pref), (acc, accref), (gu, guref)):
        assert (np.abs(_host(got) - ref) <= HALF_ULP * np.abs(ref)).all()
    assert np.array_equal(_host(u), up_g)
    assert np.array_equal(_host(gg), rref)


def _planes(torch, N, H, W, seed):
    """N stepper-layout planes (pitch >= W) of a circuit state."""
    rng = np.random.default_rng(seed)
    pitch = rdc.pitch_for(W)
    u = np.zeros((N, H, pitch), np.float32)
    v = np.zeros_like(u)
    phi = np.zeros_like(u)
    for n in range(N):
        uu, vv, pp = inputs.random_state(W, H, seed=seed + n, umax=0.9, vmax=0.2)
        u[n, :, :W], v[n, :, :W], phi[n, :, :W] = uu, vv, pp
    return pitch, u, v, phi


def test_prep_apply_loss(torch):
    N, H, W = 2, 5, 64
    pitch, u, v, phi = _planes(torch, N, H, W, 11)
    _, ut, vt, _ = _planes(torch, N, H, W, 21)
    s = _stream(torch)
    d = {k: torch.as_tensor(a).cuda() for k, a in dict(u=u, v=v, phi=phi, ut=ut, vt=vt).items()}
    plane = H * pitch
    su, sv, sp, theta, fw = 1.0, 4.0, 5.0, 0.5, 4.0
    x = torch.full((N, H, W, 32), 9.0, dtype=torch.bfloat16, device="cuda")
    rdc.nn("prep", d["u"].data_ptr(), d["v"].data_ptr(), d["phi"].data_ptr(), pitch, plane,
           x.data_ptr(), 32, N, H, W, su, sv, sp, s)
    rng = np.random.default_rng(3)
    head, hr = _bf(torch, 0.3 * rng.standard_normal((N, H, W, 32)))
    uo = torch.zeros_like(d["u"])
    vo = torch.zeros_like(d["v"])
    f, cmax = 1.4, 0.3
    rdc.nn("apply", d["u"].data_ptr(), d["v"].data_ptr(), d["phi"].data_ptr(), head.data_ptr(), 32,
           pitch, plane, uo.data_ptr(), vo.data_ptr(), N, H, W, su, sv, f, cmax, s)
    g = torch.full((N, H, W, 32), 9.0, dtype=torch.bfloat16, device="cuda")
    nb = rdc.load().rdc_nn_loss_blocks(N * H * W)
    part = torch.zeros(nb + 1, dtype=torch.float32, device="cuda")
    rdc.nn("loss", d["u"].data_ptr(), d["v"].data_ptr(), d["ut"].data_ptr(), d["vt"].data_ptr(),
           pitch, plane, head.data_ptr(), 32, g.data_ptr(), 32, N, H, W, su, sv, theta, fw,
           part.data_ptr(), s)
    _sync(torch)
    c = lambda a: a[:, :, :W].astype(np.float64)
    bfv = lambda a: torch.as_tensor(np.float32(a)).to(torch.bfloat16).double().numpy()
    xr = _host(x)
    assert np.array_equal(xr[..., 0], bfv(np.float32(su) * u[:, :, :W]))
    assert np.array_equal(xr[..., 1], bfv(np.float32(sv) * v[:, :, :W]))
    assert np.array_equal(xr[..., 2], bfv(np.float32(sp) * phi[:, :, :W]))
    assert (xr[..., 3:] == 0).all()
    ref_uo = np.clip(c(u) + hr[..., 0] / su, 0.0, 1.0)
    vcap = np.maximum((np.float32(cmax) - phi[:, :, :W]) / np.float32(f), 0).astype(np.float64)
    ref_vo = np.clip(c(v) + hr[..., 1] / sv, 0.0, vcap)
    assert (ref_uo == 0).any() and (ref_uo == 1).any() and (ref_vo == 0).any()
    assert (ref_vo == vcap).any()
    got_uo = uo.double().cpu().numpy()[:, :, :W]
    got_vo = vo.double().cpu().numpy()[:, :, :W]
    assert np.abs(got_uo - ref_uo).max() <= 2e-7 * (1 + np.abs(ref_uo).max())
    assert np.abs(got_vo - ref_vo).max() <= 2e-7 * (1 + np.abs(ref_vo).max())
    ht = torch.as_tensor(hr).requires_grad_(True)
    L = unet_ref.loss(ht, c(u), c(v), c(ut), c(vt), su, sv, theta, fw)
    L.backward()
    L = float(L.detach())
    assert abs(float(part[:nb].double().sum()) - L) <= 1e-5 * L
    assert abs(float(part[nb]) - L) <= 1e-5 * L          # the library's own total
    gref = ht.grad.numpy()
    gg = _host(g)
    assert (np.abs(gg[..., :2] - gref[..., :2]) <= HALF_ULP * np.abs(gref[..., :2]) +
            1e-6 * np.abs(gref).max()).all()
    assert (gg[..., 2:] == 0).all()


def test_adam_step(torch):
    rng = np.random.default_rng(8)
    n = 10007
    p, g, m, v = (rng.standard_normal(n).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    g[:5] = [3.0, -3.0, 0.5, 1.0, -1.0]
    dev = [torch.as_tensor(a.copy()).cuda() for a in (p, g, m, v)]
    lr_t, b1, b2, eps, clip = 1e-3, 0.9, 0.999, 1e-8, 1.0
    rdc.nn("adam", *(t.data_ptr() for t in dev), n, lr_t, b1, b2, eps, clip, _stream(torch))
    _sync(torch)
    gc = np.clip(g.astype(np.float64), -clip, clip)
    m1 = b1 * m + (1 - b1) * gc
    v1 = b2 * v + (1 - b2) * gc * gc
    p1 = p - lr_t * m1 / (np.sqrt(v1) + eps)
    for got, ref in ((dev[0], p1), (dev[2], m1), (dev[3], v1)):
        assert np.abs(got.double().cpu().numpy() - ref).max() <= 1e-6 * (1 + np.abs(ref).max())


def _front_brute(a, b, theta):
    ny, nx = a.shape
    A, B = a >= theta, b >= theta
    bad = 0
    for y in range(ny):
        for x in range(nx):
            if A[y, x] == B[y, x]:
                continue
            sl = (slice(max(0, y - 1), y + 2), slice(max(0, x - 1), x + 2))
            if A[y, x] and not B[sl].any():
                bad += 1
            if B[y, x] and not A[sl].any():
                bad += 1
    return bad


def test_front_check_counts_cells_more_than_one_cell_off(torch):
    rng = np.random.default_rng(4)
    ny, nx = 37, 45
    pitch = rdc.pitch_for(nx)
    a = np.zeros((ny, pitch), np.float32)
    b = np.zeros((ny, pitch), np.float32)
    a[:, :nx] = (rng.random((ny, nx)) < 0.1) * 0.9
    b[:, :nx] = a[:, :nx]
    b[5, 7] = 0.0              # removed: a neighbour in b? none -> counted
    b[20:22, 30:32] = 0.9      # added blob, some cells one away from a's cells
    b[:, nx - 1] = 0.9         # a column on the edge
    ref = _front_brute(a[:, :nx], b[:, :nx], 0.5)
    ad, bd = torch.as_tensor(a).cuda(), torch.as_tensor(b).cuda()
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    rdc.nn("front_check", ad.data_ptr(), bd.data_ptr(), pitch, nx, ny, 0.5, cnt.data_ptr(),
           _stream(torch))
    rdc.nn("front_check", ad.data_ptr(), ad.data_ptr(), pitch, nx, ny, 0.5, cnt.data_ptr() + 4,
           _stream(torch))
    _sync(torch)
    assert ref > 0
    assert cnt.cpu().numpy().tolist() == [ref, 0]


def test_state_check_counts_cells_the_stepper_cannot_continue(torch):
    ny, nx = 19, 70
    pitch = rdc.pitch_for(nx)
    rng = np.random.default_rng(12)
    u = rng.uniform(0, 1, (ny, pitch)).astype(np.float32)
    v = rng.uniform(0, 0.2, (ny, pitch)).astype(np.float32)
    phi = rng.choice([0.054, 0.2], (ny, pitch)).astype(np.float32)
    u[2, 3], u[4, 5], v[6, 7] = np.nan, -0.0021, np.nan
    u[8, 9] = 2.5
    v[10, 11], phi[10, 11] = 0.25, 0.054         # f v + phi = 0.404 > cmax
    u[:, nx:] = np.nan                            # padding is not part of the grid
    f, cmax, ulo, uhi = 1.4, 0.352, -0.002, 2.0
    c = np.float32(f) * v + phi
    ok = (u >= ulo) & (u <= uhi) & (c <= np.float32(cmax))
    ref = int((~ok[:, :nx]).sum())
    d = [torch.as_tensor(t).cuda() for t in (u, v, phi)]
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    rdc.nn("state_check", *(t.data_ptr() for t in d), pitch, nx, ny, ulo, uhi, f, cmax,
           cnt.data_ptr(), _stream(torch))
    _sync(torch)
    assert ref >= 5 and int(cnt.item()) == ref


# ------------------------------------------------------------------ whole network

def _host_x0(u, v, phi, W, su, sv, sp):
    """The network input as the prep kernel defines it, built on the host."""
    import torch
    b = lambda a: torch.as_tensor(np.float32(a)).to(torch.bfloat16).double().numpy()
    N, H = u.shape[:2]
    x = np.zeros((N, H, W, 32))
    x[..., 0] = b(np.float32(su) * u[:, :, :W])
    x[..., 1] = b(np.float32(sv) * v[:, :, :W])
    x[..., 2] = b(np.float32(sp) * phi[:, :, :W])
    return x


def _net(torch, seed=31):
    from paper_1901_06535_amd import surrogate as sg
    net = sg.UNet(seed=seed)
    rng = np.random.default_rng(seed)
    params = {}
    for name, cin, cout, _ in sg.LAYERS:      # nonzero biases: every bias path is exercised
        Wt, _ = net.get(name)
        params[name] = (Wt, (0.05 * rng.standard_normal(cout)).astype(np.float32))
    params["head"] = (params["head"][0] * 50.0, params["head"][1])
    net.set_all(params)
    bfw = {n: (torch.as_tensor(W).to(torch.bfloat16).double().numpy(), b.astype(np.float64))
           for n, (W, b) in params.items()}
    return sg, net, bfw


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_network_forward_and_gradients_match_fp64(torch):
    """Whole U-Net on two 16 x 256 images: forward head, loss and every
    layer's weight and bias gradient against FP64 autograd of the reference
    network (same bf16-rounded weights and input).

    The GPU stores every activation and every activation gradient in bf16,
    so the bar is a relative Frobenius error derived from that arithmetic:
    an FP32 model of this network that rounds each stored tensor to bf16
    lands 0.03-5.4% from FP64 per layer on this very case (the coarse levels
    are worst: their weight gradients sum many cancelling terms).  Each
    layer must be within 15% and the whole parameter gradient within 5%;
    a dropped path (skip, pool adjoint, bias) or a transposed operand costs
    tens of percent."""
    sg, net, bfw = _net(torch)
    N, H, W = 2, 16, 256
    pitch, u, v, phi = _planes(torch, N, H, W, 41)
    _, ut, vt, _ = _planes(torch, N, H, W, 51)
    d = {k: torch.as_tensor(a).cuda() for k, a in dict(u=u, v=v, phi=phi, ut=ut, vt=vt).items()}
    plane = H * pitch
    ws = sg.Workspace(net, N, H, W, train=True)
    net.g.fill_(5.0)                               # every gradient slot is overwritten
    sg.prep(net, ws, d["u"].data_ptr(), d["v"].data_ptr(), d["phi"].data_ptr(), pitch, plane)
    sg.forward(net, ws)
    L = sg.loss_and_grad(net, ws, d["u"].data_ptr(), d["v"].data_ptr(), d["ut"].data_ptr(),
                         d["vt"].data_ptr(), pitch, plane)
    sg.backward(net, ws)
    _sync(torch)
    x0 = _host_x0(u, v, phi, W, sg.SU, sg.SV, sg.SP)
    head, leaves = unet_ref.forward(bfw, x0, requires_grad=True)
    c = lambda a: a[:, :, :W].astype(np.float64)
    Lref = unet_ref.loss(head, c(u), c(v), c(ut), c(vt), sg.SU, sg.SV, sg.THETA, 4.0)
    Lref.backward()
    got_head = _host(ws.a["head"])
    e_head = _rel(got_head[..., :2], head.detach().numpy()[..., :2])
    print("  head rel err %.2e, loss %.6g vs %.6g" % (e_head, L, float(Lref.detach())))
    assert e_head < 2e-2
    assert abs(L - float(Lref.detach())) <= 3e-2 * float(Lref.detach())
    errs, got_all, ref_all = {}, [], []
    for name, cin, cout, _ in sg.LAYERS:
        gw = net.g[net.offsets[name][0]: net.offsets[name][0] + 9 * cout * cin]
        gb = net.g[net.offsets[name][1]: net.offsets[name][1] + cout]
        w_ref = leaves[name][0].grad.permute(2, 3, 0, 1).reshape(9, cout, cin).numpy()
        b_ref = leaves[name][1].grad.numpy()
        gw = gw.double().cpu().numpy().reshape(9, cout, cin)
        gb = gb.double().cpu().numpy()
        errs[name] = (_rel(gw, w_ref), _rel(gb, b_ref))
        got_all += [gw.ravel(), gb]
        ref_all += [w_ref.ravel(), b_ref]
    total = _rel(np.concatenate(got_all), np.concatenate(ref_all))
    print("  gradient rel err per layer (w, b): " +
          ", ".join("%s %.3f/%.3f" % (n, a, b) for n, (a, b) in errs.items()))
    print("  whole gradient rel err %.3e" % total)
    assert all(a < 0.15 and b < 0.15 for a, b in errs.values())
    assert total < 5e-2


def test_network_is_translation_equivariant_in_x(torch):
    """Shifting the input by 8 pixels along x (the coarsest level's pooling
    stride) shifts the head by the same amount away from the edges: a wrong
    tap offset or a seam between 32-pixel row segments breaks it."""
    sg, net, _ = _net(torch, seed=5)
    N, H, W = 1, 16, 256
    pitch, u, v, phi = _planes(torch, N, H, W, 61)
    us, vs, ps = (np.roll(a, 8, axis=2) for a in (u, v, phi))
    heads = []
    for uu, vv, pp in ((u, v, phi), (us, vs, ps)):
        ws = sg.Workspace(net, N, H, W, train=False)
        dd = [torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in (uu, vv, pp)]
        sg.prep(net, ws, *(t.data_ptr() for t in dd), pitch, H * pitch)
        sg.forward(net, ws)
        _sync(torch)
        heads.append(_host(ws.a["head"]))
    # the receptive field of the 4-level net is < 60 pixels: compare the middle.
    # Each output's reduction order does not depend on its position, so the
    # shifted result is bit-identical there.
    a = heads[0][:, :, 72:176]
    b = heads[1][:, :, 80:184]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("cin,up_c,cout,N,H,W", [(96, 64, 32, 2, 6, 64), (192, 128, 64, 1, 4, 128),
                                                 (256, 128, 128, 1, 4, 64), (64, 64, 32, 1, 2, 64)])
def test_conv_with_upsampled_prefix_equals_up2_then_conv(torch, cin, up_c, cout, N, H, W):
    """Reading the upsampled channels from the coarse level inside the
    convolution's loads gives the same bits as writing them with up2 first."""
    rng = np.random.default_rng(cin + up_c + cout)
    ldx = cin
    x, _ = _bf(torch, rng.standard_normal((N, H, W, ldx)))
    low, _ = _bf(torch, rng.standard_normal((N, H // 2, W // 2, up_c)))
    w, _ = _bf(torch, rng.standard_normal((9, cout, cin)) / np.sqrt(9 * cin))
    b = torch.as_tensor(rng.standard_normal(cout).astype(np.float32)).cuda()
    s = _stream(torch)
    y_fused = torch.full((N, H, W, cout), 7.0, dtype=torch.bfloat16, device="cuda")
    rdc.nn("conv3x3_up", x.data_ptr(), ldx, low.data_ptr(), up_c, up_c, w.data_ptr(),
           b.data_ptr(), y_fused.data_ptr(), cout, N, H, W, cin, cout, cout, s)
    xc = x.clone()
    rdc.nn("up2", low.data_ptr(), up_c, xc.data_ptr(), ldx, N, H, W, up_c, s)
    y_ref = torch.full((N, H, W, cout), 7.0, dtype=torch.bfloat16, device="cuda")
    rdc.nn("conv3x3", xc.data_ptr(), ldx, w.data_ptr(), b.data_ptr(), y_ref.data_ptr(), cout,
           N, H, W, cin, cout, cout, 1, s)
    _sync(torch)
    assert torch.equal(y_fused, y_ref)
    assert (y_ref.float() > 0).any()
    with pytest.raises(rdc.RdcError):                # odd height cannot be upsampled
        rdc.nn("conv3x3_up", x.data_ptr(), ldx, low.data_ptr(), up_c, up_c, w.data_ptr(),
               b.data_ptr(), y_fused.data_ptr(), cout, N, H - 1, W, cin, cout, cout, s)


def test_conv_from_planes_equals_prep_then_conv(torch):
    """Building the first layer's input from the stepper planes inside the
    convolution's loads gives the same bits as prep followed by conv3x3."""
    from paper_1901_06535_amd import surrogate as sg
    N, H, W, cout = 2, 5, 96, 32
    pitch, u, v, phi = _planes(torch, N, H, W, 71)
    d = [torch.as_tensor(a).cuda() for a in (u, v, phi)]
    plane = H * pitch
    rng = np.random.default_rng(3)
    w, _ = _bf(torch, rng.standard_normal((9, cout, sg.IN_C)) / np.sqrt(9 * 3))
    b = torch.as_tensor(rng.standard_normal(cout).astype(np.float32)).cuda()
    s = _stream(torch)
    y_fused = torch.full((N, H, W, cout), 7.0, dtype=torch.bfloat16, device="cuda")
    rdc.nn("conv3x3_planes", *(t.data_ptr() for t in d), pitch, plane, sg.SU, sg.SV, sg.SP,
           w.data_ptr(), b.data_ptr(), y_fused.data_ptr(), cout, N, H, W, sg.IN_C, cout, cout, s)
    x0 = torch.empty((N, H, W, sg.IN_C), dtype=torch.bfloat16, device="cuda")
    rdc.nn("prep", *(t.data_ptr() for t in d), pitch, plane, x0.data_ptr(), sg.IN_C, N, H, W,
           sg.SU, sg.SV, sg.SP, s)
    y_ref = torch.full((N, H, W, cout), 7.0, dtype=torch.bfloat16, device="cuda")
    rdc.nn("conv3x3", x0.data_ptr(), sg.IN_C, w.data_ptr(), b.data_ptr(), y_ref.data_ptr(), cout,
           N, H, W, sg.IN_C, cout, cout, 1, s)
    _sync(torch)
    assert torch.equal(y_fused, y_ref)


def test_inference_forward_equals_prep_and_forward(torch):
    """The coarse stepper's inference forward (first layer from the planes,
    decoders reading the coarse level) leaves the same head, bit for bit, as
    prep + the training forward."""
    sg, net, _ = _net(torch, seed=9)
    N, H, W = 2, 16, 256
    pitch, u, v, phi = _planes(torch, N, H, W, 81)
    d = [torch.as_tensor(a).cuda() for a in (u, v, phi)]
    plane = H * pitch
    ws1 = sg.Workspace(net, N, H, W, train=False)
    sg.prep(net, ws1, *(t.data_ptr() for t in d), pitch, plane)
    sg.forward(net, ws1)
    ws2 = sg.Workspace(net, N, H, W, train=False)
    sg.forward_planes(net, ws2, *(t.data_ptr() for t in d), pitch, plane)
    _sync(torch)
    assert torch.equal(ws1.a["head"], ws2.a["head"])
    assert ws1.a["head"].float().abs().max() > 0


def test_head_with_prediction_equals_head_then_apply(torch):
    """The head launch that applies the prediction itself writes the same
    (u, v) planes, bit for bit, as the head into a tensor followed by apply;
    in place, as the coarse stepper runs it."""
    sg, net, _ = _net(torch, seed=13)
    N, H, W = 2, 16, 256
    pitch, u, v, phi = _planes(torch, N, H, W, 91)
    plane = H * pitch
    params = inputs.PARAMS_WORKLOAD
    d = [torch.as_tensor(a).cuda() for a in (u, v, phi)]
    ws1 = sg.Workspace(net, N, H, W, train=False)
    sg.forward_planes(net, ws1, *(t.data_ptr() for t in d), pitch, plane)
    uo = torch.full_like(d[0], -7.0)
    vo = torch.full_like(d[1], -7.0)
    sg.apply(net, ws1, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), uo.data_ptr(),
             vo.data_ptr(), pitch, plane, params)
    ws2 = sg.Workspace(net, N, H, W, train=False)
    u2, v2 = d[0].clone(), d[1].clone()
    sg.forward_planes(net, ws2, u2.data_ptr(), v2.data_ptr(), d[2].data_ptr(), pitch, plane,
                      predict=(u2.data_ptr(), v2.data_ptr(), params))
    _sync(torch)
    c = lambda t: t[:, :, :W]
    assert torch.equal(c(u2), c(uo)) and torch.equal(c(v2), c(vo))
    assert not torch.equal(c(u2), c(d[0]))           # the prediction moved the state
    assert torch.equal(u2[:, :, W:], d[0][:, :, W:])  # padding columns untouched


def test_inference_step_at_full_size_equals_unfused_route(torch):
    """At the coarse stepper's full size (one 2048^2 grid), the inference step
    (planes input, upsampled prefixes, prediction in the head's epilogue)
    gives the same (u, v), bit for bit, as prep + forward + apply."""
    sg, net, _ = _net(torch, seed=17)
    N, H, W = 1, 2048, 2048
    wl = inputs.circuit(n=2048, seed=1005, steps=100, ndisks=8)
    pitch = rdc.pitch_for(W)
    planes = []
    for a in (wl.u0, wl.v0, wl.phi):
        t = torch.zeros((H, pitch), dtype=torch.float32, device="cuda")
        t[:, :W] = torch.as_tensor(a).cuda()
        planes.append(t)
    u, v, phi = planes
    for s in wl.stimuli:                              # excite the disks so the head is non-trivial
        yy, xx = torch.meshgrid(torch.arange(H, device="cuda"), torch.arange(W, device="cuda"),
                                indexing="ij")
        u[:, :W][(yy - s.cy) ** 2 + (xx - s.cx) ** 2 <= s.r ** 2] = 1.0
    plane = H * pitch
    params = wl.params
    ws = sg.Workspace(net, N, H, W, train=False)
    sg.prep(net, ws, u.data_ptr(), v.data_ptr(), phi.data_ptr(), pitch, plane)
    sg.forward(net, ws)
    uo, vo = torch.empty_like(u), torch.empty_like(v)
    sg.apply(net, ws, u.data_ptr(), v.data_ptr(), phi.data_ptr(), uo.data_ptr(), vo.data_ptr(),
             pitch, plane, params)
    u2, v2 = u.clone(), v.clone()
    sg.forward_planes(net, ws, u2.data_ptr(), v2.data_ptr(), phi.data_ptr(), pitch, plane,
                      predict=(u2.data_ptr(), v2.data_ptr(), params))
    _sync(torch)
    assert torch.equal(u2[:, :W], uo[:, :W]) and torch.equal(v2[:, :W], vo[:, :W])
    assert not torch.equal(u2[:, :W], u[:, :W])
