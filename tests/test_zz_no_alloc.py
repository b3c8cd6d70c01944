"""The weight-gradient entry point that allocates nothing
(rdc_nn_conv3x3_wgrad_noalloc, partials in the library's static device
scratch) against rdc_nn_conv3x3_wgrad with a caller-owned workspace, through
the C ABI: the same kernels in the same order, so the weight and bias
gradients must be bit-identical -- on two calls in a row, the second on a
smaller input (the scratch keeps the first call's partials), and once more
without the bias gradient."""
import numpy as np
import pytest

from paper_1901_06535_amd import rdc

pytestmark = pytest.mark.gpu


def _bf16(torch, shape, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(shape, generator=g).to(torch.bfloat16).cuda()


def _grads(torch, lib, n, h, w, cin, cout, seed, noalloc, with_bias=True):
    x = _bf16(torch, (n * h * w, cin), seed)
    dy = _bf16(torch, (n * h * w, cout), seed + 1)
    grad = torch.full((9, cout, cin), float("nan"), dtype=torch.float32, device="cuda")
    gb = torch.full((cout,), float("nan"), dtype=torch.float32, device="cuda") if with_bias else None
    stream = torch.cuda.current_stream().cuda_stream
    gbp = gb.data_ptr() if with_bias else None
    if noalloc:
        st = lib.rdc_nn_conv3x3_wgrad_noalloc(x.data_ptr(), cin, dy.data_ptr(), cout,
                                              grad.data_ptr(), gbp, n, h, w, cin, cout, stream)
    else:
        work = torch.empty(lib.rdc_nn_wgrad_scratch_floats(n, h, w, cin, cout),
                           dtype=torch.float32, device="cuda")
        st = lib.rdc_nn_conv3x3_wgrad(x.data_ptr(), cin, dy.data_ptr(), cout, work.data_ptr(),
                                      grad.data_ptr(), gbp, n, h, w, cin, cout, stream)
    assert st == rdc.RDC_OK, lib.rdc_nn_last_error()
    torch.cuda.synchronize()
    return grad.cpu(), (gb.cpu() if with_bias else None)


def test_noalloc_weight_gradient_equals_the_workspace_entry_point():
    import torch
    lib = rdc.load()
    cases = [(2, 64, 96, 64, 32, 11, True),      # first call: larger input
             (1, 16, 32, 32, 32, 21, True),      # second call: smaller input
             (1, 24, 64, 32, 64, 31, False)]     # no bias gradient
    for n, h, w, cin, cout, seed, bias in cases:
        print("[case] wgrad noalloc n=%d h=%d w=%d cin=%d cout=%d bias=%s"
              % (n, h, w, cin, cout, bias), flush=True)
        assert lib.rdc_nn_wgrad_scratch_floats(n, h, w, cin, cout) <= \
            lib.rdc_nn_wgrad_static_floats()
        ref_g, ref_b = _grads(torch, lib, n, h, w, cin, cout, seed, noalloc=False, with_bias=bias)
        got_g, got_b = _grads(torch, lib, n, h, w, cin, cout, seed, noalloc=True, with_bias=bias)
        assert torch.isfinite(ref_g).all()
        assert torch.equal(got_g, ref_g)
        if bias:
            assert torch.isfinite(ref_b).all() and torch.equal(got_b, ref_b)
    # a shape past the static scratch is refused with a message, nothing launched
    big = (16, 512, 512, 32, 32)
    assert lib.rdc_nn_wgrad_scratch_floats(*big) > lib.rdc_nn_wgrad_static_floats()
    x = torch.zeros(64, dtype=torch.bfloat16, device="cuda")
    g = torch.zeros(64, dtype=torch.float32, device="cuda")
    st = lib.rdc_nn_conv3x3_wgrad_noalloc(x.data_ptr(), 32, x.data_ptr(), 32, g.data_ptr(), None,
                                          *big, torch.cuda.current_stream().cuda_stream)
    assert st == rdc.RDC_E_INVAL and b"static scratch" in lib.rdc_nn_last_error()
