"""The C-ABI library loads and exports every symbol include/rdc.h declares,
and argument checks that run before any device call behave as documented.
No compute call is made (these run on machines without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1901_06535_amd import rdc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rdc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rdc.LIB_PATH):
        from paper_1901_06535_amd import build
        build.build()
    return rdc.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rdc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert set(_declared()) == set(rdc.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_status_strings(lib):
    assert rdc.load().rdc_status_string(0) == b"RDC_OK"
    assert rdc.load().rdc_status_string(-4) == b"RDC_E_NONFINITE"


def _bufs(pitch=64, base=0x10000000):
    b = rdc.rdc_buffers()
    b.u[0], b.u[1] = base, base + 0x100000
    b.v[0], b.v[1] = base + 0x200000, base + 0x300000
    b.phi = base + 0x400000
    b.pitch = pitch
    return b


@pytest.mark.parametrize("nx,ny,pitch,dtype,why", [
    (0, 4, 64, 0, "nx and ny"), (4, 0, 64, 0, "nx and ny"), (65, 4, 64, 0, "pitch"),
    (4, 4, 96, 0, "pitch"), (4, 4, 1 << 29, 0, "row too long"),
    (4, 4, 1 << 28, 1, "row too long"), (4, 1048561, 64, 0, "row limit")])
def test_create_rejects_bad_shape_before_touching_the_device(lib, nx, ny, pitch, dtype, why):
    out = ctypes.c_void_p()
    s = lib.rdc_create(nx, ny, dtype, ctypes.byref(_bufs(pitch)), None, ctypes.byref(out))
    assert s == rdc.RDC_E_INVAL and out.value is None
    assert why in rdc.rdc_last_error(None)


def test_create_rejects_misaligned_or_aliased_buffers(lib):
    out = ctypes.c_void_p()
    b = _bufs()
    b.phi = b.phi + 4
    assert lib.rdc_create(8, 8, 0, ctypes.byref(b), None, ctypes.byref(out)) == rdc.RDC_E_INVAL
    assert "aligned" in rdc.rdc_last_error(None)
    b = _bufs()
    b.v[1] = b.v[0]
    assert lib.rdc_create(8, 8, 0, ctypes.byref(b), None, ctypes.byref(out)) == rdc.RDC_E_INVAL
    assert "distinct" in rdc.rdc_last_error(None)
    b = _bufs()
    b.u[1] = None
    assert lib.rdc_create(8, 8, 0, ctypes.byref(b), None, ctypes.byref(out)) == rdc.RDC_E_INVAL
    assert lib.rdc_create(8, 8, 7, ctypes.byref(_bufs()), None, ctypes.byref(out)) == rdc.RDC_E_INVAL
    assert lib.rdc_create(8, 8, 0, None, None, ctypes.byref(out)) == rdc.RDC_E_INVAL
    assert lib.rdc_create(8, 8, 0, ctypes.byref(_bufs()), None, None) == rdc.RDC_E_INVAL


def test_null_context_is_rejected(lib):
    assert lib.rdc_step(None, 1) == rdc.RDC_E_INVAL
    assert lib.rdc_set_block(None, 4) == rdc.RDC_E_INVAL
    assert lib.rdc_read(None, None, None, 0, 0) == rdc.RDC_E_INVAL
    assert lib.rdc_destroy(None) == rdc.RDC_OK


def test_copy_argument_checks(lib):
    assert lib.rdc_copy(None, None, 16, None) == rdc.RDC_E_INVAL
    assert lib.rdc_copy(0x1000, 0x2000, 17, None) == rdc.RDC_E_INVAL
    assert lib.rdc_copy(0x1004, 0x2000, 16, None) == rdc.RDC_E_INVAL


def test_tile_rows_supported(lib):
    assert rdc.rdc_tile_rows_supported(80)
    assert not rdc.rdc_tile_rows_supported(81)


def _descs(lib, sims):
    arr = (rdc.rdc_sim_desc * len(sims))()
    for i, (nx, ny, pitch, off) in enumerate(sims):
        arr[i].nx, arr[i].ny, arr[i].pitch, arr[i].offset = nx, ny, pitch, off
        arr[i].params = rdc.rdc_params(0.022, 1.4, 0.002, 1.0, 0.001, 0.25)
    return arr


@pytest.mark.parametrize("sims,pool,why", [
    ([(10, 10, 64, 0), (10, 10, 64, 320)], 4096, "overlap"),
    ([(10, 10, 64, 0)], 100, "past the pool"),
    ([(10, 10, 60, 0)], 4096, "multiples of 64"),
    ([(10, 10, 64, 32)], 4096, "multiples of 64"),
    ([(0, 10, 64, 0)], 4096, "sizes")])
def test_batch_create_rejects_bad_layouts(lib, sims, pool, why):
    out = ctypes.c_void_p()
    d = _descs(lib, sims)
    s = lib.rdc_batch_create(len(sims), d, ctypes.byref(_bufs()), pool, None, ctypes.byref(out))
    assert s == rdc.RDC_E_INVAL and out.value is None
    assert why in lib.rdc_batch_last_error(None).decode()


def test_batch_create_rejects_bad_params(lib):
    out = ctypes.c_void_p()
    d = _descs(lib, [(10, 10, 64, 0)])
    d[0].params.dt = 0.1      # dt*D_u/dx^2 = 1.6 > 1/4
    s = lib.rdc_batch_create(1, d, ctypes.byref(_bufs()), 4096, None, ctypes.byref(out))
    assert s == rdc.RDC_E_INVAL
    assert "1/4" in lib.rdc_batch_last_error(None).decode()


def test_timelapse_argument_checks(lib):
    assert lib.rdc_set_timelapse(None, None, 0, 1) == rdc.RDC_E_INVAL


def _nn_err(lib):
    return lib.rdc_nn_last_error().decode()


FAKE = 0x10000000      # 256-byte aligned, never dereferenced: the checks reject first


@pytest.mark.parametrize("args,why", [
    # x, ldx, w, bias, y, ldy, n, h, w, cin, cout, cout_store, relu
    ((None, 32, FAKE, None, FAKE, 32, 1, 4, 64, 32, 32, 32, 1), "NULL"),
    ((FAKE, 32, FAKE, None, FAKE, 32, 1, 4, 48, 32, 32, 32, 1), "multiple of 32"),
    ((FAKE, 32, FAKE, None, FAKE, 32, 1, 4, 64, 24, 32, 32, 1), "cin % 16"),
    ((FAKE, 32, FAKE, None, FAKE, 32, 1, 4, 64, 32, 48, 32, 1), "cout in"),
    ((FAKE, 32, FAKE, None, FAKE, 32, 1, 4, 64, 32, 32, 33, 1), "cout_store"),
    ((FAKE, 36, FAKE, None, FAKE, 32, 1, 4, 64, 32, 32, 32, 1), "strides"),
    ((FAKE + 8, 32, FAKE, None, FAKE, 32, 1, 4, 64, 32, 32, 32, 1), "alignment")])
def test_conv_argument_checks_run_before_any_launch(lib, args, why):
    assert lib.rdc_nn_conv3x3(*args, None) == rdc.RDC_E_INVAL
    assert why in _nn_err(lib)


def test_nn_argument_checks(lib):
    # weight gradient: channel counts must be multiples of 32
    assert lib.rdc_nn_conv3x3_wgrad(FAKE, 32, FAKE, 32, FAKE, FAKE, None, 1, 4, 64, 16, 32,
                                    None) == rdc.RDC_E_INVAL
    assert "% 32" in _nn_err(lib)
    # the variant that allocates nothing: the same checks, and shapes whose
    # workspace exceeds its static scratch are refused before any device call
    assert lib.rdc_nn_conv3x3_wgrad_noalloc(FAKE, 32, FAKE, 32, FAKE, None, 1, 4, 64, 16, 32,
                                            None) == rdc.RDC_E_INVAL
    assert "% 32" in _nn_err(lib)
    cap = lib.rdc_nn_wgrad_static_floats()
    assert cap == 8 << 20
    assert lib.rdc_nn_wgrad_scratch_floats(16, 512, 512, 32, 32) > cap
    assert lib.rdc_nn_conv3x3_wgrad_noalloc(FAKE, 32, FAKE, 32, FAKE, FAKE, 16, 512, 512, 32, 32,
                                            None) == rdc.RDC_E_INVAL
    assert "static scratch" in _nn_err(lib)
    # scratch size is zero for shapes the kernel rejects
    assert lib.rdc_nn_wgrad_scratch_floats(1, 4, 16, 32, 32) == 0
    assert lib.rdc_nn_wgrad_scratch_floats(1, 4, 64, 32, 32) > 0
    assert lib.rdc_nn_loss_blocks(0) == 0 and lib.rdc_nn_loss_blocks(1000) >= 1
    # apply needs phi and a positive f (the Euler bound divides by it)
    assert lib.rdc_nn_apply(FAKE, FAKE, None, FAKE, 32, 64, 4096, FAKE, FAKE, 1, 4, 64, 1.0, 4.0,
                            1.4, 0.3, None) == rdc.RDC_E_INVAL
    assert lib.rdc_nn_apply(FAKE, FAKE, FAKE, FAKE, 32, 64, 4096, FAKE, FAKE, 1, 4, 64, 1.0, 4.0,
                            0.0, 0.3, None) == rdc.RDC_E_INVAL
    # front and state checks: sizes and ranges
    assert lib.rdc_nn_front_check(FAKE, FAKE, 10, 64, 4, 0.5, FAKE, None) == rdc.RDC_E_INVAL
    assert lib.rdc_nn_state_check(FAKE, FAKE, FAKE, 64, 64, 4, 1.0, -1.0, 1.4, 0.3, FAKE,
                                  None) == rdc.RDC_E_INVAL
    assert lib.rdc_nn_adam(None, FAKE, FAKE, FAKE, 10, 1e-3, 0.9, 0.999, 1e-8, 1.0,
                           None) == rdc.RDC_E_INVAL
    # fused-input convolutions: upsampling needs an even height and a whole
    # 32-channel prefix; both need a bias and cout in {32, 64, 128}
    up = lambda h, up_c, cout, bias=FAKE: lib.rdc_nn_conv3x3_up(
        FAKE, 96, FAKE, 64, up_c, FAKE, bias, FAKE, cout, 1, h, 64, 96, cout, cout, None)
    assert up(5, 64, 32) == rdc.RDC_E_INVAL and "even" in _nn_err(lib)
    assert up(4, 48, 32) == rdc.RDC_E_INVAL
    assert up(4, 128, 32) == rdc.RDC_E_INVAL         # prefix longer than cin
    assert up(4, 64, 96) == rdc.RDC_E_INVAL
    assert up(4, 64, 32, bias=None) == rdc.RDC_E_INVAL
    planes = lambda pitch, stride, cout: lib.rdc_nn_conv3x3_planes(
        FAKE, FAKE, FAKE, pitch, stride, 1.0, 4.0, 5.0, FAKE, FAKE, FAKE, cout, 1, 4, 64, 32,
        cout, cout, None)
    assert planes(32, 4096, 32) == rdc.RDC_E_INVAL    # pitch < w
    assert planes(64, 100, 32) == rdc.RDC_E_INVAL     # images overlap
    assert planes(64, 256, 256) == rdc.RDC_E_INVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with a message (and
    without touching a GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)
