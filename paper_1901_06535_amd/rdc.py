"""Python binding of ``librdc.so`` (the C ABI of ``include/rdc.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The functions ``rdc_*`` mirror the C calls one to one and take
raw addresses; :class:`Sim` wraps them for torch-owned device planes (PyTorch
provides device memory and the stream, nothing else).

The library is loaded on first use.  If it has not been built, or no GPU is
present, calls raise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librdc.so")

RDC_OK, RDC_E_INVAL, RDC_E_NOMEM, RDC_E_DEVICE, RDC_E_NONFINITE, RDC_E_STATE = 0, -1, -2, -3, -4, -5
RDC_FP32, RDC_FP64 = 0, 1
RDC_HOST, RDC_DEVICE = 0, 1
NEVER = 0x7FFFFFFF
# rdc_set_tile_rows value for the row-pipeline kernel (register-resident
# strips instead of LDS tiles)
RDC_TILE_STREAM = 1
# default cell limit of the batches' whole-grid LDS path (rdc_batch_set_resident)
RDC_BATCH_RESIDENT_DEFAULT = 16384

# Every symbol include/rdc.h declares.
EXPORTS = ("rdc_create", "rdc_destroy", "rdc_set_params", "rdc_set_phi", "rdc_write",
           "rdc_stimulate", "rdc_step", "rdc_read", "rdc_set_block", "rdc_set_tile_rows",
           "rdc_tile_rows_supported", "rdc_current", "rdc_set_arrival", "rdc_set_timelapse",
           "rdc_get_step", "rdc_set_step", "rdc_last_error", "rdc_copy", "rdc_status_string",
           "rdc_batch_create", "rdc_batch_destroy", "rdc_batch_set_block", "rdc_batch_set_phi",
           "rdc_batch_write", "rdc_batch_stimulate", "rdc_batch_step", "rdc_batch_read",
           "rdc_batch_capture", "rdc_graph_launch", "rdc_graph_destroy", "rdc_batch_last_error",
           "rdc_batch_current", "rdc_batch_set_resident", "rdc_batch_resident_count",
           "rdc_nn_conv3x3", "rdc_nn_conv3x3_up", "rdc_nn_conv3x3_planes",
           "rdc_nn_conv3x3_apply",
           "rdc_nn_dgrad_weights", "rdc_nn_wgrad_scratch_floats",
           "rdc_nn_conv3x3_wgrad", "rdc_nn_conv3x3_wgrad_noalloc", "rdc_nn_wgrad_static_floats",
           "rdc_nn_to_bf16", "rdc_nn_relu_bwd",
           "rdc_nn_pool2", "rdc_nn_pool2_bwd", "rdc_nn_up2", "rdc_nn_up2_bwd", "rdc_nn_prep",
           "rdc_nn_apply", "rdc_nn_loss_blocks", "rdc_nn_loss", "rdc_nn_adam",
           "rdc_nn_front_check", "rdc_nn_state_check", "rdc_nn_last_error")


class rdc_params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("eps", "f", "q", "D_u", "dt", "dx")]


class rdc_buffers(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p * 2), ("v", ctypes.c_void_p * 2),
                ("phi", ctypes.c_void_p), ("pitch", ctypes.c_int64)]


class rdc_sim_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("offset", ctypes.c_int64), ("params", rdc_params)]


class RdcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librdc.so (once).  Raises if it is missing: build it with
    ``python -m paper_1901_06535_amd.build``."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("librdc.so not built (%s); run python -m paper_1901_06535_amd.build"
                           % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "rdc_create": (i32, [i32, i32, i32, ctypes.POINTER(rdc_buffers), vp,
                             ctypes.POINTER(vp)]),
        "rdc_destroy": (i32, [vp]),
        "rdc_set_params": (i32, [vp, ctypes.POINTER(rdc_params)]),
        "rdc_set_phi": (i32, [vp, vp, i64, i32]),
        "rdc_write": (i32, [vp, vp, vp, i64, i32]),
        "rdc_stimulate": (i32, [vp, i32p, i32p, i32p, i32]),
        "rdc_step": (i32, [vp, i64]),
        "rdc_read": (i32, [vp, vp, vp, i64, i32]),
        "rdc_set_block": (i32, [vp, i32]),
        "rdc_set_tile_rows": (i32, [vp, i32]),
        "rdc_tile_rows_supported": (i32, [i32]),
        "rdc_current": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "rdc_set_arrival": (i32, [vp, vp, i64, ctypes.c_double]),
        "rdc_set_timelapse": (i32, [vp, vp, i64, i32]),
        "rdc_get_step": (i32, [vp, ctypes.POINTER(i64)]),
        "rdc_set_step": (i32, [vp, i64]),
        "rdc_last_error": (ctypes.c_char_p, [vp]),
        "rdc_copy": (i32, [vp, vp, i64, vp]),
        "rdc_status_string": (ctypes.c_char_p, [i32]),
        "rdc_batch_create": (i32, [i32, ctypes.POINTER(rdc_sim_desc), ctypes.POINTER(rdc_buffers),
                                   i64, vp, ctypes.POINTER(vp)]),
        "rdc_batch_destroy": (i32, [vp]),
        "rdc_batch_set_block": (i32, [vp, i32, i32]),
        "rdc_batch_set_resident": (i32, [vp, i32]),
        "rdc_batch_resident_count": (i32, [vp]),
        "rdc_batch_set_phi": (i32, [vp, i32, vp, i64, i32]),
        "rdc_batch_write": (i32, [vp, i32, vp, vp, i64, i32]),
        "rdc_batch_stimulate": (i32, [vp, i32p, i32p, i32p, i32p, i32]),
        "rdc_batch_step": (i32, [vp, i64]),
        "rdc_batch_read": (i32, [vp, i32, vp, vp, i64, i32]),
        "rdc_batch_capture": (i32, [vp, i64, ctypes.POINTER(vp)]),
        "rdc_graph_launch": (i32, [vp]),
        "rdc_graph_destroy": (i32, [vp]),
        "rdc_batch_last_error": (ctypes.c_char_p, [vp]),
        "rdc_batch_current": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "rdc_nn_conv3x3": (i32, [vp, i32, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, vp]),
        "rdc_nn_conv3x3_up": (i32, [vp, i32, vp, i32, i32, vp, vp, vp, i32, i32, i32, i32, i32,
                                    i32, i32, vp]),
        "rdc_nn_conv3x3_planes": (i32, [vp, vp, vp, i64, i64, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, vp, vp, vp, i32, i32, i32, i32, i32, i32,
                                        i32, vp]),
        "rdc_nn_conv3x3_apply": (i32, [vp, i32, vp, vp, vp, vp, vp, i64, i64, vp, vp, i32, i32,
                                       i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, vp]),
        "rdc_nn_dgrad_weights": (i32, [vp, vp, i32, i32, vp]),
        "rdc_nn_wgrad_scratch_floats": (i64, [i32, i32, i32, i32, i32]),
        "rdc_nn_conv3x3_wgrad": (i32, [vp, i32, vp, i32, vp, vp, vp, i32, i32, i32, i32, i32, vp]),
        "rdc_nn_conv3x3_wgrad_noalloc": (i32, [vp, i32, vp, i32, vp, vp, i32, i32, i32, i32, i32,
                                               vp]),
        "rdc_nn_wgrad_static_floats": (i64, []),
        "rdc_nn_to_bf16": (i32, [vp, vp, i64, vp]),
        "rdc_nn_relu_bwd": (i32, [vp, i32, vp, i32, i64, i32, vp]),
        "rdc_nn_pool2": (i32, [vp, i32, vp, i32, i32, i32, i32, i32, vp]),
        "rdc_nn_pool2_bwd": (i32, [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp]),
        "rdc_nn_up2": (i32, [vp, i32, vp, i32, i32, i32, i32, i32, vp]),
        "rdc_nn_up2_bwd": (i32, [vp, i32, vp, i32, i32, i32, i32, i32, vp]),
        "rdc_nn_prep": (i32, [vp, vp, vp, i64, i64, vp, i32, i32, i32, i32, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, vp]),
        "rdc_nn_apply": (i32, [vp, vp, vp, vp, i32, i64, i64, vp, vp, i32, i32, i32, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]),
        "rdc_nn_loss_blocks": (i32, [i64]),
        "rdc_nn_loss": (i32, [vp, vp, vp, vp, i64, i64, vp, i32, vp, i32, i32, i32, i32,
                              ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp,
                              vp]),
        "rdc_nn_adam": (i32, [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, vp]),
        "rdc_nn_front_check": (i32, [vp, vp, i64, i32, i32, ctypes.c_float, vp, vp]),
        "rdc_nn_state_check": (i32, [vp, vp, vp, i64, i32, i32, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, vp, vp]),
        "rdc_nn_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _status_name(s: int) -> str:
    return {0: "RDC_OK", -1: "RDC_E_INVAL", -2: "RDC_E_NOMEM", -3: "RDC_E_DEVICE",
            -4: "RDC_E_NONFINITE", -5: "RDC_E_STATE"}.get(s, "RDC_E_%d" % s)


def _check(status: int, ctx) -> None:
    if status != RDC_OK:
        msg = load().rdc_last_error(ctx)
        raise RdcError(status, msg.decode() if msg else "")


# ----------------------------------------------------------------- raw calls

def rdc_create(nx: int, ny: int, dtype: int, bufs: rdc_buffers, stream: int) -> int:
    out = ctypes.c_void_p()
    _check(load().rdc_create(nx, ny, dtype, ctypes.byref(bufs), stream or None,
                             ctypes.byref(out)), None)
    return out.value


def rdc_destroy(ctx) -> None:
    _check(load().rdc_destroy(ctx), None)


def rdc_set_params(ctx, p: rdc_params) -> None:
    _check(load().rdc_set_params(ctx, ctypes.byref(p)), ctx)


def rdc_set_phi(ctx, ptr: int, pitch: int, where: int) -> None:
    _check(load().rdc_set_phi(ctx, ptr, pitch, where), ctx)


def rdc_write(ctx, u_ptr: int, v_ptr: int, pitch: int, where: int) -> None:
    _check(load().rdc_write(ctx, u_ptr, v_ptr, pitch, where), ctx)


def rdc_stimulate(ctx, cx: Sequence[int], cy: Sequence[int], r: Sequence[int]) -> None:
    k = len(cx)
    arr = [np.ascontiguousarray(a, dtype=np.int32) for a in (cx, cy, r)]
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for a in arr]
    _check(load().rdc_stimulate(ctx, ptrs[0], ptrs[1], ptrs[2], k), ctx)


def rdc_step(ctx, n: int) -> None:
    _check(load().rdc_step(ctx, int(n)), ctx)


def rdc_read(ctx, u_ptr, v_ptr, pitch: int, where: int) -> int:
    """Returns the status (RDC_OK or RDC_E_NONFINITE); raises on other errors."""
    s = load().rdc_read(ctx, u_ptr, v_ptr, pitch, where)
    if s not in (RDC_OK, RDC_E_NONFINITE):
        _check(s, ctx)
    return s


def rdc_set_block(ctx, T: int) -> None:
    _check(load().rdc_set_block(ctx, T), ctx)


def rdc_set_tile_rows(ctx, rows: int) -> None:
    _check(load().rdc_set_tile_rows(ctx, rows), ctx)


def rdc_tile_rows_supported(rows: int) -> bool:
    return bool(load().rdc_tile_rows_supported(rows))


def rdc_current(ctx) -> Tuple[int, int, int]:
    """Returns (u address, v address, status); the status is RDC_OK or
    RDC_E_NONFINITE (the addresses are valid in both cases); raises on other
    errors."""
    u = ctypes.c_void_p()
    v = ctypes.c_void_p()
    s = load().rdc_current(ctx, ctypes.byref(u), ctypes.byref(v))
    if s not in (RDC_OK, RDC_E_NONFINITE):
        _check(s, ctx)
    return u.value, v.value, s


def rdc_set_arrival(ctx, ptr: Optional[int], pitch: int, theta: float) -> None:
    _check(load().rdc_set_arrival(ctx, ptr, pitch, theta), ctx)


def rdc_set_timelapse(ctx, ptr: Optional[int], pitch: int, rate: int) -> None:
    _check(load().rdc_set_timelapse(ctx, ptr, pitch, rate), ctx)


def rdc_set_step(ctx, step: int) -> None:
    _check(load().rdc_set_step(ctx, int(step)), ctx)


def rdc_get_step(ctx) -> int:
    s = ctypes.c_int64()
    _check(load().rdc_get_step(ctx, ctypes.byref(s)), ctx)
    return s.value


def rdc_last_error(ctx=None) -> str:
    m = load().rdc_last_error(ctx)
    return m.decode() if m else ""


def rdc_copy(dst: int, src: int, nbytes: int, stream: int) -> None:
    _check(load().rdc_copy(dst, src, nbytes, stream or None), None)


# ----------------------------------------------------------------- torch-owned simulation

def pitch_for(nx: int) -> int:
    return (nx + 63) // 64 * 64


class Sim:
    """One simulated grid on the current GPU: u, v (ping-pong) and phi planes
    allocated by torch with a 64-element row pitch, driven through the C ABI.

    ``params``: dict with eps, f, q, D_u, dt, dx (Eq. (1), Table 1)."""

    def __init__(self, nx: int, ny: int, params=None, dtype: str = "fp32", device=None,
                 stream=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the stepper runs only on the HIP device")
        load()
        self.nx, self.ny = int(nx), int(ny)
        self.dtype = dtype
        self.tdtype = torch.float64 if dtype == "fp64" else torch.float32
        self.np_dtype = np.float64 if dtype == "fp64" else np.float32
        self.device = torch.device(device if device is not None else "cuda")
        self.pitch = pitch_for(self.nx)
        mk = lambda: torch.zeros((self.ny, self.pitch), dtype=self.tdtype, device=self.device)
        self.planes = [mk() for _ in range(5)]  # u0, u1, v0, v1, phi
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = rdc_buffers()
        b.u[0], b.u[1] = self.planes[0].data_ptr(), self.planes[1].data_ptr()
        b.v[0], b.v[1] = self.planes[2].data_ptr(), self.planes[3].data_ptr()
        b.phi = self.planes[4].data_ptr()
        b.pitch = self.pitch
        with torch.cuda.device(self.device):
            self.ctx = rdc_create(self.nx, self.ny, RDC_FP64 if dtype == "fp64" else RDC_FP32, b,
                                  self.stream.cuda_stream)
        self.arrival_plane = None
        self.params = None
        if params is not None:
            self.set_params(params)

    # -- parameters and inputs
    def set_params(self, params) -> None:
        p = rdc_params(*(float(params[k]) for k in ("eps", "f", "q", "D_u", "dt", "dx")))
        rdc_set_params(self.ctx, p)
        self.params = dict(params)

    def _host(self, a) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=self.np_dtype)
        if a.shape != (self.ny, self.nx):
            raise ValueError("expected shape %s, got %s" % ((self.ny, self.nx), a.shape))
        return a

    def set_phi(self, phi) -> None:
        if hasattr(phi, "data_ptr"):
            t = phi.to(self.device, self.tdtype).contiguous()
            rdc_set_phi(self.ctx, t.data_ptr(), t.shape[-1], RDC_DEVICE)
            self._keep = t
        else:
            a = self._host(phi)
            rdc_set_phi(self.ctx, a.ctypes.data, self.nx, RDC_HOST)

    def write(self, u, v) -> None:
        if hasattr(u, "data_ptr"):
            tu = u.to(self.device, self.tdtype).contiguous()
            tv = v.to(self.device, self.tdtype).contiguous()
            rdc_write(self.ctx, tu.data_ptr(), tv.data_ptr(), tu.shape[-1], RDC_DEVICE)
            self._keep = (tu, tv)
        else:
            a, b = self._host(u), self._host(v)
            rdc_write(self.ctx, a.ctypes.data, b.ctypes.data, self.nx, RDC_HOST)

    def stimulate(self, disks: Iterable[Sequence[int]]) -> None:
        d = [tuple(int(t) for t in x) for x in disks]
        if d:
            rdc_stimulate(self.ctx, [t[0] for t in d], [t[1] for t in d], [t[2] for t in d])

    # -- stepping
    def set_block(self, T: int) -> None:
        rdc_set_block(self.ctx, T)

    def set_tile_rows(self, rows: int) -> None:
        rdc_set_tile_rows(self.ctx, rows)

    def autotune(self, **kw):
        """Time the launch shapes on this grid's shape (cached) and use the
        fastest; see autotune.tune_sim."""
        from . import autotune
        return autotune.tune_sim(self, **kw)

    def step(self, n: int) -> None:
        rdc_step(self.ctx, n)

    def run_schedule(self, stimuli, until: int) -> None:
        """Advance to step index ``until``, applying each stimulus ((step, cx,
        cy, r) tuples or objects) right before the step that leaves its step
        index -- the same schedule rule as the oracle's."""
        groups = {}
        for s in stimuli:
            t = (s.step, s.cx, s.cy, s.r) if hasattr(s, "step") else tuple(s)
            groups.setdefault(int(t[0]), []).append(t[1:])
        now = self.step_index
        for when in sorted(groups):
            if when < now or when > until:
                continue
            self.step(when - now)
            now = when
            self.stimulate(groups[when])
        self.step(until - now)

    @property
    def step_index(self) -> int:
        return rdc_get_step(self.ctx)

    # -- outputs
    def read(self, allow_nonfinite: bool = False) -> Tuple[np.ndarray, np.ndarray]:
        u = np.empty((self.ny, self.nx), dtype=self.np_dtype)
        v = np.empty((self.ny, self.nx), dtype=self.np_dtype)
        s = rdc_read(self.ctx, u.ctypes.data, v.ctypes.data, self.nx, RDC_HOST)
        if s == RDC_E_NONFINITE and not allow_nonfinite:
            raise RdcError(s, rdc_last_error(self.ctx))
        return u, v

    def current(self, allow_nonfinite: bool = False):
        """Torch views (ny, nx) of the planes holding the current u and v.
        Waits for the stream; raises RdcError(RDC_E_NONFINITE) if a step
        produced a non-finite value since the last write, unless
        `allow_nonfinite`."""
        pu, pv, s = rdc_current(self.ctx)
        if s == RDC_E_NONFINITE and not allow_nonfinite:
            raise RdcError(s, rdc_last_error(self.ctx))
        pick = {p.data_ptr(): p for p in self.planes[:4]}
        return pick[pu][:, : self.nx], pick[pv][:, : self.nx]

    def enable_arrival(self, theta: float = 0.5) -> None:
        t = self._torch
        self.arrival_plane = t.empty((self.ny, self.pitch), dtype=t.int32, device=self.device)
        rdc_set_arrival(self.ctx, self.arrival_plane.data_ptr(), self.pitch, theta)
        self.arrival_theta = float(theta)

    def arrival(self) -> np.ndarray:
        self.stream.synchronize()
        return self.arrival_plane[:, : self.nx].cpu().numpy()

    def enable_timelapse(self, rate: int) -> None:
        """Record the max of u over frames taken every `rate` steps (the
        current state is the first frame); see rdc_set_timelapse."""
        t = self._torch
        self.timelapse_plane = t.empty((self.ny, self.pitch), dtype=self.tdtype,
                                       device=self.device)
        rdc_set_timelapse(self.ctx, self.timelapse_plane.data_ptr(), self.pitch, rate)
        self.timelapse_rate = int(rate)

    def timelapse(self) -> np.ndarray:
        self.stream.synchronize()
        return self.timelapse_plane[:, : self.nx].cpu().numpy()

    def synchronize(self) -> None:
        self.stream.synchronize()

    # -- checkpoint / resume
    def save_checkpoint(self, path: str, seed: Optional[int] = None) -> None:
        """Write the state, phi, step index, parameters and any attached
        arrival / timelapse plane to `path`.npz + `path`.json (see
        checkpoint.py); from_checkpoint resumes bit-identically."""
        from . import checkpoint
        u, v = self.read()
        arrays = {"u": u, "v": v, "phi": self.planes[4][:, : self.nx].cpu().numpy()}
        meta = {"nx": self.nx, "ny": self.ny, "dtype": self.dtype, "params": self.params,
                "step": self.step_index, "seed": seed}
        if self.arrival_plane is not None:
            arrays["arrival"] = self.arrival()
            meta["arrival_theta"] = self.arrival_theta
        if getattr(self, "timelapse_plane", None) is not None:
            arrays["timelapse"] = self.timelapse()
            meta["timelapse_rate"] = self.timelapse_rate
        checkpoint.write(path, arrays, meta)

    @classmethod
    def from_checkpoint(cls, path: str, device=None, stream=None) -> "Sim":
        """A new context holding the checkpoint at `path` (digests checked)."""
        from . import checkpoint
        arrays, meta = checkpoint.read(path)
        s = cls(meta["nx"], meta["ny"], meta["params"], meta["dtype"], device=device,
                stream=stream)
        s.set_phi(arrays["phi"])
        s.write(arrays["u"], arrays["v"])
        rdc_set_step(s.ctx, meta["step"])
        t = s._torch
        if "arrival" in arrays:
            s.enable_arrival(meta["arrival_theta"])
            s.stream.synchronize()
            s.arrival_plane[:, : s.nx].copy_(t.as_tensor(arrays["arrival"]))
        if "timelapse" in arrays:
            s.enable_timelapse(meta["timelapse_rate"])
            s.stream.synchronize()
            s.timelapse_plane[:, : s.nx].copy_(t.as_tensor(arrays["timelapse"]))
        t.cuda.synchronize(s.device)
        return s

    def close(self) -> None:
        if getattr(self, "ctx", None):
            rdc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- batched simulations

def _bcheck(status: int, b) -> None:
    if status != RDC_OK:
        msg = load().rdc_batch_last_error(b)
        raise RdcError(status, msg.decode() if msg else "")


def _params_struct(params) -> rdc_params:
    return rdc_params(*(float(params[k]) for k in ("eps", "f", "q", "D_u", "dt", "dx")))


class BatchSim:
    """Many independent FP32 grids advanced together (rdc_batch_*): each
    spec is (nx, ny, params).  Planes are pooled in five torch tensors; each
    grid's region starts on a 64-element boundary with a 64-element pitch."""

    def __init__(self, specs, device=None, stream=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the stepper runs only on the HIP device")
        lib = load()
        self.count = len(specs)
        self.specs = [(int(nx), int(ny), dict(p)) for nx, ny, p in specs]
        self.device = torch.device(device if device is not None else "cuda")
        descs = (rdc_sim_desc * self.count)()
        self.shapes = []
        off = 0
        for i, (nx, ny, params) in enumerate(specs):
            pitch = pitch_for(int(nx))
            descs[i].nx, descs[i].ny = int(nx), int(ny)
            descs[i].pitch, descs[i].offset = pitch, off
            descs[i].params = _params_struct(params)
            self.shapes.append((int(nx), int(ny), pitch, off))
            off += pitch * int(ny)
        self.pool_elems = off
        self.planes = [torch.zeros(off, dtype=torch.float32, device=self.device) for _ in range(5)]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = rdc_buffers()
        b.u[0], b.u[1] = self.planes[0].data_ptr(), self.planes[1].data_ptr()
        b.v[0], b.v[1] = self.planes[2].data_ptr(), self.planes[3].data_ptr()
        b.phi = self.planes[4].data_ptr()
        b.pitch = 0
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _bcheck(lib.rdc_batch_create(self.count, descs, ctypes.byref(b), off,
                                         self.stream.cuda_stream or None, ctypes.byref(out)), None)
        self.b = out.value
        self.step_index = 0
        self.resident_max_cells = RDC_BATCH_RESIDENT_DEFAULT

    def _host(self, i, a):
        nx, ny, _, _ = self.shapes[i]
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.shape != (ny, nx):
            raise ValueError("expected shape %s, got %s" % ((ny, nx), a.shape))
        return a

    def set_block(self, T: int, rows: int = 56) -> None:
        _bcheck(load().rdc_batch_set_block(self.b, T, rows), self.b)

    def set_resident(self, max_cells: int) -> None:
        """Grids of at most max_cells cells (that fit) run whole in LDS; 0 = off."""
        _bcheck(load().rdc_batch_set_resident(self.b, int(max_cells)), self.b)
        self.resident_max_cells = int(max_cells)

    def resident_count(self) -> int:
        return int(load().rdc_batch_resident_count(self.b))

    def autotune(self, **kw):
        """Time the launch shapes on these grids' shapes (cached) and use the
        fastest; see autotune.tune_batch."""
        from . import autotune
        return autotune.tune_batch(self, **kw)

    def set_phi(self, i: int, phi) -> None:
        a = self._host(i, phi)
        _bcheck(load().rdc_batch_set_phi(self.b, i, a.ctypes.data, a.shape[1], RDC_HOST), self.b)

    def write(self, i: int, u, v) -> None:
        a, c = self._host(i, u), self._host(i, v)
        _bcheck(load().rdc_batch_write(self.b, i, a.ctypes.data, c.ctypes.data, a.shape[1],
                                       RDC_HOST), self.b)

    def stimulate(self, disks) -> None:
        """disks: iterable of (sim, cx, cy, r)."""
        d = [tuple(int(t) for t in x) for x in disks]
        if not d:
            return
        arr = [np.ascontiguousarray([t[j] for t in d], dtype=np.int32) for j in range(4)]
        ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for a in arr]
        _bcheck(load().rdc_batch_stimulate(self.b, *ptrs, len(d)), self.b)

    def step(self, n: int) -> None:
        _bcheck(load().rdc_batch_step(self.b, int(n)), self.b)
        self.step_index += int(n)

    def read(self, i: int, allow_nonfinite: bool = False):
        nx, ny, _, _ = self.shapes[i]
        u = np.empty((ny, nx), np.float32)
        v = np.empty((ny, nx), np.float32)
        s = load().rdc_batch_read(self.b, i, u.ctypes.data, v.ctypes.data, nx, RDC_HOST)
        if s == RDC_E_NONFINITE and allow_nonfinite:
            return u, v
        _bcheck(s, self.b)
        return u, v

    def nonfinite(self):
        """Indices of the grids whose sticky non-finite flag is set (syncs)."""
        out = []
        for i in range(len(self.shapes)):
            s = load().rdc_batch_read(self.b, i, None, None, 0, RDC_HOST)
            if s == RDC_E_NONFINITE:
                out.append(i)
            else:
                _bcheck(s, self.b)
        return out

    def current(self):
        """Flat torch views (pool_elems,) of the pool planes holding u and v."""
        u = ctypes.c_void_p()
        v = ctypes.c_void_p()
        _bcheck(load().rdc_batch_current(self.b, ctypes.byref(u), ctypes.byref(v)), self.b)
        pick = {p.data_ptr(): p for p in self.planes[:4]}
        return pick[u.value], pick[v.value]

    def capture(self, n: int) -> "BatchGraph":
        out = ctypes.c_void_p()
        _bcheck(load().rdc_batch_capture(self.b, int(n), ctypes.byref(out)), self.b)
        return BatchGraph(self, out.value, int(n))

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if getattr(self, "b", None):
            load().rdc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """A recorded rdc_batch_step(n): each launch() advances the batch by n."""

    def __init__(self, batch: BatchSim, handle, n: int):
        self.batch, self.g, self.n = batch, handle, n

    def launch(self) -> None:
        _bcheck(load().rdc_graph_launch(self.g), self.batch.b)
        self.batch.step_index += self.n

    def close(self) -> None:
        if getattr(self, "g", None):
            load().rdc_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- network kernels

def nn(name: str, *args):
    """Call rdc_nn_<name>(*args); raise RdcError with the library's message
    on failure.  Tensor arguments are passed as device addresses (ints)."""
    fn = getattr(load(), "rdc_nn_" + name)
    st = fn(*args)
    if st != RDC_OK:
        msg = load().rdc_nn_last_error()
        raise RdcError(st, msg.decode() if msg else "")
