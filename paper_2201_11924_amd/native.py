"""ctypes binding of ``libsimsense.so`` (argument marshalling only).

Every step of the depth path runs in the HIP library; this module only turns
torch tensors into device pointers and the current torch stream into a
hipStream_t.  If the library has not been built the import fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Dict, Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsimsense.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2201_11924_amd.build)")

_lib = ct.CDLL(LIB_PATH)

OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "null pointer", -3: "out of memory", -4: "device error",
          -5: "unsupported", -6: "abi mismatch", -7: "too large for the static scratch"}
ERR_TOO_LARGE = -7
FLAG_UNIQUE, FLAG_LR, FLAG_NONZERO, FLAG_VALID = 1, 2, 4, 8

PARAM_FIELDS = ("width", "height", "max_disp", "census_w", "census_h", "census_mode", "p1", "p2",
                "uniqueness_pct", "lr_max_diff", "num_paths", "median", "subpixel")


class Params(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32)] + [(n, ct.c_int32) for n in PARAM_FIELDS] + [
        ("focal_px", ct.c_float), ("baseline_m", ct.c_float), ("lr_mode", ct.c_int32),
        ("block_w", ct.c_int32), ("block_h", ct.c_int32)]

    @classmethod
    def from_dict(cls, d: Dict) -> "Params":
        p = cls()
        p.struct_size = ct.sizeof(cls)
        for n in PARAM_FIELDS:
            setattr(p, n, int(d[n]))
        p.focal_px = float(d["focal_px"])
        p.baseline_m = float(d["baseline_m"])
        p.lr_mode = int(d.get("lr_mode", 0))
        p.block_w = int(d.get("block_w", 1))
        p.block_h = int(d.get("block_h", 1))
        return p


class Outputs(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in (
        "depth", "disp", "flags", "disp_int", "cost_best", "cost_second", "disp_right", "disp_sub",
        "census_left", "census_right", "volume", "features")]


_vp, _i32, _i64 = ct.c_void_p, ct.c_int32, ct.c_int64
_lib.simsense_create.argtypes = [ct.POINTER(Params), ct.POINTER(_vp)]
_lib.simsense_destroy.argtypes = [_vp]
_lib.simsense_compute.argtypes = [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]
_lib.simsense_compute_ex.argtypes = [_vp, _vp, _vp, _i32, ct.POINTER(Outputs), _vp]
_lib.simsense_ir_noise.argtypes = [_vp, _vp, _vp, _vp, _i64, _vp]
_lib.simsense_census.argtypes = [ct.POINTER(Params), _vp, _i32, _vp, _vp]
_lib.simsense_strerror.argtypes = [ct.c_int]
_lib.simsense_strerror.restype = ct.c_char_p
_lib.simsense_scratch_bytes.argtypes = [ct.POINTER(Params)]
_lib.simsense_scratch_bytes.restype = _i64
_lib.simsense_compute_noalloc.argtypes = [ct.POINTER(Params), _vp, _vp, _i32, _vp, _vp, _vp, _vp]
_lib.simsense_profile_enable.argtypes = [_vp, ct.c_int]
_lib.simsense_profile_read.argtypes = [_vp, ct.POINTER(ct.c_double), ct.POINTER(_i32), _i32]
PASSES = ("census", "aggregate", "select", "post")


class SimSenseError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_lib.simsense_strerror(code).decode()} ({code})")
        self.code = code


def _check(code: int, what: str) -> None:
    if code != OK:
        raise SimSenseError(code, what)


def lib() -> ct.CDLL:
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to the HIP library must live on the GPU")
    return ct.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name}: need a contiguous {dtype} GPU tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")


def scratch_bytes(params: Dict) -> int:
    p = Params.from_dict(params)
    v = _lib.simsense_scratch_bytes(ct.byref(p))
    if v < 0:
        _check(int(v), "simsense_scratch_bytes")
    return int(v)


class SimSense:
    """One parameter set of the depth path and its device scratch."""

    def __init__(self, params: Dict):
        self.params = dict(params)
        self._p = Params.from_dict(params)
        h = ct.c_void_p()
        _check(_lib.simsense_create(ct.byref(self._p), ct.byref(h)), "simsense_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(_lib.simsense_destroy(self._h), "simsense_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True) -> None:
        _check(_lib.simsense_profile_enable(self._h, int(enable)), "simsense_profile_enable")

    def profile_read(self):
        """(calls, {pass: total device ms}) since the last read."""
        ms = (ct.c_double * len(PASSES))()
        calls = _i32()
        _check(_lib.simsense_profile_read(self._h, ms, ct.byref(calls), len(PASSES)), "simsense_profile_read")
        return calls.value, dict(zip(PASSES, list(ms)))

    @property
    def shape(self):
        return (self.params["height"], self.params["width"])

    def set_tuning(self, horizontal_lanes: int = 0, blocks_per_cu: int = 3) -> None:
        """Launch shape of the aggregation (blocks_per_cu 0 = one block per line block)."""
        t = Tuning(ct.sizeof(Tuning), horizontal_lanes, blocks_per_cu)
        _check(_lib.simsense_set_tuning(self._h, ct.byref(t)), "simsense_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(_lib.simsense_get_tuning(self._h, ct.byref(t)), "simsense_get_tuning")
        return dict(horizontal_lanes=t.horizontal_lanes, blocks_per_cu=t.blocks_per_cu)

    def autotune(self, left: torch.Tensor, right: torch.Tensor, reps: int = 5, stream=None):
        """Times every launch shape on this pair and keeps the fastest: (best, ms per candidate)."""
        H, W = self.shape
        _need(left, torch.uint8, (H, W), "left")
        _need(right, torch.uint8, (H, W), "right")
        best = Tuning()
        ms = (ct.c_float * 32)()
        count = _i32()
        _check(_lib.simsense_autotune(self._h, _ptr(left), _ptr(right), W, reps, ct.byref(best), ms, 32,
                                      ct.byref(count), _stream(stream)), "simsense_autotune")
        return dict(horizontal_lanes=best.horizontal_lanes, blocks_per_cu=best.blocks_per_cu), list(ms)[:count.value]

    def compute(self, left: torch.Tensor, right: torch.Tensor, depth: torch.Tensor,
                disp: Optional[torch.Tensor] = None, flags: Optional[torch.Tensor] = None, stream=None):
        H, W = self.shape
        _need(left, torch.uint8, (H, W), "left")
        _need(right, torch.uint8, (H, W), "right")
        _need(depth, torch.float32, (H, W), "depth")
        _check(_lib.simsense_compute(self._h, _ptr(left), _ptr(right), W, _ptr(depth), _ptr(disp),
                                     _ptr(flags), _stream(stream)), "simsense_compute")

    def __call__(self, left: torch.Tensor, right: torch.Tensor, stream=None):
        H, W = self.shape
        depth = torch.empty((H, W), dtype=torch.float32, device=left.device)
        disp = torch.empty_like(depth)
        flags = torch.empty((H, W), dtype=torch.uint8, device=left.device)
        self.compute(left, right, depth, disp, flags, stream)
        return depth, disp, flags

    def compute_all(self, left: torch.Tensor, right: torch.Tensor, volume: bool = False, features: bool = False,
                    stream=None):
        """Every intermediate of the path, as a dict of GPU tensors."""
        H, W = self.shape
        D = self.params["max_disp"]
        dev = left.device
        _need(left, torch.uint8, (H, W), "left")
        _need(right, torch.uint8, (H, W), "right")
        out = dict(depth=torch.empty((H, W), dtype=torch.float32, device=dev),
                   disp=torch.empty((H, W), dtype=torch.float32, device=dev),
                   flags=torch.empty((H, W), dtype=torch.uint8, device=dev),
                   disp_int=torch.empty((H, W), dtype=torch.uint8, device=dev),
                   cost_best=torch.empty((H, W), dtype=torch.int16, device=dev),
                   cost_second=torch.empty((H, W), dtype=torch.int16, device=dev),
                   disp_right=torch.empty((H, W), dtype=torch.uint8, device=dev),
                   disp_sub=torch.empty((H, W), dtype=torch.float32, device=dev),
                   census_left=torch.empty((H, W), dtype=torch.int64, device=dev),
                   census_right=torch.empty((H, W), dtype=torch.int64, device=dev))
        if volume:
            out["volume"] = torch.empty((H, W, D), dtype=torch.int16, device=dev)
        if features:
            out["features"] = torch.empty((H, W, 8), dtype=torch.int16, device=dev)
        o = Outputs(**{k: v.data_ptr() for k, v in out.items()})
        _check(_lib.simsense_compute_ex(self._h, _ptr(left), _ptr(right), W, ct.byref(o), _stream(stream)),
               "simsense_compute_ex")
        return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def compute_noalloc(params: Dict, left: torch.Tensor, right: torch.Tensor, depth: torch.Tensor,
                    disp: Optional[torch.Tensor] = None, flags: Optional[torch.Tensor] = None, stream=None) -> None:
    """simsense_compute_noalloc: the whole path without a handle, in the library's
    static per-GPU scratch (no device allocation)."""
    H, W = params["height"], params["width"]
    _need(left, torch.uint8, (H, W), "left")
    _need(right, torch.uint8, (H, W), "right")
    _need(depth, torch.float32, (H, W), "depth")
    if disp is not None:
        _need(disp, torch.float32, (H, W), "disp")
    if flags is not None:
        _need(flags, torch.uint8, (H, W), "flags")
    p = Params.from_dict(params)
    _check(_lib.simsense_compute_noalloc(ct.byref(p), _ptr(left), _ptr(right), W, _ptr(depth), _ptr(disp),
                                         _ptr(flags), _stream(stream)), "simsense_compute_noalloc")


def ir_noise(img: torch.Tensor, gamma: torch.Tensor, n: torch.Tensor, out: Optional[torch.Tensor] = None,
             stream=None) -> torch.Tensor:
    """IR noise model of Sec. VI-C, Eq. (7), applied with the caller's draws."""
    _need(gamma, torch.float32, img.shape, "gamma")
    _need(n, torch.float32, img.shape, "n")
    _need(img, torch.uint8, img.shape, "img")
    out = torch.empty_like(img) if out is None else out
    _check(_lib.simsense_ir_noise(_ptr(img), _ptr(gamma), _ptr(n), _ptr(out), img.numel(), _stream(stream)),
           "simsense_ir_noise")
    return out


class NoiseParams(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("gain_model", ct.c_int32), ("k", ct.c_float), ("theta", ct.c_float),
                ("gain_sd", ct.c_float), ("mu", ct.c_float), ("sigma", ct.c_float), ("scale", ct.c_float),
                ("seed", ct.c_uint64), ("stream", ct.c_uint32)]

    @classmethod
    def make(cls, gain_model: int, k: float = 3.98, theta: float = 0.254, gain_sd: float = 0.05, mu: float = -0.231,
             sigma: float = 0.83, scale: float = 1.0, seed: int = 0, noise_stream: int = 0) -> "NoiseParams":
        return cls(ct.sizeof(cls), gain_model, k, theta, gain_sd, mu, sigma, scale, seed, noise_stream)


_lib.simsense_noise_draws.argtypes = [ct.POINTER(NoiseParams), _i64, _vp, _vp, _vp]
_lib.simsense_ir_noise_generate.argtypes = [ct.POINTER(NoiseParams), _vp, _i32, _i32, _i32, _vp, _i32, _vp]


def noise_draws(count: int, stream=None, **kw):
    """gamma' and n' of pixels 0..count-1 from the on-device generator (GPU tensors)."""
    p = NoiseParams.make(**kw)
    g = torch.empty(count, dtype=torch.float32, device="cuda")
    n = torch.empty(count, dtype=torch.float32, device="cuda")
    _check(_lib.simsense_noise_draws(ct.byref(p), count, _ptr(g), _ptr(n), _stream(stream)), "simsense_noise_draws")
    return g, n


def ir_noise_generate(img: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None, **kw) -> torch.Tensor:
    """IR noise of Sec. VI-C drawn on the device and applied in one pass."""
    _need(img, torch.uint8, img.shape, "img")
    H, W = img.shape
    out = torch.empty_like(img) if out is None else out
    p = NoiseParams.make(**kw)
    _check(_lib.simsense_ir_noise_generate(ct.byref(p), _ptr(img), W, W, H, _ptr(out), W, _stream(stream)),
           "simsense_ir_noise_generate")
    return out


class Camera(ct.Structure):
    _fields_ = [("fx", ct.c_float), ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float)]


_lib.simsense_rectify.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _vp]
_lib.simsense_register_depth.argtypes = [_vp, _i32, _i32, ct.POINTER(Camera), ct.POINTER(ct.c_float),
                                         ct.POINTER(Camera), _i32, _i32, _vp, _vp]


def rectify(img: torch.Tensor, map_x: torch.Tensor, map_y: torch.Tensor, stream=None) -> torch.Tensor:
    """Bilinear remap of a raw IR image to the rectified frame (maps: float32, output shape)."""
    H, W = img.shape
    _need(img, torch.uint8, (H, W), "img")
    oh, ow = map_x.shape
    _need(map_x, torch.float32, (oh, ow), "map_x")
    _need(map_y, torch.float32, (oh, ow), "map_y")
    out = torch.empty((oh, ow), dtype=torch.uint8, device=img.device)
    _check(_lib.simsense_rectify(_ptr(img), W, W, H, _ptr(map_x), _ptr(map_y), ow, oh, _ptr(out), ow,
                                 _stream(stream)), "simsense_rectify")
    return out


def register_depth(depth: torch.Tensor, ir, rt, rgb, out_w: int, out_h: int, stream=None) -> torch.Tensor:
    """Depth registered into the RGB camera; ir, rgb: (fx, fy, cx, cy); rt: 12 floats (R row-major, t)."""
    H, W = depth.shape
    _need(depth, torch.float32, (H, W), "depth")
    rtv = (ct.c_float * 12)(*[float(v) for v in rt])
    out = torch.empty((out_h, out_w), dtype=torch.float32, device=depth.device)
    _check(_lib.simsense_register_depth(_ptr(depth), W, H, ct.byref(Camera(*ir)), rtv, ct.byref(Camera(*rgb)),
                                        out_w, out_h, _ptr(out), _stream(stream)), "simsense_register_depth")
    return out


def census(params: Dict, img: torch.Tensor, stream=None) -> torch.Tensor:
    p = Params.from_dict(params)
    H, W = params["height"], params["width"]
    _need(img, torch.uint8, (H, W), "img")
    out = torch.empty((H, W), dtype=torch.int64, device=img.device)
    _check(_lib.simsense_census(ct.byref(p), _ptr(img), W, _ptr(out), _stream(stream)), "simsense_census")
    return out


# ---------------------------------------------------------------- learned surrogate
_lib.simsense_net_num_params.restype = _i64
_lib.simsense_net_create.argtypes = [_i64, ct.c_uint64, ct.POINTER(_vp)]
_lib.simsense_net_destroy.argtypes = [_vp]
_fp = ct.POINTER(ct.c_float)
_lib.simsense_net_get_state.argtypes = [_vp, _fp, _fp, _fp, _i64, ct.POINTER(_i64)]
_lib.simsense_net_set_state.argtypes = [_vp, _fp, _fp, _fp, _i64, _i64]
_lib.simsense_net_get_grads.argtypes = [_vp, _fp, _i64]
_lib.simsense_net_forward.argtypes = [_vp, _vp, _i32, _i32, _i32, _vp, _vp]
_lib.simsense_net_train_step.argtypes = [_vp, _vp, _vp, _vp, _i32, _i32, _i32, ct.c_float, _vp, _vp]
_lib.simsense_net_targets.argtypes = [_vp, _vp, _vp, _vp, _vp, _i64, _vp]
_lib.simsense_net_infer.argtypes = [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, ct.c_float, _vp, _vp]
_lib.simsense_learned_compute.argtypes = [_vp, _vp, _vp, _vp, _i32, ct.POINTER(Outputs), _vp]
_lib.simsense_net_read_tensor.argtypes = [_vp, _i32, _i32, _vp, _i64]
NET_ACTIVATION, NET_OUTPUT, NET_OUTPUT_GRAD = 0, 1, 2

NUM_NET_PARAMS = int(_lib.simsense_net_num_params())


def _host_f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_fp)


class Net:
    """The learned surrogate's parameters, Adam state and device buffers."""

    def __init__(self, max_pixels: int, seed: int = 0):
        h = ct.c_void_p()
        _check(_lib.simsense_net_create(int(max_pixels), int(seed), ct.byref(h)), "simsense_net_create")
        self._h = h
        self.max_pixels = int(max_pixels)

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.simsense_net_destroy(self._h), "simsense_net_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_state(self):
        import numpy as np
        n = NUM_NET_PARAMS
        p, m, v = (np.empty(n, np.float32) for _ in range(3))
        step = _i64()
        _check(_lib.simsense_net_get_state(self._h, p.ctypes.data_as(_fp), m.ctypes.data_as(_fp),
                                           v.ctypes.data_as(_fp), n, ct.byref(step)), "simsense_net_get_state")
        return p, m, v, int(step.value)

    def set_state(self, params, m=None, v=None, step: int = 0):
        p, pp = _host_f32(params)
        mm = _host_f32(m) if m is not None else (None, None)
        vv = _host_f32(v) if v is not None else (None, None)
        _check(_lib.simsense_net_set_state(self._h, pp, mm[1], vv[1], NUM_NET_PARAMS, int(step)),
               "simsense_net_set_state")

    def get_grads(self):
        import numpy as np
        g = np.empty(NUM_NET_PARAMS, np.float32)
        _check(_lib.simsense_net_get_grads(self._h, g.ctypes.data_as(_fp), NUM_NET_PARAMS), "simsense_net_get_grads")
        return g

    def read_tensor(self, what: int, layer: int, pixels: int):
        """A tensor the last forward / training call left in the net, as a numpy
        array: bf16 bits (uint16) [pixels, C] for activations and gradients, fp32
        [pixels, 2] for the output."""
        import numpy as np
        if what == NET_OUTPUT:
            a = np.empty((pixels, 2), np.float32)
        else:
            a = np.empty((pixels, 16 if (what == NET_OUTPUT_GRAD and layer == 3) else 32), np.uint16)
        _check(_lib.simsense_net_read_tensor(self._h, what, layer, a.ctypes.data_as(_vp), a.nbytes),
               "simsense_net_read_tensor")
        return a

    def forward(self, features: torch.Tensor, stream=None) -> torch.Tensor:
        B, H, W, C = features.shape
        if C != 8 or features.element_size() != 2 or not features.is_contiguous():
            raise ValueError("features: contiguous 16-bit [B, H, W, 8] tensor (bf16 bits)")
        out = torch.empty((B, H, W, 2), dtype=torch.float32, device=features.device)
        _check(_lib.simsense_net_forward(self._h, _ptr(features), B, H, W, _ptr(out), _stream(stream)),
               "simsense_net_forward")
        return out

    def infer(self, features: torch.Tensor, d2_sub: Optional[torch.Tensor] = None, raw: bool = True,
              tau: float = 0.0, uncertain: Optional[torch.Tensor] = None, stream=None):
        """Fused inference: {"out": [B,H,W,2] (if raw), "masked", "flags" (if d2_sub is given)}."""
        B, H, W, C = features.shape
        if C != 8 or features.element_size() != 2 or not features.is_contiguous():
            raise ValueError("features: contiguous 16-bit [B, H, W, 8] tensor (bf16 bits)")
        dev = features.device
        res = {}
        if raw:
            res["out"] = torch.empty((B, H, W, 2), dtype=torch.float32, device=dev)
        if d2_sub is not None:
            _need(d2_sub, torch.float32, (B, H, W), "d2_sub")
            res["masked"] = torch.empty((B, H, W), dtype=torch.float32, device=dev)
            res["flags"] = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
        if uncertain is not None:
            _need(uncertain, torch.int32, (B,), "uncertain")
        _check(_lib.simsense_net_infer(self._h, _ptr(features), B, H, W, _ptr(d2_sub), _ptr(res.get("out")),
                                       _ptr(res.get("masked")), _ptr(res.get("flags")), float(tau),
                                       _ptr(uncertain), _stream(stream)), "simsense_net_infer")
        return res

    def train_step(self, features: torch.Tensor, t_res: torch.Tensor, t_valid: torch.Tensor, lr: float,
                   stream=None) -> torch.Tensor:
        B, H, W, C = features.shape
        _need(t_res, torch.float32, (B, H, W), "t_res")
        _need(t_valid, torch.uint8, (B, H, W), "t_valid")
        loss = torch.empty(3, dtype=torch.float32, device=features.device)
        _check(_lib.simsense_net_train_step(self._h, _ptr(features), _ptr(t_res), _ptr(t_valid), B, H, W,
                                            float(lr), _ptr(loss), _stream(stream)), "simsense_net_train_step")
        return loss


def net_targets(d8_sub: torch.Tensor, flags8: torch.Tensor, d2_sub: torch.Tensor, stream=None):
    t_res = torch.empty_like(d8_sub)
    t_valid = torch.empty(d8_sub.shape, dtype=torch.uint8, device=d8_sub.device)
    _check(_lib.simsense_net_targets(_ptr(d8_sub), _ptr(flags8), _ptr(d2_sub), _ptr(t_res), _ptr(t_valid),
                                     d8_sub.numel(), _stream(stream)), "simsense_net_targets")
    return t_res, t_valid


def learned_compute(ss: "SimSense", net: Net, left: torch.Tensor, right: torch.Tensor, extras: bool = False,
                    stream=None):
    """The learned depth path on one pair: returns a dict of GPU tensors."""
    H, W = ss.shape
    dev = left.device
    _need(left, torch.uint8, (H, W), "left")
    _need(right, torch.uint8, (H, W), "right")
    out = dict(depth=torch.empty((H, W), dtype=torch.float32, device=dev),
               disp=torch.empty((H, W), dtype=torch.float32, device=dev),
               flags=torch.empty((H, W), dtype=torch.uint8, device=dev))
    if extras:
        out.update(disp_sub=torch.empty((H, W), dtype=torch.float32, device=dev),
                   disp_int=torch.empty((H, W), dtype=torch.uint8, device=dev),
                   features=torch.empty((H, W, 8), dtype=torch.int16, device=dev))
    o = Outputs(**{k: v.data_ptr() for k, v in out.items()})
    _check(_lib.simsense_learned_compute(ss._h, net._h, _ptr(left), _ptr(right), W, ct.byref(o), _stream(stream)),
           "simsense_learned_compute")
    return out


# ---------------------------------------------------------------- batches
class Pair(ct.Structure):
    _fields_ = [("left", _vp), ("right", _vp), ("pitch", _i32), ("depth", _vp), ("disp", _vp), ("flags", _vp)]


class Tuning(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("horizontal_lanes", _i32), ("blocks_per_cu", _i32)]


_lib.simsense_set_tuning.argtypes = [_vp, ct.POINTER(Tuning)]
_lib.simsense_get_tuning.argtypes = [_vp, ct.POINTER(Tuning)]
_lib.simsense_autotune.argtypes = [_vp, _vp, _vp, _i32, _i32, ct.POINTER(Tuning), ct.POINTER(ct.c_float), _i32,
                                   ct.POINTER(_i32), _vp]
_lib.simsense_batch_create.argtypes = [ct.POINTER(Params), _i32, ct.POINTER(_vp)]
_lib.simsense_batch_destroy.argtypes = [_vp]
_lib.simsense_batch_scratch_bytes.argtypes = [_vp]
_lib.simsense_batch_scratch_bytes.restype = _i64
_lib.simsense_batch_compute.argtypes = [_vp, ct.POINTER(Pair), _vp]
_lib.simsense_batch_set_tuning.argtypes = [_vp, ct.POINTER(Tuning)]
_lib.simsense_batch_get_tuning.argtypes = [_vp, ct.POINTER(Tuning)]
_lib.simsense_batch_learned_compute.argtypes = [_vp, _vp, ct.POINTER(Pair), ct.c_float, _vp, _vp]
_lib.simsense_batch_learned_fallback.argtypes = [_vp, _vp, _vp, ct.POINTER(Pair), ct.c_float, _vp, _i32,
                                                 ct.c_float, ct.POINTER(_i32), _vp]
FALLBACK_THRESHOLD, FALLBACK_NEVER, FALLBACK_ALWAYS = 0, 1, 2
_lib.simsense_batch_autotune.argtypes = [_vp, ct.POINTER(Pair), _i32, ct.POINTER(Tuning), ct.POINTER(ct.c_float),
                                         _i32, ct.POINTER(_i32), _vp]


class Batch:
    """Many pairs of uneven sizes, computed by one graph launch per call."""

    def __init__(self, params_list):
        self.params = [dict(p) for p in params_list]
        arr = (Params * len(self.params))(*[Params.from_dict(p) for p in self.params])
        h = ct.c_void_p()
        _check(_lib.simsense_batch_create(arr, len(self.params), ct.byref(h)), "simsense_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.simsense_batch_destroy(self._h), "simsense_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def scratch_bytes(self) -> int:
        return int(_lib.simsense_batch_scratch_bytes(self._h))

    def outputs(self, device="cuda"):
        outs = []
        for p in self.params:
            H, W = p["height"], p["width"]
            outs.append(dict(depth=torch.empty((H, W), dtype=torch.float32, device=device),
                             disp=torch.empty((H, W), dtype=torch.float32, device=device),
                             flags=torch.empty((H, W), dtype=torch.uint8, device=device)))
        return outs

    def _pairs(self, lefts, rights, outs):
        arr = (Pair * len(self.params))()
        for i, (p, L, R, o) in enumerate(zip(self.params, lefts, rights, outs)):
            _need(L, torch.uint8, (p["height"], p["width"]), f"left[{i}]")
            _need(R, torch.uint8, (p["height"], p["width"]), f"right[{i}]")
            arr[i] = Pair(L.data_ptr(), R.data_ptr(), p["width"], o["depth"].data_ptr(),
                          o["disp"].data_ptr() if o.get("disp") is not None else None,
                          o["flags"].data_ptr() if o.get("flags") is not None else None)
        return arr

    def compute(self, lefts, rights, outs, stream=None):
        arr = self._pairs(lefts, rights, outs)
        _check(_lib.simsense_batch_compute(self._h, arr, _stream(stream)), "simsense_batch_compute")

    def learned_compute(self, net: "Net", lefts, rights, outs, tau: float, uncertain: torch.Tensor,
                        stream=None):
        """The learned form on every pair; `uncertain` (int32 GPU tensor, one per pair)
        receives the count of pixels whose validity logit lies within (-tau, tau)."""
        arr = self._pairs(lefts, rights, outs)
        if uncertain.dtype != torch.int32 or uncertain.numel() != len(self.params) or not uncertain.is_cuda:
            raise ValueError("uncertain: int32 GPU tensor with one entry per pair")
        _check(_lib.simsense_batch_learned_compute(self._h, net._h, arr, float(tau), _ptr(uncertain),
                                                   _stream(stream)), "simsense_batch_learned_compute")

    def learned_fallback(self, net: "Net", plain: Optional["SimSense"], lefts, rights, outs, tau: float,
                         uncertain: torch.Tensor, mode: int = FALLBACK_THRESHOLD, max_uncertain_frac: float = 0.25,
                         stream=None):
        """The learned form, then plain SGM (the `plain` handle) for the pairs that fall
        back, over their own outputs; returns the per-pair fallback decisions (list of 0/1)."""
        arr = self._pairs(lefts, rights, outs)
        if uncertain.dtype != torch.int32 or uncertain.numel() != len(self.params) or not uncertain.is_cuda:
            raise ValueError("uncertain: int32 GPU tensor with one entry per pair")
        fb = (_i32 * len(self.params))()
        _check(_lib.simsense_batch_learned_fallback(self._h, net._h, plain._h if plain is not None else None, arr,
                                                    float(tau), _ptr(uncertain), int(mode),
                                                    float(max_uncertain_frac), fb, _stream(stream)),
               "simsense_batch_learned_fallback")
        return list(fb)

    def set_tuning(self, horizontal_lanes: int = 0, blocks_per_cu: int = 2):
        t = Tuning(ct.sizeof(Tuning), horizontal_lanes, blocks_per_cu)
        _check(_lib.simsense_batch_set_tuning(self._h, ct.byref(t)), "simsense_batch_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(_lib.simsense_batch_get_tuning(self._h, ct.byref(t)), "simsense_batch_get_tuning")
        return dict(horizontal_lanes=t.horizontal_lanes, blocks_per_cu=t.blocks_per_cu)

    def autotune(self, lefts, rights, outs, reps: int = 5, stream=None):
        arr = self._pairs(lefts, rights, outs)
        best = Tuning()
        ms = (ct.c_float * 32)()
        count = _i32()
        _check(_lib.simsense_batch_autotune(self._h, arr, reps, ct.byref(best), ms, 32, ct.byref(count),
                                            _stream(stream)), "simsense_batch_autotune")
        return dict(horizontal_lanes=best.horizontal_lanes, blocks_per_cu=best.blocks_per_cu), list(ms)[:count.value]
