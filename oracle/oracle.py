"""numpy front end of the CPU oracle (``sgm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.  It
shares no code with the GPU path: the C file is compiled here with the host
compiler into its own shared object.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgm_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "noise_oracle.c"), os.path.join(_HERE, "geometry_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ct.CDLL(_LIB)
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


class OrcParams(ct.Structure):
    _fields_ = [(n, ct.c_int32) for n in (
        "width", "height", "max_disp", "census_w", "census_h", "census_mode", "p1", "p2",
        "uniqueness_pct", "lr_max_diff", "num_paths", "median", "subpixel")] + [
        ("focal_px", ct.c_float), ("baseline_m", ct.c_float), ("lr_mode", ct.c_int32),
        ("block_w", ct.c_int32), ("block_h", ct.c_int32)]


class OrcResult(ct.Structure):
    _fields_ = [("census_l", ct.c_void_p), ("census_r", ct.c_void_p), ("S", ct.c_void_p),
                ("dint", ct.c_void_p), ("s1", ct.c_void_p), ("s2", ct.c_void_p),
                ("dright", ct.c_void_p), ("flags", ct.c_void_p), ("dsub", ct.c_void_p),
                ("disp", ct.c_void_p), ("depth", ct.c_void_p)]


FLAG_UNIQUE, FLAG_LR, FLAG_NONZERO, FLAG_FINAL = 1, 2, 4, 8


def ir_noise(img: np.ndarray, gamma: np.ndarray, n: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    gamma = np.ascontiguousarray(gamma, np.float32)
    n = np.ascontiguousarray(n, np.float32)
    out = np.empty_like(img)
    lib().orc_ir_noise(_p(img), _p(gamma), _p(n), _p(out), ct.c_int64(img.size))
    return out


def census_bits(cw: int, ch: int, mode: int) -> int:
    return int(lib().orc_census_bits(cw, ch, mode))


def census(img: np.ndarray, cw: int = 7, ch: int = 9, mode: int = 0) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape
    out = np.empty((H, W), np.uint64)
    lib().orc_census(_p(img), W, H, W, cw, ch, mode, _p(out))
    return out


def popcount(v: int) -> int:
    return int(lib().orc_popcount(ct.c_uint64(int(v))))


def cost(cl: np.ndarray, cr: np.ndarray, D: int, bits: int) -> np.ndarray:
    cl = np.ascontiguousarray(cl, np.uint64)
    cr = np.ascontiguousarray(cr, np.uint64)
    H, W = cl.shape
    C = np.empty((H, W, D), np.uint16)
    lib().orc_cost(_p(cl), _p(cr), W, H, D, bits, _p(C))
    return C


def path(C: np.ndarray, dx: int, dy: int, p1: int, p2: int) -> np.ndarray:
    C = np.ascontiguousarray(C, np.uint16)
    H, W, D = C.shape
    L = np.empty((H, W, D), np.uint16)
    lib().orc_path(_p(C), W, H, D, dx, dy, p1, p2, _p(L))
    return L


def path_dirs(num_paths: int):
    out = []
    for i in range(num_paths):
        dx, dy = ct.c_int(), ct.c_int()
        lib().orc_path_dir(i, ct.byref(dx), ct.byref(dy))
        out.append((dx.value, dy.value))
    return out


def aggregate(C: np.ndarray, num_paths: int, p1: int, p2: int) -> np.ndarray:
    C = np.ascontiguousarray(C, np.uint16)
    H, W, D = C.shape
    S = np.empty((H, W, D), np.uint32)
    lib().orc_aggregate(_p(C), W, H, D, num_paths, p1, p2, _p(S))
    return S


def wta(S: np.ndarray, uniqueness_pct: int, subpixel: int = 1):
    S = np.ascontiguousarray(S, np.uint32)
    H, W, D = S.shape
    dint = np.empty((H, W), np.int32)
    s1 = np.empty((H, W), np.int32)
    s2 = np.empty((H, W), np.int32)
    vu = np.empty((H, W), np.uint8)
    dsub = np.empty((H, W), np.float64)
    lib().orc_wta(_p(S), W, H, D, uniqueness_pct, subpixel, _p(dint), _p(s1), _p(s2), _p(vu), _p(dsub))
    return dint, s1, s2, vu, dsub


def right_disp(S: np.ndarray) -> np.ndarray:
    S = np.ascontiguousarray(S, np.uint32)
    H, W, D = S.shape
    dR = np.empty((H, W), np.int32)
    lib().orc_right_disp(_p(S), W, H, D, _p(dR))
    return dR


def cost_right(cl: np.ndarray, cr: np.ndarray, D: int, bits: int) -> np.ndarray:
    cl = np.ascontiguousarray(cl, np.uint64)
    cr = np.ascontiguousarray(cr, np.uint64)
    H, W = cl.shape
    C = np.empty((H, W, D), np.uint16)
    lib().orc_cost_right(_p(cl), _p(cr), W, H, D, bits, _p(C))
    return C


def block_cost(C: np.ndarray, bw: int, bh: int) -> np.ndarray:
    C = np.ascontiguousarray(C, np.uint16)
    H, W, D = C.shape
    CB = np.empty((H, W, D), np.uint16)
    lib().orc_block_cost(_p(C), W, H, D, bw, bh, _p(CB))
    return CB


def right_disp_full(cl: np.ndarray, cr: np.ndarray, D: int, bits: int, num_paths: int, p1: int, p2: int,
                    bw: int = 1, bh: int = 1):
    cl = np.ascontiguousarray(cl, np.uint64)
    cr = np.ascontiguousarray(cr, np.uint64)
    H, W = cl.shape
    dR = np.empty((H, W), np.int32)
    lib().orc_right_disp_full(_p(cl), _p(cr), W, H, D, bits, num_paths, p1, p2, bw, bh, _p(dR))
    return dR


def lr_check(dint: np.ndarray, dR: np.ndarray, lr: int) -> np.ndarray:
    dint = np.ascontiguousarray(dint, np.int32)
    dR = np.ascontiguousarray(dR, np.int32)
    H, W = dint.shape
    out = np.empty((H, W), np.uint8)
    lib().orc_lr_check(_p(dint), _p(dR), W, H, lr, _p(out))
    return out


def median3(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    H, W = a.shape
    out = np.empty_like(a)
    lib().orc_median3(_p(a), W, H, _p(out))
    return out


def depth(disp: np.ndarray, focal_px: float, baseline_m: float) -> np.ndarray:
    disp = np.ascontiguousarray(disp, np.float64)
    out = np.empty_like(disp)
    lib().orc_depth(_p(disp), ct.c_int64(disp.size), ct.c_double(focal_px), ct.c_double(baseline_m),
                    _p(out))
    return out


# ----------------------------------------------------------------- noise generator
class OrcNoiseParams(ct.Structure):
    _fields_ = [("gain_model", ct.c_int32), ("k", ct.c_float), ("theta", ct.c_float), ("gain_sd", ct.c_float),
                ("mu", ct.c_float), ("sigma", ct.c_float), ("scale", ct.c_float),
                ("seed_lo", ct.c_uint32), ("seed_hi", ct.c_uint32), ("stream", ct.c_uint32)]


def philox4x32_10(counter, key):
    c = (ct.c_uint32 * 4)(*counter)
    k = (ct.c_uint32 * 2)(*key)
    o = (ct.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01(x: int) -> float:
    lib().orc_u01.restype = ct.c_double
    return float(lib().orc_u01(ct.c_uint32(x)))


def noise_draws(count: int, gain_model: int, k: float = 3.98, theta: float = 0.254, gain_sd: float = 0.05,
                mu: float = -0.231, sigma: float = 0.83, scale: float = 1.0, seed: int = 0, noise_stream: int = 0):
    """gamma' and n' (float32) of pixels 0..count-1, as the on-device generator defines them."""
    p = OrcNoiseParams(gain_model, k, theta, gain_sd, mu, sigma, scale, seed & 0xFFFFFFFF, seed >> 32, noise_stream)
    g = np.empty(count, np.float32)
    n = np.empty(count, np.float32)
    lib().orc_noise_draws(ct.byref(p), ct.c_int64(count), _p(g), _p(n))
    return g, n


# ----------------------------------------------------------------- rectification, registration
def rectify(img: np.ndarray, map_x: np.ndarray, map_y: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    map_x = np.ascontiguousarray(map_x, np.float32)
    map_y = np.ascontiguousarray(map_y, np.float32)
    H, W = img.shape
    oh, ow = map_x.shape
    out = np.empty((oh, ow), np.uint8)
    lib().orc_rectify(_p(img), W, W, H, _p(map_x), _p(map_y), ow, oh, _p(out))
    return out


class OrcCamera(ct.Structure):
    _fields_ = [("fx", ct.c_float), ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float)]


def register_depth(depth: np.ndarray, ir, rt, rgb, out_w: int, out_h: int) -> np.ndarray:
    """ir, rgb: (fx, fy, cx, cy); rt: 12 floats, R row-major then t."""
    depth = np.ascontiguousarray(depth, np.float32)
    H, W = depth.shape
    rt = np.ascontiguousarray(rt, np.float32).reshape(12)
    out = np.empty((out_h, out_w), np.float32)
    lib().orc_register_depth(_p(depth), W, H, ct.byref(OrcCamera(*ir)), _p(rt), ct.byref(OrcCamera(*rgb)),
                             out_w, out_h, _p(out))
    return out


@dataclass
class SGMResult:
    census_l: np.ndarray
    census_r: np.ndarray
    S: Optional[np.ndarray]
    dint: np.ndarray
    s1: np.ndarray
    s2: np.ndarray
    dright: np.ndarray
    flags: np.ndarray
    dsub: np.ndarray
    disp: np.ndarray
    depth: np.ndarray


def sgm(params: dict, left: np.ndarray, right: np.ndarray, keep_volume: bool = False) -> SGMResult:
    """The whole depth path on an already-noised pair; ``params`` as the GPU library's."""
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    H, W = left.shape
    assert params["width"] == W and params["height"] == H
    D = params["max_disp"]
    optional = {"lr_mode": 0, "block_w": 1, "block_h": 1}
    pp = OrcParams(**{k: params.get(k, optional[k]) if k in optional else params[k] for k, _ in OrcParams._fields_})
    arrs = dict(census_l=np.empty((H, W), np.uint64), census_r=np.empty((H, W), np.uint64),
                S=np.empty((H, W, D), np.uint32) if keep_volume else None,
                dint=np.empty((H, W), np.int32), s1=np.empty((H, W), np.int32),
                s2=np.empty((H, W), np.int32), dright=np.empty((H, W), np.int32),
                flags=np.empty((H, W), np.uint8), dsub=np.empty((H, W), np.float64),
                disp=np.empty((H, W), np.float64), depth=np.empty((H, W), np.float64))
    res = OrcResult(**{k: (None if v is None else v.ctypes.data) for k, v in arrs.items()})
    rc = lib().orc_sgm(ct.byref(pp), _p(left), _p(right), ct.byref(res))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return SGMResult(**arrs)
