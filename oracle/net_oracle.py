"""CPU oracle of the learned surrogate (a small convolutional net on 2-path SGM features).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  Plain numpy in fp64;
the features and the final combination can instead be evaluated in float32, the
precision in which the kernels take the decisions that follow them (a bf16
rounding, a validity test).

The net (not part of the paper; it stands in for six of the eight SGM paths):
four 3x3 convolutions with zero padding, 4 -> 32 -> 32 -> 32 -> 2 channels, ReLU
after the first three.  Output channel 0 is a disparity residual added to the
2-path sub-pixel disparity, channel 1 a validity logit.  Tensors are NHWC;
weights are [3, 3, Cin, Cout] with out(y, x) = sum_{ky,kx} in(y+ky-1, x+kx-1) w[ky,kx].

Loss: mean over pixels where the 8-path result is valid of |r - t| (L1 on the
residual) plus the mean over all pixels of the binary cross-entropy of the logit
against the 8-path validity.  Optimiser: Adam (Kingma & Ba 2015) with bias
correction.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((4, 32), (32, 32), (32, 32), (32, 2))
NUM_PARAMS = sum(9 * ci * co + co for ci, co in LAYERS)  # 20258


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int):
    """He-uniform weights, zero biases (deterministic)."""
    rng = np.random.default_rng(seed)
    ps = []
    for ci, co in LAYERS:
        bound = np.sqrt(6.0 / (9 * ci))
        ps.append((rng.uniform(-bound, bound, (3, 3, ci, co)), np.zeros(co)))
    return ps


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(v: np.ndarray):
    out, o = [], 0
    for ci, co in LAYERS:
        n = 9 * ci * co
        w = v[o:o + n].reshape(3, 3, ci, co)
        o += n
        b = v[o:o + co]
        o += co
        out.append((w.copy(), b.copy()))
    return out


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((B, H, W, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + H, kx:kx + W, :] @ w[ky, kx]
    return out + b


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dout: np.ndarray):
    """Gradients of conv3x3 with respect to its input, weights and bias."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + H, kx:kx + W, :]
            dw[ky, kx] = np.einsum("bhwc,bhwo->co", patch, dout)
            dxp[:, ky:ky + H, kx:kx + W, :] += dout @ w[ky, kx].T
    db = dout.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dw, db


def forward(params, feats: np.ndarray, round_bf16: bool = False):
    """Returns (output [B,H,W,2], list of layer inputs).  With round_bf16 the
    weights and every inter-layer activation are rounded to bf16 (as the GPU
    stores them) while all arithmetic stays fp64."""
    acts = []
    a = bf16_round(feats) if round_bf16 else feats
    for i, (w, b) in enumerate(params):
        acts.append(a)
        wq = bf16_round(w) if round_bf16 else w
        z = conv3x3(a, wq, b)
        if i < len(params) - 1:
            a = np.maximum(z, 0.0)
            if round_bf16:
                a = bf16_round(a)
        else:
            a = z
    return a, acts


def loss(out: np.ndarray, t_res: np.ndarray, t_valid: np.ndarray):
    """(total, l1, bce) and the gradient of total with respect to out."""
    r, z = out[..., 0], out[..., 1]
    v = t_valid.astype(np.float64)
    nv = max(v.sum(), 1.0)
    n = v.size
    l1 = np.sum(np.abs(r - t_res) * v) / nv
    # binary cross-entropy with logits, numerically stable form
    bce = np.sum(np.maximum(z, 0) - z * v + np.log1p(np.exp(-np.abs(z)))) / n
    g = np.zeros_like(out)
    g[..., 0] = np.sign(r - t_res) * v / nv
    g[..., 1] = (1.0 / (1.0 + np.exp(-z)) - v) / n
    return l1 + bce, l1, bce, g


def backward(params, acts, dout: np.ndarray):
    grads = [None] * len(params)
    d = dout
    for i in range(len(params) - 1, -1, -1):
        w, _ = params[i]
        dx, dw, db = conv3x3_backward(acts[i], w, d)
        grads[i] = (dw, db)
        if i > 0:
            d = dx * (acts[i] > 0)  # ReLU derivative of the previous layer
    return grads


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update of flat arrays (in place); step counts from 1."""
    m[:] = b1 * m + (1 - b1) * g
    v[:] = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p -= lr * mh / (np.sqrt(vh) + eps)


def features(ir: np.ndarray, s1: np.ndarray, s2: np.ndarray, dint: np.ndarray, max_disp: int, smax: float,
             dtype=np.float64):
    """The net's four input channels from a 2-path result: IR/255, S1/Smax, S2/Smax
    (1 where no second candidate exists) and d*/D.  Each channel is one quotient;
    with dtype=np.float32 it is the correctly rounded float32 quotient, so that the
    bf16 rounding of a feature (a quantisation decision) is taken from the same
    float32 value the kernel rounds."""
    f = lambda a: np.asarray(a).astype(dtype)
    s2f = np.minimum(np.where(np.asarray(s2) < 0, smax, s2), smax)
    sm = dtype(smax)
    return np.stack([f(ir) / dtype(255.0), f(s1) / sm, f(s2f) / sm, f(dint) / dtype(max_disp)], axis=-1)


def combine(d2_sub: np.ndarray, out: np.ndarray, dtype=np.float64) -> np.ndarray:
    """Disparity of the learned form before the median: d2 + residual where the
    logit is positive and the sum is positive, else 0 (invalid).  With
    dtype=np.float32 the sum and the validity decision are taken in float32 (the
    kernel's precision) from float32 inputs."""
    d2, r, z = (np.asarray(a).astype(dtype) for a in (d2_sub, out[..., 0], out[..., 1]))
    d = d2 + r
    return np.where((z > 0) & (d > 0), d, dtype(0.0))
