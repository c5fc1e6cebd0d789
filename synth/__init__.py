"""Seeded synthetic workloads for the block codec (inputs only).

This module holds no codec arithmetic: it makes the uint8 planes, the
quantisation tables, the image-size draws and the request traces that both
the oracle and the HIP library are fed. The same seed always gives the same
bytes, whatever the thread count.

The paper measures on 45 public 512x512 greyscale images and on the Lena
image (Section 3); neither is in this environment, so seeded "blob fields"
stand in for them: 20 isotropic Gaussian blobs (sigma 8..64 px, amplitude
0..255) plus uniform integer noise, clipped to [0, 255] (see ``synth.c``).

Workloads:
  * ``plane(w, h, seed)``                 one blob-field image
  * ``batch(sizes, seeds)``               many images packed in one buffer
  * ``video_frame(f, ...)``               4:2:0 frames of a moving field
  * ``qtable(base, s, step)``             Q_ij = base + step * s * (i + j)
  * ``loguniform_sides(...)``             multiples of 8, log-uniform
  * ``serving_trace(rate, seconds, seed)`` Poisson request stream
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lock = threading.Lock()
_lib = None
NBLOBS = 20


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _L():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_uint64, ctypes.c_double)
            L.synth_blob_plane.argtypes = [P, i64, i32, i32, u64, i32, i32, i32, f64, i32, i32,
                                           u64, i32, i32]
            L.synth_blob_batch.argtypes = [P, P, P, P, P, P, i32, i32, i32, i32]
            L.synth_blob_field.argtypes = [P, i32, i32, u64, i32, i32, i32, f64, i32]
            L.synth_window.argtypes = [P, i32, i32, i32, P, i64, i32, i32, u64, i32, i32]
            _lib = L
    return _lib


def _threads(n=None) -> int:
    if n:
        return int(n)
    return max(1, min(16, os.cpu_count() or 1))


def plane(w: int, h: int, seed: int, noise: int = 8, stride: int | None = None,
          out: np.ndarray | None = None, threads: int | None = None,
          nblobs: int = NBLOBS) -> np.ndarray:
    """One w x h blob-field image as uint8 [h, stride] (columns >= w are 0)."""
    stride = w if stride is None else stride
    if out is None:
        out = np.zeros((h, stride), np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.shape[1] >= w
    _L().synth_blob_plane(out.ctypes.data, out.strides[0], w, h, seed, nblobs, w, h, 1.0, 0, 0,
                          seed ^ 0xA5A5A5A55A5A5A5A, noise, _threads(threads))
    return out


def textured(w: int, h: int, seed: int, stride: int | None = None) -> np.ndarray:
    """A test image that exercises every coefficient and the whole pixel range
    at any size: half a two-blob field plus half a horizontal ramp over
    [0, 255], under strong noise (+-80), clipped. (The 20-blob recipe
    saturates small images to a constant.)"""
    stride = w if stride is None else stride
    base = plane(w, h, seed, noise=0, nblobs=2).astype(np.int64)
    ramp = (np.arange(w, dtype=np.int64) * 255 // max(1, w - 1))[None, :]
    noise = np.random.default_rng([seed, 99]).integers(-80, 81, size=(h, w))
    out = np.zeros((h, stride), np.uint8)
    out[:, :w] = np.clip(base // 2 + ramp // 2 + noise, 0, 255)
    return out


def batch(sizes, seeds, noise: int = 8, align: int = 256, threads: int | None = None):
    """Many images in one buffer. Returns (buf uint8[total], offsets int64[n],
    strides int64[n]); image i is buf[off[i]:] viewed as [h_i, stride_i].
    Rows are packed (stride = w); image starts are aligned to ``align`` bytes."""
    sizes = np.asarray(sizes, np.int64).reshape(-1, 2)
    n = sizes.shape[0]
    w = np.ascontiguousarray(sizes[:, 0].astype(np.int32))
    h = np.ascontiguousarray(sizes[:, 1].astype(np.int32))
    strides = w.astype(np.int64)
    nbytes = strides * h
    padded = (nbytes + align - 1) // align * align
    off = np.zeros(n, np.int64)
    if n > 1:
        off[1:] = np.cumsum(padded)[:-1]
    total = int(padded.sum()) if n else 0
    buf = np.zeros(max(total, 1), np.uint8)
    sd = np.ascontiguousarray(np.asarray(seeds, np.uint64))
    _L().synth_blob_batch(buf.ctypes.data, off.ctypes.data, strides.ctypes.data, w.ctypes.data,
                          h.ctypes.data, sd.ctypes.data, n, NBLOBS, noise, _threads(threads))
    return buf, off, strides


def batch_view(buf: np.ndarray, off, strides, sizes, i: int) -> np.ndarray:
    w, h = int(sizes[i][0]), int(sizes[i][1])
    s = int(strides[i])
    return buf[int(off[i]):int(off[i]) + s * h].reshape(h, s)[:, :w]


# ---- quantisation tables and scale draws ---------------------------------

def qtable(base: int, s: int, step: int = 1) -> np.ndarray:
    """Q_ij = base + step * s * (i + j), uint16 [8, 8]."""
    i = np.arange(8)[:, None]
    j = np.arange(8)[None, :]
    return (base + step * s * (i + j)).astype(np.uint16)


def scale_for(seed: int) -> int:
    """s uniform in {1..8}, from the image's own seed stream."""
    return int(np.random.default_rng([int(seed), 7]).integers(1, 9))


def loguniform_sides(n: int, lo: int, hi: int, rng: np.random.Generator) -> np.ndarray:
    """Multiples of 8, log-uniform in [lo, hi]: 8 * round(exp(U(ln(lo/8), ln(hi/8))))."""
    u = rng.uniform(np.log(lo / 8), np.log(hi / 8), size=n)
    return (8 * np.rint(np.exp(u))).astype(np.int64).clip(lo, hi)


# ---- named workloads ------------------------------------------------------

def single_image(seed: int = 1, w: int = 512, h: int = 512) -> np.ndarray:
    """The paper-sized 512 x 512 greyscale image (seed 1 by default)."""
    return plane(w, h, seed)


def large_batch_spec(n: int = 64, side: int = 4096, seed0: int = 1000):
    """n images of side x side, seeds seed0 + i, per-image Q = 1 + s (i + j)."""
    seeds = [seed0 + i for i in range(n)]
    sizes = [(side, side)] * n
    qs = [qtable(1, scale_for(sd)) for sd in seeds]
    return sizes, seeds, qs


def ragged_batch_spec(n: int = 10000, lo: int = 64, hi: int = 2048, seed: int = 3,
                      seed0: int = 3000):
    """n images with independent log-uniform sides in [lo, hi] (multiples of 8)."""
    rng = np.random.default_rng(seed)
    w = loguniform_sides(n, lo, hi, rng)
    h = loguniform_sides(n, lo, hi, rng)
    seeds = [seed0 + i for i in range(n)]
    sizes = list(zip(w.tolist(), h.tolist()))
    qs = [qtable(1, scale_for(sd)) for sd in seeds]
    return sizes, seeds, qs


class Video420:
    """4:2:0 frames (Y w x h, Cb/Cr w/2 x h/2) of one seeded blob field that
    moves by a random walk of integer steps in [-8, 8] per frame; chroma is
    the half-resolution view of the same field with half the motion. Noise
    is +-4 per sample, independent per frame and plane."""

    MARGIN = 256

    def __init__(self, w: int = 3840, h: int = 2160, frames: int = 256, seed: int = 4):
        self.w, self.h, self.frames, self.seed = w, h, frames, seed
        rng = np.random.default_rng([seed, 1])
        steps = rng.integers(-8, 9, size=(frames, 2))
        steps[0] = 0
        pos = np.cumsum(steps, axis=0).clip(-self.MARGIN, self.MARGIN)
        self.offsets = pos + self.MARGIN
        srng = np.random.default_rng([seed, 2])
        self.s_luma = srng.integers(1, 9, size=frames)
        self.s_chroma = srng.integers(1, 9, size=frames)

    def qtables(self, f: int):
        """(Q luma, Q chroma): 64 + s_Y (i + j) and 64 + 2 s_C (i + j)."""
        return qtable(64, int(self.s_luma[f])), qtable(64, int(self.s_chroma[f]), step=2)

    def _plane_params(self, f: int):
        w, h, M = self.w, self.h, self.MARGIN
        ox, oy = int(self.offsets[f][0]), int(self.offsets[f][1])
        out = []
        for p in range(3):
            sc, cw, ch = (1.0, w, h) if p == 0 else (0.5, w // 2, h // 2)
            px, py = (ox, oy) if p == 0 else (ox // 2, oy // 2)
            blob_seed = self.seed * 1000003 + (0 if p == 0 else 17)
            noise_seed = (self.seed << 40) ^ (f << 4) ^ p ^ 0x5851F42D4C957F2D
            out.append((sc, cw, ch, px, py, blob_seed, noise_seed))
        return out

    def _fields(self, threads):
        """The rounded, noise-free field of the whole canvas (luma and the
        half-resolution chroma view), computed once per sequence."""
        if getattr(self, "_canvas", None) is None:
            w, h, M = self.w, self.h, self.MARGIN
            fw, fh = w + 2 * M, h + 2 * M
            L = _L()
            canv = []
            for p, (sc, cw, ch) in enumerate([(1.0, fw, fh), (0.5, fw // 2, fh // 2)]):
                a = np.zeros((ch, cw), np.int16)
                seed = self.seed * 1000003 + (0 if p == 0 else 17)
                L.synth_blob_field(a.ctypes.data, cw, ch, seed, NBLOBS, fw, fh, sc, _threads(threads))
                canv.append(a)
            self._canvas = canv
        return self._canvas

    def frame(self, f: int, out=None, threads: int | None = None):
        """Returns (Y, Cb, Cr) uint8 planes of frame f (windows of the canvas
        field plus fresh noise)."""
        w, h = self.w, self.h
        if out is None:
            out = (np.zeros((h, w), np.uint8), np.zeros((h // 2, w // 2), np.uint8),
                   np.zeros((h // 2, w // 2), np.uint8))
        canv = self._fields(threads)
        L = _L()
        for p, (sc, cw, ch, px, py, _, noise_seed) in enumerate(self._plane_params(f)):
            c = canv[0 if p == 0 else 1]
            arr = out[p]
            L.synth_window(c.ctypes.data, c.shape[1], px, py, arr.ctypes.data, arr.strides[0], cw, ch,
                           noise_seed, 4, _threads(threads))
        return out

    def frame_direct(self, f: int, threads: int | None = None):
        """The same frame evaluated blob by blob at its own window (slow; used
        to check the canvas path)."""
        w, h, M = self.w, self.h, self.MARGIN
        fw, fh = w + 2 * M, h + 2 * M
        out = (np.zeros((h, w), np.uint8), np.zeros((h // 2, w // 2), np.uint8),
               np.zeros((h // 2, w // 2), np.uint8))
        L = _L()
        for p, (sc, cw, ch, px, py, blob_seed, noise_seed) in enumerate(self._plane_params(f)):
            arr = out[p]
            L.synth_blob_plane(arr.ctypes.data, arr.strides[0], cw, ch, blob_seed, NBLOBS, fw, fh,
                               sc, px, py, noise_seed, 4, _threads(threads))
        return out


def serving_trace(rate: float, seconds: float, seed: int = 5, lo: int = 32, hi: int = 8192,
                  max_aspect: float = 4.0):
    """Poisson arrivals at `rate` per second for `seconds`. Each request is
    encode (0) or decode (1) with p = 1/2, with sides log-uniform multiples of
    8 in [lo, hi] and aspect ratio <= max_aspect (resampled otherwise), and a
    scale s in {1..8}. Returns a dict of numpy arrays."""
    rng = np.random.default_rng([seed, int(rate)])
    n_est = int(rate * seconds * 1.3 + 64)
    gaps = rng.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < seconds:
        gaps = rng.exponential(1.0 / rate, size=n_est)
        t = np.concatenate([t, t[-1] + np.cumsum(gaps)])
    t = t[t < seconds]
    n = t.size
    op = rng.integers(0, 2, size=n)
    w = np.zeros(n, np.int64)
    h = np.zeros(n, np.int64)
    todo = np.arange(n)
    while todo.size:
        ww = loguniform_sides(todo.size, lo, hi, rng)
        hh = loguniform_sides(todo.size, lo, hi, rng)
        ok = np.maximum(ww, hh) <= max_aspect * np.minimum(ww, hh)
        w[todo[ok]] = ww[ok]
        h[todo[ok]] = hh[ok]
        todo = todo[~ok]
    s = rng.integers(1, 9, size=n)
    return {"t": t, "op": op, "w": w, "h": h, "s": s}
