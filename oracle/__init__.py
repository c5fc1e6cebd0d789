"""CPU oracle for the 14-addition approximate-DCT block codec.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product
library never loads it, and this package imports nothing from the product.

Two independent oracles live here:

* ``tdct_oracle.c`` (loaded through ctypes): the integer codec as the plain
  dense definition -- Y = T X T^t on level-shifted 8x8 blocks (matrix T of
  Section 2, 2-D block transform of Section 3), the D^2 fold of Section 2
  as an exact integer scale, round-half-away quantisation, zonal zigzag
  retention (Section 3) and the reconstruction T^t W' T / 64 with
  round-half-up and clamp.
* ``float_*`` (numpy, float64): the paper's own formulation with the scaled
  orthogonal matrix C^ = D T (Section 2): C = C^ X C^t, zonal mask,
  X~ = C^t C C^ (Section 3). It is used on small inputs to tie the integer
  conventions to the paper's real-valued transform.

Every function takes host numpy arrays and returns host numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_default = None


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the C oracle with gcc (``oracle/liboracle.so`` by default)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _nblk(w: int, h: int) -> int:
    return (w // 8) * (h // 8)


def _split(nblk: int, threads: int):
    threads = max(1, min(threads, nblk)) if nblk else 1
    step = (nblk + threads - 1) // threads if nblk else 0
    return [(b0, min(step, nblk - b0)) for b0 in range(0, nblk, step)] if nblk else []


def _run(fn, nblk: int, threads: int):
    parts = _split(nblk, threads)
    if threads <= 1 or len(parts) <= 1:
        for b0, n in parts:
            fn(b0, n)
        return
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        list(ex.map(lambda p: fn(*p), parts))


def _plane_args(img: np.ndarray):
    assert img.dtype == np.uint8 and img.ndim == 2
    return img.shape[0], img.strides[0]


def _qtab(Q) -> np.ndarray:
    Qa = np.ascontiguousarray(np.asarray(Q, np.uint16).reshape(64))
    assert Qa.min() >= 1
    return Qa


class Oracle:
    """The C oracle behind one shared library (the committed one, or a
    variant compiled from edited source by the tests that check the pins)."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_get_T.argtypes = [P]
        L.oracle_get_wscale.argtypes = [P]
        L.oracle_get_zigzag.argtypes = [P]
        L.oracle_round_div.argtypes = [i64, i64]
        L.oracle_round_div.restype = i64
        L.oracle_round_div_array.argtypes = [P, i64, i64, P]
        L.oracle_apply_T.argtypes = [P, P, i32]
        L.oracle_forward_block.argtypes = [P, P]
        L.oracle_inverse_block.argtypes = [P, P]
        L.oracle_forward.argtypes = [P, i64, i32, i32, i64, i64, P]
        L.oracle_quantise.argtypes = [P, i64, i32, i32, P, i32, i64, i64, P]
        L.oracle_quantise_i8_zigzag.argtypes = [P, i64, i32, i32, P, i64, i64, P]
        L.oracle_inverse.argtypes = [P, P, i32, i32, i64, i64, P, i64]
        self.L = L

    # -- constants
    def T(self) -> np.ndarray:
        out = np.zeros(64, np.int32)
        self.L.oracle_get_T(_ptr(out))
        return out.reshape(8, 8)

    def wscale(self) -> np.ndarray:
        """64 * d_i^2 * d_j^2 as exact integers, [8, 8]."""
        out = np.zeros(64, np.int32)
        self.L.oracle_get_wscale(_ptr(out))
        return out.reshape(8, 8)

    def zigzag_order(self) -> np.ndarray:
        """order[rank] = natural index 8*i + j."""
        out = np.zeros(64, np.int32)
        self.L.oracle_get_zigzag(_ptr(out))
        return out

    def zigzag_rank(self) -> np.ndarray:
        order = self.zigzag_order()
        rank = np.empty(64, np.int32)
        rank[order] = np.arange(64, dtype=np.int32)
        return rank

    def round_div(self, W: int, Q: int) -> int:
        return int(self.L.oracle_round_div(int(W), int(Q)))

    def round_div_array(self, W, Q: int) -> np.ndarray:
        Wa = np.ascontiguousarray(np.asarray(W, np.int64).reshape(-1))
        out = np.zeros_like(Wa)
        self.L.oracle_round_div_array(_ptr(Wa), Wa.size, int(Q), _ptr(out))
        return out

    def apply_T(self, x, transpose: bool = False) -> np.ndarray:
        xi = np.ascontiguousarray(np.asarray(x, np.int64).reshape(8))
        y = np.zeros(8, np.int64)
        self.L.oracle_apply_T(_ptr(xi), _ptr(y), int(transpose))
        return y

    def forward_block(self, X) -> np.ndarray:
        """Y = T X T^t for an arbitrary integer 8x8 block (no level shift)."""
        Xi = np.ascontiguousarray(np.asarray(X, np.int64).reshape(64))
        Y = np.zeros(64, np.int64)
        self.L.oracle_forward_block(_ptr(Xi), _ptr(Y))
        return Y.reshape(8, 8)

    def inverse_block(self, W) -> np.ndarray:
        """S = T^t W T for an arbitrary integer 8x8 block (no 1/64 scale)."""
        Wi = np.ascontiguousarray(np.asarray(W, np.int64).reshape(64))
        S = np.zeros(64, np.int64)
        self.L.oracle_inverse_block(_ptr(Wi), _ptr(S))
        return S.reshape(8, 8)

    # -- plane-level codec
    def forward(self, img: np.ndarray, w: int | None = None, threads: int = 1) -> np.ndarray:
        """Unscaled Y = T (X - 128) T^t, int32 [nblk, 64] in raster block order."""
        h, stride = _plane_args(img)
        w = img.shape[1] if w is None else w
        nblk = _nblk(w, h)
        out = np.zeros((nblk, 64), np.int32)
        L = self.L
        _run(lambda b0, n: L.oracle_forward(_ptr(img), stride, w, h, b0, n, _ptr(out)), nblk, threads)
        return out

    def quantise(self, img: np.ndarray, Q, keep: int = 64, w: int | None = None,
                 threads: int = 1) -> np.ndarray:
        """Fused forward + quantise, int16 [nblk, 64], natural (i, j) order."""
        h, stride = _plane_args(img)
        w = img.shape[1] if w is None else w
        nblk = _nblk(w, h)
        Qa = _qtab(Q)
        out = np.zeros((nblk, 64), np.int16)
        L = self.L
        _run(lambda b0, n: L.oracle_quantise(_ptr(img), stride, w, h, _ptr(Qa), keep, b0, n,
                                             _ptr(out)), nblk, threads)
        return out

    def quantise_i8_zigzag(self, img: np.ndarray, Q, w: int | None = None,
                           threads: int = 1) -> np.ndarray:
        """Forward + quantise, saturated to int8, stored in zigzag order [nblk, 64]."""
        h, stride = _plane_args(img)
        w = img.shape[1] if w is None else w
        nblk = _nblk(w, h)
        Qa = _qtab(Q)
        out = np.zeros((nblk, 64), np.int8)
        L = self.L
        _run(lambda b0, n: L.oracle_quantise_i8_zigzag(_ptr(img), stride, w, h, _ptr(Qa), b0, n,
                                                       _ptr(out)), nblk, threads)
        return out

    def inverse(self, q: np.ndarray, Q, w: int, h: int, dst_stride: int | None = None,
                threads: int = 1) -> np.ndarray:
        """Fused dequantise + inverse: uint8 plane [h, dst_stride] (first w columns written)."""
        qa = np.ascontiguousarray(np.asarray(q, np.int16).reshape(-1, 64))
        nblk = _nblk(w, h)
        assert qa.shape[0] >= nblk
        Qa = _qtab(Q)
        dst_stride = w if dst_stride is None else dst_stride
        out = np.zeros((h, dst_stride), np.uint8)
        L = self.L
        _run(lambda b0, n: L.oracle_inverse(_ptr(qa), _ptr(Qa), w, h, b0, n, _ptr(out), dst_stride),
             nblk, threads)
        return out

    def roundtrip(self, img: np.ndarray, Q, keep: int = 64, w: int | None = None,
                  threads: int = 1):
        """Encode then decode; returns (q, reconstruction)."""
        h = img.shape[0]
        w = img.shape[1] if w is None else w
        q = self.quantise(img, Q, keep, w=w, threads=threads)
        return q, self.inverse(q, Q, w, h, threads=threads)

    # -- the paper's float64 formulation (uses this oracle's T and zigzag)
    def float_Chat(self) -> np.ndarray:
        """C^ = D T (Section 2), float64, with the printed D."""
        return paper_D() @ self.T().astype(np.float64)

    def float_zonal_mask(self, r: int) -> np.ndarray:
        """1 where the zigzag rank is < r (Section 3), [8, 8]."""
        return (self.zigzag_rank() < r).astype(np.float64).reshape(8, 8)

    def float_block_roundtrip(self, X: np.ndarray, r: int) -> np.ndarray:
        """X~ = C^t (mask o (C^ X C^t)) C^ for one level-shifted block, float64."""
        C = self.float_Chat()
        coef = C @ np.asarray(X, np.float64) @ C.T
        return C.T @ (coef * self.float_zonal_mask(r)) @ C

    sse = staticmethod(lambda a, b: sse(a, b))
    psnr = staticmethod(lambda a, b: psnr(a, b))
    paper_D = staticmethod(lambda: paper_D())


def default() -> Oracle:
    global _default
    with _lock:
        if _default is None:
            _default = Oracle(build())
    return _default


def lib():
    return default().L


# Module-level API bound to the committed oracle.
def T(): return default().T()
def wscale(): return default().wscale()
def zigzag_order(): return default().zigzag_order()
def zigzag_rank(): return default().zigzag_rank()
def round_div(W, Q): return default().round_div(W, Q)
def round_div_array(W, Q): return default().round_div_array(W, Q)
def apply_T(x, transpose=False): return default().apply_T(x, transpose)
def forward_block(X): return default().forward_block(X)
def inverse_block(W): return default().inverse_block(W)
def forward(img, w=None, threads=1): return default().forward(img, w, threads)
def quantise(img, Q, keep=64, w=None, threads=1): return default().quantise(img, Q, keep, w, threads)
def quantise_i8_zigzag(img, Q, w=None, threads=1): return default().quantise_i8_zigzag(img, Q, w, threads)
def inverse(q, Q, w, h, dst_stride=None, threads=1): return default().inverse(q, Q, w, h, dst_stride, threads)
def roundtrip(img, Q, keep=64, w=None, threads=1): return default().roundtrip(img, Q, keep, w, threads)
def float_Chat(): return default().float_Chat()
def float_zonal_mask(r): return default().float_zonal_mask(r)
def float_block_roundtrip(X, r): return default().float_block_roundtrip(X, r)


def sse(a: np.ndarray, b: np.ndarray) -> int:
    """Exact sum of squared differences of two uint8 planes."""
    d = a.astype(np.int64) - b.astype(np.int64)
    return int((d * d).sum())


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    """PSNR = 10 log10(255^2 / MSE) in double (Section 3's figure of merit)."""
    mse = sse(a, b) / float(a.size)
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


# ---- float64 helpers ------------------------------------------------------

def paper_D() -> np.ndarray:
    """D = diag(1/sqrt 8, 1/sqrt 2, 1/2, 1/sqrt 2, 1/sqrt 8, 1/sqrt 2, 1/2, 1/sqrt 2)
    as printed in Section 2."""
    return np.diag([1 / np.sqrt(8), 1 / np.sqrt(2), 0.5, 1 / np.sqrt(2),
                    1 / np.sqrt(8), 1 / np.sqrt(2), 0.5, 1 / np.sqrt(2)])


def dct_matrix() -> np.ndarray:
    """Orthonormal 8-point DCT-II (the transform the paper approximates, Section 1)."""
    k = np.arange(8)[:, None]
    n = np.arange(8)[None, :]
    M = np.cos((2 * n + 1) * k * np.pi / 16) * np.sqrt(2 / 8)
    M[0, :] = np.sqrt(1 / 8)
    return M
