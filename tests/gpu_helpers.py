"""Device-buffer helpers for the GPU tests (torch is used for memory only)."""
import numpy as np

GUARD = 256  # bytes of sentinel on both sides of every output buffer


def torch():
    import torch as t
    return t


def to_dev(a: np.ndarray):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).cuda()


class Guarded:
    """A device buffer of `nbytes` with sentinel guard bands, so that writes
    outside the output and unwritten output bytes are both visible."""

    def __init__(self, nbytes: int, fill: int = 0xA7, offset: int = 0):
        t = torch()
        self.nbytes = nbytes
        self.offset = offset
        self.fill = fill
        self.raw = t.full((nbytes + 2 * GUARD + offset,), fill, dtype=t.uint8, device="cuda")

    @property
    def ptr(self) -> int:
        return self.raw.data_ptr() + GUARD + self.offset

    def host(self) -> np.ndarray:
        return self.raw.cpu().numpy()[GUARD + self.offset:GUARD + self.offset + self.nbytes]

    def guards_intact(self) -> bool:
        a = self.raw.cpu().numpy()
        lo = a[:GUARD + self.offset]
        hi = a[GUARD + self.offset + self.nbytes:]
        return bool((lo == self.fill).all() and (hi == self.fill).all())


def plane_dev(img: np.ndarray, offset: int = 0):
    """Upload a [h, stride] uint8 plane, optionally at a byte offset from an
    aligned allocation (to exercise unaligned loads). Returns (tensor, ptr)."""
    t = torch()
    flat = np.zeros(img.size + offset + 64, np.uint8)
    flat[offset:offset + img.size] = img.reshape(-1)
    d = t.from_numpy(flat).cuda()
    return d, d.data_ptr() + offset


def sync():
    torch().cuda.synchronize()
