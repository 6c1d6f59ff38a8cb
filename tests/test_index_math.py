"""Host checks of integer-from-float shortcuts the HIP kernels rely on (no GPU)."""
import numpy as np


def _nudge(x, ulps):
    x = np.float32(x)
    step = np.float32(np.inf) if ulps > 0 else np.float32(-np.inf)
    for _ in range(abs(ulps)):
        x = np.nextafter(x, step, dtype=np.float32)
    return x


def test_rectangle_row_from_reciprocal():
    # instance emission: row = trunc(pos * rcp(rw) + 1/128) for a hit position pos < 64 in a
    # tile rectangle of width rw <= 64; exact for a reciprocal off by up to two ulps, with
    # the fused multiply-add rounded once or the product rounded first
    for rw in range(1, 65):
        r0 = np.float32(1.0) / np.float32(rw)
        for ulps in range(-2, 3):
            r = _nudge(r0, ulps)
            for pos in range(64):
                fused = np.float32(np.float64(pos) * np.float64(r) + 1.0 / 128.0)
                split = np.float32(np.float32(np.float32(pos) * r) + np.float32(1.0 / 128.0))
                assert int(fused) == pos // rw and int(split) == pos // rw, (rw, ulps, pos)
