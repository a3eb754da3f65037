"""FP64 rescale of projected float images to 8 or 16 bits, and the RGB
composite.  Test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline use this package.

Paper, Section 2 (the three rescaling paragraphs):

1. the float image of each component is rescaled so that its page-wide
   minimum maps to 0 and its maximum to 255;
2. the minimum and maximum of the training pixels' projections map to 0 and
   255 and the whole image is rescaled on that range;
3. the 0.01, 0.1, 1 or 5 percentiles of the data are taken out and the rest
   is rescaled the same way.

Readings (the paper states none of these): the map is
q = floor(255 (y - a) / (b - a) + 1/2) clamped to [0, 255] (round half up);
q = 0 when b = a; in modes 2 and 3 values outside [a, b] clamp to 0 or 255;
mode 3 takes a and b as the p-th and (100-p)-th percentiles with NumPy's
linear interpolation.

The 16-bit output (paper Section 2, the C implementation writes 8- and
16-bit images) is the same map with 65535 levels.  The colour image (paper
Section 2: three grayscale images combined as red, green and blue; Section
4: one image may fill two channels) interleaves three 8-bit planes pixel
by pixel; a missing channel is zero.

Pinned by tests/test_oracle_cva.py: q(argmin) = 0 and q(argmax) = 255
exactly, q is monotone in y, invariant to positive scaling and shift of y,
and a sign flip maps q to 255 - q up to one grey level; a brute-force
per-element loop gives the same bytes, for 255 and for 65535 levels; the
percentiles of a shuffled arithmetic sequence are known in closed form, the
0-th percentile is the minimum and a percentile that falls between two
order statistics interpolates them; the 16-bit image divided by 257 is the
8-bit one within a level; the colour image holds each plane in its channel.
"""
from __future__ import annotations

import numpy as np


def _quantise(y: np.ndarray, a: np.ndarray, b: np.ndarray, levels: int = 255) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(y.shape, dtype=np.uint16 if levels > 255 else np.uint8)
    for j in range(y.shape[1]):
        if b[j] > a[j]:
            t = np.floor(levels * (y[:, j] - a[j]) / (b[j] - a[j]) + 0.5)
            out[:, j] = np.clip(t, 0, levels).astype(out.dtype)
    return out


def stretch_minmax(y: np.ndarray, levels: int = 255):
    """Mode 1: page-wide min-max.  y is P x C; returns (q, a, b)."""
    y = np.asarray(y, dtype=np.float64)
    a = y.min(axis=0)
    b = y.max(axis=0)
    return _quantise(y, a, b, levels), a, b


def stretch_training_range(y: np.ndarray, y_train: np.ndarray, levels: int = 255):
    """Mode 2: the training pixels' projected range maps to 0..levels."""
    y_train = np.asarray(y_train, dtype=np.float64)
    a = y_train.min(axis=0)
    b = y_train.max(axis=0)
    return _quantise(y, a, b, levels), a, b


def stretch_percentile(y: np.ndarray, pct: float, levels: int = 255):
    """Mode 3: clip the lower and upper pct percent, then rescale."""
    y = np.asarray(y, dtype=np.float64)
    a = np.percentile(y, pct, axis=0, method="linear")
    b = np.percentile(y, 100.0 - pct, axis=0, method="linear")
    return _quantise(y, a, b, levels), a, b


def compose_rgb(r, g, b) -> np.ndarray:
    """Planes of one shape (None = all zero) -> shape + (3,) uint8."""
    planes = [p for p in (r, g, b) if p is not None]
    shape = np.shape(planes[0])
    out = np.zeros(tuple(shape) + (3,), dtype=np.uint8)
    for c, p in enumerate((r, g, b)):
        if p is not None:
            out[..., c] = np.asarray(p, dtype=np.uint8)
    return out
