"""Seeded synthetic 64x64 count images for exercising the distance search at
large sizes without generating descriptors first.

Each row is a non-negative step function of the column index (what a RICI row
looks like: counts change by small even steps where a circle crosses a
surface), built from sparse random column deltas.  `delta_scale` controls how
large the steps can be, so tests can target every arithmetic range of the
search (|D| <= 11, 11 < |D| <= 127, |D| > 127).
"""

from __future__ import annotations

import numpy as np

NB = 64


def step_images(rng: np.random.Generator, n: int, density: float = 0.08, delta_scale: int = 2,
                max_delta: int | None = None, chunk: int = 16384) -> np.ndarray:
    """uint32 [n, 64, 64] images with sparse column steps of size up to
    `delta_scale` (or exactly up to `max_delta` when given).  Generated in
    chunks of `chunk` images with narrow integer types, so that haystacks of
    hundreds of thousands of images take seconds."""
    hi = max_delta if max_delta is not None else delta_scale
    sdt = np.int8 if hi <= 127 else np.int16
    out = np.empty((n, NB, NB), dtype=np.uint32)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        steps = rng.integers(-hi, hi + 1, size=(m, NB, NB), dtype=sdt)
        steps[rng.random((m, NB, NB), dtype=np.float32) >= density] = 0
        base = rng.integers(0, 4, size=(m, NB, 1), dtype=np.int32)
        rows = np.cumsum(steps, axis=-1, dtype=np.int32)
        rows += base
        rows -= np.minimum(rows.min(axis=-1, keepdims=True), 0)   # keep counts >= 0
        out[a:a + m] = rows
    return out


def perturb(rng: np.random.Generator, images: np.ndarray, frac: float = 0.02, amount: int = 2) -> np.ndarray:
    """Copies of `images` with a few pixels raised or lowered (clutter-like)."""
    out = images.astype(np.int64).copy()
    mask = rng.random(out.shape) < frac
    out += np.where(mask, rng.integers(-amount, amount + 1, size=out.shape), 0)
    return np.maximum(out, 0).astype(np.uint32)
