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
                max_delta: int | None = None) -> np.ndarray:
    """uint32 [n, 64, 64] images with sparse column steps of size up to
    `delta_scale` (or exactly up to `max_delta` when given)."""
    hi = max_delta if max_delta is not None else delta_scale
    steps = rng.integers(-hi, hi + 1, size=(n, NB, NB)).astype(np.int64)
    keep = rng.random((n, NB, NB)) < density
    steps = np.where(keep, steps, 0)
    base = rng.integers(0, 4, size=(n, NB, 1)).astype(np.int64)
    rows = base + np.cumsum(steps, axis=-1)
    rows -= np.minimum(rows.min(axis=-1, keepdims=True), 0)   # keep counts >= 0
    return rows.astype(np.uint32)


def perturb(rng: np.random.Generator, images: np.ndarray, frac: float = 0.02, amount: int = 2) -> np.ndarray:
    """Copies of `images` with a few pixels raised or lowered (clutter-like)."""
    out = images.astype(np.int64).copy()
    mask = rng.random(out.shape) < frac
    out += np.where(mask, rng.integers(-amount, amount + 1, size=out.shape), 0)
    return np.maximum(out, 0).astype(np.uint32)
