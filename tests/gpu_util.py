"""Helpers for the GPU parity tests: numpy <-> torch device tensors and the
comparison of GPU images with the oracle's images outside flagged pixels."""

from __future__ import annotations

import sys

import numpy as np


def dev_f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def dev_u32(a):
    """uint32 numpy array -> int32 device tensor with the same bits."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def host_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_images(ctx, positions, triangles, op_positions, op_normals, R) -> np.ndarray:
    say(f"  gpu generate: V={len(positions)} T={len(triangles)} N={len(op_positions)} R={R}")
    out = ctx.generate(dev_f32(np.asarray(positions).reshape(-1, 3)), dev_u32(np.asarray(triangles).reshape(-1, 3)),
                       dev_f32(np.asarray(op_positions).reshape(-1, 3)),
                       dev_f32(np.asarray(op_normals).reshape(-1, 3)), R)
    ctx.sync()
    return host_u32(out)


def assert_images_match(gpu: np.ndarray, ora: np.ndarray, flags: np.ndarray, what: str = "") -> int:
    """GPU == oracle at every pixel the oracle does not flag; returns the flag count."""
    assert gpu.shape == ora.shape, (gpu.shape, ora.shape)
    bad = (gpu != ora) & ~flags
    if bad.any():
        idx = np.argwhere(bad)
        i, r, c = idx[0]
        raise AssertionError(f"{what}: {bad.sum()} unflagged pixels differ; first at image {i} row {r} col {c}: "
                             f"gpu {gpu[i, r, c]} oracle {ora[i, r, c]}")
    return int(flags.sum())
