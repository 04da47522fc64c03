"""Learned warm start: weight file I/O for the MLP whose kernels live in the HIP library.

File format (little endian): magic b"FAWS", uint32 version = 1, uint32 count,
then count float32 parameters in the layout of fa_mlp_param_count().
"""
from __future__ import annotations

import os
import struct
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "warm_mlp.bin")   # trained on the mixed family, n = 2,000-8,000
MAGIC = b"FAWS"


def save_weights(params: np.ndarray, path: str = WEIGHTS) -> None:
    params = np.ascontiguousarray(params, dtype=np.float32).ravel()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "wb") as f:
        f.write(MAGIC + struct.pack("<II", 1, params.size))
        f.write(params.tobytes())


def read_weights(path: str = WEIGHTS) -> Optional[np.ndarray]:
    if not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        head = f.read(12)
        if len(head) != 12 or head[:4] != MAGIC:
            raise ValueError(f"{path}: not a warm-start weight file")
        version, count = struct.unpack("<II", head[4:])
        if version != 1:
            raise ValueError(f"{path}: unsupported version {version}")
        data = np.frombuffer(f.read(4 * count), dtype=np.float32)
    if data.size != count:
        raise ValueError(f"{path}: truncated")
    return data.copy()


def load_weights(device, path: str = WEIGHTS):
    """Weights as a device tensor, or None when no trained file exists."""
    import torch

    from . import api
    w = read_weights(path)
    if w is None:
        return None
    if w.size != api.mlp_param_count():
        raise ValueError(f"{path}: {w.size} parameters, the library expects {api.mlp_param_count()}")
    return torch.from_numpy(w).to(device)
