"""Helpers shared by the GPU tests (no graph arithmetic here)."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, device):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def rel_l1(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).sum() / np.abs(ref).sum())
