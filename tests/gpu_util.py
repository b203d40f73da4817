"""Helpers shared by the GPU tests (not collected by pytest)."""
import math
import sys

import numpy as np

BOX = (2 * math.pi / 1.14, 2 * math.pi / 2.5)


def say(*args):
    print("[gpu-test]", *args, flush=True)
    sys.stdout.flush()


def to_dev(a, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """Relative Frobenius error ||a - b|| / ||b|| over the whole field."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
