"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def subspace_sin(a, b):
    qa, _ = np.linalg.qr(a)
    qb, _ = np.linalg.qr(b)
    # sine of the largest principal angle, from the projection residual
    # (accurate for tiny angles, unlike sqrt(1 - cos^2))
    return float(np.linalg.norm(qb - qa @ (qa.conj().T @ qb), 2))
