"""Helpers shared by the GPU parity tests (device arrays <-> oracle layouts)."""

import sys

import numpy as np
import torch


def note(msg):
    """Name the case before any GPU step, flushed, so a failing run says where it was."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
