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


_PROBLEMS = {}


def oracle_problem(cfg):
    """The oracle's problem for a named workload, built once per test process (the 1025^2 build
    takes ~20 s)."""
    import sg_inputs
    from oracle import system
    if cfg not in _PROBLEMS:
        c = sg_inputs.CONFIGS[cfg]
        _PROBLEMS.clear()
        _PROBLEMS[cfg] = system.build_problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"])
    return _PROBLEMS[cfg]
