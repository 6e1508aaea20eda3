"""Shared helpers for the GPU tests: host <-> device marshalling of flat
column-major tensors and the comparison metric used against the oracle."""
import numpy as np
import torch

import oracle


def dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    """max |a - b| / max |b| (the gate: <= 1e-12 in FP64)."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def oracle_plan_inputs(n, A_list):
    """Oracle Schur factors (LAPACK via SciPy) for injecting into the GPU plan."""
    U, T = oracle.factors(A_list)
    return U, T


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
