"""Full-size workloads (N=28 n=2, 2^28 entries; N=7 n=19, 893,871,739 entries)
in the launch configuration the benchmark times.

Fast checks, one sampled entry at a time from the definition of the operator:
  * the solve: |B_i - (sum_k A_k x_k X)_i| <= 1e-12 max|B| at sampled i;
  * the sweep: (sum_k T_k x_k Y)_i = C_i at sampled i, with the plan's T_k;
and on the device: the forward transform preserves the Frobenius norm (the
U_k are unitary) and forward then backward returns the input.

Slow checks (marked ``slow``): every entry of the FP64 solve, and of the mixed
solve at N=7 n=19, against a full run of the oracle (about 30 GB of host
memory and a minute or two of host time at N=7 n=19)."""
import numpy as np
import pytest
import torch

import oracle
import sylt_workloads as wl
from gpu_helpers import banner

pytestmark = pytest.mark.gpu


def _sylt():
    from paper_2412_15840_amd import sylt
    return sylt


def _device_rhs(w):
    host = torch.empty(w.ntot, dtype=torch.complex128, pin_memory=True)
    wl.rhs(w, out=host.numpy())
    dev = host.cuda()
    torch.cuda.synchronize()
    return dev


def _fetch(t):
    def f(idx):
        i = torch.from_numpy(np.asarray(idx, np.int64)).cuda()
        return t[i].cpu().numpy()
    return f


@pytest.mark.parametrize("name", ["C3a", "C3b"])
def test_full_size_solve_sampled(name):
    sylt = _sylt()
    w = wl.WORKLOADS[name]
    banner(f"full size {name} {w.ntot} entries")
    A = wl.coefficient_matrices(w.n, w.seed)
    Bd = _device_rhs(w)
    plan = sylt.Plan.factor(list(w.n), [torch.from_numpy(a) for a in A])
    assert plan.separation() >= 1.0
    X = sylt.solve(plan, Bd)
    torch.cuda.synchronize()
    idx = wl.sample_indices(w.n, 48, w.seed)
    r = Bd[torch.from_numpy(idx).cuda()].cpu().numpy() - oracle.apply_at(w.n, A, _fetch(X), idx)
    bmax = float(Bd.abs().max())
    worst = float(np.max(np.abs(r)) / bmax)
    print(f"[full] {name}: sampled relative residual {worst:.3e}", flush=True)
    assert worst <= 1e-12
    del X

    # sweep against the plan's own triangular factors at sampled entries
    T = [plan.factors(k)[1].cpu().numpy() for k in range(len(w.n))]
    C = Bd.clone()
    sylt.transform(plan, C, sylt.TO_SCHUR)
    nB = float(torch.linalg.vector_norm(Bd))
    nC = float(torch.linalg.vector_norm(C))
    assert abs(nC / nB - 1) <= 1e-12
    Y = C.clone()
    sylt.sweep(plan, Y, sylt.OP_N)
    torch.cuda.synchronize()
    got = oracle.apply_at(w.n, T, _fetch(Y), idx)
    want = C[torch.from_numpy(idx).cuda()].cpu().numpy()
    sworst = float(np.max(np.abs(got - want)) / float(C.abs().max()))
    print(f"[full] {name}: sampled sweep equation residual {sworst:.3e}", flush=True)
    assert sworst <= 1e-12
    del Y
    # round trip of the transforms
    sylt.transform(plan, C, sylt.FROM_SCHUR)
    torch.cuda.synchronize()
    rt = float((C - Bd).abs().max()) / bmax
    assert rt <= 1e-13


def _compare_chunked(Xd, Xo, chunk=1 << 26):
    """max |X_gpu - X_oracle| / max |X_oracle|, streamed chunk-wise from the device."""
    num, den = 0.0, 0.0
    for a in range(0, Xo.size, chunk):
        b = min(Xo.size, a + chunk)
        g = Xd[a:b].cpu().numpy()
        num = max(num, float(np.max(np.abs(g - Xo[a:b]))))
        den = max(den, float(np.max(np.abs(Xo[a:b]))))
    return num / den


@pytest.mark.slow
@pytest.mark.parametrize("name", ["C3a", "C3b"])
def test_full_size_solve_against_full_oracle(name):
    """Every entry of the full-size FP64 solve (and, at N=7 n=19, of the mixed
    solve refined to 1e-12) against a full run of the CPU oracle (Algorithm 3
    with LAPACK Schur factors, the literal single-threaded sweep)."""
    import time
    sylt = _sylt()
    w = wl.WORKLOADS[name]
    banner(f"full oracle comparison {name} {w.ntot} entries, {oracle.num_threads()} host threads")
    A = wl.coefficient_matrices(w.n, w.seed)
    B = wl.rhs(w)
    Bd = torch.from_numpy(B).cuda()
    plan = sylt.Plan.factor(list(w.n), [torch.from_numpy(a) for a in A])
    X = sylt.solve(plan, Bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xo = oracle.solve(w.n, A, B)
    print(f"[full] {name}: oracle solve {time.perf_counter() - t0:.1f} s", flush=True)
    err = _compare_chunked(X, Xo)
    print(f"[full] {name}: FP64 relmax vs oracle {err:.3e}", flush=True)
    assert err <= 1e-12
    del X
    if name == "C3b":
        Xm, info = sylt.solve(plan, Bd, precision="mixed", rtol=1e-12, max_iter=8, info=True)
        torch.cuda.synchronize()
        errm = _compare_chunked(Xm, Xo)
        print(f"[full] C4 (mixed, same inputs): {info['iterations']} iterations, residual "
              f"{info['rel_residual']:.3e}, relmax vs FP64 oracle {errm:.3e}", flush=True)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-12
        assert errm <= 1e-11
