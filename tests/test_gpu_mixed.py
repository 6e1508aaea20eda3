"""Mixed-precision form: FP32 matrix-core transforms with FP32 accumulation,
FP64 sweep arithmetic, FP64 residual and iterative refinement.  Gate: the
refined solution reaches a 1e-12 relative residual (recomputed here by the
oracle's operator); its distance to the FP64 oracle solution is reported and
bounded by the refinement theory (residual x conditioning, <= 1e-10 here)."""
import numpy as np
import pytest
import torch

import oracle
import sylt_workloads as wl
from dense_forms import crandn, random_matrix
from gpu_helpers import banner, dev, host, relmax

pytestmark = pytest.mark.gpu


def _sylt():
    from paper_2412_15840_amd import sylt
    return sylt


@pytest.mark.parametrize("name,n,seed", [
    ("C2", None, None),
    ("n19x4", (19, 19, 19, 19), 71),
    ("n16x5", (16,) * 5, 5),
])
def test_mixed_refinement_reaches_1e12(name, n, seed):
    sylt = _sylt()
    if n is None:
        w = wl.WORKLOADS[name]
        n, seed = w.n, w.seed
    banner(f"mixed {name} {n}")
    A = wl.coefficient_matrices(n, seed)
    ntot = int(np.prod(n))
    B = wl.complex_normal(ntot, seed)
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    X, info = sylt.solve(plan, dev(B), precision="mixed", rtol=1e-12, max_iter=8, info=True)
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["rel_residual"] <= 1e-12
    Xh = host(X)
    res = oracle.relative_residual(n, A, Xh, B)
    Xo = oracle.solve(n, A, B)
    err = relmax(Xh, Xo)
    print(f"[mixed] {name}: iterations {info['iterations']}, residual (device) "
          f"{info['rel_residual']:.3e}, residual (oracle) {res:.3e}, error vs FP64 oracle {err:.3e}",
          flush=True)
    assert res <= 1e-12
    assert err <= 1e-10


@pytest.mark.parametrize("scale", [1e-42, 1e-30, 1e30, 1e36])
def test_mixed_refinement_far_from_unit_scale(scale):
    """B scaled far from unit size: 1e-42 lies below FP32's normal range and
    1e36 near its top, so a plain FP32 copy of B (or of the shrinking
    residuals) would flush or overflow.  The solve scales each right-hand side
    by a power of two before the FP32 cast; it must still reach 1e-12 and the
    FP64 oracle's solution of the same scaled problem."""
    sylt = _sylt()
    n, seed = (16, 16, 16), 83
    banner(f"mixed scale {scale:g} {n}")
    A = wl.coefficient_matrices(n, seed)
    B = wl.complex_normal(int(np.prod(n)), seed) * scale
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    X, info = sylt.solve(plan, dev(B), precision="mixed", rtol=1e-12, max_iter=8, info=True)
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["rel_residual"] <= 1e-12
    Xh = host(X)
    assert np.all(np.isfinite(Xh))
    res = oracle.relative_residual(n, A, Xh, B)
    err = relmax(Xh, oracle.solve(n, A, B))
    print(f"[mixed] scale {scale:g}: iterations {info['iterations']}, residual (oracle) {res:.3e}, "
          f"error vs FP64 oracle {err:.3e}", flush=True)
    assert res <= 1e-12
    assert err <= 1e-10


def test_mixed_reports_no_convergence():
    sylt = _sylt()
    rng = np.random.default_rng(72)
    n = (5, 6, 4)
    A = [random_matrix(k, rng) for k in n]
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    B = dev(crandn(n, rng).ravel(order="F"))
    with pytest.raises(sylt.SyltError) as ei:
        sylt.solve(plan, B, precision="mixed", rtol=1e-30, max_iter=1)
    assert ei.value.code == -3
