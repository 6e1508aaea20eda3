"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Component tests inject the oracle's Schur factors into the GPU plan
(sylt_plan_from_factors) so the transforms and the sweep are compared on
identical U_k, T_k; whole-solve tests use the library's own device Schur
factors and compare only X, which is unique (the Schur basis is not).
Gate: max|X_gpu - X_oracle| / max|X_oracle| <= 1e-12 in FP64.
"""
import numpy as np
import pytest
import torch

import oracle
import sylt_workloads as wl
from dense_forms import crandn, random_matrix, random_upper
from gpu_helpers import banner, dev, host, relmax

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _sylt():
    from paper_2412_15840_amd import sylt
    return sylt


def _rng(seed):
    return np.random.default_rng(seed)


def _flat(x):
    return np.asarray(x).ravel(order="F").copy()


SHAPES = [
    (8, 8, 8),                    # C1 shape: a single tile
    (24, 16, 1, 20, 12, 8),       # C2 shape with its singleton
    (5, 3, 7, 1, 9),              # ragged tiles in every mode
    (2,) * 12,                    # n = 2 regime
    (19, 19, 19),                 # n = 19 regime, ragged blocks
    (16, 16, 16),                 # n = 16 (matrix-core transform, no padding)
    (19, 19, 19, 19),             # two fused passes, the second with ragged tiles
    (33, 5),                      # extent > 24: generic transform path
    (64, 3),                      # the largest extent with the LDS Schur kernel
    (65, 3),                      # the smallest with the global-memory Schur kernel
    (100, 2, 3),                  # extent > 64 in the first mode
    (3, 5, 256),                  # the largest supported extent, in the last mode
    (2, 9, 33, 74),               # leading modes of the large-extent shape of Section 5.1
    (11,),                        # N = 1: a plain triangular solve
    (3, 1, 1, 4),
]


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_schur_factors_invariants(n):
    sylt = _sylt()
    banner(f"schur {n}")
    rng = _rng(100 + len(n))
    A = [random_matrix(k, rng) for k in n]
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    for k, a in enumerate(A):
        U, T = (host(t) for t in plan.factors(k))
        nk = n[k]
        assert np.all(np.tril(T, -1) == 0)
        assert np.linalg.norm(U.conj().T @ U - np.eye(nk)) <= 1e-13 * max(1, nk)
        assert np.linalg.norm(U @ T @ U.conj().T - a) <= 1e-13 * max(1, nk) * np.linalg.norm(a)
        ev = np.linalg.eigvals(a)
        d = list(np.diag(T))
        worst = 0.0
        for x in ev:
            j = int(np.argmin([abs(x - y) for y in d]))
            worst = max(worst, abs(x - d.pop(j)))
        assert worst <= 1e-11
    lam = [np.diag(oracle.schur(a)[1]) for a in A]
    assert plan.separation() == pytest.approx(oracle.separation(n, lam), rel=1e-10)


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_transform_matches_oracle(n):
    sylt = _sylt()
    banner(f"transform {n}")
    rng = _rng(200 + len(n))
    A = [random_matrix(k, rng) for k in n]
    U, T = oracle.factors(A)
    plan = sylt.Plan.from_factors(n, [torch.from_numpy(u) for u in U],
                                  [torch.from_numpy(t) for t in T])
    X = _flat(crandn(n, rng))
    for direction, adj in ((sylt.TO_SCHUR, True), (sylt.FROM_SCHUR, False)):
        ref = oracle.transform(n, U, X, adjoint=adj)
        got = sylt.transform(plan, dev(X), direction)
        torch.cuda.synchronize()
        assert relmax(host(got), ref) <= TOL
        # FP32 form: complex64 data, FP32 arithmetic
        got32 = sylt.transform(plan, dev(X, torch.complex64), direction, precision="mixed")
        torch.cuda.synchronize()
        assert relmax(host(got32), ref) <= 5e-6


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_sweep_matches_oracle(n):
    sylt = _sylt()
    banner(f"sweep {n}")
    rng = _rng(300 + len(n))
    T = [random_upper(k, rng) for k in n]
    U = [np.eye(k, dtype=np.complex128) for k in n]
    plan = sylt.Plan.from_factors(n, [torch.from_numpy(u) for u in U],
                                  [torch.from_numpy(t) for t in T])
    C = _flat(crandn(n, rng))
    ref, _ = oracle.sweep(n, T, C)
    got = sylt.sweep(plan, dev(C), sylt.OP_N)
    torch.cuda.synchronize()
    assert relmax(host(got), ref) <= TOL
    refa, _ = oracle.sweep_adjoint(n, T, C)
    gota = sylt.sweep(plan, dev(C), sylt.OP_C)
    torch.cuda.synchronize()
    assert relmax(host(gota), refa) <= TOL
    # complex64 storage, FP64 arithmetic
    got32 = sylt.sweep(plan, dev(C, torch.complex64), sylt.OP_N, precision="mixed")
    torch.cuda.synchronize()
    ref32, _ = oracle.sweep(n, T, _flat(C.astype(np.complex64).astype(np.complex128)))
    assert relmax(host(got32), ref32) <= 1e-6


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_solve_matches_oracle(name):
    sylt = _sylt()
    w = wl.WORKLOADS[name]
    banner(f"solve {name} {w.n}")
    A = wl.coefficient_matrices(w.n, w.seed)
    B = wl.rhs(w)
    Xo = oracle.solve(w.n, A, B)
    plan = sylt.Plan.factor(w.n, [torch.from_numpy(a) for a in A])
    assert plan.separation() >= 1.0
    Bd = dev(B)
    X = sylt.solve(plan, Bd)
    torch.cuda.synchronize()
    assert relmax(host(X), Xo) <= TOL
    # in place (X aliases B)
    Bd2 = dev(B)
    sylt.solve(plan, Bd2, out=Bd2)
    torch.cuda.synchronize()
    assert relmax(host(Bd2), Xo) <= TOL
    # bitwise repeatable
    X2 = sylt.solve(plan, Bd)
    torch.cuda.synchronize()
    assert torch.equal(X, X2)


@pytest.mark.parametrize("n", [(7,), (1, 1, 1), (4, 1, 1, 6), (2, 3, 2, 3, 2, 3, 2),
                               (2,) * 16 + (1,) * 16,      # N = 32, the largest supported
                               (64, 64, 2)])               # largest extent, two passes
def test_solve_edge_shapes(n):
    sylt = _sylt()
    banner(f"solve edge {n}")
    rng = _rng(400 + len(n))
    A = [random_matrix(k, rng) for k in n]
    B = _flat(crandn(n, rng))
    Xo = oracle.solve(n, A, B)
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    X = sylt.solve(plan, dev(B))
    torch.cuda.synchronize()
    assert relmax(host(X), Xo) <= TOL


def test_residual_kernel_matches_oracle_apply():
    sylt = _sylt()
    banner("residual")
    rng = _rng(500)
    n = (6, 5, 1, 7, 3)
    A = [random_matrix(k, rng) for k in n]
    X, B = _flat(crandn(n, rng)), _flat(crandn(n, rng))
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    R, r2, b2 = sylt.residual(plan, dev(B), dev(X))
    ref = B - oracle.apply(n, A, X)
    assert relmax(host(R), ref) <= TOL
    assert r2 == pytest.approx(float(np.vdot(ref, ref).real), rel=1e-12)
    assert b2 == pytest.approx(float(np.vdot(B, B).real), rel=1e-12)


def test_singular_equation_is_reported():
    """A_1 = diag(1, 2), A_2 = diag(-1, 5): the eigenvalue sum 1 + (-1) is 0."""
    sylt = _sylt()
    A = [np.diag([1.0, 2.0]).astype(complex), np.diag([-1.0, 5.0]).astype(complex)]
    with pytest.raises(sylt.SyltError) as ei:
        sylt.Plan.factor((2, 2), [torch.from_numpy(a) for a in A])
    assert ei.value.code == -2
