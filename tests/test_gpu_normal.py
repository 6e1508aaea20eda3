"""Remark 1 (eq. e:yi1i2iNdiag): when every A_k is normal its Schur factor is
diagonal and the sweep is the Hadamard product Y = Lambda o C.  The planner
detects diagonal T_k; these tests check the detection, the fast sweep against
the formula itself (eigenvalues read back from the plan) and the whole solve
and adjoint solve against the oracle's literal sweep (gate 1e-12).
"""
import numpy as np
import pytest
import torch

import oracle
import sylt_workloads as wl
from dense_forms import crandn
from gpu_helpers import banner, dev, host, relmax

pytestmark = pytest.mark.gpu


def _sylt():
    from paper_2412_15840_amd import sylt
    return sylt


def normal_matrix(n, rng, hermitian=False):
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(Z)
    lam = 3.0 + rng.standard_normal(n) + (0.0 if hermitian else 1j * rng.standard_normal(n))
    return (Q * lam) @ Q.conj().T


SHAPES = [(8, 8, 8), (5, 3, 7, 1, 9), (19, 19, 19, 19), (2,) * 12, (16,)]


@pytest.mark.parametrize("n", SHAPES)
def test_normal_solve_takes_the_hadamard_sweep(n):
    banner(f"normal n={n}")
    sylt = _sylt()
    rng = np.random.default_rng(sum(n))
    A = [normal_matrix(k, rng) for k in n]
    b = crandn(int(np.prod(n)), rng)
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is True
    X = host(sylt.solve(plan, dev(b)))
    assert relmax(X, oracle.solve(n, A, b)) <= 1e-12
    GB, _ = sylt.solve_backward(plan, dev(X), dev(b), want_A=False)
    assert relmax(host(GB), oracle.solve_adjoint(n, A, b)) <= 1e-12


def test_hermitian_inputs_are_detected():
    sylt = _sylt()
    rng = np.random.default_rng(7)
    n = (6, 5, 4)
    A = [normal_matrix(k, rng, hermitian=True) for k in n]
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is True


def test_non_normal_inputs_keep_the_tiled_sweep():
    sylt = _sylt()
    w = wl.WORKLOADS["C1"]
    A = wl.coefficient_matrices(w.n, w.seed)
    plan = sylt.Plan.factor(list(w.n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is False
    rng = np.random.default_rng(8)
    n = (6, 5, 4)
    A = [normal_matrix(6, rng), wl.coefficient_matrices((5,), 3)[0], normal_matrix(4, rng)]
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is False


@pytest.mark.parametrize("op", ["N", "C"])
def test_hadamard_sweep_matches_the_formula(op):
    sylt = _sylt()
    rng = np.random.default_rng(9)
    n = (7, 1, 6, 5)
    A = [normal_matrix(k, rng) for k in n]
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    lam = [np.diag(host(plan.factors(k)[1])) for k in range(len(n))]
    den = np.zeros(n, np.complex128)
    for k, l in enumerate(lam):
        shape = [1] * len(n)
        shape[k] = n[k]
        den = den + l.reshape(shape)
    if op == "C":
        den = den.conj()
    c = crandn(int(np.prod(n)), rng)
    Y = dev(c)
    sylt.sweep(plan, Y, sylt.OP_N if op == "N" else sylt.OP_C)
    ref = c / den.ravel(order="F")
    assert relmax(host(Y), ref) <= 1e-14


def test_mixed_precision_solve_with_normal_matrices():
    # the FP32-storage form of the Hadamard sweep inside iterative refinement
    sylt = _sylt()
    rng = np.random.default_rng(10)
    n = (8, 8, 8)
    A = [normal_matrix(k, rng) for k in n]
    b = crandn(int(np.prod(n)), rng)
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is True
    X, info = sylt.solve(plan, dev(b), precision="mixed", info=True)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-12
    assert relmax(host(X), oracle.solve(n, A, b)) <= 1e-10


def test_evolution_with_normal_matrices():
    sylt = _sylt()
    rng = np.random.default_rng(11)
    n = (6, 1, 5, 4)
    A = [normal_matrix(k, rng) for k in n]
    b, x0 = crandn(int(np.prod(n)), rng), crandn(int(np.prod(n)), rng)
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is True
    X = host(sylt.evolve(plan, 0.2, dev(b), dev(x0)))
    assert relmax(X, oracle.evolve(n, A, b, x0, 0.2)) <= 1e-11


@pytest.mark.parametrize("scale,fast", [(0.25, True), (64.0, False)])
def test_nearly_normal_threshold(scale, fast):
    """A_k = Q (D + E) Q^* with E strictly upper triangular of Frobenius norm
    `scale` times the planner's threshold 16 n eps ||T||_F: under it the
    Hadamard sweep is taken (the dropped part is a perturbation of rounding
    size), over it the tiled sweep; both solves meet the 1e-12 gate."""
    sylt = _sylt()
    rng = np.random.default_rng(11)
    n = (12, 9, 7)
    A = []
    for k in n:
        Z = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
        Q, _ = np.linalg.qr(Z)
        D = np.diag(3.0 + rng.standard_normal(k) + 1j * rng.standard_normal(k))
        E = np.triu(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)), 1)
        target = scale * 16 * k * np.finfo(float).eps * np.linalg.norm(D)
        E *= target / np.linalg.norm(E)
        A.append(Q @ (D + E) @ Q.conj().T)
    b = crandn(int(np.prod(n)), rng)
    plan = sylt.Plan.factor(list(n), [dev(a) for a in A])
    assert plan.describe()["sweep"]["diagonal"] is fast
    X = host(sylt.solve(plan, dev(b)))
    assert relmax(X, oracle.solve(n, A, b)) <= 1e-12
