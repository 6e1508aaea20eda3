"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Every oracle function is checked against something other than itself: the
worked example printed in the paper, closed forms, dense library solves on tiny
inputs (LU / triangular solve of the Kronecker-sum matrix, SciPy's Sylvester
solver), exact operation counts, invariants and finite differences.  These run
on the CPU (no GPU marker).
"""
import itertools
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import sylt_workloads as wl
from dense_forms import (crandn, kron_sum, mode_product_tensordot, random_matrix,
                         random_upper, to_flat, to_tensor)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def eig_mismatch(a, b):
    """Largest distance after greedily pairing each value of `a` with the
    nearest unused value of `b` (multisets of eigenvalues)."""
    b = list(b)
    worst = 0.0
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b.pop(j)))
    return worst


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# --------------------------------------------------------------- Algorithm 2
def test_counter_matches_worked_example():
    """Section 2.2 worked example: (5,2,3) -> 30, (4,2,3) -> 29, (3,2,3) -> 28,
    ..., (1,1,1) -> 1 (golden fixture)."""
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "index_example.txt"))
            if l.strip() and not l.startswith("#")]
    n = (5, 2, 3)
    idx, tup = oracle.counter_trace(n, 30)
    for pos, i1, i2, i3, index in rows:
        t = pos - 1 if pos > 0 else 30 + pos
        assert tuple(tup[t]) == (i1, i2, i3)
        assert idx[t] == index
    # eq. e:index for every generated tuple, and every tuple generated once
    lin = 1 + (tup[:, 0] - 1) + (tup[:, 1] - 1) * 5 + (tup[:, 2] - 1) * 10
    assert np.array_equal(lin, idx)
    assert sorted(map(tuple, tup)) == sorted(itertools.product(range(1, 6), range(1, 3), range(1, 4)))


def test_counter_matches_nested_loops():
    """Algorithm 2 reproduces the order of Algorithm 1 (i_N outermost, all
    descending)."""
    n = (3, 4, 2, 3)
    _, tup = oracle.counter_trace(n, int(np.prod(n)))
    nested = [(a, b, c, d) for d in range(3, 0, -1) for c in range(2, 0, -1)
              for b in range(4, 0, -1) for a in range(3, 0, -1)]
    assert [tuple(t) for t in tup] == nested


# ------------------------------------------------------------- cost analysis
@pytest.mark.parametrize("n", [(5, 2, 3), (8, 8, 8), (4, 1, 3, 2), (7,), (2,) * 6])
def test_sweep_step_count_is_exact(n):
    """Section 2.1: the numerator needs n_1...n_N (sum n_j - N)/2 products."""
    rng = np.random.default_rng(7)
    T = [random_upper(k, rng) for k in n]
    C = to_flat(crandn(n, rng))
    _, steps = oracle.sweep(n, T, C)
    ntot = int(np.prod(n))
    assert steps * 2 == ntot * (sum(n) - len(n))
    _, steps_adj = oracle.sweep_adjoint(n, T, C)
    assert steps_adj == steps


# -------------------------------------------------------------- mode products
@pytest.mark.parametrize("n", [(3, 4, 5), (6,), (2, 1, 3), (4, 3, 1, 2)])
def test_mode_product_matches_tensordot(n):
    rng = np.random.default_rng(11)
    X = crandn(n, rng)
    for k in range(len(n)):
        M = crandn((n[k], n[k]), rng)
        got = oracle.mode_product(n, k, M, to_flat(X))
        assert relerr(got, to_flat(mode_product_tensordot(M, X, k))) < 1e-14
        got_h = oracle.mode_product(n, k, M, to_flat(X), adjoint=True)
        assert relerr(got_h, to_flat(mode_product_tensordot(M.conj().T, X, k))) < 1e-14


def test_transform_chain_matches_kronecker_product():
    """U^*-chain(B) = (U_N x ... x U_1)^* vec(B) (Kronecker form of eq. e:CUNU2U1B)."""
    rng = np.random.default_rng(12)
    n = (3, 2, 4)
    U = [np.linalg.qr(crandn((k, k), rng))[0] for k in n]
    B = to_flat(crandn(n, rng))
    K = np.kron(U[2], np.kron(U[1], U[0]))
    assert relerr(oracle.transform(n, U, B, adjoint=True), K.conj().T @ B) < 1e-14
    assert relerr(oracle.transform(n, U, B, adjoint=False), K @ B) < 1e-14


def test_transform_unitary_invariants():
    rng = np.random.default_rng(13)
    n = (5, 4, 3, 2)
    U = [np.linalg.qr(crandn((k, k), rng))[0] for k in n]
    B = to_flat(crandn(n, rng))
    C = oracle.transform(n, U, B, adjoint=True)
    assert abs(np.linalg.norm(C) / np.linalg.norm(B) - 1) < 1e-14
    assert relerr(oracle.transform(n, U, C, adjoint=False), B) < 1e-14


# ----------------------------------------------------------------------- sweep
@pytest.mark.parametrize("n", [(4, 3, 2), (5, 2, 3), (2, 1, 3, 2), (6,), (3, 3)])
def test_sweep_matches_dense_triangular_solve(n):
    """The Kronecker sum of upper-triangular T_j is upper triangular; the sweep
    is its back substitution (Section 2, eq. e:yi1i2iN)."""
    rng = np.random.default_rng(21)
    T = [random_upper(k, rng) for k in n]
    KT = kron_sum(T)
    assert np.allclose(KT, np.triu(KT))
    C = to_flat(crandn(n, rng))
    Y, _ = oracle.sweep(n, T, C)
    ref = scipy.linalg.solve_triangular(KT, C, lower=False)
    assert relerr(Y, ref) < 1e-13
    # adjoint sweep = lower-triangular solve with the conjugate transpose
    Ya, _ = oracle.sweep_adjoint(n, T, C)
    refa = scipy.linalg.solve_triangular(KT.conj().T, C, lower=True)
    assert relerr(Ya, refa) < 1e-13


def test_sweep_corner_closed_form():
    """eq. e:yi1i2iNnormal: y_{n_1..n_N} = c / sum_j t_{j, n_j n_j}."""
    rng = np.random.default_rng(22)
    n = (4, 3, 5)
    T = [random_upper(k, rng) for k in n]
    C = to_flat(crandn(n, rng))
    Y, _ = oracle.sweep(n, T, C)
    den = sum(t[-1, -1] for t in T)
    assert Y[-1] == C[-1] / den


def test_sweep_diagonal_T_is_hadamard():
    """Remark 1 (eq. e:yi1i2iNdiag): diagonal T_j give Y = Lambda o C."""
    rng = np.random.default_rng(23)
    n = (3, 4, 2)
    lam = [crandn(k, rng) + 3 for k in n]
    T = [np.diag(l) for l in lam]
    C = crandn(n, rng)
    Y, _ = oracle.sweep(n, T, to_flat(C))
    L = lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :]
    assert relerr(Y, to_flat(C / L)) < 1e-15


def test_sweep_one_mode_is_triangular_solve():
    rng = np.random.default_rng(24)
    T = random_upper(9, rng)
    c = crandn(9, rng)
    y, _ = oracle.sweep((9,), [T], c)
    assert relerr(y, scipy.linalg.solve_triangular(T, c)) < 1e-14


# ---------------------------------------------------------------- whole solve
def test_solve_C1_matches_dense_lu():
    """Workload C1 (N=3, n=8): Algorithm 3 vs LU of the 512x512 Kronecker sum."""
    w = wl.WORKLOADS["C1"]
    A = wl.coefficient_matrices(w.n, w.seed)
    B = wl.rhs(w)
    X = oracle.solve(w.n, A, B)
    ref = np.linalg.solve(kron_sum(A), B)
    assert relerr(X, ref) < 1e-13


def test_solve_N2_is_matrix_sylvester():
    """N = 2 is A_1 X + X A_2^T = B (eq. e:sylvester, note the transpose)."""
    rng = np.random.default_rng(31)
    A1, A2 = random_matrix(7, rng), random_matrix(5, rng)
    B = crandn((7, 5), rng)
    X = oracle.solve((7, 5), [A1, A2], to_flat(B))
    ref = scipy.linalg.solve_sylvester(A1, A2.T, B)
    assert relerr(X, to_flat(ref)) < 1e-13


def test_solve_N3_with_singleton_reduces_to_matrix_sylvester():
    """N = 3 with n_3 = 1 (eq. e:sylvester3D): A_3 = (a) is a scalar that
    joins A_1, leaving A_1 + aI, X + X A_2^T = B."""
    rng = np.random.default_rng(32)
    A1, A2 = random_matrix(6, rng), random_matrix(4, rng)
    a = 0.7 - 0.4j
    B = crandn((6, 4, 1), rng)
    X = oracle.solve((6, 4, 1), [A1, A2, np.array([[a]])], to_flat(B))
    ref = scipy.linalg.solve_sylvester(A1 + a * np.eye(6), A2.T, B[:, :, 0])
    assert relerr(X, to_flat(ref)) < 1e-13


@pytest.mark.parametrize("pos", [0, 1, 2, 3])
def test_singleton_mode_anywhere(pos):
    """A singleton mode with A_j = (a) equals the problem without it and a
    added to any one other A_k (Section 4, trailing and inner singletons)."""
    rng = np.random.default_rng(33 + pos)
    base = [3, 4, 2]
    mats = [random_matrix(k, rng) for k in base]
    a = 1.3 + 0.2j
    B = crandn(base, rng)
    n_with = base[:pos] + [1] + base[pos:]
    mats_with = mats[:pos] + [np.array([[a]])] + mats[pos:]
    X_with = oracle.solve(n_with, mats_with, to_flat(B.reshape(n_with, order="F")))
    shifted = [mats[0] + a * np.eye(base[0])] + mats[1:]
    X_without = oracle.solve(base, shifted, to_flat(B))
    assert relerr(X_with, X_without) < 1e-13


def test_solve_C2_residual_and_manufactured_solution():
    """Workload C2 (N=6, with a singleton): residual of Algorithm 3 vanishes to
    rounding, and a manufactured X* is recovered (the paper's test design,
    Section 5.1)."""
    w = wl.WORKLOADS["C2"]
    A = wl.coefficient_matrices(w.n, w.seed)
    B = wl.rhs(w)
    X = oracle.solve(w.n, A, B)
    assert oracle.relative_residual(w.n, A, X, B) < 1e-14
    Xs = wl.complex_normal(w.ntot, w.seed, wl.X_STREAM)
    Bs = oracle.apply(w.n, A, Xs)
    assert relerr(oracle.solve(w.n, A, Bs), Xs) < 1e-12


def test_shift_invariance():
    """A_k -> A_k + s_k I with sum s_k = 0 leaves the operator unchanged."""
    rng = np.random.default_rng(35)
    n = (3, 4, 2)
    A = [random_matrix(k, rng) for k in n]
    s = [0.5 + 0.1j, -0.2, -0.3 - 0.1j]
    B = to_flat(crandn(n, rng))
    X1 = oracle.solve(n, A, B)
    X2 = oracle.solve(n, [a + si * np.eye(a.shape[0]) for a, si in zip(A, s)], B)
    assert relerr(X1, X2) < 1e-13


def test_apply_matches_dense():
    rng = np.random.default_rng(36)
    n = (3, 2, 4)
    A = [random_matrix(k, rng) for k in n]
    X = to_flat(crandn(n, rng))
    assert relerr(oracle.apply(n, A, X), kron_sum(A) @ X) < 1e-14
    assert relerr(oracle.apply(n, A, X, adjoint=True), kron_sum(A).conj().T @ X) < 1e-14


def test_apply_at_matches_apply():
    rng = np.random.default_rng(37)
    n = (4, 3, 1, 5)
    A = [random_matrix(k, rng) for k in n]
    X = to_flat(crandn(n, rng))
    full = kron_sum(A) @ X
    idx = np.array([0, 7, 33, 59])
    got = oracle.apply_at(n, A, lambda i: X[i], idx)
    assert relerr(got, full[idx]) < 1e-14


# ------------------------------------------------------------------- factors
def test_schur_factors():
    rng = np.random.default_rng(41)
    for nk in (1, 2, 5, 19, 24):
        A = rng.standard_normal((nk, nk)) / np.sqrt(nk) + 3 * np.eye(nk)
        U, T = oracle.schur(A.astype(np.complex128))
        assert np.array_equal(T, np.triu(T))
        assert np.linalg.norm(U.conj().T @ U - np.eye(nk)) < 1e-13
        assert np.linalg.norm(U @ T @ U.conj().T - A) < 1e-13 * max(1, np.linalg.norm(A))
        assert eig_mismatch(np.diag(T), np.linalg.eigvals(A)) < 1e-12


def test_separation_brute_force():
    rng = np.random.default_rng(42)
    n = (3, 4, 2)
    lam = [crandn(k, rng) for k in n]
    ref = min(abs(a + b + c) for a in lam[0] for b in lam[1] for c in lam[2])
    assert oracle.separation(n, lam) == pytest.approx(ref, rel=1e-15)


def test_workload_separation_at_least_one():
    """The workloads' eigenvalue sums stay away from zero (>= 1)."""
    for name in ("C1", "C2", "C5"):
        w = wl.WORKLOADS[name]
        A = wl.coefficient_matrices(w.n, w.seed)
        lam = [np.diag(oracle.schur(a)[1]) for a in A]
        assert oracle.separation(w.n, lam) >= 1.0


# ---------------------------------------------------------------- gradients
def test_adjoint_solve_matches_dense():
    rng = np.random.default_rng(51)
    n = (3, 4, 2)
    A = [random_matrix(k, rng) for k in n]
    W = to_flat(crandn(n, rng))
    G = oracle.solve_adjoint(n, A, W)
    assert relerr(G, np.linalg.solve(kron_sum(A).conj().T, W)) < 1e-13


def test_adjoint_dot_product_identity():
    """<W, A^{-1} V> = <A^{-*} W, V>."""
    rng = np.random.default_rng(52)
    n = (4, 3, 3)
    A = [random_matrix(k, rng) for k in n]
    W, V = to_flat(crandn(n, rng)), to_flat(crandn(n, rng))
    lhs = np.vdot(W, oracle.solve(n, A, V))
    rhs = np.vdot(oracle.solve_adjoint(n, A, W), V)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


@pytest.mark.parametrize("real_A", [False, True])
def test_gradients_match_central_differences(real_A):
    """L = Re<W, X(A, B)>; gradients in the convention dL = Re<grad, d(param)>
    checked along random directions with central differences (h = 1e-6)."""
    rng = np.random.default_rng(53 + real_A)
    n = (3, 4, 2)
    if real_A:
        A = [(rng.standard_normal((k, k)) / np.sqrt(k) + 3 * np.eye(k)).astype(complex) for k in n]
    else:
        A = [random_matrix(k, rng) for k in n]
    B, W = to_flat(crandn(n, rng)), to_flat(crandn(n, rng))
    X, gB, gA = oracle.gradients(n, A, B, W)

    def L(Ai, Bi):
        return float(np.real(np.vdot(W, oracle.solve(n, Ai, Bi))))

    h = 1e-6
    dB = to_flat(crandn(n, rng))
    fd = (L(A, B + h * dB) - L(A, B - h * dB)) / (2 * h)
    an = float(np.real(np.vdot(gB, dB)))
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))
    for k in range(len(n)):
        dA = rng.standard_normal((n[k], n[k])) + (0 if real_A else 1j * rng.standard_normal((n[k], n[k])))
        Ap = [a.copy() for a in A]
        Am = [a.copy() for a in A]
        Ap[k] = Ap[k] + h * dA
        Am[k] = Am[k] - h * dA
        fd = (L(Ap, B) - L(Am, B)) / (2 * h)
        g = gA[k].real if real_A else gA[k]
        an = float(np.real(np.vdot(g, dA)))
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (k, fd, an)


def test_grad_A_matches_dense_formula():
    """dL/dA_k = -G_(k) X_(k)^* via tensordot unfoldings."""
    rng = np.random.default_rng(55)
    n = (3, 4, 2)
    G, X = crandn(n, rng), crandn(n, rng)
    for k in range(3):
        Gk = np.moveaxis(G, k, 0).reshape(n[k], -1)
        Xk = np.moveaxis(X, k, 0).reshape(n[k], -1)
        ref = -Gk @ Xk.conj().T
        assert relerr(oracle.grad_A(n, k, to_flat(G), to_flat(X)), ref) < 1e-14
