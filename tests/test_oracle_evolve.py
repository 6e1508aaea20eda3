"""Pins of the oracle's Theorem 1 (time evolution) against facts that do not
go through it: the closed-form solution of the linear ODE with the dense
Kronecker-sum matrix, fourth-order Runge-Kutta integration (the paper's own
check in Section 5.2), the initial condition, the ODE itself by central
differences in t, and the exact solution of the advection-diffusion example
of Section 5.3 (with the Hermite differentiation matrices checked as the paper
checks them).  CPU only.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import sylt_workloads as wl
from dense_forms import crandn, kron_sum, random_matrix


def dense_solution(A_list, b, x0, t):
    """vec X(t) = e^{tK} x0 + K^{-1} (e^{tK} - I) b with K the Kronecker sum."""
    K = kron_sum(A_list)
    E = scipy.linalg.expm(t * K)
    return E @ x0 + np.linalg.solve(K, E @ b - b)


def case(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    A = [random_matrix(k, rng, shift) for k in n]
    ntot = int(np.prod(n))
    return A, crandn(ntot, rng), crandn(ntot, rng)


@pytest.mark.parametrize("n,t", [((2, 3, 2), 0.3), ((3, 1, 2), 0.1), ((4,), 0.7), ((2, 2, 2, 2), 0.05)])
def test_evolve_matches_dense_closed_form(n, t):
    A, b, x0 = case(n, 11 + len(n))
    ref = dense_solution(A, b, x0, t)
    got = oracle.evolve(n, A, b, x0, t)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_evolve_at_zero_time_is_initial_condition():
    n = (3, 4, 2)
    A, b, x0 = case(n, 5)
    got = oracle.evolve(n, A, b, x0, 0.0)
    assert np.max(np.abs(got - x0)) <= 1e-12 * np.max(np.abs(x0))


def test_evolve_matches_runge_kutta():
    # the paper's check: N=7 sizes 2..8 at t = 0.1 against RK4; a smaller
    # tensor keeps the dense right-hand side cheap
    n = (2, 3, 4)
    A, b, x0 = case(n, 7, shift=0.0)
    K = kron_sum(A)
    t, steps = 0.1, 200
    dt = t / steps
    x = x0.copy()
    f = lambda y: K @ y + b
    for _ in range(steps):
        k1 = f(x)
        k2 = f(x + 0.5 * dt * k1)
        k3 = f(x + 0.5 * dt * k2)
        k4 = f(x + dt * k3)
        x = x + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    got = oracle.evolve(n, A, b, x0, t)
    assert np.max(np.abs(got - x)) <= 1e-9 * np.max(np.abs(x))


def test_evolve_satisfies_the_ode():
    n = (3, 2, 3)
    A, b, x0 = case(n, 9, shift=0.0)
    t, h = 0.2, 1e-4
    d = (oracle.evolve(n, A, b, x0, t + h) - oracle.evolve(n, A, b, x0, t - h)) / (2 * h)
    rhs = oracle.apply(n, A, oracle.evolve(n, A, b, x0, t)) + b
    assert np.max(np.abs(d - rhs)) <= 1e-6 * np.max(np.abs(rhs))


def test_hermite_differentiation_matches_the_papers_check():
    # Section 5.3: D1 and D2 on m = 16 nodes with scale 1.4 applied to exp(-x^2)
    # (the paper reports 1.2e-15 and 1.5e-14 in the max norm)
    x, D1, D2 = wl.hermite_differentiation(16, 1.4)
    g = np.exp(-x * x)
    assert np.max(np.abs(D1 @ g + 2 * x * g)) <= 1e-13
    assert np.max(np.abs(D2 @ g - (4 * x * x - 2) * g)) <= 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_evolve_advection_diffusion_exact_solution(N):
    # Section 5.3: u(x, t) = (1 + e^t) exp(-x.x) at t = 1
    x, A, B, X0 = wl.advection_diffusion(N)
    X = oracle.evolve((16,) * N, A, B, X0, 1.0)
    assert np.max(np.abs(X - wl.advection_diffusion_exact(x, N, 1.0))) <= 1e-12
