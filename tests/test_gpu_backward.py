"""Differentiation through the solve: sylt_solve_backward vs the oracle
gradient (workload C5: N=5, n_k=16) and the torch.autograd.Function vs
central finite differences (h = 1e-6) and the oracle."""
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


def test_backward_C5_matches_oracle_gradient():
    sylt = _sylt()
    w = wl.WORKLOADS["C5"]
    banner(f"backward C5 {w.n}")
    A = wl.coefficient_matrices(w.n, w.seed)
    B, W = wl.rhs(w), wl.cotangent(w)
    Xo, Go, GAo = oracle.gradients(w.n, A, B, W)
    plan = sylt.Plan.factor(w.n, [torch.from_numpy(a) for a in A])
    X = sylt.solve(plan, dev(B))
    GB, GA = sylt.solve_backward(plan, X, dev(W))
    torch.cuda.synchronize()
    assert relmax(host(X), Xo) <= 1e-12
    assert relmax(host(GB), Go) <= 1e-12
    for k in range(len(w.n)):
        assert relmax(host(GA[k]), GAo[k]) <= 1e-12, k
    # GB may alias GX
    Wd = dev(W)
    sylt.solve_backward(plan, X, Wd, want_A=False, out=Wd)
    torch.cuda.synchronize()
    assert relmax(host(Wd), Go) <= 1e-12


def test_adjoint_identity_on_gpu():
    """<W, A^{-1} V> = <A^{-*} W, V> with the device solves."""
    sylt = _sylt()
    rng = np.random.default_rng(61)
    n = (6, 5, 7, 4)
    A = [random_matrix(k, rng) for k in n]
    V = crandn(n, rng).ravel(order="F")
    W = crandn(n, rng).ravel(order="F")
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    X = sylt.solve(plan, dev(V))
    G, _ = sylt.solve_backward(plan, X, dev(W), want_A=False)
    torch.cuda.synchronize()
    lhs = np.vdot(W, host(X))
    rhs = np.vdot(host(G), V)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("real_A", [False, True])
def test_autograd_function(real_A):
    """torch-facing solver on row-major tensors: forward vs the oracle (mode
    order reversed), gradients vs the oracle and central differences."""
    sylt = _sylt()
    banner(f"autograd real_A={real_A}")
    rng = np.random.default_rng(62 + real_A)
    shape = (3, 4, 5)
    if real_A:
        A_np = [rng.standard_normal((k, k)) / np.sqrt(k) + 3 * np.eye(k) for k in shape]
    else:
        A_np = [random_matrix(k, rng) for k in shape]
    B_np = crandn(shape, rng)
    W_np = crandn(shape, rng)
    A = [torch.tensor(a, device="cuda", requires_grad=True) for a in A_np]
    B = torch.tensor(B_np, device="cuda", requires_grad=True)
    X = sylt.sylvester_solve(A, B)
    W = torch.tensor(W_np, device="cuda")
    L = (W.conj() * X).real.sum()
    L.backward()
    # oracle in column-major order: reversed modes, reversed matrices
    n_cm = shape[::-1]
    A_cm = [np.asarray(a, dtype=complex) for a in A_np[::-1]]
    Xo, Go, GAo = oracle.gradients(n_cm, A_cm, B_np.ravel().copy(), W_np.ravel().copy())
    assert relmax(X.detach().cpu().numpy().ravel(), Xo) <= 1e-12
    assert relmax(B.grad.cpu().numpy().ravel(), Go) <= 1e-12
    for k in range(3):
        ref = GAo[2 - k]
        if real_A:
            ref = ref.real
            assert not A[k].grad.is_complex()
        assert relmax(A[k].grad.cpu().numpy(), ref) <= 1e-12

    def loss(As, Bv):
        with torch.no_grad():
            return float((W.conj() * sylt.sylvester_solve(As, Bv)).real.sum())

    h = 1e-6
    dB = torch.tensor(crandn(shape, rng), device="cuda")
    Bd = B.detach()
    fd = (loss([a.detach() for a in A], Bd + h * dB) - loss([a.detach() for a in A], Bd - h * dB)) / (2 * h)
    an = float((B.grad.conj() * dB).real.sum())
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))
    for k in range(3):
        dA = rng.standard_normal(A_np[k].shape)
        if not real_A:
            dA = dA + 1j * rng.standard_normal(A_np[k].shape)
        dA = torch.tensor(dA, device="cuda")
        Ap = [a.detach() for a in A]
        Am = [a.detach() for a in A]
        Ap[k] = Ap[k] + h * dA
        Am[k] = Am[k] - h * dA
        fd = (loss(Ap, Bd) - loss(Am, Bd)) / (2 * h)
        g = A[k].grad
        an = float((g.conj() * dA).real.sum()) if g.is_complex() else float((g * dA).sum())
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (k, fd, an)
