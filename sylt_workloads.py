"""Seeded synthetic inputs for the N-dimensional Sylvester tensor equation.

    sum_k A_k x_k X = B,   X, B complex tensors of shape n_1 x ... x n_N,

where [A x_k X]_{..i_k..} = sum_m A[i_k, m] X[..m..] (the mode-k product of the
paper's problem statement, Section 1, eq. e:sylvesterND).

This module only draws random numbers and describes workload shapes.  It holds
none of the method's arithmetic; both the CPU oracle (``oracle/``) and the HIP
path consume the arrays it returns.

Storage convention: every tensor is returned as a flat complex128 array in
column-major order (mode 1 fastest), i.e. element (i_1..i_N), 0-based, sits at
sum_j i_j * prod_{l<j} n_l (the paper's linear index, Section 2.2, eq. e:index).
Matrices are (n, n) numpy arrays (row/column meaning is the mathematical one).

Recipe (the design doc states it too):
  A_k = G_k / sqrt(n_k) + 3 I, G_k real N(0,1) from default_rng([seed, k]),
        k = 1..N, stored as complex128 with zero imaginary part.
  B   = P + iQ, P, Q iid N(0,1); generated in chunks of 2^24 entries, chunk c
        from default_rng([seed, 1000 + c]) filling the interleaved (re, im)
        doubles of that chunk.
  W   (cotangent for the gradient workload) likewise with stream base 2000.
  Normal A_k (normal-matrix fast path): Q_k diag(lambda_k) Q_k^* with Q_k the
        unitary QR factor of a complex Gaussian matrix and lambda_k =
        3 + N(0,1) + i N(0,1), from default_rng([seed, 100 + k]).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 24
B_STREAM = 1000
W_STREAM = 2000
X_STREAM = 3000  # manufactured solutions (tests only)


@dataclass(frozen=True)
class Workload:
    name: str
    n: tuple
    seed: int
    precision: str = "fp64"
    description: str = ""

    @property
    def N(self) -> int:
        return len(self.n)

    @property
    def ntot(self) -> int:
        return int(np.prod(self.n, dtype=np.int64))


# The workloads: the five of the benchmark description and the mixed-extent
# shape of Section 5.1 (shapes and seeds).
WORKLOADS = {
    "C1": Workload("C1", (8, 8, 8), 1, "fp64", "FP64, N=3, n_k=8 (512 entries)"),
    "C2": Workload("C2", (24, 16, 1, 20, 12, 8), 2, "fp64",
                   "FP64, N=6, n=(24,16,1,20,12,8) incl. a singleton mode"),
    "C3a": Workload("C3a", (2,) * 28, 31, "fp64", "FP64, N=28, n_k=2 (2^28 entries)"),
    "C3b": Workload("C3b", (19,) * 7, 32, "fp64", "FP64, N=7, n_k=19 (893,871,739 entries)"),
    "C4": Workload("C4", (19,) * 7, 32, "mixed", "mixed precision, N=7, n_k=19"),
    "C5": Workload("C5", (16,) * 5, 5, "fp64", "differentiation, N=5, n_k=16"),
    "E1": Workload("E1", (2, 9, 33, 74, 231), 51, "fp64",
                   "FP64, N=5, n=(2,9,33,74,231) (10,153,836 entries), the mixed-extent "
                   "shape of Section 5.1"),
}


def coefficient_matrices(n, seed):
    """A_k = G_k/sqrt(n_k) + 3 I with G_k real N(0,1) (complex128 storage)."""
    out = []
    for k, nk in enumerate(n, start=1):
        g = np.random.default_rng([seed, k]).standard_normal((nk, nk))
        a = g / math.sqrt(nk) + 3.0 * np.eye(nk)
        out.append(a.astype(np.complex128))
    return out


def normal_coefficient_matrices(n, seed):
    """Normal A_k = Q_k diag(lambda_k) Q_k^* (input recipe of the Remark 1 fast
    path): Q_k the unitary factor of a complex Gaussian matrix, lambda_k =
    3 + N(0,1) + i N(0,1), from default_rng([seed, 100 + k])."""
    out = []
    for k, nk in enumerate(n, start=1):
        rng = np.random.default_rng([seed, 100 + k])
        z = rng.standard_normal((nk, nk)) + 1j * rng.standard_normal((nk, nk))
        q, _ = np.linalg.qr(z)
        lam = 3.0 + rng.standard_normal(nk) + 1j * rng.standard_normal(nk)
        out.append((q * lam) @ q.conj().T)
    return out


def hermite_differentiation(m, b):
    """Nodes and first/second derivative matrices of Hermite-function
    interpolation (the discretisation of the advection-diffusion example,
    Section 5.3): nodes x = r / b with r the m roots of the Hermite polynomial
    H_m; u(x) ~ sum_j u_j a(x) l_j(x) / a(x_j) with the Lagrange basis l_j of
    the nodes and the weight a = exp(-(b x)^2 / 2).  Built from the barycentric
    Lagrange derivatives L1, L2 (Berrut & Trefethen 2004) in the variable r:
        D1 = A L1 A^-1 + diag(a'/a),
        D2 = A L2 A^-1 + 2 diag(a'/a) A L1 A^-1 + diag(a''/a),
    with A = diag(a), a'/a = -r, a''/a = r^2 - 1, then scaled by b and b^2."""
    r = np.sort(np.polynomial.hermite.hermroots([0] * m + [1]).real)
    d = r[:, None] - r[None, :]
    np.fill_diagonal(d, 1.0)
    w = 1.0 / np.prod(d, axis=1)                 # barycentric weights
    inv = 1.0 / d
    np.fill_diagonal(inv, 0.0)
    L1 = (w[None, :] / w[:, None]) * inv
    np.fill_diagonal(L1, 0.0)
    np.fill_diagonal(L1, -L1.sum(axis=1))
    L2 = 2.0 * L1 * (np.diag(L1)[:, None] - inv)
    np.fill_diagonal(L2, 0.0)
    np.fill_diagonal(L2, -L2.sum(axis=1))
    a = np.exp(-r * r / 2.0)
    S1 = a[:, None] * L1 / a[None, :]
    S2 = a[:, None] * L2 / a[None, :]
    D1 = S1 + np.diag(-r)
    D2 = S2 + 2.0 * np.diag(-r) @ S1 + np.diag(r * r - 1.0)
    return r / b, b * D1, b * b * D2


def advection_diffusion(N, m=16, b=1.4):
    """The advection-diffusion example of Section 5.3 on m Hermite nodes per
    axis: u_t = Lap u + 2 x.grad u + (2N+1) u - exp(-x.x), u(x,0) = 2 exp(-x.x),
    exact solution (1 + e^t) exp(-x.x).  Returns (x, [A]*N, B, X0) with
    A = D2 + 2 diag(x) D1 + (2N+1)/N I and flat column-major B, X0."""
    x, D1, D2 = hermite_differentiation(m, b)
    A = (D2 + 2.0 * np.diag(x) @ D1 + (2.0 * N + 1.0) / N * np.eye(m)).astype(np.complex128)
    g = np.exp(-x * x)
    G = g
    for _ in range(N - 1):
        G = np.multiply.outer(G, g)
    G = np.asarray(G).ravel(order="F")
    return x, [A] * N, (-G).astype(np.complex128), (2.0 * G).astype(np.complex128)


def advection_diffusion_exact(x, N, t):
    g = np.exp(-x * x)
    G = g
    for _ in range(N - 1):
        G = np.multiply.outer(G, g)
    return (1.0 + math.exp(t)) * np.asarray(G).ravel(order="F")


def _fill_chunk(buf_f64, c, seed, stream, nchunks_total):
    rng = np.random.default_rng([seed, stream + c])
    rng.standard_normal(out=buf_f64)


def complex_normal(ntot, seed, stream=B_STREAM, out=None, threads=None):
    """Flat complex128 array whose (re, im) parts are iid N(0,1).

    Chunk c (2^24 entries) is drawn from default_rng([seed, stream + c]) so the
    result is reproducible and may be produced in parallel.  ``out`` may be a
    preallocated complex128 array (e.g. pinned host memory viewed by numpy).
    """
    ntot = int(ntot)
    if out is None:
        out = np.empty(ntot, dtype=np.complex128)
    assert out.dtype == np.complex128 and out.size == ntot
    f = out.view(np.float64)
    nchunks = (ntot + CHUNK - 1) // CHUNK
    jobs = [(f[2 * c * CHUNK: 2 * min(ntot, (c + 1) * CHUNK)], c) for c in range(nchunks)]
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if nchunks <= 1 or threads <= 1:
        for buf, c in jobs:
            _fill_chunk(buf, c, seed, stream, nchunks)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda j: _fill_chunk(j[0], j[1], seed, stream, nchunks), jobs))
    return out


def rhs(wl: Workload, out=None):
    return complex_normal(wl.ntot, wl.seed, B_STREAM, out=out)


def cotangent(wl: Workload, out=None):
    return complex_normal(wl.ntot, wl.seed, W_STREAM, out=out)


def strides(n):
    """Column-major strides (prod_{l<j} n_l)."""
    s, acc = [], 1
    for nk in n:
        s.append(acc)
        acc *= int(nk)
    return s


def sample_indices(n, count, seed):
    """`count` distinct-ish linear indices spread over the tensor, always
    including the first and last entry (the two corners of the sweep)."""
    ntot = int(np.prod(n, dtype=np.int64))
    rng = np.random.default_rng([seed, 4000])
    idx = rng.integers(0, ntot, size=max(0, count - 2), dtype=np.int64)
    return np.unique(np.concatenate([[0, ntot - 1], idx]))
