"""CPU FP64 oracle for the N-dimensional Sylvester tensor equation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the HIP library (``paper_2412_15840_amd``) and never imports it.

What it computes (Cuesta & de la Hoz, arXiv 2412.15840):
  * ``solve``            -- Algorithm 3 (Section 2.2): complex Schur factors of
                            every A_j (LAPACK through SciPy), the forward chain
                            of U_j^* mode products (eq. e:CUNU2U1B), the literal
                            single-loop sweep (eq. e:yi1i2iN with the counter of
                            Algorithm 2) and the backward chain (eq. e:XUNU2U1Y).
  * ``solve_adjoint``    -- the same with the adjoint sweep (T_j^*), giving
                            dL/dB = A^{-*} W.
  * ``grad_A``           -- dL/dA_k = -G_(k) X_(k)^*.
  * ``apply``            -- the Kronecker-sum operator sum_j A_j []_j X.
  * ``apply_at``         -- that operator at a few chosen entries (pure Python).
  * ``separation``       -- min over multi-indices of |sum_j lambda_{j,i_j}|.
  * ``evolve``           -- Theorem 1 in Schur form (eqs. e:sylvesterNDG and
                            e:G): X(t) of X_t = sum_j A_j []_j X + B from X(0),
                            with exp(t T_j) from SciPy's expm (eq. e:exptAj).

All tensors are flat complex128 numpy arrays in column-major order (mode 1
fastest), the paper's linear index (eq. e:index).  Matrices are (n, n) arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.linalg

from . import build as _build

_LIB = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.ora_mode_product_range.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, _vp, ctypes.c_int,
                                             _vp, ctypes.c_int64, ctypes.c_int64]
        L.ora_mode_product.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, _vp, ctypes.c_int, _vp]
        L.ora_transform.argtypes = [ctypes.c_int, _i64p, _vp, ctypes.c_int, _vp]
        L.ora_sweep_upper.argtypes = [ctypes.c_int, _i64p, _vp, _vp, ctypes.c_int64]
        L.ora_sweep_upper.restype = ctypes.c_int64
        L.ora_sweep_adjoint.argtypes = [ctypes.c_int, _i64p, _vp, _vp]
        L.ora_sweep_adjoint.restype = ctypes.c_int64
        L.ora_counter_trace.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _i64p, _i64p]
        L.ora_apply.argtypes = [ctypes.c_int, _i64p, _vp, _vp, _vp]
        L.ora_apply_adjoint.argtypes = [ctypes.c_int, _i64p, _vp, _vp, _vp]
        L.ora_solve_factored.argtypes = [ctypes.c_int, _i64p, _vp, _vp, _vp]
        L.ora_solve_factored.restype = ctypes.c_int64
        L.ora_solve_adjoint_factored.argtypes = [ctypes.c_int, _i64p, _vp, _vp, _vp]
        L.ora_solve_adjoint_factored.restype = ctypes.c_int64
        L.ora_grad_A.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, _vp, _vp, _vp]
        L.ora_separation.argtypes = [ctypes.c_int, _i64p, _vp]
        L.ora_separation.restype = ctypes.c_double
        L.ora_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


# ---------------------------------------------------------------- marshalling
def _dims(n):
    a = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
    return a, a.ctypes.data_as(_i64p)


def _cvec(x):
    x = np.asarray(x)
    assert x.dtype == np.complex128 and x.flags.c_contiguous and x.ndim == 1, \
        "oracle tensors are flat contiguous complex128 arrays"
    return x


def _mat_colmajor(M):
    """n x n complex matrix -> contiguous column-major complex128 buffer."""
    return np.asfortranarray(np.asarray(M, dtype=np.complex128)).ravel(order="F").copy()


class _PtrArray:
    """Keeps a list of column-major matrices alive and exposes a void** array."""

    def __init__(self, mats):
        self.bufs = [_mat_colmajor(M) for M in mats]
        self.arr = (ctypes.c_void_p * len(self.bufs))(*[b.ctypes.data for b in self.bufs])

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


# ------------------------------------------------------------------- factors
def schur(A):
    """Complex Schur factorisation A = U T U^* (Section 2, via LAPACK zgees
    through SciPy).  Returns (U, T).  A 1x1 matrix gives U = 1, T = A."""
    A = np.asarray(A, dtype=np.complex128)
    if A.shape == (1, 1):
        return np.ones((1, 1), np.complex128), A.copy()
    T, U = scipy.linalg.schur(A, output="complex")
    return U, np.triu(T)


def factors(A_list):
    Us, Ts = [], []
    for A in A_list:
        U, T = schur(A)
        Us.append(U)
        Ts.append(T)
    return Us, Ts


# ----------------------------------------------------------------- operations
def mode_product(n, k, M, X, adjoint=False):
    """X <- M []_k X (or M^* []_k X), returns a new array."""
    N = len(n)
    dims, dp = _dims(n)
    out = _cvec(X).copy()
    Mb = _mat_colmajor(M)
    lib().ora_mode_product(N, dp, int(k), Mb.ctypes.data, int(bool(adjoint)), out.ctypes.data)
    return out


def transform(n, U_list, X, adjoint):
    """Chain of mode products with every U_j (adjoint=True: U_j^*, eq.
    e:CUNU2U1B; adjoint=False: U_j, eq. e:XUNU2U1Y)."""
    dims, dp = _dims(n)
    out = _cvec(X).copy()
    P = _PtrArray(U_list)
    lib().ora_transform(len(n), dp, P.ptr, int(bool(adjoint)), out.ctypes.data)
    return out


def sweep(n, T_list, C, max_entries=-1):
    """Literal sweep of Algorithm 3 (upper triangular T_j).  Returns (Y, steps)."""
    dims, dp = _dims(n)
    out = _cvec(C).copy()
    P = _PtrArray(T_list)
    steps = lib().ora_sweep_upper(len(n), dp, P.ptr, out.ctypes.data, int(max_entries))
    return out, steps


def sweep_adjoint(n, T_list, C):
    """Adjoint sweep: solves sum_j T_j^* []_j Y = C.  Returns (Y, steps)."""
    dims, dp = _dims(n)
    out = _cvec(C).copy()
    P = _PtrArray(T_list)
    steps = lib().ora_sweep_adjoint(len(n), dp, P.ptr, out.ctypes.data)
    return out, steps


def counter_trace(n, count):
    """First `count` tuples of Algorithm 2 (1-based) and their linear indices."""
    N = len(n)
    dims, dp = _dims(n)
    idx = np.zeros(count, np.int64)
    tup = np.zeros(count * N, np.int64)
    lib().ora_counter_trace(N, dp, int(count), idx.ctypes.data_as(_i64p), tup.ctypes.data_as(_i64p))
    return idx, tup.reshape(count, N)


def apply(n, A_list, X, adjoint=False):
    """sum_j A_j []_j X (or with A_j^* when adjoint)."""
    dims, dp = _dims(n)
    X = _cvec(X)
    out = np.empty_like(X)
    P = _PtrArray(A_list)
    f = lib().ora_apply_adjoint if adjoint else lib().ora_apply
    f(len(n), dp, P.ptr, X.ctypes.data, out.ctypes.data)
    return out


def solve_factored(n, U_list, T_list, B):
    dims, dp = _dims(n)
    X = _cvec(B).copy()
    PU, PT = _PtrArray(U_list), _PtrArray(T_list)
    lib().ora_solve_factored(len(n), dp, PU.ptr, PT.ptr, X.ctypes.data)
    return X


def solve(n, A_list, B):
    """Algorithm 3: the unique X with sum_j A_j []_j X = B."""
    U, T = factors(A_list)
    return solve_factored(n, U, T, B)


def solve_adjoint_factored(n, U_list, T_list, W):
    dims, dp = _dims(n)
    G = _cvec(W).copy()
    PU, PT = _PtrArray(U_list), _PtrArray(T_list)
    lib().ora_solve_adjoint_factored(len(n), dp, PU.ptr, PT.ptr, G.ctypes.data)
    return G


def evolve_factored(n, U_list, T_list, B, X0, t):
    """Theorem 1 with the Schur factors, in the order of eqs. e:sylvesterNDG
    and e:G: C = U^*-chain(B), Y(0) = U^*-chain(X(0)),
    G = exp(tT_N) []_N ( ... exp(tT_1) []_1 (sum_j T_j []_j Y(0) + C)) - C,
    then the sweep for sum_j T_j []_j Y = G and X(t) = U-chain(Y)."""
    C = transform(n, U_list, B, adjoint=True)
    Y0 = transform(n, U_list, X0, adjoint=True)
    G = apply(n, T_list, Y0) + C
    for k, T in enumerate(T_list):
        G = mode_product(n, k, scipy.linalg.expm(t * np.asarray(T, np.complex128)), G)
    G = G - C
    Y, _ = sweep(n, T_list, G)
    return transform(n, U_list, Y, adjoint=False)


def evolve(n, A_list, B, X0, t):
    """X(t) for X_t = sum_j A_j []_j X + B, X(0) = X0 (Theorem 1)."""
    U, T = factors(A_list)
    return evolve_factored(n, U, T, B, X0, t)


def solve_adjoint(n, A_list, W):
    """G with sum_j A_j^* []_j G = W (= dL/dB for L = Re<W, X>)."""
    U, T = factors(A_list)
    return solve_adjoint_factored(n, U, T, W)


def grad_A(n, k, G, X):
    """dL/dA_k = -sum G_(..a..) conj(X_(..m..)), an n_k x n_k matrix."""
    dims, dp = _dims(n)
    nk = int(n[k])
    out = np.zeros(nk * nk, np.complex128)
    lib().ora_grad_A(len(n), dp, int(k), _cvec(G).ctypes.data, _cvec(X).ctypes.data,
                     out.ctypes.data)
    return out.reshape(nk, nk, order="F")


def gradients(n, A_list, B, W):
    """(X, dL/dB, [dL/dA_k]) for L = Re<W, X(A, B)>, complex-valued A_k."""
    U, T = factors(A_list)
    X = solve_factored(n, U, T, B)
    G = solve_adjoint_factored(n, U, T, W)
    return X, G, [grad_A(n, k, G, X) for k in range(len(n))]


def separation(n, lam_list):
    dims, dp = _dims(n)
    bufs = [np.ascontiguousarray(np.asarray(l, dtype=np.complex128)) for l in lam_list]
    arr = (ctypes.c_void_p * len(bufs))(*[b.ctypes.data for b in bufs])
    return lib().ora_separation(len(n), dp, ctypes.cast(arr, ctypes.c_void_p))


def apply_at(n, A_list, fetch, indices):
    """(sum_j A_j []_j X) at the given linear indices, computed one entry at a
    time from the definition of []_j.  `fetch(idx_array)` returns X at the
    requested linear indices, so X never needs to be on the host whole."""
    n = [int(v) for v in n]
    st = [1]
    for v in n[:-1]:
        st.append(st[-1] * v)
    indices = np.asarray(indices, np.int64)
    # every entry needs the fibres through it along each mode
    need = []
    for idx in indices:
        rem = int(idx)
        for j, nj in enumerate(n):
            ij = rem % nj
            rem //= nj
            base = int(idx) - ij * st[j]
            need.extend(base + m * st[j] for m in range(nj))
    need = np.asarray(need, np.int64)
    vals = np.asarray(fetch(need), np.complex128)
    out = np.zeros(len(indices), np.complex128)
    pos = 0
    for t, idx in enumerate(indices):
        rem = int(idx)
        acc = 0j
        for j, nj in enumerate(n):
            ij = rem % nj
            rem //= nj
            A = np.asarray(A_list[j])
            for m in range(nj):
                acc += complex(A[ij, m]) * complex(vals[pos])
                pos += 1
        out[t] = acc
    return out


def num_threads():
    return int(lib().ora_num_threads())


def mode_product_fibres_inplace(n, k, M, X, f_begin, f_end, adjoint):
    """X <- M []_k X restricted to fibres [f_begin, f_end) of mode k, in place
    on the caller's array (no copy; used to time a bounded sample)."""
    dims, dp = _dims(n)
    X = _cvec(X)
    Mb = _mat_colmajor(M)
    lib().ora_mode_product_range(len(n), dp, int(k), Mb.ctypes.data, int(bool(adjoint)),
                                 X.ctypes.data, int(f_begin), int(f_end))


def sweep_inplace(n, T_list, CY, max_entries=-1):
    """Literal sweep on the caller's array, the first max_entries entries of
    Algorithm 3's order (all if -1).  Returns the multiply-subtract count."""
    dims, dp = _dims(n)
    CY = _cvec(CY)
    P = _PtrArray(T_list)
    return lib().ora_sweep_upper(len(n), dp, P.ptr, CY.ctypes.data, int(max_entries))


def relative_residual(n, A_list, X, B):
    R = np.asarray(B) - apply(n, A_list, X)
    return float(np.linalg.norm(R) / np.linalg.norm(B))
