"""Independent dense constructions used to pin the oracle on tiny inputs.

These are textbook forms that do not go through the oracle's loops:
  * the Kronecker-sum matrix A_N (+) ... (+) A_1 acting on the column-major
    vec(X) (Section 1, eq. e:systvec), built with numpy.kron;
  * the mode product through numpy.tensordot.
"""
import numpy as np


def kron_sum(mats):
    """A_N (+) ... (+) A_1 = sum_j I_{n_N} x ... x A_j x ... x I_{n_1} (x = Kronecker)."""
    n = [m.shape[0] for m in mats]
    ntot = int(np.prod(n))
    K = np.zeros((ntot, ntot), np.complex128)
    for j, A in enumerate(mats):
        left = int(np.prod(n[j + 1:])) if j + 1 < len(n) else 1   # slower modes
        right = int(np.prod(n[:j])) if j > 0 else 1               # faster modes
        K += np.kron(np.eye(left), np.kron(A, np.eye(right)))
    return K


def to_tensor(flat, n):
    return np.asarray(flat).reshape(n, order="F")


def to_flat(t):
    return np.asarray(t).ravel(order="F").copy()


def mode_product_tensordot(M, X, k):
    """[M x_k X]_{..i..} = sum_m M[i, m] X[..m..] via tensordot."""
    return np.moveaxis(np.tensordot(M, X, axes=([1], [k])), 0, k)


def random_upper(n, rng, diag_shift=3.0):
    T = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    T[np.diag_indices(n)] += diag_shift
    return T


def random_matrix(n, rng, shift=3.0):
    return ((rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
            + shift * np.eye(n))


def crandn(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
