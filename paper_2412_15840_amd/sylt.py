"""Python binding of libsylt (ctypes marshalling only; every step runs in the
HIP library).

Low-level functions mirror the C ABI in include/sylt.h one to one and take
flat, contiguous CUDA tensors holding column-major data (mode 1 fastest, the
paper's linear index, Section 2.2 eq. e:index):

    Plan.factor(n, A)                 sylt_schur_factor_ex
    Plan.set_sweep_blocks(blocks)     sylt_plan_set_sweep_blocks
    Plan.from_factors(n, U, T, A)     sylt_plan_from_factors
    transform(plan, X, direction)     sylt_transform
    sweep(plan, CY, op)               sylt_sweep
    residual(plan, B, X)              sylt_residual
    solve(plan, B)                    sylt_solve
    solve_backward(plan, X, GX)       sylt_solve_backward
    solve_backward_noalloc(...)       sylt_solve_backward_noalloc
    evolve(plan, t, B, X0)            sylt_evolve

Matrices passed to / returned from these functions are ordinary (n, n) torch
tensors with their mathematical meaning M[i, m]; the binding converts them to
the column-major buffers of the ABI.

``sylvester_solve(A_list, B)`` is the torch-facing solver for row-major
tensors, differentiable through ``SchurSolve`` (a torch.autograd.Function whose
backward calls sylt_solve_backward).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsylt.so")

FP64, MIXED = 0, 1
TO_SCHUR, FROM_SCHUR = 0, 1
OP_N, OP_C = 0, 1
_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}

_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p
_LIB = None


class SyltError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().sylt_status_string(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where} failed with status {code}: {msg}")


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("sep", ctypes.c_double),
                ("ms_transform", ctypes.c_float), ("ms_sweep", ctypes.c_float),
                ("ms_residual", ctypes.c_float)]


def lib():
    """Load libsylt.so; raise if it has not been built (no fallback exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsylt.so not found at {LIB_PATH}: build it with "
                               f"`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.sylt_schur_factor.argtypes = [ctypes.c_int, _i64p, _vp, _vp, ctypes.POINTER(_vp)]
        L.sylt_schur_factor_ex.argtypes = [ctypes.c_int, _i64p, _vp, ctypes.c_int, _vp,
                                           ctypes.POINTER(_vp)]
        L.sylt_plan_set_sweep_blocks.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.sylt_plan_from_factors.argtypes = [ctypes.c_int, _i64p, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.sylt_plan_get_factors.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
        L.sylt_plan_separation.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.sylt_plan_destroy.argtypes = [_vp]
        L.sylt_workspace_bytes.argtypes = [_vp, ctypes.c_int]
        L.sylt_workspace_bytes.restype = ctypes.c_int64
        L.sylt_transform.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
        L.sylt_sweep.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
        L.sylt_residual.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]
        L.sylt_solve.argtypes = [_vp, ctypes.POINTER(_Opts), _vp, _vp, _vp, ctypes.c_size_t, _vp,
                                 ctypes.POINTER(_Info)]
        L.sylt_solve_backward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.sylt_solve_backward_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.sylt_evolve.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.sylt_evolve_workspace_bytes.argtypes = [_vp]
        L.sylt_evolve_workspace_bytes.restype = ctypes.c_int64
        L.sylt_plan_describe.argtypes = [_vp, ctypes.c_char_p, ctypes.c_size_t]
        L.sylt_status_string.argtypes = [ctypes.c_int]
        L.sylt_status_string.restype = ctypes.c_char_p
        L.sylt_version.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(code, where):
    if code != 0:
        raise SyltError(code, where)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dims(n):
    arr = (ctypes.c_int64 * len(n))(*[int(v) for v in n])
    return arr


def _ptrs(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


def _colmajor(M, dtype=torch.complex128):
    """(n, n) matrix -> contiguous column-major buffer on the GPU."""
    M = torch.as_tensor(M)
    if not M.is_cuda:
        M = M.cuda()
    return M.to(dtype).t().contiguous()


def _from_colmajor(buf, n):
    return buf.view(n, n).t()


def _flat(X, dtype):
    if not (X.is_cuda and X.dtype == dtype and X.is_contiguous()):
        raise ValueError(f"expected a contiguous CUDA tensor of dtype {dtype}, got "
                         f"{X.dtype} on {X.device} (contiguous={X.is_contiguous()})")
    return X


class Plan:
    """Owns a sylt_plan handle (Schur factors, separation, tiling tables)."""

    def __init__(self, handle, n):
        self.handle = handle
        self.n = [int(v) for v in n]
        self.ntot = 1
        for v in self.n:
            self.ntot *= v

    @classmethod
    def factor(cls, n, A_list, stream=None, qr_iter_per_n=0):
        """sylt_schur_factor_ex; qr_iter_per_n <= 0 keeps the default QR cap."""
        A = [_colmajor(a) for a in A_list]
        h = ctypes.c_void_p()
        _check(lib().sylt_schur_factor_ex(len(n), _dims(n), ctypes.cast(_ptrs(A), _vp),
                                          int(qr_iter_per_n), _stream(stream), ctypes.byref(h)),
               "sylt_schur_factor_ex")
        return cls(h, n)

    def set_sweep_blocks(self, blocks):
        """sylt_plan_set_sweep_blocks: block sizes of the non-singleton modes."""
        arr = (ctypes.c_int * max(1, len(blocks)))(*[int(b) for b in blocks])
        _check(lib().sylt_plan_set_sweep_blocks(self.handle, len(blocks), arr),
               "sylt_plan_set_sweep_blocks")
        return self

    @classmethod
    def from_factors(cls, n, U_list, T_list, A_list=None, stream=None):
        U = [_colmajor(u) for u in U_list]
        T = [_colmajor(t) for t in T_list]
        A = [_colmajor(a) for a in A_list] if A_list is not None else None
        h = ctypes.c_void_p()
        _check(lib().sylt_plan_from_factors(len(n), _dims(n),
                                            ctypes.cast(_ptrs(A), _vp) if A else None,
                                            ctypes.cast(_ptrs(U), _vp), ctypes.cast(_ptrs(T), _vp),
                                            _stream(stream), ctypes.byref(h)),
               "sylt_plan_from_factors")
        return cls(h, n)

    def describe(self):
        """The plan's JSON self-description (passes, tiles, sweep levels)."""
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().sylt_plan_describe(self.handle, buf, len(buf)), "sylt_plan_describe")
        return json.loads(buf.value.decode())

    def separation(self):
        v = ctypes.c_double()
        _check(lib().sylt_plan_separation(self.handle, ctypes.byref(v)), "sylt_plan_separation")
        return v.value

    def factors(self, k, stream=None):
        nk = self.n[k]
        U = torch.empty(nk * nk, dtype=torch.complex128, device="cuda")
        T = torch.empty_like(U)
        _check(lib().sylt_plan_get_factors(self.handle, k, U.data_ptr(), T.data_ptr(),
                                           _stream(stream)), "sylt_plan_get_factors")
        return _from_colmajor(U, nk), _from_colmajor(T, nk)

    def workspace_bytes(self, precision="fp64"):
        v = lib().sylt_workspace_bytes(self.handle, _PREC[precision])
        if v < 0:
            raise SyltError(int(v), "sylt_workspace_bytes")
        return int(v)

    def destroy(self):
        if self.handle is not None and self.handle.value:
            lib().sylt_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def transform(plan, X, direction, precision="fp64", stream=None):
    """In-place U^* chain (TO_SCHUR) or U chain (FROM_SCHUR) of flat X."""
    prec = _PREC[precision]
    _flat(X, torch.complex128 if prec == FP64 else torch.complex64)
    _check(lib().sylt_transform(plan.handle, direction, prec, X.data_ptr(), _stream(stream)),
           "sylt_transform")
    return X


def sweep(plan, CY, op=OP_N, precision="fp64", stream=None):
    """In-place triangular sweep of flat CY."""
    prec = _PREC[precision]
    _flat(CY, torch.complex128 if prec == FP64 else torch.complex64)
    _check(lib().sylt_sweep(plan.handle, op, prec, CY.data_ptr(), _stream(stream)), "sylt_sweep")
    return CY


def residual(plan, B, X, out=None, stream=None):
    """R = B - sum_k A_k x_k X (FP64); returns (R, ||R||_F^2, ||B||_F^2)."""
    _flat(B, torch.complex128)
    _flat(X, torch.complex128)
    R = out if out is not None else torch.empty_like(B)
    norms = (ctypes.c_double * 2)()
    _check(lib().sylt_residual(plan.handle, B.data_ptr(), X.data_ptr(), R.data_ptr(), norms,
                               _stream(stream)), "sylt_residual")
    return R, norms[0], norms[1]


def solve(plan, B, precision="fp64", rtol=1e-12, max_iter=8, out=None, workspace=None,
          stream=None, info=False):
    """X with sum_k A_k x_k X = B for flat complex128 B (out may be B for
    FP64; the MIXED form rejects out aliasing B, which every residual re-reads)."""
    _flat(B, torch.complex128)
    X = out if out is not None else torch.empty_like(B)
    prec = _PREC[precision]
    ws = workspace
    nbytes = plan.workspace_bytes(prec)
    if prec == MIXED and ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=B.device)
    opts = _Opts(prec, float(rtol), int(max_iter))
    inf = _Info()
    code = lib().sylt_solve(plan.handle, ctypes.byref(opts), B.data_ptr(), X.data_ptr(),
                            ws.data_ptr() if ws is not None else None,
                            ws.numel() if ws is not None else 0, _stream(stream),
                            ctypes.byref(inf) if info else None)
    _check(code, "sylt_solve")
    if info:
        return X, {"status": inf.status, "iterations": inf.iterations,
                   "rel_residual": inf.rel_residual, "sep": inf.sep,
                   "ms_transform": inf.ms_transform, "ms_sweep": inf.ms_sweep,
                   "ms_residual": inf.ms_residual}
    return X


def solve_backward(plan, X, GX, want_A=True, out=None, stream=None):
    """(dL/dB, [dL/dA_k]) for flat X (the solution) and GX = dL/dX."""
    _flat(X, torch.complex128)
    _flat(GX, torch.complex128)
    GB = out if out is not None else torch.empty_like(GX)
    GA_bufs = [torch.empty(nk * nk, dtype=torch.complex128, device=X.device) for nk in plan.n] \
        if want_A else None
    ws = torch.empty(plan.workspace_bytes(FP64), dtype=torch.uint8, device=X.device)
    _check(lib().sylt_solve_backward(plan.handle, X.data_ptr(), GX.data_ptr(), GB.data_ptr(),
                                     ctypes.cast(_ptrs(GA_bufs), _vp) if want_A else None,
                                     ws.data_ptr(), ws.numel(), _stream(stream)),
           "sylt_solve_backward")
    GA = [_from_colmajor(g, nk) for g, nk in zip(GA_bufs, plan.n)] if want_A else None
    return GB, GA


def solve_backward_noalloc(plan, X, GX, GB, GA_bufs=None, stream=None):
    """sylt_solve_backward_noalloc into caller-allocated outputs: GB (flat
    complex128 like GX) and GA_bufs, a list of flat n_k*n_k complex128 buffers
    receiving column-major dL/dA_k (or None).  Allocates nothing."""
    _flat(X, torch.complex128)
    _flat(GX, torch.complex128)
    _flat(GB, torch.complex128)
    ptrs = ctypes.cast(_ptrs(GA_bufs), _vp) if GA_bufs is not None else None
    _check(lib().sylt_solve_backward_noalloc(plan.handle, X.data_ptr(), GX.data_ptr(),
                                             GB.data_ptr(), ptrs, _stream(stream)),
           "sylt_solve_backward_noalloc")
    return GB


# ----------------------------------------------------------- torch facing
def evolve(plan, t, B, X0, out=None, workspace=None, stream=None):
    """X(t) for X_t = sum_k A_k x_k X + B, X(0) = X0 (Theorem 1), flat
    complex128 tensors; out may be B or X0."""
    _flat(B, torch.complex128)
    _flat(X0, torch.complex128)
    X = out if out is not None else torch.empty_like(B)
    nbytes = lib().sylt_evolve_workspace_bytes(plan.handle)
    _check(nbytes if nbytes < 0 else 0, "sylt_evolve_workspace_bytes")
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                             device=B.device)
    _check(lib().sylt_evolve(plan.handle, float(t), B.data_ptr(), X0.data_ptr(), X.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream(stream)), "sylt_evolve")
    return X


class SchurSolve(torch.autograd.Function):
    """X = A^{-1} B for row-major torch tensors.

    A torch tensor of shape (n_1..n_N) has the bytes of a column-major tensor
    of shape (n_N..n_1), so the ABI receives the modes (and the A list) in
    reverse order; relabelling modes leaves sum_k A_k x_k X unchanged.
    """

    @staticmethod
    def forward(ctx, B, precision, rtol, max_iter, *A_list):
        shape = tuple(B.shape)
        n_cm = list(shape[::-1])
        A_cm = list(reversed(A_list))
        plan = Plan.factor(n_cm, A_cm)
        Bc = B.to(torch.complex128).contiguous().view(-1)
        X = solve(plan, Bc, precision=precision, rtol=rtol, max_iter=max_iter)
        ctx.plan = plan
        ctx.shape = shape
        ctx.real_B = not B.is_complex()
        ctx.real_A = [not a.is_complex() for a in A_list]
        ctx.save_for_backward(X)
        return X.view(shape)

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        need_A = any(ctx.needs_input_grad[4:])
        GB, GA_cm = solve_backward(ctx.plan, X, gX.to(torch.complex128).contiguous().view(-1),
                                   want_A=need_A)
        gB = GB.view(ctx.shape)
        if ctx.real_B:
            gB = gB.real.contiguous()
        gA = [None] * len(ctx.real_A)
        if need_A:
            for k, g in enumerate(reversed(GA_cm)):
                gA[k] = g.real.contiguous() if ctx.real_A[k] else g.contiguous()
        return (gB if ctx.needs_input_grad[0] else None, None, None, None, *gA)


def sylvester_solve(A_list, B, precision="fp64", rtol=1e-12, max_iter=8):
    """Solve sum_k A_k x_k X = B for a row-major CUDA tensor B of shape
    (n_1..n_N); A_list[k] is (n_k, n_k) acting on dimension k."""
    if len(A_list) != B.dim():
        raise ValueError("need one matrix per dimension of B")
    return SchurSolve.apply(B, precision, rtol, max_iter, *A_list)
