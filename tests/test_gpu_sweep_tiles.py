"""Element-wise parity of the sweep in the exact tiling the N=7, n=19 workload
runs with, on tensors small enough for the oracle: blocks (19,3,3,3,3,3,2),
the pencil local solve, cross-tile pulls along every blocked mode, ragged last
blocks (7 = 3+3+1, 5 = 2+2+1) and several tile levels.  The plan's own
self-description is asserted, so a planner change cannot silently drop the
coverage.  Also: tile-shape independence (two tilings agree to rounding),
bitwise repeatability, the matrix-core residual pass, and the QR iteration cap
that forces NO_CONVERGENCE from the host.

Sections: Section 2 (eq. e:yi1i2iN, solved in any dependency-respecting
order), Algorithm 3 (the oracle's literal sweep).  Gate 1e-12 in FP64.
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
HEADLINE_BLOCKS = [19, 3, 3, 3, 3, 3, 2]   # the tiling of the (19,)*7 workload
SMALL = (19, 7, 7, 7, 7, 7, 5)             # 1,596,665 entries, same tile shape


def _sylt():
    from paper_2412_15840_amd import sylt
    return sylt


def _flat(x):
    return np.asarray(x).ravel(order="F").copy()


def _assert_headline_tiling(plan):
    d = plan.describe()["sweep"]
    assert d["block"] == HEADLINE_BLOCKS
    assert d["local_solve"] == "pencil"
    assert d["tile_levels"] > 1 and d["tiles"] > 1
    assert d["diagonal"] is False
    return d


def test_headline_plan_of_the_full_workload_is_this_tiling():
    """The planner's choice for (19,)*7 is the tiling the tests below force."""
    sylt = _sylt()
    n = (19,) * 7
    T = [np.triu(np.ones((19, 19))) + 3 * np.eye(19) for _ in n]
    U = [np.eye(19, dtype=np.complex128) for _ in n]
    plan = sylt.Plan.from_factors(n, [torch.from_numpy(u) for u in U],
                                  [torch.from_numpy(t.astype(np.complex128)) for t in T])
    d = _assert_headline_tiling(plan)
    assert d["tile_levels"] == 40


@pytest.mark.parametrize("storage", ["fp64", "c64"])
def test_headline_tiling_sweep_matches_oracle(storage):
    sylt = _sylt()
    banner(f"headline tiling sweep {SMALL} {storage}")
    rng = np.random.default_rng(801)
    T = [random_upper(k, rng) for k in SMALL]
    U = [np.eye(k, dtype=np.complex128) for k in SMALL]
    plan = sylt.Plan.from_factors(SMALL, [torch.from_numpy(u) for u in U],
                                  [torch.from_numpy(t) for t in T])
    plan.set_sweep_blocks(HEADLINE_BLOCKS)
    d = _assert_headline_tiling(plan)
    print(f"[tiles] {d}", flush=True)
    C = _flat(crandn(SMALL, rng))
    if storage == "fp64":
        for op, fn in ((sylt.OP_N, oracle.sweep), (sylt.OP_C, oracle.sweep_adjoint)):
            ref, _ = fn(SMALL, T, C)
            got = sylt.sweep(plan, dev(C), op)
            torch.cuda.synchronize()
            err = relmax(host(got), ref)
            print(f"[tiles] op {op}: relmax {err:.3e}", flush=True)
            assert err <= TOL
    else:
        C32 = _flat(C.astype(np.complex64).astype(np.complex128))
        for op, fn in ((sylt.OP_N, oracle.sweep), (sylt.OP_C, oracle.sweep_adjoint)):
            ref, _ = fn(SMALL, T, C32)
            got = sylt.sweep(plan, dev(C, torch.complex64), op, precision="mixed")
            torch.cuda.synchronize()
            err = relmax(host(got), ref)
            print(f"[tiles] complex64 storage op {op}: relmax {err:.3e}", flush=True)
            # complex64 rounding of every stored entry, amplified by the solve
            assert err <= 1e-6


LONG = (19, 16, 7, 5)          # 10,640 entries
LONG_BLOCKS = [19, 3, 3, 2]


@pytest.mark.parametrize("storage", ["fp64", "c64"])
def test_pencil_pulls_with_long_and_short_ranges(storage):
    """The pencil kernel pulls a mode either one cross-section position per
    lane (k range above 8 terms) or two per lane (8 terms or fewer).  Along
    the 16-long mode in blocks of 3 the upper sweep pulls 13, 10, 7, 4 and 1
    terms and the adjoint 3, 6, 9, 12 and 15, so both forms run in both
    directions, with ragged last blocks (16 = 5*3 + 1, 7 = 3+3+1, 5 = 2+2+1).
    Element-wise against the oracle's literal sweep (Section 2, eq.
    e:yi1i2iN; Algorithm 3)."""
    sylt = _sylt()
    banner(f"pencil pulls, long and short k ranges {LONG} {storage}")
    rng = np.random.default_rng(805)
    T = [random_upper(k, rng) for k in LONG]
    U = [np.eye(k, dtype=np.complex128) for k in LONG]
    plan = sylt.Plan.from_factors(LONG, [torch.from_numpy(u) for u in U],
                                  [torch.from_numpy(t) for t in T])
    plan.set_sweep_blocks(LONG_BLOCKS)
    d = plan.describe()["sweep"]
    assert d["block"] == LONG_BLOCKS and d["local_solve"] == "pencil"
    C = _flat(crandn(LONG, rng))
    if storage == "c64":
        C = _flat(C.astype(np.complex64).astype(np.complex128))
    for op, fn in ((sylt.OP_N, oracle.sweep), (sylt.OP_C, oracle.sweep_adjoint)):
        ref, _ = fn(LONG, T, C)
        if storage == "fp64":
            got = sylt.sweep(plan, dev(C), op)
        else:
            got = sylt.sweep(plan, dev(C, torch.complex64), op, precision="mixed")
        torch.cuda.synchronize()
        err = relmax(host(got), ref)
        print(f"[tiles] long/short pulls {storage} op {op}: relmax {err:.3e}", flush=True)
        # FP64 at the parity gate; complex64 storage rounds every stored entry
        assert err <= (TOL if storage == "fp64" else 1e-6)


@pytest.fixture(scope="module")
def small_problem():
    A = wl.coefficient_matrices(SMALL, 802)
    ntot = int(np.prod(SMALL))
    B = wl.complex_normal(ntot, 802)
    Xo = oracle.solve(SMALL, A, B)
    return A, B, Xo


@pytest.mark.parametrize("blocks", [None, HEADLINE_BLOCKS])
def test_headline_tiling_solves_match_oracle(small_problem, blocks):
    """FP64 and mixed solves, element-wise against the oracle's solve (FP64 at
    1e-12; the mixed form gated on its residual, its error reported)."""
    sylt = _sylt()
    A, B, Xo = small_problem
    banner(f"headline tiling solve {SMALL} blocks {blocks}")
    plan = sylt.Plan.factor(SMALL, [torch.from_numpy(a) for a in A])
    if blocks is not None:
        plan.set_sweep_blocks(blocks)
        _assert_headline_tiling(plan)
    Bd = dev(B)
    X = sylt.solve(plan, Bd)
    torch.cuda.synchronize()
    err = relmax(host(X), Xo)
    Xm, info = sylt.solve(plan, Bd, precision="mixed", rtol=1e-12, max_iter=8, info=True)
    torch.cuda.synchronize()
    errm = relmax(host(Xm), Xo)
    print(f"[tiles] fp64 relmax {err:.3e}; mixed relmax {errm:.3e} after {info['iterations']} "
          f"iterations, residual {info['rel_residual']:.3e}", flush=True)
    assert err <= TOL
    # the mixed form's gate is its FP64 relative residual (1e-12); its distance
    # to the FP64 oracle is reported and bounded by conditioning x residual
    assert info["status"] == 0 and info["rel_residual"] <= 1e-12
    assert oracle.relative_residual(SMALL, A, host(Xm), B) <= 1e-12
    assert errm <= 1e-11


def test_tile_shape_independence_and_repeatability(small_problem):
    """Two tilings give the same X to rounding (any dependency-respecting
    order is valid, Section 2); a repeated solve is bitwise identical."""
    sylt = _sylt()
    A, B, Xo = small_problem
    banner("tile-shape independence")
    plan = sylt.Plan.factor(SMALL, [torch.from_numpy(a) for a in A])
    Bd = dev(B)
    outs = []
    for blocks in (HEADLINE_BLOCKS, [19, 7, 4, 4, 2, 2, 1], [8, 4, 4, 4, 2, 2, 2]):
        plan.set_sweep_blocks(blocks)
        assert plan.describe()["sweep"]["block"] == blocks
        X = sylt.solve(plan, Bd)
        X2 = sylt.solve(plan, Bd)
        torch.cuda.synchronize()
        assert torch.equal(X, X2), f"solve with blocks {blocks} is not bitwise repeatable"
        assert relmax(host(X), Xo) <= TOL
        outs.append(host(X))
    for o in outs[1:]:
        assert relmax(o, outs[0]) <= 1e-13


def test_set_sweep_blocks_rejects_bad_requests():
    sylt = _sylt()
    rng = np.random.default_rng(803)
    n = (5, 1, 6)
    A = [random_matrix(k, rng) for k in n]
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    before = plan.describe()["sweep"]
    for bad, code in (([5, 6, 1], -1), ([0, 6], -1), ([6, 6], -1)):
        with pytest.raises(sylt.SyltError) as ei:
            plan.set_sweep_blocks(bad)
        assert ei.value.code == code
    assert plan.describe()["sweep"] == before
    B = _flat(crandn(n, rng))
    X = sylt.solve(plan, dev(B))
    torch.cuda.synchronize()
    assert relmax(host(X), oracle.solve(n, A, B)) <= TOL


def test_matrix_core_residual_matches_oracle_apply():
    """sylt_residual through the matrix-core passes (extent 19)."""
    sylt = _sylt()
    n = (19, 19, 19, 19)
    banner(f"matrix-core residual {n}")
    rng = np.random.default_rng(804)
    A = [random_matrix(k, rng) for k in n]
    X, B = _flat(crandn(n, rng)), _flat(crandn(n, rng))
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    assert plan.describe()["residual_form"] == "mfma"
    R, r2, b2 = sylt.residual(plan, dev(B), dev(X))
    torch.cuda.synchronize()
    ref = B - oracle.apply(n, A, X)
    err = relmax(host(R), ref)
    print(f"[residual] mfma form relmax {err:.3e}", flush=True)
    assert err <= TOL
    assert r2 == pytest.approx(float(np.vdot(ref, ref).real), rel=1e-12)
    assert b2 == pytest.approx(float(np.vdot(B, B).real), rel=1e-12)


def test_qr_iteration_cap_reports_no_convergence():
    """A cap of one QR iteration per unit of extent (40 in all) cannot
    triangularise a dense 40 x 40 matrix, which takes two to four shifted
    QR steps per eigenvalue: the plan call returns NO_CONVERGENCE."""
    sylt = _sylt()
    rng = np.random.default_rng(805)
    n = (40, 3)
    A = [random_matrix(k, rng, shift=0.0) for k in n]
    with pytest.raises(sylt.SyltError) as ei:
        sylt.Plan.factor(n, [torch.from_numpy(a) for a in A], qr_iter_per_n=1)
    assert ei.value.code == -3
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])  # default cap
    assert plan.separation() > 0


def test_mixed_rejects_x_aliasing_b():
    sylt = _sylt()
    rng = np.random.default_rng(806)
    n = (5, 6, 4)
    A = [random_matrix(k, rng) for k in n]
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    B = dev(_flat(crandn(n, rng)))
    with pytest.raises(sylt.SyltError) as ei:
        sylt.solve(plan, B, precision="mixed", out=B)
    assert ei.value.code == -1


def test_info_reports_phase_times():
    sylt = _sylt()
    rng = np.random.default_rng(807)
    n = (16, 16, 16, 16)
    A = [random_matrix(k, rng) for k in n]
    plan = sylt.Plan.factor(n, [torch.from_numpy(a) for a in A])
    B = dev(_flat(crandn(n, rng)))
    _, info = sylt.solve(plan, B, info=True)
    assert info["ms_transform"] > 0 and info["ms_sweep"] > 0 and info["ms_residual"] == 0
    _, info = sylt.solve(plan, B, precision="mixed", info=True)
    assert info["ms_transform"] > 0 and info["ms_sweep"] > 0 and info["ms_residual"] > 0
