"""Batched solves: independent cells of uneven mesh and radial sizes iterate
FGMRES in lockstep; per Arnoldi step the preconditioner of all iterating
cells runs as one launch per stage depth.  Each cell solved in the batch is
compared with the same cell solved alone by the single-cell driver (the
batched kernels repeat its arithmetic unit by unit, so the two agree
exactly) and with the oracle.  Also: the lockstep driver with per-cell
preconditioner launches, a zero right-hand side among the cells, restarts in
lockstep, tile autotuning, and the 64-cell workload."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import field_errors, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def small_cells():
    cells = [
        pi.make_custom(7, 5, 19, (7, 9), seed=41, sigma_log=1.0, corr_cells=3.0),
        pi.make_custom(16, 16, 48, (8, 16), seed=42, sigma_log=0.5),
        pi.make_custom(24, 24, 72, (32, 8), seed=43, sigma_log=0.5),
        pi.make_custom(9, 12, 25, (16, 32), seed=44, sigma_log=1.0, corr_cells=3.0),
        pi.make_custom(37, 29, 61, (13, 8), seed=45, sigma_log=1.0),
        pi.make_custom(11, 10, 30, (18, 20), seed=47, sigma_log=0.5, corr_cells=3.0),
        pi.make_custom(6, 9, 16, (5, 12), seed=46, sigma_log=0.5, corr_cells=2.0),
    ]
    cells[-1].b = np.zeros_like(cells[-1].b)   # converged before the first iteration
    return cells


_cache = {}


def batch_for(key, **kw):
    from paper_2602_07225_amd import P4DBatch
    if key not in _cache:
        cells = small_cells()
        _cache[key] = (cells, P4DBatch(cells, **kw))
    return _cache[key]


def check_against_single(B, cells, xs, infos, **opts):
    for i, p in enumerate(cells):
        xb = to_np(xs[i])
        x1, i1 = B.solve_cell(i, to_dev(p.b), **opts)
        x1 = to_np(x1)
        say(f"  cell {i} N={p.N}: batch iters={infos[i].iters} restarts={infos[i].restarts} "
            f"single iters={i1.iters}, max|diff|={np.max(np.abs(xb - x1)):.1e}")
        assert infos[i].status == 0 and i1.status == 0
        assert infos[i].iters == i1.iters and infos[i].restarts == i1.restarts
        assert np.array_equal(xb, x1), f"cell {i}"


def test_batch_driver_with_per_cell_preconditioner():
    """The lockstep driver and the batched operator / Krylov kernels alone:
    the preconditioner is applied by the single-cell launches, cell after
    cell."""
    cells, B = batch_for(("small", 0, 0), pc_prec=0)
    say(f"batch of {len(cells)} cells, per-cell preconditioner launches")
    B.setup(rtol=1e-8, maxit=200)
    B.set_pc_mode(1)
    try:
        xs, infos = B.solve([p.b for p in cells])
    finally:
        B.set_pc_mode(0)
    check_against_single(B, cells, xs, infos)


@pytest.mark.parametrize("pc_prec,z_fp32", [(0, 0), (1, 0), (1, 1)])
def test_batch_equals_single_and_oracle(pc_prec, z_fp32):
    cells, B = batch_for(("small", pc_prec, z_fp32), pc_prec=pc_prec, z_fp32=bool(z_fp32))
    say(f"batch of {len(cells)} cells, pc_prec={pc_prec} z_fp32={z_fp32}")
    B.setup(rtol=1e-8, maxit=200)
    xs, infos = B.solve([p.b for p in cells])
    check_against_single(B, cells, xs, infos)
    assert infos[-1].iters == 0 and not np.any(to_np(xs[-1]))
    for i, p in enumerate(cells[:-1]):
        # reference at rtol 1e-9 (its near-null error stays out of the count)
        orc = O.Oracle(p).setup(rtol=1e-9, maxit=150)
        xo, _ = orc.solve(p.b)
        err = rel(to_np(xs[i]), xo)
        say(f"  cell {i}: rel err vs oracle {err:.2e}")
        assert err <= 1e-6


@pytest.mark.parametrize("pc_prec", [0, 1])
def test_batch_persistent_launch_equals_single(pc_prec):
    """One cooperative launch per preconditioner application (the stage
    depths walked one after another by the whole grid, with a grid barrier
    between depths): every cell equals the cell solved alone, also with
    restarts, and a repeated solve equals the first."""
    cells, B = batch_for(("small", pc_prec, 0), pc_prec=pc_prec)
    say(f"persistent launch, pc_prec={pc_prec}")
    B.setup(rtol=1e-8, maxit=200)
    B.set_pc_mode(2)
    try:
        say("  solve 1")
        xs, infos = B.solve([p.b for p in cells])
        say("  solve 2 (restart 5)")
        xs2, infos2 = B.solve([p.b for p in cells], restart=5, maxit=300)
        say("  solve 3")
        xs3, infos3 = B.solve([p.b for p in cells])
    finally:
        B.set_pc_mode(0)
    check_against_single(B, cells, xs, infos)
    check_against_single(B, cells, xs2, infos2, restart=5, maxit=300)
    for a, b in zip(xs, xs3):
        assert np.array_equal(to_np(a), to_np(b))


def test_batch_restarts_in_lockstep():
    """Restart length 3: every cell runs several cycles, finishing them at
    different steps."""
    cells, B = batch_for(("small", 0, 0), pc_prec=0)
    B.setup(rtol=1e-8)
    say("restart 3")
    xs, infos = B.solve([p.b for p in cells], restart=3, maxit=300)
    assert max(inf.restarts for inf in infos) >= 3
    check_against_single(B, cells, xs, infos, restart=3, maxit=300)


def test_batch_autotune_keeps_results():
    """The smoother tile shape changes the work split, not the arithmetic."""
    cells, B = batch_for(("small", 1, 0), pc_prec=1)
    B.setup(rtol=1e-8, maxit=200)
    say("autotune")
    x0, i0 = B.solve([p.b for p in cells])
    tiles = B.autotune()
    say(f"  tiles {tiles}")
    assert all(t[0] in (16, 32, 64) and 2 <= t[1] <= 16 for t in tiles)
    x1, i1 = B.solve([p.b for p in cells])
    for a, b, ia, ib in zip(x0, x1, i0, i1):
        assert ia.iters == ib.iters
        assert np.array_equal(to_np(a), to_np(b))


@pytest.mark.timeout(900)
def test_C4_batch_64_cells():
    """The 64-cell workload (sides 16..48, N_r in {8, 16, 32}, lognormal
    conductivities), FP32 preconditioner with autotuned tiles: every cell
    converges to rtol 1e-8 (residual confirmed with the oracle operator),
    equals the single-cell solve, and one cell of every (side, anode N_r,
    cathode N_r) class present matches the oracle's FP64 solve at the same
    tolerance to 1e-6 per field.  (Against a tighter oracle solve, rtol 1e-9,
    the largest difference is 1.1e-6, on a side-48 cell with N_r 32 / 16: the
    error that any rtol-1e-8 solution of that cell carries along its
    near-null modes -- the FP64 and FP32 preconditioners give the same
    figures on the small cells -- not a disagreement of the two solvers.)"""
    from paper_2602_07225_amd import P4DBatch
    cells = pi.make_batch(64)
    Ntot = sum(p.N for p in cells)
    say(f"C4: {len(cells)} cells, {Ntot} unknowns")
    B = P4DBatch(cells, pc_prec=1)
    B.setup(rtol=1e-8)
    tiles = B.autotune()
    say(f"  distinct tiles {sorted(set(tiles))}")
    xs, infos = B.solve([p.b for p in cells])
    say(f"  batch time {infos[0].t_solve_ms:.1f} ms, iters "
        f"{min(i.iters for i in infos)}..{max(i.iters for i in infos)}")
    check_against_single(B, cells, xs, infos)
    for i, p in enumerate(cells):
        r = rel(O.Oracle(p).apply(to_np(xs[i])), p.b)
        assert r <= 1.0001e-8, f"cell {i}: residual {r:.2e}"
    # one persistent launch per application: the same results, bit for bit
    B.set_pc_mode(2)
    try:
        xp, ip = B.solve([p.b for p in cells])
    finally:
        B.set_pc_mode(0)
    say(f"  persistent launch: batch time {ip[0].t_solve_ms:.1f} ms")
    for i in range(len(cells)):
        assert ip[i].iters == infos[i].iters
        assert np.array_equal(to_np(xp[i]), to_np(xs[i])), f"cell {i}"
    first = {}
    for i, p in enumerate(cells):
        first.setdefault((p.nx, tuple(p.nr)), i)
    say(f"  {len(first)} (side, N_r pair) classes")
    worst = 0.0
    for (side, nr), i in sorted(first.items()):
        xo, _ = O.Oracle(cells[i]).setup(rtol=1e-8).solve(cells[i].b)
        errs = field_errors(cells[i], to_np(xs[i]), xo)
        worst = max(worst, max(errs.values()))
        say(f"  cell {i} side {side} N_r {nr} N={cells[i].N}: rel err vs oracle "
            f"{errs['all']:.2e} (largest field {max(errs.values()):.2e})")
    assert worst <= 1e-6
    B.close()
