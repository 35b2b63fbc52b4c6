"""Block Gauss-Seidel preconditioner (eq. PGS) on the GPU against the oracle:
every one of the 24 field orderings, forward and transposed, multilevel
V-cycles; the FP32 preconditioner; solves and adjoint solves; option errors."""
import itertools

import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import field_errors, rel, say, solver_for, to_dev, to_np

pytestmark = pytest.mark.gpu

ORDERINGS = list(itertools.permutations(range(4)))


def mixed():
    return pi.make_custom(6, 9, 16, (5, 12), seed=31, sigma_log=0.5, corr_cells=2.0)


@pytest.mark.parametrize("transpose", [False, True])
def test_every_ordering_matches_oracle(transpose):
    p = mixed()
    orc = O.Oracle(p)
    s = solver_for(p)
    r = np.random.default_rng(4).standard_normal(p.N)
    rd = to_dev(r)
    worst = 0.0
    for fields in ORDERINGS:
        order = O.bgs_order(fields)
        orc.setup(pc=O.PC_BGS, bgs_order=order)
        s.setup(pc=2, bgs_order=order)
        z = to_np(s.apply_pc(rd, transpose))
        errs = field_errors(p, z, orc.apply_pc(r, transpose))
        worst = max(worst, max(errs.values()))
        assert max(errs.values()) <= 1e-10, (fields, errs)
    say(f"24 orderings, transpose={transpose}: worst field error {worst:.1e}")


def test_orderings_differ_on_gpu():
    """Distinct orderings give distinct results (the couplings are applied)."""
    p = mixed()
    s = solver_for(p)
    rd = to_dev(np.random.default_rng(5).standard_normal(p.N))
    zs = []
    for fields in [(1, 3, 0, 2), (2, 1, 3, 0), (0, 1, 2, 3), (3, 2, 1, 0)]:
        s.setup(pc=2, bgs_order=O.bgs_order(fields))
        zs.append(to_np(s.apply_pc(rd)))
    for i in range(len(zs)):
        for j in range(i):
            assert rel(zs[i], zs[j]) > 1e-6


def test_fp32_bgs_close_to_fp64():
    p = pi.make_custom(37, 29, 61, (13, 8), seed=23, sigma_log=1.0)
    orc = O.Oracle(p).setup(pc=O.PC_BGS)
    s = solver_for(p, pc_prec=1).setup(pc=2, pc_prec=1)
    r = np.random.default_rng(3).standard_normal(p.N)
    errs = field_errors(p, to_np(s.apply_pc(to_dev(r))), orc.apply_pc(r))
    say("  errors", {k: f"{v:.1e}" for k, v in errs.items()})
    assert errs["all"] <= 1e-3


@pytest.mark.parametrize("pc_prec", [0, 1])
def test_bgs_solve_and_adjoint(pc_prec):
    """Forward and adjoint solves (P_GS^-1 and P_GS^-T) against the oracle's
    solutions at rtol 1e-8."""
    p = pi.make_custom(7, 5, 19, (7, 9), seed=21, sigma_log=1.0, corr_cells=3.0)
    w = pi.functional_weights(p)
    orc = O.Oracle(p).setup(pc=O.PC_BGS, rtol=1e-8, cgs2=True)
    xo, io = orc.solve(p.b)
    lo, jo = orc.solve(w, transpose=True)
    s = solver_for(p, pc_prec=pc_prec).setup(pc=2, pc_prec=pc_prec, rtol=1e-8, cgs2=1)
    x, i1 = s.solve(to_dev(p.b))
    lam, i2 = s.solve_adjoint(to_dev(w))
    say(f"  pc_prec={pc_prec} iters forward gpu={i1.iters} oracle={io.iters}, "
        f"adjoint gpu={i2.iters} oracle={jo.iters}")
    assert i1.status == 0 and i2.status == 0
    tol = 1e-6 if pc_prec == 0 else 1e-5
    assert rel(to_np(x), xo) <= tol
    assert rel(to_np(lam), lo) <= tol
    assert rel(orc.apply(to_np(x)), p.b) <= 1.0001e-8
    assert rel(orc.apply(to_np(lam), True), w) <= 1.0001e-8
    if pc_prec == 0:
        assert abs(i1.iters - io.iters) <= 2 and abs(i2.iters - jo.iters) <= 2


def test_bgs_option_errors():
    from paper_2602_07225_amd import P4DBatch, P4DError, _lib
    p = mixed()
    s = solver_for(p)
    with pytest.raises(P4DError) as e:
        s.setup(pc=2, bgs_order=0)          # not a permutation
    assert e.value.status == _lib.P4D_ERR_INVALID_ARG
    s.setup(pc=2)
    assert s.opts.bgs_order == _lib.P4D_BGS_PAPER_ORDER == O.BGS_PAPER
    with pytest.raises(P4DError) as e:      # ordering differs from the setup
        s.solve(to_dev(p.b), bgs_order=O.bgs_order((0, 1, 2, 3)))
    assert e.value.status == _lib.P4D_ERR_STATE
    B = P4DBatch([p, mixed()])
    with pytest.raises(P4DError) as e:
        B.setup(pc=2)
    assert e.value.status == _lib.P4D_ERR_INVALID_ARG
    B.close()
