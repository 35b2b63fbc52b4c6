"""FGMRES over the Schur complement of the particle blocks on the GPU against
the oracle: the operator S (forward and transposed), solves and adjoint solves
in both preconditioner precisions, the equivalence with the full-space
iteration, and the cube workload."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import field_errors, rel, say, solver_for, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = {
    "C1": lambda: pi.make_config(1),
    "odd_lognormal": lambda: pi.make_custom(7, 5, 19, (7, 9), seed=21, sigma_log=1.0, corr_cells=3.0),
    "ragged_multilevel": lambda: pi.make_custom(37, 29, 61, (13, 8), seed=23, sigma_log=1.0),
}

_cache = {}


def case(name):
    if name not in _cache:
        p = CASES[name]()
        _cache[name] = (p, O.Oracle(p))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [False, True])
def test_schur_operator_parity(name, transpose):
    """S y from omega_j on the GPU against A_yy y - A_ys A_ss^-1 A_sy y
    formed by the oracle with its operator and tridiagonal solves."""
    p, orc = case(name)
    nm = p.offsets[3]
    say(f"schur operator {name} transpose={transpose} Nm={nm}")
    s = solver_for(p)
    y = np.random.default_rng(7).standard_normal(nm)
    w = to_np(s.apply_schur(to_dev(y), transpose))
    ref = orc.schur_apply(y, transpose)
    assert w.shape == (nm,)
    assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", list(CASES))
def test_schur_krylov_solve_parity(name):
    """GPU and oracle iterations over S at rtol 1e-8: solutions agree to
    <= 1e-6 per field, the full residual meets the tolerance."""
    p, orc = case(name)
    say(f"schur krylov solve {name}")
    orc.setup(rtol=1e-8, krylov=O.KRYLOV_SCHUR)
    xo, io = orc.solve(p.b)
    s = solver_for(p).setup(rtol=1e-8)
    x, info = s.solve(to_dev(p.b), krylov=1)
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  iters gpu={info.iters} oracle={io.iters} relres={info.relres_true:.2e}",
        {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and io.status == 0
    assert info.relres_true <= 1.0001e-8
    assert abs(info.iters - io.iters) <= 2
    assert max(errs.values()) <= 1e-6
    assert rel(orc.apply(x), p.b) <= 1.0001e-8
    assert info.relres_true == pytest.approx(rel(orc.apply(x), p.b), rel=1e-3)


@pytest.mark.parametrize("pc_prec,zfp32", [(1, False), (1, True)])
def test_schur_krylov_fp32_preconditioner(pc_prec, zfp32):
    p, orc = case("ragged_multilevel")
    # reference at rtol 1e-9: its own near-null error stays out of the count
    orc.setup(rtol=1e-9, maxit=150)
    xo, _ = orc.solve(p.b)
    s = solver_for(p, pc_prec=pc_prec, z_fp32=zfp32).setup(pc_prec=pc_prec, rtol=1e-8,
                                                            z_fp32=int(zfp32))
    x, info = s.solve(to_dev(p.b), krylov=1)
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  fp32 pc z_fp32={zfp32}: iters {info.iters}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and info.relres_true <= 1.0001e-8
    assert rel(orc.apply(x), p.b) <= 1.0001e-8
    # (the FP32 Z basis, an option outside the spec configuration,
    # rounds the vectors that build the solution: its error is allowed 5e-6,
    # as in the full-space test)
    assert max(errs.values()) <= (5e-6 if zfp32 else 1e-6)


@pytest.mark.parametrize("name", ["C1", "odd_lognormal"])
def test_schur_krylov_adjoint(name):
    """S^T iteration for the adjoint: the transposed operator, right-hand
    side and back-substitution."""
    p, orc = case(name)
    w = pi.functional_weights(p)
    orc.setup(rtol=1e-10)
    lo, _ = orc.solve(w, transpose=True)
    s = solver_for(p).setup(rtol=1e-10)
    lam, info = s.solve_adjoint(to_dev(w), krylov=1)
    lam = to_np(lam)
    say(f"  adjoint {name}: iters {info.iters}, rel err {rel(lam, lo):.1e}")
    assert info.status == 0
    assert rel(lam, lo) <= 1e-6
    assert rel(orc.apply(lam, True), w) <= 1.0001e-10


def test_schur_krylov_equals_full_space_solution():
    """The two Krylov spaces solve the same system: solutions agree, and the
    reduced iteration takes no more steps than the full one plus one."""
    p, _ = case("ragged_multilevel")
    s = solver_for(p).setup(rtol=1e-10)
    xf, i_f = s.solve(to_dev(p.b))
    xs, i_s = s.solve(to_dev(p.b), krylov=1)
    say(f"  iters full={i_f.iters} schur={i_s.iters}")
    assert i_f.status == 0 and i_s.status == 0
    assert rel(to_np(xs), to_np(xf)) <= 1e-7
    assert i_s.iters <= i_f.iters + 1


def test_schur_krylov_options_and_edges():
    import torch
    from paper_2602_07225_amd import P4DError, _lib
    p, _ = case("C1")
    s = solver_for(p)
    with pytest.raises(P4DError) as e:
        s.setup(pc=1, krylov=1)              # needs the SCHUR preconditioner
    assert e.value.status == _lib.P4D_ERR_INVALID_ARG
    s.setup()
    x, info = s.solve(torch.zeros(p.N, dtype=torch.float64, device="cuda"), krylov=1)
    assert info.status == 0 and info.iters == 0 and not to_np(x).any()
    x, info = s.solve(to_dev(p.b), krylov=1, maxit=2)
    assert info.status == _lib.P4D_NOT_CONVERGED and info.iters == 2
    x, info = s.solve(to_dev(p.b), krylov=1, restart=2, maxit=5000)
    assert info.status == 0 and info.relres_true <= 1.0001e-8
    from paper_2602_07225_amd import P4DBatch
    B = P4DBatch([p, case("odd_lognormal")[0]])
    B.setup()
    with pytest.raises(P4DError) as e:      # batches iterate in the full space
        B.solve([p.b, case("odd_lognormal")[0].b], krylov=1)
    assert e.value.status == _lib.P4D_ERR_INVALID_ARG
    B.close()


def test_C2_schur_krylov_solve():
    """The cube workload (15.3 M unknowns) with the Krylov space reduced to
    the 2.2 M electrode-level unknowns, against the oracle's reduced solve."""
    p = pi.make_config(2)
    orc = O.Oracle(p)
    say("C2 schur krylov solve (oracle ~30 s on the host)")
    orc.setup(rtol=1e-8, krylov=O.KRYLOV_SCHUR)
    xo, io = orc.solve(p.b)
    s = solver_for(p).setup(rtol=1e-8)
    x, info = s.solve(to_dev(p.b), krylov=1)
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  iters gpu={info.iters} oracle={io.iters} relres={info.relres_true:.2e}",
        {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and io.status == 0
    assert info.relres_true <= 1.0001e-8
    assert max(errs.values()) <= 1e-6
