"""Newton steps of the physical cube cell on the GPU (residual kernels, Newton
matrix coefficients, the scaled linear solves, the update) against the
oracle's physical model."""
import numpy as np
import pytest

import oracle as O
from oracle import phys as P
from p4d_inputs import phys as ph
from tests.gpu_util import say, to_np

pytestmark = pytest.mark.gpu


def cell(n=19, nr=(6, 7)):
    from paper_2602_07225_amd import PhysCell
    case = ph.PhysCase(n=n, nr=nr)
    grid = P.Grid(case)
    I = P.applied_current(case)
    return case, grid, I, PhysCell(case, I)


def block_errors(case, grid, a, b):
    sc = P.Scaling(case)
    ra, rb = sc.rows(grid, a), sc.rows(grid, b)
    sl = {"phi": slice(0, grid.off_ce), "ce": slice(grid.off_ce, grid.off_cs[0]),
          "cs": slice(grid.off_cs[0], grid.N)}
    return {k: np.abs(ra[s] - rb[s]).max() / max(np.abs(rb[s]).max(), 1e-300) for k, s in sl.items()}


def perturbed(case, grid, u0, seed):
    rng = np.random.default_rng(seed)
    u = u0.copy()
    u[grid.layer: grid.off_ce] += 2e-3 * rng.standard_normal(grid.off_ce - grid.layer)
    u[grid.off_ce: grid.off_cs[0]] += 20.0 * rng.standard_normal(grid.nnode)
    u[grid.off_cs[0]:] += 50.0 * rng.standard_normal(grid.N - grid.off_cs[0])
    return u


def test_initial_state_and_residual_parity():
    case, grid, I, pc = cell()
    u0 = P.initial_state(case, grid)
    g0 = to_np(pc.initial_state())
    assert np.allclose(g0, u0, rtol=1e-13, atol=0)
    # at rest the residual is the applied current alone
    r = to_np(pc.residual(u0, u0))
    ref = P.residual(case, grid, u0, u0, I)
    e = block_errors(case, grid, r, ref)
    say("  rest", {k: f"{v:.1e}" for k, v in e.items()})
    assert e["phi"] <= 1e-12
    # away from rest every term is active (kinetics, transport at the
    # element-mean c_e, storage, the particle rows)
    for seed in (1, 2):
        u = perturbed(case, grid, u0, seed)
        uold = perturbed(case, grid, u0, seed + 10)
        r = to_np(pc.residual(u, uold))
        ref = P.residual(case, grid, u, uold, I)
        e = block_errors(case, grid, r, ref)
        say(f"  perturbed {seed}", {k: f"{v:.1e}" for k, v in e.items()})
        assert max(e.values()) <= 1e-10


def test_newton_step_matches_oracle():
    case, grid, I, pc = cell()
    u0 = P.initial_state(case, grid)
    uo, hist = P.newton_step(case, grid, u0, I, lin_rtol=1e-10, coarse_max=64)
    ug, info = pc.step(u0, rtol=1e-10)
    ug = to_np(ug)
    say(f"  newton gpu iters={info.iters} lin={info.lin_iters} upd={info.update:.1e}; oracle {len(hist)}")
    assert info.status == 0
    assert abs(info.iters - len(hist)) <= 1
    sc = P.Scaling(case)
    d = sc.rows  # noqa: F841
    diff = P.scaled_update(case, grid, ug - uo)
    assert diff <= 1e-8
    # the converged state satisfies the oracle's residual
    R = P.residual(case, grid, ug, u0, I)
    assert np.abs(sc.rows(grid, R)).max() <= 1e-7


def test_steps_balance_charge_and_lithium():
    case, grid, I, pc = cell(n=28, nr=(8, 8))
    u = pc.initial_state()
    lp = P.linear_problem(case, grid, to_np(u), with_kinetics=False)
    mass = O.Oracle(lp.with_(kappa=0 * lp.kappa, kappa_d=0 * lp.kappa, dce=0 * lp.kappa,
                             sigma=0 * lp.sigma))
    m = O.Oracle(lp).lumped_weights()

    def electrolyte_li(x):
        y = np.zeros(grid.N)
        y[grid.off_ce: grid.off_cs[0]] = x[grid.off_ce: grid.off_cs[0]]
        return mass.apply(y)[grid.off_ce: grid.off_cs[0]].sum()

    li0 = electrolyte_li(to_np(u))
    for step in range(3):
        un, info = pc.step(u)
        say(f"  step {step}: newton {info.iters} lin {info.lin_iters} {info.t_ms:.0f} ms")
        assert info.status == 0 and info.iters <= 15
        x = to_np(un)
        q, _, _, _ = P.kinetics(case, grid, x)
        assert (m * q)[: grid.nea].sum() == pytest.approx(-I, rel=1e-6)
        assert (m * q)[grid.nea:].sum() == pytest.approx(I, rel=1e-6)
        u = un
    assert electrolyte_li(to_np(u)) == pytest.approx(li0, rel=1e-9)


def test_phys_argument_errors():
    from paper_2602_07225_amd import P4DError, _lib
    case = ph.PhysCase(n=19, nr=(6, 7))
    prm = _lib.phys_params(case, -1e-6)
    prm.n = 20
    with pytest.raises(P4DError):
        _lib.p4d_phys_create(prm)
    prm = _lib.phys_params(case, -1e-6)
    prm.el[1].cs0 = prm.el[1].cs_max * 1.5
    with pytest.raises(P4DError):
        _lib.p4d_phys_create(prm)


# ---------------------------------------------------------------------------
# Case II: volume fractions per element, uniform current
# ---------------------------------------------------------------------------
def cell2(n=19, nr=(6, 7), seed=3):
    from paper_2602_07225_amd import PhysCell
    case = ph.case2(n, nr, seed=seed)
    grid = P.Grid(case)
    I = P.applied_current(case)
    return case, grid, I, PhysCell(case, I)


def test_case2_residual_parity():
    case, grid, I, pc = cell2()
    u0 = P.initial_state(case, grid)
    for seed in (0, 1):
        u = u0 if seed == 0 else perturbed(case, grid, u0, seed)
        uold = u0 if seed == 0 else perturbed(case, grid, u0, seed + 10)
        r = to_np(pc.residual(u, uold))
        ref = P.residual(case, grid, u, uold, I)
        e = block_errors(case, grid, r, ref)
        say(f"  case II residual {seed}", {k: f"{v:.1e}" for k, v in e.items()})
        # at rest only the phi rows carry the applied current (c_e and c_s
        # rows are rounding noise there)
        assert (e["phi"] if seed == 0 else max(e.values())) <= 1e-10


def test_case2_newton_step_matches_oracle():
    case, grid, I, pc = cell2()
    u0 = P.initial_state(case, grid)
    uo, hist = P.newton_step(case, grid, u0, I, lin_rtol=1e-10, coarse_max=64)
    ug, info = pc.step(u0, rtol=1e-10)
    ug = to_np(ug)
    say(f"  case II newton gpu iters={info.iters} lin={info.lin_iters}; oracle {len(hist)}")
    assert info.status == 0
    assert abs(info.iters - len(hist)) <= 1
    assert P.scaled_update(case, grid, ug - uo) <= 1e-8
    sc = P.Scaling(case)
    R = P.residual(case, grid, ug, u0, I)
    assert np.abs(sc.rows(grid, R)).max() <= 1e-7
    # back to the homogeneous cell: the Case I residual (uniform current)
    pc.set_fractions(None, None)
    case1 = ph.PhysCase(n=case.n, nr=case.nr, profile="uniform")
    r = to_np(pc.residual(ug, u0))
    e = block_errors(case1, grid, r, P.residual(case1, grid, ug, u0, I))
    # (the c_s rows do not see the fractions: converged, they are rounding
    # noise in both cells)
    assert max(e["phi"], e["ce"]) <= 1e-10


def test_case2_fraction_errors():
    from paper_2602_07225_amd import P4DError, _lib
    case, grid, I, pc = cell2()
    bad = case.eps_s_e.copy()
    lay = ph.element_layers(case)
    bad[np.flatnonzero(lay == 1)[5]] = 0.95          # eps_s + eps_b > 1
    with pytest.raises(P4DError) as e:
        pc.set_fractions(bad, case.eps_b_e)
    assert e.value.status == _lib.P4D_ERR_INVALID_ARG
    with pytest.raises(P4DError):
        _lib.p4d_phys_set_fractions(pc.ctx, pc._dev(case.eps_s_e), None)
    # the failed call left the cell homogeneous: Case I residual (away from
    # rest, so that every block is active)
    u0 = P.initial_state(case, grid)
    u, uold = perturbed(case, grid, u0, 1), perturbed(case, grid, u0, 11)
    case1 = ph.PhysCase(n=case.n, nr=case.nr, profile="uniform")
    r = to_np(pc.residual(u, uold))
    e = block_errors(case1, grid, r, P.residual(case1, grid, u, uold, I))
    assert max(e.values()) <= 1e-10


@pytest.mark.parametrize("transpose", [False, True])
def test_exact_jacobian_apply_parity(transpose):
    """The Newton matrix with the c_e-derivative terms at a state with
    non-uniform c_e, in the scaled variables, against the oracle's."""
    case, grid, I, pc = cell()
    u0 = P.initial_state(case, grid)
    u = perturbed(case, grid, u0, 3)
    sc = P.Scaling(case)
    ref_orc = O.Oracle(sc.problem(P.linear_problem(case, grid, u)))
    x = np.random.default_rng(4).standard_normal(grid.N)
    y = to_np(pc.jacobian_apply(u, x, transpose))
    ref = ref_orc.apply(x, transpose)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    say(f"  exact Jacobian transpose={transpose}: max rel {err:.1e}")
    assert err <= 1e-12
    # the derivative terms are really there
    plain = O.Oracle(sc.problem(P.linear_problem(case, grid, u, exact=False))).apply(x, transpose)
    assert np.abs(plain - ref).max() > 1e3 * err * np.abs(ref).max()


def test_newton_step_schur_krylov_matches_oracle():
    """Newton steps with FGMRES over the Schur complement of the particle
    blocks (exact Newton matrix, its particle blocks eliminated exactly)."""
    case, grid, I, pc = cell()
    u0 = P.initial_state(case, grid)
    uo, hist = P.newton_step(case, grid, u0, I, lin_rtol=1e-10, coarse_max=64)
    ug, info = pc.step(u0, rtol=1e-10, krylov=1)
    ug = to_np(ug)
    say(f"  newton (Schur-Krylov) gpu iters={info.iters} lin={info.lin_iters}; oracle {len(hist)}")
    assert info.status == 0
    assert abs(info.iters - len(hist)) <= 1
    assert P.scaled_update(case, grid, ug - uo) <= 1e-8
