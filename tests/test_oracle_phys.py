"""Pins of the oracle's physical model (Sec. 2 equations with the appendix
parameters, Case I cube of Sec. 5): material functions, the rest state, the
Newton matrix against finite differences of the residual, charge balance and
electrolyte lithium conservation of converged steps."""
import numpy as np
import pytest

import oracle as O
from oracle import phys as P
from p4d_inputs import phys as ph


@pytest.fixture(scope="module")
def cube():
    case = ph.PhysCase(n=19, nr=(6, 7))
    grid = P.Grid(case)
    return case, grid


def test_material_function_derivatives():
    """Open-circuit potentials: the returned derivatives equal central
    differences over the stoichiometry range; kappa stays positive and D_e
    decreases over 0..3000 mol/m^3."""
    th = np.linspace(0.05, 0.95, 37)
    h = 1e-6
    for f in (P.ocp_negative, P.ocp_positive):
        u, du = f(th)
        fd = (f(th + h)[0] - f(th - h)[0]) / (2 * h)
        assert np.allclose(du, fd, rtol=1e-6, atol=1e-6)
    c = np.linspace(1.0, 3000.0, 301)
    assert np.all(P.kappa_bulk(c) > 0)
    assert np.all(np.diff(P.de_bulk(c)) < 0)


def test_layers_and_grid(cube):
    case, grid = cube
    # 225 um cube: 100 / 25 / 100 um on element faces
    h = case.h
    assert (case.na - 1) * h == pytest.approx(100e-6)
    assert (case.na + case.ns) * h == pytest.approx(125e-6)
    assert grid.nc == case.na
    assert (grid.emat == 0).sum() == (grid.emat == 1).sum()


def test_rest_state_is_a_solution_at_zero_current(cube):
    """c_e = c_e0, c_s = c_s0 and zero overpotential: every residual row
    vanishes (to rounding) when no current is applied."""
    case, grid = cube
    u0 = P.initial_state(case, grid)
    R = P.residual(case, grid, u0, u0, 0.0)
    q, _, _, _ = P.kinetics(case, grid, u0)
    assert np.abs(q).max() < 1e-9
    sc = P.Scaling(case)
    assert np.abs(sc.rows(grid, R)).max() < 1e-9


def _fd(case, grid, u, u_old, I, v, eps):
    return (P.residual(case, grid, u + eps * v, u_old, I) -
            P.residual(case, grid, u - eps * v, u_old, I)) / (2 * eps)


def _block_errors(case, grid, a, b, rows=("phis", "phie", "ce", "cs")):
    """Relative error per field block of the scaled rows D_r a against D_r b
    (in SI units the blocks differ by ten orders of magnitude)."""
    sc = P.Scaling(case)
    ra, rb = sc.rows(grid, a), sc.rows(grid, b)
    sl = {"phis": slice(grid.layer, grid.off_pe), "phie": slice(grid.off_pe, grid.off_ce),
          "ce": slice(grid.off_ce, grid.off_cs[0]), "cs": slice(grid.off_cs[0], grid.N)}
    return {k: np.linalg.norm(ra[sl[k]] - rb[sl[k]]) / np.linalg.norm(rb[sl[k]]) for k in rows}


def _direction(grid, rng, ce=True):
    v = rng.standard_normal(grid.N)
    v[: grid.off_ce] *= 1e-3            # volts
    v[grid.off_ce: grid.off_cs[0]] *= 1.0 if ce else 0.0
    v[grid.off_cs[0]:] *= 10.0
    v[: grid.layer] = 0.0               # grounded phi_s
    return v


def test_newton_matrix_is_the_jacobian_at_rest(cube):
    """At the rest state the transport coefficients are stationary in c_e
    (uniform c_e, no gradients), so the Newton matrix is the exact Jacobian:
    it matches central differences of the residual to O(eps^2)."""
    case, grid = cube
    u0 = P.initial_state(case, grid)
    I = P.applied_current(case)
    J = O.Oracle(P.linear_problem(case, grid, u0))
    v = _direction(grid, np.random.default_rng(1))
    Jv = J.apply(v)
    e2 = _block_errors(case, grid, _fd(case, grid, u0, u0, I, v, 1e-2), Jv)
    e3 = _block_errors(case, grid, _fd(case, grid, u0, u0, I, v, 1e-3), Jv)
    for k in e3:
        assert e3[k] < 1e-7, (k, e2, e3)


def test_newton_matrix_is_the_jacobian_after_a_step(cube):
    """After a discharge step c_e is no longer uniform and the transport
    coefficients move with it: the Newton matrix, with the c_e-derivative
    terms of the element coefficients, still equals central differences of
    the residual in every direction (c_e-only directions included), and its
    transpose is the adjoint of it."""
    case, grid = cube
    u0 = P.initial_state(case, grid)
    I = P.applied_current(case)
    u1, _ = P.newton_step(case, grid, u0, I)
    J = O.Oracle(P.linear_problem(case, grid, u1))
    for seed, ce in ((2, True), (3, False)):
        v = _direction(grid, np.random.default_rng(seed), ce=ce)
        Jv = J.apply(v)
        err = _block_errors(case, grid, _fd(case, grid, u1, u0, I, v, 1e-3), Jv)
        assert max(err.values()) < 1e-7, err
    w = np.zeros(grid.N)
    w[grid.off_ce: grid.off_cs[0]] = np.random.default_rng(4).standard_normal(grid.nnode)
    err = _block_errors(case, grid, _fd(case, grid, u1, u0, I, w, 1e-3), J.apply(w),
                        rows=("phie", "ce"))
    assert max(err.values()) < 1e-7, err
    # without the derivative terms the c_e rows miss the transport derivative
    Jp = O.Oracle(P.linear_problem(case, grid, u1, exact=False))
    errp = _block_errors(case, grid, _fd(case, grid, u1, u0, I, w, 1e-3), Jp.apply(w),
                         rows=("phie", "ce"))
    assert max(errp.values()) > 1e-4, errp
    # adjoint: <J x, y> = <x, J^T y>
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(grid.N), rng.standard_normal(grid.N)
    lhs, rhs = J.apply(x) @ y, x @ J.apply(y, True)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(J.apply(x)) * np.linalg.norm(y)


def test_newton_converges_quadratically(cube):
    """The second 60 s step from the first converges quadratically: each
    scaled update is at most a constant times the square of the previous."""
    case, grid = cube
    u0 = P.initial_state(case, grid)
    I = P.applied_current(case)
    u1, _ = P.newton_step(case, grid, u0, I)
    _, hist = P.newton_step(case, grid, u1, I)
    d = [h[0] for h in hist]
    assert len(d) <= 5 and d[-1] <= 1e-9
    for a, b in zip(d[:-1], d[1:]):
        if a < 1e-2:
            assert b <= 10.0 * a * a, d


def test_converged_step_balances_charge_and_conserves_electrolyte_lithium(cube):
    """Two 60 s steps at 1C: Newton converges; the reaction current of each
    electrode equals the applied current (negative electrode +|I|, positive
    -|I|, discharge); the electrolyte lithium sum_e eps int c_e is conserved;
    the negative particles lose lithium at the surface and the positive ones
    gain it."""
    case, grid = cube
    u = P.initial_state(case, grid)
    I = P.applied_current(case)
    lp = P.linear_problem(case, grid, u, with_kinetics=False)
    mass = O.Oracle(lp.with_(kappa=0 * lp.kappa, kappa_d=0 * lp.kappa, dce=0 * lp.kappa,
                             sigma=0 * lp.sigma))
    m = O.Oracle(lp).lumped_weights()

    def electrolyte_li(x):
        y = np.zeros(grid.N)
        y[grid.off_ce: grid.off_cs[0]] = x[grid.off_ce: grid.off_cs[0]]
        return mass.apply(y)[grid.off_ce: grid.off_cs[0]].sum() * case.dt

    li0 = electrolyte_li(u)
    for _ in range(2):
        un, hist = P.newton_step(case, grid, u, I)
        assert hist[-1][0] <= 1e-9 and len(hist) < 15
        q, _, _, _ = P.kinetics(case, grid, un)
        assert (m * q)[: grid.nea].sum() == pytest.approx(-I, rel=1e-7)
        assert (m * q)[grid.nea:].sum() == pytest.approx(I, rel=1e-7)
        assert np.all(grid.surface(un, 0) < grid.surface(u, 0))
        assert np.all(grid.surface(un, 1) > grid.surface(u, 1))
        u = un
    assert electrolyte_li(u) == pytest.approx(li0, rel=1e-10)


# ---------------------------------------------------------------------------
# Case II: volume fractions per element
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def hetero():
    case = ph.case2(19, (6, 7), seed=3)
    return case, P.Grid(case)


def test_case2_fields_and_uniform_current(hetero):
    """Fractions inside (0, 1) with the porosity as the remainder; the
    uniform top-face current is the lumped face weight times I / area."""
    case, grid = hetero
    lay = ph.element_layers(case)
    por = ph.porosity(case)
    el = lay >= 0
    assert np.all(case.eps_s_e[el] > 0) and np.all(case.eps_b_e[el] > 0) and np.all(por[el] > 0)
    assert np.allclose(por[el], 1.0 - case.eps_s_e[el] - case.eps_b_e[el], rtol=0, atol=0)
    assert np.all(por[~el] == ph.SEPARATOR_EPS)
    assert np.std(por[el]) > 0.02                       # really heterogeneous
    I = P.applied_current(case)
    f = P.face_source(case, grid, I)
    top = f[grid.ne - grid.layer:]
    h, n = case.h, case.n
    w1 = np.full(n, h)
    w1[0] = w1[-1] = h / 2
    assert np.allclose(top, (I / ph.CELL_EDGE ** 2) * np.outer(w1, w1).reshape(-1), rtol=1e-13, atol=0)
    assert np.all(f[: grid.ne - grid.layer] == 0)


def test_case2_coefficients_follow_the_local_fractions(hetero):
    """sigma_eff = eps_s^1.5 sigma and kappa_eff = eps^1.5 kappa(c_e) per
    element at the rest state (uniform c_e)."""
    case, grid = hetero
    u0 = P.initial_state(case, grid)
    sig, kap, kd, dce = P.element_coefficients(case, grid, u0)
    lay = ph.element_layers(case)
    por = ph.porosity(case)
    for el in (0, 1):
        sel = lay == el
        assert np.allclose(sig[sel], case.eps_s_e[sel] ** 1.5 * case.electrodes[el].sigma, rtol=1e-14)
    assert np.all(sig[lay < 0] == 0)
    assert np.allclose(kap, por ** 1.5 * P.kappa_bulk(ph.CE0), rtol=1e-14)
    assert np.allclose(dce, por ** 1.5 * P.de_bulk(ph.CE0), rtol=1e-14)


def test_case2_zero_variance_is_the_homogeneous_cell():
    """Fractions fixed at the table means reproduce the homogeneous cell
    (same residual up to the rounding of 1 - eps_s - eps_b)."""
    case1 = ph.PhysCase(n=19, nr=(6, 7), profile="uniform")
    grid = P.Grid(case1)
    lay = ph.element_layers(case1)
    fs = np.where(lay == 0, 0.6, 0.5)
    fb = np.where(lay == 0, 0.1, 0.2)
    case = ph.PhysCase(n=19, nr=(6, 7), profile="uniform", eps_s_e=fs, eps_b_e=fb)
    u0 = P.initial_state(case1, grid)
    rng = np.random.default_rng(4)
    u = u0.copy()
    u[grid.off_ce: grid.off_cs[0]] += 30.0 * rng.standard_normal(grid.nnode)
    I = P.applied_current(case1)
    sc = P.Scaling(case1)
    r1 = sc.rows(grid, P.residual(case1, grid, u, u0, I))
    r2 = sc.rows(grid, P.residual(case, grid, u, u0, I))
    assert np.abs(r1 - r2).max() <= 1e-12 * np.abs(r1).max()


def test_case2_newton_matrix_is_the_jacobian_at_rest(hetero):
    """At the rest state (uniform c_e) the Newton matrix of the heterogeneous
    cell is the exact Jacobian: central differences agree to O(eps^2)."""
    case, grid = hetero
    u0 = P.initial_state(case, grid)
    I = P.applied_current(case)
    J = O.Oracle(P.linear_problem(case, grid, u0))
    v = _direction(grid, np.random.default_rng(5))
    Jv = J.apply(v)
    e3 = _block_errors(case, grid, _fd(case, grid, u0, u0, I, v, 1e-3), Jv)
    for k in e3:
        assert e3[k] < 1e-7, (k, e3)


def test_case2_step_balances_charge_and_conserves_lithium(hetero):
    """A converged 60 s step of the heterogeneous cell: reaction currents
    equal the applied current per electrode, and the electrolyte lithium
    int eps c_e (mass matrix of the porosity field, assembled here by
    quadrature) is unchanged."""
    from tests import qref
    case, grid = hetero
    u = P.initial_state(case, grid)
    I = P.applied_current(case)
    n, h = case.n, case.h
    coords = [np.arange(n) * h] * 3
    M = qref.assemble_box(n, n, n, np.zeros(grid.nelem), ph.porosity(case), *coords)
    li = lambda x: M @ x[grid.off_ce: grid.off_cs[0]]  # noqa: E731
    li0 = li(u).sum()
    un, hist = P.newton_step(case, grid, u, I)
    assert hist[-1][0] <= 1e-9 and len(hist) < 15
    m = O.Oracle(P.linear_problem(case, grid, un)).lumped_weights()
    q, _, _, _ = P.kinetics(case, grid, un)
    assert (m * q)[: grid.nea].sum() == pytest.approx(-I, rel=1e-7)
    assert (m * q)[grid.nea:].sum() == pytest.approx(I, rel=1e-7)
    assert li(un).sum() == pytest.approx(li0, rel=1e-10)
    # heterogeneity shows: c_e differs from the homogeneous cell's step
    case1 = ph.PhysCase(n=19, nr=(6, 7), profile="uniform")
    u1, _ = P.newton_step(case1, grid, P.initial_state(case1, grid), I)
    d = np.abs(un - u1)[grid.off_ce: grid.off_cs[0]].max()
    assert d > 1e-3 * np.abs(u1[grid.off_ce: grid.off_cs[0]] - ph.CE0).max()
