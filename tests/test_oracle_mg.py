"""Pins of the oracle's multigrid pieces (the electrode-level block solves
of Sec. 4.2, here geometric Galerkin multigrid)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle as O
import p4d_inputs as pi
from tests import qref


@pytest.mark.parametrize("dims", [(9, 9, 9), (8, 7, 6), (5, 6, 4), (4, 3, 7)])
@pytest.mark.parametrize("lognormal", [False, True])
def test_G1_galerkin_equals_coarse_assembly(dims, lognormal):
    """P^T K_h(sigma) P equals the stiffness of the coarse Q1 basis under the
    fine-level bilinear form (nested conforming spaces, including the odd
    last interval of 'even plus last' coarsening)."""
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    ne = (nx - 1) * (ny - 1) * (nz - 1)
    coef = np.exp(rng.standard_normal(ne)) if lognormal else np.ones(ne)
    Kf = qref.assemble_box(nx, ny, nz, coef)
    S = qref.dense_to_stencil(dims, Kf)
    Sc, cdims = O.rap(dims, S)
    Ac = qref.stencil_to_dense(cdims, Sc)
    xs = [np.arange(n, dtype=float) for n in dims]
    Aq, qdims = qref.galerkin_by_quadrature(*xs, coef)
    assert qdims == cdims
    assert np.allclose(Ac, Aq, atol=1e-12 * np.abs(Aq).max())


def test_G1_mass_term():
    """Galerkin product of a mass + stiffness operator equals the coarse
    assembly of both (here against the dense triple product with the
    tensor-product interpolation built from the coarse coordinates)."""
    dims = (6, 5, 7)
    rng = np.random.default_rng(1)
    ne = 5 * 4 * 6
    A = qref.assemble_box(*dims, rng.uniform(0.5, 2, ne), rng.uniform(0.5, 2, ne))
    S = qref.dense_to_stencil(dims, A)
    Sc, cdims = O.rap(dims, S)

    def P1(n):
        xc = qref.coarse_coords(np.arange(n, dtype=float))
        P = np.zeros((n, len(xc)))
        for i in range(n):
            I = min(np.searchsorted(xc, i, side="right") - 1, len(xc) - 2)
            t = (i - xc[I]) / (xc[I + 1] - xc[I])
            P[i, I] += 1 - t
            P[i, I + 1] += t
        return P
    Px, Py, Pz = (P1(n) for n in dims)
    P = np.kron(Pz, np.kron(Py, Px))
    ref = P.T @ A.toarray() @ P
    assert np.allclose(qref.stencil_to_dense(cdims, Sc), ref, atol=1e-13 * np.abs(ref).max())


def spd_box(dims, seed=0):
    rng = np.random.default_rng(seed)
    ne = (dims[0] - 1) * (dims[1] - 1) * (dims[2] - 1)
    A = qref.assemble_box(*dims, rng.uniform(0.5, 2, ne), 0.05 * np.ones(ne))
    return qref.dense_to_stencil(dims, A), A.toarray()


def test_gershgorin_bound():
    dims = (4, 5, 3)
    S, A = spd_box(dims)
    ref = np.max(np.abs(A).sum(axis=1) / np.diag(A))
    assert O.gershgorin(dims, S) == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_chebyshev_closed_form(deg):
    """From x0 = 0, degree-k Chebyshev smoothing on D^-1 S over
    [lmax/4, lmax] leaves the error E x* with
    E = q(D^-1 S), q(l) = T_k((theta - l)/delta) / T_k(theta/delta)."""
    dims = (4, 4, 5)
    S, A = spd_box(dims, seed=deg)
    n = A.shape[0]
    lmax = O.gershgorin(dims, S)
    lmin = lmax / 4
    theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
    d = np.diag(A)
    C = A / np.sqrt(np.outer(d, d))
    lam, Q = np.linalg.eigh(C)
    Tk = np.zeros(deg + 1); Tk[-1] = 1.0
    q = npcheb.chebval((theta - lam) / delta, Tk) / npcheb.chebval(theta / delta, Tk)
    E = (Q * q) @ Q.T
    E = np.diag(1 / np.sqrt(d)) @ E @ np.diag(np.sqrt(d))
    b = np.random.default_rng(9).standard_normal(n)
    xstar = np.linalg.solve(A, b)
    ref = xstar - E @ xstar
    got = O.chebyshev(dims, S, deg, b)
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def mg_problem(nx, ny, nz, seed=2, sigma_log=1.0):
    p = pi.make_custom(nx, ny, nz, (6, 6), seed=seed, sigma_log=sigma_log, corr_cells=3.0)
    orc = O.Oracle(p)
    orc.setup()
    return p, orc


@pytest.mark.parametrize("shape", [(10, 9, 30), (16, 16, 48)])
def test_hierarchy_shapes(shape):
    p, orc = mg_problem(*shape)
    for box in range(4):
        lv = orc.mg_levels(box)
        for (d0, _), (d1, _) in zip(lv[:-1], lv[1:]):
            assert d1 == tuple(n if n <= 2 else n // 2 + 1 for n in d0)
            assert d0[0] * d0[1] * d0[2] > 64      # default coarse_max
        last = lv[-1][0]
        assert last[0] * last[1] * last[2] <= 64 or len(lv) == 1


@pytest.mark.parametrize("shape", [(10, 9, 30), (16, 16, 48)])
def test_G2_vcycle_symmetric(shape):
    p, orc = mg_problem(*shape)
    rng = np.random.default_rng(4)
    for box in range(4):
        n = orc.box_slice(box).stop - orc.box_slice(box).start
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        a = orc.vcycle(box, x) @ y
        b = x @ orc.vcycle(box, y)
        assert a == pytest.approx(b, rel=1e-11)


@pytest.mark.parametrize("shape", [(10, 9, 30), (16, 16, 48)])
def test_vcycle_contracts(shape):
    """Used as a stationary iteration x += V(b - S x) on its own fine
    operator, the V-cycle reduces the residual by a mesh-independent factor
    (well below 1)."""
    p, orc = mg_problem(*shape)
    rng = np.random.default_rng(8)
    for box in range(4):
        dims = orc.mg_levels(box)[0][0]
        S = orc.mg_stencil(box, 0)
        b = rng.standard_normal(dims[0] * dims[1] * dims[2])
        x = np.zeros_like(b)
        r0 = np.linalg.norm(b)
        for _ in range(6):
            x = x + orc.vcycle(box, b - O.stencil_apply(dims, S, x))
        rate = (np.linalg.norm(b - O.stencil_apply(dims, S, x)) / r0) ** (1 / 6)
        assert rate < 0.35, (box, rate)


def test_fine_operator_is_schur_block():
    """Level-0 operator of the phi_e box = K_kappa + diag(omega m g) and of
    the c_e box = M_eps/dt + K_kappa - diag(omega tc m e), assembled
    independently."""
    p, orc = mg_problem(6, 5, 13)
    h = p.h
    nodes = (p.nx, p.ny, p.nz)
    coords = [np.arange(n) * h for n in nodes]
    lay = np.repeat(np.array([0 if k + 1 < p.na else (1 if k >= p.na + p.ns else -1)
                              for k in range(p.nz - 1)]), (p.nx - 1) * (p.ny - 1))
    eps = np.where(lay >= 0, p.eps_elec, p.eps_sep)
    Kk = qref.assemble_box(*nodes, p.kappa, None, *coords).toarray()
    Me = qref.assemble_box(*nodes, np.zeros(p.n_elem), eps / p.dt, *coords).toarray()
    m, w = orc.lumped_weights(), orc.omega()
    k = np.repeat(np.arange(p.nz), p.nx * p.ny)
    elec = (k < p.na) | (k >= p.na + p.ns)
    dg = np.zeros(p.n_nodes); dg[elec] = w * m * p.g
    de = np.zeros(p.n_nodes); de[elec] = -w * p.tc * m * p.e
    S2 = qref.stencil_to_dense(nodes, orc.mg_stencil(2, 0))
    S3 = qref.stencil_to_dense(nodes, orc.mg_stencil(3, 0))
    assert np.allclose(S2, Kk + np.diag(dg), atol=1e-14 * np.abs(Kk).max())
    assert np.allclose(S3, Me + Kk + np.diag(de), atol=1e-14 * np.abs(Kk).max())


def _interp_1d(n):
    """Linear interpolation from the coarse points ('even indices plus the
    last') to the n fine points, from the coarse coordinates."""
    xc = qref.coarse_coords(np.arange(n, dtype=float))
    P = np.zeros((n, len(xc)))
    for i in range(n):
        I = min(np.searchsorted(xc, i, side="right") - 1, len(xc) - 2)
        t = (i - xc[I]) / (xc[I + 1] - xc[I])
        P[i, I] += 1 - t
        P[i, I + 1] += t
    return P


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_two_grid_vcycle_is_the_composed_error_propagation(deg):
    """With the coarse level solved exactly, the V-cycle from x = 0 is
    V = (I - E) S^-1 with the error propagation
        E = q(D^-1 S) (I - P S_c^-1 P^T S) q(D^-1 S),   S_c = P^T S P,
    q the degree-k Chebyshev polynomial on [lmax/4, lmax] (lmax the
    Gershgorin bound of D^-1 S), P the tensor-product linear interpolation.
    Everything on the right is built densely here from the fine stencil
    alone, so a restriction that is not P^T (a scaled one), a coarse
    operator that is not the Galerkin product, or a post-smoother that
    differs from the pre-smoother fails, although each keeps V symmetric."""
    p = pi.make_custom(6, 5, 13, (6, 6), seed=3, sigma_log=1.0, corr_cells=3.0)
    orc = O.Oracle(p)
    orc.setup(coarse_max=100, cheb_degree=deg)
    for box in range(4):
        lv = orc.mg_levels(box)
        assert len(lv) == 2, lv
        dims = lv[0][0]
        n = dims[0] * dims[1] * dims[2]
        S = qref.stencil_to_dense(dims, orc.mg_stencil(box, 0))
        d = np.diag(S)
        lmax = np.max(np.abs(S).sum(axis=1) / d)
        lmin = lmax / 4
        theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
        C = S / np.sqrt(np.outer(d, d))
        lam, Q = np.linalg.eigh(C)
        Tk = np.zeros(deg + 1); Tk[-1] = 1.0
        q = npcheb.chebval((theta - lam) / delta, Tk) / npcheb.chebval(theta / delta, Tk)
        Qp = np.diag(1 / np.sqrt(d)) @ ((Q * q) @ Q.T) @ np.diag(np.sqrt(d))
        P = np.kron(_interp_1d(dims[2]), np.kron(_interp_1d(dims[1]), _interp_1d(dims[0])))
        Sc = P.T @ S @ P
        cgc = np.eye(n) - P @ np.linalg.solve(Sc, P.T @ S)
        E = Qp @ cgc @ Qp
        ref = (np.eye(n) - E) @ np.linalg.inv(S)
        got = np.stack([orc.vcycle(box, e) for e in np.eye(n)], axis=1)
        assert np.allclose(got, ref, atol=1e-11 * np.abs(ref).max()), (box, np.abs(got - ref).max())
