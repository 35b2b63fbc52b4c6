"""Pins of the oracle on anisotropic meshes (box elements with edges hx, hy
along the cell and hz through it, as in the flattened jelly roll of Case III,
Sec. 5) and of its z-line multigrid (block Gauss-Seidel over the z-lines,
coarsening in x and y only): quadrature assembly of every block with the
element edges, the Galerkin product of the semicoarsened hierarchy as a
dense triple product, one colour sweep against dense block Gauss-Seidel,
symmetry of the V-cycle, the solution against a dense solve."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests import qref
from tests.test_oracle_operator import block, elem_mat_array, phis_nodes


def aniso(nx=6, ny=5, nz=13, nr=(5, 6), hxy=(3.7, 0.6), seed=21, bv=True, length=1.0):
    p = pi.make_custom(nx, ny, nz, nr, seed=seed, sigma_log=0.7, corr_cells=2.0)
    h = length / (nz - 1)
    p = p.with_(hxy=(hxy[0] * h, hxy[1] * h), length=length)
    if not bv:
        z = np.zeros(p.n_e)
        p = p.with_(g=z, s=z, e=z)
    return p


def coords(p):
    hx, hy = p.hxy
    return np.arange(p.nx) * hx, np.arange(p.ny) * hy, np.arange(p.nz) * p.h


def test_anisotropic_blocks_match_quadrature_assembly():
    """Every diffusion and storage block equals the Q1 assembly on box
    elements of edges (hx, hy, hz); the lumped reaction weights are an
    eighth of the element volume per electrode element."""
    p = aniso(bv=False)
    orc = O.Oracle(p)
    xs, ys, zs = coords(p)
    emat = elem_mat_array(p)
    is_elec = emat >= 0
    eps = np.where(is_elec, p.eps_elec, p.eps_sep)
    nodes = (p.nx, p.ny, p.nz)
    Kk = qref.assemble_box(*nodes, p.kappa, None, xs, ys, zs).toarray()
    Ks = qref.assemble_box(*nodes, np.where(is_elec, p.sigma, 0.0), None, xs, ys, zs)
    Me = qref.assemble_box(*nodes, np.zeros(p.n_elem), eps / p.dt, xs, ys, zs).toarray()
    ps = phis_nodes(p)
    Ks_ps = Ks[ps][:, ps].toarray()
    dirichlet = np.zeros(len(ps), bool)
    dirichlet[: p.nx * p.ny] = True
    Ks_ps[dirichlet, :] = 0.0
    Ks_ps[:, dirichlet] = 0.0
    Ks_ps[dirichlet, dirichlet] = 1.0
    tol = 1e-13 * np.abs(Kk).max()
    assert np.allclose(block(orc, p, 0, 0), Ks_ps, atol=tol)
    assert np.allclose(block(orc, p, 1, 1), Kk, atol=tol)
    assert np.allclose(block(orc, p, 1, 2), p.chi * Kk, atol=tol)
    assert np.allclose(block(orc, p, 2, 2), Me + Kk, atol=tol)
    # row-sum lumped electrode mass
    vol = p.hxy[0] * p.hxy[1] * p.h
    m = orc.lumped_weights()
    Mel = qref.assemble_box(*nodes, np.zeros(p.n_elem), is_elec.astype(float), xs, ys, zs)
    lump = np.asarray(Mel.sum(axis=1)).ravel()[ps]
    assert np.allclose(m, lump, rtol=1e-13, atol=0)
    assert m.sum() == pytest.approx(vol * is_elec.sum(), rel=1e-13)


def test_isotropic_edges_reproduce_the_default_operator():
    """hxy equal to h is the isotropic operator, bit for bit."""
    p = aniso()
    q = p.with_(hxy=(p.h, p.h))
    x = np.random.default_rng(1).standard_normal(p.N)
    base = p.with_(hxy=(0.0, 0.0))
    assert np.array_equal(O.Oracle(q).apply(x), O.Oracle(base).apply(x))


@pytest.mark.parametrize("dims", [(7, 6, 5), (9, 4, 8)])
def test_semicoarsened_galerkin_is_the_triple_product(dims):
    """With z left uncoarsened, S_c = P^T S P for P = P_x (x) P_y (x) I on an
    anisotropic mass + stiffness operator."""
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    ne = (nx - 1) * (ny - 1) * (nz - 1)
    xs, ys, zs = np.arange(nx) * 5.0, np.arange(ny) * 3.0, np.arange(nz) * 0.1
    A = qref.assemble_box(nx, ny, nz, rng.uniform(0.5, 2, ne), rng.uniform(0.5, 2, ne), xs, ys, zs)
    S = qref.dense_to_stencil(dims, A)
    Sc, cdims = O.rap(dims, S, coarsen_z=False)
    assert cdims[2] == nz

    def P1(n):
        xc = qref.coarse_coords(np.arange(n, dtype=float))
        P = np.zeros((n, len(xc)))
        for i in range(n):
            I = min(np.searchsorted(xc, i, side="right") - 1, len(xc) - 2)
            t = (i - xc[I]) / (xc[I + 1] - xc[I])
            P[i, I] += 1 - t
            P[i, I + 1] += t
        return P
    P = np.kron(np.eye(nz), np.kron(P1(ny), P1(nx)))
    ref = P.T @ A.toarray() @ P
    assert np.allclose(qref.stencil_to_dense(cdims, Sc), ref, atol=1e-13 * np.abs(ref).max())


def _line_ids(dims, i, j):
    nx, ny, nz = dims
    return [i + nx * (j + ny * k) for k in range(nz)]


@pytest.mark.parametrize("backward", [False, True])
def test_zline_sweep_is_dense_block_gauss_seidel(backward):
    """One pass over the four colours equals block Gauss-Seidel written with
    dense blocks: for each line l of a colour, x_l = A_ll^-1 (b_l - sum_m
    A_lm x_m), colours (even x, even y), (odd, even), (even, odd), (odd,
    odd), reversed for the backward pass."""
    dims = (5, 4, 6)
    nx, ny, nz = dims
    rng = np.random.default_rng(3)
    ne = (nx - 1) * (ny - 1) * (nz - 1)
    xs, ys, zs = np.arange(nx) * 4.0, np.arange(ny) * 2.5, np.arange(nz) * 0.2
    A = qref.assemble_box(nx, ny, nz, rng.uniform(0.5, 2, ne), rng.uniform(0.5, 2, ne), xs, ys,
                          zs).toarray()
    S = qref.dense_to_stencil(dims, A)
    b = rng.standard_normal(nx * ny * nz)
    x0 = rng.standard_normal(nx * ny * nz)
    got = O.zline_sweep(dims, S, b, x0, backward=backward)
    x = x0.copy()
    colours = [(0, 0), (1, 0), (0, 1), (1, 1)]
    if backward:
        colours = colours[::-1]
    for cx, cy in colours:
        for j in range(cy, ny, 2):
            for i in range(cx, nx, 2):
                ids = _line_ids(dims, i, j)
                rest = b[ids] - A[ids] @ x + A[np.ix_(ids, ids)] @ x[ids]
                x[ids] = np.linalg.solve(A[np.ix_(ids, ids)], rest)
    assert np.allclose(got, x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_zline_vcycle_is_symmetric_and_semicoarsened():
    """The z-line V-cycle (pre-sweeps forward, post-sweeps backward) is
    self-adjoint; every level keeps the box's z extent."""
    p = aniso(nx=17, ny=9, nz=13, hxy=(30.0, 25.0))
    orc = O.Oracle(p).setup(smoother=O.SMOOTH_ZLINE, coarse_max=64)
    rng = np.random.default_rng(4)
    for box in range(4):
        levels = orc.mg_levels(box)
        assert len(levels) > 1
        assert len({d[2] for d, _ in levels}) == 1
        n = levels[0][0][0] * levels[0][0][1] * levels[0][0][2]
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        vx, vy = orc.vcycle(box, x), orc.vcycle(box, y)
        assert abs(vx @ y - x @ vy) <= 1e-12 * np.sqrt((vx @ vx) * (y @ y))


@pytest.mark.parametrize("smoother", [O.SMOOTH_CHEB, O.SMOOTH_ZLINE])
def test_anisotropic_solution_matches_dense_solve(smoother):
    p = aniso(nx=6, ny=5, nz=13, hxy=(8.0, 6.0))
    orc = O.Oracle(p).setup(smoother=smoother, rtol=1e-12, coarse_max=64, maxit=2000)
    x, info = orc.solve(p.b)
    assert info.status == 0
    A = np.column_stack([orc.apply(e) for e in np.eye(p.N)])
    ref = np.linalg.solve(A, p.b)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_zline_smoothing_is_robust_to_the_aspect_ratio():
    """Strongly flattened elements (edges along the cell 40x the one through
    it): the point-smoothed hierarchy needs many more iterations, the z-line
    one stays at a handful (iteration counts reported, the bound loose)."""
    p = aniso(nx=33, ny=17, nz=13, nr=(5, 5), hxy=(40.0, 40.0))
    its = {}
    for sm in (O.SMOOTH_CHEB, O.SMOOTH_ZLINE):
        orc = O.Oracle(p).setup(smoother=sm, rtol=1e-8, coarse_max=64, maxit=3000)
        _, info = orc.solve(p.b)
        assert info.status == 0
        its[sm] = info.iters
    print("iterations point / z-line:", its)
    assert its[O.SMOOTH_ZLINE] <= 20
    assert its[O.SMOOTH_ZLINE] * 2 <= its[O.SMOOTH_CHEB]
