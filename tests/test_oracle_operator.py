"""Pins of the oracle's linearized operator (Sec. 3.2 weak forms, Sec. 4.1
block Jacobian) against independent quadrature assembly and conservation
laws of the model equations (Sec. 2)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import p4d_inputs as pi
from tests import qref


def elem_layers(p):
    """material per element layer: 0 anode, 1 cathode, -1 separator"""
    out = []
    for k in range(p.nz - 1):
        if k + 1 < p.na:
            out.append(0)
        elif k >= p.na + p.ns:
            out.append(1)
        else:
            out.append(-1)
    return np.array(out)


def elem_mat_array(p):
    lay = elem_layers(p)
    return np.repeat(lay, (p.nx - 1) * (p.ny - 1))


def node_layers(p):
    k = np.repeat(np.arange(p.nz), p.nx * p.ny)
    return k


def phis_nodes(p):
    """global node ids of the phi_s entries (anode then cathode)"""
    k = node_layers(p)
    ids = np.arange(p.n_nodes)
    return np.concatenate([ids[k < p.na], ids[k >= p.na + p.ns]])


def problem(nx=5, ny=4, nz=13, nr=(6, 5), sigma_log=0.7, seed=11, bv=True):
    p = pi.make_custom(nx, ny, nz, nr, seed=seed, sigma_log=sigma_log, corr_cells=2.0)
    if not bv:
        z = np.zeros(p.n_e)
        p = p.with_(g=z, s=z, e=z)
    return p


def field_slices(p):
    o = p.offsets
    return (slice(o[0], o[1]), slice(o[1], o[2]), slice(o[2], o[3]), slice(o[3], o[5]))


def block(orc, p, row, col, transpose=False):
    """Dense block A[row, col] by probing with unit vectors."""
    sl = field_slices(p)
    rs, cs = sl[row], sl[col]
    ncol = cs.stop - cs.start
    B = np.zeros((rs.stop - rs.start, ncol))
    x = np.zeros(p.N)
    for c in range(ncol):
        x[cs.start + c] = 1.0
        B[:, c] = orc.apply(x, transpose)[rs]
        x[cs.start + c] = 0.0
    return B


def test_q1_reference_stencils():
    """Interior assembled stencils of the unit-cube Q1 element matrices."""
    K, M = qref.element_matrices()
    A = qref.assemble_box(3, 3, 3, np.ones(8))
    Mm = qref.assemble_box(3, 3, 3, np.zeros(8), np.ones(8))
    c = 13
    row = A.toarray()[c]
    mrow = Mm.toarray()[c]
    for o in range(27):
        d = abs(o % 3 - 1) + abs((o // 3) % 3 - 1) + abs(o // 9 - 1)
        kexp = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[d]
        mexp = {0: 64, 1: 16, 2: 4, 3: 1}[d] / 216
        assert row[o] == pytest.approx(kexp, abs=1e-14)
        assert mrow[o] == pytest.approx(mexp, abs=1e-14)


@pytest.mark.parametrize("seed", [11, 12])
def test_blocks_match_quadrature_assembly(seed):
    """With zero Butler-Volmer derivatives the operator is A_diff; every block
    equals the Q1 assembly of the weak forms (phis-weak, phie-weak, ce-weak)
    and the backward-Euler radial rows (FD)."""
    p = problem(seed=seed, bv=False)
    orc = O.Oracle(p)
    h = p.h
    emat = elem_mat_array(p)
    is_elec = emat >= 0
    eps = np.where(is_elec, p.eps_elec, p.eps_sep)
    nodes = (p.nx, p.ny, p.nz)
    coords = [np.arange(n) * h for n in nodes]
    Kk = qref.assemble_box(*nodes, p.kappa, None, *coords)
    Ks = qref.assemble_box(*nodes, np.where(is_elec, p.sigma, 0.0), None, *coords)
    Me = qref.assemble_box(*nodes, np.zeros(p.n_elem), eps / p.dt, *coords)
    ps = phis_nodes(p)
    Ks_ps = Ks[ps][:, ps].toarray()
    dirichlet = np.zeros(len(ps), bool)
    dirichlet[: p.nx * p.ny] = True
    Ks_ps[dirichlet, :] = 0.0
    Ks_ps[:, dirichlet] = 0.0
    Ks_ps[dirichlet, dirichlet] = 1.0
    tol = 1e-13
    assert np.allclose(block(orc, p, 0, 0), Ks_ps, atol=tol * h)
    assert np.allclose(block(orc, p, 1, 1), Kk.toarray(), atol=tol * h)
    assert np.allclose(block(orc, p, 1, 2), p.chi * Kk.toarray(), atol=tol * h)
    assert np.allclose(block(orc, p, 2, 2), (Me + Kk).toarray(), atol=tol * h)
    assert np.abs(block(orc, p, 2, 1)).max() == 0.0
    assert np.abs(block(orc, p, 0, 1)).max() == 0.0
    # radial rows: T0 = I/dt - L_h per electrode node, SoA layout [r][node]
    Bss = block(orc, p, 3, 3)
    off = 0
    for el, nn in ((0, p.n_ea), (1, p.n_ec)):
        N = p.nr[el]
        rho = O.radial_mesh(N, p.theta_bar[el])
        sub, dia, sup, _ = O.radial_rows(N, p.Ds[el], rho)
        T0 = np.eye(N) / p.dt - (np.diag(dia) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1))
        for jn in (0, nn // 2, nn - 1):
            idx = off + np.arange(N) * nn + jn
            assert np.allclose(Bss[np.ix_(idx, idx)], T0, atol=1e-15)
        off += N * nn
    # transposed operator
    assert np.allclose(block(orc, p, 2, 1, True), p.chi * Kk.toarray(), atol=tol * h)


def test_general_transport_coefficients_and_length():
    """Separate element coefficients for the diffusion-potential block and
    the c_e diffusion, a physical cell length and per-electrode coupling
    scales: every block equals the Q1 assembly with those coefficients on the
    scaled grid, and the surface coupling scales per electrode."""
    p = problem(seed=13, bv=False)
    rng = np.random.default_rng(5)
    kd = np.exp(0.5 * rng.standard_normal(p.n_elem))
    dc = np.exp(0.5 * rng.standard_normal(p.n_elem))
    L = 2.25e-4
    q = p.with_(kappa_d=kd, dce=dc, length=L, lambda_el=(0.7, 1.9))
    orc = O.Oracle(q)
    h = q.h
    assert h == pytest.approx(L / (p.nz - 1))
    emat = elem_mat_array(p)
    eps = np.where(emat >= 0, p.eps_elec, p.eps_sep)
    nodes = (p.nx, p.ny, p.nz)
    coords = [np.arange(n) * h for n in nodes]
    Kk = qref.assemble_box(*nodes, p.kappa, None, *coords).toarray()
    Kd = qref.assemble_box(*nodes, kd, None, *coords).toarray()
    Kc = qref.assemble_box(*nodes, dc, None, *coords).toarray()
    Me = qref.assemble_box(*nodes, np.zeros(p.n_elem), eps / p.dt, *coords).toarray()
    tol = 1e-13 * h
    assert np.allclose(block(orc, q, 1, 1), Kk, atol=tol)
    assert np.allclose(block(orc, q, 1, 2), Kd, atol=tol)
    assert np.allclose(block(orc, q, 2, 2), Me + Kc, atol=max(tol, 1e-13 * np.abs(Me).max()))
    assert np.allclose(block(orc, q, 2, 1, True), Kd, atol=tol)
    assert np.abs(block(orc, q, 1, 2, True)).max() == 0.0
    # the default coefficients reproduce the plain operator
    q0 = p.with_(kappa_d=p.chi * p.kappa, dce=p.kappa)
    x = rng.standard_normal(p.N)
    ref = O.Oracle(p).apply(x)
    assert np.allclose(O.Oracle(q0).apply(x), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # surface coupling: lambda per electrode replaces lambda_c
    g0 = [O.Oracle(p).radial(el)[4] for el in (0, 1)]
    g1 = [orc.radial(el)[4] for el in (0, 1)]
    assert g1[0] == pytest.approx(0.7 * g0[0] / p.lambda_c)
    assert g1[1] == pytest.approx(1.9 * g0[1] / p.lambda_c)


def test_porosity_per_element():
    """A porosity field per element (Case II volume fractions, Sec. 5) enters
    only the c_e storage: that block equals the Q1 mass assembly of the field
    over dt (plus the unchanged stiffness), the mass of a uniform c_e is the
    integral of the porosity, and the per-material values reproduce the
    default operator exactly."""
    p = problem(seed=14, bv=False)
    rng = np.random.default_rng(6)
    ep = 0.1 + 0.8 * rng.random(p.n_elem)
    q = p.with_(eps_e=ep, length=3.0)
    orc = O.Oracle(q)
    h = q.h
    nodes = (p.nx, p.ny, p.nz)
    coords = [np.arange(n) * h for n in nodes]
    Kk = qref.assemble_box(*nodes, p.kappa, None, *coords).toarray()
    Me = qref.assemble_box(*nodes, np.zeros(p.n_elem), ep / p.dt, *coords).toarray()
    B = block(orc, q, 2, 2)
    assert np.allclose(B, Me + Kk, rtol=0, atol=1e-13 * np.abs(B).max())
    # the other blocks do not see it
    ref = O.Oracle(p.with_(length=3.0))
    for r, c in ((1, 1), (1, 2), (0, 0)):
        assert np.array_equal(block(orc, q, r, c), block(ref, q, r, c))
    # storage of c_e = 1 (no transport): sum of rows = h^3 sum(eps_e) / dt
    z = np.zeros(p.n_elem)
    q0 = q.with_(kappa=z, sigma=z)
    x = np.zeros(p.N)
    x[p.offsets[2]: p.offsets[3]] = 1.0
    y = O.Oracle(q0).apply(x)[p.offsets[2]: p.offsets[3]]
    assert y.sum() == pytest.approx(h ** 3 * ep.sum() / p.dt, rel=1e-13)
    # per-material values as a field: the default operator, bit for bit
    emat = elem_mat_array(p)
    pm = p.with_(eps_e=np.where(emat >= 0, p.eps_elec, p.eps_sep))
    x = rng.standard_normal(p.N)
    assert np.array_equal(O.Oracle(pm).apply(x), O.Oracle(p).apply(x))
    assert np.array_equal(O.Oracle(pm).apply(x, True), O.Oracle(p).apply(x, True))


def test_lumped_weights_are_row_sum_lumped_electrode_mass():
    p = problem()
    orc = O.Oracle(p)
    h = p.h
    emat = elem_mat_array(p)
    nodes = (p.nx, p.ny, p.nz)
    coords = [np.arange(n) * h for n in nodes]
    Mel = qref.assemble_box(*nodes, np.zeros(p.n_elem), (emat >= 0).astype(float), *coords)
    lump = np.asarray(Mel.sum(axis=1)).ravel()
    assert np.allclose(orc.lumped_weights(), lump[phis_nodes(p)], rtol=1e-13)


def test_charge_conservation():
    """Charge leaving the solid enters the electrolyte (the same a*i_n with
    opposite signs in eq. phis and the phi_e equation): for any x vanishing
    near the grounded face, sum(y_phis) + sum(y_phie) = 0."""
    p = problem()
    orc = O.Oracle(p)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(p.N)
    k = node_layers(p)
    sl = field_slices(p)
    x[sl[1]][k <= 1] = 0.0
    x[sl[2]][k <= 1] = 0.0
    ps_k = k[phis_nodes(p)]
    x[sl[0]][ps_k <= 1] = 0.0
    csa = x[p.offsets[3]:p.offsets[4]].reshape(p.nr[0], p.n_ea)
    csa[:, ps_k[: p.n_ea] <= 1] = 0.0
    y = orc.apply(x)
    tot = y[sl[0]].sum() + y[sl[1]].sum()
    scale = np.abs(y[sl[0]]).sum() + np.abs(y[sl[1]]).sum()
    assert abs(tot) <= 1e-13 * scale
    # and the reaction does not vanish in this test
    yz = O.Oracle(problem(bv=False)).apply(x)
    assert np.abs(y[sl[1]] - yz[sl[1]]).max() > 1e-6 * np.abs(y[sl[1]]).max()


def test_lithium_balance():
    """Lithium leaving the particles (measured with the conservation weights
    w of the radial scheme) enters the electrolyte equation with the factor
    (1 - t+): sum(y_ce) - 1^T M_eps x_ce / dt = -(1-t+) sum_j m_j Q_j, where
    Q_j = (w.y_s,j - w.x_s,j/dt) / (Gamma w_N) is the node's surface
    exchange read off the particle rows."""
    p = problem()
    orc = O.Oracle(p)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(p.N)
    y = orc.apply(x)
    sl = field_slices(p)
    h = p.h
    emat = elem_mat_array(p)
    eps = np.where(emat >= 0, p.eps_elec, p.eps_sep)
    nodes = (p.nx, p.ny, p.nz)
    coords = [np.arange(n) * h for n in nodes]
    Me = qref.assemble_box(*nodes, np.zeros(p.n_elem), eps / p.dt, *coords)
    lhs = y[sl[2]].sum() - (Me @ x[sl[2]]).sum()
    m = orc.lumped_weights()
    Q = []
    for el, nn, off in ((0, p.n_ea, p.offsets[3]), (1, p.n_ec, p.offsets[4])):
        N = p.nr[el]
        rho, sub, dia, sup, gam = orc.radial(el)
        L = np.diag(dia) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
        w = np.linalg.svd(L.T)[2][-1]
        ys = y[off:off + N * nn].reshape(N, nn)
        xs = x[off:off + N * nn].reshape(N, nn)
        Q.append((w @ ys - w @ xs / p.dt) / (gam * w[-1]))
    Q = np.concatenate(Q)
    rhs = -p.tc * (m * Q).sum()
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_reaction_depends_on_overpotential_difference():
    """eta = phi_s - phi_e: raising phi_s and phi_e together changes no
    reaction term, so away from the grounded face and domain borders A maps
    (phi_s, phi_e) = (1, 1) to zero in the phi_s, phi_e and c_s rows."""
    p = problem(nx=6, ny=6)
    orc = O.Oracle(p)
    x = np.zeros(p.N)
    sl = field_slices(p)
    x[sl[0]] = 1.0
    x[sl[1]] = 1.0
    y = orc.apply(x)
    k = node_layers(p)
    ps_k = k[phis_nodes(p)]
    # phi_e rows of nodes above the first two layers: K 1 = 0 and q = 0
    assert np.abs(y[sl[1]][k >= 2]).max() <= 1e-14
    cathode = np.arange(p.n_ea, p.n_e)
    assert np.abs(y[sl[0]][cathode]).max() <= 1e-14
    ys = y[p.offsets[4]:p.offsets[5]]
    assert np.abs(ys).max() <= 1e-13


def test_diffusion_consistency_order():
    """(K u)_j / h^3 -> -Lap u at interior nodes, O(h^2) (Q1 on a uniform
    grid), through the phi_e block of the oracle operator."""
    errs = []
    for nz in (13, 25, 49):
        nx = (nz - 1) // 2 + 1
        p = pi.make_custom(nx, nx, nz, (4, 4), seed=1)
        p = p.with_(g=np.zeros(p.n_e), s=np.zeros(p.n_e), e=np.zeros(p.n_e))
        orc = O.Oracle(p)
        h = p.h
        i = np.tile(np.arange(nx), nx * nz)
        j = np.tile(np.repeat(np.arange(nx), nx), nz)
        k = np.repeat(np.arange(nz), nx * nx)
        X, Y, Z = i * h, j * h, k * h
        u = np.cos(2 * X) * np.sin(1.5 * Y + 0.3) * np.cos(Z + 0.2)
        lap = -(4 + 2.25 + 1) * u
        x = np.zeros(p.N)
        sl = field_slices(p)
        x[sl[1]] = u
        y = orc.apply(x)[sl[1]] / h ** 3
        inner = (i > 0) & (i < nx - 1) & (j > 0) & (j < nx - 1) & (k > 0) & (k < nz - 1)
        errs.append(np.max(np.abs(y[inner] + lap[inner])))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


def test_symmetry_and_transpose():
    """Diffusion blocks (with the reaction diagonal) are symmetric, T0 is
    symmetric in the conservation-weighted inner product, and the transposed
    apply satisfies <A x, y> = <x, A^T y>."""
    p = problem()
    orc = O.Oracle(p)
    for f in (0, 1):
        B = block(orc, p, f, f)
        assert np.allclose(B, B.T, atol=1e-14 * np.abs(B).max())
    B = block(orc, p, 2, 2)
    assert np.allclose(B, B.T, atol=1e-14 * np.abs(B).max())
    for el in range(2):
        rho, sub, dia, sup, gam = orc.radial(el)
        L = np.diag(dia) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
        w = np.abs(np.linalg.svd(L.T)[2][-1])
        T0 = np.eye(len(rho)) / p.dt - L
        WT = np.diag(w) @ T0
        assert np.allclose(WT, WT.T, atol=1e-14 * np.abs(WT).max())
    rng = np.random.default_rng(3)
    for _ in range(3):
        x, y = rng.standard_normal(p.N), rng.standard_normal(p.N)
        a = orc.apply(x) @ y
        b = x @ orc.apply(y, True)
        assert a == pytest.approx(b, rel=1e-12)
