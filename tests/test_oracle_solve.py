"""Pins of the oracle's preconditioner (Sec. 4.2: eq. PJ, eq. PGS in every
field ordering, and the exact elimination of the particle blocks), the Schur
complement of the particle blocks and the Krylov iteration over it, FGMRES
solve and parameter gradients."""
import itertools

import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi


def tiny(seed=0, sigma_log=0.5, nx=4, ny=4, nz=6, nr=(4, 5)):
    return pi.make_custom(nx, ny, nz, nr, seed=seed, sigma_log=sigma_log,
                          na=2, ns=2, corr_cells=2.0)


def schur_blocks(p, A):
    """Dense blocks of A split into macro (y) and particle (s) unknowns."""
    nm = p.offsets[3]
    return A[:nm, :nm], A[:nm, nm:], A[nm:, :nm], A[nm:, nm:]


def field_ranges(p):
    o = p.offsets
    return [(o[0], o[1]), (o[1], o[2]), (o[2], o[3])]


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("seed", [0, 1])
def test_schur_preconditioner_is_exact_block_ldu(seed, transpose):
    """With direct block solves (single-level grids), P^-1 of mode SCHUR is
    the inverse of [[St + Ays Ass^-1 Asy, Ays], [Asy, Ass]] with St the
    field-block diagonal of the exact Schur complement
    S = Ayy - Ays Ass^-1 Asy, all blocks taken from the assembled A."""
    p = tiny(seed)
    orc = O.Oracle(p).setup(pc=O.PC_SCHUR, coarse_max=512)
    A = orc.dense()
    Ayy, Ays, Asy, Ass = schur_blocks(p, A)
    S = Ayy - Ays @ np.linalg.solve(Ass, Asy)
    St = np.zeros_like(S)
    for a, b in field_ranges(p):
        St[a:b, a:b] = S[a:b, a:b]
    P = np.block([[St + Ays @ np.linalg.solve(Ass, Asy), Ays], [Asy, Ass]])
    if transpose:
        P = P.T
    r = np.random.default_rng(seed + 10).standard_normal(p.N)
    z = orc.apply_pc(r, transpose)
    ref = np.linalg.solve(P, r)
    assert np.allclose(z, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("transpose", [False, True])
def test_block_jacobi_is_eq_PJ(transpose):
    """Mode BJ with direct block solves applies diag(A_phis, A_phie, A_ce,
    A_cs)^-1 (eq. PJ)."""
    p = tiny(3)
    orc = O.Oracle(p).setup(pc=O.PC_BJ, coarse_max=512)
    A = orc.dense()
    PJ = np.zeros_like(A)
    o = p.offsets
    for a, b in [(o[0], o[1]), (o[1], o[2]), (o[2], o[3]), (o[3], o[5])]:
        PJ[a:b, a:b] = A[a:b, a:b]
    if transpose:
        PJ = PJ.T
    r = np.random.default_rng(1).standard_normal(p.N)
    ref = np.linalg.solve(PJ, r)
    assert np.allclose(orc.apply_pc(r, transpose), ref, atol=1e-10 * np.abs(ref).max())


def field_blocks(p):
    """Index ranges of phi_s, phi_e, c_e and c_s (both electrodes)."""
    o = p.offsets
    return [(o[0], o[1]), (o[1], o[2]), (o[2], o[3]), (o[3], o[5])]


def pgs_dense(A, blocks, fields):
    """eq. PGS written in the field ordering `fields` (first block first):
    the blocks A_{f,g} with g at or before f in the ordering, zero after."""
    P = np.zeros_like(A)
    pos = {f: i for i, f in enumerate(fields)}
    for f in range(4):
        for g in range(4):
            if pos[g] <= pos[f]:
                (a, b), (c, d) = blocks[f], blocks[g]
                P[a:b, c:d] = A[a:b, c:d]
    return P


ALL_ORDERINGS = list(itertools.permutations(range(4)))


@pytest.mark.parametrize("transpose", [False, True])
def test_block_gauss_seidel_is_eq_PGS_in_every_ordering(transpose):
    """Mode BGS with direct block solves applies P_GS^-1 (P_GS^-T) of eq. PGS
    for each of the 24 orderings; P_GS is built from the assembled A."""
    p = tiny(4, sigma_log=1.0)
    orc = O.Oracle(p)
    A = orc.dense()
    blocks = field_blocks(p)
    r = np.random.default_rng(5).standard_normal(p.N)
    for fields in ALL_ORDERINGS:
        orc.setup(pc=O.PC_BGS, coarse_max=512, bgs_order=O.bgs_order(fields))
        P = pgs_dense(A, blocks, fields)
        ref = np.linalg.solve(P.T if transpose else P, r)
        z = orc.apply_pc(r, transpose)
        assert np.allclose(z, ref, rtol=0, atol=1e-10 * np.abs(ref).max()), fields


def test_block_gauss_seidel_orderings_differ():
    """The off-diagonal blocks are not zero: orderings give different P_GS^-1,
    and reversing the ordering is not the transpose (a mistake that swapped
    the sweep direction would pass a symmetric test)."""
    p = tiny(6)
    orc = O.Oracle(p)
    r = np.random.default_rng(7).standard_normal(p.N)
    zs = []
    for fields in [(1, 3, 0, 2), (2, 1, 3, 0), (0, 1, 2, 3), (3, 2, 1, 0)]:
        orc.setup(pc=O.PC_BGS, coarse_max=512, bgs_order=O.bgs_order(fields))
        zs.append(orc.apply_pc(r))
    for i in range(len(zs)):
        for j in range(i):
            assert np.linalg.norm(zs[i] - zs[j]) > 1e-6 * np.linalg.norm(zs[i])
    orc.setup(pc=O.PC_BGS, coarse_max=512, bgs_order=O.bgs_order((0, 1, 2, 3)))
    zt = orc.apply_pc(r, True)
    assert np.linalg.norm(zt - zs[3]) > 1e-6 * np.linalg.norm(zt)


def tiny_general(seed):
    """tiny() with separate diffusion-potential and c_e diffusion
    coefficients, a physical length and per-electrode coupling scales."""
    p = tiny(seed, sigma_log=1.0)
    rng = np.random.default_rng(seed + 100)
    return p.with_(kappa_d=np.exp(0.5 * rng.standard_normal(p.n_elem)),
                   dce=np.exp(0.5 * rng.standard_normal(p.n_elem)), length=3.0,
                   lambda_el=(0.6, 1.7))


@pytest.mark.parametrize("transpose", [False, True])
def test_preconditioners_exact_with_general_transport(transpose):
    """The field blocks given to the direct coarse solves follow the general
    coefficients: SCHUR is the exact block LDU, BGS is eq. PGS."""
    p = tiny_general(8)
    orc = O.Oracle(p).setup(pc=O.PC_SCHUR, coarse_max=512)
    A = orc.dense()
    Ayy, Ays, Asy, Ass = schur_blocks(p, A)
    S = Ayy - Ays @ np.linalg.solve(Ass, Asy)
    St = np.zeros_like(S)
    for a, b in field_ranges(p):
        St[a:b, a:b] = S[a:b, a:b]
    P = np.block([[St + Ays @ np.linalg.solve(Ass, Asy), Ays], [Asy, Ass]])
    r = np.random.default_rng(3).standard_normal(p.N)
    ref = np.linalg.solve(P.T if transpose else P, r)
    assert np.allclose(orc.apply_pc(r, transpose), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    for fields in [(1, 3, 0, 2), (2, 0, 3, 1)]:
        orc.setup(pc=O.PC_BGS, coarse_max=512, bgs_order=O.bgs_order(fields))
        Pg = pgs_dense(A, field_blocks(p), fields)
        ref = np.linalg.solve(Pg.T if transpose else Pg, r)
        assert np.allclose(orc.apply_pc(r, transpose), ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_bgs_order_packing():
    assert O.BGS_PAPER == O.bgs_order((O.F_PHIE, O.F_CS, O.F_PHIS, O.F_CE))
    for fields in ALL_ORDERINGS:
        assert O.bgs_order_fields(O.bgs_order(fields)) == fields
    with pytest.raises(ValueError):
        O.bgs_order((0, 1, 1, 3))
    with pytest.raises(ValueError):
        O.Oracle(tiny(0)).setup(pc=O.PC_BGS, bgs_order=0)


def omega_closed_form(p, orc):
    """S = A_diff,yy + sum_j omega_j a_j b_j^T with omega_j = 1/(1 + Gamma s_j
    tau0), tau0 = (T0^-1)_NN (Sherman-Morrison on A_ss,j = T0 + Gamma s_j
    e_N e_N^T): the reaction coupling of A_yy scaled by omega_j, built here
    from the radial rows and the node coefficients alone."""
    tau0, gam = [], []
    for el in range(2):
        rho, sub, dia, sup, G = orc.radial(el)
        N = p.nr[el]
        T0 = np.diag(1.0 / p.dt - dia) - np.diag(sub[1:], -1) - np.diag(sup[:-1], 1)
        tau0.append(np.linalg.solve(T0, np.eye(N)[:, -1])[-1])
        gam.append(G)
    return tau0, gam


@pytest.mark.parametrize("transpose", [False, True])
def test_schur_complement_is_dense_schur_and_omega_form(transpose):
    """S from the oracle equals A_yy - A_ys A_ss^-1 A_sy of the assembled A,
    and the closed form A_yy + sum_j (omega_j - 1) a_j b_j^T."""
    p = tiny(9, sigma_log=1.0)
    orc = O.Oracle(p)
    A = orc.dense(transpose)
    nm = p.offsets[3]
    Ayy, Ays, Asy, Ass = A[:nm, :nm], A[:nm, nm:], A[nm:, :nm], A[nm:, nm:]
    S_dense = Ayy - Ays @ np.linalg.solve(Ass, Asy)
    S = np.column_stack([orc.schur_apply(e, transpose) for e in np.eye(nm)])
    assert np.allclose(S, S_dense, rtol=0, atol=1e-12 * np.abs(S_dense).max())
    # closed form: per electrode node the rank-1 reaction block of A_yy,
    # scaled by omega_j instead of 1
    tau0, gam = omega_closed_form(p, orc)
    m = orc.lumped_weights()
    S_cf = Ayy.copy()
    o = p.offsets
    layer = p.nx * p.ny
    for je in range(p.n_ea + p.n_ec):
        el = 0 if je < p.n_ea else 1
        k = je // layer if el == 0 else p.na + p.ns + (je - p.n_ea) // layer
        n = k * layer + je % layer
        dirn = k == 0
        a = np.array([0.0 if dirn else m[je], -m[je], -p.tc * m[je]])
        bb = np.array([0.0 if dirn else p.g[je], -p.g[je], p.e[je]])
        if transpose:
            a, bb = bb, a
        om = 1.0 / (1.0 + gam[el] * p.s[je] * tau0[el])
        rows = [o[0] + je, o[1] + n, o[2] + n]
        S_cf[np.ix_(rows, rows)] += (om - 1.0) * np.outer(a, bb)
    assert np.allclose(S, S_cf, rtol=0, atol=1e-12 * np.abs(S_cf).max())


@pytest.mark.parametrize("transpose", [False, True])
def test_schur_rhs_and_back_substitution(transpose):
    """With y the exact solution of S y = b^, [y | back(y)] solves A x = b."""
    p = tiny(10)
    orc = O.Oracle(p)
    A = orc.dense(transpose)
    nm = p.offsets[3]
    bhat = orc.schur_rhs(p.b, transpose)
    S = np.column_stack([orc.schur_apply(e, transpose) for e in np.eye(nm)])
    y = np.linalg.solve(S, bhat)
    x = orc.schur_back(p.b, y, transpose)
    ref = np.linalg.solve(A, p.b)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("transpose", [False, True])
def test_schur_krylov_matches_dense_lu_and_full_space(transpose):
    """FGMRES over the Schur complement (multilevel V-cycles on its field
    blocks) reaches the dense-LU solution, with the full residual at the
    requested level and no more iterations than the full-space iteration
    with the same preconditioner blocks plus one."""
    p = tiny(7, nx=5, ny=4, nz=8, nr=(4, 6))
    A = O.Oracle(p).dense(transpose)
    ref = np.linalg.solve(A, p.b)
    full = O.Oracle(p).setup(rtol=1e-10, coarse_max=20)
    xf, inf_f = full.solve(p.b, transpose)
    red = O.Oracle(p).setup(rtol=1e-10, coarse_max=20, krylov=O.KRYLOV_SCHUR)
    x, info = red.solve(p.b, transpose)
    assert info.status == 0 and inf_f.status == 0
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(A @ x - p.b) / np.linalg.norm(p.b) == pytest.approx(info.relres_true, rel=1e-6)
    assert info.relres_true <= 1e-10
    assert info.iters <= inf_f.iters + 1


def test_schur_krylov_requires_schur_mode():
    with pytest.raises(ValueError):
        O.Oracle(tiny(0)).setup(pc=O.PC_BJ, krylov=O.KRYLOV_SCHUR)


def test_preconditioner_transpose_identity():
    """<P^-1 x, y> = <x, P^-T y> with multilevel V-cycles."""
    p = pi.make_custom(10, 9, 30, (6, 8), seed=5, sigma_log=1.0, corr_cells=3.0)
    orc = O.Oracle(p).setup()
    assert orc.mg_levels(2)[0][0] == (10, 9, 30) and len(orc.mg_levels(2)) >= 2
    rng = np.random.default_rng(2)
    for _ in range(2):
        x, y = rng.standard_normal(p.N), rng.standard_normal(p.N)
        assert orc.apply_pc(x) @ y == pytest.approx(x @ orc.apply_pc(y, True), rel=1e-11)


@pytest.mark.parametrize("pc", [O.PC_SCHUR, O.PC_BJ, O.PC_BGS])
@pytest.mark.parametrize("coarse_max", [512, 20])
@pytest.mark.parametrize("transpose", [False, True])
def test_L1_solution_matches_dense_lu(pc, coarse_max, transpose):
    p = tiny(7, nx=5, ny=4, nz=8, nr=(4, 6))
    orc = O.Oracle(p).setup(pc=pc, rtol=1e-10, coarse_max=coarse_max, maxit=3000,
                            cgs2=(pc == O.PC_BJ))
    A = orc.dense(transpose)
    x, info = orc.solve(p.b, transpose)
    ref = np.linalg.solve(A, p.b)
    assert info.status == 0
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_L2_manufactured_solution():
    """x* smooth in the macro fields and quadratic in rho; b = A x*.  (cond(A)
    is ~1e7 here, so residuals below ~1e-11 are not attainable.)"""
    p = pi.make_config(1)
    orc = O.Oracle(p).setup(rtol=1e-10)
    h = p.h
    k = np.repeat(np.arange(p.nz), p.nx * p.ny)
    j = np.tile(np.repeat(np.arange(p.ny), p.nx), p.nz)
    i = np.tile(np.arange(p.nx), p.ny * p.nz)
    X, Y, Z = i * h, j * h, k * h
    xs = np.zeros(p.N)
    o = p.offsets
    elec = (k < p.na) | (k >= p.na + p.ns)
    phis = np.cos(np.pi * X) * np.cos(np.pi * Y) * (1 + Z)
    xs[o[0]:o[1]] = phis[elec]
    xs[o[0]:o[0] + p.nx * p.ny] = 0.0            # grounded layer
    xs[o[1]:o[2]] = np.cos(2 * X) * np.sin(Y + 1) * np.cos(3 * Z)
    xs[o[2]:o[3]] = 1 + 0.2 * np.cos(np.pi * Z)
    for el, nn, off in ((0, p.n_ea, o[3]), (1, p.n_ec, o[4])):
        rho = O.radial_mesh(p.nr[el], p.theta_bar[el])
        base = 0.5 + 0.1 * np.arange(nn) / nn
        xs[off:off + p.nr[el] * nn] = (base[None, :] + 0.3 * rho[:, None] ** 2).reshape(-1)
    b = orc.apply(xs)
    x, info = orc.solve(b)
    assert info.status == 0
    # relative error <= cond(A) * rtol with cond ~1e7; the error sits in the
    # weakly controlled modes (the cathode phi_s / phi_e shift against the
    # grounded anode, a constant shift of c_e), measured 2e-5..1.4e-4 per field
    # depending on the Krylov path
    assert np.linalg.norm(x - xs) <= 1e-3 * np.linalg.norm(xs)
    o = p.offsets
    for a, b2 in zip(o[:-1], o[1:]):
        if b2 > a:
            assert np.linalg.norm(x[a:b2] - xs[a:b2]) <= 1e-3 * np.linalg.norm(xs[a:b2])
    # and the residual of the recovered x is at the requested level
    assert np.linalg.norm(orc.apply(x) - b) <= 1.0001e-10 * np.linalg.norm(b)


def test_zero_rhs_and_iteration_cap():
    p = tiny(2)
    orc = O.Oracle(p).setup()
    x, info = orc.solve(np.zeros(p.N))
    assert info.status == 0 and info.iters == 0 and not x.any()
    orc.setup(maxit=2)
    x, info = orc.solve(p.b)
    assert info.status == 1 and info.iters == 2


def test_schur_mode_beats_block_gauss_seidel_and_jacobi_on_C1():
    p = pi.make_config(1)
    o1 = O.Oracle(p).setup(pc=O.PC_SCHUR)
    x1, i1 = o1.solve(p.b)
    o2 = O.Oracle(p).setup(pc=O.PC_BJ)
    x2, i2 = o2.solve(p.b)
    o3 = O.Oracle(p).setup(pc=O.PC_BGS)
    x3, i3 = o3.solve(p.b)
    assert i1.status == 0 and i2.status == 0 and i3.status == 0
    # Sec. 5: block Gauss-Seidel needs fewer iterations than block Jacobi
    assert i1.iters < i3.iters < i2.iters
    assert np.linalg.norm(x1 - x2) <= 1e-6 * np.linalg.norm(x1)
    assert np.linalg.norm(x1 - x3) <= 1e-6 * np.linalg.norm(x1)


def test_J2_gradient_matches_finite_differences():
    """dJ/dsigma and dJ/dDs (-lambda^T dA/dp x, Sec. 4.1 operator) against
    central differences of J = w.x, J the mean phi_s on the cathode top face.
    Solves are dense LU here so that the differences carry only rounding
    noise, eps * cond(A) / h with cond(A) ~ 1e7; with h = 1e-3 both that and
    the O(h^2) truncation stay near 1e-7 relative (measured), so a 1e-5
    bound separates them from any structural mistake."""
    p = pi.make_custom(5, 4, 13, (5, 4), seed=8, sigma_log=1.0, corr_cells=3.0)
    w = pi.functional_weights(p)

    def J(sigma, Ds):
        A = O.Oracle(p.with_(sigma=sigma, Ds=tuple(Ds))).dense()
        return w @ np.linalg.solve(A, p.b)

    orc = O.Oracle(p)
    A = orc.dense()
    x = np.linalg.solve(A, p.b)
    lam = np.linalg.solve(A.T, w)
    gs, gD = orc.gradient(x, lam)
    lay = np.repeat(np.array([0 if k + 1 < p.na else (1 if k >= p.na + p.ns else -1)
                              for k in range(p.nz - 1)]), (p.nx - 1) * (p.ny - 1))
    assert np.all(gs[lay < 0] == 0.0)
    rng = np.random.default_rng(3)
    hstep = 1e-3
    sig0, D0 = p.sigma.copy(), np.array(p.Ds)
    for _ in range(3):
        v = rng.standard_normal(p.n_elem)
        vD = rng.standard_normal(2)
        fd = (J(sig0 * (1 + hstep * v), D0 * (1 + hstep * vD)) -
              J(sig0 * (1 - hstep * v), D0 * (1 - hstep * vD))) / (2 * hstep)
        ad = gs @ (sig0 * v) + gD @ (D0 * vD)
        assert ad == pytest.approx(fd, rel=1e-5, abs=1e-12)
    # each parameter group on its own
    fdD = (J(sig0, D0 * np.array([1 + hstep, 1])) - J(sig0, D0 * np.array([1 - hstep, 1]))) / (2 * hstep)
    assert gD[0] * D0[0] == pytest.approx(fdD, rel=1e-5, abs=1e-14)
