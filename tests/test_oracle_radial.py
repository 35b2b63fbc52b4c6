"""Pins of the oracle's particle discretization (Sec. 3.1: eq. L1, L2, L0, LR,
the geometric mesh after Remark 3.1) against closed forms."""
import numpy as np
import pytest

import oracle as O


def dense_L(N, D, theta):
    rho = O.radial_mesh(N, theta)
    sub, dia, sup, flux = O.radial_rows(N, D, rho)
    L = np.diag(dia) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
    return rho, L, flux


@pytest.mark.parametrize("N", [3, 8, 16, 20, 32])
@pytest.mark.parametrize("theta", [1.0, 0.5, 0.3])
def test_mesh_geometry(N, theta):
    rho = O.radial_mesh(N, theta)
    d = np.diff(rho)
    assert rho[0] == 0.0 and rho[-1] == 1.0
    assert np.all(d > 0)
    # geometric progression with last/first interval ratio theta
    assert d[-1] / d[0] == pytest.approx(theta, rel=1e-12)
    if N > 2:
        q = d[1:] / d[:-1]
        assert np.allclose(q, theta ** (1.0 / (N - 2)), rtol=1e-12)


@pytest.mark.parametrize("N", [8, 16, 20, 32])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_R1_zero_row_sums(N, theta):
    """Constants are in the kernel of L_h (no flux => no change)."""
    _, L, _ = dense_L(N, 1e-4, theta)
    assert np.max(np.abs(L @ np.ones(N))) <= 1e-13 * np.max(np.abs(L))


@pytest.mark.parametrize("N", [5, 10, 20, 32])
@pytest.mark.parametrize("theta", [1.0, 0.5, 0.3])
def test_R2_exact_on_quadratics_and_flux_sign(N, theta):
    """c = rho^2 has (1/r^2)(r^2 D c')' = 6D everywhere, and its surface flux
    -D c'(R) = -2 D R = i_n/F.  The scheme is exact on quadratics only if the
    flux term of eq. (LR) enters with the sign of eq. (particleBC2)."""
    D = 0.37
    rho, L, flux = dense_L(N, D, theta)
    c = rho ** 2
    inF = -2.0 * D * 1.0
    Lc = L @ c
    Lc[-1] += flux * inF
    assert np.allclose(Lc, 6.0 * D, rtol=0, atol=1e-11 * max(1.0, np.abs(L).max()))
    # the sign printed in eq. (LR) (+2 i_n/(F dr)(1+dr/R)) is not exact
    Lbad = L @ c
    Lbad[-1] -= flux * inF
    assert abs(Lbad[-1] - 6.0 * D) > 1.0


@pytest.mark.parametrize("N", [8, 16, 20, 32])
@pytest.mark.parametrize("theta", [1.0, 0.5, 0.3])
def test_R4_conservation_weights(N, theta):
    """The left null vector w of L_h is non-negative and diag(w) L_h is
    symmetric (the scheme conserves sum_i w_i c_i under zero flux)."""
    _, L, _ = dense_L(N, 1.0, theta)
    u, s, vt = np.linalg.svd(L.T)
    w = vt[-1]
    w = w / w[np.argmax(np.abs(w))]
    assert s[-1] <= 1e-12 * s[0]
    assert np.all(w >= -1e-12)
    WL = np.diag(w) @ L
    assert np.allclose(WL, WL.T, atol=1e-12 * np.abs(WL).max())


@pytest.mark.parametrize("N", [8, 16, 20, 32])
def test_R4_closed_form_uniform(N):
    """Uniform mesh: w = (0, 1, 4, ..., (N-2)^2, (N-1)(N-2)/2) dr^3."""
    _, L, _ = dense_L(N, 1.0, 1.0)
    dr = 1.0 / (N - 1)
    w = np.array([i * i for i in range(N - 1)] + [(N - 1) * (N - 2) / 2.0]) * dr ** 3
    assert np.max(np.abs(w @ L)) <= 1e-12 * np.abs(L).max()


@pytest.mark.parametrize("N", [8, 16, 20, 32])
def test_R5_flux_consistency(N):
    """Uniform mesh: w.L_h c = -(R^2 - dr^2) i_n/F for any c, an O(dr^2)
    approximation of the exact lithium loss -R^2 i_n/F of int r^2 c dr."""
    rng = np.random.default_rng(N)
    rho, L, flux = dense_L(N, 0.7, 1.0)
    dr = 1.0 / (N - 1)
    w = np.array([i * i for i in range(N - 1)] + [(N - 1) * (N - 2) / 2.0]) * dr ** 3
    c = rng.standard_normal(N)
    inF = 0.83
    Lc = L @ c
    Lc[-1] += flux * inF
    assert w @ Lc == pytest.approx(-(1.0 - dr * dr) * inF, rel=1e-11)


def test_R6_second_order_on_regular_meshes():
    """Truncation error of L_h on c = rho^4 ((1/r^2)(r^2 c')' = 20 rho^2,
    surface flux i_n/F = -4 D R^3) is O(dr^2) at the centre and interior
    nodes of a geometric mesh with fixed theta (locally regular, Remark 3.1).
    At the surface node the ghost-point row of eq. (LR) gives exactly
    20 D - 8 D dr + 2 D dr^2 on rho^4 (Taylor expansion of (1-dr)^4)."""
    D = 1.0
    errs = []
    for N in (11, 21, 41, 81):
        rho, L, flux = dense_L(N, D, 0.5)
        c = rho ** 4
        Lc = L @ c
        Lc[-1] += flux * (-4.0 * D)
        errs.append(np.max(np.abs(Lc[:-1] - 20.0 * D * rho[:-1] ** 2)))
        dr = rho[-1] - rho[-2]
        assert Lc[-1] == pytest.approx(20 * D - 8 * D * dr + 2 * D * dr * dr, rel=1e-10)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


def test_surface_coupling_scale(oracle_mod):
    """Gamma = lambda_c * 2 (1 + dr/R) / dr with dr the last interval."""
    import p4d_inputs as pi
    p = pi.make_custom(4, 4, 12, (10, 7), seed=3, lambda_c=0.25)
    o = O.Oracle(p)
    for el in range(2):
        rho, sub, dia, sup, gam = o.radial(el)
        dr = rho[-1] - rho[-2]
        assert gam == pytest.approx(0.25 * 2 * (1 + dr) / dr, rel=1e-14)
        assert sub[-1] == pytest.approx(2 * p.Ds[el] / dr ** 2, rel=1e-14)
