"""Separate transport coefficients (diffusion-potential block and c_e
diffusion with their own element coefficients), a physical cell length and
per-electrode surface coupling scales: operator, preconditioners and solves
on the GPU against the oracle."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import field_errors, rel, say, solver_for, to_dev, to_np

pytestmark = pytest.mark.gpu


def general(seed=51, nx=9, ny=7, nz=23, nr=(7, 11)):
    """Separate coefficients, a cell length and coupling scales.  (With a
    physical length such as 225 um and unit coefficients the c_e and phi_e
    blocks would be nearly singular, storage ~h^3 against stiffness ~h, and
    two FP64 summation orders would differ by ~1e-5; the physical cell
    scales its Newton systems instead.)"""
    p = pi.make_custom(nx, ny, nz, nr, seed=seed, sigma_log=1.0, corr_cells=3.0)
    rng = np.random.default_rng(seed + 7)
    return p.with_(kappa_d=np.exp(0.7 * rng.standard_normal(p.n_elem)),
                   dce=np.exp(0.7 * rng.standard_normal(p.n_elem)),
                   length=3.0, lambda_el=(0.4, 2.5))


@pytest.mark.parametrize("transpose", [False, True])
def test_general_operator_parity(transpose):
    p = general()
    orc = O.Oracle(p)
    s = solver_for(p)
    x = np.random.default_rng(1).standard_normal(p.N)
    y = to_np(s.apply(to_dev(x), transpose))
    ref = orc.apply(x, transpose)
    say(f"general operator transpose={transpose}: max rel {np.max(np.abs(y - ref)) / np.max(np.abs(ref)):.1e}")
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("pc", [O.PC_SCHUR, O.PC_BJ, O.PC_BGS])
@pytest.mark.parametrize("transpose", [False, True])
def test_general_preconditioner_parity(pc, transpose):
    p = general()
    orc = O.Oracle(p).setup(pc=pc)
    s = solver_for(p).setup(pc=pc)
    r = np.random.default_rng(2).standard_normal(p.N)
    errs = field_errors(p, to_np(s.apply_pc(to_dev(r), transpose)), orc.apply_pc(r, transpose))
    say(f"  pc={pc} transpose={transpose}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-10


@pytest.mark.parametrize("pc", [O.PC_SCHUR, O.PC_BGS])
def test_general_solve_parity(pc):
    p = general()
    cgs2 = pc != O.PC_SCHUR
    orc = O.Oracle(p).setup(pc=pc, rtol=1e-8, cgs2=cgs2)
    xo, io = orc.solve(p.b)
    s = solver_for(p).setup(pc=pc, rtol=1e-8, cgs2=int(cgs2))
    x, info = s.solve(to_dev(p.b))
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  pc={pc} iters gpu={info.iters} oracle={io.iters}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and io.status == 0
    assert abs(info.iters - io.iters) <= 2
    assert max(errs.values()) <= 1e-6
    assert rel(orc.apply(x), p.b) <= 1.0001e-8


@pytest.mark.parametrize("transpose", [False, True])
def test_general_schur_operator_parity(transpose):
    """The Schur complement of the particle blocks in its per-node form
    (separate coefficients, per-element storage)."""
    p = general().with_(eps_e=0.1 + 0.8 * np.random.default_rng(8).random(general().n_elem))
    orc = O.Oracle(p)
    s = solver_for(p)
    y = np.random.default_rng(9).standard_normal(orc.n_macro)
    w = to_np(s.apply_schur(to_dev(y), transpose))
    ref = orc.schur_apply(y, transpose)
    assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_general_schur_krylov_solve_parity():
    p = general()
    orc = O.Oracle(p).setup(rtol=1e-8, krylov=O.KRYLOV_SCHUR)
    xo, io = orc.solve(p.b)
    s = solver_for(p).setup(rtol=1e-8)
    x, info = s.solve(to_dev(p.b), krylov=1)
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  general Schur-Krylov iters gpu={info.iters} oracle={io.iters}",
        {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and io.status == 0
    assert abs(info.iters - io.iters) <= 2
    assert max(errs.values()) <= 1e-6
    assert rel(orc.apply(x), p.b) <= 1.0001e-8


def test_transport_reset():
    p = general()
    plain = p.with_(kappa_d=None, dce=None)
    s = solver_for(p)
    x = np.random.default_rng(3).standard_normal(p.N)
    s.set_transport(None, None)          # back to chi * kappa and kappa
    y = to_np(s.apply(to_dev(x)))
    ref = O.Oracle(plain).apply(x)
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))
    # explicit defaults take the general kernels and agree
    s.set_transport(p.chi * p.kappa, p.kappa)
    y2 = to_np(s.apply(to_dev(x)))
    assert np.max(np.abs(y2 - ref)) <= 1e-13 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# porosity per element (c_e storage), alone and with separate coefficients
# ---------------------------------------------------------------------------
def porous(seed=52, with_transport=False):
    p = pi.make_custom(9, 7, 23, (7, 11), seed=seed, sigma_log=1.0, corr_cells=3.0)
    rng = np.random.default_rng(seed + 9)
    q = p.with_(eps_e=0.1 + 0.8 * rng.random(p.n_elem), length=3.0)
    if with_transport:
        q = q.with_(kappa_d=np.exp(0.7 * rng.standard_normal(p.n_elem)),
                    dce=np.exp(0.7 * rng.standard_normal(p.n_elem)))
    return q


@pytest.mark.parametrize("with_transport", [False, True])
@pytest.mark.parametrize("transpose", [False, True])
def test_storage_operator_parity(with_transport, transpose):
    p = porous(with_transport=with_transport)
    orc = O.Oracle(p)
    s = solver_for(p)
    x = np.random.default_rng(4).standard_normal(p.N)
    y = to_np(s.apply(to_dev(x), transpose))
    ref = orc.apply(x, transpose)
    say(f"storage operator transport={with_transport} transpose={transpose}: "
        f"max rel {np.max(np.abs(y - ref)) / np.max(np.abs(ref)):.1e}")
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("pc", [O.PC_SCHUR, O.PC_BJ, O.PC_BGS])
@pytest.mark.parametrize("transpose", [False, True])
def test_storage_preconditioner_parity(pc, transpose):
    p = porous()
    orc = O.Oracle(p).setup(pc=pc)
    s = solver_for(p).setup(pc=pc)
    r = np.random.default_rng(5).standard_normal(p.N)
    errs = field_errors(p, to_np(s.apply_pc(to_dev(r), transpose)), orc.apply_pc(r, transpose))
    say(f"  storage pc={pc} transpose={transpose}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-10


@pytest.mark.parametrize("with_transport", [False, True])
def test_storage_solve_parity(with_transport):
    p = porous(with_transport=with_transport)
    orc = O.Oracle(p).setup(rtol=1e-8)
    xo, io = orc.solve(p.b)
    s = solver_for(p).setup(rtol=1e-8)
    x, info = s.solve(to_dev(p.b))
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  storage transport={with_transport} iters gpu={info.iters} oracle={io.iters}",
        {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and io.status == 0
    assert abs(info.iters - io.iters) <= 2
    assert max(errs.values()) <= 1e-6
    assert rel(orc.apply(x), p.b) <= 1.0001e-8


def test_storage_reset_restores_the_tiled_path():
    """Clearing the storage returns to the per-material (tiled) operator."""
    p = porous()
    plain = p.with_(eps_e=None)
    s = solver_for(p)
    s.set_storage(None)
    x = np.random.default_rng(6).standard_normal(p.N)
    ref = O.Oracle(plain).apply(x)
    y = to_np(s.apply(to_dev(x)))
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))
    s.setup(rtol=1e-8)
    xs, info = s.solve(to_dev(p.b), krylov=1)
    assert info.status == 0
    assert rel(O.Oracle(plain).apply(to_np(xs)), p.b) <= 1.0001e-8
    # a re-upload (new sigma) keeps a storage that is set
    s.set_storage(p.eps_e)
    s.upload(p.sigma * 1.5, p.kappa, p.g, p.s, p.e)
    ref2 = O.Oracle(p.with_(sigma=p.sigma * 1.5)).apply(x)
    y2 = to_np(s.apply(to_dev(x)))
    assert np.max(np.abs(y2 - ref2)) <= 1e-13 * np.max(np.abs(ref2))
