"""Adjoint solve and parameter gradients through torch autograd (the
transposed operator and transposed preconditioner of the HIP library),
against the oracle and against finite differences; at a small size and at
the large-cell size (128 x 128 x 256 nodes, 68 M unknowns)."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def J_and_grads(s, p, sigma, Ds, w, **opts):
    import torch
    from paper_2602_07225_amd import solve
    sig = torch.as_tensor(sigma, device="cuda").clone().requires_grad_(True)
    D = torch.tensor(list(Ds), dtype=torch.float64, requires_grad=True)
    b = torch.as_tensor(p.b, device="cuda").clone().requires_grad_(True)
    x = solve(s, sig, D, b, **opts)
    J = (torch.as_tensor(w, device="cuda") * x).sum()
    J.backward()
    return J.item(), sig.grad, D.grad, b.grad, x


def test_autograd_matches_oracle():
    from paper_2602_07225_amd import P4DSolver
    p = pi.make_custom(7, 6, 19, (7, 9), seed=31, sigma_log=1.0, corr_cells=3.0)
    say(f"autograd small N={p.N}")
    w = pi.functional_weights(p)
    s = P4DSolver(p)
    J, gs, gD, gb, x = J_and_grads(s, p, p.sigma, p.Ds, w, rtol=1e-10)
    orc = O.Oracle(p).setup(rtol=1e-10)
    xo, _ = orc.solve(p.b)
    lo, _ = orc.solve(w, transpose=True)
    gso, gDo = orc.gradient(xo, lo)
    assert rel(to_np(x), xo) <= 1e-6
    assert rel(to_np(gb), lo) <= 1e-6
    assert rel(to_np(gs), gso) <= 1e-6
    assert np.allclose(to_np(gD), gDo, rtol=1e-6)


def test_autograd_finite_differences():
    """Central differences of GPU forward solves (relative step 1e-3, where
    the O(h^2) truncation and the solver noise are both ~1e-7)."""
    from paper_2602_07225_amd import P4DSolver, solve
    import torch
    p = pi.make_custom(7, 6, 19, (7, 9), seed=32, sigma_log=1.0, corr_cells=3.0)
    w = pi.functional_weights(p)
    s = P4DSolver(p)
    J0, gs, gD, _, _ = J_and_grads(s, p, p.sigma, p.Ds, w, rtol=1e-10)
    gs, gD = to_np(gs), to_np(gD)
    wt = torch.as_tensor(w, device="cuda")

    def J(sig, D):
        x = solve(s, torch.as_tensor(sig, device="cuda"), torch.tensor(D), to_dev(p.b), rtol=1e-10)
        return (wt * x).sum().item()

    rng = np.random.default_rng(5)
    h = 1e-3
    for t in range(5):
        v, vD = rng.standard_normal(p.n_elem), rng.standard_normal(2)
        fd = (J(p.sigma * (1 + h * v), np.array(p.Ds) * (1 + h * vD)) -
              J(p.sigma * (1 - h * v), np.array(p.Ds) * (1 - h * vD))) / (2 * h)
        ad = gs @ (p.sigma * v) + gD @ (np.array(p.Ds) * vD)
        say(f"  direction {t}: fd={fd:.10e} adjoint={ad:.10e}")
        assert ad == pytest.approx(fd, rel=1e-5)


@pytest.fixture(scope="module")
def c5():
    from paper_2602_07225_amd import P4DSolver
    p = pi.make_config(5)
    say(f"C5 N={p.N}")
    return p, P4DSolver(p)


def test_C5_forward_adjoint_gradient(c5):
    """The large-cell workload: forward and adjoint solves to rtol 1e-8,
    residuals confirmed by the oracle operator, gradients equal to the
    oracle's gradient formula evaluated at the GPU's x and lambda."""
    import torch
    p, s = c5
    w = pi.functional_weights(p)
    s.upload(p.sigma, p.kappa, p.g, p.s, p.e)
    s.set_diffusivity(p.Ds)
    s.setup(rtol=1e-8)
    x, i1 = s.solve(to_dev(p.b))
    lam, i2 = s.solve_adjoint(to_dev(w))
    say(f"  forward iters={i1.iters} t={i1.t_solve_ms:.1f} ms, adjoint iters={i2.iters} "
        f"t={i2.t_solve_ms:.1f} ms")
    assert i1.status == 0 and i2.status == 0
    orc = O.Oracle(p)
    xn, ln = to_np(x), to_np(lam)
    assert rel(orc.apply(xn), p.b) <= 1.0001e-8
    assert rel(orc.apply(ln, transpose=True), w) <= 1.0001e-8
    gs, gD = s.gradient(x, lam)
    gso, gDo = orc.gradient(xn, ln)
    # lambda^T K x cancels the large near-constant parts of x and lambda; the
    # oracle sums K x in standard form, the GPU in difference form, so they
    # agree to ~1e-8 here (1.3e-8 measured), not to machine precision
    assert rel(to_np(gs), gso) <= 1e-6
    assert np.allclose(to_np(gD), gDo, rtol=1e-10)


def test_C5_transpose_identity(c5):
    """<A x, y> = <x, A^T y> and <P^-1 x, y> = <x, P^-T y> at full size."""
    p, s = c5
    s.setup()
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal(p.N), rng.standard_normal(p.N)
    xd, yd = to_dev(x), to_dev(y)
    a = float(to_np(s.apply(xd)) @ y)
    b = float(x @ to_np(s.apply(yd, transpose=True)))
    assert a == pytest.approx(b, rel=1e-12)
    a = float(to_np(s.apply_pc(xd)) @ y)
    b = float(x @ to_np(s.apply_pc(yd, transpose=True)))
    assert a == pytest.approx(b, rel=1e-8)


def test_C5_finite_differences_20_directions(c5):
    """dJ/dsigma (per element) and dJ/dDs against central differences with
    relative step 1e-6 in 20 random directions.  The FD solves run at twice
    the attainable residual floor (eps * cond(A), measured first), since the
    solver noise in J has to stay well below h * |dJ|."""
    import torch
    p, s = c5
    w = pi.functional_weights(p)
    wt = torch.as_tensor(w, device="cuda")
    b = to_dev(p.b)
    s.upload(p.sigma, p.kappa, p.g, p.s, p.e)
    s.set_diffusivity(p.Ds)
    s.setup(rtol=1e-13, maxit=120)
    _, probe = s.solve(b)
    floor = probe.relres_true
    rtol = max(2.0 * floor, 1e-11)
    say(f"  residual floor {floor:.2e}, FD solves at rtol {rtol:.2e}")
    J0, gs, gD, _, _ = J_and_grads(s, p, p.sigma, p.Ds, w, rtol=rtol, maxit=3000)
    gs, gD = to_np(gs), to_np(gD)

    def J(sig, D):
        s.upload(sig, p.kappa, p.g, p.s, p.e)
        s.set_diffusivity(D)
        s.setup(rtol=rtol, maxit=3000)
        x, info = s.solve(b)
        assert info.relres_true <= rtol
        return (wt * x).sum().item()

    rng = np.random.default_rng(20)
    h = 1e-6
    worst = 0.0
    for t in range(20):
        v, vD = rng.standard_normal(p.n_elem), rng.standard_normal(2)
        fd = (J(p.sigma * (1 + h * v), np.array(p.Ds) * (1 + h * vD)) -
              J(p.sigma * (1 - h * v), np.array(p.Ds) * (1 - h * vD))) / (2 * h)
        ad = gs @ (p.sigma * v) + gD @ (np.array(p.Ds) * vD)
        err = abs(fd - ad) / abs(ad)
        worst = max(worst, err)
        say(f"  direction {t}: fd={fd:.8e} adjoint={ad:.8e} rel={err:.1e}")
    assert worst <= 1e-4


def test_autograd_backward_after_another_forward():
    """Two differentiable solves on one solver at different parameters, then
    the backward of each: every gradient is the oracle's at its own
    forward's parameters (the backward restores the state it recorded)."""
    import torch
    from paper_2602_07225_amd import P4DSolver, solve
    p = pi.make_custom(7, 6, 19, (7, 9), seed=34, sigma_log=1.0, corr_cells=3.0)
    w = pi.functional_weights(p)
    wt = torch.as_tensor(w, device="cuda")
    s = P4DSolver(p)
    pts = [(p.sigma, np.array(p.Ds)), (p.sigma * np.exp(0.3 * np.sin(np.arange(p.n_elem))),
                                       np.array(p.Ds) * np.array([0.5, 2.0]))]
    outs = []
    for sig, D in pts:
        st = torch.as_tensor(sig, device="cuda").clone().requires_grad_(True)
        Dt = torch.tensor(D, dtype=torch.float64, requires_grad=True)
        x = solve(s, st, Dt, to_dev(p.b), rtol=1e-10)
        outs.append((st, Dt, (wt * x).sum()))
    for k in (0, 1):
        st, Dt, J = outs[k]
        J.backward()
        q = p.with_(sigma=pts[k][0], Ds=tuple(pts[k][1]))
        orc = O.Oracle(q).setup(rtol=1e-10)
        xo, _ = orc.solve(q.b)
        lo, _ = orc.solve(w, transpose=True)
        gso, gDo = orc.gradient(xo, lo)
        say(f"  forward {k}: dJ/dsigma rel err {rel(to_np(st.grad), gso):.1e}")
        assert rel(to_np(st.grad), gso) <= 1e-6
        assert np.allclose(to_np(Dt.grad), gDo, rtol=1e-6)


def test_autograd_keeps_separate_coefficients_and_storage():
    """A differentiable solve on a cell with separate transport coefficients
    and a per-element porosity: forward, adjoint and gradients equal the
    oracle's for that operator, and a plain solve afterwards still sees the
    same coefficients."""
    from paper_2602_07225_amd import P4DSolver
    rng = np.random.default_rng(35)
    p = pi.make_custom(7, 6, 19, (7, 9), seed=35, sigma_log=1.0, corr_cells=3.0)
    p = p.with_(kappa_d=1.2 * p.kappa * np.exp(0.3 * rng.standard_normal(p.n_elem)),
                dce=np.exp(0.5 * rng.standard_normal(p.n_elem)),
                eps_e=0.2 + 0.6 * rng.random(p.n_elem))
    w = pi.functional_weights(p)
    s = P4DSolver(p)
    J, gs, gD, gb, x = J_and_grads(s, p, p.sigma, p.Ds, w, rtol=1e-10)
    orc = O.Oracle(p).setup(rtol=1e-10)
    xo, _ = orc.solve(p.b)
    lo, _ = orc.solve(w, transpose=True)
    gso, gDo = orc.gradient(xo, lo)
    say(f"  x {rel(to_np(x), xo):.1e} lambda {rel(to_np(gb), lo):.1e} dsigma {rel(to_np(gs), gso):.1e}")
    assert rel(to_np(x), xo) <= 1e-6
    assert rel(to_np(gb), lo) <= 1e-6
    assert rel(to_np(gs), gso) <= 1e-6
    assert np.allclose(to_np(gD), gDo, rtol=1e-6)
    x2, info = s.solve(to_dev(p.b))
    assert info.status == 0 and rel(to_np(x2), xo) <= 1e-6
