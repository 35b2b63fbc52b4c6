"""The solve's host-device protocol: the setup returns before its kernels
end and hands its Chebyshev bounds over at the first use; a solve enqueues
the next Arnoldi step before the host has read the current step's
Hessenberg column; profiling can time a sample of a class's launches.
None of this may change a result."""
import numpy as np
import pytest

import p4d_inputs as pi
from paper_2602_07225_amd import _lib as L
from paper_2602_07225_amd._lib import P4DError
from tests.gpu_util import say, solver_for, to_dev, to_np

pytestmark = pytest.mark.gpu


def problem():
    return pi.make_custom(37, 29, 61, (13, 8), seed=23, sigma_log=1.0)


def test_setup_and_solve_on_different_streams():
    """Setup on one stream, solve on another: the solve waits for the setup
    (its bounds and its stencils) and gives the same-stream result."""
    import torch
    p = problem()
    s = solver_for(p)
    b = to_dev(p.b)
    s.setup(rtol=1e-10)
    x0, i0 = s.solve(b)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(2):
        say(f"two streams, repetition {rep}")
        with torch.cuda.stream(sa):
            s.setup(rtol=1e-10)
        with torch.cuda.stream(sb):
            x1, i1 = s.solve(b)
        torch.cuda.synchronize()
        assert i1.status == 0 and i1.iters == i0.iters
        assert np.array_equal(to_np(x1), to_np(x0))


@pytest.mark.parametrize("maxit", [1, 2, 3, 5])
def test_solve_stopped_at_maxit_equals_one_cycle(maxit):
    """maxit = k with the default restart (the host may enqueue step k + 1
    before it reads step k) equals one cycle of restart k (no step beyond
    the cycle is ever enqueued): x after k steps, bit for bit."""
    p = problem()
    s = solver_for(p)
    b = to_dev(p.b)
    s.setup(rtol=1e-12)
    xa, ia = s.solve(b, maxit=maxit)
    xb, ib = s.solve(b, maxit=maxit, restart=maxit)
    say(f"maxit {maxit}: iters {ia.iters} / {ib.iters}, status {ia.status} / {ib.status}")
    assert ia.iters == ib.iters == maxit
    assert ia.status == ib.status == L.P4D_NOT_CONVERGED
    assert np.array_equal(to_np(xa), to_np(xb))


@pytest.mark.parametrize("krylov", [0, 1])
def test_solve_without_an_update_leaves_x_zero(krylov):
    """The first update assigns x = Z y (x is not cleared before it): a solve
    that stops before any update (maxit = 0) returns x = 0 in the Krylov
    space (all unknowns, or the electrode-level ones over the Schur
    complement, whose particle unknowns then follow from them), and the
    next solve is unaffected."""
    p = problem()
    s = solver_for(p)
    b = to_dev(p.b)
    s.setup(rtol=1e-10)
    x1, i1 = s.solve(b, krylov=krylov)
    x0, i0 = s.solve(b, maxit=0, krylov=krylov)
    say(f"krylov {krylov}: maxit 0 status {i0.status} iters {i0.iters}")
    assert i0.iters == 0 and i0.status == L.P4D_NOT_CONVERGED
    nk = p.N if krylov == 0 else p.offsets[3]   # phi_s, phi_e, c_e
    assert not np.any(to_np(x0)[:nk])
    x2, i2 = s.solve(b, krylov=krylov)
    assert i2.status == 0 and np.array_equal(to_np(x2), to_np(x1))


def test_nonfinite_bound_reported_at_first_use():
    """A coefficient that makes a Gershgorin bound non-finite: the setup
    returns (it does not wait for its kernels), the first solve reports
    P4D_ERR_NONFINITE, and a later valid setup solves again."""
    p = problem()
    s = solver_for(p)
    b = to_dev(p.b)
    sig = np.array(p.sigma, dtype=np.float64)
    sig[0] = np.nan   # an anode element (sigma is read on electrode elements only)
    s.upload(sig, p.kappa, p.g, p.s, p.e)
    s.setup()
    with pytest.raises(P4DError) as e:
        s.solve(b)
    assert e.value.status == L.P4D_ERR_NONFINITE
    with pytest.raises(P4DError) as e:   # the failed bounds leave no setup behind
        s.solve(b)
    assert e.value.status == L.P4D_ERR_STATE
    s.upload(p.sigma, p.kappa, p.g, p.s, p.e)
    s.setup(rtol=1e-8)
    x, info = s.solve(b)
    assert info.status == 0 and np.all(np.isfinite(to_np(x)))


@pytest.mark.parametrize("degree", [2, 3])
def test_sampled_profiling_counts_every_nth_interval(degree):
    """p4d_profile_every(n): one event pair in n of each class is timed, and
    the solve's result does not depend on it.  The level-0 smoothing steps
    share a pair per side of the coarse correction: degree - 1 launches
    before, degree after, so the timed launches are those of every n-th of
    these intervals."""
    p = problem()
    s = solver_for(p)
    b = to_dev(p.b)
    s.setup(rtol=1e-8, cheb_degree=degree)
    x0, _ = s.solve(b)
    cls = next(k for k, v in L.KERNEL_CLASSES.items() if v == "smooth0")
    counts, per = {}, {}
    for every in (1, 3, 7):
        L.p4d_profile(s.ctx, 1 << cls)
        L.p4d_profile_every(s.ctx, every)
        x, _ = s.solve(b)
        ms, n, by = L.p4d_profile_read(s.ctx, cls)
        L.p4d_profile(s.ctx, 0)
        L.p4d_profile_every(s.ctx, 1)
        counts[every] = n
        per[every] = ms / n
        say(f"degree {degree}, every {every}: {n} timed launches, {ms:.3f} ms")
        assert n > 0 and ms > 0.0 and by > 0.0
        assert np.array_equal(to_np(x), to_np(x0))
    cycles, rem = divmod(counts[1], 2 * degree - 1)
    assert rem == 0
    sizes = [n for _ in range(cycles) for n in (degree - 1, degree) if n > 0]
    for every in (3, 7):
        assert counts[every] == sum(sizes[::every])
    with pytest.raises(P4DError):
        L.p4d_profile_every(s.ctx, 0)
