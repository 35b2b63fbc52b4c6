"""Parity at the benchmark sizes (15.3 M unknowns), in the configuration that
bench.py times: the oracle is fast enough at this size to compare whole
vectors (operator, preconditioner) and whole solutions."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import field_errors, rel, say, solver_for, to_dev, to_np

pytestmark = pytest.mark.gpu

_cache = {}


def big(cid):
    if cid not in _cache:
        p = pi.make_config(cid)
        _cache[cid] = (p, O.Oracle(p))
    return _cache[cid]


@pytest.mark.parametrize("transpose", [False, True])
def test_C2_operator_full(transpose):
    p, orc = big(2)
    say(f"C2 operator transpose={transpose} N={p.N}")
    s = solver_for(p)
    x = np.random.default_rng(5).standard_normal(p.N)
    y = to_np(s.apply(to_dev(x), transpose))
    ref = orc.apply(x, transpose)
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("deg", [2, 3])
def test_C2_preconditioner_full(deg):
    p, orc = big(2)
    say(f"C2 preconditioner, Chebyshev degree {deg}")
    orc.setup(cheb_degree=deg)
    s = solver_for(p).setup(cheb_degree=deg)
    r = np.random.default_rng(6).standard_normal(p.N)
    errs = field_errors(p, to_np(s.apply_pc(to_dev(r))), orc.apply_pc(r))
    say("  errors", {k: f"{v:.1e}" for k, v in errs.items()})
    # The field operators given to the V-cycles have condition ~1e7 here
    # (constant-mode eigenvalue ~ omega m g ~ h^3 against stiffness ~ h), so
    # FP64 results that differ only in summation order agree to ~1e-16 * 1e7.
    assert max(errs.values()) <= 1e-8


def test_C2_solve_full():
    """The benchmark solve: FP64, SCHUR, V(3,3) Chebyshev, FGMRES(30), rtol
    1e-8."""
    p, orc = big(2)
    say("C2 solve (oracle ~20 s on the host)")
    orc.setup(rtol=1e-8, cheb_degree=3)
    xo, io = orc.solve(p.b)
    s = solver_for(p).setup(rtol=1e-8, cheb_degree=3)
    x, info = s.solve(to_dev(p.b))
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  iters gpu={info.iters} oracle={io.iters}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0 and io.status == 0
    assert max(errs.values()) <= 1e-6
    assert rel(orc.apply(x), p.b) <= 1.0001e-8


def test_C3_fp32_preconditioned_solve_full():
    """Lognormal cube with the FP32 preconditioner and FP32 Z basis, against
    the FP64 oracle solution."""
    p, orc = big(3)
    say("C3 fp32 solve (oracle ~20 s on the host)")
    orc.setup(rtol=1e-8)
    xo, io = orc.solve(p.b)
    s = solver_for(p, pc_prec=1, z_fp32=True).setup(pc_prec=1, z_fp32=1, rtol=1e-8)
    x, info = s.solve(to_dev(p.b))
    x = to_np(x)
    errs = field_errors(p, x, xo)
    say(f"  iters gpu={info.iters} oracle={io.iters}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert info.status == 0
    assert max(errs.values()) <= 1e-6
    assert rel(orc.apply(x), p.b) <= 1.0001e-8
