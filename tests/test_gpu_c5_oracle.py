"""The large-cell workload (128 x 128 x 256 nodes, N_r = 16, lognormal
conductivities, 67,993,600 unknowns) against full oracle solves on the host
cores: the GPU's forward and adjoint solutions at rtol 1e-8, per field,
against the oracle's FP64 solutions at rtol 1e-8 (the spec bar 1e-6),
and the gradient formula on the two pairs.  About 40 GB of host memory and a
few minutes of the host's cores for the two oracle solves."""
import numpy as np
import pytest

import oracle as O
import p4d_inputs as pi
from tests.gpu_util import field_errors, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1500)
def test_C5_forward_and_adjoint_against_oracle_solves():
    from paper_2602_07225_amd import P4DSolver
    p = pi.make_config(5)
    w = pi.functional_weights(p)
    say(f"C5 N={p.N}: GPU solves")
    s = P4DSolver(p)
    s.setup(rtol=1e-8)
    x, i1 = s.solve(to_dev(p.b))
    lam, i2 = s.solve_adjoint(to_dev(w))
    gs, gD = s.gradient(x, lam)
    x, lam, gs, gD = to_np(x), to_np(lam), to_np(gs), to_np(gD)
    assert i1.status == 0 and i2.status == 0
    s.close()
    del s
    say(f"  GPU iters {i1.iters} / {i2.iters}; oracle setup on {O.num_threads()} threads")
    orc = O.Oracle(p).setup(rtol=1e-8)
    xo, io = orc.solve(p.b)
    ex = field_errors(p, x, xo)
    say(f"  forward: oracle iters {io.iters}", {k: f"{v:.1e}" for k, v in ex.items()})
    lo, jo = orc.solve(w, transpose=True)
    el = field_errors(p, lam, lo)
    say(f"  adjoint: oracle iters {jo.iters}", {k: f"{v:.1e}" for k, v in el.items()})
    assert io.status == 0 and jo.status == 0
    assert max(ex.values()) <= 1e-6
    assert max(el.values()) <= 1e-6
    gso, gDo = orc.gradient(xo, lo)
    rg = np.linalg.norm(gs - gso) / np.linalg.norm(gso)
    say(f"  dJ/dsigma rel err {rg:.1e}, dJ/dDs {gD} vs {gDo}")
    assert rg <= 1e-6
    assert np.allclose(gD, gDo, rtol=1e-6)
