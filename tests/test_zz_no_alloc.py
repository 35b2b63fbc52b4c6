"""The entry point that allocates nothing (p4d_solve_noalloc): upload +
setup + solve on the library's static scratch array, called through the C
ABI, against the existing entry points (p4d_upload + p4d_setup + p4d_solve
on a caller workspace) on the same inputs, for two calls in a row, the
second on a smaller problem; and its host-side rejection of a problem too
large for the scratch."""
import numpy as np
import pytest

import p4d_inputs as pi
from tests.gpu_util import field_errors, say, to_dev, to_np


def _noalloc(p, opts_kw):
    import torch
    from paper_2602_07225_amd import _lib as L
    desc = L.desc_from(p)
    ctx = L.p4d_create(desc)
    try:
        arrs = [to_dev(a) for a in (p.sigma, p.kappa, p.g, p.s, p.e)]
        b = to_dev(p.b)
        x = torch.full_like(b, float("nan"))
        st, info = L.p4d_solve_noalloc(ctx, *arrs, b, x, L.default_opts(**opts_kw))
        torch.cuda.synchronize()
        return st, info, to_np(x)
    finally:
        L.p4d_destroy(ctx)


def _existing(p, opts_kw):
    from paper_2602_07225_amd import P4DSolver
    s = P4DSolver(p)
    s.setup(**opts_kw)
    x, info = s.solve(to_dev(p.b))
    return info, to_np(x)


@pytest.mark.gpu
@pytest.mark.parametrize("pc_prec", [0, 1])
def test_noalloc_equals_existing_entry_points(pc_prec):
    from paper_2602_07225_amd import _lib as L
    opts = dict(rtol=1e-8, pc_prec=pc_prec)
    # the second call is smaller than the first and reuses the same scratch
    for p in (pi.make_config(1), pi.make_custom(6, 5, 13, (5, 7), seed=61, sigma_log=1.0,
                                                corr_cells=2.0)):
        say(f"noalloc N={p.N} pc_prec={pc_prec}")
        st, info, x = _noalloc(p, opts)
        ref_info, xr = _existing(p, opts)
        errs = field_errors(p, x, xr)
        say(f"  iters {info.iters} / {ref_info.iters}", {k: f"{v:.1e}" for k, v in errs.items()})
        assert st == L.P4D_OK and info.status == 0
        assert info.iters == ref_info.iters
        assert np.all(np.isfinite(x))
        assert max(errs.values()) <= 1e-12


@pytest.mark.gpu
def test_noalloc_rejects_too_large_problem():
    from paper_2602_07225_amd import P4DError, _lib as L
    p = pi.make_custom(64, 64, 96, (20, 20), seed=62)
    ctx = L.p4d_create(L.desc_from(p))
    try:
        need = L.p4d_workspace_size(ctx, L.default_opts())
        assert need > L.P4D_NOALLOC_MAX_BYTES
        dummy = to_dev(np.zeros(4))
        with pytest.raises(P4DError) as e:
            L.p4d_solve_noalloc(ctx, dummy, dummy, dummy, dummy, dummy, dummy, to_dev(np.zeros(4)),
                                L.default_opts())
        assert e.value.status == L.P4D_ERR_OOM
        assert "scratch" in str(e.value)
    finally:
        L.p4d_destroy(ctx)
