"""Helpers for the GPU tests: build a solver for a seeded problem, move
vectors between numpy and the device, compare per field."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def solver_for(p, **kw):
    from paper_2602_07225_amd import P4DSolver
    return P4DSolver(p, **kw)


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def field_errors(p, x, ref):
    o = p.offsets
    names = ["phi_s", "phi_e", "c_e", "c_s_anode", "c_s_cathode"]
    out = {"all": rel(x, ref)}
    for nm, a, b in zip(names, o[:-1], o[1:]):
        out[nm] = rel(x[a:b], ref[a:b])
    return out
