"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/p4d.h, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(p4d_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2602_07225_amd import _lib
    return _lib.lib()


def test_library_exports_every_declared_symbol(L):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), f"{s} declared in include/ but not exported"


def test_binding_names_match_header():
    from paper_2602_07225_amd import _lib
    for s in declared_symbols():
        assert s in _lib.EXPORTED, s


def test_invalid_descriptions_rejected_on_host(L):
    from paper_2602_07225_amd import _lib
    base = dict(nx=8, ny=8, nz=24, na=10, ns=4, nr=(10, 10), Ds=(1e-4, 4e-5),
                theta_bar=(0.5, 0.5), dt=1.0, chi=1.2, tc=0.6, lambda_c=1.0,
                eps_elec=0.3, eps_sep=1.0)

    class P:
        pass

    bad = [dict(nx=1), dict(nz=4), dict(na=1), dict(ns=0), dict(na=12, ns=11),
           dict(nr=(2, 10)), dict(nr=(10, 65)), dict(Ds=(0.0, 1.0)), dict(theta_bar=(1.5, 0.5)),
           dict(dt=0.0), dict(eps_elec=0.0)]
    for b in bad:
        p = P()
        for k, v in {**base, **b}.items():
            setattr(p, k, v)
        h = C.c_void_p()
        st = L.p4d_create(C.byref(_lib.desc_from(p)), C.byref(h))
        assert st == _lib.P4D_ERR_INVALID_ARG, b
        assert not h.value
    assert L.p4d_create(None, None) == _lib.P4D_ERR_INVALID_ARG
    assert L.p4d_solve(None, None, None, None, None, None) == _lib.P4D_ERR_INVALID_ARG
    assert L.p4d_status_string(_lib.P4D_ERR_STATE) == b"call out of order"


def test_default_options(L):
    from paper_2602_07225_amd import _lib
    o = _lib.default_opts()
    assert (o.pc, o.pc_prec, o.restart, o.maxit, o.cheb_degree, o.coarse_max) == (0, 0, 30, 1000, 2, 64)
    assert o.rtol == 1e-8
    # block Gauss-Seidel: the paper's ordering (phi_e, c_s, phi_s, c_e)
    assert o.bgs_order == _lib.P4D_BGS_PAPER_ORDER == 1 | 3 << 2 | 0 << 4 | 2 << 6


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the C layout: sizes and member offsets as the
    host compiler lays out the header's structs."""
    import ctypes as C
    import os
    import subprocess
    from paper_2602_07225_amd import _lib
    hdr = os.path.join(os.path.dirname(__file__), "..", "include", "p4d.h")
    checks = {"p4d_solve_opts": (_lib.SolveOpts, ["rtol", "bgs_order", "krylov"]),
              "p4d_problem_desc": (_lib.ProblemDesc, ["Ds", "dt", "length", "lambda_el"]),
              "p4d_phys_params": (_lib.PhysParams, ["theta_bar", "current", "eps_sep", "el"]),
              "p4d_newton_info": (_lib.NewtonInfo, ["update", "t_ms"])}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{os.path.abspath(hdr)}"',
             "int main(void) {"]
    for cname, (_, members) in checks.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for m in members:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {m}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-o", str(exe), str(src)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    expect = []
    for cname, (cls, members) in checks.items():
        expect.append(C.sizeof(cls))
        expect += [getattr(cls, m).offset for m in members]
    assert vals == expect


def test_header_constants_match_binding():
    import os
    import re
    from paper_2602_07225_amd import _lib
    h = open(os.path.join(os.path.dirname(__file__), "..", "include", "p4d.h")).read()
    for name in ("P4D_PC_SCHUR", "P4D_PC_BJ", "P4D_PC_BGS", "P4D_F_PHIS", "P4D_F_PHIE",
                 "P4D_F_CE", "P4D_F_CS", "P4D_K_OPERATOR", "P4D_K_RADIAL", "P4D_K_BATCH_PC",
                 "P4D_K_COUPLING", "P4D_K_COUNT", "P4D_KRYLOV_FULL", "P4D_KRYLOV_SCHUR"):
        m = re.search(name + r"\s*=\s*(\d+)", h)
        assert m and int(m.group(1)) == getattr(_lib, name), name
