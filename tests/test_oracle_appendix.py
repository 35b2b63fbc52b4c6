"""Pins of the oracle's material functions and case constants against the
appendix "Model Parameters" as printed.

The fixture ``golden/appendix_model_parameters.txt`` holds the printed LaTeX
of the open-circuit potential fits (eq. ocp_cathode, ocp_anode), of the bulk
electrolyte diffusivity and conductivity (eq. De_app, kappa_app), of the
theoretical capacity that defines the 1C current (eq.
theoretical-capacity-electrode, theoretical-capacity-cell,
applied-current-crate) and the parameter tables.  A small reader turns that
LaTeX into numpy expressions mechanically, so the oracle's own hand-written
forms (the cathode fit rewritten as ``amp tanh(p + q theta~)``, derivative
formulas, the capacity) are checked against an independent reading of the
printed text: a changed coefficient, a dropped term or a slip in the
rewriting fails here.  Derivatives are checked against the complex-step
derivative of the printed form (exact to rounding)."""
import os
import re

import numpy as np
import pytest

from oracle import phys as P
from p4d_inputs import phys as ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_model_parameters.txt")


def _sections():
    sec, name = {}, None
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#"):
                continue
            if line.startswith("== "):
                name = line[3:].strip()
                sec[name] = []
            elif name is not None and line.strip():
                sec[name].append(line.rstrip("\n"))
    return {k: "\n".join(v) for k, v in sec.items()}


SEC = _sections()

# printed symbols -> names of the reader's namespace
_SYMBOLS = [(r"\tilde{\theta}", " tt "), (r"\theta", " th "), (r"E_{D_e}", " ED "),
            (r"c_e", " ce "), (r"\varepsilon_{s,i}", " eps_s "), (r"c_{s,i}^{\max}", " cs_max "),
            (r"V_i", " V "), (r"\mathsf{C}", " Crate "), (r"Q_n", " Qn "), (r"Q_p", " Qp "),
            (r"\tanh", " TANH"), (r"\exp", " EXP"), (r"\min", " MIN")]


def _frac(s):
    """\\frac{A}{B} -> ((A)/(B)), innermost first, braces balanced."""
    while True:
        i = s.find(r"\frac{")
        if i < 0:
            return s
        parts, j = [], i + len(r"\frac")
        for _ in range(2):
            assert s[j] == "{", s[i:i + 40]
            depth, k = 0, j
            while True:
                depth += {"{": 1, "}": -1}.get(s[k], 0)
                if depth == 0:
                    break
                k += 1
            parts.append(s[j + 1:k])
            j = k + 1
        s = s[:i] + "((" + parts[0] + ")/(" + parts[1] + "))" + s[j:]


def latex_to_numpy(tex: str) -> str:
    s = re.sub(r"\\label\{[^}]*\}", "", tex)
    for tok in (r"\nonumber", r"\quad", r"\!", "&"):
        s = s.replace(tok, " ")
    s = s.replace("\\\\", " ").replace(r"\,", " ").replace("\n", " ")
    s = s.replace(r"\left(", "(").replace(r"\right)", ")")
    s = s.replace(r"\{", "(").replace(r"\}", ")")
    for a, b in _SYMBOLS:
        s = s.replace(a, b)
    s = s.replace(r"\times", "*")
    s = re.sub(r"10\^\{([^}]*)\}", r"10**(\1)", s)
    s = _frac(s)
    s = re.sub(r"\b([A-Za-z]\w*)\^(\d)", r"\1**\2", s)
    s = s.strip().rstrip(",.").strip()
    assert "\\" not in s and "{" not in s, s
    # implicit products: an operand (number, name, closing parenthesis)
    # followed, after a space, by a name or an opening parenthesis, or a
    # closing parenthesis directly followed by one; function names first take
    # their argument
    s = re.sub(r"(TANH|EXP|MIN)\s*\(", r"\1(", s)
    s = re.sub(r"([\w.)])\s+(?=[A-Za-z(])", r"\1*", s)
    s = re.sub(r"\)(?=[\w(])", ")*", s)
    s = s.replace("TANH", "np.tanh").replace("EXP", "np.exp").replace("MIN", "min")
    return s


def printed(name: str, **vals):
    expr = latex_to_numpy(SEC[name].split("=", 1)[1] if name.startswith("eq:theor")
                          or name.startswith("eq:appl") else SEC[name])
    ns = {"np": np, **vals}
    return eval(expr, ns)   # noqa: S307 - the fixture is a committed test file


def table(name: str) -> dict:
    return {k: float(v) for k, v in (l.split() for l in SEC[name].splitlines())}


def test_reader_on_known_forms():
    """The reader itself: fractions, implicit products, powers, exponents."""
    assert eval(latex_to_numpy(r"\frac{\theta - 0.5}{0.034}"), {"th": 0.534}) == pytest.approx(1.0)
    assert eval(latex_to_numpy(r"\frac{4}{R}\left(\frac{1}{2} - 1\right)"), {"R": 2.0}) == -1.0
    assert eval(latex_to_numpy(r"\frac{F}{3600}\,\varepsilon_{s,i}\,V_i"),
                {"F": 7200.0, "eps_s": 0.5, "V": 3.0}) == 3.0
    assert eval(latex_to_numpy(r"2 \tanh\!\left(\frac{1}{4}\right)"), {"np": np}) == \
        pytest.approx(2 * np.tanh(0.25))
    assert eval(latex_to_numpy(r"1.5 c^2 - 5.34 \times 10^{-10}"), {"np": np, "c": 2.0}) == \
        pytest.approx(6.0 - 5.34e-10)
    assert eval(latex_to_numpy("\\left(1 + c\\right)\n\\left(2\\right)"), {"np": np, "c": 1.0}) == 4.0


def _tilde(th):
    lhs, rhs = SEC["where tilde"].split("=")
    assert "tt" in latex_to_numpy(lhs)
    return eval(latex_to_numpy(rhs), {"np": np, "th": th})


def _ocp_printed(el, th):
    name = "eq:ocp_anode theta" if el == 0 else "eq:ocp_cathode theta"
    return printed(name, th=th, tt=_tilde(th))


THETA = np.linspace(0.02, 0.98, 241)


@pytest.mark.parametrize("el", [0, 1])
def test_ocp_equals_printed_fit(el):
    f = P.ocp_negative if el == 0 else P.ocp_positive
    u, _ = f(THETA)
    ref = _ocp_printed(el, THETA)
    assert np.allclose(u, ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("el", [0, 1])
def test_ocp_derivative_equals_complex_step_of_printed_fit(el):
    f = P.ocp_negative if el == 0 else P.ocp_positive
    _, du = f(THETA)
    h = 1e-30
    ref = np.imag(_ocp_printed(el, THETA + 1j * h)) / h
    assert np.allclose(du, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_ocp_physical_range_and_rest_voltage():
    """Graphite sits below 1 V and LiCoO2 near 4 V over the stoichiometries
    the cell visits; at the tables' initial concentrations the open-circuit
    cell voltage U_p - U_n is the usual LiCoO2/graphite 3.8-3.9 V."""
    neg, pos = ph.NEGATIVE, ph.POSITIVE
    un = _ocp_printed(0, np.linspace(0.05, 0.95, 19))
    up = _ocp_printed(1, np.linspace(0.45, 0.95, 11))
    assert np.all((un > 0.0) & (un < 1.0)) and np.all((up > 3.5) & (up < 4.5))
    v0 = _ocp_printed(1, pos.cs0 / pos.cs_max) - _ocp_printed(0, neg.cs0 / neg.cs_max)
    assert 3.8 < v0 < 3.9
    assert P.ocp_positive(pos.cs0 / pos.cs_max)[0] - P.ocp_negative(neg.cs0 / neg.cs_max)[0] == \
        pytest.approx(v0, rel=1e-14)


CE = np.linspace(50.0, 3000.0, 119)


def test_transport_functions_equal_printed_forms_at_reference_temperature():
    """kappa(c_e, T) and D_e(c_e, T) at the tables' temperature (the oracle
    drops the Arrhenius factors, which are exactly 1 there)."""
    T = table("tab:constants")["T"]
    R = table("tab:constants")["R"]
    ed = float(SEC["where E_De"].split("=")[1])
    c = eval(latex_to_numpy(SEC["where c"].split("=")[1]), {"np": np, "ce": CE})
    kap = printed("eq:kappa_app c_e T", ce=CE, c=c, T=T, R=R)
    de = printed("eq:De_app c_e T", ce=CE, T=T, R=R, ED=ed)
    assert np.allclose(P.kappa_bulk(CE), kap, rtol=1e-14, atol=0)
    assert np.allclose(P.de_bulk(CE), de, rtol=1e-14, atol=0)
    # away from that temperature the factors differ from 1 (the reader
    # really evaluates them)
    assert printed("eq:kappa_app c_e T", ce=1000.0, c=1.0, T=310.0, R=R) > \
        printed("eq:kappa_app c_e T", ce=1000.0, c=1.0, T=T, R=R)


def test_transport_derivatives_equal_complex_step():
    T, R = table("tab:constants")["T"], table("tab:constants")["R"]
    ed = float(SEC["where E_De"].split("=")[1])
    h = 1e-30
    z = CE + 1j * h
    kap = printed("eq:kappa_app c_e T", ce=z, c=z / 1000.0, T=T, R=R)
    de = printed("eq:De_app c_e T", ce=z, T=T, R=R, ED=ed)
    assert np.allclose(P.dkappa_bulk(CE), np.imag(kap) / h, rtol=1e-12, atol=0)
    assert np.allclose(P.dde_bulk(CE), np.imag(de) / h, rtol=1e-12, atol=0)


def test_parameter_tables():
    """The case data used by the oracle and the library equals the printed
    tables."""
    cst = table("tab:constants")
    assert (ph.F, ph.R_GAS, ph.T_REF) == (cst["F"], cst["R"], cst["T"])
    el = table("tab:electrolyte")
    assert (ph.CE0, ph.T_PLUS, ph.BRUGGEMAN) == (el["c_e0"], el["t_plus"], el["bruggeman"])
    for e, name in ((ph.NEGATIVE, "tab:anode"), (ph.POSITIVE, "tab:cathode")):
        t = table(name)
        for k, v in t.items():
            assert getattr(e, k) == v, (name, k)
    assert ph.SEPARATOR_EPS == table("tab:separator")["eps"]


@pytest.mark.parametrize("n", [19, 28])
def test_one_c_current_is_the_theoretical_capacity(n):
    """I_app = C min(Q_n, Q_p), Q_i = F/3600 eps_s,i V_i c_s,max,i with the
    electrode volumes of the cube (225 um square, 100 um thick); the
    negative electrode limits (Q_n < Q_p, as the appendix notes).  The
    oracle returns it with the discharge sign (current leaving the top
    face)."""
    case = ph.PhysCase(n=n, nr=(6, 6))
    F = table("tab:constants")["F"]
    V = 225e-6 * 225e-6 * 100e-6
    q = [printed("eq:theoretical-capacity-electrode", F=F, V=V, eps_s=t["eps_s"], cs_max=t["cs_max"])
         for t in (table("tab:anode"), table("tab:cathode"))]
    assert q[0] < q[1]
    Q = printed("eq:theoretical-capacity-cell", Qn=q[0], Qp=q[1])
    assert Q == q[0]
    I = printed("eq:applied-current-crate", Crate=1.0, Q=Q)
    assert case.electrode_volume == pytest.approx(V, rel=1e-15)
    assert P.applied_current(case) == pytest.approx(-I, rel=1e-14)
    assert I == pytest.approx(2.035e-6, rel=1e-3)
