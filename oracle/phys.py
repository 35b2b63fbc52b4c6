"""Physical P4D-DFN model around the linear oracle: the nonlinear residual of
one backward-Euler step, its linearization and Newton steps, for the cube
cell of the paper (Sec. 2 model, Sec. 3 discretization, Sec. 5 Case I,
appendix parameter tables).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.
Plain numpy loops over nodes and elements; the linear algebra is the C
oracle (pinned separately).

Parity status: the material functions (open-circuit potentials, bulk
conductivity and diffusivity, their derivatives) and the 1C current are
pinned against the appendix's printed formulas and tables read by a separate
LaTeX reader (tests/test_oracle_appendix.py); the residual and Newton matrix
against central differences, the rest state, charge balance and lithium
conservation (tests/test_oracle_phys.py).

Readings (each also listed in the design notes):
  - the transport coefficients of an element are evaluated at the mean of
    its eight nodal c_e (kappa_eff, D_e_eff and the diffusion-potential
    factor kappa_eff 2RT(1 - t+) / (F c_e));
  - the Newton matrix is the exact Jacobian: besides the transport
    coefficients at the iterate and the kinetics derivatives it holds the
    derivative of each element's coefficients with respect to its mean c_e,
    applied to the state (rank-one terms per element); the preconditioner
    is built without those terms;
  - the reaction is lumped per node (weight m_j), as in the linear model;
  - the applied current enters through the top face with the paper's
    Gaussian profile, lumped per face node and normalized so that the nodal
    currents sum to the applied current; a discharge (lithium leaving the
    negative particles) has the current leave through the top face;
  - temperature 298.15 K, so the Arrhenius factors of kappa and D_e are 1;
  - Case II: the volume fractions vary per element; sigma_eff takes the
    local active fraction and kappa_eff, D_e_eff and the c_e storage the
    local porosity (Bruggeman), while the specific area a keeps its table
    value (the tables give it as a constant) and the 1C current uses the
    mean fractions; the current enters uniformly through the top face.
"""
from __future__ import annotations

import numpy as np

import p4d_inputs as pi
from p4d_inputs import phys as ph

from . import Oracle, PC_SCHUR

FRT = ph.F / (ph.R_GAS * ph.T_REF)


# ---------------------------------------------------------------------------
# material functions (appendix): open-circuit potentials and electrolyte
# transport, with their derivatives
# ---------------------------------------------------------------------------
def ocp_negative(theta):
    """Graphite open-circuit potential and its derivative in theta."""
    t = np.asarray(theta, dtype=float)
    terms = [(0.0351, 0.286, 0.083), (-0.0045, 0.849, 0.119), (-0.035, 0.9233, 0.05),
             (-0.0147, 0.5, 0.034), (-0.102, 0.194, 0.142), (-0.022, 0.9, 0.0164),
             (-0.011, 0.124, 0.0226), (0.0155, 0.105, 0.029)]
    u = 0.194 + 1.5 * np.exp(-120.0 * t)
    du = -180.0 * np.exp(-120.0 * t)
    for amp, c, w in terms:
        th = np.tanh((t - c) / w)
        u = u + amp * th
        du = du + amp * (1.0 - th * th) / w
    return u, du


def ocp_positive(theta):
    """LiCoO2 open-circuit potential (of 1.062 theta) and its derivative in
    theta."""
    t = 1.062 * np.asarray(theta, dtype=float)
    # amp * tanh(p + q t)
    terms = [(0.07645, 30.834, -54.4806), (2.1581, 52.294, -50.294),
             (-0.14169, 11.0923, -19.8543), (0.2051, 1.4684, -5.4888),
             (0.2531, 0.56478 / 0.1316, -1.0 / 0.1316), (-0.02167, -0.525 / 0.006, 1.0 / 0.006)]
    u = 2.16216 + 0.0 * t
    du = 0.0 * t
    for amp, p, q in terms:
        th = np.tanh(p + q * t)
        u = u + amp * th
        du = du + amp * q * (1.0 - th * th)
    return u, 1.062 * du


def kappa_bulk(ce):
    c = np.asarray(ce, dtype=float) / 1000.0
    return 0.0911 + 1.9101 * c - 1.052 * c * c + 0.1554 * c * c * c


def dkappa_bulk(ce):
    """d kappa / d c_e (S/m per mol/m^3)."""
    c = np.asarray(ce, dtype=float) / 1000.0
    return (1.9101 - 2.0 * 1.052 * c + 3.0 * 0.1554 * c * c) / 1000.0


def de_bulk(ce):
    return 5.34e-10 * np.exp(-0.65 * np.asarray(ce, dtype=float) / 1000.0)


def dde_bulk(ce):
    return -0.65 / 1000.0 * de_bulk(ce)


OCP = (ocp_negative, ocp_positive)


# ---------------------------------------------------------------------------
# grid bookkeeping
# ---------------------------------------------------------------------------
class Grid:
    def __init__(self, case: ph.PhysCase):
        self.case = case
        n = case.n
        self.nx = self.ny = self.nz = n
        self.na, self.ns = case.na, case.ns
        self.nc = n - case.na - case.ns
        self.layer = n * n
        self.nnode = n ** 3
        self.nelem = (n - 1) ** 3
        self.nea = self.layer * self.na
        self.nec = self.layer * self.nc
        self.ne = self.nea + self.nec
        self.off_pe = self.ne
        self.off_ce = self.ne + self.nnode
        self.off_cs = (self.off_ce + self.nnode, self.off_ce + self.nnode + case.nr[0] * self.nea)
        self.N = self.off_cs[1] + case.nr[1] * self.nec
        # electrode node -> global node id, electrode index
        k = np.repeat(np.arange(n), self.layer)
        ids = np.arange(self.nnode)
        self.enode = np.concatenate([ids[k < self.na], ids[k >= self.na + self.ns]])
        self.eel = np.concatenate([np.zeros(self.nea, int), np.ones(self.nec, int)])
        self.ek = k[self.enode]
        # element material per element: 0, 1, or -1 (separator)
        kk = np.repeat(np.arange(n - 1), (n - 1) ** 2)
        self.emat = np.where(kk + 1 < self.na, 0, np.where(kk >= self.na + self.ns, 1, -1))
        # corner node ids of every element
        ei, ej, ek = np.meshgrid(np.arange(n - 1), np.arange(n - 1), np.arange(n - 1), indexing="ij")
        ei, ej, ek = (a.transpose(2, 1, 0).reshape(-1) for a in (ei, ej, ek))
        corners = []
        for b in range(8):
            corners.append((ei + (b & 1)) + n * ((ej + ((b >> 1) & 1)) + n * (ek + ((b >> 2) & 1))))
        self.corners = np.stack(corners, axis=1)

    def surface(self, u, el):
        """c_s at the particle surface of the electrode's nodes."""
        nn = self.nea if el == 0 else self.nec
        N = self.case.nr[el]
        return u[self.off_cs[el] + (N - 1) * nn: self.off_cs[el] + N * nn]


# ---------------------------------------------------------------------------
# case data derived from the tables
# ---------------------------------------------------------------------------
def applied_current(case: ph.PhysCase) -> float:
    """1C current of the cell (A): Q_i = F / 3600 eps_s,i V_i c_s,max,i (Ah),
    Q = min(Q_n, Q_p), I = C Q; negative = discharge (current leaves through
    the top face)."""
    q = [ph.F / 3600.0 * el.eps_s * case.electrode_volume * el.cs_max for el in case.electrodes]
    return -case.c_rate * min(q)


def face_source(case: ph.PhysCase, grid: Grid, current: float) -> np.ndarray:
    """Nodal currents on the top face (phi_s rows of the positive electrode):
    the Gaussian profile of Sec. 5 centred on the face with spreads
    gauss_frac * edge (or a uniform one, Case II), lumped (face weight per
    node) and normalized to sum to `current`."""
    n, h = case.n, case.h
    L = ph.CELL_EDGE
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    sx = sy = case.gauss_frac * L
    G = np.exp(-(X - L / 2) ** 2 / (2 * sx * sx) - (Y - L / 2) ** 2 / (2 * sy * sy))
    if case.profile == "uniform":
        G = np.ones_like(G)
    w1 = np.full(n, h)
    w1[0] = w1[-1] = h / 2
    W = np.outer(w1, w1)
    gw = (G * W).reshape(-1)
    f = np.zeros(grid.ne)
    top = grid.ne - grid.layer     # last layer of the positive electrode
    f[top:] = current * gw / gw.sum()
    return f


def initial_state(case: ph.PhysCase, grid: Grid) -> np.ndarray:
    """Rest state: c_e = c_e0, c_s = c_s0, zero overpotential everywhere
    (phi_s = 0 in the negative electrode, phi_e = -U_n, phi_s = U_p - U_n in
    the positive electrode)."""
    u = np.zeros(grid.N)
    neg, pos = case.electrodes
    un, _ = ocp_negative(neg.cs0 / neg.cs_max)
    up, _ = ocp_positive(pos.cs0 / pos.cs_max)
    u[: grid.nea] = 0.0
    u[grid.nea: grid.ne] = up - un
    u[grid.off_pe: grid.off_ce] = -un
    u[grid.off_ce: grid.off_ce + grid.nnode] = ph.CE0
    u[grid.off_cs[0]: grid.off_cs[1]] = neg.cs0
    u[grid.off_cs[1]:] = pos.cs0
    return u


# ---------------------------------------------------------------------------
# coefficients of one state
# ---------------------------------------------------------------------------
def element_coefficients(case, grid, u, derivatives=False):
    """sigma_eff, kappa_eff, the diffusion-potential coefficient and D_e_eff
    per element, at the element-mean c_e (and, with derivatives, the
    derivatives of the last three with respect to that mean)."""
    ce = u[grid.off_ce: grid.off_ce + grid.nnode]
    cbar = ce[grid.corners].mean(axis=1)
    eps = ph.porosity(case)
    act = ph.active_fraction(case)
    sig = np.zeros(grid.nelem)
    for el in range(2):
        sel = grid.emat == el
        sig[sel] = act[sel] ** ph.BRUGGEMAN * case.electrodes[el].sigma
    kap = eps ** ph.BRUGGEMAN * kappa_bulk(cbar)
    kd = kap * 2.0 * (1.0 - ph.T_PLUS) / (FRT * cbar)
    dce = eps ** ph.BRUGGEMAN * de_bulk(cbar)
    if not derivatives:
        return sig, kap, kd, dce
    dkap = eps ** ph.BRUGGEMAN * dkappa_bulk(cbar)
    dkd = 2.0 * (1.0 - ph.T_PLUS) / FRT * (dkap * cbar - kap) / (cbar * cbar)
    ddce = eps ** ph.BRUGGEMAN * dde_bulk(cbar)
    return sig, kap, kd, dce, (dkap, dkd, ddce)


def kinetics(case, grid, u):
    """Per electrode node: the volumetric reaction q = a i_n and its
    derivatives (a di/d phi_s, a di/d c_e, a di/d c_s,surf)."""
    q = np.zeros(grid.ne)
    g = np.zeros(grid.ne)
    e = np.zeros(grid.ne)
    s = np.zeros(grid.ne)
    ce = u[grid.off_ce: grid.off_ce + grid.nnode]
    for el in range(2):
        sl = slice(0, grid.nea) if el == 0 else slice(grid.nea, grid.ne)
        prm = case.electrodes[el]
        nodes = grid.enode[sl]
        phis = u[sl]
        phie = u[grid.off_pe + nodes]
        cen = ce[nodes]
        css = grid.surface(u, el)
        U, dU = OCP[el](css / prm.cs_max)
        eta = phis - phie - U
        al = prm.alpha
        i0 = prm.k * cen ** al * (prm.cs_max - css) ** al * css ** al
        ea, ec = np.exp(al * FRT * eta), np.exp(-al * FRT * eta)
        i_n = i0 * (ea - ec)
        i_eta = i0 * al * FRT * (ea + ec)
        i_ce = al * i_n / cen
        i_cs = i_n * (-al / (prm.cs_max - css) + al / css) - i_eta * dU / prm.cs_max
        q[sl] = prm.a * i_n
        g[sl] = prm.a * i_eta
        e[sl] = prm.a * i_ce
        s[sl] = prm.a * i_cs
    return q, g, e, s


def linear_problem(case, grid, u, with_kinetics=True, exact=None) -> pi.Problem:
    """The Newton matrix at u as a linear-operator description: transport
    coefficients at u, kinetics derivatives (or zero) and, when exact (by
    default with the kinetics), the c_e-derivative terms of the transport
    coefficients applied to the state."""
    exact = with_kinetics if exact is None else exact
    sig, kap, kd, dce, der = element_coefficients(case, grid, u, derivatives=True)
    if with_kinetics:
        _, g, e, s = kinetics(case, grid, u)
    else:
        g = e = s = np.zeros(grid.ne)
    neg, pos = case.electrodes
    d = ph.case_desc(case)
    return pi.Problem(
        nx=d["nx"], ny=d["ny"], nz=d["nz"], na=d["na"], ns=d["ns"], nr=d["nr"],
        Ds=(neg.Ds / neg.Rs ** 2, pos.Ds / pos.Rs ** 2), theta_bar=d["theta_bar"], dt=d["dt"],
        chi=0.0, tc=(1.0 - ph.T_PLUS) / ph.F, lambda_c=1.0, eps_elec=d["eps_elec"],
        eps_sep=d["eps_sep"], sigma=sig, kappa=kap, g=g, s=s, e=e, b=np.zeros(grid.N),
        length=d["length"], lambda_el=(1.0 / (ph.F * neg.Rs * neg.a), 1.0 / (ph.F * pos.Rs * pos.a)),
        kappa_d=kd, dce=dce, eps_e=ph.porosity(case) if case.heterogeneous else None,
        newton=(u[grid.off_pe: grid.off_ce].copy(), u[grid.off_ce: grid.off_cs[0]].copy()) + der
        if exact else None,
        name="phys")


# ---------------------------------------------------------------------------
# residual of one backward-Euler step
# ---------------------------------------------------------------------------
def residual(case, grid, u, u_old, current):
    """R(u) for the step from u_old: the transport operator at u (diffusion,
    storage and radial rows) applied to u, minus the previous-step storage,
    plus the lumped reaction (phi_s +m q, phi_e -m q, c_e -(1-t+)/F m q,
    surface c_s +Gamma q) and minus the applied current."""
    lp = linear_problem(case, grid, u, with_kinetics=False)
    orc = Oracle(lp)
    R = orc.apply(u)
    # previous-step storage: M_eps c_e_old / dt (operator with the transport
    # coefficients set to zero) and c_s_old / dt
    lp0 = lp.with_(kappa=np.zeros(grid.nelem), kappa_d=np.zeros(grid.nelem),
                   dce=np.zeros(grid.nelem), sigma=np.zeros(grid.nelem))
    xold = np.zeros(grid.N)
    xold[grid.off_ce: grid.off_ce + grid.nnode] = u_old[grid.off_ce: grid.off_ce + grid.nnode]
    R[grid.off_ce: grid.off_ce + grid.nnode] -= Oracle(lp0).apply(xold)[grid.off_ce: grid.off_ce + grid.nnode]
    R[grid.off_cs[0]:] -= u_old[grid.off_cs[0]:] / case.dt
    q, _, _, _ = kinetics(case, grid, u)
    m = orc.lumped_weights()
    dirn = grid.ek == 0
    R[: grid.ne] += np.where(dirn, 0.0, m * q)
    R[grid.off_pe + grid.enode] -= m * q
    R[grid.off_ce + grid.enode] -= lp.tc * m * q
    for el in range(2):
        nn = grid.nea if el == 0 else grid.nec
        N = case.nr[el]
        sl = slice(0, grid.nea) if el == 0 else slice(grid.nea, grid.ne)
        gam = orc.radial(el)[4]
        R[grid.off_cs[el] + (N - 1) * nn: grid.off_cs[el] + N * nn] += gam * q[sl]
    R[: grid.ne] -= face_source(case, grid, current)
    return R


SCALES = (ph.R_GAS * ph.T_REF / ph.F, ph.R_GAS * ph.T_REF / ph.F, ph.CE0, None)


# ---------------------------------------------------------------------------
# scaling of the Newton system
# ---------------------------------------------------------------------------
class Scaling:
    """Per-field unknown scales (x: RT/F for both potentials, c_e0, the mean
    c_s,max for c_s) and equation scales (r: the inverse diagonal magnitude
    of the phi_e, c_e and c_s rows at the rest state, with the phi_s rows
    sharing the phi_e scale), so that D_r J D_c has O(1) blocks.  In SI
    units the blocks differ by ten orders of magnitude and FGMRES on the 2-norm
    of the unscaled residual stagnates.  The scaled matrix is again an
    operator of the same family, with scaled coefficients."""

    def __init__(self, case: ph.PhysCase):
        h, dt = case.h, case.dt
        eps = case.electrodes[0].eps
        self.x_phi = ph.R_GAS * ph.T_REF / ph.F
        self.x_c = ph.CE0
        self.x_s = 0.5 * (case.electrodes[0].cs_max + case.electrodes[1].cs_max)
        kap0 = eps ** ph.BRUGGEMAN * float(kappa_bulk(ph.CE0))
        d0 = eps ** ph.BRUGGEMAN * float(de_bulk(ph.CE0))
        self.r_phi = 1.0 / (kap0 * h * self.x_phi)
        self.r_c = 1.0 / ((eps * h ** 3 / dt + d0 * h) * self.x_c)
        self.r_s = dt / self.x_s

    def problem(self, lp: pi.Problem) -> pi.Problem:
        """D_r A D_c for the operator lp: every coefficient takes its row and
        column scale (the storage of c_e also the change of time step that
        carries the c_s row scale)."""
        rp, rc, rs = self.r_phi, self.r_c, self.r_s
        xp, xc, xs = self.x_phi, self.x_c, self.x_s
        tfac = rs * xs            # dt' = dt / tfac, Ds' = Ds * tfac
        return lp.with_(sigma=rp * xp * lp.sigma, kappa=rp * xp * lp.kappa,
                        kappa_d=rp * xc * lp.kappa_d, dce=rc * xc * lp.dce,
                        eps_elec=rc * xc * lp.eps_elec / tfac, eps_sep=rc * xc * lp.eps_sep / tfac,
                        eps_e=None if lp.eps_e is None else rc * xc * lp.eps_e / tfac,
                        newton=None if lp.newton is None else
                        lp.newton[:2] + (rp * xc * lp.newton[2], rp * xc * lp.newton[3],
                                         rc * xc * lp.newton[4]),
                        g=rp * xp * lp.g, e=rp * xc * lp.e, s=rp * xs * lp.s,
                        tc=lp.tc * rc / rp, lambda_el=tuple(l * rs / rp for l in lp.lambda_el),
                        dt=lp.dt / tfac, Ds=tuple(d * tfac for d in lp.Ds))

    def rows(self, grid, R):
        """D_r R (the grounded phi_s rows take 1 / x_phi: they are identity rows)."""
        out = R.copy()
        out[: grid.off_ce] *= self.r_phi
        out[: grid.layer] = R[: grid.layer] / self.x_phi
        out[grid.off_ce: grid.off_cs[0]] *= self.r_c
        out[grid.off_cs[0]:] *= self.r_s
        return out

    def cols(self, grid, x):
        """D_c x."""
        out = x.copy()
        out[: grid.off_ce] *= self.x_phi
        out[grid.off_ce: grid.off_cs[0]] *= self.x_c
        out[grid.off_cs[0]:] *= self.x_s
        return out


def scaled_update(case, grid, du):
    """max over the fields of |du| / field scale (RT/F for the potentials,
    c_e0 for c_e, c_s,max per electrode for c_s)."""
    out = max(np.abs(du[: grid.off_pe]).max(), np.abs(du[grid.off_pe: grid.off_ce]).max()) / SCALES[0]
    out = max(out, np.abs(du[grid.off_ce: grid.off_cs[0]]).max() / ph.CE0)
    for el in range(2):
        hi = grid.off_cs[1] if el == 0 else grid.N
        out = max(out, np.abs(du[grid.off_cs[el]: hi]).max() / case.electrodes[el].cs_max)
    return out


def newton_step(case, grid, u_old, current, tol=1e-9, maxit=30, lin_rtol=1e-10, coarse_max=512):
    """One backward-Euler step by Newton iterations from u_old: each solves
    the scaled system (D_r J D_c) dx = -D_r R with the oracle's FGMRES
    (Schur preconditioner), du = D_c dx; stops when the scaled update falls
    below tol.  Returns (u, list of (scaled update, linear iterations))."""
    sc = Scaling(case)
    u = u_old.copy()
    hist = []
    for _ in range(maxit):
        R = residual(case, grid, u, u_old, current)
        lp = sc.problem(linear_problem(case, grid, u))
        orc = Oracle(lp).setup(pc=PC_SCHUR, rtol=lin_rtol, coarse_max=coarse_max, maxit=3000)
        dx, info = orc.solve(-sc.rows(grid, R))
        du = sc.cols(grid, dx)
        u = u + du
        hist.append((scaled_update(case, grid, du), info.iters))
        if hist[-1][0] <= tol:
            break
    return u, hist
