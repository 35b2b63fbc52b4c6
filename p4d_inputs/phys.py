"""Physical parameters and geometry of the paper's homogeneous cube cell
(Case I, Sec. 5; parameter tables of the appendix).  Data only: no step of
the method is computed here (kinetics, open-circuit potentials, transport
functions and the residual are written separately by the oracle and the GPU
library).

Case II (Sec. 5) keeps the geometry and draws the active-material and
binder volume fractions per element from filtered Gaussian random fields
with the table of prescribed means and variances; the porosity is what
remains, and the current enters uniformly through the top face.

Geometry: a cube of edge 225 um along x, y and z; the negative electrode
(graphite) occupies z in [0, 100 um], the separator (100, 125) and the
positive electrode (LiCoO2) [125, 225].  The node grid is n x n x n with
n - 1 a multiple of 9 (at least 18), so that every layer boundary falls on
element faces: 25 um is (n - 1) / 9 elements.  phi_s = 0 on the bottom face (the negative
collector); the applied current enters through the top face.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

# universal constants (table "Universal physical constants")
F = 96485.33       # C / mol
R_GAS = 8.31446    # J / (mol K)
T_REF = 298.15     # K

# electrolyte (table "Electrolyte parameters")
CE0 = 1000.0       # mol / m^3
T_PLUS = 0.4
BRUGGEMAN = 1.5


@dataclass(frozen=True)
class Electrode:
    eps_s: float       # active material volume fraction
    eps: float         # porosity
    sigma: float       # solid conductivity, S/m
    k: float           # reaction rate constant, A/m^2 (m^3/mol)^1.5
    alpha: float       # charge-transfer coefficients (anodic = cathodic)
    cs_max: float      # mol / m^3
    cs0: float         # initial solid concentration, mol / m^3
    a: float           # specific interfacial area, 1/m
    Ds: float          # solid diffusivity, m^2/s
    Rs: float          # particle radius, m


# tables "Anode (negative electrode) parameters" and "Cathode (positive
# electrode) parameters"
NEGATIVE = Electrode(eps_s=0.6, eps=0.3, sigma=100.0, k=2e-5, alpha=0.5, cs_max=2.50e4,
                     cs0=2.00e4, a=1.8e5, Ds=3.9e-14, Rs=1.0e-5)
POSITIVE = Electrode(eps_s=0.5, eps=0.3, sigma=10.0, k=6e-7, alpha=0.5, cs_max=5.12e4,
                     cs0=3.07e4, a=1.5e5, Ds=1.0e-13, Rs=1.0e-5)
SEPARATOR_EPS = 1.0

# table "Prescribed mean and variance values for volume fractions of solid
# components" (Case II): (mean, variance) per electrode (negative, positive)
FRACTION_STATS = {"active": ((0.60, 0.004), (0.50, 0.004)),
                  "binder": ((0.10, 0.0001), (0.20, 0.0001))}

CELL_EDGE = 225e-6                                 # m
LAYERS_UM = (100.0, 25.0, 100.0)                   # negative, separator, positive


@dataclass
class PhysCase:
    """The cube cell on an n^3 node grid with N_r radial points per particle."""
    n: int
    nr: Tuple[int, int]
    dt: float = 60.0                   # s (one minute, Sec. 5)
    c_rate: float = 1.0
    theta_bar: Tuple[float, float] = (0.5, 0.5)
    gauss_frac: float = 0.1            # spread of the applied current / collector edge
    electrodes: Tuple[Electrode, Electrode] = field(default_factory=lambda: (NEGATIVE, POSITIVE))
    # Case II: active-material and binder volume fractions per element
    # (element-id order; separator entries unused), and the current profile
    # on the top face ("gauss" or "uniform")
    eps_s_e: Optional[np.ndarray] = None
    eps_b_e: Optional[np.ndarray] = None
    profile: str = "gauss"

    def __post_init__(self):
        if (self.n - 1) % 9 != 0 or self.n < 19:
            raise ValueError("n - 1 must be a multiple of 9, at least 18 (two elements per 25 um)")
        if self.profile not in ("gauss", "uniform"):
            raise ValueError("profile is 'gauss' or 'uniform'")
        if (self.eps_s_e is None) != (self.eps_b_e is None):
            raise ValueError("give both volume-fraction fields or neither")

    @property
    def heterogeneous(self) -> bool:
        return self.eps_s_e is not None

    # node layers: elements kk with kk + 1 < na are negative-electrode
    # elements, kk >= na + ns positive ones (the library's convention)
    @property
    def elems_25um(self) -> int:
        return (self.n - 1) // 9

    @property
    def na(self) -> int:
        return 4 * self.elems_25um + 1

    @property
    def ns(self) -> int:
        return self.elems_25um - 1

    @property
    def nz(self) -> int:
        return self.n

    @property
    def h(self) -> float:
        return CELL_EDGE / (self.n - 1)

    @property
    def electrode_volume(self) -> float:
        return CELL_EDGE * CELL_EDGE * LAYERS_UM[0] * 1e-6


def case_desc(case: PhysCase) -> dict:
    """Fields of the problem description that are plain data of the case:
    grid, radial sizes, time step, porosities and the cell edge."""
    return dict(nx=case.n, ny=case.n, nz=case.n, na=case.na, ns=case.ns, nr=tuple(case.nr),
                theta_bar=tuple(case.theta_bar), dt=case.dt,
                eps_elec=case.electrodes[0].eps, eps_sep=SEPARATOR_EPS, length=CELL_EDGE)


def element_layers(case: PhysCase) -> np.ndarray:
    """Material per element (0 negative, 1 positive, -1 separator), element
    ids x fastest."""
    n = case.n
    kk = np.repeat(np.arange(n - 1), (n - 1) ** 2)
    return np.where(kk + 1 < case.na, 0, np.where(kk >= case.na + case.ns, 1, -1))


def case2(n: int, nr: Tuple[int, int], seed: int = 2, corr_um: float = 25.0, **kw) -> PhysCase:
    """Case II: the cube with volume fractions from two independent filtered
    Gaussian random fields (active material, binder), each standardized over
    the domain and mapped per electrode to the prescribed mean and variance:
    eps_i = mean_i + sqrt(var_i) G_i.  The correlation length (the filter's
    h_c) is corr_um micrometres, the separator thickness by default.  Draw
    order: G_active, then G_binder, from PCG64(seed)."""
    from . import grf
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = (n - 1, n - 1, n - 1)
    hc = corr_um * 1e-6 / (CELL_EDGE / (n - 1))
    g_act = grf(rng, cells, hc)
    g_bin = grf(rng, cells, hc)
    probe = PhysCase(n=n, nr=nr)
    lay = element_layers(probe)
    fs, fb = np.zeros(g_act.size), np.zeros(g_act.size)
    for el in (0, 1):
        (ms, vs), (mb, vb) = FRACTION_STATS["active"][el], FRACTION_STATS["binder"][el]
        sel = lay == el
        fs[sel] = ms + np.sqrt(vs) * g_act[sel]
        fb[sel] = mb + np.sqrt(vb) * g_bin[sel]
    elec = lay >= 0
    por = 1.0 - fs - fb
    if np.any(fs[elec] <= 0) or np.any(fb[elec] <= 0) or np.any(por[elec] <= 0):
        raise ValueError("a volume fraction left (0, 1); draw another seed")
    return PhysCase(n=n, nr=nr, eps_s_e=fs, eps_b_e=fb, profile="uniform", **kw)


def porosity(case: PhysCase) -> np.ndarray:
    """Porosity per element: 1 - eps_s - eps_b in the electrodes (Case II) or
    the table value, and the separator's."""
    lay = element_layers(case)
    if case.heterogeneous:
        por = 1.0 - case.eps_s_e - case.eps_b_e
    else:
        por = np.full(lay.size, case.electrodes[0].eps)
    return np.where(lay >= 0, por, SEPARATOR_EPS)


def active_fraction(case: PhysCase) -> np.ndarray:
    """Active-material volume fraction per element (zero in the separator)."""
    lay = element_layers(case)
    if case.heterogeneous:
        return np.where(lay >= 0, case.eps_s_e, 0.0)
    return np.where(lay == 0, case.electrodes[0].eps_s,
                    np.where(lay == 1, case.electrodes[1].eps_s, 0.0))
