"""Seeded synthetic inputs for the linearized pseudo-4D DFN Jacobian solve.

This module is shared by the CPU oracle and the GPU path, so it holds only
input generation: mesh sizes and layer split, coefficient fields, linearized
Butler-Volmer derivatives, right-hand sides and functional weights.  None of
the method's arithmetic (operator, preconditioner, Krylov) lives here.

Problem definition (all quantities nondimensional):

* Structured node grid ``nx x ny x nz`` with isotropic spacing
  ``h = 1/(nz-1)``; node id ``i + nx*(j + ny*k)``.  Layers along ``k``:
  anode ``k < na``, separator ``na <= k < na+ns``, cathode above
  (the cell stack of the paper's Case I, Section 5.1).
* Element ``(i,j,k)`` spans node layers ``k..k+1``; it belongs to an electrode
  only if both of its node layers do, otherwise to the separator.
* ``sigma`` (solid conductivity, used on electrode elements) and ``kappa``
  (electrolyte conductivity, all elements), one value per element, element id
  ``i + (nx-1)*(j + (ny-1)*k)``.  Uniform 1 or lognormal
  ``exp(sigma_log * G)`` with ``G`` a filtered Gaussian random field built as
  in the paper's Case II (coarse Gaussian samples, trilinear interpolation, a
  reaction-diffusion filter ``(I - h_c^2 Lap) g~ = g``), here normalized to
  mean 0 and variance 1.
* ``g, s, e``: per electrode node, derivatives of the reaction term
  ``a*i_n`` (Butler-Volmer, Section 2.4) with respect to the overpotential,
  the particle surface concentration and the electrolyte concentration.
  ``g, s ~ U(0.5, 2)``; ``e = sign * 0.1 * U(0.5, 2)`` with sign +1 in the
  anode and -1 in the cathode.
* Particle radius 1 after scaling by ``R_s = 1e-5 m`` (Tables of the model
  parameters appendix); ``Ds_hat = D_s * dt / R_s^2``.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

R_S = 1.0e-5          # particle radius [m], both electrodes (parameter tables)
T_PLUS = 0.4          # cation transference number (electrolyte table)


def layer_split(nz: int) -> Tuple[int, int, int]:
    """Anode / separator / cathode node layers for ``nz`` layers.

    Electrodes get ``round(5*nz/12)`` layers each (the 100/25/100 um stack of
    Case I, i.e. 5:1:... with the separator the remainder)."""
    na = int(np.floor(5.0 * nz / 12.0 + 0.5))
    ns = nz - 2 * na
    if na < 2 or ns < 1:
        raise ValueError(f"nz={nz} too small for an anode/separator/cathode split")
    return na, ns, na


@dataclass
class Problem:
    """One linearized P4D Jacobian instance (see module docstring)."""
    nx: int
    ny: int
    nz: int
    na: int
    ns: int
    nr: Tuple[int, int]
    Ds: Tuple[float, float]            # nondimensional particle diffusivity
    theta_bar: Tuple[float, float] = (0.5, 0.5)
    dt: float = 1.0
    chi: float = 2.0 * (1.0 - T_PLUS)  # diffusion-potential factor
    tc: float = 1.0 - T_PLUS           # electrolyte source factor
    lambda_c: float = 1.0              # surface coupling scale
    eps_elec: float = 0.3              # porosity in electrode elements
    eps_sep: float = 1.0               # porosity in separator elements
    sigma: Optional[np.ndarray] = None  # (n_elem,)
    kappa: Optional[np.ndarray] = None  # (n_elem,)
    g: Optional[np.ndarray] = None      # (n_e,)
    s: Optional[np.ndarray] = None
    e: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None      # (N,)
    name: str = ""
    # cell edge along z (0: 1, i.e. nondimensional), surface coupling scale
    # per electrode (0: lambda_c), and element coefficients of the
    # diffusion-potential block and the c_e diffusion (None: chi * kappa,
    # kappa); porosity per element for the c_e storage (None: eps_elec,
    # eps_sep by material)
    length: float = 0.0
    lambda_el: Tuple[float, float] = (0.0, 0.0)
    kappa_d: Optional[np.ndarray] = None  # (n_elem,)
    dce: Optional[np.ndarray] = None      # (n_elem,)
    eps_e: Optional[np.ndarray] = None    # (n_elem,)
    # element edges along x and y (0: h, the edge along z)
    hxy: Tuple[float, float] = (0.0, 0.0)
    # Newton terms of a state (phi_e, c_e per node; per element the c_e-
    # derivatives of kappa_eff, the diffusion-potential coefficient, D_eff)
    newton: Optional[Tuple[np.ndarray, ...]] = None

    # ---- sizes -----------------------------------------------------------
    @property
    def nc(self) -> int:
        return self.nz - self.na - self.ns

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_elem(self) -> int:
        return (self.nx - 1) * (self.ny - 1) * (self.nz - 1)

    @property
    def n_ea(self) -> int:
        return self.nx * self.ny * self.na

    @property
    def n_ec(self) -> int:
        return self.nx * self.ny * self.nc

    @property
    def n_e(self) -> int:
        return self.n_ea + self.n_ec

    @property
    def offsets(self) -> Tuple[int, int, int, int, int, int]:
        """(phi_s, phi_e, c_e, c_s anode, c_s cathode, N)."""
        o_ps = 0
        o_pe = self.n_e
        o_ce = o_pe + self.n_nodes
        o_csa = o_ce + self.n_nodes
        o_csc = o_csa + self.nr[0] * self.n_ea
        n = o_csc + self.nr[1] * self.n_ec
        return o_ps, o_pe, o_ce, o_csa, o_csc, n

    @property
    def N(self) -> int:
        return self.offsets[5]

    @property
    def h(self) -> float:
        return (self.length if self.length > 0 else 1.0) / (self.nz - 1)

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Random fields
# ---------------------------------------------------------------------------
def grf(rng: np.random.Generator, shape_cells: Tuple[int, int, int],
        corr_cells: float = 8.0) -> np.ndarray:
    """Filtered Gaussian random field on an element grid, mean 0, variance 1.

    ``shape_cells`` = (ncx, ncy, ncz) elements.  Coarse standard-normal
    samples on a grid of spacing ``corr_cells`` elements are trilinearly
    interpolated to element centres, then filtered with
    ``(I - h_c^2 Lap) g~ = g`` (7-point Laplacian, zero-flux boundaries,
    solved exactly in the cosine basis), then standardized.  Returns an array
    in element-id order (x fastest)."""
    from scipy.fft import dctn, idctn
    ncx, ncy, ncz = shape_cells
    hc = float(corr_cells)
    cdims = [int(np.ceil(n / hc)) + 1 for n in (ncx, ncy, ncz)]
    coarse = rng.standard_normal(size=(cdims[2], cdims[1], cdims[0]))

    def axis_weights(n):
        t = (np.arange(n) + 0.5) / hc
        i0 = np.floor(t).astype(np.int64)
        w = t - i0
        return i0, w

    ix, wx = axis_weights(ncx)
    iy, wy = axis_weights(ncy)
    iz, wz = axis_weights(ncz)
    g = np.zeros((ncz, ncy, ncx))
    for dz in (0, 1):
        fz = (wz if dz else 1 - wz)[:, None, None]
        for dy in (0, 1):
            fy = (wy if dy else 1 - wy)[None, :, None]
            for dx in (0, 1):
                fx = (wx if dx else 1 - wx)[None, None, :]
                g += fz * fy * fx * coarse[np.ix_(iz + dz, iy + dy, ix + dx)]
    # filter in units of element size: (I - hc^2 Lap) with unit spacing
    lam = 0.0
    lam_z = 2.0 - 2.0 * np.cos(np.pi * np.arange(ncz) / ncz)
    lam_y = 2.0 - 2.0 * np.cos(np.pi * np.arange(ncy) / ncy)
    lam_x = 2.0 - 2.0 * np.cos(np.pi * np.arange(ncx) / ncx)
    lam = lam_z[:, None, None] + lam_y[None, :, None] + lam_x[None, None, :]
    gh = dctn(g, type=2, norm="ortho")
    gt = idctn(gh / (1.0 + hc * hc * lam), type=2, norm="ortho")
    gt = gt - gt.mean()
    sd = gt.std()
    if sd > 0:
        gt = gt / sd
    return np.ascontiguousarray(gt.reshape(-1))


# ---------------------------------------------------------------------------
# Problem factories
# ---------------------------------------------------------------------------
D_S_ANODE = 1.0e-14    # solid diffusivity of the benchmark cells [m^2/s]
D_S_CATHODE = 4.0e-15


def make_custom(nx: int, ny: int, nz: int, nr=(10, 10), *, seed: int = 0,
                sigma_log: float = 0.0, na: Optional[int] = None,
                ns: Optional[int] = None, rng: Optional[np.random.Generator] = None,
                Ds_phys=(D_S_ANODE, D_S_CATHODE), dt: float = 1.0,
                lambda_c: float = 1.0, theta_bar=(0.5, 0.5),
                corr_cells: float = 8.0, name: str = "") -> Problem:
    """Build a seeded problem.  Draw order: GRF(sigma), GRF(kappa), g, s,
    e-magnitude, b."""
    if na is None or ns is None:
        na_, ns_, _ = layer_split(nz)
        na = na_ if na is None else na
        ns = ns_ if ns is None else ns
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    Ds = (Ds_phys[0] * dt / R_S ** 2, Ds_phys[1] * dt / R_S ** 2)
    p = Problem(nx=nx, ny=ny, nz=nz, na=na, ns=ns, nr=(int(nr[0]), int(nr[1])),
                Ds=Ds, theta_bar=tuple(theta_bar), dt=dt, lambda_c=lambda_c,
                name=name)
    if p.nc < 2 or p.na < 2 or p.ns < 1:
        raise ValueError("need >= 2 layers per electrode and >= 1 separator layer")
    cells = (nx - 1, ny - 1, nz - 1)
    if sigma_log > 0.0:
        p.sigma = np.exp(sigma_log * grf(rng, cells, corr_cells))
        p.kappa = np.exp(sigma_log * grf(rng, cells, corr_cells))
    else:
        p.sigma = np.ones(p.n_elem)
        p.kappa = np.ones(p.n_elem)
    ne = p.n_e
    p.g = rng.uniform(0.5, 2.0, size=ne)
    p.s = rng.uniform(0.5, 2.0, size=ne)
    emag = rng.uniform(0.5, 2.0, size=ne)
    sign = np.concatenate([np.ones(p.n_ea), -np.ones(p.n_ec)])
    p.e = sign * 0.1 * emag
    p.b = rng.standard_normal(size=p.N)
    return p


# flattened jelly roll (Case III, Sec. 5): a stack 120 um thick (50 / 20 /
# 50 um), 5 cm high and 1 m long on 56 x 85 x 1800 elements; here 60
# elements through the stack so that the layers fall on element faces
CASE3_STACK_UM = 120.0
CASE3_HX_M = 1.0 / 1800      # element edge along the roll
CASE3_HY_M = 0.05 / 85       # element edge along the height


def make_case3_like(nx: int = 1801, ny: int = 86, nz: int = 61, nr=(10, 10), *,
                    seed: int = 6) -> Problem:
    """Linearized system on the Case III mesh: nz - 1 elements through the
    stack (z, nondimensional thickness 1, layers 5/12, 1/6, 5/12 of it) and
    the paper's element edges along the roll and the height (about 280x the
    edge through the stack at nz = 61); nx - 1 by ny - 1 elements cover the
    whole roll at the defaults, a section of it otherwise.  Coefficients,
    Butler-Volmer derivatives and the right-hand side as make_custom with
    uniform sigma = kappa = 1."""
    if (nz - 1) % 12 != 0:
        raise ValueError("nz - 1 must be a multiple of 12 (25/10/25 of 60 elements)")
    e = (nz - 1) // 12
    hz_m = CASE3_STACK_UM * 1e-6 / (nz - 1)
    hx_m, hy_m = CASE3_HX_M, CASE3_HY_M
    p = make_custom(nx, ny, nz, nr, seed=seed, na=5 * e + 1, ns=2 * e,
                    name=f"Case III-like flattened roll {nx}x{ny}x{nz} Nr={nr[0]}")
    h = p.h
    return p.with_(hxy=(h * hx_m / hz_m, h * hy_m / hz_m))


def make_config(cid: int, seed: Optional[int] = None) -> Problem:
    """Benchmark configurations C1, C2, C3, C5 (C4 is ``make_batch``)."""
    seed = cid if seed is None else seed
    if cid == 1:
        return make_custom(8, 8, 24, (10, 10), seed=seed, name="C1 tiny cube 8x8x24 Nr=10")
    if cid == 2:
        return make_custom(64, 64, 192, (20, 20), seed=seed,
                           name="C2 homogeneous cube 64x64x192 Nr=20")
    if cid == 3:
        return make_custom(64, 64, 192, (20, 20), seed=seed, sigma_log=1.0,
                           name="C3 lognormal cube 64x64x192 Nr=20 sigma_log=1")
    if cid == 5:
        return make_custom(128, 128, 256, (16, 16), seed=seed, sigma_log=1.0,
                           name="C5 large cell 128x128x256 Nr=16 sigma_log=1")
    raise ValueError(f"unknown config {cid}")


def make_batch(ncells: int = 64, seed: int = 4, sides=(16, 24, 32, 48),
               nrs=(8, 16, 32), sigma_log: float = 0.5) -> List[Problem]:
    """C4: independent cells of uneven mesh and radial sizes.  Per cell
    (its own spawned stream): side, Nr anode, Nr cathode, then the draws of
    ``make_custom``."""
    ss = np.random.SeedSequence(seed)
    out = []
    for c, child in enumerate(ss.spawn(ncells)):
        rng = np.random.Generator(np.random.PCG64(child))
        side = int(rng.choice(sides))
        nra = int(rng.choice(nrs))
        nrc = int(rng.choice(nrs))
        out.append(make_custom(side, side, 3 * side, (nra, nrc), rng=rng,
                               sigma_log=sigma_log,
                               name=f"C4 cell {c}: {side}x{side}x{3*side} Nr=({nra},{nrc})"))
    return out


def functional_weights(p: Problem) -> np.ndarray:
    """Weights ``w`` with ``J = w . x`` = mean of phi_s over the cathode top
    face (Gamma_p, where the applied current enters): lumped Q1 face
    quadrature 1, 1/2, 1/4 for interior, edge and corner nodes, normalized to
    sum 1."""
    w = np.zeros(p.N)
    fx = np.ones(p.nx); fx[0] = fx[-1] = 0.5
    fy = np.ones(p.ny); fy[0] = fy[-1] = 0.5
    face = (fy[:, None] * fx[None, :]).reshape(-1)
    face = face / face.sum()
    start = p.n_ea + p.nx * p.ny * (p.nc - 1)   # top layer of cathode phi_s
    w[start:start + p.nx * p.ny] = face
    return w
