"""Plain FP64 CPU oracle for the linearized pseudo-4D DFN Jacobian solve.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The product (the HIP library and
its Python binding) never does.

The arithmetic lives in ``p4d_oracle.c`` (plain loops, each function citing
the section or equation of arXiv 2602.07225 it follows); this module only
marshals numpy arrays through ctypes.

Parity status of each oracle function (pins in ``tests/test_oracle_*.py``):
  radial rows, mesh, Gamma        pinned (exactness on quadratics, zero row
                                  sums, mass conservation, truncation order)
  Q1 operator blocks              pinned (quadrature element matrices, row
                                  sums, linear exactness, consistency order)
  reaction coupling               pinned (charge conservation, lithium balance)
  full operator / transpose       pinned (above + dot-product identity)
  Galerkin RAP                    pinned (equals coarse-grid Q1 assembly)
  Chebyshev smoother              pinned (closed-form Chebyshev polynomial)
  V-cycle                         pinned (symmetry, convergence as iteration,
                                  two-grid cycle equal to the dense composed
                                  error propagation)
  preconditioner                  pinned (dense block-LDU with exact Schur
                                  diagonal blocks on tiny meshes)
  FGMRES solve                    pinned (dense LU; manufactured solution)
  parameter gradients             pinned (central finite differences of
                                  oracle solves)
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PC_SCHUR = 0
PC_BJ = 1
PC_BGS = 2

# Krylov space: all unknowns, or the Schur complement of the c_s blocks
KRYLOV_FULL = 0
KRYLOV_SCHUR = 1
# multigrid smoothing: Chebyshev with full coarsening, or symmetric z-line
# block Gauss-Seidel with coarsening in x and y only
SMOOTH_CHEB = 0
SMOOTH_ZLINE = 1

# fields of the 4x4 block system as numbered in a block ordering
F_PHIS, F_PHIE, F_CE, F_CS = 0, 1, 2, 3
FIELD_NAMES = ("phi_s", "phi_e", "c_e", "c_s")


def bgs_order(fields):
    """Pack a field ordering (a permutation of 0..3, first block first) as
    the preconditioner option: the field at block position p in bits
    [2p, 2p + 2)."""
    fields = tuple(int(f) for f in fields)
    if sorted(fields) != [0, 1, 2, 3]:
        raise ValueError(f"{fields} is not an ordering of the four fields")
    return sum(f << (2 * p) for p, f in enumerate(fields))


def bgs_order_fields(order):
    """Inverse of bgs_order."""
    fields = tuple((int(order) >> (2 * p)) & 3 for p in range(4))
    if sorted(fields) != [0, 1, 2, 3] or int(order) >> 8:
        raise ValueError(f"{order} is not a packed field ordering")
    return fields


# the ordering of the paper's scaling runs (Sec. 5): (phi_e, c_s, phi_s, c_e)
BGS_PAPER = bgs_order((F_PHIE, F_CS, F_PHIS, F_CE))

_dp = C.POINTER(C.c_double)


class Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("na", C.c_int32), ("ns", C.c_int32), ("nr", C.c_int32 * 2),
                ("Ds", C.c_double * 2), ("theta_bar", C.c_double * 2),
                ("dt", C.c_double), ("chi", C.c_double), ("tc", C.c_double),
                ("lambda_c", C.c_double), ("eps_elec", C.c_double),
                ("eps_sep", C.c_double), ("length", C.c_double),
                ("lambda_el", C.c_double * 2), ("hxy", C.c_double * 2)]


class Opts(C.Structure):
    _fields_ = [("pc", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("cgs2", C.c_int32), ("rtol", C.c_double),
                ("coarse_max", C.c_int32), ("cheb_degree", C.c_int32),
                ("bgs_order", C.c_int32), ("krylov", C.c_int32), ("smoother", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("relres_est", C.c_double), ("relres_true", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Desc), _dp, _dp, _dp, _dp, _dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_apply.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_setup.argtypes = [C.c_void_p, C.POINTER(Opts)]
        L.orc_apply_pc.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_fgmres.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.POINTER(Info)]
        L.orc_fgmres.restype = C.c_int
        L.orc_gradient.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_schur_apply.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_set_transport.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_set_storage.argtypes = [C.c_void_p, _dp]
        L.orc_set_newton.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.orc_schur_rhs.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_schur_back.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_radial_mesh.argtypes = [C.c_int, C.c_double, _dp]
        L.orc_radial_rows.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_radial_rows.restype = C.c_double
        L.orc_radial_info.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_lumped_weights.argtypes = [C.c_void_p, _dp]
        L.orc_mg_nlev.argtypes = [C.c_void_p, C.c_int]
        L.orc_mg_nlev.restype = C.c_int
        L.orc_mg_level.argtypes = [C.c_void_p, C.c_int, C.c_int,
                                   C.POINTER(C.c_int32), _dp]
        L.orc_mg_stencil.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp]
        L.orc_vcycle.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_omega.argtypes = [C.c_void_p, _dp]
        L.orc_rap.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp]
        L.orc_stencil_apply.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_zline_sweep.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_int, _dp, _dp]
        L.orc_chebyshev.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_int, _dp, _dp]
        L.orc_gershgorin.argtypes = [C.c_int, C.c_int, C.c_int, _dp]
        L.orc_gershgorin.restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# Radial helpers (Sec. 3.1)
# ---------------------------------------------------------------------------
def radial_mesh(N: int, theta_bar: float) -> np.ndarray:
    rho = np.zeros(N)
    lib().orc_radial_mesh(N, theta_bar, _p(rho))
    return rho


def radial_rows(N: int, D: float, rho: np.ndarray):
    """(sub, diag, sup, flux) of L_h without its flux term; ``flux`` is the
    coefficient of i_n/F in the surface row."""
    rho = _f64(rho)
    sub, dia, sup = np.zeros(N), np.zeros(N), np.zeros(N)
    flux = lib().orc_radial_rows(N, D, _p(rho), _p(sub), _p(dia), _p(sup))
    return sub, dia, sup, flux


# ---------------------------------------------------------------------------
# Stencil helpers (test pins of the multigrid pieces)
# ---------------------------------------------------------------------------
def rap(dims, S: np.ndarray, coarsen_z: bool = True) -> np.ndarray:
    nx, ny, nz = dims
    cdim = [n if n <= 2 else n // 2 + 1 for n in dims]
    if not coarsen_z:
        cdim[2] = nz
    Sc = np.zeros(27 * cdim[0] * cdim[1] * cdim[2])
    lib().orc_rap(nx, ny, nz, int(coarsen_z), _p(_f64(S).reshape(-1)), _p(Sc))
    return Sc.reshape(-1, 27), tuple(cdim)


def stencil_apply(dims, S, x):
    y = np.zeros(len(x))
    lib().orc_stencil_apply(*dims, _p(_f64(S).reshape(-1)), _p(_f64(x)), _p(y))
    return y


def chebyshev(dims, S, deg, b, x0=None):
    x = np.zeros(len(b)) if x0 is None else _f64(x0).copy()
    lib().orc_chebyshev(*dims, _p(_f64(S).reshape(-1)), deg, _p(_f64(b)), _p(x))
    return x


def zline_sweep(dims, S, b, x0, backward=False):
    """One pass of z-line block Gauss-Seidel over the four colours."""
    x = _f64(x0).copy()
    lib().orc_zline_sweep(*dims, _p(_f64(S).reshape(-1)), int(backward), _p(_f64(b)), _p(x))
    return x


def gershgorin(dims, S):
    return lib().orc_gershgorin(*dims, _p(_f64(S).reshape(-1)))


# ---------------------------------------------------------------------------
# The problem object
# ---------------------------------------------------------------------------
@dataclass
class SolveInfo:
    iters: int
    restarts: int
    status: int
    relres_est: float
    relres_true: float


class Oracle:
    """Oracle instance for one ``p4d_inputs.Problem``."""

    def __init__(self, prob):
        self.prob = prob
        d = Desc()
        d.nx, d.ny, d.nz, d.na, d.ns = prob.nx, prob.ny, prob.nz, prob.na, prob.ns
        d.nr[0], d.nr[1] = prob.nr
        d.Ds[0], d.Ds[1] = prob.Ds
        d.theta_bar[0], d.theta_bar[1] = prob.theta_bar
        d.dt, d.chi, d.tc, d.lambda_c = prob.dt, prob.chi, prob.tc, prob.lambda_c
        d.eps_elec, d.eps_sep = prob.eps_elec, prob.eps_sep
        d.length = getattr(prob, "length", 0.0)
        lel = getattr(prob, "lambda_el", (0.0, 0.0))
        d.lambda_el[0], d.lambda_el[1] = lel
        d.hxy[0], d.hxy[1] = getattr(prob, "hxy", (0.0, 0.0))
        self.desc = d
        self._keep = [_f64(prob.sigma), _f64(prob.kappa), _f64(prob.g),
                      _f64(prob.s), _f64(prob.e)]
        self.h = lib().orc_create(C.byref(d), *[_p(a) for a in self._keep])
        kd, dc = getattr(prob, "kappa_d", None), getattr(prob, "dce", None)
        if kd is not None or dc is not None:
            self._keep_t = [None if a is None else _f64(a) for a in (kd, dc)]
            lib().orc_set_transport(self.h, *[None if a is None else _p(a) for a in self._keep_t])
        ep = getattr(prob, "eps_e", None)
        if ep is not None:
            self._keep_e = _f64(ep)
            lib().orc_set_storage(self.h, _p(self._keep_e))
        nw = getattr(prob, "newton", None)
        if nw is not None:
            self._keep_n = [_f64(a) for a in nw]
            lib().orc_set_newton(self.h, *[_p(a) for a in self._keep_n])
        sz = (C.c_int64 * 8)()
        lib().orc_sizes(self.h, sz)
        self.sizes = list(sz)
        self.N = int(sz[5])
        self.opts = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- operator ------------------------------------------------------------
    def apply(self, x, transpose=False):
        x = _f64(x)
        assert x.shape == (self.N,)
        y = np.zeros(self.N)
        lib().orc_apply(self.h, int(transpose), _p(x), _p(y))
        return y

    def dense(self, transpose=False):
        """Assemble A column by column (tiny meshes only)."""
        A = np.zeros((self.N, self.N))
        e = np.zeros(self.N)
        for c in range(self.N):
            e[c] = 1.0
            A[:, c] = self.apply(e, transpose)
            e[c] = 0.0
        return A

    # -- preconditioner --------------------------------------------------------
    def setup(self, pc=PC_SCHUR, restart=30, maxit=1000, rtol=1e-8, cgs2=False,
              coarse_max=64, cheb_degree=2, bgs_order=BGS_PAPER, krylov=KRYLOV_FULL,
              smoother=SMOOTH_CHEB):
        o = Opts()
        o.pc, o.restart, o.maxit, o.cgs2 = pc, restart, maxit, int(cgs2)
        o.rtol, o.coarse_max, o.cheb_degree = rtol, coarse_max, cheb_degree
        o.bgs_order = bgs_order
        o.krylov = krylov
        o.smoother = smoother
        if smoother not in (SMOOTH_CHEB, SMOOTH_ZLINE):
            raise ValueError("smoother must be SMOOTH_CHEB or SMOOTH_ZLINE")
        if krylov not in (KRYLOV_FULL, KRYLOV_SCHUR) or (krylov == KRYLOV_SCHUR and pc != PC_SCHUR):
            raise ValueError("krylov must be KRYLOV_FULL, or KRYLOV_SCHUR with PC_SCHUR")
        if restart > 63:
            raise ValueError("restart must be <= 63")
        if pc == PC_BGS:
            bgs_order_fields(bgs_order)   # raises unless a permutation
        self.opts = o
        lib().orc_setup(self.h, C.byref(o))
        return self

    # -- Schur complement of the c_s blocks ------------------------------------
    @property
    def n_macro(self):
        return int(self.sizes[3])

    def schur_apply(self, y, transpose=False):
        """S y (S^T y), S = A_yy - A_ys A_ss^-1 A_sy over [phi_s | phi_e | c_e]."""
        y = _f64(y)
        out = np.zeros(self.n_macro)
        lib().orc_schur_apply(self.h, int(transpose), _p(y), _p(out))
        return out

    def schur_rhs(self, b, transpose=False):
        """b_y - A_ys A_ss^-1 b_s."""
        b = _f64(b)
        out = np.zeros(self.n_macro)
        lib().orc_schur_rhs(self.h, int(transpose), _p(b), _p(out))
        return out

    def schur_back(self, b, y, transpose=False):
        """The full solution [y | A_ss^-1 (b_s - A_sy y)]."""
        b = _f64(b)
        x = np.zeros(self.N)
        x[:self.n_macro] = y
        lib().orc_schur_back(self.h, int(transpose), _p(b), _p(x))
        return x

    def apply_pc(self, r, transpose=False):
        r = _f64(r)
        z = np.zeros(self.N)
        lib().orc_apply_pc(self.h, int(transpose), _p(r), _p(z))
        return z

    def solve(self, b, transpose=False):
        b = _f64(b)
        x = np.zeros(self.N)
        info = Info()
        lib().orc_fgmres(self.h, int(transpose), _p(b), _p(x), C.byref(info))
        return x, SolveInfo(info.iters, info.restarts, info.status,
                            info.relres_est, info.relres_true)

    def gradient(self, x, lam):
        ds = np.zeros(self.prob.n_elem)
        dD = np.zeros(2)
        lib().orc_gradient(self.h, _p(_f64(x)), _p(_f64(lam)), _p(ds), _p(dD))
        return ds, dD

    # -- inspection -------------------------------------------------------------
    def radial(self, el):
        N = self.prob.nr[el]
        rho, sub, dia, sup = (np.zeros(N) for _ in range(4))
        g = C.c_double()
        lib().orc_radial_info(self.h, el, _p(rho), _p(sub), _p(dia), _p(sup), C.byref(g))
        return rho, sub, dia, sup, g.value

    def lumped_weights(self):
        m = np.zeros(self.prob.n_e)
        lib().orc_lumped_weights(self.h, _p(m))
        return m

    def omega(self):
        w = np.zeros(self.prob.n_e)
        lib().orc_omega(self.h, _p(w))
        return w

    def mg_levels(self, box):
        out = []
        for l in range(lib().orc_mg_nlev(self.h, box)):
            dims = (C.c_int32 * 3)()
            lm = C.c_double()
            lib().orc_mg_level(self.h, box, l, dims, C.byref(lm))
            out.append((tuple(dims), lm.value))
        return out

    def mg_stencil(self, box, level):
        dims = self.mg_levels(box)[level][0]
        S = np.zeros(27 * dims[0] * dims[1] * dims[2])
        lib().orc_mg_stencil(self.h, box, level, _p(S))
        return S.reshape(-1, 27)

    def vcycle(self, box, b):
        b = _f64(b)
        x = np.zeros(len(b))
        lib().orc_vcycle(self.h, box, _p(b), _p(x))
        return x

    def box_slice(self, box):
        p = self.prob
        layer = p.nx * p.ny
        o = p.offsets
        if box == 0:
            return slice(o[0] + layer, o[0] + p.n_ea)
        if box == 1:
            return slice(o[0] + p.n_ea, o[0] + p.n_e)
        if box == 2:
            return slice(o[1], o[1] + p.n_nodes)
        return slice(o[2], o[2] + p.n_nodes)
