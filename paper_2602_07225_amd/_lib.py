"""ctypes binding of ``libp4d.so`` (the C ABI in ``include/p4d.h``).

Argument marshalling only: torch tensors are passed as raw device pointers,
the current HIP stream as ``void*``.  Function names equal the C ones.  There
is no fallback: if the library is missing or fails to load, every call
raises."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libp4d.so")

P4D_OK = 0
P4D_NOT_CONVERGED = 1
P4D_BREAKDOWN = 2
P4D_ERR_INVALID_ARG = -1
P4D_ERR_OOM = -2
P4D_ERR_HIP = -3
P4D_ERR_STATE = -4
P4D_ERR_NONFINITE = -5

P4D_PC_SCHUR = 0
P4D_PC_BJ = 1
P4D_PC_BGS = 2
# field codes of a block Gauss-Seidel ordering (bits [2p, 2p + 2) hold the
# field at block position p)
P4D_F_PHIS, P4D_F_PHIE, P4D_F_CE, P4D_F_CS = 0, 1, 2, 3
P4D_BGS_PAPER_ORDER = P4D_F_PHIE | (P4D_F_CS << 2) | (P4D_F_PHIS << 4) | (P4D_F_CE << 6)
P4D_FP64 = 0
P4D_FP32 = 1
P4D_KRYLOV_FULL = 0
P4D_KRYLOV_SCHUR = 1
P4D_SMOOTH_CHEB = 0
P4D_SMOOTH_ZLINE = 1
# size of the static scratch of p4d_solve_noalloc (per GPU)
P4D_NOALLOC_MAX_BYTES = 64 << 20

(P4D_K_OPERATOR, P4D_K_MDOT, P4D_K_ORTH, P4D_K_RADIAL, P4D_K_SMOOTH0, P4D_K_ZY,
 P4D_K_BATCH_PC, P4D_K_COUPLING) = range(1, 9)
P4D_K_COUNT = 9
KERNEL_CLASSES = {P4D_K_OPERATOR: "operator", P4D_K_MDOT: "mdot", P4D_K_ORTH: "orth",
                  P4D_K_RADIAL: "radial", P4D_K_SMOOTH0: "smooth0", P4D_K_ZY: "zy",
                  P4D_K_BATCH_PC: "batch_pc", P4D_K_COUPLING: "coupling"}

EXPORTED = [
    "p4d_default_opts", "p4d_create", "p4d_destroy", "p4d_vector_size", "p4d_workspace_size",
    "p4d_set_workspace", "p4d_upload", "p4d_set_transport", "p4d_set_storage", "p4d_set_diffusivity",
    "p4d_setup",
    "p4d_apply_operator",
    "p4d_apply_schur_operator", "p4d_apply_preconditioner", "p4d_solve", "p4d_solve_adjoint", "p4d_param_gradient",
    "p4d_solve_noalloc",
    "p4d_profile", "p4d_profile_every", "p4d_profile_read", "p4d_status_string", "p4d_last_error", "p4d_autotune",
    "p4d_batch_create", "p4d_batch_destroy", "p4d_batch_cell", "p4d_batch_workspace_size",
    "p4d_batch_set_workspace", "p4d_batch_upload", "p4d_batch_setup", "p4d_batch_autotune",
    "p4d_batch_solve", "p4d_batch_set_pc_mode", "p4d_batch_profile", "p4d_batch_profile_read",
    "p4d_batch_last_error",
    "p4d_phys_create", "p4d_phys_workspace_size", "p4d_phys_set_workspace", "p4d_phys_initial_state",
    "p4d_phys_residual", "p4d_phys_newton_step", "p4d_phys_set_fractions", "p4d_phys_jacobian_apply",
]


class ProblemDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("na", C.c_int32), ("ns", C.c_int32), ("nr", C.c_int32 * 2),
                ("Ds", C.c_double * 2), ("theta_bar", C.c_double * 2),
                ("dt", C.c_double), ("chi", C.c_double), ("tc", C.c_double),
                ("lambda_c", C.c_double), ("eps_elec", C.c_double), ("eps_sep", C.c_double),
                ("length", C.c_double), ("lambda_el", C.c_double * 2), ("hxy", C.c_double * 2)]


class SolveOpts(C.Structure):
    _fields_ = [("pc", C.c_int32), ("pc_prec", C.c_int32), ("restart", C.c_int32),
                ("maxit", C.c_int32), ("cheb_degree", C.c_int32), ("coarse_max", C.c_int32),
                ("cgs2", C.c_int32), ("z_fp32", C.c_int32), ("rtol", C.c_double),
                ("bgs_order", C.c_int32), ("krylov", C.c_int32), ("smoother", C.c_int32)]


class Electrode(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("eps_s", "eps", "sigma", "k", "alpha", "cs_max", "cs0", "a", "Ds", "Rs")]


class PhysParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("nr", C.c_int32 * 2), ("theta_bar", C.c_double * 2),
                ("dt", C.c_double), ("current", C.c_double), ("gauss_frac", C.c_double),
                ("edge", C.c_double), ("F", C.c_double), ("R", C.c_double), ("T", C.c_double),
                ("t_plus", C.c_double), ("brug", C.c_double), ("ce0", C.c_double),
                ("eps_sep", C.c_double), ("el", Electrode * 2), ("profile", C.c_int32)]


class NewtonOpts(C.Structure):
    _fields_ = [("maxit", C.c_int32), ("tol", C.c_double)]


class NewtonInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("lin_iters", C.c_int32),
                ("update", C.c_double), ("t_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("relres_est", C.c_double), ("relres_true", C.c_double),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class P4DError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"p4d status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                               "(the solver has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.p4d_default_opts.argtypes = [C.POINTER(SolveOpts)]
        L.p4d_default_opts.restype = None
        L.p4d_create.argtypes = [C.POINTER(ProblemDesc), C.POINTER(vp)]
        L.p4d_destroy.argtypes = [vp]
        L.p4d_destroy.restype = None
        L.p4d_vector_size.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.p4d_workspace_size.argtypes = [vp, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]
        L.p4d_set_workspace.argtypes = [vp, vp, C.c_size_t, C.POINTER(SolveOpts)]
        L.p4d_upload.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.p4d_setup.argtypes = [vp, C.POINTER(SolveOpts), vp]
        L.p4d_set_diffusivity.argtypes = [vp, C.POINTER(C.c_double), vp]
        L.p4d_set_transport.argtypes = [vp, vp, vp, vp]
        L.p4d_set_storage.argtypes = [vp, vp, vp]
        L.p4d_apply_operator.argtypes = [vp, C.c_int, vp, vp, vp]
        L.p4d_apply_preconditioner.argtypes = [vp, C.c_int, vp, vp, vp]
        L.p4d_apply_schur_operator.argtypes = [vp, C.c_int, vp, vp, vp]
        L.p4d_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.p4d_solve_adjoint.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.p4d_param_gradient.argtypes = [vp, vp, vp, vp, vp, vp]
        L.p4d_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(SolveOpts),
                                        C.POINTER(SolveInfo), vp]
        L.p4d_profile.argtypes = [vp, C.c_int]
        L.p4d_profile_every.argtypes = [vp, C.c_int]
        L.p4d_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.p4d_status_string.argtypes = [C.c_int]
        L.p4d_status_string.restype = C.c_char_p
        L.p4d_last_error.argtypes = [vp]
        L.p4d_last_error.restype = C.c_char_p
        L.p4d_autotune.argtypes = [vp, vp, C.POINTER(C.c_int32)]
        for name in ["p4d_autotune", "p4d_create", "p4d_vector_size", "p4d_workspace_size", "p4d_set_workspace",
                     "p4d_upload", "p4d_set_transport", "p4d_set_storage", "p4d_set_diffusivity", "p4d_setup",
                     "p4d_apply_operator",
                     "p4d_apply_preconditioner", "p4d_apply_schur_operator",
                     "p4d_solve", "p4d_solve_adjoint", "p4d_param_gradient", "p4d_profile",
                     "p4d_profile_every", "p4d_profile_read", "p4d_solve_noalloc"]:
            getattr(L, name).restype = C.c_int
        _bind_batch(L)
        _bind_phys(L)
        _lib = L
    return _lib


def _bind_phys(L):
    vp = C.c_void_p
    L.p4d_phys_create.argtypes = [C.POINTER(PhysParams), C.POINTER(vp)]
    L.p4d_phys_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.p4d_phys_set_workspace.argtypes = [vp, vp, C.c_size_t]
    L.p4d_phys_initial_state.argtypes = [vp, vp, vp]
    L.p4d_phys_residual.argtypes = [vp, vp, vp, vp, vp]
    L.p4d_phys_newton_step.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(NewtonOpts),
                                       C.POINTER(NewtonInfo), vp]
    L.p4d_phys_set_fractions.argtypes = [vp, vp, vp, vp]
    L.p4d_phys_jacobian_apply.argtypes = [vp, vp, C.c_int, vp, vp, vp]
    for name in ("p4d_phys_create", "p4d_phys_workspace_size", "p4d_phys_set_workspace",
                 "p4d_phys_initial_state", "p4d_phys_residual", "p4d_phys_newton_step",
                 "p4d_phys_set_fractions", "p4d_phys_jacobian_apply"):
        getattr(L, name).restype = C.c_int


def phys_params(case, current: float) -> PhysParams:
    """PhysParams from a p4d_inputs.phys.PhysCase (data of the case) and the
    applied current."""
    from p4d_inputs import phys as ph
    p = PhysParams()
    p.n = case.n
    p.nr[0], p.nr[1] = case.nr
    p.theta_bar[0], p.theta_bar[1] = case.theta_bar
    p.dt, p.current, p.gauss_frac, p.edge = case.dt, current, case.gauss_frac, ph.CELL_EDGE
    p.F, p.R, p.T = ph.F, ph.R_GAS, ph.T_REF
    p.t_plus, p.brug, p.ce0, p.eps_sep = ph.T_PLUS, ph.BRUGGEMAN, ph.CE0, ph.SEPARATOR_EPS
    for i, e in enumerate(case.electrodes):
        for k, _ in Electrode._fields_:
            setattr(p.el[i], k, getattr(e, k))
    p.profile = 1 if getattr(case, "profile", "gauss") == "uniform" else 0
    return p


def p4d_phys_create(params: PhysParams) -> int:
    h = C.c_void_p()
    check(lib().p4d_phys_create(C.byref(params), C.byref(h)), None, "p4d_phys_create")
    return h.value


def p4d_phys_workspace_size(ctx) -> int:
    n = C.c_size_t()
    check(lib().p4d_phys_workspace_size(ctx, C.byref(n)), ctx, "p4d_phys_workspace_size")
    return n.value


def p4d_phys_set_workspace(ctx, ptr_, nbytes):
    return check(lib().p4d_phys_set_workspace(ctx, ptr_, nbytes), ctx, "p4d_phys_set_workspace")


def p4d_phys_initial_state(ctx, u, stream=None):
    return check(lib().p4d_phys_initial_state(ctx, ptr(u), stream_ptr(stream)), ctx,
                 "p4d_phys_initial_state")


def p4d_phys_residual(ctx, u, uold, r, stream=None):
    return check(lib().p4d_phys_residual(ctx, ptr(u), ptr(uold), ptr(r), stream_ptr(stream)), ctx,
                 "p4d_phys_residual")


def p4d_phys_newton_step(ctx, u, uold, solve: SolveOpts | None = None, newton: NewtonOpts | None = None,
                         stream=None):
    info = NewtonInfo()
    st = check(lib().p4d_phys_newton_step(ctx, ptr(u), ptr(uold), C.byref(solve) if solve else None,
                                          C.byref(newton) if newton else None, C.byref(info),
                                          stream_ptr(stream)), ctx, "p4d_phys_newton_step")
    return st, info


def _bind_batch(L):
    vp = C.c_void_p
    L.p4d_batch_create.argtypes = [C.POINTER(ProblemDesc), C.c_int32, C.POINTER(vp)]
    L.p4d_batch_destroy.argtypes = [vp]
    L.p4d_batch_destroy.restype = None
    L.p4d_batch_cell.argtypes = [vp, C.c_int32, C.POINTER(vp)]
    L.p4d_batch_workspace_size.argtypes = [vp, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]
    L.p4d_batch_set_workspace.argtypes = [vp, vp, C.c_size_t, C.POINTER(SolveOpts)]
    L.p4d_batch_upload.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp]
    L.p4d_batch_setup.argtypes = [vp, C.POINTER(SolveOpts), vp]
    L.p4d_batch_autotune.argtypes = [vp, vp, C.POINTER(C.c_int32)]
    L.p4d_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveOpts),
                                  C.POINTER(SolveInfo), vp]
    L.p4d_batch_set_pc_mode.argtypes = [vp, C.c_int32]
    L.p4d_batch_profile.argtypes = [vp, C.c_int]
    L.p4d_batch_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.p4d_batch_last_error.argtypes = [vp]
    L.p4d_batch_last_error.restype = C.c_char_p
    for name in ["p4d_batch_create", "p4d_batch_cell", "p4d_batch_workspace_size",
                 "p4d_batch_set_workspace", "p4d_batch_upload", "p4d_batch_setup",
                 "p4d_batch_autotune", "p4d_batch_solve", "p4d_batch_set_pc_mode",
                 "p4d_batch_profile", "p4d_batch_profile_read"]:
        getattr(L, name).restype = C.c_int


def check(status, ctx=None, what="", batch=None):
    """Raise on negative statuses; return the status otherwise."""
    if status < 0:
        msg = lib().p4d_status_string(status).decode()
        if ctx:
            msg += ": " + lib().p4d_last_error(ctx).decode()
        if batch:
            msg += ": " + lib().p4d_batch_last_error(batch).decode()
        raise P4DError(status, f"{what}: {msg}")
    return status


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().p4d_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def desc_from(p) -> ProblemDesc:
    """ProblemDesc from any object with the fields of the problem description
    (nx, ny, nz, na, ns, nr, Ds, theta_bar, dt, chi, tc, lambda_c, eps_elec,
    eps_sep)."""
    d = ProblemDesc()
    d.nx, d.ny, d.nz, d.na, d.ns = p.nx, p.ny, p.nz, p.na, p.ns
    d.nr[0], d.nr[1] = p.nr
    d.Ds[0], d.Ds[1] = p.Ds
    d.theta_bar[0], d.theta_bar[1] = p.theta_bar
    d.dt, d.chi, d.tc, d.lambda_c = p.dt, p.chi, p.tc, p.lambda_c
    d.eps_elec, d.eps_sep = p.eps_elec, p.eps_sep
    d.length = getattr(p, "length", 0.0)
    lel = getattr(p, "lambda_el", (0.0, 0.0))
    d.lambda_el[0], d.lambda_el[1] = lel
    d.hxy[0], d.hxy[1] = getattr(p, "hxy", (0.0, 0.0))
    return d


def ptr(t) -> int:
    """Device pointer of a torch tensor (contiguous, on the GPU)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return t.data_ptr()


def stream_ptr(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# ---- thin same-name wrappers ------------------------------------------------
def p4d_create(desc: ProblemDesc) -> int:
    h = C.c_void_p()
    check(lib().p4d_create(C.byref(desc), C.byref(h)), None, "p4d_create")
    return h.value


def p4d_destroy(ctx: int) -> None:
    lib().p4d_destroy(ctx)


def p4d_vector_size(ctx: int):
    n = C.c_int64()
    offs = (C.c_int64 * 6)()
    ne, nel = C.c_int64(), C.c_int64()
    check(lib().p4d_vector_size(ctx, C.byref(n), offs, C.byref(nel), C.byref(ne)), ctx,
          "p4d_vector_size")
    return n.value, list(offs), nel.value, ne.value


def p4d_workspace_size(ctx: int, opts: SolveOpts | None = None) -> int:
    b = C.c_size_t()
    check(lib().p4d_workspace_size(ctx, C.byref(opts) if opts else None, C.byref(b)), ctx,
          "p4d_workspace_size")
    return b.value


def p4d_set_workspace(ctx: int, d_work: int, nbytes: int, opts: SolveOpts | None = None):
    return check(lib().p4d_set_workspace(ctx, d_work, nbytes, C.byref(opts) if opts else None),
                 ctx, "p4d_set_workspace")


def p4d_upload(ctx, sigma, kappa, g, s, e, stream=None):
    return check(lib().p4d_upload(ctx, ptr(sigma), ptr(kappa), ptr(g), ptr(s), ptr(e),
                                  stream_ptr(stream)), ctx, "p4d_upload")


def p4d_set_diffusivity(ctx, Ds, stream=None):
    arr = (C.c_double * 2)(float(Ds[0]), float(Ds[1]))
    return check(lib().p4d_set_diffusivity(ctx, arr, stream_ptr(stream)), ctx,
                 "p4d_set_diffusivity")


def p4d_setup(ctx, opts: SolveOpts | None = None, stream=None):
    return check(lib().p4d_setup(ctx, C.byref(opts) if opts else None, stream_ptr(stream)),
                 ctx, "p4d_setup")


def p4d_set_transport(ctx, kappa_d=None, dce=None, stream=None):
    return check(lib().p4d_set_transport(ctx, ptr(kappa_d) if kappa_d is not None else None,
                                         ptr(dce) if dce is not None else None, stream_ptr(stream)),
                 ctx, "p4d_set_transport")


def p4d_set_storage(ctx, eps_e=None, stream=None):
    return check(lib().p4d_set_storage(ctx, ptr(eps_e) if eps_e is not None else None,
                                       stream_ptr(stream)), ctx, "p4d_set_storage")


def p4d_phys_jacobian_apply(ctx, u, transpose, x, y, stream=None):
    return check(lib().p4d_phys_jacobian_apply(ctx, ptr(u), int(transpose), ptr(x), ptr(y),
                                               stream_ptr(stream)), ctx, "p4d_phys_jacobian_apply")


def p4d_phys_set_fractions(ctx, eps_s=None, eps_b=None, stream=None):
    return check(lib().p4d_phys_set_fractions(ctx, ptr(eps_s) if eps_s is not None else None,
                                              ptr(eps_b) if eps_b is not None else None,
                                              stream_ptr(stream)), ctx, "p4d_phys_set_fractions")


def p4d_apply_operator(ctx, transpose, x, y, stream=None):
    return check(lib().p4d_apply_operator(ctx, int(transpose), ptr(x), ptr(y),
                                          stream_ptr(stream)), ctx, "p4d_apply_operator")


def p4d_apply_schur_operator(ctx, transpose, y, w, stream=None):
    return check(lib().p4d_apply_schur_operator(ctx, int(transpose), ptr(y), ptr(w),
                                                stream_ptr(stream)), ctx,
                 "p4d_apply_schur_operator")


def p4d_apply_preconditioner(ctx, transpose, r, z, stream=None):
    return check(lib().p4d_apply_preconditioner(ctx, int(transpose), ptr(r), ptr(z),
                                                stream_ptr(stream)), ctx,
                 "p4d_apply_preconditioner")


def p4d_solve(ctx, b, x, opts: SolveOpts | None = None, stream=None):
    info = SolveInfo()
    st = check(lib().p4d_solve(ctx, ptr(b), ptr(x), C.byref(opts) if opts else None,
                               C.byref(info), stream_ptr(stream)), ctx, "p4d_solve")
    return st, info


def p4d_solve_adjoint(ctx, g, lam, opts: SolveOpts | None = None, stream=None):
    info = SolveInfo()
    st = check(lib().p4d_solve_adjoint(ctx, ptr(g), ptr(lam), C.byref(opts) if opts else None,
                                       C.byref(info), stream_ptr(stream)), ctx,
               "p4d_solve_adjoint")
    return st, info


def p4d_solve_noalloc(ctx, sigma, kappa, g, s, e, b, x, opts: SolveOpts | None = None, stream=None):
    """Upload + setup + solve on the library's static scratch (no workspace)."""
    info = SolveInfo()
    st = check(lib().p4d_solve_noalloc(ctx, ptr(sigma), ptr(kappa), ptr(g), ptr(s), ptr(e), ptr(b),
                                       ptr(x), C.byref(opts) if opts else None, C.byref(info),
                                       stream_ptr(stream)), ctx, "p4d_solve_noalloc")
    return st, info


def p4d_param_gradient(ctx, x, lam, dsigma, dDs, stream=None):
    return check(lib().p4d_param_gradient(ctx, ptr(x), ptr(lam), ptr(dsigma), ptr(dDs),
                                          stream_ptr(stream)), ctx, "p4d_param_gradient")


def p4d_profile(ctx, class_mask: int):
    return check(lib().p4d_profile(ctx, class_mask), ctx, "p4d_profile")


def p4d_profile_every(ctx, every: int):
    return check(lib().p4d_profile_every(ctx, every), ctx, "p4d_profile_every")


def p4d_profile_read(ctx, kernel_class: int):
    ms, n, by = C.c_double(), C.c_int64(), C.c_double()
    check(lib().p4d_profile_read(ctx, kernel_class, C.byref(ms), C.byref(n), C.byref(by)), ctx,
          "p4d_profile_read")
    return ms.value, n.value, by.value


def p4d_autotune(ctx, stream=None):
    tile = (C.c_int32 * 2)()
    check(lib().p4d_autotune(ctx, stream_ptr(stream), tile), ctx, "p4d_autotune")
    return tile[0], tile[1]


# ---- batched solves ------------------------------------------------------------
def p4d_batch_create(descs) -> int:
    arr = (ProblemDesc * len(descs))(*descs)
    h = C.c_void_p()
    check(lib().p4d_batch_create(arr, len(descs), C.byref(h)), None, "p4d_batch_create")
    return h.value


def p4d_batch_destroy(batch: int) -> None:
    lib().p4d_batch_destroy(batch)


def p4d_batch_cell(batch: int, cell: int) -> int:
    h = C.c_void_p()
    check(lib().p4d_batch_cell(batch, cell, C.byref(h)), None, "p4d_batch_cell", batch)
    return h.value


def p4d_batch_workspace_size(batch: int, opts: SolveOpts | None = None) -> int:
    b = C.c_size_t()
    check(lib().p4d_batch_workspace_size(batch, C.byref(opts) if opts else None, C.byref(b)),
          None, "p4d_batch_workspace_size", batch)
    return b.value


def p4d_batch_set_workspace(batch, d_work: int, nbytes: int, opts: SolveOpts | None = None):
    return check(lib().p4d_batch_set_workspace(batch, d_work, nbytes,
                                               C.byref(opts) if opts else None),
                 None, "p4d_batch_set_workspace", batch)


def p4d_batch_upload(batch, cell, sigma, kappa, g, s, e, stream=None):
    return check(lib().p4d_batch_upload(batch, cell, ptr(sigma), ptr(kappa), ptr(g), ptr(s),
                                        ptr(e), stream_ptr(stream)),
                 None, "p4d_batch_upload", batch)


def p4d_batch_setup(batch, opts: SolveOpts | None = None, stream=None):
    return check(lib().p4d_batch_setup(batch, C.byref(opts) if opts else None,
                                       stream_ptr(stream)), None, "p4d_batch_setup", batch)


def p4d_batch_autotune(batch, ncells, stream=None):
    tiles = (C.c_int32 * (2 * ncells))()
    check(lib().p4d_batch_autotune(batch, stream_ptr(stream), tiles), None,
          "p4d_batch_autotune", batch)
    return [(tiles[2 * i], tiles[2 * i + 1]) for i in range(ncells)]


def p4d_batch_solve(batch, bs, xs, opts: SolveOpts | None = None, stream=None):
    n = len(bs)
    bp = (C.c_void_p * n)(*[ptr(b) for b in bs])
    xp = (C.c_void_p * n)(*[ptr(x) for x in xs])
    infos = (SolveInfo * n)()
    st = check(lib().p4d_batch_solve(batch, bp, xp, C.byref(opts) if opts else None, infos,
                                     stream_ptr(stream)), None, "p4d_batch_solve", batch)
    return st, list(infos)


def p4d_batch_set_pc_mode(batch, mode: int):
    return check(lib().p4d_batch_set_pc_mode(batch, int(mode)), None, "p4d_batch_set_pc_mode",
                 batch)


def p4d_batch_profile(batch, class_mask: int):
    return check(lib().p4d_batch_profile(batch, class_mask), None, "p4d_batch_profile", batch)


def p4d_batch_profile_read(batch, kernel_class: int):
    ms, n, by = C.c_double(), C.c_int64(), C.c_double()
    check(lib().p4d_batch_profile_read(batch, kernel_class, C.byref(ms), C.byref(n),
                                       C.byref(by)), None, "p4d_batch_profile_read", batch)
    return ms.value, n.value, by.value


def p4d_batch_last_error(batch) -> str:
    return lib().p4d_batch_last_error(batch).decode()
