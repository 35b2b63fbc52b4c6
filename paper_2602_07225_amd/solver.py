"""Torch-facing wrapper of one solver context: owns the device workspace
(a torch uint8 tensor) and forwards every call to the C ABI."""
from __future__ import annotations

import torch

from . import _lib as L


class P4DSolver:
    """One linearized P4D-DFN Jacobian on the current GPU.

    ``prob`` is any object carrying the problem description fields and the
    coefficient arrays ``sigma, kappa`` (per element) and ``g, s, e`` (per
    electrode node), as numpy arrays or torch tensors."""

    def __init__(self, prob, restart: int = 30, z_fp32: bool = False, pc_prec: int = L.P4D_FP64,
                 coarse_max: int = 512, device: str = "cuda", smoother: int = L.P4D_SMOOTH_CHEB):
        self.device = torch.device(device)
        self.desc = L.desc_from(prob)
        self.ctx = L.p4d_create(self.desc)
        self.N, self.offsets, self.n_elem, self.n_e = L.p4d_vector_size(self.ctx)
        # the workspace is laid out for these options (the multigrid hierarchy
        # depends on the precision, coarse size and smoother)
        self.ws_opts = L.default_opts(restart=restart, z_fp32=int(z_fp32), pc_prec=pc_prec,
                                      coarse_max=coarse_max, smoother=smoother)
        nbytes = L.p4d_workspace_size(self.ctx, self.ws_opts)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        L.p4d_set_workspace(self.ctx, self.ws.data_ptr(), nbytes, self.ws_opts)
        self._kd = self._dc = self._ep = None
        # bumped by every call that changes the operator or the
        # preconditioner, so that a differentiable solve can tell whether the
        # context still holds the state of its forward pass
        self.version = 0
        self.upload(prob.sigma, prob.kappa, prob.g, prob.s, prob.e)
        kd, dc = getattr(prob, "kappa_d", None), getattr(prob, "dce", None)
        if kd is not None or dc is not None:
            self.set_transport(kd, dc)
        ep = getattr(prob, "eps_e", None)
        if ep is not None:
            self.set_storage(ep)
        self.opts = None

    def _dev(self, a):
        if isinstance(a, torch.Tensor):
            return a.to(self.device, torch.float64).contiguous()
        return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()

    def upload(self, sigma, kappa, g, s, e):
        arrs = [self._dev(a) for a in (sigma, kappa, g, s, e)]
        assert arrs[0].numel() == self.n_elem and arrs[1].numel() == self.n_elem
        assert all(a.numel() == self.n_e for a in arrs[2:])
        L.p4d_upload(self.ctx, *arrs)
        # kept for re-uploads with a new sigma (differentiable solves)
        self._sigma, self._kappa, self._g, self._s, self._e = arrs
        # the upload resets the separate coefficients: keep those set
        if self._kd is not None or self._dc is not None:
            L.p4d_set_transport(self.ctx, self._kd, self._dc)
        if self._ep is not None:
            L.p4d_set_storage(self.ctx, self._ep)
        self.opts = None
        self.version += 1

    def set_transport(self, kappa_d=None, dce=None):
        """Separate element coefficients of the diffusion-potential block and
        the c_e diffusion (None: chi * kappa and kappa)."""
        self._kd = None if kappa_d is None else self._dev(kappa_d)
        self._dc = None if dce is None else self._dev(dce)
        if any(t is not None and t.numel() != self.n_elem for t in (self._kd, self._dc)):
            raise ValueError(f"transport coefficients need {self.n_elem} values per element")
        L.p4d_set_transport(self.ctx, self._kd, self._dc)
        self.opts = None
        self.version += 1

    def set_storage(self, eps_e=None):
        """Porosity per element for the c_e storage (None: per material)."""
        self._ep = None if eps_e is None else self._dev(eps_e)
        if self._ep is not None and self._ep.numel() != self.n_elem:
            raise ValueError(f"eps_e needs {self.n_elem} values per element")
        L.p4d_set_storage(self.ctx, self._ep)
        self.opts = None
        self.version += 1

    def set_diffusivity(self, Ds):
        """Particle diffusivities (nondimensional, anode/cathode)."""
        L.p4d_set_diffusivity(self.ctx, Ds)
        self.desc.Ds[0], self.desc.Ds[1] = float(Ds[0]), float(Ds[1])
        self.opts = None
        self.version += 1

    def setup(self, **kw):
        o = L.default_opts(**kw)
        L.p4d_setup(self.ctx, o)
        self.opts = o
        self.version += 1
        return self

    def state(self):
        """The uploaded coefficients and diffusivities (device tensors held
        by reference; every upload makes new ones)."""
        return dict(sigma=self._sigma, kappa=self._kappa, g=self._g, s=self._s, e=self._e,
                    kappa_d=self._kd, dce=self._dc, eps_e=self._ep,
                    Ds=(float(self.desc.Ds[0]), float(self.desc.Ds[1])))

    def restore(self, st, **setup_kw):
        """Upload a state taken by ``state()`` and build its preconditioner."""
        self._kd, self._dc, self._ep = st["kappa_d"], st["dce"], st["eps_e"]
        self.upload(st["sigma"], st["kappa"], st["g"], st["s"], st["e"])
        self.set_diffusivity(st["Ds"])
        return self.setup(**setup_kw)

    def apply(self, x, transpose=False):
        x = self._dev(x)
        y = torch.empty_like(x)
        L.p4d_apply_operator(self.ctx, transpose, x, y)
        return y

    def apply_schur(self, y, transpose=False):
        """S y (S^T y) over the electrode-level unknowns (the Schur complement
        of the particle blocks)."""
        y = self._dev(y)
        w = torch.empty_like(y)
        L.p4d_apply_schur_operator(self.ctx, transpose, y, w)
        return w

    def apply_pc(self, r, transpose=False):
        r = self._dev(r)
        z = torch.empty_like(r)
        L.p4d_apply_preconditioner(self.ctx, transpose, r, z)
        return z

    def _opts(self, kw):
        if self.opts is None:
            raise RuntimeError("call setup() first")
        o = L.SolveOpts.from_buffer_copy(self.opts)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def solve(self, b, **kw):
        b = self._dev(b)
        x = torch.empty_like(b)
        st, info = L.p4d_solve(self.ctx, b, x, self._opts(kw))
        return x, info

    def solve_adjoint(self, g, **kw):
        g = self._dev(g)
        lam = torch.empty_like(g)
        st, info = L.p4d_solve_adjoint(self.ctx, g, lam, self._opts(kw))
        return lam, info

    def gradient(self, x, lam):
        ds = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
        dD = torch.empty(2, dtype=torch.float64, device=self.device)
        L.p4d_param_gradient(self.ctx, self._dev(x), self._dev(lam), ds, dD)
        return ds, dD

    def close(self):
        if getattr(self, "ctx", None):
            L.p4d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class P4DBatch:
    """Independent cells of uneven mesh and radial sizes solved together:
    FGMRES in lockstep; per Arnoldi step, one preconditioner launch per stage
    depth for all iterating cells (``p4d_batch_*`` in the C ABI).

    ``probs``: objects with the problem description fields and coefficient
    arrays, one per cell (at most 64)."""

    def __init__(self, probs, restart: int = 30, z_fp32: bool = False,
                 pc_prec: int = L.P4D_FP32, coarse_max: int = 64, device: str = "cuda"):
        self.device = torch.device(device)
        self.n = len(probs)
        self.descs = [L.desc_from(p) for p in probs]
        self.batch = L.p4d_batch_create(self.descs)
        self.cells = [L.p4d_batch_cell(self.batch, i) for i in range(self.n)]
        sizes = [L.p4d_vector_size(c) for c in self.cells]
        self.N = [s[0] for s in sizes]
        self.n_elem = [s[2] for s in sizes]
        self.n_e = [s[3] for s in sizes]
        self.ws_opts = L.default_opts(restart=restart, z_fp32=int(z_fp32), pc_prec=pc_prec,
                                      coarse_max=coarse_max)
        nbytes = L.p4d_batch_workspace_size(self.batch, self.ws_opts)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        L.p4d_batch_set_workspace(self.batch, self.ws.data_ptr(), nbytes, self.ws_opts)
        for i, p in enumerate(probs):
            self.upload(i, p.sigma, p.kappa, p.g, p.s, p.e)
        self.opts = None

    def _dev(self, a):
        if isinstance(a, torch.Tensor):
            return a.to(self.device, torch.float64).contiguous()
        return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()

    def upload(self, i, sigma, kappa, g, s, e):
        arrs = [self._dev(a) for a in (sigma, kappa, g, s, e)]
        assert arrs[0].numel() == self.n_elem[i] and arrs[1].numel() == self.n_elem[i]
        assert all(a.numel() == self.n_e[i] for a in arrs[2:])
        L.p4d_batch_upload(self.batch, i, *arrs)
        torch.cuda.current_stream().synchronize()
        self.opts = None

    def setup(self, **kw):
        o = L.SolveOpts.from_buffer_copy(self.ws_opts)
        for k, v in kw.items():
            setattr(o, k, v)
        L.p4d_batch_setup(self.batch, o)
        self.opts = o
        return self

    def autotune(self):
        """Level-0 smoother tiles per distinct cell geometry: [(TX, CZ)] per cell."""
        return L.p4d_batch_autotune(self.batch, self.n)

    def _opts(self, kw):
        if self.opts is None:
            raise RuntimeError("call setup() first")
        o = L.SolveOpts.from_buffer_copy(self.opts)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def solve(self, bs, **kw):
        """x_i = A_i^-1 b_i for all cells; returns (list of x, list of SolveInfo)."""
        bs = [self._dev(b) for b in bs]
        assert len(bs) == self.n and all(b.numel() == n for b, n in zip(bs, self.N))
        xs = [torch.empty_like(b) for b in bs]
        _, infos = L.p4d_batch_solve(self.batch, bs, xs, self._opts(kw))
        return xs, infos

    def solve_cell(self, i, b, **kw):
        """The same cell solved alone (single-cell driver on the cell's context)."""
        b = self._dev(b)
        x = torch.empty_like(b)
        _, info = L.p4d_solve(self.cells[i], b, x, self._opts(kw))
        return x, info

    def apply(self, i, x):
        x = self._dev(x)
        y = torch.empty_like(x)
        L.p4d_apply_operator(self.cells[i], 0, x, y)
        return y

    def set_pc_mode(self, mode: int):
        """0: batched stage launches, one per stage depth (default); 1: per-cell
        launches; 2: one persistent launch per preconditioner application."""
        L.p4d_batch_set_pc_mode(self.batch, mode)

    def profile(self, class_mask: int):
        L.p4d_batch_profile(self.batch, class_mask)

    def profile_read(self, kernel_class: int):
        return L.p4d_batch_profile_read(self.batch, kernel_class)

    def close(self):
        if getattr(self, "batch", None):
            torch.cuda.synchronize()
            L.p4d_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PhysCell:
    """The physical cube cell (``p4d_inputs.phys.PhysCase``): backward-Euler
    steps of the P4D-DFN model by Newton iterations on the GPU
    (``p4d_phys_*`` in the C ABI).  States are SI-unit device vectors in the
    global layout."""

    def __init__(self, case, current: float, restart: int = 30, pc_prec: int = L.P4D_FP64,
                 coarse_max: int = 64, device: str = "cuda"):
        self.device = torch.device(device)
        self.case = case
        self.params = L.phys_params(case, current)
        self.ctx = L.p4d_phys_create(self.params)
        self.N, self.offsets, self.n_elem, self.n_e = L.p4d_vector_size(self.ctx)
        self.ws_opts = L.default_opts(restart=restart, pc_prec=pc_prec, coarse_max=coarse_max)
        nbytes = L.p4d_workspace_size(self.ctx, self.ws_opts)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        L.p4d_set_workspace(self.ctx, self.ws.data_ptr(), nbytes, self.ws_opts)
        pbytes = L.p4d_phys_workspace_size(self.ctx)
        self.pws = torch.empty(pbytes, dtype=torch.uint8, device=self.device)
        L.p4d_phys_set_workspace(self.ctx, self.pws.data_ptr(), pbytes)
        if getattr(case, "eps_s_e", None) is not None:
            self.set_fractions(case.eps_s_e, case.eps_b_e)

    def set_fractions(self, eps_s=None, eps_b=None):
        """Case II volume fractions per element (None, None: homogeneous)."""
        a = None if eps_s is None else self._dev(eps_s)
        b = None if eps_b is None else self._dev(eps_b)
        if any(t is not None and t.numel() != self.n_elem for t in (a, b)):
            raise ValueError(f"volume fractions need {self.n_elem} values per element")
        L.p4d_phys_set_fractions(self.ctx, a, b)

    def _dev(self, a):
        if isinstance(a, torch.Tensor):
            return a.to(self.device, torch.float64).contiguous()
        return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()

    def initial_state(self):
        u = torch.empty(self.N, dtype=torch.float64, device=self.device)
        L.p4d_phys_initial_state(self.ctx, u)
        return u

    def jacobian_apply(self, u, x, transpose=False):
        """J(u) x (J^T x) in the scaled variables of the Newton system."""
        y = torch.empty(self.N, dtype=torch.float64, device=self.device)
        L.p4d_phys_jacobian_apply(self.ctx, self._dev(u), transpose, self._dev(x), y)
        return y

    def residual(self, u, u_old):
        r = torch.empty(self.N, dtype=torch.float64, device=self.device)
        L.p4d_phys_residual(self.ctx, self._dev(u), self._dev(u_old), r)
        return r

    def step(self, u_old, guess=None, maxit: int = 30, tol: float = 1e-9, **solve):
        """One backward-Euler step from u_old; returns (u, NewtonInfo)."""
        u_old = self._dev(u_old)
        u = (self._dev(guess) if guess is not None else u_old).clone()
        o = self.ws_opts.__class__.from_buffer_copy(self.ws_opts)
        for k, v in solve.items():
            setattr(o, k, v)
        _, info = L.p4d_phys_newton_step(self.ctx, u, u_old, o, L.NewtonOpts(maxit, tol))
        return u, info

    def close(self):
        if getattr(self, "ctx", None):
            L.p4d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
