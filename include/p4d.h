/*
 * p4d.h -- C ABI of the MI355X (gfx950) solver for one linearized pseudo-4D
 * DFN (Doyle-Fuller-Newman) Jacobian system, after arXiv 2602.07225
 * ("Scalable Preconditioners for the Pseudo-4D DFN Lithium-ion Battery
 * Model").
 *
 * The system (paper Sec. 4.1, eq. blocks) couples, on a structured Q1 hex
 * node grid, the solid potential phi_s (electrode nodes), the electrolyte
 * potential phi_e and concentration c_e (all nodes) with one radial particle
 * concentration profile c_s of N_r points per electrode node (Sec. 3.1,
 * eq. FD).  It is solved by restarted flexible GMRES (Sec. 4.2) with a block
 * preconditioner: exact tridiagonal eliminations of the particle blocks
 * (element-wise block Jacobi, Sec. 4.2), coupled back to the macro fields
 * through the particle surface, and one multigrid V-cycle per
 * electrode-level field.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are DEVICE pointers (HIP global memory) of the GPU
 *    that is current when the call is made; all other pointers are host
 *    pointers.  Device arrays are FP64 unless stated otherwise.
 *  - Every call only enqueues work on `stream` (a hipStream_t, passed as
 *    void* so this header needs no HIP include) except where stated: calls
 *    that must read device results (setup, solve) synchronize that stream.
 *  - The caller owns all memory it passes in.  The library keeps no pointer
 *    to caller arrays after a call returns, except the workspace given to
 *    p4d_set_workspace, which must stay valid and untouched until the
 *    context is destroyed or another workspace is set.
 *  - Errors are reported by status codes only; argument checks happen before
 *    any device work is enqueued.  p4d_last_error() gives a message.
 *  - A context is not thread safe; calls on one context (or on contexts
 *    sharing a workspace) must not overlap.
 *
 * Global vector layout (length N, paper block order phi_s, phi_e, c_e, c_s,
 * eq. blocks):
 *    [ phi_s (n_e) | phi_e (n_nodes) | c_e (n_nodes) |
 *      c_s anode  (N_r,a x n_ea, index r*n_ea + j) |
 *      c_s cathode(N_r,c x n_ec, index r*n_ec + j) ]
 *  node id n = i + nx*(j + ny*k); the anode holds node layers k < na, the
 *  separator na <= k < na+ns, the cathode the rest; phi_s and c_s list the
 *  anode nodes then the cathode nodes, each in node-id order; the first
 *  nx*ny phi_s entries (layer k = 0, the grounded face Gamma_n, eq. Dirichlet)
 *  are identity rows.  Element e = i + (nx-1)*(j + (ny-1)*k) spans node
 *  layers k, k+1 and is an electrode element only if both layers are.
 */
#ifndef P4D_H
#define P4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    P4D_OK = 0,
    P4D_NOT_CONVERGED = 1,      /* iteration cap reached; x holds the last iterate */
    P4D_BREAKDOWN = 2,          /* Krylov breakdown without convergence            */
    P4D_ERR_INVALID_ARG = -1,   /* bad pointer, size or option; nothing enqueued   */
    P4D_ERR_OOM = -2,           /* workspace too small                             */
    P4D_ERR_HIP = -3,           /* a HIP runtime call failed                       */
    P4D_ERR_STATE = -4,         /* call out of order (e.g. solve before setup)     */
    P4D_ERR_NONFINITE = -5      /* NaN/Inf met in the right-hand side or residual  */
} p4d_status;

typedef enum {
    P4D_PC_SCHUR = 0,   /* particle blocks eliminated exactly, field-block diagonal
                           of the Schur complement to the V-cycles                 */
    P4D_PC_BJ = 1,      /* block Jacobi, paper eq. (PJ)                            */
    P4D_PC_BGS = 2      /* block Gauss-Seidel, paper eq. (PGS), in the field ordering
                           of p4d_solve_opts.bgs_order (single cells only)         */
} p4d_pc_type;

/* Field codes of a block Gauss-Seidel ordering: the field solved at block
 * position p (p = 0 first) sits in bits [2p, 2p + 2) of bgs_order.  The
 * paper's scaling runs use (phi_e, c_s, phi_s, c_e) (Sec. 5, ordering study),
 * packed P4D_BGS_PAPER_ORDER. */
enum { P4D_F_PHIS = 0, P4D_F_PHIE = 1, P4D_F_CE = 2, P4D_F_CS = 3 };
#define P4D_BGS_PAPER_ORDER (P4D_F_PHIE | (P4D_F_CS << 2) | (P4D_F_PHIS << 4) | (P4D_F_CE << 6))

typedef enum { P4D_FP64 = 0, P4D_FP32 = 1 } p4d_prec;

/* Krylov space of the solve.  P4D_KRYLOV_SCHUR: the particle blocks are
 * eliminated exactly (A_cs,cs is block diagonal with one tridiagonal block
 * per electrode node and couples to the electrode-level fields only through
 * the surface value, paper Sec. 4.1), FGMRES runs on the Schur complement
 * S = A_yy - A_ys A_ss^-1 A_sy over [phi_s | phi_e | c_e] with the SCHUR-mode
 * V-cycles as preconditioner, and c_s follows by back-substitution.  The
 * stopping rule and the reported true residual refer to the whole system.
 * Needs pc = P4D_PC_SCHUR. */
typedef enum { P4D_KRYLOV_FULL = 0, P4D_KRYLOV_SCHUR = 1 } p4d_krylov;

/* Multigrid smoothing of the field blocks.  P4D_SMOOTH_CHEB: Chebyshev on
 * diag(S)^-1 S of degree cheb_degree, full coarsening.  P4D_SMOOTH_ZLINE:
 * symmetric block Gauss-Seidel over the z-lines of each box (lines coloured
 * by the parity of x and y; colours 0..3 before the coarse correction, 3..0
 * after; cheb_degree passes each), coarsening in x and y only: robust when
 * the elements are much thinner along z than across, as in the flattened
 * jelly roll of paper Sec. 5 (Case III), where point smoothers stall.  FP64
 * preconditioner, pc SCHUR or BJ; either Krylov space; at most 2016 node
 * layers (p4d_setup returns P4D_ERR_INVALID_ARG above).                   */
typedef enum { P4D_SMOOTH_CHEB = 0, P4D_SMOOTH_ZLINE = 1 } p4d_smoother;

/* Problem geometry and scalars, all nondimensional.  The particle radius is
 * scaled to 1; Ds = D_s dt / R_s^2; theta_bar = last/first radial interval. */
typedef struct {
    int32_t nx, ny, nz;        /* node counts, nx, ny >= 2, nz >= 5              */
    int32_t na, ns;            /* anode and separator node layers (na >= 2)      */
    int32_t nr[2];             /* radial points per particle, anode/cathode, 3..64 */
    double Ds[2];              /* particle diffusivity, anode/cathode            */
    double theta_bar[2];       /* radial grading, (0, 1]                          */
    double dt;                 /* backward-Euler step                             */
    double chi;                /* diffusion-potential factor 2(1 - t+)            */
    double tc;                 /* electrolyte source factor (1 - t+)              */
    double lambda_c;           /* scale of the surface coupling                   */
    double eps_elec, eps_sep;  /* porosity in electrode and separator elements    */
    double length;             /* cell edge along z: h = length / (nz - 1); 0: 1  */
    double lambda_el[2];       /* surface coupling scale per electrode; 0 keeps
                                  lambda_c                                        */
    double hxy[2];             /* element edges along x and y; 0: h (cubes).  Box
                                  elements take the Q1 stiffness sum_d (vol /
                                  h_d^2) Khat_d and the mass vol Mhat; the
                                  operator then runs one thread per node, and
                                  block Gauss-Seidel (P4D_PC_BGS),
                                  p4d_param_gradient and batches do not apply   */
} p4d_problem_desc;

typedef struct {
    int32_t pc;            /* p4d_pc_type                                         */
    int32_t pc_prec;       /* p4d_prec of the preconditioner (radial + V-cycle)   */
    int32_t restart;       /* FGMRES restart length m, 1..64                      */
    int32_t maxit;         /* cap on total inner iterations                       */
    int32_t cheb_degree;   /* Chebyshev smoothing degree, 1..4 (default 2)        */
    int32_t coarse_max;    /* dense coarse solve at <= this many nodes, 8..1024   */
    int32_t cgs2;          /* 1: Gram-Schmidt applied twice                       */
    int32_t z_fp32;        /* 1: store the preconditioned basis Z in FP32         */
    double rtol;           /* stop when ||b - A x|| <= rtol ||b||                 */
    int32_t bgs_order;     /* P4D_PC_BGS: packed field ordering (see above); fixed
                              at p4d_setup, a solve must pass the same value     */
    int32_t krylov;        /* p4d_krylov; may differ between solves             */
    int32_t smoother;      /* p4d_smoother (default P4D_SMOOTH_CHEB)              */
} p4d_solve_opts;

typedef struct {
    int32_t iters, restarts, status;
    double relres_est;     /* Givens estimate at exit                             */
    double relres_true;    /* true residual ||b - A x|| / ||b|| at exit           */
    double t_setup_ms, t_solve_ms;
} p4d_solve_info;

typedef struct p4d_ctx p4d_ctx;

/* Fill opts with the defaults: SCHUR, FP64, restart 30, maxit 1000, Chebyshev
 * degree 2, coarse_max 64, one Gram-Schmidt pass, FP64 Z, rtol 1e-8, block
 * Gauss-Seidel ordering P4D_BGS_PAPER_ORDER, full Krylov space.            */
void p4d_default_opts(p4d_solve_opts *opts);

/* Create a context for the problem `desc` on the current device.  Computes
 * the per-electrode radial tables (mesh after Remark 3.1, rows of eq. L0, L1,
 * L2, LR; the shared factorization of the backward-Euler radial matrix).
 * Errors: INVALID_ARG for inconsistent sizes.                               */
p4d_status p4d_create(const p4d_problem_desc *desc, p4d_ctx **out);
void p4d_destroy(p4d_ctx *ctx);

/* Sizes: n_dof = N; offsets[0..5] = start of phi_s, phi_e, c_e, c_s anode,
 * c_s cathode, and N.  n_elem = (nx-1)(ny-1)(nz-1), n_e = electrode nodes.  */
p4d_status p4d_vector_size(const p4d_ctx *ctx, int64_t *n_dof, int64_t offsets[6],
                           int64_t *n_elem, int64_t *n_e);

/* Bytes of device workspace needed for the given options (NULL = defaults;
 * the largest restart and precision that will be used must be passed).     */
p4d_status p4d_workspace_size(const p4d_ctx *ctx, const p4d_solve_opts *opts,
                              size_t *bytes);
/* Hand the context a device workspace of at least p4d_workspace_size(opts)
 * bytes; opts (NULL = defaults) are the options it was sized for and fix its
 * layout: later solves may use a restart length up to opts->restart; a
 * workspace sized with z_fp32 = 1 holds only an FP32 Z basis, one sized with
 * z_fp32 = 0 holds either; a setup with another pc_prec or coarse_max re-lays
 * the preconditioner part if it still fits.  Invalidates earlier uploads and
 * setup.                                                                    */
p4d_status p4d_set_workspace(p4d_ctx *ctx, void *d_work, size_t bytes,
                             const p4d_solve_opts *opts);

/* Copy the linearization coefficients into the workspace (assemble/upload
 * the Jacobian, Sec. 4.1).  d_sigma, d_kappa: per element, solid and
 * electrolyte conductivity (sigma is read on electrode elements only);
 * d_g, d_s, d_e: per electrode node (phi_s order), derivatives of the
 * reaction term a*i_n (Butler-Volmer, Sec. 2.4) with respect to the
 * overpotential, the particle surface concentration and c_e.              */
p4d_status p4d_upload(p4d_ctx *ctx, const double *d_sigma, const double *d_kappa,
                      const double *d_g, const double *d_s, const double *d_e,
                      void *stream);

/* Replace the particle diffusivities Ds[2] (host array, anode/cathode) of the
 * problem: recomputes the radial tables (eq. FD rows and their shared
 * factorization) and copies them to the device on `stream`; invalidates the
 * last setup.                                                               */
p4d_status p4d_set_diffusivity(p4d_ctx *ctx, const double Ds[2], void *stream);

/* Build the preconditioner (surface-coupling weights, Galerkin multigrid
 * hierarchies, Chebyshev bounds, dense coarse inverses) on `stream`.  Returns
 * without waiting for its kernels: the Chebyshev bounds reach the host at
 * the first use of the preconditioner (p4d_solve, p4d_solve_adjoint,
 * p4d_apply_preconditioner, p4d_autotune, batch solves), which then reports
 * a non-positive or non-finite bound as P4D_ERR_NONFINITE.                  */
p4d_status p4d_setup(p4d_ctx *ctx, const p4d_solve_opts *opts, void *stream);

/* Separate element coefficients (device, one per element, caller-owned, read
 * during the call) of the electrolyte equations (paper Sec. 2, eq. phie-weak
 * and ce-weak): d_kappa_d for the diffusion-potential block (phi_e row, c_e
 * column; kappa_eff 2RT(1 - t+)/(F c_e) in the physical model) and d_dce for
 * the c_e diffusion (D_e_eff).  NULL keeps the default (chi * kappa, and
 * kappa, the operator of p4d_upload); both NULL restores it.  Needs
 * p4d_upload, which resets them; invalidates p4d_setup.  With separate
 * coefficients the operator runs one thread per node (also in its
 * Schur-complement form) and batches do not apply.                          */
p4d_status p4d_set_transport(p4d_ctx *ctx, const double *d_kappa_d, const double *d_dce,
                             void *stream);

/* Porosity per element for the c_e storage term (paper Sec. 2 electrolyte
 * mass balance, eq. ce-weak; Case II of Sec. 5 varies it): the element mass
 * becomes eps_e h^3 Mhat / dt.  d_eps_e: device, one value per element
 * (element ids x fastest), caller-owned, read during the call; NULL restores
 * the per-material eps_elec / eps_sep.  Values are not checked (a
 * non-positive porosity leaves S_ce indefinite).  Needs p4d_upload, which
 * resets it; invalidates p4d_setup.  As with p4d_set_transport the operator
 * then runs one thread per node and batches do not apply; every
 * preconditioner and Krylov space does.  INVALID_ARG on a
 * physical cell (p4d_phys_set_fractions sets its storage).                */
p4d_status p4d_set_storage(p4d_ctx *ctx, const double *d_eps_e, void *stream);

/* d_y = A d_x, or A^T d_x if transpose (eq. blocks).  d_x, d_y: length N,
 * must not alias.  Needs p4d_upload.                                       */
p4d_status p4d_apply_operator(p4d_ctx *ctx, int transpose, const double *d_x,
                              double *d_y, void *stream);

/* d_w = S d_y (S^T d_y if transpose), S = A_yy - A_ys A_ss^-1 A_sy the Schur
 * complement of the particle blocks (see p4d_krylov), formed as A_diff,yy +
 * sum_j omega_j a_j b_j^T with omega_j = 1/(1 + Gamma s_j (T0^-1)_NN).  d_y,
 * d_w: device, length off_cs[0] (the electrode-level unknowns), must not
 * alias.  Needs p4d_upload.                                                */
p4d_status p4d_apply_schur_operator(p4d_ctx *ctx, int transpose, const double *d_y,
                                    double *d_w, void *stream);

/* d_z = P^-1 d_r (P^-T if transpose) with the preconditioner of the last
 * p4d_setup (in its precision; d_r and d_z stay FP64).  Needs p4d_setup.   */
p4d_status p4d_apply_preconditioner(p4d_ctx *ctx, int transpose, const double *d_r,
                                    double *d_z, void *stream);

/* Solve A x = b by restarted flexible GMRES from x0 = 0 (d_x is output only).
 * Synchronizes `stream`.  Returns OK, NOT_CONVERGED (x = last iterate),
 * BREAKDOWN, NONFINITE or an error.  opts: NULL = those of p4d_setup; the
 * preconditioner options (pc, pc_prec, cheb_degree, coarse_max) must match
 * the last setup.  info may be NULL.                                       */
p4d_status p4d_solve(p4d_ctx *ctx, const double *d_b, double *d_x,
                     const p4d_solve_opts *opts, p4d_solve_info *info, void *stream);

/* Adjoint solve A^T lambda = g with the transposed operator and transposed
 * preconditioner (same algorithm as p4d_solve).                            */
p4d_status p4d_solve_adjoint(p4d_ctx *ctx, const double *d_g, double *d_lambda,
                             const p4d_solve_opts *opts, p4d_solve_info *info,
                             void *stream);

/* Upload + setup + solve in one call with no workspace argument, for callers
 * that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as p4d_upload(d_sigma,
 * d_kappa, d_g, d_s, d_e) then p4d_setup(opts) then p4d_solve(d_b, d_x,
 * opts, info) on the problem of `ctx`, with the per-material operator (no
 * separate transport coefficients or per-element porosity).  The workspace
 * is carved from a device array of P4D_NOALLOC_MAX_BYTES that the library
 * holds statically, one copy per GPU until the process ends: the call makes
 * no hipMalloc, hipFree or pinned-memory allocation (only small host-heap
 * bookkeeping).  A problem whose workspace for `opts` exceeds that size is
 * rejected with P4D_ERR_OOM before any device work (p4d_workspace_size gives
 * the size, plus 256 bytes of alignment).  `ctx` itself is left as it was:
 * its workspace, uploads and setup are neither used nor changed (only its
 * error message).  All calls on one GPU share that GPU's scratch array and
 * the last call's contents stay in it: calls that overlap on one GPU (other
 * threads, other streams) race.  Nothing in it needs to start at zero.
 * Synchronizes `stream`.                                                   */
#define P4D_NOALLOC_MAX_BYTES (64u << 20)
p4d_status p4d_solve_noalloc(p4d_ctx *ctx, const double *d_sigma, const double *d_kappa,
                             const double *d_g, const double *d_s, const double *d_e,
                             const double *d_b, double *d_x, const p4d_solve_opts *opts,
                             p4d_solve_info *info, void *stream);

/* Gradients of J = w.x for A x = b, given x and lambda = A^-T w:
 * dJ/dp = -lambda^T (dA/dp) x.  d_dsigma: per element (zero on separator
 * elements); d_dDs: 2 values (anode, cathode), derivative with respect to Ds.
 * Both are device arrays.                                                  */
p4d_status p4d_param_gradient(p4d_ctx *ctx, const double *d_x, const double *d_lambda,
                              double *d_dsigma, double *d_dDs, void *stream);

/* Kernel timing with HIP events recorded on `stream` around every launch of
 * the kernel classes in `class_mask` (bit 1 << p4d_kernel_class; 0 switches
 * timing off and clears the totals); the level-0 smoothing steps on one side
 * of a V-cycle's coarse correction, which run back to back, share one event
 * pair (an interval of cheb_degree - 1 or cheb_degree launches).
 * P4D_K_COUPLING: the kernels around the V-cycles of the block Gauss-Seidel
 * and Schur-complement preconditioners (right-hand sides with the
 * off-diagonal blocks, precision casts, output).                          */
typedef enum {
    P4D_K_OPERATOR = 1, P4D_K_MDOT = 2, P4D_K_ORTH = 3, P4D_K_RADIAL = 4,
    P4D_K_SMOOTH0 = 5, P4D_K_ZY = 6, P4D_K_BATCH_PC = 7, P4D_K_COUPLING = 8,
    P4D_K_COUNT = 9
} p4d_kernel_class;
p4d_status p4d_profile(p4d_ctx *ctx, int class_mask);
/* Time only one interval (event pair) in `every` (>= 1, default 1) of each
 * class in the mask, counted per class from this call or the last
 * p4d_profile: fewer event pairs on the stream while the average over the
 * timed launches stays that of the class (a pair costs a few microseconds
 * of the stream's time).  The totals of p4d_profile_read then cover the
 * launches of the timed intervals only.                                    */
p4d_status p4d_profile_every(p4d_ctx *ctx, int every);
/* For one class: total_ms = summed kernel durations, launches, and bytes =
 * algorithmic bytes of those launches (the data each launch must read and
 * write once).                                                              */
p4d_status p4d_profile_read(p4d_ctx *ctx, int kernel_class, double *total_ms,
                            int64_t *launches, double *bytes);

const char *p4d_status_string(p4d_status s);
const char *p4d_last_error(const p4d_ctx *ctx);

/* Level-0 smoother tile autotuning: times one Chebyshev step over the four
 * multigrid boxes for each tile shape TX x (256/TX) nodes by CZ layers,
 * TX in {16, 32, 64}, 2 <= CZ <= 16, and keeps the fastest for this context
 * (without it, CZ is chosen from the grid and the number of resident
 * workgroups).  Needs p4d_setup; synchronizes `stream`; only preconditioner
 * buffers are written.  tile (host, may be NULL) receives {TX, CZ}.        */
p4d_status p4d_autotune(p4d_ctx *ctx, void *stream, int32_t tile[2]);

/* ---------------------------------------------------------------------------
 * Batched solves: up to 64 independent cells, each with its own mesh, radial
 * sizes, coefficients and right-hand side, solved together by FGMRES
 * iterating in lockstep.  Per Arnoldi step the preconditioner of every
 * iterating cell is applied by one launch per stage depth (stage d of all
 * cells in one work list of tiles and blocks; the same stages and arithmetic
 * as the single-cell path), followed by batched operator, Gram-Schmidt and
 * norm kernels over the table of cells.  A cell that converges stops
 * iterating; the others go on.  Each cell is a full context
 * (p4d_batch_cell), so every single-cell call also works on it.
 *
 * Sequence: p4d_batch_create, p4d_batch_workspace_size,
 * p4d_batch_set_workspace, p4d_batch_upload (each cell), p4d_batch_setup,
 * optionally p4d_batch_autotune, then p4d_batch_solve any number of times.
 * -------------------------------------------------------------------------*/
typedef struct p4d_batch p4d_batch;

/* descs: host array of ncells problem descriptions, 1 <= ncells <= 64.      */
p4d_status p4d_batch_create(const p4d_problem_desc *descs, int32_t ncells, p4d_batch **out);
void p4d_batch_destroy(p4d_batch *batch);
/* The context of one cell (owned by the batch; valid until it is destroyed). */
p4d_status p4d_batch_cell(p4d_batch *batch, int32_t cell, p4d_ctx **out);
/* Bytes of device workspace for all cells (their contexts' workspaces) plus
 * the batch tables, for the options `opts` (NULL: defaults).                */
p4d_status p4d_batch_workspace_size(const p4d_batch *batch, const p4d_solve_opts *opts,
                                    size_t *bytes);
/* Carves d_work (device, caller-owned, kept until destroy or the next call)
 * into the cells' workspaces and the batch tables.  OOM if too small.       */
p4d_status p4d_batch_set_workspace(p4d_batch *batch, void *d_work, size_t bytes,
                                   const p4d_solve_opts *opts);
/* p4d_upload for one cell (device arrays sized for that cell).              */
p4d_status p4d_batch_upload(p4d_batch *batch, int32_t cell, const double *d_sigma,
                            const double *d_kappa, const double *d_g, const double *d_s,
                            const double *d_e, void *stream);
/* p4d_setup of every cell with the same options; these must keep the
 * preconditioner precision, coarse size and Z precision of the workspace
 * options and a restart no larger (STATE otherwise).                        */
p4d_status p4d_batch_setup(p4d_batch *batch, const p4d_solve_opts *opts, void *stream);
/* Level-0 smoother tiles of the batch: every candidate layer depth CZ
 * (2..16, the same for all cells; TX follows each cell's grid width) is
 * timed on whole batched preconditioner applications and the fastest is
 * kept (without it, CZ is chosen from the number of tiles and of resident
 * workgroups).  Synchronizes `stream`; writes only preconditioner buffers.
 * tiles (host, may be NULL) receives {TX, CZ} per cell.                     */
p4d_status p4d_batch_autotune(p4d_batch *batch, void *stream, int32_t *tiles);
/* Solves A_i x_i = b_i for every cell i.  d_b, d_x: host arrays of ncells
 * device pointers (vectors of each cell's length N_i, global layout above).
 * infos (host, may be NULL): ncells entries; t_solve_ms is the time of the
 * whole batch.  Returns OK when every cell converged, else the status of the
 * first cell that did not (each cell's own status is in infos).
 * Synchronizes `stream` once per Arnoldi step.                              */
p4d_status p4d_batch_solve(p4d_batch *batch, const double *const *d_b, double *const *d_x,
                           const p4d_solve_opts *opts, p4d_solve_info *infos, void *stream);
/* mode 0 (default): batched stage launches, one per stage depth; mode 1: the
 * single-cell preconditioner launches, cell after cell (a reference); mode 2:
 * one cooperative launch per application: the whole grid walks the stage
 * depths with a grid barrier between depths (P4D_ERR_HIP where the device
 * cannot launch it cooperatively).  The three give the same results bit for
 * bit.                                                                      */
p4d_status p4d_batch_set_pc_mode(p4d_batch *batch, int32_t mode);
/* Kernel timing of the batched launches, as p4d_profile / p4d_profile_read;
 * P4D_K_BATCH_PC times all preconditioner launches of one Arnoldi step
 * together and counts their level-0 and particle bytes (coarse levels not
 * counted).                                                                 */
p4d_status p4d_batch_profile(p4d_batch *batch, int class_mask);
p4d_status p4d_batch_profile_read(p4d_batch *batch, int kernel_class, double *total_ms,
                                  int64_t *launches, double *bytes);
const char *p4d_batch_last_error(const p4d_batch *batch);

/* ------------------------------------------------------------------------ */
/* Physical cell: the Newton step around the linear solve (paper Sec. 4.1)   */
/* for the cube cell of Sec. 5 (Case I) with the model of Sec. 2 and the     */
/* appendix parameters: Butler-Volmer kinetics with the open-circuit         */
/* potentials, kappa(c_e), D_e(c_e), Bruggeman corrections, the Gaussian     */
/* (or uniform) applied current on the top face; Case II volume fractions   */
/* per element by p4d_phys_set_fractions.  The state u is in SI units (V, V,       */
/* mol/m^3, mol/m^3) in the global layout above.  The context's linear       */
/* operator is the Newton matrix in scaled variables (unknowns divided and   */
/* equations multiplied by per-field scales), with transport coefficients   */
/* at the element-mean c_e of the current iterate; p4d_solve and the other  */
/* linear calls work on it as on any context.                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double eps_s;      /* active material volume fraction                     */
    double eps;        /* porosity (the same in both electrodes)              */
    double sigma;      /* solid conductivity, S/m                             */
    double k;          /* reaction rate constant                              */
    double alpha;      /* anodic = cathodic charge-transfer coefficient       */
    double cs_max, cs0;/* maximum and initial solid concentration, mol/m^3    */
    double a;          /* specific interfacial area, 1/m                      */
    double Ds;         /* solid diffusivity, m^2/s                            */
    double Rs;         /* particle radius, m                                  */
} p4d_electrode;

typedef struct {
    int32_t n;            /* nodes per edge of the cube: n - 1 a multiple of 9, >= 18
                             (negative 4/9, separator 1/9, positive 4/9 of the edge) */
    int32_t nr[2];        /* radial points, negative / positive, 3..64           */
    double theta_bar[2];  /* radial grading                                      */
    double dt;            /* backward-Euler step, s                              */
    double current;       /* applied current, A (negative: discharge, the current
                             leaves through the top face)                        */
    double gauss_frac;    /* spread of the Gaussian current profile / cube edge  */
    double edge;          /* cube edge, m                                        */
    double F, R, T;       /* Faraday constant, gas constant, temperature         */
    double t_plus, brug;  /* transference number, Bruggeman exponent            */
    double ce0;           /* initial electrolyte concentration, mol/m^3          */
    double eps_sep;       /* separator porosity                                  */
    p4d_electrode el[2];  /* negative (bottom, grounded), positive (top)         */
    int32_t profile;      /* applied current over the top face: 0 Gaussian, 1
                             uniform (Case II)                                   */
} p4d_phys_params;

typedef struct {
    int32_t maxit;        /* Newton iterations per step (default 30)             */
    double tol;           /* stop when max |du_f| / scale_f <= tol (RT/F for the
                             potentials, c_e0, c_s,max per electrode); 1e-9      */
} p4d_newton_opts;

typedef struct {
    int32_t iters;        /* Newton iterations taken                             */
    int32_t status;       /* 0 converged, 1 not converged, else a p4d_status     */
    int32_t lin_iters;    /* FGMRES iterations summed over the step              */
    double update;        /* the last scaled update                              */
    double t_ms;          /* wall time of the step                               */
} p4d_newton_info;

/* Context for the cube cell described by prm (validated: INVALID_ARG).      */
p4d_status p4d_phys_create(const p4d_phys_params *prm, p4d_ctx **ctx);
/* Device bytes of the Newton buffers (four state-sized vectors and two per
 * electrode node), beyond p4d_workspace_size.                               */
p4d_status p4d_phys_workspace_size(const p4d_ctx *ctx, size_t *bytes);
/* Hands the context its Newton buffers (device, caller-owned, kept until
 * destroy); needs p4d_set_workspace first.                                  */
p4d_status p4d_phys_set_workspace(p4d_ctx *ctx, void *d_work, size_t bytes);
/* Case II (Sec. 5): active-material and binder volume fractions per element
 * (device, element ids x fastest, caller-owned, read during the call;
 * separator entries ignored).  sigma_eff takes eps_s^brug, kappa_eff, D_e_eff
 * and the c_e storage the porosity 1 - eps_s - eps_b (brug for the
 * transport); the specific area keeps el[].a.  Both NULL restores the
 * homogeneous cell.  INVALID_ARG if only one is NULL or if a fraction is
 * outside (0, 1) or no porosity is left (the cell is then homogeneous).
 * Needs p4d_phys_set_workspace, which resets it; synchronizes `stream`.    */
p4d_status p4d_phys_set_fractions(p4d_ctx *ctx, const double *d_eps_s, const double *d_eps_b,
                                  void *stream);
/* d_u = the rest state: c_e0, c_s0 and zero overpotential (phi_s = 0 in the
 * negative electrode, phi_e = -U_n, phi_s = U_p - U_n in the positive one). */
p4d_status p4d_phys_initial_state(p4d_ctx *ctx, double *d_u, void *stream);
/* d_r = R(d_u), the residual of the backward-Euler step from d_uold in SI
 * units per row (phi rows in A, c_e rows in mol/s, c_s rows in mol/(m^3 s);
 * grounded phi_s rows: phi_s).  Leaves the Newton matrix at d_u in the
 * context.                                                                 */
p4d_status p4d_phys_residual(p4d_ctx *ctx, const double *d_u, const double *d_uold, double *d_r,
                             void *stream);
/* d_y = J(d_u) d_x (J^T if transpose): the Newton matrix of the cell at the
 * state d_u in the scaled variables (D_r J D_c, see above), with the
 * c_e-derivatives of the transport coefficients; d_x, d_y length N, must not
 * alias.  Leaves the coefficients of d_u in the context.                   */
p4d_status p4d_phys_jacobian_apply(p4d_ctx *ctx, const double *d_u, int transpose, const double *d_x,
                                   double *d_y, void *stream);
/* One backward-Euler step from d_uold: Newton iterations from the guess in
 * d_u (overwritten with the result), each a p4d_setup and an FGMRES solve of
 * the scaled Newton system (the exact Jacobian; its preconditioner is built
 * from the transport coefficients at the iterate without their
 * c_e-derivatives) with solve (may be NULL: defaults; either Krylov space),
 * until the scaled update meets newton->tol.
 * Synchronizes `stream` once per iteration.                                */
p4d_status p4d_phys_newton_step(p4d_ctx *ctx, double *d_u, const double *d_uold,
                                const p4d_solve_opts *solve, const p4d_newton_opts *newton,
                                p4d_newton_info *info, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* P4D_H */
