/*
 * Plain FP64 CPU oracle for one linearized pseudo-4D DFN Jacobian solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU library: the two
 * meet only through the seeded input arrays.
 *
 * It is written for a reader holding the paper (arXiv 2602.07225), favouring
 * plain loops over speed.  Sections and equations cited:
 *
 *   Sec. 3.1   radial finite differences: eq. (L1), (L2), (Lh), (L0), (LR),
 *              (FD); the geometric radial mesh after Remark 3.1.
 *   Sec. 3.2   Q1 finite elements for c_e, phi_e, phi_s: the weak forms
 *              (ce-weak), (phie-weak), (phis-weak); Dirichlet phi_s = 0 on
 *              Gamma_n (eq. Dirichlet).
 *   Sec. 3.3   backward Euler.
 *   Sec. 4.1   block residual and 4x4 block Jacobian (eq. blocks), c_s
 *              block-diagonal with one tridiagonal N_c x N_c block per point.
 *   Sec. 4.2   block preconditioners: block Jacobi (eq. PJ), block
 *              Gauss-Seidel in any of the 24 field orderings (eq. PGS, the
 *              ordering study of Sec. 5); multigrid for the electrode-level
 *              blocks; exact element-wise block Jacobi (tridiagonal solves)
 *              for c_s.
 *
 * Readings where the paper is silent or ambiguous (each also listed in the
 * design notes of the repository):
 *   - c_s lives on electrode NODES with a lumped reaction weight m_j;
 *   - the surface flux term of eq. (LR) enters with the sign implied by the
 *     boundary condition eq. (particleBC2), i.e. +Gamma*q in the c_s surface
 *     row of the Jacobian;
 *   - radial grading: Delta_{N-1} / Delta_1 = theta_bar (refined to surface);
 *   - SCHUR preconditioner mode: the c_s blocks are eliminated exactly and
 *     the field-block diagonal of the resulting Schur complement is given to
 *     the V-cycles (mode BJ is the paper's eq. (PJ));
 *   - geometric Galerkin multigrid V(2,2) with degree-2 Chebyshev smoothing
 *     on diag(S)^-1 S over [lmax/4, lmax], lmax the Gershgorin bound, dense
 *     Cholesky at <= 512 nodes, in place of BoomerAMG;
 *   - restarted right-preconditioned flexible GMRES, classical Gram-Schmidt;
 *   - optionally FGMRES over the Schur complement of the c_s blocks only
 *     (not a variant the paper runs: an algebraic consequence of the block
 *     structure of Sec. 4.1, exact up to rounding), with the SCHUR-mode
 *     V-cycles as its preconditioner.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads an OpenMP region of the oracle uses (1 without OpenMP) */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Problem description (mirrors p4d_inputs.Problem)                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, nz, na, ns;
    int32_t nr[2];
    double Ds[2];          /* nondimensional particle diffusivity per electrode */
    double theta_bar[2];   /* radial grading Delta_{N-1}/Delta_1                */
    double dt, chi, tc, lambda_c, eps_elec, eps_sep;
    double length;         /* cell edge along z (h = length / (nz - 1)); 0: 1   */
    double lambda_el[2];   /* surface coupling scale per electrode; 0: lambda_c */
    double hxy[2];         /* element edges along x and y; 0: h (isotropic)     */
} orc_desc;

enum { ORC_PC_SCHUR = 0, ORC_PC_BJ = 1, ORC_PC_BGS = 2 };

/* fields of the 4x4 block system, as numbered in a block ordering           */
enum { ORC_F_PHIS = 0, ORC_F_PHIE = 1, ORC_F_CE = 2, ORC_F_CS = 3 };

typedef struct {
    int32_t pc;            /* ORC_PC_SCHUR, ORC_PC_BJ or ORC_PC_BGS             */
    int32_t restart;       /* FGMRES restart length m                          */
    int32_t maxit;         /* total inner iterations                           */
    int32_t cgs2;          /* 1: classical Gram-Schmidt applied twice           */
    double rtol;
    int32_t coarse_max;    /* direct solve once a grid has <= this many nodes */
    int32_t cheb_degree;
    int32_t bgs_order;     /* BGS: field at block position p is bits [2p, 2p+2) */
    int32_t krylov;        /* ORC_KRYLOV_FULL or ORC_KRYLOV_SCHUR               */
    int32_t smoother;      /* ORC_SMOOTH_CHEB or ORC_SMOOTH_ZLINE              */
} orc_opts;

/* Multigrid smoothing: Chebyshev on diag(S)^-1 S with full coarsening, or
 * symmetric block Gauss-Seidel over the z-lines of the box (four colours of
 * lines by the parity of x and y) with coarsening in x and y only.          */
enum { ORC_SMOOTH_CHEB = 0, ORC_SMOOTH_ZLINE = 1 };

/* Krylov space: all unknowns, or the electrode-level unknowns of the Schur
 * complement left when the c_s blocks are eliminated exactly (SCHUR mode). */
enum { ORC_KRYLOV_FULL = 0, ORC_KRYLOV_SCHUR = 1 };

typedef struct {
    int32_t iters, restarts, status;   /* status 0 converged, 1 not, 2 breakdown */
    double relres_est, relres_true;
} orc_info;

/* one multigrid level: a node box with a stored 27-point stencil            */
typedef struct {
    int nx, ny, nz;
    long n;
    double *S;      /* [n][27], offset o = (dx+1) + 3(dy+1) + 9(dz+1)          */
    double lmax;    /* Gershgorin bound of diag(S)^-1 S                        */
    double *L;      /* coarsest only: dense Cholesky factor (row-major, lower) */
} orc_level;

typedef struct {
    int nlev;
    orc_level lev[16];
} orc_mg;

typedef struct {
    orc_desc d;
    double h;              /* element edge along z                          */
    double hx, hy, vol;    /* edges along x and y, element volume            */
    int aniso;             /* hx or hy differs from h                        */
    double kw[3];          /* stiffness weights vol / (h_d^2 h) per axis     */
    int nc;
    long nnode, nelem, nea, nec, ne;
    long off_ps, off_pe, off_ce, off_cs[2], N;
    double *sigma, *kappa, *g, *s, *e, *m;
    /* optional element coefficients of the diffusion-potential block and of
     * the c_e diffusion (NULL: chi * kappa and kappa)                       */
    double *kappad, *dce;
    double *epse;              /* porosity per element (NULL: per material) */
    /* Newton terms: state phi_e and c_e per node, per element the
     * c_e-derivatives of kappa_eff, of the diffusion-potential coefficient
     * and of D_eff (NULL: off)                                              */
    double *nw_up, *nw_uc, *nw_a, *nw_b, *nw_c;
    /* radial: node coordinates and rows of L~_h (flux term excluded) */
    double *rho[2], *Lsub[2], *Ldia[2], *Lsup[2];
    double Gamma[2];
    /* preconditioner */
    int pc_ready, pc_type;
    orc_opts opts;
    double *omega;         /* per electrode node                            */
    orc_mg mg[4];          /* boxes: 0 phi_s anode, 1 phi_s cathode, 2 phi_e, 3 c_e */
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int popc3(int v) { return (v & 1) + ((v >> 1) & 1) + ((v >> 2) & 1); }

/* Q1 reference element on the unit cube, local node a = bx | by<<1 | bz<<2.
 * Stiffness int grad(phi_a).grad(phi_b) and mass int phi_a phi_b; both depend
 * only on how many coordinates the two corners differ in.                    */
static double khat(int a, int b)
{
    switch (popc3(a ^ b)) {
    case 0: return 1.0 / 3.0;
    case 1: return 0.0;
    default: return -1.0 / 12.0;
    }
}
static double mhat(int a, int b)
{
    switch (popc3(a ^ b)) {
    case 0: return 1.0 / 27.0;
    case 1: return 1.0 / 54.0;
    case 2: return 1.0 / 108.0;
    default: return 1.0 / 216.0;
    }
}

static void *xmalloc(size_t n)
{
    void *p = calloc(1, n ? n : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

/* material of an element layer kk: 0 anode, 1 cathode, -1 separator         */
static int elem_mat(const orc_problem *P, int kk)
{
    if (kk + 1 < P->d.na) return 0;
    if (kk >= P->d.na + P->d.ns) return 1;
    return -1;
}
/* material of a node layer k                                               */
static int node_mat(const orc_problem *P, int k)
{
    if (k < P->d.na) return 0;
    if (k >= P->d.na + P->d.ns) return 1;
    return -1;
}
/* electrode-node index (phi_s / c_s numbering) of node (i,j,k), -1 if none */
static long enode(const orc_problem *P, int i, int j, int k)
{
    int nx = P->d.nx, ny = P->d.ny;
    if (k < P->d.na) return i + (long)nx * (j + (long)ny * k);
    if (k >= P->d.na + P->d.ns)
        return P->nea + i + (long)nx * (j + (long)ny * (k - P->d.na - P->d.ns));
    return -1;
}
static long node_id(const orc_problem *P, int i, int j, int k)
{
    return i + (long)P->d.nx * (j + (long)P->d.ny * k);
}
static long elem_id(const orc_problem *P, int i, int j, int k)
{
    return i + (long)(P->d.nx - 1) * (j + (long)(P->d.ny - 1) * k);
}
static int is_dirichlet(const orc_problem *P, int k) { (void)P; return k == 0; }

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: radial mesh and finite-difference rows                          */
/* ------------------------------------------------------------------------ */
/* Geometric mesh on [0,1]: Delta_i = Delta_1 q^(i-1), q = theta_bar^(1/(N-2)),
 * sum of the N-1 intervals = 1.                                             */
void orc_radial_mesh(int N, double theta_bar, double *rho)
{
    double q = pow(theta_bar, 1.0 / (double)(N - 2));
    double sum = 0.0, dq = 1.0;
    for (int i = 0; i < N - 1; i++) { sum += dq; dq *= q; }
    double d1 = 1.0 / sum;
    rho[0] = 0.0;
    dq = d1;
    for (int i = 1; i < N; i++) { rho[i] = rho[i - 1] + dq; dq *= q; }
    rho[N - 1] = 1.0;
}

/* Rows of the discrete radial operator L_h for c (0-based r = 0..N-1):
 *   r = 0      eq. (L0):  6D/Delta_1^2 (c_2 - c_1)
 *   0<r<N-1    eq. (L1)+(L2) with theta = Delta_r / Delta_{r-1}
 *   r = N-1    eq. (LR) without its flux term: 2D/Delta^2 (c_{N-1} - c_N)
 * Returns the flux-term factor multiplying i_n/F in row N-1 of L_h with the
 * sign taken from (particleBC2): -2/Delta (1 + Delta/R), R = 1.            */
double orc_radial_rows(int N, double D, const double *rho,
                       double *sub, double *dia, double *sup)
{
    for (int r = 0; r < N; r++) sub[r] = dia[r] = sup[r] = 0.0;
    double d1 = rho[1] - rho[0];
    dia[0] = -6.0 * D / (d1 * d1);
    sup[0] = 6.0 * D / (d1 * d1);
    for (int r = 1; r < N - 1; r++) {
        double dm = rho[r] - rho[r - 1];       /* Delta r_{i-1} */
        double dp = rho[r + 1] - rho[r];       /* Delta r_i     */
        double th = dp / dm;
        /* L1: 2D/r_i * (c_{i+1} - th^2 c_{i-1} - (1-th^2) c_i) / (dp (1+th)) */
        double f1 = 2.0 * D / (rho[r] * dp * (1.0 + th));
        double l1_m = -th * th * f1, l1_0 = -(1.0 - th * th) * f1, l1_p = f1;
        /* L2: 2D/(dp dm (1+th)) (c_{i+1} + th c_{i-1} - (1+th) c_i)          */
        double f2 = 2.0 * D / (dp * dm * (1.0 + th));
        double l2_m = th * f2, l2_0 = -(1.0 + th) * f2, l2_p = f2;
        sub[r] = l1_m + l2_m;
        dia[r] = l1_0 + l2_0;
        sup[r] = l1_p + l2_p;
    }
    double dl = rho[N - 1] - rho[N - 2];
    sub[N - 1] = 2.0 * D / (dl * dl);
    dia[N - 1] = -2.0 * D / (dl * dl);
    return -2.0 / dl * (1.0 + dl / 1.0);
}

/* ------------------------------------------------------------------------ */
/* Problem construction                                                      */
/* ------------------------------------------------------------------------ */
orc_problem *orc_create(const orc_desc *d, const double *sigma, const double *kappa,
                        const double *g, const double *s, const double *e)
{
    orc_problem *P = xmalloc(sizeof(orc_problem));
    P->d = *d;
    P->h = (d->length > 0.0 ? d->length : 1.0) / (d->nz - 1);
    P->hx = d->hxy[0] > 0.0 ? d->hxy[0] : P->h;
    P->hy = d->hxy[1] > 0.0 ? d->hxy[1] : P->h;
    P->aniso = P->hx != P->h || P->hy != P->h;
    P->vol = P->hx * P->hy * P->h;
    P->kw[0] = P->hy / P->hx;
    P->kw[1] = P->hx / P->hy;
    P->kw[2] = P->hx * P->hy / (P->h * P->h);
    P->kappad = NULL;
    P->dce = NULL;
    P->epse = NULL;
    P->nw_up = P->nw_uc = P->nw_a = P->nw_b = P->nw_c = NULL;
    P->nc = d->nz - d->na - d->ns;
    P->nnode = (long)d->nx * d->ny * d->nz;
    P->nelem = (long)(d->nx - 1) * (d->ny - 1) * (d->nz - 1);
    P->nea = (long)d->nx * d->ny * d->na;
    P->nec = (long)d->nx * d->ny * P->nc;
    P->ne = P->nea + P->nec;
    P->off_ps = 0;
    P->off_pe = P->ne;
    P->off_ce = P->off_pe + P->nnode;
    P->off_cs[0] = P->off_ce + P->nnode;
    P->off_cs[1] = P->off_cs[0] + (long)d->nr[0] * P->nea;
    P->N = P->off_cs[1] + (long)d->nr[1] * P->nec;

    P->sigma = xmalloc(sizeof(double) * P->nelem);
    P->kappa = xmalloc(sizeof(double) * P->nelem);
    memcpy(P->sigma, sigma, sizeof(double) * P->nelem);
    memcpy(P->kappa, kappa, sizeof(double) * P->nelem);
    P->g = xmalloc(sizeof(double) * P->ne);
    P->s = xmalloc(sizeof(double) * P->ne);
    P->e = xmalloc(sizeof(double) * P->ne);
    memcpy(P->g, g, sizeof(double) * P->ne);
    memcpy(P->s, s, sizeof(double) * P->ne);
    memcpy(P->e, e, sizeof(double) * P->ne);

    /* lumped reaction weight: the node's share (1/8 of each) of the volume of
     * the electrode elements that contain it                                */
    P->m = xmalloc(sizeof(double) * P->ne);
    double h3 = P->vol;
    for (int k = 0; k < d->nz; k++)
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                long je = enode(P, i, j, k);
                if (je < 0) continue;
                int cnt = 0;
                for (int bz = 0; bz < 2; bz++)
                    for (int by = 0; by < 2; by++)
                        for (int bx = 0; bx < 2; bx++) {
                            int ei = i - 1 + bx, ej = j - 1 + by, ek = k - 1 + bz;
                            if (ei < 0 || ej < 0 || ek < 0 || ei >= d->nx - 1 ||
                                ej >= d->ny - 1 || ek >= d->nz - 1) continue;
                            if (elem_mat(P, ek) >= 0) cnt++;
                        }
                P->m[je] = h3 / 8.0 * cnt;
            }

    for (int el = 0; el < 2; el++) {
        int N = d->nr[el];
        P->rho[el] = xmalloc(sizeof(double) * N);
        P->Lsub[el] = xmalloc(sizeof(double) * N);
        P->Ldia[el] = xmalloc(sizeof(double) * N);
        P->Lsup[el] = xmalloc(sizeof(double) * N);
        orc_radial_mesh(N, d->theta_bar[el], P->rho[el]);
        double flux = orc_radial_rows(N, d->Ds[el], P->rho[el], P->Lsub[el],
                                      P->Ldia[el], P->Lsup[el]);
        /* R_cs,N = (c_N - c_N^old)/dt - L_h(c)_N contains -flux * i_n/F;
         * the nondimensional surface coupling scale is lambda_c            */
        P->Gamma[el] = -flux * (d->lambda_el[el] > 0.0 ? d->lambda_el[el] : d->lambda_c);
    }
    return P;
}

/* Element coefficients of the diffusion-potential block (kappa_d: the
 * (phi_e row, c_e column) stiffness, chi * kappa by default) and of the c_e
 * diffusion (dce: kappa by default), for transport coefficients that differ
 * (Sec. 2: kappa_eff 2RT(1 - t+)/(F c_e) and D_e_eff).  NULL keeps the
 * default.                                                                  */
void orc_set_transport(orc_problem *P, const double *kappa_d, const double *dce)
{
    free(P->kappad); free(P->dce);
    P->kappad = P->dce = NULL;
    if (kappa_d) {
        P->kappad = xmalloc(sizeof(double) * P->nelem);
        memcpy(P->kappad, kappa_d, sizeof(double) * P->nelem);
    }
    if (dce) {
        P->dce = xmalloc(sizeof(double) * P->nelem);
        memcpy(P->dce, dce, sizeof(double) * P->nelem);
    }
    P->pc_ready = 0;
}

/* Porosity per element for the c_e storage term (Sec. 2 electrolyte mass
 * balance; Case II of Sec. 5 draws it from volume-fraction fields): the
 * element mass matrix becomes eps_e h^3 Mhat / dt.  NULL restores the
 * per-material values eps_elec, eps_sep.                                    */
void orc_set_storage(orc_problem *P, const double *eps_e)
{
    free(P->epse);
    P->epse = NULL;
    if (eps_e) {
        P->epse = xmalloc(sizeof(double) * P->nelem);
        memcpy(P->epse, eps_e, sizeof(double) * P->nelem);
    }
    P->pc_ready = 0;
}

/* The c_e-derivative terms of the transport coefficients in the Newton
 * matrix at a state (Sec. 4.1: the Jacobian of the residual; the element
 * coefficients kappa_eff, kappa_eff 2RT(1-t+)/(F c) and D_eff are functions
 * of the element's mean c_e): up, uc the state's phi_e and c_e per node,
 * da, db, dc per element the derivatives of the three coefficients with
 * respect to the element mean.  All NULL removes the terms (Picard matrix).
 * The preconditioner does not use them.                                     */
void orc_set_newton(orc_problem *P, const double *up, const double *uc, const double *da,
                    const double *db, const double *dc)
{
    double **dst[5] = {&P->nw_up, &P->nw_uc, &P->nw_a, &P->nw_b, &P->nw_c};
    const double *src[5] = {up, uc, da, db, dc};
    for (int q = 0; q < 5; q++) {
        free(*dst[q]);
        *dst[q] = NULL;
    }
    if (!up) return;
    for (int q = 0; q < 5; q++) {
        long n = q < 2 ? P->nnode : P->nelem;
        *dst[q] = xmalloc(sizeof(double) * n);
        memcpy(*dst[q], src[q], sizeof(double) * n);
    }
}

static void mg_free(orc_mg *M)
{
    for (int l = 0; l < M->nlev; l++) {
        free(M->lev[l].S);
        free(M->lev[l].L);
    }
    M->nlev = 0;
}

void orc_destroy(orc_problem *P)
{
    if (!P) return;
    free(P->sigma); free(P->kappa); free(P->g); free(P->s); free(P->e); free(P->m);
    free(P->kappad); free(P->dce); free(P->epse);
    free(P->nw_up); free(P->nw_uc); free(P->nw_a); free(P->nw_b); free(P->nw_c);
    for (int el = 0; el < 2; el++) {
        free(P->rho[el]); free(P->Lsub[el]); free(P->Ldia[el]); free(P->Lsup[el]);
    }
    free(P->omega);
    for (int b = 0; b < 4; b++) mg_free(&P->mg[b]);
    free(P);
}

void orc_sizes(const orc_problem *P, int64_t *out /* [8] */)
{
    out[0] = P->off_ps; out[1] = P->off_pe; out[2] = P->off_ce;
    out[3] = P->off_cs[0]; out[4] = P->off_cs[1]; out[5] = P->N;
    out[6] = P->ne; out[7] = P->nnode;
}

void orc_radial_info(const orc_problem *P, int el, double *rho, double *sub,
                     double *dia, double *sup, double *gamma)
{
    int N = P->d.nr[el];
    memcpy(rho, P->rho[el], sizeof(double) * N);
    memcpy(sub, P->Lsub[el], sizeof(double) * N);
    memcpy(dia, P->Ldia[el], sizeof(double) * N);
    memcpy(sup, P->Lsup[el], sizeof(double) * N);
    *gamma = P->Gamma[el];
}

void orc_lumped_weights(const orc_problem *P, double *m)
{
    memcpy(m, P->m, sizeof(double) * P->ne);
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2: Q1 element sums at one node                                     */
/* ------------------------------------------------------------------------ */
/* Stiffness of a box element with edges hx, hy, hz over h: the sum over the
 * axes d of (vol / h_d^2) / h times the tensor product of the 1D stiffness
 * along d (1 on the diagonal, -1 off) with the 1D masses (1/3, 1/6) along
 * the other two; for equal edges this is khat.                              */
static double kelem(const orc_problem *P, int a, int b)
{
    if (!P->aniso) return khat(a, b);
    int p = a ^ b;
    double acc = 0.0;
    for (int d = 0; d < 3; d++) {
        double v = (p >> d) & 1 ? -1.0 : 1.0;
        for (int q = 0; q < 3; q++)
            if (q != d) v *= (p >> q) & 1 ? 1.0 / 6.0 : 1.0 / 3.0;
        acc += P->kw[d] * v;
    }
    return acc;
}

/* sum over the elements e containing node (i,j,k) that pass `use`, of
 *   coef(e) * sum_b Ahat(a,b) * x[node b]     (a = local index of the node)
 * where x is read through `xv` (returns the value at node (i,j,k)).         */
typedef double (*elem_coef_fn)(const orc_problem *, int, int, int, const void *);
typedef double (*node_val_fn)(const orc_problem *, int, int, int, const void *);

static double elem_sum(const orc_problem *P, int i, int j, int k, int stiff,
                       elem_coef_fn cf, const void *cctx, node_val_fn xv,
                       const void *xctx)
{
    const orc_desc *d = &P->d;
    double acc = 0.0;
    for (int bz = 0; bz < 2; bz++)
        for (int by = 0; by < 2; by++)
            for (int bx = 0; bx < 2; bx++) {
                int ei = i - 1 + bx, ej = j - 1 + by, ek = k - 1 + bz;
                if (ei < 0 || ej < 0 || ek < 0 || ei >= d->nx - 1 ||
                    ej >= d->ny - 1 || ek >= d->nz - 1) continue;
                double c = cf(P, ei, ej, ek, cctx);
                if (c == 0.0) continue;
                int a = (1 - bx) | ((1 - by) << 1) | ((1 - bz) << 2);
                double part = 0.0;
                for (int b = 0; b < 8; b++) {
                    double w = stiff ? kelem(P, a, b) : mhat(a, b);
                    if (w == 0.0) continue;
                    part += w * xv(P, ei + (b & 1), ej + ((b >> 1) & 1),
                                   ek + ((b >> 2) & 1), xctx);
                }
                acc += c * part;
            }
    return acc;
}

/* element coefficients */
static double cf_sigma(const orc_problem *P, int i, int j, int k, const void *c)
{
    (void)c;
    if (elem_mat(P, k) < 0) return 0.0;   /* phi_s lives on electrode elements */
    return P->sigma[elem_id(P, i, j, k)] * P->h;
}
static double cf_kappa(const orc_problem *P, int i, int j, int k, const void *c)
{
    (void)c;
    return P->kappa[elem_id(P, i, j, k)] * P->h;
}
/* diffusion-potential block and c_e diffusion (defaults chi kappa, kappa) */
static double cf_kappad(const orc_problem *P, int i, int j, int k, const void *c)
{
    (void)c;
    long id = elem_id(P, i, j, k);
    return (P->kappad ? P->kappad[id] : P->d.chi * P->kappa[id]) * P->h;
}
static double cf_dce(const orc_problem *P, int i, int j, int k, const void *c)
{
    (void)c;
    return (P->dce ? P->dce : P->kappa)[elem_id(P, i, j, k)] * P->h;
}
static double cf_mass(const orc_problem *P, int i, int j, int k, const void *c)
{
    (void)c;
    double eps = P->epse ? P->epse[elem_id(P, i, j, k)]
                         : (elem_mat(P, k) >= 0 ? P->d.eps_elec : P->d.eps_sep);
    return eps * P->vol / P->d.dt;
}

/* node value readers */
static double xv_node(const orc_problem *P, int i, int j, int k, const void *c)
{
    return ((const double *)c)[node_id(P, i, j, k)];
}
/* phi_s column: Dirichlet columns are zero (strongly imposed phi_s = 0)     */
static double xv_phis(const orc_problem *P, int i, int j, int k, const void *c)
{
    long je = enode(P, i, j, k);
    if (je < 0 || is_dirichlet(P, k)) return 0.0;
    return ((const double *)c)[je];
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1: the linearized operator y = A x (or A^T x)                      */
/* ------------------------------------------------------------------------ */
/* Per electrode node j the reaction term a*i_n is linearized as
 *   q_j = g_j (x_phis - x_phie) + e_j x_ce + s_j x_cs,N
 * and enters (phis-weak) with +m_j, (phie-weak) with -m_j, (ce-weak) with
 * -(1-t+) m_j and the c_s surface row (FD)/(LR) with +Gamma.  So
 *   A = A_diff + sum_j P_j^T a_j b_j^T P_j,
 *   a_j = (m_j, -m_j, -tc m_j, Gamma),  b_j = (g_j, -g_j, e_j, s_j)
 * over (phi_s, phi_e, c_e, c_s,N) of node j, with the phi_s entries of a_j and
 * b_j zero on the Dirichlet layer.  A^T swaps a_j and b_j, transposes the
 * radial rows and moves chi K_kappa to the (c_e row, phi_e column) block.  */
void orc_apply(const orc_problem *P, int transpose, const double *x, double *y)
{
    const orc_desc *d = &P->d;
    const double *xps = x + P->off_ps, *xpe = x + P->off_pe, *xce = x + P->off_ce;
    double *yps = y + P->off_ps, *ype = y + P->off_pe, *yce = y + P->off_ce;
    memset(y, 0, sizeof(double) * P->N);

    /* diffusion / storage blocks of the three electrode-level equations */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < d->nz; k++)
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                long n = node_id(P, i, j, k);
                double Kpe = elem_sum(P, i, j, k, 1, cf_kappa, NULL, xv_node, xpe);
                double Mce = elem_sum(P, i, j, k, 0, cf_mass, NULL, xv_node, xce);
                if (!P->kappad && !P->dce) {
                    double Kce = elem_sum(P, i, j, k, 1, cf_kappa, NULL, xv_node, xce);
                    if (!transpose) {
                        ype[n] = Kpe + d->chi * Kce;
                        yce[n] = Mce + Kce;
                    } else {
                        ype[n] = Kpe;
                        yce[n] = Mce + Kce + d->chi * Kpe;
                    }
                } else {   /* separate transport coefficients */
                    double Dce = elem_sum(P, i, j, k, 1, cf_dce, NULL, xv_node, xce);
                    double Kx = elem_sum(P, i, j, k, 1, cf_kappad, NULL, xv_node,
                                         transpose ? xpe : xce);
                    if (!transpose) {
                        ype[n] = Kpe + Kx;
                        yce[n] = Mce + Dce;
                    } else {
                        ype[n] = Kpe;
                        yce[n] = Mce + Dce + Kx;
                    }
                }
                long je = enode(P, i, j, k);
                if (je >= 0) {
                    if (is_dirichlet(P, k))
                        yps[je] = xps[je];                 /* identity row */
                    else
                        yps[je] = elem_sum(P, i, j, k, 1, cf_sigma, NULL, xv_phis, xps);
                }
            }

    /* c_e-derivatives of the transport coefficients (Newton terms): element
     * e adds to its corner rows a the rank-one terms
     *   (h K_e (da_e up + db_e uc))_a * mean_e(x_ce)     (phi_e rows)
     *   (h K_e  dc_e uc)_a            * mean_e(x_ce)     (c_e rows)
     * (up, uc the state); the transpose returns w_e^T (...) / 8 to the c_e
     * columns of the corners.  Element by element, serially.               */
    if (P->nw_up) {
        for (int ek = 0; ek < d->nz - 1; ek++)
            for (int ej = 0; ej < d->ny - 1; ej++)
                for (int ei = 0; ei < d->nx - 1; ei++) {
                    long id = elem_id(P, ei, ej, ek), cn[8];
                    for (int b = 0; b < 8; b++)
                        cn[b] = node_id(P, ei + (b & 1), ej + ((b >> 1) & 1), ek + ((b >> 2) & 1));
                    double sp[8], sc[8];
                    for (int a = 0; a < 8; a++) {
                        sp[a] = sc[a] = 0.0;
                        for (int b = 0; b < 8; b++) {
                            double w = P->h * kelem(P, a, b);
                            sp[a] += w * P->nw_up[cn[b]];
                            sc[a] += w * P->nw_uc[cn[b]];
                        }
                    }
                    double A = P->nw_a[id], B = P->nw_b[id], Cc = P->nw_c[id];
                    if (!transpose) {
                        double xm = 0.0;
                        for (int b = 0; b < 8; b++) xm += xce[cn[b]];
                        xm /= 8.0;
                        for (int a = 0; a < 8; a++) {
                            ype[cn[a]] += (A * sp[a] + B * sc[a]) * xm;
                            yce[cn[a]] += Cc * sc[a] * xm;
                        }
                    } else {
                        double t = 0.0;
                        for (int a = 0; a < 8; a++)
                            t += xpe[cn[a]] * (A * sp[a] + B * sc[a]) + xce[cn[a]] * Cc * sc[a];
                        for (int b = 0; b < 8; b++) yce[cn[b]] += t / 8.0;
                    }
                }
    }

    /* radial blocks: c_s rows = c/dt - L~_h c (backward Euler of (FD)) */
    for (int el = 0; el < 2; el++) {
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec;
        const double *xs = x + P->off_cs[el];
        double *ys = y + P->off_cs[el];
        const double *lo = P->Lsub[el], *di = P->Ldia[el], *up = P->Lsup[el];
#pragma omp parallel for schedule(static)
        for (long jn = 0; jn < nn; jn++)
            for (int r = 0; r < N; r++) {
                double v = xs[(long)r * nn + jn] / d->dt;
                if (!transpose) {
                    v -= di[r] * xs[(long)r * nn + jn];
                    if (r > 0) v -= lo[r] * xs[(long)(r - 1) * nn + jn];
                    if (r < N - 1) v -= up[r] * xs[(long)(r + 1) * nn + jn];
                } else {
                    v -= di[r] * xs[(long)r * nn + jn];
                    if (r > 0) v -= up[r - 1] * xs[(long)(r - 1) * nn + jn];
                    if (r < N - 1) v -= lo[r + 1] * xs[(long)(r + 1) * nn + jn];
                }
                ys[(long)r * nn + jn] = v;
            }
    }

    /* reaction coupling, node by node */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < d->nz; k++) {
        int el = node_mat(P, k);
        if (el < 0) continue;
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec;
        long base = el == 0 ? 0 : P->nea;
        double Gam = P->Gamma[el];
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                long n = node_id(P, i, j, k);
                long je = enode(P, i, j, k);
                long jl = je - base;
                int dir = is_dirichlet(P, k);
                double a[4] = { dir ? 0.0 : P->m[je], -P->m[je], -d->tc * P->m[je], Gam };
                double b[4] = { dir ? 0.0 : P->g[je], -P->g[je], P->e[je], P->s[je] };
                double xl[4] = { xps[je], xpe[n], xce[n],
                                 x[P->off_cs[el] + (long)(N - 1) * nn + jl] };
                const double *rowc = transpose ? b : a;   /* row coefficients    */
                const double *colc = transpose ? a : b;   /* column coefficients */
                double q = 0.0;
                for (int t = 0; t < 4; t++) q += colc[t] * xl[t];
                yps[je] += rowc[0] * q;   /* zero on Dirichlet rows */
                ype[n] += rowc[1] * q;
                yce[n] += rowc[2] * q;
                y[P->off_cs[el] + (long)(N - 1) * nn + jl] += rowc[3] * q;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Tridiagonal solves for the c_s blocks (Sec. 4.2, element-wise block       */
/* Jacobi): A_ss,j = T0 + Gamma s_j e_N e_N^T, T0 = I/dt - L~_h.            */
/* ------------------------------------------------------------------------ */
static void radial_solve(const orc_problem *P, int el, double sj, int transpose,
                         const double *rhs, double *out, double *work)
{
    int N = P->d.nr[el];
    double *lo = work, *di = work + N, *up = work + 2 * N, *cp = work + 3 * N;
    for (int r = 0; r < N; r++) {
        di[r] = 1.0 / P->d.dt - P->Ldia[el][r];
        lo[r] = r > 0 ? -P->Lsub[el][r] : 0.0;      /* A[r][r-1] */
        up[r] = r < N - 1 ? -P->Lsup[el][r] : 0.0;  /* A[r][r+1] */
    }
    di[N - 1] += P->Gamma[el] * sj;
    if (transpose) {   /* A^T[r][r-1] = A[r-1][r], A^T[r][r+1] = A[r+1][r] */
        double *tl = cp;
        for (int r = 0; r < N; r++) tl[r] = r > 0 ? up[r - 1] : 0.0;
        for (int r = 0; r < N - 1; r++) up[r] = lo[r + 1];
        up[N - 1] = 0.0;
        for (int r = 0; r < N; r++) lo[r] = tl[r];
    }
    /* Thomas algorithm */
    double *c2 = cp, *d2 = out;
    c2[0] = up[0] / di[0];
    d2[0] = rhs[0] / di[0];
    for (int r = 1; r < N; r++) {
        double den = di[r] - lo[r] * c2[r - 1];
        c2[r] = r < N - 1 ? up[r] / den : 0.0;
        d2[r] = (rhs[r] - lo[r] * d2[r - 1]) / den;
    }
    for (int r = N - 2; r >= 0; r--) d2[r] -= c2[r] * d2[r + 1];
}

/* (T0^-1)_{NN} for electrode el                                             */
static double tau0(const orc_problem *P, int el)
{
    int N = P->d.nr[el];
    double *rhs = xmalloc(sizeof(double) * N), *out = xmalloc(sizeof(double) * N);
    double *w = xmalloc(sizeof(double) * 4 * N);
    rhs[N - 1] = 1.0;
    radial_solve(P, el, 0.0, 0, rhs, out, w);
    double t = out[N - 1];
    free(rhs); free(out); free(w);
    return t;
}

/* ------------------------------------------------------------------------ */
/* Multigrid (replaces the paper's BoomerAMG V-cycle, Sec. 4.2)              */
/* ------------------------------------------------------------------------ */
/* Fine boxes:  0: phi_s anode, node layers 1..na-1 (the Dirichlet layer is
 * eliminated); 1: phi_s cathode, layers na+ns..nz-1; 2: phi_e, 3: c_e, all
 * layers.  The field operators are the diagonal blocks of the (approximate)
 * Schur complement: S_f = A_diff,ff + diag(omega_j a_f,j b_f,j).            */
static void box_geom(const orc_problem *P, int box, int *nz, int *k0)
{
    switch (box) {
    case 0: *nz = P->d.na - 1; *k0 = 1; break;
    case 1: *nz = P->nc; *k0 = P->d.na + P->d.ns; break;
    default: *nz = P->d.nz; *k0 = 0; break;
    }
}

static int st_off(int dx, int dy, int dz) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1); }

/* assemble the 27-point stencil of the fine operator of a box              */
static void assemble_fine(const orc_problem *P, int box, double *S)
{
    const orc_desc *d = &P->d;
    int NZ, k0;
    box_geom(P, box, &NZ, &k0);
    int nx = d->nx, ny = d->ny;
    long n = (long)nx * ny * NZ;
    memset(S, 0, sizeof(double) * 27 * n);
#pragma omp parallel for schedule(static)
    for (int kl = 0; kl < NZ; kl++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int k = kl + k0;
                double *row = S + 27 * (i + (long)nx * (j + (long)ny * kl));
                for (int bz = 0; bz < 2; bz++)
                    for (int by = 0; by < 2; by++)
                        for (int bx = 0; bx < 2; bx++) {
                            int ei = i - 1 + bx, ej = j - 1 + by, ek = k - 1 + bz;
                            if (ei < 0 || ej < 0 || ek < 0 || ei >= nx - 1 ||
                                ej >= ny - 1 || ek >= d->nz - 1) continue;
                            double cK, cM = 0.0;
                            if (box <= 1) {
                                if (elem_mat(P, ek) != box) continue;
                                cK = cf_sigma(P, ei, ej, ek, NULL);
                            } else if (box == 2) {
                                cK = cf_kappa(P, ei, ej, ek, NULL);
                            } else {
                                cK = cf_dce(P, ei, ej, ek, NULL);
                                cM = cf_mass(P, ei, ej, ek, NULL);
                            }
                            int a = (1 - bx) | ((1 - by) << 1) | ((1 - bz) << 2);
                            for (int b = 0; b < 8; b++) {
                                int gi = ei + (b & 1), gj = ej + ((b >> 1) & 1),
                                    gk = ek + ((b >> 2) & 1);
                                int lk = gk - k0;
                                if (lk < 0 || lk >= NZ) continue;   /* eliminated */
                                row[st_off(gi - i, gj - j, gk - k)] +=
                                    cK * kelem(P, a, b) + cM * mhat(a, b);
                            }
                        }
                /* reaction diagonal of the Schur-complement field block */
                long je = enode(P, i, j, k);
                if (je >= 0) {
                    double w = P->omega[je];
                    double dg;
                    if (box <= 2) dg = w * P->m[je] * P->g[je];
                    else dg = -w * d->tc * P->m[je] * P->e[je];
                    row[st_off(0, 0, 0)] += dg;
                }
            }
}

/* 1D linear interpolation for the "even indices plus the last" coarsening.
 * Lists the coarse points (and weights) that fine index i interpolates from. */
static int coarse_of_fine(int n, int i, int *I, double *w)
{
    int nc = n / 2 + 1;
    if (n <= 2) { I[0] = i; w[0] = 1.0; return 1; }
    if ((i & 1) == 0) { I[0] = i / 2; w[0] = 1.0; return 1; }
    if (i == n - 1) { I[0] = nc - 1; w[0] = 1.0; return 1; }
    I[0] = (i - 1) / 2; w[0] = 0.5;
    I[1] = (i + 1) / 2; w[1] = 0.5;
    return 2;
}
static int coarse_size(int n) { return n <= 2 ? n : n / 2 + 1; }

/* the same along z, which z-line smoothing leaves uncoarsened (P_z = I)      */
static int z_of_fine(int zc, int n, int i, int *I, double *w)
{
    if (!zc) { I[0] = i; w[0] = 1.0; return 1; }
    return coarse_of_fine(n, i, I, w);
}
static int z_size(int zc, int n) { return zc ? coarse_size(n) : n; }

/* Galerkin product S_c = P^T S P, P = P_x (x) P_y (x) P_z (P_z = I unless
 * zc), by brute force over fine rows (serial scatter, obviously correct)    */
void orc_rap(int nx, int ny, int nz, int zc, const double *S, double *Sc)
{
    int cx = coarse_size(nx), cy = coarse_size(ny), cz = z_size(zc, nz);
    memset(Sc, 0, sizeof(double) * 27 * (long)cx * cy * cz);
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int Ii[2], Ij[2], Ik[2];
                double wi[2], wj[2], wk[2];
                int ni = coarse_of_fine(nx, i, Ii, wi);
                int nj = coarse_of_fine(ny, j, Ij, wj);
                int nk = z_of_fine(zc, nz, k, Ik, wk);
                const double *row = S + 27 * (i + (long)nx * (j + (long)ny * k));
                for (int o = 0; o < 27; o++) {
                    double sv = row[o];
                    if (sv == 0.0) continue;
                    int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                    int ii = i + dx, jj = j + dy, kk = k + dz;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    int Ji[2], Jj[2], Jk[2];
                    double vi[2], vj[2], vk[2];
                    int mi = coarse_of_fine(nx, ii, Ji, vi);
                    int mj = coarse_of_fine(ny, jj, Jj, vj);
                    int mk = z_of_fine(zc, nz, kk, Jk, vk);
                    for (int a3 = 0; a3 < nk; a3++) for (int a2 = 0; a2 < nj; a2++)
                    for (int a1 = 0; a1 < ni; a1++) {
                        double wa = wi[a1] * wj[a2] * wk[a3] * sv;
                        long Irow = Ii[a1] + (long)cx * (Ij[a2] + (long)cy * Ik[a3]);
                        for (int b3 = 0; b3 < mk; b3++) for (int b2 = 0; b2 < mj; b2++)
                        for (int b1 = 0; b1 < mi; b1++) {
                            int ox = Ji[b1] - Ii[a1], oy = Jj[b2] - Ij[a2], oz = Jk[b3] - Ik[a3];
                            if (ox < -1 || ox > 1 || oy < -1 || oy > 1 || oz < -1 || oz > 1) {
                                fprintf(stderr, "oracle: RAP stencil overflow\n");
                                abort();
                            }
                            Sc[27 * Irow + st_off(ox, oy, oz)] +=
                                wa * vi[b1] * vj[b2] * vk[b3];
                        }
                    }
                }
            }
}

/* y = S x for a stored stencil on a box                                     */
static void st_apply(const orc_level *L, const double *x, double *y)
{
    int nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long n = i + (long)nx * (j + (long)ny * k);
                double acc = 0.0;
                for (int o = 0; o < 27; o++) {
                    int ii = i + o % 3 - 1, jj = j + (o / 3) % 3 - 1, kk = k + o / 9 - 1;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    acc += L->S[27 * n + o] * x[ii + (long)nx * (jj + (long)ny * kk)];
                }
                y[n] = acc;
            }
}

/* Gershgorin bound of diag(S)^-1 S: max_i sum_j |s_ij| / s_ii               */
static double gershgorin(const orc_level *L)
{
    double mx = 0.0;
    for (long n = 0; n < L->n; n++) {
        double sum = 0.0;
        for (int o = 0; o < 27; o++) sum += fabs(L->S[27 * n + o]);
        double r = sum / L->S[27 * n + 13];
        if (r > mx) mx = r;
    }
    return mx;
}

/* dense Cholesky of the coarsest operator                                   */
static void coarse_factor(orc_level *L)
{
    long n = L->n;
    double *A = xmalloc(sizeof(double) * n * n);
    for (int k = 0; k < L->nz; k++)
        for (int j = 0; j < L->ny; j++)
            for (int i = 0; i < L->nx; i++) {
                long r = i + (long)L->nx * (j + (long)L->ny * k);
                for (int o = 0; o < 27; o++) {
                    int ii = i + o % 3 - 1, jj = j + (o / 3) % 3 - 1, kk = k + o / 9 - 1;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= L->nx || jj >= L->ny || kk >= L->nz)
                        continue;
                    A[r * n + ii + (long)L->nx * (jj + (long)L->ny * kk)] += L->S[27 * r + o];
                }
            }
    /* symmetrize (Galerkin products are symmetric up to rounding) */
    for (long r = 0; r < n; r++)
        for (long c = 0; c < r; c++) {
            double v = 0.5 * (A[r * n + c] + A[c * n + r]);
            A[r * n + c] = A[c * n + r] = v;
        }
    for (long j = 0; j < n; j++) {
        double dsum = A[j * n + j];
        for (long k = 0; k < j; k++) dsum -= A[j * n + k] * A[j * n + k];
        if (dsum <= 0.0) { fprintf(stderr, "oracle: coarse matrix not SPD\n"); abort(); }
        double ljj = sqrt(dsum);
        A[j * n + j] = ljj;
        for (long i = j + 1; i < n; i++) {
            double v = A[i * n + j];
            for (long k = 0; k < j; k++) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / ljj;
        }
    }
    L->L = A;
}

static void coarse_solve(const orc_level *L, const double *b, double *x)
{
    long n = L->n;
    const double *A = L->L;
    for (long i = 0; i < n; i++) {
        double v = b[i];
        for (long k = 0; k < i; k++) v -= A[i * n + k] * x[k];
        x[i] = v / A[i * n + i];
    }
    for (long i = n - 1; i >= 0; i--) {
        double v = x[i];
        for (long k = i + 1; k < n; k++) v -= A[k * n + i] * x[k];
        x[i] = v / A[i * n + i];
    }
}

static void mg_build(orc_problem *P, int box)
{
    orc_mg *M = &P->mg[box];
    mg_free(M);
    int NZ, k0;
    box_geom(P, box, &NZ, &k0);
    orc_level *L0 = &M->lev[0];
    L0->nx = P->d.nx; L0->ny = P->d.ny; L0->nz = NZ;
    L0->n = (long)L0->nx * L0->ny * L0->nz;
    L0->S = xmalloc(sizeof(double) * 27 * L0->n);
    assemble_fine(P, box, L0->S);
    M->nlev = 1;
    const int zc = P->opts.smoother != ORC_SMOOTH_ZLINE;
    for (;;) {
        orc_level *L = &M->lev[M->nlev - 1];
        L->lmax = gershgorin(L);
        int cx = coarse_size(L->nx), cy = coarse_size(L->ny), cz = z_size(zc, L->nz);
        long cn = (long)cx * cy * cz;
        if (L->n <= P->opts.coarse_max || cn == L->n || M->nlev == 16) {
            coarse_factor(L);
            break;
        }
        orc_level *C = &M->lev[M->nlev];
        C->nx = cx; C->ny = cy; C->nz = cz; C->n = cn;
        C->S = xmalloc(sizeof(double) * 27 * cn);
        orc_rap(L->nx, L->ny, L->nz, zc, L->S, C->S);
        M->nlev++;
    }
}

/* Chebyshev smoothing of degree `deg` on diag(S)^-1 S over [lmax/4, lmax]
 * (three-term recurrence for the shifted and scaled Chebyshev polynomials,
 * Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1)            */
static void chebyshev(const orc_level *L, int deg, const double *b, double *x,
                      double *r, double *dv)
{
    double lmax = L->lmax, lmin = lmax / 4.0;
    double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    double sigma = theta / delta, rho = 1.0 / sigma;
    long n = L->n;
    st_apply(L, x, r);
    for (long i = 0; i < n; i++) dv[i] = (b[i] - r[i]) / L->S[27 * i + 13] / theta;
    for (int it = 1; it <= deg; it++) {
        for (long i = 0; i < n; i++) x[i] += dv[i];
        if (it == deg) break;
        st_apply(L, x, r);
        double rho_new = 1.0 / (2.0 * sigma - rho);
        for (long i = 0; i < n; i++)
            dv[i] = rho_new * rho * dv[i] +
                    2.0 * rho_new / delta * (b[i] - r[i]) / L->S[27 * i + 13];
        rho = rho_new;
    }
}

/* Block Gauss-Seidel over the z-lines of one colour (x parity cx, y parity
 * cy): on each line (i, j) the rows' couplings to other lines are moved to
 * the right-hand side with the current x, and the line's tridiagonal block
 * (couplings to k-1, k, k+1 in the same column) is solved by elimination.
 * Lines of one colour do not couple (27-point stencil), so their order does
 * not matter.                                                               */
static void zline_colour(const orc_level *L, int cx, int cy, const double *b, double *x)
{
    int nx = L->nx, ny = L->ny, nz = L->nz;
    double *cp = xmalloc(sizeof(double) * nz), *dp = xmalloc(sizeof(double) * nz);
    for (int j = cy; j < ny; j += 2)
        for (int i = cx; i < nx; i += 2) {
            for (int k = 0; k < nz; k++) {
                long n = i + (long)nx * (j + (long)ny * k);
                const double *row = L->S + 27 * n;
                double rhs = b[n];
                for (int o = 0; o < 27; o++) {
                    int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                    if (dx == 0 && dy == 0) continue;
                    int ii = i + dx, jj = j + dy, kk = k + dz;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    rhs -= row[o] * x[ii + (long)nx * (jj + (long)ny * kk)];
                }
                double lo = k > 0 ? row[st_off(0, 0, -1)] : 0.0;
                double up = k < nz - 1 ? row[st_off(0, 0, 1)] : 0.0;
                double den = row[13] - (k > 0 ? lo * cp[k - 1] : 0.0);
                cp[k] = up / den;
                dp[k] = (rhs - (k > 0 ? lo * dp[k - 1] : 0.0)) / den;
            }
            double nxt = 0.0;
            for (int k = nz - 1; k >= 0; k--) {
                nxt = dp[k] - (k < nz - 1 ? cp[k] * nxt : 0.0);
                x[i + (long)nx * (j + (long)ny * k)] = nxt;
            }
        }
    free(cp); free(dp);
}

/* one symmetric sweep pass: colours 0..3 (pre) or 3..0 (post)              */
static void zline_sweep(const orc_level *L, int backward, const double *b, double *x)
{
    for (int q = 0; q < 4; q++) {
        int c = backward ? 3 - q : q;
        zline_colour(L, c & 1, c >> 1, b, x);
    }
}

/* one V-cycle x = V_l(b), x zero on entry not required (it is overwritten)  */
static void vcycle(const orc_problem *P, const orc_mg *M, int l, const double *b, double *x)
{
    const orc_level *L = &M->lev[l];
    long n = L->n;
    if (l == M->nlev - 1) { coarse_solve(L, b, x); return; }
    const orc_level *C = &M->lev[l + 1];
    double *r = xmalloc(sizeof(double) * n), *dv = xmalloc(sizeof(double) * n);
    double *bc = xmalloc(sizeof(double) * C->n), *xc = xmalloc(sizeof(double) * C->n);
    int deg = P->opts.cheb_degree;
    const int line = P->opts.smoother == ORC_SMOOTH_ZLINE, zc = !line;
    memset(x, 0, sizeof(double) * n);
    if (line)                                             /* pre-smoothing  */
        for (int t = 0; t < deg; t++) zline_sweep(L, 0, b, x);
    else
        chebyshev(L, deg, b, x, r, dv);
    st_apply(L, x, r);
    for (long i = 0; i < n; i++) r[i] = b[i] - r[i];      /* residual       */
    memset(bc, 0, sizeof(double) * C->n);                 /* b_c = P^T r    */
    for (int k = 0; k < L->nz; k++)
        for (int j = 0; j < L->ny; j++)
            for (int i = 0; i < L->nx; i++) {
                int Ii[2], Ij[2], Ik[2];
                double wi[2], wj[2], wk[2];
                int ni = coarse_of_fine(L->nx, i, Ii, wi);
                int nj = coarse_of_fine(L->ny, j, Ij, wj);
                int nk = z_of_fine(zc, L->nz, k, Ik, wk);
                double rv = r[i + (long)L->nx * (j + (long)L->ny * k)];
                for (int c = 0; c < nk; c++) for (int bq = 0; bq < nj; bq++)
                for (int a = 0; a < ni; a++)
                    bc[Ii[a] + (long)C->nx * (Ij[bq] + (long)C->ny * Ik[c])] +=
                        wi[a] * wj[bq] * wk[c] * rv;
            }
    vcycle(P, M, l + 1, bc, xc);
    for (int k = 0; k < L->nz; k++)                       /* x += P x_c     */
        for (int j = 0; j < L->ny; j++)
            for (int i = 0; i < L->nx; i++) {
                int Ii[2], Ij[2], Ik[2];
                double wi[2], wj[2], wk[2];
                int ni = coarse_of_fine(L->nx, i, Ii, wi);
                int nj = coarse_of_fine(L->ny, j, Ij, wj);
                int nk = z_of_fine(zc, L->nz, k, Ik, wk);
                double v = 0.0;
                for (int c = 0; c < nk; c++) for (int bq = 0; bq < nj; bq++)
                for (int a = 0; a < ni; a++)
                    v += wi[a] * wj[bq] * wk[c] *
                         xc[Ii[a] + (long)C->nx * (Ij[bq] + (long)C->ny * Ik[c])];
                x[i + (long)L->nx * (j + (long)L->ny * k)] += v;
            }
    if (line)                                             /* post-smoothing */
        for (int t = 0; t < deg; t++) zline_sweep(L, 1, b, x);
    else
        chebyshev(L, deg, b, x, r, dv);
    free(r); free(dv); free(bc); free(xc);
}

/* ------------------------------------------------------------------------ */
/* Preconditioner setup and apply (Sec. 4.2)                                 */
/* ------------------------------------------------------------------------ */
void orc_setup(orc_problem *P, const orc_opts *o)
{
    if (o->krylov != ORC_KRYLOV_FULL && !(o->krylov == ORC_KRYLOV_SCHUR && o->pc == ORC_PC_SCHUR)) {
        fprintf(stderr, "oracle: krylov %d needs pc SCHUR\n", o->krylov);
        abort();
    }
    if (o->pc == ORC_PC_BGS) {   /* the ordering must be a permutation */
        int seen = 0;
        for (int p = 0; p < 4; p++) seen |= 1 << ((o->bgs_order >> (2 * p)) & 3);
        if (seen != 15 || (o->bgs_order >> 8) != 0) {
            fprintf(stderr, "oracle: bgs_order %d is not a field ordering\n", o->bgs_order);
            abort();
        }
    }
    P->opts = *o;
    if (P->opts.coarse_max <= 0) P->opts.coarse_max = 512;
    if (P->opts.cheb_degree <= 0) P->opts.cheb_degree = 2;
    P->pc_type = o->pc;
    free(P->omega);
    P->omega = xmalloc(sizeof(double) * P->ne);
    for (int el = 0; el < 2; el++) {
        double t0 = tau0(P, el);
        long nn = el == 0 ? P->nea : P->nec, base = el == 0 ? 0 : P->nea;
        for (long jl = 0; jl < nn; jl++) {
            long je = base + jl;
            /* Sherman-Morrison: 1 - Gamma s (A_ss^-1)_NN = 1/(1 + Gamma s tau0) */
            P->omega[je] = o->pc != ORC_PC_SCHUR ? 1.0
                                                 : 1.0 / (1.0 + P->Gamma[el] * P->s[je] * t0);
        }
    }
    for (int b = 0; b < 4; b++) mg_build(P, b);
    P->pc_ready = 1;
}

/* field slices of a macro vector for the four multigrid boxes               */
static void box_slice(const orc_problem *P, int box, long *off, long *n)
{
    long layer = (long)P->d.nx * P->d.ny;
    switch (box) {
    case 0: *off = P->off_ps + layer; *n = P->nea - layer; break;
    case 1: *off = P->off_ps + P->nea; *n = P->nec; break;
    case 2: *off = P->off_pe; *n = P->nnode; break;
    default: *off = P->off_ce; *n = P->nnode; break;
    }
}

/* ------------------------------------------------------------------------ */
/* Block Gauss-Seidel (eq. PGS) in a chosen field ordering o_0, ..., o_3.    */
/* ------------------------------------------------------------------------ */
/* Rows of field f minus the blocks A_{f,g} z_g of the fields g already solved
 * (done[g] != 0).  The off-diagonal blocks of A are the node-local reaction
 * terms a_f,j b_g,j (over phi_s, phi_e, c_e and the c_s surface value, the
 * c_s row being the surface row) and chi K_kappa in the (phi_e row, c_e
 * column) block.  Transposed, the blocks are those of A^T: the roles of a
 * and b swap and chi K_kappa sits in the (c_e row, phi_e column) block.     */
static void bgs_subtract(const orc_problem *P, int transpose, int f, const int *done,
                         const double *z, double *t)
{
    const orc_desc *d = &P->d;
    const double *zps = z + P->off_ps, *zpe = z + P->off_pe, *zce = z + P->off_ce;
    for (int k = 0; k < d->nz; k++) {
        int el = node_mat(P, k);
        if (el < 0) continue;
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec, base = el == 0 ? 0 : P->nea;
        int dir = is_dirichlet(P, k);
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                long n = node_id(P, i, j, k), je = enode(P, i, j, k), jl = je - base;
                long srow = P->off_cs[el] + (long)(N - 1) * nn + jl;
                double a[4] = { dir ? 0.0 : P->m[je], -P->m[je], -d->tc * P->m[je],
                                P->Gamma[el] };
                double b[4] = { dir ? 0.0 : P->g[je], -P->g[je], P->e[je], P->s[je] };
                double zl[4] = { zps[je], zpe[n], zce[n], z[srow] };
                const double *rowc = transpose ? b : a, *colc = transpose ? a : b;
                double q = 0.0;
                for (int g = 0; g < 4; g++)
                    if (done[g]) q += colc[g] * zl[g];
                long row = f == ORC_F_PHIS ? P->off_ps + je
                         : f == ORC_F_PHIE ? P->off_pe + n
                         : f == ORC_F_CE   ? P->off_ce + n : srow;
                t[row] -= rowc[f] * q;
            }
    }
    /* chi K_kappa: A_{phi_e, c_e} (A^T_{c_e, phi_e} when transposed) */
    int krow = transpose ? ORC_F_CE : ORC_F_PHIE, kcol = transpose ? ORC_F_PHIE : ORC_F_CE;
    if (f == krow && done[kcol]) {
        const double *zk = kcol == ORC_F_CE ? zce : zpe;
        double *tk = t + (krow == ORC_F_PHIE ? P->off_pe : P->off_ce);
        for (int k = 0; k < d->nz; k++)
            for (int j = 0; j < d->ny; j++)
                for (int i = 0; i < d->nx; i++)
                    tk[node_id(P, i, j, k)] -=
                        P->kappad ? elem_sum(P, i, j, k, 1, cf_kappad, NULL, xv_node, zk)
                                  : d->chi * elem_sum(P, i, j, k, 1, cf_kappa, NULL, xv_node, zk);
    }
}

/* z_f = A_{f,f}^-1 t_f (A_{f,f}^-T when transposed): a V-cycle for the
 * electrode-level fields (omega = 1, so the multigrid operator is the
 * diagonal block itself), the exact tridiagonal solve for each c_s block.    */
static void bgs_block_solve(const orc_problem *P, int transpose, int f, const double *t,
                            double *z)
{
    const orc_desc *d = &P->d;
    long off, n;
    switch (f) {
    case ORC_F_PHIS:
        for (long q = 0; q < (long)d->nx * d->ny; q++) z[P->off_ps + q] = t[P->off_ps + q];
        for (int b = 0; b < 2; b++) {
            box_slice(P, b, &off, &n);
            vcycle(P, &P->mg[b], 0, t + off, z + off);
        }
        break;
    case ORC_F_PHIE:
    case ORC_F_CE:
        box_slice(P, f == ORC_F_PHIE ? 2 : 3, &off, &n);
        vcycle(P, &P->mg[f == ORC_F_PHIE ? 2 : 3], 0, t + off, z + off);
        break;
    default:
        for (int el = 0; el < 2; el++) {
            int N = d->nr[el];
            long nn = el == 0 ? P->nea : P->nec, base = el == 0 ? 0 : P->nea;
            double *rhs = xmalloc(sizeof(double) * N), *sol = xmalloc(sizeof(double) * N);
            double *w = xmalloc(sizeof(double) * 4 * N);
            for (long jl = 0; jl < nn; jl++) {
                for (int q = 0; q < N; q++) rhs[q] = t[P->off_cs[el] + (long)q * nn + jl];
                radial_solve(P, el, P->s[base + jl], transpose, rhs, sol, w);
                for (int q = 0; q < N; q++) z[P->off_cs[el] + (long)q * nn + jl] = sol[q];
            }
            free(rhs); free(sol); free(w);
        }
    }
}

/* P_GS is block lower triangular in the ordering: z_{o_p} = A_{o_p,o_p}^-1
 * (r_{o_p} - sum_{q<p} A_{o_p,o_q} z_{o_q}), p = 0..3.  P_GS^T is block upper
 * triangular, so the transposed sweep runs p = 3..0 with the blocks of A^T.  */
static void apply_bgs(const orc_problem *P, int transpose, const double *r, double *z)
{
    double *t = xmalloc(sizeof(double) * P->N);
    memcpy(t, r, sizeof(double) * P->N);
    memset(z, 0, sizeof(double) * P->N);
    int done[4] = { 0, 0, 0, 0 };
    for (int s = 0; s < 4; s++) {
        int p = transpose ? 3 - s : s;
        int f = (P->opts.bgs_order >> (2 * p)) & 3;
        bgs_subtract(P, transpose, f, done, z, t);
        bgs_block_solve(P, transpose, f, t, z);
        done[f] = 1;
    }
    free(t);
}

/* z = P^-1 r (or P^-T r).  SCHUR mode, per electrode node j:
 *   1. zeta_j = (A_ss,j^-1 r_s,j)_N                (A_ss,j^-T when transposed)
 *   2. r~_y  = r_y - a_y,j s_j zeta_j              (transposed: - b_y,j Gamma zeta_j)
 *   3. z_f   = V_f(r~_f) for f in {phi_s, phi_e, c_e}
 *   4. z_s,j = A_ss,j^-1 (r_s,j - Gamma (b_y,j . z_y,j) e_N)
 *                                                  (transposed: s_j (a_y,j . z_y,j))
 * BJ mode (eq. PJ): steps 2 and the correction in 4 are skipped.  BGS mode:
 * apply_bgs above.                                                          */
void orc_apply_pc(const orc_problem *P, int transpose, const double *r, double *z)
{
    const orc_desc *d = &P->d;
    if (P->pc_type == ORC_PC_BGS) {
        apply_bgs(P, transpose, r, z);
        return;
    }
    int schur = P->pc_type == ORC_PC_SCHUR;
    long Nm = P->off_cs[0];
    double *rt = xmalloc(sizeof(double) * Nm);
    memcpy(rt, r, sizeof(double) * Nm);
    memset(z, 0, sizeof(double) * P->N);

    for (int k = 0; k < d->nz && schur; k++) {
        int el = node_mat(P, k);
        if (el < 0) continue;
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec, base = el == 0 ? 0 : P->nea;
        double *rhs = xmalloc(sizeof(double) * N), *sol = xmalloc(sizeof(double) * N);
        double *w = xmalloc(sizeof(double) * 4 * N);
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                long n = node_id(P, i, j, k), je = enode(P, i, j, k), jl = je - base;
                for (int q = 0; q < N; q++) rhs[q] = r[P->off_cs[el] + (long)q * nn + jl];
                radial_solve(P, el, P->s[je], transpose, rhs, sol, w);
                double zeta = sol[N - 1];
                int dir = is_dirichlet(P, k);
                double a[3] = { dir ? 0.0 : P->m[je], -P->m[je], -d->tc * P->m[je] };
                double b[3] = { dir ? 0.0 : P->g[je], -P->g[je], P->e[je] };
                double coef[3];
                for (int f = 0; f < 3; f++)
                    coef[f] = transpose ? b[f] * P->Gamma[el] : a[f] * P->s[je];
                rt[P->off_ps + je] -= coef[0] * zeta;
                rt[P->off_pe + n] -= coef[1] * zeta;
                rt[P->off_ce + n] -= coef[2] * zeta;
            }
        free(rhs); free(sol); free(w);
    }

    /* Dirichlet rows of the phi_s block are identity rows */
    for (long q = 0; q < (long)d->nx * d->ny; q++) z[P->off_ps + q] = rt[P->off_ps + q];
    for (int b = 0; b < 4; b++) {
        long off, n;
        box_slice(P, b, &off, &n);
        vcycle(P, &P->mg[b], 0, rt + off, z + off);
    }

    for (int k = 0; k < d->nz; k++) {
        int el = node_mat(P, k);
        if (el < 0) continue;
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec, base = el == 0 ? 0 : P->nea;
        double *rhs = xmalloc(sizeof(double) * N), *sol = xmalloc(sizeof(double) * N);
        double *w = xmalloc(sizeof(double) * 4 * N);
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                long n = node_id(P, i, j, k), je = enode(P, i, j, k), jl = je - base;
                for (int q = 0; q < N; q++) rhs[q] = r[P->off_cs[el] + (long)q * nn + jl];
                if (schur) {
                    int dir = is_dirichlet(P, k);
                    double a[3] = { dir ? 0.0 : P->m[je], -P->m[je], -d->tc * P->m[je] };
                    double b[3] = { dir ? 0.0 : P->g[je], -P->g[je], P->e[je] };
                    double zy[3] = { z[P->off_ps + je], z[P->off_pe + n], z[P->off_ce + n] };
                    double delta = 0.0;
                    for (int f = 0; f < 3; f++)
                        delta += (transpose ? a[f] * P->s[je] : b[f] * P->Gamma[el]) * zy[f];
                    rhs[N - 1] -= delta;
                }
                radial_solve(P, el, P->s[je], transpose, rhs, sol, w);
                for (int q = 0; q < N; q++) z[P->off_cs[el] + (long)q * nn + jl] = sol[q];
            }
        free(rhs); free(sol); free(w);
    }
    free(rt);
}

/* ------------------------------------------------------------------------ */
/* Multigrid inspection (for the tests)                                      */
/* ------------------------------------------------------------------------ */
int orc_mg_nlev(const orc_problem *P, int box) { return P->mg[box].nlev; }
void orc_mg_level(const orc_problem *P, int box, int l, int32_t *dims, double *lmax)
{
    const orc_level *L = &P->mg[box].lev[l];
    dims[0] = L->nx; dims[1] = L->ny; dims[2] = L->nz;
    *lmax = L->lmax;
}
void orc_mg_stencil(const orc_problem *P, int box, int l, double *S)
{
    const orc_level *L = &P->mg[box].lev[l];
    memcpy(S, L->S, sizeof(double) * 27 * L->n);
}
void orc_vcycle(const orc_problem *P, int box, const double *b, double *x)
{
    vcycle(P, &P->mg[box], 0, b, x);
}
void orc_omega(const orc_problem *P, double *w) { memcpy(w, P->omega, sizeof(double) * P->ne); }

/* stand-alone stencil helpers on a single box (test pins) */
void orc_stencil_apply(int nx, int ny, int nz, const double *S, const double *x, double *y)
{
    orc_level L = { nx, ny, nz, (long)nx * ny * nz, (double *)S, 0.0, NULL };
    st_apply(&L, x, y);
}
void orc_chebyshev(int nx, int ny, int nz, const double *S, int deg,
                   const double *b, double *x)
{
    orc_level L = { nx, ny, nz, (long)nx * ny * nz, (double *)S, 0.0, NULL };
    L.lmax = gershgorin(&L);
    double *r = xmalloc(sizeof(double) * L.n), *dv = xmalloc(sizeof(double) * L.n);
    chebyshev(&L, deg, b, x, r, dv);
    free(r); free(dv);
}
void orc_zline_sweep(int nx, int ny, int nz, const double *S, int backward, const double *b,
                     double *x)
{
    orc_level L = {nx, ny, nz, (long)nx * ny * nz, (double *)S, 0.0, NULL};
    zline_sweep(&L, backward, b, x);
}
double orc_gershgorin(int nx, int ny, int nz, const double *S)
{
    orc_level L = { nx, ny, nz, (long)nx * ny * nz, (double *)S, 0.0, NULL };
    return gershgorin(&L);
}

/* ------------------------------------------------------------------------ */
/* Flexible GMRES (Saad 1993), right preconditioned, restarted              */
/* ------------------------------------------------------------------------ */
/* Inner product summed over fixed chunks, the chunk sums added in order, so
 * that the result does not depend on the number or timing of threads.     */
static double dot(const double *a, const double *b, long n)
{
    const long CH = 8192;
    long nch = (n + CH - 1) / CH;
    double *part = xmalloc(sizeof(double) * (nch > 0 ? nch : 1));
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nch; c++) {
        long hi = (c + 1) * CH < n ? (c + 1) * CH : n;
        double s = 0.0;
        for (long i = c * CH; i < hi; i++) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (long c = 0; c < nch; c++) s += part[c];
    free(part);
    return s;
}

/* ------------------------------------------------------------------------ */
/* The Schur complement of the c_s blocks (Sec. 4.1: A_cs,cs is block        */
/* diagonal, one tridiagonal block per electrode node, and the c_s unknowns  */
/* couple to the electrode-level fields only through the surface value).     */
/* With y the electrode-level unknowns [phi_s | phi_e | c_e]:                 */
/*   S = A_yy - A_ys A_ss^-1 A_sy,  b^ = b_y - A_ys A_ss^-1 b_s,              */
/*   x_s = A_ss^-1 (b_s - A_sy y),                                           */
/* each written out with the operator and the per-node tridiagonal solves    */
/* (transposed: the same with the blocks of A^T).                            */
/* ------------------------------------------------------------------------ */
/* out_s = A_ss^-1 in_s (A_ss^-T when transposed), per electrode node        */
static void particle_solve(const orc_problem *P, int transpose, const double *in, double *out)
{
    const orc_desc *d = &P->d;
    for (int el = 0; el < 2; el++) {
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec, base = el == 0 ? 0 : P->nea;
#pragma omp parallel
        {
            double *rhs = xmalloc(sizeof(double) * N), *sol = xmalloc(sizeof(double) * N);
            double *w = xmalloc(sizeof(double) * 4 * N);
#pragma omp for schedule(static)
            for (long jl = 0; jl < nn; jl++) {
                for (int q = 0; q < N; q++) rhs[q] = in[P->off_cs[el] + (long)q * nn + jl];
                radial_solve(P, el, P->s[base + jl], transpose, rhs, sol, w);
                for (int q = 0; q < N; q++) out[P->off_cs[el] + (long)q * nn + jl] = sol[q];
            }
            free(rhs); free(sol); free(w);
        }
    }
}

/* out = S y (S^T y), y and out of length off_cs[0] */
void orc_schur_apply(const orc_problem *P, int transpose, const double *y, double *out)
{
    long Nm = P->off_cs[0], N = P->N;
    double *x = xmalloc(sizeof(double) * N), *t = xmalloc(sizeof(double) * N);
    double *u = xmalloc(sizeof(double) * N);
    memset(x, 0, sizeof(double) * N);
    memcpy(x, y, sizeof(double) * Nm);
    orc_apply(P, transpose, x, t);                 /* t_y = A_yy y, t_s = A_sy y */
    memset(x, 0, sizeof(double) * N);
    particle_solve(P, transpose, t, x);            /* x_s = A_ss^-1 A_sy y      */
    orc_apply(P, transpose, x, u);                 /* u_y = A_ys x_s            */
    for (long i = 0; i < Nm; i++) out[i] = t[i] - u[i];
    free(x); free(t); free(u);
}

/* bhat = b_y - A_ys A_ss^-1 b_s (length off_cs[0]) */
void orc_schur_rhs(const orc_problem *P, int transpose, const double *b, double *bhat)
{
    long Nm = P->off_cs[0], N = P->N;
    double *x = xmalloc(sizeof(double) * N), *u = xmalloc(sizeof(double) * N);
    memset(x, 0, sizeof(double) * N);
    particle_solve(P, transpose, b, x);
    orc_apply(P, transpose, x, u);
    for (long i = 0; i < Nm; i++) bhat[i] = b[i] - u[i];
    free(x); free(u);
}

/* x_s = A_ss^-1 (b_s - A_sy y), with y = x[0 .. off_cs[0]) given */
void orc_schur_back(const orc_problem *P, int transpose, const double *b, double *x)
{
    long Nm = P->off_cs[0], N = P->N;
    double *xy = xmalloc(sizeof(double) * N), *t = xmalloc(sizeof(double) * N);
    memset(xy, 0, sizeof(double) * N);
    memcpy(xy, x, sizeof(double) * Nm);
    orc_apply(P, transpose, xy, t);                /* t_s = A_sy y */
    for (long i = Nm; i < N; i++) t[i] = b[i] - t[i];
    particle_solve(P, transpose, t, xy);
    memcpy(x + Nm, xy + Nm, sizeof(double) * (N - Nm));
    free(xy); free(t);
}

/* preconditioner of the Schur-complement iteration: the V-cycles on the
 * field blocks S~_f (step 3 of the SCHUR mode), identity on the grounded
 * layer of phi_s                                                            */
static void schur_pc(const orc_problem *P, const double *r, double *z)
{
    const orc_desc *d = &P->d;
    for (long q = 0; q < (long)d->nx * d->ny; q++) z[P->off_ps + q] = r[P->off_ps + q];
    for (int b = 0; b < 4; b++) {
        long off, n;
        box_slice(P, b, &off, &n);
        vcycle(P, &P->mg[b], 0, r + off, z + off);
    }
}

typedef void (*orc_lin_fn)(const orc_problem *, int, const double *, double *);
static void full_op(const orc_problem *P, int t, const double *x, double *y) { orc_apply(P, t, x, y); }
static void full_pc(const orc_problem *P, int t, const double *r, double *z) { orc_apply_pc(P, t, r, z); }
static void schur_op(const orc_problem *P, int t, const double *x, double *y) { orc_schur_apply(P, t, x, y); }
static void schur_pcf(const orc_problem *P, int t, const double *r, double *z) { (void)t; schur_pc(P, r, z); }

/* Restarted right-preconditioned FGMRES on an operator of size n from x0 = 0.
 * Stopping rule: the Givens estimate reaches rtol * bref, after which the
 * true residual is formed; the solve stops when the true residual meets
 * rtol * bref.                                                             */
static int fgmres_core(const orc_problem *P, int transpose, long N, orc_lin_fn op, orc_lin_fn pc,
                       const double *b, double bref, double *x, orc_info *info)
{
    const orc_opts *o = &P->opts;
    int m = o->restart;
    double *V = xmalloc(sizeof(double) * N * (m + 1));
    double *Z = xmalloc(sizeof(double) * N * m);
    double *w = xmalloc(sizeof(double) * N);
    double *H = xmalloc(sizeof(double) * (m + 1) * m);    /* H[i*m + k] */
    double *cs = xmalloc(sizeof(double) * m), *sn = xmalloc(sizeof(double) * m);
    double *gv = xmalloc(sizeof(double) * (m + 1)), *yv = xmalloc(sizeof(double) * m);
    double *hc = xmalloc(sizeof(double) * (m + 1));
    memset(info, 0, sizeof(*info));
    memset(x, 0, sizeof(double) * N);
    double bnorm = bref;
    int status = 1, total = 0;
    if (bnorm == 0.0) {      /* x = 0 is exact */
        status = 0;
        goto done;
    }
    for (;;) {
        op(P, transpose, x, w);
        for (long i = 0; i < N; i++) w[i] = b[i] - w[i];
        double beta = sqrt(dot(w, w, N));
        info->relres_true = beta / bnorm;
        if (beta <= o->rtol * bnorm) { status = 0; break; }
        if (total >= o->maxit) { status = 1; break; }
        for (long i = 0; i < N; i++) V[i] = w[i] / beta;
        memset(gv, 0, sizeof(double) * (m + 1));
        gv[0] = beta;
        int k, kused = 0, breakdown = 0;
        for (k = 0; k < m; k++) {
            double *vk = V + (long)k * N, *zk = Z + (long)k * N;
            pc(P, transpose, vk, zk);
            op(P, transpose, zk, w);
            for (int i = 0; i <= k; i++) hc[i] = 0.0;
            for (int pass = 0; pass < (o->cgs2 ? 2 : 1); pass++) {
                double hp[64];
                for (int i = 0; i <= k; i++) hp[i] = dot(V + (long)i * N, w, N);
                for (int i = 0; i <= k; i++) {
                    const double *vi = V + (long)i * N;
                    for (long q = 0; q < N; q++) w[q] -= hp[i] * vi[q];
                    hc[i] += hp[i];
                }
            }
            double hn = sqrt(dot(w, w, N));
            hc[k + 1] = hn;
            double colnorm = 0.0;
            for (int i = 0; i <= k + 1; i++) colnorm += hc[i] * hc[i];
            colnorm = sqrt(colnorm);
            /* apply earlier rotations, then a new one zeroing hc[k+1] */
            for (int i = 0; i < k; i++) {
                double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
                hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
                hc[i] = t;
            }
            double den = sqrt(hc[k] * hc[k] + hc[k + 1] * hc[k + 1]);
            cs[k] = hc[k] / den;
            sn[k] = hc[k + 1] / den;
            hc[k] = den;
            hc[k + 1] = 0.0;
            gv[k + 1] = -sn[k] * gv[k];
            gv[k] = cs[k] * gv[k];
            for (int i = 0; i <= k; i++) H[i * m + k] = hc[i];
            total++;
            kused = k + 1;
            info->relres_est = fabs(gv[k + 1]) / bnorm;
            if (hn <= 1e-14 * colnorm) { breakdown = 1; break; }
            double *vn = V + (long)(k + 1) * N;
            for (long q = 0; q < N; q++) vn[q] = w[q] / hn;
            if (fabs(gv[k + 1]) <= o->rtol * bnorm || total >= o->maxit) break;
        }
        /* y = H^-1 g (upper triangular), x += Z y */
        for (int i = kused - 1; i >= 0; i--) {
            double v = gv[i];
            for (int j = i + 1; j < kused; j++) v -= H[i * m + j] * yv[j];
            yv[i] = v / H[i * m + i];
        }
        for (int i = 0; i < kused; i++) {
            const double *zi = Z + (long)i * N;
            for (long q = 0; q < N; q++) x[q] += yv[i] * zi[q];
        }
        info->restarts++;
        if (breakdown) {
            op(P, transpose, x, w);
            for (long i = 0; i < N; i++) w[i] = b[i] - w[i];
            info->relres_true = sqrt(dot(w, w, N)) / bnorm;
            status = info->relres_true <= o->rtol ? 0 : 2;
            break;
        }
    }
done:
    info->iters = total;
    info->status = status;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(gv); free(yv); free(hc);
    return status;
}

/* Solves A x = b (A^T x = b if transpose) from x0 = 0 by FGMRES over all
 * unknowns, or (krylov = SCHUR) over the Schur complement S y = b^ followed
 * by x_s = A_ss^-1 (b_s - A_sy y).  Both stop on rtol ||b||: with the c_s
 * rows solved exactly, b - A x is zero in the c_s rows and equals b^ - S y
 * in the others.  relres_true is ||b - A x|| / ||b|| of the returned x.     */
int orc_fgmres(orc_problem *P, int transpose, const double *b, double *x, orc_info *info)
{
    long N = P->N, Nm = P->off_cs[0];
    double bnorm = sqrt(dot(b, b, N));
    if (P->opts.krylov != ORC_KRYLOV_SCHUR)
        return fgmres_core(P, transpose, N, full_op, full_pc, b, bnorm, x, info);
    double *bhat = xmalloc(sizeof(double) * Nm);
    orc_schur_rhs(P, transpose, b, bhat);
    int status = fgmres_core(P, transpose, Nm, schur_op, schur_pcf, bhat, bnorm, x, info);
    orc_schur_back(P, transpose, b, x);
    double *r = xmalloc(sizeof(double) * N);
    orc_apply(P, transpose, x, r);
    for (long i = 0; i < N; i++) r[i] = b[i] - r[i];
    if (bnorm > 0.0) info->relres_true = sqrt(dot(r, r, N)) / bnorm;
    free(r);
    free(bhat);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Parameter gradients of J = w.x with A x = b, A^T lambda = w               */
/* dJ/dp = -lambda^T (dA/dp) x                                               */
/* ------------------------------------------------------------------------ */
/* dJ/dsigma_e for every element (zero on separator elements): only the
 * phi_s stiffness block depends on sigma_e, with element matrix h Khat; the
 * Dirichlet entries carry no sigma dependence.  dJ/dDs[el]: T0 = I/dt - L~,
 * L~ linear in D, so dT0/dD = -L~(D=1).                                    */
void orc_gradient(const orc_problem *P, const double *x, const double *lam,
                  double *dsigma, double *dDs)
{
    const orc_desc *d = &P->d;
#pragma omp parallel for schedule(static)
    for (int ek = 0; ek < d->nz - 1; ek++)
        for (int ej = 0; ej < d->ny - 1; ej++)
            for (int ei = 0; ei < d->nx - 1; ei++) {
                long id = elem_id(P, ei, ej, ek);
                if (elem_mat(P, ek) < 0) { dsigma[id] = 0.0; continue; }
                double xl[8], ll[8];
                for (int a = 0; a < 8; a++) {
                    int i = ei + (a & 1), j = ej + ((a >> 1) & 1), k = ek + ((a >> 2) & 1);
                    long je = enode(P, i, j, k);
                    int dir = is_dirichlet(P, k);
                    xl[a] = dir ? 0.0 : x[P->off_ps + je];
                    ll[a] = dir ? 0.0 : lam[P->off_ps + je];
                }
                double acc = 0.0;
                for (int a = 0; a < 8; a++)
                    for (int b = 0; b < 8; b++) acc += ll[a] * P->h * kelem(P, a, b) * xl[b];
                dsigma[id] = -acc;
            }
    for (int el = 0; el < 2; el++) {
        int N = d->nr[el];
        long nn = el == 0 ? P->nea : P->nec;
        double *lo = xmalloc(sizeof(double) * N), *di = xmalloc(sizeof(double) * N),
               *up = xmalloc(sizeof(double) * N);
        orc_radial_rows(N, 1.0, P->rho[el], lo, di, up);
        const double *xs = x + P->off_cs[el], *ls = lam + P->off_cs[el];
        double acc = 0.0;
        for (long jn = 0; jn < nn; jn++)
            for (int r = 0; r < N; r++) {
                double Lx = di[r] * xs[(long)r * nn + jn];
                if (r > 0) Lx += lo[r] * xs[(long)(r - 1) * nn + jn];
                if (r < N - 1) Lx += up[r] * xs[(long)(r + 1) * nn + jn];
                acc += ls[(long)r * nn + jn] * Lx;
            }
        dDs[el] = acc;
        free(lo); free(di); free(up);
    }
}
