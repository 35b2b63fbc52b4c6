// Internal declarations of the gfx950 solver library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p4d {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxNr = 64;           // radial points per particle
constexpr int kMaxRestart = 64;      // FGMRES restart length
constexpr int kMaxLevels = 16;
constexpr int kRedBlocks = 2048;     // partial-sum slots of the streaming reductions

// Structured grid and model scalars, passed by value to every kernel.
struct Geom {
    int nx, ny, nz, na, ns, nc;
    int nr[2];
    long long nnode, nelem, nea, nec, ne;
    long long off_pe, off_ce, off_cs[2], N, Nm;
    double h, dt, chi, tc;
    double mass_elec, mass_sep;      // eps * vol / dt per element material
    const double *meh = nullptr;     // eps_e * vol / dt per element (device), or by material
    // box elements (edges hx, hy along x, y; h along z): vol = hx hy h, and
    // the Q1 stiffness over h is sum_d (vol / (h_d^2 h)) Khat_d; kw[0] is its
    // diagonal, kw[p] minus its entry between corners differing in the axes
    // of bit pattern p (isotropic: 1/3, and 1/12 for two or three axes)
    int aniso = 0;
    double vol = 0.0;
    double kw[8] = {};
    // Newton terms of a physical cell, set only for its linear solves: the
    // state (SI; phi_e at nwu + off_pe, c_e at nwu + off_ce) and per element
    // h times the scaled c_e-derivatives of kappa_eff, of the
    // diffusion-potential coefficient and of D_eff (null: none)
    const double *nwu = nullptr, *nwa = nullptr, *nwb = nullptr, *nwc = nullptr;
};

__host__ __device__ inline int elem_mat(const Geom &g, int kk)
{
    return kk + 1 < g.na ? 0 : (kk >= g.na + g.ns ? 1 : -1);
}
// storage coefficient eps h^3 / dt of element id (in element layer kk); the
// array is device memory, read as such (through the generic pointer the
// compiler would emit a flat load, which also holds up every LDS wait)
__device__ inline double elem_storage(const Geom &g, long long id, int kk)
{
    return g.meh ? ((const __attribute__((address_space(1))) double *)g.meh)[id]
                 : (elem_mat(g, kk) >= 0 ? g.mass_elec : g.mass_sep);
}
__host__ __device__ inline int node_mat(const Geom &g, int k)
{
    return k < g.na ? 0 : (k >= g.na + g.ns ? 1 : -1);
}

// Per-electrode radial tables (T0 = I/dt - L_h and its shared factorizations).
struct RadialTab {
    int N;
    double Gamma;                    // surface coupling factor (flux term of eq. LR)
    double tau0;                     // (T0^-1)_{NN}
    double tsub[kMaxNr], tdia[kMaxNr], tsup[kMaxNr];   // rows of T0
    double l[kMaxNr], ipiv[kMaxNr], piv[kMaxNr];       // T0 = L U, unit L multipliers
    double lT[kMaxNr];                                 // T0^T = L' U' (same pivots)
    double tN[kMaxNr], tNT[kMaxNr];                    // T0^-1 e_N and T0^-T e_N
    double hsub[kMaxNr], hdia[kMaxNr], hsup[kMaxNr];   // dL_h/dDs
};

// One multigrid level of one box, as seen by a batched launch.  Iterates x
// are FP64 in every precision mode (their near-null component can exceed the
// rest by 1e4..1e6, which FP32 storage would not resolve); T is the storage
// type of everything else.
template <typename T>
struct LevelArgs {
    int nx, ny, nz, n;
    int blk0;                        // first workgroup of this box in the launch
    int k0;                          // level 0: global node layer of local layer 0
    int ek_lo, ek_hi;                // level 0: element layers taking part
    int mass;                        // level 0: add the c_e storage term
    const double *cK;                // level 0: element coefficient (x h)
    const T *S;                      // level >= 1: upper-half stencil, SoA [14][n]
    const T *invd;                   // inverse diagonal
    const T *dcorr;                  // level 0: diagonal reaction correction
    const T *b;
    const double *xin;
    double *xout;
    const T *din;
    T *dout;
    T *rout;
    double c1, c2;                   // Chebyshev step: d' = c1 d + c2 D^-1 r
    int din_x;                       // 1: the previous direction equals x (first
                                     // step from x = 0), read it from xin
};

template <typename T>
struct LevelBatch {
    int nbox;
    LevelArgs<T> a[4];
};

// Restriction / prolongation between level l (fine) and l+1 (coarse).
template <typename T>
struct TransferArgs {
    int fx, fy, fz, cx, cy, cz;
    int blk0;
    const T *rf;                     // fine residual (restriction)
    T *bc;                           // coarse right-hand side (restriction)
    double *xc1;                     // coarse first smoothing iterate, may be null
    const T *invdc;                  // coarse inverse diagonal
    double c2c;                      // coarse first-step coefficient
    const double *xc;                // coarse solution (prolongation)
    double *xf;                      // fine iterate, updated in place
};
template <typename T>
struct TransferBatch {
    int nbox;
    TransferArgs<T> a[4];
};

template <typename T>
struct CoarseArgs {
    int n;
    const double *Ainv;              // dense inverse, column-major
    const T *b;
    double *x;
};
template <typename T>
struct CoarseBatch {
    int nbox;
    CoarseArgs<T> a[4];
};

// The last two levels of a box's V-cycle in one workgroup: the last smoothed
// level F (from the first iterate the restriction left there: smoothing
// steps 2..deg, residual, restriction to the coarsest level, dense coarse
// solve, prolongation, smoothing steps 1..deg) with F's stencil and vectors
// held in LDS.  The arithmetic is that of the per-stage kernels (the same
// device functions), so the results are identical.
template <typename T>
struct TailArgs {
    int nx, ny, nz, n;               // level F
    int cx, cy, cz, nc;              // coarsest level
    const T *S, *invd, *b;           // level F stencil (upper half, [14][n]), inverse diagonal, rhs
    const double *x1;                // level F first iterate
    double *xout;                    // level F final iterate
    const double *Ainv;              // coarsest level: dense inverse, column-major
    double c1[5], c2[5];             // level F Chebyshev steps 1..deg
};
template <typename T>
struct TailBatch {
    int nbox, deg;
    TailArgs<T> a[4];
};
constexpr int kTailLds = 96 * 1024;  // LDS of the tail kernel
constexpr int kTailThreads = 1024;
// LDS bytes the tail needs for a level of n nodes above a coarsest level of nc
template <typename T>
__host__ __device__ constexpr long long tail_lds_bytes(long long n, long long nc)
{
    return 8 * (2 * n + 5 * nc + nc * nc) + (long long)sizeof(T) * (18 * n + nc) + 64;
}

// ---- launchers (each defined beside its kernels) ---------------------------
// operator.hip
// tile_tx > 0 (and qbuf, n_e doubles): macro rows by 2.5D tiles, then the
// particle rows (for y = A x without b or partial sums)
template <typename TX>
void launch_operator(const Geom &g, const RadialTab *tabs, const double *sigh,
                     const double *kaph, const double *gg, const double *ss, const double *ee,
                     const double *mm, const TX *x, double *y, const double *b,
                     double *partial, int transpose, int tile_tx, int tile_cz, double *qbuf,
                     const double *kdh, const double *dch, hipStream_t st);
int operator_blocks(const Geom &g);
int operator_tiles(const Geom &g, int TX, int CZ);
int operator_tile_slots();
void launch_grad(const Geom &g, const RadialTab *tabs, const double *x, const double *lam,
                 double *dsigma, double *partial, hipStream_t st);
void launch_grad_final(const double *partial, int nblk, double *dDs, hipStream_t st);

// radial.hip (RadArgs in p4d_kernels.hpp)
struct RadArgs;
template <typename T>
void launch_rad_fwd(const Geom &g, const RadArgs &R, const double *r, const double *rscale, int transpose,
                    int schur, hipStream_t st);
template <typename T, typename TZ>
void launch_rad_back(const Geom &g, const RadArgs &R, const double *r, const double *rscale, TZ *z,
                     int transpose, int schur, hipStream_t st);
// size class of the per-thread radial register arrays: the largest N_r of
// the two electrodes rounded up to 8, 12, 16, 20, 24, 32 or 64
int rad_nrmax(const Geom &g);
constexpr int kNrClasses = 7;
constexpr int kNrClass[kNrClasses] = {8, 12, 16, 20, 24, 32, 64};
#define P4D_NR_SWITCH(nr, M)   \
    switch (nr) {              \
    case 8: M(8); break;       \
    case 12: M(12); break;     \
    case 16: M(16); break;     \
    case 20: M(20); break;     \
    case 24: M(24); break;     \
    case 32: M(32); break;     \
    default: M(64); break;     \
    }

// mg.hip
// level-0 smoother, 2.5D tiles of TX x (256/TX) nodes and CZ layers;
// TX in {16, 32, 64}
template <typename T>
void launch_smooth0(const Geom &g, const LevelBatch<T> &lb, int nblk, int resid_only, int TX,
                    int CZ, hipStream_t st);
int smooth0_tiles(int nx, int ny, int nz, int TX, int CZ);
int smooth0_slots();
template <typename T>
void launch_smooth(const LevelBatch<T> &lb, int nblk, int resid_only, hipStream_t st);
template <typename T>
void launch_restrict(const TransferBatch<T> &tb, int nblk, hipStream_t st);
template <typename T>
void launch_prolong(const TransferBatch<T> &tb, int nblk, hipStream_t st);
template <typename T>
void launch_coarse(const CoarseBatch<T> &cb, hipStream_t st);
template <typename T>
void launch_tail(const TailBatch<T> &tb, hipStream_t st);
void launch_assemble0(const Geom &g, int box, int nz, int k0, int ek_lo, int ek_hi, int mass,
                      const double *cK, const double *dcorr, double *S, hipStream_t st);
// Galerkin product P^T S P as three 1D coarsenings (x, y, z), for up to four
// boxes per launch; tmp of each job needs 27 * (cx*fy*fz + cx*cy*fz) doubles
// Level-0 rows of one multigrid box from its element data (the arguments of
// the level-0 assembly): formed on the fly where the stored stencil would
// only be read once
struct Elem0 {
    int nzb, k0, ek_lo, ek_hi, mass;
    const double *cK, *dcorr;
};
// Per-box arguments of the batched level preparation: at level 0 the
// inverse diagonal from the element rows, at levels >= 1 the difference
// form and inverse diagonal from the stored stencil; both raise the box's
// Gershgorin bound, kept as the bits of a non-negative double so that an
// integer atomic maximum gives it exactly (in any order)
struct PrepArgs {
    int n, blk0;
    const double *S;                 // levels >= 1: Galerkin stencil [27][n]
    void *D, *invd;                  // levels >= 1: difference form [14][n], inverse diagonal (T)
    Elem0 E;                         // level 0: element data of the box
    double *invd0;                   // level 0: FP64 inverse diagonal
    unsigned long long *lmax;
};
struct PrepBatch {
    int nbox;
    PrepArgs a[4];
};
constexpr int kLmaxSlots = 32;       // atomic slots per Gershgorin bound
template <typename T>
void launch_level_prep_batch(const PrepBatch &pb, int nblk, hipStream_t st);
void launch_diag0_batch(const Geom &g, const PrepBatch &pb, int nblk, hipStream_t st);
struct RapArgs {
    int nx, ny, nz;          // input dims of this 1D coarsening
    int blk0;
    const double *Sf;        // null: level-0 rows from e0
    double *Sc;
    Elem0 e0;
};
struct RapBatch {
    int nbox;
    RapArgs a[4];
};
struct RapJob {
    int fx, fy, fz;
    const double *Sf;        // null: level-0 rows formed from e0
    double *Sc;
    double *tmp;
    Elem0 e0;
};
// zc = 0: z is not coarsened (P_z = I), the x and y passes only; the jobs
// either all read a stored stencil or all form level-0 rows
void launch_rap(const Geom &g, const RapJob *jobs, int njobs, int zc, hipStream_t st);

// z-line smoothing of up to four boxes of one level (FP64, full stencils
// [27][n]): block Gauss-Seidel over the lines of one colour (x parity
// colour & 1, y parity colour >> 1), in place in x.  A box's z extent is at
// most kZlineMaxNz (a line's rows and a chunk of staged x planes must fit
// the 64 KB of LDS).
constexpr int kZlineLds = 65536;
constexpr int kZlineMaxNz = 2016;
struct LineArgs {
    int nx, ny, nz, n, blk0;
    int lt, kc;                      // sweep tile width and chunk depth (set by launch_zline)
    const double *S;                 // [27][n], natural node order (residual)
    const double *Sz;                // the same rows in the sweeps' order (launch_zline_order)
    const double *b;
    double *x;
    double *r;
};
struct LineBatch {
    int nbox;
    LineArgs a[4];
};
void launch_zline(LineBatch lb, int colour, hipStream_t st);
// r = b - S x on the same boxes
void launch_resid_full(LineBatch lb, hipStream_t st);
// Sz = the rows of S ([27][n] on an nx x ny x nz box) reordered as the
// z-line sweeps read them: colour by colour, then by tiles of up to 8 lines
// consecutive along x, then layer k, coefficient and line; a coefficient
// whose neighbour lies off the box is stored as +0
void launch_zline_order(int nx, int ny, int nz, const double *S, double *Sz, hipStream_t st);
void launch_diag(int n, const double *S, double *invd, unsigned long long *lmax, int nblk,
                 hipStream_t st);
// levels >= 1 in one pass: the smoother's stored stencil D in T (slot 0 the
// row sum formed in FP64, slots 1..13 the upper half), the inverse diagonal
// in T, Gershgorin ratio block maxima in ratio_partial
template <typename T>
void launch_level_prep(int n, const double *S, T *D, T *invd, double *ratio_partial, int nblk,
                       hipStream_t st);
// the same for level 0 with its rows formed from the element data
void launch_diag0(const Geom &g, const Elem0 &E, int n, double *invd, double *ratio_partial, int nblk,
                  hipStream_t st);
void launch_max_final(const double *partial, int nblk, double *out, hipStream_t st);
void launch_dense_from_stencil(int nx, int ny, int nz, const double *S, double *A,
                               hipStream_t st);
struct InvBatch {
    int nbox;
    int n[4];
    double *A[4];
    double *Ainv[4];
};
void launch_invert(const InvBatch &ib, hipStream_t st);
// out = factor * in per element, or factor * def where in is null
void launch_scale_elem(const Geom &g, const double *in, double factor, const double *def, double *out,
                       hipStream_t st);
void launch_setup_nodes(const Geom &g, const RadialTab *tabs, const double *sigma,
                        const double *kappa, double *sigh, double *kaph, double *mm,
                        hipStream_t st);
template <typename T>
void launch_dcorr(const Geom &g, const double *gg, const double *ee, const double *mm,
                  const double *omega, T *dcorr0, hipStream_t st);
void launch_omega(const Geom &g, const RadialTab *tabs, const double *ss, int schur,
                  double *omega, hipStream_t st);
template <typename T>
void launch_cast(long long n, const double *src, T *dst, hipStream_t st);

// operator.hip: the Schur complement of the particle blocks (electrode-level
// vectors of length Nm)
template <typename TX>
void launch_operator_schur(const Geom &g, const RadialTab *tabs, const double *sigh,
                           const double *kaph, const double *gg, const double *ss, const double *ee,
                           const double *mm, const double *om, const TX *y, double *w, int transpose,
                           int tile_tx, int tile_cz, const double *kdh, const double *dch, hipStream_t st);
// reduced.hip
void launch_red_rhs(const Geom &g, const RadialTab *tabs, const double *gg, const double *ss,
                    const double *ee, const double *mm, const double *b, double *bhat, int transpose,
                    hipStream_t st);
void launch_red_back(const Geom &g, const RadialTab *tabs, const double *gg, const double *ss,
                     const double *ee, const double *mm, const double *b, double *x, int transpose,
                     hipStream_t st);
void launch_red_resid(long long n, const double *bhat, double *w, double *partial, int nblk,
                      hipStream_t st);

// krylov.hip
int stream_blocks(long long n);
// basis vector q at V + q ldv, except vector 0 at v0 (the first cycle's
// right-hand side, read in place)
void launch_mdot(long long n, const double *w, const double *V, const double *v0, long long ldv, int nv,
                 double *partial, int nblk, hipStream_t st);
void launch_mdot_final(int nv, const double *partial, int nblk, const double *invbeta,
                       double *h, double *c, hipStream_t st);
void launch_orth(long long n, double *w, const double *V, const double *v0, long long ldv, int nv,
                 const double *c, double *partial, int nblk, hipStream_t st);
void launch_norm_final(const double *partial, int nblk, double *beta_out, double *invbeta_out,
                       hipStream_t st);
// x += Z y, or x = Z y with assign (x is not read)
template <typename TZ>
void launch_zy(long long n, double *x, const TZ *Z, long long ldz, int nv, const double *y, int assign,
               hipStream_t st);
void launch_dot_partial(long long n, const double *a, const double *b, double *partial,
                        int nblk, hipStream_t st);
// n 64-bit values from src (device) to dst (mapped host memory, its device
// address), then seq to seq_out (mapped host memory) once they are visible
void launch_publish(const void *src, int n, void *dst, unsigned long long *seq_out, unsigned long long seq,
                    hipStream_t st);

}  // namespace p4d
