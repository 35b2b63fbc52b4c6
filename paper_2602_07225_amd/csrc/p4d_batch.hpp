// Internal declarations of the batched solver: many independent cells, each
// with its own mesh, radial sizes and coefficients, iterate in lockstep.
#pragma once
#include "p4d_internal.hpp"
#include "p4d_kernels.hpp"

namespace p4d {

constexpr int kMaxBatch = 64;            // cells per batch (one bit each in a 64-bit mask)
constexpr int kMaxStagesPerCell = 256;   // preconditioner stages recorded per cell

// Stages of one preconditioner application of one cell, in execution order.
enum StageKind : int {
    SK_RADF = 0,     // particle forward elimination and Schur right-hand side
    SK_SM0,          // level-0 Chebyshev step (2.5D tiles)
    SK_SM0R,         // level-0 residual
    SK_SM,           // level >= 1 Chebyshev step
    SK_SMR,          // level >= 1 residual
    SK_RESTRICT,
    SK_PROLONG,
    SK_COARSE,       // dense coarsest-level solve
    SK_RADB          // particle back-substitution and output
};

template <typename T>
union StageArgs {
    LevelBatch<T> lb;
    TransferBatch<T> tb;
    CoarseBatch<T> cb;
};

template <typename T>
struct PStage {
    int kind;
    int cell;
    int nunits;          // workgroup-sized units of work
    int TX, CZ;          // level-0 smoother tile shape
    int aux;             // coarse solve: 64-row blocks per box
    StageArgs<T> u;
};

// Per-cell constants of the batched preconditioner.
struct PCell {
    Geom g;
    RadArgs R;               // tables, coefficients, level-0 buffers and final iterates
    const double *V;         // Krylov basis, [m+1][N], unnormalized
    void *Z;                 // preconditioned directions, [m][N]
    const double *invbeta;   // 1 / ||V_k||
    int schur;
};

// One launch: the work list of one stage depth (queue positions
// [pos0, pos0 + npos), units [item0, item0 + nitems)).
struct StageRun {
    const void *stages;      // PStage<T>[]
    const PCell *cells;
    const int *order;        // queue position -> stage index
    const int *ustart;       // queue position -> first unit of that stage
    int pos0, npos;
    int item0, nitems;
    int transpose;
    int k;                   // Arnoldi step: r = V_k / beta_k, z -> Z_k
    unsigned long long active;
};

// Stage families: each has its own batched kernel.
enum StageFamily : int {
    SF_RADF = 0,     // SK_RADF
    SF_RADB,         // SK_RADB
    SF_SM0,          // SK_SM0, SK_SM0R
    SF_MISC          // coarse levels: SK_SM, SK_SMR, SK_RESTRICT, SK_PROLONG, SK_COARSE
};
__host__ __device__ inline int stage_family(int kind)
{
    return kind == SK_RADF ? SF_RADF
                           : (kind == SK_RADB ? SF_RADB
                                              : (kind == SK_SM0 || kind == SK_SM0R ? SF_SM0 : SF_MISC));
}

template <typename T, typename TZ>
void launch_batch_stage(const StageRun &run, int family, int nrmax, int kinds, hipStream_t st);

// One launch for a whole preconditioner application of all cells: the work
// items of all stage depths (the units of the per-depth work lists, depth
// after depth), walked depth by depth by a cooperative grid with a grid
// barrier between depths.
struct PersistRun {
    const void *stages;          // PStage<T>[]
    const PCell *cells;
    const int *order;            // queue position -> stage index
    const int *ustart;           // queue position -> first item of that stage
    const int *dstart;           // depth -> first item; [ndepth]: item count
    int npos, ndepth;
    int transpose, k;
    unsigned long long active;
};
template <typename T, typename TZ>
hipError_t launch_batch_persist(const PersistRun &run, int nrmax, int grid, hipStream_t st);
template <typename T, typename TZ>
int batch_persist_slots(int nrmax);   // 0: no cooperative launch
template <typename T>
int bstage_sm0_slots();

// Per-cell constants of the batched operator and Krylov kernels.
struct BCell {
    Geom g;
    OpArgs op;               // tables and coefficients (x, y, b set per launch)
    int op_blk0, op_nblk;    // one-thread-per-node operator workgroups in the batched grid
    int st_blk0, st_nblk;    // streaming workgroups
    int tile_blk0, tile_n;   // tiled operator workgroups
    int rad_blk0, rad_n;     // particle-row workgroups
    int op_tx, op_cz;        // operator tile shape
    double *qbuf;            // reaction q per electrode node
    double *V;
    void *Z;
    double *x;
    const double *b;
    double *red;             // partial sums
    double *h;               // [0,64): pass-1 h, [64,128): pass-2 h, [128]: a norm
    double *coef;            // Gram-Schmidt coefficients
    double *invbeta;
    const double *y;         // least-squares coefficients of the finished cycle
    const int *kused;        // their number
};

void launch_bstart(const BCell *cells, int ncells, int nblk_st, hipStream_t st);
// resid: V_0 = b - A x (one thread per node, with partial sums); else
// V_{k+1} = A Z_k (tiled macro rows, then the particle rows)
template <typename TZ>
void launch_bop(const BCell *cells, int ncells, unsigned long long active, int k, int resid,
                int transpose, int nblk_op, int nblk_tile, int nblk_rad, int nrmax, hipStream_t st);
void launch_bmdot(const BCell *cells, int ncells, unsigned long long active, int k, int nblk_st,
                  int pass, hipStream_t st);
void launch_borth(const BCell *cells, int ncells, unsigned long long active, int k, int nblk_st,
                  hipStream_t st);
void launch_bnorm_final(const BCell *cells, int ncells, unsigned long long active, int slot, int op,
                        hipStream_t st);
template <typename TZ>
void launch_bzy(const BCell *cells, int ncells, unsigned long long active, int kmax, int nblk_st,
                hipStream_t st);

}  // namespace p4d
