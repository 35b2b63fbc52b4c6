// Batched solves of many independent cells of uneven size in lockstep:
//  - the preconditioner of every iterating cell by a few launches per stage
//    depth, each over all cells;
//  - batched operator and Krylov streaming kernels over a table of cells.
//
// Every cell's preconditioner application is a fixed sequence of stages
// (particle forward elimination, the V-cycle stages of its four boxes level
// by level, particle back-substitution), recorded once with the same
// schedule as the single-cell path.  A stage splits into workgroup-sized
// units (tiles, 256-node blocks, 64-row blocks).  The stages are placed at
// depths: the descending half of a V-cycle from the first depth on, the
// ascending half (from the first prolongation) so that it ends at the last
// depth, so the stages with the same role in cells of different depth line
// up.  The units of one depth, split by stage family (and, for the particle
// stages, by radial size class), form work lists, larger cells first; one
// launch runs one list, one unit per workgroup.  The launches of one
// application are ordered by the stream and no workgroup ever waits for
// another.
//
// Each unit computes exactly what the single-cell kernels compute for the
// same block or tile (the same device functions), so a cell solved in a
// batch follows the same arithmetic as the cell solved alone.
#include <hip/hip_cooperative_groups.h>

#include "p4d_batch.hpp"

namespace p4d {

// The stage, cell and queue tables do not change while a kernel runs.  Read
// through the constant address space, their fields arrive by scalar loads
// and the compiler knows that the pointers among them address global
// memory; read through a generic pointer, every access through those
// pointers stays a flat access, which also holds every LDS and scalar-load
// wait behind the outstanding memory operations.
template <typename X>
using Ctab = __attribute__((address_space(4))) const X;
template <typename X>
__device__ inline Ctab<X> *ctab(const X *p)
{
    return (Ctab<X> *)p;
}
// a copy of a table entry (for types whose copy constructor does not take a
// constant-address-space source)
template <typename X>
__device__ inline X ld(Ctab<X> &r)
{
    X v;
    __builtin_memcpy(&v, (const void *)&r, sizeof(X));
    return v;
}

// ---------------------------------------------------------------------------
// Batched preconditioner stages.  Every launch runs one work list: units of
// one stage family (see StageFamily) from the stages of one depth, one unit
// per workgroup.  A kernel per family keeps the register and LDS footprint
// of that family's block function only.
// ---------------------------------------------------------------------------
__device__ inline int find_pos(Ctab<int> *ustart, int npos, int item)
{
    int lo = 0, hi = npos - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ustart[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct UnitRef {
    int si;      // stage index
    int unit;    // unit within the stage
};

// The unit of this workgroup; the values are the same in every lane, and
// marking them so lets the stage arguments be read into scalar registers.
__device__ inline UnitRef unit_of(const StageRun &run)
{
    const int item = run.item0 + xcd_block(blockIdx.x, gridDim.x);
    const int pos = __builtin_amdgcn_readfirstlane(run.pos0 + find_pos(ctab(run.ustart + run.pos0), run.npos, item));
    const int si = __builtin_amdgcn_readfirstlane(ctab(run.order)[pos]);
    const int unit = __builtin_amdgcn_readfirstlane(item - ctab(run.ustart)[pos]);
    return UnitRef{si, unit};
}

template <typename T, int NRMAX>
__global__ __launch_bounds__(kBlock) void k_bstage_radf(StageRun run)
{
    const UnitRef u = unit_of(run);
    Ctab<PStage<T>> &S = ctab((const PStage<T> *)run.stages)[u.si];
    if (!((run.active >> S.cell) & 1ULL)) return;   // the cell is not iterating
    // local copies: the cell's constants stay in registers across the
    // unit's stores
    const PCell Cm = ld(ctab(run.cells)[S.cell]);
    const Geom g = Cm.g;
    const RadArgs R = Cm.R;
    const double *r = Cm.V + (long long)run.k * g.N;
    const double rs = Cm.invbeta[run.k];
    if (Cm.schur) {
        if (run.transpose) rad_fwd_block<T, NRMAX, true, true>(g, R, r, rs, u.unit);
        else rad_fwd_block<T, NRMAX, false, true>(g, R, r, rs, u.unit);
    } else {
        rad_fwd_block<T, NRMAX, false, false>(g, R, r, rs, u.unit);
    }
}

template <typename T, typename TZ, int NRMAX>
__global__ __launch_bounds__(kBlock) void k_bstage_radb(StageRun run)
{
    const UnitRef u = unit_of(run);
    Ctab<PStage<T>> &S = ctab((const PStage<T> *)run.stages)[u.si];
    if (!((run.active >> S.cell) & 1ULL)) return;
    const PCell Cm = ld(ctab(run.cells)[S.cell]);
    const Geom g = Cm.g;
    const RadArgs R = Cm.R;
    const double *r = Cm.V + (long long)run.k * g.N;
    const double rs = Cm.invbeta[run.k];
    TZ *z = (TZ *)Cm.Z + (long long)run.k * g.N;
    if (Cm.schur) {
        if (run.transpose) rad_back_block<T, TZ, NRMAX, true, true>(g, R, r, rs, z, u.unit);
        else rad_back_block<T, TZ, NRMAX, false, true>(g, R, r, rs, z, u.unit);
    } else {
        if (run.transpose) rad_back_block<T, TZ, NRMAX, true, false>(g, R, r, rs, z, u.unit);
        else rad_back_block<T, TZ, NRMAX, false, false>(g, R, r, rs, z, u.unit);
    }
}

// KINDS: the stage kinds in the list (1: smoothing steps only, 2: residuals
// only, 3: both), so that a list of one kind carries the registers of that
// kind's tile function only
template <typename T, int KINDS>
__global__ __launch_bounds__(kBlock) void k_bstage_sm0(StageRun run)
{
    __shared__ Smooth0Lds lds;
    const UnitRef u = unit_of(run);
    Ctab<PStage<T>> &S = ctab((const PStage<T> *)run.stages)[u.si];
    if (!((run.active >> S.cell) & 1ULL)) return;
    const LevelArgs<T> A = ld(S.u.lb.a[__builtin_amdgcn_readfirstlane(find_box(S.u.lb, u.unit))]);
    const Geom g = ld(ctab(run.cells)[S.cell]).g;
    const int TX = S.TX, CZ = S.CZ;
    if (KINDS == 1 || (KINDS == 3 && S.kind == SK_SM0)) smooth0_tile<T, false>(g, A, u.unit - A.blk0, TX, CZ, lds);
    else smooth0_tile<T, true>(g, A, u.unit - A.blk0, TX, CZ, lds);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bstage_misc(StageRun run)
{
    __shared__ CoarseLds lds;
    const UnitRef u = unit_of(run);
    Ctab<PStage<T>> &S = ctab((const PStage<T> *)run.stages)[u.si];
    if (!((run.active >> S.cell) & 1ULL)) return;
    const int unit = u.unit;
    switch (S.kind) {
    case SK_SM:
    case SK_SMR: {
        const LevelArgs<T> A = ld(S.u.lb.a[find_box(S.u.lb, unit)]);
        if (S.kind == SK_SM) smooth_block<T, false>(A, unit - A.blk0);
        else smooth_block<T, true>(A, unit - A.blk0);
        break;
    }
    case SK_RESTRICT: {
        const TransferArgs<T> A = ld(S.u.tb.a[find_box(S.u.tb, unit)]);
        restrict_block<T>(A, unit - A.blk0);
        break;
    }
    case SK_PROLONG: {
        const TransferArgs<T> A = ld(S.u.tb.a[find_box(S.u.tb, unit)]);
        prolong_block<T>(A, unit - A.blk0);
        break;
    }
    case SK_COARSE: {
        const int box = unit / S.aux, rb = unit % S.aux;
        if (box < S.u.cb.nbox) {
            const CoarseArgs<T> A = ld(S.u.cb.a[box]);
            if (rb * 64 < A.n) coarse_block<T>(A, rb, lds);
        }
        break;
    }
    default:
        break;
    }
}

template <typename T, typename TZ>
void launch_batch_stage(const StageRun &run, int family, int nrmax, int kinds, hipStream_t st)
{
    if (run.nitems <= 0) return;
    const dim3 grid(run.nitems), block(kBlock);
    switch (family) {
    case SF_RADF:
#define P4D_BF(NR) hipLaunchKernelGGL((k_bstage_radf<T, NR>), grid, block, 0, st, run)
        P4D_NR_SWITCH(nrmax, P4D_BF)
#undef P4D_BF
        break;
    case SF_RADB:
#define P4D_BB(NR) hipLaunchKernelGGL((k_bstage_radb<T, TZ, NR>), grid, block, 0, st, run)
        P4D_NR_SWITCH(nrmax, P4D_BB)
#undef P4D_BB
        break;
    case SF_SM0:
        if (kinds == 1) hipLaunchKernelGGL((k_bstage_sm0<T, 1>), grid, block, 0, st, run);
        else if (kinds == 2) hipLaunchKernelGGL((k_bstage_sm0<T, 2>), grid, block, 0, st, run);
        else hipLaunchKernelGGL((k_bstage_sm0<T, 3>), grid, block, 0, st, run);
        break;
    default:
        hipLaunchKernelGGL((k_bstage_misc<T>), grid, block, 0, st, run);
        break;
    }
}
#define P4D_INST(T, TZ) template void launch_batch_stage<T, TZ>(const StageRun &, int, int, int, hipStream_t);
P4D_INST(double, double)
P4D_INST(float, double)
P4D_INST(double, float)
P4D_INST(float, float)
#undef P4D_INST

// ---------------------------------------------------------------------------
// Persistent application (see PersistRun)
// ---------------------------------------------------------------------------
union PersistLds {
    Smooth0Lds s0;
    CoarseLds co;
};

// one unit of a stage: the device function of its family, as in the
// per-depth kernels above
template <typename T, typename TZ, int NRMAX>
__device__ inline void persist_unit(const PersistRun &run, Ctab<PStage<T>> &S, int unit, PersistLds &L)
{
    const PCell Cm = ld(ctab(run.cells)[S.cell]);
    switch (stage_family(S.kind)) {
    case SF_RADF: {
        const Geom g = Cm.g;
        const RadArgs R = Cm.R;
        const double *r = Cm.V + (long long)run.k * g.N;
        const double rs = Cm.invbeta[run.k];
        if (Cm.schur) {
            if (run.transpose) rad_fwd_block<T, NRMAX, true, true>(g, R, r, rs, unit);
            else rad_fwd_block<T, NRMAX, false, true>(g, R, r, rs, unit);
        } else {
            rad_fwd_block<T, NRMAX, false, false>(g, R, r, rs, unit);
        }
        break;
    }
    case SF_RADB: {
        const Geom g = Cm.g;
        const RadArgs R = Cm.R;
        const double *r = Cm.V + (long long)run.k * g.N;
        const double rs = Cm.invbeta[run.k];
        TZ *z = (TZ *)Cm.Z + (long long)run.k * g.N;
        if (Cm.schur) {
            if (run.transpose) rad_back_block<T, TZ, NRMAX, true, true>(g, R, r, rs, z, unit);
            else rad_back_block<T, TZ, NRMAX, false, true>(g, R, r, rs, z, unit);
        } else {
            if (run.transpose) rad_back_block<T, TZ, NRMAX, true, false>(g, R, r, rs, z, unit);
            else rad_back_block<T, TZ, NRMAX, false, false>(g, R, r, rs, z, unit);
        }
        break;
    }
    case SF_SM0: {
        const LevelArgs<T> A = ld(S.u.lb.a[__builtin_amdgcn_readfirstlane(find_box(S.u.lb, unit))]);
        const Geom g = Cm.g;
        if (S.kind == SK_SM0) smooth0_tile<T, false>(g, A, unit - A.blk0, S.TX, S.CZ, L.s0);
        else smooth0_tile<T, true>(g, A, unit - A.blk0, S.TX, S.CZ, L.s0);
        break;
    }
    default:
        switch (S.kind) {
        case SK_SM:
        case SK_SMR: {
            const LevelArgs<T> A = ld(S.u.lb.a[find_box(S.u.lb, unit)]);
            if (S.kind == SK_SM) smooth_block<T, false>(A, unit - A.blk0);
            else smooth_block<T, true>(A, unit - A.blk0);
            break;
        }
        case SK_RESTRICT: {
            const TransferArgs<T> A = ld(S.u.tb.a[find_box(S.u.tb, unit)]);
            restrict_block<T>(A, unit - A.blk0);
            break;
        }
        case SK_PROLONG: {
            const TransferArgs<T> A = ld(S.u.tb.a[find_box(S.u.tb, unit)]);
            prolong_block<T>(A, unit - A.blk0);
            break;
        }
        case SK_COARSE: {
            const int box = unit / S.aux, rb = unit % S.aux;
            if (box < S.u.cb.nbox) {
                const CoarseArgs<T> A = ld(S.u.cb.a[box]);
                if (rb * 64 < A.n) coarse_block<T>(A, rb, L.co);
            }
            break;
        }
        default:
            break;
        }
        break;
    }
}

// All stage depths of one application in one cooperative launch: the grid
// walks the work items of a depth (item = workgroup + j x grid size, every
// family in one list), then meets at the runtime's grid barrier before the
// next depth, so each depth sees the whole previous depth complete, as with
// one launch per depth.  No workgroup waits for another except at that
// barrier, which every workgroup reaches once per depth.
template <typename T, typename TZ, int NRMAX>
__global__ __launch_bounds__(kBlock) void k_bpc_persist(PersistRun run)
{
    __shared__ PersistLds lds;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int d = 0; d < run.ndepth; d++) {
        const int i0 = run.dstart[d], i1 = run.dstart[d + 1];
        for (int item = i0 + (int)blockIdx.x; item < i1; item += (int)gridDim.x) {
            const int pos = __builtin_amdgcn_readfirstlane(find_pos(ctab(run.ustart), run.npos, item));
            const int si = __builtin_amdgcn_readfirstlane(ctab(run.order)[pos]);
            Ctab<PStage<T>> &S = ctab((const PStage<T> *)run.stages)[si];
            if (!((run.active >> S.cell) & 1ULL)) continue;   // (uniform in the workgroup)
            persist_unit<T, TZ, NRMAX>(run, S, item - run.ustart[pos], lds);
        }
        grid.sync();
    }
}

template <typename T, typename TZ>
hipError_t launch_batch_persist(const PersistRun &run, int nrmax, int grid, hipStream_t st)
{
    void *args[] = {(void *)&run};
    const void *f = nullptr;
#define P4D_BPF(NR) f = (const void *)k_bpc_persist<T, TZ, NR>
    P4D_NR_SWITCH(nrmax, P4D_BPF)
#undef P4D_BPF
    return hipLaunchCooperativeKernel(f, dim3(grid), dim3(kBlock), args, 0, st);
}

// workgroups of the cooperative kernel resident at once (its grid size)
template <typename T, typename TZ>
int batch_persist_slots(int nrmax)
{
    int dev = 0, ncu = 0, per = 0, coop = 0;
    const void *f = nullptr;
#define P4D_BPF(NR) f = (const void *)k_bpc_persist<T, TZ, NR>
    P4D_NR_SWITCH(nrmax, P4D_BPF)
#undef P4D_BPF
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kBlock, 0) != hipSuccess || per < 1)
        return 0;
    return per * ncu;
}
#define P4D_INST(T, TZ)                                                                           \
    template hipError_t launch_batch_persist<T, TZ>(const PersistRun &, int, int, hipStream_t);  \
    template int batch_persist_slots<T, TZ>(int);
P4D_INST(double, double)
P4D_INST(float, double)
P4D_INST(double, float)
P4D_INST(float, float)
#undef P4D_INST

// workgroups of the batched level-0 smoother (its smoothing steps) resident at once
template <typename T>
int bstage_sm0_slots()
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_bstage_sm0<T, 1>, kBlock, 0) !=
            hipSuccess)
        return 1024;
    return (per < 1 ? 1 : per) * (ncu < 1 ? 1 : ncu);
}
template int bstage_sm0_slots<double>();
template int bstage_sm0_slots<float>();

// ---------------------------------------------------------------------------
// Batched operator and Krylov streaming kernels.  The workgroups of the
// cells follow each other in the grid (offsets in the cell table); those of
// cells outside the active mask return at once.  Per cell, the partition of
// the work and the order of every reduction are those of the single-cell
// kernels.
// ---------------------------------------------------------------------------
// the cell of batched workgroup b, by the offsets of one launch kind
enum { SEL_OP = 0, SEL_ST, SEL_TILE, SEL_RAD };
template <int SEL>
__device__ inline int find_cell(const BCell *cells, int ncells, int b)
{
    int lo = 0, hi = ncells - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        Ctab<BCell> &M = ctab(cells)[mid];
        const int b0 = SEL == SEL_OP ? M.op_blk0
                                     : (SEL == SEL_ST ? M.st_blk0 : (SEL == SEL_TILE ? M.tile_blk0 : M.rad_blk0));
        if (b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// V_0 = b - A x with per-workgroup sums of squares, one thread per node
template <typename TX, int NRMAX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_bop_resid(const BCell *__restrict__ cells, int ncells,
                                                      unsigned long long active)
{
    __shared__ double red[4];
    const int gb = xcd_block(blockIdx.x, gridDim.x);
    const int c = find_cell<SEL_OP>(cells, ncells, gb);
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const int lb = gb - C.op_blk0;
    const long long n = (long long)lb * kBlock + threadIdx.x;
    OpArgs O = C.op;
    O.x = C.x;
    O.y = C.V;
    O.b = C.b;
    const Geom g = C.g;
    double sq = 0.0;
    if (n < g.nnode) sq = operator_node<TX, NRMAX, TRANS, true>(g, O, n);
    const double s = block_sum(sq, red);
    if (threadIdx.x == 0) C.red[lb] = s;
}

// V_{k+1} = A Z_k: macro rows over 2.5D tiles of every cell ...
template <typename TX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_bop_tile(const BCell *__restrict__ cells, int ncells,
                                                     unsigned long long active, int k)
{
    __shared__ OpLds L;
    const int gb = xcd_block(blockIdx.x, gridDim.x);
    const int c = find_cell<SEL_TILE>(cells, ncells, gb);
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const Geom g = C.g;
    OpArgs O = C.op;
    O.x = (const TX *)C.Z + (long long)k * g.N;
    O.y = C.V + (long long)(k + 1) * g.N;
    O.b = nullptr;
    operator_tile<TX, TRANS>(g, O, C.qbuf, gb - C.tile_blk0, C.op_tx, C.op_cz, L);
}

// ... then the particle rows of every cell
template <typename TX, int NRMAX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_bop_radial(const BCell *__restrict__ cells, int ncells,
                                                       unsigned long long active, int k)
{
    const int c = find_cell<SEL_RAD>(cells, ncells, blockIdx.x);
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const Geom g = C.g;
    const long long je = (long long)(blockIdx.x - C.rad_blk0) * kBlock + threadIdx.x;
    if (je >= g.ne) return;
    OpArgs O = C.op;
    O.x = (const TX *)C.Z + (long long)k * g.N;
    O.y = C.V + (long long)(k + 1) * g.N;
    O.b = nullptr;
    operator_radial<TX, NRMAX, TRANS>(g, O, C.qbuf, je);
}

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_bmdot(const BCell *__restrict__ cells, int ncells,
                                                  unsigned long long active, int k)
{
    __shared__ double red[4][KMAX];
    const int c = find_cell<SEL_ST>(cells, ncells, blockIdx.x);
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const int lb = blockIdx.x - C.st_blk0, nb = C.st_nblk;
    const long long N = C.g.N;
    const int nv = k + 1;
    const double *__restrict__ V = C.V;
    const double *__restrict__ w = V + (long long)(k + 1) * N;
    double acc[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; q++) acc[q] = 0.0;
    for (long long i = (long long)lb * kBlock + threadIdx.x; i < N; i += (long long)nb * kBlock) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < KMAX; q++)
            if (q < nv) acc[q] += wi * V[(long long)q * N + i];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < KMAX; q++) {
        if (q < nv) {
            const double s = wave_sum(acc[q]);
            if (lane == 0) red[wv][q] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv)
        C.red[(long long)threadIdx.x * nb + lb] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// grid (nv, ncells): h_q = invbeta_q * sum_b partial[q][b], c_q = h_q * invbeta_q
__global__ __launch_bounds__(kBlock) void k_bmdot_final(const BCell *__restrict__ cells,
                                                        unsigned long long active, int pass)
{
    __shared__ double red[4];
    const int q = blockIdx.x, c = blockIdx.y;
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const int nb = C.st_nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += C.red[(long long)q * nb + b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double hq = s * C.invbeta[q];
        C.h[64 * pass + q] = hq;
        C.coef[q] = hq * C.invbeta[q];
    }
}

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_borth(const BCell *__restrict__ cells, int ncells,
                                                  unsigned long long active, int k)
{
    __shared__ double red[4];
    const int c = find_cell<SEL_ST>(cells, ncells, blockIdx.x);
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const int lb = blockIdx.x - C.st_blk0, nb = C.st_nblk;
    const long long N = C.g.N;
    const int nv = k + 1;
    const double *__restrict__ V = C.V;
    double *__restrict__ w = C.V + (long long)(k + 1) * N;
    double cq[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; q++) cq[q] = q < nv ? C.coef[q] : 0.0;
    double sq = 0.0;
    for (long long i = (long long)lb * kBlock + threadIdx.x; i < N; i += (long long)nb * kBlock) {
        double wi = w[i];
#pragma unroll
        for (int q = 0; q < KMAX; q++)
            if (q < nv) wi -= cq[q] * V[(long long)q * N + i];
        w[i] = wi;
        sq += wi * wi;
    }
    const double s = block_sum(sq, red);
    if (threadIdx.x == 0) C.red[lb] = s;
}

// grid ncells: beta = sqrt(sum of the cell's partials) into h[128] and
// 1/beta into invbeta[slot] (0 when beta = 0); op = 1 reduces the operator
// partials
__global__ __launch_bounds__(kBlock) void k_bnorm_final(const BCell *__restrict__ cells,
                                                        unsigned long long active, int slot, int op)
{
    __shared__ double red[4];
    const int c = blockIdx.x;
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const int nb = op ? C.op_nblk : C.st_nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += C.red[b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double bt = sqrt(s);
        C.h[128] = bt;
        C.invbeta[slot] = bt > 0.0 ? 1.0 / bt : 0.0;
    }
}

template <typename TZ, int KMAX>
__global__ __launch_bounds__(kBlock) void k_bzy(const BCell *__restrict__ cells, int ncells,
                                                unsigned long long active)
{
    const int c = find_cell<SEL_ST>(cells, ncells, blockIdx.x);
    const BCell C = ld(ctab(cells)[c]);
    if (!((active >> c) & 1ULL)) return;
    const int lb = blockIdx.x - C.st_blk0, nb = C.st_nblk;
    const long long N = C.g.N;
    const int nv = *C.kused;
    double yq[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; q++) yq[q] = q < nv ? C.y[q] : 0.0;
    const TZ *__restrict__ Z = (const TZ *)C.Z;
    double *__restrict__ x = C.x;
    for (long long i = (long long)lb * kBlock + threadIdx.x; i < N; i += (long long)nb * kBlock) {
        double xi = x[i];
#pragma unroll
        for (int q = 0; q < KMAX; q++)
            if (q < nv) xi += yq[q] * (double)Z[(long long)q * N + i];
        x[i] = xi;
    }
}

// per cell: partial sums of ||b||^2, x = 0, V_0 = b
__global__ __launch_bounds__(kBlock) void k_bstart(const BCell *__restrict__ cells, int ncells)
{
    __shared__ double red[4];
    const int c = find_cell<SEL_ST>(cells, ncells, blockIdx.x);
    const BCell C = ld(ctab(cells)[c]);
    const int lb = blockIdx.x - C.st_blk0, nb = C.st_nblk;
    const long long N = C.g.N;
    double s = 0.0;
    for (long long i = (long long)lb * kBlock + threadIdx.x; i < N; i += (long long)nb * kBlock) {
        const double bi = C.b[i];
        s += bi * bi;
        C.x[i] = 0.0;
        C.V[i] = bi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) C.red[lb] = s;
}

void launch_bstart(const BCell *cells, int ncells, int nblk_st, hipStream_t st)
{
    hipLaunchKernelGGL(k_bstart, dim3(nblk_st), dim3(kBlock), 0, st, cells, ncells);
}

template <typename TZ>
void launch_bop(const BCell *cells, int ncells, unsigned long long active, int k, int resid,
                int transpose, int nblk_op, int nblk_tile, int nblk_rad, int nrmax, hipStream_t st)
{
    if (resid) {
#define P4D_BR(NR)                                                                                \
    do {                                                                                          \
        if (transpose)                                                                            \
            hipLaunchKernelGGL((k_bop_resid<double, NR, true>), dim3(nblk_op), dim3(kBlock), 0, st, \
                               cells, ncells, active);                                            \
        else                                                                                      \
            hipLaunchKernelGGL((k_bop_resid<double, NR, false>), dim3(nblk_op), dim3(kBlock), 0, st,\
                               cells, ncells, active);                                            \
    } while (0)
        P4D_NR_SWITCH(nrmax, P4D_BR)
#undef P4D_BR
        return;
    }
    if (transpose)
        hipLaunchKernelGGL((k_bop_tile<TZ, true>), dim3(nblk_tile), dim3(kBlock), 0, st, cells, ncells,
                           active, k);
    else
        hipLaunchKernelGGL((k_bop_tile<TZ, false>), dim3(nblk_tile), dim3(kBlock), 0, st, cells, ncells,
                           active, k);
#define P4D_BRA(NR)                                                                                \
    do {                                                                                           \
        if (transpose)                                                                             \
            hipLaunchKernelGGL((k_bop_radial<TZ, NR, true>), dim3(nblk_rad), dim3(kBlock), 0, st,     \
                               cells, ncells, active, k);                                          \
        else                                                                                       \
            hipLaunchKernelGGL((k_bop_radial<TZ, NR, false>), dim3(nblk_rad), dim3(kBlock), 0, st,    \
                               cells, ncells, active, k);                                          \
    } while (0)
    P4D_NR_SWITCH(nrmax, P4D_BRA)
#undef P4D_BRA
}
template void launch_bop<double>(const BCell *, int, unsigned long long, int, int, int, int, int, int,
                                 int, hipStream_t);
template void launch_bop<float>(const BCell *, int, unsigned long long, int, int, int, int, int, int,
                                int, hipStream_t);

void launch_bmdot(const BCell *cells, int ncells, unsigned long long active, int k, int nblk_st,
                  int pass, hipStream_t st)
{
    const int nv = k + 1;
#define P4D_BM(K) \
    hipLaunchKernelGGL((k_bmdot<K>), dim3(nblk_st), dim3(kBlock), 0, st, cells, ncells, active, k)
    if (nv <= 4) P4D_BM(4);
    else if (nv <= 8) P4D_BM(8);
    else if (nv <= 16) P4D_BM(16);
    else if (nv <= 32) P4D_BM(32);
    else P4D_BM(64);
#undef P4D_BM
    hipLaunchKernelGGL(k_bmdot_final, dim3(nv, ncells), dim3(kBlock), 0, st, cells, active, pass);
}

void launch_borth(const BCell *cells, int ncells, unsigned long long active, int k, int nblk_st,
                  hipStream_t st)
{
    const int nv = k + 1;
#define P4D_BR(K) \
    hipLaunchKernelGGL((k_borth<K>), dim3(nblk_st), dim3(kBlock), 0, st, cells, ncells, active, k)
    if (nv <= 4) P4D_BR(4);
    else if (nv <= 8) P4D_BR(8);
    else if (nv <= 16) P4D_BR(16);
    else if (nv <= 32) P4D_BR(32);
    else P4D_BR(64);
#undef P4D_BR
}

void launch_bnorm_final(const BCell *cells, int ncells, unsigned long long active, int slot, int op,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_bnorm_final, dim3(ncells), dim3(kBlock), 0, st, cells, active, slot, op);
}

template <typename TZ>
void launch_bzy(const BCell *cells, int ncells, unsigned long long active, int kmax, int nblk_st,
                hipStream_t st)
{
#define P4D_BZ(K) \
    hipLaunchKernelGGL((k_bzy<TZ, K>), dim3(nblk_st), dim3(kBlock), 0, st, cells, ncells, active)
    if (kmax <= 4) P4D_BZ(4);
    else if (kmax <= 8) P4D_BZ(8);
    else if (kmax <= 16) P4D_BZ(16);
    else if (kmax <= 32) P4D_BZ(32);
    else P4D_BZ(64);
#undef P4D_BZ
}
template void launch_bzy<double>(const BCell *, int, unsigned long long, int, int, hipStream_t);
template void launch_bzy<float>(const BCell *, int, unsigned long long, int, int, hipStream_t);

}  // namespace p4d
