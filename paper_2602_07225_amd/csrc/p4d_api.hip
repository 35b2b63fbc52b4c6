// C ABI of the solver (include/p4d.h): context and workspace management,
// the per-electrode radial tables, preconditioner setup and application,
// and the restarted flexible GMRES driver.  All per-node, per-element and
// per-DOF work runs in the HIP kernels of operator.hip, radial.hip, mg.hip
// and krylov.hip; the host only computes O(N_r) radial tables, O(levels)
// Chebyshev coefficients and the (m+1) x m Hessenberg least-squares problem.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/p4d.h"
#include "p4d_batch.hpp"
#include "p4d_bgs.hpp"
#include "p4d_phys.hpp"

using namespace p4d;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Level {
    int nx = 0, ny = 0, nz = 0, n = 0;
    double lmax = 0.0;
    double *S64 = nullptr;   // persistent FP64 Galerkin stencil (levels >= 1)
    double *Sz = nullptr;    // z-line smoothing: S64's rows in the sweeps' order
    void *S = nullptr;       // smoother copy in the preconditioner precision,
                             // centre slot = FP64 row sum (difference form)
    void *invd = nullptr, *b = nullptr, *xa = nullptr, *xb = nullptr, *d = nullptr, *r = nullptr;
    double *Ainv = nullptr;  // coarsest level
};

struct Box {
    int nlev = 0;
    int k0 = 0, ek_lo = 0, ek_hi = 0, mass = 0;
    long long off = 0;       // offset of level 0 in the macro layout
    const double *cK = nullptr;
    Level lev[kMaxLevels];
};

// Newton state of a physical cell
struct PhysState {
    p4d_phys_params prm{};
    PhysDev P{};
    double *uh = nullptr, *rh = nullptr, *dh = nullptr, *old = nullptr, *fh = nullptr, *qh = nullptr;
    double *por = nullptr, *act = nullptr;   // porosity, active fraction per element (Case II)
    double *nwa = nullptr, *nwb = nullptr, *nwc = nullptr;   // Newton-term coefficients per element
    bool ready = false;
};

struct Prof {
    int mask = 0;
    int every = 1;                // time one launch in `every` of each class
    long long seen[P4D_K_COUNT] = {};
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<double> bytes;    // per pair
    std::vector<int> cls;         // per pair
    std::vector<int> count;       // launches per pair
    int used = 0;
    double total_ms[P4D_K_COUNT] = {}, total_bytes[P4D_K_COUNT] = {};
    long long launches[P4D_K_COUNT] = {};
};

}  // namespace

struct p4d_ctx {
    p4d_problem_desc desc{};
    Geom g{};
    RadialTab tabs_h[2];
    std::string err;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    p4d_solve_opts ws_opts{};
    // device arrays
    RadialTab *tabs = nullptr;
    double *sigh = nullptr, *kaph = nullptr, *gg = nullptr, *ss = nullptr, *ee = nullptr,
           *mm = nullptr, *omega = nullptr, *qbuf = nullptr;
    double *oms = nullptr;         // omega_j of the Schur complement (whatever the preconditioner)
    double *kdh = nullptr, *dch = nullptr;   // h * separate transport coefficients
    double *meh = nullptr;         // eps_e vol / dt per element (when storage is set)
    int storage = 0;               // 1: g.meh points at meh
    int transport_set = 0;         // 1: kdh / dch hold caller coefficients
    int general = 0;               // 1: kdh / dch hold the transport coefficients
    PhysState *phys = nullptr;     // physical cell (p4d_phys_create)
    double *red = nullptr;         // partial sums
    size_t red_len = 0;
    double *hdev = nullptr, *cdev = nullptr, *invbeta = nullptr, *ydev = nullptr, *scal = nullptr;
    // preconditioner
    int uploaded = 0, pc_ready = 0;
    p4d_solve_opts pc{};
    int prec = 0;                  // 0 FP64, 1 FP32
    Box box[4];
    void *b0 = nullptr, *x0a = nullptr, *x0b = nullptr, *d0 = nullptr, *r0 = nullptr,
         *invd0 = nullptr, *dcorr0 = nullptr;
    char *scratch = nullptr;       // Krylov basis region, also setup scratch
    size_t scratch_bytes = 0;
    double *hhost = nullptr;       // pinned host staging
    // values handed from the device to the host (launch_publish): mapped,
    // coherent pinned memory (slots of kPubMax values and a sequence number)
    unsigned long long *hpub = nullptr, *hpub_dev = nullptr;
    unsigned long long pub_seq = 0;
    // Gershgorin bounds of the last setup still on their way (finish_setup)
    int lmax_pending = 0;
    unsigned long long lmax_seq = 0;
    hipStream_t lmax_stream = nullptr;
    int tile_tx = 64, tile_cz = 8; // level-0 smoother tiles
    int tiles_tuned = 0;           // set by the autotuner; else chosen at layout time
    int op_tx = 64, op_cz = 4;     // operator tiles (op_tx = 0: one thread per node)
    int box_mask = 15;             // multigrid boxes a V-cycle runs on (bit per box)
    Prof prof;
    // record mode: the preconditioner schedule is appended to a stage list
    // (std::vector<PStage<T>>) instead of being launched
    void *rec = nullptr;
    int rec_cell = 0;
    RadArgs rec_R{};
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static p4d_status fail(p4d_ctx *c, p4d_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}
static p4d_status hipchk(p4d_ctx *c, hipError_t e, const char *where)
{
    if (e == hipSuccess) return P4D_OK;
    return fail(c, P4D_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIPCHK(c, call)                                            \
    do {                                                           \
        p4d_status _s = hipchk((c), (call), #call);                \
        if (_s != P4D_OK) return _s;                               \
    } while (0)

static int coarse_n_h(int n) { return n <= 2 ? n : n / 2 + 1; }

// Device values the host waits for (norms, Hessenberg columns, Gershgorin
// bounds): a one-workgroup kernel copies them into mapped host memory and
// then raises a sequence number, on which the host spins.  The handoff costs
// a few microseconds less than a copy and a stream synchronization, and the
// solve makes one per Arnoldi step.  Two slots for the solve, so that the
// values of one step can be on their way while the host still reads the
// previous step's, and one for the setup.
constexpr int kPubMax = 2048;
constexpr int kPubStride = kPubMax + 16;   // slot: kPubMax values, then the sequence number
constexpr int kPubSlots = 3;               // 0, 1: the solve; 2: the setup's bounds
constexpr int kPubSetup = 2;
static p4d_status alloc_pub(p4d_ctx *c)
{
    void *h = nullptr, *d = nullptr;
    if (hipHostMalloc(&h, 8 * kPubSlots * kPubStride, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return P4D_ERR_HIP;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        hipHostFree(h);
        return P4D_ERR_HIP;
    }
    c->hpub = (unsigned long long *)h;
    c->hpub_dev = (unsigned long long *)d;
    for (int q = 0; q < kPubSlots; q++) c->hpub[q * kPubStride + kPubMax] = 0;
    c->pub_seq = 0;
    return P4D_OK;
}

// n (<= kPubMax) 64-bit values at src (device) to slot `slot` of c->hpub,
// after the work already on st; returns the sequence number to wait for
static unsigned long long publish(p4d_ctx *c, const void *src, int n, int slot, hipStream_t st)
{
    const unsigned long long seq = ++c->pub_seq;
    launch_publish(src, n, c->hpub_dev + slot * kPubStride, c->hpub_dev + slot * kPubStride + kPubMax, seq,
                   st);
    return seq;
}

// Wait until slot `slot` holds the values of publish number seq.  An error
// of the stream ends the wait with that error.
static p4d_status await_pub(p4d_ctx *c, int slot, unsigned long long seq, hipStream_t st)
{
    HIPCHK(c, hipGetLastError());
    volatile unsigned long long *flag = c->hpub + slot * kPubStride + kPubMax;
    for (long long polls = 1; *flag != seq; polls++) {
        if ((polls & 1023) == 0) {
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) {
                if (*flag == seq) break;
                return fail(c, P4D_ERR_HIP, "a value handed to the host did not arrive");
            }
            if (e != hipErrorNotReady) return hipchk(c, e, "hipStreamQuery");
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return P4D_OK;
}

// publish into slot 0 and wait: the values are then at c->hpub
static p4d_status pull(p4d_ctx *c, const void *src, int n, hipStream_t st)
{
    return await_pub(c, 0, publish(c, src, n, 0, st), st);
}

// Geometric radial mesh on [0, 1] with Delta_{i+1} = q Delta_i and
// Delta_{N-1} / Delta_1 = theta_bar (Sec. 3.1, after Remark 3.1).
static void radial_table(const p4d_problem_desc &d, int el, RadialTab &T)
{
    const int N = d.nr[el];
    std::vector<double> rho(N), dr(N - 1);
    const double q = std::pow(d.theta_bar[el], 1.0 / (N - 2));
    double s = 0.0, f = 1.0;
    for (int i = 0; i < N - 1; i++) { s += f; f *= q; }
    f = 1.0 / s;
    rho[0] = 0.0;
    for (int i = 0; i < N - 1; i++) { dr[i] = f; rho[i + 1] = rho[i] + f; f *= q; }
    rho[N - 1] = 1.0;
    for (int i = 0; i < N - 1; i++) dr[i] = rho[i + 1] - rho[i];
    // L_h rows for unit diffusivity: centre eq. (L0), interior eq. (L1)+(L2),
    // surface eq. (LR) without the flux term.
    std::memset(&T, 0, sizeof(T));
    T.N = N;
    std::vector<double> lo(N, 0.0), di(N, 0.0), up(N, 0.0);
    di[0] = -6.0 / (dr[0] * dr[0]);
    up[0] = 6.0 / (dr[0] * dr[0]);
    for (int i = 1; i < N - 1; i++) {
        const double hm = dr[i - 1], hp = dr[i], th = hp / hm;
        const double a1 = 2.0 / (rho[i] * hp * (1.0 + th));   // first-derivative part
        const double a2 = 2.0 / (hp * hm * (1.0 + th));       // second-derivative part
        lo[i] = -th * th * a1 + th * a2;
        di[i] = -(1.0 - th * th) * a1 - (1.0 + th) * a2;
        up[i] = a1 + a2;
    }
    const double hl = dr[N - 2];
    lo[N - 1] = 2.0 / (hl * hl);
    di[N - 1] = -2.0 / (hl * hl);
    // surface coupling: the flux term 2 i_n/(F dr)(1 + dr/R) of eq. (LR), with
    // the sign of eq. (particleBC2), enters R_cs,N with +Gamma
    T.Gamma = (d.lambda_el[el] > 0.0 ? d.lambda_el[el] : d.lambda_c) * 2.0 * (1.0 + hl) / hl;
    const double D = d.Ds[el];
    for (int i = 0; i < N; i++) {
        T.hsub[i] = lo[i];
        T.hdia[i] = di[i];
        T.hsup[i] = up[i];
        T.tsub[i] = -D * lo[i];
        T.tdia[i] = 1.0 / d.dt - D * di[i];
        T.tsup[i] = -D * up[i];
    }
    T.tsub[0] = 0.0;
    T.tsup[N - 1] = 0.0;
    // T0 = L U (unit lower bidiagonal L, U with diagonal piv and T0's
    // superdiagonal); T0^T = L' U' has the same pivots.
    T.piv[0] = T.tdia[0];
    for (int i = 1; i < N; i++) {
        T.l[i] = T.tsub[i] / T.piv[i - 1];
        T.lT[i] = T.tsup[i - 1] / T.piv[i - 1];
        T.piv[i] = T.tdia[i] - T.l[i] * T.tsup[i - 1];
    }
    for (int i = 0; i < N; i++) T.ipiv[i] = 1.0 / T.piv[i];
    T.tau0 = 1.0 / T.piv[N - 1];   // (T0^-1)_{NN}
    // T0^-1 e_N and T0^-T e_N: forward elimination of e_N leaves e_N, then
    // back substitution with U (superdiagonal tsup) or U' (tsub shifted)
    T.tN[N - 1] = T.tNT[N - 1] = T.ipiv[N - 1];
    for (int i = N - 2; i >= 0; i--) {
        T.tN[i] = -T.tsup[i] * T.tN[i + 1] * T.ipiv[i];
        T.tNT[i] = -T.tsub[i + 1] * T.tNT[i + 1] * T.ipiv[i];
    }
}

static void fill_geom(const p4d_problem_desc &d, Geom &g)
{
    g.nx = d.nx; g.ny = d.ny; g.nz = d.nz; g.na = d.na; g.ns = d.ns;
    g.nc = d.nz - d.na - d.ns;
    g.nr[0] = d.nr[0]; g.nr[1] = d.nr[1];
    g.nnode = (long long)d.nx * d.ny * d.nz;
    g.nelem = (long long)(d.nx - 1) * (d.ny - 1) * (d.nz - 1);
    g.nea = (long long)d.nx * d.ny * d.na;
    g.nec = (long long)d.nx * d.ny * g.nc;
    g.ne = g.nea + g.nec;
    g.off_pe = g.ne;
    g.off_ce = g.ne + g.nnode;
    g.off_cs[0] = g.off_ce + g.nnode;
    g.off_cs[1] = g.off_cs[0] + (long long)d.nr[0] * g.nea;
    g.N = g.off_cs[1] + (long long)d.nr[1] * g.nec;
    g.Nm = g.off_cs[0];
    g.h = (d.length > 0.0 ? d.length : 1.0) / (d.nz - 1);
    g.dt = d.dt;
    g.chi = d.chi;
    g.tc = d.tc;
    const double hx = d.hxy[0] > 0.0 ? d.hxy[0] : g.h, hy = d.hxy[1] > 0.0 ? d.hxy[1] : g.h;
    g.aniso = hx != g.h || hy != g.h;
    g.vol = hx * hy * g.h;
    g.mass_elec = d.eps_elec * g.vol / d.dt;
    g.mass_sep = d.eps_sep * g.vol / d.dt;
    if (!g.aniso) {
        g.kw[0] = 1.0 / 3.0;
        for (int p = 1; p < 8; p++) g.kw[p] = p == 1 || p == 2 || p == 4 ? 0.0 : 1.0 / 12.0;
    } else {
        const double w[3] = {hy / hx, hx / hy, hx * hy / (g.h * g.h)};
        for (int p = 0; p < 8; p++) {
            double k = 0.0;
            for (int ax = 0; ax < 3; ax++) {
                double v = (p >> ax) & 1 ? -1.0 : 1.0;
                for (int q = 0; q < 3; q++)
                    if (q != ax) v *= (p >> q) & 1 ? 1.0 / 6.0 : 1.0 / 3.0;
                k += w[ax] * v;
            }
            g.kw[p] = p == 0 ? k : -k;
        }
    }
}

// level dims of the four multigrid boxes
// (z-line smoothing keeps z: coarsening in x and y only)
static void box_dims(const p4d_ctx *c, int b, int coarse_max, int zline, int *nlev, int dims[][3])
{
    const Geom &g = c->g;
    int nz = b == 0 ? g.na - 1 : (b == 1 ? g.nc : g.nz);
    int d0[3] = {g.nx, g.ny, nz};
    int L = 0;
    for (;;) {
        dims[L][0] = d0[0]; dims[L][1] = d0[1]; dims[L][2] = d0[2];
        const long long n = (long long)d0[0] * d0[1] * d0[2];
        const int cx = coarse_n_h(d0[0]), cy = coarse_n_h(d0[1]);
        const int cz = zline ? d0[2] : coarse_n_h(d0[2]);
        L++;
        if (n <= coarse_max || (long long)cx * cy * cz == n || L == kMaxLevels) break;
        d0[0] = cx; d0[1] = cy; d0[2] = cz;
    }
    *nlev = L;
}

// Carves the workspace (base == nullptr: sizing only).  Returns bytes.
static size_t carve(p4d_ctx *c, const p4d_solve_opts &o, char *base)
{
    const Geom &g = c->g;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    const size_t ts = o.pc_prec == P4D_FP32 ? sizeof(float) : sizeof(double);
    c->tabs = (RadialTab *)take(2 * sizeof(RadialTab));
    c->sigh = (double *)take(8 * g.nelem);
    c->kaph = (double *)take(8 * g.nelem);
    c->gg = (double *)take(8 * g.ne);
    c->ss = (double *)take(8 * g.ne);
    c->ee = (double *)take(8 * g.ne);
    c->mm = (double *)take(8 * g.ne);
    c->omega = (double *)take(8 * g.ne);
    c->qbuf = (double *)take(8 * g.ne);          // reaction q of the tiled operator
    c->oms = (double *)take(8 * g.ne);
    c->kdh = (double *)take(8 * g.nelem);
    c->dch = (double *)take(8 * g.nelem);
    c->meh = (double *)take(8 * g.nelem);
    // reduction partials: streaming (kRedBlocks x 64), operator, gradient
    size_t rl = (size_t)kRedBlocks * 64;
    const size_t opb = (size_t)operator_blocks(g) + 1;
    const size_t grb = 2 * (size_t)(((g.nelem > g.ne ? g.nelem : g.ne) + kBlock - 1) / kBlock) + 2;
    rl = rl > opb ? rl : opb;
    rl = rl > grb ? rl : grb;
    c->red_len = rl;
    c->red = (double *)take(8 * rl);
    c->hdev = (double *)take(8 * 256);
    c->cdev = (double *)take(8 * 256);
    c->invbeta = (double *)take(8 * 128);
    c->ydev = (double *)take(8 * 128);
    c->scal = (double *)take(8 * 128);
    const long long Nm = g.Nm;
    c->b0 = take(ts * Nm);
    c->x0a = take(8 * Nm);          // iterates are FP64 in every mode
    c->x0b = take(8 * Nm);
    c->d0 = take(ts * Nm);
    c->r0 = take(ts * Nm);
    c->invd0 = take(ts * Nm);
    c->dcorr0 = take(ts * Nm);
    const long long layer = (long long)g.nx * g.ny;
    size_t setup_need = 0;
    for (int b = 0; b < 4; b++) {
        Box &B = c->box[b];
        int dims[kMaxLevels][3];
        box_dims(c, b, o.coarse_max, o.smoother == P4D_SMOOTH_ZLINE, &B.nlev, dims);
        B.k0 = b == 0 ? 1 : (b == 1 ? g.na + g.ns : 0);
        B.ek_lo = b == 0 ? 0 : (b == 1 ? g.na + g.ns : 0);
        B.ek_hi = b == 0 ? g.na - 2 : g.nz - 2;
        B.mass = b == 3;
        B.off = b == 0 ? layer : (b == 1 ? g.nea : (b == 2 ? g.off_pe : g.off_ce));
        B.cK = b <= 1 ? c->sigh : ((b == 3 && c->general) ? c->dch : c->kaph);
        for (int l = 0; l < B.nlev; l++) {
            Level &L = B.lev[l];
            L.nx = dims[l][0]; L.ny = dims[l][1]; L.nz = dims[l][2];
            L.n = L.nx * L.ny * L.nz;
            if (l == 0) {
                auto at = [&](void *p, size_t es) -> void * {
                    return base ? (void *)((char *)p + es * B.off) : nullptr;
                };
                L.b = at(c->b0, ts); L.xa = at(c->x0a, 8); L.xb = at(c->x0b, 8);
                L.d = at(c->d0, ts); L.r = at(c->r0, ts); L.invd = at(c->invd0, ts);
                L.S = nullptr;
                // z-line smoothing reads the assembled level-0 stencil
                L.S64 = o.smoother == P4D_SMOOTH_ZLINE ? (double *)take(8 * 27 * (size_t)L.n) : nullptr;
            } else {
                L.S64 = (double *)take(8 * 27 * (size_t)L.n);
                L.S = take(ts * 14 * (size_t)L.n);   // upper half, difference form
                L.invd = take(ts * L.n);
                L.b = take(ts * L.n);
                L.xa = take(8 * (size_t)L.n);
                L.xb = take(8 * (size_t)L.n);
                L.d = take(ts * L.n);
                L.r = take(ts * L.n);
            }
            L.Sz = o.smoother == P4D_SMOOTH_ZLINE && l < B.nlev - 1 ? (double *)take(8 * 27 * (size_t)L.n)
                                                                     : nullptr;
            if (l == B.nlev - 1) {
                L.Ainv = (double *)take(8 * (size_t)L.n * L.n);
                setup_need += align_up(8 * (size_t)L.n * L.n);   // dense copy per box
            }
        }
    }
    // setup scratch: level-0 FP64 stencils of all boxes + FP64 dcorr and
    // inverse diagonal + dense coarse matrix
    size_t s0 = 0;
    for (int b = 0; b < 4; b++) s0 += align_up(8 * 27 * (size_t)c->box[b].lev[0].n);
    size_t rapmax = 0;
    for (int b = 0; b < 4; b++) {
        const Box &B = c->box[b];
        for (int l = 0; l + 1 < B.nlev; l++) {
            const Level &F = B.lev[l];
            const size_t cx = coarse_n_h(F.nx), cy = coarse_n_h(F.ny);
            const size_t t = 27 * (cx * F.ny * F.nz + cx * cy * F.nz);
            rapmax = t > rapmax ? t : rapmax;
        }
    }
    s0 += 2 * align_up(8 * (size_t)Nm) + align_up(8 * 4 * rapmax) + align_up(setup_need);
    // Krylov basis
    const int m = o.restart;
    const size_t zs = o.z_fp32 ? sizeof(float) : sizeof(double);
    const size_t kry_full = align_up(8 * (size_t)(m + 1) * g.N) + align_up(zs * (size_t)m * g.N);
    // the Schur-complement iteration: V and Z over the electrode-level
    // unknowns plus its right-hand side
    const size_t kry_red = align_up(8 * (size_t)(m + 1) * Nm) + align_up(zs * (size_t)m * Nm) +
                           align_up(8 * (size_t)Nm);
    const size_t kry = kry_full > kry_red ? kry_full : kry_red;
    c->scratch_bytes = kry > s0 ? kry : s0;
    c->scratch = take(c->scratch_bytes);
    return off;
}

static bool opts_valid(const p4d_solve_opts &o, std::string &why)
{
    if (o.pc != P4D_PC_SCHUR && o.pc != P4D_PC_BJ && o.pc != P4D_PC_BGS) { why = "pc"; return false; }
    if (o.krylov != P4D_KRYLOV_FULL && o.krylov != P4D_KRYLOV_SCHUR) { why = "krylov"; return false; }
    if (o.krylov == P4D_KRYLOV_SCHUR && o.pc != P4D_PC_SCHUR) {
        why = "the Schur-complement Krylov space needs pc P4D_PC_SCHUR";
        return false;
    }
    if (o.pc == P4D_PC_BGS) {
        int seen = 0;
        for (int p = 0; p < 4; p++) seen |= 1 << ((o.bgs_order >> (2 * p)) & 3);
        if (seen != 15 || (o.bgs_order >> 8) != 0) {
            why = "bgs_order must pack an ordering of the four fields";
            return false;
        }
    }
    if (o.pc_prec != P4D_FP64 && o.pc_prec != P4D_FP32) { why = "pc_prec"; return false; }
    if (o.restart < 1 || o.restart > kMaxRestart) { why = "restart must be in 1..64"; return false; }
    if (o.maxit < 0) { why = "maxit"; return false; }
    if (o.cheb_degree < 1 || o.cheb_degree > 4) { why = "cheb_degree must be in 1..4"; return false; }
    if (o.coarse_max < 8 || o.coarse_max > 1024) { why = "coarse_max must be in 8..1024"; return false; }
    if (!(o.rtol > 0.0) || !(o.rtol < 1.0)) { why = "rtol must be in (0,1)"; return false; }
    if (o.smoother != P4D_SMOOTH_CHEB && o.smoother != P4D_SMOOTH_ZLINE) { why = "smoother"; return false; }
    if (o.smoother == P4D_SMOOTH_ZLINE && (o.pc_prec != P4D_FP64 || o.pc == P4D_PC_BGS)) {
        why = "z-line smoothing needs an FP64 preconditioner and pc SCHUR or BJ";
        return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// profiling: event pairs around launches of one kernel class
// ---------------------------------------------------------------------------
static void prof_harvest(Prof &P)
{
    for (int i = 0; i < P.used; i++) {
        hipEventSynchronize(P.ev[2 * i + 1]);
        float ms = 0.f;
        hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]);
        P.total_ms[P.cls[i]] += ms;
        P.total_bytes[P.cls[i]] += P.bytes[i];
        P.launches[P.cls[i]] += P.count[i];
    }
    P.used = 0;
}
static void prof_init(Prof &P)
{
    P.ev.resize(2 * 512);
    P.bytes.resize(512);
    P.cls.resize(512);
    P.count.resize(512);
    for (auto &e : P.ev) hipEventCreate(&e);
}
static void prof_free(Prof &P)
{
    for (auto &e : P.ev) hipEventDestroy(e);
    P.ev.clear();
}
static void prof_reset(Prof &P, int mask)
{
    prof_harvest(P);
    P.mask = mask;
    for (int k = 0; k < P4D_K_COUNT; k++) {
        P.total_ms[k] = 0.0;
        P.total_bytes[k] = 0.0;
        P.launches[k] = 0;
        P.seen[k] = 0;
    }
}
// An event pair around `count` back-to-back launches of one class (their
// bytes added with add() when the pair is opened with bytes 0); one pair in
// P.every of each class is recorded
struct ProfScope {
    Prof &P;
    bool on;
    hipStream_t st;
    ProfScope(Prof &P_, int cls, double bytes, hipStream_t s, int count = 1) : P(P_), on(false), st(s)
    {
        if (!(P.mask & (1 << cls)) || count < 1) return;
        if (P.seen[cls]++ % P.every) return;
        if (P.used * 2 + 2 > (int)P.ev.size()) prof_harvest(P);
        P.bytes[P.used] = bytes;
        P.cls[P.used] = cls;
        P.count[P.used] = count;
        hipEventRecord(P.ev[2 * P.used], st);
        on = true;
    }
    void add(double bytes)
    {
        if (on) P.bytes[P.used] += bytes;
    }
    ~ProfScope()
    {
        if (!on) return;
        hipEventRecord(P.ev[2 * P.used + 1], st);
        P.used++;
    }
};

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
template <typename TX>
static void apply_op(p4d_ctx *c, int transpose, const TX *x, double *y, const double *b,
                     double *partial, hipStream_t st)
{
    const Geom &g = c->g;
    const double bytes = (double)sizeof(TX) * g.N + 8.0 * g.N + (b ? 8.0 * g.N : 0.0) +
                         16.0 * g.nelem + 32.0 * g.ne;
    ProfScope ps(c->prof, P4D_K_OPERATOR, bytes, st);
    launch_operator<TX>(g, c->tabs, c->sigh, c->kaph, c->gg, c->ss, c->ee, c->mm, x, y, b,
                        partial, transpose, c->op_tx, c->op_cz, c->qbuf,
                        c->general ? c->kdh : nullptr, c->general ? c->dch : nullptr, st);
}

// w = S y (S^T y) over the electrode-level unknowns
template <typename TX>
static void apply_op_schur(p4d_ctx *c, int transpose, const TX *y, double *w, hipStream_t st)
{
    const Geom &g = c->g;
    const double bytes = (double)(sizeof(TX) + 8) * g.Nm + 16.0 * g.nelem + 40.0 * g.ne;
    ProfScope ps(c->prof, P4D_K_OPERATOR, bytes, st);
    launch_operator_schur<TX>(g, c->tabs, c->sigh, c->kaph, c->gg, c->ss, c->ee, c->mm, c->oms, y, w,
                              transpose, c->op_tx, c->op_cz, c->general ? c->kdh : nullptr,
                              c->general ? c->dch : nullptr, st);
}

// ---------------------------------------------------------------------------
// multigrid V-cycle over the four boxes, level by level
// ---------------------------------------------------------------------------
namespace {
struct ChebCoef {
    double c1[5], c2[5];   // per step t = 1..deg (index t)
};
ChebCoef cheb_coef(double lmax, int deg)
{
    ChebCoef C{};
    const double lmin = lmax / 4.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    C.c1[1] = 0.0;
    C.c2[1] = 1.0 / theta;
    for (int t = 2; t <= deg; t++) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        C.c1[t] = rn * rho;
        C.c2[t] = 2.0 * rn / delta;
        rho = rn;
    }
    return C;
}
}  // namespace

template <typename T>
struct VState {
    int xcur[4][kMaxLevels];   // 0: xa, 1: xb holds the current iterate
};

static double *lvx(Level &L, int which) { return (double *)(which ? L.xb : L.xa); }

template <typename T>
static PStage<T> &rec_stage(p4d_ctx *c, int kind, int nunits)
{
    auto &v = *(std::vector<PStage<T>> *)c->rec;
    v.emplace_back();
    PStage<T> &S = v.back();
    std::memset((void *)&S, 0, sizeof(S));
    S.kind = kind;
    S.cell = c->rec_cell;
    S.nunits = nunits;
    S.TX = c->tile_tx;
    S.CZ = c->tile_cz;
    return S;
}

// grp: the event pair of the level-0 steps it belongs to (or null: a pair
// of its own)
template <typename T>
static void smooth_step(p4d_ctx *c, VState<T> &vs, int l, const int *boxes, int nb, int step,
                        int post, hipStream_t st, ProfScope *grp = nullptr)
{
    // step index t (1-based); post-smoothing step 1 starts from a nonzero x
    LevelBatch<T> lb{};
    lb.nbox = nb;
    int blk = 0;
    for (int q = 0; q < nb; q++) {
        const int b = boxes[q];
        Box &B = c->box[b];
        Level &L = B.lev[l];
        const ChebCoef C = cheb_coef(L.lmax, c->pc.cheb_degree);
        LevelArgs<T> &A = lb.a[q];
        A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.n = L.n;
        A.blk0 = blk;
        blk += l == 0 ? smooth0_tiles(L.nx, L.ny, L.nz, c->tile_tx, c->tile_cz)
                      : (L.n + kBlock - 1) / kBlock;
        A.k0 = B.k0; A.ek_lo = B.ek_lo; A.ek_hi = B.ek_hi; A.mass = B.mass;
        A.cK = B.cK;
        A.S = (const T *)L.S;
        A.invd = (const T *)L.invd;
        A.dcorr = l == 0 ? (const T *)c->dcorr0 + B.off : nullptr;
        A.b = (const T *)L.b;
        const int cur = vs.xcur[b][l];
        A.xin = lvx(L, cur);
        A.xout = lvx(L, 1 - cur);
        A.c1 = C.c1[step];
        A.c2 = C.c2[step];
        // direction: after the fused first pre-smoothing step it equals x
        // after the fused first pre-smoothing step (from x = 0) the direction
        // equals the iterate itself
        A.din = (const T *)L.d;
        A.din_x = (!post && step == 2) ? 1 : 0;
        A.dout = step < c->pc.cheb_degree ? (T *)L.d : nullptr;
        A.rout = nullptr;
        vs.xcur[b][l] = 1 - cur;
    }
    if (c->rec) {
        rec_stage<T>(c, l == 0 ? SK_SM0 : SK_SM, blk).u.lb = lb;
        return;
    }
    if (l == 0) {
        // algorithmic bytes: x read and written (FP64), b, D^-1, reaction
        // diagonal (+ direction in/out) in T, one element coefficient per node
        double bytes = 0.0;
        for (int q = 0; q < nb; q++) {
            const LevelArgs<T> &A = lb.a[q];
            const double per = 16.0 + 8.0 + sizeof(T) * (3 + (A.c1 != 0.0 && !A.din_x) + (A.dout != nullptr));
            bytes += per * A.n;
        }
        if (grp) {
            grp->add(bytes);
            launch_smooth0<T>(c->g, lb, blk, 0, c->tile_tx, c->tile_cz, st);
        } else {
            ProfScope ps(c->prof, P4D_K_SMOOTH0, bytes, st);
            launch_smooth0<T>(c->g, lb, blk, 0, c->tile_tx, c->tile_cz, st);
        }
    } else {
        launch_smooth<T>(lb, blk, 0, st);
    }
}

template <typename T>
static void residual_step(p4d_ctx *c, VState<T> &vs, int l, const int *boxes, int nb,
                          hipStream_t st)
{
    LevelBatch<T> lb{};
    lb.nbox = nb;
    int blk = 0;
    for (int q = 0; q < nb; q++) {
        const int b = boxes[q];
        Box &B = c->box[b];
        Level &L = B.lev[l];
        LevelArgs<T> &A = lb.a[q];
        A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.n = L.n;
        A.blk0 = blk;
        blk += l == 0 ? smooth0_tiles(L.nx, L.ny, L.nz, c->tile_tx, c->tile_cz)
                      : (L.n + kBlock - 1) / kBlock;
        A.k0 = B.k0; A.ek_lo = B.ek_lo; A.ek_hi = B.ek_hi; A.mass = B.mass;
        A.cK = B.cK;
        A.S = (const T *)L.S;
        A.invd = (const T *)L.invd;
        A.dcorr = l == 0 ? (const T *)c->dcorr0 + B.off : nullptr;
        A.b = (const T *)L.b;
        A.xin = lvx(L, vs.xcur[b][l]);
        A.rout = (T *)L.r;
    }
    if (c->rec) rec_stage<T>(c, l == 0 ? SK_SM0R : SK_SMR, blk).u.lb = lb;
    else if (l == 0) launch_smooth0<T>(c->g, lb, blk, 1, c->tile_tx, c->tile_cz, st);
    else launch_smooth<T>(lb, blk, 1, st);
}

template <typename T>
static void vcycle_rest(p4d_ctx *c, VState<T> &vs, int l, int *act, int na, hipStream_t st);

template <typename T>
static void vcycle_level(p4d_ctx *c, VState<T> &vs, int l, hipStream_t st)
{
    int act[4], na = 0, crs[4], nc = 0;
    for (int b = 0; b < 4; b++) {
        if (!((c->box_mask >> b) & 1)) continue;
        if (c->box[b].nlev - 1 > l) act[na++] = b;
        else if (c->box[b].nlev - 1 == l) crs[nc++] = b;
    }
    if (nc) {
        CoarseBatch<T> cb{};
        cb.nbox = nc;
        for (int q = 0; q < nc; q++) {
            Level &L = c->box[crs[q]].lev[l];
            cb.a[q].n = L.n;
            cb.a[q].Ainv = L.Ainv;
            cb.a[q].b = (const T *)L.b;
            cb.a[q].x = (double *)L.xa;
            vs.xcur[crs[q]][l] = 0;
        }
        if (c->rec) {
            int nmax = 1;
            for (int q = 0; q < nc; q++) nmax = cb.a[q].n > nmax ? cb.a[q].n : nmax;
            const int rows = (nmax + 63) / 64;
            PStage<T> &S = rec_stage<T>(c, SK_COARSE, rows * nc);
            S.aux = rows;
            S.u.cb = cb;
        } else {
            launch_coarse<T>(cb, st);
        }
    }
    if (!na) return;
    const int deg = c->pc.cheb_degree;
    if (l >= 1 && !c->rec) {
        // boxes whose level l is their last smoothed level and fits the
        // LDS of one workgroup run the rest of their cycle in the tail kernel
        TailBatch<T> tb{};
        tb.deg = deg;
        int rest[4], nr = 0, tmask = 0;
        for (int q = 0; q < na; q++) {
            Box &B = c->box[act[q]];
            const Level &F = B.lev[l], &Cl = B.lev[l + 1];
            if (B.nlev - 2 != l || tail_lds_bytes<T>(F.n, Cl.n) > kTailLds) {
                rest[nr++] = act[q];
                continue;
            }
            TailArgs<T> &A = tb.a[tb.nbox++];
            A.nx = F.nx; A.ny = F.ny; A.nz = F.nz; A.n = F.n;
            A.cx = Cl.nx; A.cy = Cl.ny; A.cz = Cl.nz; A.nc = Cl.n;
            A.S = (const T *)F.S;
            A.invd = (const T *)F.invd;
            A.b = (const T *)F.b;
            A.x1 = lvx(const_cast<Level &>(F), vs.xcur[act[q]][l]);
            // the per-stage schedule flips the iterate buffer once per
            // smoothing step: deg - 1 before and deg after the correction
            const int fin = (vs.xcur[act[q]][l] + 2 * deg - 1) & 1;
            A.xout = lvx(const_cast<Level &>(F), fin);
            vs.xcur[act[q]][l] = fin;
            A.Ainv = Cl.Ainv;
            const ChebCoef C = cheb_coef(F.lmax, deg);
            for (int t = 0; t < 5; t++) {
                A.c1[t] = C.c1[t];
                A.c2[t] = C.c2[t];
            }
            tmask |= 1 << act[q];
        }
        if (tb.nbox) launch_tail<T>(tb, st);
        if (!nr) return;
        // the other boxes continue level by level; the tail's boxes sit out
        // the coarser levels
        for (int q = 0; q < nr; q++) act[q] = rest[q];
        na = nr;
        const int keep = c->box_mask;
        c->box_mask &= ~tmask;
        vcycle_rest<T>(c, vs, l, act, na, st);
        c->box_mask = keep;
        return;
    }
    vcycle_rest<T>(c, vs, l, act, na, st);
}

// level l of the V-cycle for the boxes in act (levels below l + 1 by
// recursion): pre-smoothing, residual, restriction, coarser levels,
// prolongation, post-smoothing
template <typename T>
static void vcycle_rest(p4d_ctx *c, VState<T> &vs, int l, int *act, int na, hipStream_t st)
{
    const int deg = c->pc.cheb_degree;
    // the level-0 smoothing steps on either side of the coarse correction
    // run back to back: each side is one timed interval
    const bool grouped = l == 0 && !c->rec;
    {
        ProfScope grp(c->prof, P4D_K_SMOOTH0, 0.0, st, grouped ? deg - 1 : 0);
        for (int t = 2; t <= deg; t++) smooth_step<T>(c, vs, l, act, na, t, 0, st, grouped ? &grp : nullptr);
    }
    residual_step<T>(c, vs, l, act, na, st);
    {   // restriction (+ first smoothing iterate of the coarse level)
        TransferBatch<T> tb{};
        tb.nbox = na;
        int blk = 0;
        for (int q = 0; q < na; q++) {
            Box &B = c->box[act[q]];
            Level &F = B.lev[l], &Cl = B.lev[l + 1];
            TransferArgs<T> &A = tb.a[q];
            A.fx = F.nx; A.fy = F.ny; A.fz = F.nz;
            A.cx = Cl.nx; A.cy = Cl.ny; A.cz = Cl.nz;
            A.blk0 = blk;
            blk += (Cl.n + kBlock - 1) / kBlock;
            A.rf = (const T *)F.r;
            A.bc = (T *)Cl.b;
            const bool coarsest = (l + 1 == B.nlev - 1);
            A.xc1 = coarsest ? nullptr : (double *)Cl.xa;
            A.invdc = (const T *)Cl.invd;
            A.c2c = coarsest ? 0.0 : cheb_coef(Cl.lmax, deg).c2[1];
            vs.xcur[act[q]][l + 1] = 0;
        }
        if (c->rec) rec_stage<T>(c, SK_RESTRICT, blk).u.tb = tb;
        else launch_restrict<T>(tb, blk, st);
    }
    vcycle_level<T>(c, vs, l + 1, st);
    {   // prolongation and correction
        TransferBatch<T> tb{};
        tb.nbox = na;
        int blk = 0;
        for (int q = 0; q < na; q++) {
            Box &B = c->box[act[q]];
            Level &F = B.lev[l], &Cl = B.lev[l + 1];
            TransferArgs<T> &A = tb.a[q];
            A.fx = F.nx; A.fy = F.ny; A.fz = F.nz;
            A.cx = Cl.nx; A.cy = Cl.ny; A.cz = Cl.nz;
            A.blk0 = blk;
            blk += (F.n + kBlock - 1) / kBlock;
            A.xc = lvx(Cl, vs.xcur[act[q]][l + 1]);
            A.xf = lvx(F, vs.xcur[act[q]][l]);
        }
        if (c->rec) rec_stage<T>(c, SK_PROLONG, blk).u.tb = tb;
        else launch_prolong<T>(tb, blk, st);
    }
    {
        ProfScope grp(c->prof, P4D_K_SMOOTH0, 0.0, st, grouped ? deg : 0);
        for (int t = 1; t <= deg; t++) smooth_step<T>(c, vs, l, act, na, t, 1, st, grouped ? &grp : nullptr);
    }
}

// One V-cycle at level l with z-line smoothing (FP64; levels keep their z
// extent): x = 0, cheb_degree passes of colours 0..3, residual, restriction,
// the coarser level, prolongation, cheb_degree passes of colours 3..0.  The
// iterate of every level stays in its xa buffer.
static void vcycle_line(p4d_ctx *c, int l, hipStream_t st)
{
    int act[4], na = 0, crs[4], nc = 0;
    for (int b = 0; b < 4; b++) {
        if (!((c->box_mask >> b) & 1)) continue;
        if (c->box[b].nlev - 1 > l) act[na++] = b;
        else if (c->box[b].nlev - 1 == l) crs[nc++] = b;
    }
    if (nc) {
        CoarseBatch<double> cb{};
        cb.nbox = nc;
        for (int q = 0; q < nc; q++) {
            Level &L = c->box[crs[q]].lev[l];
            cb.a[q].n = L.n;
            cb.a[q].Ainv = L.Ainv;
            cb.a[q].b = (const double *)L.b;
            cb.a[q].x = (double *)L.xa;
        }
        launch_coarse<double>(cb, st);
    }
    if (!na) return;
    LineBatch lb{};
    lb.nbox = na;
    double bytes = 0.0;
    for (int q = 0; q < na; q++) {
        Box &B = c->box[act[q]];
        Level &L = B.lev[l];
        LineArgs &A = lb.a[q];
        A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.n = L.n;
        A.S = L.S64;
        A.Sz = L.Sz;
        A.b = (const double *)L.b;
        A.x = (double *)L.xa;
        A.r = (double *)L.r;
        hipMemsetAsync(A.x, 0, 8 * (size_t)L.n, st);
        // stencil, b, x read and written
        bytes += (27.0 * 8 + 8 + 16) * L.n;
    }
    const int deg = c->pc.cheb_degree;
    auto pass = [&](bool backward) {
        if (l == 0) {   // level-0 passes are timed as the level-0 smoother class
            ProfScope ps(c->prof, P4D_K_SMOOTH0, bytes, st);
            for (int q = 0; q < 4; q++) launch_zline(lb, backward ? 3 - q : q, st);
        } else {
            for (int q = 0; q < 4; q++) launch_zline(lb, backward ? 3 - q : q, st);
        }
    };
    for (int t = 0; t < deg; t++) pass(false);
    launch_resid_full(lb, st);
    {
        TransferBatch<double> tb{};
        tb.nbox = na;
        int blk = 0;
        for (int q = 0; q < na; q++) {
            Box &B = c->box[act[q]];
            Level &F = B.lev[l], &Cl = B.lev[l + 1];
            TransferArgs<double> &A = tb.a[q];
            A.fx = F.nx; A.fy = F.ny; A.fz = F.nz;
            A.cx = Cl.nx; A.cy = Cl.ny; A.cz = Cl.nz;
            A.blk0 = blk;
            blk += (Cl.n + kBlock - 1) / kBlock;
            A.rf = (const double *)F.r;
            A.bc = (double *)Cl.b;
            A.xc1 = nullptr;
            A.invdc = nullptr;
            A.c2c = 0.0;
        }
        launch_restrict<double>(tb, blk, st);
    }
    vcycle_line(c, l + 1, st);
    {
        TransferBatch<double> tb{};
        tb.nbox = na;
        int blk = 0;
        for (int q = 0; q < na; q++) {
            Box &B = c->box[act[q]];
            Level &F = B.lev[l], &Cl = B.lev[l + 1];
            TransferArgs<double> &A = tb.a[q];
            A.fx = F.nx; A.fy = F.ny; A.fz = F.nz;
            A.cx = Cl.nx; A.cy = Cl.ny; A.cz = Cl.nz;
            A.blk0 = blk;
            blk += (F.n + kBlock - 1) / kBlock;
            A.xc = (const double *)Cl.xa;
            A.xf = (double *)F.xa;
        }
        launch_prolong<double>(tb, blk, st);
    }
    for (int t = 0; t < deg; t++) pass(true);
}

// fixed part of the particle-block arguments
static RadArgs rad_args(const p4d_ctx *c)
{
    RadArgs R{};
    R.tabs = c->tabs;
    R.gg = c->gg; R.ss = c->ss; R.ee = c->ee; R.mm = c->mm; R.om = c->omega;
    R.b0 = c->b0;
    R.x1 = (double *)c->x0a;
    R.invd0 = c->invd0;
    for (int b = 0; b < 4; b++) R.c2box[b] = cheb_coef(c->box[b].lev[0].lmax, c->pc.cheb_degree).c2[1];
    return R;
}

// z = P^-1 (s r), or P^-T, with the scale s read from device memory (rscale;
// null: 1)
template <typename T, typename TZ>
static void apply_pc_t(p4d_ctx *c, int transpose, const double *r, const double *rscale, TZ *z,
                       hipStream_t st)
{
    const Geom &g = c->g;
    const int schur = c->pc.pc == P4D_PC_SCHUR;
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
    RadArgs R = rad_args(c);
    if (c->rec) {
        rec_stage<T>(c, SK_RADF, nb);
    } else {
        ProfScope ps(c->prof, P4D_K_RADIAL, 8.0 * g.N + 32.0 * g.ne + (sizeof(T) * 2 + 8.0) * g.Nm, st);
        launch_rad_fwd<T>(g, R, r, rscale, transpose, schur, st);
    }
    VState<T> vs{};
    for (int b = 0; b < 4; b++) vs.xcur[b][0] = 0;
    if (c->pc.smoother == P4D_SMOOTH_ZLINE) vcycle_line(c, 0, st);   // (FP64 only)
    else vcycle_level<T>(c, vs, 0, st);
    // each box's final level-0 iterate (the two buffers alternate)
    for (int b = 0; b < 4; b++) R.x0[b] = (const double *)(vs.xcur[b][0] ? c->x0b : c->x0a);
    if (c->rec) {
        rec_stage<T>(c, SK_RADB, nb);
        c->rec_R = R;
        return;
    }
    ProfScope ps(c->prof, P4D_K_RADIAL, 8.0 * (g.N - g.Nm) + 8.0 * g.ne + 8.0 * g.Nm +
                                           sizeof(TZ) * g.N + 40.0 * g.ne, st);
    launch_rad_back<T, TZ>(g, R, r, rscale, z, transpose, schur, st);
}

// z = P_GS^-1 (rscale r), or P_GS^-T (eq. PGS): the fields in the chosen
// ordering (backwards when transposed), each V-cycle on the boxes of its own
// field only; the level-0 iterates of the fields solved stay in place (each
// box owns its slice of the level-0 buffers) and feed the later couplings.
template <typename T, typename TZ>
static void apply_bgs_t(p4d_ctx *c, int transpose, const double *r, const double *rscale, TZ *z,
                        hipStream_t st)
{
    const Geom &g = c->g;
    BgsArgs B{};
    B.R = rad_args(c);
    B.kx = c->general ? c->kdh : c->kaph;
    B.kx_scale = c->general ? 1.0 : c->g.chi;
    B.zsN = c->qbuf;
    VState<T> vs{};
    for (int b = 0; b < 4; b++) {
        vs.xcur[b][0] = 0;
        B.R.x0[b] = (const double *)c->x0a;
    }
    for (int s = 0; s < 4; s++) {
        const int p = transpose ? 3 - s : s;
        const int f = (c->pc.bgs_order >> (2 * p)) & 3;
        B.field = f;
        if (f == BF_CS) {
            ProfScope ps(c->prof, P4D_K_RADIAL, 8.0 * (g.N - g.Nm) + 56.0 * g.ne + 16.0 * g.nnode +
                                                   sizeof(TZ) * (g.N - g.Nm), st);
            launch_bgs_cs<T, TZ>(g, B, r, rscale, z, transpose, st);
        } else {
            const double n = f == BF_PHIS ? (double)g.ne : (double)g.nnode;
            {
                ProfScope ps(c->prof, P4D_K_COUPLING, n * (8.0 + sizeof(T) * 2 + 8.0) + 48.0 * g.ne, st);
                launch_bgs_rhs<T>(g, B, r, rscale, transpose, st);
            }
            const int boxes = f == BF_PHIS ? 3 : (f == BF_PHIE ? 4 : 8);   // phi_s: both electrodes
            c->box_mask = boxes;
            vcycle_level<T>(c, vs, 0, st);
            c->box_mask = 15;
            for (int b = 0; b < 4; b++)
                if ((boxes >> b) & 1) B.R.x0[b] = (const double *)(vs.xcur[b][0] ? c->x0b : c->x0a);
        }
        B.done |= 1 << f;
    }
    ProfScope ps(c->prof, P4D_K_COUPLING, (8.0 + sizeof(TZ)) * g.Nm, st);
    launch_bgs_out<TZ>(g, B, r, rscale, z, st);
}

// z = P_S^-1 (rscale r) for the Schur-complement iteration: one V-cycle per
// field on S~_f (the field blocks of S, the SCHUR-mode boxes), identity on
// the grounded layer; r and z hold the electrode-level unknowns only.
template <typename T, typename TZ>
static void apply_pc_schur_t(p4d_ctx *c, const double *r, const double *rscale, TZ *z, hipStream_t st)
{
    const Geom &g = c->g;
    BgsArgs B{};
    B.R = rad_args(c);
    {
        ProfScope ps(c->prof, P4D_K_COUPLING, (8.0 + sizeof(T) + 8.0) * g.Nm, st);
        launch_rad_fwd<T>(g, B.R, r, rscale, 0, 0, st);   // cast + first Chebyshev iterate
    }
    VState<T> vs{};
    for (int b = 0; b < 4; b++) vs.xcur[b][0] = 0;
    if (c->pc.smoother == P4D_SMOOTH_ZLINE) vcycle_line(c, 0, st);   // (FP64 only)
    else vcycle_level<T>(c, vs, 0, st);
    for (int b = 0; b < 4; b++) B.R.x0[b] = (const double *)(vs.xcur[b][0] ? c->x0b : c->x0a);
    ProfScope ps(c->prof, P4D_K_COUPLING, (8.0 + sizeof(TZ)) * g.Nm, st);
    launch_bgs_out<TZ>(g, B, r, rscale, z, st);
}

template <typename TZ>
static void apply_pc_schur(p4d_ctx *c, const double *r, const double *rscale, TZ *z, hipStream_t st)
{
    if (c->prec == 1) apply_pc_schur_t<float, TZ>(c, r, rscale, z, st);
    else apply_pc_schur_t<double, TZ>(c, r, rscale, z, st);
}

template <typename TZ>
static void apply_pc(p4d_ctx *c, int transpose, const double *r, const double *rscale, TZ *z,
                     hipStream_t st)
{
    if (c->pc.pc == P4D_PC_BGS) {
        if (c->prec == 1) apply_bgs_t<float, TZ>(c, transpose, r, rscale, z, st);
        else apply_bgs_t<double, TZ>(c, transpose, r, rscale, z, st);
        return;
    }
    if (c->prec == 1) apply_pc_t<float, TZ>(c, transpose, r, rscale, z, st);
    else apply_pc_t<double, TZ>(c, transpose, r, rscale, z, st);
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
template <typename T>
static p4d_status setup_t(p4d_ctx *c, hipStream_t st)
{
    const Geom &g = c->g;
    const int schur = c->pc.pc == P4D_PC_SCHUR;
    launch_omega(g, c->tabs, c->ss, schur, c->omega, st);
    // scratch: FP64 stencils of level 0, FP64 dcorr / inverse diagonal, dense
    char *sp = c->scratch;
    auto take = [&](size_t bytes) { char *p = sp; sp += align_up(bytes); return p; };
    const int zline = c->pc.smoother == P4D_SMOOTH_ZLINE;
    double *S0[4];
    for (int b = 0; b < 4; b++)
        S0[b] = zline ? c->box[b].lev[0].S64 : (double *)take(8 * 27 * (size_t)c->box[b].lev[0].n);
    double *dc64 = (double *)take(8 * (size_t)g.Nm);
    double *id64 = (double *)take(8 * (size_t)g.Nm);
    size_t rapmax = 0;
    for (int b = 0; b < 4; b++) {
        const Box &B = c->box[b];
        for (int l = 0; l + 1 < B.nlev; l++) {
            const Level &F = B.lev[l];
            const size_t cx = coarse_n_h(F.nx), cy = coarse_n_h(F.ny);
            const size_t t = 27 * (cx * F.ny * F.nz + cx * cy * F.nz);
            rapmax = t > rapmax ? t : rapmax;
        }
    }
    double *raptmp = (double *)take(8 * 4 * (rapmax ? rapmax : 1));   // one slice per box
    InvBatch ib{};
    Elem0 E0[4];
    for (int b = 0; b < 4; b++) {
        const Box &B = c->box[b];
        E0[b] = Elem0{B.lev[0].nz, B.k0, B.ek_lo, B.ek_hi, B.mass, B.cK, dc64 + B.off};
    }
    launch_dcorr<double>(g, c->gg, c->ee, c->mm, c->omega, dc64, st);
    launch_cast<T>(g.Nm, dc64, (T *)c->dcorr0, st);
    // inverse diagonal of level 0 defaults to 0 outside the boxes (the
    // grounded layer of phi_s)
    HIPCHK(c, hipMemsetAsync(id64, 0, 8 * (size_t)g.Nm, st));
    // Gershgorin bounds, raised by atomic maxima: kLmaxSlots slots for box b,
    // level l at (16 b + l) kLmaxSlots of the reduction buffer
    unsigned long long *lmx = (unsigned long long *)c->red;
    const size_t nlmx = 64 * (size_t)kLmaxSlots;
    HIPCHK(c, hipMemsetAsync(lmx, 0, 8 * nlmx, st));
    int maxlev = 0;
    for (int b = 0; b < 4; b++) maxlev = c->box[b].nlev > maxlev ? c->box[b].nlev : maxlev;
    for (int l = 0; l < maxlev; l++) {
        if (l > 0) {   // Galerkin products of this level, all boxes in one batch
            RapJob jobs[4];
            int nj = 0;
            for (int b = 0; b < 4; b++) {
                Box &B = c->box[b];
                if (B.nlev <= l) continue;
                const Level &F = B.lev[l - 1];
                jobs[nj] = RapJob{F.nx, F.ny, F.nz, l == 1 ? (zline ? S0[b] : nullptr) : F.S64,
                                  B.lev[l].S64, raptmp + (size_t)nj * rapmax, l == 1 ? E0[b] : Elem0{}};
                nj++;
            }
            launch_rap(g, jobs, nj, !zline, st);
        }
        // difference form, inverse diagonal and bound of this level, all
        // boxes in one launch (level 0: from the element rows)
        PrepBatch pb{};
        int pblk = 0;
        for (int b = 0; b < 4; b++) {
            Box &B = c->box[b];
            if (B.nlev <= l) continue;
            Level &L = B.lev[l];
            if (l == 0 && (zline || B.nlev == 1)) continue;   // stored-stencil path below
            PrepArgs &A = pb.a[pb.nbox++];
            A.n = L.n;
            A.blk0 = pblk;
            pblk += (L.n + kBlock - 1) / kBlock;
            A.S = L.S64;
            A.D = L.S;
            A.invd = L.invd;
            A.E = E0[b];
            A.invd0 = id64 + B.off;
            A.lmax = lmx + (16 * b + l) * kLmaxSlots;
        }
        if (pb.nbox) {
            if (l > 0) launch_level_prep_batch<T>(pb, pblk, st);
            else launch_diag0_batch(g, pb, pblk, st);
        }
        for (int b = 0; b < 4; b++) {
            Box &B = c->box[b];
            if (B.nlev <= l) continue;
            Level &L = B.lev[l];
            const double *Sl;
            if (l == 0) {
                // the stored level-0 stencil is needed only by z-line smoothing
                // and by a level-0 coarsest grid; otherwise its rows are formed
                // where they are used (diagonal, first Galerkin product)
                if (zline || B.nlev == 1) {
                    launch_assemble0(g, b, L.nz, B.k0, B.ek_lo, B.ek_hi, B.mass, B.cK, dc64 + B.off,
                                     S0[b], st);
                    launch_diag(L.n, S0[b], id64 + B.off, lmx + 16 * b * kLmaxSlots, (L.n + kBlock - 1) / kBlock,
                                st);
                }
                Sl = S0[b];
            } else {
                Sl = L.S64;
            }
            if (zline && L.Sz) launch_zline_order(L.nx, L.ny, L.nz, Sl, L.Sz, st);
            if (l == B.nlev - 1) {
                if (L.n > 1024) return fail(c, P4D_ERR_INVALID_ARG, "coarsest grid above 1024 nodes");
                double *dense = (double *)take(8 * (size_t)L.n * L.n);
                launch_dense_from_stencil(L.nx, L.ny, L.nz, Sl, dense, st);
                ib.n[ib.nbox] = L.n;
                ib.A[ib.nbox] = dense;
                ib.Ainv[ib.nbox] = L.Ainv;
                ib.nbox++;
            }
        }
    }
    launch_invert(ib, st);
    launch_cast<T>(g.Nm, id64, (T *)c->invd0, st);
    HIPCHK(c, hipGetLastError());
    // the Gershgorin maxima go to the host in a slot of their own; the first
    // use of the preconditioner waits for them (finish_setup), so the setup
    // returns without waiting for its kernels
    static_assert(4 * kMaxLevels * kLmaxSlots <= kPubMax, "Gershgorin slots exceed the handoff buffer");
    c->lmax_seq = publish(c, lmx, (int)nlmx, kPubSetup, st);
    c->lmax_stream = st;
    c->lmax_pending = 1;
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

// The Chebyshev bounds of the last setup (the largest Gershgorin ratio of
// every level), once its kernels have handed them over
static p4d_status finish_setup(p4d_ctx *c)
{
    if (!c->lmax_pending) return P4D_OK;
    c->lmax_pending = 0;
    const p4d_status ps = await_pub(c, kPubSetup, c->lmax_seq, c->lmax_stream);
    if (ps != P4D_OK) {
        c->pc_ready = 0;
        return ps;
    }
    const unsigned long long *lmh = c->hpub + kPubSetup * kPubStride;
    for (int b = 0; b < 4; b++)
        for (int l = 0; l < c->box[b].nlev; l++) {
            unsigned long long bits = 0;   // bits of the maximum (non-negative doubles order as integers)
            for (int q = 0; q < kLmaxSlots; q++)
                bits = std::max(bits, lmh[(16 * (size_t)b + l) * kLmaxSlots + q]);
            double lm;
            std::memcpy(&lm, &bits, sizeof(lm));
            if (!(lm > 0.0) || !std::isfinite(lm)) {
                c->pc_ready = 0;
                return fail(c, P4D_ERR_NONFINITE, "non-positive or non-finite Gershgorin bound");
            }
            c->box[b].lev[l].lmax = lm;
        }
    return P4D_OK;
}

// ---------------------------------------------------------------------------
// FGMRES (Saad's flexible variant, right preconditioned, restarted)
// ---------------------------------------------------------------------------
// The Krylov space is either all unknowns, or (krylov = SCHUR) the
// electrode-level unknowns of the Schur complement S of the particle blocks:
// FGMRES on S y = bhat, then x_s = A_ss^-1 (b_s - A_sy y).  Both stop on
// rtol ||b|| with b the full right-hand side: with the particle rows solved
// exactly, b - A x vanishes in them and equals bhat - S y in the others.
template <typename TZ>
static p4d_status fgmres(p4d_ctx *c, int transpose, const double *b, double *x,
                         const p4d_solve_opts &o, p4d_solve_info *info, hipStream_t st)
{
    const Geom &g = c->g;
    const bool schur = o.krylov == P4D_KRYLOV_SCHUR;
    const long long N = schur ? g.Nm : g.N;   // Krylov vector length
    const int m = o.restart;
    double *V = (double *)c->scratch;
    TZ *Z = (TZ *)(c->scratch + align_up(8 * (size_t)(m + 1) * N));
    // the Krylov right-hand side: b, or bhat (after Z; the region is sized
    // for the full space, which leaves room)
    double *bk = schur ? (double *)((char *)Z + align_up(sizeof(TZ) * (size_t)m * N)) : (double *)b;
    double *red = c->red;
    const int sb = stream_blocks(N);
    const int sbf = stream_blocks(g.N);
    const int ob = operator_blocks(g);
    const double *hh = (const double *)c->hpub;   // values handed to the host (pull)
    double *hout = c->hhost + 256;                 // host-to-device staging
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), yv(m), hc(m + 2),
        beta(m + 1), res(m + 1);
    p4d_solve_info inf{};
    auto t0 = std::chrono::steady_clock::now();
    // the setup's bounds: waited for before the first preconditioner
    // application, or now if the setup ran on another stream (this stream
    // does not follow its kernels)
    if (c->lmax_pending && c->lmax_stream != st) {
        const p4d_status fs = finish_setup(c);
        if (fs != P4D_OK) return fs;
    }
    // r = bk - op(x) into V_0 with its norm (restarts and breakdown)
    auto residual = [&]() -> p4d_status {
        if (schur) {
            apply_op_schur<double>(c, transpose, x, V, st);
            launch_red_resid(N, bk, V, red, sb, st);
            launch_norm_final(red, sb, c->hdev + 200, c->invbeta, st);
        } else {
            apply_op<double>(c, transpose, x, V, b, red, st);
            launch_norm_final(red, ob, c->hdev + 200, c->invbeta, st);
        }
        const p4d_status ps = pull(c, c->hdev + 200, 1, st);
        if (ps != P4D_OK) return ps;
        prof_harvest(c->prof);
        return P4D_OK;
    };

    // ||b|| over all unknowns
    launch_dot_partial(g.N, b, b, red, sbf, st);
    launch_norm_final(red, sbf, c->hdev, nullptr, st);
    {
        const p4d_status ps = pull(c, c->hdev, 1, st);
        if (ps != P4D_OK) return ps;
    }
    const double bnorm = hh[0];
    // set when the last handoff follows every write to x (no final one needed)
    bool synced = false;
    // x = 0 until the first update, which assigns x = Z y instead of adding
    // (a solve that stops before it clears x at the end)
    bool x_zero = true;
    // the first basis vector: the first cycle reads the right-hand side in
    // place, later cycles their residual in V
    const double *v0 = bk;
    if (!std::isfinite(bnorm)) {
        HIPCHK(c, hipMemsetAsync(x, 0, 8 * (size_t)g.N, st));
        HIPCHK(c, hipStreamSynchronize(st));
        return fail(c, P4D_ERR_NONFINITE, "non-finite right-hand side");
    }
    p4d_status status = P4D_NOT_CONVERGED;
    int total = 0;
    bool first = true;
    if (bnorm == 0.0) {
        status = P4D_OK;
        goto done;
    }
    if (schur) {
        ProfScope ps(c->prof, P4D_K_RADIAL, 8.0 * g.N + 8.0 * g.Nm + 32.0 * g.ne, st);
        launch_red_rhs(g, c->tabs, c->gg, c->ss, c->ee, c->mm, b, bk, transpose, st);
    }
    for (;;) {
        // r = bk - op(x) into V_0 (x = 0 in the first cycle: r = bk)
        if (first) {
            if (schur) {
                launch_dot_partial(N, bk, bk, red, sb, st);
                launch_norm_final(red, sb, c->hdev + 200, c->invbeta, st);
                const p4d_status ps = pull(c, c->hdev + 200, 1, st);
                if (ps != P4D_OK) return ps;
                beta[0] = hh[0];
            } else {
                hout[0] = 1.0 / bnorm;
                HIPCHK(c, hipMemcpyAsync(c->invbeta, hout, 8, hipMemcpyHostToDevice, st));
                beta[0] = bnorm;
            }
            first = false;
        } else {
            const p4d_status rs = residual();
            if (rs != P4D_OK) return rs;
            beta[0] = hh[0];
            synced = true;
            v0 = V;
        }
        inf.relres_true = beta[0] / bnorm;
        if (!std::isfinite(beta[0])) { status = P4D_ERR_NONFINITE; break; }
        if (beta[0] <= o.rtol * bnorm) { status = P4D_OK; break; }
        if (total >= o.maxit) { status = P4D_NOT_CONVERGED; break; }
        synced = false;
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta[0];
        res[0] = beta[0];
        int kused = 0;
        bool breakdown = false, nonfinite = false;
        // one Arnoldi step on the device: z_k = P^-1 v_k / beta_k, w = A z_k,
        // Gram-Schmidt against V_0..V_k, ||w|| and 1 / ||w|| (every input it
        // needs is in device memory), then its Hessenberg column to the host
        unsigned long long step_seq[2] = {0, 0};
        auto enqueue_step = [&](int k) {
            const double *vk = k == 0 ? v0 : V + (long long)k * N;
            TZ *zk = Z + (long long)k * N;
            double *w = V + (long long)(k + 1) * N;
            if (schur) {
                apply_pc_schur<TZ>(c, vk, c->invbeta + k, zk, st);
                apply_op_schur<TZ>(c, transpose, zk, w, st);
            } else {
                apply_pc<TZ>(c, transpose, vk, c->invbeta + k, zk, st);
                apply_op<TZ>(c, transpose, zk, w, nullptr, nullptr, st);
            }
            const int nv = k + 1;
            const int passes = o.cgs2 ? 2 : 1;
            for (int p = 0; p < passes; p++) {
                {
                    ProfScope ps(c->prof, P4D_K_MDOT, 8.0 * (nv + 1) * N, st);
                    launch_mdot(N, w, V, v0, N, nv, red, sb, st);
                }
                launch_mdot_final(nv, red, sb, c->invbeta, c->hdev + 64 * p, c->cdev, st);
                {
                    ProfScope ps(c->prof, P4D_K_ORTH, 8.0 * (nv + 2) * N, st);
                    launch_orth(N, w, V, v0, N, nv, c->cdev, red, sb, st);
                }
            }
            launch_norm_final(red, sb, c->hdev + 128, c->invbeta + k + 1, st);
            step_seq[k & 1] = publish(c, c->hdev, 129, k & 1, st);
        };
        // The next step is enqueued before the host reads this step's column
        // when the residual estimate is expected to stay above the tolerance
        // (its rate of decrease so far, with a margin): the device then runs
        // on while the host waits.  If the solve stops after all, the extra
        // step's results are never used.
        {
            const p4d_status fs = finish_setup(c);
            if (fs != P4D_OK) return fs;
        }
        int ahead = -1;   // the step already enqueued, if any
        for (int k = 0; k < m; k++) {
            if (ahead != k) enqueue_step(k);
            ahead = -1;
            const double est = res[k];   // residual estimate after k steps
            const double prev = k > 0 ? res[k - 1] : est;
            const double rate = prev > 0.0 && est < prev ? est / prev : 1.0;
            if (k + 1 < m && total + 1 < o.maxit && est * rate > 2.0 * o.rtol * bnorm) {
                enqueue_step(k + 1);
                ahead = k + 1;
            }
            {
                const p4d_status ps = await_pub(c, k & 1, step_seq[k & 1], st);
                if (ps != P4D_OK) return ps;
            }
            // (with a step in flight its events are still pending)
            if (ahead < 0) prof_harvest(c->prof);
            const double *hh = (const double *)c->hpub + (k & 1) * kPubStride;
            for (int i = 0; i <= k; i++) hc[i] = hh[i] + (o.cgs2 ? hh[64 + i] : 0.0);
            const double hn = hh[128];
            hc[k + 1] = hn;
            double colnorm = 0.0;
            for (int i = 0; i <= k + 1; i++) colnorm += hc[i] * hc[i];
            colnorm = std::sqrt(colnorm);
            if (!std::isfinite(colnorm)) { nonfinite = true; break; }
            for (int i = 0; i < k; i++) {
                const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
                hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
                hc[i] = t;
            }
            const double den = std::sqrt(hc[k] * hc[k] + hc[k + 1] * hc[k + 1]);
            cs[k] = hc[k] / den;
            sn[k] = hc[k + 1] / den;
            hc[k] = den;
            gv[k + 1] = -sn[k] * gv[k];
            gv[k] = cs[k] * gv[k];
            for (int i = 0; i <= k; i++) H[(size_t)i * m + k] = hc[i];
            total++;
            kused = k + 1;
            beta[k + 1] = hn;
            inf.relres_est = std::fabs(gv[k + 1]) / bnorm;
            res[k + 1] = std::fabs(gv[k + 1]);
            if (hn <= 1e-14 * colnorm) { breakdown = true; break; }
            if (std::fabs(gv[k + 1]) <= o.rtol * bnorm || total >= o.maxit) break;
        }
        if (nonfinite) { status = P4D_ERR_NONFINITE; break; }
        for (int i = kused - 1; i >= 0; i--) {
            double v = gv[i];
            for (int j = i + 1; j < kused; j++) v -= H[(size_t)i * m + j] * yv[j];
            yv[i] = v / H[(size_t)i * m + i];
        }
        // the previous host-to-device copy from hout has completed: the host
        // has since waited for a handoff enqueued after it
        for (int i = 0; i < kused; i++) hout[i] = yv[i];
        HIPCHK(c, hipMemcpyAsync(c->ydev, hout, 8 * kused, hipMemcpyHostToDevice, st));
        {
            // x written, and read unless this update assigns it
            ProfScope ps(c->prof, P4D_K_ZY, ((x_zero ? 8.0 : 16.0) + sizeof(TZ) * kused) * N, st);
            launch_zy<TZ>(N, x, Z, N, kused, c->ydev, x_zero ? 1 : 0, st);
        }
        if (kused > 0) x_zero = false;
        inf.restarts++;
        if (breakdown) {
            const p4d_status rs = residual();
            if (rs != P4D_OK) return rs;
            synced = true;
            inf.relres_true = hh[0] / bnorm;
            status = inf.relres_true <= o.rtol ? P4D_OK : P4D_BREAKDOWN;
            break;
        }
    }
    if (x_zero) {   // no update happened
        HIPCHK(c, hipMemsetAsync(x, 0, 8 * (size_t)g.N, st));
        x_zero = false;
    }
    if (schur && status != P4D_ERR_NONFINITE) {
        // particle unknowns from the electrode-level ones, then the true
        // residual of the whole system (V has room for one full vector)
        {
            ProfScope ps(c->prof, P4D_K_RADIAL, 16.0 * (g.N - g.Nm) + 8.0 * g.Nm + 32.0 * g.ne, st);
            launch_red_back(g, c->tabs, c->gg, c->ss, c->ee, c->mm, b, x, transpose, st);
        }
        apply_op<double>(c, transpose, x, V, b, red, st);
        launch_norm_final(red, ob, c->hdev + 200, nullptr, st);
        const p4d_status ps = pull(c, c->hdev + 200, 1, st);
        if (ps != P4D_OK) return ps;
        synced = true;
        inf.relres_true = hh[0] / bnorm;
    }
done:
    if (x_zero) HIPCHK(c, hipMemsetAsync(x, 0, 8 * (size_t)g.N, st));   // (b = 0)
    HIPCHK(c, hipGetLastError());
    if (!synced) {   // the solution is complete when the handoff after it arrives
        const p4d_status ps = pull(c, c->hdev, 0, st);
        if (ps != P4D_OK) return ps;
    }
    prof_harvest(c->prof);
    inf.iters = total;
    inf.status = status;
    inf.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    if (status == P4D_ERR_NONFINITE) c->err = "non-finite value during the solve";
    return status;
}

// ---------------------------------------------------------------------------
// physical cell: Newton iterations around the linear solve
// ---------------------------------------------------------------------------
namespace {
double kappa_bulk_h(double ce)   // bulk conductivity at 298.15 K (appendix)
{
    const double c = ce / 1000.0;
    return 0.0911 + c * (1.9101 + c * (-1.052 + c * 0.1554));
}
double de_bulk_h(double ce) { return 5.34e-10 * std::exp(-0.65 * ce / 1000.0); }
}  // namespace

// Newton terms of the physical cell in the operator (u = null: off)
static void newton_terms_on(p4d_ctx *c, const double *u)
{
    PhysState &S = *c->phys;
    c->g.nwu = u;
    c->g.nwa = u ? S.nwa : nullptr;
    c->g.nwb = u ? S.nwb : nullptr;
    c->g.nwc = u ? S.nwc : nullptr;
}

// Arrays of the operator for the state u (SI): transport coefficients at the
// element-mean c_e and the kinetics derivatives, scaled; the reaction q^.
static void phys_coef(p4d_ctx *c, const double *u, hipStream_t st)
{
    PhysState &S = *c->phys;
    launch_phys_coef(c->g, S.P, u, c->sigh, c->kaph, c->kdh, c->dch, c->gg, c->ss, c->ee, S.qh, S.nwa, S.nwb,
                     S.nwc, st);
    launch_omega(c->g, c->tabs, c->ss, 1, c->oms, st);   // the Schur-complement operator's weights
    c->general = 1;
    c->box[3].cK = c->dch;
    c->uploaded = 1;
    c->pc_ready = 0;
}

// radial tables, lumped weights (geometry only) and the applied current
static p4d_status phys_prepare(p4d_ctx *c, hipStream_t st)
{
    PhysState &S = *c->phys;
    HIPCHK(c, hipMemcpyAsync(c->tabs, c->tabs_h, sizeof(c->tabs_h), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemsetAsync(c->kdh, 0, 8 * (size_t)c->g.nelem, st));
    launch_setup_nodes(c->g, c->tabs, c->kdh, c->kdh, c->sigh, c->kaph, c->mm, st);
    HIPCHK(c, hipGetLastError());
    if (!S.ready) {
        // nodal currents of the top face: the Gaussian profile (spread
        // gauss_frac * edge around the face centre; or uniform) times the
        // lumped face weight, normalized to the applied current, scaled by
        // r_phi
        const int n = c->g.nx;
        const double h = c->g.h, L = S.prm.edge, sd = S.prm.gauss_frac * L;
        std::vector<double> f((size_t)c->g.ne, 0.0);
        double sum = 0.0;
        const size_t top = (size_t)(c->g.ne - (long long)n * n);
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                const double x = i * h - 0.5 * L, y = j * h - 0.5 * L;
                const double w = (i == 0 || i == n - 1 ? 0.5 * h : h) * (j == 0 || j == n - 1 ? 0.5 * h : h);
                const double v = (S.prm.profile == 1 ? 1.0 : std::exp(-(x * x + y * y) / (2.0 * sd * sd))) * w;
                f[top + i + (size_t)n * j] = v;
                sum += v;
            }
        for (size_t t = top; t < f.size(); t++) f[t] *= S.prm.current * S.P.rphi / sum;
        HIPCHK(c, hipMemcpyAsync(S.fh, f.data(), 8 * f.size(), hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
        S.ready = true;
    }
    return P4D_OK;
}

// previous-step storage in the scaled rows: M' c_e,old^ (the operator with
// every coefficient but the storage set to zero) and c_s,old^ / dt'
static p4d_status phys_old(p4d_ctx *c, const double *uold, hipStream_t st)
{
    PhysState &S = *c->phys;
    const Geom &g = c->g;
    for (double *p : {c->sigh, c->kaph, c->kdh, c->dch})
        HIPCHK(c, hipMemsetAsync(p, 0, 8 * (size_t)g.nelem, st));
    for (double *p : {c->gg, c->ss, c->ee})
        HIPCHK(c, hipMemsetAsync(p, 0, 8 * (size_t)g.ne, st));
    c->general = 1;
    c->box[3].cK = c->dch;
    c->uploaded = 1;
    c->pc_ready = 0;
    launch_phys_scale(g, S.P, uold, S.dh, 0, st);
    HIPCHK(c, hipMemsetAsync(S.dh, 0, 8 * (size_t)g.off_ce, st));
    HIPCHK(c, hipMemsetAsync(S.dh + g.off_cs[0], 0, 8 * (size_t)(g.N - g.off_cs[0]), st));
    apply_op<double>(c, 0, S.dh, S.old, nullptr, nullptr, st);
    launch_phys_old_cs(g, S.P, uold, c->desc.dt, S.old, st);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

// r = R^(u) (scaled rows), or -R^ when neg; leaves the Newton matrix at u
static p4d_status phys_residual(p4d_ctx *c, const double *u, double *r, int neg, hipStream_t st)
{
    PhysState &S = *c->phys;
    const Geom &g = c->g;
    phys_coef(c, u, st);
    launch_phys_scale(g, S.P, u, S.uh, 0, st);
    apply_op<double>(c, 0, S.uh, r, nullptr, nullptr, st);
    PhysFix F{};
    F.uh = S.uh; F.old = S.old; F.fh = S.fh; F.qh = S.qh;
    F.gg = c->gg; F.ss = c->ss; F.ee = c->ee; F.mm = c->mm;
    F.gam[0] = c->tabs_h[0].Gamma;
    F.gam[1] = c->tabs_h[1].Gamma;
    launch_phys_fix(g, F, r, neg, st);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

void p4d_default_opts(p4d_solve_opts *o)
{
    if (!o) return;
    o->pc = P4D_PC_SCHUR;
    o->pc_prec = P4D_FP64;
    o->restart = 30;
    o->maxit = 1000;
    o->cheb_degree = 2;
    o->coarse_max = 64;
    o->cgs2 = 0;
    o->z_fp32 = 0;
    o->rtol = 1e-8;
    o->bgs_order = 1 | (3 << 2) | (0 << 4) | (2 << 6);   // (phi_e, c_s, phi_s, c_e)
    o->krylov = P4D_KRYLOV_FULL;
    o->smoother = P4D_SMOOTH_CHEB;
}

const char *p4d_status_string(p4d_status s)
{
    switch (s) {
    case P4D_OK: return "ok";
    case P4D_NOT_CONVERGED: return "not converged";
    case P4D_BREAKDOWN: return "breakdown";
    case P4D_ERR_INVALID_ARG: return "invalid argument";
    case P4D_ERR_OOM: return "workspace too small";
    case P4D_ERR_HIP: return "HIP error";
    case P4D_ERR_STATE: return "call out of order";
    case P4D_ERR_NONFINITE: return "non-finite value";
    }
    return "unknown";
}

const char *p4d_last_error(const p4d_ctx *c) { return c ? c->err.c_str() : "null context"; }

p4d_status p4d_create(const p4d_problem_desc *d, p4d_ctx **out)
{
    if (!d || !out) return P4D_ERR_INVALID_ARG;
    *out = nullptr;
    const int nc = d->nz - d->na - d->ns;
    if (d->nx < 2 || d->ny < 2 || d->nz < 5 || d->na < 2 || d->ns < 1 || nc < 2)
        return P4D_ERR_INVALID_ARG;
    for (int el = 0; el < 2; el++) {
        if (d->nr[el] < 3 || d->nr[el] > kMaxNr) return P4D_ERR_INVALID_ARG;
        if (!(d->Ds[el] > 0.0) || !(d->theta_bar[el] > 0.0) || d->theta_bar[el] > 1.0)
            return P4D_ERR_INVALID_ARG;
    }
    if (!(d->dt > 0.0) || !std::isfinite(d->chi) || !std::isfinite(d->tc) ||
        !std::isfinite(d->lambda_c) || !(d->eps_elec > 0.0) || !(d->eps_sep > 0.0))
        return P4D_ERR_INVALID_ARG;
    if (!(d->length >= 0.0) || !std::isfinite(d->length) || !(d->lambda_el[0] >= 0.0) ||
        !(d->lambda_el[1] >= 0.0) || !std::isfinite(d->lambda_el[0]) || !std::isfinite(d->lambda_el[1]))
        return P4D_ERR_INVALID_ARG;
    if (!(d->hxy[0] >= 0.0) || !(d->hxy[1] >= 0.0) || !std::isfinite(d->hxy[0]) || !std::isfinite(d->hxy[1]))
        return P4D_ERR_INVALID_ARG;
    if ((long long)d->nx * d->ny * d->nz > (1LL << 30)) return P4D_ERR_INVALID_ARG;
    p4d_ctx *c = new p4d_ctx();
    c->desc = *d;
    fill_geom(*d, c->g);
    radial_table(*d, 0, c->tabs_h[0]);
    radial_table(*d, 1, c->tabs_h[1]);
    if (hipHostMalloc((void **)&c->hhost, 8 * 512, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return P4D_ERR_HIP;
    }
    if (alloc_pub(c) != P4D_OK) {
        hipHostFree(c->hhost);
        delete c;
        return P4D_ERR_HIP;
    }
    c->tile_tx = d->nx >= 48 ? 64 : (d->nx >= 24 ? 32 : 16);
    c->tile_cz = 8;
    prof_init(c->prof);
    p4d_default_opts(&c->ws_opts);
    *out = c;
    return P4D_OK;
}

void p4d_destroy(p4d_ctx *c)
{
    if (!c) return;
    prof_free(c->prof);
    if (c->hhost) hipHostFree(c->hhost);
    if (c->hpub) hipHostFree(c->hpub);
    delete c->phys;
    delete c;
}

p4d_status p4d_vector_size(const p4d_ctx *c, int64_t *n_dof, int64_t offsets[6], int64_t *n_elem,
                           int64_t *n_e)
{
    if (!c) return P4D_ERR_INVALID_ARG;
    if (n_dof) *n_dof = c->g.N;
    if (offsets) {
        offsets[0] = 0; offsets[1] = c->g.off_pe; offsets[2] = c->g.off_ce;
        offsets[3] = c->g.off_cs[0]; offsets[4] = c->g.off_cs[1]; offsets[5] = c->g.N;
    }
    if (n_elem) *n_elem = c->g.nelem;
    if (n_e) *n_e = c->g.ne;
    return P4D_OK;
}

p4d_status p4d_workspace_size(const p4d_ctx *cc, const p4d_solve_opts *opts, size_t *bytes)
{
    if (!cc || !bytes) return P4D_ERR_INVALID_ARG;
    p4d_ctx *c = const_cast<p4d_ctx *>(cc);
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return fail(c, P4D_ERR_INVALID_ARG, why);
    // sizing must not disturb a configured context
    p4d_ctx tmp;
    tmp.desc = c->desc;
    tmp.g = c->g;
    *bytes = carve(&tmp, o, nullptr) + kAlign;
    return P4D_OK;
}

static p4d_status ensure_layout(p4d_ctx *c, const p4d_solve_opts &o);

p4d_status p4d_set_workspace(p4d_ctx *c, void *d_work, size_t bytes, const p4d_solve_opts *opts)
{
    if (!c || !d_work) return P4D_ERR_INVALID_ARG;
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return fail(c, P4D_ERR_INVALID_ARG, why);
    c->ws = (char *)d_work;
    c->ws_bytes = bytes;
    c->uploaded = 0;
    c->pc_ready = 0;
    c->storage = 0;
    c->g.meh = nullptr;
    if (c->phys) {
        c->phys->P.por = c->phys->P.act = nullptr;
        c->phys->ready = false;
    }
    return ensure_layout(c, o);
}

// Default level-0 smoother tiles: TX by the grid width, and the layer depth
// CZ that minimizes (rounds of resident workgroups) x (CZ + 2 halo planes),
// so that the last round of tiles is not nearly empty.
static void default_tiles(p4d_ctx *c)
{
    // tile width: the one whose tiles cover the x-y plane with the fewest
    // idle lanes (the wider one on ties, for longer contiguous rows)
    const int nx = c->g.nx, ny = c->g.ny;
    double bestcov = -1.0;
    for (int tx = 16; tx <= 64; tx *= 2) {
        const int ty = kBlock / tx;
        const double cov = (double)nx * ny / ((double)((nx + tx - 1) / tx) * tx * ((ny + ty - 1) / ty) * ty);
        if (cov >= bestcov) {
            bestcov = cov;
            c->tile_tx = tx;
        }
    }
    const long long slots = smooth0_slots();
    long long best = -1;
    for (int cz = 2; cz <= 16; cz++) {
        long long tiles = 0;
        for (int b = 0; b < 4; b++) {
            const Level &L = c->box[b].lev[0];
            tiles += smooth0_tiles(L.nx, L.ny, L.nz, c->tile_tx, cz);
        }
        const long long cost = ((tiles + slots - 1) / slots) * (cz + 2);
        if (best < 0 || cost < best) {
            best = cost;
            c->tile_cz = cz;
        }
    }
    // operator tiles: the same rule over the whole node grid
    c->op_tx = c->tile_tx;
    const long long oslots = operator_tile_slots();
    best = -1;
    for (int cz = 2; cz <= 16; cz++) {
        const long long tiles = operator_tiles(c->g, c->op_tx, cz);
        const long long cost = ((tiles + oslots - 1) / oslots) * (cz + 2);
        if (best < 0 || cost < best) {
            best = cost;
            c->op_cz = cz;
        }
    }
}

static p4d_status ensure_layout(p4d_ctx *c, const p4d_solve_opts &o)
{
    if (!c->ws) return fail(c, P4D_ERR_STATE, "no workspace");
    char *base = (char *)align_up((size_t)c->ws);
    p4d_ctx probe;
    probe.desc = c->desc;
    probe.g = c->g;
    const size_t need = carve(&probe, o, nullptr);
    if (need + (size_t)(base - c->ws) > c->ws_bytes)
        return fail(c, P4D_ERR_OOM, "workspace too small for these options");
    carve(c, o, base);
    c->ws_opts = o;
    if (!c->tiles_tuned) default_tiles(c);
    return P4D_OK;
}

static p4d_status refresh_general(p4d_ctx *c, hipStream_t st);

p4d_status p4d_upload(p4d_ctx *c, const double *sigma, const double *kappa, const double *g,
                      const double *s, const double *e, void *stream)
{
    if (!c || !sigma || !kappa || !g || !s || !e) return P4D_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (!c->ws) return fail(c, P4D_ERR_STATE, "p4d_set_workspace first");
    HIPCHK(c, hipMemcpyAsync(c->tabs, c->tabs_h, sizeof(c->tabs_h), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->gg, g, 8 * c->g.ne, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->ss, s, 8 * c->g.ne, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->ee, e, 8 * c->g.ne, hipMemcpyDeviceToDevice, st));
    launch_setup_nodes(c->g, c->tabs, sigma, kappa, c->sigh, c->kaph, c->mm, st);
    launch_omega(c->g, c->tabs, c->ss, 1, c->oms, st);
    c->general = 0;
    c->box[3].cK = c->kaph;
    c->storage = 0;
    c->transport_set = 0;
    c->g.meh = nullptr;
    HIPCHK(c, hipGetLastError());
    // the host copy of the radial tables must outlive the async copy
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->g.aniso) {
        p4d_status rs = refresh_general(c, st);
        if (rs != P4D_OK) return rs;
    }
    c->uploaded = 1;
    c->pc_ready = 0;
    return P4D_OK;
}

// The per-node operator with its own element arrays (GEN) runs when the
// caller set transport coefficients or a per-element storage, or the
// elements are boxes; otherwise kdh / dch take the defaults chi h kappa and
// h kappa.
static p4d_status refresh_general(p4d_ctx *c, hipStream_t st)
{
    const bool gen = c->transport_set || c->storage || c->g.aniso;
    if (gen && !c->transport_set) {
        launch_scale_elem(c->g, nullptr, c->g.chi, c->kaph, c->kdh, st);
        launch_scale_elem(c->g, nullptr, 1.0, c->kaph, c->dch, st);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(st));
    }
    c->general = gen ? 1 : 0;
    c->box[3].cK = gen ? c->dch : c->kaph;
    return P4D_OK;
}

p4d_status p4d_set_transport(p4d_ctx *c, const double *kappa_d, const double *dce, void *stream)
{
    if (!c) return P4D_ERR_INVALID_ARG;
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    hipStream_t st = (hipStream_t)stream;
    c->pc_ready = 0;
    if (!kappa_d && !dce) {
        c->transport_set = 0;
        return refresh_general(c, st);
    }
    // h * coefficient, or the default from h * kappa
    launch_scale_elem(c->g, kappa_d, kappa_d ? c->g.h : c->g.chi, c->kaph, c->kdh, st);
    launch_scale_elem(c->g, dce, dce ? c->g.h : 1.0, c->kaph, c->dch, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->transport_set = 1;
    return refresh_general(c, st);
}

p4d_status p4d_set_storage(p4d_ctx *c, const double *eps_e, void *stream)
{
    if (!c) return P4D_ERR_INVALID_ARG;
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    if (c->phys) return fail(c, P4D_ERR_INVALID_ARG, "a physical cell sets its storage from its fractions");
    hipStream_t st = (hipStream_t)stream;
    c->pc_ready = 0;
    if (!eps_e) {
        c->storage = 0;
        c->g.meh = nullptr;
        return refresh_general(c, st);
    }
    launch_scale_elem(c->g, eps_e, c->g.vol / c->g.dt, nullptr, c->meh, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->storage = 1;
    c->g.meh = c->meh;
    return refresh_general(c, st);
}

p4d_status p4d_set_diffusivity(p4d_ctx *c, const double Ds[2], void *stream)
{
    if (!c || !Ds || !(Ds[0] > 0.0) || !(Ds[1] > 0.0)) return P4D_ERR_INVALID_ARG;
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    hipStream_t st = (hipStream_t)stream;
    // the previous copy of the tables may still be in flight
    HIPCHK(c, hipStreamSynchronize(st));
    c->desc.Ds[0] = Ds[0];
    c->desc.Ds[1] = Ds[1];
    radial_table(c->desc, 0, c->tabs_h[0]);
    radial_table(c->desc, 1, c->tabs_h[1]);
    HIPCHK(c, hipMemcpyAsync(c->tabs, c->tabs_h, sizeof(c->tabs_h), hipMemcpyHostToDevice, st));
    launch_omega(c->g, c->tabs, c->ss, 1, c->oms, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->pc_ready = 0;
    return P4D_OK;
}

p4d_status p4d_setup(p4d_ctx *c, const p4d_solve_opts *opts, void *stream)
{
    if (!c) return P4D_ERR_INVALID_ARG;
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return fail(c, P4D_ERR_INVALID_ARG, why);
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    if (o.pc == P4D_PC_BGS && c->g.aniso)
        return fail(c, P4D_ERR_INVALID_ARG, "block Gauss-Seidel needs cube elements");
    if (o.smoother == P4D_SMOOTH_ZLINE && c->g.nz > kZlineMaxNz)
        return fail(c, P4D_ERR_INVALID_ARG, "z-line smoothing takes at most 2016 node layers");
    // keep the Krylov sizing of the layout (it is set by the workspace size
    // the caller asked for); the preconditioner part must match o
    p4d_solve_opts lay = c->ws_opts;
    lay.pc_prec = o.pc_prec;
    lay.coarse_max = o.coarse_max;
    lay.smoother = o.smoother;
    if (o.restart > lay.restart) lay.restart = o.restart;
    const bool relayout = lay.pc_prec != c->ws_opts.pc_prec || lay.coarse_max != c->ws_opts.coarse_max ||
                          lay.restart != c->ws_opts.restart || lay.z_fp32 != c->ws_opts.z_fp32 ||
                          lay.smoother != c->ws_opts.smoother;
    if (relayout) {
        // coefficient arrays sit at the start of every layout, so they
        // survive a change of the preconditioner part
        p4d_status rs = ensure_layout(c, lay);
        if (rs != P4D_OK) return rs;
    }
    c->pc = o;
    c->prec = o.pc_prec == P4D_FP32 ? 1 : 0;
    c->lmax_pending = 0;
    hipStream_t st = (hipStream_t)stream;
    p4d_status s = c->prec ? setup_t<float>(c, st) : setup_t<double>(c, st);
    if (s != P4D_OK) return s;
    c->pc_ready = 1;
    return P4D_OK;
}

p4d_status p4d_apply_operator(p4d_ctx *c, int transpose, const double *x, double *y, void *stream)
{
    if (!c || !x || !y || x == y) return P4D_ERR_INVALID_ARG;
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    apply_op<double>(c, transpose, x, y, nullptr, nullptr, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

p4d_status p4d_apply_schur_operator(p4d_ctx *c, int transpose, const double *y, double *w,
                                    void *stream)
{
    if (!c || !y || !w || y == w) return P4D_ERR_INVALID_ARG;
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    apply_op_schur<double>(c, transpose, y, w, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

p4d_status p4d_apply_preconditioner(p4d_ctx *c, int transpose, const double *r, double *z,
                                    void *stream)
{
    if (!c || !r || !z || r == z) return P4D_ERR_INVALID_ARG;
    if (!c->pc_ready) return fail(c, P4D_ERR_STATE, "p4d_setup first");
    const p4d_status fs = finish_setup(c);
    if (fs != P4D_OK) return fs;
    apply_pc<double>(c, transpose, r, nullptr, z, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

static p4d_status solve_common(p4d_ctx *c, int transpose, const double *b, double *x,
                               const p4d_solve_opts *opts, p4d_solve_info *info, void *stream)
{
    if (!c || !b || !x || b == x) return P4D_ERR_INVALID_ARG;
    if (!c->pc_ready) return fail(c, P4D_ERR_STATE, "p4d_setup first");
    p4d_solve_opts o = opts ? *opts : c->pc;
    std::string why;
    if (!opts_valid(o, why)) return fail(c, P4D_ERR_INVALID_ARG, why);
    if (o.pc != c->pc.pc || o.pc_prec != c->pc.pc_prec || o.cheb_degree != c->pc.cheb_degree ||
        o.coarse_max != c->pc.coarse_max || o.smoother != c->pc.smoother ||
        (o.pc == P4D_PC_BGS && o.bgs_order != c->pc.bgs_order))
        return fail(c, P4D_ERR_STATE, "preconditioner options differ from the last setup");
    if (o.restart > c->ws_opts.restart || (!o.z_fp32 && c->ws_opts.z_fp32))
        return fail(c, P4D_ERR_OOM, "workspace sized for a smaller restart or an FP32 Z basis");
    hipStream_t st = (hipStream_t)stream;
    if (o.z_fp32) return fgmres<float>(c, transpose, b, x, o, info, st);
    return fgmres<double>(c, transpose, b, x, o, info, st);
}

p4d_status p4d_solve(p4d_ctx *c, const double *b, double *x, const p4d_solve_opts *opts,
                     p4d_solve_info *info, void *stream)
{
    return solve_common(c, 0, b, x, opts, info, stream);
}

p4d_status p4d_solve_adjoint(p4d_ctx *c, const double *g, double *lam, const p4d_solve_opts *opts,
                             p4d_solve_info *info, void *stream)
{
    return solve_common(c, 1, g, lam, opts, info, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// upload + setup + solve with no workspace argument: the whole workspace is
// carved from a file-scope device array (one copy per GPU, held until the
// process ends), so the call allocates no device or pinned memory.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char noalloc_scratch[P4D_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
void *noalloc_ptr[kMaxDevices];   // device address of noalloc_scratch, per device
}  // namespace

// The device address of the scratch array on the current device, looked up
// once per device with that device current (in host code the array's name
// is only a host-side stand-in).
static p4d_status noalloc_base(p4d_ctx *c, char **out)
{
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, P4D_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p)
            return fail(c, P4D_ERR_HIP, std::string("hipGetSymbolAddress(noalloc_scratch): ") +
                                            hipGetErrorString(e));
        noalloc_ptr[dev] = p;
    }
    *out = (char *)noalloc_ptr[dev];
    return P4D_OK;
}

extern "C" {

p4d_status p4d_solve_noalloc(p4d_ctx *c, const double *sigma, const double *kappa, const double *g,
                             const double *s, const double *e, const double *b, double *x,
                             const p4d_solve_opts *opts, p4d_solve_info *info, void *stream)
{
    if (!c || !sigma || !kappa || !g || !s || !e || !b || !x || b == x) return P4D_ERR_INVALID_ARG;
    if (c->phys) return fail(c, P4D_ERR_INVALID_ARG, "a physical cell solves through p4d_phys_newton_step");
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return fail(c, P4D_ERR_INVALID_ARG, why);
    // a context of its own, on the caller's problem, bound to the scratch:
    // the caller's context (its workspace, uploads and setup) is untouched
    p4d_ctx t;
    t.desc = c->desc;
    t.g = c->g;
    t.g.meh = nullptr;
    t.tabs_h[0] = c->tabs_h[0];
    t.tabs_h[1] = c->tabs_h[1];
    t.tile_tx = c->tile_tx;
    t.tile_cz = c->tile_cz;
    t.tiles_tuned = c->tiles_tuned;
    t.op_tx = c->op_tx;
    t.op_cz = c->op_cz;
    const size_t need = carve(&t, o, nullptr) + kAlign;
    if (need > (size_t)P4D_NOALLOC_MAX_BYTES)
        return fail(c, P4D_ERR_OOM, "p4d_solve_noalloc: this problem needs " + std::to_string(need) +
                                        " bytes of scratch, more than the " +
                                        std::to_string((size_t)P4D_NOALLOC_MAX_BYTES) + " it holds");
    char *base = nullptr;
    p4d_status st = noalloc_base(c, &base);
    if (st != P4D_OK) return st;
    t.hhost = c->hhost;   // the caller context's pinned staging (no allocation)
    t.hpub = c->hpub;
    t.hpub_dev = c->hpub_dev;
    t.pub_seq = c->pub_seq;
    t.ws = base;
    t.ws_bytes = P4D_NOALLOC_MAX_BYTES;
    // every array of the layout is written before it is read (as with a
    // fresh caller workspace), so nothing in the scratch is cleared here
    st = ensure_layout(&t, o);
    if (st == P4D_OK) st = p4d_upload(&t, sigma, kappa, g, s, e, stream);
    if (st == P4D_OK) st = p4d_setup(&t, &o, stream);
    if (st == P4D_OK) st = p4d_solve(&t, b, x, &o, info, stream);
    if (st != P4D_OK) c->err = t.err;
    c->pub_seq = t.pub_seq;
    t.hhost = nullptr;
    t.hpub = t.hpub_dev = nullptr;
    return st;
}

p4d_status p4d_phys_create(const p4d_phys_params *p, p4d_ctx **out)
{
    if (!p || !out) return P4D_ERR_INVALID_ARG;
    *out = nullptr;
    const int n = p->n;
    if (n < 19 || (n - 1) % 9 != 0 || n > 1024) return P4D_ERR_INVALID_ARG;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(p->dt) || !pos(p->edge) || !pos(p->F) || !pos(p->R) || !pos(p->T) || !pos(p->ce0) ||
        !pos(p->eps_sep) || !pos(p->brug) || !pos(p->gauss_frac) || !std::isfinite(p->current) ||
        !(p->t_plus >= 0.0 && p->t_plus < 1.0) || (p->profile != 0 && p->profile != 1))
        return P4D_ERR_INVALID_ARG;
    for (int el = 0; el < 2; el++) {
        const p4d_electrode &e = p->el[el];
        if (!pos(e.eps_s) || !pos(e.eps) || !pos(e.sigma) || !pos(e.k) || !pos(e.alpha) ||
            !pos(e.cs_max) || !pos(e.cs0) || !(e.cs0 < e.cs_max) || !pos(e.a) || !pos(e.Ds) ||
            !pos(e.Rs))
            return P4D_ERR_INVALID_ARG;
    }
    if (p->el[0].eps != p->el[1].eps) return P4D_ERR_INVALID_ARG;
    // scales: unknowns x (RT/F, c_e0, the mean c_s,max), equations r (inverse
    // diagonal magnitude of the phi_e, c_e and c_s rows at the rest state)
    PhysDev P{};
    P.F = p->F;
    P.RT = p->R * p->T;
    P.tplus = p->t_plus;
    P.brug = p->brug;
    P.ce0 = p->ce0;
    P.eps_el = p->el[0].eps;
    P.eps_sep = p->eps_sep;
    for (int el = 0; el < 2; el++) {
        const p4d_electrode &e = p->el[el];
        P.eps_s[el] = e.eps_s; P.sigma[el] = e.sigma; P.k[el] = e.k; P.alpha[el] = e.alpha;
        P.csmax[el] = e.cs_max; P.cs0[el] = e.cs0; P.a[el] = e.a;
    }
    const double h = p->edge / (n - 1), eps = p->el[0].eps;
    P.xphi = P.RT / P.F;
    P.xc = p->ce0;
    P.xs = 0.5 * (p->el[0].cs_max + p->el[1].cs_max);
    const double kap0 = std::pow(eps, p->brug) * kappa_bulk_h(p->ce0);
    const double d0 = std::pow(eps, p->brug) * de_bulk_h(p->ce0);
    P.rphi = 1.0 / (kap0 * h * P.xphi);
    P.rc = 1.0 / ((eps * h * h * h / p->dt + d0 * h) * P.xc);
    P.rs = p->dt / P.xs;
    const double tfac = P.rs * P.xs;
    // the scaled Newton matrix as an operator description
    p4d_problem_desc d{};
    const int e25 = (n - 1) / 9;
    d.nx = d.ny = d.nz = n;
    d.na = 4 * e25 + 1;
    d.ns = e25 - 1;
    for (int el = 0; el < 2; el++) {
        const p4d_electrode &e = p->el[el];
        d.nr[el] = p->nr[el];
        d.Ds[el] = e.Ds / (e.Rs * e.Rs) * tfac;
        d.theta_bar[el] = p->theta_bar[el];
        d.lambda_el[el] = 1.0 / (p->F * e.Rs * e.a) * P.rs / P.rphi;
    }
    d.dt = p->dt / tfac;
    d.chi = 0.0;
    d.tc = (1.0 - p->t_plus) / p->F * P.rc / P.rphi;
    d.lambda_c = 1.0;
    d.eps_elec = P.rc * P.xc * eps / tfac;
    d.eps_sep = P.rc * P.xc * p->eps_sep / tfac;
    d.length = p->edge;
    const p4d_status s = p4d_create(&d, out);
    if (s != P4D_OK) return s;
    (*out)->phys = new PhysState();
    (*out)->phys->prm = *p;
    (*out)->phys->P = P;
    return P4D_OK;
}

p4d_status p4d_phys_workspace_size(const p4d_ctx *c, size_t *bytes)
{
    if (!c || !bytes || !c->phys) return P4D_ERR_INVALID_ARG;
    *bytes = 4 * align_up(8 * (size_t)c->g.N) + 2 * align_up(8 * (size_t)c->g.ne) +
             5 * align_up(8 * (size_t)c->g.nelem) + 256;
    return P4D_OK;
}

p4d_status p4d_phys_set_workspace(p4d_ctx *c, void *d_work, size_t bytes)
{
    if (!c || !d_work || !c->phys) return P4D_ERR_INVALID_ARG;
    if (!c->ws) return fail(c, P4D_ERR_STATE, "p4d_set_workspace first");
    size_t need;
    p4d_phys_workspace_size(c, &need);
    if (bytes < need) return fail(c, P4D_ERR_OOM, "Newton buffers too small");
    char *p = (char *)align_up((size_t)d_work);
    auto take = [&](size_t b) { char *q = p; p += align_up(b); return (double *)q; };
    PhysState &S = *c->phys;
    S.uh = take(8 * (size_t)c->g.N);
    S.rh = take(8 * (size_t)c->g.N);
    S.dh = take(8 * (size_t)c->g.N);
    S.old = take(8 * (size_t)c->g.N);
    S.fh = take(8 * (size_t)c->g.ne);
    S.qh = take(8 * (size_t)c->g.ne);
    S.por = take(8 * (size_t)c->g.nelem);
    S.act = take(8 * (size_t)c->g.nelem);
    S.nwa = take(8 * (size_t)c->g.nelem);
    S.nwb = take(8 * (size_t)c->g.nelem);
    S.nwc = take(8 * (size_t)c->g.nelem);
    S.P.por = S.P.act = nullptr;
    c->storage = 0;
    c->g.meh = nullptr;
    S.ready = false;
    return P4D_OK;
}

p4d_status p4d_phys_set_fractions(p4d_ctx *c, const double *eps_s, const double *eps_b, void *stream)
{
    if (!c || !c->phys || (!eps_s) != (!eps_b)) return P4D_ERR_INVALID_ARG;
    PhysState &S = *c->phys;
    if (!S.uh) return fail(c, P4D_ERR_STATE, "p4d_phys_set_workspace first");
    c->pc_ready = 0;
    S.P.por = S.P.act = nullptr;
    c->storage = 0;
    c->g.meh = nullptr;
    if (!eps_s) return P4D_OK;
    hipStream_t st = (hipStream_t)stream;
    const double h = c->g.h;
    const double ms = S.P.rc * S.P.xc * h * h * h / S.prm.dt;
    const int nb = launch_phys_fractions(c->g, S.P, eps_s, eps_b, S.por, S.act, c->meh, ms, c->red, st);
    launch_max_final(c->red, nb, c->scal + 100, st);
    HIPCHK(c, hipMemcpyAsync(c->hhost, c->scal + 100, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->hhost[0] != 0.0)
        return fail(c, P4D_ERR_INVALID_ARG, "volume fractions outside (0, 1) or no porosity left");
    S.P.por = S.por;
    S.P.act = S.act;
    c->storage = 1;
    c->g.meh = c->meh;
    return P4D_OK;
}

p4d_status p4d_phys_initial_state(p4d_ctx *c, double *u, void *stream)
{
    if (!c || !u || !c->phys) return P4D_ERR_INVALID_ARG;
    launch_phys_init(c->g, c->phys->P, u, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

p4d_status p4d_phys_residual(p4d_ctx *c, const double *u, const double *uold, double *r, void *stream)
{
    if (!c || !u || !uold || !r || !c->phys) return P4D_ERR_INVALID_ARG;
    if (!c->phys->uh) return fail(c, P4D_ERR_STATE, "p4d_phys_set_workspace first");
    hipStream_t st = (hipStream_t)stream;
    p4d_status s = phys_prepare(c, st);
    if (s == P4D_OK) s = phys_old(c, uold, st);
    if (s == P4D_OK) s = phys_residual(c, u, c->phys->rh, 0, st);
    if (s != P4D_OK) return s;
    launch_phys_unscale_rows(c->g, c->phys->P, c->phys->rh, r, st);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

p4d_status p4d_phys_jacobian_apply(p4d_ctx *c, const double *u, int transpose, const double *x, double *y,
                                   void *stream)
{
    if (!c || !u || !x || !y || x == y || !c->phys) return P4D_ERR_INVALID_ARG;
    if (!c->phys->uh) return fail(c, P4D_ERR_STATE, "p4d_phys_set_workspace first");
    hipStream_t st = (hipStream_t)stream;
    p4d_status s = phys_prepare(c, st);
    if (s != P4D_OK) return s;
    phys_coef(c, u, st);
    newton_terms_on(c, u);
    apply_op<double>(c, transpose, x, y, nullptr, nullptr, st);
    newton_terms_on(c, nullptr);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

p4d_status p4d_phys_newton_step(p4d_ctx *c, double *u, const double *uold, const p4d_solve_opts *solve,
                                const p4d_newton_opts *newton, p4d_newton_info *info, void *stream)
{
    if (!c || !u || !uold || u == uold || !c->phys) return P4D_ERR_INVALID_ARG;
    PhysState &S = *c->phys;
    if (!S.uh) return fail(c, P4D_ERR_STATE, "p4d_phys_set_workspace first");
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (solve) o = *solve;
    std::string why;
    if (!opts_valid(o, why)) return fail(c, P4D_ERR_INVALID_ARG, why);
    if (o.restart > c->ws_opts.restart || (!o.z_fp32 && c->ws_opts.z_fp32))
        return fail(c, P4D_ERR_OOM, "workspace sized for a smaller restart or an FP32 Z basis");
    const int maxit = newton ? newton->maxit : 30;
    const double tol = newton ? newton->tol : 1e-9;
    if (maxit < 1 || !(tol > 0.0)) return fail(c, P4D_ERR_INVALID_ARG, "newton options");
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    p4d_newton_info inf{};
    inf.status = 1;
    p4d_status s = phys_prepare(c, st);
    if (s == P4D_OK) s = phys_old(c, uold, st);
    if (s != P4D_OK) return s;
    for (int it = 0; it < maxit; it++) {
        s = phys_residual(c, u, S.rh, 1, st);   // right-hand side -R^
        if (s != P4D_OK) return s;
        s = p4d_setup(c, &o, st);
        if (s != P4D_OK) return s;
        p4d_solve_info li{};
        // the exact Newton matrix: with the c_e-derivative terms at u (the
        // preconditioner above is built without them)
        newton_terms_on(c, u);
        s = o.z_fp32 ? fgmres<float>(c, 0, S.rh, S.dh, o, &li, st) : fgmres<double>(c, 0, S.rh, S.dh, o, &li, st);
        newton_terms_on(c, nullptr);
        if (s != P4D_OK && s != P4D_NOT_CONVERGED) {
            inf.status = s;
            break;
        }
        inf.lin_iters += li.iters;
        const int nb = launch_phys_update(c->g, S.P, S.dh, u, c->red, st);
        launch_max_final(c->red, nb, c->scal + 100, st);
        {
            const p4d_status ps = pull(c, c->scal + 100, 1, st);
            if (ps != P4D_OK) return ps;
        }
        inf.iters = it + 1;
        inf.update = *(const double *)c->hpub;
        if (!std::isfinite(inf.update)) {
            inf.status = P4D_ERR_NONFINITE;
            break;
        }
        if (inf.update <= tol) {
            inf.status = 0;
            break;
        }
    }
    inf.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    if (inf.status == 0) return P4D_OK;
    return inf.status == 1 ? P4D_NOT_CONVERGED : (p4d_status)inf.status;
}

p4d_status p4d_param_gradient(p4d_ctx *c, const double *x, const double *lam, double *dsigma,
                              double *dDs, void *stream)
{
    if (!c || !x || !lam || !dsigma || !dDs) return P4D_ERR_INVALID_ARG;
    if (!c->uploaded) return fail(c, P4D_ERR_STATE, "p4d_upload first");
    if (c->g.aniso) return fail(c, P4D_ERR_INVALID_ARG, "parameter gradients need cube elements");
    hipStream_t st = (hipStream_t)stream;
    launch_grad(c->g, c->tabs, x, lam, dsigma, c->red, st);
    const long long n = c->g.nelem > c->g.ne ? c->g.nelem : c->g.ne;
    launch_grad_final(c->red, (int)((n + kBlock - 1) / kBlock), dDs, st);
    HIPCHK(c, hipGetLastError());
    return P4D_OK;
}

p4d_status p4d_profile(p4d_ctx *c, int mask)
{
    if (!c || mask < 0 || mask >= (1 << P4D_K_COUNT)) return P4D_ERR_INVALID_ARG;
    prof_reset(c->prof, mask);
    return P4D_OK;
}

p4d_status p4d_profile_every(p4d_ctx *c, int every)
{
    if (!c || every < 1) return P4D_ERR_INVALID_ARG;
    c->prof.every = every;
    for (int k = 0; k < P4D_K_COUNT; k++) c->prof.seen[k] = 0;
    return P4D_OK;
}

p4d_status p4d_profile_read(p4d_ctx *c, int cls, double *total_ms, int64_t *launches,
                            double *bytes)
{
    if (!c || cls < 1 || cls >= P4D_K_COUNT) return P4D_ERR_INVALID_ARG;
    prof_harvest(c->prof);
    if (total_ms) *total_ms = c->prof.total_ms[cls];
    if (launches) *launches = c->prof.launches[cls];
    if (bytes) *bytes = c->prof.total_bytes[cls];
    return P4D_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Tile autotuning of the level-0 smoother: every candidate shape is timed on
// one Chebyshev step over the four boxes of this context and the fastest is
// kept.  The step writes only preconditioner buffers, which every
// preconditioner application overwrites before reading.
// ---------------------------------------------------------------------------
template <typename T>
static p4d_status tune_tiles_t(p4d_ctx *c, hipStream_t st)
{
    static const int txs[3] = {16, 32, 64};
    const int boxes[4] = {0, 1, 2, 3};
    const int mask = c->prof.mask;
    c->prof.mask = 0;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(c, P4D_ERR_HIP, "hipEventCreate");
    }
    float best = 0.f;
    int btx = c->tile_tx, bcz = c->tile_cz;
    hipError_t he = hipSuccess;
    for (int a = 0; a < 3 && he == hipSuccess; a++)
        for (int cz = 2; cz <= 16 && he == hipSuccess; cz++) {
            c->tile_tx = txs[a];
            c->tile_cz = cz;
            VState<T> vs{};
            smooth_step<T>(c, vs, 0, boxes, 4, 1, 1, st);   // warm-up
            hipEventRecord(e0, st);
            for (int rep = 0; rep < 4; rep++) smooth_step<T>(c, vs, 0, boxes, 4, 1, 1, st);
            hipEventRecord(e1, st);
            he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he == hipSuccess && (best == 0.f || ms < best)) {
                best = ms;
                btx = txs[a];
                bcz = cz;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tile_tx = btx;
    c->tile_cz = bcz;
    c->tiles_tuned = 1;
    c->prof.mask = mask;
    if (he != hipSuccess) return hipchk(c, he, "smoother tile timing");
    return hipchk(c, hipGetLastError(), "smoother tile timing");
}

static p4d_status tune_tiles(p4d_ctx *c, hipStream_t st)
{
    const p4d_status fs = finish_setup(c);
    if (fs != P4D_OK) return fs;
    return c->prec ? tune_tiles_t<float>(c, st) : tune_tiles_t<double>(c, st);
}

// ---------------------------------------------------------------------------
// Batched solves: independent cells, each a full context with its own slice
// of the batch workspace, iterate FGMRES in lockstep.  Per Arnoldi step there
// are the preconditioner launches for all iterating cells (one per stage
// depth), then
// batched operator, Gram-Schmidt and norm launches, and one device-to-host
// copy of every cell's Hessenberg column; the Givens updates run on the host
// per cell exactly as in the single-cell driver.
// ---------------------------------------------------------------------------
struct p4d_batch {
    int n = 0;
    std::vector<p4d_ctx *> cell;
    std::string err;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    p4d_solve_opts ws_opts{};
    int ready = 0;                  // workspace carved
    // device tables
    BCell *bcell = nullptr;
    PCell *pcell = nullptr;
    void *stages = nullptr;
    int *order = nullptr, *ustart = nullptr;
    double *hb = nullptr;           // per cell 256 values (h, norms)
    double *yb = nullptr;           // per cell 64 least-squares coefficients
    int *kused = nullptr;
    // pinned host mirrors
    double *hb_h = nullptr, *yb_h = nullptr;
    int *kused_h = nullptr;
    // recorded schedule
    int recorded = 0, rec_prec = -1;
    int nstages = 0, nrmax = 8;
    struct WorkList {
        int family, nr;             // stage family, radial size class
        int kinds = 0;              // level-0 smoothing lists: 1 steps, 2 residuals, 3 both
        int pos0, npos;             // queue positions
        int item0, nitems;          // units
        int depth;                  // stage depth
    };
    std::vector<WorkList> lists;    // in launch order
    int tile_cz = 0;                // level-0 tile depth of the batch (0: chosen at recording)
    std::vector<double> pc_bytes;   // per cell: level-0 and particle bytes of one application
    int pc_mode = 0;                // 0: batched stage launches, 1: per-cell launches,
                                    // 2: one persistent launch per application
    // persistent application: first item of every stage depth, grid size
    int *dstart = nullptr;
    int npos = 0, ndepth = 0, pgrid = 0;
    hipError_t plaunch = hipSuccess;   // status of the last cooperative launch
    Prof prof;
};

static p4d_status bfail(p4d_batch *B, p4d_status s, const std::string &msg)
{
    if (B) B->err = msg;
    return s;
}
#define BHIPCHK(B, call)                                                              \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess)                                                         \
            return bfail((B), P4D_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

static size_t batch_carve(p4d_batch *B, const p4d_solve_opts &o, char *base, p4d_status *st)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    *st = P4D_OK;
    for (int i = 0; i < B->n; i++) {
        p4d_ctx *c = B->cell[i];
        p4d_ctx probe;
        probe.desc = c->desc;
        probe.g = c->g;
        const size_t need = carve(&probe, o, nullptr);
        char *p = take(need);
        if (base) {
            c->ws = p;
            c->ws_bytes = need;
            c->uploaded = 0;
            c->pc_ready = 0;
            const p4d_status s = ensure_layout(c, o);
            if (s != P4D_OK) {
                *st = s;
                B->err = "cell " + std::to_string(i) + ": " + c->err;
            }
        }
    }
    const size_t maxst = (size_t)B->n * kMaxStagesPerCell;
    static_assert(sizeof(PStage<double>) >= sizeof(PStage<float>), "stage size");
    B->bcell = (BCell *)take(sizeof(BCell) * B->n);
    B->pcell = (PCell *)take(sizeof(PCell) * B->n);
    B->stages = take(sizeof(PStage<double>) * maxst);
    B->order = (int *)take(4 * maxst);
    B->ustart = (int *)take(4 * maxst);
    B->dstart = (int *)take(4 * (maxst + 1));
    B->hb = (double *)take(8 * 256 * (size_t)B->n);
    B->yb = (double *)take(8 * 64 * (size_t)B->n);
    B->kused = (int *)take(4 * (size_t)B->n);
    return off;
}

template <typename T>
static double stage_bytes(const PStage<T> &S, const Geom &g)
{
    double bytes = 0.0;
    switch (S.kind) {
    case SK_RADF:
        return 8.0 * g.N + 32.0 * g.ne + (sizeof(T) * 2 + 8.0) * g.Nm;
    case SK_RADB:
        return 8.0 * (g.N - g.Nm) + 8.0 * g.ne + 8.0 * g.Nm + 8.0 * g.N + 40.0 * g.ne;
    case SK_SM0:
        for (int q = 0; q < S.u.lb.nbox; q++) {
            const LevelArgs<T> &A = S.u.lb.a[q];
            bytes += (16.0 + 8.0 + sizeof(T) * (3 + (A.c1 != 0.0 && !A.din_x) + (A.dout != nullptr))) * A.n;
        }
        return bytes;
    case SK_SM0R:
        for (int q = 0; q < S.u.lb.nbox; q++) bytes += (8.0 + 8.0 + sizeof(T) * 3) * S.u.lb.a[q].n;
        return bytes;
    default:
        return 0.0;   // coarse levels: not counted
    }
}

// Level-0 tile depth for the whole batch: the one that minimizes (rounds of
// resident workgroups over all cells' tiles) x (CZ + 2 halo planes).
template <typename T>
static int batch_default_cz(p4d_batch *B)
{
    const long long slots = bstage_sm0_slots<T>();
    long long best = -1;
    int bcz = 8;
    for (int cz = 2; cz <= 16; cz++) {
        long long tiles = 0;
        for (p4d_ctx *c : B->cell)
            for (int b = 0; b < 4; b++) {
                const Level &L = c->box[b].lev[0];
                tiles += smooth0_tiles(L.nx, L.ny, L.nz, c->tile_tx, cz);
            }
        const long long cost = ((tiles + slots - 1) / slots) * (cz + 2);
        if (best < 0 || cost < best) {
            best = cost;
            bcz = cz;
        }
    }
    return bcz;
}

// Records every cell's preconditioner schedule and builds the work lists.
// Depths: the stages before a cell's first prolongation keep their index,
// the rest are placed so that every cell's last stage falls on the last
// depth.  Per depth, one list per stage family (per radial size class for
// the particle stages), larger cells first.
template <typename T>
static p4d_status batch_record(p4d_batch *B)
{
    const int n = B->n;
    std::vector<std::vector<PStage<T>>> per(n);
    B->pc_bytes.assign(n, 0.0);
    B->nrmax = 8;
    const int cz = B->tile_cz > 0 ? B->tile_cz : batch_default_cz<T>(B);
    for (int i = 0; i < n; i++) {
        const p4d_status fs = finish_setup(B->cell[i]);
        if (fs != P4D_OK) return bfail(B, fs, "cell " + std::to_string(i) + ": " + B->cell[i]->err);
    }
    for (int i = 0; i < n; i++) {
        p4d_ctx *c = B->cell[i];
        const int keep = c->tile_cz;
        c->tile_cz = cz;
        c->rec = &per[i];
        c->rec_cell = i;
        apply_pc_t<T, double>(c, 0, nullptr, nullptr, (double *)nullptr, nullptr);
        c->rec = nullptr;
        c->tile_cz = keep;
        if ((int)per[i].size() > kMaxStagesPerCell)
            return bfail(B, P4D_ERR_INVALID_ARG, "too many preconditioner stages in a cell");
        for (const PStage<T> &S : per[i]) B->pc_bytes[i] += stage_bytes(S, c->g);
        const int nr = rad_nrmax(c->g);
        B->nrmax = nr > B->nrmax ? nr : B->nrmax;
    }
    std::vector<PStage<T>> all;
    std::vector<int> base(n), split(n);
    int A = 0, Bm = 0;
    for (int i = 0; i < n; i++) {
        base[i] = (int)all.size();
        all.insert(all.end(), per[i].begin(), per[i].end());
        const int L = (int)per[i].size();
        int p = L;
        for (int j = 0; j < L; j++)
            if (per[i][j].kind == SK_PROLONG) { p = j; break; }
        split[i] = p;
        A = p > A ? p : A;
        Bm = L - p > Bm ? L - p : Bm;
    }
    const int depth = A + Bm;
    // stage of cell i at depth d, or -1
    std::vector<int> at((size_t)n * depth, -1);
    for (int i = 0; i < n; i++) {
        const int L = (int)per[i].size();
        for (int j = 0; j < L; j++) {
            const int d = j < split[i] ? j : depth - (L - j);
            at[(size_t)i * depth + d] = j;
        }
    }
    std::vector<int> bysize(n);
    for (int i = 0; i < n; i++) bysize[i] = i;
    std::stable_sort(bysize.begin(), bysize.end(),
                     [&](int a, int b) { return B->cell[a]->g.N > B->cell[b]->g.N; });
    std::vector<int> order, ustart;
    B->lists.clear();
    long long items = 0;
    for (int d = 0; d < depth; d++)
        for (int fam = SF_RADF; fam <= SF_MISC; fam++) {
            const bool radial = fam == SF_RADF || fam == SF_RADB;
            for (int ci = 0; ci < (radial ? kNrClasses : 1); ci++) {
                p4d_batch::WorkList W{fam, radial ? kNrClass[ci] : 8, 0, (int)order.size(), 0, (int)items, 0, d};
                for (int i : bysize) {
                    const int j = at[(size_t)i * depth + d];
                    if (j < 0 || stage_family(per[i][j].kind) != fam) continue;
                    if (radial && rad_nrmax(B->cell[i]->g) != kNrClass[ci]) continue;
                    if (fam == SF_SM0) W.kinds |= per[i][j].kind == SK_SM0 ? 1 : 2;
                    order.push_back(base[i] + j);
                    ustart.push_back((int)items);
                    items += per[i][j].nunits;
                }
                W.npos = (int)order.size() - W.pos0;
                W.nitems = (int)(items - W.item0);
                if (W.npos > 0) B->lists.push_back(W);
                if (items >= (1LL << 31) - (1LL << 20))
                    return bfail(B, P4D_ERR_INVALID_ARG, "work list too long");
            }
        }
    BHIPCHK(B, hipMemcpy(B->stages, all.data(), sizeof(PStage<T>) * all.size(), hipMemcpyHostToDevice));
    BHIPCHK(B, hipMemcpy(B->order, order.data(), 4 * order.size(), hipMemcpyHostToDevice));
    BHIPCHK(B, hipMemcpy(B->ustart, ustart.data(), 4 * ustart.size(), hipMemcpyHostToDevice));
    // the persistent application walks the same items depth by depth: the
    // first item of every depth (the work lists are in depth order)
    std::vector<int> dstart(depth + 1, (int)items);
    for (int d = depth - 1, li = (int)B->lists.size() - 1; d >= 0; d--) {
        dstart[d] = dstart[d + 1];
        for (; li >= 0 && B->lists[li].depth == d; li--) dstart[d] = B->lists[li].item0;
    }
    BHIPCHK(B, hipMemcpy(B->dstart, dstart.data(), 4 * dstart.size(), hipMemcpyHostToDevice));
    B->npos = (int)order.size();
    B->ndepth = depth;
    B->pgrid = batch_persist_slots<T, double>(B->nrmax);
    B->nstages = (int)all.size();
    B->recorded = 1;
    B->rec_prec = B->cell[0]->prec;
    return P4D_OK;
}

namespace {
struct CellRun {
    std::vector<double> H, cs, sn, gv, yv, hc, beta;
    double bnorm = 0.0;
    int total = 0, kused = 0;
    bool done = false, first = true, in_cycle = false, breakdown = false, nonfinite = false;
    p4d_status status = P4D_NOT_CONVERGED;
    p4d_solve_info inf{};
};
}  // namespace

// Cell tables of the batched kernels for restart length m (b and x may be
// null when only the preconditioner is used); copied to the device.
struct BatchGrid {
    int op = 0, st = 0, tile = 0, rad = 0;   // workgroups of each batched launch kind
};
static p4d_status batch_tables(p4d_batch *B, int m, const double *const *bv, double *const *xv,
                               std::vector<BCell> &bc, BatchGrid &G, hipStream_t st)
{
    const int n = B->n;
    bc.assign(n, BCell{});
    std::vector<PCell> pcl(n);
    G = BatchGrid{};
    // operator tile depth for the batch as a whole (same rule as the
    // single-cell default, over the tiles of all cells)
    int opcz = 8;
    {
        const long long slots = operator_tile_slots();
        long long best = -1;
        for (int cz = 2; cz <= 16; cz++) {
            long long tiles = 0;
            for (p4d_ctx *c : B->cell) tiles += operator_tiles(c->g, c->op_tx > 0 ? c->op_tx : 64, cz);
            const long long cost = ((tiles + slots - 1) / slots) * (cz + 2);
            if (best < 0 || cost < best) {
                best = cost;
                opcz = cz;
            }
        }
    }
    for (int i = 0; i < n; i++) {
        p4d_ctx *c = B->cell[i];
        const Geom &g = c->g;
        BCell &C = bc[i];
        std::memset((void *)&C, 0, sizeof(C));
        C.g = g;
        C.op = OpArgs{c->tabs, c->sigh, c->kaph, c->gg, c->ss, c->ee, c->mm, nullptr, nullptr, nullptr};
        C.op_blk0 = G.op;
        C.op_nblk = operator_blocks(g);
        G.op += C.op_nblk;
        C.st_blk0 = G.st;
        C.st_nblk = stream_blocks(g.N);
        G.st += C.st_nblk;
        C.op_tx = c->op_tx > 0 ? c->op_tx : 64;
        C.op_cz = opcz;
        C.tile_blk0 = G.tile;
        C.tile_n = operator_tiles(g, C.op_tx, C.op_cz);
        G.tile += C.tile_n;
        C.rad_blk0 = G.rad;
        C.rad_n = (int)((g.ne + kBlock - 1) / kBlock);
        G.rad += C.rad_n;
        C.qbuf = c->qbuf;
        C.V = (double *)c->scratch;
        C.Z = c->scratch + align_up(8 * (size_t)(m + 1) * g.N);
        C.x = xv ? xv[i] : nullptr;
        C.b = bv ? bv[i] : nullptr;
        C.red = c->red;
        C.h = B->hb + 256 * (size_t)i;
        C.coef = c->cdev;
        C.invbeta = c->invbeta;
        C.y = B->yb + 64 * (size_t)i;
        C.kused = B->kused + i;
        PCell &P = pcl[i];
        std::memset((void *)&P, 0, sizeof(P));
        P.g = g;
        P.R = c->rec_R;
        P.V = C.V;
        P.Z = C.Z;
        P.invbeta = c->invbeta;
        P.schur = c->pc.pc == P4D_PC_SCHUR;
    }
    BHIPCHK(B, hipStreamSynchronize(st));
    BHIPCHK(B, hipMemcpy(B->bcell, bc.data(), sizeof(BCell) * n, hipMemcpyHostToDevice));
    BHIPCHK(B, hipMemcpy(B->pcell, pcl.data(), sizeof(PCell) * n, hipMemcpyHostToDevice));
    return P4D_OK;
}

// One batched preconditioner application z_k = P^-1 V_k / beta_k for the
// cells in `active` (work lists of the recorded schedule, in order).
template <typename T, typename TZ>
static void batch_apply_pc(p4d_batch *B, int transpose, int k, unsigned long long active, hipStream_t st)
{
    if (B->pc_mode == 2) {   // one cooperative launch for all depths
        PersistRun pr{};
        pr.stages = B->stages;
        pr.cells = B->pcell;
        pr.order = B->order;
        pr.ustart = B->ustart;
        pr.dstart = B->dstart;
        pr.npos = B->npos;
        pr.ndepth = B->ndepth;
        pr.transpose = transpose;
        pr.k = k;
        pr.active = active;
        B->plaunch = launch_batch_persist<T, TZ>(pr, B->nrmax, B->pgrid, st);
        return;
    }
    StageRun run{};
    run.stages = B->stages;
    run.cells = B->pcell;
    run.order = B->order;
    run.ustart = B->ustart;
    run.transpose = transpose;
    run.k = k;
    run.active = active;
    for (const p4d_batch::WorkList &W : B->lists) {
        run.pos0 = W.pos0;
        run.npos = W.npos;
        run.item0 = W.item0;
        run.nitems = W.nitems;
        launch_batch_stage<T, TZ>(run, W.family, W.nr, W.kinds, st);
    }
}

// Batch tile tuning: every candidate level-0 tile depth is recorded and
// timed on whole batched preconditioner applications (all cells, step 0;
// only preconditioner buffers and the first preconditioned direction are
// written); the fastest is kept.
template <typename T, typename TZ>
static p4d_status batch_tune_t(p4d_batch *B, hipStream_t st)
{
    std::vector<BCell> bc;
    BatchGrid G;
    const unsigned long long all = B->n == 64 ? ~0ULL : ((1ULL << B->n) - 1);
    static const int czs[9] = {2, 3, 4, 5, 6, 8, 10, 12, 16};
    hipEvent_t e0, e1;
    BHIPCHK(B, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(B, P4D_ERR_HIP, "hipEventCreate");
    }
    float best = 0.f;
    int bcz = 8;
    p4d_status s = P4D_OK;
    for (int q = 0; q < 9 && s == P4D_OK; q++) {
        B->tile_cz = czs[q];
        s = batch_record<T>(B);
        if (s == P4D_OK) s = batch_tables(B, B->ws_opts.restart, nullptr, nullptr, bc, G, st);
        if (s != P4D_OK) break;
        batch_apply_pc<T, TZ>(B, 0, 0, all, st);   // warm-up
        (void)hipEventRecord(e0, st);
        for (int rep = 0; rep < 3; rep++) batch_apply_pc<T, TZ>(B, 0, 0, all, st);
        (void)hipEventRecord(e1, st);
        float ms = 0.f;
        hipError_t he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            s = bfail(B, P4D_ERR_HIP, std::string("batch tile timing: ") + hipGetErrorString(he));
            break;
        }
        if (best == 0.f || ms < best) {
            best = ms;
            bcz = czs[q];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->tile_cz = bcz;
    B->recorded = 0;
    return s;
}

template <typename T, typename TZ>
static p4d_status batch_fgmres(p4d_batch *B, int transpose, const double *const *bv,
                               double *const *xv, const p4d_solve_opts &o, p4d_solve_info *infos,
                               hipStream_t st)
{
    const int n = B->n, m = o.restart;
    auto t0 = std::chrono::steady_clock::now();
    std::vector<BCell> bc;
    BatchGrid G;
    {
        const p4d_status ts = batch_tables(B, m, bv, xv, bc, G, st);
        if (ts != P4D_OK) return ts;
    }
    const int opb = G.op, stb = G.st;

    std::vector<CellRun> S(n);
    for (auto &R : S) {
        R.H.assign((size_t)(m + 1) * m, 0.0);
        R.cs.assign(m, 0.0); R.sn.assign(m, 0.0); R.gv.assign(m + 1, 0.0);
        R.yv.assign(m, 0.0); R.hc.assign(m + 2, 0.0); R.beta.assign(m + 1, 0.0);
    }
    const size_t hcopy = 8 * 256 * (size_t)n;
    if (B->pc_mode == 2 && B->pgrid < 1)
        return bfail(B, P4D_ERR_HIP, "this device runs no cooperative launch of the persistent kernel");
    B->plaunch = hipSuccess;
    auto fetch = [&]() -> p4d_status {
        BHIPCHK(B, hipMemcpyAsync(B->hb_h, B->hb, hcopy, hipMemcpyDeviceToHost, st));
        BHIPCHK(B, hipStreamSynchronize(st));
        prof_harvest(B->prof);
        BHIPCHK(B, B->plaunch);
        return P4D_OK;
    };
    auto sum_n = [&](unsigned long long mk, double per_cell_factor, bool stream_len) {
        double s = 0.0;
        for (int i = 0; i < n; i++)
            if ((mk >> i) & 1ULL) s += per_cell_factor * (stream_len ? (double)B->cell[i]->g.N : 1.0);
        return s;
    };
    const unsigned long long all = n == 64 ? ~0ULL : ((1ULL << n) - 1);
    p4d_status ps;
    // ||b||, x = 0, V_0 = b
    launch_bstart(B->bcell, n, stb, st);
    launch_bnorm_final(B->bcell, n, all, 0, 0, st);
    if ((ps = fetch()) != P4D_OK) return ps;
    for (int i = 0; i < n; i++) {
        CellRun &R = S[i];
        R.bnorm = B->hb_h[256 * i + 128];
        if (!std::isfinite(R.bnorm)) { R.status = P4D_ERR_NONFINITE; R.done = true; }
        else if (R.bnorm == 0.0) { R.status = P4D_OK; R.done = true; }
    }
    for (;;) {
        // true residual of the cells that finished a cycle: V_0 = b - A x
        unsigned long long rmask = 0;
        for (int i = 0; i < n; i++)
            if (!S[i].done && !S[i].first) rmask |= 1ULL << i;
        if (rmask) {
            {
                double bytes = 0.0;
                for (int i = 0; i < n; i++)
                    if ((rmask >> i) & 1ULL) {
                        const Geom &g = B->cell[i]->g;
                        bytes += 24.0 * g.N + 16.0 * g.nelem + 32.0 * g.ne;
                    }
                ProfScope pr(B->prof, P4D_K_OPERATOR, bytes, st);
                launch_bop<double>(B->bcell, n, rmask, 0, 1, transpose, opb, G.tile, G.rad, B->nrmax, st);
            }
            launch_bnorm_final(B->bcell, n, rmask, 0, 1, st);
            if ((ps = fetch()) != P4D_OK) return ps;
        }
        unsigned long long act = 0;
        for (int i = 0; i < n; i++) {
            CellRun &R = S[i];
            if (R.done) continue;
            const double beta0 = R.first ? R.bnorm : B->hb_h[256 * i + 128];
            R.first = false;
            R.inf.relres_true = beta0 / R.bnorm;
            if (R.breakdown) {
                R.status = R.inf.relres_true <= o.rtol ? P4D_OK : P4D_BREAKDOWN;
                R.done = true;
                continue;
            }
            if (!std::isfinite(beta0)) { R.status = P4D_ERR_NONFINITE; R.done = true; continue; }
            if (beta0 <= o.rtol * R.bnorm) { R.status = P4D_OK; R.done = true; continue; }
            if (R.total >= o.maxit) { R.status = P4D_NOT_CONVERGED; R.done = true; continue; }
            std::fill(R.gv.begin(), R.gv.end(), 0.0);
            R.gv[0] = beta0;
            R.beta[0] = beta0;
            R.kused = 0;
            R.in_cycle = true;
            act |= 1ULL << i;
        }
        if (!act) break;
        const unsigned long long cyc = act;
        for (int k = 0; k < m && act; k++) {
            {
                double bytes = 0.0;
                for (int i = 0; i < n; i++)
                    if ((act >> i) & 1ULL) bytes += B->pc_bytes[i];
                ProfScope pr(B->prof, P4D_K_BATCH_PC, bytes, st);
                if (B->pc_mode != 1) {
                    batch_apply_pc<T, TZ>(B, transpose, k, act, st);
                } else {
                    for (int i = 0; i < n; i++)
                        if ((act >> i) & 1ULL) {
                            p4d_ctx *c = B->cell[i];
                            apply_pc_t<T, TZ>(c, transpose, bc[i].V + (long long)k * c->g.N,
                                              bc[i].invbeta + k,
                                              (TZ *)bc[i].Z + (long long)k * c->g.N, st);
                        }
                }
            }
            {
                double bytes = 0.0;
                for (int i = 0; i < n; i++)
                    if ((act >> i) & 1ULL) {
                        const Geom &g = B->cell[i]->g;
                        bytes += (sizeof(TZ) + 8.0) * g.N + 16.0 * g.nelem + 32.0 * g.ne;
                    }
                ProfScope pr(B->prof, P4D_K_OPERATOR, bytes, st);
                launch_bop<TZ>(B->bcell, n, act, k, 0, transpose, opb, G.tile, G.rad, B->nrmax, st);
            }
            const int nv = k + 1;
            const int passes = o.cgs2 ? 2 : 1;
            for (int p = 0; p < passes; p++) {
                {
                    ProfScope pr(B->prof, P4D_K_MDOT, sum_n(act, 8.0 * (nv + 1), true), st);
                    launch_bmdot(B->bcell, n, act, k, stb, p, st);
                }
                ProfScope pr(B->prof, P4D_K_ORTH, sum_n(act, 8.0 * (nv + 2), true), st);
                launch_borth(B->bcell, n, act, k, stb, st);
            }
            launch_bnorm_final(B->bcell, n, act, k + 1, 0, st);
            if ((ps = fetch()) != P4D_OK) return ps;
            for (int i = 0; i < n; i++) {
                if (!((act >> i) & 1ULL)) continue;
                CellRun &R = S[i];
                const double *hh = B->hb_h + 256 * (size_t)i;
                std::vector<double> &hc = R.hc;
                for (int q = 0; q <= k; q++) hc[q] = hh[q] + (o.cgs2 ? hh[64 + q] : 0.0);
                const double hn = hh[128];
                hc[k + 1] = hn;
                double colnorm = 0.0;
                for (int q = 0; q <= k + 1; q++) colnorm += hc[q] * hc[q];
                colnorm = std::sqrt(colnorm);
                if (!std::isfinite(colnorm)) {
                    R.nonfinite = true;
                    act &= ~(1ULL << i);
                    continue;
                }
                for (int q = 0; q < k; q++) {
                    const double t = R.cs[q] * hc[q] + R.sn[q] * hc[q + 1];
                    hc[q + 1] = -R.sn[q] * hc[q] + R.cs[q] * hc[q + 1];
                    hc[q] = t;
                }
                const double den = std::sqrt(hc[k] * hc[k] + hc[k + 1] * hc[k + 1]);
                R.cs[k] = hc[k] / den;
                R.sn[k] = hc[k + 1] / den;
                hc[k] = den;
                R.gv[k + 1] = -R.sn[k] * R.gv[k];
                R.gv[k] = R.cs[k] * R.gv[k];
                for (int q = 0; q <= k; q++) R.H[(size_t)q * m + k] = hc[q];
                R.total++;
                R.kused = k + 1;
                R.beta[k + 1] = hn;
                R.inf.relres_est = std::fabs(R.gv[k + 1]) / R.bnorm;
                if (hn <= 1e-14 * colnorm) {
                    R.breakdown = true;
                    act &= ~(1ULL << i);
                } else if (std::fabs(R.gv[k + 1]) <= o.rtol * R.bnorm || R.total >= o.maxit) {
                    act &= ~(1ULL << i);
                }
            }
        }
        // x += Z y for the cells of this cycle
        unsigned long long zmask = 0;
        int kmax = 1;
        for (int i = 0; i < n; i++) {
            if (!((cyc >> i) & 1ULL)) continue;
            CellRun &R = S[i];
            R.in_cycle = false;
            if (R.nonfinite) {
                R.status = P4D_ERR_NONFINITE;
                R.done = true;
                continue;
            }
            const int ku = R.kused;
            for (int q = ku - 1; q >= 0; q--) {
                double v = R.gv[q];
                for (int j = q + 1; j < ku; j++) v -= R.H[(size_t)q * m + j] * R.yv[j];
                R.yv[q] = v / R.H[(size_t)q * m + q];
            }
            for (int q = 0; q < 64; q++) B->yb_h[64 * i + q] = q < ku ? R.yv[q] : 0.0;
            B->kused_h[i] = ku;
            kmax = ku > kmax ? ku : kmax;
            R.inf.restarts++;
            zmask |= 1ULL << i;
        }
        if (zmask) {
            // the previous copies from these staging buffers have completed:
            // every step synchronizes the stream
            BHIPCHK(B, hipMemcpyAsync(B->yb, B->yb_h, 8 * 64 * (size_t)n, hipMemcpyHostToDevice, st));
            BHIPCHK(B, hipMemcpyAsync(B->kused, B->kused_h, 4 * (size_t)n, hipMemcpyHostToDevice, st));
            double bytes = 0.0;
            for (int i = 0; i < n; i++)
                if ((zmask >> i) & 1ULL) bytes += (16.0 + sizeof(TZ) * S[i].kused) * B->cell[i]->g.N;
            ProfScope pr(B->prof, P4D_K_ZY, bytes, st);
            launch_bzy<TZ>(B->bcell, n, zmask, kmax, stb, st);
        }
    }
    BHIPCHK(B, hipGetLastError());
    BHIPCHK(B, hipStreamSynchronize(st));
    prof_harvest(B->prof);
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    p4d_status overall = P4D_OK;
    for (int i = 0; i < n; i++) {
        CellRun &R = S[i];
        R.inf.iters = R.total;
        R.inf.status = R.status;
        R.inf.t_solve_ms = ms;
        if (infos) infos[i] = R.inf;
        if (R.status != P4D_OK && overall == P4D_OK) overall = R.status;
    }
    if (overall != P4D_OK) B->err = std::string("a cell ended with: ") + p4d_status_string(overall);
    return overall;
}

extern "C" {

p4d_status p4d_autotune(p4d_ctx *c, void *stream, int32_t tile[2])
{
    if (!c) return P4D_ERR_INVALID_ARG;
    if (!c->pc_ready) return fail(c, P4D_ERR_STATE, "p4d_setup first");
    const p4d_status s = tune_tiles(c, (hipStream_t)stream);
    if (tile) {
        tile[0] = c->tile_tx;
        tile[1] = c->tile_cz;
    }
    return s;
}

p4d_status p4d_batch_create(const p4d_problem_desc *descs, int32_t ncells, p4d_batch **out)
{
    if (!descs || !out || ncells < 1 || ncells > kMaxBatch) return P4D_ERR_INVALID_ARG;
    *out = nullptr;
    for (int i = 0; i < ncells; i++)   // batches run the cube-element kernels
        if (descs[i].hxy[0] != 0.0 || descs[i].hxy[1] != 0.0) return P4D_ERR_INVALID_ARG;
    p4d_batch *B = new p4d_batch();
    B->n = ncells;
    for (int i = 0; i < ncells; i++) {
        p4d_ctx *c = nullptr;
        const p4d_status s = p4d_create(&descs[i], &c);
        if (s != P4D_OK) {
            for (p4d_ctx *q : B->cell) p4d_destroy(q);
            delete B;
            return s;
        }
        B->cell.push_back(c);
    }
    if (hipHostMalloc((void **)&B->hb_h, 8 * (256 * (size_t)ncells + 1), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&B->yb_h, 8 * 64 * (size_t)ncells, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&B->kused_h, 4 * (size_t)ncells, hipHostMallocDefault) != hipSuccess) {
        if (B->hb_h) hipHostFree(B->hb_h);
        if (B->yb_h) hipHostFree(B->yb_h);
        for (p4d_ctx *q : B->cell) p4d_destroy(q);
        delete B;
        return P4D_ERR_HIP;
    }
    prof_init(B->prof);
    p4d_default_opts(&B->ws_opts);
    *out = B;
    return P4D_OK;
}

void p4d_batch_destroy(p4d_batch *B)
{
    if (!B) return;
    for (p4d_ctx *c : B->cell) p4d_destroy(c);
    if (B->hb_h) hipHostFree(B->hb_h);
    if (B->yb_h) hipHostFree(B->yb_h);
    if (B->kused_h) hipHostFree(B->kused_h);
    prof_free(B->prof);
    delete B;
}

p4d_status p4d_batch_cell(p4d_batch *B, int32_t cell, p4d_ctx **out)
{
    if (!B || !out || cell < 0 || cell >= B->n) return P4D_ERR_INVALID_ARG;
    *out = B->cell[cell];
    return P4D_OK;
}

p4d_status p4d_batch_workspace_size(const p4d_batch *Bc, const p4d_solve_opts *opts, size_t *bytes)
{
    if (!Bc || !bytes) return P4D_ERR_INVALID_ARG;
    p4d_batch *B = const_cast<p4d_batch *>(Bc);
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return bfail(B, P4D_ERR_INVALID_ARG, why);
    p4d_status s;
    // sizing only: no pointer of the batch or its cells changes
    p4d_batch probe;
    probe.n = B->n;
    probe.cell = B->cell;
    *bytes = batch_carve(&probe, o, nullptr, &s) + kAlign;
    probe.cell.clear();
    return P4D_OK;
}

p4d_status p4d_batch_set_workspace(p4d_batch *B, void *d_work, size_t bytes, const p4d_solve_opts *opts)
{
    if (!B || !d_work) return P4D_ERR_INVALID_ARG;
    p4d_solve_opts o;
    p4d_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return bfail(B, P4D_ERR_INVALID_ARG, why);
    char *base = (char *)align_up((size_t)d_work);
    p4d_status s;
    p4d_batch probe;
    probe.n = B->n;
    probe.cell = B->cell;
    const size_t need = batch_carve(&probe, o, nullptr, &s);
    probe.cell.clear();
    if (need + (size_t)(base - (char *)d_work) > bytes)
        return bfail(B, P4D_ERR_OOM, "workspace too small for these options");
    B->ws = (char *)d_work;
    B->ws_bytes = bytes;
    B->ready = 0;
    B->recorded = 0;
    batch_carve(B, o, base, &s);
    if (s != P4D_OK) return s;
    B->ws_opts = o;
    B->ready = 1;
    return P4D_OK;
}

p4d_status p4d_batch_upload(p4d_batch *B, int32_t cell, const double *sigma, const double *kappa,
                            const double *g, const double *s, const double *e, void *stream)
{
    if (!B || cell < 0 || cell >= B->n) return P4D_ERR_INVALID_ARG;
    if (!B->ready) return bfail(B, P4D_ERR_STATE, "p4d_batch_set_workspace first");
    const p4d_status st = p4d_upload(B->cell[cell], sigma, kappa, g, s, e, stream);
    if (st != P4D_OK) B->err = "cell " + std::to_string(cell) + ": " + B->cell[cell]->err;
    B->recorded = 0;
    return st;
}

p4d_status p4d_batch_setup(p4d_batch *B, const p4d_solve_opts *opts, void *stream)
{
    if (!B) return P4D_ERR_INVALID_ARG;
    if (!B->ready) return bfail(B, P4D_ERR_STATE, "p4d_batch_set_workspace first");
    p4d_solve_opts o = B->ws_opts;
    if (opts) o = *opts;
    if (o.pc == P4D_PC_BGS)
        return bfail(B, P4D_ERR_INVALID_ARG, "block Gauss-Seidel is available for single cells only");
    if (o.pc_prec != B->ws_opts.pc_prec || o.coarse_max != B->ws_opts.coarse_max ||
        o.restart > B->ws_opts.restart || (!o.z_fp32 && B->ws_opts.z_fp32))
        return bfail(B, P4D_ERR_STATE, "options differ from those the workspace was carved for");
    B->recorded = 0;
    for (int i = 0; i < B->n; i++) {
        const p4d_status s = p4d_setup(B->cell[i], &o, stream);
        if (s != P4D_OK) return bfail(B, s, "cell " + std::to_string(i) + ": " + B->cell[i]->err);
    }
    return P4D_OK;
}

p4d_status p4d_batch_autotune(p4d_batch *B, void *stream, int32_t *tiles)
{
    if (!B) return P4D_ERR_INVALID_ARG;
    for (int i = 0; i < B->n; i++)
        if (!B->cell[i]->pc_ready) return bfail(B, P4D_ERR_STATE, "p4d_batch_setup first");
    const p4d_ctx *c0 = B->cell[0];
    const hipStream_t st = (hipStream_t)stream;
    p4d_status s;
    if (c0->prec) s = B->ws_opts.z_fp32 ? batch_tune_t<float, float>(B, st) : batch_tune_t<float, double>(B, st);
    else s = B->ws_opts.z_fp32 ? batch_tune_t<double, float>(B, st) : batch_tune_t<double, double>(B, st);
    if (s != P4D_OK) return s;
    if (tiles)
        for (int i = 0; i < B->n; i++) {
            tiles[2 * i] = B->cell[i]->tile_tx;
            tiles[2 * i + 1] = B->tile_cz;
        }
    return P4D_OK;
}

p4d_status p4d_batch_solve(p4d_batch *B, const double *const *d_b, double *const *d_x,
                           const p4d_solve_opts *opts, p4d_solve_info *infos, void *stream)
{
    if (!B || !d_b || !d_x) return P4D_ERR_INVALID_ARG;
    for (int i = 0; i < B->n; i++)
        if (!d_b[i] || !d_x[i] || d_b[i] == d_x[i]) return bfail(B, P4D_ERR_INVALID_ARG, "null or aliased vectors");
    if (!B->ready) return bfail(B, P4D_ERR_STATE, "p4d_batch_set_workspace first");
    p4d_ctx *c0 = B->cell[0];
    for (int i = 0; i < B->n; i++)
        if (!B->cell[i]->pc_ready) return bfail(B, P4D_ERR_STATE, "p4d_batch_setup first");
    p4d_solve_opts o = opts ? *opts : c0->pc;
    std::string why;
    if (!opts_valid(o, why)) return bfail(B, P4D_ERR_INVALID_ARG, why);
    if (o.krylov != P4D_KRYLOV_FULL)
        return bfail(B, P4D_ERR_INVALID_ARG, "the Schur-complement Krylov space is for single cells only");
    for (int i = 0; i < B->n; i++) {
        const p4d_ctx *c = B->cell[i];
        if (o.pc != c->pc.pc || o.pc_prec != c->pc.pc_prec || o.cheb_degree != c->pc.cheb_degree ||
            o.coarse_max != c->pc.coarse_max)
            return bfail(B, P4D_ERR_STATE, "preconditioner options differ from the last setup");
        if (o.restart > c->ws_opts.restart || (!o.z_fp32 && c->ws_opts.z_fp32))
            return bfail(B, P4D_ERR_OOM, "workspace sized for a smaller restart or an FP32 Z basis");
    }
    hipStream_t st = (hipStream_t)stream;
    if (!B->recorded || B->rec_prec != c0->prec) {
        const p4d_status s = c0->prec ? batch_record<float>(B) : batch_record<double>(B);
        if (s != P4D_OK) return s;
    }
    if (c0->prec) {
        if (o.z_fp32) return batch_fgmres<float, float>(B, 0, d_b, d_x, o, infos, st);
        return batch_fgmres<float, double>(B, 0, d_b, d_x, o, infos, st);
    }
    if (o.z_fp32) return batch_fgmres<double, float>(B, 0, d_b, d_x, o, infos, st);
    return batch_fgmres<double, double>(B, 0, d_b, d_x, o, infos, st);
}

p4d_status p4d_batch_set_pc_mode(p4d_batch *B, int32_t mode)
{
    if (!B || mode < 0 || mode > 2) return P4D_ERR_INVALID_ARG;
    B->pc_mode = mode;
    return P4D_OK;
}

p4d_status p4d_batch_profile(p4d_batch *B, int mask)
{
    if (!B || mask < 0 || mask >= (1 << P4D_K_COUNT)) return P4D_ERR_INVALID_ARG;
    prof_reset(B->prof, mask);
    return P4D_OK;
}

p4d_status p4d_batch_profile_read(p4d_batch *B, int cls, double *total_ms, int64_t *launches,
                                  double *bytes)
{
    if (!B || cls < 1 || cls >= P4D_K_COUNT) return P4D_ERR_INVALID_ARG;
    prof_harvest(B->prof);
    if (total_ms) *total_ms = B->prof.total_ms[cls];
    if (launches) *launches = B->prof.launches[cls];
    if (bytes) *bytes = B->prof.total_bytes[cls];
    return P4D_OK;
}

const char *p4d_batch_last_error(const p4d_batch *B) { return B ? B->err.c_str() : "null batch"; }

}  // extern "C"
