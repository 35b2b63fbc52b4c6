// Block-level device functions of the operator and the preconditioner.  The
// single-cell kernels (operator.hip, radial.hip, mg.hip) and the batched stage
// kernels (batch.hip, one launch per stage depth over work lists spanning all
// cells) call the same functions, each for one workgroup-sized unit of work
// given by an explicit block or tile index.
#pragma once
#include "p4d_device.hpp"

namespace p4d {

// ---------------------------------------------------------------------------
// 1D transfer helpers for 'even indices plus the last' coarsening of n points
// ---------------------------------------------------------------------------
__host__ __device__ inline int coarse_n(int n) { return n <= 2 ? n : n / 2 + 1; }

// coarse points (and weights) that fine point i interpolates from
__device__ inline int coarse_of(int n, int i, int I[2], double w[2])
{
    // (an unused second slot repeats the first point with weight 0)
    if (n <= 2) { I[0] = I[1] = i; w[0] = 1.0; w[1] = 0.0; return 1; }
    if (!(i & 1)) { I[0] = I[1] = i >> 1; w[0] = 1.0; w[1] = 0.0; return 1; }
    if (i == n - 1) { I[0] = I[1] = n / 2; w[0] = 1.0; w[1] = 0.0; return 1; }
    I[0] = (i - 1) >> 1; w[0] = 0.5;
    I[1] = (i + 1) >> 1; w[1] = 0.5;
    return 2;
}
// fine points (and weights) that interpolate from coarse point I, in the
// order: the coincident point, its odd left neighbour, its odd right
// neighbour; unused slots repeat the coincident point with weight 0
// (selects instead of a running index keep the arrays in registers)
__device__ inline int fine_of(int n, int I, int f[3], double w[3])
{
    if (n <= 2) {
        f[0] = f[1] = f[2] = I;
        w[0] = 1.0; w[1] = w[2] = 0.0;
        return 1;
    }
    const int nc = n / 2 + 1;
    const int c = (I == nc - 1) ? n - 1 : 2 * I;
    const bool lft = c - 1 >= 0 && ((c - 1) & 1) && c - 1 != n - 1;
    const bool rgt = c + 1 <= n - 1 && ((c + 1) & 1) && c + 1 != n - 1;
    f[0] = c; w[0] = 1.0;
    f[1] = lft ? c - 1 : (rgt ? c + 1 : c);
    w[1] = (lft || rgt) ? 0.5 : 0.0;
    f[2] = (lft && rgt) ? c + 1 : c;
    w[2] = (lft && rgt) ? 0.5 : 0.0;
    return 1 + (int)lft + (int)rgt;
}

template <typename B>
__device__ inline int find_box(const B &bt, int b)
{
    int q = 0;
#pragma unroll
    for (int t = 1; t < 4; t++)
        if (t < bt.nbox && b >= bt.a[t].blk0) q = t;
    return q;
}

// ---------------------------------------------------------------------------
// Level-0 smoother, 2.5D tiled.  A workgroup owns a TX x TY tile of an x-y
// plane and marches through a chunk of CZ node layers; three planes of x
// (with a one-node halo) and two layers of element coefficients sit in LDS
// rings, so every value is read from memory once per tile and the 27-point
// neighbourhood comes from LDS.  TX in {16, 32, 64}, TY = 256 / TX.
// ---------------------------------------------------------------------------
constexpr int kXpLds = 396;   // largest plane with halo: 66 x 6
constexpr int kCkLds = 325;   // largest element tile: 65 x 5
struct Smooth0Lds {
    double xp[3][kXpLds];
    double ck[2][kCkLds];
};

__host__ __device__ inline int smooth0_box_tiles(int nx, int ny, int nz, int TX, int CZ)
{
    const int TY = kBlock / TX;
    return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * ((nz + CZ - 1) / CZ);
}

// Q1 stiffness at a node: box-element weights g.kw in the general (GEN)
// instantiations, the cube stencil otherwise
template <bool GEN, typename R>
__device__ inline R stiff_of(const Geom &g, const R c[8], const R X[27])
{
    if (GEN) return q1_stiff_w(c, X, g.kw);
    return q1_stiff(c, X);
}

// The cube stencil as the level-0 smoother evaluates it.  The rows sum to
// zero, so the node's row is (4 x_i sum_e c_e - sum_e c_e F_e) / 12, with
// F_e the sum of x over the four corners of element e that differ from the
// node in at least two axes.  That is ~41 FP64 operations per node against
// ~72 for the difference form; the rounding differs by a few ulps of
// |x_i| sum_e c_e, which is far below what a smoothing step resolves.
template <typename R>
__device__ inline R q1_stiff_sum(const R c[8], const R X[27])
{
    R acc = R(0), cs = R(0);
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int a = (1 - ex) | ((1 - ey) << 1) | ((1 - ez) << 2);
        R far = R(0);
        bool first = true;
#pragma unroll
        for (int bb = 0; bb < 8; bb++) {
            if (popc3(a ^ bb) < 2) continue;
            const R v = X[nb_index(ex - 1 + (bb & 1), ey - 1 + ((bb >> 1) & 1), ez - 1 + ((bb >> 2) & 1))];
            far = first ? v : far + v;
            first = false;
        }
        acc = e == 0 ? c[e] * far : acc + c[e] * far;
        cs = e == 0 ? c[e] : cs + c[e];
    }
    return (R(4) * X[13] * cs - acc) * R(1.0 / 12.0);
}

// MEH: the storage of the mass box per element (g.meh) and the box-element
// stiffness weights (a separate instantiation keeps the per-material cube
// one free of their registers)
template <typename T, bool RESID_ONLY, bool MEH = false>
__device__ inline void smooth0_tile(const Geom &g, const LevelArgs<T> &A, int tile, int TX, int CZ,
                                    Smooth0Lds &L)
{
    const int TY = kBlock / TX;
    const int PX = TX + 2, PY = TY + 2;
    const int EX = TX + 1, EY = TY + 1;
    const int ntx = (A.nx + TX - 1) / TX, nty = (A.ny + TY - 1) / TY;
    const int tix = tile % ntx, tiy = (tile / ntx) % nty, tch = tile / (ntx * nty);
    const int i0 = tix * TX, j0 = tiy * TY, k0l = tch * CZ;
    const int k1l = k0l + CZ < A.nz ? k0l + CZ : A.nz;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < A.nx && j < A.ny;
    const int planeN = A.nx * A.ny;
    // elements on either side of the node in x and y (the box spans the
    // whole node plane)
    const bool inx0 = i > 0, inx1 = i < g.nx - 1, iny0 = j > 0, iny1 = j < g.ny - 1;

    // One plane of x with its halo (PX*PY <= 2*kBlock values) and one layer
    // of element coefficients (EX*EY <= 2*kBlock) per workgroup: each thread
    // holds at most two of each.  They are fetched into registers one layer
    // ahead and written to LDS after the layer that used the slot is done,
    // so the global loads overlap the arithmetic of the previous layer.
    double px[2], pc[2];
    auto fetch_plane_to = [&](int kl, double v[2]) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            const int ii = i0 - 1 + q % PX, jj = j0 - 1 + q / PX;
            const bool ok = q < PX * PY && kl >= 0 && kl < A.nz && ii >= 0 && ii < A.nx && jj >= 0 &&
                            jj < A.ny;
            v[h] = ok ? A.xin[ii + A.nx * (jj + A.ny * kl)] : 0.0;
        }
    };
    auto store_plane_from = [&](int slot, const double v[2]) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            if (q < PX * PY) L.xp[slot][q] = v[h];
        }
    };
    auto fetch_elems_to = [&](int kl, double v[2]) {
        const int ek = kl + A.k0;
        const bool lay = ek >= A.ek_lo && ek <= A.ek_hi;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            const int ei = i0 - 1 + q % EX, ej = j0 - 1 + q / EX;
            const bool ok = q < EX * EY && lay && ei >= 0 && ei < g.nx - 1 && ej >= 0 && ej < g.ny - 1;
            v[h] = ok ? A.cK[ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek)] : 0.0;
        }
    };
    auto store_elems_from = [&](int slot, const double v[2]) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            if (q < EX * EY) L.ck[slot][q] = v[h];
        }
    };
    auto fetch_plane = [&](int kl) { fetch_plane_to(kl, px); };
    auto store_plane = [&](int slot) { store_plane_from(slot, px); };
    auto fetch_elems = [&](int kl) { fetch_elems_to(kl, pc); };
    auto store_elems = [&](int slot) { store_elems_from(slot, pc); };
    // per-node data of a layer (right-hand side, reaction diagonal, inverse
    // diagonal, previous direction), also fetched one layer ahead
    double nb[4] = {0.0, 0.0, 0.0, 0.0};
    auto fetch_node = [&](int kl) {
        const int n = i + A.nx * j + planeN * kl;
        if (own) {
            nb[0] = (double)A.b[n];
            nb[1] = (double)A.dcorr[n];
            if (!RESID_ONLY) {
                nb[2] = (double)A.invd[n];
                if (A.c1 != 0.0 && !A.din_x) nb[3] = (double)A.din[n];
            }
        }
    };
    {   // prologue: every load of the first layer is issued before any of
        // them is stored, so the tile waits for one memory latency, not four
        double p0[2], p1[2], e0[2];
        fetch_plane_to(k0l - 1, p0);
        fetch_plane_to(k0l, p1);
        fetch_elems_to(k0l - 1, e0);
        fetch_plane(k0l + 1);
        fetch_elems(k0l);
        fetch_node(k0l);
        store_plane_from((k0l + 2) % 3, p0);
        store_plane_from(k0l % 3, p1);
        store_elems_from((k0l + 1) & 1, e0);
    }
    for (int kl = k0l; kl < k1l; kl++) {
        store_plane((kl + 1) % 3);
        store_elems(kl & 1);
        const int n = i + A.nx * j + planeN * kl;
        const double bn = nb[0], dcn = nb[1], idn = nb[2], dnn = nb[3];
        __syncthreads();
        if (kl + 1 < k1l) {
            fetch_plane(kl + 2);
            fetch_elems(kl + 1);
            fetch_node(kl + 1);
        }
        if (own) {
            double X[27];
#pragma unroll
            for (int dz = -1; dz <= 1; dz++) {
                const double *P = L.xp[(kl + dz + 3) % 3];
#pragma unroll
                for (int dy = -1; dy <= 1; dy++)
#pragma unroll
                    for (int dx = -1; dx <= 1; dx++)
                        X[nb_index(dx, dy, dz)] = P[(tx + 1 + dx) + PX * (ty + 1 + dy)];
            }
            double cK[8], cM[8];
            const int k = kl + A.k0;
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                cK[e] = L.ck[(kl - 1 + ez) & 1][(tx + ex) + EX * (ty + ey)];
                // storage of the elements inside the box, whatever their
                // stiffness coefficient (which may be zero)
                const int ek = k - 1 + ez;
                const bool in = A.mass && (ex ? inx1 : inx0) && (ey ? iny1 : iny0) &&
                                ek >= A.ek_lo && ek <= A.ek_hi;
                if (MEH) {
                    const int ei = i - 1 + ex, ej = j - 1 + ey;
                    cM[e] = in ? elem_storage(g, ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek), ek)
                               : 0.0;
                } else {
                    cM[e] = in ? (elem_mat(g, ek) >= 0 ? g.mass_elec : g.mass_sep) : 0.0;
                }
            }
            double Sx = (MEH ? q1_stiff_w(cK, X, g.kw) : q1_stiff_sum(cK, X)) + dcn * X[13];
            if (A.mass) Sx += q1_mass(cM, X);
            const double r = bn - Sx;
            if (RESID_ONLY) {
                A.rout[n] = (T)r;
            } else {
                double d = A.c2 * idn * r;
                if (A.c1 != 0.0) d += A.c1 * (A.din_x ? X[13] : dnn);
                A.xout[n] = X[13] + d;
                if (A.dout) A.dout[n] = (T)d;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Levels >= 1: Galerkin stencil of a symmetric operator, stored by its upper
// half in difference form: slot 0 holds the row sum, slot 1 + u the coupling
// to the neighbour at stencil offset 14 + u; the coupling to a neighbour at
// a lower offset o is that neighbour's coupling at offset 26 - o.
//   S x = rowsum x_i + sum_{j != i} s_ij (x_j - x_i)
// ---------------------------------------------------------------------------
template <typename T, bool RESID_ONLY>
__device__ inline void smooth_block(const LevelArgs<T> &A, int blk)
{
    const int n = blk * kBlock + threadIdx.x;
    if (n >= A.n) return;
    const int i = n % A.nx, t = n / A.nx;
    const int j = t % A.ny, kl = t / A.ny;
    // all coefficients and neighbours are loaded before any arithmetic (a
    // missing neighbour's index is clamped to the node, its term skipped),
    // so the loads are in flight together
    T sv[27];
    double xv[27];
    bool okv[27];
#pragma unroll
    for (int o = 0; o < 27; o++) {
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        okv[o] = (i + dx >= 0) && (i + dx < A.nx) && (j + dy >= 0) && (j + dy < A.ny) &&
                 (kl + dz >= 0) && (kl + dz < A.nz);
        const int nbr = okv[o] ? n + dx + A.nx * (dy + A.ny * dz) : n;
        xv[o] = A.xin[nbr];
        if (o > 13) sv[o] = A.S[(long long)(o - 13) * A.n + n];
        else if (o < 13) sv[o] = A.S[(long long)(13 - o) * A.n + nbr];
        else sv[o] = A.S[n];
    }
    const double xc = xv[13];
    double Sx = (double)sv[13] * xc;
#pragma unroll
    for (int o = 0; o < 27; o++) {
        if (o == 13) continue;
        if (okv[o]) Sx += (double)sv[o] * (xv[o] - xc);
    }
    const double r = (double)A.b[n] - Sx;
    if (RESID_ONLY) {
        A.rout[n] = (T)r;
        return;
    }
    double d = A.c2 * (double)A.invd[n] * r;
    if (A.c1 != 0.0) d += A.c1 * (A.din_x ? xc : (double)A.din[n]);
    A.xout[n] = xc + d;
    if (A.dout) A.dout[n] = (T)d;
}

// b_c = P^T r_f; also the first Chebyshev iterate x_c1 = c2 D_c^-1 b_c
template <typename T>
__device__ inline void restrict_block(const TransferArgs<T> &A, int blk)
{
    const int nc = A.cx * A.cy * A.cz;
    const int n = blk * kBlock + threadIdx.x;
    if (n >= nc) return;
    const int I = n % A.cx, t = n / A.cx;
    const int J = t % A.cy, K = t / A.cy;
    int fi[3], fj[3], fk[3];
    double wi[3], wj[3], wk[3];
    const int ni = fine_of(A.fx, I, fi, wi);
    const int nj = fine_of(A.fy, J, fj, wj);
    const int nk = fine_of(A.cz == A.fz ? 1 : A.fz, K, fk, wk);   // (z kept: identity)
    (void)ni; (void)nj; (void)nk;
    // issued with the residual loads (after the store below it would wait
    // for them first)
    const double idc = A.xc1 ? (double)A.invdc[n] : 0.0;
    // all 27 slots, without tests: an unused slot reads a point that a used
    // slot reads too and adds an exact zero to a sum that starts at +0 (and
    // so never holds -0), leaving it as it is bit for bit; unguarded, the
    // loads are all in flight at once
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
#pragma unroll
        for (int bq = 0; bq < 3; bq++) {
            const long long row = (long long)A.fx * (fj[bq] + (long long)A.fy * fk[c]);
            double part = 0.0;
#pragma unroll
            for (int a = 0; a < 3; a++) part += wi[a] * (double)A.rf[row + fi[a]];
            acc += wj[bq] * wk[c] * part;
        }
    }
    const T bc = (T)acc;
    A.bc[n] = bc;
    if (A.xc1) A.xc1[n] = A.c2c * idc * (double)bc;
}

// x_f += P x_c
template <typename T>
__device__ inline void prolong_block(const TransferArgs<T> &A, int blk)
{
    const int nf = A.fx * A.fy * A.fz;
    const int n = blk * kBlock + threadIdx.x;
    if (n >= nf) return;
    const int i = n % A.fx, t = n / A.fx;
    const int j = t % A.fy, k = t / A.fy;
    int Ci[2], Cj[2], Ck[2];
    double wi[2], wj[2], wk[2];
    const int ni = coarse_of(A.fx, i, Ci, wi);
    const int nj = coarse_of(A.fy, j, Cj, wj);
    const int nk = coarse_of(A.cz == A.fz ? 1 : A.fz, k, Ck, wk);
    (void)ni; (void)nj; (void)nk;
    // all 8 slots, without tests (an unused slot adds an exact zero; see
    // restrict_block)
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int bq = 0; bq < 2; bq++) {
            const long long row = (long long)A.cx * (Cj[bq] + (long long)A.cy * Ck[c]);
            double part = 0.0;
#pragma unroll
            for (int a = 0; a < 2; a++) part += wi[a] * A.xc[row + Ci[a]];
            acc += wj[bq] * wk[c] * part;
        }
    }
    A.xf[n] += acc;
}

// Coarsest level, 64 rows of x = A^-1 b per workgroup (FP64); the 4 waves
// split the columns, then add up.
struct CoarseLds {
    double bl[1024];
    double part[4][64];
};
template <typename T>
__device__ inline void coarse_block(const CoarseArgs<T> &A, int rowblk, CoarseLds &L)
{
    const int n = A.n;
    for (int q = threadIdx.x; q < n; q += kBlock) L.bl[q] = (double)A.b[q];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = rowblk * 64 + lane;
    double acc = 0.0;
    if (row < n) {
#pragma unroll 4
        for (int c = w; c < n; c += 4) acc += A.Ainv[(long long)c * n + row] * L.bl[c];
    }
    L.part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < n)
        A.x[row] = (L.part[0][lane] + L.part[1][lane]) + (L.part[2][lane] + L.part[3][lane]);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Particle blocks (Sec. 4.2: one tridiagonal system per point, inverted
// exactly).  A_ss,j = T0 + Gamma s_j e_N e_N^T shares the LU of T0; only the
// last pivot depends on the node.
// ---------------------------------------------------------------------------
// A radial table read through the constant address space: loads from a
// wave-uniform address become scalar loads (the tables do not change while
// a kernel runs)
typedef __attribute__((address_space(4))) const RadialTab ConstTab;

struct RadArgs {
    const RadialTab *tabs;
    const double *gg, *ss, *ee, *mm, *om;
    void *b0;            // T, macro layout
    double *x1;          // first Chebyshev iterate of each box
    const void *invd0;   // T
    double c2box[4];
    const double *x0[4]; // final level-0 iterates per box (rad_back)
};

// zeta_j = (A_ss,j^-1 r_s,j)_N; r~_y = r_y - a_y s_j zeta_j (transposed:
// r_y - Gamma b_y zeta_j); written in precision T with the first Chebyshev
// iterate of each box.
template <typename T, int NRMAX, bool TRANS, bool SCHUR>
__device__ inline void rad_fwd_block(const Geom &g, const RadArgs &R, const double *r, double rscale,
                                     int blk)
{
    const long long n = (long long)blk * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    T *b0 = (T *)R.b0;
    const T *invd0 = (const T *)R.invd0;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    double rpe = r[g.off_pe + n] * rscale;
    double rce = r[g.off_ce + n] * rscale;
    // every load is issued before the first store (a load after a store of
    // a computed value would wait for that computation's loads first)
    const double idpe = (double)invd0[g.off_pe + n], idce = (double)invd0[g.off_ce + n];
    const int el = node_mat(g, k);
    if (el >= 0) {
        const long long base = el == 0 ? 0 : g.nea;
        const long long klo = el == 0 ? 0 : g.na + g.ns;
        const long long je = base + n - klo * g.nx * g.ny;
        const bool dir = (k == 0);
        double rps = r[je] * rscale;
        const double idps = dir ? 0.0 : (double)invd0[je];
        if (SCHUR) {
            auto elim = [&](const auto &Tb) {
                const int N = Tb.N;
                const long long nn = el == 0 ? g.nea : g.nec;
                const double *rs = r + (el == 0 ? g.off_cs[0] : g.off_cs[1]) + (je - base);
                // all radial values first (indices clamped to the last point), so
                // the loads are in flight together
                double rv[NRMAX];
#pragma unroll
                for (int q = 0; q < NRMAX; q++) rv[q] = rs[(long long)(q < N ? q : N - 1) * nn];
                T y = (T)(rv[0] * rscale);
#pragma unroll
                for (int q = 1; q < NRMAX; q++) {
                    if (q < N) {
                        const T lq = (T)(TRANS ? Tb.lT[q] : Tb.l[q]);
                        y = (T)(rv[q] * rscale) - lq * y;
                    }
                }
                const double sj = R.ss[je];
                const T pivN = (T)(Tb.piv[N - 1] + Tb.Gamma * sj);
                const double zeta = (double)(y / pivN);
                const double m = R.mm[je];
                if (!TRANS) {   // a_y s_j zeta, a_y = (m, -m, -tc m)
                    const double f = sj * zeta;
                    if (!dir) rps -= m * f;
                    rpe += m * f;
                    rce += g.tc * m * f;
                } else {        // Gamma b_y zeta, b_y = (g, -g, e)
                    const double f = Tb.Gamma * zeta;
                    const double gj = R.gg[je];
                    if (!dir) rps -= gj * f;
                    rpe += gj * f;
                    rce -= R.ee[je] * f;
                }
            };
            // the tables of the node's electrode: through a wave-uniform pointer
            // in the constant address space (scalar loads) when the whole wave
            // lies in one electrode, per lane otherwise
            const int elw = __builtin_amdgcn_readfirstlane(el);
            if (__builtin_amdgcn_ballot_w64(el != elw) == 0) elim(*(const ConstTab *)(R.tabs + elw));
            else elim(R.tabs[el]);
        }
        const T bps = (T)rps;
        b0[je] = bps;
        if (!dir) R.x1[je] = (el == 0 ? R.c2box[0] : R.c2box[1]) * idps * (double)bps;
    }
    const T bpe = (T)rpe, bce = (T)rce;
    b0[g.off_pe + n] = bpe;
    b0[g.off_ce + n] = bce;
    R.x1[g.off_pe + n] = R.c2box[2] * idpe * (double)bpe;
    R.x1[g.off_ce + n] = R.c2box[3] * idce * (double)bce;
}

// z_s,j = A_ss,j^-1 r_s,j - delta_j A_ss,j^-1 e_N, and by Sherman-Morrison
// A_ss,j^-1 e_N = omega_j T0^-1 e_N: the elimination in precision T only
// sees r_s, while delta_j = Gamma b_y . z_y (transposed s_j a_y . z_y),
// which carries the large near-null part of z_y, is applied in FP64.
template <typename T, typename TZ, int NRMAX, bool TRANS, bool SCHUR>
__device__ inline void rad_back_block(const Geom &g, const RadArgs &R, const double *r, double rscale,
                                      TZ *z, int blk)
{
    const long long n = (long long)blk * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const int el = node_mat(g, k);
    const double zpe = R.x0[2][g.off_pe + n];
    const double zce = R.x0[3][g.off_ce + n];
    if (el < 0) {
        z[g.off_pe + n] = (TZ)zpe;
        z[g.off_ce + n] = (TZ)zce;
        return;
    }
    const long long base = el == 0 ? 0 : g.nea;
    const long long klo = el == 0 ? 0 : g.na + g.ns;
    const long long je = base + n - klo * g.nx * g.ny;
    const bool dir = (k == 0);
    const double zps = dir ? r[je] * rscale : (el == 0 ? R.x0[0] : R.x0[1])[je];
    auto solve = [&](const auto &Tb) {
        const int N = Tb.N;
        const long long nn = el == 0 ? g.nea : g.nec;
        const double *rs = r + (el == 0 ? g.off_cs[0] : g.off_cs[1]) + (je - base);
        TZ *zs = z + (el == 0 ? g.off_cs[0] : g.off_cs[1]) + (je - base);
        const double sj = R.ss[je];
        double dw = 0.0;   // delta_j * omega_j
        if (SCHUR) {
            const double m = R.mm[je];
            double delta;
            if (!TRANS)
                delta = Tb.Gamma * ((dir ? 0.0 : R.gg[je]) * zps - R.gg[je] * zpe + R.ee[je] * zce);
            else
                delta = sj * ((dir ? 0.0 : m) * zps - m * zpe - g.tc * m * zce);
            dw = delta * R.om[je];
        }
        // forward elimination; the register arrays are only indexed by unrolled
        // constants, the last entry is carried separately; all radial values are
        // loaded first (indices clamped to the last point)
        double rv[NRMAX];
#pragma unroll
        for (int q = 0; q < NRMAX; q++) rv[q] = rs[(long long)(q < N ? q : N - 1) * nn];
        // the electrode-level outputs are stored only now, after every load is
        // issued (a load after them would wait for the loads they depend on)
        z[g.off_pe + n] = (TZ)zpe;
        z[g.off_ce + n] = (TZ)zce;
        z[je] = (TZ)zps;
        T y[NRMAX];
        y[0] = (T)(rv[0] * rscale);
        T ylast = y[0];
#pragma unroll
        for (int q = 1; q < NRMAX; q++) {
            if (q < N) {
                const T lq = (T)(TRANS ? Tb.lT[q] : Tb.l[q]);
                y[q] = (T)(rv[q] * rscale) - lq * y[q - 1];
                ylast = y[q];
            }
        }
        T zn = ylast / (T)(Tb.piv[N - 1] + Tb.Gamma * sj);
        zs[(long long)(N - 1) * nn] = (TZ)((double)zn - dw * (TRANS ? Tb.tNT[N - 1] : Tb.tN[N - 1]));
#pragma unroll
        for (int q = NRMAX - 2; q >= 0; q--) {
            if (q < N - 1) {
                const T u = (T)(TRANS ? Tb.tsub[q + 1] : Tb.tsup[q]);
                zn = (y[q] - u * zn) * (T)Tb.ipiv[q];
                zs[(long long)q * nn] = (TZ)((double)zn - dw * (TRANS ? Tb.tNT[q] : Tb.tN[q]));
            }
        }
    };
    // the tables of the node's electrode: through a wave-uniform pointer in the
    // constant address space (scalar loads) when the whole wave lies in one
    // electrode, per lane otherwise
    const int elw = __builtin_amdgcn_readfirstlane(el);
    if (__builtin_amdgcn_ballot_w64(el != elw) == 0) solve(*(const ConstTab *)(R.tabs + elw));
    else solve(R.tabs[el]);
}

// ---------------------------------------------------------------------------
// The operator y = A x (or A^T x, or b - A x) for the nodes of one block,
// with the sum of squares of what the thread writes (paper Sec. 4.1,
// eq. blocks; see operator.hip).
// ---------------------------------------------------------------------------
struct OpArgs {
    const RadialTab *tabs;
    const double *sigh, *kaph, *gg, *ss, *ee, *mm;
    const void *x;       // TX
    double *y;
    const double *b;     // b - A x when not null
    const double *om;    // omega per electrode node (Schur complement operator)
    const double *kdh;   // h * diffusion-potential coefficient per element (GEN)
    const double *dch;   // h * c_e diffusion coefficient per element (GEN)
};

template <typename TX>
__device__ inline double ldx(const TX *p) { return (double)*p; }

template <typename TX>
__device__ inline void load_nb(const Geom &g, const TX *f, long long n, int i, int j, int k,
                               double X[27])
{
#pragma unroll
    for (int o = 0; o < 27; o++) {
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const bool ok = (i + dx >= 0) && (i + dx < g.nx) && (j + dy >= 0) && (j + dy < g.ny) &&
                        (k + dz >= 0) && (k + dz < g.nz);
        X[o] = ok ? ldx(f + n + dx + (long long)g.nx * (dy + (long long)g.ny * dz)) : 0.0;
    }
}

// Stencil parts of the operator at one node, gathered either per node from
// memory or from an LDS tile: K_kappa phi_e, K_kappa c_e, M_eps c_e and, on
// electrode nodes, K_sigma phi_s, with the centre values (xpsc is phi_s as a
// neighbour value: zero on the grounded layer).
struct OpStencil {
    double Kpe, xpe, Kce, Mce, xce, Kps, xpsc;
    double Kx;   // GEN: the diffusion-potential stiffness applied to c_e (phi_e if transposed)
    double Npe = 0.0, Nce = 0.0;   // GEN: Newton terms of the phi_e and c_e rows
};

// Newton terms at one node (GEN, g.nwu set): each element e of the node
// has coefficients that depend on its mean c_e, so it adds to its corner
// rows (K_e u)_a times the mean of x_ce over its corners, with K_e the
// element stiffness (over h) and u the state: phi_e rows da_e (K_e phi_e) +
// db_e (K_e c_e), c_e rows dc_e (K_e c_e).  Transposed, the node (a c_e
// column) collects w_e^T (...) / 8 from each of its elements, w the input's
// phi_e and c_e on the element's corners.  Xc: the input's c_e around the
// node (the forward form).  (K_e u)_a = sum_{b != a} kw[a^b] (u_a - u_b).
template <typename TX, bool TRANS>
__device__ inline void newton_terms(const Geom &g, const TX *x, long long n, int i, int j, int k,
                                    const double Xc[27], OpStencil &P)
{
    const double *up = g.nwu + g.off_pe, *uc = g.nwu + g.off_ce;
    const long long layer = (long long)g.nx * g.ny;
    double npe = 0.0, nce = 0.0;
    for (int e = 0; e < 8; e++) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
        if (ei < 0 || ej < 0 || ek < 0 || ei >= g.nx - 1 || ej >= g.ny - 1 || ek >= g.nz - 1) continue;
        const long long id = ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek);
        // corner b of the element is node n + off(b); this node is corner a
        const long long c0 = ei + (long long)g.nx * ej + layer * ek;
        auto node = [&](int b) { return c0 + (b & 1) + (long long)g.nx * ((b >> 1) & 1) + layer * ((b >> 2) & 1); };
        const double A = g.nwa[id], B = g.nwb[id], C = g.nwc[id];
        if (!TRANS) {
            const int a = (1 - ex) | ((1 - ey) << 1) | ((1 - ez) << 2);
            double sp = 0.0, sc = 0.0, xm = 0.0;
            const double upa = up[n], uca = uc[n];
            for (int b = 0; b < 8; b++) {
                xm += Xc[nb_index(ex - 1 + (b & 1), ey - 1 + ((b >> 1) & 1), ez - 1 + ((b >> 2) & 1))];
                if (b == a) continue;
                const long long nb = node(b);
                const double w = g.kw[a ^ b];
                sp += w * (upa - up[nb]);
                sc += w * (uca - uc[nb]);
            }
            xm *= 0.125;
            npe += (A * sp + B * sc) * xm;
            nce += C * sc * xm;
        } else {
            double t = 0.0;
            for (int a = 0; a < 8; a++) {
                const long long na = node(a);
                double kup = 0.0, kuc = 0.0;
                for (int b = 0; b < 8; b++) {
                    if (b == a) continue;
                    const long long nb = node(b);
                    const double w = g.kw[a ^ b];
                    kup += w * (up[na] - up[nb]);
                    kuc += w * (uc[na] - uc[nb]);
                }
                t += ldx(x + g.off_pe + na) * (A * kup + B * kuc) + ldx(x + g.off_ce + na) * C * kuc;
            }
            nce += 0.125 * t;
        }
    }
    P.Npe = npe;
    P.Nce = nce;
}

// Reaction coupling of one electrode node: the linearized reaction q and the
// weights with which it enters the phi_s, phi_e, c_e and surface c_s rows
// (a = (m, -m, -tc m, Gamma), b = (g, -g, e, s); transposed: a and b swap).
struct OpCoupling {
    double q, r0, r1, r2, r3;
};
template <bool TRANS, typename Tab>
__device__ inline OpCoupling op_coupling(const Geom &g, const Tab &T, bool dir, double m,
                                         double gj, double sj, double ej, double xpsc, double xpe,
                                         double xce, double xsN)
{
    OpCoupling c;
    const double a0 = dir ? 0.0 : m, b0 = dir ? 0.0 : gj;
    if (!TRANS) {
        c.q = b0 * xpsc - gj * xpe + ej * xce + sj * xsN;
        c.r0 = a0; c.r1 = -m; c.r2 = -g.tc * m; c.r3 = T.Gamma;
    } else {
        c.q = a0 * xpsc - m * xpe - g.tc * m * xce + T.Gamma * xsN;
        c.r0 = b0; c.r1 = -gj; c.r2 = ej; c.r3 = sj;
    }
    return c;
}

// Row r of T0 (or T0^T) applied to a particle column, without the coupling
template <typename Tab>
__device__ inline double op_radial_row(const Tab &T, bool trans, int r, int N, double xm, double x0,
                                       double xp)
{
    if (!trans) return T.tdia[r] * x0 + T.tsub[r] * xm + T.tsup[r] * xp;
    return T.tdia[r] * x0 + (r > 0 ? T.tsup[r > 0 ? r - 1 : 0] : 0.0) * xm +
           (r < N - 1 ? T.tsub[r + 1 < kMaxNr ? r + 1 : r] : 0.0) * xp;
}

// Everything after the stencil parts: reaction coupling, radial rows and
// the output (y, or b - A x when RESID); returns the sum of squares written.
// GEN: separate element coefficients for the diffusion-potential block
// (P.Kx) and the c_e diffusion (P.Kce), instead of chi * kappa and kappa.
// RED: the Schur complement of the particle blocks (see operator_tile): the
// reaction enters scaled by omega_j, no particle column (x, y hold the
// electrode-level unknowns only)
template <typename TX, int NRMAX, bool TRANS, bool RESID, bool GEN = false, bool RED = false>
__device__ inline double operator_finish(const Geom &g, const OpArgs &O, long long n, int i, int j,
                                         int k, const OpStencil &P)
{
    const TX *x = (const TX *)O.x;
    double *y = O.y;
    const double *b = O.b;
    double sq = 0.0;
    const double xpe = P.xpe, xce = P.xce;
    // b - A x: every value of b this node needs is loaded before its first
    // store (a load after a store may not be hoisted above it, pointers may
    // alias, and would wait for the loads the stored value depends on)
    double bpe = 0.0, bce = 0.0;
    if (RESID) {
        bpe = b[g.off_pe + n];
        bce = b[g.off_ce + n];
    }
    double ype, yce;
    if (GEN) {
        ype = (TRANS ? P.Kpe : P.Kpe + P.Kx) + P.Npe;
        yce = (TRANS ? P.Mce + P.Kce + P.Kx : P.Mce + P.Kce) + P.Nce;
    } else if (!TRANS) {
        ype = P.Kpe + g.chi * P.Kce;
        yce = P.Mce + P.Kce;
    } else {
        ype = P.Kpe;
        yce = P.Mce + P.Kce + g.chi * P.Kpe;
    }
    const int el = node_mat(g, k);
    if (el >= 0) {
        const long long base = el == 0 ? 0 : g.nea;
        const int klo = el == 0 ? 0 : g.na + g.ns;
        const long long je = base + i + (long long)g.nx * (j + (long long)g.ny * (k - klo));
        const bool dir = (k == 0);
        const double xps = ldx(x + je);
        auto rows = [&](const auto &T) {
            const int N = T.N;
            const long long nn = el == 0 ? g.nea : g.nec;
            const long long jl = je - base;
            const long long offs = el == 0 ? g.off_cs[0] : g.off_cs[1];
            const TX *xs = x + offs + jl;
            double *ys = y + offs + jl;
            const double m = O.mm[je], gj = O.gg[je], sj = O.ss[je], ej = O.ee[je];
            // the particle column, loaded at once (indices clamped to the last point)
            double xr[NRMAX], bv[NRMAX];
            double xsN = 0.0, bps = 0.0;
            if (!RED) {
#pragma unroll
                for (int r = 0; r < NRMAX; r++) xr[r] = ldx(xs + (long long)(r < N ? r : N - 1) * nn);
                if (RESID) {
#pragma unroll
                    for (int r = 0; r < NRMAX; r++) bv[r] = b[offs + jl + (long long)(r < N ? r : N - 1) * nn];
                }
                xsN = xr[0];
#pragma unroll
                for (int r = 1; r < NRMAX; r++)
                    if (r == N - 1) xsN = xr[r];
            }
            if (RESID) bps = b[je];
            const OpCoupling cp = op_coupling<TRANS>(g, T, dir, m, gj, sj, ej, P.xpsc, xpe, xce, xsN);
            const double q = RED ? cp.q * O.om[je] : cp.q, r3 = cp.r3;
            double yps = dir ? xps : P.Kps + cp.r0 * q;
            ype += cp.r1 * q;
            yce += cp.r2 * q;
            if (RESID) yps = bps - yps;
            y[je] = yps;
            sq += yps * yps;
#pragma unroll
            for (int r = 0; r < NRMAX; r++) {
                if (RED) break;
                if (r < N) {
                    const double xm = r > 0 ? xr[r > 0 ? r - 1 : 0] : 0.0;
                    const double x0 = xr[r];
                    const double xp = r < N - 1 ? xr[r + 1 < NRMAX ? r + 1 : r] : 0.0;
                    double v = op_radial_row(T, TRANS, r, N, xm, x0, xp);
                    if (r == N - 1) v += r3 * q;
                    if (RESID) v = bv[r] - v;
                    ys[(long long)r * nn] = v;
                    sq += v * v;
                }
            }
        };
        // the electrode's table through a wave-uniform pointer (scalar loads)
        // when the whole wave lies in one electrode, per lane otherwise
        const int elw = __builtin_amdgcn_readfirstlane(el);
        if (__builtin_amdgcn_ballot_w64(el != elw) == 0) rows(*(const ConstTab *)(O.tabs + elw));
        else rows(O.tabs[el]);
    }
    if (RESID) {
        ype = bpe - ype;
        yce = bce - yce;
    }
    y[g.off_pe + n] = ype;
    y[g.off_ce + n] = yce;
    sq += ype * ype + yce * yce;
    return sq;
}

// The operator y = A x (or A^T x, or b - A x) at one node, every stencil
// value read from memory (paper Sec. 4.1, eq. blocks; see operator.hip).
template <typename TX, int NRMAX, bool TRANS, bool RESID, bool GEN = false, bool RED = false>
__device__ inline double operator_node(const Geom &g, const OpArgs &O, long long n)
{
    const TX *x = (const TX *)O.x;
    const int i = (int)(n % g.nx);
    const long long t = n / g.nx;
    const int j = (int)(t % g.ny), k = (int)(t / g.ny);
    // element coefficients of the node's eight elements; each set is read
    // beside the neighbourhood that uses it, so only one set is live at a time
    auto elem_of = [&](const double *C, double c[8]) {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + ((e >> 2) & 1);
            const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < g.nx - 1 && ej < g.ny - 1 &&
                            ek < g.nz - 1;
            c[e] = ok ? C[ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek)] : 0.0;
        }
    };
    double ck[8], cs[8], cm[8];
    elem_of(O.kaph, ck);
    OpStencil P;
    double X[27];
    P.Kx = 0.0;
    load_nb(g, x + g.off_pe, n, i, j, k, X);
    P.Kpe = stiff_of<GEN>(g, ck, X);
    P.xpe = X[13];
    if (GEN && TRANS) {
        double cx[8];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + ((e >> 2) & 1);
            const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < g.nx - 1 && ej < g.ny - 1 &&
                            ek < g.nz - 1;
            cx[e] = ok ? O.kdh[ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek)] : 0.0;
        }
        P.Kx = stiff_of<GEN>(g, cx, X);
    }
    // an empty statement that takes the finished sums: they may not be
    // deferred past it nor the next neighbourhood's loads hoisted above it,
    // so one 27-value neighbourhood is live at a time (register use)
    __asm__ volatile("" : "+v"(P.Kpe), "+v"(P.Kx) : : "memory");
    load_nb(g, x + g.off_ce, n, i, j, k, X);
    if (GEN) {
        double cd[8], cx[8];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + ((e >> 2) & 1);
            const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < g.nx - 1 && ej < g.ny - 1 &&
                            ek < g.nz - 1;
            const long long id = ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek);
            cd[e] = ok ? O.dch[id] : 0.0;
            cx[e] = (ok && !TRANS) ? O.kdh[id] : 0.0;
        }
        P.Kce = stiff_of<GEN>(g, cd, X);
        if (!TRANS) P.Kx = stiff_of<GEN>(g, cx, X);
    } else {
        P.Kce = stiff_of<GEN>(g, ck, X);
    }
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + ((e >> 2) & 1);
        const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < g.nx - 1 && ej < g.ny - 1 &&
                        ek < g.nz - 1;
        const long long id = ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek);
        // per-element storage only with separate coefficients (GEN)
        cm[e] = ok ? (GEN ? elem_storage(g, id, ek) : (elem_mat(g, ek) >= 0 ? g.mass_elec : g.mass_sep))
                   : 0.0;
    }
    P.Mce = q1_mass(cm, X);
    P.xce = X[13];
    if (GEN && g.nwu) newton_terms<TX, TRANS>(g, x, n, i, j, k, X, P);
    __asm__ volatile("" : "+v"(P.Kce), "+v"(P.Mce), "+v"(P.Kx), "+v"(P.Npe), "+v"(P.Nce) : : "memory");
    P.Kps = 0.0;
    P.xpsc = 0.0;
    const int el = node_mat(g, k);
    if (el >= 0) {
        elem_of(O.sigh, cs);
        const long long base = el == 0 ? 0 : g.nea;
        const int klo = el == 0 ? 0 : g.na + g.ns;
        const int khi = el == 0 ? g.na - 1 : g.nz - 1;
        const long long je = base + i + (long long)g.nx * (j + (long long)g.ny * (k - klo));
        // phi_s neighbours: same electrode, grounded layer as a zero column
#pragma unroll
        for (int o = 0; o < 27; o++) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            const bool ok = (i + dx >= 0) && (i + dx < g.nx) && (j + dy >= 0) && (j + dy < g.ny) &&
                            (k + dz >= klo) && (k + dz <= khi) && (k + dz != 0);
            X[o] = ok ? ldx(x + je + dx + (long long)g.nx * (dy + (long long)g.ny * dz)) : 0.0;
        }
        P.Kps = stiff_of<GEN>(g, cs, X);
        P.xpsc = X[13];
    }
    return operator_finish<TX, NRMAX, TRANS, RESID, GEN, RED>(g, O, n, i, j, k, P);
}

// ---------------------------------------------------------------------------
// The operator over a 2.5D tile (the level-0 smoother's scheme): a TX x TY
// block of nodes marches through CZ node layers; three planes of phi_e, c_e
// and phi_s with a one-node halo and two layers of element coefficients sit
// in LDS rings, fetched into registers one layer ahead.  Each node's
// arithmetic is operator_finish on the same stencil values as operator_node,
// so both give the same result.
// ---------------------------------------------------------------------------
struct OpLds {
    double pe[3][kXpLds], ce[3][kXpLds], ps[3][kXpLds];
    double kap[2][kCkLds], sig[2][kCkLds];
};

__host__ __device__ inline int op_tiles(int nx, int ny, int nz, int TX, int CZ)
{
    return smooth0_box_tiles(nx, ny, nz, TX, CZ);
}

// RED: the Schur complement S = A_yy - A_ys A_ss^-1 A_sy of the particle
// blocks instead of A, over the electrode-level unknowns only: the reaction
// coupling of each electrode node enters scaled by omega_j (Sherman-Morrison:
// 1 - Gamma s_j (A_ss,j^-1)_NN = omega_j) and there is no particle column.
template <typename TX_T, bool TRANS, bool RED = false>
__device__ inline void operator_tile(const Geom &g, const OpArgs &O, double *qout, int tile, int TX,
                                     int CZ, OpLds &L)
{
    const TX_T *x = (const TX_T *)O.x;
    const int TY = kBlock / TX;
    const int PX = TX + 2, PY = TY + 2;
    const int EX = TX + 1, EY = TY + 1;
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY;
    const int tix = tile % ntx, tiy = (tile / ntx) % nty, tch = tile / (ntx * nty);
    const int i0 = tix * TX, j0 = tiy * TY, k0 = tch * CZ;
    const int k1 = k0 + CZ < g.nz ? k0 + CZ : g.nz;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < g.nx && j < g.ny;
    const long long layer = (long long)g.nx * g.ny;

    double pe[2], ce[2], ps[2], kp[2], sg[2];
    auto fetch_planes_to = [&](int kk, double vpe[2], double vce[2], double vps[2]) {
        const int el = (kk >= 0 && kk < g.nz) ? node_mat(g, kk) : -1;
        const bool has_ps = el >= 0 && kk != 0;
        const long long psb = el == 0 ? 0 : g.nea - (long long)(g.na + g.ns) * layer;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            const int ii = i0 - 1 + q % PX, jj = j0 - 1 + q / PX;
            const bool ok = q < PX * PY && kk >= 0 && kk < g.nz && ii >= 0 && ii < g.nx && jj >= 0 &&
                            jj < g.ny;
            const long long nd = ii + g.nx * (jj + (long long)g.ny * kk);
            vpe[h] = ok ? ldx(x + g.off_pe + nd) : 0.0;
            vce[h] = ok ? ldx(x + g.off_ce + nd) : 0.0;
            vps[h] = (ok && has_ps) ? ldx(x + (psb + nd)) : 0.0;
        }
    };
    auto store_planes_from = [&](int slot, const double vpe[2], const double vce[2], const double vps[2]) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            if (q < PX * PY) {
                L.pe[slot][q] = vpe[h];
                L.ce[slot][q] = vce[h];
                L.ps[slot][q] = vps[h];
            }
        }
    };
    auto fetch_elems_to = [&](int ek, double vkp[2], double vsg[2]) {
        const bool lay = ek >= 0 && ek < g.nz - 1;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            const int ei = i0 - 1 + q % EX, ej = j0 - 1 + q / EX;
            const bool ok = q < EX * EY && lay && ei >= 0 && ei < g.nx - 1 && ej >= 0 && ej < g.ny - 1;
            const long long id = ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek);
            vkp[h] = ok ? O.kaph[id] : 0.0;
            vsg[h] = ok ? O.sigh[id] : 0.0;
        }
    };
    auto store_elems_from = [&](int slot, const double vkp[2], const double vsg[2]) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int q = threadIdx.x + h * kBlock;
            if (q < EX * EY) {
                L.kap[slot][q] = vkp[h];
                L.sig[slot][q] = vsg[h];
            }
        }
    };
    auto fetch_planes = [&](int kk) { fetch_planes_to(kk, pe, ce, ps); };
    auto store_planes = [&](int slot) { store_planes_from(slot, pe, ce, ps); };
    auto fetch_elems = [&](int ek) { fetch_elems_to(ek, kp, sg); };
    auto store_elems = [&](int slot) { store_elems_from(slot, kp, sg); };
    {   // prologue: every load of the first layer is issued before any of
        // them is stored, so the tile waits for one memory latency, not four
        double pe0[2], ce0[2], ps0[2], pe1[2], ce1[2], ps1[2], kp0[2], sg0[2];
        fetch_planes_to(k0 - 1, pe0, ce0, ps0);
        fetch_planes_to(k0, pe1, ce1, ps1);
        fetch_elems_to(k0 - 1, kp0, sg0);
        fetch_planes(k0 + 1);
        fetch_elems(k0);
        store_planes_from((k0 + 2) % 3, pe0, ce0, ps0);
        store_planes_from(k0 % 3, pe1, ce1, ps1);
        store_elems_from((k0 + 1) & 1, kp0, sg0);
    }
    for (int k = k0; k < k1; k++) {
        store_planes((k + 1) % 3);
        store_elems(k & 1);
        __syncthreads();
        if (k + 1 < k1) {
            fetch_planes(k + 2);
            fetch_elems(k + 1);
        }
        if (own) {
            // element coefficients are read from LDS (or formed) just before
            // the field that uses them, so only one set is live at a time
            auto elem_coef = [&](const double (*C)[kCkLds], double c[8]) {
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                    c[e] = C[(k - 1 + ez) & 1][(tx + ex) + EX * (ty + ey)];
                }
            };
            auto mass_coef = [&](double c[8]) {
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
                    const int ek = k - 1 + ez;
                    // the element exists iff its kappa coefficient slot was
                    // filled; decide by the indices, as the per-node gather does
                    const int ei = i - 1 + ex, ej = j - 1 + ey;
                    const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < g.nx - 1 && ej < g.ny - 1 &&
                                    ek < g.nz - 1;
                    c[e] = ok ? (elem_mat(g, ek) >= 0 ? g.mass_elec : g.mass_sep) : 0.0;
                }
            };
            double ck[8], cs[8], cm[8];
            elem_coef(L.kap, ck);
            OpStencil P;
            double X[27];
            auto gather = [&](const double (*F)[kXpLds]) {
#pragma unroll
                for (int dz = -1; dz <= 1; dz++) {
                    const double *Pl = F[(k + dz + 3) % 3];
#pragma unroll
                    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
                        for (int dx = -1; dx <= 1; dx++)
                            X[nb_index(dx, dy, dz)] = Pl[(tx + 1 + dx) + PX * (ty + 1 + dy)];
                }
            };
            // one field at a time: the scheduling barriers keep the three
            // 27-value gathers from being hoisted together (register use)
            gather(L.pe);
            P.Kpe = q1_stiff(ck, X);
            P.xpe = X[13];
            // an empty statement that takes the finished sum: the compiler
            // may neither defer the sum nor hoist the next gather above it,
            // so only one 27-value neighbourhood is live at a time
            __asm__ volatile("" : "+v"(P.Kpe) : : "memory");
            gather(L.ce);
            P.Kce = q1_stiff(ck, X);
            mass_coef(cm);
            P.Mce = q1_mass(cm, X);
            P.xce = X[13];
            __asm__ volatile("" : "+v"(P.Kce), "+v"(P.Mce) : : "memory");
            P.Kps = 0.0;
            P.xpsc = 0.0;
            if (node_mat(g, k) >= 0) {
                elem_coef(L.sig, cs);
                gather(L.ps);
                P.Kps = q1_stiff(cs, X);
                P.xpsc = X[13];
            }
            const long long n = i + (long long)g.nx * j + layer * k;
            double ype, yce;
            if (!TRANS) {
                ype = P.Kpe + g.chi * P.Kce;
                yce = P.Mce + P.Kce;
            } else {
                ype = P.Kpe;
                yce = P.Mce + P.Kce + g.chi * P.Kpe;
            }
            const int el = node_mat(g, k);
            if (el >= 0) {
                const long long base = el == 0 ? 0 : g.nea;
                const int klo = el == 0 ? 0 : g.na + g.ns;
                const long long je = base + i + (long long)g.nx * (j + (long long)g.ny * (k - klo));
                const bool dir = (k == 0);
                // the tile's layer lies in one electrode: its table through a
                // wave-uniform pointer (scalar loads)
                const ConstTab &T = *(const ConstTab *)(O.tabs + __builtin_amdgcn_readfirstlane(el));
                double xsN = 0.0;
                if (!RED) {
                    const long long nn = el == 0 ? g.nea : g.nec;
                    const long long offs = el == 0 ? g.off_cs[0] : g.off_cs[1];
                    xsN = ldx(x + offs + (je - base) + (long long)(T.N - 1) * nn);
                }
                const OpCoupling cp = op_coupling<TRANS>(g, T, dir, O.mm[je], O.gg[je], O.ss[je],
                                                         O.ee[je], P.xpsc, P.xpe, P.xce, xsN);
                const double q = RED ? cp.q * O.om[je] : cp.q;
                O.y[je] = dir ? ldx(x + je) : P.Kps + cp.r0 * q;
                ype += cp.r1 * q;
                yce += cp.r2 * q;
                if (!RED) qout[je] = q;
            }
            O.y[g.off_pe + n] = ype;
            O.y[g.off_ce + n] = yce;
        }
        __syncthreads();
    }
}


// The particle rows of y = A x (or A^T x) for one electrode node je: row r
// of T0 applied to its column (loaded at once, indices clamped to the last
// point), plus the coupling weight times q (stored by operator_tile) on the
// surface row.
template <typename TX_T, int NRMAX, bool TRANS>
__device__ inline void operator_radial(const Geom &g, const OpArgs &O, const double *q, long long je)
{
    const TX_T *x = (const TX_T *)O.x;
    const int el = je < g.nea ? 0 : 1;
    const long long nn = el == 0 ? g.nea : g.nec;
    const long long jl = el == 0 ? je : je - g.nea;
    const long long offs = el == 0 ? g.off_cs[0] : g.off_cs[1];
    const TX_T *xs = x + offs + jl;
    double *ys = O.y + offs + jl;
    auto rows = [&](const auto &T) {
        const int N = T.N;
        double xr[NRMAX];
#pragma unroll
        for (int r = 0; r < NRMAX; r++) xr[r] = ldx(xs + (long long)(r < N ? r : N - 1) * nn);
        const double r3 = TRANS ? O.ss[je] : T.Gamma, qj = q[je];
        // all rows first, then the stores: a table read after a store may not
        // be hoisted above it (the pointers may alias), which would chain the
        // rows' cache latencies
        double v[NRMAX];
#pragma unroll
        for (int r = 0; r < NRMAX; r++) {
            if (r < N) {
                const double xm = r > 0 ? xr[r > 0 ? r - 1 : 0] : 0.0;
                const double xp = r < N - 1 ? xr[r + 1 < NRMAX ? r + 1 : r] : 0.0;
                v[r] = op_radial_row(T, TRANS, r, N, xm, xr[r], xp);
                if (r == N - 1) v[r] += r3 * qj;   // the same expression as in operator_finish
            }
        }
#pragma unroll
        for (int r = 0; r < NRMAX; r++)
            if (r < N) ys[(long long)r * nn] = v[r];
    };
    // the electrode's table through a wave-uniform pointer (scalar loads) when
    // the whole wave lies in one electrode, per lane otherwise
    const int elw = __builtin_amdgcn_readfirstlane(el);
    if (__builtin_amdgcn_ballot_w64(el != elw) == 0) rows(*(const ConstTab *)(O.tabs + elw));
    else rows(O.tabs[el]);
}

}  // namespace p4d
