// The linearized P4D operator y = A x (or A^T x, or b - A x) and the
// parameter-gradient kernels.
//
// A (paper Sec. 4.1, eq. blocks) per node, matrix-free:
//   phi_s rows: K_sigma phi_s + m q            (phis-weak; grounded layer: identity)
//   phi_e rows: K_kappa phi_e + chi K_kappa c_e - m q              (phie-weak)
//   c_e rows:   M_eps/dt c_e + K_kappa c_e - tc m q        (ce-weak, backward Euler)
//   c_s rows:   T0 c_s + Gamma q e_N                       (eq. FD with eq. LR)
// with the linearized reaction q = g (phi_s - phi_e) + e c_e + s c_s,N of
// the Butler-Volmer term (Sec. 2.4) and m the lumped electrode weight.  With
// separate transport coefficients (GEN) the diffusion-potential block and
// the c_e diffusion take their own element coefficients instead of chi kappa
// and kappa.
#include "p4d_kernels.hpp"

namespace p4d {

template <typename TX, int NRMAX, bool TRANS, bool RESID, bool GEN>
__global__ __launch_bounds__(kBlock) void k_operator(Geom g, OpArgs O, double *__restrict__ partial)
{
    __shared__ double red[4];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const long long n = (long long)lb * kBlock + threadIdx.x;
    double sq = 0.0;
    if (n < g.nnode) sq = operator_node<TX, NRMAX, TRANS, RESID, GEN>(g, O, n);
    if (partial) {
        const double s = block_sum(sq, red);
        if (threadIdx.x == 0) partial[lb] = s;
    }
}

int operator_blocks(const Geom &g) { return (int)((g.nnode + kBlock - 1) / kBlock); }

template <typename TX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_operator_tile(Geom g, OpArgs O, double *qout, int TXn, int CZ)
{
    __shared__ OpLds L;
    operator_tile<TX, TRANS>(g, O, qout, xcd_block(blockIdx.x, gridDim.x), TXn, CZ, L);
}

// the Schur complement of the particle blocks over the electrode-level unknowns
template <typename TX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_operator_schur(Geom g, OpArgs O, int TXn, int CZ)
{
    __shared__ OpLds L;
    operator_tile<TX, TRANS, true>(g, O, nullptr, xcd_block(blockIdx.x, gridDim.x), TXn, CZ, L);
}

template <typename TX, int NRMAX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_operator_radial(Geom g, OpArgs O, const double *q)
{
    const long long je = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (je < g.ne) operator_radial<TX, NRMAX, TRANS>(g, O, q, je);
}

// workgroups of the tiled operator resident at once on the current device
int operator_tile_slots()
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_operator_tile<double, false>,
                                                     kBlock, 0) != hipSuccess)
        return 1024;
    return (per < 1 ? 1 : per) * (ncu < 1 ? 1 : ncu);
}
int operator_tiles(const Geom &g, int TX, int CZ) { return op_tiles(g.nx, g.ny, g.nz, TX, CZ); }

// y = A x (or A^T x): the macro rows by 2.5D tiles of TX x (256/TX) nodes by
// CZ layers (storing the reaction q per electrode node in qbuf), then the
// particle rows one thread per value, when tile_tx > 0.  b - A x (b given)
// and the per-workgroup sums of squares (partial given) use one thread per
// node for everything.
template <typename TX>
void launch_operator(const Geom &g, const RadialTab *tabs, const double *sigh, const double *kaph,
                     const double *gg, const double *ss, const double *ee, const double *mm,
                     const TX *x, double *y, const double *b, double *partial, int transpose,
                     int tile_tx, int tile_cz, double *qbuf, const double *kdh, const double *dch,
                     hipStream_t st)
{
    OpArgs O{tabs, sigh, kaph, gg, ss, ee, mm, x, y, b, nullptr, kdh, dch};
    const bool gen = kdh && dch;
    if (!gen && !b && !partial && tile_tx > 0 && qbuf) {
        const int nt = operator_tiles(g, tile_tx, tile_cz);
        const int nr = (int)((g.ne + kBlock - 1) / kBlock);
        if (transpose)
            hipLaunchKernelGGL((k_operator_tile<TX, true>), dim3(nt), dim3(kBlock), 0, st, g, O, qbuf,
                               tile_tx, tile_cz);
        else
            hipLaunchKernelGGL((k_operator_tile<TX, false>), dim3(nt), dim3(kBlock), 0, st, g, O, qbuf,
                               tile_tx, tile_cz);
#define P4D_OR(NR)                                                                                  \
    do {                                                                                            \
        if (transpose)                                                                              \
            hipLaunchKernelGGL((k_operator_radial<TX, NR, true>), dim3(nr), dim3(kBlock), 0, st, g, O, \
                               qbuf);                                                               \
        else                                                                                        \
            hipLaunchKernelGGL((k_operator_radial<TX, NR, false>), dim3(nr), dim3(kBlock), 0, st, g,   \
                               O, qbuf);                                                            \
    } while (0)
        P4D_NR_SWITCH(rad_nrmax(g), P4D_OR)
#undef P4D_OR
        return;
    }
    const int nb = operator_blocks(g);
#define P4D_OP(NR, TR, RS)                                                                          \
    do {                                                                                            \
        if (gen)                                                                                    \
            hipLaunchKernelGGL((k_operator<TX, NR, TR, RS, true>), dim3(nb), dim3(kBlock), 0, st, g, O, \
                               partial);                                                            \
        else                                                                                        \
            hipLaunchKernelGGL((k_operator<TX, NR, TR, RS, false>), dim3(nb), dim3(kBlock), 0, st, g,   \
                               O, partial);                                                         \
    } while (0)
#define P4D_OP2(NR)                                        \
    do {                                                   \
        if (!transpose) {                                  \
            if (b) P4D_OP(NR, false, true);                \
            else P4D_OP(NR, false, false);                 \
        } else {                                           \
            if (b) P4D_OP(NR, true, true);                 \
            else P4D_OP(NR, true, false);                  \
        }                                                  \
    } while (0)
    P4D_NR_SWITCH(rad_nrmax(g), P4D_OP2)
#undef P4D_OP2
#undef P4D_OP
}
template void launch_operator<double>(const Geom &, const RadialTab *, const double *,
                                      const double *, const double *, const double *,
                                      const double *, const double *, const double *, double *,
                                      const double *, double *, int, int, int, double *,
                                      const double *, const double *, hipStream_t);
template void launch_operator<float>(const Geom &, const RadialTab *, const double *,
                                     const double *, const double *, const double *,
                                     const double *, const double *, const float *, double *,
                                     const double *, double *, int, int, int, double *,
                                     const double *, const double *, hipStream_t);

// the Schur-complement operator one thread per node, with the separate
// element arrays (GEN: transport coefficients, storage, box elements,
// Newton terms)
template <typename TX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_operator_schur_gen(Geom g, OpArgs O)
{
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const long long n = (long long)lb * kBlock + threadIdx.x;
    if (n < g.nnode) operator_node<TX, 1, TRANS, false, true, true>(g, O, n);
}

// w = S y (or S^T y), S = A_yy - A_ys A_ss^-1 A_sy: y and w hold the
// electrode-level unknowns only (length Nm); omega per electrode node.
// kdh, dch given: the per-node form with the separate element arrays.
template <typename TX>
void launch_operator_schur(const Geom &g, const RadialTab *tabs, const double *sigh,
                           const double *kaph, const double *gg, const double *ss, const double *ee,
                           const double *mm, const double *om, const TX *y, double *w, int transpose,
                           int tile_tx, int tile_cz, const double *kdh, const double *dch, hipStream_t st)
{
    OpArgs O{tabs, sigh, kaph, gg, ss, ee, mm, y, w, nullptr, om, kdh, dch};
    if (kdh && dch) {
        const int nb = operator_blocks(g);
        if (transpose)
            hipLaunchKernelGGL((k_operator_schur_gen<TX, true>), dim3(nb), dim3(kBlock), 0, st, g, O);
        else
            hipLaunchKernelGGL((k_operator_schur_gen<TX, false>), dim3(nb), dim3(kBlock), 0, st, g, O);
        return;
    }
    const int nt = operator_tiles(g, tile_tx, tile_cz);
    if (transpose)
        hipLaunchKernelGGL((k_operator_schur<TX, true>), dim3(nt), dim3(kBlock), 0, st, g, O, tile_tx,
                           tile_cz);
    else
        hipLaunchKernelGGL((k_operator_schur<TX, false>), dim3(nt), dim3(kBlock), 0, st, g, O, tile_tx,
                           tile_cz);
}
template void launch_operator_schur<double>(const Geom &, const RadialTab *, const double *,
                                            const double *, const double *, const double *,
                                            const double *, const double *, const double *,
                                            const double *, double *, int, int, int, const double *,
                                            const double *, hipStream_t);
template void launch_operator_schur<float>(const Geom &, const RadialTab *, const double *,
                                           const double *, const double *, const double *,
                                           const double *, const double *, const double *,
                                           const float *, double *, int, int, int, const double *,
                                           const double *, hipStream_t);

// ---------------------------------------------------------------------------
// Gradients of J = w.x:  dJ/dp = -lambda^T (dA/dp) x.
//  sigma_e enters only the phi_s stiffness block through h sigma_e Khat, so
//  dJ/dsigma_e = -h lambda_e^T Khat x_e over the element's phi_s corners
//  (grounded corners excluded).  Ds enters T0 = I/dt - L_h linearly, so
//  dJ/dDs = sum_j lambda_s,j^T (dL_h/dDs) x_s,j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_grad(Geom g, const RadialTab *__restrict__ tabs,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ dsigma,
                                                 double *__restrict__ partial)
{
    __shared__ double red[4];
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    // elements: one per thread
    if (t < g.nelem) {
        const int ei = (int)(t % (g.nx - 1));
        const long long u = t / (g.nx - 1);
        const int ej = (int)(u % (g.ny - 1)), ek = (int)(u / (g.ny - 1));
        const int el = elem_mat(g, ek);
        double val = 0.0;
        if (el >= 0) {
            const long long base = el == 0 ? 0 : g.nea;
            const int klo = el == 0 ? 0 : g.na + g.ns;
            double xl[8], ll[8];
#pragma unroll
            for (int a = 0; a < 8; a++) {
                const int i = ei + (a & 1), j = ej + ((a >> 1) & 1), k = ek + ((a >> 2) & 1);
                const long long je = base + i + (long long)g.nx * (j + (long long)g.ny * (k - klo));
                xl[a] = k == 0 ? 0.0 : x[je];
                ll[a] = k == 0 ? 0.0 : lam[je];
            }
            // (Khat x)_a = sum_b Khat_ab (x_b - x_a): rows of Khat sum to zero,
            // so the large near-constant parts of x cancel exactly
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 8; a++) {
                double row = 0.0;
#pragma unroll
                for (int bb = 0; bb < 8; bb++)
                    if (popc3(a ^ bb) >= 2) row += xl[a] - xl[bb];
                s += ll[a] * row;
            }
            val = -g.h * s * (1.0 / 12.0);
        }
        dsigma[t] = val;
    }
    // electrode nodes: radial part
    if (t < g.ne) {
        const int el = t < g.nea ? 0 : 1;
        const RadialTab &T = tabs[el];
        const long long nn = el == 0 ? g.nea : g.nec;
        const long long jl = el == 0 ? t : t - g.nea;
        const double *xs = x + g.off_cs[el] + jl;
        const double *ls = lam + g.off_cs[el] + jl;
        double s = 0.0;
        for (int r = 0; r < T.N; r++) {
            double Lx = T.hdia[r] * xs[(long long)r * nn];
            if (r > 0) Lx += T.hsub[r] * xs[(long long)(r - 1) * nn];
            if (r < T.N - 1) Lx += T.hsup[r] * xs[(long long)(r + 1) * nn];
            s += ls[(long long)r * nn] * Lx;
        }
        acc[el] = s;
    }
    const double s0 = block_sum(acc[0], red);
    const double s1 = block_sum(acc[1], red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s0;
        partial[2 * blockIdx.x + 1] = s1;
    }
}

__global__ __launch_bounds__(kBlock) void k_grad_final(const double *__restrict__ partial,
                                                       int nblk, double *__restrict__ out)
{
    __shared__ double red[4];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        s0 += partial[2 * b];
        s1 += partial[2 * b + 1];
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
    }
}

void launch_grad(const Geom &g, const RadialTab *tabs, const double *x, const double *lam,
                 double *dsigma, double *partial, hipStream_t st)
{
    const long long n = g.nelem > g.ne ? g.nelem : g.ne;
    const int nb = (int)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_grad, dim3(nb), dim3(kBlock), 0, st, g, tabs, x, lam, dsigma, partial);
}

void launch_grad_final(const double *partial, int nblk, double *dDs, hipStream_t st)
{
    hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(kBlock), 0, st, partial, nblk, dDs);
}

}  // namespace p4d
