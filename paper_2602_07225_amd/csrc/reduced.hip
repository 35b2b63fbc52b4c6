// Krylov iteration over the Schur complement of the particle blocks.  The
// c_s block A_ss is block diagonal (one tridiagonal block per electrode node,
// paper Sec. 4.1) and c_s couples to the electrode-level fields only through
// its surface value, so
//   S = A_yy - A_ys A_ss^-1 A_sy,   bhat = b_y - A_ys A_ss^-1 b_s,
//   x_s = A_ss^-1 (b_s - A_sy y)
// are exact; FGMRES runs on S y = bhat over y = [phi_s | phi_e | c_e] only
// (S is the operator's RED mode).  With A_ys = a_y s_j e_N^T and A_sy =
// Gamma e_N b_y^T per node (transposed: the roles of a and b swap):
//   red_rhs  : zeta_j = (A_ss,j^-1 b_s,j)_N, bhat_f = b_f - a_f s_j zeta_j,
//   red_back : x_s,j = A_ss,j^-1 (b_s,j - delta_j e_N), delta_j = Gamma b_j . y,
//   red_resid: w = bhat - w and its sum of squares (restart residuals).
// All in FP64: these steps are part of the solution, not of the
// preconditioner.
#include "p4d_kernels.hpp"

namespace p4d {

struct RedArgs {
    const RadialTab *tabs;
    const double *gg, *ss, *ee, *mm;
};

template <int NRMAX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_red_rhs(Geom g, RedArgs R, const double *__restrict__ b,
                                                    double *__restrict__ bhat)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    double bpe = b[g.off_pe + n], bce = b[g.off_ce + n];
    const int el = node_mat(g, k);
    if (el >= 0) {
        const long long base = el == 0 ? 0 : g.nea;
        const long long klo = el == 0 ? 0 : g.na + g.ns;
        const long long je = base + n - klo * g.nx * g.ny;
        const bool dir = (k == 0);
        double bps = b[je];
        const RadialTab &Tb = R.tabs[el];
        const int N = Tb.N;
        const long long nn = el == 0 ? g.nea : g.nec;
        const double *bs = b + (el == 0 ? g.off_cs[0] : g.off_cs[1]) + (je - base);
        double rv[NRMAX];
#pragma unroll
        for (int q = 0; q < NRMAX; q++) rv[q] = bs[(long long)(q < N ? q : N - 1) * nn];
        double y = rv[0];
#pragma unroll
        for (int q = 1; q < NRMAX; q++)
            if (q < N) y = rv[q] - (TRANS ? Tb.lT[q] : Tb.l[q]) * y;
        const double sj = R.ss[je];
        const double zeta = y / (Tb.piv[N - 1] + Tb.Gamma * sj);
        const double m = R.mm[je];
        if (!TRANS) {   // a_y s_j zeta, a_y = (m, -m, -tc m)
            const double f = sj * zeta;
            if (!dir) bps -= m * f;
            bpe += m * f;
            bce += g.tc * m * f;
        } else {        // Gamma b_y zeta, b_y = (g, -g, e)
            const double f = Tb.Gamma * zeta;
            const double gj = R.gg[je];
            if (!dir) bps -= gj * f;
            bpe += gj * f;
            bce -= R.ee[je] * f;
        }
        bhat[je] = bps;
    }
    bhat[g.off_pe + n] = bpe;
    bhat[g.off_ce + n] = bce;
}

template <int NRMAX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_red_back(Geom g, RedArgs R, const double *__restrict__ b,
                                                     double *__restrict__ x)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const int el = node_mat(g, k);
    if (el < 0) return;
    const long long base = el == 0 ? 0 : g.nea;
    const long long klo = el == 0 ? 0 : g.na + g.ns;
    const long long je = base + n - klo * g.nx * g.ny;
    const bool dir = (k == 0);
    const RadialTab &Tb = R.tabs[el];
    const int N = Tb.N;
    const long long nn = el == 0 ? g.nea : g.nec;
    const long long offs = el == 0 ? g.off_cs[0] : g.off_cs[1];
    const double *bs = b + offs + (je - base);
    double *xs = x + offs + (je - base);
    const double yps = dir ? 0.0 : x[je], ype = x[g.off_pe + n], yce = x[g.off_ce + n];
    const double sj = R.ss[je], m = R.mm[je], gj = R.gg[je];
    const double delta = TRANS ? sj * (m * yps - m * ype - g.tc * m * yce)
                               : Tb.Gamma * (gj * yps - gj * ype + R.ee[je] * yce);
    double rv[NRMAX];
#pragma unroll
    for (int q = 0; q < NRMAX; q++) rv[q] = bs[(long long)(q < N ? q : N - 1) * nn];
    // forward elimination with the shared unit-lower factor; the surface
    // entry carries -delta
    double yv[NRMAX];
    yv[0] = rv[0];   // N >= 3: the surface entry is not the first
    double ylast = yv[0];
#pragma unroll
    for (int q = 1; q < NRMAX; q++) {
        if (q < N) {
            const double rq = q == N - 1 ? rv[q] - delta : rv[q];
            yv[q] = rq - (TRANS ? Tb.lT[q] : Tb.l[q]) * yv[q - 1];
            ylast = yv[q];
        }
    }
    double zn = ylast / (Tb.piv[N - 1] + Tb.Gamma * sj);
    xs[(long long)(N - 1) * nn] = zn;
#pragma unroll
    for (int q = NRMAX - 2; q >= 0; q--) {
        if (q < N - 1) {
            zn = (yv[q] - (TRANS ? Tb.tsub[q + 1] : Tb.tsup[q]) * zn) * Tb.ipiv[q];
            xs[(long long)q * nn] = zn;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_red_resid(long long n, const double *__restrict__ bhat,
                                                      double *__restrict__ w, double *__restrict__ partial)
{
    __shared__ double lds[4];
    double sq = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const double v = bhat[i] - w[i];
        w[i] = v;
        sq += v * v;
    }
    sq = block_sum(sq, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = sq;
}

static RedArgs red_args(const RadialTab *tabs, const double *gg, const double *ss, const double *ee,
                        const double *mm)
{
    RedArgs R;
    R.tabs = tabs;
    R.gg = gg; R.ss = ss; R.ee = ee; R.mm = mm;
    return R;
}

void launch_red_rhs(const Geom &g, const RadialTab *tabs, const double *gg, const double *ss,
                    const double *ee, const double *mm, const double *b, double *bhat, int transpose,
                    hipStream_t st)
{
    const RedArgs R = red_args(tabs, gg, ss, ee, mm);
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
#define P4D_RR(NR)                                                                                 \
    do {                                                                                           \
        if (transpose)                                                                             \
            hipLaunchKernelGGL((k_red_rhs<NR, true>), dim3(nb), dim3(kBlock), 0, st, g, R, b, bhat); \
        else                                                                                       \
            hipLaunchKernelGGL((k_red_rhs<NR, false>), dim3(nb), dim3(kBlock), 0, st, g, R, b, bhat); \
    } while (0)
    P4D_NR_SWITCH(rad_nrmax(g), P4D_RR)
#undef P4D_RR
}

void launch_red_back(const Geom &g, const RadialTab *tabs, const double *gg, const double *ss,
                     const double *ee, const double *mm, const double *b, double *x, int transpose,
                     hipStream_t st)
{
    const RedArgs R = red_args(tabs, gg, ss, ee, mm);
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
#define P4D_RB(NR)                                                                                \
    do {                                                                                          \
        if (transpose)                                                                            \
            hipLaunchKernelGGL((k_red_back<NR, true>), dim3(nb), dim3(kBlock), 0, st, g, R, b, x);  \
        else                                                                                      \
            hipLaunchKernelGGL((k_red_back<NR, false>), dim3(nb), dim3(kBlock), 0, st, g, R, b, x); \
    } while (0)
    P4D_NR_SWITCH(rad_nrmax(g), P4D_RB)
#undef P4D_RB
}

void launch_red_resid(long long n, const double *bhat, double *w, double *partial, int nblk,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_red_resid, dim3(nblk), dim3(kBlock), 0, st, n, bhat, w, partial);
}

}  // namespace p4d
