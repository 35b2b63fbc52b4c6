// Particle-block kernels of the preconditioner (paper Sec. 4.2: the c_s
// block is block diagonal with one tridiagonal N_c x N_c matrix per point,
// inverted exactly).  With A_ss,j = T0 + Gamma s_j e_N e_N^T, T0 shared by
// all points of an electrode, one LU of T0 serves every node: only the last
// pivot depends on j.
//
//   rad_fwd : zeta_j = (A_ss,j^-1 r_s,j)_N by forward elimination, then the
//             macro right-hand side r~_y = r_y - a_y s_j zeta_j (SCHUR mode;
//             transposed: r_y - Gamma b_y zeta_j), written in the
//             preconditioner precision together with the first Chebyshev
//             iterate of each V-cycle box.
//   rad_back: delta_j = Gamma b_y . z_y (transposed: s_j a_y . z_y),
//             z_s,j = A_ss,j^-1 (r_s,j - delta_j e_N), and the macro output.
// Eliminations run in the preconditioner precision T; the surface coupling
// (r~_y, delta_j) is formed in FP64.
#include "p4d_device.hpp"

namespace p4d {

template <typename T, bool TRANS, bool SCHUR>
__global__ __launch_bounds__(kBlock) void k_rad_fwd(
    Geom g, const RadialTab *__restrict__ tabs, const double *__restrict__ gg,
    const double *__restrict__ ss, const double *__restrict__ ee, const double *__restrict__ mm,
    const double *__restrict__ r, double rscale, T *__restrict__ b0, double *__restrict__ x1,
    const T *__restrict__ invd0, double c2a, double c2c, double c2e, double c2ce)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    double rpe = r[g.off_pe + n] * rscale;
    double rce = r[g.off_ce + n] * rscale;
    const int el = node_mat(g, k);
    if (el >= 0) {
        const long long base = el == 0 ? 0 : g.nea;
        const long long klo = el == 0 ? 0 : g.na + g.ns;
        const long long je = base + n - klo * g.nx * g.ny;
        const bool dir = (k == 0);
        double rps = r[je] * rscale;
        if (SCHUR) {
            const RadialTab &Tb = tabs[el];
            const int N = Tb.N;
            const long long nn = el == 0 ? g.nea : g.nec;
            const double *rs = r + g.off_cs[el] + (je - base);
            T y = (T)(rs[0] * rscale);
            for (int q = 1; q < N; q++) {
                const T lq = (T)(TRANS ? Tb.lT[q] : Tb.l[q]);
                y = (T)(rs[(long long)q * nn] * rscale) - lq * y;
            }
            const double sj = ss[je];
            const T pivN = (T)(Tb.piv[N - 1] + Tb.Gamma * sj);
            const double zeta = (double)(y / pivN);
            const double m = mm[je];
            if (!TRANS) {   // a_y s_j zeta, a_y = (m, -m, -tc m)
                const double f = sj * zeta;
                if (!dir) rps -= m * f;
                rpe += m * f;
                rce += g.tc * m * f;
            } else {        // Gamma b_y zeta, b_y = (g, -g, e)
                const double f = Tb.Gamma * zeta;
                const double gj = gg[je];
                if (!dir) rps -= gj * f;
                rpe += gj * f;
                rce -= ee[je] * f;
            }
        }
        const T bps = (T)rps;
        b0[je] = bps;
        if (!dir) x1[je] = (el == 0 ? c2a : c2c) * (double)invd0[je] * (double)bps;
    }
    const T bpe = (T)rpe, bce = (T)rce;
    b0[g.off_pe + n] = bpe;
    b0[g.off_ce + n] = bce;
    x1[g.off_pe + n] = c2e * (double)invd0[g.off_pe + n] * (double)bpe;
    x1[g.off_ce + n] = c2ce * (double)invd0[g.off_ce + n] * (double)bce;
}

template <typename T>
void launch_rad_fwd(const Geom &g, const RadialTab *tabs, const double *gg, const double *ss,
                    const double *ee, const double *mm, const double *r, double rscale, T *b0,
                    double *x1, const T *invd0, const double c2box[4], int transpose, int schur,
                    hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
#define P4D_RF(TR, SC)                                                                       \
    hipLaunchKernelGGL((k_rad_fwd<T, TR, SC>), dim3(nb), dim3(kBlock), 0, st, g, tabs, gg, \
                       ss, ee, mm, r, rscale, b0, x1, invd0, c2box[0], c2box[1], c2box[2],  \
                       c2box[3])
    if (schur) {
        if (transpose) P4D_RF(true, true); else P4D_RF(false, true);
    } else {
        P4D_RF(false, false);
    }
#undef P4D_RF
}
template void launch_rad_fwd<double>(const Geom &, const RadialTab *, const double *,
                                     const double *, const double *, const double *,
                                     const double *, double, double *, double *, const double *,
                                     const double *, int, int, hipStream_t);
template void launch_rad_fwd<float>(const Geom &, const RadialTab *, const double *,
                                    const double *, const double *, const double *,
                                    const double *, double, float *, double *, const float *,
                                    const double *, int, int, hipStream_t);

// z_s,j = A_ss,j^-1 r_s,j - delta_j A_ss,j^-1 e_N, and by Sherman-Morrison
// A_ss,j^-1 e_N = omega_j T0^-1 e_N: the elimination in precision T only
// sees r_s, while delta_j, which carries the large near-null part of z_y, is
// applied in FP64 with the precomputed T0^-1 e_N.
template <typename T, typename TZ, int NRMAX, bool TRANS, bool SCHUR>
__global__ __launch_bounds__(kBlock) void k_rad_back(
    Geom g, const RadialTab *__restrict__ tabs, const double *__restrict__ gg,
    const double *__restrict__ ss, const double *__restrict__ ee, const double *__restrict__ mm,
    const double *__restrict__ om, const double *__restrict__ r, double rscale,
    const double *__restrict__ x0, TZ *__restrict__ z)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const double zpe = x0[g.off_pe + n];
    const double zce = x0[g.off_ce + n];
    z[g.off_pe + n] = (TZ)zpe;
    z[g.off_ce + n] = (TZ)zce;
    const int el = node_mat(g, k);
    if (el < 0) return;
    const long long base = el == 0 ? 0 : g.nea;
    const long long klo = el == 0 ? 0 : g.na + g.ns;
    const long long je = base + n - klo * g.nx * g.ny;
    const bool dir = (k == 0);
    const double zps = dir ? r[je] * rscale : x0[je];
    z[je] = (TZ)zps;
    const RadialTab &Tb = tabs[el];
    const int N = Tb.N;
    const long long nn = el == 0 ? g.nea : g.nec;
    const double *rs = r + g.off_cs[el] + (je - base);
    TZ *zs = z + g.off_cs[el] + (je - base);
    const double sj = ss[je];
    double dw = 0.0;   // delta_j * omega_j
    if (SCHUR) {
        const double m = mm[je];
        double delta;
        if (!TRANS)
            delta = Tb.Gamma * ((dir ? 0.0 : gg[je]) * zps - gg[je] * zpe + ee[je] * zce);
        else
            delta = sj * ((dir ? 0.0 : m) * zps - m * zpe - g.tc * m * zce);
        dw = delta * om[je];
    }
    // forward elimination; the register array is only indexed by unrolled
    // constants, the last entry is carried separately
    T y[NRMAX];
    y[0] = (T)(rs[0] * rscale);
    T ylast = y[0];
#pragma unroll
    for (int q = 1; q < NRMAX; q++) {
        if (q < N) {
            const T lq = (T)(TRANS ? Tb.lT[q] : Tb.l[q]);
            y[q] = (T)(rs[(long long)q * nn] * rscale) - lq * y[q - 1];
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
}

template <typename T, typename TZ>
void launch_rad_back(const Geom &g, const RadialTab *tabs, const double *gg, const double *ss,
                     const double *ee, const double *mm, const double *om, const double *r,
                     double rscale, const double *x0, TZ *z, int transpose, int schur,
                     hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
    const int nrm = g.nr[0] > g.nr[1] ? g.nr[0] : g.nr[1];
#define P4D_RB(NR, TR, SC)                                                                      \
    hipLaunchKernelGGL((k_rad_back<T, TZ, NR, TR, SC>), dim3(nb), dim3(kBlock), 0, st, g, tabs, \
                       gg, ss, ee, mm, om, r, rscale, x0, z)
#define P4D_RB2(NR)                                          \
    do {                                                     \
        if (schur) {                                         \
            if (transpose) P4D_RB(NR, true, true);           \
            else P4D_RB(NR, false, true);                    \
        } else {                                             \
            if (transpose) P4D_RB(NR, true, false);          \
            else P4D_RB(NR, false, false);                   \
        }                                                    \
    } while (0)
    if (nrm <= 8) P4D_RB2(8);
    else if (nrm <= 16) P4D_RB2(16);
    else if (nrm <= 32) P4D_RB2(32);
    else P4D_RB2(64);
#undef P4D_RB2
#undef P4D_RB
}
template void launch_rad_back<double, double>(const Geom &, const RadialTab *, const double *,
                                              const double *, const double *, const double *, const double *,
                                              const double *, double, const double *, double *,
                                              int, int, hipStream_t);
template void launch_rad_back<float, double>(const Geom &, const RadialTab *, const double *,
                                             const double *, const double *, const double *, const double *,
                                             const double *, double, const double *, double *,
                                             int, int, hipStream_t);
template void launch_rad_back<float, float>(const Geom &, const RadialTab *, const double *,
                                            const double *, const double *, const double *, const double *,
                                            const double *, double, const double *, float *, int,
                                            int, hipStream_t);
template void launch_rad_back<double, float>(const Geom &, const RadialTab *, const double *,
                                             const double *, const double *, const double *, const double *,
                                             const double *, double, const double *, float *,
                                             int, int, hipStream_t);

}  // namespace p4d
