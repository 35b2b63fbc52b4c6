// Block Gauss-Seidel preconditioner kernels (paper Sec. 4.2, eq. PGS).  The
// fields are solved one after another in a chosen ordering; before a field is
// solved, the off-diagonal blocks of A times the fields solved before it are
// subtracted from its rows.  Those blocks are
//   - the node-local reaction terms a_f,j b_g,j (a = (m, -m, -tc m, Gamma),
//     b = (g, -g, e, s) over phi_s, phi_e, c_e and the c_s surface value, the
//     phi_s entries zero on the grounded layer), entering the c_s surface row
//     for f = c_s; transposed, a and b swap;
//   - the diffusion-potential block (chi K_kappa, or its own element
//     coefficients) in the (phi_e row, c_e column) block; transposed, in the
//     (c_e row, phi_e column) block.
// Solved values are read in FP64: the final level-0 V-cycle iterates of the
// electrode-level fields and the c_s surface values kept per electrode node.
#include "p4d_bgs.hpp"

namespace p4d {

template <typename T, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_bgs_rhs(Geom g, BgsArgs B, const double *__restrict__ r,
                                                    const double *rscale_p)
{
    const double rscale = rscale_p ? *rscale_p : 1.0;
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int f = B.field, done = B.done;
    const int i = (int)(n % g.nx);
    const long long t2 = n / g.nx;
    const int j = (int)(t2 % g.ny), k = (int)(t2 / g.ny);
    const int el = node_mat(g, k);
    if (f == BF_PHIS && el < 0) return;
    const RadArgs &R = B.R;
    long long je = 0;
    if (el >= 0) {
        const long long base = el == 0 ? 0 : g.nea;
        const int klo = el == 0 ? 0 : g.na + g.ns;
        je = base + n - (long long)klo * g.nx * g.ny;
    }
    const long long slot = f == BF_PHIS ? je : (f == BF_PHIE ? g.off_pe + n : g.off_ce + n);
    const bool dir = (k == 0);
    double t = r[slot] * rscale;
    if (el >= 0 && done) {
        const double m = R.mm[je], gj = R.gg[je], ej = R.ee[je], sj = R.ss[je];
        const double Gam = el == 0 ? R.tabs[0].Gamma : R.tabs[1].Gamma;
        // column coefficients (b, or a when transposed) times the solved values
        double q = 0.0;
        if ((done & (1 << BF_PHIS)) && !dir)
            q += (TRANS ? m : gj) * (el == 0 ? R.x0[0] : R.x0[1])[je];
        if (done & (1 << BF_PHIE)) q += (TRANS ? -m : -gj) * R.x0[2][g.off_pe + n];
        if (done & (1 << BF_CE)) q += (TRANS ? -g.tc * m : ej) * R.x0[3][g.off_ce + n];
        if (done & (1 << BF_CS)) q += (TRANS ? Gam : sj) * B.zsN[je];
        // row coefficient of field f (a, or b when transposed)
        const double rc = f == BF_PHIS ? (dir ? 0.0 : (TRANS ? gj : m))
                                       : (f == BF_PHIE ? (TRANS ? -gj : -m) : (TRANS ? ej : -g.tc * m));
        t -= rc * q;
    }
    const bool kterm = TRANS ? (f == BF_CE && (done & (1 << BF_PHIE)))
                             : (f == BF_PHIE && (done & (1 << BF_CE)));
    if (kterm) {
        double ck[8], X[27];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int ei = i - 1 + (e & 1), ej2 = j - 1 + ((e >> 1) & 1), ek = k - 1 + ((e >> 2) & 1);
            const bool ok = ei >= 0 && ej2 >= 0 && ek >= 0 && ei < g.nx - 1 && ej2 < g.ny - 1 &&
                            ek < g.nz - 1;
            const long long id = ei + (long long)(g.nx - 1) * (ej2 + (long long)(g.ny - 1) * ek);
            ck[e] = ok ? B.kx[id] : 0.0;
        }
        load_nb(g, TRANS ? R.x0[2] + g.off_pe : R.x0[3] + g.off_ce, n, i, j, k, X);
        t -= B.kx_scale * q1_stiff(ck, X);
    }
    const T bt = (T)t;
    ((T *)R.b0)[slot] = bt;
    if (!(f == BF_PHIS && dir)) {
        const double c2 = f == BF_PHIS ? (el == 0 ? R.c2box[0] : R.c2box[1])
                                       : (f == BF_PHIE ? R.c2box[2] : R.c2box[3]);
        R.x1[slot] = c2 * (double)((const T *)R.invd0)[slot] * (double)bt;
    }
}

template <typename T>
void launch_bgs_rhs(const Geom &g, const BgsArgs &B, const double *r, const double *rscale, int transpose,
                    hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
    if (transpose)
        hipLaunchKernelGGL((k_bgs_rhs<T, true>), dim3(nb), dim3(kBlock), 0, st, g, B, r, rscale);
    else
        hipLaunchKernelGGL((k_bgs_rhs<T, false>), dim3(nb), dim3(kBlock), 0, st, g, B, r, rscale);
}
template void launch_bgs_rhs<double>(const Geom &, const BgsArgs &, const double *, const double *, int,
                                     hipStream_t);
template void launch_bgs_rhs<float>(const Geom &, const BgsArgs &, const double *, const double *, int,
                                    hipStream_t);

// A_ss,j = T0 + Gamma s_j e_N e_N^T, so A_ss,j^-1 e_N = omega_j T0^-1 e_N with
// omega_j = 1 / (1 + Gamma s_j tau0) (Sherman-Morrison): the elimination in
// precision T sees r_s only and the coupling delta_j is applied in FP64.
template <typename T, typename TZ, int NRMAX, bool TRANS>
__global__ __launch_bounds__(kBlock) void k_bgs_cs(Geom g, BgsArgs B, const double *__restrict__ r,
                                                   const double *rscale_p, TZ *__restrict__ z)
{
    const double rscale = rscale_p ? *rscale_p : 1.0;
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const int el = node_mat(g, k);
    if (el < 0) return;
    const RadArgs &R = B.R;
    const int done = B.done;
    const long long base = el == 0 ? 0 : g.nea;
    const long long klo = el == 0 ? 0 : g.na + g.ns;
    const long long je = base + n - klo * g.nx * g.ny;
    const bool dir = (k == 0);
    auto solve = [&](const auto &Tb) {
        const int N = Tb.N;
        const long long nn = el == 0 ? g.nea : g.nec;
        const long long offs = el == 0 ? g.off_cs[0] : g.off_cs[1];
        const double *rs = r + offs + (je - base);
        TZ *zs = z + offs + (je - base);
        const double sj = R.ss[je], m = R.mm[je], gj = R.gg[je];
        double pz = 0.0;   // column coefficients times the solved values
        if ((done & (1 << BF_PHIS)) && !dir) pz += (TRANS ? m : gj) * (el == 0 ? R.x0[0] : R.x0[1])[je];
        if (done & (1 << BF_PHIE)) pz += (TRANS ? -m : -gj) * R.x0[2][g.off_pe + n];
        if (done & (1 << BF_CE)) pz += (TRANS ? -g.tc * m : R.ee[je]) * R.x0[3][g.off_ce + n];
        const double delta = (TRANS ? sj : Tb.Gamma) * pz;
        const double dw = delta / (1.0 + Tb.Gamma * sj * Tb.tau0);
        double rv[NRMAX];
#pragma unroll
        for (int q = 0; q < NRMAX; q++) rv[q] = rs[(long long)(q < N ? q : N - 1) * nn];
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
        const double zN = (double)zn - dw * (TRANS ? Tb.tNT[N - 1] : Tb.tN[N - 1]);
        zs[(long long)(N - 1) * nn] = (TZ)zN;
        B.zsN[je] = zN;
#pragma unroll
        for (int q = NRMAX - 2; q >= 0; q--) {
            if (q < N - 1) {
                const T u = (T)(TRANS ? Tb.tsub[q + 1] : Tb.tsup[q]);
                zn = (y[q] - u * zn) * (T)Tb.ipiv[q];
                zs[(long long)q * nn] = (TZ)((double)zn - dw * (TRANS ? Tb.tNT[q] : Tb.tN[q]));
            }
        }
    };
    // the electrode's table through a wave-uniform pointer (scalar loads) when
    // the whole wave lies in one electrode, per lane otherwise
    const int elw = __builtin_amdgcn_readfirstlane(el);
    if (__builtin_amdgcn_ballot_w64(el != elw) == 0) solve(*(const ConstTab *)(R.tabs + elw));
    else solve(R.tabs[el]);
}

template <typename T, typename TZ>
void launch_bgs_cs(const Geom &g, const BgsArgs &B, const double *r, const double *rscale, TZ *z,
                   int transpose, hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
#define P4D_BC(NR, TR) \
    hipLaunchKernelGGL((k_bgs_cs<T, TZ, NR, TR>), dim3(nb), dim3(kBlock), 0, st, g, B, r, rscale, z)
#define P4D_BC2(NR)                        \
    do {                                   \
        if (transpose) P4D_BC(NR, true);   \
        else P4D_BC(NR, false);            \
    } while (0)
    P4D_NR_SWITCH(rad_nrmax(g), P4D_BC2)
#undef P4D_BC2
#undef P4D_BC
}
template void launch_bgs_cs<double, double>(const Geom &, const BgsArgs &, const double *, const double *,
                                            double *, int, hipStream_t);
template void launch_bgs_cs<float, double>(const Geom &, const BgsArgs &, const double *, const double *,
                                           double *, int, hipStream_t);
template void launch_bgs_cs<double, float>(const Geom &, const BgsArgs &, const double *, const double *,
                                           float *, int, hipStream_t);
template void launch_bgs_cs<float, float>(const Geom &, const BgsArgs &, const double *, const double *,
                                          float *, int, hipStream_t);

template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_bgs_out(Geom g, BgsArgs B, const double *__restrict__ r,
                                                    const double *rscale_p, TZ *__restrict__ z)
{
    const double rscale = rscale_p ? *rscale_p : 1.0;
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const RadArgs &R = B.R;
    z[g.off_pe + n] = (TZ)R.x0[2][g.off_pe + n];
    z[g.off_ce + n] = (TZ)R.x0[3][g.off_ce + n];
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const int el = node_mat(g, k);
    if (el < 0) return;
    const long long base = el == 0 ? 0 : g.nea;
    const long long klo = el == 0 ? 0 : g.na + g.ns;
    const long long je = base + n - klo * g.nx * g.ny;
    z[je] = (TZ)(k == 0 ? r[je] * rscale : (el == 0 ? R.x0[0] : R.x0[1])[je]);
}

template <typename TZ>
void launch_bgs_out(const Geom &g, const BgsArgs &B, const double *r, const double *rscale, TZ *z,
                    hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_bgs_out<TZ>), dim3(nb), dim3(kBlock), 0, st, g, B, r, rscale, z);
}
template void launch_bgs_out<double>(const Geom &, const BgsArgs &, const double *, const double *, double *,
                                     hipStream_t);
template void launch_bgs_out<float>(const Geom &, const BgsArgs &, const double *, const double *, float *,
                                    hipStream_t);

}  // namespace p4d
