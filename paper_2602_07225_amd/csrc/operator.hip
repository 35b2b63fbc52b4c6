// The linearized P4D operator y = A x (or A^T x, or b - A x) and the
// parameter-gradient kernels.
//
// A (paper Sec. 4.1, eq. blocks) per node, matrix-free:
//   phi_s rows: K_sigma phi_s + m q            (phis-weak; grounded layer: identity)
//   phi_e rows: K_kappa phi_e + chi K_kappa c_e - m q              (phie-weak)
//   c_e rows:   M_eps/dt c_e + K_kappa c_e - tc m q        (ce-weak, backward Euler)
//   c_s rows:   T0 c_s + Gamma q e_N                       (eq. FD with eq. LR)
// with the linearized reaction q = g (phi_s - phi_e) + e c_e + s c_s,N of
// the Butler-Volmer term (Sec. 2.4) and m the lumped electrode weight.
#include "p4d_device.hpp"

namespace p4d {

template <typename TX>
__device__ inline double ldx(const TX *p) { return (double)*p; }

// Loads the 27 neighbours of node (i,j,k) from a node-indexed field.
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

template <typename TX, bool TRANS, bool RESID>
__global__ __launch_bounds__(kBlock) void k_operator(
    Geom g, const RadialTab *__restrict__ tabs, const double *__restrict__ sigh,
    const double *__restrict__ kaph, const double *__restrict__ gg, const double *__restrict__ ss,
    const double *__restrict__ ee, const double *__restrict__ mm, const TX *__restrict__ x,
    double *__restrict__ y, const double *__restrict__ b, double *__restrict__ partial)
{
    __shared__ double red[4];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const long long n = (long long)lb * kBlock + threadIdx.x;
    double sq = 0.0;
    if (n < g.nnode) {
        const int i = (int)(n % g.nx);
        const long long t = n / g.nx;
        const int j = (int)(t % g.ny), k = (int)(t / g.ny);
        double ck[8], cs[8], cm[8];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + ((e >> 2) & 1);
            const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < g.nx - 1 && ej < g.ny - 1 &&
                            ek < g.nz - 1;
            const long long id = ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek);
            ck[e] = ok ? kaph[id] : 0.0;
            cs[e] = ok ? sigh[id] : 0.0;
            cm[e] = ok ? (elem_mat(g, ek) >= 0 ? g.mass_elec : g.mass_sep) : 0.0;
        }
        double X[27];
        load_nb(g, x + g.off_pe, n, i, j, k, X);
        const double Kpe = q1_stiff(ck, X);
        const double xpe = X[13];
        load_nb(g, x + g.off_ce, n, i, j, k, X);
        const double Kce = q1_stiff(ck, X);
        const double Mce = q1_mass(cm, X);
        const double xce = X[13];
        double ype, yce;
        if (!TRANS) {
            ype = Kpe + g.chi * Kce;
            yce = Mce + Kce;
        } else {
            ype = Kpe;
            yce = Mce + Kce + g.chi * Kpe;
        }
        const int el = node_mat(g, k);
        if (el >= 0) {
            const long long base = el == 0 ? 0 : g.nea;
            const int klo = el == 0 ? 0 : g.na + g.ns;
            const int khi = el == 0 ? g.na - 1 : g.nz - 1;
            const long long je = base + i + (long long)g.nx * (j + (long long)g.ny * (k - klo));
            const bool dir = (k == 0);
            // phi_s neighbours: same electrode, grounded layer as a zero column
#pragma unroll
            for (int o = 0; o < 27; o++) {
                const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                const bool ok = (i + dx >= 0) && (i + dx < g.nx) && (j + dy >= 0) &&
                                (j + dy < g.ny) && (k + dz >= klo) && (k + dz <= khi) &&
                                (k + dz != 0);
                X[o] = ok ? ldx(x + je + dx + (long long)g.nx * (dy + (long long)g.ny * dz)) : 0.0;
            }
            const double xps = ldx(x + je);
            const RadialTab &T = tabs[el];
            const int N = T.N;
            const long long nn = el == 0 ? g.nea : g.nec;
            const long long jl = je - base;
            const TX *xs = x + g.off_cs[el] + jl;
            double *ys = y + g.off_cs[el] + jl;
            const double m = mm[je], gj = gg[je], sj = ss[je], ej = ee[je];
            const double xsN = ldx(xs + (long long)(N - 1) * nn);
            // a = (m, -m, -tc m, Gamma) rows, b = (g, -g, e, s) columns
            const double a0 = dir ? 0.0 : m, b0 = dir ? 0.0 : gj;
            double q, r0, r1, r2, r3;
            if (!TRANS) {
                q = b0 * X[13] - gj * xpe + ej * xce + sj * xsN;
                r0 = a0; r1 = -m; r2 = -g.tc * m; r3 = T.Gamma;
            } else {
                q = a0 * X[13] - m * xpe - g.tc * m * xce + T.Gamma * xsN;
                r0 = b0; r1 = -gj; r2 = ej; r3 = sj;
            }
            double yps = dir ? xps : q1_stiff(cs, X) + r0 * q;
            ype += r1 * q;
            yce += r2 * q;
            if (RESID) yps = b[je] - yps;
            y[je] = yps;
            sq += yps * yps;
            // radial rows
            double xm = 0.0, x0 = ldx(xs);
            for (int r = 0; r < N; r++) {
                const double xp = r < N - 1 ? ldx(xs + (long long)(r + 1) * nn) : 0.0;
                double v;
                if (!TRANS)
                    v = T.tdia[r] * x0 + T.tsub[r] * xm + T.tsup[r] * xp;
                else
                    v = T.tdia[r] * x0 + (r > 0 ? T.tsup[r - 1] : 0.0) * xm +
                        (r < N - 1 ? T.tsub[r + 1] : 0.0) * xp;
                if (r == N - 1) v += r3 * q;
                if (RESID) v = b[g.off_cs[el] + jl + (long long)r * nn] - v;
                ys[(long long)r * nn] = v;
                sq += v * v;
                xm = x0;
                x0 = xp;
            }
        }
        if (RESID) {
            ype = b[g.off_pe + n] - ype;
            yce = b[g.off_ce + n] - yce;
        }
        y[g.off_pe + n] = ype;
        y[g.off_ce + n] = yce;
        sq += ype * ype + yce * yce;
    }
    if (partial) {
        const double s = block_sum(sq, red);
        if (threadIdx.x == 0) partial[lb] = s;
    }
}

int operator_blocks(const Geom &g) { return (int)((g.nnode + kBlock - 1) / kBlock); }

template <typename TX>
void launch_operator(const Geom &g, const RadialTab *tabs, const double *sigh, const double *kaph,
                     const double *gg, const double *ss, const double *ee, const double *mm,
                     const TX *x, double *y, const double *b, double *partial, int transpose,
                     hipStream_t st)
{
    const int nb = operator_blocks(g);
#define P4D_OP(TR, RS)                                                                    \
    hipLaunchKernelGGL((k_operator<TX, TR, RS>), dim3(nb), dim3(kBlock), 0, st, g, tabs, \
                       sigh, kaph, gg, ss, ee, mm, x, y, b, partial)
    if (!transpose) {
        if (b) P4D_OP(false, true); else P4D_OP(false, false);
    } else {
        if (b) P4D_OP(true, true); else P4D_OP(true, false);
    }
#undef P4D_OP
}
template void launch_operator<double>(const Geom &, const RadialTab *, const double *,
                                      const double *, const double *, const double *,
                                      const double *, const double *, const double *, double *,
                                      const double *, double *, int, hipStream_t);
template void launch_operator<float>(const Geom &, const RadialTab *, const double *,
                                     const double *, const double *, const double *,
                                     const double *, const double *, const float *, double *,
                                     const double *, double *, int, hipStream_t);

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
