// Physical P4D-DFN cell around the linear solve (paper Sec. 2 model with the
// appendix parameters; the Newton step of Sec. 4.1): coefficients of the
// Newton matrix from the state, the residual of one backward-Euler step and
// the update.  Every linear quantity lives in the scaled variables of the
// context (unknowns divided by x_f, equations multiplied by r_f per field),
// whose operator is D_r J D_c; the state u stays in SI units.
//   phys_elem : per element, the transport coefficients at the mean c_e of
//               its corners (sigma_eff, kappa_eff, kappa_eff 2RT(1-t+)/(F c),
//               D_e_eff), scaled and times h, into the operator's arrays;
//   phys_node : per electrode node, Butler-Volmer kinetics with the
//               open-circuit potential of the surface stoichiometry: the
//               scaled reaction q^ = r_phi a i_n and the derivative
//               coefficients g, e, s of the linearized reaction;
//   phys_fix  : residual rows from the operator's J u^: the reaction
//               correction a_j (q^_j - b_j . u^_j), the previous-step storage
//               and the applied current;
//   phys_update: u += D_c du^ with the largest scaled change per field.
#include "p4d_phys.hpp"

namespace p4d {

// graphite open-circuit potential U(theta) and dU/dtheta (appendix fit)
__device__ inline double ocp_neg(double t, double &du)
{
    const double amp[8] = {0.0351, -0.0045, -0.035, -0.0147, -0.102, -0.022, -0.011, 0.0155};
    const double cen[8] = {0.286, 0.849, 0.9233, 0.5, 0.194, 0.9, 0.124, 0.105};
    const double wid[8] = {0.083, 0.119, 0.05, 0.034, 0.142, 0.0164, 0.0226, 0.029};
    const double ex = exp(-120.0 * t);
    double u = 0.194 + 1.5 * ex;
    du = -180.0 * ex;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const double th = tanh((t - cen[q]) / wid[q]);
        u += amp[q] * th;
        du += amp[q] * (1.0 - th * th) / wid[q];
    }
    return u;
}

// LiCoO2 open-circuit potential of 1.062 theta and its theta-derivative
__device__ inline double ocp_pos(double t, double &du)
{
    const double s = 1.062 * t;
    // amp * tanh(p + q s)
    const double amp[6] = {0.07645, 2.1581, -0.14169, 0.2051, 0.2531, -0.02167};
    const double p[6] = {30.834, 52.294, 11.0923, 1.4684, 0.56478 / 0.1316, -0.525 / 0.006};
    const double qq[6] = {-54.4806, -50.294, -19.8543, -5.4888, -1.0 / 0.1316, 1.0 / 0.006};
    double u = 2.16216, d = 0.0;
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const double th = tanh(p[q] + qq[q] * s);
        u += amp[q] * th;
        d += amp[q] * qq[q] * (1.0 - th * th);
    }
    du = 1.062 * d;
    return u;
}

// bulk electrolyte conductivity and diffusivity at 298.15 K (appendix)
__device__ inline double kappa_bulk(double ce)
{
    const double c = ce / 1000.0;
    return 0.0911 + c * (1.9101 + c * (-1.052 + c * 0.1554));
}
__device__ inline double de_bulk(double ce) { return 5.34e-10 * exp(-0.65 * ce / 1000.0); }
__device__ inline double dkappa_bulk(double ce)   // d kappa / d c_e
{
    const double c = ce / 1000.0;
    return (1.9101 + c * (-2.0 * 1.052 + c * 3.0 * 0.1554)) / 1000.0;
}

__global__ __launch_bounds__(kBlock) void k_phys_elem(Geom g, PhysDev P, const double *__restrict__ u,
                                                      double *__restrict__ sigh, double *__restrict__ kaph,
                                                      double *__restrict__ kdh, double *__restrict__ dch,
                                                      double *__restrict__ nwa, double *__restrict__ nwb,
                                                      double *__restrict__ nwc)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.nelem) return;
    const int ei = (int)(t % (g.nx - 1));
    const long long r = t / (g.nx - 1);
    const int ej = (int)(r % (g.ny - 1)), ek = (int)(r / (g.ny - 1));
    const double *ce = u + g.off_ce;
    double cbar = 0.0;
#pragma unroll
    for (int b = 0; b < 8; b++)
        cbar += ce[(ei + (b & 1)) + (long long)g.nx * ((ej + ((b >> 1) & 1)) + (long long)g.ny * (ek + ((b >> 2) & 1)))];
    cbar *= 0.125;
    const int mat = elem_mat(g, ek);
    const double eps = P.por ? P.por[t] : (mat >= 0 ? P.eps_el : P.eps_sep);
    const double eb = pow(eps, P.brug);
    const double kap = eb * kappa_bulk(cbar);
    const double kd = kap * 2.0 * (1.0 - P.tplus) * P.RT / (P.F * cbar);
    const double dce = eb * de_bulk(cbar);
    const double act = P.act ? P.act[t] : (mat == 0 ? P.eps_s[0] : P.eps_s[1]);
    const double sig = mat >= 0 ? pow(act, P.brug) * (mat == 0 ? P.sigma[0] : P.sigma[1]) : 0.0;
    sigh[t] = g.h * P.rphi * P.xphi * sig;
    kaph[t] = g.h * P.rphi * P.xphi * kap;
    kdh[t] = g.h * P.rphi * P.xc * kd;
    dch[t] = g.h * P.rc * P.xc * dce;
    // derivatives with respect to the element mean c_e (Newton terms; the
    // column scale x_c of c_e and the row scales)
    const double dkap = eb * dkappa_bulk(cbar);
    const double dkd = 2.0 * (1.0 - P.tplus) * P.RT / P.F * (dkap * cbar - kap) / (cbar * cbar);
    const double ddce = eb * (-0.65 / 1000.0) * de_bulk(cbar);
    nwa[t] = g.h * P.rphi * P.xc * dkap;
    nwb[t] = g.h * P.rphi * P.xc * dkd;
    nwc[t] = g.h * P.rc * P.xc * ddce;
}

__global__ __launch_bounds__(kBlock) void k_phys_node(Geom g, PhysDev P, const double *__restrict__ u,
                                                      double *__restrict__ gg, double *__restrict__ ss,
                                                      double *__restrict__ ee, double *__restrict__ qh)
{
    const long long je = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (je >= g.ne) return;
    const int el = je < g.nea ? 0 : 1;
    const long long jl = el == 0 ? je : je - g.nea;
    const long long nn = el == 0 ? g.nea : g.nec;
    const long long n = jl + (el == 0 ? 0LL : (long long)(g.na + g.ns) * g.nx * g.ny);
    const int N = el == 0 ? g.nr[0] : g.nr[1];
    const double csmax = el == 0 ? P.csmax[0] : P.csmax[1];
    const double alpha = el == 0 ? P.alpha[0] : P.alpha[1];
    const double kr = el == 0 ? P.k[0] : P.k[1];
    const double a = el == 0 ? P.a[0] : P.a[1];
    const double phis = u[je], phie = u[g.off_pe + n], ce = u[g.off_ce + n];
    const double cs = u[(el == 0 ? g.off_cs[0] : g.off_cs[1]) + (long long)(N - 1) * nn + jl];
    double dU;
    const double U = el == 0 ? ocp_neg(cs / csmax, dU) : ocp_pos(cs / csmax, dU);
    const double f = P.F / P.RT;
    const double eta = phis - phie - U;
    const double i0 = kr * pow(ce, alpha) * pow(csmax - cs, alpha) * pow(cs, alpha);
    const double ea = exp(alpha * f * eta), ec = exp(-alpha * f * eta);
    const double in = i0 * (ea - ec);
    const double i_eta = i0 * alpha * f * (ea + ec);
    const double i_ce = alpha * in / ce;
    const double i_cs = in * (alpha / cs - alpha / (csmax - cs)) - i_eta * dU / csmax;
    gg[je] = P.rphi * P.xphi * a * i_eta;
    ee[je] = P.rphi * P.xc * a * i_ce;
    ss[je] = P.rphi * P.xs * a * i_cs;
    qh[je] = P.rphi * a * in;
}

// Case II volume fractions: porosity 1 - eps_s - eps_b and active fraction
// eps_s in electrode elements (separator: its porosity, no solid), the
// scaled storage ms * eps (ms = r_c x_c h^3 / dt) of the c_e rows; flags fractions
// outside (0, 1) or a porosity outside (0, 1]
__global__ __launch_bounds__(kBlock) void k_phys_fractions(Geom g, PhysDev P, const double *__restrict__ eps_s,
                                                           const double *__restrict__ eps_b,
                                                           double *__restrict__ por, double *__restrict__ act,
                                                           double *__restrict__ meh, double ms,
                                                           double *__restrict__ partial)
{
    __shared__ double lds[4];
    double bad = 0.0;
    for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < g.nelem;
         t += (long long)gridDim.x * kBlock) {
        const int ek = (int)(t / ((long long)(g.nx - 1) * (g.ny - 1)));
        double p = P.eps_sep, a = 0.0;
        if (elem_mat(g, ek) >= 0) {
            const double fs = eps_s[t], fb = eps_b[t];
            a = fs;
            p = 1.0 - fs - fb;
            if (!(fs > 0.0 && fs < 1.0 && fb > 0.0 && fb < 1.0 && p > 0.0 && p <= 1.0)) bad = 1.0;
        }
        por[t] = p;
        act[t] = a;
        meh[t] = ms * p;
    }
    bad = block_max(bad, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = bad;
}

// u^ = D_c^-1 u (or u = D_c u^ when up), per field
__global__ __launch_bounds__(kBlock) void k_phys_scale(Geom g, PhysDev P, const double *__restrict__ in,
                                                       double *__restrict__ out, int up)
{
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.N) return;
    const double x = i < g.off_ce ? P.xphi : (i < g.off_cs[0] ? P.xc : P.xs);
    out[i] = up ? in[i] * x : in[i] / x;
}

// residual rows: r (holding J u^ from the operator) += a_j (q^_j - b_j . u^_j)
// at electrode nodes, - old, - f; written negated when neg
__global__ __launch_bounds__(kBlock) void k_phys_fix(Geom g, PhysFix F, double *__restrict__ r, int neg)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const double sgn = neg ? -1.0 : 1.0;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const int el = node_mat(g, k);
    double rpe = r[g.off_pe + n] - F.old[g.off_pe + n];
    double rce = r[g.off_ce + n] - F.old[g.off_ce + n];
    if (el >= 0) {
        const long long base = el == 0 ? 0 : g.nea;
        const long long klo = el == 0 ? 0 : g.na + g.ns;
        const long long je = base + n - klo * g.nx * g.ny;
        const long long jl = je - base;
        const long long nn = el == 0 ? g.nea : g.nec;
        const int N = el == 0 ? g.nr[0] : g.nr[1];
        const long long offs = el == 0 ? g.off_cs[0] : g.off_cs[1];
        const bool dir = (k == 0);
        const double m = F.mm[je], gj = F.gg[je];
        const double bu = (dir ? 0.0 : gj * F.uh[je]) - gj * F.uh[g.off_pe + n] + F.ee[je] * F.uh[g.off_ce + n] +
                          F.ss[je] * F.uh[offs + (long long)(N - 1) * nn + jl];
        const double corr = F.qh[je] - bu;
        double rps = r[je] - F.old[je] - F.fh[je];
        if (!dir) rps += m * corr;
        rpe -= m * corr;
        rce -= g.tc * m * corr;
        r[je] = sgn * rps;
        const double gam = el == 0 ? F.gam[0] : F.gam[1];
        for (int q = 0; q < N; q++) {
            const long long id = offs + (long long)q * nn + jl;
            double v = r[id] - F.old[id];
            if (q == N - 1) v += gam * corr;
            r[id] = sgn * v;
        }
    }
    r[g.off_pe + n] = sgn * rpe;
    r[g.off_ce + n] = sgn * rce;
}

// u += D_c du^; per workgroup the largest |du^| over phi (x_phi is RT/F),
// c_e (x_c is c_e0) and c_s (times x_s / c_s,max of the electrode)
__global__ __launch_bounds__(kBlock) void k_phys_update(Geom g, PhysDev P, const double *__restrict__ dh,
                                                        double *__restrict__ u, double *__restrict__ partial)
{
    __shared__ double lds[4];
    double m = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * kBlock) {
        const double d = dh[i];
        double x, w;
        if (i < g.off_ce) { x = P.xphi; w = 1.0; }
        else if (i < g.off_cs[0]) { x = P.xc; w = P.xc / P.ce0; }
        else if (i < g.off_cs[1]) { x = P.xs; w = P.xs / P.csmax[0]; }
        else { x = P.xs; w = P.xs / P.csmax[1]; }
        u[i] += x * d;
        m = fmax(m, fabs(d) * w);
    }
    m = block_max(m, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// the rest state: c_e0, c_s0, phi_s = 0 (negative), phi_e = -U_n, phi_s = U_p - U_n
__global__ __launch_bounds__(kBlock) void k_phys_init(Geom g, PhysDev P, double *__restrict__ u)
{
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.N) return;
    double d;
    const double un = ocp_neg(P.cs0[0] / P.csmax[0], d);
    const double up = ocp_pos(P.cs0[1] / P.csmax[1], d);
    double v;
    if (i < g.nea) v = 0.0;
    else if (i < g.ne) v = up - un;
    else if (i < g.off_ce) v = -un;
    else if (i < g.off_cs[0]) v = P.ce0;
    else if (i < g.off_cs[1]) v = P.cs0[0];
    else v = P.cs0[1];
    u[i] = v;
}

// SI residual rows from scaled ones: R = D_r^-1 R^ (grounded phi_s rows are
// identity rows in the scaled variables: R = x_phi R^)
__global__ __launch_bounds__(kBlock) void k_phys_unscale_rows(Geom g, PhysDev P, const double *__restrict__ rh,
                                                              double *__restrict__ r)
{
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.N) return;
    double f;
    if (i < (long long)g.nx * g.ny) f = P.xphi;
    else if (i < g.off_ce) f = 1.0 / P.rphi;
    else if (i < g.off_cs[0]) f = 1.0 / P.rc;
    else f = 1.0 / P.rs;
    r[i] = rh[i] * f;
}

// previous-step storage of the particle rows: c_s,old^ / dt' (scaled)
__global__ __launch_bounds__(kBlock) void k_phys_old_cs(Geom g, PhysDev P, const double *__restrict__ uold,
                                                       double dtp, double *__restrict__ old)
{
    const long long i = g.off_cs[0] + (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.N) return;
    old[i] = uold[i] / (P.xs * dtp);
}

static int blocks(long long n) { return (int)((n + kBlock - 1) / kBlock); }

void launch_phys_old_cs(const Geom &g, const PhysDev &P, const double *uold, double dtp, double *old,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_phys_old_cs, dim3(blocks(g.N - g.off_cs[0])), dim3(kBlock), 0, st, g, P, uold, dtp,
                       old);
}

void launch_phys_coef(const Geom &g, const PhysDev &P, const double *u, double *sigh, double *kaph,
                      double *kdh, double *dch, double *gg, double *ss, double *ee, double *qh,
                      double *nwa, double *nwb, double *nwc, hipStream_t st)
{
    hipLaunchKernelGGL(k_phys_elem, dim3(blocks(g.nelem)), dim3(kBlock), 0, st, g, P, u, sigh, kaph, kdh,
                       dch, nwa, nwb, nwc);
    hipLaunchKernelGGL(k_phys_node, dim3(blocks(g.ne)), dim3(kBlock), 0, st, g, P, u, gg, ss, ee, qh);
}

void launch_phys_scale(const Geom &g, const PhysDev &P, const double *in, double *out, int up,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_phys_scale, dim3(blocks(g.N)), dim3(kBlock), 0, st, g, P, in, out, up);
}

void launch_phys_fix(const Geom &g, const PhysFix &F, double *r, int neg, hipStream_t st)
{
    hipLaunchKernelGGL(k_phys_fix, dim3(blocks(g.nnode)), dim3(kBlock), 0, st, g, F, r, neg);
}

int launch_phys_update(const Geom &g, const PhysDev &P, const double *dh, double *u, double *partial,
                       hipStream_t st)
{
    const int nb = stream_blocks(g.N);
    hipLaunchKernelGGL(k_phys_update, dim3(nb), dim3(kBlock), 0, st, g, P, dh, u, partial);
    return nb;
}

void launch_phys_init(const Geom &g, const PhysDev &P, double *u, hipStream_t st)
{
    hipLaunchKernelGGL(k_phys_init, dim3(blocks(g.N)), dim3(kBlock), 0, st, g, P, u);
}

int launch_phys_fractions(const Geom &g, const PhysDev &P, const double *eps_s, const double *eps_b,
                          double *por, double *act, double *meh, double ms, double *partial, hipStream_t st)
{
    const int nb = stream_blocks(g.nelem);
    hipLaunchKernelGGL(k_phys_fractions, dim3(nb), dim3(kBlock), 0, st, g, P, eps_s, eps_b, por, act, meh,
                       ms, partial);
    return nb;
}

void launch_phys_unscale_rows(const Geom &g, const PhysDev &P, const double *rh, double *r, hipStream_t st)
{
    hipLaunchKernelGGL(k_phys_unscale_rows, dim3(blocks(g.N)), dim3(kBlock), 0, st, g, P, rh, r);
}

}  // namespace p4d
