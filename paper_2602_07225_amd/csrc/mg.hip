// Geometric Galerkin multigrid for the electrode-level blocks (in place of
// the paper's BoomerAMG V-cycle, Sec. 4.2).  Four node boxes are processed
// together in every launch: phi_s anode (layers 1..na-1, the grounded layer
// eliminated), phi_s cathode, phi_e and c_e.  Each box operator is the
// field-block diagonal of the Schur complement,
//   S_f = A_diff,ff + diag(omega_j a_f,j b_f,j),
// applied matrix-free from element coefficients on the finest level and as
// a stored 27-point Galerkin stencil S_{l+1} = P^T S_l P on coarser levels.
// Smoother: Chebyshev on D^-1 S over [lmax/4, lmax] (lmax: Gershgorin bound),
// one fused kernel per step.  Coarsening per direction keeps the even indices
// plus the last one; P is tensor-product linear interpolation.
#include "p4d_kernels.hpp"

namespace p4d {

// ---------------------------------------------------------------------------
// Single-cell kernels: all four boxes of one V-cycle stage per launch
// ---------------------------------------------------------------------------
template <typename T, bool RESID_ONLY, bool MEH>
__global__ __launch_bounds__(kBlock) void k_smooth0(Geom g, LevelBatch<T> lb, int TX, int CZ)
{
    __shared__ Smooth0Lds L;
    const int bx = find_box(lb, blockIdx.x);
    const LevelArgs<T> &A = lb.a[bx];
    const int nt = smooth0_box_tiles(A.nx, A.ny, A.nz, TX, CZ);
    smooth0_tile<T, RESID_ONLY, MEH>(g, A, xcd_block(blockIdx.x - A.blk0, nt), TX, CZ, L);
}

int smooth0_tiles(int nx, int ny, int nz, int TX, int CZ) { return smooth0_box_tiles(nx, ny, nz, TX, CZ); }

// workgroups of the level-0 smoother resident at once on the current device
int smooth0_slots()
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_smooth0<double, false, false>,
                                                     kBlock, 0) != hipSuccess)
        return 1024;
    return (per < 1 ? 1 : per) * (ncu < 1 ? 1 : ncu);
}

template <typename T>
void launch_smooth0(const Geom &g, const LevelBatch<T> &lb, int nblk, int resid_only, int TX,
                    int CZ, hipStream_t st)
{
    if (g.meh || g.aniso) {
        if (resid_only)
            hipLaunchKernelGGL((k_smooth0<T, true, true>), dim3(nblk), dim3(kBlock), 0, st, g, lb, TX, CZ);
        else
            hipLaunchKernelGGL((k_smooth0<T, false, true>), dim3(nblk), dim3(kBlock), 0, st, g, lb, TX, CZ);
    } else if (resid_only) {
        hipLaunchKernelGGL((k_smooth0<T, true, false>), dim3(nblk), dim3(kBlock), 0, st, g, lb, TX, CZ);
    } else {
        hipLaunchKernelGGL((k_smooth0<T, false, false>), dim3(nblk), dim3(kBlock), 0, st, g, lb, TX, CZ);
    }
}
template void launch_smooth0<double>(const Geom &, const LevelBatch<double> &, int, int, int, int,
                                     hipStream_t);
template void launch_smooth0<float>(const Geom &, const LevelBatch<float> &, int, int, int, int,
                                    hipStream_t);

template <typename T, bool RESID_ONLY>
__global__ __launch_bounds__(kBlock) void k_smooth(LevelBatch<T> lb)
{
    const int bx = find_box(lb, blockIdx.x);
    const LevelArgs<T> &A = lb.a[bx];
    const int nblk = (A.n + kBlock - 1) / kBlock;
    smooth_block<T, RESID_ONLY>(A, xcd_block(blockIdx.x - A.blk0, nblk));
}

template <typename T>
void launch_smooth(const LevelBatch<T> &lb, int nblk, int resid_only, hipStream_t st)
{
    if (resid_only)
        hipLaunchKernelGGL((k_smooth<T, true>), dim3(nblk), dim3(kBlock), 0, st, lb);
    else
        hipLaunchKernelGGL((k_smooth<T, false>), dim3(nblk), dim3(kBlock), 0, st, lb);
}
template void launch_smooth<double>(const LevelBatch<double> &, int, int, hipStream_t);
template void launch_smooth<float>(const LevelBatch<float> &, int, int, hipStream_t);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(TransferBatch<T> tb)
{
    const int bx = find_box(tb, blockIdx.x);
    restrict_block<T>(tb.a[bx], blockIdx.x - tb.a[bx].blk0);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(TransferBatch<T> tb)
{
    const int bx = find_box(tb, blockIdx.x);
    prolong_block<T>(tb.a[bx], blockIdx.x - tb.a[bx].blk0);
}
template <typename T>
void launch_restrict(const TransferBatch<T> &tb, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL((k_restrict<T>), dim3(nblk), dim3(kBlock), 0, st, tb);
}
template <typename T>
void launch_prolong(const TransferBatch<T> &tb, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL((k_prolong<T>), dim3(nblk), dim3(kBlock), 0, st, tb);
}
template void launch_restrict<double>(const TransferBatch<double> &, int, hipStream_t);
template void launch_restrict<float>(const TransferBatch<float> &, int, hipStream_t);
template void launch_prolong<double>(const TransferBatch<double> &, int, hipStream_t);
template void launch_prolong<float>(const TransferBatch<float> &, int, hipStream_t);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(CoarseBatch<T> cb)
{
    __shared__ CoarseLds L;
    const int box = blockIdx.y;
    if (box >= cb.nbox) return;
    if (blockIdx.x * 64 >= cb.a[box].n) return;
    coarse_block<T>(cb.a[box], blockIdx.x, L);
}

template <typename T>
void launch_coarse(const CoarseBatch<T> &cb, hipStream_t st)
{
    int nmax = 1;
    for (int b = 0; b < cb.nbox; b++) nmax = cb.a[b].n > nmax ? cb.a[b].n : nmax;
    hipLaunchKernelGGL((k_coarse<T>), dim3((nmax + 63) / 64, cb.nbox), dim3(kBlock), 0, st, cb);
}
template void launch_coarse<double>(const CoarseBatch<double> &, hipStream_t);
template void launch_coarse<float>(const CoarseBatch<float> &, hipStream_t);

// Tail of the V-cycle, one 1024-thread workgroup per box (see TailArgs).  The
// per-stage device functions run here on LDS arrays through generic
// pointers: node n of a stage is base + threadIdx.x over bases stepping by
// the workgroup size, which is what smooth_block / restrict_block /
// prolong_block compute from a block index base / kBlock.
template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailBatch<T> tb)
{
    __shared__ __align__(16) char lds[kTailLds];
    if ((int)blockIdx.x >= tb.nbox) return;
    const TailArgs<T> &A = tb.a[blockIdx.x];
    const int n = A.n, nc = A.nc, deg = tb.deg;
    // doubles: x1 and the coarse inverse first (filled together), then the
    // second iterate buffer, the coarse solution and the partial sums; then
    // the stencil, inverse diagonal and right-hand side (filled together),
    // direction, residual and coarse right-hand side in T
    double *xa = (double *)lds;
    double *Ainv = xa + n;             // [nc][nc] coarse inverse
    double *xb = Ainv + nc * nc;
    double *xc = xb + n;
    double *part = xc + nc;            // [4][nc] partial sums of the coarse solve
    T *S = (T *)(part + 4 * nc);
    T *invd = S + 14 * n;
    T *b = invd + n;
    T *d = b + n;
    T *r = d + n;
    T *bc = r + n;
    {   // every global load is issued, kU per thread and array group, before
        // any of them is stored to LDS (a load-store loop waits for each)
        constexpr int kU = 8;
        const int cT = 16 * n, cD = n + nc * nc;
        const int cmax = cT > cD ? cT : cD;
        for (int base = 0; base < cmax; base += kU * kTailThreads) {
            T vt[kU];
            double vd[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                // indexes clamped into range and sources chosen by select, so
                // that the loads are issued without branches (stored only if
                // q is in range)
                const int q = base + u * kTailThreads + (int)threadIdx.x;
                const int qt = q < cT ? q : cT - 1, qd = q < cD ? q : cD - 1;
                const T *pt = qt < 14 * n ? A.S + qt : (qt < 15 * n ? A.invd + (qt - 14 * n) : A.b + (qt - 15 * n));
                const double *pd = qd < n ? A.x1 + qd : A.Ainv + (qd - n);
                vt[u] = *pt;
                vd[u] = *pd;
            }
#pragma unroll
            for (int u = 0; u < kU; u++) {
                const int q = base + u * kTailThreads + (int)threadIdx.x;
                if (q < cT) S[q] = vt[u];
                if (q < cD) xa[q] = vd[u];
            }
        }
    }
    __syncthreads();
    LevelArgs<T> L{};
    L.nx = A.nx; L.ny = A.ny; L.nz = A.nz; L.n = n;
    L.S = S; L.invd = invd; L.b = b; L.din = d;
    int cur = 0;   // 0: the iterate is in xa
    auto smooth = [&](int t, bool post) {
        L.xin = cur ? xb : xa;
        L.xout = cur ? xa : xb;
        L.c1 = A.c1[t];
        L.c2 = A.c2[t];
        // (first pre-smoothing step from x = 0: its direction is x itself)
        L.din_x = (!post && t == 2) ? 1 : 0;
        L.dout = t < deg ? d : nullptr;
        L.rout = nullptr;
        for (int base = 0; base < n; base += kTailThreads) smooth_block<T, false>(L, base / kBlock);
        __syncthreads();
        cur ^= 1;
    };
    for (int t = 2; t <= deg; t++) smooth(t, false);
    L.xin = cur ? xb : xa;
    L.rout = r;
    for (int base = 0; base < n; base += kTailThreads) smooth_block<T, true>(L, base / kBlock);
    __syncthreads();
    TransferArgs<T> P{};
    P.fx = A.nx; P.fy = A.ny; P.fz = A.nz;
    P.cx = A.cx; P.cy = A.cy; P.cz = A.cz;
    P.rf = r;
    P.bc = bc;
    P.xc1 = nullptr;
    for (int base = 0; base < nc; base += kTailThreads) restrict_block<T>(P, base / kBlock);
    __syncthreads();
    // x_c = Ainv b_c with the per-stage coarse kernel's summation: four
    // partial sums over the columns c = w (mod 4), ascending, then paired
    for (int q = threadIdx.x; q < 4 * nc; q += kTailThreads) {
        const int w = q / nc, row = q - w * nc;
        double acc = 0.0;
        for (int c = w; c < nc; c += 4) acc += Ainv[c * nc + row] * (double)bc[c];
        part[w * nc + row] = acc;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nc; q += kTailThreads)
        xc[q] = (part[q] + part[nc + q]) + (part[2 * nc + q] + part[3 * nc + q]);
    __syncthreads();
    P.xc = xc;
    P.xf = cur ? xb : xa;
    for (int base = 0; base < n; base += kTailThreads) prolong_block<T>(P, base / kBlock);
    __syncthreads();
    for (int t = 1; t <= deg; t++) smooth(t, true);
    const double *xf = cur ? xb : xa;
    for (int q = threadIdx.x; q < n; q += kTailThreads) A.xout[q] = xf[q];
}

template <typename T>
void launch_tail(const TailBatch<T> &tb, hipStream_t st)
{
    hipLaunchKernelGGL((k_tail<T>), dim3(tb.nbox), dim3(kTailThreads), 0, st, tb);
}
template void launch_tail<double>(const TailBatch<double> &, hipStream_t);
template void launch_tail<float>(const TailBatch<float> &, hipStream_t);

// ---------------------------------------------------------------------------
// Setup kernels (FP64)
// ---------------------------------------------------------------------------
// per element: h sigma (electrode elements only), h kappa; per electrode node:
// the lumped weight m_j = (vol/8) * #(electrode elements containing j)
__global__ __launch_bounds__(kBlock) void k_setup_nodes(Geom g, const double *__restrict__ sigma,
                                                        const double *__restrict__ kappa,
                                                        double *__restrict__ sigh,
                                                        double *__restrict__ kaph,
                                                        double *__restrict__ mm)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < g.nelem) {
        const long long u = t / (g.nx - 1);
        const int ek = (int)(u / (g.ny - 1));
        sigh[t] = elem_mat(g, ek) >= 0 ? g.h * sigma[t] : 0.0;
        kaph[t] = g.h * kappa[t];
    }
    if (t < g.ne) {
        const int el = t < g.nea ? 0 : 1;
        const long long jl = el == 0 ? t : t - g.nea;
        const int i = (int)(jl % g.nx);
        const long long u = jl / g.nx;
        const int j = (int)(u % g.ny);
        const int k = (int)(u / g.ny) + (el == 0 ? 0 : g.na + g.ns);
        const int cx = (i > 0) + (i < g.nx - 1), cy = (j > 0) + (j < g.ny - 1);
        int cz = 0;
        if (k - 1 >= 0 && elem_mat(g, k - 1) == el) cz++;
        if (k < g.nz - 1 && elem_mat(g, k) == el) cz++;
        mm[t] = g.vol / 8.0 * (double)(cx * cy * cz);
    }
}

__global__ __launch_bounds__(kBlock) void k_scale_elem(long long n, const double *__restrict__ in,
                                                       double factor, const double *__restrict__ def,
                                                       double *__restrict__ out)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) out[t] = factor * (in ? in[t] : def[t]);
}

void launch_scale_elem(const Geom &g, const double *in, double factor, const double *def, double *out,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_elem, dim3((int)((g.nelem + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       g.nelem, in, factor, def, out);
}

void launch_setup_nodes(const Geom &g, const RadialTab *, const double *sigma, const double *kappa,
                        double *sigh, double *kaph, double *mm, hipStream_t st)
{
    const long long n = g.nelem > g.ne ? g.nelem : g.ne;
    hipLaunchKernelGGL(k_setup_nodes, dim3((int)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       g, sigma, kappa, sigh, kaph, mm);
}

// omega_j = 1 / (1 + Gamma s_j tau0) (Sherman-Morrison: 1 - Gamma s_j (A_ss,j^-1)_NN)
__global__ __launch_bounds__(kBlock) void k_omega(Geom g, const RadialTab *__restrict__ tabs,
                                                  const double *__restrict__ ss, int schur,
                                                  double *__restrict__ om)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.ne) return;
    const RadialTab &T = tabs[t < g.nea ? 0 : 1];
    om[t] = schur ? 1.0 / (1.0 + T.Gamma * ss[t] * T.tau0) : 1.0;
}

void launch_omega(const Geom &g, const RadialTab *tabs, const double *ss, int schur, double *om,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_omega, dim3((int)((g.ne + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, g,
                       tabs, ss, schur, om);
}

// diagonal reaction correction of the box operators, macro layout:
// phi_s, phi_e: omega m g; c_e: -omega tc m e (zero off the electrodes)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dcorr(Geom g, const double *__restrict__ gg,
                                                  const double *__restrict__ ee,
                                                  const double *__restrict__ mm,
                                                  const double *__restrict__ om, T *__restrict__ dc)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnode) return;
    const int k = (int)(n / ((long long)g.nx * g.ny));
    const int el = node_mat(g, k);
    double dpe = 0.0, dce = 0.0;
    if (el >= 0) {
        const long long je = (el == 0 ? 0 : g.nea) + n - (long long)(el == 0 ? 0 : g.na + g.ns) * g.nx * g.ny;
        const double w = om[je] * mm[je];
        dpe = w * gg[je];
        dce = -g.tc * w * ee[je];
        dc[je] = (T)(k == 0 ? 0.0 : dpe);
    }
    dc[g.off_pe + n] = (T)dpe;
    dc[g.off_ce + n] = (T)dce;
}

template <typename T>
void launch_dcorr(const Geom &g, const double *gg, const double *ee, const double *mm,
                  const double *omega, T *dcorr0, hipStream_t st)
{
    hipLaunchKernelGGL((k_dcorr<T>), dim3((int)((g.nnode + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, g, gg, ee, mm, omega, dcorr0);
}
template void launch_dcorr<double>(const Geom &, const double *, const double *, const double *,
                                   const double *, double *, hipStream_t);
template void launch_dcorr<float>(const Geom &, const double *, const double *, const double *,
                                  const double *, float *, hipStream_t);

// row n (box-local) of the level-0 operator of one box, 27-point pattern
__device__ inline void assemble0_row(const Geom &g, const Elem0 &E, int n, double row[27])
{
    const int nzb = E.nzb, k0 = E.k0, ek_lo = E.ek_lo, ek_hi = E.ek_hi, mass = E.mass;
    const double *cK = E.cK, *dcorr = E.dcorr;
    const int i = n % g.nx, t = n / g.nx;
    const int j = t % g.ny, kl = t / g.ny;
    const int k = kl + k0;
#pragma unroll
    for (int o = 0; o < 27; o++) row[o] = 0.0;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
        const bool ok = ei >= 0 && ej >= 0 && ei < g.nx - 1 && ej < g.ny - 1 && ek >= ek_lo &&
                        ek <= ek_hi;
        const long long id = ei + (long long)(g.nx - 1) * (ej + (long long)(g.ny - 1) * ek);
        const double c = ok ? cK[id] : 0.0;
        const double cm = (ok && mass) ? elem_storage(g, id, ek) : 0.0;
        const int a = (1 - ex) | ((1 - ey) << 1) | ((1 - ez) << 2);
#pragma unroll
        for (int bb = 0; bb < 8; bb++) {
            const int dx = ex - 1 + (bb & 1), dy = ey - 1 + ((bb >> 1) & 1), dz = ez - 1 + ((bb >> 2) & 1);
            const int d = popc3(a ^ bb);
            const double kab = g.aniso ? (d == 0 ? g.kw[0] : -g.kw[a ^ bb])
                                       : (d == 0 ? 1.0 / 3.0 : (d == 1 ? 0.0 : -1.0 / 12.0));
            const double mab = d == 0 ? 8.0 / 216 : d == 1 ? 4.0 / 216 : d == 2 ? 2.0 / 216 : 1.0 / 216;
            const bool in = (kl + dz >= 0) && (kl + dz < nzb);
            if (in) row[nb_index(dx, dy, dz)] += c * kab + cm * mab;
        }
    }
    row[13] += dcorr[n];
}

// 27-point stencil (SoA [27][n]) of the level-0 operator of one box
__global__ __launch_bounds__(kBlock) void k_assemble0(Geom g, int nzb, int k0, int ek_lo, int ek_hi,
                                                      int mass, const double *__restrict__ cK,
                                                      const double *__restrict__ dcorr,
                                                      double *__restrict__ S)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    const int nb = g.nx * g.ny * nzb;
    if (n >= nb) return;
    double row[27];
    assemble0_row(g, Elem0{nzb, k0, ek_lo, ek_hi, mass, cK, dcorr}, n, row);
#pragma unroll
    for (int o = 0; o < 27; o++) S[(long long)o * nb + n] = row[o];
}

void launch_assemble0(const Geom &g, int, int nz, int k0, int ek_lo, int ek_hi, int mass,
                      const double *cK, const double *dcorr, double *S, hipStream_t st)
{
    const int nb = g.nx * g.ny * nz;
    hipLaunchKernelGGL(k_assemble0, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g, nz,
                       k0, ek_lo, ek_hi, mass, cK, dcorr, S);
}

// Galerkin coarse stencil S_c = P^T S P with P = P_x (x) P_y (x) P_z, done as
// three 1D Galerkin coarsenings (along x, then y, then z): each keeps the
// 27-point pattern.  Along the coarsened axis, coarse row I gathers the fine
// rows g1 in {c-1, c, c+1} around its fine point c, each with weight
// P(g1, I), and the fine couplings g1 -> g1 + da land on coarse offsets dJ
// with weight P(g1 + da, I + dJ); all loops have fixed trip counts and the
// weights are computed by selects, so there is no divergent branching.

// 1D interpolation weight P(g, J) of the 'even indices plus the last' rule
__device__ inline double pweight(int n, int g, int J)
{
    if (g < 0 || g >= n) return 0.0;
    if (n <= 2) return g == J ? 1.0 : 0.0;
    if (!(g & 1)) return (g >> 1) == J ? 1.0 : 0.0;
    if (g == n - 1) return (n >> 1) == J ? 1.0 : 0.0;
    return ((g - 1) >> 1) == J || ((g + 1) >> 1) == J ? 0.5 : 0.0;
}

// stencil slot of offset a along axis AX and (d1, d2) along the other two
template <int AX>
__device__ constexpr int slot_ax(int a, int d1, int d2)
{
    return nb_index(AX == 0 ? a : d1, AX == 0 ? d1 : (AX == 1 ? a : d2), AX == 2 ? a : d2);
}

// ELEM (x pass of the first coarsening only): the fine rows are formed from
// the level-0 element data instead of read from a stored stencil
template <int AX, bool ELEM>
__global__ __launch_bounds__(kBlock) void k_rap1d(Geom g, RapBatch rb)
{
    const RapArgs &A = rb.a[find_box(rb, blockIdx.x)];
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int fa = AX == 0 ? nx : (AX == 1 ? ny : nz);
    const int ca = coarse_n(fa);
    const int ox = AX == 0 ? ca : nx, oy = AX == 1 ? ca : ny, oz = AX == 2 ? ca : nz;
    const int no = ox * oy * oz, nf = nx * ny * nz;
    const int n = (blockIdx.x - A.blk0) * kBlock + threadIdx.x;
    if (n >= no) return;
    const int I0 = n % ox, t = n / ox, J0 = t % oy, K0 = t / oy;
    const int Ia = AX == 0 ? I0 : (AX == 1 ? J0 : K0);   // coarse index along AX
    const int c = fa <= 2 ? Ia : (Ia == ca - 1 ? fa - 1 : 2 * Ia);
    double acc[27];
#pragma unroll
    for (int o = 0; o < 27; o++) acc[o] = 0.0;
#pragma unroll 1
    for (int q = 0; q < 3; q++) {   // one fine row at a time keeps 27 loads in flight
        const int g1 = c - 1 + q;
        const double w1 = pweight(fa, g1, Ia);
        const int gc = g1 < 0 ? 0 : (g1 >= fa ? fa - 1 : g1);   // any valid row when w1 = 0
        const int i = AX == 0 ? gc : I0, j = AX == 1 ? gc : J0, k = AX == 2 ? gc : K0;
        const long long row = i + (long long)nx * (j + (long long)ny * k);
        const double *__restrict__ S = A.Sf;
        double sv[27];
        if (ELEM) {
            assemble0_row(g, A.e0, (int)row, sv);
        } else {
#pragma unroll
            for (int o = 0; o < 27; o++) sv[o] = S[(long long)o * nf + row];
        }
#pragma unroll
        for (int da = -1; da <= 1; da++) {
            double W[3];
#pragma unroll
            for (int dJ = -1; dJ <= 1; dJ++) W[dJ + 1] = w1 * pweight(fa, g1 + da, Ia + dJ);
#pragma unroll
            for (int m = 0; m < 9; m++) {
                const int d1 = m % 3 - 1, d2 = m / 3 - 1;
                const double v = sv[slot_ax<AX>(da, d1, d2)];
#pragma unroll
                for (int dJ = -1; dJ <= 1; dJ++) acc[slot_ax<AX>(dJ, d1, d2)] += W[dJ + 1] * v;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 27; o++) A.Sc[(long long)o * no + n] = acc[o];
}

// P^T S P for up to four boxes at once; job b needs job.tmp with room for
// 27 * (cx*fy*fz + cx*cy*fz) doubles
void launch_rap(const Geom &g, const RapJob *jobs, int njobs, int zc, hipStream_t st)
{
    RapBatch r[3] = {};
    int blk[3] = {0, 0, 0};
    for (int a = 0; a < 3; a++) r[a].nbox = njobs;
    for (int b = 0; b < njobs; b++) {
        const RapJob &J = jobs[b];
        const int cx = coarse_n(J.fx), cy = coarse_n(J.fy), cz = coarse_n(J.fz);
        double *t1 = J.tmp;                                  // (cx, fy, fz)
        double *t2 = J.tmp + 27LL * cx * J.fy * J.fz;        // (cx, cy, fz)
        const int n1 = cx * J.fy * J.fz, n2 = cx * cy * J.fz, n3 = cx * cy * cz;
        r[0].a[b] = RapArgs{J.fx, J.fy, J.fz, blk[0], J.Sf, t1, J.e0};
        r[1].a[b] = RapArgs{cx, J.fy, J.fz, blk[1], t1, zc ? t2 : J.Sc, Elem0{}};
        r[2].a[b] = RapArgs{cx, cy, J.fz, blk[2], t2, J.Sc, Elem0{}};
        blk[0] += (n1 + kBlock - 1) / kBlock;
        blk[1] += (n2 + kBlock - 1) / kBlock;
        blk[2] += (n3 + kBlock - 1) / kBlock;
    }
    if (!njobs) return;
    if (jobs[0].Sf) hipLaunchKernelGGL((k_rap1d<0, false>), dim3(blk[0]), dim3(kBlock), 0, st, g, r[0]);
    else hipLaunchKernelGGL((k_rap1d<0, true>), dim3(blk[0]), dim3(kBlock), 0, st, g, r[0]);
    hipLaunchKernelGGL((k_rap1d<1, false>), dim3(blk[1]), dim3(kBlock), 0, st, g, r[1]);
    if (zc) hipLaunchKernelGGL((k_rap1d<2, false>), dim3(blk[2]), dim3(kBlock), 0, st, g, r[2]);
}

// ---------------------------------------------------------------------------
// z-line block Gauss-Seidel (boxes much thinner along z than across).  The
// lines of a colour (every other line in x and y) are cut into tiles of LT
// lines that are consecutive along x; Sz holds a tile's rows together,
// layer by layer, and in a layer the 27 coefficients of its lines one after
// the other, so that a workgroup streams one contiguous block of the stencil
// (runs of a few lines per coefficient and layer read back poorly from HBM).
// The workgroup marches through z in chunks of KC layers: it stages the x
// planes around the tile (2 LT + 1 by 3 nodes, layers k0 - 1 .. k0 + KC) in
// LDS; its threads form, one (line, layer) each, the right-hand side with
// the couplings to other lines moved over (lines of one colour do not
// couple) and copy the line's tridiagonal block (offsets (0,0,-1), centre,
// (0,0,1)).  Then one thread per line eliminates down the line and
// substitutes back up in LDS, and all threads write x.  LDS [k][line] keeps
// the threads of the elimination on consecutive banks.
// ---------------------------------------------------------------------------
// Sz index of coefficient o of the row of line (a, bl) of a colour in layer
// k; base = 27 x the rows of the lower colours, ncx the colour's lines
// along x, LT the tile width
__device__ inline long long zline_index(long long base, int ncx, int nz, int LT, int a, int bl, int k, int o)
{
    const int a0 = a - a % LT;
    const int w = ncx - a0 < LT ? ncx - a0 : LT;
    return base + ((long long)bl * ncx + a0) * 27 * nz + (long long)(k * 27 + o) * w + (a - a0);
}

__device__ inline long long zline_rows_below(int nx, int ny, int nz, int colour)
{
    long long offc = 0;
    for (int c = 0; c < colour; c++)
        offc += (long long)((nx - (c & 1) + 1) / 2) * ((ny - (c >> 1) + 1) / 2) * nz;
    return offc;
}

__global__ __launch_bounds__(kBlock) void k_zline(LineBatch lb, int colour)
{
    extern __shared__ double lds[];
    const LineArgs &A = lb.a[find_box(lb, blockIdx.x)];
    const int LT = A.lt, KC = A.kc;   // KC * LT <= kBlock
    const int cx = colour & 1, cy = colour >> 1;
    const int ncx = (A.nx - cx + 1) / 2;
    const int tX = (ncx + LT - 1) / LT;
    const int tile = blockIdx.x - A.blk0;
    const int a0 = (tile % tX) * LT, bl = tile / tX;
    const int w = ncx - a0 < LT ? ncx - a0 : LT;   // lines in this tile
    const int FX = 2 * LT + 1, plane = 3 * FX;
    const int fi0 = cx + 2 * a0 - 1, fj0 = cy + 2 * bl - 1;   // footprint origin (node indices)
    const int nz = A.nz;
    const long long layer = (long long)A.nx * A.ny;
    const double *Z = A.Sz + 27 * zline_rows_below(A.nx, A.ny, nz, colour) + ((long long)bl * ncx + a0) * 27 * nz;
    double *Llo = lds, *Ldg = lds + LT * nz, *Lup = Ldg + LT * nz, *Lrh = Lup + LT * nz;
    double *Lx = Lrh + LT * nz;   // [KC + 2][3][FX]
    const int j = cy + 2 * bl;
    for (int k0 = 0; k0 < nz; k0 += KC) {
        for (int q = threadIdx.x; q < (KC + 2) * plane; q += kBlock) {
            const int pl = q / plane, r = q - pl * plane;
            const int ii = fi0 + r % FX, jj = fj0 + r / FX, kk = k0 - 1 + pl;
            const bool ok = ii >= 0 && ii < A.nx && jj >= 0 && jj < A.ny && kk >= 0 && kk < nz;
            Lx[q] = ok ? A.x[ii + (long long)A.nx * jj + layer * kk] : 0.0;
        }
        __syncthreads();
        {
            const int l = threadIdx.x % LT, kk = threadIdx.x / LT, k = k0 + kk;
            if (kk < KC && k < nz && l < w) {
                const int i = cx + 2 * (a0 + l);
                const long long n = i + (long long)A.nx * j + layer * k;
                const double *Zr = Z + (long long)k * 27 * w + l;   // coefficient o at Zr[o * w]
                const double *P = Lx + (kk + 1) * plane + (i - fi0) + FX;
                double rhs = A.b[n];
                // no bounds tests: Sz holds +0 for a neighbour off the box and
                // the staged x is +0 there, so that such a term subtracts an
                // exact -0 and leaves rhs as it is, bit for bit; unguarded,
                // the loads are all in flight at once
#pragma unroll
                for (int o = 0; o < 27; o++) {
                    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                    if (dx == 0 && dy == 0) continue;
                    rhs -= Zr[o * w] * P[dx + FX * dy + plane * dz];
                }
                const int q = k * LT + l;
                Llo[q] = Zr[4 * w];    // offset (0,0,-1), +0 in the bottom layer
                Lup[q] = Zr[22 * w];   // offset (0,0,+1), +0 in the top layer
                Ldg[q] = Zr[13 * w];
                Lrh[q] = rhs;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < w) {
        // the next row's values are read one step ahead (ahead of this
        // step's stores), so that the LDS latency leaves the chain of
        // dependent divisions
        const int ll = threadIdx.x;
        double cprev = 0.0, dprev = 0.0;
        double lo = Llo[ll], dg = Ldg[ll], up = Lup[ll], rh = Lrh[ll];
        for (int k = 0; k < nz; k++) {
            const int q = k * LT + ll;
            const int qn = k + 1 < nz ? q + LT : q;
            const double lo1 = Llo[qn], dg1 = Ldg[qn], up1 = Lup[qn], rh1 = Lrh[qn];
            const double den = dg - lo * cprev;
            cprev = up / den;
            dprev = (rh - lo * dprev) / den;
            Lup[q] = cprev;
            Lrh[q] = dprev;
            lo = lo1; dg = dg1; up = up1; rh = rh1;
        }
        double nxt = 0.0;
        double c = Lup[(nz - 1) * LT + ll], d = Lrh[(nz - 1) * LT + ll];
        for (int k = nz - 1; k >= 0; k--) {
            const int q = k * LT + ll;
            const int qn = k > 0 ? q - LT : q;
            const double c1 = Lup[qn], d1 = Lrh[qn];
            nxt = d - (k < nz - 1 ? c * nxt : 0.0);
            Lrh[q] = nxt;
            c = c1; d = d1;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < LT * nz; p += kBlock) {
        const int l = p % LT, k = p / LT;
        if (l >= w) continue;
        A.x[cx + 2 * (a0 + l) + (long long)A.nx * j + layer * k] = Lrh[k * LT + l];
    }
}

__global__ __launch_bounds__(kBlock) void k_resid_full(LineBatch lb)
{
    const LineArgs &A = lb.a[find_box(lb, blockIdx.x)];
    const int n = (blockIdx.x - A.blk0) * kBlock + threadIdx.x;
    if (n >= A.n) return;
    const int i = n % A.nx, t = n / A.nx, j = t % A.ny, k = t / A.ny;
    const long long layer = (long long)A.nx * A.ny, N = A.n;
    double acc = A.b[n];
#pragma unroll
    for (int o = 0; o < 27; o++) {
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const bool ok = ((unsigned)(i + dx) < (unsigned)A.nx) & ((unsigned)(j + dy) < (unsigned)A.ny) &
                        ((unsigned)(k + dz) < (unsigned)A.nz);
        // loads at valid addresses (the node itself off the box) and a select
        const double sv = A.S[o * N + n];
        const double xv = A.x[ok ? n + dx + (long long)A.nx * dy + layer * dz : (long long)n];
        acc = ok ? acc - sv * xv : acc;
    }
    A.r[n] = acc;
}

__global__ __launch_bounds__(kBlock) void k_zline_order(int nx, int ny, int nz, int LT, const double *__restrict__ S,
                                                        double *__restrict__ Sz)
{
    const long long N = (long long)nx * ny * nz;
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const int i = (int)(n % nx);
    const long long u = n / nx;
    const int j = (int)(u % ny), k = (int)(u / ny);
    const int colour = (i & 1) | ((j & 1) << 1);
    const long long base = 27 * zline_rows_below(nx, ny, nz, colour);
    const int ncx = (nx - (i & 1) + 1) / 2;
#pragma unroll
    for (int o = 0; o < 27; o++) {
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const bool ok = i + dx >= 0 && i + dx < nx && j + dy >= 0 && j + dy < ny && k + dz >= 0 && k + dz < nz;
        Sz[zline_index(base, ncx, nz, LT, i >> 1, j >> 1, k, o)] = ok ? S[o * N + n] : 0.0;   // +0 off the box
    }
}

// Tile width LT (lines along x, a power of two) and chunk depth KC (layers,
// a power of two, KC * LT <= kBlock) of an nx x ny x nz box: 8-line tiles on
// boxes with many lines (HBM-bound sweeps), 2-line tiles on boxes with few
// (latency-bound sweeps, where one deep chunk per workgroup pays); then the
// widest tile and deepest chunk, at most the z extent rounded up, whose line
// rows (four doubles each) and staged x planes fit the 64 KB LDS budget.
// The stencil reordering and the sweeps both take the tile from here.
static size_t zline_lds(int LT, int KC, int nz)
{
    return (size_t)32 * LT * nz + (size_t)8 * (KC + 2) * (2 * LT + 1) * 3;
}
static bool zline_tile(int nx, int ny, int nz, int &LT, int &KC)
{
    const long long lines = (long long)((nx + 1) / 2) * ((ny + 1) / 2);   // colour 0, the most
    int kfull = 1;
    while (kfull < nz && kfull < kBlock) kfull *= 2;
    for (LT = lines >= 4096 ? 8 : 2; LT >= 1; LT /= 2)
        for (KC = kfull < kBlock / LT ? kfull : kBlock / LT; KC >= 1; KC /= 2)
            if (zline_lds(LT, KC, nz) <= (size_t)kZlineLds) return true;
    return false;
}

void launch_zline_order(int nx, int ny, int nz, const double *S, double *Sz, hipStream_t st)
{
    int LT, KC;
    if (!zline_tile(nx, ny, nz, LT, KC)) return;   // z extents beyond the limit are refused at setup
    const long long N = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_zline_order, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, nx,
                       ny, nz, LT, S, Sz);
}

void launch_zline(LineBatch lb, int colour, hipStream_t st)
{
    int blk = 0;
    size_t lds = 0;
    for (int q = 0; q < lb.nbox; q++) {
        LineArgs &A = lb.a[q];
        if (!zline_tile(A.nx, A.ny, A.nz, A.lt, A.kc)) return;
        const size_t need = zline_lds(A.lt, A.kc, A.nz);
        lds = need > lds ? need : lds;
        const int cx = colour & 1, cy = colour >> 1;
        const int ncx = (A.nx - cx + 1) / 2, ncy = (A.ny - cy + 1) / 2;
        A.blk0 = blk;
        blk += ((ncx + A.lt - 1) / A.lt) * ncy;
    }
    if (blk) hipLaunchKernelGGL(k_zline, dim3(blk), dim3(kBlock), lds, st, lb, colour);
}

void launch_resid_full(LineBatch lb, hipStream_t st)
{
    int blk = 0;
    for (int q = 0; q < lb.nbox; q++) {
        lb.a[q].blk0 = blk;
        blk += (lb.a[q].n + kBlock - 1) / kBlock;
    }
    if (blk) hipLaunchKernelGGL(k_resid_full, dim3(blk), dim3(kBlock), 0, st, lb);
}

// inverse diagonal and per-block maxima of the Gershgorin ratio sum|s_ij|/s_ii
// Raise the bound (the bits of a non-negative double) to the workgroup's
// largest Gershgorin ratio; a negative, infinite or NaN ratio (a
// non-positive or non-finite diagonal) becomes +inf, which the host rejects.
// The bound is kept in kLmaxSlots slots, workgroup b raising slot b mod
// kLmaxSlots (one atomic per workgroup, spread over the slots so that they do
// not queue on one address); the host takes the maximum of the slots.
__device__ inline void gershgorin_max(double ratio, unsigned long long *lmax)
{
    __shared__ double red[4];
    if (!(ratio >= 0.0) || !(ratio < INFINITY)) ratio = INFINITY;
    const double m = block_max(ratio, red);
    if (threadIdx.x == 0)
        atomicMax(lmax + (blockIdx.x % kLmaxSlots), (unsigned long long)__double_as_longlong(m));
}

__global__ __launch_bounds__(kBlock) void k_diag(int n, const double *__restrict__ S,
                                                 double *__restrict__ invd,
                                                 unsigned long long *__restrict__ lmax)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double ratio = 0.0;
    if (t < n) {
        double sum = 0.0;
        for (int o = 0; o < 27; o++) sum += fabs(S[(long long)o * n + t]);
        const double dg = S[13LL * n + t];
        invd[t] = 1.0 / dg;
        ratio = sum / dg;
    }
    gershgorin_max(ratio, lmax);
}

__global__ __launch_bounds__(kBlock) void k_max_final(const double *__restrict__ part, int nblk,
                                                      double *__restrict__ out)
{
    __shared__ double red[4];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) m = fmax(m, part[b]);
    m = block_max(m, red);
    if (threadIdx.x == 0) *out = m;
}

void launch_diag(int n, const double *S, double *invd, unsigned long long *lmax, int nblk,
                 hipStream_t st)
{
    hipLaunchKernelGGL(k_diag, dim3(nblk), dim3(kBlock), 0, st, n, S, invd, lmax);
}

// level 0 of all boxes: inverse diagonal of the rows formed from the element
// data, and the Gershgorin bound
__global__ __launch_bounds__(kBlock) void k_diag0_batch(Geom g, PrepBatch pb)
{
    // (the box index is uniform: in a scalar register the box's arguments
    // are read without a private copy)
    const int bx = __builtin_amdgcn_readfirstlane(find_box(pb, blockIdx.x));
    const PrepArgs A = pb.a[bx];
    const int t = (blockIdx.x - A.blk0) * kBlock + threadIdx.x;
    double ratio = 0.0;
    if (t < A.n) {
        double row[27];
        assemble0_row(g, A.E, t, row);
        double sum = 0.0;
        for (int o = 0; o < 27; o++) sum += fabs(row[o]);
        const double dg = row[13];
        A.invd0[t] = 1.0 / dg;
        ratio = sum / dg;
    }
    gershgorin_max(ratio, A.lmax);
}
void launch_diag0_batch(const Geom &g, const PrepBatch &pb, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag0_batch, dim3(nblk), dim3(kBlock), 0, st, g, pb);
}

__global__ __launch_bounds__(kBlock) void k_diag0(Geom g, Elem0 E, int n, double *__restrict__ invd,
                                                  double *__restrict__ part)
{
    __shared__ double red[4];
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double ratio = 0.0;
    if (t < n) {
        double row[27];
        assemble0_row(g, E, t, row);
        double sum = 0.0;
        for (int o = 0; o < 27; o++) sum += fabs(row[o]);
        const double dg = row[13];
        invd[t] = 1.0 / dg;
        ratio = sum / dg;
    }
    const double m = block_max(ratio, red);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

void launch_diag0(const Geom &g, const Elem0 &E, int n, double *invd, double *part, int nblk,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_diag0, dim3(nblk), dim3(kBlock), 0, st, g, E, n, invd, part);
}
void launch_max_final(const double *part, int nblk, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kBlock), 0, st, part, nblk, out);
}

// dense symmetric matrix (row-major) from a stencil, symmetrized
__global__ __launch_bounds__(kBlock) void k_dense(int nx, int ny, int nz,
                                                  const double *__restrict__ S,
                                                  double *__restrict__ A)
{
    const int n = nx * ny * nz;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)n * n) return;
    const int r = (int)(t / n), c = (int)(t % n);
    auto entry = [&](int row, int col) -> double {
        const int i = row % nx, u = row / nx, j = u % ny, k = u / ny;
        const int ci = col % nx, cu = col / nx, cj = cu % ny, ck = cu / ny;
        const int dx = ci - i, dy = cj - j, dz = ck - k;
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return 0.0;
        return S[(long long)nb_index(dx, dy, dz) * n + row];
    };
    A[t] = 0.5 * (entry(r, c) + entry(c, r));
}

// In-place Gauss-Jordan inversion of SPD matrices (no pivoting), one
// workgroup per matrix; each wave sweeps rows, its lanes the columns.  The
// result is written column-major (equal to row-major for the symmetric
// inverse).
__global__ __launch_bounds__(1024) void k_invert(InvBatch ib)
{
    __shared__ double rowp[1024];
    __shared__ double colp[1024];
    const int box = blockIdx.x;
    const int n = ib.n[box];
    double *A = ib.A[box];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int p = 0; p < n; p++) {
        __syncthreads();
        const double d = 1.0 / A[(long long)p * n + p];
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            rowp[q] = A[(long long)p * n + q] * d;
            colp[q] = A[(long long)q * n + p];
        }
        __syncthreads();
        for (int i = wave; i < n; i += nw) {
            const double ci = colp[i];
            double *Ai = A + (long long)i * n;
            for (int j = lane; j < n; j += 64) {
                double v;
                if (i == p) v = j == p ? d : rowp[j];
                else v = j == p ? -ci * d : Ai[j] - ci * rowp[j];
                Ai[j] = v;
            }
        }
    }
    __syncthreads();
    double *out = ib.Ainv[box];
    for (long long t = threadIdx.x; t < (long long)n * n; t += blockDim.x) out[t] = A[t];
}

void launch_dense_from_stencil(int nx, int ny, int nz, const double *S, double *A, hipStream_t st)
{
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_dense, dim3((int)((n * n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, nx,
                       ny, nz, S, A);
}
// Same elimination for n <= kInvLds with the matrix held in registers, at
// most kInvE entries per thread at fixed positions: per pivot only the pivot
// row and column pass through LDS.  Each entry is updated by the same
// expressions as above, so the inverse is the same.
constexpr int kInvLds = 80;
constexpr int kInvE = (kInvLds * kInvLds + 1023) / 1024;
__global__ __launch_bounds__(1024) void k_invert_lds(InvBatch ib)
{
    __shared__ double rowp[kInvLds], colp[kInvLds];
    const int box = blockIdx.x;
    const int n = ib.n[box];
    const int nn = n * n;
    double v[kInvE];
    int ii[kInvE], jj[kInvE];
#pragma unroll
    for (int e = 0; e < kInvE; e++) {
        const int t = threadIdx.x + e * 1024;
        ii[e] = t < nn ? t / n : -1;
        jj[e] = t < nn ? t - ii[e] * n : -1;
        v[e] = t < nn ? ib.A[box][t] : 0.0;
    }
    for (int p = 0; p < n; p++) {
#pragma unroll
        for (int e = 0; e < kInvE; e++) {
            if (ii[e] == p) rowp[jj[e]] = v[e];
            if (jj[e] == p) colp[ii[e]] = v[e];
        }
        __syncthreads();
        const double d = 1.0 / colp[p];
#pragma unroll
        for (int e = 0; e < kInvE; e++) {
            if (ii[e] < 0) continue;
            const double rp = rowp[jj[e]] * d;
            double w;
            if (ii[e] == p) w = jj[e] == p ? d : rp;
            else w = jj[e] == p ? -colp[ii[e]] * d : v[e] - colp[ii[e]] * rp;
            v[e] = w;
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kInvE; e++) {
        const int t = threadIdx.x + e * 1024;
        if (t < nn) ib.Ainv[box][t] = v[e];
    }
}

// The same elimination for n <= 64, laid out so that publishing a pivot row
// and column needs no search: thread t holds column j = t % 64 in rows
// t / 64 + 16 s (s = 0..3).  Row and column p + 1 and the reciprocal of
// their diagonal entry are stored, into the other of two buffers, by their
// holders right after the update of pivot p (wave t / 64 = (p + 1) % 16 the
// row, lane j = p + 1 of every wave its part of the column), so that one
// barrier per pivot suffices.  Each entry is updated by the expressions
// above, so the inverse is the same.
constexpr int kInvW = 64;
__global__ __launch_bounds__(1024) void k_invert_w64(InvBatch ib)
{
    __shared__ double rowp[2][kInvW], colp[2][kInvW], dp[2];
    const int box = blockIdx.x;
    const int n = ib.n[box];
    const int j = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    double v[4];
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int i = r0 + 16 * s;
        v[s] = i < n && j < n ? ib.A[box][i * n + j] : 0.0;
    }
    // row, column and diagonal reciprocal of pivot q into buffer q & 1
    auto publish = [&](int q) {
        const int b = q & 1;
        if (r0 == (q & 15) && j < n) {
            const int sq = q >> 4;   // row q's slot in its wave
            const double a = sq == 0 ? v[0] : (sq == 1 ? v[1] : (sq == 2 ? v[2] : v[3]));
            rowp[b][j] = a;
            if (j == q) dp[b] = 1.0 / a;
        }
        if (j == q) {
#pragma unroll
            for (int s = 0; s < 4; s++)
                if (r0 + 16 * s < n) colp[b][r0 + 16 * s] = v[s];
        }
    };
    if (n > 0) publish(0);
    __syncthreads();
    for (int p = 0; p < n; p++) {
        const int b = p & 1;
        const double d = dp[b];
        const double rp = rowp[b][j] * d;   // (unused where j >= n)
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int i = r0 + 16 * s;
            if (i >= n || j >= n) continue;
            double w;
            if (i == p) w = j == p ? d : rp;
            else w = j == p ? -colp[b][i] * d : v[s] - colp[b][i] * rp;
            v[s] = w;
        }
        if (p + 1 < n) publish(p + 1);
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int i = r0 + 16 * s;
        if (i < n && j < n) ib.Ainv[box][i * n + j] = v[s];
    }
}

void launch_invert(const InvBatch &ib, hipStream_t st)
{
    int nmax = 0;
    for (int b = 0; b < ib.nbox; b++) nmax = ib.n[b] > nmax ? ib.n[b] : nmax;
    if (nmax <= kInvW)
        hipLaunchKernelGGL(k_invert_w64, dim3(ib.nbox), dim3(1024), 0, st, ib);
    else if (nmax <= kInvLds)
        hipLaunchKernelGGL(k_invert_lds, dim3(ib.nbox), dim3(1024), 0, st, ib);
    else
        hipLaunchKernelGGL(k_invert, dim3(ib.nbox), dim3(1024), 0, st, ib);
}


// A coarse level's smoother data in one pass over its stored Galerkin
// stencil: the difference form in T (slot 0 the row sum formed in FP64,
// slots 1..13 the upper half as they are), the inverse diagonal in T (formed
// in FP64), and the block maximum of the Gershgorin ratio
template <typename T>
__global__ __launch_bounds__(kBlock) void k_level_prep(int n, const double *__restrict__ S,
                                                       T *__restrict__ D, T *__restrict__ invd,
                                                       double *__restrict__ part)
{
    __shared__ double red[4];
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double ratio = 0.0;
    if (t < n) {
        double rs = 0.0, sum = 0.0;
        for (int o = 0; o < 27; o++) {
            const double v = S[(long long)o * n + t];
            rs += v;
            sum += fabs(v);
            if (o > 13) D[(long long)(o - 13) * n + t] = (T)v;
        }
        D[t] = (T)rs;
        const double dg = S[13LL * n + t];
        invd[t] = (T)(1.0 / dg);
        ratio = sum / dg;
    }
    const double m = block_max(ratio, red);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}
template <typename T>
void launch_level_prep(int n, const double *S, T *D, T *invd, double *part, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL((k_level_prep<T>), dim3(nblk), dim3(kBlock), 0, st, n, S, D, invd, part);
}

// the same for one level of all boxes, the bound by atomic maximum
template <typename T>
__global__ __launch_bounds__(kBlock) void k_level_prep_batch(PrepBatch pb)
{
    const int bx = __builtin_amdgcn_readfirstlane(find_box(pb, blockIdx.x));
    const PrepArgs A = pb.a[bx];
    const int n = A.n;
    const int t = (blockIdx.x - A.blk0) * kBlock + threadIdx.x;
    T *D = (T *)A.D;
    double ratio = 0.0;
    if (t < n) {
        double rs = 0.0, sum = 0.0;
        for (int o = 0; o < 27; o++) {
            const double v = A.S[(long long)o * n + t];
            rs += v;
            sum += fabs(v);
            if (o > 13) D[(long long)(o - 13) * n + t] = (T)v;
        }
        D[t] = (T)rs;
        const double dg = A.S[13LL * n + t];
        ((T *)A.invd)[t] = (T)(1.0 / dg);
        ratio = sum / dg;
    }
    gershgorin_max(ratio, A.lmax);
}
template <typename T>
void launch_level_prep_batch(const PrepBatch &pb, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL((k_level_prep_batch<T>), dim3(nblk), dim3(kBlock), 0, st, pb);
}
template void launch_level_prep_batch<double>(const PrepBatch &, int, hipStream_t);
template void launch_level_prep_batch<float>(const PrepBatch &, int, hipStream_t);
template void launch_level_prep<double>(int, const double *, double *, double *, double *, int,
                                        hipStream_t);
template void launch_level_prep<float>(int, const double *, float *, float *, double *, int,
                                       hipStream_t);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cast(long long n, const double *__restrict__ s,
                                                 T *__restrict__ d)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) d[t] = (T)s[t];
}
template <typename T>
void launch_cast(long long n, const double *src, T *dst, hipStream_t st)
{
    hipLaunchKernelGGL((k_cast<T>), dim3((int)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n,
                       src, dst);
}
template void launch_cast<double>(long long, const double *, double *, hipStream_t);
template void launch_cast<float>(long long, const double *, float *, hipStream_t);

}  // namespace p4d
