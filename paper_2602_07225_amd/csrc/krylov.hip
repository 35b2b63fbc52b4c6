// Streaming kernels of flexible GMRES (the paper's Krylov solver, Sec. 4.2):
// classical Gram-Schmidt as one fused multi-dot (h = V^T w in one pass over w
// and the basis) and one fused update (w -= V c together with ||w||^2).
// Reductions are two-stage with a fixed grid, hence deterministic.
// The basis is stored unnormalized: v_i = V_i / beta_i, the scale 1/beta_i
// being folded into the coefficients.
#include "p4d_device.hpp"

namespace p4d {

constexpr int kPStride = 64;   // partial-sum stride per workgroup

int stream_blocks(long long n)
{
    long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_mdot(long long n, const double *__restrict__ w,
                                                 const double *__restrict__ V,
                                                 const double *__restrict__ v0, long long ldv,
                                                 int nv, double *__restrict__ partial)
{
    __shared__ double red[4][KMAX];
    double acc[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; q++) acc[q] = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < KMAX; q++)
            if (q < nv) acc[q] += wi * (q == 0 ? v0 : V + (long long)q * ldv)[i];
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
    // partial sums stored [q][block] so that the final reduction reads them
    // contiguously
    if (threadIdx.x < nv)
        partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

void launch_mdot(long long n, const double *w, const double *V, const double *v0, long long ldv, int nv,
                 double *partial, int nblk, hipStream_t st)
{
#define P4D_MD(K) \
    hipLaunchKernelGGL((k_mdot<K>), dim3(nblk), dim3(kBlock), 0, st, n, w, V, v0, ldv, nv, partial)
    if (nv <= 4) P4D_MD(4);
    else if (nv <= 8) P4D_MD(8);
    else if (nv <= 16) P4D_MD(16);
    else if (nv <= 32) P4D_MD(32);
    else P4D_MD(64);
#undef P4D_MD
}

// h_q = invbeta_q * sum_b partial[q][b];  c_q = h_q * invbeta_q; one
// workgroup per q
__global__ __launch_bounds__(kBlock) void k_mdot_final(int nv, const double *__restrict__ partial,
                                                       int nblk, const double *__restrict__ invbeta,
                                                       double *__restrict__ h,
                                                       double *__restrict__ c)
{
    __shared__ double red[4];
    const int q = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) s += partial[(long long)q * nblk + b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double hq = s * invbeta[q];
        h[q] = hq;
        c[q] = hq * invbeta[q];
    }
}

void launch_mdot_final(int nv, const double *partial, int nblk, const double *invbeta, double *h,
                       double *c, hipStream_t st)
{
    hipLaunchKernelGGL(k_mdot_final, dim3(nv), dim3(kBlock), 0, st, nv, partial, nblk, invbeta, h, c);
}

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_orth(long long n, double *__restrict__ w,
                                                 const double *__restrict__ V,
                                                 const double *__restrict__ v0, long long ldv,
                                                 int nv, const double *__restrict__ c,
                                                 double *__restrict__ partial)
{
    __shared__ double red[4];
    double cq[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; q++) cq[q] = q < nv ? c[q] : 0.0;
    double sq = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double wi = w[i];
#pragma unroll
        for (int q = 0; q < KMAX; q++)
            if (q < nv) wi -= cq[q] * (q == 0 ? v0 : V + (long long)q * ldv)[i];
        w[i] = wi;
        sq += wi * wi;
    }
    const double s = block_sum(sq, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_orth(long long n, double *w, const double *V, const double *v0, long long ldv, int nv,
                 const double *c, double *partial, int nblk, hipStream_t st)
{
#define P4D_OR(K) \
    hipLaunchKernelGGL((k_orth<K>), dim3(nblk), dim3(kBlock), 0, st, n, w, V, v0, ldv, nv, c, partial)
    if (nv <= 4) P4D_OR(4);
    else if (nv <= 8) P4D_OR(8);
    else if (nv <= 16) P4D_OR(16);
    else if (nv <= 32) P4D_OR(32);
    else P4D_OR(64);
#undef P4D_OR
}

// beta = sqrt(sum partial); invbeta = 1/beta (0 if beta == 0)
__global__ __launch_bounds__(kBlock) void k_norm_final(const double *__restrict__ partial, int nblk,
                                                       double *__restrict__ beta,
                                                       double *__restrict__ invbeta)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) s += partial[b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double bt = sqrt(s);
        *beta = bt;
        if (invbeta) *invbeta = bt > 0.0 ? 1.0 / bt : 0.0;
    }
}

void launch_norm_final(const double *partial, int nblk, double *beta, double *invbeta,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kBlock), 0, st, partial, nblk, beta, invbeta);
}

// assign: x = Z y (x not read; the first update from x = 0), else x += Z y
template <typename TZ, int KMAX>
__global__ __launch_bounds__(kBlock) void k_zy(long long n, double *__restrict__ x,
                                               const TZ *__restrict__ Z, long long ldz, int nv,
                                               const double *__restrict__ y, int assign)
{
    double yq[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; q++) yq[q] = q < nv ? y[q] : 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double xi = assign ? 0.0 : x[i];
#pragma unroll
        for (int q = 0; q < KMAX; q++)
            if (q < nv) xi += yq[q] * (double)Z[(long long)q * ldz + i];
        x[i] = xi;
    }
}

template <typename TZ>
void launch_zy(long long n, double *x, const TZ *Z, long long ldz, int nv, const double *y, int assign,
               hipStream_t st)
{
    const int nblk = stream_blocks(n);
#define P4D_ZY(K) \
    hipLaunchKernelGGL((k_zy<TZ, K>), dim3(nblk), dim3(kBlock), 0, st, n, x, Z, ldz, nv, y, assign)
    if (nv <= 4) P4D_ZY(4);
    else if (nv <= 8) P4D_ZY(8);
    else if (nv <= 16) P4D_ZY(16);
    else if (nv <= 32) P4D_ZY(32);
    else P4D_ZY(64);
#undef P4D_ZY
}
template void launch_zy<double>(long long, double *, const double *, long long, int, const double *, int,
                                hipStream_t);
template void launch_zy<float>(long long, double *, const float *, long long, int, const double *, int,
                               hipStream_t);

__global__ __launch_bounds__(kBlock) void k_dot(long long n, const double *__restrict__ a,
                                                const double *__restrict__ b,
                                                double *__restrict__ partial)
{
    __shared__ double red[4];
    double s = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        s += a[i] * b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_dot_partial(long long n, const double *a, const double *b, double *partial, int nblk,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_dot, dim3(nblk), dim3(kBlock), 0, st, n, a, b, partial);
}

// Hand n device values (the bits of doubles or of 64-bit integers) to the
// host: copied into mapped host memory, then the sequence number is raised.
// Every thread releases its copies at system scope before the barrier, after
// which one thread stores the number; a host that sees the number sees the
// values.
__global__ __launch_bounds__(kBlock) void k_publish(const unsigned long long *__restrict__ src, int n,
                                                    unsigned long long *dst, unsigned long long *seq_out,
                                                    unsigned long long seq)
{
    for (int i = threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(seq_out, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish(const void *src, int n, void *dst, unsigned long long *seq_out, unsigned long long seq,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(kBlock), 0, st, (const unsigned long long *)src, n,
                       (unsigned long long *)dst, seq_out, seq);
}

}  // namespace p4d
