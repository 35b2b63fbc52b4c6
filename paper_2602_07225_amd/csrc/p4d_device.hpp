// Device helpers shared by the kernel files of the library.
#pragma once
#include "p4d_internal.hpp"

namespace p4d {

// Workgroup b of nb as dispatched round-robin over the 8 XCDs is mapped to a
// logical tile so that each XCD works on one contiguous range of tiles (its
// stencil halos then stay in that XCD's L2).
__device__ inline int xcd_block(int b, int nb)
{
    int q = nb >> 3, r = nb & 7;
    int x = b & 7, pos = b >> 3;
    int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + pos;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over a 256-thread workgroup; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds /* >= 4 */)
{
    v = wave_sum(v);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return r;
}
__device__ inline double block_max(double v, double *lds)
{
    v = wave_max(v);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
    __syncthreads();
    return r;
}

__host__ __device__ constexpr int popc3(int v) { return (v & 1) + ((v >> 1) & 1) + ((v >> 2) & 1); }
__host__ __device__ constexpr int nb_index(int dx, int dy, int dz)
{
    return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

// Q1 element sums at one node.  c[e], e = ex | ey<<1 | ez<<2, is the
// coefficient of the element spanning node offsets ex-1..ex (etc.); X holds
// the 27 neighbour values.  Reference stiffness on the unit cube: 1/3 on the
// diagonal, 0 between corners differing in one coordinate, -1/12 otherwise.
// Its rows sum to zero, so it is applied to differences x_b - x_a: constants
// cancel exactly, which keeps near-null modes accurate in FP32.
template <typename R>
__device__ inline R q1_stiff(const R c[8], const R X[27])
{
    R acc = R(0);
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int a = (1 - ex) | ((1 - ey) << 1) | ((1 - ez) << 2);
        R far = R(0);
#pragma unroll
        for (int bb = 0; bb < 8; bb++) {
            if (popc3(a ^ bb) >= 2)
                far += X[13] - X[nb_index(ex - 1 + (bb & 1), ey - 1 + ((bb >> 1) & 1),
                                          ez - 1 + ((bb >> 2) & 1))];
        }
        acc += c[e] * far;
    }
    return acc * R(1.0 / 12.0);
}

// The same for box elements: kw[p] weighs the difference to the corner that
// differs in the axes of bit pattern p (kw[0], the diagonal, is not used:
// rows sum to zero).  With kw = {., 0, 0, 1/12, 0, 1/12, 1/12, 1/12} it is
// q1_stiff.
template <typename R>
__device__ inline R q1_stiff_w(const R c[8], const R X[27], const double kw[8])
{
    R acc = R(0);
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int a = (1 - ex) | ((1 - ey) << 1) | ((1 - ez) << 2);
        R part = R(0);
#pragma unroll
        for (int bb = 0; bb < 8; bb++) {
            if (bb == a) continue;
            part += R(kw[a ^ bb]) * (X[13] - X[nb_index(ex - 1 + (bb & 1), ey - 1 + ((bb >> 1) & 1),
                                                      ez - 1 + ((bb >> 2) & 1))]);
        }
        acc += c[e] * part;
    }
    return acc;
}

// Reference mass on the unit cube: (8, 4, 2, 1)/216 by the number of
// differing coordinates.
template <typename R>
__device__ inline R q1_mass(const R c[8], const R X[27])
{
    R acc = R(0);
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        const int a = (1 - ex) | ((1 - ey) << 1) | ((1 - ez) << 2);
        R part = R(0);
#pragma unroll
        for (int bb = 0; bb < 8; bb++) {
            const int d = popc3(a ^ bb);
            const R w = d == 0 ? R(8.0 / 216.0) : d == 1 ? R(4.0 / 216.0)
                                                         : d == 2 ? R(2.0 / 216.0) : R(1.0 / 216.0);
            part += w * X[nb_index(ex - 1 + (bb & 1), ey - 1 + ((bb >> 1) & 1),
                                   ez - 1 + ((bb >> 2) & 1))];
        }
        acc += c[e] * part;
    }
    return acc;
}

}  // namespace p4d
