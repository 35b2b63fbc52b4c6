// Particle-block kernels of the preconditioner (paper Sec. 4.2: the c_s
// block is block diagonal with one tridiagonal N_c x N_c matrix per point,
// inverted exactly); the bodies live in p4d_kernels.hpp.
//   rad_fwd : zeta_j and the macro right-hand side r~_y (SCHUR mode), written
//             in the preconditioner precision with the first Chebyshev
//             iterate of each V-cycle box.
//   rad_back: delta_j, the particle solution and the macro output.
#include "p4d_kernels.hpp"

namespace p4d {

template <typename T, int NRMAX, bool TRANS, bool SCHUR>
__global__ __launch_bounds__(kBlock) void k_rad_fwd(Geom g, RadArgs R, const double *r, const double *rscale)
{
    rad_fwd_block<T, NRMAX, TRANS, SCHUR>(g, R, r, rscale ? *rscale : 1.0, blockIdx.x);
}

int rad_nrmax(const Geom &g)
{
    const int nrm = g.nr[0] > g.nr[1] ? g.nr[0] : g.nr[1];
    for (int c = 0; c < kNrClasses - 1; c++)
        if (nrm <= kNrClass[c]) return kNrClass[c];
    return kNrClass[kNrClasses - 1];
}

template <typename T>
void launch_rad_fwd(const Geom &g, const RadArgs &R, const double *r, const double *rscale, int transpose,
                    int schur, hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
#define P4D_RF(NR, TR, SC) \
    hipLaunchKernelGGL((k_rad_fwd<T, NR, TR, SC>), dim3(nb), dim3(kBlock), 0, st, g, R, r, rscale)
#define P4D_RF2(NR)                                  \
    do {                                             \
        if (schur) {                                 \
            if (transpose) P4D_RF(NR, true, true);   \
            else P4D_RF(NR, false, true);            \
        } else {                                     \
            P4D_RF(NR, false, false);                \
        }                                            \
    } while (0)
    P4D_NR_SWITCH(rad_nrmax(g), P4D_RF2)
#undef P4D_RF2
#undef P4D_RF
}
template void launch_rad_fwd<double>(const Geom &, const RadArgs &, const double *, const double *, int,
                                     int, hipStream_t);
template void launch_rad_fwd<float>(const Geom &, const RadArgs &, const double *, const double *, int, int,
                                    hipStream_t);

template <typename T, typename TZ, int NRMAX, bool TRANS, bool SCHUR>
__global__ __launch_bounds__(kBlock) void k_rad_back(Geom g, RadArgs R, const double *r,
                                                    const double *rscale, TZ *z)
{
    rad_back_block<T, TZ, NRMAX, TRANS, SCHUR>(g, R, r, rscale ? *rscale : 1.0, z, blockIdx.x);
}


template <typename T, typename TZ>
void launch_rad_back(const Geom &g, const RadArgs &R, const double *r, const double *rscale, TZ *z,
                     int transpose, int schur, hipStream_t st)
{
    const int nb = (int)((g.nnode + kBlock - 1) / kBlock);
#define P4D_RB(NR, TR, SC) \
    hipLaunchKernelGGL((k_rad_back<T, TZ, NR, TR, SC>), dim3(nb), dim3(kBlock), 0, st, g, R, r, rscale, z)
#define P4D_RB2(NR)                                  \
    do {                                             \
        if (schur) {                                 \
            if (transpose) P4D_RB(NR, true, true);   \
            else P4D_RB(NR, false, true);            \
        } else {                                     \
            if (transpose) P4D_RB(NR, true, false);  \
            else P4D_RB(NR, false, false);           \
        }                                            \
    } while (0)
    P4D_NR_SWITCH(rad_nrmax(g), P4D_RB2)
#undef P4D_RB2
#undef P4D_RB
}
template void launch_rad_back<double, double>(const Geom &, const RadArgs &, const double *, const double *,
                                                double *, int, int, hipStream_t);
template void launch_rad_back<float, double>(const Geom &, const RadArgs &, const double *, const double *,
                                                double *, int, int, hipStream_t);
template void launch_rad_back<double, float>(const Geom &, const RadArgs &, const double *, const double *,
                                                float *, int, int, hipStream_t);
template void launch_rad_back<float, float>(const Geom &, const RadArgs &, const double *, const double *,
                                                float *, int, int, hipStream_t);

}  // namespace p4d
