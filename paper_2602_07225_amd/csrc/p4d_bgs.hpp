// Block Gauss-Seidel preconditioner (paper Sec. 4.2, eq. PGS): declarations
// shared by the kernels (bgs.hip) and the driver (p4d_api.hip).
#pragma once
#include "p4d_kernels.hpp"

namespace p4d {

// Fields of the 4x4 block system as numbered in a block ordering (the
// ordering option holds the field at block position p in bits [2p, 2p + 2)).
enum BgsField : int { BF_PHIS = 0, BF_PHIE = 1, BF_CE = 2, BF_CS = 3 };

struct BgsArgs {
    RadArgs R;            // tables, coefficients, level-0 buffers, final iterates
    const double *kx;     // element coefficient of the diffusion-potential block (x h) ...
    double kx_scale;      // ... times this factor (chi with h kappa, or 1)
    double *zsN;          // solved c_s surface value per electrode node (FP64)
    int field;            // field whose right-hand side bgs_rhs forms
    int done;             // bit f set: field f solved
};

// Right-hand side r_f - sum_{g done} A_{f,g} z_g of one electrode-level field
// (precision T, level-0 multigrid layout) with the first Chebyshev iterate of
// its boxes.
template <typename T>
void launch_bgs_rhs(const Geom &g, const BgsArgs &B, const double *r, const double *rscale, int transpose,
                    hipStream_t st);
// z_s,j = A_ss,j^-1 (r_s,j - delta_j e_N), delta_j the coupling to the
// electrode-level fields solved before; keeps z_s,N in FP64 in zsN.
template <typename T, typename TZ>
void launch_bgs_cs(const Geom &g, const BgsArgs &B, const double *r, const double *rscale, TZ *z,
                   int transpose, hipStream_t st);
// phi_s (identity rows on the grounded layer), phi_e and c_e of z from the
// final level-0 iterates.
template <typename TZ>
void launch_bgs_out(const Geom &g, const BgsArgs &B, const double *r, const double *rscale, TZ *z,
                    hipStream_t st);

}  // namespace p4d
