// Physical cell around the linear solve: device-side constants and the
// launchers of phys.hip (used by the Newton driver in p4d_api.hip).
#pragma once
#include "p4d_kernels.hpp"

namespace p4d {

// constants of the physical cell and the per-field scales of the Newton
// system (unknowns u = x_f u^, equations R^ = r_f R)
struct PhysDev {
    double F, RT, tplus, brug, ce0, eps_el, eps_sep;
    double eps_s[2], sigma[2], k[2], alpha[2], csmax[2], cs0[2], a[2];
    double xphi, xc, xs, rphi, rc, rs;
    // Case II: porosity and active-material fraction per element (device),
    // or the per-material values when null
    const double *por = nullptr, *act = nullptr;
};

// arrays of the residual correction (scaled variables)
struct PhysFix {
    const double *uh;      // scaled state
    const double *old;     // previous-step storage terms (scaled rows)
    const double *fh;      // applied current per phi_s row (scaled)
    const double *qh;      // scaled reaction per electrode node
    const double *gg, *ss, *ee, *mm;
    double gam[2];         // scaled surface coupling per electrode
};

// also the scaled c_e-derivatives of the transport coefficients (times h)
// per element, for the Newton terms
void launch_phys_coef(const Geom &g, const PhysDev &P, const double *u, double *sigh, double *kaph,
                      double *kdh, double *dch, double *gg, double *ss, double *ee, double *qh,
                      double *nwa, double *nwb, double *nwc, hipStream_t st);
void launch_phys_scale(const Geom &g, const PhysDev &P, const double *in, double *out, int up,
                       hipStream_t st);
void launch_phys_fix(const Geom &g, const PhysFix &F, double *r, int neg, hipStream_t st);
// returns the number of partial maxima written
int launch_phys_update(const Geom &g, const PhysDev &P, const double *dh, double *u, double *partial,
                       hipStream_t st);
void launch_phys_init(const Geom &g, const PhysDev &P, double *u, hipStream_t st);
void launch_phys_old_cs(const Geom &g, const PhysDev &P, const double *uold, double dtp, double *old,
                        hipStream_t st);
// por, act and the scaled storage meh = ms * por from the volume fractions
// (device, per element); per workgroup a 1 where a fraction is out of range
int launch_phys_fractions(const Geom &g, const PhysDev &P, const double *eps_s, const double *eps_b,
                          double *por, double *act, double *meh, double ms, double *partial,
                          hipStream_t st);
void launch_phys_unscale_rows(const Geom &g, const PhysDev &P, const double *rh, double *r, hipStream_t st);

}  // namespace p4d
