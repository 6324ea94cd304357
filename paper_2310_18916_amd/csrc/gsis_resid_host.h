// Host side of the convergence criterion of Sec. 5, Eq. (convergence_critertion):
// the relative changes from the reduced sums, and the divergence watch.
// Plain C++ (no HIP), so the logic is compiled and tested on the host alone.
#pragma once
#include <cmath>

namespace gsis {

// sums[0..2]: sum over fluid cells of (rho^n - rho^{n-1})^2, |u^n - u^{n-1}|^2,
// (Tt^n - Tt^{n-1})^2; sums[3..5]: of (rho^{n-1})^2, |u^{n-1}|^2, (Tt^{n-1})^2
// (uniform cells: the volume weights cancel).
//
// A denominator at or below its noise floor counts as zero and the absolute
// change is reported.  Density and temperature are positive, so their floor is
// zero.  The velocity of a gas at rest is the rounding noise of the moment
// reduction, so its floor is (1e3 eps)^2 sum Tt^2, eps the unit roundoff of
// the VDF precision: a root-mean-square speed below 1e3 eps thermal speeds is
// taken as no flow at all.
struct ResidEval {
    double eps[3];
    bool relative[3];   // the denominator was above its floor
};

inline double resid_u_floor(const double *sums, bool fp32)
{
    const double em = fp32 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
    const double k = 1e3 * em;
    return k * k * sums[5];
}

inline ResidEval resid_eval(const double *sums, bool fp32)
{
    ResidEval r;
    const double floor_[3] = {0.0, resid_u_floor(sums, fp32), 0.0};
    for (int k = 0; k < 3; ++k) {
        r.relative[k] = sums[3 + k] > floor_[k];
        r.eps[k] = r.relative[k] ? std::sqrt(sums[k] / sums[3 + k]) : std::sqrt(sums[k]);
    }
    return r;
}

// Divergence: a component whose relative change exceeds `factor` times its
// reference.  The reference of a component is its first relative value (an
// absolute change against noise is no scale for later ones).
struct DivWatch {
    bool have[3] = {false, false, false};
    double first[3] = {0.0, 0.0, 0.0};
};

inline bool resid_diverged(DivWatch &w, const ResidEval &r, double factor)
{
    bool grew = false;
    for (int k = 0; k < 3; ++k) {
        if (!r.relative[k]) continue;
        if (!w.have[k]) {
            if (r.eps[k] > 0.0) {
                w.have[k] = true;
                w.first[k] = r.eps[k];
            }
        } else if (r.eps[k] > factor * w.first[k]) {
            grew = true;
        }
    }
    return grew;
}

}  // namespace gsis
