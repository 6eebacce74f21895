// HOMO/LUMO estimates from the history of a finished expansion (host code), for the
// accelerated layers of a later call (Sec. Accelerated Deep-NN SP2: the values can be
// taken from previous expansions, as in a molecular-dynamics run).
//
// Near convergence IdErr_k = Tr[S_{k-1} - S_{k-1}^2] is dominated by the two eigenvalues
// closest to the step: the LUMO image a (near 0) and the HOMO image 1 - c (near 1), so
// IdErr_k ~ a + c.  An ordinary layer x^2 maps (a, c) to (a^2, 2c - c^2) and 2x - x^2 maps it
// to (2a - a^2, c^2); two consecutive values then fix a and c through one quadratic.  The
// layers before S_{k-1} are undone exactly: sigma_n = +-1/(1 - 2v) gives the branch and the
// shift v of an accelerated layer (v = 0 for an ordinary one), and each map is inverted on
// its increasing branch.  S_0 = (emax I - H)/(emax - emin) turns the images into energies.
// Further eigenvalues near the step only enlarge IdErr, which moves both estimates toward
// the middle of the gap; every usable pair of layers contributes, the highest HOMO and
// lowest LUMO estimates are kept, and the interval is narrowed by 10 % of its width.
#include "sp2_internal.h"

#include <math.h>

namespace {

constexpr double kUpper = 0.25;    // IdErr_k above this: more than two states matter
constexpr double kMargin = 0.1;    // inward narrowing, as a fraction of the interval

// x from y = map(x) on the increasing branch; branch +1: y = ((x - v)/(1 - v))^2,
// branch -1: y = 1 - ((1 - v - x)/(1 - v))^2
double undo_layer(double y, int branch, double v) {
    if (y < 0.0) y = 0.0;
    if (y > 1.0) y = 1.0;
    if (branch > 0) return v + (1.0 - v) * sqrt(y);
    return (1.0 - v) * (1.0 - sqrt(1.0 - y));
}

}  // namespace

extern "C" {

int sp2_estimate_gap(const sp2_info* info, int n, int precision, double* homo, double* lumo) {
    if (!info || !homo || !lumo || n <= 0 || precision < SP2_FP64 || precision > SP2_BF16X2) return SP2_EINVAL;
    const int m = info->layers;
    if (m < 3 || m > SP2_MAX_LAYERS || !(info->emax > info->emin)) return SP2_EINVAL;
    // rounding floor of IdErr in the state precision
    const double floor_abs = (precision == SP2_FP64 ? 1e-12 : 1e-6) * n;
    const double span = info->emax - info->emin;
    double best_homo = -INFINITY, best_lumo = INFINITY;
    int used = 0;
    // layer j (1-based) applied to S_{j-1} gives S_j; history index j - 1
    for (int k = 0; k + 1 < m - 1; ++k) {
        const double s = info->sigma_c[k];
        if (fabs(s) != 1.0) continue;                     // the pair's layer must be an ordinary one
        const double e0 = info->iderr[k], e1 = info->iderr[k + 1];
        if (!(e0 <= kUpper) || !(e1 >= floor_abs)) continue;
        const double disc = 1.0 - (2.0 * e0 - e1);
        if (disc < 0.0) continue;
        const double r = 1.0 - sqrt(disc);
        double a, c;
        if (s > 0) {
            a = r;
            c = e0 - r;
        } else {
            c = r;
            a = e0 - r;
        }
        if (!(a > 0.0) || !(c > 0.0)) continue;
        double xl = a, xh = 1.0 - c;
        for (int j = k - 1; j >= 0; --j) {
            const double sj = info->sigma_c[j];
            const int branch = sj > 0 ? 1 : -1;
            const double v = 0.5 * (1.0 - 1.0 / fabs(sj));
            xl = undo_layer(xl, branch, v);
            xh = undo_layer(xh, branch, v);
        }
        const double eh = info->emax - xh * span, el = info->emax - xl * span;
        if (eh > best_homo) best_homo = eh;
        if (el < best_lumo) best_lumo = el;
        ++used;
    }
    if (used == 0 || !(best_lumo > best_homo)) return SP2_EINVAL;
    const double w = best_lumo - best_homo;
    *homo = best_homo + kMargin * w;
    *lumo = best_lumo - kMargin * w;
    return SP2_OK;
}

}  // extern "C"
