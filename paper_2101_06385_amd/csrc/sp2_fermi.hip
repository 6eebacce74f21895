// Fit of the optimized finite-temperature expansion (Sec. "Optimized SP2 Finite
// Temperature Fermi-Operator Expansion"), host code.
//
// Scalar model on the rescaled energy x in [0, 1]:
//   x_0 = x,  x_k = t_{k-1,1} x_{k-1}^2 + t_{k-1,2} x_{k-1} + t_{k-1,3}   (Eq. general SP2)
//   F~(x) = 1 - sum_{i=0}^{L} c_i x_i                                      (its read-out)
// fitted to F(x) = 1 / (exp(beta (x - m)) + 1) (Eq. fermi), with beta = (emax - emin)/kT and
// m = (mu - emin)/(emax - emin), by minimizing sum_i w_i [F~(x_i) - F(x_i)]^2 over `grid`
// equally spaced points with trapezoid weights (an approximation of the integral of the
// squared error).  Levenberg-Marquardt: solve (J^T J + lambda diag(J^T J)) d = -J^T r by
// Cholesky, accept a step that lowers the loss and divide lambda by 10, else multiply it
// by 10; lambda starts at 1e-3; stop after max_iter steps or once lambda exceeds 1e12.
// The start is the truncated SP2 expansion whose branch at each layer keeps the image of
// m closest to 1/2 (x^2 on a tie), read out as 1 - x_L.
#include "sp2_internal.h"

#include <math.h>

#include <vector>

namespace {

struct FitProblem {
    int L, m;
    std::vector<double> x, sw, target;   // grid, sqrt(weights), F on the grid
};

// residuals r_i = sqrt(w_i) (F~(x_i) - F(x_i)); returns sum r_i^2; jac (m x P, row major)
// filled when non-null, by the chain rule backwards through the layers
double evaluate(const FitProblem& fp, const std::vector<double>& p, std::vector<double>* r,
                std::vector<double>* jac, std::vector<double>& xs) {
    const int L = fp.L, P = 4 * L + 1;
    const double* th = p.data();
    const double* c = p.data() + 3 * L;
    double sum = 0.0;
    for (int i = 0; i < fp.m; ++i) {
        xs[0] = fp.x[i];
        for (int k = 0; k < L; ++k) {
            const double v = xs[k];
            xs[k + 1] = th[3 * k] * v * v + th[3 * k + 1] * v + th[3 * k + 2];
        }
        double f = 1.0;
        for (int k = 0; k <= L; ++k) f -= c[k] * xs[k];
        const double ri = fp.sw[i] * (f - fp.target[i]);
        if (r) (*r)[i] = ri;
        sum += ri * ri;
        if (jac) {
            double* row = jac->data() + (size_t)i * P;
            for (int k = 0; k <= L; ++k) row[3 * L + k] = -fp.sw[i] * xs[k];
            double g = -c[L];   // dF~/dx_L
            for (int k = L - 1; k >= 0; --k) {
                const double v = xs[k];
                row[3 * k] = fp.sw[i] * g * v * v;
                row[3 * k + 1] = fp.sw[i] * g * v;
                row[3 * k + 2] = fp.sw[i] * g;
                g = -c[k] + g * (2.0 * th[3 * k] * v + th[3 * k + 1]);
            }
        }
    }
    return sum;
}

// In-place Cholesky solve of the SPD system a d = b (P x P, row major); false if not SPD.
bool cholesky_solve(std::vector<double>& a, std::vector<double>& b, int P) {
    for (int j = 0; j < P; ++j) {
        double d = a[(size_t)j * P + j];
        for (int k = 0; k < j; ++k) d -= a[(size_t)j * P + k] * a[(size_t)j * P + k];
        if (!(d > 0.0) || !isfinite(d)) return false;
        d = sqrt(d);
        a[(size_t)j * P + j] = d;
        for (int i = j + 1; i < P; ++i) {
            double s = a[(size_t)i * P + j];
            for (int k = 0; k < j; ++k) s -= a[(size_t)i * P + k] * a[(size_t)j * P + k];
            a[(size_t)i * P + j] = s / d;
        }
    }
    for (int i = 0; i < P; ++i) {   // L y = b
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= a[(size_t)i * P + k] * b[k];
        b[i] = s / a[(size_t)i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {   // L^T d = y
        double s = b[i];
        for (int k = i + 1; k < P; ++k) s -= a[(size_t)k * P + i] * b[k];
        b[i] = s / a[(size_t)i * P + i];
    }
    return true;
}

}  // namespace

extern "C" {

int sp2_fermi_fit(int layers, double mu, double kT, double emin, double emax, int grid, int max_iter,
                  double* theta, double* c, double* loss) {
    if (layers < 1 || layers >= SP2_MAX_LAYERS || grid < 3 || grid > 1000000 || max_iter < 0 || !theta || !c)
        return SP2_EINVAL;
    if (!(isfinite(mu) && isfinite(kT) && isfinite(emin) && isfinite(emax) && kT > 0.0 && emax > emin))
        return SP2_EINVAL;
    const double span = emax - emin;
    const double beta = span / kT, m0 = (mu - emin) / span;
    FitProblem fp;
    fp.L = layers;
    fp.m = grid;
    fp.x.resize(grid);
    fp.sw.resize(grid);
    fp.target.resize(grid);
    for (int i = 0; i < grid; ++i) {
        const double x = (double)i / (grid - 1);
        const double w = (i == 0 || i == grid - 1) ? 0.5 / (grid - 1) : 1.0 / (grid - 1);
        const double z = beta * (x - m0);
        fp.x[i] = x;
        fp.sw[i] = sqrt(w);
        fp.target[i] = z > 0.0 ? exp(-z) / (1.0 + exp(-z)) : 1.0 / (1.0 + exp(z));
    }
    const int L = layers, P = 4 * L + 1;
    std::vector<double> p(P, 0.0);
    double im = m0;
    for (int k = 0; k < L; ++k) {
        const double sq = im * im, pr = 2.0 * im - im * im;
        if (fabs(sq - 0.5) <= fabs(pr - 0.5)) {
            p[3 * k] = 1.0;
            im = sq;
        } else {
            p[3 * k] = -1.0;
            p[3 * k + 1] = 2.0;
            im = pr;
        }
    }
    p[3 * L + L] = 1.0;
    std::vector<double> xs(L + 1), r(grid), jac((size_t)grid * P), a((size_t)P * P), g(P), trial(P);
    double cur = evaluate(fp, p, nullptr, nullptr, xs);
    double lam = 1e-3;
    for (int it = 0; it < max_iter && lam <= 1e12; ++it) {
        evaluate(fp, p, &r, &jac, xs);
        for (int u = 0; u < P; ++u) {
            double gs = 0.0;
            for (int i = 0; i < grid; ++i) gs += jac[(size_t)i * P + u] * r[i];
            g[u] = -gs;
            for (int v = 0; v <= u; ++v) {
                double s = 0.0;
                for (int i = 0; i < grid; ++i) s += jac[(size_t)i * P + u] * jac[(size_t)i * P + v];
                a[(size_t)u * P + v] = s;
                a[(size_t)v * P + u] = s;
            }
        }
        for (int u = 0; u < P; ++u) a[(size_t)u * P + u] *= 1.0 + lam;
        std::vector<double> d = g;
        bool ok = cholesky_solve(a, d, P);
        double nw = INFINITY;
        if (ok) {
            for (int u = 0; u < P; ++u) trial[u] = p[u] + d[u];
            nw = evaluate(fp, trial, nullptr, nullptr, xs);
        }
        if (ok && nw < cur) {
            p.swap(trial);
            cur = nw;
            lam /= 10.0;
        } else {
            lam *= 10.0;
        }
    }
    for (int k = 0; k < 3 * L; ++k) theta[k] = p[k];
    for (int k = 0; k <= L; ++k) c[k] = p[3 * L + k];
    if (loss) *loss = cur;
    return isfinite(cur) ? SP2_OK : SP2_ENONFINITE;
}

}  // extern "C"
