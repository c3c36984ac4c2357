// Lowest eigenpair of the Lanczos tridiagonal matrix T_n (Sec. 3.4), host FP64.
//
// Eigenvalue: bisection on the Sturm count (number of negative pivots of the
// LDL^T factorization of T - x I) inside the Gershgorin interval.
// Eigenvector: inverse iteration with Gaussian elimination with partial
// pivoting on the tridiagonal T - lambda I.
#include <cmath>
#include <vector>

#include "hphi_internal.h"

namespace hphi {
namespace {

int sturm_count(const double* a, const double* b, int n, double x) {
    int neg = 0;
    double d = a[0] - x;
    const double tiny = 1e-300;
    if (d < 0) ++neg;
    for (int i = 1; i < n; ++i) {
        if (std::fabs(d) < tiny) d = -tiny;
        d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
        if (d < 0) ++neg;
    }
    return neg;
}

// Solve (T - lam I) z = rhs in place (partial pivoting, 2 super-diagonals).
void tridiag_solve(const double* a, const double* b, int n, double lam, std::vector<double>& z) {
    std::vector<double> d(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a[i] - lam;
    for (int i = 0; i + 1 < n; ++i) {
        du[i] = b[i];
        dl[i] = b[i];
    }
    std::vector<int> piv(n, 0);
    const double eps = 1e-300;
    for (int i = 0; i + 1 < n; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
            if (std::fabs(d[i]) < eps) d[i] = eps;
            const double f = dl[i] / d[i];
            dl[i] = f;
            d[i + 1] -= f * du[i];
            du2[i] = 0.0;
        } else {
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = d[i + 1];
            d[i + 1] = t - f * d[i + 1];
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
            piv[i] = 1;
        }
    }
    if (std::fabs(d[n - 1]) < eps) d[n - 1] = eps;
    // forward: apply L^{-1} with the recorded interchanges
    for (int i = 0; i + 1 < n; ++i) {
        if (piv[i]) {
            const double t = z[i];
            z[i] = z[i + 1];
            z[i + 1] = t - dl[i] * z[i + 1];
        } else {
            z[i + 1] -= dl[i] * z[i];
        }
    }
    // back substitution with U (diag d, super du, super-2 du2)
    z[n - 1] /= d[n - 1];
    if (n > 1) z[n - 2] = (z[n - 2] - du[n - 2] * z[n - 1]) / d[n - 2];
    for (int i = n - 3; i >= 0; --i) z[i] = (z[i] - du[i] * z[i + 1] - du2[i] * z[i + 2]) / d[i];
}

}  // namespace

double tridiag_lowest(const double* a, const double* b, int n, double* evec) {
    if (n == 1) {
        if (evec) evec[0] = 1.0;
        return a[0];
    }
    double lo = a[0], hi = a[0];
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        if (i > 0) r += std::fabs(b[i - 1]);
        if (i + 1 < n) r += std::fabs(b[i]);
        lo = std::fmin(lo, a[i] - r);
        hi = std::fmax(hi, a[i] + r);
    }
    // bisection for the smallest eigenvalue: count(x) >= 1 iff x > lambda_0
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, n, mid) >= 1) hi = mid; else lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    if (evec) {
        std::vector<double> z(n, 1.0);
        double scale = 0.0;
        for (int i = 0; i < n; ++i) scale = std::fmax(scale, std::fabs(a[i]) + std::fabs(i + 1 < n ? b[i] : 0.0));
        const double shift = lam - 4.0 * 2.220446049250313e-16 * (scale > 1.0 ? scale : 1.0);
        for (int it = 0; it < 4; ++it) {
            tridiag_solve(a, b, n, shift, z);
            double nrm = 0.0;
            for (double x : z) nrm += x * x;
            nrm = std::sqrt(nrm);
            for (double& x : z) x /= nrm;
        }
        // fixed sign: largest-magnitude component positive
        int imax = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(z[i]) > std::fabs(z[imax])) imax = i;
        const double sgn = z[imax] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) evec[i] = sgn * z[i];
    }
    return lam;
}

}  // namespace hphi
