// Lowest eigenpair of the Lanczos tridiagonal H_eff (host, float64).
//
// Diagonal a[0..m), off-diagonal b[1..m) (b[i] couples i-1 and i).
// Eigenvalue: bisection on the Sturm count of T - x I (the number of negative
// pivots of its LDL^T factorisation equals the number of eigenvalues below x)
// inside the Gershgorin interval, down to the last bit.
// Eigenvector: inverse iteration with the shift placed just below that
// eigenvalue, where T - shift I is positive definite and its LDL^T
// factorisation needs no pivoting.
#pragma once

#include <math.h>

#include <algorithm>
#include <vector>

namespace mcd {

inline int sturm_below(const double *a, const double *b, int m, double x) {
    int c = 0;
    double q = a[0] - x;
    const double tiny = 1e-300;
    if (q < 0.0) c++;
    for (int i = 1; i < m; i++) {
        if (q == 0.0) q = tiny;
        q = (a[i] - x) - b[i] * b[i] / q;
        if (q < 0.0) c++;
    }
    return c;
}

inline double tri_lowest(const double *a, const double *b, int m) {
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < m; i++) {
        const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < m ? fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    if (m == 1) return a[0];
    for (int it = 0; it < 200; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, b, m, mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

inline std::vector<double> tri_vector(const double *a, const double *b, int m, double lam) {
    std::vector<double> z(m, 1.0);
    if (m == 1) return z;
    double scale = 0.0;
    for (int i = 0; i < m; i++) scale = std::max(scale, fabs(a[i]) + (i ? fabs(b[i]) : 0.0));
    const double shift = lam - 1e-10 * std::max(1.0, scale);
    std::vector<double> d(m), l(m);
    d[0] = a[0] - shift;
    for (int i = 1; i < m; i++) {
        l[i] = b[i] / d[i - 1];
        d[i] = (a[i] - shift) - l[i] * b[i];
    }
    for (int it = 0; it < 4; it++) {
        for (int i = 1; i < m; i++) z[i] -= l[i] * z[i - 1];     // L y = z
        for (int i = 0; i < m; i++) z[i] /= d[i];                 // D w = y
        for (int i = m - 2; i >= 0; i--) z[i] -= l[i + 1] * z[i + 1];  // L^T x = w
        double nr = 0.0;
        for (int i = 0; i < m; i++) nr += z[i] * z[i];
        nr = sqrt(nr);
        for (int i = 0; i < m; i++) z[i] /= nr;
    }
    // fix the sign: largest component positive
    int im = 0;
    for (int i = 1; i < m; i++)
        if (fabs(z[i]) > fabs(z[im])) im = i;
    if (z[im] < 0)
        for (int i = 0; i < m; i++) z[i] = -z[i];
    return z;
}

}  // namespace mcd
