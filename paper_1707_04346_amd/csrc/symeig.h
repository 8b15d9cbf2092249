// symeig.h -- eigenvalues and eigenvectors of a small dense real symmetric
// matrix on the host: Householder reduction to tridiagonal form with the
// transformations accumulated, then the implicit-shift QL iteration on the
// tridiagonal matrix (the Wilkinson-Reinsch method).  O(n^3); used for the
// Davidson projected matrix (n <= 512) and the P-space block (n <= 2048).
// Header-only, plain C++: no device code.
#pragma once

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace cis {

// A: n x n row-major symmetric (taken by value).  On return w holds the
// eigenvalues in ascending order and V (n x n row-major) the matching
// orthonormal eigenvectors in its columns: V[i * n + r] is component i of
// eigenvector r.  Returns false if the QL iteration failed to converge (the
// results are then those reached).
inline bool sym_eig(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &V) {
    w.assign(n, 0.0);
    V.assign(size_t(n) * n, 0.0);
    if (n <= 0) return true;
    auto a = [&](int i, int j) -> double & { return A[size_t(i) * n + j]; };
    auto z = [&](int i, int j) -> double & { return V[size_t(i) * n + j]; };
    for (int i = 0; i < n; ++i) z(i, i) = 1.0;
    std::vector<double> v(n), p(n), e(n, 0.0);
    // Householder: for column k, reflect A[k+1.., k] onto a multiple of the first unit vector
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;                     // length of the reflected part
        double xn = 0;
        for (int i = 0; i < m; ++i) xn += a(k + 1 + i, k) * a(k + 1 + i, k);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const double alpha = a(k + 1, k) > 0 ? -xn : xn;
        double vn = 0;
        for (int i = 0; i < m; ++i) {
            v[i] = a(k + 1 + i, k) - (i == 0 ? alpha : 0.0);
            vn += v[i] * v[i];
        }
        if (vn == 0.0) continue;
        const double beta = 2.0 / vn;
        // p = beta * A_sub v, K = beta/2 * v.p, q = p - K v; A_sub -= v q^T + q v^T
        double vp = 0;
        for (int i = 0; i < m; ++i) {
            double s = 0;
            for (int j = 0; j < m; ++j) s += a(k + 1 + i, k + 1 + j) * v[j];
            p[i] = beta * s;
            vp += v[i] * p[i];
        }
        const double K = 0.5 * beta * vp;
        for (int i = 0; i < m; ++i) p[i] -= K * v[i];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) a(k + 1 + i, k + 1 + j) -= v[i] * p[j] + p[i] * v[j];
        a(k + 1, k) = a(k, k + 1) = alpha;
        for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
        // V <- V H on columns k+1..n-1
        for (int r = 0; r < n; ++r) {
            double s = 0;
            for (int j = 0; j < m; ++j) s += z(r, k + 1 + j) * v[j];
            s *= beta;
            if (s != 0.0)
                for (int j = 0; j < m; ++j) z(r, k + 1 + j) -= s * v[j];
        }
    }
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i) d[i] = a(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);   // e[i] couples i and i + 1
    // implicit-shift QL on (d, e), rotations accumulated into the columns of V,
    // held transposed (Zt row r = column r of V) so a rotation updates two rows
    std::vector<double> Zt(size_t(n) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Zt[size_t(j) * n + i] = V[size_t(i) * n + j];
    bool ok = true;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (iter == 60) { ok = false; break; }
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, pp = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {                      // split: the chase ends early
                    d[i + 1] -= pp;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * s + 2.0 * c * b;
                pp = s * r;
                d[i + 1] = g + pp;
                g = c * r - b;
                double *zi = &Zt[size_t(i) * n], *zf = &Zt[size_t(i + 1) * n];
                for (int k = 0; k < n; ++k) {
                    const double f1 = zf[k], f0 = zi[k];
                    zf[k] = s * f0 + c * f1;
                    zi[k] = c * f0 - s * f1;
                }
            }
            if (deflated) continue;
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // ascending order
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        const double *col = &Zt[size_t(idx[j]) * n];
        for (int i = 0; i < n; ++i) V[size_t(i) * n + j] = col[i];
    }
    return ok;
}

}  // namespace cis
