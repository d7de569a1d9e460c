// Small dense complex linear algebra on the host (FP64), for the projected
// problems of the eigensolver and the shifted solver: matrices of order up to
// a few hundred, row-major std::vector<std::complex<double>>.
//
//   eig_general   eigenvalues and right eigenvectors of a general matrix:
//                 Householder reduction to Hessenberg form, then the
//                 single-shift (Wilkinson) QR iteration with Givens rotations
//                 to complex Schur form T = Z^dag A Z, then back substitution
//                 on T (Golub & Van Loan, Matrix Computations, ch. 7);
//   inverse       Gauss-Jordan with partial pivoting.
// Host only; no device code.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace ovd {
namespace dense {

using cd = std::complex<double>;
using Mat = std::vector<cd>;   // row-major n x n

inline double cabs2(cd z) { return z.real() * z.real() + z.imag() * z.imag(); }

// Givens rotation [c s; -conj(s) c] (c real) with G [x; y] = [r; 0]
inline void givens(cd x, cd y, double& c, cd& s) {
    const double ax = std::abs(x), ay = std::abs(y);
    if (ay == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (ax == 0.0) {
        c = 0.0;
        s = std::conj(y) / ay;
        return;
    }
    const double nrm = std::hypot(ax, ay);
    c = ax / nrm;
    s = (x / ax) * std::conj(y) / nrm;
}

// Eigen-decomposition of a general n x n matrix.  w: n eigenvalues; V: right
// eigenvectors as columns (V[i * n + j] = component i of vector j), unit
// 2-norm.  Returns false if the QR iteration did not converge.
inline bool eig_general(int n, Mat A, std::vector<cd>& w, Mat& V) {
    w.assign(n, cd(0));
    V.assign((size_t)n * n, cd(0));
    Mat Z((size_t)n * n, cd(0));
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
    auto z = [&](int i, int j) -> cd& { return Z[(size_t)i * n + j]; };
    // 1. Hessenberg reduction by Householder reflections, accumulated into Z
    std::vector<cd> v(n);
    for (int k = 0; k + 2 < n; ++k) {
        double xn = 0.0;
        for (int i = k + 1; i < n; ++i) xn += cabs2(a(i, k));
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const cd x0 = a(k + 1, k);
        const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
        v[k + 1] += ph * xn;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += cabs2(v[i]);
        if (vn == 0.0) continue;
        const double f = 2.0 / vn;
        // A <- (I - f v v^dag) A
        for (int j = 0; j < n; ++j) {
            cd t = 0.0;
            for (int i = k + 1; i < n; ++i) t += std::conj(v[i]) * a(i, j);
            t *= f;
            for (int i = k + 1; i < n; ++i) a(i, j) -= v[i] * t;
        }
        // A <- A (I - f v v^dag),  Z <- Z (I - f v v^dag)
        for (int i = 0; i < n; ++i) {
            cd t = 0.0, u = 0.0;
            for (int j = k + 1; j < n; ++j) {
                t += a(i, j) * v[j];
                u += z(i, j) * v[j];
            }
            t *= f;
            u *= f;
            for (int j = k + 1; j < n; ++j) {
                a(i, j) -= t * std::conj(v[j]);
                z(i, j) -= u * std::conj(v[j]);
            }
        }
        for (int i = k + 2; i < n; ++i) a(i, k) = 0.0;
    }
    // 2. shifted QR iteration to upper triangular T, rotations accumulated into Z
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, iter = 0, total = 0;
    while (hi > 0) {
        int lo = hi;
        while (lo > 0) {
            const double sc = std::abs(a(lo, lo)) + std::abs(a(lo - 1, lo - 1));
            if (std::abs(a(lo, lo - 1)) <= eps * (sc > 0 ? sc : 1.0)) {
                a(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {   // a(hi, hi) converged
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 100 * n) return false;
        ++iter;
        // Wilkinson shift: eigenvalue of the trailing 2 x 2 closer to a(hi, hi)
        cd sigma;
        if (iter % 11 == 0) {
            sigma = a(hi, hi) + std::abs(a(hi, hi - 1)) * 0.75;   // exceptional shift
        } else {
            const cd p = a(hi - 1, hi - 1), q = a(hi - 1, hi), r = a(hi, hi - 1), s = a(hi, hi);
            const cd tr = p + s, det = p * s - q * r;
            const cd disc = std::sqrt(tr * tr * 0.25 - det);
            const cd e1 = tr * 0.5 + disc, e2 = tr * 0.5 - disc;
            sigma = std::abs(e1 - s) < std::abs(e2 - s) ? e1 : e2;
        }
        // implicit single-shift bulge chase on rows/columns lo..hi
        cd x = a(lo, lo) - sigma, y = a(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            double c;
            cd s;
            givens(x, y, c, s);
            // rows k, k+1 (columns from max(lo, k-1) to n-1)
            for (int j = std::max(lo, k - 1); j < n; ++j) {
                const cd t1 = a(k, j), t2 = a(k + 1, j);
                a(k, j) = c * t1 + s * t2;
                a(k + 1, j) = -std::conj(s) * t1 + c * t2;
            }
            // columns k, k+1 (rows 0 .. min(k+2, hi)), and Z
            const int imax = std::min(k + 2, hi);
            for (int i = 0; i <= imax; ++i) {
                const cd t1 = a(i, k), t2 = a(i, k + 1);
                a(i, k) = c * t1 + std::conj(s) * t2;
                a(i, k + 1) = -s * t1 + c * t2;
            }
            for (int i = 0; i < n; ++i) {
                const cd t1 = z(i, k), t2 = z(i, k + 1);
                z(i, k) = c * t1 + std::conj(s) * t2;
                z(i, k + 1) = -s * t1 + c * t2;
            }
            if (k + 1 < hi) {
                x = a(k + 1, k);
                y = a(k + 2, k);
            }
        }
    }
    // 3. eigenvectors of T by back substitution, then V = Z X
    for (int i = 0; i < n; ++i) w[i] = a(i, i);
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) tnorm = std::max(tnorm, std::abs(a(i, j)));
    const double small = eps * (tnorm > 0 ? tnorm : 1.0);
    Mat X((size_t)n * n, cd(0));
    std::vector<cd> xv(n);
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < n; ++i) xv[i] = 0.0;
        xv[k] = 1.0;
        for (int j = k - 1; j >= 0; --j) {
            cd t = 0.0;
            for (int i = j + 1; i <= k; ++i) t += a(j, i) * xv[i];
            cd d = a(j, j) - w[k];
            if (std::abs(d) < small) d = small;
            xv[j] = -t / d;
        }
        for (int i = 0; i <= k; ++i) X[(size_t)i * n + k] = xv[i];
    }
    for (int j = 0; j < n; ++j) {
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            cd t = 0.0;
            for (int q = 0; q <= j; ++q) t += z(i, q) * X[(size_t)q * n + j];
            V[(size_t)i * n + j] = t;
            nrm += cabs2(t);
        }
        nrm = std::sqrt(nrm);
        if (nrm > 0)
            for (int i = 0; i < n; ++i) V[(size_t)i * n + j] /= nrm;
    }
    return true;
}

// general inverse (Gauss-Jordan, partial pivoting); false if singular
inline bool inverse(int n, Mat A, Mat& X) {
    X.assign((size_t)n * n, cd(0));
    for (int i = 0; i < n; ++i) X[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (std::abs(A[(size_t)i * n + c]) > std::abs(A[(size_t)p * n + c])) p = i;
        if (std::abs(A[(size_t)p * n + c]) == 0.0) return false;
        if (p != c)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)p * n + j], A[(size_t)c * n + j]);
                std::swap(X[(size_t)p * n + j], X[(size_t)c * n + j]);
            }
        const cd piv = A[(size_t)c * n + c];
        for (int j = 0; j < n; ++j) {
            A[(size_t)c * n + j] /= piv;
            X[(size_t)c * n + j] /= piv;
        }
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            const cd f = A[(size_t)i * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)i * n + j] -= f * A[(size_t)c * n + j];
                X[(size_t)i * n + j] -= f * X[(size_t)c * n + j];
            }
        }
    }
    return true;
}

}  // namespace dense
}  // namespace ovd
