// Host check of the small dense algebra used by the eigensolver: reads a
// matrix from stdin (n, then n*n pairs re im, row-major), prints its
// eigenvalues and the max residual |A v - w v| of the eigenvectors, then the
// error of A A^{-1}.
#include "../../paper_1611_00195_amd/csrc/dense.hpp"

#include <cstdio>

using namespace ovd::dense;

int main() {
    int n = 0;
    if (std::scanf("%d", &n) != 1 || n < 1) return 2;
    Mat A((size_t)n * n);
    for (auto& x : A) {
        double re, im;
        if (std::scanf("%lf %lf", &re, &im) != 2) return 2;
        x = cd(re, im);
    }
    std::vector<cd> w;
    Mat V;
    if (!eig_general(n, A, w, V)) return 3;
    double res = 0.0;
    for (int j = 0; j < n; ++j) {
        double r = 0.0;
        for (int i = 0; i < n; ++i) {
            cd t = 0.0;
            for (int k = 0; k < n; ++k) t += A[(size_t)i * n + k] * V[(size_t)k * n + j];
            r += std::norm(t - w[j] * V[(size_t)i * n + j]);
        }
        res = std::max(res, std::sqrt(r));
    }
    for (int j = 0; j < n; ++j) std::printf("%.17g %.17g\n", w[j].real(), w[j].imag());
    Mat X;
    double e2 = -1.0;
    if (inverse(n, A, X)) {
        e2 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cd t = 0.0;
                for (int k = 0; k < n; ++k) t += A[(size_t)i * n + k] * X[(size_t)k * n + j];
                e2 = std::max(e2, std::abs(t - (i == j ? 1.0 : 0.0)));
            }
    }
    std::printf("residual %.6e\ninverse %.6e\n", res, e2);
    return 0;
}
