// Deflation data on the GPU: the m eigenvalues of smallest |lambda| of
// H(mu) = gamma5 Dw(mu) with right and left eigenvectors (L^dag R = 1, Sec. 3,
// eq. 8), and the derivatives of the first l eigenvector pairs along mu or a
// link direction (Sec. 3, eq. 10-11 with the eigenvector derivative of the
// perturbation expansion).
//
// Eigenpairs: Chebyshev-filtered subspace iteration on H^2.  The wanted
// eigenvalues are the smallest |lambda|, interior for H but at the lower end
// of the spectrum of H^2 (lambda^2, close to the positive real axis), so a
// Chebyshev polynomial of H^2 that is bounded on [a, b] (b an upper bound of
// |lambda|^2, a the largest Ritz value of the current subspace) amplifies
// them.  Each outer iteration: filter the p = m + extra vectors, orthonormalise
// (Cholesky QR, twice), Rayleigh-Ritz with H itself (projected p x p problem
// solved on the host by the QR algorithm), residual norms from the Gram matrix
// of H Q - Q G.  The same run on H^dag = H(-mu) gives the left subspace; the
// left vectors are then the dual basis of the right ones in it (L^dag R = 1).
//
// Derivatives (gauge L_j^dag dR_j = 0, dL_j^dag R_j = 0), with P = sum_{i<m} R_i L_i^dag:
//   dR_j = sum_{i != j} R_i (L_i^dag dA R_j) / (lambda_j - lambda_i)
//          + (lambda_j - A)^{-1} (1 - P) dA R_j            (solved on range(1 - P))
//   dL_j = sum_{i != j} L_i conj((L_j^dag dA R_i) / (lambda_j - lambda_i))
//          + (conj(lambda_j) - A^dag)^{-1} (1 - P)^dag dA^dag L_j
// The shifted systems are solved by restarted GMRES with classical
// Gram-Schmidt applied twice; every long-vector product is a stencil launch
// or an MFMA projection (kernels_defl.hip), the small problems run on the host.
#include "ovd_internal.h"
#include "dense.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace ovd {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// seeded start vectors: every component uniform in (-1/2, 1/2) + i (-1/2, 1/2)
// from a counter-based hash (splitmix64 of seed and position); padding sites zero
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ void fill_random_kernel(long long n_elem, long long nf, int V, int Vp, uint64_t seed, c64* __restrict__ out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    const int s = (int)((e % nf) % Vp);
    if (s >= V) {
        out[e] = c64{0.0, 0.0};
        return;
    }
    const uint64_t a = mix64(seed * 0x100000001B3ull + 2 * (uint64_t)e);
    const uint64_t b = mix64(seed * 0x100000001B3ull + 2 * (uint64_t)e + 1);
    const double inv = 1.0 / 9007199254740992.0;   // 2^-53
    out[e] = c64{(double)(a >> 11) * inv - 0.5, (double)(b >> 11) * inv - 0.5};
}

// out = a X + b Y + c Z (complex scalars; Y, Z may be null)
__global__ void lincomb_kernel(long long n_elem, c64 a, const c64* __restrict__ X, c64 b, const c64* __restrict__ Y,
                               c64 c, const c64* __restrict__ Z, c64* __restrict__ out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        c64 r = a * X[e];
        if (Y) r += b * Y[e];
        if (Z) r += c * Z[e];
        out[e] = r;
    }
}

namespace {

// progress lines on stderr when OVDERIV_VERBOSE is set (long setup runs)
bool verbose() {
    static const bool v = std::getenv("OVDERIV_VERBOSE") != nullptr;
    return v;
}

// ---------------------------------------------------------------------------
// host-side helpers
// ---------------------------------------------------------------------------
struct Ctx {
    Geom g;
    const c64* U;
    const c64* dU;
    double md;
    hipStream_t s;
    long long nf;
    std::string err;
    std::vector<void*> owned;
    c64* scr = nullptr;      // projection scratch
    size_t scr_elems = 0;
    c64* small = nullptr;    // device staging of small matrices
    size_t small_elems = 0;
    double* emu = nullptr;   // device (e^{m}, e^{-m}) per field, 2 x max fields
    int emu_n = 0;
    double emu_mu = 1e300;

    ~Ctx() {
        for (void* p : owned) (void)hipFree(p);
    }
    bool ok(hipError_t e, const char* what) {
        if (e != hipSuccess && err.empty()) err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipSuccess;
    }
    c64* fields(int n) {
        void* p = nullptr;
        const size_t bytes = sizeof(c64) * (size_t)(n > 0 ? n : 1) * nf;
        if (!ok(hipMalloc(&p, bytes), "hipMalloc")) return nullptr;
        owned.push_back(p);
        if (!ok(hipMemsetAsync(p, 0, bytes, s), "hipMemsetAsync")) return nullptr;
        return (c64*)p;
    }
    bool ensure_scratch(int m, int nr) {
        const size_t need = defl_proj_scratch(m, nr, nf);
        if (need <= scr_elems) return true;
        void* p = nullptr;
        if (!ok(hipMalloc(&p, sizeof(c64) * need), "hipMalloc")) return false;
        owned.push_back(p);
        scr = (c64*)p;
        scr_elems = need;
        return true;
    }
    bool ensure_small(size_t n) {
        if (n <= small_elems) return true;
        void* p = nullptr;
        if (!ok(hipMalloc(&p, sizeof(c64) * n), "hipMalloc")) return false;
        owned.push_back(p);
        small = (c64*)p;
        small_elems = n;
        return true;
    }
    // (e^{mu}, e^{-mu}) for n fields
    bool set_mu(double mu, int n) {
        if (mu == emu_mu && n <= emu_n) return true;
        const int cap = std::max(n, emu_n);
        if (cap > emu_n) {
            void* p = nullptr;
            if (!ok(hipMalloc(&p, sizeof(double) * 2 * cap), "hipMalloc")) return false;
            owned.push_back(p);
            emu = (double*)p;
            emu_n = cap;
        }
        std::vector<double> h(2 * (size_t)emu_n);
        for (int i = 0; i < emu_n; ++i) {
            h[2 * i] = std::exp(mu);
            h[2 * i + 1] = std::exp(-mu);
        }
        if (!ok(hipMemcpyAsync(emu, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s), "copy"))
            return false;
        if (!ok(hipStreamSynchronize(s), "sync")) return false;
        emu_mu = mu;
        return true;
    }
    // out = op(mu) in, n fields (op: 0 H, 2 dH/dmu, 3 dH/dlink)
    bool apply(int op, double mu, const c64* in, c64* out, int n) {
        if (!set_mu(mu, n)) return false;
        launch_apply_op<double>(g, op, n, emu, U, dU, md, in, out, s);
        return ok(hipGetLastError(), "apply_op");
    }
    // C (m x nr, host) = A^dag B
    bool proj(const c64* A, int m, const c64* B, int nr, std::vector<cd>& C) {
        if (!ensure_scratch(m, nr) || !ensure_small((size_t)m * nr)) return false;
        launch_defl_proj(A, nf, m, B, nf, nr, nf, small, scr, s);
        C.resize((size_t)m * nr);
        if (!ok(hipMemcpyAsync(C.data(), small, sizeof(c64) * m * nr, hipMemcpyDeviceToHost, s), "copy")) return false;
        return ok(hipStreamSynchronize(s), "sync");
    }
    // Y += A C (C host, m x nr)
    bool comb(const c64* A, int m, const std::vector<cd>& C, int nr, c64* Y) {
        if (!ensure_small((size_t)m * nr)) return false;
        if (!ok(hipMemcpyAsync(small, C.data(), sizeof(c64) * m * nr, hipMemcpyHostToDevice, s), "copy")) return false;
        launch_defl_comb(A, nf, m, small, nr, Y, nf, nf, s);
        if (!ok(hipGetLastError(), "defl_comb")) return false;
        return ok(hipStreamSynchronize(s), "sync");   // the staging buffer is reused next
    }
    bool lincomb(long long n_elem, cd a, const c64* X, cd b, const c64* Y, cd c, const c64* Z, c64* out) {
        long long nb = (n_elem + 255) / 256;
        if (nb > 8192) nb = 8192;
        lincomb_kernel<<<(unsigned)nb, 256, 0, s>>>(n_elem, c64{a.real(), a.imag()}, X, c64{b.real(), b.imag()}, Y,
                                                   c64{c.real(), c.imag()}, Z, out);
        return ok(hipGetLastError(), "lincomb");
    }
    bool copy(c64* dst, const c64* src, int n) {
        return ok(hipMemcpyAsync(dst, src, sizeof(c64) * (size_t)n * nf, hipMemcpyDeviceToDevice, s), "copy");
    }
    double norm(const c64* x) {
        std::vector<cd> c;
        if (!proj(x, 1, x, 1, c)) return -1.0;
        return std::sqrt(std::max(0.0, c[0].real()));
    }
};

// Q = Y R^{-1} with Y^dag Y = R^dag R, twice (Cholesky QR 2); Y is overwritten by Q
bool orthonormalise(Ctx& c, c64* Y, c64* T, int p) {
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<cd> G, R;
        if (!c.proj(Y, p, Y, p, G)) return false;
        // symmetrise and lift the diagonal slightly for a safe factorisation
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) {
                const cd a = 0.5 * (G[(size_t)i * p + j] + std::conj(G[(size_t)j * p + i]));
                G[(size_t)i * p + j] = a;
                G[(size_t)j * p + i] = std::conj(a);
            }
        double dmax = 0.0;
        for (int i = 0; i < p; ++i) dmax = std::max(dmax, G[(size_t)i * p + i].real());
        for (int i = 0; i < p; ++i) G[(size_t)i * p + i] += 1e-15 * dmax;
        if (!dense::cholesky_upper(p, G, R)) {
            c.err = "Cholesky QR failed: the filtered vectors lost rank";
            return false;
        }
        const std::vector<cd> Ri = dense::inv_upper(p, R);
        if (!c.ok(hipMemsetAsync(T, 0, sizeof(c64) * (size_t)p * c.nf, c.s), "memset")) return false;
        if (!c.comb(Y, p, Ri, p, T)) return false;
        if (!c.copy(Y, T, p)) return false;
    }
    return true;
}

// Chebyshev filter of degree d in H(mu)^2 on [a, b]: out = T_d(((H^2) - c)/e) X
// (three buffers rotate; the result ends up in *res)
bool cheb_filter(Ctx& c, double mu, const c64* X, c64* B0, c64* B1, c64* B2, c64* T, int p, int d, double a,
                 double b, c64** res) {
    const long long ne = (long long)p * c.nf;
    const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
    // B1 = (H^2 X - cc X) / e
    if (!c.apply(0, mu, X, T, p) || !c.apply(0, mu, T, B1, p)) return false;
    if (!c.lincomb(ne, 1.0 / e, B1, -cc / e, X, 0.0, nullptr, B1)) return false;
    if (!c.copy(B0, X, p)) return false;
    c64 *y0 = B0, *y1 = B1, *y2 = B2;
    for (int k = 2; k <= d; ++k) {
        if (!c.apply(0, mu, y1, T, p) || !c.apply(0, mu, T, y2, p)) return false;
        if (!c.lincomb(ne, 2.0 / e, y2, -2.0 * cc / e, y1, -1.0, y0, y2)) return false;
        c64* t = y0;
        y0 = y1;
        y1 = y2;
        y2 = t;
    }
    *res = y1;
    return true;
}

struct SideResult {
    std::vector<cd> theta;   // m Ritz values, increasing |theta|
    int outer = 0;
    double max_res = 0.0;
};

// sort the eigenpairs (w, S) of a p x p projected matrix by |w| (S columns)
void sort_by_modulus(int p, std::vector<cd>& w, std::vector<cd>& S) {
    std::vector<int> ord(p);
    for (int i = 0; i < p; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int i, int j) { return std::abs(w[i]) < std::abs(w[j]); });
    std::vector<cd> Ss((size_t)p * p), ws(p);
    for (int j = 0; j < p; ++j) {
        ws[j] = w[ord[j]];
        for (int i = 0; i < p; ++i) Ss[(size_t)i * p + j] = S[(size_t)i * p + ord[j]];
    }
    w.swap(ws);
    S.swap(Ss);
}

// residual norms |(W - Q G) s_j| (Q orthonormal, G = Q^dag W) of the first n columns of S
bool ritz_residuals(Ctx& c, const c64* Q, const c64* W, c64* Z, int p, const std::vector<cd>& G,
                    const std::vector<cd>& S, int n, std::vector<double>& res) {
    if (!c.copy(Z, W, p)) return false;
    std::vector<cd> mG(G.size());
    for (size_t i = 0; i < G.size(); ++i) mG[i] = -G[i];
    if (!c.comb(Q, p, mG, p, Z)) return false;
    std::vector<cd> E;
    if (!c.proj(Z, p, Z, p, E)) return false;
    res.assign(n, 0.0);
    for (int j = 0; j < n; ++j) {
        cd acc = 0.0;
        for (int i = 0; i < p; ++i) {
            cd t = 0.0;
            for (int k = 0; k < p; ++k) t += E[(size_t)i * p + k] * S[(size_t)k * p + j];
            acc += std::conj(S[(size_t)i * p + j]) * t;
        }
        res[j] = std::sqrt(std::max(0.0, acc.real()));
    }
    return true;
}

// Subspace iteration for one side (mu or -mu).  The filter and the subspace
// update use Rayleigh-Ritz with H^2, whose wanted eigenvalues lambda^2 are at
// the edge of its spectrum (Rayleigh-Ritz with H itself would produce spurious
// Ritz values near zero from mixtures of eigenvectors of opposite sign); the
// m best vectors are then projected with H to separate lambda from -lambda and
// to measure the residual |H r - lambda r|.  The m eigenvectors of H end up in
// Out (unit norm), increasing |lambda|.
bool subspace_side(Ctx& c, double mu, int m, int p, double tol, int max_outer, int degree, uint64_t seed, c64* Out,
                   SideResult& sr) {
    c64* X = c.fields(p);
    c64* B0 = c.fields(p);
    c64* B1 = c.fields(p);
    c64* B2 = c.fields(p);
    c64* T = c.fields(p);
    c64* Qm = c.fields(p);
    c64* Wm = c.fields(p);
    c64* Zm = c.fields(p);
    if (!X || !B0 || !B1 || !B2 || !T || !Qm || !Wm || !Zm) return false;
    {
        const long long ne = (long long)p * c.nf;
        fill_random_kernel<<<(unsigned)((ne + 255) / 256), 256, 0, c.s>>>(ne, c.nf, c.g.V, c.g.Vp, seed, X);
        if (!c.ok(hipGetLastError(), "fill_random")) return false;
    }
    if (!orthonormalise(c, X, T, p)) return false;
    // upper bound of |lambda|^2: ||Dw|| <= |m0 + 4| + 3 + e^{|mu|} (r = 1, unit-norm links)
    const double hb = std::fabs(c.md) + 3.0 + std::exp(std::fabs(mu));
    const double b = 1.02 * hb * hb;
    double a = 0.25 * b;
    double best = 1e300;
    int best_it = 0;
    for (int it = 1; it <= max_outer; ++it) {
        c64* Y = nullptr;
        if (!cheb_filter(c, mu, X, B0, B1, B2, T, p, degree, a, b, &Y)) return false;
        c64* Q = Y;
        c64* Wb = (Q == B0) ? B1 : B0;     // H Q, then H^2 Q
        c64* Zb = (Q == B2) ? B1 : B2;
        if (!orthonormalise(c, Q, T, p)) return false;
        if (!c.apply(0, mu, Q, T, p) || !c.apply(0, mu, T, Wb, p)) return false;
        std::vector<cd> G2;
        if (!c.proj(Q, p, Wb, p, G2)) return false;
        std::vector<cd> w2, S2;
        if (!dense::eig_general(p, G2, w2, S2)) {
            c.err = "QR iteration of the projected problem did not converge";
            return false;
        }
        sort_by_modulus(p, w2, S2);
        // next start: all p Ritz vectors of H^2
        if (!c.ok(hipMemsetAsync(X, 0, sizeof(c64) * (size_t)p * c.nf, c.s), "memset")) return false;
        if (!c.comb(Q, p, S2, p, X)) return false;
        // H is projected on the first mq >= m Ritz vectors of H^2, mq at the
        // largest relative gap of |theta^2| in [m, p - 4].  A weak gauge field
        // leaves the spectrum of H close to symmetric (lambda next to some
        // -lambda'), H^2 cannot tell such a pair apart and its Ritz vectors mix
        // the two; H separates them only when the whole cluster is in the space.
        int mq = m;
        {
            double gbest = -1.0;
            const int jmax = std::min(p - 1, std::max(m, p - 4));
            for (int j = m; j <= jmax; ++j) {
                const double gap = (std::abs(w2[j]) - std::abs(w2[j - 1])) / std::max(std::abs(w2[j - 1]), 1e-300);
                if (gap > gbest) {
                    gbest = gap;
                    mq = j;
                }
            }
        }
        // orthonormalise, project H, keep the m smallest |lambda|, residuals |H r - lambda r|
        if (!c.copy(Qm, X, mq)) return false;
        if (!orthonormalise(c, Qm, Zm, mq)) return false;
        if (!c.apply(0, mu, Qm, Wm, mq)) return false;
        std::vector<cd> G, w, S;
        if (!c.proj(Qm, mq, Wm, mq, G)) return false;
        if (!dense::eig_general(mq, G, w, S)) {
            c.err = "QR iteration of the projected problem did not converge";
            return false;
        }
        sort_by_modulus(mq, w, S);
        std::vector<double> res;
        if (!ritz_residuals(c, Qm, Wm, Zm, mq, G, S, m, res)) return false;
        const double rmax = *std::max_element(res.begin(), res.end());
        sr.theta.assign(w.begin(), w.begin() + m);
        sr.outer = it;
        sr.max_res = rmax;
        if (verbose()) {
            int nconv = 0;
            while (nconv < m && res[nconv] <= tol) ++nconv;
            std::fprintf(stderr,
                         "eigs mu=%+.3f outer %d: max residual %.3e, first %d converged, res_1 %.1e, |lambda_m| %.6f, "
                         "a %.4f, H on %d of %d\n",
                         mu, it, rmax, nconv, res[0], std::abs(w[m - 1]), a, mq, p);
            std::fflush(stderr);
        }
        // stagnation: no halving of the best residual in 20 outer iterations
        if (rmax < 0.5 * best) {
            best = rmax;
            best_it = it;
        }
        const bool stalled = it - best_it >= 20;
        if (rmax <= tol || it == max_outer || stalled) {
            // eigenvectors r = Qm s (unit norm), the first m columns of S
            std::vector<cd> Sm((size_t)mq * m);
            for (int i = 0; i < mq; ++i)
                for (int j = 0; j < m; ++j) Sm[(size_t)i * m + j] = S[(size_t)i * mq + j];
            if (!c.ok(hipMemsetAsync(Out, 0, sizeof(c64) * (size_t)m * c.nf, c.s), "memset")) return false;
            if (!c.comb(Qm, mq, Sm, m, Out)) return false;
            break;
        }
        // damp everything above the largest Ritz value of H^2 in the subspace
        a = std::max(w2[p - 1].real(), 1e-6 * b);
        if (a >= b) a = 0.5 * b;
        (void)Zb;
    }
    return true;
}

// restarted GMRES for (shift - A) z = rhs on range(1 - P), P = sum R_i L_i^dag
// (adjoint side: A^dag = H(-mu), P^dag = sum L_i R_i^dag); z in Z.
bool gmres_shifted(Ctx& c, double mu, bool adjoint, cd shift, const c64* Rv, const c64* Lv, int m, const c64* rhs,
                   c64* Z, double tol, int restart, int max_it, int& iters, double& relres) {
    const c64* Pa = adjoint ? Rv : Lv;   // projector P z = Pb (Pa^dag z)
    const c64* Pb = adjoint ? Lv : Rv;
    const double amu = adjoint ? -mu : mu;
    c64* Vb = c.fields(restart + 1);
    c64* w = c.fields(1);
    c64* u = c.fields(1);
    c64* r = c.fields(1);
    if (!Vb || !w || !u || !r) return false;
    // op(z) = shift (1-P) z - A (1-P) z + P z
    auto op = [&](const c64* zin, c64* out) -> bool {
        std::vector<cd> pc;
        if (!c.proj(Pa, m, zin, 1, pc)) return false;        // Pa^dag z
        if (!c.copy(u, zin, 1)) return false;
        for (auto& v : pc) v = -v;
        if (!c.comb(Pb, m, pc, 1, u)) return false;          // u = (1 - P) z
        if (!c.apply(0, amu, u, out, 1)) return false;       // out = A u
        // out = shift u - A u + (z - u)
        return c.lincomb(c.nf, shift - 1.0, u, -1.0, out, 1.0, zin, out);
    };
    const double bn = c.norm(rhs);
    if (!(bn > 0)) {
        iters = 0;
        relres = 0.0;
        return c.ok(hipMemsetAsync(Z, 0, sizeof(c64) * c.nf, c.s), "memset");
    }
    if (!c.ok(hipMemsetAsync(Z, 0, sizeof(c64) * c.nf, c.s), "memset")) return false;
    iters = 0;
    relres = 1.0;
    while (iters < max_it) {
        // r = rhs - op(Z)
        if (!op(Z, w)) return false;
        if (!c.lincomb(c.nf, 1.0, rhs, -1.0, w, 0.0, nullptr, r)) return false;
        const double beta = c.norm(r);
        relres = beta / bn;
        if (relres <= tol) break;
        if (!c.lincomb(c.nf, 1.0 / beta, r, 0.0, nullptr, 0.0, nullptr, Vb)) return false;
        std::vector<cd> H((size_t)(restart + 1) * restart, cd(0)), g(restart + 1, cd(0)), sn(restart);
        std::vector<double> cs(restart);
        g[0] = beta;
        int j = 0;
        for (; j < restart && iters < max_it; ++j, ++iters) {
            c64* vj = Vb + (size_t)j * c.nf;
            c64* vn = Vb + (size_t)(j + 1) * c.nf;
            if (!op(vj, vn)) return false;
            // classical Gram-Schmidt, twice
            std::vector<cd> h(j + 1, cd(0));
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<cd> hp;
                if (!c.proj(Vb, j + 1, vn, 1, hp)) return false;
                for (int i = 0; i <= j; ++i) h[i] += hp[i];
                for (auto& v : hp) v = -v;
                if (!c.comb(Vb, j + 1, hp, 1, vn)) return false;
            }
            const double hn = c.norm(vn);
            for (int i = 0; i <= j; ++i) H[(size_t)i * restart + j] = h[i];
            H[(size_t)(j + 1) * restart + j] = hn;
            // apply the previous rotations, then a new one
            for (int i = 0; i < j; ++i) {
                const cd t1 = H[(size_t)i * restart + j], t2 = H[(size_t)(i + 1) * restart + j];
                H[(size_t)i * restart + j] = cs[i] * t1 + sn[i] * t2;
                H[(size_t)(i + 1) * restart + j] = -std::conj(sn[i]) * t1 + cs[i] * t2;
            }
            dense::givens(H[(size_t)j * restart + j], H[(size_t)(j + 1) * restart + j], cs[j], sn[j]);
            const cd t1 = H[(size_t)j * restart + j], t2 = H[(size_t)(j + 1) * restart + j];
            H[(size_t)j * restart + j] = cs[j] * t1 + sn[j] * t2;
            H[(size_t)(j + 1) * restart + j] = 0.0;
            const cd g1 = g[j], g2 = g[j + 1];
            g[j] = cs[j] * g1 + sn[j] * g2;
            g[j + 1] = -std::conj(sn[j]) * g1 + cs[j] * g2;
            relres = std::abs(g[j + 1]) / bn;
            if (hn > 0 && !c.lincomb(c.nf, 1.0 / hn, vn, 0.0, nullptr, 0.0, nullptr, vn)) return false;
            if (relres <= tol || !(hn > 0)) {
                ++j;
                ++iters;
                break;
            }
        }
        // y = H(0:j, 0:j)^{-1} g, Z += V y
        std::vector<cd> y(j, cd(0));
        for (int i = j - 1; i >= 0; --i) {
            cd t = g[i];
            for (int k = i + 1; k < j; ++k) t -= H[(size_t)i * restart + k] * y[k];
            y[i] = t / H[(size_t)i * restart + i];
        }
        if (j > 0 && !c.comb(Vb, j, y, 1, Z)) return false;
        if (relres <= tol) {
            // true residual of the final iterate
            if (!op(Z, w)) return false;
            if (!c.lincomb(c.nf, 1.0, rhs, -1.0, w, 0.0, nullptr, r)) return false;
            relres = c.norm(r) / bn;
            break;
        }
    }
    return true;
}

}  // namespace

int eigs_compute(const EigParams& P, EigResult& out) {
    const auto t0 = std::chrono::steady_clock::now();
    Ctx c;
    c.g = P.g;
    c.U = P.U;
    c.dU = P.dU;
    c.md = P.md;
    c.s = P.stream;
    c.nf = (long long)12 * P.g.Vp;
    const int m = P.m, l = P.l;
    const int p = P.p > m ? P.p : m + std::max(16, m / 2);
    const int degree = P.degree;
    out = EigResult{};
    auto fail = [&](int code) {
        out.err = c.err.empty() ? "eigensolver failed" : c.err;
        return code;
    };
    c64* Rv = c.fields(m);
    c64* Lraw = c.fields(m);
    if (!Rv || !Lraw) return fail(-2);
    SideResult right, left;
    if (!subspace_side(c, P.mu, m, p, P.tol, P.max_outer, degree, P.seed, Rv, right)) return fail(-3);
    if (!subspace_side(c, -P.mu, m, p, P.tol, P.max_outer, degree, P.seed + 1, Lraw, left)) return fail(-3);
    out.outer_right = right.outer;
    out.outer_left = left.outer;
    out.res_right = right.max_res;
    out.res_left = left.max_res;
    if (right.max_res > P.tol || left.max_res > P.tol) {
        c.err = "eigenpairs not converged: residual " + std::to_string(std::max(right.max_res, left.max_res)) +
                " after " + std::to_string(std::max(right.outer, left.outer)) + " outer iterations";
        return fail(-7);
    }
    // the two sides must hold the same eigenvalues (conjugated)
    double setdiff = 0.0;
    for (int i = 0; i < m; ++i) {
        double best = 1e300;
        for (int j = 0; j < m; ++j) best = std::min(best, std::abs(std::conj(left.theta[j]) - right.theta[i]));
        setdiff = std::max(setdiff, best);
    }
    if (setdiff > 1e3 * P.tol + 1e-9) {
        c.err = "left and right eigenvalue sets differ by " + std::to_string(setdiff) +
                " (a cluster straddles the m-th eigenvalue; choose another m)";
        return fail(-7);
    }
    // left vectors: dual basis of R in span(Lraw): L = Lraw (M^{-1})^dag, M = Lraw^dag R
    std::vector<cd> M, Mi;
    if (!c.proj(Lraw, m, Rv, m, M)) return fail(-3);
    if (!dense::inverse(m, M, Mi)) {
        c.err = "left and right eigenvectors are not in duality (singular L^dag R)";
        return fail(-7);
    }
    std::vector<cd> K((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) K[(size_t)i * m + j] = std::conj(Mi[(size_t)j * m + i]);
    c64* Lv = c.fields(m);
    if (!Lv || !c.comb(Lraw, m, K, m, Lv)) return fail(-3);
    {
        std::vector<cd> G;
        if (!c.proj(Lv, m, Rv, m, G)) return fail(-3);
        double dev = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) dev = std::max(dev, std::abs(G[(size_t)i * m + j] - cd(i == j ? 1.0 : 0.0)));
        out.biorth = dev;
    }
    out.lam.resize(m);
    for (int i = 0; i < m; ++i) out.lam[i] = c64{right.theta[i].real(), right.theta[i].imag()};
    out.R = Rv;
    out.L = Lv;
    // derivatives of the first l pairs
    if (l > 0) {
        const int dop = P.dir_link ? 3 : 2;
        c64* D = c.fields(m);       // dA R_i
        c64* DL = c.fields(l);      // dA^dag L_j
        c64* dR = c.fields(l);
        c64* dL = c.fields(l);
        c64* rhs = c.fields(1);
        c64* z = c.fields(1);
        if (!D || !DL || !dR || !dL || !rhs || !z) return fail(-2);
        if (!c.apply(dop, P.mu, Rv, D, m)) return fail(-3);
        // (d/dmu H)^dag = -(d/dmu H)(-mu); for a link direction dH^dag = dH(-mu)
        if (!c.apply(dop, -P.mu, Lv, DL, l)) return fail(-3);
        if (!P.dir_link && !c.lincomb((long long)l * c.nf, -1.0, DL, 0.0, nullptr, 0.0, nullptr, DL)) return fail(-3);
        std::vector<cd> C;   // C[i][j] = L_i^dag dA R_j
        if (!c.proj(Lv, m, D, m, C)) return fail(-3);
        std::vector<cd> lam(m);
        for (int i = 0; i < m; ++i) lam[i] = right.theta[i];
        // GMRES restart length: long (the shifts are interior), at most the dimension
        const int restart = (int)std::min<long long>(150, 12LL * c.g.V - 1);
        for (int j = 0; j < l; ++j) {
            for (int i = 0; i < m; ++i)
                if (i != j && std::abs(lam[j] - lam[i]) < 1e-9 * (1.0 + std::abs(lam[j]))) {
                    c.err = "degenerate eigenvalues among the derivative pairs";
                    return fail(-7);
                }
            // right: rhs = (1 - P) dA R_j
            if (!c.copy(rhs, D + (size_t)j * c.nf, 1)) return fail(-3);
            std::vector<cd> cj(m);
            for (int i = 0; i < m; ++i) cj[i] = -C[(size_t)i * m + j];
            if (!c.comb(Rv, m, cj, 1, rhs)) return fail(-3);
            int it = 0;
            double rr = 0.0;
            if (!gmres_shifted(c, P.mu, false, lam[j], Rv, Lv, m, rhs, z, P.gmres_tol, restart, P.gmres_max, it, rr))
                return fail(-3);
            if (verbose()) {
                std::fprintf(stderr, "eigs dR_%d: %d GMRES iterations, residual %.2e\n", j, it, rr);
                std::fflush(stderr);
            }
            out.gmres_iters += it;
            out.gmres_res = std::max(out.gmres_res, rr);
            c64* dRj = dR + (size_t)j * c.nf;
            if (!c.copy(dRj, z, 1)) return fail(-3);
            std::vector<cd> sr(m, cd(0));
            for (int i = 0; i < m; ++i)
                if (i != j) sr[i] = C[(size_t)i * m + j] / (lam[j] - lam[i]);
            if (!c.comb(Rv, m, sr, 1, dRj)) return fail(-3);
            // left: rhs = (1 - P)^dag dA^dag L_j = e - L (R^dag e)
            const c64* e = DL + (size_t)j * c.nf;
            std::vector<cd> pr;
            if (!c.proj(Rv, m, e, 1, pr)) return fail(-3);
            if (!c.copy(rhs, e, 1)) return fail(-3);
            for (auto& v : pr) v = -v;
            if (!c.comb(Lv, m, pr, 1, rhs)) return fail(-3);
            if (!gmres_shifted(c, P.mu, true, std::conj(lam[j]), Rv, Lv, m, rhs, z, P.gmres_tol, restart, P.gmres_max,
                               it, rr))
                return fail(-3);
            if (verbose()) {
                std::fprintf(stderr, "eigs dL_%d: %d GMRES iterations, residual %.2e\n", j, it, rr);
                std::fflush(stderr);
            }
            out.gmres_iters += it;
            out.gmres_res = std::max(out.gmres_res, rr);
            c64* dLj = dL + (size_t)j * c.nf;
            if (!c.copy(dLj, z, 1)) return fail(-3);
            std::vector<cd> sl(m, cd(0));
            for (int i = 0; i < m; ++i)
                if (i != j) sl[i] = std::conj(C[(size_t)j * m + i] / (lam[j] - lam[i]));
            if (!c.comb(Lv, m, sl, 1, dLj)) return fail(-3);
        }
        if (out.gmres_res > 1e3 * P.gmres_tol) {
            c.err = "shifted solves for the eigenvector derivatives did not converge (residual " +
                    std::to_string(out.gmres_res) + ")";
            return fail(-7);
        }
        out.dR = dR;
        out.dL = dL;
    }
    if (!c.ok(hipStreamSynchronize(c.s), "sync")) return fail(-3);
    // hand the result buffers over to the caller
    for (void* q : {(void*)out.R, (void*)out.L, (void*)out.dR, (void*)out.dL}) {
        auto it = std::find(c.owned.begin(), c.owned.end(), q);
        if (q && it != c.owned.end()) c.owned.erase(it);
    }
    out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

}  // namespace ovd
