// Deflation data on the GPU: the m eigenvalues of smallest |lambda| of
// H(mu) = gamma5 Dw(mu) with right and left eigenvectors (L^dag R = 1, Sec. 3,
// eq. 8), and the derivatives of the first l eigenvector pairs along mu or a
// link direction (Sec. 3, eq. 10-11 with the eigenvector derivative of the
// perturbation expansion).
//
// Eigenpairs: thick-restart Arnoldi on B = H^{-1}.  The wanted eigenvalues
// (smallest |lambda|) are interior for H, but 1/lambda are the eigenvalues of
// largest modulus of B, outside the disk that holds the rest of its spectrum,
// where a Krylov space converges to them whatever their phase.  Every
// application of B is a conjugate-gradient solve of the normal equations
// H^dag H z = H^dag v (H^dag = H(-mu)); the basis is orthogonalised by
// classical Gram-Schmidt twice (MFMA projections), the projected problem is
// solved on the host by the QR algorithm, and each restart keeps the Ritz
// vectors of largest |theta| (a Krylov decomposition with a full leading
// block).  The same run on H^dag gives the left subspace; the left vectors are
// then the dual basis of the right ones in it (L^dag R = 1).
//
// Derivatives (gauge L_j^dag dR_j = 0, dL_j^dag R_j = 0), with P = sum_{i<m} R_i L_i^dag:
//   dR_j = sum_{i != j} R_i (L_i^dag dA R_j) / (lambda_j - lambda_i)
//          + (lambda_j - A)^{-1} (1 - P) dA R_j            (solved on range(1 - P))
//   dL_j = sum_{i != j} L_i conj((L_j^dag dA R_i) / (lambda_j - lambda_i))
//          + (conj(lambda_j) - A^dag)^{-1} (1 - P)^dag dA^dag L_j
// The shifted systems are solved by conjugate gradients on their normal
// equations (CGLS); every long-vector product is a stencil launch or an MFMA
// projection (kernels_defl.hip), the small problems run on the host.
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
#include <thread>
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

// x^dag y of two fields in two launches with a fixed summation order: each of
// kDotBlocks blocks sums a strided share of the elements (wave shuffles, then
// the block's waves in order), and one block adds the partials in order.
constexpr int kDotBlocks = 512;
__device__ __forceinline__ void block_sum2(double& re, double& im, double* lds) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        re += __shfl_xor(re, m, 64);
        im += __shfl_xor(im, m, 64);
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        lds[2 * w] = re;
        lds[2 * w + 1] = im;
    }
    __syncthreads();
    re = 0.0;
    im = 0.0;
    for (int q = 0; q < nw; ++q) {
        re += lds[2 * q];
        im += lds[2 * q + 1];
    }
}
__global__ __launch_bounds__(256) void dot_partial_kernel(long long n_elem, const c64* __restrict__ x,
                                                          const c64* __restrict__ y, c64* __restrict__ part) {
    __shared__ double lds[8];
    double re = 0.0, im = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        const c64 a = x[e], b = y[e];
        re += a.re * b.re + a.im * b.im;
        im += a.re * b.im - a.im * b.re;
    }
    block_sum2(re, im, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = c64{re, im};
}
__global__ __launch_bounds__(256) void dot_final_kernel(int nb, const c64* __restrict__ part, c64* __restrict__ out) {
    __shared__ double lds[8];
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        re += part[i].re;
        im += part[i].im;
    }
    block_sum2(re, im, lds);
    if (threadIdx.x == 0) *out = c64{re, im};
}

// out = X + f Y with f = sgn num / den from device scalars, so that a CG step
// needs no host round trip (f = 0 when den = 0); X and out may be the same
__global__ void axpy_ratio_kernel(long long n_elem, const c64* X, double sgn, const c64* __restrict__ num,
                                  const c64* __restrict__ den, const c64* __restrict__ Y, c64* out) {
    const c64 a = *num, b = *den;
    const double bb = b.re * b.re + b.im * b.im;
    const c64 f = bb > 0 ? c64{sgn * (a.re * b.re + a.im * b.im) / bb, sgn * (a.im * b.re - a.re * b.im) / bb}
                         : c64{0.0, 0.0};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        const c64 y = Y[e];
        c64 r = X[e];
        r.re += f.re * y.re - f.im * y.im;
        r.im += f.re * y.im + f.im * y.re;
        out[e] = r;
    }
}

// out_j = a_j X_j + b_j Y_j + c_j Z_j for nr columns of nf elements (column j
// at offset j nf), coefficients coef[j][3] on the device; Y, Z may be null;
// out may be X or Y (each element is read before it is written)
__global__ void blincomb_kernel(long long nf, int nr, const c64* __restrict__ coef, const c64* X, const c64* Y,
                                const c64* Z, c64* out) {
    const int j = blockIdx.y;
    const c64 a = coef[3 * j], b = coef[3 * j + 1], c = coef[3 * j + 2];
    const size_t o = (size_t)j * nf;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += stride) {
        c64 r = a * X[o + e];
        if (Y) r += b * Y[o + e];
        if (Z) r += c * Z[o + e];
        out[o + e] = r;
    }
}

// CGLS scalars of nr systems on the device (one thread per system), so that an
// iteration needs no host round trip; the coefficient triples feed
// blincomb_kernel.
struct CglsState {
    double *bn, *gam, *qq, *rn, *gn, *relres;
    int *active, *iters;
    c64 *cz, *cr, *cp;   // Z += alpha p,  r -= alpha q,  p = s + beta p
};
// squared 2-norms of nr columns (column j at offset j nf) in two launches with
// a fixed summation order: kDotBlocks partial sums per column, then one block
// per column adds them in order
__global__ __launch_bounds__(256) void colnorm2_partial_kernel(long long nf, const c64* __restrict__ X,
                                                               double* __restrict__ part) {
    __shared__ double lds[8];
    const c64* x = X + (size_t)blockIdx.y * nf;
    double re = 0.0, im = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += stride) {
        const c64 a = x[e];
        re += a.re * a.re + a.im * a.im;
    }
    block_sum2(re, im, lds);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = re;
}
__global__ __launch_bounds__(256) void colnorm2_final_kernel(int nb, const double* __restrict__ part,
                                                             double* __restrict__ out) {
    __shared__ double lds[8];
    const double* pj = part + (size_t)blockIdx.x * nb;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) re += pj[i];
    block_sum2(re, im, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = re;
}
// start: bn = |rhs_j| (from its squared norm), systems with a zero right-hand side inactive
__global__ void cgls_init_kernel(int nr, CglsState d) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr) return;
    d.bn[j] = sqrt(d.bn[j]);
    d.active[j] = d.bn[j] > 0 ? 1 : 0;
    d.relres[j] = d.active[j] ? 1.0 : 0.0;
    d.iters[j] = 0;
}
// alpha = gam / |q|^2 for the active systems (a system with |q| = 0 stops)
__global__ void cgls_alpha_kernel(int nr, CglsState d) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr) return;
    const c64 one{1.0, 0.0}, zero{0.0, 0.0};
    if (d.active[j] && !(d.qq[j] > 0)) d.active[j] = 0;
    if (!d.active[j]) {
        d.cz[3 * j] = one; d.cz[3 * j + 1] = zero; d.cz[3 * j + 2] = zero;
        d.cr[3 * j] = one; d.cr[3 * j + 1] = zero; d.cr[3 * j + 2] = zero;
        return;
    }
    const double alpha = d.gam[j] / d.qq[j];
    d.cz[3 * j] = one; d.cz[3 * j + 1] = c64{alpha, 0.0}; d.cz[3 * j + 2] = zero;
    d.cr[3 * j] = one; d.cr[3 * j + 1] = c64{-alpha, 0.0}; d.cr[3 * j + 2] = zero;
    ++d.iters[j];
}
// relative residual of the active systems; a system at tolerance stops
__global__ void cgls_conv_kernel(int nr, CglsState d, double tol) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr || !d.active[j]) return;
    d.relres[j] = sqrt(d.rn[j]) / d.bn[j];
    if (d.relres[j] <= tol) d.active[j] = 0;
}
// beta = |s|^2 / gam for the active systems (p unchanged for the others)
__global__ void cgls_beta_kernel(int nr, CglsState d) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr) return;
    const c64 zero{0.0, 0.0};
    if (!d.active[j]) {
        d.cp[3 * j] = zero; d.cp[3 * j + 1] = c64{1.0, 0.0}; d.cp[3 * j + 2] = zero;
        return;
    }
    d.cp[3 * j] = c64{1.0, 0.0}; d.cp[3 * j + 1] = c64{d.gn[j] / d.gam[j], 0.0}; d.cp[3 * j + 2] = zero;
    d.gam[j] = d.gn[j];
}
__global__ void cneg_kernel(int n, const c64* __restrict__ in, c64* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = -in[i];
}

// One CG step's vector updates and the next residual norm in one pass:
//   z += f d,  r -= f t  (f = num / den from device scalars, 0 when den = 0),
// and the kDotBlocks block partial sums of r^dag r for the new r, with the
// same element-to-thread map and arithmetic as axpy_ratio_kernel and
// dot_partial_kernel (dot_final_kernel then adds them in order): the results
// are those of the three separate launches.
__global__ __launch_bounds__(256) void cg_update_kernel(long long n_elem, c64* z, const c64* __restrict__ d, c64* r,
                                                        const c64* __restrict__ t, const c64* __restrict__ num,
                                                        const c64* __restrict__ den, c64* __restrict__ part) {
    __shared__ double lds[8];
    const c64 a = *num, b = *den;
    const double bb = b.re * b.re + b.im * b.im;
    const c64 fz = bb > 0 ? c64{1.0 * (a.re * b.re + a.im * b.im) / bb, 1.0 * (a.im * b.re - a.re * b.im) / bb}
                          : c64{0.0, 0.0};
    const c64 fr = bb > 0 ? c64{-1.0 * (a.re * b.re + a.im * b.im) / bb, -1.0 * (a.im * b.re - a.re * b.im) / bb}
                          : c64{0.0, 0.0};
    double re = 0.0, im = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        {
            const c64 y = d[e];
            c64 v = z[e];
            v.re += fz.re * y.re - fz.im * y.im;
            v.im += fz.re * y.im + fz.im * y.re;
            z[e] = v;
        }
        const c64 y = t[e];
        c64 v = r[e];
        v.re += fr.re * y.re - fr.im * y.im;
        v.im += fr.re * y.im + fr.im * y.re;
        r[e] = v;
        re += v.re * v.re + v.im * v.im;
        im += v.re * v.im - v.im * v.re;
    }
    block_sum2(re, im, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = c64{re, im};
}

namespace {

// progress lines on stderr when OVDERIV_VERBOSE is set (long setup runs)
bool verbose() {
    static const bool v = std::getenv("OVDERIV_VERBOSE") != nullptr;
    return v;
}
// seconds since the first call (time stamps of the verbose log)
double vclock() {
    static const auto t0 = std::chrono::steady_clock::now();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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
    // device tables (e^{mu}, e^{-mu}) per field for the two values of mu used
    // last: a solve alternates H(mu) and H(-mu) = H(mu)^dag, which then costs
    // no upload and no wait inside its iterations
    struct MuTable {
        double mu = 1e300;
        int n = 0;
        double* d = nullptr;
    };
    MuTable mu_tab[2];
    int mu_next = 0;

    ~Ctx() {
        for (void* p : owned) (void)hipFree(p);
    }
    bool ok(hipError_t e, const char* what) {
        if (e != hipSuccess && err.empty()) err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipSuccess;
    }
    // one block of n fields kept for repeated solves (grown on demand)
    c64* reuse_buf = nullptr;
    int reuse_n = 0;
    c64* reuse(int n) {
        if (n <= reuse_n) return reuse_buf;
        reuse_buf = fields(n);
        reuse_n = reuse_buf ? n : 0;
        return reuse_buf;
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
    // the table of mu for n fields (built on first use; one of two slots)
    const double* mu_table(double mu, int n) {
        for (const MuTable& t : mu_tab)
            if (t.d && t.mu == mu && n <= t.n) return t.d;
        MuTable& t = mu_tab[mu_next];
        mu_next ^= 1;
        if (n > t.n) {
            void* p = nullptr;
            if (!ok(hipMalloc(&p, sizeof(double) * 2 * n), "hipMalloc")) return nullptr;
            owned.push_back(p);
            t.d = (double*)p;
            t.n = n;
        }
        std::vector<double> h(2 * (size_t)t.n);
        for (int i = 0; i < t.n; ++i) {
            h[2 * i] = std::exp(mu);
            h[2 * i + 1] = std::exp(-mu);
        }
        // stream-ordered after every launch that read the slot's previous table
        if (!ok(hipMemcpyAsync(t.d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s), "copy"))
            return nullptr;
        if (!ok(hipStreamSynchronize(s), "sync")) return nullptr;   // h is released on return
        t.mu = mu;
        return t.d;
    }
    // out = op(mu) in, n fields (op: 0 H, 2 dH/dmu, 3 dH/dlink)
    bool apply(int op, double mu, const c64* in, c64* out, int n) {
        const double* emu = mu_table(mu, n);
        if (!emu) return false;
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
    // Cd (device, m x nr) = A^dag B, no wait
    // (reduction chunks of `chunk` elements, see launch_defl_proj)
    bool proj_dev(const c64* A, int m, const c64* B, int nr, c64* Cd, long long chunk = 0) {
        if (!ensure_scratch(m, nr)) return false;
        launch_defl_proj(A, nf, m, B, nf, nr, nf, Cd, scr, s, chunk);
        return ok(hipGetLastError(), "defl_proj");
    }
    // Y = Y0 + A Cd (Cd device, m x nr), no wait
    bool comb_dev(const c64* A, int m, const c64* Cd, int nr, const c64* Y0, c64* Y) {
        launch_defl_comb(A, nf, m, Cd, nr, Y, nf, nf, s, Y0, nf);
        return ok(hipGetLastError(), "defl_comb");
    }
    // out_j = a_j X_j + b_j Y_j + c_j Z_j over nr columns, coefficients on the device
    bool blincomb(int nr, const c64* coef, const c64* X, const c64* Y, const c64* Z, c64* out) {
        long long nb = (nf + 255) / 256;
        if (nb > 2048) nb = 2048;
        blincomb_kernel<<<dim3((unsigned)nb, (unsigned)nr), 256, 0, s>>>(nf, nr, coef, X, Y, Z, out);
        return ok(hipGetLastError(), "blincomb");
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
    // dst (device, one complex) = x^dag y, left on the device
    c64* dot_part = nullptr;
    bool dot_dev(const c64* x, const c64* y, c64* dst) {
        if (!dot_part) {
            void* p = nullptr;
            if (!ok(hipMalloc(&p, kDotBlocks * sizeof(c64)), "hipMalloc")) return false;
            owned.push_back(p);
            dot_part = (c64*)p;
        }
        dot_partial_kernel<<<kDotBlocks, 256, 0, s>>>(nf, x, y, dot_part);
        dot_final_kernel<<<1, 256, 0, s>>>(kDotBlocks, dot_part, dst);
        return ok(hipGetLastError(), "dot");
    }
    // z += (num/den) d, r -= (num/den) t, dst = r^dag r of the new r (device scalars)
    bool cg_update(c64* z, const c64* d, c64* r, const c64* t, const c64* num, const c64* den, c64* dst) {
        if (!dot_part) {
            void* p = nullptr;
            if (!ok(hipMalloc(&p, kDotBlocks * sizeof(c64)), "hipMalloc")) return false;
            owned.push_back(p);
            dot_part = (c64*)p;
        }
        cg_update_kernel<<<kDotBlocks, 256, 0, s>>>(nf, z, d, r, t, num, den, dot_part);
        dot_final_kernel<<<1, 256, 0, s>>>(kDotBlocks, dot_part, dst);
        return ok(hipGetLastError(), "cg_update");
    }
    bool axpy_ratio(const c64* X, double sgn, const c64* num, const c64* den, const c64* Y, c64* out) {
        long long nb = (nf + 255) / 256;
        if (nb > 8192) nb = 8192;
        axpy_ratio_kernel<<<(unsigned)nb, 256, 0, s>>>(nf, X, sgn, num, den, Y, out);
        return ok(hipGetLastError(), "axpy_ratio");
    }
    // host copy of a device scalar (waits for the stream)
    bool read_scalar(const c64* src, cd& out) {
        c64 v{};
        if (!ok(hipMemcpyAsync(&v, src, sizeof(c64), hipMemcpyDeviceToHost, s), "copy")) return false;
        if (!ok(hipStreamSynchronize(s), "sync")) return false;
        out = cd(v.re, v.im);
        return true;
    }
    // three device scalars for the CG recurrence
    c64* cg_sc = nullptr;
    c64* cg_scalars() {
        if (cg_sc) return cg_sc;
        void* p = nullptr;
        if (!ok(hipMalloc(&p, 3 * sizeof(c64)), "hipMalloc")) return nullptr;
        owned.push_back(p);
        cg_sc = (c64*)p;
        return cg_sc;
    }
    bool copy(c64* dst, const c64* src, int n) {
        return ok(hipMemcpyAsync(dst, src, sizeof(c64) * (size_t)n * nf, hipMemcpyDeviceToDevice, s), "copy");
    }
    double norm(const c64* x) {
        c64* sc = cg_scalars();
        cd v;
        if (!sc || !dot_dev(x, x, sc) || !read_scalar(sc, v)) return -1.0;
        return std::sqrt(std::max(0.0, v.real()));
    }
};

struct SideResult {
    std::vector<cd> theta;   // m eigenvalues of H, increasing |theta|
    cd next{0.0, 0.0};       // the (m+1)-th Ritz value of H at convergence (0 when the basis has no more)
    int outer = 0;
    double max_res = 0.0;
    long long solves = 0, cg_iters = 0;
};

// sort the eigenpairs (w, S) of a p x p projected matrix by decreasing |w| (S columns)
void sort_by_modulus_desc(int p, std::vector<cd>& w, std::vector<cd>& S) {
    std::vector<int> ord(p);
    for (int i = 0; i < p; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int i, int j) { return std::abs(w[i]) > std::abs(w[j]); });
    std::vector<cd> Ss((size_t)p * p), ws(p);
    for (int j = 0; j < p; ++j) {
        ws[j] = w[ord[j]];
        for (int i = 0; i < p; ++i) Ss[(size_t)i * p + j] = S[(size_t)i * p + ord[j]];
    }
    w.swap(ws);
    S.swap(Ss);
}

// z = H(mu)^{-1} v by conjugate gradients on the normal equations
// H^dag H z = H^dag v (H^dag = H(-mu)); r, d, q, t: work fields.  The CG
// scalars stay on the device; the residual is read every kCgCheck iterations,
// so a solve may run up to kCgCheck - 1 iterations past the tolerance.
constexpr int kCgCheck = 8;
bool solve_h(Ctx& c, double mu, const c64* v, c64* z, c64* r, c64* d, c64* q, c64* t, double tol, int max_it,
             long long& iters) {
    c64* sc = c.cg_scalars();
    if (!sc) return false;
    c64 *rr = sc, *qq = sc + 1, *rn = sc + 2;
    if (!c.ok(hipMemsetAsync(z, 0, sizeof(c64) * c.nf, c.s), "memset")) return false;
    if (!c.apply(0, -mu, v, r, 1)) return false;   // r = H^dag v (z = 0)
    if (!c.copy(d, r, 1)) return false;
    cd h;
    if (!c.dot_dev(r, r, rr) || !c.read_scalar(rr, h)) return false;
    const double r0 = std::sqrt(h.real());
    if (!(r0 > 0)) return true;
    for (int it = 0; it < max_it; ++it) {
        if (!c.apply(0, mu, d, q, 1) || !c.apply(0, -mu, q, t, 1)) return false;   // t = H^dag H d
        if (!c.dot_dev(q, q, qq)) return false;
        if (!c.cg_update(z, d, r, t, rr, qq, rn)) return false;   // z += a d, r -= a t, rn = r^dag r
        ++iters;
        if ((it + 1) % kCgCheck == 0 || it + 1 == max_it) {
            if (!c.read_scalar(rn, h)) return false;
            if (std::sqrt(std::max(0.0, h.real())) <= tol * r0) break;
        }
        if (!c.axpy_ratio(r, 1.0, rn, rr, d, d)) return false;
        std::swap(rr, rn);   // stream order: the next dot overwrites the old rr after this step's reads
    }
    return c.ok(hipStreamSynchronize(c.s), "sync");
}

// One side (mu, or -mu for the left vectors): the m eigenpairs of H(mu) of
// smallest |lambda| by thick-restart Arnoldi on B = H(mu)^{-1}.  The wanted
// eigenvalues 1/lambda are those of largest modulus of B: outside the disk that
// holds the rest of its spectrum, where a Krylov space finds them whatever
// their phase (a polynomial filter in H^2 cannot separate |lambda| from the
// imaginary parts of lambda^2).  Each cycle extends the Arnoldi basis to n
// vectors (one CG solve per vector), takes the Ritz pairs of the n x n
// projected matrix, and restarts from the k Ritz vectors of largest |theta|
// plus the last Arnoldi vector (a Krylov decomposition with a full k x k
// block).  The m eigenvectors of H end up in Out (unit norm), increasing |lambda|.
bool arnoldi_side(Ctx& c, double mu, int m, int n, double tol, int max_cycles, uint64_t seed, c64* Out,
                  SideResult& sr) {
    const int kkeep = std::min(n - 4, m + std::max(8, (n - m) / 2));
    c64* Vb = c.fields(n + 1);
    c64* T = c.fields(n);
    c64* Zm = c.fields(m);
    c64* w4[4] = {c.fields(1), c.fields(1), c.fields(1), c.fields(1)};
    if (!Vb || !T || !Zm || !w4[0] || !w4[1] || !w4[2] || !w4[3]) return false;
    auto V = [&](int i) { return Vb + (size_t)i * c.nf; };
    {
        fill_random_kernel<<<(unsigned)((c.nf + 255) / 256), 256, 0, c.s>>>(c.nf, c.nf, c.g.V, c.g.Vp, seed, Vb);
        if (!c.ok(hipGetLastError(), "fill_random")) return false;
        const double nv = c.norm(V(0));
        if (!c.lincomb(c.nf, 1.0 / nv, V(0), 0.0, nullptr, 0.0, nullptr, V(0))) return false;
    }
    // ||H|| <= |m0 + 4| + 3 + e^{|mu|} (r = 1, unit-norm links)
    const double hb = std::fabs(c.md) + 3.0 + std::exp(std::fabs(mu));
    std::vector<cd> Hm((size_t)(n + 1) * n, cd(0));   // (n + 1) x n, row-major
    auto h = [&](int i, int j) -> cd& { return Hm[(size_t)i * n + j]; };
    int k = 0;
    for (int cyc = 1; cyc <= max_cycles; ++cyc) {
        for (int j = k; j < n; ++j) {
            if (!solve_h(c, mu, V(j), V(j + 1), w4[0], w4[1], w4[2], w4[3], 1e-13, 5000, sr.cg_iters)) return false;
            ++sr.solves;
            std::vector<cd> hc(j + 1, cd(0));
            for (int pass = 0; pass < 2; ++pass) {   // classical Gram-Schmidt, twice
                std::vector<cd> hp;
                if (!c.proj(Vb, j + 1, V(j + 1), 1, hp)) return false;
                for (int i = 0; i <= j; ++i) hc[i] += hp[i];
                for (auto& x : hp) x = -x;
                if (!c.comb(Vb, j + 1, hp, 1, V(j + 1))) return false;
            }
            const double hn = c.norm(V(j + 1));
            for (int i = 0; i <= j; ++i) h(i, j) = hc[i];
            h(j + 1, j) = hn;
            if (!(hn > 0)) {
                c.err = "Arnoldi breakdown (invariant subspace); choose another seed";
                return false;
            }
            if (!c.lincomb(c.nf, 1.0 / hn, V(j + 1), 0.0, nullptr, 0.0, nullptr, V(j + 1))) return false;
        }
        // Ritz pairs of B in the n-dimensional space, decreasing |theta|
        std::vector<cd> Hn((size_t)n * n), th, S;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Hn[(size_t)i * n + j] = h(i, j);
        if (!dense::eig_general(n, Hn, th, S)) {
            c.err = "QR iteration of the projected problem did not converge";
            return false;
        }
        sort_by_modulus_desc(n, th, S);
        // estimated residual of H: |H x - lambda x| <= |lambda| ||H|| |B x - theta x|,
        // |B x - theta x| = |row n of the decomposition . s|
        double est = 0.0;
        for (int i = 0; i < m; ++i) {
            cd rb = 0.0;
            for (int j = 0; j < n; ++j) rb += h(n, j) * S[(size_t)j * n + i];
            est = std::max(est, std::abs(rb) * hb / std::abs(th[i]));
        }
        sr.outer = cyc;
        const bool last = cyc == max_cycles;
        if (est <= tol || last) {
            // eigenvectors x = V s (unit norm), eigenvalues 1/theta, true residuals |H x - lambda x|
            std::vector<cd> Sm((size_t)n * m);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < m; ++j) Sm[(size_t)i * m + j] = S[(size_t)i * n + j];
            if (!c.ok(hipMemsetAsync(Out, 0, sizeof(c64) * (size_t)m * c.nf, c.s), "memset")) return false;
            if (!c.comb(Vb, n, Sm, m, Out)) return false;
            if (!c.apply(0, mu, Out, Zm, m)) return false;
            sr.theta.assign(m, cd(0));
            sr.next = n > m && std::abs(th[m]) > 0.0 ? 1.0 / th[m] : cd(0.0);
            double rmax = 0.0;
            for (int i = 0; i < m; ++i) {
                c64* xi = Out + (size_t)i * c.nf;
                c64* zi = Zm + (size_t)i * c.nf;
                const double nx = c.norm(xi);
                if (!c.lincomb(c.nf, 1.0 / nx, xi, 0.0, nullptr, 0.0, nullptr, xi)) return false;
                const cd lam = 1.0 / th[i];
                sr.theta[i] = lam;
                if (!c.lincomb(c.nf, 1.0 / nx, zi, -lam, xi, 0.0, nullptr, zi)) return false;
                rmax = std::max(rmax, c.norm(zi));
            }
            sr.max_res = rmax;
            if (verbose()) {
                std::fprintf(stderr, "[%.2f s] eigs mu=%+.3f cycle %d: estimate %.2e, residual %.3e, |lambda_m| %.6f, %lld solves, %lld CG\n",
                             vclock(), mu, cyc, est, rmax, std::abs(sr.theta[m - 1]), sr.solves, sr.cg_iters);
                std::fflush(stderr);
            }
            if (rmax <= tol || last) return true;
        } else if (verbose()) {
            std::fprintf(stderr, "[%.2f s] eigs mu=%+.3f cycle %d: estimate %.2e, |lambda_m| %.6f, %lld solves, %lld CG\n",
                         vclock(), mu, cyc, est, std::abs(1.0 / th[m - 1]), sr.solves, sr.cg_iters);
            std::fflush(stderr);
        }
        // thick restart: keep kk >= kkeep Ritz vectors, kk at the largest
        // relative gap of |theta| in [kkeep, kkeep + 4] (a cluster at the cut
        // is kept whole; the rest of the basis is new Krylov directions)
        int kk = kkeep;
        {
            double gbest = -1.0;
            for (int j = kkeep; j <= std::min(n - 2, kkeep + 4); ++j) {
                const double gap = (std::abs(th[j - 1]) - std::abs(th[j])) / std::abs(th[j - 1]);
                if (gap > gbest) {
                    gbest = gap;
                    kk = j;
                }
            }
        }
        // orthonormal basis Q of the kept Ritz vectors (host Gram-Schmidt, twice)
        std::vector<cd> Q((size_t)n * kk);
        for (int j = 0; j < kk; ++j) {
            for (int i = 0; i < n; ++i) Q[(size_t)i * kk + j] = S[(size_t)i * n + j];
            for (int pass = 0; pass < 2; ++pass)
                for (int q = 0; q < j; ++q) {
                    cd d = 0.0;
                    for (int i = 0; i < n; ++i) d += std::conj(Q[(size_t)i * kk + q]) * Q[(size_t)i * kk + j];
                    for (int i = 0; i < n; ++i) Q[(size_t)i * kk + j] -= d * Q[(size_t)i * kk + q];
                }
            double nq = 0.0;
            for (int i = 0; i < n; ++i) nq += std::norm(Q[(size_t)i * kk + j]);
            nq = std::sqrt(nq);
            for (int i = 0; i < n; ++i) Q[(size_t)i * kk + j] /= nq;
        }
        // new basis [V Q, v_n], new decomposition: B (V Q) = (V Q) (Q^dag H Q) + v_n (h_n Q)
        if (!c.ok(hipMemsetAsync(T, 0, sizeof(c64) * (size_t)kk * c.nf, c.s), "memset")) return false;
        if (!c.comb(Vb, n, Q, kk, T)) return false;
        if (!c.copy(V(kk), V(n), 1)) return false;
        if (!c.copy(Vb, T, kk)) return false;
        std::vector<cd> HQ((size_t)n * kk, cd(0)), M((size_t)kk * kk, cd(0)), brow(kk, cd(0));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < kk; ++j) {
                cd t = 0.0;
                for (int l = 0; l < n; ++l) t += Hn[(size_t)i * n + l] * Q[(size_t)l * kk + j];
                HQ[(size_t)i * kk + j] = t;
            }
        for (int i = 0; i < kk; ++i)
            for (int j = 0; j < kk; ++j) {
                cd t = 0.0;
                for (int l = 0; l < n; ++l) t += std::conj(Q[(size_t)l * kk + i]) * HQ[(size_t)l * kk + j];
                M[(size_t)i * kk + j] = t;
            }
        for (int j = 0; j < kk; ++j) {
            cd t = 0.0;
            for (int l = 0; l < n; ++l) t += h(n, l) * Q[(size_t)l * kk + j];
            brow[j] = t;
        }
        std::fill(Hm.begin(), Hm.end(), cd(0));
        for (int i = 0; i < kk; ++i)
            for (int j = 0; j < kk; ++j) h(i, j) = M[(size_t)i * kk + j];
        for (int j = 0; j < kk; ++j) h(kk, j) = brow[j];
        k = kk;
    }
    return true;
}

// (shift_j - A) z_j = rhs_j, j < nr, on the range of 1 - P (P = sum R_i L_i^dag;
// adjoint side: A^dag = H(-mu), P^dag = sum L_i R_i^dag), each solved as
// op_j z = rhs_j with op_j = shift_j (1 - P) - A (1 - P) + P by CGLS: conjugate
// gradients on the normal equations op_j^dag op_j z = op_j^dag rhs_j with the
// residual rhs_j - op_j z kept explicitly.  The shift sits inside the spectrum
// of A (an interior eigenvalue), so op_j is indefinite with a small gap; CGLS
// converges monotonically there, where restarted GMRES stalls.  The nr systems
// run side by side, each with its own CGLS scalars, so that one pass over the m
// projector vectors serves all of them; a converged system is left as it is.
// The scalars, the projection coefficients and the per-system combinations stay
// on the device; the host reads which systems are still running every
// kCgCheck iterations (the iterations past the last system's convergence
// change nothing).  rhs, Z: nr fields; iters, relres: per system.
bool cgls_shifted(Ctx& c, double mu, bool adjoint, const std::vector<cd>& shift, const c64* Rv, const c64* Lv, int m,
                  const c64* rhs, c64* Z, double tol, int max_it, std::vector<int>& iters,
                  std::vector<double>& relres) {
    const int nr = (int)shift.size();
    const c64* Pa = adjoint ? Rv : Lv;   // P z = Pb (Pa^dag z), P^dag y = Pa (Pb^dag y)
    const c64* Pb = adjoint ? Lv : Rv;
    const double amu = adjoint ? -mu : mu;
    c64* W = c.reuse(6 * nr);
    if (!W) return false;
    const long long blk = (long long)nr * c.nf;
    c64 *r = W, *s = W + blk, *p = W + 2 * blk, *q = W + 3 * blk, *u = W + 4 * blk, *t = W + 5 * blk;
    // device state: 5 coefficient triples per system, two m x nr coefficient
    // blocks, 6 nr doubles, the partial sums of the column norms and 2 nr ints
    const size_t nsc = ((size_t)6 * nr + (size_t)kDotBlocks * nr) * sizeof(double) + (size_t)2 * nr * sizeof(int);
    const size_t ncoef = (size_t)5 * 3 * nr, nmat = (size_t)2 * m * nr;
    void* mem = nullptr;
    if (!c.ok(hipMalloc(&mem, nsc + sizeof(c64) * (ncoef + nmat)), "hipMalloc")) return false;
    c.owned.push_back(mem);
    c64* cbase = (c64*)mem;
    c64 *cop = cbase, *copd = cbase + 3 * nr;
    CglsState d;
    d.cz = cbase + 6 * nr;
    d.cr = cbase + 9 * nr;
    d.cp = cbase + 12 * nr;
    c64* Cd = cbase + ncoef;                  // m x nr projection coefficients
    c64* Cn = Cd + (size_t)m * nr;            // their negation
    double* dd = (double*)(cbase + ncoef + nmat);
    double* npart = dd + 6 * nr;              // [nr][kDotBlocks] partial norms
    d.bn = dd;
    d.gam = dd + nr;
    d.qq = dd + 2 * nr;
    d.rn = dd + 3 * nr;
    d.gn = dd + 4 * nr;
    d.relres = dd + 5 * nr;
    d.active = (int*)(npart + (size_t)kDotBlocks * nr);
    d.iters = d.active + nr;
    const unsigned g1 = (unsigned)((nr + 63) / 64);
    // the per-system coefficients of op and op^dag, fixed for the whole solve
    {
        std::vector<c64> h((size_t)6 * nr);
        for (int j = 0; j < nr; ++j) {
            const cd a = shift[j] - 1.0, ac = std::conj(shift[j]);
            h[3 * j] = c64{a.real(), a.imag()};
            h[3 * j + 1] = c64{-1.0, 0.0};
            h[3 * j + 2] = c64{1.0, 0.0};
            h[3 * nr + 3 * j] = c64{ac.real(), ac.imag()};
            h[3 * nr + 3 * j + 1] = c64{-1.0, 0.0};
            h[3 * nr + 3 * j + 2] = c64{0.0, 0.0};
        }
        if (!c.ok(hipMemcpyAsync(cop, h.data(), sizeof(c64) * h.size(), hipMemcpyHostToDevice, c.s), "copy") ||
            !c.ok(hipStreamSynchronize(c.s), "sync"))   // h is released on return
            return false;
    }
    if (!c.ensure_scratch(m, nr)) return false;
    // squared 2-norms of the nr columns of x into n2 (device)
    auto norms2 = [&](const c64* x, double* n2) -> bool {
        colnorm2_partial_kernel<<<dim3(kDotBlocks, (unsigned)nr), 256, 0, c.s>>>(c.nf, x, npart);
        colnorm2_final_kernel<<<(unsigned)nr, 256, 0, c.s>>>(kDotBlocks, npart, n2);
        return c.ok(hipGetLastError(), "colnorm2");
    };
    // the m-vector projections reduce over chunks of kCglsChunk elements
    // (fewer partial sums than the default, which suits one-vector products)
    constexpr long long kCglsChunk = 512;
    // out = op(zin): u = (1 - P) zin, out_j = shift_j u_j - A u_j + (zin_j - u_j)
    auto op = [&](const c64* zin, c64* out) -> bool {
        if (!c.proj_dev(Pa, m, zin, nr, Cd, kCglsChunk)) return false;
        cneg_kernel<<<(unsigned)((m * nr + 255) / 256), 256, 0, c.s>>>(m * nr, Cd, Cn);
        if (!c.comb_dev(Pb, m, Cn, nr, zin, u)) return false;
        if (!c.apply(0, amu, u, out, nr)) return false;
        return c.blincomb(nr, cop, u, out, zin, out);
    };
    // out = op_j^dag(y) = (1 - P^dag)(conj(shift_j) y - A^dag y) + P^dag y = t + Pa (Pb^dag (y - t))
    auto opd = [&](const c64* y, c64* out) -> bool {
        if (!c.apply(0, -amu, y, t, nr)) return false;
        if (!c.blincomb(nr, copd, y, t, nullptr, t)) return false;
        if (!c.lincomb(blk, 1.0, y, -1.0, t, 0.0, nullptr, u)) return false;
        if (!c.proj_dev(Pb, m, u, nr, Cd, kCglsChunk)) return false;
        return c.comb_dev(Pa, m, Cd, nr, t, out);
    };
    iters.assign(nr, 0);
    relres.assign(nr, 0.0);
    if (!c.ok(hipMemsetAsync(Z, 0, sizeof(c64) * blk, c.s), "memset")) return false;
    if (!norms2(rhs, d.bn)) return false;
    cgls_init_kernel<<<g1, 64, 0, c.s>>>(nr, d);
    if (!c.copy(r, rhs, nr) || !opd(r, s) || !c.copy(p, s, nr) || !norms2(s, d.gam)) return false;
    std::vector<int> act(nr);
    for (int it = 0; it < max_it; ++it) {
        if (it % kCgCheck == 0) {
            if (!c.ok(hipMemcpyAsync(act.data(), d.active, sizeof(int) * nr, hipMemcpyDeviceToHost, c.s), "copy") ||
                !c.ok(hipStreamSynchronize(c.s), "sync"))
                return false;
            if (std::none_of(act.begin(), act.end(), [](int a) { return a != 0; })) break;
        }
        if (!op(p, q) || !norms2(q, d.qq)) return false;
        cgls_alpha_kernel<<<g1, 64, 0, c.s>>>(nr, d);
        if (!c.blincomb(nr, d.cz, Z, p, nullptr, Z) || !c.blincomb(nr, d.cr, r, q, nullptr, r)) return false;
        if (!norms2(r, d.rn)) return false;
        cgls_conv_kernel<<<g1, 64, 0, c.s>>>(nr, d, tol);
        if (!opd(r, s) || !norms2(s, d.gn)) return false;
        cgls_beta_kernel<<<g1, 64, 0, c.s>>>(nr, d);
        if (!c.blincomb(nr, d.cp, s, p, nullptr, p)) return false;
        if (!c.ok(hipGetLastError(), "cgls")) return false;
    }
    if (!c.ok(hipMemcpyAsync(iters.data(), d.iters, sizeof(int) * nr, hipMemcpyDeviceToHost, c.s), "copy")) return false;
    // true residuals of the final iterates
    std::vector<double> bn(nr), rn(nr);
    if (!op(Z, q)) return false;
    if (!c.lincomb(blk, 1.0, rhs, -1.0, q, 0.0, nullptr, r)) return false;
    if (!norms2(r, d.rn)) return false;
    if (!c.ok(hipMemcpyAsync(bn.data(), d.bn, sizeof(double) * nr, hipMemcpyDeviceToHost, c.s), "copy") ||
        !c.ok(hipMemcpyAsync(rn.data(), d.rn, sizeof(double) * nr, hipMemcpyDeviceToHost, c.s), "copy") ||
        !c.ok(hipStreamSynchronize(c.s), "sync"))
        return false;
    for (int j = 0; j < nr; ++j) relres[j] = bn[j] > 0 ? std::sqrt(rn[j]) / bn[j] : 0.0;
    return true;
}

}  // namespace

int eigs_compute(const EigParams& P, EigResult& out) {
    const auto t0 = std::chrono::steady_clock::now();
    if (verbose()) (void)vclock();
    Ctx c;
    c.g = P.g;
    c.U = P.U;
    c.dU = P.dU;
    c.md = P.md;
    c.s = P.stream;
    c.nf = (long long)12 * P.g.Vp;
    const int m = P.m, l = P.l;
    const int p = P.p > m ? P.p : 2 * m + 20;   // Arnoldi basis size
    out = EigResult{};
    // on failure the context still owns (and frees) every buffer, including
    // those already named in out: the caller must not free them again
    auto fail = [&](int code) {
        out.err = c.err.empty() ? "eigensolver failed" : c.err;
        out.R = out.L = out.dR = out.dL = nullptr;
        return code;
    };
    c64* Rv = c.fields(m);
    c64* Lraw = c.fields(m);
    if (!Rv || !Lraw) return fail(-2);
    SideResult right, left;
    {
        // The two sides are independent.  The left one runs from a second host
        // thread on a second stream with workspaces of its own, so that the
        // small launches of the two sides (one field each) overlap on the GPU.
        hipStream_t s2 = nullptr;
        hipEvent_t ready = nullptr;
        if (!c.ok(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking), "hipStreamCreate")) return fail(-3);
        bool ok1 = c.ok(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "hipEventCreate") &&
                   c.ok(hipEventRecord(ready, c.s), "hipEventRecord") &&
                   c.ok(hipStreamWaitEvent(s2, ready, 0), "hipStreamWaitEvent");   // links and Lraw are ready
        bool ok2 = ok1;
        std::string err2;
        if (ok1) {
            Ctx c2;
            c2.g = c.g;
            c2.U = c.U;
            c2.dU = c.dU;
            c2.md = c.md;
            c2.s = s2;
            c2.nf = c.nf;
            std::thread left_side([&] {
                ok2 = arnoldi_side(c2, -P.mu, m, p, P.tol, P.max_outer, P.seed + 1, Lraw, left);
            });
            ok1 = arnoldi_side(c, P.mu, m, p, P.tol, P.max_outer, P.seed, Rv, right);
            left_side.join();
            ok2 = c2.ok(hipStreamSynchronize(s2), "sync") && ok2;   // before c2's workspaces are freed
            err2 = c2.err;
        }
        if (ready) (void)hipEventDestroy(ready);
        (void)hipStreamDestroy(s2);
        if (!ok1) return fail(-3);
        if (!ok2) {
            if (c.err.empty()) c.err = err2;
            return fail(-3);
        }
    }
    out.outer_right = right.outer;
    out.outer_left = left.outer;
    out.res_right = right.max_res;
    out.res_left = left.max_res;
    if (right.max_res > P.tol || left.max_res > P.tol) {
        c.err = "eigenpairs not converged: residual " + std::to_string(std::max(right.max_res, left.max_res)) +
                " after " + std::to_string(std::max(right.outer, left.outer)) + " restart cycles";
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
        c64* rhs = c.fields(l);
        c64* z = c.fields(l);
        if (!D || !DL || !dR || !dL || !rhs || !z) return fail(-2);
        if (!c.apply(dop, P.mu, Rv, D, m)) return fail(-3);
        // (d/dmu H)^dag = -(d/dmu H)(-mu); for a link direction dH^dag = dH(-mu)
        if (!c.apply(dop, -P.mu, Lv, DL, l)) return fail(-3);
        if (!P.dir_link && !c.lincomb((long long)l * c.nf, -1.0, DL, 0.0, nullptr, 0.0, nullptr, DL)) return fail(-3);
        std::vector<cd> C;   // C[i][j] = L_i^dag dA R_j
        if (!c.proj(Lv, m, D, m, C)) return fail(-3);
        std::vector<cd> lam(m);
        for (int i = 0; i < m; ++i) lam[i] = right.theta[i];
        // the derivatives of pair j divide by lam_j - lam_i and invert lam_j - H
        // outside the set: an eigenvalue equal to lam_j elsewhere in the set, or
        // just beyond it (the next Ritz value), makes them undefined
        for (int j = 0; j < l; ++j) {
            for (int i = 0; i < m; ++i)
                if (i != j && std::abs(lam[j] - lam[i]) < 1e-9 * (1.0 + std::abs(lam[j]))) {
                    c.err = "degenerate eigenvalues among the derivative pairs";
                    return fail(-7);
                }
            if (std::abs(right.next) > 0.0 && std::abs(lam[j] - right.next) < 1e-9 * (1.0 + std::abs(lam[j]))) {
                c.err = "a derivative pair's eigenvalue recurs just beyond the m-th (a degenerate cluster "
                        "straddles the cut; choose another m)";
                return fail(-7);
            }
        }
        auto record = [&](const char* side, const std::vector<int>& its, const std::vector<double>& res) {
            for (int j = 0; j < l; ++j) {
                if (verbose()) {
                    std::fprintf(stderr, "[%.2f s] eigs %s_%d: %d CGLS iterations, residual %.2e\n", vclock(), side, j, its[j],
                                 res[j]);
                    std::fflush(stderr);
                }
                out.shift_iters += its[j];
                out.shift_res = std::max(out.shift_res, res[j]);
            }
        };
        // right, all l at once: rhs_j = (1 - P) dA R_j, then dR_j = z_j + sum_{i != j} R_i C_ij / (lam_j - lam_i)
        auto right_side = [&](Ctx& cx, c64* rb, c64* zb, std::vector<int>& its, std::vector<double>& res) -> bool {
            if (!cx.copy(rb, D, l)) return false;
            std::vector<cd> cm((size_t)m * l), sr((size_t)m * l, cd(0));
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < l; ++j) {
                    cm[(size_t)i * l + j] = -C[(size_t)i * m + j];
                    if (i != j) sr[(size_t)i * l + j] = C[(size_t)i * m + j] / (lam[j] - lam[i]);
                }
            if (!cx.comb(Rv, m, cm, l, rb)) return false;
            if (!cgls_shifted(cx, P.mu, false, std::vector<cd>(lam.begin(), lam.begin() + l), Rv, Lv, m, rb, zb,
                              P.shift_tol, P.shift_max, its, res))
                return false;
            return cx.copy(dR, zb, l) && cx.comb(Rv, m, sr, l, dR);
        };
        // left: rhs_j = (1 - P)^dag dA^dag L_j = e_j - L (R^dag e_j), then
        // dL_j = z_j + sum_{i != j} L_i conj(C_ji / (lam_j - lam_i))
        auto left_side = [&](Ctx& cx, c64* rb, c64* zb, std::vector<int>& its, std::vector<double>& res) -> bool {
            std::vector<cd> pr;
            if (!cx.proj(Rv, m, DL, l, pr)) return false;
            if (!cx.copy(rb, DL, l)) return false;
            for (auto& v : pr) v = -v;
            if (!cx.comb(Lv, m, pr, l, rb)) return false;
            std::vector<cd> shl(l), sl((size_t)m * l, cd(0));
            for (int j = 0; j < l; ++j) shl[j] = std::conj(lam[j]);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < l; ++j)
                    if (i != j) sl[(size_t)i * l + j] = std::conj(C[(size_t)j * m + i] / (lam[j] - lam[i]));
            if (!cgls_shifted(cx, P.mu, true, shl, Rv, Lv, m, rb, zb, P.shift_tol, P.shift_max, its, res))
                return false;
            return cx.copy(dL, zb, l) && cx.comb(Lv, m, sl, l, dL);
        };
        // the two sets of systems are independent: the left one runs from a
        // second host thread on a second stream with workspaces of its own
        {
            c64* rhs2 = c.fields(l);
            c64* z2 = c.fields(l);
            if (!rhs2 || !z2) return fail(-2);
            std::vector<int> its_r, its_l;
            std::vector<double> res_r, res_l;
            hipStream_t s2 = nullptr;
            hipEvent_t ready = nullptr;
            if (!c.ok(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking), "hipStreamCreate")) return fail(-3);
            bool ok1 = c.ok(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "hipEventCreate") &&
                       c.ok(hipEventRecord(ready, c.s), "hipEventRecord") &&
                       c.ok(hipStreamWaitEvent(s2, ready, 0), "hipStreamWaitEvent");   // D, DL, R, L are ready
            bool ok2 = ok1;
            std::string err2;
            if (ok1) {
                Ctx c2;
                c2.g = c.g;
                c2.U = c.U;
                c2.dU = c.dU;
                c2.md = c.md;
                c2.s = s2;
                c2.nf = c.nf;
                std::thread left_thread([&] { ok2 = left_side(c2, rhs2, z2, its_l, res_l); });
                ok1 = right_side(c, rhs, z, its_r, res_r);
                left_thread.join();
                ok2 = c2.ok(hipStreamSynchronize(s2), "sync") && ok2;   // before c2's workspaces are freed
                err2 = c2.err;
            }
            if (ready) (void)hipEventDestroy(ready);
            (void)hipStreamDestroy(s2);
            if (!ok1) return fail(-3);
            if (!ok2) {
                if (c.err.empty()) c.err = err2;
                return fail(-3);
            }
            record("dR", its_r, res_r);
            record("dL", its_l, res_l);
        }
        if (out.shift_res > 1e3 * P.shift_tol) {
            c.err = "shifted solves for the eigenvector derivatives did not converge (residual " +
                    std::to_string(out.shift_res) + ")";
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
