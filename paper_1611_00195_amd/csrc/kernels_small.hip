// sgn(T_k) e_1 for the k x k complex tridiagonal Ritz matrices of two-sided
// Lanczos, in FP64 on gfx950.
//
// The sign is discontinuous on the imaginary axis (Sec. 3); for a matrix with
// no eigenvalue there,
//     sgn(T) = (2/pi) int_0^inf T (T^2 + y^2)^{-1} dy
//            = (1/pi) int_0^inf [(T + iy)^{-1} + (T - iy)^{-1}] dy,
// because (2/pi) int_0^inf z/(z^2 + y^2) dy = sgn(Re z).  With y = e^s the
// integrand is analytic in a strip of half-width d = pi/2 - max|arg(+-theta)|
// around the real s axis, so the trapezoidal rule in s converges geometrically
// (error ~ exp(-2 pi d / h)).  Each node costs two tridiagonal solves with
// right-hand side e_1, O(k) each and independent: one GPU thread per solve, no
// eigendecomposition, and unlike the spectral form the result stays accurate
// when Ritz values pair up (the block matrix of eq. 6 is not diagonalisable,
// Sec. 3, and its Ritz matrices are close to defective).
//
// Adaptivity: the step is halved level by level (new nodes at the midpoints,
// the sums of earlier levels are reused) until two successive levels agree to
// a tolerance; in the geometric regime the error of the finer level is about
// the square of that difference.  Ritz values close to the imaginary axis
// (small d) thus cost more levels instead of silently losing accuracy.
//
// Nodes: s = smin + q h, smin = log(theta_max) - 54, up to log(theta_max) + 11.5,
// theta_max the Gershgorin bound of T.  Below the first node the integrand is
// < e^{-38} relative for every |theta| >= e^{-16} theta_max; above the last
// node the sum is continued analytically with the large-y expansion
// (T + iy)^{-1} + (T - iy)^{-1} = 2 (T/y^2 - T^3/y^4 + ...), summed over the
// remaining trapezoidal nodes as a geometric series.
//
// Each solve is Gaussian elimination with partial pivoting on the tridiagonal
// T + sigma I (rows swapped when the subdiagonal entry is larger in modulus),
// which fills one extra superdiagonal; the factors are kept in a scratch array
// laid out [field][row][solve] so that the 64 solves of a wave store and load
// contiguously.
#include "ovd_internal.h"

#include <vector>

namespace ovd {

static constexpr double kLowSpan = 54.0;
static constexpr double kHighSpan = 11.5;
static constexpr int kMaxLevels = 9;
static constexpr int kChunkSolves = 16384;   // solves per launch over all rhs (bounds the scratch)

size_t small_sign_scratch_elems(int nrhs, int k, double quad_step) {
    (void)quad_step;
    (void)nrhs;
    return 4 * (size_t)k * kChunkSolves + (size_t)4 * nrhs * k + 2 * (size_t)nrhs;
}

__device__ __forceinline__ c64 tdiag(const TslCoeffs& co, int r, int i) { return co.alpha[(size_t)r * co.kmax + i]; }
// T[i][i+1] = beta[i+1],  T[i+1][i] = delta[i+1]
__device__ __forceinline__ c64 tsup(const TslCoeffs& co, int r, int i) { return co.beta[(size_t)r * co.kmax + i + 1]; }
__device__ __forceinline__ c64 tsub(const TslCoeffs& co, int r, int i) { return co.delta[(size_t)r * co.kmax + i + 1]; }

// smin[r] = log(Gershgorin bound of T_r) - kLowSpan, one thread per rhs
__global__ void small_sign_setup_kernel(int nrhs, int k, TslCoeffs co, double* __restrict__ smin) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double m = 0.0;
    for (int i = 0; i < k; ++i) {
        double a = sqrt(norm2(tdiag(co, r, i)));
        if (i + 1 < k) a += sqrt(norm2(tsup(co, r, i)));
        if (i > 0) a += sqrt(norm2(tsub(co, r, i - 1)));
        m = a > m ? a : m;
    }
    smin[r] = log(m > 0.0 ? m : 1.0) - kLowSpan;
}

// Solves for nodes s = smin[r] + (off + q) h, q in [q0, q0 + nq), both signs of
// the shift; thread = (rhs, q, sign).  Writes e^s x into the B slot.
__global__ __launch_bounds__(64) void small_sign_solve_kernel(int nrhs, int k, TslCoeffs co,
                                                              const double* __restrict__ smin, double h,
                                                              double off, int q0, int nq,
                                                              c64* __restrict__ scr, int transpose, int scale) {
    const int nsol = nrhs * 2 * nq;
    const int sol = blockIdx.x * blockDim.x + threadIdx.x;
    if (sol >= nsol) return;
    const int r = sol / (2 * nq);
    const int q = q0 + ((sol % (2 * nq)) >> 1);
    const double sgn = (sol & 1) ? -1.0 : 1.0;
    const double y = exp(smin[r] + (off + q) * h);
    const c64 sigma{0.0, sgn * y};
    c64* D = scr;                              // pivot row diagonal
    c64* DU = scr + (size_t)k * nsol;          // first superdiagonal
    c64* DU2 = scr + (size_t)2 * k * nsol;     // second superdiagonal (fill from pivoting)
    c64* B = scr + (size_t)3 * k * nsol;       // right-hand side, then solution
#define AT(P, i) P[(size_t)(i) * nsol + sol]
    // forward elimination with partial pivoting
    c64 cd = tdiag(co, r, 0) + sigma;
    c64 cu = (k > 1) ? (transpose ? tsub(co, r, 0) : tsup(co, r, 0)) : c64{0.0, 0.0};
    c64 cb{1.0, 0.0};
    for (int i = 0; i + 1 < k; ++i) {
        const c64 dl = transpose ? tsup(co, r, i) : tsub(co, r, i);
        const c64 dn = tdiag(co, r, i + 1) + sigma;
        const c64 un = (i + 2 < k) ? (transpose ? tsub(co, r, i + 1) : tsup(co, r, i + 1)) : c64{0.0, 0.0};
        if (cabs1(cd) >= cabs1(dl)) {
            const c64 f = cdiv(dl, cd);
            AT(D, i) = cd; AT(DU, i) = cu; AT(DU2, i) = c64{0.0, 0.0}; AT(B, i) = cb;
            cd = dn - f * cu;
            cu = un;
            cb = -(f * cb);
        } else {
            // swap rows i and i+1; the new row i+1 is the old row i minus f
            // times the swapped-in row, whose right-hand side is zero
            const c64 f = cdiv(cd, dl);
            AT(D, i) = dl; AT(DU, i) = dn; AT(DU2, i) = un; AT(B, i) = c64{0.0, 0.0};
            const c64 nd = cu - f * dn;
            cu = -(f * un);
            cd = nd;
        }
    }
    if (cabs1(cd) == 0.0) cd = c64{1e-300, 0.0};
    // back substitution, scaled by the node weight e^s when asked
    const double wgt = scale ? y : 1.0;
    c64 x1 = cdiv(cb, cd);
    AT(B, k - 1) = wgt * x1;
    c64 x2{0.0, 0.0};
    for (int i = k - 2; i >= 0; --i) {
        const c64 xi = cdiv(AT(B, i) - AT(DU, i) * x1 - AT(DU2, i) * x2, AT(D, i));
        AT(B, i) = wgt * xi;
        x2 = x1;
        x1 = xi;
    }
#undef AT
}

// acc[r][i] += sum over the chunk's nodes (in order) of e^s (x+ [i] + x- [i])
__global__ void small_sign_accum_kernel(int nrhs, int k, int nq, const c64* __restrict__ scr,
                                        c64* __restrict__ acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= k) return;
    const int nsol = nrhs * 2 * nq;
    const c64* B = scr + (size_t)3 * k * nsol + (size_t)i * nsol + (size_t)r * 2 * nq;
    c64 a = acc[(size_t)r * k + i];
    for (int q = 0; q < nq; ++q) a += B[2 * q] + B[2 * q + 1];
    acc[(size_t)r * k + i] = a;
}

// c = (h/pi) acc + tail(h); diff[r] = max_i |c - c_prev| (one block per rhs); c_prev <- c
__global__ void small_sign_finalize_kernel(int k, TslCoeffs co, const double* __restrict__ smin, double h,
                                           int qlast, const c64* __restrict__ acc, c64* __restrict__ c_out,
                                           c64* __restrict__ c_prev, double* __restrict__ diff) {
    __shared__ double red[256];
    __shared__ c64 tail[4];
    const int r = blockIdx.x;
    if (threadIdx.x == 0) {
        // tail beyond the last node sL: sum_{m>=1} (2/pi) h [T e^{-s} - T^3 e^{-3s}] e_1, s = sL + m h
        const double sL = smin[r] + qlast * h;
        const double E = exp(-h);
        const double w1 = (2.0 / M_PI) * h * exp(-sL) * E / (1.0 - E);
        const double w3 = (2.0 / M_PI) * h * exp(-3.0 * sL) * E * E * E / (1.0 - E * E * E);
        c64 v1[4] = {}, v2[4] = {}, v3[4] = {};
        auto T = [&](int a, int b) -> c64 {
            if (a >= k || b >= k) return c64{0.0, 0.0};
            if (a == b) return tdiag(co, r, a);
            if (b == a + 1) return tsup(co, r, a);
            if (a == b + 1) return tsub(co, r, b);
            return c64{0.0, 0.0};
        };
        for (int a = 0; a < 4; ++a) v1[a] = T(a, 0);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) v2[a] += T(a, b) * v1[b];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) v3[a] += T(a, b) * v2[b];
        for (int a = 0; a < 4; ++a) tail[a] = w1 * v1[a] - w3 * v3[a];
    }
    __syncthreads();
    double dmax = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        c64 c = (h / M_PI) * acc[(size_t)r * k + i];
        if (i < 4) c += tail[i];
        const c64 d = c - c_prev[(size_t)r * k + i];
        const double ad = sqrt(norm2(d));
        dmax = ad > dmax ? ad : dmax;
        c_prev[(size_t)r * k + i] = c;
        c_out[(size_t)r * k + i] = c;
    }
    red[threadIdx.x] = dmax;
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
        if (threadIdx.x < m) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + m] ? red[threadIdx.x] : red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) diff[r] = red[0];
}

// Host driver: level 0 with step h0 = 2 quad_step, then midpoint refinements
// until max_r diff_r <= tol (at least one refinement, at most kMaxLevels).
// Returns the last difference (an error estimate of the previous level, an
// upper bound of the final error in the geometric regime) in *check.
void launch_small_sign(int nrhs, int k, TslCoeffs co, double quad_step, c64* scratch, size_t scratch_elems,
                       c64* c_out, double* check, hipStream_t s) {
    (void)scratch_elems;
    c64* scr = scratch;
    c64* acc = scratch + 4 * (size_t)k * kChunkSolves;
    c64* cprev = acc + (size_t)nrhs * k;
    double* smin = (double*)(cprev + (size_t)nrhs * k);
    double* diff = smin + nrhs;
    (void)hipMemsetAsync(acc, 0, sizeof(c64) * 2 * nrhs * k, s);
    small_sign_setup_kernel<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, k, co, smin);
    const double h0 = 2.0 * quad_step;
    const int Q0 = (int)ceil((kLowSpan + kHighSpan) / h0) + 1;
    const int chunk = kChunkSolves / (2 * nrhs) > 0 ? kChunkSolves / (2 * nrhs) : 1;
    const double tol = 1e-10;
    std::vector<double> hd(nrhs);
    double last = 0.0;
    for (int lev = 0; lev <= kMaxLevels; ++lev) {
        // nodes of this level: level 0 all Q0 nodes at spacing h0; level l >= 1
        // the (Q0 - 1) 2^{l-1} midpoints at spacing h0 / 2^{l-1}
        const double sp = lev == 0 ? h0 : h0 / (double)(1 << (lev - 1));
        const double off = lev == 0 ? 0.0 : 0.5;
        const int nq = lev == 0 ? Q0 : (Q0 - 1) * (1 << (lev - 1));
        for (int q0 = 0; q0 < nq; q0 += chunk) {
            const int n = (nq - q0) < chunk ? (nq - q0) : chunk;
            const int nsol = nrhs * 2 * n;
            small_sign_solve_kernel<<<(nsol + 63) / 64, 64, 0, s>>>(nrhs, k, co, smin, sp, off, q0, n, scr, 0, 1);
            dim3 g((k + 127) / 128, nrhs);
            small_sign_accum_kernel<<<g, 128, 0, s>>>(nrhs, k, n, scr, acc);
        }
        const double hl = h0 / (double)(1 << lev);
        // the last node is s = smin + (Q0 - 1) h0 = smin + qlast * hl
        const int qlast = (Q0 - 1) * (1 << lev);
        small_sign_finalize_kernel<<<nrhs, 256, 0, s>>>(k, co, smin, hl, qlast, acc, c_out, cprev, diff);
        if (lev == 0) continue;
        (void)hipMemcpyAsync(hd.data(), diff, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s);
        (void)hipStreamSynchronize(s);
        last = 0.0;
        for (double d : hd) last = d > last ? d : last;
        if (last <= tol) break;
    }
    if (check) *check = last;
}


// ===========================================================================
// Frechet derivative M = L_sgn(T, e_1 e_1^T) for the gradient of
// <x|sgn(H)|b>, by differentiating the same integral:
//   M = -(1/pi) int_0^inf [(T + iy)^{-1} E (T + iy)^{-1} + (T - iy)^{-1} E (T - iy)^{-1}] dy,
//   E = e_1 e_1^T,  (T + iy)^{-1} E (T + iy)^{-1} = x x~^T with
//   x = (T + iy)^{-1} e_1,  x~ = (T^T + iy)^{-1} e_1,
// on the same nodes and with the same level-by-level refinement as the sign;
// the tail beyond the last node is w1 E - w3 (E T^2 + T E T + T^2 E).
// The node sum  sum_q e^{s_q} x_q x~_q^T  is a complex (k x S)(S x k) product,
// accumulated on the matrix cores.
// ===========================================================================
typedef double v4d __attribute__((ext_vector_type(4)));

// Msum[i][j] += sum_sol XA[i][sol] XB[j][sol]  (k x k, XA/XB laid out [row][sol], nsol solves)
__global__ __launch_bounds__(64) void frechet_accum_kernel(int k, int nsol, const c64* __restrict__ XA,
                                                           const c64* __restrict__ XB, c64* __restrict__ M) {
    const int l = threadIdx.x;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    const int ia = i0 + (l & 15), jb = j0 + (l & 15), kk = l >> 4;
    const bool va = ia < k, vb = jb < k;
    v4d re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
    for (int s = 0; s < nsol; s += 4) {
        const int sl = s + kk;
        c64 a{0.0, 0.0}, b{0.0, 0.0};
        if (va && sl < nsol) a = XA[(size_t)ia * nsol + sl];
        if (vb && sl < nsol) b = XB[(size_t)jb * nsol + sl];
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.im, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.re, im, 0, 0, 0);
    }
    const int jj = j0 + (l & 15);
    for (int v = 0; v < 4; ++v) {
        const int ii = i0 + 4 * v + (l >> 4);
        if (ii < k && jj < k) M[(size_t)ii * k + jj] = M[(size_t)ii * k + jj] + c64{re[v], im[v]};
    }
}

// Mout = -(h/pi) Msum + tail; diff = max |Mout - Mprev|; Mprev <- Mout   (one block)
__global__ void frechet_finalize_kernel(int k, TslCoeffs co, const double* __restrict__ smin, double h, int qlast,
                                        const c64* __restrict__ Msum, c64* __restrict__ Mout,
                                        c64* __restrict__ Mprev, double* __restrict__ diff) {
    __shared__ double red[256];
    __shared__ c64 T2[3][3], Tm[3][3];
    __shared__ double w1s, w3s;
    const int r = 0;
    if (threadIdx.x == 0) {
        const double sL = smin[r] + qlast * h;
        const double E = exp(-h);
        w1s = (2.0 / M_PI) * h * exp(-sL) * E / (1.0 - E);
        w3s = (2.0 / M_PI) * h * exp(-3.0 * sL) * E * E * E / (1.0 - E * E * E);
        auto T = [&](int a, int b) -> c64 {
            if (a >= k || b >= k) return c64{0.0, 0.0};
            if (a == b) return tdiag(co, r, a);
            if (b == a + 1) return tsup(co, r, a);
            if (a == b + 1) return tsub(co, r, b);
            return c64{0.0, 0.0};
        };
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                Tm[a][b] = T(a, b);
                c64 s{0.0, 0.0};
                for (int c = 0; c < 4; ++c) s += T(a, c) * T(c, b);
                T2[a][b] = s;
            }
    }
    __syncthreads();
    double dmax = 0.0;
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
        const int i = t / k, j = t % k;
        c64 m = (-h / M_PI) * Msum[t];
        // tail: w1 E - w3 (E T^2 + T E T + T^2 E), E = e_1 e_1^T
        if (i == 0 && j == 0) m += c64{w1s, 0.0};
        c64 t3{0.0, 0.0};
        if (i == 0 && j < 3) t3 += T2[0][j];
        if (i < 2 && j < 2) t3 += Tm[i][0] * Tm[0][j];
        if (j == 0 && i < 3) t3 += T2[i][0];
        m -= w3s * t3;
        const c64 d = m - Mprev[t];
        const double ad = sqrt(norm2(d));
        dmax = ad > dmax ? ad : dmax;
        Mprev[t] = m;
        Mout[t] = m;
    }
    red[threadIdx.x] = dmax;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) diff[0] = red[0];
}

size_t small_frechet_scratch_elems(int k) {
    return 2 * (4 * (size_t)k * kChunkSolves) + 3 * (size_t)k * k + 4;
}

// M (k x k, row-major) = L_sgn(T, e_1 e_1^T) for one tridiagonal (rhs 0 of co)
void launch_small_frechet(int k, TslCoeffs co, double quad_step, c64* scratch, c64* M_out, double* check,
                          hipStream_t s) {
    c64* scrA = scratch;
    c64* scrB = scrA + 4 * (size_t)k * kChunkSolves;
    c64* Msum = scrB + 4 * (size_t)k * kChunkSolves;
    c64* Mprev = Msum + (size_t)k * k;
    double* smin = (double*)(Mprev + (size_t)k * k);
    double* diff = smin + 2;
    (void)hipMemsetAsync(Msum, 0, sizeof(c64) * 2 * k * k, s);
    small_sign_setup_kernel<<<1, 64, 0, s>>>(1, k, co, smin);
    const double h0 = 2.0 * quad_step;
    const int Q0 = (int)ceil((kLowSpan + kHighSpan) / h0) + 1;
    const int chunk = kChunkSolves / 2;
    double hd = 0.0, last = 0.0;
    for (int lev = 0; lev <= kMaxLevels; ++lev) {
        const double sp = lev == 0 ? h0 : h0 / (double)(1 << (lev - 1));
        const double off = lev == 0 ? 0.0 : 0.5;
        const int nq = lev == 0 ? Q0 : (Q0 - 1) * (1 << (lev - 1));
        for (int q0 = 0; q0 < nq; q0 += chunk) {
            const int n = (nq - q0) < chunk ? (nq - q0) : chunk;
            const int nsol = 2 * n;
            // scaled solves with T (weight e^s folded in), unscaled with T^T
            small_sign_solve_kernel<<<(nsol + 63) / 64, 64, 0, s>>>(1, k, co, smin, sp, off, q0, n, scrA, 0, 1);
            small_sign_solve_kernel<<<(nsol + 63) / 64, 64, 0, s>>>(1, k, co, smin, sp, off, q0, n, scrB, 1, 0);
            dim3 g((k + 15) / 16, (k + 15) / 16);
            frechet_accum_kernel<<<g, 64, 0, s>>>(k, nsol, scrA + (size_t)3 * k * nsol, scrB + (size_t)3 * k * nsol,
                                                  Msum);
        }
        const double hl = h0 / (double)(1 << lev);
        const int qlast = (Q0 - 1) * (1 << lev);
        frechet_finalize_kernel<<<1, 256, 0, s>>>(k, co, smin, hl, qlast, Msum, M_out, Mprev, diff);
        if (lev == 0) continue;
        (void)hipMemcpyAsync(&hd, diff, sizeof(double), hipMemcpyDeviceToHost, s);
        (void)hipStreamSynchronize(s);
        last = hd;
        if (last <= 1e-10) break;
    }
    if (check) *check = last;
}

}  // namespace ovd
