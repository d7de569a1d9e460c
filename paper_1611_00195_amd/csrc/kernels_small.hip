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
static constexpr double kSignTol = 1e-10;   // agreement of two refinement levels

size_t small_sign_scratch_elems(int nrhs, int k, int chunk) {
    if (chunk < 1) chunk = kDefaultChunkSolves;
    return 4 * (size_t)k * chunk + (size_t)4 * nrhs * k + 2 * (size_t)nrhs;
}

__device__ __forceinline__ c64 tdiag(const TslCoeffs& co, int r, int i) { return co.alpha[(size_t)r * co.kmax + i]; }
// T[i][i+1] = beta[i+1],  T[i+1][i] = delta[i+1]
__device__ __forceinline__ c64 tsup(const TslCoeffs& co, int r, int i) { return co.beta[(size_t)r * co.kmax + i + 1]; }
__device__ __forceinline__ c64 tsub(const TslCoeffs& co, int r, int i) { return co.delta[(size_t)r * co.kmax + i + 1]; }

// smin[r] = log(Gershgorin bound of T_r) - kLowSpan, one block of 256 per rhs
// (the rows spread over the block, then a max over its threads)
__global__ __launch_bounds__(256) void small_sign_setup_kernel(int nrhs, int k, TslCoeffs co,
                                                               double* __restrict__ smin) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    if (r >= nrhs) return;
    double m = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        double a = sqrt(norm2(tdiag(co, r, i)));
        if (i + 1 < k) a += sqrt(norm2(tsup(co, r, i)));
        if (i > 0) a += sqrt(norm2(tsub(co, r, i - 1)));
        m = a > m ? a : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x] : red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) smin[r] = log(red[0] > 0.0 ? red[0] : 1.0) - kLowSpan;
}

// 1 / z, scaled against overflow as in Smith's division; written with selects
// so that the lanes of a wave (different shifts) do not diverge
__device__ __forceinline__ c64 crecip(c64 z) {
    const bool big = fabs(z.re) >= fabs(z.im);
    const double p = big ? z.re : z.im, q = big ? z.im : z.re;
    const double r = q / p, d = 1.0 / (p + q * r);
    return big ? c64{d, -r * d} : c64{r * d, -d};
}

// Solves for nodes s = smin[r] + (off + q) h, q in [q0, q0 + nq), both signs of
// the shift; thread = (rhs, q, sign).  Writes e^s x into the B slot.
// Each row is a short dependent chain, so the loads that feed it (the entries
// of T in the elimination, the stored factor rows in the back substitution)
// are issued a group of kPf rows ahead; the elimination stores the reciprocal
// of each pivot, so the back substitution has no division on its chain.
constexpr int kPf = 4;
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
    const c64 zero{0.0, 0.0};
    c64* IP = scr;                             // reciprocal of the pivot row's diagonal
    c64* DU = scr + (size_t)k * nsol;          // first superdiagonal
    c64* DU2 = scr + (size_t)2 * k * nsol;     // second superdiagonal (fill from pivoting)
    c64* B = scr + (size_t)3 * k * nsol;       // right-hand side, then solution
#define AT(P, i) P[(size_t)(i) * nsol + sol]
    // entries of row i + 1 of T + sigma (dl: its subdiagonal entry, dn: its
    // diagonal, un: its superdiagonal), in the orientation of the solve
    auto row = [&](int i, c64& dl, c64& dn, c64& un) {
        dl = transpose ? tsup(co, r, i) : tsub(co, r, i);
        dn = tdiag(co, r, i + 1) + sigma;
        un = (i + 2 < k) ? (transpose ? tsub(co, r, i + 1) : tsup(co, r, i + 1)) : zero;
    };
    // forward elimination with partial pivoting
    c64 cd = tdiag(co, r, 0) + sigma;
    c64 cu = (k > 1) ? (transpose ? tsub(co, r, 0) : tsup(co, r, 0)) : zero;
    c64 cb{1.0, 0.0};
    c64 gl[kPf], gn[kPf], gu[kPf];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        gl[u] = gn[u] = gu[u] = zero;
        if (u + 1 < k) row(u, gl[u], gn[u], gu[u]);
    }
    for (int i0 = 0; i0 + 1 < k; i0 += kPf) {
        c64 nl[kPf], nn[kPf], nu[kPf];
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            nl[u] = nn[u] = nu[u] = zero;
            if (i0 + kPf + u + 1 < k) row(i0 + kPf + u, nl[u], nn[u], nu[u]);
        }
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            const int i = i0 + u;
            if (i + 1 >= k) break;
            const c64 dl = gl[u], dn = gn[u], un = gu[u];
            // sw: swap rows i and i+1 (the subdiagonal entry is the larger); the
            // new row i+1 is then the old row i minus f times the swapped-in
            // row, whose right-hand side is zero.  Selects, not branches: the
            // lanes choose their pivots independently.
            const bool sw = !(cabs1(cd) >= cabs1(dl));
            const c64 ip = crecip(sw ? dl : cd);
            const c64 f = (sw ? cd : dl) * ip;
            AT(IP, i) = ip;
            AT(DU, i) = sw ? dn : cu;
            AT(DU2, i) = sw ? un : zero;
            AT(B, i) = sw ? zero : cb;
            const c64 ncd = sw ? cu - f * dn : dn - f * cu;
            cu = sw ? -(f * un) : un;
            cb = sw ? cb : -(f * cb);
            cd = ncd;
        }
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            gl[u] = nl[u];
            gn[u] = nn[u];
            gu[u] = nu[u];
        }
    }
    if (cabs1(cd) == 0.0) cd = c64{1e-300, 0.0};
    // back substitution, scaled by the node weight e^s when asked
    const double wgt = scale ? y : 1.0;
    c64 x1 = cb * crecip(cd);
    AT(B, k - 1) = wgt * x1;
    c64 x2 = zero;
    c64 fb[kPf], fu[kPf], fu2[kPf], fp[kPf];
    auto fetch = [&](int i, c64& b, c64& du, c64& du2, c64& ip) {
        b = AT(B, i); du = AT(DU, i); du2 = AT(DU2, i); ip = AT(IP, i);
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        fb[u] = fu[u] = fu2[u] = fp[u] = zero;
        if (k - 2 - u >= 0) fetch(k - 2 - u, fb[u], fu[u], fu2[u], fp[u]);
    }
    for (int i0 = k - 2; i0 >= 0; i0 -= kPf) {
        c64 nb[kPf], nu[kPf], nu2[kPf], np[kPf];
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            nb[u] = nu[u] = nu2[u] = np[u] = zero;
            if (i0 - kPf - u >= 0) fetch(i0 - kPf - u, nb[u], nu[u], nu2[u], np[u]);
        }
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            const int i = i0 - u;
            if (i < 0) break;
            const c64 xi = (fb[u] - fu[u] * x1 - fu2[u] * x2) * fp[u];
            AT(B, i) = wgt * xi;
            x2 = x1;
            x1 = xi;
        }
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            fb[u] = nb[u];
            fu[u] = nu[u];
            fu2[u] = nu2[u];
            fp[u] = np[u];
        }
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
                                           long long qlast, const c64* __restrict__ acc, c64* __restrict__ c_out,
                                           c64* __restrict__ c_prev, double* __restrict__ diff, int transpose) {
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
            if (transpose) {
                const int t = a;
                a = b;
                b = t;
            }
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
// until max_r diff_r <= kSignTol (at least one refinement, at most
// cfg.max_levels).  The last difference (an error estimate of the previous
// level, an upper bound of the final error in the geometric regime) goes to
// *check.  Returns 0 when converged, 1 when the levels ran out first, or the
// HIP error of the first failing runtime call (negated).
int launch_small_sign(int nrhs, int k, TslCoeffs co, const SmallSignCfg& cfg, c64* scratch, c64* c_out,
                      double* check, hipStream_t s, int transpose) {
    const int chunk_solves = cfg.chunk > 0 ? cfg.chunk : kDefaultChunkSolves;
    const int max_levels = cfg.max_levels > 0 ? cfg.max_levels : kDefaultMaxLevels;
    c64* scr = scratch;
    c64* acc = scratch + 4 * (size_t)k * chunk_solves;
    c64* cprev = acc + (size_t)nrhs * k;
    double* smin = (double*)(cprev + (size_t)nrhs * k);
    double* diff = smin + nrhs;
    hipError_t e = hipMemsetAsync(acc, 0, sizeof(c64) * 2 * nrhs * k, s);
    if (e != hipSuccess) return -(int)e;
    small_sign_setup_kernel<<<nrhs, 256, 0, s>>>(nrhs, k, co, smin);
    const double h0 = 2.0 * cfg.quad_step;
    const int Q0 = (int)ceil((kLowSpan + kHighSpan) / h0) + 1;
    const int chunk = chunk_solves / (2 * nrhs) > 0 ? chunk_solves / (2 * nrhs) : 1;
    std::vector<double> hd(nrhs);
    double last = 0.0;
    int rc = 1;
    for (int lev = 0; lev <= max_levels; ++lev) {
        // nodes of this level: level 0 all Q0 nodes at spacing h0; level l >= 1
        // the (Q0 - 1) 2^{l-1} midpoints at spacing h0 / 2^{l-1}
        const double sp = lev == 0 ? h0 : h0 / (double)(1LL << (lev - 1));
        const double off = lev == 0 ? 0.0 : 0.5;
        const long long nql = lev == 0 ? Q0 : (long long)(Q0 - 1) * (1LL << (lev - 1));
        const int nq = (int)nql;
        for (int q0 = 0; q0 < nq; q0 += chunk) {
            const int n = (nq - q0) < chunk ? (nq - q0) : chunk;
            const int nsol = nrhs * 2 * n;
            small_sign_solve_kernel<<<(nsol + 63) / 64, 64, 0, s>>>(nrhs, k, co, smin, sp, off, q0, n, scr, transpose, 1);
            dim3 g((k + 127) / 128, nrhs);
            small_sign_accum_kernel<<<g, 128, 0, s>>>(nrhs, k, n, scr, acc);
        }
        const double hl = h0 / (double)(1LL << lev);
        // the last node is s = smin + (Q0 - 1) h0 = smin + qlast * hl
        const long long qlast = (long long)(Q0 - 1) * (1LL << lev);
        small_sign_finalize_kernel<<<nrhs, 256, 0, s>>>(k, co, smin, hl, qlast, acc, c_out, cprev, diff, transpose);
        if (lev == 0) continue;
        if ((e = hipMemcpyAsync(hd.data(), diff, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return -(int)e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return -(int)e;
        last = 0.0;
        for (double d : hd) last = (d > last || d != d) ? d : last;
        if (last <= kSignTol) {
            rc = 0;
            break;
        }
    }
    if (check) *check = last;
    if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
    return rc;
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
// M = -(h/pi) Msum + tail, elementwise over kFinBlocks blocks; each block's
// largest change against the previous level goes to part[block] (the max over
// blocks, taken by fin_max_kernel, is independent of the order)
constexpr int kFinBlocks = 64;
__global__ __launch_bounds__(256) void frechet_finalize_kernel(int k, TslCoeffs co, const double* __restrict__ smin,
                                                               double h, long long qlast,
                                                               const c64* __restrict__ Msum, c64* __restrict__ Mout,
                                                               c64* __restrict__ Mprev, double* __restrict__ part) {
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
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k * k; t += gridDim.x * blockDim.x) {
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
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void fin_max_kernel(int n, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = part[i] > m ? part[i] : m;
    *out = m;
}

size_t small_frechet_scratch_elems(int k) {
    return 2 * (4 * (size_t)k * kDefaultChunkSolves) + 3 * (size_t)k * k + 4 + kFinBlocks;
}

// M (k x k, row-major) = L_sgn(T, e_1 e_1^T) for one tridiagonal (rhs 0 of co);
// return codes as launch_small_sign
int launch_small_frechet(int k, TslCoeffs co, const SmallSignCfg& cfg, c64* scratch, c64* M_out, double* check,
                         hipStream_t s) {
    const int max_levels = cfg.max_levels > 0 ? cfg.max_levels : kDefaultMaxLevels;
    c64* scrA = scratch;
    c64* scrB = scrA + 4 * (size_t)k * kDefaultChunkSolves;
    c64* Msum = scrB + 4 * (size_t)k * kDefaultChunkSolves;
    c64* Mprev = Msum + (size_t)k * k;
    double* smin = (double*)(Mprev + (size_t)k * k);
    double* diff = smin + 2;
    double* fpart = smin + 8;   // kFinBlocks partial maxima
    hipError_t e = hipMemsetAsync(Msum, 0, sizeof(c64) * 2 * k * k, s);
    if (e != hipSuccess) return -(int)e;
    small_sign_setup_kernel<<<1, 256, 0, s>>>(1, k, co, smin);
    const double h0 = 2.0 * cfg.quad_step;
    const int Q0 = (int)ceil((kLowSpan + kHighSpan) / h0) + 1;
    const int chunk = kDefaultChunkSolves / 2;
    double hd = 0.0, last = 0.0;
    int rc = 1;
    for (int lev = 0; lev <= max_levels; ++lev) {
        const double sp = lev == 0 ? h0 : h0 / (double)(1LL << (lev - 1));
        const double off = lev == 0 ? 0.0 : 0.5;
        const int nq = lev == 0 ? Q0 : (int)((long long)(Q0 - 1) * (1LL << (lev - 1)));
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
        const double hl = h0 / (double)(1LL << lev);
        const long long qlast = (long long)(Q0 - 1) * (1LL << lev);
        frechet_finalize_kernel<<<kFinBlocks, 256, 0, s>>>(k, co, smin, hl, qlast, Msum, M_out, Mprev, fpart);
        fin_max_kernel<<<1, 64, 0, s>>>(kFinBlocks, fpart, diff);
        if (lev == 0) continue;
        if ((e = hipMemcpyAsync(&hd, diff, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return -(int)e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return -(int)e;
        last = hd;
        if (last <= kSignTol) {
            rc = 0;
            break;
        }
    }
    if (check) *check = last;
    if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
    return rc;
}

// ===========================================================================
// Nested two-sided Lanczos for sgn(T_k) e_1 (the paper computes the sign of its
// outer Ritz matrix with one level of nesting and an inner Krylov size of 100,
// Sec. 4; the construction is that of the cited nested Krylov-Ritz method).
//
// A Krylov space of the tridiagonal T_k itself started at e_1 is spanned by
// e_1 .. e_kp and would only reproduce the outer run truncated at kp steps.
// The inner run therefore works on Tt = (T_k + T_k^{-1}) / 2, which has the
// same sign function as T_k (Re(z + 1/z) = Re z (1 + 1/|z|^2)) and whose
// Krylov space holds rational functions of T_k:
//   v_1 = w_1 = e_1;  kp steps of the same two-sided recurrence as the outer
//   run (Tt^dag = (T^dag + T^{-dag}) / 2);  T' the kp x kp Ritz matrix;
//   sgn(T_k) e_1 ~ V' sgn(T') e_1,
// with sgn(T') e_1 from the quadrature above.
//
// One block of 256 threads per right-hand side.  The two solves of a step
// (T^{-1} v and T^{-dag} w) are sequential recurrences; they run at the same
// time on lane 0 of waves 0 and 1, from pivoted LU factors computed once.
// Everything else (tridiagonal products, three-term updates, inner products
// with a fixed summation order) is spread over the block.
// ===========================================================================

// LU factors of a tridiagonal matrix with partial pivoting (rows i and i+1
// exchanged when the subdiagonal entry is larger in modulus): unit lower
// factor with multipliers ml[i], upper factor with diagonal d, superdiagonals
// du, du2; piv[i] = 1 when rows i, i+1 were exchanged.
struct TriLU {
    c64 *d, *du, *du2, *ml;
    int* piv;
};

// a: diagonal (n), up[i] = A[i][i+1], lo[i] = A[i+1][i] (n - 1 each), into f
__device__ void tri_factor(int n, const c64* a_diag, const c64* up, const c64* lo, TriLU f) {
    for (int i = 0; i < n; ++i) {
        f.d[i] = a_diag[i];
        f.du[i] = i + 1 < n ? up[i] : c64{0.0, 0.0};
        f.du2[i] = c64{0.0, 0.0};
    }
    for (int i = 0; i + 1 < n; ++i) {
        const c64 l = lo[i];
        if (cabs1(f.d[i]) >= cabs1(l)) {
            f.piv[i] = 0;
            const c64 m = cabs1(f.d[i]) > 0.0 ? cdiv(l, f.d[i]) : c64{0.0, 0.0};
            f.ml[i] = m;
            f.d[i + 1] = f.d[i + 1] - m * f.du[i];
        } else {
            // rows i, i+1 exchanged: row i = (l, d[i+1], du[i+1]), then eliminate
            f.piv[i] = 1;
            const c64 m = cdiv(f.d[i], l);
            f.ml[i] = m;
            const c64 old_du = f.du[i];
            f.d[i] = l;
            f.du[i] = f.d[i + 1];
            f.d[i + 1] = old_du - m * f.du[i];
            if (i + 2 < n) {
                f.du2[i] = f.du[i + 1];
                f.du[i + 1] = -(m * f.du2[i]);
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (cabs1(f.d[i]) == 0.0) f.d[i] = c64{1e-300, 0.0};
}

// x <- A^{-1} x with the factors of A
__device__ void tri_solve(int n, TriLU f, c64* x) {
    for (int i = 0; i + 1 < n; ++i) {
        if (f.piv[i] == 0) {
            x[i + 1] = x[i + 1] - f.ml[i] * x[i];
        } else {
            const c64 t = x[i];
            x[i] = x[i + 1];
            x[i + 1] = t - f.ml[i] * x[i];
        }
    }
    x[n - 1] = cdiv(x[n - 1], f.d[n - 1]);
    if (n >= 2) x[n - 2] = cdiv(x[n - 2] - f.du[n - 2] * x[n - 1], f.d[n - 2]);
    for (int i = n - 3; i >= 0; --i) x[i] = cdiv(x[i] - f.du[i] * x[i + 1] - f.du2[i] * x[i + 2], f.d[i]);
}

// deterministic block sum of NV doubles (256 threads): fixed shuffle tree in
// each wave, then the four wave sums in order; the result is returned to all
template <int NV>
__device__ void nested_block_sum(double (&v)[NV], double* lds /* [4 * NV + NV] */) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
        v[i] = x;
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int i = 0; i < NV; ++i) lds[w * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) lds[4 * NV + i] = ((lds[i] + lds[NV + i]) + lds[2 * NV + i]) + lds[3 * NV + i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = lds[4 * NV + i];
}

// per-rhs scratch of the inner run (complex elements): 2 x 4k factors, the
// six k-vectors v, v_prev, w, w_prev, u, z, and the inner basis kp x k
__host__ __device__ inline size_t nested_rhs_elems(int k, int kp) { return (size_t)8 * k + 6 * (size_t)k + (size_t)kp * k; }

__global__ __launch_bounds__(256) void nested_tsl_kernel(int k, TslCoeffs co, int kp, double tau,
                                                         c64* __restrict__ scr, int* __restrict__ ipiv,
                                                         TslCoeffs ico, int* __restrict__ flags) {
    __shared__ double lds[64];
    const int r = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    c64* base = scr + (size_t)r * nested_rhs_elems(k, kp);
    TriLU fa{base, base + k, base + 2 * k, base + 3 * k, ipiv + (size_t)r * 2 * k};
    TriLU fh{base + 4 * k, base + 5 * k, base + 6 * k, base + 7 * k, ipiv + (size_t)r * 2 * k + k};
    c64* v = base + 8 * k;
    c64* vp = v + k;
    c64* w = vp + k;
    c64* wp = w + k;
    c64* u = wp + k;
    c64* z = u + k;
    c64* Vb = z + k;      // inner basis, [kp][k]
    const c64* al = co.alpha + (size_t)r * co.kmax;
    const c64* be = co.beta + (size_t)r * co.kmax;    // T[i][i+1] = be[i + 1]
    const c64* de = co.delta + (size_t)r * co.kmax;   // T[i+1][i] = de[i + 1]
    c64* ia = ico.alpha + (size_t)r * ico.kmax;
    c64* ib = ico.beta + (size_t)r * ico.kmax;
    c64* id = ico.delta + (size_t)r * ico.kmax;
    // factors of T (lane 0 of wave 0) and of T^dag (lane 0 of wave 1); the
    // diagonals and off-diagonals are staged through u and z
    for (int i = tid; i < k; i += nt) {
        u[i] = al[i];                               // diagonal of T
        v[i] = i + 1 < k ? be[i + 1] : c64{0.0, 0.0};   // T[i][i+1]
        vp[i] = i + 1 < k ? de[i + 1] : c64{0.0, 0.0};  // T[i+1][i]
        z[i] = conj(al[i]);                         // diagonal of T^dag
        w[i] = i + 1 < k ? conj(de[i + 1]) : c64{0.0, 0.0};   // T^dag[i][i+1] = conj(T[i+1][i])
        wp[i] = i + 1 < k ? conj(be[i + 1]) : c64{0.0, 0.0};  // T^dag[i+1][i] = conj(T[i][i+1])
    }
    __syncthreads();
    if (tid == 0) tri_factor(k, u, v, vp, fa);
    if (tid == 64) tri_factor(k, z, w, wp, fh);
    __syncthreads();
    for (int i = tid; i < k; i += nt) {
        v[i] = c64{i == 0 ? 1.0 : 0.0, 0.0};
        w[i] = v[i];
        vp[i] = c64{0.0, 0.0};
        wp[i] = c64{0.0, 0.0};
    }
    if (tid == 0) {
        ib[0] = c64{0.0, 0.0};
        id[0] = c64{1.0, 0.0};
        flags[r] = -1;
    }
    c64 beta{0.0, 0.0};
    double delta = 0.0;
    for (int j = 0; j < kp; ++j) {
        __syncthreads();
        // the basis vector, and the right-hand sides of the two solves
        for (int i = tid; i < k; i += nt) {
            Vb[(size_t)j * k + i] = v[i];
            u[i] = v[i];
            z[i] = w[i];
        }
        __syncthreads();
        if (tid == 0) tri_solve(k, fa, u);      // u = T^{-1} v
        if (tid == 64) tri_solve(k, fh, z);     // z = T^{-dag} w
        __syncthreads();
        // u = (T v + T^{-1} v) / 2,  z = (T^dag w + T^{-dag} w) / 2,  alpha = w^dag u
        double pa[2] = {0.0, 0.0};
        for (int i = tid; i < k; i += nt) {
            c64 tv = al[i] * v[i];
            c64 tw = conj(al[i]) * w[i];
            if (i > 0) {
                tv += de[i] * v[i - 1];             // T[i][i-1]
                tw += conj(be[i]) * w[i - 1];       // conj(T[i-1][i])
            }
            if (i + 1 < k) {
                tv += be[i + 1] * v[i + 1];         // T[i][i+1]
                tw += conj(de[i + 1]) * w[i + 1];   // conj(T[i+1][i])
            }
            const c64 uu = 0.5 * (tv + u[i]);
            const c64 zz = 0.5 * (tw + z[i]);
            u[i] = uu;
            z[i] = zz;
            const c64 d = cdot(w[i], uu);
            pa[0] += d.re;
            pa[1] += d.im;
        }
        nested_block_sum<2>(pa, lds);
        const c64 alpha{pa[0], pa[1]};
        if (tid == 0) ia[j] = alpha;
        if (j == kp - 1) break;
        // three-term update and omega = what^dag vhat
        double po[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = tid; i < k; i += nt) {
            const c64 vh = u[i] - alpha * v[i] - beta * vp[i];
            const c64 wh = z[i] - conj(alpha) * w[i] - c64{delta, 0.0} * wp[i];
            u[i] = vh;
            z[i] = wh;
            const c64 d = cdot(wh, vh);
            po[0] += d.re;
            po[1] += d.im;
            po[2] += norm2(vh);
            po[3] += norm2(wh);
        }
        nested_block_sum<4>(po, lds);
        const c64 omega{po[0], po[1]};
        const double aom = sqrt(norm2(omega));
        const double margin = aom / sqrt(po[2] * po[3]);
        if (!(margin > tau)) {   // breakdown (or a non-finite value): T' has j + 1 rows
            if (tid == 0) flags[r] = j + 1;
            return;
        }
        const double dn = sqrt(aom);
        const c64 bn = (1.0 / dn) * omega;
        const c64 sw = cdiv(c64{1.0, 0.0}, conj(bn));
        for (int i = tid; i < k; i += nt) {
            vp[i] = v[i];
            wp[i] = w[i];
            v[i] = (1.0 / dn) * u[i];
            w[i] = sw * z[i];
        }
        if (tid == 0) {
            ib[j + 1] = bn;
            id[j + 1] = c64{dn, 0.0};
        }
        // the next update subtracts beta_{j+1} v_j and conj(delta_{j+1}) w_j
        beta = bn;
        delta = dn;
    }
}

// c[r][i] = sum_j Vb[r][j][i] cp[r][j]  (fixed order in j)
__global__ void nested_combine_kernel(int k, int kp, const c64* __restrict__ scr, const c64* __restrict__ cp,
                                      c64* __restrict__ c_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= k) return;
    const c64* Vb = scr + (size_t)r * nested_rhs_elems(k, kp) + (size_t)14 * k;
    c64 a{0.0, 0.0};
    for (int j = 0; j < kp; ++j) a += Vb[(size_t)j * k + i] * cp[(size_t)r * kp + j];
    c_out[(size_t)r * k + i] = a;
}

size_t nested_sign_scratch_elems(int nrhs, int k, int kp, int chunk) {
    return (size_t)nrhs * nested_rhs_elems(k, kp)   // factors, vectors, inner bases
           + (size_t)nrhs * k                      // pivots (2 k ints per rhs)
           + (size_t)5 * nrhs * kp                 // inner alpha, beta, delta, proj, sgn(T') e_1
           + (size_t)nrhs                          // flags
           + small_sign_scratch_elems(nrhs, kp, chunk);
}

int launch_nested_sign(int nrhs, int k, TslCoeffs co, int kp, double tau, const SmallSignCfg& cfg, c64* scratch,
                       c64* c_out, double* check, int* bstep, hipStream_t s) {
    if (kp > k) kp = k;
    c64* scr = scratch;
    int* ipiv = (int*)(scr + (size_t)nrhs * nested_rhs_elems(k, kp));
    c64* ic = scr + (size_t)nrhs * nested_rhs_elems(k, kp) + (size_t)nrhs * k;
    TslCoeffs ico{ic, ic + (size_t)nrhs * kp, ic + (size_t)2 * nrhs * kp, ic + (size_t)3 * nrhs * kp, kp};
    c64* cp = ic + (size_t)4 * nrhs * kp;
    int* flags = (int*)(cp + (size_t)nrhs * kp);
    c64* sscr = (c64*)(flags) + nrhs;
    hipError_t e = hipMemsetAsync(ic, 0, sizeof(c64) * 4 * nrhs * kp, s);
    if (e != hipSuccess) return -(int)e;
    nested_tsl_kernel<<<nrhs, 256, 0, s>>>(k, co, kp, tau, scr, ipiv, ico, flags);
    std::vector<int> hf(nrhs);
    if ((e = hipMemcpyAsync(hf.data(), flags, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return -(int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return -(int)e;
    for (int r = 0; r < nrhs; ++r)
        if (hf[r] >= 0) {
            if (bstep) *bstep = hf[r];
            return 2;
        }
    const int rc = launch_small_sign(nrhs, kp, ico, cfg, sscr, cp, check, s, 0);
    if (rc < 0) return rc;
    dim3 g((k + 127) / 128, nrhs);
    nested_combine_kernel<<<g, 128, 0, s>>>(k, kp, scr, cp, c_out);
    if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
    return rc;
}

// ===========================================================================
// Coefficients of the deflated gradient of <x|sgn(H)|b> (Sec. 3 deflation of
// the bilinear two-sided Lanczos run with right start b' = (1 - P) b and left
// start x' = (1 - P)^dag x).  With g_j(z) = (sgn z - s_j)/(z - lam_j):
//   A[p][j] = delta_0 conj(d_j) [g_j(T) e_1]_p / delta_p      (the vectors
//             |b'| (x^dag R_j) g_j(H) b' in the stored right basis),
//   B[q][i] = conj(c_i beta_0 [g_i(T)^T e_1]_q / beta_q)      (the vectors
//             conj((L_i^dag b)(x'^dag v_1)) W conj(g_i(T)^T e_1) in the left basis),
// c_i = L_i^dag b, d_i = R_i^dag x; g_j(T) e_1 = (T - lam_j)^{-1} (sgn(T) e_1 - s_j e_1)
// and g_i(T)^T e_1 = (T - lam_i)^{-T} (sgn(T)^T e_1 - s_i e_1), one pivoted
// tridiagonal solve per thread.
// ===========================================================================
__global__ void defl_vjp_coef_kernel(int k, TslCoeffs co, int m, const c64* __restrict__ lam,
                                     const double* __restrict__ sg, const c64* __restrict__ scol,
                                     const c64* __restrict__ srow, const c64* __restrict__ cv,
                                     const c64* __restrict__ dv, c64* __restrict__ A, c64* __restrict__ B,
                                     c64* __restrict__ scr, int* __restrict__ ipiv) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * m) return;
    const int side = t / m, j = t % m;
    c64* base = scr + (size_t)t * 8 * k;
    TriLU f{base, base + k, base + 2 * k, base + 3 * k, ipiv + (size_t)t * k};
    c64* dg = base + 4 * k;      // diagonal, upper, lower of T - lam_j (or of its transpose)
    c64* up = base + 5 * k;
    c64* lo = base + 6 * k;
    c64* x = base + 7 * k;
    for (int i = 0; i < k; ++i) {
        dg[i] = co.alpha[i] - lam[j];
        const c64 bu = i + 1 < k ? co.beta[i + 1] : c64{0.0, 0.0};    // T[i][i+1]
        const c64 dl = i + 1 < k ? co.delta[i + 1] : c64{0.0, 0.0};   // T[i+1][i]
        up[i] = side == 0 ? bu : dl;
        lo[i] = side == 0 ? dl : bu;
        x[i] = (side == 0 ? scol[i] : srow[i]) - c64{i == 0 ? sg[j] : 0.0, 0.0};
    }
    tri_factor(k, dg, up, lo, f);
    tri_solve(k, f, x);
    const c64 b0 = co.beta[0];
    const double d0 = co.delta[0].re;
    for (int p = 0; p < k; ++p) {
        if (side == 0) {
            A[(size_t)p * m + j] = cdiv((d0 * conj(dv[j])) * x[p], co.delta[p]);
        } else {
            B[(size_t)p * m + j] = conj(cdiv(cv[j] * b0 * x[p], co.beta[p]));
        }
    }
}

// Cm[j][i] = conj(f_ij c_i) d_j, f_ij = (s_i - s_j) / (lam_i - lam_j) (0 when s_i = s_j)
__global__ void defl_vjp_dd_kernel(int m, const c64* __restrict__ lam, const double* __restrict__ sg,
                                   const c64* __restrict__ cv, const c64* __restrict__ dv, c64* __restrict__ Cm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * m) return;
    const int j = t / m, i = t % m;
    c64 v{0.0, 0.0};
    if (sg[i] != sg[j]) {
        const c64 fij = cdiv(c64{sg[i] - sg[j], 0.0}, lam[i] - lam[j]);
        v = conj(fij * cv[i]) * dv[j];
    }
    Cm[t] = v;
}

size_t defl_vjp_coef_scratch(int k, int m) { return (size_t)2 * m * 8 * k + (size_t)m * k; }

void launch_defl_vjp_coef(int k, TslCoeffs co, int m, const c64* lam, const double* sg, const c64* scol,
                          const c64* srow, const c64* cv, const c64* dv, c64* A, c64* B, c64* Cm, c64* scratch,
                          hipStream_t s) {
    int* ipiv = (int*)(scratch + (size_t)2 * m * 8 * k);
    defl_vjp_coef_kernel<<<(2 * m + 63) / 64, 64, 0, s>>>(k, co, m, lam, sg, scol, srow, cv, dv, A, B, scratch, ipiv);
    defl_vjp_dd_kernel<<<(m * m + 255) / 256, 256, 0, s>>>(m, lam, sg, cv, dv, Cm);
}

}  // namespace ovd
