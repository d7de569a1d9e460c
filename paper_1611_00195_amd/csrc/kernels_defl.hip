// Deflation projections (Sec. 3, eq. 8 and eq. 10-11) as tall-skinny complex
// FP64 GEMMs on the MFMA units of gfx950.
//
// The deflation vectors R_i, L_i, dR_i, dL_i are long (12 V complex) and few
// (m <= a few hundred); the sources are few too (nrhs).  The two products are
//   projection:   C = A^dag B          (m x nrhs, a reduction over 12 V)
//   combination:  Y = Y + s A C        (12 V x nrhs, a sum over m)
// with A the deflation vectors and B / Y the sources.  Both are bound by
// reading A from HBM; the matrix cores do the arithmetic in 16 x 16 tiles
// (V_MFMA_F64_16X16X4_F64), complex products as four real ones:
//   conj(a)^T b:  re = ar^T br + ai^T bi,   im = ar^T bi - ai^T br
//   a c:          re = ar cr - ai ci,        im = ar ci + ai cr.
// Operand layout of the 16x16x4 FP64 instruction (lane l of the wave):
//   A operand: row l % 16, k = l / 16;  B operand: k = l / 16, column l % 16;
//   result register v (v = 0..3): row 4 v + l / 16, column l % 16
// (checked on gfx950 with a one-wave probe of known operands).
// Fields are the FP64 internal layout [12][Vp] (flattened to 12 Vp complex,
// padding sites zero), so a field is a plain complex vector of length
// nf = 12 Vp here.
#include "ovd_internal.h"

namespace ovd {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// projection C = A^dag B, split over the reduction index.
// grid: (ceil(m/16), ceil(nr/16), nsplit), one wave per block.  The partial
// tile of split z goes to part[z][i][r]; defl_proj_reduce sums the splits in
// order.  A column i lives at A + i sA, B column r at B + r sB.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void defl_proj_kernel(const c64* __restrict__ A, long long sA, int m,
                                                       const c64* __restrict__ B, long long sB, int nr,
                                                       long long nf, long long chunk, c64* __restrict__ part) {
    const int l = threadIdx.x;
    const int i0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
    const int z = blockIdx.z;
    const long long k0 = (long long)z * chunk;
    long long k1 = k0 + chunk;
    if (k1 > nf) k1 = nf;
    const int ia = i0 + (l & 15);   // A row (vector index) of this lane
    const int rb = r0 + (l & 15);   // B column (rhs index) of this lane
    const int kk = l >> 4;
    const bool va = ia < m, vb = rb < nr;
    const c64* Ap = A + (va ? ia : 0) * sA;
    const c64* Bp = B + (vb ? rb : 0) * sB;
    v4d cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    // groups of 8 steps: the 16 loads of a group are issued before its first
    // product, so a wave has them in flight together instead of waiting on one
    // load per step; the products run in the same order as in the tail loop
    // (an invalid row or column loads row 0 and uses zero)
    long long k = k0;
    const long long kg = k0 + (k1 - k0) / 32 * 32;
    for (; k < kg; k += 32) {
        c64 a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = Ap[k + 4 * u + kk];
            b[u] = Bp[k + 4 * u + kk];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const c64 au = va ? a[u] : c64{0.0, 0.0};
            const c64 bu = vb ? b[u] : c64{0.0, 0.0};
            cre = mfma(au.re, bu.re, cre);
            cre = mfma(au.im, bu.im, cre);
            cim = mfma(au.re, bu.im, cim);
            cim = mfma(-au.im, bu.re, cim);
        }
    }
    for (; k < k1; k += 4) {
        const long long kl = k + kk;
        c64 a{0.0, 0.0}, b{0.0, 0.0};
        if (va && kl < k1) a = Ap[kl];
        if (vb && kl < k1) b = Bp[kl];
        cre = mfma(a.re, b.re, cre);
        cre = mfma(a.im, b.im, cre);
        cim = mfma(a.re, b.im, cim);
        cim = mfma(-a.im, b.re, cim);
    }
    // result register v: row (vector i) 4 v + l/16, column (rhs) l % 16
    const int rr = r0 + (l & 15);
    for (int v = 0; v < 4; ++v) {
        const int ii = i0 + 4 * v + (l >> 4);
        if (ii < m && rr < nr) part[((size_t)z * m + ii) * nr + rr] = c64{cre[v], cim[v]};
    }
}

// one block per output: each thread sums a strided subset of the splits, then
// a tree over the block (fixed order, so the result is deterministic)
__global__ __launch_bounds__(256) void defl_proj_reduce(int m, int nr, int nsplit, const c64* __restrict__ part,
                                                        c64* __restrict__ C) {
    __shared__ double re[256], im[256];
    const int t = blockIdx.x;
    c64 s{0.0, 0.0};
    for (int z = threadIdx.x; z < nsplit; z += blockDim.x) s += part[(size_t)z * m * nr + t];
    re[threadIdx.x] = s.re;
    im[threadIdx.x] = s.im;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            re[threadIdx.x] += re[threadIdx.x + w];
            im[threadIdx.x] += im[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) C[t] = c64{re[0], im[0]};
}

// reduction index split into chunks of this many elements (a multiple of 4):
// short enough that a single-vector projection (a Krylov or CG inner product)
// still runs many independent waves
constexpr long long kProjChunk = 256;

size_t defl_proj_scratch(int m, int nr, long long nf, long long chunk) {
    if (chunk <= 0) chunk = kProjChunk;
    const long long nsplit = (nf + chunk - 1) / chunk;
    return (size_t)nsplit * m * nr;
}

void launch_defl_proj(const c64* A, long long sA, int m, const c64* B, long long sB, int nr, long long nf,
                      c64* C, c64* scratch, hipStream_t s, long long chunk) {
    if (m <= 0 || nr <= 0) return;
    if (chunk <= 0) chunk = kProjChunk;
    const int nsplit = (int)((nf + chunk - 1) / chunk);
    dim3 grid((m + 15) / 16, (nr + 15) / 16, nsplit);
    defl_proj_kernel<<<grid, 64, 0, s>>>(A, sA, m, B, sB, nr, nf, chunk, scratch);
    defl_proj_reduce<<<m * nr, 256, 0, s>>>(m, nr, nsplit, scratch, C);
}

// ---------------------------------------------------------------------------
// combination Y[:, r] += sum_i A[:, i] C[i][r] (C given as [m][nr], already
// scaled by the caller).  grid: (ceil(nf/16), ceil(nr/16)), one wave per block;
// the reduction over i runs in steps of 4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void defl_comb_kernel(const c64* __restrict__ A, long long sA, int m,
                                                       const c64* __restrict__ C, int nr,
                                                       c64* __restrict__ Y, long long sY, long long nf,
                                                       const c64* __restrict__ Y0, long long sY0) {
    const int l = threadIdx.x;
    const long long n0 = (long long)blockIdx.x * 16;
    const int r0 = blockIdx.y * 16;
    const long long na = n0 + (l & 15);   // A row (element index) of this lane
    const int rb = r0 + (l & 15);         // C column (rhs) of this lane
    const int kk = l >> 4;
    v4d yre = {0, 0, 0, 0}, yim = {0, 0, 0, 0};
    for (int i = 0; i < m; i += 4) {
        const int ik = i + kk;
        c64 a{0.0, 0.0}, c{0.0, 0.0};
        if (ik < m && na < nf) a = A[(size_t)ik * sA + na];
        if (ik < m && rb < nr) c = C[(size_t)ik * nr + rb];
        yre = mfma(a.re, c.re, yre);
        yre = mfma(-a.im, c.im, yre);
        yim = mfma(a.re, c.im, yim);
        yim = mfma(a.im, c.re, yim);
    }
    const int rr = r0 + (l & 15);
    if (rr >= nr) return;
    for (int v = 0; v < 4; ++v) {
        const long long nn = n0 + 4 * v + (l >> 4);
        if (nn < nf) {
            c64* y = Y + (size_t)rr * sY + nn;
            const c64 y0 = Y0 ? Y0[(size_t)rr * sY0 + nn] : *y;
            *y = y0 + c64{yre[v], yim[v]};
        }
    }
}

void launch_defl_comb(const c64* A, long long sA, int m, const c64* C, int nr, c64* Y, long long sY, long long nf,
                      hipStream_t s, const c64* Y0, long long sY0) {
    dim3 grid((unsigned)((nf + 15) / 16), (nr + 15) / 16);
    defl_comb_kernel<<<grid, 64, 0, s>>>(A, sA, m, C, nr, Y, sY, nf, Y0, sY0);
}

// out[i][r] = sign * f[i] * in[i][r]
__global__ void defl_scale_kernel(int m, int nr, const double* __restrict__ f, const c64* __restrict__ in,
                                  c64* __restrict__ out, double sign) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * nr) return;
    out[t] = (sign * f[t / nr]) * in[t];
}

void launch_defl_scale(int m, int nr, const double* f, const c64* in, c64* out, double sign, hipStream_t s) {
    defl_scale_kernel<<<(m * nr + 255) / 256, 256, 0, s>>>(m, nr, f, in, out, sign);
}

// xdy[r] += sum_i conj(P1[i][r]) sD[i][r] + conj(P2[i][r]) sC[i][r]   (one thread per rhs, fixed order)
__global__ void defl_scalar_kernel(int l, int nr, const c64* __restrict__ P1, const c64* __restrict__ sD,
                                   const c64* __restrict__ P2, const c64* __restrict__ sC, c64* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    c64 s{0.0, 0.0};
    for (int i = 0; i < l; ++i) {
        s += cdot(P1[(size_t)i * nr + r], sD[(size_t)i * nr + r]);
        s += cdot(P2[(size_t)i * nr + r], sC[(size_t)i * nr + r]);
    }
    out[r] = out[r] + s;
}

void launch_defl_scalar(int l, int nr, const c64* P1, const c64* sD, const c64* P2, const c64* sC, c64* out,
                        hipStream_t s) {
    defl_scalar_kernel<<<(nr + 63) / 64, 64, 0, s>>>(l, nr, P1, sD, P2, sC, out);
}

// AoS complex128 output [n][V][12] += SoA FP64 field(s) [n][12][Vp]
__global__ void add_soa_to_aos_kernel(Geom g, const c64* __restrict__ in, long long stride, c64* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
    const c64* src = in + r * stride;
    c64* dst = out + ((size_t)r * g.V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = dst[c] + src[(size_t)c * g.Vp + s];
}

void launch_add_soa_to_aos(const Geom& g, int n, const c64* in, long long stride, void* out_aos, hipStream_t s) {
    dim3 grid((g.V + 255) / 256, n);
    add_soa_to_aos_kernel<<<grid, 256, 0, s>>>(g, in, stride, (c64*)out_aos);
}

// FP64 SoA -> T SoA (same layout semantics, fidx<T>), n fields with strides
template <typename T>
__global__ void convert_field_kernel(Geom g, const c64* __restrict__ in, long long sin, cpx<T>* __restrict__ out,
                                     long long sout) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
#pragma unroll
    for (int c = 0; c < 12; ++c)
        out[r * sout + fidx<T>(c, s, g.Vp)] = cast<T>(in[r * sin + (size_t)c * g.Vp + s]);
}

template <typename T>
void launch_convert_field(const Geom& g, int n, const c64* in, long long sin, cpx<T>* out, long long sout,
                          hipStream_t s) {
    dim3 grid((g.V + 255) / 256, n);
    convert_field_kernel<T><<<grid, 256, 0, s>>>(g, in, sin, out, sout);
}
template void launch_convert_field<double>(const Geom&, int, const c64*, long long, c64*, long long, hipStream_t);
template void launch_convert_field<float>(const Geom&, int, const c64*, long long, c32*, long long, hipStream_t);

// FP32 internal layout -> FP64 internal layout (padding sites zero)
__global__ void widen_field_kernel(Geom g, const c32* __restrict__ in, long long sin, c64* __restrict__ out,
                                   long long sout) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.Vp) return;
#pragma unroll
    for (int c = 0; c < 12; ++c)
        out[r * sout + (size_t)c * g.Vp + s] = s < g.V ? cast<double>(in[r * sin + fidx<float>(c, s, g.Vp)]) : c64{0.0, 0.0};
}

void launch_widen_field(const Geom& g, int n, const c32* in, long long sin, c64* out, long long sout, hipStream_t s) {
    dim3 grid((g.Vp + 255) / 256, n);
    widen_field_kernel<<<grid, 256, 0, s>>>(g, in, sin, out, sout);
}

}  // namespace ovd

namespace ovd {

// ---------------------------------------------------------------------------
// out = conj(in), n complex: conj(M') for the gradient's product Z = W M'^dag,
// which runs as the plain library GEMM Z = W conj(M'^T) (rocblas_zgemm, in
// api.hip)
__global__ void conj_c64_kernel(long long n, const c64* __restrict__ in, c64* __restrict__ out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) out[e] = conj(in[e]);
}

void launch_conj_c64(long long n, const c64* in, c64* out, hipStream_t s) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    conj_c64_kernel<<<(unsigned)nb, 256, 0, s>>>(n, in, out);
}

// M'[p][q] = xb M[p][q] / (delta_p beta_q), xb = beta_0 delta_0 = x^dag b
__global__ void vjp_scale_m_kernel(int k, TslCoeffs co, const c64* __restrict__ M, c64* __restrict__ Mp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k * k) return;
    const int p = t / k, q = t % k;
    const c64 xb = co.beta[0] * co.delta[0];
    const c64 den = co.delta[p] * co.beta[q];
    Mp[t] = cdiv(xb * M[t], den);
}

void launch_vjp_scale_m(int k, TslCoeffs co, const c64* M, c64* Mp, hipStream_t s) {
    vjp_scale_m_kernel<<<(k * k + 255) / 256, 256, 0, s>>>(k, co, M, Mp);
}

}  // namespace ovd
