// Layout conversion, reconstruction of the Krylov-Ritz result and the
// storage-free scalar, for libovderiv on gfx950.  All kernels are
// bandwidth-bound element-wise passes.
#include "ovd_internal.h"

namespace ovd {

// links: AoS complex128 [4][V][3][3] -> SoA [4][9][Vp] in FP64 and (optionally) FP32
__global__ void pack_links_kernel(Geom g, const c64* __restrict__ in, c64* __restrict__ o64,
                                  c32* __restrict__ o32) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int nu = blockIdx.y;
    if (s >= g.V) return;
    const c64* src = in + ((size_t)nu * g.V + s) * 9;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const c64 u = src[i];
        if (o64) o64[lidx<double>(nu, i, s, g.Vp)] = u;
        if (o32) o32[lidx<float>(nu, i, s, g.Vp)] = cast<float>(u);
    }
    if (o32) o32[lidx<float>(nu, 9, s, g.Vp)] = c32{0.f, 0.f};
}

void launch_pack_links(const Geom& g, const void* U_aos, c64* U64, c32* U32, hipStream_t s) {
    dim3 grid((g.V + 255) / 256, 4);
    pack_links_kernel<<<grid, 256, 0, s>>>(g, (const c64*)U_aos, U64, U32);
}

template <typename T>
__global__ void pack_spinor_kernel(Geom g, const c64* __restrict__ in, cpx<T>* __restrict__ out,
                                   long long stride) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
    const c64* src = in + ((size_t)r * g.V + s) * 12;
    cpx<T>* dst = out + r * stride;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx<T>(c, s, g.Vp)] = cast<T>(src[c]);
}

template <typename T>
__global__ void unpack_spinor_kernel(Geom g, const cpx<T>* __restrict__ in, long long stride,
                                     c64* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
    const cpx<T>* src = in + r * stride;
    c64* dst = out + ((size_t)r * g.V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = cast<double>(src[fidx<T>(c, s, g.Vp)]);
}

template <typename T>
void launch_pack_spinor(const Geom& g, int n, const void* in_aos, cpx<T>* out, long long stride, hipStream_t s) {
    dim3 grid((g.V + 255) / 256, n);
    pack_spinor_kernel<T><<<grid, 256, 0, s>>>(g, (const c64*)in_aos, out, stride);
}
template <typename T>
void launch_unpack_spinor(const Geom& g, int n, const cpx<T>* in, long long stride, void* out_aos, hipStream_t s) {
    dim3 grid((g.V + 255) / 256, n);
    unpack_spinor_kernel<T><<<grid, 256, 0, s>>>(g, in, stride, (c64*)out_aos);
}
template void launch_pack_spinor<double>(const Geom&, int, const void*, c64*, long long, hipStream_t);
template void launch_pack_spinor<float>(const Geom&, int, const void*, c32*, long long, hipStream_t);
template void launch_unpack_spinor<double>(const Geom&, int, const c64*, long long, void*, hipStream_t);
template void launch_unpack_spinor<float>(const Geom&, int, const c32*, long long, void*, hipStream_t);

// ---------------------------------------------------------------------------
// y[rhs] = sum_j coef_j basis[rhs][j] (one half of a block vector, or a plain
// spinor field), written as AoS complex128.  coef_j = |psi| c_j / delta_j
// turns the unnormalised stored vectors into |psi| V_k c.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void reconstruct_kernel(Geom g, int k, const cpx<T>* __restrict__ basis, long long s_rhs,
                                   long long s_j, int half, const c64* __restrict__ coef, int coef_ld,
                                   c64* __restrict__ out, int accumulate) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
    const cpx<T>* B = basis + r * s_rhs + (size_t)half * 12 * g.Vp;
    const c64* cf = coef + (size_t)r * coef_ld;
    c64 acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0.0, 0.0};
    for (int j = 0; j < k; ++j) {
        const c64 w = cf[j];
        const cpx<T>* Bj = B + j * s_j;
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] += w * cast<double>(Bj[fidx<T>(c, s, g.Vp)]);
    }
    c64* dst = out + ((size_t)r * g.V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = accumulate ? dst[c] + acc[c] : acc[c];
}

template <typename T>
void launch_reconstruct(const Geom& g, int nrhs, int k, const cpx<T>* basis, long long s_rhs,
                        long long s_j, int half, const c64* coef, int coef_ld, void* out_aos,
                        hipStream_t s, bool accumulate) {
    dim3 grid((g.V + 255) / 256, nrhs);
    reconstruct_kernel<T><<<grid, 256, 0, s>>>(g, k, basis, s_rhs, s_j, half, coef, coef_ld, (c64*)out_aos,
                                               accumulate ? 1 : 0);
}
template void launch_reconstruct<double>(const Geom&, int, int, const c64*, long long, long long, int,
                                         const c64*, int, void*, hipStream_t, bool);
template void launch_reconstruct<float>(const Geom&, int, int, const c32*, long long, long long, int,
                                        const c64*, int, void*, hipStream_t, bool);

// out[rhs] = scale[rhs] * sum_j c[rhs][j] proj[rhs][j], one block per rhs,
// fixed summation order
__global__ void scalar_dot_kernel(int k, const c64* __restrict__ c, const c64* __restrict__ proj, int ld,
                                  const c64* __restrict__ scale, c64* __restrict__ out) {
    __shared__ double re[256], im[256];
    const int r = blockIdx.x;
    c64 acc{0.0, 0.0};
    for (int j = threadIdx.x; j < k; j += blockDim.x) acc += c[(size_t)r * k + j] * proj[(size_t)r * ld + j];
    re[threadIdx.x] = acc.re;
    im[threadIdx.x] = acc.im;
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
        if (threadIdx.x < m) {
            re[threadIdx.x] += re[threadIdx.x + m];
            im[threadIdx.x] += im[threadIdx.x + m];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = scale[(size_t)r * ld] * c64{re[0], im[0]};
}

void launch_scalar_dot(int nrhs, int k, const c64* c, const c64* proj, int ld, const c64* scale, c64* out,
                       hipStream_t s) {
    scalar_dot_kernel<<<nrhs, 256, 0, s>>>(k, c, proj, ld, scale, out);
}

// AoS complex128 [n][V][4][3]: out = cb b + cy gamma5 y  (gamma5 = diag(1, 1, -1, -1) on the spin)
__global__ void gamma5_axpy_kernel(long long n_sites, double cb, const c64* __restrict__ b, double cy,
                                   const c64* __restrict__ y, c64* __restrict__ out) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_sites * 12) return;
    const int spin = (int)((t % 12) / 3);
    const double g = spin < 2 ? cy : -cy;
    c64 r = g * y[t];
    if (b) r += cb * b[t];
    out[t] = r;
}

void launch_gamma5_axpy(long long n_sites, double cb, const void* b, double cy, const void* y, void* out,
                        hipStream_t s) {
    const long long n = n_sites * 12;
    gamma5_axpy_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n_sites, cb, (const c64*)b, cy, (const c64*)y,
                                                                   (c64*)out);
}

// per field: out[r] = sqrt(|top[r]|^2 + |a[r] - b[r]|^2) / (2 |b[r]|)  (AoS complex128, m
// elements each, top nullable: the block vector (top; a) against (0; b)); one block per field
__global__ void half_rel_diff_kernel(long long m, const c64* __restrict__ top, const c64* __restrict__ a,
                                     const c64* __restrict__ b, double* __restrict__ out) {
    __shared__ double sd[256], sb[256];
    const c64* A = a + (size_t)blockIdx.x * m;
    const c64* B = b + (size_t)blockIdx.x * m;
    double d = 0.0, n = 0.0;
    for (long long i = threadIdx.x; i < m; i += blockDim.x) {
        d += norm2(A[i] - B[i]);
        n += norm2(B[i]);
    }
    if (top) {
        const c64* Tp = top + (size_t)blockIdx.x * m;
        for (long long i = threadIdx.x; i < m; i += blockDim.x) d += norm2(Tp[i]);
    }
    sd[threadIdx.x] = d;
    sb[threadIdx.x] = n;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            sd[threadIdx.x] += sd[threadIdx.x + k];
            sb[threadIdx.x] += sb[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(sd[0]) / (2.0 * sqrt(sb[0]));
}

void launch_half_rel_diff(int n, long long m, const void* a, const void* b, double* out, hipStream_t s,
                          const void* top) {
    half_rel_diff_kernel<<<n, 256, 0, s>>>(m, (const c64*)top, (const c64*)a, (const c64*)b, out);
}

// flag |= 1 when two arrays of n complex differ anywhere (bit for bit)
__global__ void field_differs_kernel(long long n, const c64* __restrict__ a, const c64* __restrict__ b,
                                     unsigned* __restrict__ flag) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool diff = false;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const c64 x = a[i], y = b[i];
        diff |= (x.re != y.re) || (x.im != y.im);
    }
    if (__any(diff) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

void launch_field_differs(long long n, const c64* a, const c64* b, unsigned* flag, hipStream_t s) {
    long long nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    field_differs_kernel<<<(unsigned)nb, 256, 0, s>>>(n, a, b, flag);
}

}  // namespace ovd
