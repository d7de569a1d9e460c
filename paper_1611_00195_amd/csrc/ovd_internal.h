// Internal declarations of libovderiv: device complex arithmetic, the
// lattice geometry passed to kernels, and the host-side launchers that the
// C ABI in api.hip calls.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

namespace ovd {

// ---------------------------------------------------------------------------
// complex numbers (interleaved re, im; 16-byte aligned in FP64, 8 in FP32)
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T> __host__ __device__ inline cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <typename T> __host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cpx<T>& operator+=(cpx<T>& a, cpx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T> __host__ __device__ inline cpx<T>& operator-=(cpx<T>& a, cpx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T> __host__ __device__ inline cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ inline T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
template <typename T> __host__ __device__ inline cpx<T> cdot(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a / b, scaled to avoid overflow (Smith's algorithm)
template <typename T> __host__ __device__ inline cpx<T> cdiv(cpx<T> a, cpx<T> b) {
    T ar = b.re < 0 ? -b.re : b.re, ai = b.im < 0 ? -b.im : b.im;
    if (ar >= ai) {
        T r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        T r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
template <typename T> __host__ __device__ inline T cabs1(cpx<T> a) {
    return (a.re < 0 ? -a.re : a.re) + (a.im < 0 ? -a.im : a.im);
}
template <typename D, typename S> __host__ __device__ inline cpx<D> cast(cpx<S> a) {
    return {static_cast<D>(a.re), static_cast<D>(a.im)};
}

using c64 = cpx<double>;
using c32 = cpx<float>;

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];     // Lx, Ly, Lz, Lt
    int V;        // sites
    int Vp;       // padded site stride of the internal field layout (multiple of 64)
    int bc_t;     // +1 periodic, -1 antiperiodic time boundary
};

// Internal field layout: component-major so that a wave reads 64 consecutive
// sites of one component at once, and every lane loads 16 bytes:
//   FP64: spinor [12][Vp] complex, links [4][9][Vp] complex;
//   FP32: spinor [6][Vp][2] complex (components 2q, 2q+1 side by side),
//         links [4][5][Vp][2] complex (entries 2q, 2q+1; entry 9 is zero padding).
// A block vector (top, bottom) is two spinor fields; right-hand sides are
// stacked with an explicit stride.  Both layouts hold 12 Vp complex per field.
template <typename T> __host__ __device__ inline size_t fidx(int c, int s, int Vp);
template <> __host__ __device__ inline size_t fidx<double>(int c, int s, int Vp) { return (size_t)c * Vp + s; }
template <> __host__ __device__ inline size_t fidx<float>(int c, int s, int Vp) {
    return ((size_t)(c >> 1) * Vp + s) * 2 + (c & 1);
}
template <typename T> __host__ __device__ inline size_t lidx(int nu, int i, int s, int Vp);
template <> __host__ __device__ inline size_t lidx<double>(int nu, int i, int s, int Vp) {
    return ((size_t)nu * 9 + i) * Vp + s;
}
template <> __host__ __device__ inline size_t lidx<float>(int nu, int i, int s, int Vp) {
    return ((size_t)nu * 5 + (i >> 1)) * Vp * 2 + (size_t)s * 2 + (i & 1);
}
// complex elements of one link field
template <typename T> inline size_t link_elems(int Vp) { return sizeof(T) == 8 ? (size_t)36 * Vp : (size_t)40 * Vp; }

// Per-right-hand-side scalar state of the Lanczos recurrence, FP64.
struct TslState {
    c64 av, bv, cv;       // next vhat = av*X + bv*Y + cv*Z   (v side)
    c64 aw, bw, cw;       // next what = aw*X + bw*Y + cw*Z   (w side)
    c64 beta_prev;        // beta_j of the last completed step
    double delta_prev;    // delta_j
    double min_margin;    // min |omega| / (|v||w|)
    double emu, emu_inv;  // e^{mu}, e^{-mu}
    int step;             // number of completed reductions
    int flag;             // 0 ok, 1 breakdown, 2 non-finite
    int bstep;            // step of the breakdown
    int pad;
};

// Per-step coefficient arrays, [rhs][kmax] complex each.
struct TslCoeffs {
    c64* alpha;
    c64* beta;
    c64* delta;   // real, stored complex for uniformity
    c64* proj;    // <x|v_j> (normalised v_j); only for the scalar mode
    int kmax;
};

// Kernel arguments of one fused Lanczos step.
struct StepPtrs {
    const void* Xv; const void* Yv; const void* Zv;   // v side inputs
    const void* Xw; const void* Yw; const void* Zw;   // w side inputs
    void* outV; void* outU;                          // vhat, A vhat
    void* outW; void* outZ;                          // what, A^dag what
    const void* xproj;                               // projection vector or null
    long long sXv, sYv, sZv, sXw, sYw, sZw, sV, sU, sW, sZ, sx;   // rhs strides (elements)
};

// ---------------------------------------------------------------------------
// launchers (kernels_*.hip)
// ---------------------------------------------------------------------------
// links: AoS complex128 [4][V][3][3] -> SoA [4][9][Vp] (double and/or float)
void launch_pack_links(const Geom& g, const void* U_aos, c64* U64, c32* U32, hipStream_t s);
// spinors: AoS complex128 [n][V][12] <-> SoA [n][12][Vp] (stride per rhs)
template <typename T>
void launch_pack_spinor(const Geom& g, int n, const void* in_aos, cpx<T>* out, long long stride, hipStream_t s);
template <typename T>
void launch_unpack_spinor(const Geom& g, int n, const cpx<T>* in, long long stride, void* out_aos, hipStream_t s);

// launch shape of the stencil kernels: XCD work order (0: nrhs/8 sources per
// XCD over the whole lattice, needs nrhs % 8 == 0; 1: contiguous site-group
// ranges per XCD, rhs innermost; < 0: default) and site groups per block
// (apply_op: 2 or 4; Lanczos stencil DIR 0: 2 or 4, DIR 1/2: 1 or 2, and 8 for one
// block per xy-plane with the plane in LDS when 128 <= Lx Ly <= 256; <= 0: default)
struct StencilVariant {
    int map = -1;
    int gpb = 0;
    int seq = 0;   // 1: the two outputs of a pair one after the other (DIR 0/1, not the plane shape);
                   // 2: split, the two outputs of a site in two waves (DIR 0, 1 or 2 groups per block);
                   // 3: time-marching (DIR 1, plane shape applies; gpb = number of time segments)
    int rp = 1;    // Dw.v (H, Dw): right-hand sides per thread, 1 or 2 (2 needs an even count)
};
inline int default_map(int nrhs) { return (nrhs >= 16 && nrhs % 8 == 0) ? 0 : 1; }

// standalone operator: out = op(in) on SoA fields, per-rhs mu
template <typename T>
void launch_apply_op(const Geom& g, int op, int nrhs, const double* d_emu, const cpx<T>* U,
                     const cpx<T>* dU, double m_diag, const cpx<T>* in, cpx<T>* out, hipStream_t s,
                     StencilVariant v = StencilVariant{});

// Lanczos step part 1: vhat/what = a X + b Y (+ c Z) element-wise on both
// sides (nterms 2 or 3), fsz elements per rhs and side.
template <typename T>
void launch_tsl_update(int nrhs, int nterms, long long fsz, const StepPtrs& p, const TslState* st,
                       hipStream_t s);
// Lanczos step part 2: stencil on outV/outW into outU/outZ plus the step's
// reductions and scalar recurrence.  dir: 0 plain H, 1 block d/dmu, 2 block d/dlink.
// blocks per right-hand side of the stencil kernel (size of its partial sums)
int tsl_stencil_blocks(const Geom& g, int dir, int gpb = 0);
// the plane-in-LDS launch shape (gpb 8) applies: 128 <= Lx Ly <= 256
bool tsl_plane_ok(const Geom& g);
// the time-marching form (seq 3, d/dmu only) applies at this precision
// (bytes per real): the plane shape applies and two planes of both input
// fields fit the LDS
bool tsl_march_ok(const Geom& g, int real_bytes);
// blocks per right-hand side of the time-marching form with nseg time segments
int tsl_march_blocks(const Geom& g, int nseg);
template <typename T>
void launch_tsl_stencil(const Geom& g, int dir, int nrhs, const StepPtrs& p, const cpx<T>* U,
                        const cpx<T>* dU, double m_diag, TslState* st, TslCoeffs co, double* partials,
                        unsigned* counters, int j, double tau, hipStream_t s, StencilVariant v = StencilVariant{});

// One lattice of a multi-lattice Lanczos step (several handles' recurrences
// advanced by one stencil launch and one update launch per step).  Stencil
// blocks [block0, block0 + nblocks) and update x-blocks [ublock0, ublock0 +
// unblocks) belong to this lattice; block0 and nblocks are multiples of 8.
struct TslSegment {
    Geom g;
    int ngroups, nrhs, map;
    int block0, nblocks;       // stencil blocks: tsl_stencil_blocks(g, dir, gpb) * nrhs
    int ublock0, unblocks;     // update x-blocks per (rhs, side)
    long long fsz;             // elements per rhs and side
    double tau;                // breakdown tolerance of the lattice's handle
    StepPtrs p;
    const void* U;
    const void* dU;
    double mdiag;
    TslState* st;
    TslCoeffs co;
    double* partials;
    unsigned* counters;
};
// update x-blocks per (rhs, side) of launch_tsl_update
int tsl_update_xblocks(long long fsz);
// the two kernels of step j over nseg lattices (device table seg[nseg]);
// gpb 1 or 2, seq 1 for the sequential form (dir 1 only); nterms as
// launch_tsl_update (0: no update, step 0)
template <typename T>
void launch_tsl_step_multi(int dir, int gpb, int seq, int nterms, const TslSegment* seg, int nseg, int nblocks,
                           int ublocks, int max_nrhs, int j, hipStream_t s);

// sgn(T_k) e_1 for nrhs tridiagonal matrices by the resolvent quadrature.
// quad_step: first refined step of the trapezoidal rule in log(y); max_levels:
// refinement levels before giving up (<= 0: kDefaultMaxLevels); chunk: solves
// per launch, which sizes the scratch (<= 0: kDefaultChunkSolves).  The result
// does not depend on chunk (the node sums are accumulated in one fixed order).
constexpr int kDefaultMaxLevels = 9;
constexpr int kMaxLevelsLimit = 20;
constexpr int kDefaultChunkSolves = 16384;
struct SmallSignCfg {
    double quad_step = 0.1;
    int max_levels = kDefaultMaxLevels;
    int chunk = kDefaultChunkSolves;
};
// Return codes of the small dense solvers: 0 converged, 1 not converged within
// max_levels (the result is the last level's), < 0 the negated HIP error.
// transpose: sgn(T^T) e_1 (the first row of sgn(T)) instead of sgn(T) e_1.
int launch_small_sign(int nrhs, int k, TslCoeffs co, const SmallSignCfg& cfg, c64* scratch, c64* c_out,
                      double* check, hipStream_t s, int transpose = 0);
size_t small_sign_scratch_elems(int nrhs, int k, int chunk);
// M = L_sgn(T_k, e_1 e_1^T) (k x k, row-major) for rhs 0 of co
int launch_small_frechet(int k, TslCoeffs co, const SmallSignCfg& cfg, c64* scratch, c64* M_out, double* check,
                         hipStream_t s);
size_t small_frechet_scratch_elems(int k);
// Nested two-sided Lanczos for sgn(T_k) e_1: an inner Krylov-Ritz run of kp
// steps on Tt = (T_k + T_k^{-1}) / 2 (same sign as T_k) from e_1, whose kp x kp
// Ritz matrix is signed by the quadrature above; c = V' sgn(T') e_1.  Return
// codes: 0, 1 (quadrature of T' not converged), 2 (inner breakdown, step in
// *bstep), < 0 HIP error.
size_t nested_sign_scratch_elems(int nrhs, int k, int kp, int chunk);
int launch_nested_sign(int nrhs, int k, TslCoeffs co, int kp, double tau, const SmallSignCfg& cfg, c64* scratch,
                       c64* c_out, double* check, int* bstep, hipStream_t s);

// coefficient matrices of the deflated gradient (rhs 0 of co, m deflated pairs):
// A, B [k][m], Cm [m][m] (see kernels_small.hip); scol / srow: sgn(T) e_1 and
// sgn(T)^T e_1; cv = L^dag b, dv = R^dag x; lam device [m], sg device [m]
size_t defl_vjp_coef_scratch(int k, int m);
void launch_defl_vjp_coef(int k, TslCoeffs co, int m, const c64* lam, const double* sg, const c64* scol,
                          const c64* srow, const c64* cv, const c64* dv, c64* A, c64* B, c64* Cm, c64* scratch,
                          hipStream_t s);

// y = sum_j coef[rhs][j] * basis[rhs][j]  (top/bottom halves selected by half_off);
// with accumulate, y += the sum (the basis taken a chunk of vectors at a time)
template <typename T>
void launch_reconstruct(const Geom& g, int nrhs, int k, const cpx<T>* basis, long long s_rhs,
                        long long s_j, int half, const c64* coef, int coef_ld, void* out_aos,
                        hipStream_t s, bool accumulate = false);

// scalar result: out[rhs] = scale[rhs] * sum_j c[rhs][j] * proj[rhs][j]
void launch_scalar_dot(int nrhs, int k, const c64* c, const c64* proj, int ld,
                       const c64* scale, c64* out, hipStream_t s);

// deflation products (kernels_defl.hip), FP64 fields flattened to nf = 12 Vp
// complex: C (m x nr, row-major) = A^dag B;  Y += A C
// The projection's reduction is split into chunks of `chunk` elements (a
// multiple of 4; 0 = the default, short enough that a one-vector projection
// runs many waves); its scratch depends on the chunk.
size_t defl_proj_scratch(int m, int nr, long long nf, long long chunk = 0);
void launch_defl_proj(const c64* A, long long sA, int m, const c64* B, long long sB, int nr, long long nf,
                      c64* C, c64* scratch, hipStream_t s, long long chunk = 0);
// Y += A C, or with Y0: Y = Y0 + A C (Y0 columns at stride sY0)
void launch_defl_comb(const c64* A, long long sA, int m, const c64* C, int nr, c64* Y, long long sY, long long nf,
                      hipStream_t s, const c64* Y0 = nullptr, long long sY0 = 0);
// out[i][r] = sign * f[i] * in[i][r]
void launch_defl_scale(int m, int nr, const double* f, const c64* in, c64* out, double sign, hipStream_t s);
// out[r] += sum_i conj(P1[i][r]) sD[i][r] + conj(P2[i][r]) sC[i][r]
void launch_defl_scalar(int l, int nr, const c64* P1, const c64* sD, const c64* P2, const c64* sC, c64* out,
                        hipStream_t s);
void launch_add_soa_to_aos(const Geom& g, int n, const c64* in, long long stride, void* out_aos, hipStream_t s);
template <typename T>
void launch_convert_field(const Geom& g, int n, const c64* in, long long sin, cpx<T>* out, long long sout,
                          hipStream_t s);

// AoS complex128 fields: out = cb b + cy gamma5 y (b may be null)
void launch_gamma5_axpy(long long n_sites, double cb, const void* b, double cy, const void* y, void* out,
                        hipStream_t s);
// out[r] = |a_r - b_r| / (2 |b_r|) for n AoS complex128 fields of m complex each (device out);
// with top: sqrt(|top_r|^2 + |a_r - b_r|^2) / (2 |b_r|), the block vector (top; a) against (0; b)
void launch_half_rel_diff(int n, long long m, const void* a, const void* b, double* out, hipStream_t s,
                          const void* top = nullptr);

// *flag |= 1 when the n complex of a and b differ anywhere (flag cleared by the caller)
void launch_field_differs(long long n, const c64* a, const c64* b, unsigned* flag, hipStream_t s);

// FP32 internal fields -> FP64 internal fields (n fields, strides in elements)
void launch_widen_field(const Geom& g, int n, const c32* in, long long sin, c64* out, long long sout, hipStream_t s);

// gradient of <x|sgn(H)|b> (kernels_defl.hip / kernels_stencil.hip)
// out = conj(in), n complex (elementwise)
void launch_conj_c64(long long n, const c64* in, c64* out, hipStream_t s);
void launch_vjp_scale_m(int k, TslCoeffs co, const c64* M, c64* Mp, hipStream_t s);
// force of the gradient from the basis pairs p < k; the sum over p may be
// split over launches that carry Kf, Kb in Kacc ([18][4V], needed unless
// first && last): first starts from zero, last writes F, dU, dUc, trF.
// With Kpart (vjp_force_scratch_elems(g, nchunk) elements) and nchunk > 1, a
// first launch splits its sum over p into nchunk ranges run side by side and
// summed in order (vjp_force_chunks: the number that fills the GPU).
void launch_vjp_force(const Geom& g, int k, const c64* Vb, long long sV, const c64* Zb, long long sZ, const c64* U64,
                      double emu, c64* F, c64* dU, c64* dUc, c64* trF, c64* dth, hipStream_t s, c64* Kacc = nullptr,
                      bool first = true, bool last = true, c64* Kpart = nullptr, int nchunk = 1);
int vjp_force_chunks(const Geom& g, int k);
size_t vjp_force_scratch_elems(const Geom& g, int nchunk);
void launch_sum_c64(int n, const c64* v, c64* out, hipStream_t s);

// eigenpairs of smallest |lambda| and eigenvector derivatives for deflation (eigs.hip)
struct EigParams {
    Geom g;
    const c64* U = nullptr;     // FP64 internal links
    const c64* dU = nullptr;    // FP64 internal link direction (dir_link)
    double md = 0.0;            // m0 + 4 r
    double mu = 0.0;
    int m = 0, l = 0, p = 0;    // pairs, derivative pairs, Arnoldi basis size (0: 2 m + 20)
    bool dir_link = false;
    double tol = 1e-10;         // residual |H r - theta r| of the wanted pairs
    int max_outer = 80;         // restart cycles of the Arnoldi iteration
    double shift_tol = 1e-11;   // relative residual of the shifted derivative solves
    int shift_max = 60000;      // and their iteration limit (rough links need 40 000)
    uint64_t seed = 1611;
    hipStream_t stream = nullptr;
};
struct EigResult {
    std::vector<c64> lam;                 // m eigenvalues, increasing |lambda|
    c64 *R = nullptr, *L = nullptr;       // device [m][12][Vp], caller frees
    c64 *dR = nullptr, *dL = nullptr;     // device [l][12][Vp] or null, caller frees
    int outer_right = 0, outer_left = 0, shift_iters = 0;
    double res_right = 0, res_left = 0, biorth = 0, shift_res = 0, ms = 0;
    std::string err;
};
// 0 on success; -2 allocation, -3 HIP error, -7 no convergence (err says why)
int eigs_compute(const EigParams& p, EigResult& out);

}  // namespace ovd
