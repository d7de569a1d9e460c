// Wilson-Dirac stencil kernels for gfx950: the standalone operator apply, and
// the two kernels of one two-sided Lanczos step (three-term update, then the
// stencil with the step's inner products).
//
// Operator (Sec. 1, eq. 1): H(mu) = gamma5 Dw(mu) with
//   Dw(mu) psi(x) = (m0 + 4) psi(x) - 1/2 sum_nu [ e^{mu d_nu4} (1 - gamma_nu) U_nu(x) psi(x+nu)
//                   + e^{-mu d_nu4} (1 + gamma_nu) U_nu(x-nu)^dag psi(x-nu) ]   (r = 1)
// in the chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]].
// With r = 1 each (1 -+ gamma_nu) has rank two, so a hop projects the four
// spin components to two ("half spinor"), multiplies those by the 3x3 link and
// rebuilds the lower two spin components from the upper two.  The time
// boundary factor is applied on the hops that cross t = Lt-1 <-> 0.
//
// Memory: fields are stored [12][Vp] (component-major), so the 64 lanes of a
// wave read 64 consecutive sites of one component in one coalesced access;
// links are [4][9][Vp].  The kernels are bound by memory bandwidth and
// latency, not arithmetic: no MFMA and no LDS staging of neighbours (the 4D
// halo of any tile small enough for LDS would be larger than the tile);
// neighbour reuse comes from L1/L2, helped by an XCD-aware block order that
// gives each of the eight XCDs a contiguous slab of sites.  Every hop issues
// all of its loads before any arithmetic (branch-free, one load batch per
// hop), which is what keeps enough bytes in flight.
#include "ovd_internal.h"

// occupancy hint for the stencil kernels (waves per SIMD); empty = compiler's choice
#ifndef OVD_OCC
#define OVD_OCC
#endif

namespace ovd {

// ---------------------------------------------------------------------------
// spin projection table
// ---------------------------------------------------------------------------
// (1 - gamma_nu) (forward hop) and (1 + gamma_nu) (backward hop) in the chiral
// basis, hop index i = 2 nu + (backward):
//   h0 = psi_0 + F0 psi_P0,  h1 = psi_1 + F1 psi_P1  (P1 = 5 - P0)
//   result spins 0,1 = h0, h1;  spin 2 = G0 h_Q0,  spin 3 = G1 h_Q1  (Q1 = 1 - Q0)
// with F, G in {+1, -1, +i, -i} (codes 0..3).  Packed per hop as
//   bit 0: P0 == 3,  bits 1-2: F0, 3-4: F1,  bit 5: Q0,  bits 6-7: G0, 8-9: G1.
enum { F_P1 = 0, F_M1 = 1, F_PI = 2, F_MI = 3 };
#define OVD_HOP(P0, F0, F1, Q0, G0, G1) \
    ((P0 == 3 ? 1 : 0) | ((F0) << 1) | ((F1) << 3) | ((Q0) << 5) | ((G0) << 6) | ((G1) << 8))
__constant__ int kHop[8] = {
    OVD_HOP(3, F_PI, F_PI, 1, F_MI, F_MI),   // x forward
    OVD_HOP(3, F_MI, F_MI, 1, F_PI, F_PI),   // x backward
    OVD_HOP(3, F_P1, F_M1, 1, F_M1, F_P1),   // y forward
    OVD_HOP(3, F_M1, F_P1, 1, F_P1, F_M1),   // y backward
    OVD_HOP(2, F_PI, F_MI, 0, F_MI, F_PI),   // z forward
    OVD_HOP(2, F_MI, F_PI, 0, F_PI, F_MI),   // z backward
    OVD_HOP(2, F_M1, F_M1, 0, F_M1, F_M1),   // t forward
    OVD_HOP(2, F_P1, F_P1, 0, F_P1, F_P1)};  // t backward
#undef OVD_HOP

// z times the constant with code f (0: +1, 1: -1, 2: +i, 3: -i), branch-free:
// +1: (re, im), -1: (-re, -im), +i: (-im, re), -i: (im, -re)
template <typename T>
__device__ __forceinline__ cpx<T> mulc(cpx<T> z, int f) {
    const bool sw = f >= 2;
    const T re = sw ? z.im : z.re;
    const T im = sw ? z.re : z.im;
    const T sr = (f == 1 || f == 2) ? T(-1) : T(1);
    const T si = (f == 1 || f == 3) ? T(-1) : T(1);
    return {sr * re, si * im};
}

struct Nbr {
    int f[4], b[4];
    bool wf, wb;   // forward / backward time hop crosses the boundary
};

__device__ __forceinline__ Nbr neighbours(const Geom& g, int s) {
    Nbr N;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    int r = s;
    const int x = r % Lx; r /= Lx;
    const int y = r % Ly; r /= Ly;
    const int z = r % Lz;
    const int t = r / Lz;
    const int sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
    N.f[0] = (x == Lx - 1) ? s - (Lx - 1) : s + 1;
    N.b[0] = (x == 0) ? s + (Lx - 1) : s - 1;
    N.f[1] = (y == Ly - 1) ? s - (Ly - 1) * sy : s + sy;
    N.b[1] = (y == 0) ? s + (Ly - 1) * sy : s - sy;
    N.f[2] = (z == Lz - 1) ? s - (Lz - 1) * sz : s + sz;
    N.b[2] = (z == 0) ? s + (Lz - 1) * sz : s - sz;
    N.f[3] = (t == Lt - 1) ? s - (Lt - 1) * st : s + st;
    N.b[3] = (t == 0) ? s + (Lt - 1) * st : s - st;
    N.wf = (t == Lt - 1);
    N.wb = (t == 0);
    return N;
}

// Whole-site loads and stores of a spinor field and of one link matrix, 16
// bytes per lane (one complex in FP64, two in FP32).
template <typename T>
__device__ __forceinline__ void load12(const cpx<T>* __restrict__ F, int n, int Vp, cpx<T> (&v)[12]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = F[(size_t)c * Vp + n];
    } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float4 t = *reinterpret_cast<const float4*>(F + ((size_t)q * Vp + n) * 2);
            v[2 * q] = {t.x, t.y};
            v[2 * q + 1] = {t.z, t.w};
        }
    }
}

template <typename T>
__device__ __forceinline__ void store12(cpx<T>* __restrict__ F, int n, int Vp, const cpx<T> (&v)[12]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int c = 0; c < 12; ++c) F[(size_t)c * Vp + n] = v[c];
    } else {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            *reinterpret_cast<float4*>(F + ((size_t)q * Vp + n) * 2) =
                float4{v[2 * q].re, v[2 * q].im, v[2 * q + 1].re, v[2 * q + 1].im};
    }
}

// the 3x3 link U_nu(ls), entries 3a + b
template <typename T>
__device__ __forceinline__ void load_link(const cpx<T>* __restrict__ W, int nu, int ls, int Vp, cpx<T> (&u)[9]) {
    if constexpr (sizeof(T) == 8) {
        const cpx<T>* Wn = W + (size_t)nu * 9 * Vp + ls;
#pragma unroll
        for (int i = 0; i < 9; ++i) u[i] = Wn[(size_t)i * Vp];
    } else {
        const cpx<T>* Wn = W + (size_t)nu * 5 * Vp * 2 + (size_t)ls * 2;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const float4 t = *reinterpret_cast<const float4*>(Wn + (size_t)q * Vp * 2);
            u[2 * q] = {t.x, t.y};
            if (2 * q + 1 < 9) u[2 * q + 1] = {t.z, t.w};
        }
    }
}

// half spinor of field F at site n for hop code `code`
template <typename T>
__device__ __forceinline__ void project(const cpx<T>* __restrict__ F, int n, int Vp, int code,
                                        cpx<T> (&h0)[3], cpx<T> (&h1)[3]) {
    cpx<T> v[12];
    load12(F, n, Vp, v);
    const bool p3 = code & 1;
    const int f0 = (code >> 1) & 3, f1 = (code >> 3) & 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> a = p3 ? v[9 + c] : v[6 + c];   // spin P0
        const cpx<T> b = p3 ? v[6 + c] : v[9 + c];   // spin P1
        h0[c] = v[c] + mulc(a, f0);
        h1[c] = v[3 + c] + mulc(b, f1);
    }
}

// acc += coef * reconstruct(W h), W = U_nu(ls) (forward) or U_nu(ls)^dag (backward)
template <typename T>
__device__ __forceinline__ void link_mult_acc(cpx<T> (&acc)[12], const cpx<T> (&h0)[3], const cpx<T> (&h1)[3],
                                              const cpx<T>* __restrict__ W, int hidx, int code, int ls, int Vp,
                                              T coef) {
    const bool fwd = (hidx & 1) == 0;
    const int q0 = (code >> 5) & 1;
    const int g0c = (code >> 6) & 3, g1c = (code >> 8) & 3;
    cpx<T> u[9];
    load_link(W, hidx >> 1, ls, Vp, u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // row a of U:  U[a][b] = u[3a + b];  row a of U^dag: conj(U[b][a]) = conj(u[3b + a])
        const cpx<T> r0 = fwd ? u[3 * a] : conj(u[a]);
        const cpx<T> r1 = fwd ? u[3 * a + 1] : conj(u[3 + a]);
        const cpx<T> r2 = fwd ? u[3 * a + 2] : conj(u[6 + a]);
        const cpx<T> g0 = r0 * h0[0] + r1 * h0[1] + r2 * h0[2];
        const cpx<T> g1 = r0 * h1[0] + r1 * h1[1] + r2 * h1[2];
        acc[a] += coef * g0;
        acc[3 + a] += coef * g1;
        acc[6 + a] += coef * mulc(q0 == 0 ? g0 : g1, g0c);
        acc[9 + a] += coef * mulc(q0 == 0 ? g1 : g0, g1c);
    }
}

// The eight hops of field P (links W).  On the two time hops the field
// P + sf Q (forward) / P + sb Q (backward) is used instead, sf, sb in {0, +-1}
// (the mu derivative of the block matrix combines its two halves there);
// spatial hops get -1/2 cs, time hops -1/2 cf / -1/2 cb and the boundary
// factor.  With space == false only the time hops are applied.
template <typename T>
__device__ __forceinline__ void hops(cpx<T> (&acc)[12], const cpx<T>* __restrict__ P, const cpx<T>* __restrict__ Q,
                                     int sf, int sb, const Nbr& N, int s, const cpx<T>* __restrict__ W, int Vp,
                                     T cs, T cf, T cb, int bc, bool space) {
    const T h = T(-0.5);
#pragma unroll 1
    for (int i = space ? 0 : 6; i < 8; ++i) {
        const int nu = i >> 1;
        const bool fwd = (i & 1) == 0;
        const int nf = nu == 0 ? N.f[0] : nu == 1 ? N.f[1] : nu == 2 ? N.f[2] : N.f[3];
        const int nbk = nu == 0 ? N.b[0] : nu == 1 ? N.b[1] : nu == 2 ? N.b[2] : N.b[3];
        const int n = fwd ? nf : nbk;
        const int ls = fwd ? s : nbk;
        const int code = kHop[i];
        T coef = h * cs;
        if (nu == 3) coef = fwd ? h * cf * (N.wf ? T(bc) : T(1)) : h * cb * (N.wb ? T(bc) : T(1));
        cpx<T> h0[3], h1[3];
        project(P, n, Vp, code, h0, h1);
        const int sg = (nu < 3) ? 0 : (fwd ? sf : sb);
        if (sg != 0) {   // uniform per wave
            cpx<T> q0[3], q1[3];
            project(Q, n, Vp, code, q0, q1);
            const T sgn = T(sg);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                h0[c] += sgn * q0[c];
                h1[c] += sgn * q1[c];
            }
        }
        link_mult_acc(acc, h0, h1, W, i, code, ls, Vp, coef);
    }
}

// Work decomposition over the 8 XCDs.  Blocks are dispatched round-robin over
// the XCDs (block b runs on XCD b % 8, in order of b / 8), and each XCD has its
// own 4 MB L2.  A stencil re-reads every field at the neighbouring sites, the
// furthest (the time neighbours) one time slice (Lx Ly Lz sites) away, so an
// XCD keeps its neighbour data in L2 only if it sweeps a compact piece of
// work in site order.  The (rhs, site group) work items are therefore split
// into 8 compact chunks, one per XCD:
//   nrhs a multiple of 8:  XCD x takes right-hand sides x m .. x m + m - 1
//                          (m = nrhs / 8) over the whole lattice, site group
//                          major, so those m share each link read;
//   nrhs dividing 8:       XCD x takes one right-hand side over 1/(8/nrhs) of
//                          the lattice (a contiguous range of time slices);
//   otherwise:             contiguous ranges of (site group, rhs) pairs.
// nb (site groups per rhs, padded) is a multiple of 8.
struct Work {
    int rhs, grp;
};
__device__ __forceinline__ Work xcd_work(int bid, int nb, int nrhs) {
    const int x = bid & 7, idx = bid >> 3;
    Work w;
    if ((nrhs & 7) == 0) {
        const int m = nrhs >> 3;
        w.grp = idx / m;
        w.rhs = x * m + idx % m;
    } else if ((8 % nrhs) == 0) {
        const int parts = 8 / nrhs;
        w.rhs = x / parts;
        w.grp = (x % parts) * (nb / parts) + idx;
    } else {
        const int i = x * (nb * nrhs / 8) + idx;
        w.grp = i / nrhs;
        w.rhs = i % nrhs;
    }
    return w;
}

// ---------------------------------------------------------------------------
// standalone operator
// ---------------------------------------------------------------------------
template <typename T, int OP>
__global__ __launch_bounds__(256) OVD_OCC void apply_op_kernel(Geom g, const double* __restrict__ emu,
                                                       const cpx<T>* __restrict__ U,
                                                       const cpx<T>* __restrict__ dU, T mdiag,
                                                       const cpx<T>* __restrict__ in,
                                                       cpx<T>* __restrict__ out, int ngroups, int nrhs) {
    const Work w = xcd_work(blockIdx.x, gridDim.x / nrhs, nrhs);
    const int rhs = w.rhs;
    const int grp = w.grp * 4 + (threadIdx.x >> 6);
    const int s = grp * 64 + (threadIdx.x & 63);
    if (grp >= ngroups || s >= g.V) return;
    const int Vp = g.Vp;
    const size_t roff = (size_t)rhs * 12 * Vp;
    const T ep = T(emu[2 * rhs]), em = T(emu[2 * rhs + 1]);
    const cpx<T>* P = in + roff;
    const Nbr N = neighbours(g, s);
    cpx<T> acc[12];
    if constexpr (OP == 0 || OP == 1) {          // H or Dw
        load12(P, s, Vp, acc);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = mdiag * acc[c];
        hops(acc, P, P, 0, 0, N, s, U, Vp, T(1), ep, em, g.bc_t, true);
    } else if constexpr (OP == 2) {             // dH/dmu: time hops, e^{mu} and -e^{-mu}
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
        hops(acc, P, P, 0, 0, N, s, U, Vp, T(0), ep, -em, g.bc_t, false);
    } else {                                    // dH/dt along dU: hops with dU, no mass term
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
        hops(acc, P, P, 0, 0, N, s, dU, Vp, T(1), ep, em, g.bc_t, true);
    }
    if (OP != 1) {
#pragma unroll
        for (int c = 6; c < 12; ++c) acc[c] = -acc[c];   // gamma5
    }
    store12(out + roff, s, Vp, acc);
}

template <typename T>
void launch_apply_op(const Geom& g, int op, int nrhs, const double* d_emu, const cpx<T>* U,
                     const cpx<T>* dU, double m_diag, const cpx<T>* in, cpx<T>* out, hipStream_t s) {
    const int ngroups = (g.V + 63) / 64;
    const int nq = ((ngroups + 3) / 4 + 7) / 8 * 8;   // blocks of 4 site groups, padded to 8
    dim3 grid(nq * nrhs), block(256);
    const T md = T(m_diag);
    switch (op) {
        case 0: apply_op_kernel<T, 0><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups, nrhs); break;
        case 1: apply_op_kernel<T, 1><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups, nrhs); break;
        case 2: apply_op_kernel<T, 2><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups, nrhs); break;
        default: apply_op_kernel<T, 3><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups, nrhs); break;
    }
}
template void launch_apply_op<double>(const Geom&, int, int, const double*, const c64*, const c64*, double,
                                      const c64*, c64*, hipStream_t);
template void launch_apply_op<float>(const Geom&, int, int, const double*, const c32*, const c32*, double,
                                     const c32*, c32*, hipStream_t);

// ---------------------------------------------------------------------------
// deterministic block reduction of NV doubles (fixed shuffle tree, then waves
// in order); the result is valid in thread 0
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* lds /* [16][NV] */) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
        v[i] = x;
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int i = 0; i < NV; ++i) lds[w * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < NV; ++i) {
            double x = lds[i];
            for (int q = 1; q < nw; ++q) x += lds[q * NV + i];
            v[i] = x;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Lanczos step, part 1: three-term update (element-wise)
//     vhat_{j+1} = av X + bv Y + cv Z,   what_{j+1} = aw X' + bw Y' + cw Z'
// with X = A vhat_j, Y = vhat_j, Z = vhat_{j-1} (all unnormalised; the
// coefficients fold in the normalisations, see the stencil kernel below).
// blockIdx.z = side (0: v, 1: w); NT = number of terms (2 on the first update).
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ __launch_bounds__(256) void tsl_update_kernel(StepPtrs p, long long n_elem,
                                                         const TslState* __restrict__ st) {
    const int rhs = blockIdx.y;
    const TslState* S = st + rhs;
    if (S->flag) return;
    const bool vside = blockIdx.z == 0;
    const cpx<T> a = cast<T>(vside ? S->av : S->aw);
    const cpx<T> b = cast<T>(vside ? S->bv : S->bw);
    const cpx<T> c = cast<T>(vside ? S->cv : S->cw);
    const cpx<T>* X = vside ? (const cpx<T>*)p.Xv + rhs * p.sXv : (const cpx<T>*)p.Xw + rhs * p.sXw;
    const cpx<T>* Y = vside ? (const cpx<T>*)p.Yv + rhs * p.sYv : (const cpx<T>*)p.Yw + rhs * p.sYw;
    const cpx<T>* Z = vside ? (const cpx<T>*)p.Zv + rhs * p.sZv : (const cpx<T>*)p.Zw + rhs * p.sZw;
    cpx<T>* O = vside ? (cpx<T>*)p.outV + rhs * p.sV : (cpx<T>*)p.outW + rhs * p.sW;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        cpx<T> r = a * X[e] + b * Y[e];
        if constexpr (NT == 3) r += c * Z[e];
        O[e] = r;
    }
}

// ---------------------------------------------------------------------------
// Lanczos step, part 2: stencil and inner products.
//
// Reads the new unnormalised vectors vhat, what, writes A vhat and A^dag what
// and the block partial sums of
//     omega = what^dag vhat,  gamma = what^dag A vhat = (A^dag what)^dag vhat,
//     p = x^dag vhat_top,  |vhat|^2, |what|^2.
// The last block to finish sums the partials in a fixed order and advances the
// recurrence: delta = sqrt|omega|, beta = omega/delta, alpha = gamma/omega
// (= w^dag A v for the normalised vectors), and the coefficients of the next
// update.  One grid-wide reduction per Lanczos step, no host round trip.
//
// Work split: a block is NK waves over the same 64 sites, wave = output kind.
//   DIR 0 (A = H):                kind 0 = H vhat,  kind 1 = H^dag what
//   DIR 1/2 (A = B = [[H, dH], [0, H]], B^dag = [[H^dag, 0], [dH^dag, H^dag]]):
//     kind 0 = H vt + dH vb,  kind 1 = H vb,  kind 2 = H^dag wt,  kind 3 = dH^dag wt + H^dag wb
// with H^dag = H(-mu); for d/dmu, dH only has time hops (e^{mu}, -e^{-mu}) and
// dH^dag = -dH/dmu(-mu) (time hops -e^{-mu}, e^{mu}); for a link direction,
// dH is the hopping term with links dU, and dH^dag that with dU at -mu.
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__global__ __launch_bounds__(256) OVD_OCC void tsl_stencil_kernel(Geom g, StepPtrs p, const cpx<T>* __restrict__ U,
                                                          const cpx<T>* __restrict__ dU, T mdiag,
                                                          TslState* __restrict__ st, TslCoeffs co,
                                                          double* __restrict__ partials,
                                                          unsigned* __restrict__ counters, int j, double tau,
                                                          int ngroups, int nrhs) {
    constexpr int NK = (DIR == 0) ? 2 : 4;
    __shared__ double lds[16 * 8];
    __shared__ int am_last;
    const int nb = gridDim.x / nrhs;                // blocks per rhs
    const Work wk = xcd_work(blockIdx.x, nb, nrhs);
    const int rhs = wk.rhs;
    const int grp = wk.grp;                         // in [0, ngroups padded to 8)
    TslState* S = st + rhs;
    if (S->flag) return;   // uniform over the rhs: breakdown in an earlier step
    const int Vp = g.Vp;
    const int kind = threadIdx.x >> 6;
    const int s = grp * 64 + (threadIdx.x & 63);
    const bool active = (grp < ngroups) && (s < g.V) && (kind < NK);
    const T ep = T(S->emu), em = T(S->emu_inv);
    const size_t HALF = (size_t)12 * Vp;
    // Per-kind configuration (uniform per wave):
    //   vside: output on the v side (A, i.e. H(mu)) or the w side (A^dag, H(-mu));
    //   hp / hq: half-field index (0 top, 1 bottom) of the primary / secondary input;
    //   sf, sb: sign of the secondary input on the forward / backward time hop (d/dmu);
    //   sec: secondary input hopped with dU (d/dlink).
    const bool vside = (kind == 0) || (kind == 1 && DIR != 0);
    int hp = 0, hq = 0, sf = 0, sb = 0;
    bool sec = false;
    if (DIR != 0) {
        if (kind == 0) { hp = 0; hq = 1; }
        else if (kind == 1) { hp = 1; hq = 1; }
        else if (kind == 2) { hp = 0; hq = 0; }
        else { hp = 1; hq = 0; }
        if (DIR == 1 && kind == 0) { sf = +1; sb = -1; }   // H vt + dH/dmu vb
        if (DIR == 1 && kind == 3) { sf = -1; sb = +1; }   // dH/dmu^dag wt + H^dag wb
        if (DIR == 2 && (kind == 0 || kind == 3)) sec = true;
    }
    const cpx<T>* F = vside ? (const cpx<T>*)p.outV + rhs * p.sV : (const cpx<T>*)p.outW + rhs * p.sW;
    const cpx<T>* P = F + hp * HALF;
    const cpx<T>* Q = F + hq * HALF;
    const T cf = vside ? ep : em, cbk = vside ? em : ep;

    double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (active) {
        const Nbr N = neighbours(g, s);
        cpx<T> acc[12];
        load12(P, s, Vp, acc);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = mdiag * acc[c];
        hops(acc, P, Q, sf, sb, N, s, U, Vp, T(1), cf, cbk, g.bc_t, true);
        if (DIR == 2 && sec) hops(acc, Q, Q, 0, 0, N, s, dU, Vp, T(1), cf, cbk, g.bc_t, true);
        cpx<T>* oA = vside ? (cpx<T>*)p.outU + rhs * p.sU : (cpx<T>*)p.outZ + rhs * p.sZ;
        oA += hp * HALF;
#pragma unroll
        for (int c = 6; c < 12; ++c) acc[c] = -acc[c];   // gamma5
        store12(oA, s, Vp, acc);
        // reduction terms.  v side: omega = what^dag vhat, |vhat|^2, p = x^dag vhat_top;
        // w side: gamma = what^dag A vhat = (A^dag what)^dag vhat, |what|^2.
        // Each thread holds at most its output and one loaded field at a time.
        if (vside) {
            cpx<T> vv[12], wv[12];
            load12(P, s, Vp, vv);
            load12((const cpx<T>*)p.outW + rhs * p.sW + hp * HALF, s, Vp, wv);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const c64 om = cdot(cast<double>(wv[c]), cast<double>(vv[c]));
                part[0] += om.re; part[1] += om.im;
                part[6] += norm2(cast<double>(vv[c]));
            }
            if (hp == 0 && p.xproj) {
                load12((const cpx<T>*)p.xproj + rhs * p.sx, s, Vp, wv);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const c64 pr = cdot(cast<double>(wv[c]), cast<double>(vv[c]));
                    part[4] += pr.re; part[5] += pr.im;
                }
            }
        } else {
            cpx<T> vv[12];
            load12((const cpx<T>*)p.outV + rhs * p.sV + hp * HALF, s, Vp, vv);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const c64 ga = cdot(cast<double>(acc[c]), cast<double>(vv[c]));
                part[2] += ga.re; part[3] += ga.im;
            }
            load12(P, s, Vp, vv);
#pragma unroll
            for (int c = 0; c < 12; ++c) part[7] += norm2(cast<double>(vv[c]));
        }
    }

    block_reduce<8>(part, lds);
    if (threadIdx.x == 0) {
        double* dst = partials + ((size_t)rhs * nb + grp) * 8;
        for (int i = 0; i < 8; ++i) __hip_atomic_store(dst + i, part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned prev = atomicAdd(counters + rhs, 1u);
        am_last = (prev == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!am_last) return;
    __threadfence();
    double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double* src = partials + ((size_t)rhs * nb + b) * 8;
        for (int i = 0; i < 8; ++i) tot[i] += __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_reduce<8>(tot, lds);
    if (threadIdx.x != 0) return;
    __hip_atomic_store(counters + rhs, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const c64 omega{tot[0], tot[1]}, gam{tot[2], tot[3]}, pr{tot[4], tot[5]};
    const double nv = tot[6], nw = tot[7];
    const double aom = sqrt(norm2(omega));
    const double margin = aom / sqrt(nv * nw);
    const size_t ci = (size_t)rhs * co.kmax + j;
    if (!(margin == margin) || !(nv < 1e300) || !(nw < 1e300) || !(norm2(gam) < 1e300)) {
        S->flag = 2;
        S->bstep = j;
        return;
    }
    if (margin < S->min_margin) S->min_margin = margin;
    if (margin <= tau) {
        S->flag = 1;
        S->bstep = j;
        return;
    }
    // j = 0: v_1 = psi/|psi|, w_1 = phi/conj(phi^dag v_1); later delta = sqrt|omega|
    const double delta = (j == 0) ? sqrt(nv) : sqrt(aom);
    const c64 beta = (1.0 / delta) * omega;
    const c64 alpha = cdiv(gam, omega);
    co.alpha[ci] = alpha;
    co.beta[ci] = beta;
    co.delta[ci] = c64{delta, 0.0};
    co.proj[ci] = (1.0 / delta) * pr;
    // next update: vhat = (A vhat - alpha vhat)/delta - beta vhat_prev/delta_prev,
    //              what = (A^dag what - conj(alpha) what)/conj(beta) - delta what_prev/conj(beta_prev)
    const c64 one{1.0, 0.0};
    S->av = c64{1.0 / delta, 0.0};
    S->bv = -((1.0 / delta) * alpha);
    S->aw = cdiv(one, conj(beta));
    S->bw = -cdiv(conj(alpha), conj(beta));
    if (j == 0) {
        S->cv = c64{0.0, 0.0};
        S->cw = c64{0.0, 0.0};
    } else {
        S->cv = -((1.0 / S->delta_prev) * beta);
        S->cw = -cdiv(c64{delta, 0.0}, conj(S->beta_prev));
    }
    S->delta_prev = delta;
    S->beta_prev = beta;
    S->step = j + 1;
}

template <typename T>
void launch_tsl_update(int nrhs, int nterms, long long fsz, const StepPtrs& p, const TslState* st,
                       hipStream_t s) {
    long long nblk = (fsz + 255) / 256;
    if (nblk > 2048) nblk = 2048;
    dim3 grid((unsigned)nblk, nrhs, 2);
    if (nterms == 3)
        tsl_update_kernel<T, 3><<<grid, 256, 0, s>>>(p, fsz, st);
    else
        tsl_update_kernel<T, 2><<<grid, 256, 0, s>>>(p, fsz, st);
}

template <typename T>
void launch_tsl_stencil(const Geom& g, int dir, int nrhs, const StepPtrs& p, const cpx<T>* U,
                        const cpx<T>* dU, double m_diag, TslState* st, TslCoeffs co, double* partials,
                        unsigned* counters, int j, double tau, hipStream_t s) {
    const int ngroups = (g.V + 63) / 64;
    const int nb = (ngroups + 7) / 8 * 8;   // blocks per rhs; nb * nrhs is a multiple of 8
    dim3 grid(nb * nrhs);
    const T md = T(m_diag);
    if (dir == 0)
        tsl_stencil_kernel<T, 0><<<grid, dim3(128), 0, s>>>(g, p, U, dU, md, st, co, partials, counters, j, tau, ngroups, nrhs);
    else if (dir == 1)
        tsl_stencil_kernel<T, 1><<<grid, dim3(256), 0, s>>>(g, p, U, dU, md, st, co, partials, counters, j, tau, ngroups, nrhs);
    else
        tsl_stencil_kernel<T, 2><<<grid, dim3(256), 0, s>>>(g, p, U, dU, md, st, co, partials, counters, j, tau, ngroups, nrhs);
}

#define OVD_INST(T)                                                                                        \
    template void launch_tsl_update<T>(int, int, long long, const StepPtrs&, const TslState*, hipStream_t); \
    template void launch_tsl_stencil<T>(const Geom&, int, int, const StepPtrs&, const cpx<T>*, const cpx<T>*, \
                                        double, TslState*, TslCoeffs, double*, unsigned*, int, double,     \
                                        hipStream_t);
OVD_INST(double)
OVD_INST(float)
#undef OVD_INST

// ---------------------------------------------------------------------------
// Link force of s = <x|sgn(H)|b> from K = sum_p v_p z_p^dag (vhat_p, z_p from the
// two-sided Lanczos basis and Z = W M'^dag).  For link U_nu(y) with forward
// hop y -> y + nu:
//   Kf[b][a] = sum_p sum_{s,t} (gamma5 (1 - gamma_nu))_{st} v_p(y+nu)[t][b] conj(z_p(y)[s][a])
//   Kb[b][a] = sum_p sum_{s,t} (gamma5 (1 + gamma_nu))_{st} v_p(y)[t][b] conj(z_p(y+nu)[s][a])
//   ds/dU[a][b] = -1/2 cf sgn Kf[b][a],   ds/dconj(U)[a][b] = -1/2 cb sgn Kb[a][b],
//   F = -1/2 cf sgn U Kf + 1/2 cb sgn Kb U^dag  (ds/dt = tr(F X) for U -> e^{tX} U),
// cf = e^{mu}, cb = e^{-mu} on time links (1 in space), sgn the boundary
// factor of the hop.  One thread per (site, direction), direction fastest.
// trF[y] = tr F_t(y), summed later into ds/dmu.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void vjp_force_kernel(Geom g, int k, const c64* __restrict__ Vb, long long sV,
                                                        const c64* __restrict__ Zb, long long sZ,
                                                        const c64* __restrict__ U, double emu,
                                                        c64* __restrict__ F, c64* __restrict__ dU,
                                                        c64* __restrict__ dUc, c64* __restrict__ trF) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    const int y = t >> 2, nu = t & 3;
    const int Vp = g.Vp;
    const Nbr N = neighbours(g, y);
    const int yp = nu == 0 ? N.f[0] : nu == 1 ? N.f[1] : nu == 2 ? N.f[2] : N.f[3];
    const double sg = (nu == 3 && N.wf) ? double(g.bc_t) : 1.0;
    const double cf = nu == 3 ? emu : 1.0, cb = nu == 3 ? 1.0 / emu : 1.0;
    c64 Kf[9], Kb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Kf[i] = Kb[i] = c64{0.0, 0.0};
    const int cfw = kHop[2 * nu], cbw = kHop[2 * nu + 1];
    for (int p = 0; p < k; ++p) {
        const c64* Vp_ = Vb + (size_t)p * sV;
        const c64* Zp_ = Zb + (size_t)p * sZ;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            // pass 0: (gamma5 (1 - gamma_nu) v(y+nu)) x conj(z(y));  pass 1: (gamma5 (1 + gamma_nu) v(y)) x conj(z(y+nu))
            const int code = pass == 0 ? cfw : cbw;
            c64 h0[3], h1[3];
            project(Vp_, pass == 0 ? yp : y, Vp, code, h0, h1);
            c64 z[12];
            load12(Zp_, pass == 0 ? y : yp, Vp, z);
            const int q0 = (code >> 5) & 1;
            const int g0c = (code >> 6) & 3, g1c = (code >> 8) & 3;
            c64* K = pass == 0 ? Kf : Kb;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                // u spins: 0 h0, 1 h1, 2 -G0 h_Q0, 3 -G1 h_Q1 (the minus from gamma5)
                const c64 u0 = h0[b], u1 = h1[b];
                const c64 u2 = -mulc(q0 == 0 ? h0[b] : h1[b], g0c);
                const c64 u3 = -mulc(q0 == 0 ? h1[b] : h0[b], g1c);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    K[3 * b + a] += u0 * conj(z[a]) + u1 * conj(z[3 + a]) + u2 * conj(z[6 + a]) + u3 * conj(z[9 + a]);
                }
            }
        }
    }
    // link U_nu(y) from the FP64 internal link field
    c64 u[9];
    load_link(U, nu, y, Vp, u);
    const double af = -0.5 * cf * sg, ab = 0.5 * cb * sg;
    const size_t o = ((size_t)nu * g.V + y) * 9;
    c64 tr{0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            c64 f{0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                f += af * (u[3 * a + c] * Kf[3 * c + b]);      // (U Kf)[a][b]
                f += ab * (Kb[3 * a + c] * conj(u[3 * b + c])); // (Kb U^dag)[a][b]
            }
            if (F) F[o + 3 * a + b] = f;
            if (a == b) tr += f;
            if (dU) dU[o + 3 * a + b] = af * Kf[3 * b + a];
            if (dUc) dUc[o + 3 * a + b] = (-ab) * Kb[3 * a + b];
        }
    if (nu == 3) trF[y] = tr;
}

void launch_vjp_force(const Geom& g, int k, const c64* Vb, long long sV, const c64* Zb, long long sZ, const c64* U64,
                      double emu, c64* F, c64* dU, c64* dUc, c64* trF, hipStream_t s) {
    vjp_force_kernel<<<(4 * g.V + 255) / 256, 256, 0, s>>>(g, k, Vb, sV, Zb, sZ, U64, emu, F, dU, dUc, trF);
}

// out = sum_y trF[y] (one block, fixed order)
__global__ void sum_c64_kernel(int n, const c64* __restrict__ v, c64* __restrict__ out) {
    __shared__ double re[256], im[256];
    c64 a{0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += v[i];
    re[threadIdx.x] = a.re;
    im[threadIdx.x] = a.im;
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
        if (threadIdx.x < m) {
            re[threadIdx.x] += re[threadIdx.x + m];
            im[threadIdx.x] += im[threadIdx.x + m];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = c64{re[0], im[0]};
}

void launch_sum_c64(int n, const c64* v, c64* out, hipStream_t s) { sum_c64_kernel<<<1, 256, 0, s>>>(n, v, out); }

}  // namespace ovd
