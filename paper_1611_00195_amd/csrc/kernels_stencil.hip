// Wilson-Dirac stencil kernels for gfx950: the standalone operator apply and
// the fused two-sided Lanczos step.
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
// links are [4][9][Vp].  The kernels are bound by HBM/MALL bandwidth, not by
// arithmetic: no MFMA, no LDS staging of neighbours (the 4D halo of any tile
// small enough for LDS would be larger than the tile); neighbour reuse comes
// from L1/L2, helped by an XCD-aware block order that gives each of the eight
// XCDs a contiguous slab of sites.
#include "ovd_internal.h"

namespace ovd {

// ---------------------------------------------------------------------------
// multiplication by the constants +1, -1, +i, -i
// ---------------------------------------------------------------------------
enum { F_P1 = 0, F_M1 = 1, F_PI = 2, F_MI = 3 };
template <int F, typename T>
__device__ __forceinline__ cpx<T> mulf(cpx<T> z) {
    if constexpr (F == F_P1) return z;
    else if constexpr (F == F_M1) return {-z.re, -z.im};
    else if constexpr (F == F_PI) return {-z.im, z.re};
    else return {z.im, -z.re};
}

// Spin projection of (1 - gamma_nu) (forward hop) and (1 + gamma_nu)
// (backward hop) in the chiral basis, for hop index i = 2 nu + (backward):
//   h0 = psi_0 + F0 psi_P0,  h1 = psi_1 + F1 psi_P1  (P1 = 5 - P0)
//   result spins 0,1 = h0, h1;  spin 2 = G0 h_Q0,  spin 3 = G1 h_Q1  (Q1 = 1 - Q0)
// with F, G in {+1, -1, +i, -i} (codes 0..3).  Packed per hop as
//   bit 0: P0 == 3,  bits 1-2: F0, 3-4: F1,  bit 5: Q0,  bits 6-7: G0, 8-9: G1.
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

// z times the constant with code f (0: +1, 1: -1, 2: +i, 3: -i)
template <typename T>
__device__ __forceinline__ cpx<T> mulc(cpx<T> z, int f) {
    const T re = (f == 0) ? z.re : (f == 1) ? -z.re : (f == 2) ? -z.im : z.im;
    const T im = (f == 0) ? z.im : (f == 1) ? -z.im : (f == 2) ? z.re : -z.re;
    return {re, im};
}

// ---------------------------------------------------------------------------
// field loaders
// ---------------------------------------------------------------------------
// a X + b Y + c Z on one [12][Vp] field; nt = 0 reads X unscaled.
template <typename T>
struct Lin3 {
    const cpx<T>* __restrict__ X;
    const cpx<T>* __restrict__ Y;
    const cpx<T>* __restrict__ Z;
    cpx<T> a, b, c;
    int nt, Vp;
    __device__ __forceinline__ cpx<T> operator()(int comp, int n) const {
        const size_t o = (size_t)comp * Vp + n;
        cpx<T> x = X[o];
        if (nt == 0) return x;
        cpx<T> r = a * x;
        if (nt >= 2) r += b * Y[o];
        if (nt >= 3) r += c * Z[o];
        return r;
    }
    __device__ __forceinline__ cpx<T> operator()(int comp, int n, int) const { return (*this)(comp, n); }
};

// P + s Q with s in {0, +1, -1} (uniform per wave): the mu-derivative
// combines the two halves of a block vector on the time hops.
template <typename T>
struct Src2 {
    Lin3<T> p, q;
    __device__ __forceinline__ cpx<T> operator()(int comp, int n, int sg) const {
        cpx<T> v = p(comp, n);
        if (sg > 0) v += q(comp, n);
        else if (sg < 0) v -= q(comp, n);
        return v;
    }
};

// ---------------------------------------------------------------------------
// one hop: acc += coef * (1 -+ gamma_nu) W psi(n), W = U_nu(x) forward or
// U_nu(x-nu)^dag backward (ls = site of the link)
// ---------------------------------------------------------------------------
template <typename T, class SRC>
__device__ __forceinline__ void hop(cpx<T> (&acc)[12], const SRC& src, int sg, int n, int hidx,
                                    const cpx<T>* __restrict__ W, int ls, int Vp, T coef) {
    const int code = kHop[hidx];
    const int p0 = (code & 1) ? 3 : 2, p1 = 5 - p0;
    const int f0 = (code >> 1) & 3, f1 = (code >> 3) & 3;
    const int q0 = (code >> 5) & 1;
    const int g0c = (code >> 6) & 3, g1c = (code >> 8) & 3;
    const bool fwd = (hidx & 1) == 0;
    cpx<T> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = src(c, n, sg) + mulc(src(p0 * 3 + c, n, sg), f0);
        h1[c] = src(3 + c, n, sg) + mulc(src(p1 * 3 + c, n, sg), f1);
    }
    const cpx<T>* Wn = W + (size_t)(hidx >> 1) * 9 * Vp + ls;
    // forward: row a of U is U[a][b] at 3a+b;  backward: row a of U^dag is conj(U[b][a]) at 3b+a
    const int ra = fwd ? 3 : 1, rb = fwd ? 1 : 3;
    const T cs = fwd ? T(1) : T(-1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> u[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cpx<T> w = Wn[(size_t)(ra * a + rb * b) * Vp];
            u[b] = {w.re, cs * w.im};
        }
        const cpx<T> g0 = u[0] * h0[0] + u[1] * h0[1] + u[2] * h0[2];
        const cpx<T> g1 = u[0] * h1[0] + u[1] * h1[1] + u[2] * h1[2];
        acc[a] += coef * g0;
        acc[3 + a] += coef * g1;
        acc[6 + a] += coef * mulc(q0 == 0 ? g0 : g1, g0c);
        acc[9 + a] += coef * mulc(q0 == 0 ? g1 : g0, g1c);
    }
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

// All eight hops, one loop iteration each, sharing one code path (the loop is
// not unrolled so that the loads of later hops are not hoisted).  Spatial hops
// read `src` with sign 0, the forward / backward time hops with signs sf / sb
// (a two-field source then combines the two halves of a block vector).  Coefficients: -1/2 cs in space, -1/2 cf
// and -1/2 cb in time, times the boundary factor on a wrapping time hop.
template <typename T, class SRC>
__device__ __forceinline__ void hops8(cpx<T> (&acc)[12], const SRC& src, int sf, int sb,
                                      const Nbr& N, int s, const cpx<T>* __restrict__ W, int Vp,
                                      T cs, T cf, T cb, int bc, bool space = true) {
    const T h = T(-0.5);
    const T ctf = h * cf * (N.wf ? T(bc) : T(1));
    const T ctb = h * cb * (N.wb ? T(bc) : T(1));
#pragma unroll 1
    for (int i = space ? 0 : 6; i < 8; ++i) {
        const int nu = i >> 1;
        const bool fwd = (i & 1) == 0;
        const int nf = nu == 0 ? N.f[0] : nu == 1 ? N.f[1] : nu == 2 ? N.f[2] : N.f[3];
        const int nbk = nu == 0 ? N.b[0] : nu == 1 ? N.b[1] : nu == 2 ? N.b[2] : N.b[3];
        const int n = fwd ? nf : nbk;
        const int ls = fwd ? s : nbk;
        const T coef = (nu < 3) ? h * cs : (fwd ? ctf : ctb);
        const int sg = (nu < 3) ? 0 : (fwd ? sf : sb);
        hop(acc, src, sg, n, i, W, ls, Vp, coef);
    }
}

__device__ __forceinline__ int xcd_group(int bid, int nb) {
    // blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of site groups (nb is a multiple of 8)
    return (bid & 7) * (nb >> 3) + (bid >> 3);
}

// ---------------------------------------------------------------------------
// standalone operator
// ---------------------------------------------------------------------------
template <typename T, int OP>
__global__ __launch_bounds__(256) void apply_op_kernel(Geom g, const double* __restrict__ emu,
                                                       const cpx<T>* __restrict__ U,
                                                       const cpx<T>* __restrict__ dU, T mdiag,
                                                       const cpx<T>* __restrict__ in,
                                                       cpx<T>* __restrict__ out, int ngroups) {
    const int rhs = blockIdx.y;
    const int grp = xcd_group(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    const int s = grp * 64 + (threadIdx.x & 63);
    if (grp >= ngroups || s >= g.V) return;
    const int Vp = g.Vp;
    const size_t roff = (size_t)rhs * 12 * Vp;
    const T ep = T(emu[2 * rhs]), em = T(emu[2 * rhs + 1]);
    Lin3<T> P{in + roff, nullptr, nullptr, {}, {}, {}, 0, Vp};
    const Nbr N = neighbours(g, s);
    cpx<T> acc[12];
    if constexpr (OP == 0 || OP == 1) {          // H or Dw
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = mdiag * P(c, s);
        hops8(acc, P, 0, 0, N, s, U, Vp, T(1), ep, em, g.bc_t);
    } else if constexpr (OP == 2) {             // dH/dmu: time hops, e^{mu} and -e^{-mu}
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
        hops8(acc, P, 0, 0, N, s, U, Vp, T(0), ep, -em, g.bc_t, false);
    } else {                                    // dH/dt along dU: hops with dU, no mass term
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
        hops8(acc, P, 0, 0, N, s, dU, Vp, T(1), ep, em, g.bc_t);
    }
    cpx<T>* o = out + roff;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        cpx<T> v = acc[c];
        if (OP != 1 && c >= 6) v = -v;          // gamma5
        o[(size_t)c * Vp + s] = v;
    }
}

template <typename T>
void launch_apply_op(const Geom& g, int op, int nrhs, const double* d_emu, const cpx<T>* U,
                     const cpx<T>* dU, double m_diag, const cpx<T>* in, cpx<T>* out, hipStream_t s) {
    const int ngroups = (g.V + 63) / 64;
    const int nb = ((ngroups + 3) / 4 + 7) / 8 * 8;
    dim3 grid(nb, nrhs), block(256);
    const T md = T(m_diag);
    switch (op) {
        case 0: apply_op_kernel<T, 0><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups); break;
        case 1: apply_op_kernel<T, 1><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups); break;
        case 2: apply_op_kernel<T, 2><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups); break;
        default: apply_op_kernel<T, 3><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups); break;
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
// fused two-sided Lanczos step
//
// Step j (0-based) forms the next unnormalised Lanczos vectors
//     vhat = av X_v + bv Y_v + cv Z_v,   what = aw X_w + bw Y_w + cw Z_w
// (X = A v_j, Y = v_j, Z = v_{j-1}, all unnormalised, the coefficients fold
// in the normalisations) at every site and, because the stencil needs them,
// at the eight neighbours; it writes vhat, A vhat, what, A^dag what and the
// block partial sums of
//     omega = what^dag vhat,  gamma = what^dag A vhat,  p = x^dag vhat_top,
//     |vhat|^2, |what|^2.
// The last block to finish sums the partials in a fixed order and advances the
// recurrence: delta = sqrt|omega|, beta = omega/delta, alpha = gamma/omega
// (= w^dag A v for the normalised vectors), so each step costs one launch and
// one grid-wide reduction.
//
// Work split: a block is NK waves over the same 64 sites, wave = output kind.
//   DIR 0 (A = H):                kind 0 = H vhat,  kind 1 = H^dag what
//   DIR 1/2 (A = B = [[H, dH], [0, H]], B^dag = [[H^dag, 0], [dH^dag, H^dag]]):
//     kind 0 = H vt + dH vb,  kind 1 = H vb,  kind 2 = H^dag wt,  kind 3 = dH^dag wt + H^dag wb
// with H^dag = H(-mu); for d/dmu, dH only has time hops (e^{mu}, -e^{-mu}) and
// dH^dag = -dH/dmu(-mu) (time hops -e^{-mu}, e^{mu}); for a link direction,
// dH is the hopping term with links dU and dH^dag that with dU at -mu.
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__global__ __launch_bounds__(256) void tsl_step_kernel(Geom g, StepPtrs p, const cpx<T>* __restrict__ U,
                                                       const cpx<T>* __restrict__ dU, T mdiag,
                                                       TslState* __restrict__ st, TslCoeffs co,
                                                       double* __restrict__ partials,
                                                       unsigned* __restrict__ counters, int j, double tau,
                                                       int nt, int ngroups) {
    constexpr int NK = (DIR == 0) ? 2 : 4;
    __shared__ double lds[16 * 8];
    __shared__ int am_last;
    const int rhs = blockIdx.y;
    TslState* S = st + rhs;
    if (S->flag) return;   // uniform over the grid: breakdown in an earlier step
    const int Vp = g.Vp;
    const int kind = threadIdx.x >> 6;
    const int grp = xcd_group(blockIdx.x, gridDim.x);
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
    const cpx<T> ca = cast<T>(vside ? S->av : S->aw);
    const cpx<T> cb_ = cast<T>(vside ? S->bv : S->bw);
    const cpx<T> cc = cast<T>(vside ? S->cv : S->cw);
    const cpx<T>* X = vside ? (const cpx<T>*)p.Xv + rhs * p.sXv : (const cpx<T>*)p.Xw + rhs * p.sXw;
    const cpx<T>* Y = vside ? (const cpx<T>*)p.Yv + rhs * p.sYv : (const cpx<T>*)p.Yw + rhs * p.sYw;
    const cpx<T>* Z = vside ? (const cpx<T>*)p.Zv + rhs * p.sZv : (const cpx<T>*)p.Zw + rhs * p.sZw;
    const Lin3<T> P{X + hp * HALF, Y + hp * HALF, Z + hp * HALF, ca, cb_, cc, nt, Vp};
    const Lin3<T> Q{X + hq * HALF, Y + hq * HALF, Z + hq * HALF, ca, cb_, cc, nt, Vp};
    const T cf = vside ? ep : em, cbk = vside ? em : ep;

    double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (active) {
        const Nbr N = neighbours(g, s);
        cpx<T> acc[12];
        cpx<T>* oV = vside ? (cpx<T>*)p.outV + rhs * p.sV : (cpx<T>*)p.outW + rhs * p.sW;
        oV += hp * HALF;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cpx<T> v = P(c, s);
            oV[(size_t)c * Vp + s] = v;
            acc[c] = mdiag * v;
        }
        const Src2<T> pq{P, Q};
        hops8(acc, pq, sf, sb, N, s, U, Vp, T(1), cf, cbk, g.bc_t);
        if (DIR == 2 && sec) hops8(acc, Q, 0, 0, N, s, dU, Vp, T(1), cf, cbk, g.bc_t);
        cpx<T>* oA = vside ? (cpx<T>*)p.outU + rhs * p.sU : (cpx<T>*)p.outZ + rhs * p.sZ;
        oA += hp * HALF;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            if (c >= 6) acc[c] = -acc[c];   // gamma5
            oA[(size_t)c * Vp + s] = acc[c];
        }
        // reduction terms
        if (vside) {
            const cpx<T>* Xw = (const cpx<T>*)p.Xw + rhs * p.sXw + hp * HALF;
            const cpx<T>* Yw = (const cpx<T>*)p.Yw + rhs * p.sYw + hp * HALF;
            const cpx<T>* Zw = (const cpx<T>*)p.Zw + rhs * p.sZw + hp * HALF;
            const Lin3<T> Wc{Xw, Yw, Zw, cast<T>(S->aw), cast<T>(S->bw), cast<T>(S->cw), nt, Vp};
            const cpx<T>* xp = (hp == 0 && p.xproj) ? (const cpx<T>*)p.xproj + rhs * p.sx : nullptr;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const c64 w = cast<double>(Wc(c, s));
                const c64 v = cast<double>(P(c, s));
                const c64 a = cast<double>(acc[c]);
                const c64 om = cdot(w, v), ga = cdot(w, a);
                part[0] += om.re; part[1] += om.im;
                part[2] += ga.re; part[3] += ga.im;
                part[6] += norm2(v);
                if (xp) {
                    const c64 pr = cdot(cast<double>(xp[(size_t)c * Vp + s]), v);
                    part[4] += pr.re; part[5] += pr.im;
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) part[7] += norm2(cast<double>(P(c, s)));
        }
    }

    block_reduce<8>(part, lds);
    const int nb = gridDim.x;
    if (threadIdx.x == 0) {
        double* dst = partials + ((size_t)rhs * nb + blockIdx.x) * 8;
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
    const double delta = (j == 0) ? sqrt(nv) : sqrt(aom);
    const c64 beta = (1.0 / delta) * omega;
    const c64 alpha = cdiv(gam, omega);
    co.alpha[ci] = alpha;
    co.beta[ci] = beta;
    co.delta[ci] = c64{delta, 0.0};
    co.proj[ci] = (1.0 / delta) * pr;
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
void launch_tsl_step(const Geom& g, int dir, int nrhs, int nterms, const StepPtrs& p,
                     const cpx<T>* U, const cpx<T>* dU, double m_diag, TslState* st,
                     TslCoeffs co, double* partials, unsigned* counters, int j, double tau,
                     hipStream_t s) {
    const int ngroups = (g.V + 63) / 64;
    const int nb = (ngroups + 7) / 8 * 8;
    dim3 grid(nb, nrhs);
    const T md = T(m_diag);
    if (dir == 0)
        tsl_step_kernel<T, 0><<<grid, dim3(128), 0, s>>>(g, p, U, dU, md, st, co, partials, counters, j, tau, nterms, ngroups);
    else if (dir == 1)
        tsl_step_kernel<T, 1><<<grid, dim3(256), 0, s>>>(g, p, U, dU, md, st, co, partials, counters, j, tau, nterms, ngroups);
    else
        tsl_step_kernel<T, 2><<<grid, dim3(256), 0, s>>>(g, p, U, dU, md, st, co, partials, counters, j, tau, nterms, ngroups);
}
template void launch_tsl_step<double>(const Geom&, int, int, int, const StepPtrs&, const c64*, const c64*,
                                      double, TslState*, TslCoeffs, double*, unsigned*, int, double, hipStream_t);
template void launch_tsl_step<float>(const Geom&, int, int, int, const StepPtrs&, const c32*, const c32*,
                                     double, TslState*, TslCoeffs, double*, unsigned*, int, double, hipStream_t);

}  // namespace ovd
