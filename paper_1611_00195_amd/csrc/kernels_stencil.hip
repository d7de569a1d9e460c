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
#include <type_traits>

#include "ovd_internal.h"

// scheduling fence between the hops of a site (limits how far the compiler
// hoists the next hop's loads, and so the register count); empty = none
#ifndef OVD_HOP_FENCE
#define OVD_HOP_FENCE
#endif

// scheduling fence between the two inputs of a paired hop; empty = none
#ifndef OVD_PAIR_FENCE
#define OVD_PAIR_FENCE
#endif

// scheduling fence between the hops of the sequential form (without it the
// compiler hoists the loads of all eight hops and spills); empty = none
#ifndef OVD_SEQ_FENCE
#define OVD_SEQ_FENCE __builtin_amdgcn_sched_barrier(0)
#endif

// scheduling fence between the hops of the time-marching form; empty = none
#ifndef OVD_MARCH_FENCE
#define OVD_MARCH_FENCE __builtin_amdgcn_sched_barrier(0)
#endif

// occupancy hint for the stencil kernels (waves per SIMD), by precision T;
// empty = compiler's choice
#ifndef OVD_OCC
#define OVD_OCC(T)
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

// ---------------------------------------------------------------------------
// Compile-time hops.  The same spin table as kHop, known to the compiler, so
// that the constants of each hop fold into sign flips and re/im swaps (no
// selects), with the field and link addresses as a uniform base plus a 32-bit
// per-lane byte offset (16 bytes per site in every plane, in both precisions).
// ---------------------------------------------------------------------------
struct HopC {
    int p3, f0, f1, q0, g0, g1;
};
constexpr HopC kHopCT[8] = {{1, F_PI, F_PI, 1, F_MI, F_MI}, {1, F_MI, F_MI, 1, F_PI, F_PI},
                            {1, F_P1, F_M1, 1, F_M1, F_P1}, {1, F_M1, F_P1, 1, F_P1, F_M1},
                            {0, F_PI, F_MI, 0, F_MI, F_PI}, {0, F_MI, F_PI, 0, F_PI, F_MI},
                            {0, F_M1, F_M1, 0, F_M1, F_M1}, {0, F_P1, F_P1, 0, F_P1, F_P1}};

template <int F, typename T>
__device__ __forceinline__ cpx<T> mulk(cpx<T> z) {
    if constexpr (F == F_P1) return z;
    else if constexpr (F == F_M1) return {-z.re, -z.im};
    else if constexpr (F == F_PI) return {-z.im, z.re};
    else return {z.im, -z.re};
}

typedef double ovd_d2 __attribute__((ext_vector_type(2)));
typedef float ovd_f4 __attribute__((ext_vector_type(4)));

// one 16-byte plane entry: one complex in FP64, two in FP32
template <typename T>
__device__ __forceinline__ void ld_plane(const char* __restrict__ base, uint32_t off, cpx<T>* dst) {
    if constexpr (sizeof(T) == 8) {
        const double2 d = *reinterpret_cast<const double2*>(base + off);
        dst[0] = {d.x, d.y};
    } else {
        const float4 t = *reinterpret_cast<const float4*>(base + off);
        dst[0] = {t.x, t.y};
        dst[1] = {t.z, t.w};
    }
}

template <typename T>
__device__ __forceinline__ void ld_site(const char* __restrict__ P, uint32_t Vp16, uint32_t off, cpx<T> (&v)[12]) {
    constexpr int per = sizeof(T) == 8 ? 1 : 2;
#pragma unroll
    for (int q = 0; q < 12 / per; ++q) ld_plane<T>(P + (size_t)q * Vp16, off, v + q * per);
}

// a site read once per launch (the x projection field), non-temporal
template <typename T>
__device__ __forceinline__ void ld_site_nt(const char* __restrict__ P, uint32_t Vp16, uint32_t off, cpx<T> (&v)[12]) {
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        if constexpr (sizeof(T) == 8) {
            const ovd_d2 d = __builtin_nontemporal_load(reinterpret_cast<const ovd_d2*>(P + (size_t)q * Vp16 + off));
            v[q] = {d.x, d.y};
        } else if (q < 6) {
            const ovd_f4 t = __builtin_nontemporal_load(reinterpret_cast<const ovd_f4*>(P + (size_t)q * Vp16 + off));
            v[2 * q] = {t.x, t.y};
            v[2 * q + 1] = {t.z, t.w};
        }
    }
}

template <typename T>
__device__ __forceinline__ void ld_link(const char* __restrict__ W, uint32_t Vp16, int nu, uint32_t off,
                                        cpx<T> (&u)[9]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int e = 0; e < 9; ++e) ld_plane<T>(W + (size_t)(nu * 9 + e) * Vp16, off, u + e);
    } else {
        cpx<T> t[10];
#pragma unroll
        for (int q = 0; q < 5; ++q) ld_plane<T>(W + (size_t)(nu * 5 + q) * Vp16, off, t + 2 * q);
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = t[e];
    }
}

// The stencil's outputs are written once and not read again by the launch:
// non-temporal stores keep them from displacing the neighbour planes and
// links that the launch still reuses from the L2.
template <typename T>
__device__ __forceinline__ void store_site(char* __restrict__ P, uint32_t Vp16, uint32_t off, const cpx<T> (&v)[12]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int c = 0; c < 12; ++c)
            __builtin_nontemporal_store(ovd_d2{v[c].re, v[c].im}, reinterpret_cast<ovd_d2*>(P + (size_t)c * Vp16 + off));
    } else {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            __builtin_nontemporal_store(ovd_f4{v[2 * q].re, v[2 * q].im, v[2 * q + 1].re, v[2 * q + 1].im},
                                        reinterpret_cast<ovd_f4*>(P + (size_t)q * Vp16 + off));
    }
}

// half spinor of hop I from a loaded site
template <typename T, int I>
__device__ __forceinline__ void proj_ct(const cpx<T> (&v)[12], cpx<T> (&h0)[3], cpx<T> (&h1)[3]) {
    constexpr HopC H = kHopCT[I];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> a = H.p3 ? v[9 + c] : v[6 + c];
        const cpx<T> b = H.p3 ? v[6 + c] : v[9 + c];
        h0[c] = v[c] + mulk<H.f0>(a);
        h1[c] = v[3 + c] + mulk<H.f1>(b);
    }
}

// acc += coef * reconstruct(W proj(P(neighbour))) for hop I
template <typename T, int I>
__device__ __forceinline__ void hop_ct(cpx<T> (&acc)[12], const char* __restrict__ P, const char* __restrict__ W,
                                       uint32_t Vp16, uint32_t noff, uint32_t loff, T coef) {
    constexpr HopC H = kHopCT[I];
    constexpr bool fwd = (I & 1) == 0;
    cpx<T> h0[3], h1[3];
    {
        cpx<T> v[12];
        ld_site<T>(P, Vp16, noff, v);
        proj_ct<T, I>(v, h0, h1);
    }
    cpx<T> u[9];
    ld_link<T>(W, Vp16, I >> 1, loff, u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = coef * h0[c];
        h1[c] = coef * h1[c];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // row a of U: U[a][b] = u[3a + b];  row a of U^dag: conj(U[b][a])
        const cpx<T> r0 = fwd ? u[3 * a] : conj(u[a]);
        const cpx<T> r1 = fwd ? u[3 * a + 1] : conj(u[3 + a]);
        const cpx<T> r2 = fwd ? u[3 * a + 2] : conj(u[6 + a]);
        const cpx<T> g0 = r0 * h0[0] + r1 * h0[1] + r2 * h0[2];
        const cpx<T> g1 = r0 * h1[0] + r1 * h1[1] + r2 * h1[2];
        acc[a] += g0;
        acc[3 + a] += g1;
        acc[6 + a] += mulk<H.g0>(H.q0 == 0 ? g0 : g1);
        acc[9 + a] += mulk<H.g1>(H.q0 == 0 ? g1 : g0);
    }
}

// The eight hops of field P (links W).  On the two time hops the field
// P + sf Q (forward) / P + sb Q (backward) is used instead, sf, sb in {0, +-1}
// (the mu derivative of the block matrix combines its two halves there);
// spatial hops get -1/2 cs, time hops -1/2 cf / -1/2 cb and the boundary
// factor.  With SPACE false only the time hops are applied.
template <bool SPACE, typename T>
__device__ __forceinline__ void hops(cpx<T> (&acc)[12], const cpx<T>* __restrict__ Pf, const cpx<T>* __restrict__ Qf,
                                     int sf, int sb, const Nbr& N, int s, const cpx<T>* __restrict__ Wf, int Vp,
                                     T cs, T cf, T cb, int bc) {
    const char* P = reinterpret_cast<const char*>(Pf);
    const char* Q = reinterpret_cast<const char*>(Qf);
    const char* W = reinterpret_cast<const char*>(Wf);
    const uint32_t Vp16 = (uint32_t)Vp * 16u;
    const uint32_t so = (uint32_t)s * 16u;
    const T h = T(-0.5);
    if constexpr (SPACE) {
        const T c = h * cs;
        hop_ct<T, 0>(acc, P, W, Vp16, (uint32_t)N.f[0] * 16u, so, c);
        OVD_HOP_FENCE;
        hop_ct<T, 1>(acc, P, W, Vp16, (uint32_t)N.b[0] * 16u, (uint32_t)N.b[0] * 16u, c);
        OVD_HOP_FENCE;
        hop_ct<T, 2>(acc, P, W, Vp16, (uint32_t)N.f[1] * 16u, so, c);
        OVD_HOP_FENCE;
        hop_ct<T, 3>(acc, P, W, Vp16, (uint32_t)N.b[1] * 16u, (uint32_t)N.b[1] * 16u, c);
        OVD_HOP_FENCE;
        hop_ct<T, 4>(acc, P, W, Vp16, (uint32_t)N.f[2] * 16u, so, c);
        OVD_HOP_FENCE;
        hop_ct<T, 5>(acc, P, W, Vp16, (uint32_t)N.b[2] * 16u, (uint32_t)N.b[2] * 16u, c);
        OVD_HOP_FENCE;
    }
    // time hops; the second field enters as a hop of its own (linear in the
    // field, and one field at a time keeps the register count of a single hop)
    const T ctf = h * cf * (N.wf ? T(bc) : T(1));
    const T ctb = h * cb * (N.wb ? T(bc) : T(1));
    const uint32_t of = (uint32_t)N.f[3] * 16u, ob = (uint32_t)N.b[3] * 16u;
    hop_ct<T, 6>(acc, P, W, Vp16, of, so, ctf);
    if (sf != 0) {   // uniform per wave
        OVD_HOP_FENCE;
        hop_ct<T, 6>(acc, Q, W, Vp16, of, so, T(sf) * ctf);
    }
    OVD_HOP_FENCE;
    hop_ct<T, 7>(acc, P, W, Vp16, ob, ob, ctb);
    if (sb != 0) {
        OVD_HOP_FENCE;
        hop_ct<T, 7>(acc, Q, W, Vp16, ob, ob, T(sb) * ctb);
    }
}

// Work decomposition over the 8 XCDs.  Blocks are dispatched round-robin over
// the XCDs (block b runs on XCD b % 8, in order of b / 8), and each XCD has its
// own 4 MB L2.  A stencil re-reads every field at the neighbouring sites, the
// furthest (the time neighbours) one time slice (Lx Ly Lz sites) away, so an
// XCD keeps its neighbour data in L2 only if it sweeps a compact piece of
// work in site order.  The (rhs, site group) work items are therefore split
// into 8 compact chunks, one per XCD:
//   map 0 (nrhs a multiple of 8): XCD x takes right-hand sides x m .. x m + m - 1
//                          (m = nrhs / 8) over the whole lattice, site group
//                          major, so those m share each link read;
//   map 1:                 XCD x takes a contiguous range of site groups for
//                          all right-hand sides (rhs innermost), so that the
//                          links and neighbours of a range stay in its L2.
// Measured on Dw.v at 14^4, map 0 wins from 16 sources up and map 1 below
// (the default); the autotuner of the library times both.
// nb (site groups per rhs, padded) is a multiple of 8.
struct Work {
    int rhs, grp;
};
__device__ __forceinline__ Work xcd_work(int bid, int nb, int nrhs, int map) {
    const int x = bid & 7, idx = bid >> 3;
    Work w;
    if (map == 0 && (nrhs & 7) == 0) {
        const int m = nrhs >> 3;
        w.grp = idx / m;
        w.rhs = x * m + idx % m;
    } else {
        const int i = x * (nb * nrhs / 8) + idx;
        w.grp = i / nrhs;
        w.rhs = i % nrhs;
    }
    return w;
}

// GPB site groups (of 64) per block: DIR 0 has one pair per site (GPB waves),
// DIR 1/2 two pairs per site (GPB groups x (v, w) waves)
// GPB == PLANE_GPB: one block per (xy-plane, rhs, side) (DIR 0: (xy-plane,
// rhs)), thread t at site t of the plane (Lx Ly <= 256), the plane's two input
// fields staged in LDS for the x and y hops.
constexpr int PLANE_GPB = 8;

template <typename T, int I, int DIR, typename LoadA, typename LoadB>
__device__ __forceinline__ void pair_hop(cpx<T> (&accA)[12], cpx<T> (&accB)[12], LoadA loadA, LoadB loadB,
                                         const char* __restrict__ W, const char* __restrict__ W2, uint32_t Vp16,
                                         uint32_t loff, T cA, T cB, T xAB, T xBA, bool vside);

// ---------------------------------------------------------------------------
// standalone operator
// ---------------------------------------------------------------------------
template <typename T, int OP, int GPB>
__global__ __launch_bounds__(256) OVD_OCC(T) void apply_op_kernel(Geom g, const double* __restrict__ emu,
                                                       const cpx<T>* __restrict__ U,
                                                       const cpx<T>* __restrict__ dU, T mdiag,
                                                       const cpx<T>* __restrict__ in,
                                                       cpx<T>* __restrict__ out, int ngroups, int nrhs, int map) {
    const Work w = xcd_work(blockIdx.x, gridDim.x / nrhs, nrhs, map);
    const int rhs = w.rhs;
    const int grp = w.grp * GPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
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
        hops<true>(acc, P, P, 0, 0, N, s, U, Vp, T(1), ep, em, g.bc_t);
    } else if constexpr (OP == 2) {             // dH/dmu: time hops, e^{mu} and -e^{-mu}
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
        hops<false>(acc, P, P, 0, 0, N, s, U, Vp, T(0), ep, -em, g.bc_t);
    } else {                                    // dH/dt along dU: hops with dU, no mass term
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
        hops<true>(acc, P, P, 0, 0, N, s, dU, Vp, T(1), ep, em, g.bc_t);
    }
    if (OP != 1) {
#pragma unroll
        for (int c = 6; c < 12; ++c) acc[c] = -acc[c];   // gamma5
    }
    store12(out + roff, s, Vp, acc);
}

// H or Dw on two right-hand sides per thread (OP 0 or 1): the link of every
// hop is loaded once for both, through the paired hops of the Lanczos stencil
// (pair r holds right-hand sides 2 r and 2 r + 1, each with its own mu).
template <typename T, int DIR, bool PLANE>
__device__ __forceinline__ void pair_hops(cpx<T> (&accA)[12], cpx<T> (&accB)[12], const cpx<T>* Af,
                                          const cpx<T>* Bf, const cpx<T>* Wf, const cpx<T>* W2f, const Nbr& N, int s,
                                          int Vp, T cfA, T cbA, T cfB, T cbB, T xfAB, T xbAB, T xfBA, T xbBA, int bc,
                                          bool vside);

template <typename T, int OP, int GPB>
__global__ __launch_bounds__(256) OVD_OCC(T) void apply_op_pair_kernel(Geom g, const double* __restrict__ emu,
                                                            const cpx<T>* __restrict__ U, T mdiag,
                                                            const cpx<T>* __restrict__ in,
                                                            cpx<T>* __restrict__ out, int ngroups, int npairs,
                                                            int map) {
    static_assert(OP == 0 || OP == 1, "paired form: H or Dw");
    const Work w = xcd_work(blockIdx.x, gridDim.x / npairs, npairs, map);
    const int r0 = 2 * w.rhs;
    const int grp = w.grp * GPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int s = grp * 64 + (threadIdx.x & 63);
    if (grp >= ngroups || s >= g.V) return;
    const int Vp = g.Vp;
    const cpx<T>* A = in + (size_t)r0 * 12 * Vp;
    const cpx<T>* B = A + (size_t)12 * Vp;
    const T epA = T(emu[2 * r0]), emA = T(emu[2 * r0 + 1]);
    const T epB = T(emu[2 * r0 + 2]), emB = T(emu[2 * r0 + 3]);
    const Nbr N = neighbours(g, s);
    cpx<T> accA[12], accB[12];
    load12(A, s, Vp, accA);
    load12(B, s, Vp, accB);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        accA[c] = mdiag * accA[c];
        accB[c] = mdiag * accB[c];
    }
    const T z = T(0);
    pair_hops<T, 0, false>(accA, accB, A, B, U, U, N, s, Vp, epA, emA, epB, emB, z, z, z, z, g.bc_t, true);
    if (OP == 0) {
#pragma unroll
        for (int c = 6; c < 12; ++c) {   // gamma5
            accA[c] = -accA[c];
            accB[c] = -accB[c];
        }
    }
    store12(out + (size_t)r0 * 12 * Vp, s, Vp, accA);
    store12(out + (size_t)(r0 + 1) * 12 * Vp, s, Vp, accB);
}

// H or Dw on two right-hand sides per thread with the xy-plane in LDS: one
// block per (xy-plane, pair), thread t at site t of the plane (Lx Ly <= 256).
// The block stages the plane's two input fields in LDS; the x and y hops read
// their neighbours there and the z and t hops from memory.  Hops, order and
// arithmetic are those of apply_op_pair_kernel, so the outputs are the same.
template <typename T, int OP>
__global__ __launch_bounds__(256) OVD_OCC(T) void apply_op_plane_kernel(Geom g, const double* __restrict__ emu,
                                                             const cpx<T>* __restrict__ U, T mdiag,
                                                             const cpx<T>* __restrict__ in,
                                                             cpx<T>* __restrict__ out, int npairs, int map) {
    static_assert(OP == 0 || OP == 1, "paired form: H or Dw");
    constexpr int NQ = sizeof(T) == 8 ? 12 : 6;   // 16-byte entries per site
    extern __shared__ float4 plane_lds[];          // [field 2][NQ][P]
    const int nb = (int)(gridDim.x / (unsigned)npairs);
    const Work w = xcd_work((int)blockIdx.x, nb, npairs, map);
    const int r0 = 2 * w.rhs;
    const int Lx = g.L[0], Ly = g.L[1], P = Lx * Ly, Vp = g.Vp;
    const int tid = (int)threadIdx.x;
    const bool act = w.grp < g.V / P && tid < P;
    const int s = w.grp * P + tid;
    const cpx<T>* A = in + (size_t)r0 * 12 * Vp;
    const cpx<T>* B = A + (size_t)12 * Vp;
    auto lds_at = [&](int f, int q, int t) -> float4& { return plane_lds[((size_t)f * NQ + q) * P + t]; };
    auto to_lds = [&](int f, int t, const cpx<T> (&v)[12]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float4 e;
            if constexpr (sizeof(T) == 8) {
                const double2 d{(double)v[q].re, (double)v[q].im};
                e = *reinterpret_cast<const float4*>(&d);
            } else {
                e = float4{(float)v[2 * q].re, (float)v[2 * q].im, (float)v[2 * q + 1].re, (float)v[2 * q + 1].im};
            }
            lds_at(f, q, t) = e;
        }
    };
    auto from_lds = [&](int f, int t, cpx<T> (&v)[12]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float4 e = lds_at(f, q, t);
            if constexpr (sizeof(T) == 8) {
                const double2 d = *reinterpret_cast<const double2*>(&e);
                v[q] = cpx<T>{(T)d.x, (T)d.y};
            } else {
                v[2 * q] = cpx<T>{(T)e.x, (T)e.y};
                v[2 * q + 1] = cpx<T>{(T)e.z, (T)e.w};
            }
        }
    };
    cpx<T> accA[12], accB[12];
    if (act) {
        load12(A, s, Vp, accA);
        to_lds(0, tid, accA);
        load12(B, s, Vp, accB);
        to_lds(1, tid, accB);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            accA[c] = mdiag * accA[c];
            accB[c] = mdiag * accB[c];
        }
    }
    __syncthreads();   // the plane's inputs are in LDS (the block's only barrier)
    if (!act) return;
    const T epA = T(emu[2 * r0]), emA = T(emu[2 * r0 + 1]);
    const T epB = T(emu[2 * r0 + 2]), emB = T(emu[2 * r0 + 3]);
    const Nbr N = neighbours(g, s);
    const char* W = reinterpret_cast<const char*>(U);
    const uint32_t Vp16 = (uint32_t)Vp * 16u;
    const int x = tid % Lx, y = tid / Lx;
    const int txf = y * Lx + (x == Lx - 1 ? 0 : x + 1), txb = y * Lx + (x == 0 ? Lx - 1 : x - 1);
    const int tyf = (y == Ly - 1 ? 0 : y + 1) * Lx + x, tyb = (y == 0 ? Ly - 1 : y - 1) * Lx + x;
    const T h = T(-0.5), z = T(0);
#define OVD_PO(I, TN, LS)                                                                                  \
    pair_hop<T, I, 0>(                                                                                     \
        accA, accB, [&](cpx<T>(&v)[12]) { from_lds(0, TN, v); }, [&](cpx<T>(&v)[12]) { from_lds(1, TN, v); }, \
        W, W, Vp16, (uint32_t)(LS) * 16u, h, h, z, z, true);                                               \
    OVD_HOP_FENCE;
    OVD_PO(0, txf, s)
    OVD_PO(1, txb, N.b[0])
    OVD_PO(2, tyf, s)
    OVD_PO(3, tyb, N.b[1])
#undef OVD_PO
    pair_hops<T, 0, true>(accA, accB, A, B, U, U, N, s, Vp, epA, emA, epB, emB, z, z, z, z, g.bc_t, true);
    if (OP == 0) {
#pragma unroll
        for (int c = 6; c < 12; ++c) {   // gamma5
            accA[c] = -accA[c];
            accB[c] = -accB[c];
        }
    }
    store12(out + (size_t)r0 * 12 * Vp, s, Vp, accA);
    store12(out + (size_t)(r0 + 1) * 12 * Vp, s, Vp, accB);
}

template <typename T, int OP>
static void launch_apply_op_v(const Geom& g, int nrhs, const double* d_emu, const cpx<T>* U, const cpx<T>* dU, T md,
                              const cpx<T>* in, cpx<T>* out, StencilVariant v, hipStream_t s) {
    const int ngroups = (g.V + 63) / 64;
    const int gpb = v.gpb == 2 ? 2 : 4;
    const int nq = ((ngroups + gpb - 1) / gpb + 7) / 8 * 8;   // blocks of gpb site groups, padded to 8
    if constexpr (OP == 0 || OP == 1) {
        if (v.rp == 2 && nrhs % 2 == 0 && v.gpb == PLANE_GPB && tsl_plane_ok(g)) {
            const int np = nrhs / 2;
            const int map = (v.map == 0 && np % 8 != 0) ? 1 : v.map;
            const int planes = g.V / (g.L[0] * g.L[1]);
            static bool attr = false;
            if (!attr) {
                (void)hipFuncSetAttribute((const void*)apply_op_plane_kernel<T, OP>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
                attr = true;
            }
            apply_op_plane_kernel<T, OP><<<dim3((planes + 7) / 8 * 8 * np), dim3(256),
                                           (size_t)2 * 12 * g.L[0] * g.L[1] * sizeof(cpx<T>), s>>>(
                g, d_emu, U, md, in, out, np, map);
            return;
        }
        if (v.rp == 2 && nrhs % 2 == 0) {
            const int np = nrhs / 2;
            const int map = (v.map == 0 && np % 8 != 0) ? 1 : v.map;
            dim3 grid(nq * np), block(64 * gpb);
            if (gpb == 2)
                apply_op_pair_kernel<T, OP, 2><<<grid, block, 0, s>>>(g, d_emu, U, md, in, out, ngroups, np, map);
            else
                apply_op_pair_kernel<T, OP, 4><<<grid, block, 0, s>>>(g, d_emu, U, md, in, out, ngroups, np, map);
            return;
        }
    }
    dim3 grid(nq * nrhs), block(64 * gpb);
    if (gpb == 2)
        apply_op_kernel<T, OP, 2><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups, nrhs, v.map);
    else
        apply_op_kernel<T, OP, 4><<<grid, block, 0, s>>>(g, d_emu, U, dU, md, in, out, ngroups, nrhs, v.map);
}

template <typename T>
void launch_apply_op(const Geom& g, int op, int nrhs, const double* d_emu, const cpx<T>* U,
                     const cpx<T>* dU, double m_diag, const cpx<T>* in, cpx<T>* out, hipStream_t s,
                     StencilVariant v) {
    if (v.map < 0) v.map = default_map(nrhs);
    if (v.gpb <= 0) v.gpb = 4;
    const T md = T(m_diag);
    switch (op) {
        case 0: launch_apply_op_v<T, 0>(g, nrhs, d_emu, U, dU, md, in, out, v, s); break;
        case 1: launch_apply_op_v<T, 1>(g, nrhs, d_emu, U, dU, md, in, out, v, s); break;
        case 2: launch_apply_op_v<T, 2>(g, nrhs, d_emu, U, dU, md, in, out, v, s); break;
        default: launch_apply_op_v<T, 3>(g, nrhs, d_emu, U, dU, md, in, out, v, s); break;
    }
}
template void launch_apply_op<double>(const Geom&, int, int, const double*, const c64*, const c64*, double,
                                      const c64*, c64*, hipStream_t, StencilVariant);
template void launch_apply_op<float>(const Geom&, int, int, const double*, const c32*, const c32*, double,
                                     const c32*, c32*, hipStream_t, StencilVariant);

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
// The arithmetic is FP64 for either storage type, with the single rounding at
// the store: FP32 vectors then follow the FP64 recurrence coefficients of T_k
// up to that one rounding, instead of coefficients rounded to FP32 and three
// FP32 products and sums.  The kernel is HBM-bound; FP64 costs nothing here.
// ---------------------------------------------------------------------------
// The update streams each element once: non-temporal loads and stores (the
// fields are far larger than the L2, and the hint keeps them from evicting
// lines still in use).
typedef float ovd_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ c64 ld_nt(const cpx<double>* p) {
    const ovd_d2 v = __builtin_nontemporal_load(reinterpret_cast<const ovd_d2*>(p));
    return c64{v.x, v.y};
}
__device__ __forceinline__ c64 ld_nt(const cpx<float>* p) {
    const ovd_f2 v = __builtin_nontemporal_load(reinterpret_cast<const ovd_f2*>(p));
    return c64{(double)v.x, (double)v.y};
}
__device__ __forceinline__ void st_nt(cpx<double>* p, c64 r) {
    __builtin_nontemporal_store(ovd_d2{r.re, r.im}, reinterpret_cast<ovd_d2*>(p));
}
__device__ __forceinline__ void st_nt(cpx<float>* p, c64 r) {
    __builtin_nontemporal_store(ovd_f2{(float)r.re, (float)r.im}, reinterpret_cast<ovd_f2*>(p));
}

template <typename T, int NT>
__device__ __forceinline__ void tsl_update_body(const int bx, const int nbx, const int rhs, const bool vside,
                                                const StepPtrs& p, long long n_elem,
                                                const TslState* __restrict__ st) {
    const TslState* S = st + rhs;
    if (S->flag) return;
    const c64 a = vside ? S->av : S->aw;
    const c64 b = vside ? S->bv : S->bw;
    const c64 c = vside ? S->cv : S->cw;
    const cpx<T>* X = vside ? (const cpx<T>*)p.Xv + rhs * p.sXv : (const cpx<T>*)p.Xw + rhs * p.sXw;
    const cpx<T>* Y = vside ? (const cpx<T>*)p.Yv + rhs * p.sYv : (const cpx<T>*)p.Yw + rhs * p.sYw;
    const cpx<T>* Z = vside ? (const cpx<T>*)p.Zv + rhs * p.sZv : (const cpx<T>*)p.Zw + rhs * p.sZw;
    cpx<T>* O = vside ? (cpx<T>*)p.outV + rhs * p.sV : (cpx<T>*)p.outW + rhs * p.sW;
    const long long stride = (long long)nbx * blockDim.x;
    for (long long e = (long long)bx * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        c64 r = a * ld_nt(X + e) + b * ld_nt(Y + e);
        if constexpr (NT == 3) r += c * ld_nt(Z + e);
        st_nt(O + e, r);
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(256) void tsl_update_kernel(StepPtrs p, long long n_elem,
                                                         const TslState* __restrict__ st) {
    tsl_update_body<T, NT>((int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y, blockIdx.z == 0, p, n_elem, st);
}

// The update of several lattices in one launch: x ranges of blocks per
// lattice (as in its own launch), y the rhs (blocks past a lattice's count
// return), z the side.
template <typename T, int NT>
__global__ __launch_bounds__(256) void tsl_update_multi_kernel(const TslSegment* __restrict__ seg, int nseg) {
    int i = 0;
    for (int q = 1; q < nseg; ++q)
        if ((int)blockIdx.x >= seg[q].ublock0) i = q;
    const TslSegment& S = seg[i];
    if ((int)blockIdx.y >= S.nrhs) return;
    tsl_update_body<T, NT>((int)blockIdx.x - S.ublock0, S.unblocks, (int)blockIdx.y, blockIdx.z == 0, S.p, S.fsz,
                           S.st);
}

// ---------------------------------------------------------------------------
// Lanczos step, part 2: stencil and inner products.
//
// Reads the new unnormalised vectors vhat, what, writes A vhat and A^dag what
// and the block partial sums of
//     omega = what^dag vhat,  gamma = what^dag A vhat,  p = x^dag vhat_top,
//     |vhat|^2, |what|^2.
// The last block to finish sums the partials in a fixed order and advances the
// recurrence: delta = sqrt|omega|, beta = omega/delta, alpha = gamma/omega
// (= w^dag A v for the normalised vectors), and the coefficients of the next
// update.  One grid-wide reduction per Lanczos step, no host round trip.
//
// Each thread computes two output fields at one site from two input fields
// ("pair"), loading every link once for both and every neighbour of each
// input once:
//   DIR 0 (A = H):  A = vhat -> H vhat,  B = what -> H^dag what  (one wave each);
//   DIR 1/2 (A = B = [[H, dH], [0, H]]):
//     v wave: A = vt, B = vb;  top = H vt + dH vb,  bottom = H vb;
//     w wave: A = wt, B = wb;  top = H^dag wt,      bottom = dH^dag wt + H^dag wb,
// with H^dag = H(-mu).  For d/dmu, dH has only time hops, with the factors
// (+e^{mu}, -e^{-mu}) where H has (e^{mu}, e^{-mu}), and dH^dag those of
// -dH/dmu(-mu); by linearity these enter as "mix" terms of the time hops
// (top += x_AB B, bottom += x_BA A before the link multiply).  For a link
// direction, dH is the hopping term with links dU (dH^dag: dU at -mu).
// A block is 4 waves: (v, w) on site group 2b and (v, w) on group 2b + 1.
// ---------------------------------------------------------------------------

// acc += reconstruct_I(g0, g1): spins 0, 1 = g0, g1; spins 2, 3 from the hop table
template <typename T, int I>
__device__ __forceinline__ void recon_add(cpx<T> (&acc)[12], const cpx<T> (&g0)[3], const cpx<T> (&g1)[3]) {
    constexpr HopC H = kHopCT[I];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] += g0[a];
        acc[3 + a] += g1[a];
        acc[6 + a] += mulk<H.g0>(H.q0 == 0 ? g0[a] : g1[a]);
        acc[9 + a] += mulk<H.g1>(H.q0 == 0 ? g1[a] : g0[a]);
    }
}

// g = U h (forward hop) or U^dag h (backward hop), h a half spinor (2 x 3 colours)
template <typename T, bool FWD>
__device__ __forceinline__ void link_mul(const cpx<T> (&u)[9], const cpx<T> (&h0)[3], const cpx<T> (&h1)[3],
                                         cpx<T> (&g0)[3], cpx<T> (&g1)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<T> r0 = FWD ? u[3 * a] : conj(u[a]);
        const cpx<T> r1 = FWD ? u[3 * a + 1] : conj(u[3 + a]);
        const cpx<T> r2 = FWD ? u[3 * a + 2] : conj(u[6 + a]);
        g0[a] = r0 * h0[0] + r1 * h0[1] + r2 * h0[2];
        g1[a] = r0 * h1[0] + r1 * h1[1] + r2 * h1[2];
    }
}

// Hop I of a pair.  cA, cB: hop factors of the two outputs; xAB, xBA: mix
// factors (time hops of the mu derivative, else 0); with DIR 2 the second
// link field W2 carries the derivative hop of B into top (v side) or of A into
// bottom (w side).
template <typename T, int I, int DIR, typename LoadA, typename LoadB>
__device__ __forceinline__ void pair_hop(cpx<T> (&accA)[12], cpx<T> (&accB)[12], LoadA loadA, LoadB loadB,
                                         const char* __restrict__ W, const char* __restrict__ W2, uint32_t Vp16,
                                         uint32_t loff, T cA, T cB, T xAB, T xBA, bool vside) {
    constexpr bool fwd = (I & 1) == 0;
    constexpr bool mix = (DIR == 1) && (I >= 6);
    cpx<T> u[9];
    ld_link<T>(W, Vp16, I >> 1, loff, u);
    cpx<T> a0[3], a1[3], b0[3], b1[3], g0[3], g1[3];
    {
        cpx<T> v[12];
        loadA(v);
        proj_ct<T, I>(v, a0, a1);
    }
    if constexpr (!mix) {
        // A and B independent: one input at a time (fewer live registers)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b0[c] = cA * a0[c];
            b1[c] = cA * a1[c];
        }
        link_mul<T, fwd>(u, b0, b1, g0, g1);
        recon_add<T, I>(accA, g0, g1);
        OVD_PAIR_FENCE;
        {
            cpx<T> v[12];
            loadB(v);
            proj_ct<T, I>(v, b0, b1);
        }
        if constexpr (DIR == 2) {
            // derivative hop with the second link field: B into top (v side), A into bottom (w side)
            cpx<T> w[9], d0[3], d1[3];
            ld_link<T>(W2, Vp16, I >> 1, loff, w);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                d0[c] = vside ? cA * b0[c] : cB * a0[c];
                d1[c] = vside ? cA * b1[c] : cB * a1[c];
            }
            link_mul<T, fwd>(w, d0, d1, g0, g1);
            if (vside) recon_add<T, I>(accA, g0, g1);
            else recon_add<T, I>(accB, g0, g1);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b0[c] = cB * b0[c];
            b1[c] = cB * b1[c];
        }
        link_mul<T, fwd>(u, b0, b1, g0, g1);
        recon_add<T, I>(accB, g0, g1);
    } else {
        // time hops of the mu derivative: top += x_AB B, bottom += x_BA A
        {
            cpx<T> v[12];
            loadB(v);
            proj_ct<T, I>(v, b0, b1);
        }
        cpx<T> h0[3], h1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c] = cA * a0[c] + (cA * xAB) * b0[c];
            h1[c] = cA * a1[c] + (cA * xAB) * b1[c];
        }
        link_mul<T, fwd>(u, h0, h1, g0, g1);
        recon_add<T, I>(accA, g0, g1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c] = cB * b0[c] + (cB * xBA) * a0[c];
            h1[c] = cB * b1[c] + (cB * xBA) * a1[c];
        }
        link_mul<T, fwd>(u, h0, h1, g0, g1);
        recon_add<T, I>(accB, g0, g1);
    }
}

template <typename T, int DIR, bool PLANE>
__device__ __forceinline__ void pair_hops(cpx<T> (&accA)[12], cpx<T> (&accB)[12], const cpx<T>* Af,
                                          const cpx<T>* Bf, const cpx<T>* Wf, const cpx<T>* W2f, const Nbr& N, int s,
                                          int Vp, T cfA, T cbA, T cfB, T cbB, T xfAB, T xbAB, T xfBA, T xbBA, int bc,
                                          bool vside) {
    const char* A = reinterpret_cast<const char*>(Af);
    const char* B = reinterpret_cast<const char*>(Bf);
    const char* W = reinterpret_cast<const char*>(Wf);
    const char* W2 = reinterpret_cast<const char*>(W2f);
    const uint32_t Vp16 = (uint32_t)Vp * 16u;
    const uint32_t so = (uint32_t)s * 16u;
    const T h = T(-0.5), z = T(0);
#define OVD_PH(I, NB, LS, CA, CB, XAB, XBA)                                                                    \
    {                                                                                                          \
        const uint32_t noff = (uint32_t)(NB) * 16u;                                                            \
        pair_hop<T, I, DIR>(                                                                                   \
            accA, accB, [&](cpx<T>(&v)[12]) { ld_site<T>(A, Vp16, noff, v); },                                 \
            [&](cpx<T>(&v)[12]) { ld_site<T>(B, Vp16, noff, v); }, W, W2, Vp16, (uint32_t)(LS) * 16u, CA, CB, \
            XAB, XBA, vside);                                                                                  \
    }                                                                                                          \
    OVD_HOP_FENCE;
    if constexpr (!PLANE) {   // x and y hops from memory (with a plane in LDS the caller has done them)
        OVD_PH(0, N.f[0], s, h, h, z, z)
        OVD_PH(1, N.b[0], N.b[0], h, h, z, z)
        OVD_PH(2, N.f[1], s, h, h, z, z)
        OVD_PH(3, N.b[1], N.b[1], h, h, z, z)
    }
    OVD_PH(4, N.f[2], s, h, h, z, z)
    OVD_PH(5, N.b[2], N.b[2], h, h, z, z)
    const T sf = N.wf ? T(bc) : T(1), sb = N.wb ? T(bc) : T(1);
    OVD_PH(6, N.f[3], s, h * cfA * sf, h * cfB * sf, xfAB, xfBA)
    OVD_PH(7, N.b[3], N.b[3], h * cbA * sb, h * cbB * sb, xbAB, xbBA)
#undef OVD_PH
    (void)so;
}

// One output of a pair, hop I ("sequential" form: the thread finishes one
// output before it starts the other, so only one 12-entry accumulator is live):
//   acc += recon(link * proj(c P(n) + c x Q(n)))
// where Q, the other input of the pair, enters only on the time hops of the mu
// derivative for the output that has them (MIX; x = its mix factor).
template <typename T, int I, bool MIX, typename LoadP, typename LoadQ>
__device__ __forceinline__ void single_hop(cpx<T> (&acc)[12], LoadP loadP, LoadQ loadQ, const char* __restrict__ W,
                                           uint32_t Vp16, uint32_t loff, T c, T x) {
    constexpr bool fwd = (I & 1) == 0;
    cpx<T> u[9];
    ld_link<T>(W, Vp16, I >> 1, loff, u);
    cpx<T> h0[3], h1[3], g0[3], g1[3];
    {
        cpx<T> v[12];
        loadP(v);
        proj_ct<T, I>(v, h0, h1);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h0[a] = c * h0[a];
        h1[a] = c * h1[a];
    }
    if constexpr (MIX) {
        cpx<T> v[12], q0[3], q1[3];
        loadQ(v);
        proj_ct<T, I>(v, q0, q1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0[a] += (c * x) * q0[a];
            h1[a] += (c * x) * q1[a];
        }
    }
    link_mul<T, fwd>(u, h0, h1, g0, g1);
    recon_add<T, I>(acc, g0, g1);
}

// The same pointer, opaque to the optimiser: the loads of the second pass of
// the sequential form are issued again instead of being forwarded from the
// first pass (which would keep all eight links live between the passes).
template <typename P>
__device__ __forceinline__ P opaque_ptr(P p) {
    asm volatile("" : "+s"(p));
    return p;
}

// All eight hops of one output (DIR 0 or 1): P the input of this output, Q the
// other input of the pair, cf/cb the forward/backward hop factors; USEQ: the
// output has the mix terms xf/xb on its time hops.
template <typename T, bool USEQ>
__device__ __forceinline__ void single_hops(cpx<T> (&acc)[12], const cpx<T>* Pf, const cpx<T>* Qf,
                                            const cpx<T>* Wf, const Nbr& N, int s, int Vp, T cf, T cb, T xf, T xb,
                                            int bc) {
    const char* P = reinterpret_cast<const char*>(Pf);
    const char* Q = reinterpret_cast<const char*>(Qf);
    const char* W = reinterpret_cast<const char*>(Wf);
    const uint32_t Vp16 = (uint32_t)Vp * 16u;
    const T h = T(-0.5), z = T(0);
#define OVD_SH(I, NB, LS, C, X)                                                                               \
    {                                                                                                         \
        const uint32_t noff = (uint32_t)(NB) * 16u;                                                           \
        single_hop<T, I, USEQ && (I >= 6)>(                                                                   \
            acc, [&](cpx<T>(&v)[12]) { ld_site<T>(P, Vp16, noff, v); },                                       \
            [&](cpx<T>(&v)[12]) { ld_site<T>(Q, Vp16, noff, v); }, W, Vp16, (uint32_t)(LS) * 16u, C, X);      \
    }                                                                                                         \
    OVD_SEQ_FENCE;
    OVD_SH(0, N.f[0], s, h, z)
    OVD_SH(1, N.b[0], N.b[0], h, z)
    OVD_SH(2, N.f[1], s, h, z)
    OVD_SH(3, N.b[1], N.b[1], h, z)
    OVD_SH(4, N.f[2], s, h, z)
    OVD_SH(5, N.b[2], N.b[2], h, z)
    const T sf = N.wf ? T(bc) : T(1), sb = N.wb ? T(bc) : T(1);
    OVD_SH(6, N.f[3], s, h * cf * sf, xf)
    OVD_SH(7, N.b[3], N.b[3], h * cb * sb, xb)
#undef OVD_SH
}

// partial sums of the step: 0,1 omega; 2,3 gamma; 4,5 p; 6 |vhat|^2; 7 |what|^2
template <typename T>
__device__ __forceinline__ void dot_acc(double* part, int i, const cpx<T> (&a)[12], const cpx<T> (&b)[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const c64 d = cdot(cast<double>(a[c]), cast<double>(b[c]));
        part[i] += d.re;
        part[i + 1] += d.im;
    }
}
template <typename T>
__device__ __forceinline__ void nrm_acc(double* part, int i, const cpx<T> (&a)[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) part[i] += norm2(cast<double>(a[c]));
}


// The end of a stencil block: its partial sums into the step's grid reduction,
// and in the last block of the rhs the step's scalars and the coefficients of
// the next update.
__device__ __forceinline__ void tsl_step_tail(double (&part)[8], double* lds, int* am_last, TslState* S,
                                              TslCoeffs co, double* __restrict__ partials,
                                              unsigned* __restrict__ counters, int rhs, int nb, int grp, int j,
                                              double tau) {
    // Grid reduction without a device-wide fence.  The block's partial sums are
    // stored with device-scope relaxed atomic stores, which are written through
    // to the level that all XCDs see; the wait for those stores to complete
    // orders them before the counter increment; the last block reads the
    // partials with device-scope loads from that same level.  A full fence
    // (__threadfence) here would write back and invalidate the XCD's L2 at the
    // end of every block, costing the stencil a third of its time.
    block_reduce<8>(part, lds);
    if (threadIdx.x == 0) {
        double* dst = partials + ((size_t)rhs * nb + grp) * 8;
        for (int i = 0; i < 8; ++i) __hip_atomic_store(dst + i, part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);   // the partials have reached the device-coherent level
        const unsigned prev = __hip_atomic_fetch_add(counters + rhs, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *am_last = (prev == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!*am_last) return;
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

// The body of one launch's block `bid` of `nblocks` (blocks per rhs = nblocks / nrhs);
// a standalone launch passes its own grid, a multi-lattice launch the block's
// place inside its lattice's range of blocks.
// FORM 0: paired (one thread computes both outputs of its pair, loading each
// link once for both); 1: sequential (one output after the other in the same
// thread, one accumulator live); 2: split (DIR 0 only: the two outputs of a
// site in the two waves of a (v, w) wave pair, twice the waves of the paired
// form for a launch too small to fill the GPU).
template <typename T, int DIR, int GPB, int FORM>
__device__ __forceinline__ void tsl_stencil_body(const int bid, const int nblocks, Geom g, StepPtrs p,
                                                 const cpx<T>* __restrict__ U, const cpx<T>* __restrict__ dU, T mdiag,
                                                 TslState* __restrict__ st, TslCoeffs co,
                                                 double* __restrict__ partials, unsigned* __restrict__ counters, int j,
                                                 double tau, int ngroups, int nrhs, int map) {
    constexpr bool PLANE = GPB == PLANE_GPB;
    constexpr bool SEQ = FORM != 0;              // the sequential body, whole or split over two waves
    constexpr bool SPLIT = FORM == 2;
    static_assert(!SEQ || (!PLANE && DIR != 2), "sequential form: DIR 0/1 without the plane in LDS");
    static_assert(!SPLIT || DIR == 0, "split form: DIR 0 only");
    constexpr int NQ = sizeof(T) == 8 ? 12 : 6;     // 16-byte entries per site
    extern __shared__ float4 plane_lds[];           // PLANE: [2][NQ][P]
    __shared__ double lds[16 * 8];
    __shared__ int am_last;
    const int nb = (int)((unsigned)nblocks / (unsigned)nrhs);   // blocks per rhs
    const Work wk = xcd_work(bid, nb, nrhs, map);
    const int rhs = wk.rhs;
    TslState* S = st + rhs;
    if (S->flag) return;   // uniform over the rhs: breakdown in an earlier step
    const int Vp = g.Vp;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int P = g.L[0] * g.L[1];
    bool vside;
    int s;
    bool active;
    if constexpr (PLANE) {
        const int plane = (DIR == 0) ? wk.grp : (wk.grp >> 1);
        vside = (DIR == 0) || (wk.grp & 1) == 0;
        s = plane * P + (int)threadIdx.x;
        active = plane < g.V / P && (int)threadIdx.x < P;
    } else {
        // DIR 0: one pair per wave; DIR 1/2 and the split form: (v, w) wave pairs
        constexpr bool VW = DIR != 0 || SPLIT;
        vside = !VW || (wave & 1) == 0;
        const int grp = VW ? wk.grp * GPB + (wave >> 1) : wk.grp * GPB + wave;
        s = grp * 64 + (threadIdx.x & 63);
        active = (grp < ngroups) && (s < g.V);
    }
    const T ep = T(S->emu), em = T(S->emu_inv);
    const size_t HALF = (size_t)12 * Vp;
    const cpx<T>* Vf = (const cpx<T>*)p.outV + rhs * p.sV;
    const cpx<T>* Wf = (const cpx<T>*)p.outW + rhs * p.sW;
    cpx<T>* oV = (cpx<T>*)p.outU + rhs * p.sU;
    cpx<T>* oW = (cpx<T>*)p.outZ + rhs * p.sZ;
    // the pair: DIR 0 (A, B) = (vhat, what); DIR 1/2 the two halves of one side
    const cpx<T>* Ain = (DIR == 0 || vside) ? Vf : Wf;
    const cpx<T>* Bin = (DIR == 0) ? Wf : Ain + HALF;
    cpx<T>* Aout = (DIR == 0 || vside) ? oV : oW;
    cpx<T>* Bout = (DIR == 0) ? oW : Aout + HALF;
    // hop factors: v side H(mu), w side H(-mu)
    T cfA, cbA, cfB, cbB, xfAB = 0, xbAB = 0, xfBA = 0, xbBA = 0;
    if (DIR == 0) {
        cfA = ep; cbA = em; cfB = em; cbB = ep;
    } else {
        cfA = cfB = vside ? ep : em;
        cbA = cbB = vside ? em : ep;
        if (DIR == 1) {
            if (vside) { xfAB = T(1); xbAB = T(-1); }    // top += (d/dmu H) vb
            else { xfBA = T(-1); xbBA = T(1); }          // bottom += (d/dmu H)^dag wt
        }
    }
    // LDS entry q of field f at plane site t (PLANE only)
    auto lds_at = [&](int f, int q, int t) -> float4& { return plane_lds[((size_t)f * NQ + q) * P + t]; };
    auto to_lds = [&](int f, int t, const cpx<T> (&v)[12]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float4 e;
            if constexpr (sizeof(T) == 8) {
                const double2 d{(double)v[q].re, (double)v[q].im};
                e = *reinterpret_cast<const float4*>(&d);
            } else {
                e = float4{(float)v[2 * q].re, (float)v[2 * q].im, (float)v[2 * q + 1].re, (float)v[2 * q + 1].im};
            }
            lds_at(f, q, t) = e;
        }
    };
    auto from_lds = [&](int f, int t, cpx<T> (&v)[12]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float4 e = lds_at(f, q, t);
            if constexpr (sizeof(T) == 8) {
                const double2 d = *reinterpret_cast<const double2*>(&e);
                v[q] = cpx<T>{(T)d.x, (T)d.y};
            } else {
                v[2 * q] = cpx<T>{(T)e.x, (T)e.y};
                v[2 * q + 1] = cpx<T>{(T)e.z, (T)e.w};
            }
        }
    };
    (void)to_lds;
    (void)from_lds;

    double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const char* Ab = reinterpret_cast<const char*>(Ain);
    const char* Bb = reinterpret_cast<const char*>(Bin);
    const char* Xb = p.xproj ? reinterpret_cast<const char*>((const cpx<T>*)p.xproj + rhs * p.sx) : nullptr;
    const uint32_t Vp16 = (uint32_t)Vp * 16u, so = (uint32_t)s * 16u;
    if constexpr (SEQ) {
        // the two outputs one after the other, each with its own-site terms,
        // eight hops, store and gamma contribution; one straight-line body per
        // side (VS: the v side; DIR 0 has one side).  PARTS: 1 the first
        // output, 2 the second, 3 both (the split form gives each to one wave).
        auto body = [&](auto vs_tag, auto parts_tag) {
            constexpr bool VS = decltype(vs_tag)::value;
            constexpr int PARTS = decltype(parts_tag)::value;
            const Nbr N = neighbours(g, s);
            cpx<T> acc[12];
            if constexpr ((PARTS & 1) != 0) {
            {
                cpx<T> a[12];
                ld_site<T>(Ab, Vp16, so, a);
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = mdiag * a[c];
                nrm_acc(part, (DIR == 0 || VS) ? 6 : 7, a);
                if ((DIR == 0 || VS) && Xb) {             // p = x^dag vhat_top
                    cpx<T> x[12];
                    ld_site<T>(Xb, Vp16, so, x);
                    dot_acc(part, 4, x, a);
                }
                if constexpr (DIR == 0) {                 // omega = what^dag vhat
                    cpx<T> b[12];
                    ld_site<T>(Bb, Vp16, so, b);
                    dot_acc(part, 0, b, a);
                } else if constexpr (!VS) {               // omega, top halves: wt^dag vt
                    cpx<T> v[12];
                    ld_site<T>(reinterpret_cast<const char*>(Vf), Vp16, so, v);
                    dot_acc(part, 0, a, v);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            single_hops<T, DIR == 1 && VS>(acc, Ain, Bin, U, N, s, Vp, cfA, cbA, xfAB, xbAB, g.bc_t);
#pragma unroll
            for (int c = 6; c < 12; ++c) acc[c] = -acc[c];   // gamma5
            store_site<T>(reinterpret_cast<char*>(Aout), Vp16, so, acc);
            if constexpr (DIR == 1 && VS) {               // gamma, top halves: wt^dag (A vhat)_top
                cpx<T> w[12];
                ld_site<T>(reinterpret_cast<const char*>(Wf), Vp16, so, w);
                dot_acc(part, 2, w, acc);
            }
            __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr ((PARTS & 2) != 0) {
            {
                cpx<T> b[12];
                ld_site<T>(Bb, Vp16, so, b);
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = mdiag * b[c];
                nrm_acc(part, (DIR != 0 && VS) ? 6 : 7, b);
                if constexpr (DIR != 0 && !VS) {          // omega, bottom halves: wb^dag vb
                    cpx<T> v[12];
                    ld_site<T>(reinterpret_cast<const char*>(Vf + HALF), Vp16, so, v);
                    dot_acc(part, 0, b, v);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            single_hops<T, DIR == 1 && !VS>(acc, opaque_ptr(Bin), opaque_ptr(Ain), opaque_ptr(U), N, s, Vp, cfB, cbB,
                                            xfBA, xbBA, g.bc_t);
#pragma unroll
            for (int c = 6; c < 12; ++c) acc[c] = -acc[c];   // gamma5
            store_site<T>(reinterpret_cast<char*>(Bout), Vp16, so, acc);
            if constexpr (DIR == 0) {                     // gamma = (A^dag what)^dag vhat
                cpx<T> v[12];
                ld_site<T>(Ab, Vp16, so, v);
                dot_acc(part, 2, acc, v);
            } else if constexpr (VS) {                    // gamma, bottom halves: wb^dag (A vhat)_bottom
                cpx<T> w[12];
                ld_site<T>(reinterpret_cast<const char*>(Wf + HALF), Vp16, so, w);
                dot_acc(part, 2, w, acc);
            }
            }
        };
        using both = std::integral_constant<int, 3>;
        if (active) {
            if constexpr (SPLIT) {   // DIR 0: the v wave H vhat, the w wave H^dag what
                if (vside) body(std::integral_constant<bool, true>{}, std::integral_constant<int, 1>{});
                else body(std::integral_constant<bool, true>{}, std::integral_constant<int, 2>{});
            } else if (DIR == 0 || vside) {
                body(std::integral_constant<bool, true>{}, both{});
            } else {
                body(std::integral_constant<bool, false>{}, both{});
            }
        }
    } else {
        cpx<T> accA[12], accB[12];
        if (active) {
            // own site: mass term, and the reductions that need only the inputs,
            // one loaded field at a time (fences keep the loads of the phases apart)
            {
                cpx<T> a[12];
                ld_site<T>(Ab, Vp16, so, a);
                if constexpr (PLANE) to_lds(0, (int)threadIdx.x, a);
    #pragma unroll
                for (int c = 0; c < 12; ++c) accA[c] = mdiag * a[c];
                nrm_acc(part, (DIR == 0 || vside) ? 6 : 7, a);
                if ((DIR == 0 || vside) && Xb) {          // p = x^dag vhat_top
                    cpx<T> x[12];
                                        if constexpr (sizeof(T) == 8) ld_site_nt<T>(Xb, Vp16, so, x);   // measured: FP32 gains nothing
                    else ld_site<T>(Xb, Vp16, so, x);
                    dot_acc(part, 4, x, a);
                }
                if (DIR == 0) {                           // omega = what^dag vhat
                    cpx<T> b[12];
                    ld_site<T>(Bb, Vp16, so, b);
                    dot_acc(part, 0, b, a);
                } else if (!vside) {                      // omega, top halves: wt^dag vt
                    cpx<T> v[12];
                    ld_site<T>(reinterpret_cast<const char*>(Vf), Vp16, so, v);
                    dot_acc(part, 0, a, v);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                cpx<T> b[12];
                ld_site<T>(Bb, Vp16, so, b);
                if constexpr (PLANE) to_lds(1, (int)threadIdx.x, b);
    #pragma unroll
                for (int c = 0; c < 12; ++c) accB[c] = mdiag * b[c];
                nrm_acc(part, (DIR != 0 && vside) ? 6 : 7, b);
                if (DIR != 0 && !vside) {                 // omega, bottom halves: wb^dag vb
                    cpx<T> v[12];
                    ld_site<T>(reinterpret_cast<const char*>(Vf + HALF), Vp16, so, v);
                    dot_acc(part, 0, b, v);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (PLANE) __syncthreads();   // the plane's inputs are in LDS
        if (active) {
            const Nbr N = neighbours(g, s);
            if constexpr (PLANE) {
                // x and y hops from the plane in LDS (periodic within the plane)
                const char* W = reinterpret_cast<const char*>(U);
                const char* W2 = reinterpret_cast<const char*>(dU);
                const int t = (int)threadIdx.x, Lx = g.L[0], Ly = g.L[1];
                const int x = t % Lx, y = t / Lx;
                const int txf = y * Lx + (x == Lx - 1 ? 0 : x + 1), txb = y * Lx + (x == 0 ? Lx - 1 : x - 1);
                const int tyf = (y == Ly - 1 ? 0 : y + 1) * Lx + x, tyb = (y == 0 ? Ly - 1 : y - 1) * Lx + x;
                const T h = T(-0.5), z = T(0);
    #define OVD_PL(I, TN, LS)                                                                                   \
        pair_hop<T, I, DIR>(                                                                                    \
            accA, accB, [&](cpx<T>(&v)[12]) { from_lds(0, TN, v); }, [&](cpx<T>(&v)[12]) { from_lds(1, TN, v); }, \
            W, W2, Vp16, (uint32_t)(LS) * 16u, h, h, z, z, vside);                                              \
        OVD_HOP_FENCE;
                OVD_PL(0, txf, s)
                OVD_PL(1, txb, N.b[0])
                OVD_PL(2, tyf, s)
                OVD_PL(3, tyb, N.b[1])
    #undef OVD_PL
            }
            pair_hops<T, DIR, PLANE>(accA, accB, Ain, Bin, U, dU, N, s, Vp, cfA, cbA, cfB, cbB, xfAB, xbAB, xfBA,
                                     xbBA, g.bc_t, vside);
    #pragma unroll
            for (int c = 6; c < 12; ++c) {   // gamma5
                accA[c] = -accA[c];
                accB[c] = -accB[c];
            }
            store_site<T>(reinterpret_cast<char*>(Aout), Vp16, so, accA);
            store_site<T>(reinterpret_cast<char*>(Bout), Vp16, so, accB);
            // gamma = what^dag (A vhat)
            if (DIR == 0) {                // = (A^dag what)^dag vhat = accB^dag vhat
                cpx<T> v[12];
                ld_site<T>(Ab, Vp16, so, v);
                dot_acc(part, 2, accB, v);
            } else if (vside) {
                {
                    cpx<T> w[12];
                    ld_site<T>(reinterpret_cast<const char*>(Wf), Vp16, so, w);
                    dot_acc(part, 2, w, accA);
                }
                __builtin_amdgcn_sched_barrier(0);
                {
                    cpx<T> w[12];
                    ld_site<T>(reinterpret_cast<const char*>(Wf + HALF), Vp16, so, w);
                    dot_acc(part, 2, w, accB);
                }
            }
        }

    }

    tsl_step_tail(part, lds, &am_last, S, co, partials, counters, rhs, nb, wk.grp, j, tau);
}

template <typename T, int DIR, int GPB, bool SEQ>
__global__ __launch_bounds__(256) OVD_OCC(T) void tsl_stencil_kernel(Geom g, StepPtrs p, const cpx<T>* __restrict__ U,
                                                          const cpx<T>* __restrict__ dU, T mdiag,
                                                          TslState* __restrict__ st, TslCoeffs co,
                                                          double* __restrict__ partials,
                                                          unsigned* __restrict__ counters, int j, double tau,
                                                          int ngroups, int nrhs, int map) {
    tsl_stencil_body<T, DIR, GPB, SEQ ? 1 : 0>((int)blockIdx.x, (int)gridDim.x, g, p, U, dU, mdiag, st, co, partials,
                                       counters, j, tau, ngroups, nrhs, map);
}

// The split form of the plain pair (DIR 0): GPB site groups per block, each
// with a v wave (H vhat) and a w wave (H^dag what).
template <typename T, int GPB>
__global__ __launch_bounds__(256) OVD_OCC(T) void tsl_stencil_split_kernel(Geom g, StepPtrs p,
                                                                           const cpx<T>* __restrict__ U, T mdiag,
                                                                           TslState* __restrict__ st, TslCoeffs co,
                                                                           double* __restrict__ partials,
                                                                           unsigned* __restrict__ counters, int j,
                                                                           double tau, int ngroups, int nrhs, int map) {
    tsl_stencil_body<T, 0, GPB, 2>((int)blockIdx.x, (int)gridDim.x, g, p, U, U, mdiag, st, co, partials, counters, j,
                                   tau, ngroups, nrhs, map);
}

// The time-marching form of the d/dmu block stencil (DIR 1).  One block per
// (rhs, side, z, segment of time slices); thread t holds site t of the
// xy-plane (Lx Ly <= 256) and the block walks its slices in time order.  The
// plane of slice t + 1, loaded for the forward time hop of slice t, goes into
// the second LDS buffer and serves as slice t + 1's own plane (own-site terms,
// x and y hops).  The backward time hop into slice t + 1 is formed at slice t
// from the own plane and the link U_4 of the forward hop, and carried in
// registers (the half spinors after the link, before reconstruction).  A
// slice thus reads from memory the next plane, the two z neighbour planes, the
// x field, the other side's own site and the links; the plane shape also reads
// both time neighbours, a whole time slice (Lx Ly Lz sites) away, which an
// XCD's L2 does not keep.  The hops are those of the plane shape, with the
// backward time hop added first (the carry is then dead before the other
// hops' loads), so the outputs agree with that shape to rounding.
// Blocks per rhs: 2 Lz nseg, padded to a multiple of 8 (padding blocks and
// empty segments run no slice but take part in the reduction).
template <typename T>
__global__ __launch_bounds__(256) void tsl_march_kernel(Geom g, StepPtrs p, const cpx<T>* __restrict__ U, T mdiag,
                                                        TslState* __restrict__ st, TslCoeffs co,
                                                        double* __restrict__ partials, unsigned* __restrict__ counters,
                                                        int j, double tau, int nseg, int nrhs, int map) {
    constexpr int NQ = sizeof(T) == 8 ? 12 : 6;   // 16-byte entries per site
    extern __shared__ float4 plane_lds[];          // [buffer 2][field 2][NQ][P]
    __shared__ double lds[16 * 8];
    __shared__ int am_last;
    const int nb = (int)(gridDim.x / (unsigned)nrhs);
    const Work wk = xcd_work((int)blockIdx.x, nb, nrhs, map);
    const int rhs = wk.rhs;
    TslState* S = st + rhs;
    if (S->flag) return;   // uniform over the rhs: breakdown in an earlier step
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int P = Lx * Ly, Vp = g.Vp;
    const int tid = (int)threadIdx.x;
    const bool vside = (wk.grp & 1) == 0;
    const int zz = (wk.grp >> 1) % Lz, seg = (wk.grp >> 1) / Lz;
    const int tlen = (Lt + nseg - 1) / nseg;
    const int t0 = seg * tlen, t1 = min(Lt, t0 + tlen);   // no slice when t0 >= t1
    const bool act = tid < P;
    const T ep = T(S->emu), em = T(S->emu_inv);
    const size_t HALF = (size_t)12 * Vp;
    const cpx<T>* Vf = (const cpx<T>*)p.outV + rhs * p.sV;
    const cpx<T>* Wf = (const cpx<T>*)p.outW + rhs * p.sW;
    const cpx<T>* Ain = vside ? Vf : Wf;
    cpx<T>* Aout = vside ? (cpx<T>*)p.outU + rhs * p.sU : (cpx<T>*)p.outZ + rhs * p.sZ;
    const char* Ab = reinterpret_cast<const char*>(Ain);
    const char* Bb = reinterpret_cast<const char*>(Ain + HALF);
    char* Ao = reinterpret_cast<char*>(Aout);
    char* Bo = reinterpret_cast<char*>(Aout + HALF);
    const char* Xb = p.xproj ? reinterpret_cast<const char*>((const cpx<T>*)p.xproj + rhs * p.sx) : nullptr;
    const char* W = reinterpret_cast<const char*>(U);
    // hop factors (v side H(mu), w side H(-mu)) and the mix factors of the time hops
    const T cf = vside ? ep : em, cb = vside ? em : ep;
    const T xfAB = vside ? T(1) : T(0), xbAB = vside ? T(-1) : T(0);
    const T xfBA = vside ? T(0) : T(-1), xbBA = vside ? T(0) : T(1);
    const uint32_t Vp16 = (uint32_t)Vp * 16u;
    const T h = T(-0.5), zr = T(0);
    const int x = tid % Lx, y = tid / Lx;
    const int txf = y * Lx + (x == Lx - 1 ? 0 : x + 1), txb = y * Lx + (x == 0 ? Lx - 1 : x - 1);
    const int tyf = (y == Ly - 1 ? 0 : y + 1) * Lx + x, tyb = (y == 0 ? Ly - 1 : y - 1) * Lx + x;

    auto lds_at = [&](int b, int f, int q, int t) -> float4& {
        return plane_lds[(((size_t)b * 2 + f) * NQ + q) * P + t];
    };
    auto to_lds = [&](int b, int f, int t, const cpx<T> (&v)[12]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float4 e;
            if constexpr (sizeof(T) == 8) {
                const double2 d{(double)v[q].re, (double)v[q].im};
                e = *reinterpret_cast<const float4*>(&d);
            } else {
                e = float4{(float)v[2 * q].re, (float)v[2 * q].im, (float)v[2 * q + 1].re, (float)v[2 * q + 1].im};
            }
            lds_at(b, f, q, t) = e;
        }
    };
    auto from_lds = [&](int b, int f, int t, cpx<T> (&v)[12]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float4 e = lds_at(b, f, q, t);
            if constexpr (sizeof(T) == 8) {
                const double2 d = *reinterpret_cast<const double2*>(&e);
                v[q] = cpx<T>{(T)d.x, (T)d.y};
            } else {
                v[2 * q] = cpx<T>{(T)e.x, (T)e.y};
                v[2 * q + 1] = cpx<T>{(T)e.z, (T)e.w};
            }
        }
    };
    // carry: the backward time hop into the next slice, U_4(s)^dag applied
    // to the projected own fields of site s (as the plane shape's hop 7 does
    // at the next slice); sb: the boundary factor of that hop
    cpx<T> kA0[3], kA1[3], kB0[3], kB1[3];
    auto make_carry = [&](const cpx<T> (&a)[12], const cpx<T> (&b)[12], uint32_t loff, T sb) {
        cpx<T> u[9];
        ld_link<T>(W, Vp16, 3, loff, u);
        cpx<T> a0[3], a1[3], b0[3], b1[3], h0[3], h1[3];
        proj_ct<T, 7>(a, a0, a1);
        proj_ct<T, 7>(b, b0, b1);
        const T cA = h * cb * sb;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c] = cA * a0[c] + (cA * xbAB) * b0[c];
            h1[c] = cA * a1[c] + (cA * xbAB) * b1[c];
        }
        link_mul<T, false>(u, h0, h1, kA0, kA1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c] = cA * b0[c] + (cA * xbBA) * a0[c];
            h1[c] = cA * b1[c] + (cA * xbBA) * a1[c];
        }
        link_mul<T, false>(u, h0, h1, kB0, kB1);
    };

    double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int buf = 0;
    if (t0 < t1 && act) {   // the first slice's own plane, and the carry into it
        const uint32_t s0 = (uint32_t)((t0 * Lz + zz) * P + tid) * 16u;
        const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
        const uint32_t sp = (uint32_t)((tp * Lz + zz) * P + tid) * 16u;
        cpx<T> a[12], b[12];
        ld_site<T>(Ab, Vp16, s0, a);
        to_lds(0, 0, tid, a);
        ld_site<T>(Bb, Vp16, s0, b);
        to_lds(0, 1, tid, b);
        __builtin_amdgcn_sched_barrier(0);
        ld_site<T>(Ab, Vp16, sp, a);
        ld_site<T>(Bb, Vp16, sp, b);
        make_carry(a, b, sp, t0 == 0 ? T(g.bc_t) : T(1));
    }
    for (int tt = t0; tt < t1; ++tt) {
        __syncthreads();   // slice tt's plane is in buffer buf; buffer buf ^ 1 is free
        if (act) {
            const int s = (tt * Lz + zz) * P + tid;
            const uint32_t so = (uint32_t)s * 16u;
            const Nbr N = neighbours(g, s);
            const bool keep = tt + 1 < t1;   // the next slice is this block's
            cpx<T> accA[12], accB[12];
            {
                cpx<T> a[12];
                from_lds(buf, 0, tid, a);
#pragma unroll
                for (int c = 0; c < 12; ++c) accA[c] = mdiag * a[c];
                nrm_acc(part, vside ? 6 : 7, a);
                if (vside && Xb) {                         // p = x^dag vhat_top
                    cpx<T> xv[12];
                    if constexpr (sizeof(T) == 8) ld_site_nt<T>(Xb, Vp16, so, xv);
                    else ld_site<T>(Xb, Vp16, so, xv);
                    dot_acc(part, 4, xv, a);
                }
                if (!vside) {                              // omega, top halves: wt^dag vt
                    cpx<T> v[12];
                    ld_site<T>(reinterpret_cast<const char*>(Vf), Vp16, so, v);
                    dot_acc(part, 0, a, v);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                cpx<T> b[12];
                from_lds(buf, 1, tid, b);
#pragma unroll
                for (int c = 0; c < 12; ++c) accB[c] = mdiag * b[c];
                nrm_acc(part, vside ? 6 : 7, b);
                if (!vside) {                              // omega, bottom halves: wb^dag vb
                    cpx<T> v[12];
                    ld_site<T>(reinterpret_cast<const char*>(Vf + HALF), Vp16, so, v);
                    dot_acc(part, 0, b, v);
                }
            }
            // backward time hop: the carry formed at the previous slice
            recon_add<T, 7>(accA, kA0, kA1);
            recon_add<T, 7>(accB, kB0, kB1);
            __builtin_amdgcn_sched_barrier(0);
            // x and y hops from the plane in LDS
#define OVD_ML(I, TN, LS)                                                                                  \
    pair_hop<T, I, 1>(                                                                                     \
        accA, accB, [&](cpx<T>(&v)[12]) { from_lds(buf, 0, TN, v); },                                      \
        [&](cpx<T>(&v)[12]) { from_lds(buf, 1, TN, v); }, W, W, Vp16, (uint32_t)(LS) * 16u, h, h, zr, zr, \
        vside);                                                                                            \
    OVD_MARCH_FENCE;
            OVD_ML(0, txf, s)
            OVD_ML(1, txb, N.b[0])
            OVD_ML(2, tyf, s)
            OVD_ML(3, tyb, N.b[1])
#undef OVD_ML
            // z hops from memory
            {
                const uint32_t nf = (uint32_t)N.f[2] * 16u, nbk = (uint32_t)N.b[2] * 16u;
                pair_hop<T, 4, 1>(
                    accA, accB, [&](cpx<T>(&v)[12]) { ld_site<T>(Ab, Vp16, nf, v); },
                    [&](cpx<T>(&v)[12]) { ld_site<T>(Bb, Vp16, nf, v); }, W, W, Vp16, so, h, h, zr, zr, vside);
                OVD_MARCH_FENCE;
                pair_hop<T, 5, 1>(
                    accA, accB, [&](cpx<T>(&v)[12]) { ld_site<T>(Ab, Vp16, nbk, v); },
                    [&](cpx<T>(&v)[12]) { ld_site<T>(Bb, Vp16, nbk, v); }, W, W, Vp16, nbk, h, h, zr, zr, vside);
                OVD_MARCH_FENCE;
            }
            // forward time hop; its neighbour plane is the next slice's own plane
            {
                const uint32_t nf = (uint32_t)N.f[3] * 16u;
                const T sf = N.wf ? T(g.bc_t) : T(1);
                const int nbuf = buf ^ 1;   // free in this slice; on the last slice the store is unused
                {
                    cpx<T> v[12];
                    ld_site<T>(Ab, Vp16, nf, v);
                    to_lds(nbuf, 0, tid, v);
                }
                {
                    cpx<T> v[12];
                    ld_site<T>(Bb, Vp16, nf, v);
                    to_lds(nbuf, 1, tid, v);
                }
                // the thread reads back its own entries: no barrier needed
                pair_hop<T, 6, 1>(
                    accA, accB, [&](cpx<T>(&v)[12]) { from_lds(nbuf, 0, tid, v); },
                    [&](cpx<T>(&v)[12]) { from_lds(nbuf, 1, tid, v); }, W, W, Vp16, so, h * cf * sf, h * cf * sf,
                    xfAB, xfBA, vside);
                OVD_MARCH_FENCE;
            }
#pragma unroll
            for (int c = 6; c < 12; ++c) {   // gamma5
                accA[c] = -accA[c];
                accB[c] = -accB[c];
            }
            store_site<T>(Ao, Vp16, so, accA);
            store_site<T>(Bo, Vp16, so, accB);
            if (vside) {   // gamma: wt^dag (A vhat)_top + wb^dag (A vhat)_bottom
                {
                    cpx<T> w[12];
                    ld_site<T>(reinterpret_cast<const char*>(Wf), Vp16, so, w);
                    dot_acc(part, 2, w, accA);
                }
                __builtin_amdgcn_sched_barrier(0);
                {
                    cpx<T> w[12];
                    ld_site<T>(reinterpret_cast<const char*>(Wf + HALF), Vp16, so, w);
                    dot_acc(part, 2, w, accB);
                }
            }
            if (keep) {   // the carry into the next slice (its backward hop crosses no boundary)
                __builtin_amdgcn_sched_barrier(0);
                cpx<T> a[12], b[12];
                from_lds(buf, 0, tid, a);
                from_lds(buf, 1, tid, b);
                make_carry(a, b, so, T(1));
            }
        }
        buf ^= 1;
    }
    tsl_step_tail(part, lds, &am_last, S, co, partials, counters, rhs, nb, wk.grp, j, tau);
}

// One Lanczos step of several lattices in one launch: the blocks are split
// into consecutive ranges, one per lattice (each range a multiple of 8 blocks
// long and starting at a multiple of 8, so a block's XCD is the one it has in
// the lattice's own launch), and every block runs the standalone body with
// its lattice's arguments: results identical to the lattice's own launch.
template <typename T, int DIR, int GPB, bool SEQ>
__global__ __launch_bounds__(256) OVD_OCC(T) void tsl_stencil_multi_kernel(const TslSegment* __restrict__ seg,
                                                                           int nseg, int j) {
    int i = 0;
    for (int q = 1; q < nseg; ++q)
        if ((int)blockIdx.x >= seg[q].block0) i = q;
    const TslSegment& S = seg[i];
    tsl_stencil_body<T, DIR, GPB, SEQ ? 1 : 0>((int)blockIdx.x - S.block0, S.nblocks, S.g, S.p, (const cpx<T>*)S.U,
                                         (const cpx<T>*)S.dU, T(S.mdiag), S.st, S.co, S.partials, S.counters, j, S.tau,
                                         S.ngroups, S.nrhs, S.map);
}

int tsl_update_xblocks(long long fsz) {
    long long nblk = (fsz + 255) / 256;
    return (int)(nblk > 2048 ? 2048 : nblk);
}

template <typename T>
void launch_tsl_update(int nrhs, int nterms, long long fsz, const StepPtrs& p, const TslState* st,
                       hipStream_t s) {
    dim3 grid((unsigned)tsl_update_xblocks(fsz), nrhs, 2);
    if (nterms == 3)
        tsl_update_kernel<T, 3><<<grid, 256, 0, s>>>(p, fsz, st);
    else
        tsl_update_kernel<T, 2><<<grid, 256, 0, s>>>(p, fsz, st);
}

int tsl_stencil_blocks(const Geom& g, int dir, int gpb) {
    if (gpb == PLANE_GPB) {   // one block per plane (and side)
        const int items = (g.V / (g.L[0] * g.L[1])) * (dir == 0 ? 1 : 2);
        return (items + 7) / 8 * 8;
    }
    const int ngroups = (g.V + 63) / 64;
    if (gpb <= 0) gpb = dir == 0 ? 4 : 2;
    return ((ngroups + gpb - 1) / gpb + 7) / 8 * 8;   // nb * nrhs is a multiple of 8
}

bool tsl_plane_ok(const Geom& g) {
    const int P = g.L[0] * g.L[1];
    return P >= 128 && P <= 256;
}

// the time-marching form: two LDS buffers of the plane's two input fields
static size_t march_lds_bytes(const Geom& g, size_t real_bytes) {
    return (size_t)2 * 2 * 12 * g.L[0] * g.L[1] * 2 * real_bytes;
}

bool tsl_march_ok(const Geom& g, int real_bytes) {
    return tsl_plane_ok(g) && march_lds_bytes(g, (size_t)real_bytes) + 2048 <= 160 * 1024;
}

static int march_segments(const Geom& g, int nseg) {
    return nseg < 1 ? 1 : nseg > g.L[3] ? g.L[3] : nseg;
}

int tsl_march_blocks(const Geom& g, int nseg) {
    return (2 * g.L[2] * march_segments(g, nseg) + 7) / 8 * 8;
}

template <typename T>
void launch_tsl_stencil(const Geom& g, int dir, int nrhs, const StepPtrs& p, const cpx<T>* U,
                        const cpx<T>* dU, double m_diag, TslState* st, TslCoeffs co, double* partials,
                        unsigned* counters, int j, double tau, hipStream_t s, StencilVariant v) {
    const int ngroups = (g.V + 63) / 64;
    if (v.map < 0) v.map = default_map(nrhs);
    if (v.gpb <= 0) v.gpb = dir == 0 ? 4 : 2;
    dim3 grid(tsl_stencil_blocks(g, dir, v.gpb) * nrhs);
    const T md = T(m_diag);
    // dynamic LDS: the plane's two input fields (PLANE_GPB only)
    const size_t plds = (size_t)2 * 12 * g.L[0] * g.L[1] * sizeof(cpx<T>);
#define OVD_TSL(D, G, THREADS, SHM, SQ)                                                                    \
    tsl_stencil_kernel<T, D, G, SQ><<<grid, dim3(THREADS), SHM, s>>>(g, p, U, dU, md, st, co, partials, counters, \
                                                                    j, tau, ngroups, nrhs, v.map)
#define OVD_TSL_PLANE(D)                                                                                   \
    do {                                                                                                   \
        static bool attr = false;                                                                          \
        if (!attr) {                                                                                       \
            (void)hipFuncSetAttribute((const void*)tsl_stencil_kernel<T, D, PLANE_GPB, false>,              \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);      \
            attr = true;                                                                                   \
        }                                                                                                  \
        OVD_TSL(D, PLANE_GPB, 256, plds, false);                                                           \
    } while (0)
    if (dir == 1 && v.seq == 3 && tsl_march_ok(g, (int)sizeof(T))) {
        const int nseg = march_segments(g, v.gpb);
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void*)tsl_march_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      160 * 1024 - 2048);
            attr = true;
        }
        tsl_march_kernel<T><<<dim3(tsl_march_blocks(g, nseg) * nrhs), dim3(256), march_lds_bytes(g, sizeof(T)), s>>>(
            g, p, U, md, st, co, partials, counters, j, tau, nseg, nrhs, v.map);
        return;
    }
    if (v.gpb == PLANE_GPB && !tsl_plane_ok(g)) v.gpb = dir == 0 ? 4 : 2;
    const bool split = dir == 0 && v.seq == 2 && (v.gpb == 1 || v.gpb == 2);
    const bool seq = v.seq == 1 && dir != 2 && v.gpb != PLANE_GPB;
    grid = dim3(tsl_stencil_blocks(g, dir, v.gpb) * nrhs);
    if (split) {
        if (v.gpb == 1)
            tsl_stencil_split_kernel<T, 1><<<grid, 128, 0, s>>>(g, p, U, md, st, co, partials, counters, j, tau,
                                                                ngroups, nrhs, v.map);
        else
            tsl_stencil_split_kernel<T, 2><<<grid, 256, 0, s>>>(g, p, U, md, st, co, partials, counters, j, tau,
                                                                ngroups, nrhs, v.map);
    } else if (dir == 0) {
        if (v.gpb == PLANE_GPB) OVD_TSL_PLANE(0);
        else if (v.gpb == 2) {
            if (seq) OVD_TSL(0, 2, 128, 0, true);
            else OVD_TSL(0, 2, 128, 0, false);
        } else {
            if (seq) OVD_TSL(0, 4, 256, 0, true);
            else OVD_TSL(0, 4, 256, 0, false);
        }
    } else if (dir == 1) {
        if (v.gpb == PLANE_GPB) OVD_TSL_PLANE(1);
        else if (v.gpb == 1) {
            if (seq) OVD_TSL(1, 1, 128, 0, true);
            else OVD_TSL(1, 1, 128, 0, false);
        } else {
            if (seq) OVD_TSL(1, 2, 256, 0, true);
            else OVD_TSL(1, 2, 256, 0, false);
        }
    } else {
        if (v.gpb == PLANE_GPB) OVD_TSL_PLANE(2);
        else if (v.gpb == 1) OVD_TSL(2, 1, 128, 0, false);
        else OVD_TSL(2, 2, 256, 0, false);
    }
#undef OVD_TSL_PLANE
#undef OVD_TSL
}

template <typename T>
void launch_tsl_step_multi(int dir, int gpb, int seq, int nterms, const TslSegment* seg, int nseg, int nblocks,
                           int ublocks, int max_nrhs, int j, hipStream_t s) {
    if (nterms == 3)
        tsl_update_multi_kernel<T, 3><<<dim3(ublocks, max_nrhs, 2), 256, 0, s>>>(seg, nseg);
    else if (nterms == 2)
        tsl_update_multi_kernel<T, 2><<<dim3(ublocks, max_nrhs, 2), 256, 0, s>>>(seg, nseg);
    if (dir == 1) {
        if (gpb == 1) {
            if (seq) tsl_stencil_multi_kernel<T, 1, 1, true><<<nblocks, 128, 0, s>>>(seg, nseg, j);
            else tsl_stencil_multi_kernel<T, 1, 1, false><<<nblocks, 128, 0, s>>>(seg, nseg, j);
        } else {
            if (seq) tsl_stencil_multi_kernel<T, 1, 2, true><<<nblocks, 256, 0, s>>>(seg, nseg, j);
            else tsl_stencil_multi_kernel<T, 1, 2, false><<<nblocks, 256, 0, s>>>(seg, nseg, j);
        }
    } else {
        if (gpb == 1) tsl_stencil_multi_kernel<T, 2, 1, false><<<nblocks, 128, 0, s>>>(seg, nseg, j);
        else tsl_stencil_multi_kernel<T, 2, 2, false><<<nblocks, 256, 0, s>>>(seg, nseg, j);
    }
}

#define OVD_INST(T)                                                                                        \
    template void launch_tsl_step_multi<T>(int, int, int, int, const TslSegment*, int, int, int, int, int, \
                                           hipStream_t);                                                   \
    template void launch_tsl_update<T>(int, int, long long, const StepPtrs&, const TslState*, hipStream_t); \
    template void launch_tsl_stencil<T>(const Geom&, int, int, const StepPtrs&, const cpx<T>*, const cpx<T>*, \
                                        double, TslState*, TslCoeffs, double*, unsigned*, int, double,     \
                                        hipStream_t, StencilVariant);
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
// trF[y] = tr F_t(y), summed later into ds/dmu; dth[nu][y] = i tr F_nu(y), the
// derivative along a U(1) phase U_nu(y) -> e^{i theta} U_nu(y) (nullable).
// The sum over p may be split into chunks (the basis regenerated a chunk at a
// time): Kacc [18][4V] carries Kf, Kb between the launches of one gradient;
// `first` starts from zero instead of Kacc, `last` turns K into the outputs
// (else K is stored to Kacc).
// ---------------------------------------------------------------------------
// Kf, Kb += the terms of basis pairs p0 <= p < p1 for thread t = 4 y + nu
__device__ __forceinline__ void force_acc(const Geom& g, int t, int p0, int p1, const c64* __restrict__ Vb,
                                          long long sV, const c64* __restrict__ Zb, long long sZ, c64 (&Kf)[9],
                                          c64 (&Kb)[9]) {
    const int y = t >> 2, nu = t & 3;
    const int Vp = g.Vp;
    const Nbr N = neighbours(g, y);
    const int yp = nu == 0 ? N.f[0] : nu == 1 ? N.f[1] : nu == 2 ? N.f[2] : N.f[3];
    const int cfw = kHop[2 * nu], cbw = kHop[2 * nu + 1];
    for (int p = p0; p < p1; ++p) {
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
}

// the outputs of link U_nu(y), t = 4 y + nu, from its finished Kf, Kb
__device__ __forceinline__ void force_out(const Geom& g, int t, const c64 (&Kf)[9], const c64 (&Kb)[9],
                                          const c64* __restrict__ U, double emu, c64* __restrict__ F,
                                          c64* __restrict__ dU, c64* __restrict__ dUc, c64* __restrict__ trF,
                                          c64* __restrict__ dth) {
    const int y = t >> 2, nu = t & 3;
    const Nbr N = neighbours(g, y);
    const double sg = (nu == 3 && N.wf) ? double(g.bc_t) : 1.0;
    const double cf = nu == 3 ? emu : 1.0, cb = nu == 3 ? 1.0 / emu : 1.0;
    // link U_nu(y) from the FP64 internal link field
    c64 u[9];
    load_link(U, nu, y, g.Vp, u);
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
    if (dth) dth[(size_t)nu * g.V + y] = c64{-tr.im, tr.re};   // i tr F: the U(1) phase of this link
}

__global__ __launch_bounds__(256) void vjp_force_kernel(Geom g, int k, const c64* __restrict__ Vb, long long sV,
                                                        const c64* __restrict__ Zb, long long sZ,
                                                        const c64* __restrict__ U, double emu,
                                                        c64* __restrict__ F, c64* __restrict__ dU,
                                                        c64* __restrict__ dUc, c64* __restrict__ trF,
                                                        c64* __restrict__ dth, c64* __restrict__ Kacc, int first,
                                                        int last) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    const size_t n4 = (size_t)4 * g.V;
    c64 Kf[9], Kb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Kf[i] = first ? c64{0.0, 0.0} : Kacc[(size_t)i * n4 + t];
        Kb[i] = first ? c64{0.0, 0.0} : Kacc[(size_t)(9 + i) * n4 + t];
    }
    force_acc(g, t, 0, k, Vb, sV, Zb, sZ, Kf, Kb);
    if (!last) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            Kacc[(size_t)i * n4 + t] = Kf[i];
            Kacc[(size_t)(9 + i) * n4 + t] = Kb[i];
        }
        return;
    }
    force_out(g, t, Kf, Kb, U, emu, F, dU, dUc, trF, dth);
}

// The sum over p split into nchunk consecutive ranges that run side by side
// (blockIdx.y = range): each range's Kf, Kb go to Kpart [nchunk][18][4V];
// vjp_force_fin_kernel then sums the ranges in order and writes the outputs.
__global__ __launch_bounds__(256) void vjp_force_part_kernel(Geom g, int k, int nchunk, const c64* __restrict__ Vb,
                                                             long long sV, const c64* __restrict__ Zb, long long sZ,
                                                             c64* __restrict__ Kpart) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    const size_t n4 = (size_t)4 * g.V;
    const int c = blockIdx.y;
    const int p0 = (int)((long long)k * c / nchunk), p1 = (int)((long long)k * (c + 1) / nchunk);
    c64 Kf[9], Kb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Kf[i] = Kb[i] = c64{0.0, 0.0};
    force_acc(g, t, p0, p1, Vb, sV, Zb, sZ, Kf, Kb);
    c64* Kc = Kpart + (size_t)c * 18 * n4;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Kc[(size_t)i * n4 + t] = Kf[i];
        Kc[(size_t)(9 + i) * n4 + t] = Kb[i];
    }
}

__global__ __launch_bounds__(256) void vjp_force_fin_kernel(Geom g, int nchunk, const c64* __restrict__ Kpart,
                                                            const c64* __restrict__ U, double emu,
                                                            c64* __restrict__ F, c64* __restrict__ dU,
                                                            c64* __restrict__ dUc, c64* __restrict__ trF,
                                                            c64* __restrict__ dth, c64* __restrict__ Kacc, int last) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.V) return;
    const size_t n4 = (size_t)4 * g.V;
    c64 Kf[9], Kb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Kf[i] = Kb[i] = c64{0.0, 0.0};
    for (int c = 0; c < nchunk; ++c) {
        const c64* Kc = Kpart + (size_t)c * 18 * n4;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            Kf[i] += Kc[(size_t)i * n4 + t];
            Kb[i] += Kc[(size_t)(9 + i) * n4 + t];
        }
    }
    if (!last) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            Kacc[(size_t)i * n4 + t] = Kf[i];
            Kacc[(size_t)(9 + i) * n4 + t] = Kb[i];
        }
        return;
    }
    force_out(g, t, Kf, Kb, U, emu, F, dU, dUc, trF, dth);
}

int vjp_force_chunks(const Geom& g, int k) {
    const int nblk = (4 * g.V + 255) / 256;
    int nc = (2048 + nblk - 1) / nblk;   // about 2048 blocks in all
    nc = std::min(nc, 8);
    nc = std::min(nc, k / 16);           // at least 16 basis pairs per range
    return std::max(nc, 1);
}

size_t vjp_force_scratch_elems(const Geom& g, int nchunk) {
    return nchunk > 1 ? (size_t)nchunk * 18 * 4 * g.V : 0;
}

void launch_vjp_force(const Geom& g, int k, const c64* Vb, long long sV, const c64* Zb, long long sZ, const c64* U64,
                      double emu, c64* F, c64* dU, c64* dUc, c64* trF, c64* dth, hipStream_t s, c64* Kacc, bool first,
                      bool last, c64* Kpart, int nchunk) {
    const unsigned nblk = (unsigned)((4 * g.V + 255) / 256);
    if (nchunk > 1 && Kpart && first) {
        vjp_force_part_kernel<<<dim3(nblk, (unsigned)nchunk), 256, 0, s>>>(g, k, nchunk, Vb, sV, Zb, sZ, Kpart);
        vjp_force_fin_kernel<<<nblk, 256, 0, s>>>(g, nchunk, Kpart, U64, emu, F, dU, dUc, trF, dth, Kacc,
                                                  last ? 1 : 0);
        return;
    }
    vjp_force_kernel<<<nblk, 256, 0, s>>>(g, k, Vb, sV, Zb, sZ, U64, emu, F, dU, dUc, trF, dth, Kacc, first ? 1 : 0,
                                          last ? 1 : 0);
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
