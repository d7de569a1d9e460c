// C ABI of libovderiv and the host-side driver of the two-sided Lanczos
// pipeline (see include/ovderiv.h for the contract of every entry point).
//
// Pipeline of one call (all on the handle's stream, no host round trip until
// the end):
//   1. pack the AoS complex128 inputs into the internal [12][Vp] layout and
//      form the right / left start vectors (block system: (0; b) and, for the
//      left start, (b; b));
//   2. k fused Lanczos steps (one kernel each, one grid reduction each; the
//      scalar recurrence advances on the device);
//   3. sgn(T_k) e_1 by the resolvent quadrature (FP64);
//   4. |psi| V_k sgn(T_k) e_1 from the stored basis, or the storage-free
//      scalar |psi| sum_j c_j <x|v_j>.
#include "ovd_internal.h"
#include "../../include/ovderiv.h"

#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <thread>
#include <vector>

using namespace ovd;

struct DeflSet {
    double mu = 0;
    int m = 0, l = 0;
    int dir_kind = OVD_DIR_MU;
    std::vector<c64> lam;
    c64* R = nullptr;   // FP64 [m][12][Vp] (padding sites zero)
    c64* L = nullptr;
    c64* dR = nullptr;  // [l][12][Vp]
    c64* dL = nullptr;
    c64* dir_ref = nullptr;  // link direction of dR, dL (FP64 internal layout); null for mu
    double* sgn = nullptr;   // device [m]: sgn(Re lambda_i)
    double* ones = nullptr;  // device [m]: 1
};

struct ovd_lattice {
    Geom g{};
    rocblas_handle blas = nullptr;   // the gradient's Z = W M'^dag (created on first use)
    double m0 = -1.5, r = 1.0;
    ovd_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    c64* U64 = nullptr;
    c32* U32 = nullptr;
    c64* dU64 = nullptr;
    c32* dU32 = nullptr;
    bool links_set = false;
    std::map<std::string, std::pair<void*, size_t>> ws;
    std::vector<DeflSet> defl;
    // coefficients of the last Lanczos run
    int last_nrhs = 0, last_k = 0;
    TslCoeffs last_co{};
    // event pool for per-kernel timing of the Lanczos loop
    std::vector<hipEvent_t> ev;
    // recorded Lanczos loops (HIP graphs), keyed by everything baked into them
    struct GraphEntry {
        std::vector<uintptr_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;   // capture only; replays run on `stream`
    // autotuned launch shapes, keyed by kernel, precision, direction / operator and batch size
    std::map<std::string, StencilVariant> tuned;
    // while a call runs without allocations: workspaces are carved from this
    // region (the per-device static scratch) instead of hipMalloc
    struct Arena {
        char* base = nullptr;
        size_t size = 0, used = 0;
        bool active = false;
    } arena;
};

namespace {

ovd_status fail(ovd_h h, ovd_status st, const std::string& msg) {
    if (h) h->err = msg;
    return st;
}

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(h, OVD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// grow-only named workspace (or, during an allocation-free call, the next
// 256-byte aligned piece of the call's scratch region)
void* ws_get(ovd_h h, const std::string& name, size_t bytes, ovd_status* st) {
    if (h->arena.active) {
        const size_t off = (h->arena.used + 255) / 256 * 256;
        if (off + bytes > h->arena.size) {
            *st = fail(h, OVD_ENOMEM, "the no-allocation scratch (" + std::to_string(h->arena.size) +
                                          " bytes) is too small for workspace '" + name + "'");
            return nullptr;
        }
        h->arena.used = off + bytes;
        return h->arena.base + off;
    }
    auto it = h->ws.find(name);
    if (it != h->ws.end() && it->second.second >= bytes) return it->second.first;
    if (it != h->ws.end()) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(it->second.first);
        h->ws.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
        *st = fail(h, OVD_ENOMEM, "hipMalloc of workspace '" + name + "' (" + std::to_string(bytes) + " bytes) failed");
        return nullptr;
    }
    h->ws[name] = {p, bytes};
    return p;
}

#define WS(var, type, name, count)                                                   \
    type* var = (type*)ws_get(h, name, sizeof(type) * (size_t)(count), &wst);        \
    if (!var) return wst;

struct Timer {
    hipEvent_t a{}, b{};
    bool ok = false;
    void start(hipStream_t s, bool enable = true) {
        if (!enable) return;
        ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
        if (ok) (void)hipEventRecord(a, s);
    }
    void stop(hipStream_t s) {
        if (ok) (void)hipEventRecord(b, s);
    }
    double ms() {
        float t = 0.f;
        if (ok && hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(&t, a, b);
        return t;
    }
    ~Timer() {
        if (ok) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    }
};

// Autotuner: time every candidate launch shape with `launch(v)` (1 warm-up
// and 3 timed launches each, on the handle's stream) and keep the fastest.
// `reset()` runs before each candidate.
template <typename Launch, typename Reset>
StencilVariant autotune(ovd_h h, const std::vector<StencilVariant>& cands, Launch launch, Reset reset) {
    StencilVariant best = cands.front();
    float best_ms = 1e30f;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return best;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return best;
    }
    // three rounds over the candidates (each: a warm-up launch, then three timed
    // launches), the best of its rounds per candidate: shapes within a few per
    // cent of each other are then ranked by more than one sample, and drift
    // over the rounds does not favour one of them
    std::vector<float> tmin(cands.size(), 1e30f);
    for (int round = 0; round < 3; ++round)
        for (size_t i = 0; i < cands.size(); ++i) {
            const auto& v = cands[i];
            reset();
            launch(v);
            (void)hipEventRecord(a, h->stream);
            for (int r = 0; r < 3; ++r) launch(v);
            (void)hipEventRecord(b, h->stream);
            float ms = 0.f;
            if (hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess)
                tmin[i] = std::min(tmin[i], ms);
        }
    for (size_t i = 0; i < cands.size(); ++i)
        if (tmin[i] < best_ms) {
            best_ms = tmin[i];
            best = cands[i];
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipGetLastError();
    return best;
}

// a shape forced through the options, completed with defaults; false if none is forced
bool forced_shape(ovd_h h, int nrhs, int def_gpb, StencilVariant* v) {
    if (h->opt.shape_map < 0 && h->opt.shape_gpb <= 0 && h->opt.shape_seq < 0 && h->opt.shape_rp <= 0) return false;
    v->map = h->opt.shape_map >= 0 ? h->opt.shape_map : default_map(nrhs);
    if (v->map == 0 && nrhs % 8 != 0) v->map = 1;
    v->gpb = h->opt.shape_gpb > 0 ? h->opt.shape_gpb : def_gpb;
    v->seq = h->opt.shape_seq == 2 ? 2 : h->opt.shape_seq == 3 ? 3 : h->opt.shape_seq > 0 ? 1 : 0;
    v->rp = h->opt.shape_rp == 2 ? 2 : 1;
    return true;
}

// launch shapes to time: both work orders, the given groups per block, with
// seq_too the sequential form of each (the LDS-plane shape has none), and with
// split_too the split form of DIR 0 with 1 and 2 groups per block
std::vector<StencilVariant> shape_candidates(int nrhs, const std::vector<int>& gpbs, bool seq_too = false,
                                             bool split_too = false) {
    std::vector<StencilVariant> c;
    for (int map : {1, 0}) {
        if (map == 0 && nrhs % 8 != 0) continue;
        for (int gpb : gpbs) {
            c.push_back(StencilVariant{map, gpb, 0});
            if (seq_too && gpb != 8) c.push_back(StencilVariant{map, gpb, 1});
        }
        if (split_too) {
            c.push_back(StencilVariant{map, 1, 2});
            c.push_back(StencilVariant{map, 2, 2});
        }
    }
    return c;
}

// Dw.v launch shapes: the stencil shapes, and for H and Dw on an even number
// of right-hand sides each of them also with two right-hand sides per thread,
// and (plane: the xy-plane fits a block) two per thread with the plane in LDS
std::vector<StencilVariant> op_candidates(int nrhs, int op, bool plane) {
    std::vector<StencilVariant> c = shape_candidates(nrhs, {4, 2});
    if ((op == 0 || op == 1) && nrhs % 2 == 0) {
        const size_t n = c.size();
        for (size_t i = 0; i < n; ++i) {
            StencilVariant v = c[i];
            v.rp = 2;
            if (v.map == 0 && (nrhs / 2) % 8 != 0) continue;   // the XCD order over pairs
            c.push_back(v);
        }
        if (plane)
            for (int map : {1, 0})
                if (map == 1 || (nrhs / 2) % 8 == 0) c.push_back(StencilVariant{map, 8, 0, 2});
    }
    return c;
}

// a forced Dw.v shape made valid: 2 or 4 groups per block, or the plane in
// LDS (8) with two right-hand sides per thread where that applies
void op_shape_sanitize(StencilVariant& fv, int op, int nrhs, const Geom& g) {
    fv.seq = 0;
    if (!(op == 0 || op == 1) || nrhs % 2 != 0) fv.rp = 1;
    if (fv.gpb == 8 && fv.rp == 2 && tsl_plane_ok(g)) return;
    if (fv.gpb != 2) fv.gpb = 4;
}

// Whether a call keeps its Krylov basis (need bytes) or regenerates it:
// basis_recompute > 0 always regenerates, 0 never, < 0 when the stored basis
// does not fit in the free device memory plus what the named workspaces
// already hold.
bool recompute_basis(ovd_h h, size_t need, std::initializer_list<const char*> held_names, ovd_status* st) {
    if (h->opt.basis_recompute > 0) return true;
    if (h->opt.basis_recompute == 0) return false;
    if (h->opt.mem_budget > 0 && need > (size_t)h->opt.mem_budget) return true;
    size_t held = 0;
    for (const char* n : held_names) {
        auto it = h->ws.find(n);
        if (it != h->ws.end()) held += it->second.second;
    }
    size_t fr = 0, tot = 0;
    const hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) {
        *st = fail(h, OVD_EHIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
        return false;
    }
    return need > held + fr / 10 * 9;
}

// fill per-rhs coefficient vector coef[r][j] = delta[r][0] * c[r][j] / delta[r][j]
__global__ void make_coef_kernel(int k, TslCoeffs co, const c64* __restrict__ c, c64* __restrict__ coef) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= k) return;
    const double d0 = co.delta[(size_t)r * co.kmax].re;
    const double dj = co.delta[(size_t)r * co.kmax + j].re;
    coef[(size_t)r * k + j] = (d0 / dj) * c[(size_t)r * k + j];
}

// left start of the block system: dst = (src_top + src_bot; src_bot)
template <typename T>
__global__ void left_sum_kernel(Geom g, const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst, long long stride) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
    const size_t HALF = (size_t)12 * g.Vp;
    const cpx<T>* a = src + r * stride;
    cpx<T>* o = dst + r * stride;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t i = fidx<T>(c, s, g.Vp);
        const cpx<T> t = a[i], b = a[HALF + i];
        o[i] = t + b;
        o[HALF + i] = b;
    }
}

// block start vectors from FP64 halves: src_v = (t; b), src_w = (t + b; b) or (t; b)
template <typename T>
__global__ void make_block_src_kernel(Geom g, const c64* __restrict__ t64, const c64* __restrict__ b64, long long sh,
                                      cpx<T>* __restrict__ sv, cpx<T>* __restrict__ sw, long long fsz, int same) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V) return;
    const size_t HALF = (size_t)12 * g.Vp;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const c64 t = t64[r * sh + (size_t)c * g.Vp + s], b = b64[r * sh + (size_t)c * g.Vp + s];
        const size_t i = fidx<T>(c, s, g.Vp);
        sv[r * fsz + i] = cast<T>(t);
        sv[r * fsz + HALF + i] = cast<T>(b);
        sw[r * fsz + i] = cast<T>(same ? t : t + b);
        sw[r * fsz + HALF + i] = cast<T>(b);
    }
}

const DeflSet* find_defl(ovd_h h, double mu) {
    for (const auto& d : h->defl)
        if (std::fabs(d.mu - mu) <= 1e-12) return &d;
    return nullptr;
}

// maximal runs of consecutive right-hand sides that share one deflation set
struct Run {
    const DeflSet* set;
    int r0, n;
};
std::vector<Run> defl_runs(ovd_h h, int nrhs, const double* mu) {
    std::vector<Run> runs;
    for (int r = 0; r < nrhs; ++r) {
        const DeflSet* d = find_defl(h, mu[r]);
        if (!runs.empty() && runs.back().set == d) runs.back().n++;
        else runs.push_back({d, r, 1});
    }
    return runs;
}

ovd_status check_handle(ovd_h h) {
    if (!h) return OVD_EINVAL;
    (void)hipGetLastError();   // a failed runtime call of an earlier, finished call is not this call's error
    if (!h->links_set) return fail(h, OVD_EINVAL, "links not set (call ovd_set_links first)");
    return OVD_OK;
}

SmallSignCfg sign_cfg(const ovd_options& o) {
    SmallSignCfg c;
    c.quad_step = o.quad_step;
    c.max_levels = o.quad_max_levels > 0 ? o.quad_max_levels : kDefaultMaxLevels;
    c.chunk = kDefaultChunkSolves;
    return c;
}

// solves per launch of the small sign during an allocation-free call (the
// result does not depend on it; it sizes the scratch: 4 k chunk complex)
constexpr int kNoAllocChunkSolves = 1024;

// map a return code of the small dense solvers to a status
ovd_status small_status(ovd_h h, int rc, const char* what, double chk, int bstep) {
    if (rc == 0) return OVD_OK;
    if (rc == 1)
        return fail(h, OVD_ENOCONV, std::string(what) + ": two successive quadrature levels still differ by " +
                                        std::to_string(chk) + " (> 1e-10) after the last allowed level");
    if (rc == 2)
        return fail(h, OVD_EBREAKDOWN, std::string(what) + ": breakdown of the inner Lanczos run at step " +
                                           std::to_string(bstep));
    return fail(h, OVD_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)(-rc)));
}

// sgn(T_k) e_1 for the nrhs Ritz matrices in co, by the handle's method
ovd_status small_sign(ovd_h h, int nrhs, int k, TslCoeffs co, c64* c_out, double* chk, int* bstep) {
    ovd_status wst = OVD_OK;
    SmallSignCfg cfg = sign_cfg(h->opt);
    if (h->arena.active) cfg.chunk = kNoAllocChunkSolves;
    if (h->opt.sign_method == OVD_SIGN_NESTED) {
        const int kp = std::min(k, h->opt.nested_inner > 0 ? h->opt.nested_inner : 100);
        WS(scr, c64, "small_scratch", nested_sign_scratch_elems(nrhs, k, kp, cfg.chunk));
        const int rc = launch_nested_sign(nrhs, k, co, kp, h->opt.breakdown_tol, cfg, scr, c_out, chk, bstep,
                                          h->stream);
        return small_status(h, rc, "sgn(T_k) e_1 (nested)", *chk, *bstep);
    }
    WS(scr, c64, "small_scratch", small_sign_scratch_elems(nrhs, k, cfg.chunk));
    const int rc = launch_small_sign(nrhs, k, co, cfg, scr, c_out, chk, h->stream);
    return small_status(h, rc, "sgn(T_k) e_1", *chk, -1);
}

// Core two-sided Lanczos run on nrhs systems.
//   dir 0: A = H;  dir 1/2: A = B (d/dmu, d/dlink).
//   src_v/src_w: SoA start vectors (stride fsz per rhs).  xproj: SoA (stride 12*Vp) or null.
//   basis: if non-null, V-hat_1..V-hat_k are kept there ([rhs][k][fsz]).
// ---------------------------------------------------------------------------
// Shared Lanczos steps of an uneven batch.  Each job's host thread runs its
// call up to the Lanczos loop and then hands the loop to the batch: it
// records an event after its preparation and publishes the kernel arguments
// of its k steps (a plan).  The thread that completes the set (the last to
// publish, or the last job to leave without publishing) enqueues, on the
// batch's stream and after every plan's event, one update launch and one
// stencil launch per step for all lattices still running at that step.  Each
// job's stream then waits for that work, and the job finishes on its own.
// ---------------------------------------------------------------------------
struct MultiPlan {
    ovd_h h = nullptr;
    int dir = 0, nrhs = 0, k = 0;
    long long fsz = 0;
    std::vector<StepPtrs> steps;   // kernel arguments of steps 0 .. k-1
    const void* U = nullptr;
    const void* dU = nullptr;
    double md = 0.0;
    TslState* st = nullptr;
    TslCoeffs co{};
    double* partials = nullptr;
    unsigned* counters = nullptr;
    StencilVariant var;            // in: the handle's shape; out: the shape used
};

struct MultiCoord {
    std::mutex m;
    std::condition_variable cv;
    int n = 0, arrived = 0, resigned = 0;
    bool done = false;
    ovd_status status = OVD_OK;
    std::string err;
    std::vector<MultiPlan*> plans;
    std::vector<hipEvent_t> ready;
    void (*lead)(MultiCoord&) = nullptr;   // enqueue the shared steps (precision of the plans)
    hipStream_t stream = nullptr;
    hipEvent_t finished = nullptr;
    void* table = nullptr;                 // TslSegment [max k][plans] on the device

    ~MultiCoord() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (table) (void)hipFree(table);
        for (hipEvent_t e : ready) (void)hipEventDestroy(e);
        if (finished) (void)hipEventDestroy(finished);
        if (stream) (void)hipStreamDestroy(stream);
    }
    // called with m held, once every job has published or left
    void complete() {
        if (lead && !plans.empty()) lead(*this);
        done = true;
        cv.notify_all();
    }
};

// the batch the calling thread's job belongs to (set by ovd_sign_apply_deriv_batch)
thread_local MultiCoord* tls_multi = nullptr;

void multi_resign(MultiCoord& C) {
    std::lock_guard<std::mutex> lk(C.m);
    ++C.resigned;
    if (C.arrived + C.resigned == C.n) C.complete();
}

template <typename T>
void multi_lead(MultiCoord& C) {
    auto bad = [&](const std::string& what, hipError_t e) {
        C.status = OVD_EHIP;
        C.err = "shared Lanczos steps of the batch: " + what + ": " + hipGetErrorString(e);
    };
    const std::vector<MultiPlan*>& P = C.plans;
    const size_t np = P.size();
    // one launch shape for all, by consensus of the lattices' own shapes: one
    // site group per block if every lattice has one, else two; the sequential
    // form (d/dmu only) if every lattice has it, else the paired form; each
    // lattice keeps its XCD order
    int gpb = 1, seq = P[0]->dir == 1 ? 1 : 0;
    for (const MultiPlan* q : P) {
        if (q->var.gpb != 1) gpb = 2;
        if (q->var.seq != 1 || (q->var.gpb != 1 && q->var.gpb != 2)) seq = 0;
    }
    int maxk = 0, maxr = 0;
    for (MultiPlan* q : P) {
        q->var.gpb = gpb;
        q->var.seq = seq;
        if (q->var.map < 0) q->var.map = default_map(q->nrhs);
        maxk = std::max(maxk, q->k);
        maxr = std::max(maxr, q->nrhs);
    }
    std::vector<TslSegment> tab((size_t)maxk * np);
    std::vector<int> nseg(maxk), nblk(maxk), nub(maxk);
    for (int j = 0; j < maxk; ++j) {
        int b0 = 0, u0 = 0, c = 0;
        for (const MultiPlan* q : P) {
            if (q->k <= j) continue;
            TslSegment& S = tab[(size_t)j * np + c++];
            S.g = q->h->g;
            S.ngroups = (S.g.V + 63) / 64;
            S.nrhs = q->nrhs;
            S.map = q->var.map;
            S.nblocks = tsl_stencil_blocks(S.g, q->dir, gpb) * q->nrhs;
            S.block0 = b0;
            b0 += S.nblocks;
            S.unblocks = tsl_update_xblocks(q->fsz);
            S.ublock0 = u0;
            u0 += S.unblocks;
            S.fsz = q->fsz;
            S.tau = q->h->opt.breakdown_tol;
            S.p = q->steps[j];
            S.U = q->U;
            S.dU = q->dU;
            S.mdiag = q->md;
            S.st = q->st;
            S.co = q->co;
            S.partials = q->partials;
            S.counters = q->counters;
        }
        nseg[j] = c;
        nblk[j] = b0;
        nub[j] = u0;
    }
    hipError_t e;
    if ((e = hipMalloc(&C.table, sizeof(TslSegment) * tab.size())) != hipSuccess) return bad("table", e);
    if ((e = hipMemcpy(C.table, tab.data(), sizeof(TslSegment) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return bad("table upload", e);
    if ((e = hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking)) != hipSuccess) return bad("stream", e);
    for (hipEvent_t ev : C.ready)
        if ((e = hipStreamWaitEvent(C.stream, ev, 0)) != hipSuccess) return bad("wait for the jobs", e);
    const TslSegment* dtab = (const TslSegment*)C.table;
    for (int j = 0; j < maxk; ++j)
        launch_tsl_step_multi<T>(P[0]->dir, gpb, seq, j == 0 ? 0 : (j == 1 ? 2 : 3), dtab + (size_t)j * np,
                                 nseg[j], nblk[j], nub[j], maxr, j, C.stream);
    if ((e = hipGetLastError()) != hipSuccess) return bad("launch", e);
    if ((e = hipEventCreateWithFlags(&C.finished, hipEventDisableTiming)) != hipSuccess) return bad("event", e);
    if ((e = hipEventRecord(C.finished, C.stream)) != hipSuccess) return bad("event", e);
}

// publish plan and wait until the batch's steps are enqueued; then the
// handle's stream waits for them
template <typename T>
ovd_status multi_join(ovd_h h, MultiCoord& C, MultiPlan& plan) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, h->stream);
    std::unique_lock<std::mutex> lk(C.m);
    if (e != hipSuccess) {   // leave the batch
        if (ev) (void)hipEventDestroy(ev);
        ++C.resigned;
        if (C.arrived + C.resigned == C.n) C.complete();
        return fail(h, OVD_EHIP, std::string("batch event: ") + hipGetErrorString(e));
    }
    C.ready.push_back(ev);
    C.plans.push_back(&plan);
    C.lead = &multi_lead<T>;
    ++C.arrived;
    if (C.arrived + C.resigned == C.n) C.complete();
    else C.cv.wait(lk, [&] { return C.done; });
    if (C.status != OVD_OK) return fail(h, C.status, C.err);
    HIPCHK(hipStreamWaitEvent(h->stream, C.finished, 0));
    return OVD_OK;
}

template <typename T>
ovd_status run_tsl(ovd_h h, int nrhs, int k, int dir, const double* mu, const cpx<T>* src_v,
                   const cpx<T>* src_w, const cpx<T>* xproj, cpx<T>* basis, c64* c_out, ovd_stats* stats,
                   cpx<T>* basis_w = nullptr, int basis_ring = 0,
                   const std::function<void(int, hipStream_t)>* after_step = nullptr) {
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    const int halves = dir == 0 ? 1 : 2;
    const long long fsz = (long long)halves * 12 * g.Vp;
    const cpx<T>* U = std::is_same<T, double>::value ? (const cpx<T>*)h->U64 : (const cpx<T>*)h->U32;
    const cpx<T>* dU = std::is_same<T, double>::value ? (const cpx<T>*)h->dU64 : (const cpx<T>*)h->dU32;
    const int nb = tsl_stencil_blocks(g, dir, 1);   // the most blocks of any launch shape

    WS(ring, cpx<T>, "tsl_ring", (size_t)10 * nrhs * fsz);
    WS(st, TslState, "tsl_state", nrhs);
    WS(coef, c64, "tsl_coef", (size_t)4 * nrhs * k);
    WS(partials, double, "tsl_partials", (size_t)nrhs * nb * 8);
    WS(counters, unsigned, "tsl_counters", nrhs);
    HIPCHK(hipMemsetAsync(counters, 0, sizeof(unsigned) * nrhs, h->stream));
    HIPCHK(hipMemsetAsync(coef, 0, sizeof(c64) * 4 * nrhs * k, h->stream));
    std::vector<TslState> hs(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        TslState s{};
        s.emu = std::exp(mu[r]);
        s.emu_inv = std::exp(-mu[r]);
        s.min_margin = 1e300;
        hs[r] = s;
    }
    HIPCHK(hipMemcpyAsync(st, hs.data(), sizeof(TslState) * nrhs, hipMemcpyHostToDevice, h->stream));
    TslCoeffs co{coef, coef + (size_t)nrhs * k, coef + (size_t)2 * nrhs * k, coef + (size_t)3 * nrhs * k, k};

    // rotating buffers: V-hat x3, U-hat x2, W-hat x3, Z-hat x2
    auto slot = [&](int base, int i) { return ring + (size_t)(base + i) * nrhs * fsz; };
    // basis: all k right vectors, or with basis_ring > 0 a ring of that many
    // (vector i in slot (i - 1) % basis_ring)
    auto Vs = [&](int i) -> cpx<T>* {
        if (!basis) return slot(0, i % 3);
        return basis + (size_t)(basis_ring > 0 ? (i - 1) % basis_ring : i - 1) * fsz;
    };
    auto Us = [&](int i) -> cpx<T>* { return slot(3, i % 2); };
    auto Ws = [&](int i) -> cpx<T>* { return basis_w ? basis_w + (size_t)(i - 1) * fsz : slot(5, i % 3); };
    auto Zs = [&](int i) -> cpx<T>* { return slot(8, i % 2); };
    const long long sV = basis ? (long long)(basis_ring > 0 ? basis_ring : k) * fsz : fsz;
    const long long sW = basis_w ? (long long)k * fsz : fsz;

    Timer tl, ts;
    // per-kernel events: 4 per step (update start/end, stencil start/end)
    const size_t nev = h->arena.active ? 0 : (size_t)4 * k;
    while (h->ev.size() < nev) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        h->ev.push_back(e);
    }
    tl.start(h->stream, !h->arena.active);
    const double md = h->m0 + 4.0 * h->r;
    // start vectors into slot 1
    HIPCHK(hipMemcpy2DAsync(Vs(1), sizeof(cpx<T>) * sV, src_v, sizeof(cpx<T>) * fsz, sizeof(cpx<T>) * fsz, nrhs,
                            hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemcpy2DAsync(Ws(1), sizeof(cpx<T>) * sW, src_w, sizeof(cpx<T>) * fsz, sizeof(cpx<T>) * fsz, nrhs,
                            hipMemcpyDeviceToDevice, h->stream));
    const bool timing = h->opt.step_timing != 0 && !h->arena.active;
    // launch shape of the stencil: autotuned once per precision, direction and batch size
    StencilVariant var{default_map(nrhs), dir == 0 ? 4 : 2};
    {
        const std::string key = std::string("tsl:") + (sizeof(T) == 8 ? "d" : "f") + ":" + std::to_string(dir) + ":" +
                                std::to_string(nrhs);
        auto it = h->tuned.find(key);
        if (forced_shape(h, nrhs, dir == 0 ? 4 : 2, &var) && var.seq == 3 && dir == 1 &&
            tsl_march_ok(g, (int)sizeof(T))) {
            if (var.gpb > g.L[3]) var.gpb = g.L[3];   // time segments
            h->tuned[key] = var;
        } else if (forced_shape(h, nrhs, dir == 0 ? 4 : 2, &var)) {
            if (var.seq == 3) var.seq = 0;   // the time-marching form does not apply: paired
            if (var.gpb == 8 && !tsl_plane_ok(g)) var.gpb = 0;
            if (var.seq == 2 && (dir != 0 || var.gpb == 8)) var.seq = 0;   // the split form: DIR 0, 1 or 2 groups
            if (dir == 0 && var.seq == 2) {
                if (var.gpb != 1) var.gpb = 2;
            } else if (dir == 0 && var.gpb != 2 && var.gpb != 8) {
                var.gpb = 4;
            }
            if (dir != 0 && var.gpb != 1 && var.gpb != 8) var.gpb = 2;
            if (dir == 2 || var.gpb == 8) var.seq = 0;
            h->tuned[key] = var;
        } else if (it != h->tuned.end()) {
            var = it->second;
        } else if (h->opt.autotune && !h->arena.active) {
            // time step 0 on the start vectors with a scratch copy of the recurrence state
            WS(tst, TslState, "tune_state", nrhs);
            WS(tcoef, c64, "tune_coef", (size_t)4 * nrhs);
            WS(tpart, double, "tune_partials", (size_t)nrhs * nb * 8);
            WS(tcnt, unsigned, "tune_counters", nrhs);
            TslCoeffs tco{tcoef, tcoef + nrhs, tcoef + (size_t)2 * nrhs, tcoef + (size_t)3 * nrhs, 1};
            StepPtrs p0{};
            p0.outV = Vs(1); p0.sV = sV;
            p0.outU = Us(1); p0.sU = fsz;
            p0.outW = Ws(1); p0.sW = sW;
            p0.outZ = Zs(1); p0.sZ = fsz;
            p0.xproj = xproj;
            p0.sx = (long long)12 * g.Vp;
            std::vector<StencilVariant> cands =
                shape_candidates(nrhs,
                                 tsl_plane_ok(g) ? (dir == 0 ? std::vector<int>{4, 2, 8} : std::vector<int>{2, 1, 8})
                                                 : (dir == 0 ? std::vector<int>{4, 2} : std::vector<int>{2, 1}),
                                 dir != 2, dir == 0);
            // the time-marching form (1, 2 or 4 time segments) from 16 right-hand
            // sides on: at 8 the timing of single launches favoured it by a margin
            // that the replayed steps did not show
            if (dir == 1 && nrhs >= 16 && tsl_march_ok(g, (int)sizeof(T)))
                for (int map : {1, 0}) {
                    if (map == 0 && nrhs % 8 != 0) continue;
                    for (int ns : {1, 2, 4})
                        if (ns <= g.L[3]) cands.push_back(StencilVariant{map, ns, 3});
                }
            var = autotune(
                h, cands,
                [&](StencilVariant v) {
                    launch_tsl_stencil<T>(g, dir, nrhs, p0, U, dU, md, tst, tco, tpart, tcnt, 0, h->opt.breakdown_tol,
                                          h->stream, v);
                },
                [&]() {
                    (void)hipMemcpyAsync(tst, hs.data(), sizeof(TslState) * nrhs, hipMemcpyHostToDevice, h->stream);
                    (void)hipMemsetAsync(tcnt, 0, sizeof(unsigned) * nrhs, h->stream);
                });
            HIPCHK(hipGetLastError());
            h->tuned[key] = var;
        }
    }
    // kernel arguments of step j
    auto step_ptrs = [&](int j) {
        StepPtrs p{};
        if (j > 0) {
            p.Xv = Us(j); p.sXv = fsz;
            p.Yv = Vs(j); p.sYv = sV;
            p.Zv = (j >= 2) ? Vs(j - 1) : Vs(j); p.sZv = sV;
            p.Xw = Zs(j); p.sXw = fsz;
            p.Yw = Ws(j); p.sYw = sW;
            p.Zw = (j >= 2) ? Ws(j - 1) : Ws(j); p.sZw = sW;
        }
        p.outV = Vs(j + 1); p.sV = sV;
        p.outU = Us(j + 1); p.sU = fsz;
        p.outW = Ws(j + 1); p.sW = sW;
        p.outZ = Zs(j + 1); p.sZ = fsz;
        p.xproj = xproj;
        p.sx = (long long)12 * g.Vp;
        return p;
    };
    // the k steps: update (from the second step on) and stencil with the step's reductions
    auto enqueue_steps = [&](hipStream_t stream) -> hipError_t {
        for (int j = 0; j < k; ++j) {
            const StepPtrs p = step_ptrs(j);
            if (j > 0) {
                if (timing) (void)hipEventRecord(h->ev[4 * j], stream);
                launch_tsl_update<T>(nrhs, j == 1 ? 2 : 3, fsz, p, st, stream);
                if (timing) (void)hipEventRecord(h->ev[4 * j + 1], stream);
            }
            if (timing) (void)hipEventRecord(h->ev[4 * j + 2], stream);
            launch_tsl_stencil<T>(g, dir, nrhs, p, U, dU, md, st, co, partials, counters, j,
                                  h->opt.breakdown_tol, stream, var);
            if (timing) (void)hipEventRecord(h->ev[4 * j + 3], stream);
            if (after_step) (*after_step)(j, stream);   // right vectors 1 .. j + 1 are final
        }
        return hipGetLastError();
    };
    bool launched = false;
    // the first Lanczos run of a job of a shared-step batch hands its steps to the batch
    if (MultiCoord* C = tls_multi) {
        tls_multi = nullptr;
        if (dir != 0 && !timing && !after_step && !h->arena.active && !h->opt.batch_separate) {
            MultiPlan plan;
            plan.h = h;
            plan.dir = dir;
            plan.nrhs = nrhs;
            plan.k = k;
            plan.fsz = fsz;
            plan.steps.reserve(k);
            for (int j = 0; j < k; ++j) plan.steps.push_back(step_ptrs(j));
            plan.U = U;
            plan.dU = dU;
            plan.md = md;
            plan.st = st;
            plan.co = co;
            plan.partials = partials;
            plan.counters = counters;
            plan.var = var;
            const ovd_status js = multi_join<T>(h, *C, plan);
            if (js != OVD_OK) return js;
            h->tuned[std::string("tsl:") + (sizeof(T) == 8 ? "d" : "f") + ":" + std::to_string(dir) + ":" +
                     std::to_string(nrhs)] = plan.var;
            launched = true;
        } else {
            multi_resign(*C);
        }
    }
    // events and per-call hooks stay out of graphs; an allocation-free call launches one by one
    if (!launched && h->opt.use_graph && !timing && !after_step && !h->arena.active) {
        double tau = h->opt.breakdown_tol;
        uint64_t tb, mb;
        std::memcpy(&tb, &tau, 8);
        std::memcpy(&mb, &md, 8);
        const std::vector<uintptr_t> key = {
            sizeof(T), (uintptr_t)dir, (uintptr_t)nrhs, (uintptr_t)k, (uintptr_t)ring, (uintptr_t)basis,
            (uintptr_t)basis_w, (uintptr_t)xproj, (uintptr_t)U, (uintptr_t)dU, (uintptr_t)st, (uintptr_t)coef,
            (uintptr_t)partials, (uintptr_t)counters, (uintptr_t)tb, (uintptr_t)mb, (uintptr_t)g.V,
            (uintptr_t)var.map, (uintptr_t)var.gpb, (uintptr_t)var.seq};
        hipGraphExec_t exec = nullptr;
        for (auto& e : h->graphs)
            if (e.key == key) exec = e.exec;
        if (!exec) {
            if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
            const hipError_t le = enqueue_steps(h->cap_stream);
            const hipError_t ce = hipStreamEndCapture(h->cap_stream, &graph);
            if (le != hipSuccess || ce != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(h, OVD_EHIP, std::string("recording the Lanczos steps into a graph failed: ") +
                                             hipGetErrorString(le != hipSuccess ? le : ce));
            }
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return fail(h, OVD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
            }
            if (h->graphs.size() >= 8) {   // keep a few shapes; drop the oldest
                (void)hipStreamSynchronize(h->stream);
                (void)hipGraphExecDestroy(h->graphs.front().exec);
                (void)hipGraphDestroy(h->graphs.front().graph);
                h->graphs.erase(h->graphs.begin());
            }
            h->graphs.push_back({key, graph, exec});
        }
        HIPCHK(hipGraphLaunch(exec, h->stream));
        launched = true;
    }
    if (!launched) HIPCHK(enqueue_steps(h->stream));
    HIPCHK(hipGetLastError());
    tl.stop(h->stream);

    // state check (synchronises)
    HIPCHK(hipMemcpyAsync(hs.data(), st, sizeof(TslState) * nrhs, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double minm = 1e300;
    int bstep = -1;
    int bad = 0;
    for (int r = 0; r < nrhs; ++r) {
        if (hs[r].min_margin < minm) minm = hs[r].min_margin;
        if (hs[r].flag) {
            bad = hs[r].flag;
            bstep = hs[r].bstep;
        }
    }
    h->last_nrhs = nrhs;
    h->last_k = k;
    h->last_co = co;
    if (stats) {
        stats->k = k;
        stats->breakdown_step = bstep;
        stats->min_margin = minm;
        stats->ms_lanczos = tl.ms();
        double msu = 0.0, mss = 0.0;
        for (int j = 0; j < (timing ? k : 0); ++j) {
            float t = 0.f;
            if (j > 0 && hipEventElapsedTime(&t, h->ev[4 * j], h->ev[4 * j + 1]) == hipSuccess) msu += t;
            if (hipEventElapsedTime(&t, h->ev[4 * j + 2], h->ev[4 * j + 3]) == hipSuccess) mss += t;
        }
        stats->ms_update = msu;
        stats->ms_stencil = mss;
    }
    if (bad == 1) return fail(h, OVD_EBREAKDOWN, "two-sided Lanczos breakdown at step " + std::to_string(bstep));
    if (bad == 2) return fail(h, OVD_ENAN, "non-finite value in the Lanczos recurrence at step " + std::to_string(bstep));

    // sgn(T_k) e_1
    ts.start(h->stream, !h->arena.active);
    double chk = 0.0;
    int bst = -1;
    const ovd_status ss = small_sign(h, nrhs, k, co, c_out, &chk, &bst);
    ts.stop(h->stream);
    if (stats) {
        stats->ms_small_sign = ts.ms();
        stats->sign_check = chk;
        if (ss == OVD_EBREAKDOWN) stats->breakdown_step = bst;
    }
    return ss;
}

// The vector outputs without a stored basis: the Lanczos run again (same
// kernels, launch shape and inputs, so the same right vectors) with the right
// vectors in a ring of 2C per right-hand side; after every C steps the C
// finished vectors are added into out0 (half 0) and out1 (half 1, nullable)
// with the coefficients cf [nrhs][k].
template <typename T>
ovd_status reconstruct_two_pass(ovd_h h, int nrhs, int k, int dir, const double* mu, const cpx<T>* srcv,
                                const cpx<T>* srcw, const cpx<T>* xp, const c64* cf, long long fsz, void* out0,
                                void* out1) {
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    const int C = std::min(k, 32);
    WS(ring, cpx<T>, "recon_ring", (size_t)nrhs * 2 * C * fsz);
    WS(c2, c64, "ritz_c_pass2", (size_t)nrhs * k);
    int done = 0;   // right vectors already added
    const std::function<void(int, hipStream_t)> hook = [&](int j, hipStream_t stream) {
        const int avail = j + 1;   // right vectors 1 .. j + 1 are final
        if (avail - done < C && avail < k) return;
        const int n = avail - done;
        const cpx<T>* base = ring + (size_t)(done % (2 * C)) * fsz;   // done is a multiple of C: no wrap
        if (out0) launch_reconstruct<T>(g, nrhs, n, base, (long long)2 * C * fsz, fsz, 0, cf + done, k, out0, stream,
                                        done > 0);
        if (out1) launch_reconstruct<T>(g, nrhs, n, base, (long long)2 * C * fsz, fsz, 1, cf + done, k, out1, stream,
                                        done > 0);
        done = avail;
    };
    ovd_status s = run_tsl<T>(h, nrhs, k, dir, mu, srcv, srcw, xp, ring, c2, nullptr, nullptr, 2 * C, &hook);
    if (s != OVD_OK) return s;
    if (done != k) return fail(h, OVD_EHIP, "the regenerated basis did not reach step k");
    return OVD_OK;
}

template <typename T>
ovd_status sign_apply_impl(ovd_h h, int nrhs, const double* mu, int k, const void* b, void* y, ovd_stats* stats) {
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    const long long fsz = (long long)12 * g.Vp;
    const auto runs = defl_runs(h, nrhs, mu);
    int mmax = 0;
    for (const auto& rn : runs)
        if (rn.set && rn.set->m > mmax) mmax = rn.set->m;
    WS(b64, c64, "stage_b", (size_t)nrhs * fsz);
    const bool recompute = recompute_basis(h, sizeof(cpx<T>) * (size_t)nrhs * k * fsz, {"basis_v"}, &wst);
    if (wst != OVD_OK) return wst;
    cpx<T>* basis = nullptr;
    if (!recompute) {
        WS(bb, cpx<T>, "basis_v", (size_t)nrhs * k * fsz);
        basis = bb;
    }
    WS(c, c64, "ritz_c", (size_t)nrhs * k);
    WS(cf, c64, "ritz_coef", (size_t)nrhs * k);
    Timer tt;
    tt.start(h->stream, !h->arena.active);
    HIPCHK(hipMemsetAsync(b64, 0, sizeof(c64) * nrhs * fsz, h->stream));
    launch_pack_spinor<double>(g, nrhs, b, b64, fsz, h->stream);
    // eq. 8: c = L^dag b, b' = b - R c, exact part R (sgn(lambda) c)
    c64* sC = nullptr;
    if (mmax > 0) {
        WS(Cm, c64, "defl_C", (size_t)mmax * nrhs);
        WS(sCm, c64, "defl_sC", (size_t)mmax * nrhs);
        WS(scr, c64, "defl_scr", defl_proj_scratch(mmax, nrhs, fsz));
        sC = sCm;
        for (const auto& rn : runs) {
            if (!rn.set) continue;
            const DeflSet& d = *rn.set;
            c64* bb = b64 + (size_t)rn.r0 * fsz;
            c64* sc = sC + (size_t)rn.r0 * mmax;
            launch_defl_proj(d.L, fsz, d.m, bb, fsz, rn.n, fsz, Cm, scr, h->stream);
            launch_defl_scale(d.m, rn.n, d.ones, Cm, sc, -1.0, h->stream);
            launch_defl_comb(d.R, fsz, d.m, sc, rn.n, bb, fsz, fsz, h->stream);
            launch_defl_scale(d.m, rn.n, d.sgn, Cm, sc, 1.0, h->stream);
        }
    }
    const cpx<T>* src;
    if constexpr (std::is_same<T, double>::value) {
        src = b64;
    } else {
        WS(sv, cpx<T>, "src_v", (size_t)nrhs * fsz);
        launch_convert_field<T>(g, nrhs, b64, fsz, sv, fsz, h->stream);
        src = sv;
    }
    HIPCHK(hipGetLastError());
    ovd_status s = run_tsl<T>(h, nrhs, k, 0, mu, src, src, nullptr, basis, c, stats);
    if (s != OVD_OK) return s;
    dim3 grid((k + 127) / 128, nrhs);
    make_coef_kernel<<<grid, 128, 0, h->stream>>>(k, h->last_co, c, cf);
    if (basis) {
        launch_reconstruct<T>(g, nrhs, k, basis, (long long)k * fsz, fsz, 0, cf, k, y, h->stream);
    } else {
        s = reconstruct_two_pass<T>(h, nrhs, k, 0, mu, src, src, nullptr, cf, fsz, y, nullptr);
        if (s != OVD_OK) return s;
        if (stats) stats->basis_recomputed = 1;
    }
    if (mmax > 0) {
        HIPCHK(hipMemsetAsync(b64, 0, sizeof(c64) * nrhs * fsz, h->stream));
        for (const auto& rn : runs) {
            if (!rn.set) continue;
            c64* bb = b64 + (size_t)rn.r0 * fsz;
            launch_defl_comb(rn.set->R, fsz, rn.set->m, sC + (size_t)rn.r0 * mmax, rn.n, bb, fsz, fsz, h->stream);
        }
        launch_add_soa_to_aos(g, nrhs, b64, fsz, y, h->stream);
    }
    HIPCHK(hipGetLastError());
    tt.stop(h->stream);
    if (stats) stats->ms_total = tt.ms();
    return OVD_OK;
}

// s = (x'^dag b') [sgn(T_k)]_11 + sum_i sgn(lambda_i) conj(d_i) c_i (one thread)
__global__ void vjp_value_kernel(TslCoeffs co, const c64* __restrict__ c, int m, const double* __restrict__ sg,
                                 const c64* __restrict__ cv, const c64* __restrict__ dv, c64* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    c64 v = (co.beta[0] * co.delta[0]) * c[0];
    for (int i = 0; i < m; ++i) v += sg[i] * (conj(dv[i]) * cv[i]);
    *out = v;
}

void launch_vjp_value(TslCoeffs co, const c64* c, int m, const double* sg, const c64* cv, const c64* dv, c64* out,
                      hipStream_t s) {
    vjp_value_kernel<<<1, 64, 0, s>>>(co, c, m, sg, cv, dv, out);
}

// a[i] += b[i] for n complex
__global__ void cadd_kernel(int n, c64* __restrict__ a, const c64* __restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += b[i];
}

// The block method (eq. 6-7) on the source psi = (t; b) (t = 0 when null):
// dy, y = top and bottom halves of sgn(B) psi, deflated by eq. 11 when a set
// for mu exists; with x, the storage-free <x|dy>.
template <typename T>
ovd_status deriv_impl(ovd_h h, int nrhs, const double* mu, int dirk, int k, const void* b, void* y, void* dy,
                      const void* x, double* xdy, ovd_stats* stats, const void* t = nullptr) {
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    const long long half = (long long)12 * g.Vp;
    const long long fsz = 2 * half;
    const bool need_vec = (y != nullptr) || (dy != nullptr);
    const auto runs = defl_runs(h, nrhs, mu);
    int lmax = 0;
    for (const auto& rn : runs)
        if (rn.set && rn.set->l > lmax) lmax = rn.set->l;
    for (const auto& rn : runs)
        if (rn.set && rn.set->l > 0 && rn.set->dir_kind != (dirk == 2 ? OVD_DIR_LINK : OVD_DIR_MU))
            return fail(h, OVD_EINVAL, "deflation set derivatives belong to another direction");
    if (dirk == 2) {   // a set built along one link direction must not serve another
        WS(flag, unsigned, "dir_flag", 1);
        bool any = false;
        HIPCHK(hipMemsetAsync(flag, 0, sizeof(unsigned), h->stream));
        for (const auto& rn : runs)
            if (rn.set && rn.set->l > 0) {
                launch_field_differs((long long)link_elems<double>(g.Vp), h->dU64, rn.set->dir_ref, flag, h->stream);
                any = true;
            }
        if (any) {
            unsigned hf = 0;
            HIPCHK(hipMemcpyAsync(&hf, flag, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            if (hf) return fail(h, OVD_EINVAL, "the deflation set's derivatives belong to another link direction");
        }
    }
    WS(b64, c64, "stage_b", (size_t)nrhs * half);
    WS(t64, c64, "stage_t", (size_t)nrhs * half);
    WS(srcv, cpx<T>, "src_v", (size_t)nrhs * fsz);
    WS(srcw, cpx<T>, "src_w", (size_t)nrhs * fsz);
    cpx<T>* xp = nullptr;
    if (x) {
        WS(xb, cpx<T>, "xproj", (size_t)nrhs * half);
        xp = xb;
    }
    cpx<T>* basis = nullptr;
    bool recompute = false;
    if (need_vec) {
        recompute = recompute_basis(h, sizeof(cpx<T>) * (size_t)nrhs * k * fsz, {"basis_v"}, &wst);
        if (wst != OVD_OK) return wst;
        if (!recompute) {
            WS(bb, cpx<T>, "basis_v", (size_t)nrhs * k * fsz);
            basis = bb;
        }
    }
    WS(c, c64, "ritz_c", (size_t)nrhs * k);
    Timer tt;
    tt.start(h->stream, !h->arena.active);
    // psi = (t; b), deflated by eq. 11: psi' = psi - P_{2l} psi = (t - (R d + dR c); b - R c)
    // with c = L^dag b, d = dL^dag b + L^dag t over the first l pairs
    HIPCHK(hipMemsetAsync(b64, 0, sizeof(c64) * nrhs * half, h->stream));
    HIPCHK(hipMemsetAsync(t64, 0, sizeof(c64) * nrhs * half, h->stream));
    launch_pack_spinor<double>(g, nrhs, b, b64, half, h->stream);
    if (t) launch_pack_spinor<double>(g, nrhs, t, t64, half, h->stream);
    c64 *sC = nullptr, *sD = nullptr;
    if (lmax > 0) {
        WS(Cm, c64, "defl_C", (size_t)lmax * nrhs);
        WS(Dm, c64, "defl_D", (size_t)lmax * nrhs);
        WS(tmp, c64, "defl_tmp", (size_t)lmax * nrhs);
        WS(sCm, c64, "defl_sC", (size_t)lmax * nrhs);
        WS(sDm, c64, "defl_sD", (size_t)lmax * nrhs);
        WS(scr, c64, "defl_scr", defl_proj_scratch(lmax, nrhs, half));
        sC = sCm;
        sD = sDm;
        for (const auto& rn : runs) {
            if (!rn.set || rn.set->l == 0) continue;
            const DeflSet& d = *rn.set;
            const int l = d.l;
            c64* bb = b64 + (size_t)rn.r0 * half;
            c64* tb = t64 + (size_t)rn.r0 * half;
            launch_defl_proj(d.L, half, l, bb, half, rn.n, half, Cm, scr, h->stream);
            launch_defl_proj(d.dL, half, l, bb, half, rn.n, half, Dm, scr, h->stream);
            if (t) {   // d += L^dag t
                launch_defl_proj(d.L, half, l, tb, half, rn.n, half, tmp, scr, h->stream);
                cadd_kernel<<<(l * rn.n + 255) / 256, 256, 0, h->stream>>>(l * rn.n, Dm, tmp);
            }
            launch_defl_scale(l, rn.n, d.ones, Cm, tmp, -1.0, h->stream);
            launch_defl_comb(d.dR, half, l, tmp, rn.n, tb, half, half, h->stream);   // t -= dR c
            launch_defl_comb(d.R, half, l, tmp, rn.n, bb, half, half, h->stream);    // b -= R c
            launch_defl_scale(l, rn.n, d.ones, Dm, tmp, -1.0, h->stream);
            launch_defl_comb(d.R, half, l, tmp, rn.n, tb, half, half, h->stream);    // t -= R d
            launch_defl_scale(l, rn.n, d.sgn, Cm, sC + (size_t)rn.r0 * lmax, 1.0, h->stream);
            launch_defl_scale(l, rn.n, d.sgn, Dm, sD + (size_t)rn.r0 * lmax, 1.0, h->stream);
        }
    }
    {
        dim3 grid((g.V + 255) / 256, nrhs);
        make_block_src_kernel<T><<<grid, 256, 0, h->stream>>>(g, t64, b64, half, srcv, srcw, fsz,
                                                              h->opt.left_start == OVD_LEFT_SAME);
    }
    if (xp) launch_pack_spinor<T>(g, nrhs, x, xp, half, h->stream);
    HIPCHK(hipGetLastError());
    ovd_status s = run_tsl<T>(h, nrhs, k, dirk, mu, srcv, srcw, xp, basis, c, stats);
    if (s != OVD_OK) return s;
    if (need_vec) {
        WS(cf, c64, "ritz_coef", (size_t)nrhs * k);
        dim3 grid((k + 127) / 128, nrhs);
        make_coef_kernel<<<grid, 128, 0, h->stream>>>(k, h->last_co, c, cf);
        if (basis) {
            if (dy) launch_reconstruct<T>(g, nrhs, k, basis, (long long)k * fsz, fsz, 0, cf, k, dy, h->stream);
            if (y) launch_reconstruct<T>(g, nrhs, k, basis, (long long)k * fsz, fsz, 1, cf, k, y, h->stream);
        } else {
            s = reconstruct_two_pass<T>(h, nrhs, k, dirk, mu, srcv, srcw, xp, cf, fsz, dy, y);
            if (s != OVD_OK) return s;
            if (stats) stats->basis_recomputed = 1;
        }
        if (lmax > 0) {
            // exact part: top R (s d) + dR (s c), bottom R (s c)
            HIPCHK(hipMemsetAsync(b64, 0, sizeof(c64) * nrhs * half, h->stream));
            HIPCHK(hipMemsetAsync(t64, 0, sizeof(c64) * nrhs * half, h->stream));
            for (const auto& rn : runs) {
                if (!rn.set || rn.set->l == 0) continue;
                const DeflSet& d = *rn.set;
                c64* bb = b64 + (size_t)rn.r0 * half;
                c64* tb = t64 + (size_t)rn.r0 * half;
                launch_defl_comb(d.R, half, d.l, sD + (size_t)rn.r0 * lmax, rn.n, tb, half, half, h->stream);
                launch_defl_comb(d.dR, half, d.l, sC + (size_t)rn.r0 * lmax, rn.n, tb, half, half, h->stream);
                launch_defl_comb(d.R, half, d.l, sC + (size_t)rn.r0 * lmax, rn.n, bb, half, half, h->stream);
            }
            if (dy) launch_add_soa_to_aos(g, nrhs, t64, half, dy, h->stream);
            if (y) launch_add_soa_to_aos(g, nrhs, b64, half, y, h->stream);
        }
    }
    if (xdy) {
        WS(outd, c64, "scalar_out", nrhs);
        launch_scalar_dot(nrhs, k, c, h->last_co.proj, k, h->last_co.delta, outd, h->stream);
        if (lmax > 0) {
            // <x| R (s d) + dR (s c)> = sum_i conj(R_i^dag x) s_i d_i + conj(dR_i^dag x) s_i c_i
            WS(x64, c64, "stage_x", (size_t)nrhs * half);
            WS(P1, c64, "defl_P1", (size_t)lmax * nrhs);
            WS(P2, c64, "defl_P2", (size_t)lmax * nrhs);
            WS(scr, c64, "defl_scr", defl_proj_scratch(lmax, nrhs, half));
            HIPCHK(hipMemsetAsync(x64, 0, sizeof(c64) * nrhs * half, h->stream));
            launch_pack_spinor<double>(g, nrhs, x, x64, half, h->stream);
            for (const auto& rn : runs) {
                if (!rn.set || rn.set->l == 0) continue;
                const DeflSet& d = *rn.set;
                const c64* xb = x64 + (size_t)rn.r0 * half;
                launch_defl_proj(d.R, half, d.l, xb, half, rn.n, half, P1, scr, h->stream);
                launch_defl_proj(d.dR, half, d.l, xb, half, rn.n, half, P2, scr, h->stream);
                launch_defl_scalar(d.l, rn.n, P1, sD + (size_t)rn.r0 * lmax, P2, sC + (size_t)rn.r0 * lmax,
                                   outd + rn.r0, h->stream);
            }
        }
        HIPCHK(hipMemcpyAsync(xdy, outd, sizeof(c64) * nrhs, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipGetLastError());
    tt.stop(h->stream);
    if (stats) stats->ms_total = tt.ms();
    HIPCHK(hipStreamSynchronize(h->stream));
    return OVD_OK;
}

ovd_status upload_dir(ovd_h h, const ovd_dir* dir, int* dirk) {
    ovd_status wst = OVD_OK;
    if (!dir || dir->kind == OVD_DIR_MU) {
        *dirk = 1;
        return OVD_OK;
    }
    if (dir->kind != OVD_DIR_LINK || !dir->dU) return fail(h, OVD_EINVAL, "bad derivative direction");
    WS(d64, c64, "dU64", link_elems<double>(h->g.Vp));
    c32* d32 = nullptr;
    if (h->opt.precision == OVD_MIXED) {
        WS(t32, c32, "dU32", link_elems<float>(h->g.Vp));
        d32 = t32;
    }
    launch_pack_links(h->g, dir->dU, d64, d32, h->stream);
    HIPCHK(hipGetLastError());
    h->dU64 = d64;
    h->dU32 = d32;
    *dirk = 2;
    return OVD_OK;
}

}  // namespace

bool options_ok(const ovd_options& o) {
    return (o.precision == OVD_FP64 || o.precision == OVD_MIXED) && o.quad_max_levels >= 0 &&
           o.quad_max_levels <= kMaxLevelsLimit && (o.sign_method == OVD_SIGN_QUAD || o.sign_method == OVD_SIGN_NESTED) &&
           o.nested_inner >= 0 && o.mem_budget >= 0 && o.eig_shift_max >= 0 &&
           (o.batch_separate == 0 || o.batch_separate == 1);
}

extern "C" {

ovd_status ovd_create_lattice(const int dims[4], double m0, double r, int t_bc, const ovd_options* opt,
                              void* stream, ovd_h* out) {
    if (!dims || !out) return OVD_EINVAL;
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2) return OVD_EINVAL;
    if (r != 1.0) return OVD_EINVAL;
    if (t_bc != 1 && t_bc != -1) return OVD_EINVAL;
    const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    if (V > (1LL << 28)) return OVD_EINVAL;
    ovd_lattice* h = new ovd_lattice();
    for (int i = 0; i < 4; ++i) h->g.L[i] = dims[i];
    h->g.V = (int)V;
    h->g.Vp = (int)((V + 63) / 64 * 64);
    h->g.bc_t = t_bc;
    h->m0 = m0;
    h->r = r;
    h->opt.precision = OVD_FP64;
    h->opt.left_start = OVD_LEFT_SUM;
    h->opt.breakdown_tol = 1e-14;
    h->opt.quad_step = 0.1;
    h->opt.step_timing = 0;
    h->opt.use_graph = 1;
    h->opt.autotune = 1;
    h->opt.shape_map = -1;
    h->opt.shape_gpb = 0;
    h->opt.shape_seq = -1;
    h->opt.shape_rp = 0;
    h->opt.basis_recompute = -1;
    h->opt.quad_max_levels = 0;
    h->opt.sign_method = OVD_SIGN_QUAD;
    h->opt.nested_inner = 0;
    h->opt.mem_budget = 0;
    h->opt.eig_shift_max = 0;
    if (opt) {
        if (!options_ok(*opt)) {
            delete h;
            return OVD_EINVAL;
        }
        h->opt = *opt;
        if (h->opt.breakdown_tol <= 0) h->opt.breakdown_tol = 1e-14;
        if (h->opt.quad_step <= 0) h->opt.quad_step = 0.1;
    }
    h->stream = (hipStream_t)stream;
    *out = h;
    return OVD_OK;
}

ovd_status ovd_destroy(ovd_h h) {
    if (!h) return OVD_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->ws) (void)hipFree(kv.second.first);
    for (auto e : h->ev) (void)hipEventDestroy(e);
    for (auto& e : h->graphs) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
    }
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->U64) (void)hipFree(h->U64);
    if (h->U32) (void)hipFree(h->U32);
    if (h->blas) (void)rocblas_destroy_handle(h->blas);
    ovd_clear_deflation(h);
    delete h;
    return OVD_OK;
}

const char* ovd_last_error(ovd_h h) { return h ? h->err.c_str() : "null handle"; }

ovd_status ovd_set_stream(ovd_h h, void* stream) {
    if (!h) return OVD_EINVAL;
    h->stream = (hipStream_t)stream;
    return OVD_OK;
}

ovd_status ovd_set_links(ovd_h h, const void* U) {
    if (!h) return OVD_EINVAL;
    (void)hipGetLastError();
    if (!U) return fail(h, OVD_EINVAL, "null link pointer");
    if (!h->U64) HIPCHK(hipMalloc(&h->U64, link_elems<double>(h->g.Vp) * sizeof(c64)));
    if (h->opt.precision == OVD_MIXED && !h->U32) HIPCHK(hipMalloc(&h->U32, link_elems<float>(h->g.Vp) * sizeof(c32)));
    // the eigenvectors of any deflation set belong to the old links
    if (!h->defl.empty()) ovd_clear_deflation(h);
    launch_pack_links(h->g, U, h->U64, h->U32, h->stream);
    HIPCHK(hipGetLastError());
    h->links_set = true;
    return OVD_OK;
}

ovd_status ovd_apply_op(ovd_h h, int op, double mu, const ovd_dir* dir, int nrhs, const void* in, void* out,
                        double* ms) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (!in || !out || nrhs < 1 || op < 0 || op > 3) return fail(h, OVD_EINVAL, "bad ovd_apply_op arguments");
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    if (op == OVD_OP_DH_DLINK) {
        if (!dir || dir->kind != OVD_DIR_LINK) return fail(h, OVD_EINVAL, "OVD_OP_DH_DLINK needs a link direction");
        int dk;
        s = upload_dir(h, dir, &dk);
        if (s != OVD_OK) return s;
    }
    const long long fsz = (long long)12 * g.Vp;
    WS(emu, double, "emu", 2 * nrhs);
    std::vector<double> he(2 * nrhs);
    for (int r = 0; r < nrhs; ++r) {
        he[2 * r] = std::exp(mu);
        he[2 * r + 1] = std::exp(-mu);
    }
    HIPCHK(hipMemcpyAsync(emu, he.data(), sizeof(double) * 2 * nrhs, hipMemcpyHostToDevice, h->stream));
    Timer t;
    const double md = h->m0 + 4 * h->r;
    const bool f32 = h->opt.precision == OVD_MIXED;
    const std::string key = std::string("op:") + (f32 ? "f" : "d") + ":" + std::to_string(op) + ":" +
                            std::to_string(nrhs);
    if (f32) {
        WS(a, c32, "op_in", (size_t)nrhs * fsz);
        WS(b, c32, "op_out", (size_t)nrhs * fsz);
        launch_pack_spinor<float>(g, nrhs, in, a, fsz, h->stream);
        auto launch = [&](StencilVariant v) {
            launch_apply_op<float>(g, op, nrhs, emu, h->U32, h->dU32, md, a, b, h->stream, v);
        };
        StencilVariant fv;
        if (forced_shape(h, nrhs, 4, &fv)) {
            op_shape_sanitize(fv, op, nrhs, g);
            h->tuned[key] = fv;
        } else if (!h->tuned.count(key)) {
            h->tuned[key] = h->opt.autotune ? autotune(h, op_candidates(nrhs, op, tsl_plane_ok(g)), launch, [] {})
                                            : StencilVariant{default_map(nrhs), 4};
        }
        t.start(h->stream);
        launch(h->tuned[key]);
        t.stop(h->stream);
        launch_unpack_spinor<float>(g, nrhs, b, fsz, out, h->stream);
    } else {
        WS(a, c64, "op_in", (size_t)nrhs * fsz);
        WS(b, c64, "op_out", (size_t)nrhs * fsz);
        launch_pack_spinor<double>(g, nrhs, in, a, fsz, h->stream);
        auto launch = [&](StencilVariant v) {
            launch_apply_op<double>(g, op, nrhs, emu, h->U64, h->dU64, md, a, b, h->stream, v);
        };
        StencilVariant fv;
        if (forced_shape(h, nrhs, 4, &fv)) {
            op_shape_sanitize(fv, op, nrhs, g);
            h->tuned[key] = fv;
        } else if (!h->tuned.count(key)) {
            h->tuned[key] = h->opt.autotune ? autotune(h, op_candidates(nrhs, op, tsl_plane_ok(g)), launch, [] {})
                                            : StencilVariant{default_map(nrhs), 4};
        }
        t.start(h->stream);
        launch(h->tuned[key]);
        t.stop(h->stream);
        launch_unpack_spinor<double>(g, nrhs, b, fsz, out, h->stream);
    }
    HIPCHK(hipGetLastError());
    if (ms) *ms = t.ms();
    return OVD_OK;
}

ovd_status ovd_sign_apply(ovd_h h, int nrhs, const double* mu, int k, const void* b, void* y, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !b || !y) return fail(h, OVD_EINVAL, "bad ovd_sign_apply arguments");
    if (st) std::memset(st, 0, sizeof(*st));
    if (h->opt.precision == OVD_MIXED) return sign_apply_impl<float>(h, nrhs, mu, k, b, y, st);
    return sign_apply_impl<double>(h, nrhs, mu, k, b, y, st);
}

ovd_status ovd_sign_apply_deriv(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* b,
                                void* y, void* dy, const void* x, double* xdy, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !b) return fail(h, OVD_EINVAL, "bad ovd_sign_apply_deriv arguments");
    if (!y && !dy && !(x && xdy)) return fail(h, OVD_EINVAL, "no output requested");
    if (xdy && !x) return fail(h, OVD_EINVAL, "xdy requested without x");
    if (st) std::memset(st, 0, sizeof(*st));
    int dirk = 1;
    s = upload_dir(h, dir, &dirk);
    if (s != OVD_OK) return s;
    if (h->opt.precision == OVD_MIXED) return deriv_impl<float>(h, nrhs, mu, dirk, k, b, y, dy, x, xdy, st);
    return deriv_impl<double>(h, nrhs, mu, dirk, k, b, y, dy, x, xdy, st);
}

ovd_status ovd_block_sign_apply(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* t,
                                const void* b, void* yt, void* yb, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !b || (!yt && !yb)) return fail(h, OVD_EINVAL, "bad ovd_block_sign_apply arguments");
    if (st) std::memset(st, 0, sizeof(*st));
    int dirk = 1;
    s = upload_dir(h, dir, &dirk);
    if (s != OVD_OK) return s;
    if (h->opt.precision == OVD_MIXED)
        return deriv_impl<float>(h, nrhs, mu, dirk, k, b, yb, yt, nullptr, nullptr, st, t);
    return deriv_impl<double>(h, nrhs, mu, dirk, k, b, yb, yt, nullptr, nullptr, st, t);
}

ovd_status ovd_deriv_error_estimate(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* phi,
                                    double* eps, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !phi || !eps) return fail(h, OVD_EINVAL, "bad ovd_deriv_error_estimate arguments");
    ovd_status wst = OVD_OK;
    const long long ns = (long long)nrhs * h->g.V;
    WS(t1, c64, "eps_t1", (size_t)ns * 12);
    WS(b1, c64, "eps_b1", (size_t)ns * 12);
    WS(t2, c64, "eps_t2", (size_t)ns * 12);
    WS(b2, c64, "eps_b2", (size_t)ns * 12);
    WS(e, double, "eps_out", nrhs);
    // sgn(B) (0; phi), then sgn(B) applied to that full block vector
    s = ovd_block_sign_apply(h, nrhs, mu, dir, k, nullptr, phi, t1, b1, st);
    if (s != OVD_OK) return s;
    s = ovd_block_sign_apply(h, nrhs, mu, dir, k, t1, b1, t2, b2, nullptr);
    if (s != OVD_OK) return s;
    launch_half_rel_diff(nrhs, (long long)h->g.V * 12, b2, phi, e, h->stream, t2);
    HIPCHK(hipMemcpyAsync(eps, e, sizeof(double) * nrhs, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return OVD_OK;
}

ovd_status ovd_overlap_apply(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* b,
                             void* Db, void* dDb, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !b || (!Db && !dDb)) return fail(h, OVD_EINVAL, "bad ovd_overlap_apply arguments");
    const long long ns = (long long)nrhs * h->g.V;
    if (!dDb) {
        s = ovd_sign_apply(h, nrhs, mu, k, b, Db, st);                       // Db = sgn(H) b
        if (s != OVD_OK) return s;
        launch_gamma5_axpy(ns, 1.0, b, 1.0, Db, Db, h->stream);             // Db = b + gamma5 sgn(H) b
    } else {
        ovd_status wst = OVD_OK;
        void* y = Db;
        if (!y) {
            WS(tmp, c64, "overlap_y", (size_t)ns * 12);
            y = tmp;
        }
        s = ovd_sign_apply_deriv(h, nrhs, mu, dir, k, b, y, dDb, nullptr, nullptr, st);
        if (s != OVD_OK) return s;
        launch_gamma5_axpy(ns, 0.0, nullptr, 1.0, dDb, dDb, h->stream);      // d D b = gamma5 d sgn(H) b
        if (Db) launch_gamma5_axpy(ns, 1.0, b, 1.0, Db, Db, h->stream);
    }
    HIPCHK(hipGetLastError());
    return OVD_OK;
}

ovd_status ovd_sign_error_estimate(ovd_h h, int nrhs, const double* mu, int k, const void* b, double* eps,
                                   ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !b || !eps) return fail(h, OVD_EINVAL, "bad ovd_sign_error_estimate arguments");
    ovd_status wst = OVD_OK;
    const long long ns = (long long)nrhs * h->g.V;
    WS(y, c64, "eps_y", (size_t)ns * 12);
    WS(z, c64, "eps_z", (size_t)ns * 12);
    WS(e, double, "eps_out", nrhs);
    s = ovd_sign_apply(h, nrhs, mu, k, b, y, st);
    if (s != OVD_OK) return s;
    s = ovd_sign_apply(h, nrhs, mu, k, y, z, nullptr);
    if (s != OVD_OK) return s;
    launch_half_rel_diff(nrhs, (long long)h->g.V * 12, z, b, e, h->stream);
    HIPCHK(hipMemcpyAsync(eps, e, sizeof(double) * nrhs, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return OVD_OK;
}

ovd_status ovd_sign_apply_deriv_batch(int njobs, ovd_deriv_job* jobs) {
    if (njobs < 1 || !jobs) return OVD_EINVAL;
    for (int i = 0; i < njobs; ++i) {
        if (!jobs[i].h) return OVD_EINVAL;
        for (int j = 0; j < i; ++j)
            if (jobs[j].h == jobs[i].h) {
                jobs[i].status = fail(jobs[i].h, OVD_EINVAL, "a handle appears twice in one batch");
                return OVD_EINVAL;
            }
    }
    // shared Lanczos steps when the lattices allow one kernel for all of them
    bool shared = njobs > 1;
    const int kind0 = jobs[0].dir ? jobs[0].dir->kind : OVD_DIR_MU;
    for (int i = 0; i < njobs; ++i) {
        const int kind = jobs[i].dir ? jobs[i].dir->kind : OVD_DIR_MU;
        if (jobs[i].h->opt.precision != jobs[0].h->opt.precision || kind != kind0 || jobs[i].h->opt.batch_separate)
            shared = false;
    }
    MultiCoord C;
    C.n = njobs;
    // one host thread per lattice: each call enqueues on its handle's stream
    // and waits only for its own results (and for the shared steps), so the
    // lattices run side by side
    auto run = [&](int i) {
        ovd_deriv_job& J = jobs[i];
        tls_multi = shared ? &C : nullptr;
        J.status = ovd_sign_apply_deriv(J.h, J.nrhs, J.mu, J.dir, J.k, J.b, J.y, J.dy, J.x, J.xdy, J.st);
        if (tls_multi) {   // left before its Lanczos steps
            tls_multi = nullptr;
            multi_resign(C);
        }
    };
    std::vector<std::thread> pool;
    pool.reserve(njobs - 1);
    for (int i = 1; i < njobs; ++i) pool.emplace_back(run, i);
    run(0);
    for (auto& t : pool) t.join();
    for (int i = 0; i < njobs; ++i)
        if (jobs[i].status != OVD_OK) return jobs[i].status;
    return OVD_OK;
}

ovd_status ovd_get_tuned(ovd_h h, char* buf, int len) {
    if (!h || !buf || len < 1) return OVD_EINVAL;
    std::string out;
    for (const auto& kv : h->tuned)
        out += kv.first + "=map" + std::to_string(kv.second.map) + ",gpb" + std::to_string(kv.second.gpb) +
               (kv.second.seq == 3 ? ",march" : kv.second.seq == 2 ? ",split" : kv.second.seq ? ",seq" : "") +
               (kv.second.rp == 2 ? ",rp2;" : ";");
    std::strncpy(buf, out.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
    return OVD_OK;
}

ovd_status ovd_get_tridiag(ovd_h h, int rhs, int k, double* alpha, double* beta, double* delta) {
    if (!h) return OVD_EINVAL;
    if (rhs < 0 || rhs >= h->last_nrhs || k < 1 || k > h->last_k)
        return fail(h, OVD_EINVAL, "no such Lanczos run / rhs / k");
    const TslCoeffs& co = h->last_co;
    const size_t off = (size_t)rhs * co.kmax;
    if (alpha) HIPCHK(hipMemcpy(alpha, co.alpha + off, sizeof(c64) * k, hipMemcpyDeviceToHost));
    if (beta) HIPCHK(hipMemcpy(beta, co.beta + off, sizeof(c64) * k, hipMemcpyDeviceToHost));
    if (delta) HIPCHK(hipMemcpy(delta, co.delta + off, sizeof(c64) * k, hipMemcpyDeviceToHost));
    return OVD_OK;
}

}  // extern "C"

void free_defl(DeflSet& d) {
    for (void* q : {(void*)d.R, (void*)d.L, (void*)d.dR, (void*)d.dL, (void*)d.dir_ref, (void*)d.sgn, (void*)d.ones})
        if (q) (void)hipFree(q);
    d = DeflSet{};
}

// a device copy of the packed link direction that dR, dL belong to
ovd_status tag_direction(ovd_h h, DeflSet& d, const c64* packed) {
    const size_t n = link_elems<double>(h->g.Vp);
    if (hipMalloc(&d.dir_ref, sizeof(c64) * n) != hipSuccess) return fail(h, OVD_ENOMEM, "deflation direction copy");
    HIPCHK(hipMemcpyAsync(d.dir_ref, packed, sizeof(c64) * n, hipMemcpyDeviceToDevice, h->stream));
    return OVD_OK;
}

// finish a deflation set whose vectors are on the device: upload sgn(lambda),
// check L^dag R = 1, replace any set of the same mu
template <typename Release>
ovd_status install_defl(ovd_h h, DeflSet& d, const std::vector<double>& sg, const std::vector<double>& on,
                        Release release) {
    ovd_status wst = OVD_OK;
    const int m = d.m;
    const long long nf = (long long)12 * h->g.Vp;
    const double mu = d.mu;
    (void)hipMemcpyAsync(d.sgn, sg.data(), sizeof(double) * m, hipMemcpyHostToDevice, h->stream);
    (void)hipMemcpyAsync(d.ones, on.data(), sizeof(double) * m, hipMemcpyHostToDevice, h->stream);
    // biorthonormality L^dag R = 1 (checked on the device, FP64)
    c64* G = (c64*)ws_get(h, "defl_gram", sizeof(c64) * (size_t)m * m, &wst);
    c64* scr = (c64*)ws_get(h, "defl_scr", sizeof(c64) * defl_proj_scratch(m, m, nf), &wst);
    if (!G || !scr) {
        release();
        return wst;
    }
    launch_defl_proj(d.L, nf, m, d.R, nf, m, nf, G, scr, h->stream);
    std::vector<c64> hg((size_t)m * m);
    if (hipMemcpyAsync(hg.data(), G, sizeof(c64) * m * m, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        release();
        return fail(h, OVD_EHIP, "deflation set upload failed");
    }
    double dev = 0.0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            const c64 e = hg[(size_t)i * m + j] - c64{i == j ? 1.0 : 0.0, 0.0};
            dev = std::max(dev, std::sqrt(norm2(e)));
        }
    if (!(dev <= 1e-8)) {
        release();
        return fail(h, OVD_EINVAL, "deflation vectors are not biorthonormal: max |L^dag R - 1| = " + std::to_string(dev));
    }
    for (auto it = h->defl.begin(); it != h->defl.end(); ++it) {
        if (std::fabs(it->mu - mu) <= 1e-12) {
            free_defl(*it);
            h->defl.erase(it);
            break;
        }
    }
    h->defl.push_back(d);
    return OVD_OK;
}


extern "C" {

ovd_status ovd_set_deflation(ovd_h h, double mu, int m, const double* lam, const void* R, const void* L, int l,
                             const void* dR, const void* dL, const ovd_dir* dir) {
    if (!h) return OVD_EINVAL;
    if (m < 1 || !lam || !R || !L || l < 0 || l > m || (l > 0 && (!dR || !dL)))
        return fail(h, OVD_EINVAL, "bad ovd_set_deflation arguments");
    if (l > 0 && dir && dir->kind == OVD_DIR_LINK && !dir->dU)
        return fail(h, OVD_EINVAL, "deflation derivatives along a link direction need that direction (dir->dU)");
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    const long long nf = (long long)12 * g.Vp;
    DeflSet d;
    d.mu = mu;
    d.m = m;
    d.l = l;
    d.dir_kind = (dir && dir->kind == OVD_DIR_LINK) ? OVD_DIR_LINK : OVD_DIR_MU;
    d.lam.resize(m);
    std::vector<double> sg(m), on(m, 1.0);
    for (int i = 0; i < m; ++i) {
        d.lam[i] = c64{lam[2 * i], lam[2 * i + 1]};
        sg[i] = lam[2 * i] >= 0.0 ? 1.0 : -1.0;   // sgn(Re lambda)
    }
    auto alloc = [&](c64** p, int n) -> hipError_t {
        hipError_t e = hipMalloc(p, sizeof(c64) * (size_t)n * nf);
        if (e == hipSuccess) e = hipMemsetAsync(*p, 0, sizeof(c64) * (size_t)n * nf, h->stream);
        return e;
    };
    auto release = [&]() { free_defl(d); };
    if (alloc(&d.R, m) != hipSuccess || alloc(&d.L, m) != hipSuccess ||
        (l > 0 && (alloc(&d.dR, l) != hipSuccess || alloc(&d.dL, l) != hipSuccess)) ||
        hipMalloc(&d.sgn, sizeof(double) * m) != hipSuccess || hipMalloc(&d.ones, sizeof(double) * m) != hipSuccess) {
        release();
        return fail(h, OVD_ENOMEM, "device allocation of the deflation set failed");
    }
    launch_pack_spinor<double>(g, m, R, d.R, nf, h->stream);
    launch_pack_spinor<double>(g, m, L, d.L, nf, h->stream);
    if (l > 0) {
        launch_pack_spinor<double>(g, l, dR, d.dR, nf, h->stream);
        launch_pack_spinor<double>(g, l, dL, d.dL, nf, h->stream);
    }
    if (l > 0 && d.dir_kind == OVD_DIR_LINK) {
        int dk = 0;
        ovd_status s2 = upload_dir(h, dir, &dk);
        if (s2 == OVD_OK) s2 = tag_direction(h, d, h->dU64);
        if (s2 != OVD_OK) {
            release();
            return s2;
        }
    }
    return install_defl(h, d, sg, on, release);
}

ovd_status ovd_compute_deflation(ovd_h h, double mu, int m, int l, const ovd_dir* dir, double tol, double* lam,
                                 ovd_eig_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (m < 1 || l < 0 || l > m || m > 512) return fail(h, OVD_EINVAL, "bad ovd_compute_deflation arguments");
    if (st) std::memset(st, 0, sizeof(*st));
    int dk = 1;
    if (l > 0) {
        s = upload_dir(h, dir, &dk);
        if (s != OVD_OK) return s;
    }
    EigParams P;
    P.g = h->g;
    P.U = h->U64;
    P.dU = h->dU64;
    P.md = h->m0 + 4.0 * h->r;
    P.mu = mu;
    P.m = m;
    P.l = l;
    P.dir_link = dk == 2;
    if (tol > 0) P.tol = tol;
    if (h->opt.eig_shift_max > 0) P.shift_max = h->opt.eig_shift_max;
    P.stream = h->stream;
    EigResult R;
    const int rc = eigs_compute(P, R);
    if (st) {
        st->outer_right = R.outer_right;
        st->outer_left = R.outer_left;
        st->max_res_right = R.res_right;
        st->max_res_left = R.res_left;
        st->max_biorth = R.biorth;
        st->shift_iters = R.shift_iters;
        st->max_shift_res = R.shift_res;
        st->ms = R.ms;
    }
    if (rc != 0) {
        for (void* q : {(void*)R.R, (void*)R.L, (void*)R.dR, (void*)R.dL})
            if (q) (void)hipFree(q);
        const ovd_status code = rc == -2 ? OVD_ENOMEM : rc == -3 ? OVD_EHIP : OVD_ENOCONV;
        return fail(h, code, R.err);
    }
    DeflSet d;
    d.mu = mu;
    d.m = m;
    d.l = l;
    d.dir_kind = dk == 2 ? OVD_DIR_LINK : OVD_DIR_MU;
    d.lam = R.lam;
    d.R = R.R;
    d.L = R.L;
    d.dR = R.dR;
    d.dL = R.dL;
    std::vector<double> sg(m), on(m, 1.0);
    for (int i = 0; i < m; ++i) {
        sg[i] = R.lam[i].re >= 0.0 ? 1.0 : -1.0;
        if (lam) {
            lam[2 * i] = R.lam[i].re;
            lam[2 * i + 1] = R.lam[i].im;
        }
    }
    auto release = [&]() { free_defl(d); };
    if (hipMalloc(&d.sgn, sizeof(double) * m) != hipSuccess || hipMalloc(&d.ones, sizeof(double) * m) != hipSuccess) {
        release();
        return fail(h, OVD_ENOMEM, "device allocation of the deflation set failed");
    }
    if (l > 0 && d.dir_kind == OVD_DIR_LINK) {
        const ovd_status s2 = tag_direction(h, d, h->dU64);
        if (s2 != OVD_OK) {
            release();
            return s2;
        }
    }
    return install_defl(h, d, sg, on, release);
}

ovd_status ovd_get_deflation(ovd_h h, double mu, int* m, int* l, double* lam, void* R, void* L, void* dR, void* dL) {
    if (!h) return OVD_EINVAL;
    const DeflSet* d = find_defl(h, mu);
    if (!d) return fail(h, OVD_ENODEFL, "no deflation set for this mu");
    if (m) *m = d->m;
    if (l) *l = d->l;
    if (lam)
        for (int i = 0; i < d->m; ++i) {
            lam[2 * i] = d->lam[i].re;
            lam[2 * i + 1] = d->lam[i].im;
        }
    const long long nf = (long long)12 * h->g.Vp;
    if (R) launch_unpack_spinor<double>(h->g, d->m, d->R, nf, R, h->stream);
    if (L) launch_unpack_spinor<double>(h->g, d->m, d->L, nf, L, h->stream);
    if (dR && d->l > 0) launch_unpack_spinor<double>(h->g, d->l, d->dR, nf, dR, h->stream);
    if (dL && d->l > 0) launch_unpack_spinor<double>(h->g, d->l, d->dL, nf, dL, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return OVD_OK;
}

ovd_status ovd_clear_deflation(ovd_h h) {
    if (!h) return OVD_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    for (auto& d : h->defl) free_defl(d);
    h->defl.clear();
    return OVD_OK;
}

// Z = W M'^dag for k fields W (field q at W + q sW, nf elements each):
// z_p[n] = sum_q w_q[n] conj(M'[p][q]).  A plain N x k x k complex GEMM, run by
// rocBLAS (column-major: Z (nf x k, ld sZ) = W (nf x k, ld sW) Mc (k x k,
// ld k) with Mc = conj(M') elementwise, the k x k matrix M' being stored
// row-major), with atomics off so that the result does not depend on the run.
ovd_status zgemm_w_mdag(ovd_h h, const c64* W, long long sW, int k, const c64* Mc, c64* Z, long long sZ,
                        long long nf) {
    if (nf > INT32_MAX || sW > INT32_MAX || sZ > INT32_MAX) return fail(h, OVD_EINVAL, "field too long for the GEMM");
    if (!h->blas) {
        if (rocblas_create_handle(&h->blas) != rocblas_status_success) {
            h->blas = nullptr;
            return fail(h, OVD_EHIP, "rocblas_create_handle failed");
        }
        (void)rocblas_set_atomics_mode(h->blas, rocblas_atomics_not_allowed);
    }
    if (rocblas_set_stream(h->blas, h->stream) != rocblas_status_success)
        return fail(h, OVD_EHIP, "rocblas_set_stream failed");
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    const rocblas_status rs =
        rocblas_zgemm(h->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)nf, k, k, &one,
                      reinterpret_cast<const rocblas_double_complex*>(W), (rocblas_int)sW,
                      reinterpret_cast<const rocblas_double_complex*>(Mc), k, &zero,
                      reinterpret_cast<rocblas_double_complex*>(Z), (rocblas_int)sZ);
    if (rs != rocblas_status_success)
        return fail(h, OVD_EHIP, std::string("rocblas_zgemm: ") + rocblas_status_to_string(rs));
    return OVD_OK;
}

ovd_status ovd_sign_apply_vjp(ovd_h h, double mu, int k, const void* x, const void* b, double* s_out,
                              double* ds_dmu, void* F, void* dsdU, void* dsdUc, void* dsdtheta, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (k < 1 || !x || !b) return fail(h, OVD_EINVAL, "bad ovd_sign_apply_vjp arguments");
    if (st) std::memset(st, 0, sizeof(*st));
    ovd_status wst = OVD_OK;
    const Geom& g = h->g;
    const long long fsz = (long long)12 * g.Vp;
    const bool mixed = h->opt.precision == OVD_MIXED;
    const bool grad = ds_dmu || F || dsdU || dsdUc || dsdtheta;
    const DeflSet* dset = find_defl(h, mu);
    const int md = dset ? dset->m : 0;
    // stored form: both bases and Z (3 k FP64 fields, plus the two FP32 bases
    // in mixed precision); recompute form: the left basis only (turned into Z
    // in place), the right basis regenerated by a second, identical run
    bool recompute = false;
    if (grad) {
        const size_t f64 = sizeof(c64) * fsz, f32 = sizeof(c32) * fsz;
        const size_t need = (size_t)3 * k * f64 + (mixed ? (size_t)2 * k * f32 : 0) +
                            sizeof(c64) * vjp_force_scratch_elems(g, vjp_force_chunks(g, k));
        recompute = recompute_basis(
            h, need, {"vjp_basis_v", "vjp_basis_w", "vjp_Z", "vjp_basis_v32", "vjp_basis_w32", "vjp_kpart"}, &wst);
        if (wst != OVD_OK) return wst;
    }
    if (st) st->basis_recomputed = recompute ? 1 : 0;
    WS(bw, c64, "vjp_basis_w", (size_t)k * fsz);
    c64* bv = nullptr;
    if (!recompute) {
        WS(bv_, c64, "vjp_basis_v", (size_t)k * fsz);
        bv = bv_;
    }
    WS(c, c64, "ritz_c", k);
    Timer tt;
    tt.start(h->stream, !h->arena.active);
    const double mus[1] = {mu};
    // sources in FP64: b' = (1 - P) b and x' = (1 - P)^dag x when the m pairs of
    // the set for mu are deflated (eq. 8): c = L^dag b, d = R^dag x
    WS(srcv64, c64, "vjp_src_v", fsz);
    WS(srcw64, c64, "vjp_src_w", fsz);
    HIPCHK(hipMemsetAsync(srcv64, 0, sizeof(c64) * fsz, h->stream));
    HIPCHK(hipMemsetAsync(srcw64, 0, sizeof(c64) * fsz, h->stream));
    launch_pack_spinor<double>(g, 1, b, srcv64, fsz, h->stream);
    launch_pack_spinor<double>(g, 1, x, srcw64, fsz, h->stream);
    c64 *cvec = nullptr, *dvec = nullptr;
    if (md > 0) {
        WS(cv, c64, "vjp_defl_c", md);
        WS(dv, c64, "vjp_defl_d", md);
        WS(tmp, c64, "vjp_defl_tmp", md);
        WS(pscr, c64, "defl_scr", defl_proj_scratch(md, 1, fsz));
        cvec = cv;
        dvec = dv;
        launch_defl_proj(dset->L, fsz, md, srcv64, fsz, 1, fsz, cv, pscr, h->stream);
        launch_defl_proj(dset->R, fsz, md, srcw64, fsz, 1, fsz, dv, pscr, h->stream);
        launch_defl_scale(md, 1, dset->ones, cv, tmp, -1.0, h->stream);
        launch_defl_comb(dset->R, fsz, md, tmp, 1, srcv64, fsz, fsz, h->stream);   // b' = b - R c
        launch_defl_scale(md, 1, dset->ones, dv, tmp, -1.0, h->stream);
        launch_defl_comb(dset->L, fsz, md, tmp, 1, srcw64, fsz, fsz, h->stream);   // x' = x - L d
    }
    // bilinear two-sided Lanczos: right start b', left start x' (FP64, or FP32
    // vectors for OVD_MIXED, widened to FP64 for the gradient)
    c32 *srcv32 = nullptr, *srcw32 = nullptr;
    if (mixed) {
        WS(srcv, c32, "vjp_src_v32", fsz);
        WS(srcw, c32, "vjp_src_w32", fsz);
        WS(bw32, c32, "vjp_basis_w32", (size_t)k * fsz);
        c32* bv32 = nullptr;
        if (!recompute) {
            WS(bv32_, c32, "vjp_basis_v32", (size_t)k * fsz);
            bv32 = bv32_;
        }
        srcv32 = srcv;
        srcw32 = srcw;
        launch_convert_field<float>(g, 1, srcv64, fsz, srcv, fsz, h->stream);
        launch_convert_field<float>(g, 1, srcw64, fsz, srcw, fsz, h->stream);
        s = run_tsl<float>(h, 1, k, 0, mus, srcv, srcw, nullptr, bv32, c, st, bw32);
        if (s != OVD_OK) return s;
        if (bv32) launch_widen_field(g, k, bv32, fsz, bv, fsz, h->stream);
        launch_widen_field(g, k, bw32, fsz, bw, fsz, h->stream);
        HIPCHK(hipGetLastError());
    } else {
        s = run_tsl<double>(h, 1, k, 0, mus, srcv64, srcw64, nullptr, bv, c, st, bw);
        if (s != OVD_OK) return s;
    }
    const TslCoeffs co = h->last_co;
    // s = (x'^dag b') [sgn(T_k)]_11 + sum_i sgn(lambda_i) conj(d_i) c_i, x'^dag b' = beta_0 delta_0
    WS(sdev, c64, "vjp_s", 1);
    launch_vjp_value(co, c, md, dset ? dset->sgn : nullptr, cvec, dvec, sdev, h->stream);
    c64 sv;
    HIPCHK(hipMemcpyAsync(&sv, sdev, sizeof(c64), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (s_out) {
        s_out[0] = sv.re;
        s_out[1] = sv.im;
    }
    if (grad) {
        // M = L_sgn(T_k, e_1 e_1^T), M' = (x'^dag b') M / (delta_p beta_q), Z = W-hat M'^dag
        WS(scr, c64, "frechet_scr", small_frechet_scratch_elems(k));
        WS(M, c64, "vjp_M", (size_t)k * k);
        WS(Mp, c64, "vjp_Mp", (size_t)k * k);
        WS(Mc, c64, "vjp_Mc", (size_t)k * k);
        WS(trF, c64, "vjp_trF", g.V);
        WS(dsum, c64, "vjp_dsum", 1);
        double chk = 0.0;
        const int frc = launch_small_frechet(k, co, sign_cfg(h->opt), scr, M, &chk, h->stream);
        if (st) st->sign_check = std::max(st->sign_check, chk);
        s = small_status(h, frc, "L_sgn(T_k, e_1 e_1^T)", chk, -1);
        if (s != OVD_OK) return s;
        launch_vjp_scale_m(k, co, M, Mp, h->stream);
        launch_conj_c64((long long)k * k, Mp, Mc, h->stream);
        // deflated: the cross and exact parts of the Frechet kernel as 2 m more
        // (v, z) pairs: (V-hat A, L_j) and (R_i, W-hat B + L Cm)
        c64 *AV = nullptr, *ZW = nullptr, *Amat = nullptr;
        const bool last_krylov = md == 0;
        c64* Kacc = nullptr;
        if (recompute || md > 0) {
            WS(ka, c64, "vjp_kacc", (size_t)18 * 4 * g.V);
            Kacc = ka;
        }
        if (md > 0) {
            WS(srow, c64, "vjp_sgn_row", k);
            WS(sscr, c64, "small_scratch", small_sign_scratch_elems(1, k, kDefaultChunkSolves));
            WS(lamd, c64, "vjp_defl_lam", md);
            WS(Am, c64, "vjp_defl_A", (size_t)k * md);
            WS(Bm, c64, "vjp_defl_B", (size_t)k * md);
            WS(Cm, c64, "vjp_defl_Cm", (size_t)md * md);
            WS(cscr, c64, "vjp_defl_scr", defl_vjp_coef_scratch(k, md));
            WS(av, c64, "vjp_defl_AV", (size_t)md * fsz);
            WS(zw, c64, "vjp_defl_ZW", (size_t)md * fsz);
            AV = av;
            ZW = zw;
            Amat = Am;
            double chk2 = 0.0;
            const int rrc = launch_small_sign(1, k, co, sign_cfg(h->opt), sscr, srow, &chk2, h->stream, 1);
            if (st) st->sign_check = std::max(st->sign_check, chk2);
            s = small_status(h, rrc, "sgn(T_k)^T e_1", chk2, -1);
            if (s != OVD_OK) return s;
            HIPCHK(hipMemcpyAsync(lamd, dset->lam.data(), sizeof(c64) * md, hipMemcpyHostToDevice, h->stream));
            launch_defl_vjp_coef(k, co, md, lamd, dset->sgn, c, srow, cvec, dvec, Am, Bm, Cm, cscr, h->stream);
            HIPCHK(hipMemsetAsync(av, 0, sizeof(c64) * md * fsz, h->stream));
            HIPCHK(hipMemsetAsync(zw, 0, sizeof(c64) * md * fsz, h->stream));
            // the left basis is still W-hat here (the recompute form turns it into Z below)
            launch_defl_comb(bw, fsz, k, Bm, md, zw, fsz, fsz, h->stream);
            launch_defl_comb(dset->L, fsz, md, Cm, md, zw, fsz, fsz, h->stream);
            if (bv) launch_defl_comb(bv, fsz, k, Am, md, av, fsz, fsz, h->stream);
            HIPCHK(hipGetLastError());
        }
        if (!recompute) {
            WS(Z, c64, "vjp_Z", (size_t)k * fsz);
            s = zgemm_w_mdag(h, bw, fsz, k, Mc, Z, fsz, fsz);
            if (s != OVD_OK) return s;
            const int nchunk = vjp_force_chunks(g, k);
            c64* Kpart = nullptr;
            if (nchunk > 1) {
                WS(kp, c64, "vjp_kpart", vjp_force_scratch_elems(g, nchunk));
                Kpart = kp;
            }
            launch_vjp_force(g, k, bv, fsz, Z, fsz, h->U64, std::exp(mu), (c64*)F, (c64*)dsdU, (c64*)dsdUc, trF,
                             (c64*)dsdtheta, h->stream, Kacc, true, last_krylov, Kpart, nchunk);
        } else {
            // Z over W in place, a slab of field elements at a time through a
            // k x E copy
            const long long E = ((fsz + 15) / 16 + 15) / 16 * 16;
            WS(slab, c64, "vjp_zslab", (size_t)k * E);
            for (long long e0 = 0; e0 < fsz; e0 += E) {
                const long long ne = std::min(E, fsz - e0);
                HIPCHK(hipMemcpy2DAsync(slab, sizeof(c64) * E, bw + e0, sizeof(c64) * fsz, sizeof(c64) * ne, k,
                                        hipMemcpyDeviceToDevice, h->stream));
                s = zgemm_w_mdag(h, slab, E, k, Mc, bw + e0, fsz, ne);
                if (s != OVD_OK) return s;
            }
            // the Lanczos run again: same kernels, launch shape and inputs, so
            // the same right vectors, now in a ring of 2C; after every C steps
            // the C finished vectors enter the force sum (Kf, Kb carried in Kacc)
            // and, deflated, the combinations V-hat A
            const int C = std::min(k, 32);
            c32* ring32 = nullptr;
            c64* ring64 = nullptr;
            c64* chunk64 = nullptr;
            if (mixed) {
                WS(r32, c32, "vjp_vring32", (size_t)2 * C * fsz);
                WS(ch, c64, "vjp_vchunk", (size_t)C * fsz);
                ring32 = r32;
                chunk64 = ch;
            } else {
                WS(r64, c64, "vjp_vring", (size_t)2 * C * fsz);
                ring64 = r64;
            }
            int done = 0;   // right vectors already in the force sum
            const double emu = std::exp(mu);
            const std::function<void(int, hipStream_t)> hook = [&](int j, hipStream_t stream) {
                const int avail = j + 1;   // right vectors 1 .. j + 1 are final
                if (avail - done < C && avail < k) return;
                const int n = avail - done;
                const size_t slot0 = (size_t)(done % (2 * C));   // done is a multiple of C: no wrap
                const c64* vch = ring64 ? ring64 + slot0 * fsz : chunk64;
                if (ring32) launch_widen_field(g, n, ring32 + slot0 * fsz, fsz, chunk64, fsz, stream);
                launch_vjp_force(g, n, vch, fsz, bw + (size_t)done * fsz, fsz, h->U64, emu, (c64*)F, (c64*)dsdU,
                                 (c64*)dsdUc, trF, (c64*)dsdtheta, stream, Kacc, done == 0, avail == k && last_krylov);
                if (AV) launch_defl_comb(vch, fsz, n, Amat + (size_t)done * md, md, AV, fsz, fsz, stream);
                done = avail;
            };
            ovd_stats st2{};
            if (mixed) s = run_tsl<float>(h, 1, k, 0, mus, srcv32, srcw32, nullptr, ring32, c, &st2, nullptr, 2 * C, &hook);
            else s = run_tsl<double>(h, 1, k, 0, mus, srcv64, srcw64, nullptr, ring64, c, &st2, nullptr, 2 * C, &hook);
            if (s != OVD_OK) return s;
            if (done != k) return fail(h, OVD_EHIP, "gradient: the regenerated basis did not reach step k");
            if (st) st->ms_lanczos += st2.ms_lanczos;
        }
        if (md > 0) {
            // K_CD = sum_j (V-hat A)_j L_j^dag and K_DC + K_DD = sum_i R_i (W-hat B + L Cm)_i^dag
            const double emu = std::exp(mu);
            launch_vjp_force(g, md, AV, fsz, dset->L, fsz, h->U64, emu, (c64*)F, (c64*)dsdU, (c64*)dsdUc, trF,
                             (c64*)dsdtheta, h->stream, Kacc, false, false);
            launch_vjp_force(g, md, dset->R, fsz, ZW, fsz, h->U64, emu, (c64*)F, (c64*)dsdU, (c64*)dsdUc, trF,
                             (c64*)dsdtheta, h->stream, Kacc, false, true);
        }
        launch_sum_c64(g.V, trF, dsum, h->stream);
        c64 dm;
        HIPCHK(hipMemcpyAsync(&dm, dsum, sizeof(c64), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->stream));
        if (ds_dmu) {
            ds_dmu[0] = dm.re;
            ds_dmu[1] = dm.im;
        }
        if (st) st->sign_check = std::max(st->sign_check, chk);
    }
    tt.stop(h->stream);
    if (st) st->ms_total = tt.ms();
    return OVD_OK;
}

ovd_status ovd_tridiag_sign(int nt, int k, const double* alpha, const double* beta, const double* delta,
                            const ovd_options* opt, double* c, double* check, void* stream) {
    if (nt < 1 || k < 1 || !alpha || !beta || !delta || !c) return OVD_EINVAL;
    ovd_options o{};
    o.breakdown_tol = 1e-14;
    o.quad_step = 0.1;
    if (opt) {
        if (!options_ok(*opt)) return OVD_EINVAL;
        o = *opt;
        if (o.breakdown_tol <= 0) o.breakdown_tol = 1e-14;
        if (o.quad_step <= 0) o.quad_step = 0.1;
    }
    hipStream_t s = (hipStream_t)stream;
    const SmallSignCfg cfg = sign_cfg(o);
    const int kp = std::min(k, o.nested_inner > 0 ? o.nested_inner : 100);
    const bool nested = o.sign_method == OVD_SIGN_NESTED;
    const size_t nscr = nested ? nested_sign_scratch_elems(nt, k, kp, cfg.chunk) : small_sign_scratch_elems(nt, k, cfg.chunk);
    const size_t ncoef = (size_t)4 * nt * k;
    c64* d = nullptr;
    if (hipMalloc(&d, sizeof(c64) * (ncoef + (size_t)nt * k + nscr)) != hipSuccess) return OVD_ENOMEM;
    TslCoeffs co{d, d + (size_t)nt * k, d + (size_t)2 * nt * k, d + (size_t)3 * nt * k, k};
    c64* cd = d + ncoef;
    c64* scr = cd + (size_t)nt * k;
    ovd_status st = OVD_OK;
    double chk = 0.0;
    int bstep = -1;
    if (hipMemcpyAsync(co.alpha, alpha, sizeof(c64) * nt * k, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(co.beta, beta, sizeof(c64) * nt * k, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(co.delta, delta, sizeof(c64) * nt * k, hipMemcpyHostToDevice, s) != hipSuccess) {
        st = OVD_EHIP;
    } else {
        const int rc = nested ? launch_nested_sign(nt, k, co, kp, o.breakdown_tol, cfg, scr, cd, &chk, &bstep, s)
                              : launch_small_sign(nt, k, co, cfg, scr, cd, &chk, s);
        if (rc < 0) st = OVD_EHIP;
        else if (rc == 2) st = OVD_EBREAKDOWN;
        else {
            if (hipMemcpyAsync(c, cd, sizeof(c64) * nt * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                st = OVD_EHIP;
            else if (rc == 1)
                st = OVD_ENOCONV;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(d);
    if (check) *check = chk;
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Derivative evaluation without device allocations.
//
// The storage-free scalar form of ovd_sign_apply_deriv with every workspace
// (staging, start vectors, the Lanczos ring, recurrence state, coefficients,
// partial sums, the small-sign scratch, deflation scratch) carved from one
// static device array of kNoAllocBytes per device instead of hipMalloc.
// Same kernels; launched one by one (no graph instantiation, no events, no
// autotuning: the call uses the shape tuned by an earlier allocating call of
// the same precision, direction and batch size, else the default shape).
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)256 << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (looked up once per
// device, with that device current; the array's name is not a device address
// in host code)
ovd_status noalloc_scratch(ovd_h h, void** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(h, OVD_EINVAL, "device index out of range for the no-allocation scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(h, OVD_EHIP, std::string("hipGetSymbolAddress of the no-allocation scratch: ") +
                                         hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return OVD_OK;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// bytes the scalar-mode derivative takes from the scratch: the workspaces of
// deriv_impl, run_tsl and the small sign in their order, each 256-aligned
size_t noalloc_need(ovd_h h, int nrhs, int k, bool link, int lmax) {
    const Geom& g = h->g;
    const bool mixed = h->opt.precision == OVD_MIXED;
    const size_t bT = mixed ? sizeof(c32) : sizeof(c64);
    const size_t half = (size_t)12 * g.Vp, fsz = 2 * half;
    size_t n = 0;
    if (link) {
        n += al256(sizeof(c64) * link_elems<double>(g.Vp));
        if (mixed) n += al256(sizeof(c32) * link_elems<float>(g.Vp));
        n += al256(sizeof(unsigned));
    }
    n += 2 * al256(sizeof(c64) * nrhs * half);                      // stage_b, stage_t
    n += 2 * al256(bT * nrhs * fsz);                                // src_v, src_w
    n += al256(bT * nrhs * half);                                   // xproj
    n += al256(sizeof(c64) * nrhs * k);                             // ritz_c
    if (lmax > 0) {
        n += 5 * al256(sizeof(c64) * lmax * nrhs);
        n += 2 * al256(sizeof(c64) * defl_proj_scratch(lmax, nrhs, (long long)half));
        n += al256(sizeof(c64) * nrhs * half) + 2 * al256(sizeof(c64) * lmax * nrhs);
    }
    const int nb = tsl_stencil_blocks(g, 1, 1);
    n += al256(bT * 10 * nrhs * fsz);                               // Lanczos ring
    n += al256(sizeof(TslState) * nrhs) + al256(sizeof(c64) * 4 * nrhs * k);
    n += al256(sizeof(double) * nrhs * nb * 8) + al256(sizeof(unsigned) * nrhs);
    if (h->opt.sign_method == OVD_SIGN_NESTED) {
        const int kp = std::min(k, h->opt.nested_inner > 0 ? h->opt.nested_inner : 100);
        n += al256(sizeof(c64) * nested_sign_scratch_elems(nrhs, k, kp, kNoAllocChunkSolves));
    } else {
        n += al256(sizeof(c64) * small_sign_scratch_elems(nrhs, k, kNoAllocChunkSolves));
    }
    n += al256(sizeof(c64) * nrhs);                                 // scalar_out
    return n;
}

}  // namespace

extern "C" {

ovd_status ovd_sign_apply_deriv_noalloc(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k,
                                        const void* b, const void* x, double* xdy, ovd_stats* st) {
    ovd_status s = check_handle(h);
    if (s != OVD_OK) return s;
    if (nrhs < 1 || !mu || k < 1 || !b || !x || !xdy)
        return fail(h, OVD_EINVAL, "bad ovd_sign_apply_deriv_noalloc arguments");
    if (h->arena.active) return fail(h, OVD_EINVAL, "ovd_sign_apply_deriv_noalloc re-entered");
    const bool link = dir && dir->kind == OVD_DIR_LINK;
    int lmax = 0;
    for (int r = 0; r < nrhs; ++r) {
        const DeflSet* d = find_defl(h, mu[r]);
        if (d && d->l > lmax) lmax = d->l;
    }
    const size_t need = noalloc_need(h, nrhs, k, link, lmax);
    if (need > kNoAllocBytes)
        return fail(h, OVD_EINVAL, "ovd_sign_apply_deriv_noalloc needs " + std::to_string(need) +
                                       " bytes of scratch for this lattice, batch and k; its static scratch holds " +
                                       std::to_string(kNoAllocBytes) + " (use ovd_sign_apply_deriv)");
    void* base = nullptr;
    s = noalloc_scratch(h, &base);
    if (s != OVD_OK) return s;
    if (st) std::memset(st, 0, sizeof(*st));
    c64* keep64 = h->dU64;
    c32* keep32 = h->dU32;
    h->arena.base = (char*)base;
    h->arena.size = kNoAllocBytes;
    h->arena.used = 0;
    h->arena.active = true;
    int dirk = 1;
    s = upload_dir(h, dir, &dirk);
    if (s == OVD_OK) {
        if (h->opt.precision == OVD_MIXED)
            s = deriv_impl<float>(h, nrhs, mu, dirk, k, b, nullptr, nullptr, x, xdy, st);
        else
            s = deriv_impl<double>(h, nrhs, mu, dirk, k, b, nullptr, nullptr, x, xdy, st);
    }
    h->arena = ovd_lattice::Arena{};
    // a link direction packed into the scratch is not the handle's own copy
    h->dU64 = keep64;
    h->dU32 = keep32;
    return s;
}

}  // extern "C"
