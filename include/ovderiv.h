/*
 * libovderiv -- two-sided Lanczos approximation of sgn(H(mu)) b, its
 * derivative by the block-matrix method, generalised deflation and the
 * gradient of <x|sgn(H)|b>, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Puhr & Buividovich, "A method to compute derivatives of functions
 * of large complex matrices" (Lattice 2016, arXiv:1611.00195).
 *   Sec. 1, eq. 1   kernel H(mu) = gamma5 Dw(mu) of the overlap operator;
 *   Sec. 2          only the action y = f(A) x is needed; d_t y = (d_t f(A)) x;
 *   Sec. 2, eq. 6-7 f([[A, dA], [0, A]]) (0; x) = (d_t f(A) x ; f(A) x);
 *   Sec. 2 (end)    two-sided Lanczos (TSL) for the sign of a non-Hermitian matrix;
 *   Sec. 3, eq. 8   standard deflation;  eq. 9-11  generalised deflation.
 *
 * Conventions shared by every call
 *   Lattice dims = {Lx, Ly, Lz, Lt}; site index s = x + Lx*(y + Ly*(z + Lz*t)).
 *   Spinor field: complex128 (interleaved re, im) [V][4 spin][3 colour],
 *     component index 3*spin + colour.  Chiral basis, gamma5 = diag(1,1,-1,-1).
 *   Link field:   complex128 [4][V][3][3], direction order x, y, z, t,
 *     row-major 3x3.  The time boundary factor t_bc (-1 antiperiodic) is
 *     applied by the stencil on the hops crossing t = Lt-1 <-> 0, never
 *     stored in the links.
 *   Dw(mu) psi(x) = (m0 + 4r) psi(x) - 1/2 sum_nu [ e^{mu d_nu4} (r - gamma_nu) U_nu(x) psi(x+nu)
 *                    + e^{-mu d_nu4} (r + gamma_nu) U_nu(x-nu)^dag psi(x-nu) ].
 *   Only r = 1 is supported on the GPU path (the spin-projection trick).
 *
 * Memory and streams
 *   Every array argument marked "device" is a device pointer owned by the
 *   caller (for example a torch tensor on the handle's device); "host"
 *   pointers are ordinary host memory.  Work is enqueued on the stream given
 *   at creation (NULL = the null stream).  Calls that return host scalars
 *   (xdy, s, ds_dmu, stats) synchronise that stream before returning; the
 *   others return after enqueueing.  The handle owns its workspaces, a copy
 *   of the links and the deflation data, all freed by ovd_destroy.
 *
 * Errors
 *   Every call returns an ovd_status; on failure ovd_last_error(h) holds a
 *   message.  A handle is not thread-safe: use one handle per host thread.
 */
#ifndef OVDERIV_H
#define OVDERIV_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ovd_lattice* ovd_h;

typedef enum {
    OVD_OK = 0,
    OVD_EINVAL = -1,      /* bad argument (sizes, null pointers, unsupported r, ...); every
                             batched call needs nrhs >= 1 and k >= 1, and an empty batch is
                             rejected before any device work */
    OVD_ENOMEM = -2,      /* device allocation failed */
    OVD_EHIP = -3,        /* a HIP runtime call failed */
    OVD_EBREAKDOWN = -4,  /* serious Lanczos breakdown: |w^dag v| <= tau |w| |v| */
    OVD_ENODEFL = -5,     /* deflation requested for a mu with no deflation set */
    OVD_ENAN = -6,        /* non-finite value detected in the recurrence */
    OVD_ENOCONV = -7      /* an iterative solver did not converge: eigenpairs, shifted solves,
                             or the sgn(T_k) e_1 quadrature (see quad_max_levels) */
} ovd_status;

enum { OVD_FP64 = 0, OVD_MIXED = 1 };        /* precision of Krylov vectors and stencil */
enum { OVD_LEFT_SUM = 0, OVD_LEFT_SAME = 1 };  /* left start of the block system */
enum { OVD_DIR_MU = 0, OVD_DIR_LINK = 1 };     /* derivative direction t */
enum { OVD_OP_H = 0, OVD_OP_DW = 1, OVD_OP_DH_DMU = 2, OVD_OP_DH_DLINK = 3 };
enum { OVD_SIGN_QUAD = 0, OVD_SIGN_NESTED = 1 };   /* method for sgn(T_k) e_1 */

typedef struct {
    int precision;          /* OVD_FP64 (default) or OVD_MIXED: FP32 vectors, links and
                               stencil arithmetic; the three-term update in FP64 with one
                               rounding at the FP32 store; FP64 inner products, Lanczos
                               scalars, T_k, sgn(T_k) and deflation */
    int left_start;         /* left start of the block system, see ovd_sign_apply_deriv */
    double breakdown_tol;   /* tau, default 1e-14 */
    double quad_step;       /* first refined step of the trapezoidal rule in log(y) used for
                               sgn(T_k) e_1 (halved until two levels agree to 1e-10),
                               default 0.1 */
    int step_timing;        /* 1: time every Lanczos kernel with events (ovd_stats.ms_stencil,
                               ms_update); 0 (default): only the totals */
    int use_graph;          /* 1 (default): the k Lanczos steps of a call are recorded once
                               into a HIP graph (per shape and workspace) and replayed;
                               0: launched one by one */
    int autotune;           /* 1 (default): the first call of each precision, direction and
                               batch size times the stencil's launch shapes (XCD work order,
                               site groups per block) and keeps the fastest; 0: fixed shapes */
    int shape_map;          /* >= 0: force the XCD work order of the stencils (0: nrhs/8
                               sources per XCD, only when nrhs % 8 == 0; 1: contiguous site
                               ranges per XCD); -1 (default): tuned or default */
    int shape_gpb;          /* > 0: force the site groups per block (Lanczos stencil: 1 or 2
                               for derivatives, 2 or 4 otherwise, or 8: one block per
                               xy-plane staged in LDS, when 128 <= Lx Ly <= 256; Dw.v: 2 or 4,
                               or 8 with shape_rp 2 under the same condition;
                               with shape_seq 3 the number of time segments, at most Lt);
                               0: tuned */
    int shape_seq;          /* Lanczos stencil without the derivative of a link field, not the
                               LDS-plane shape: 1 forces the sequential form (each thread
                               finishes one of its two outputs before the other: half the
                               live accumulators, twice the waves per SIMD in FP64), 0 the
                               paired form (both outputs at once, every link loaded once);
                               2 (plain sgn(H) and the gradient only, 1 or 2 groups per
                               block) the split form (the two outputs of a site in two
                               waves: twice the waves of the paired form, for launches too
                               small to fill the GPU); 3 (the mu derivative only, when the
                               LDS-plane shape applies and two planes of both input fields
                               fit the LDS) the time-marching form (one block per xy-plane
                               column of shape_gpb time segments, walking its time slices
                               in order and reusing each loaded plane from LDS);
                               -1 (default): tuned, else paired */
    int shape_rp;           /* ovd_apply_op with OVD_OP_H or OVD_OP_DW on an even number of
                               right-hand sides: 2 forces two per thread (each link loaded
                               once for both), 1 one per thread; 0 (default): tuned */
    int basis_recompute;    /* calls that need a Krylov basis (vector outputs of
                               ovd_sign_apply and ovd_sign_apply_deriv, the gradient of
                               ovd_sign_apply_vjp): 0 stores it; 1 regenerates it with a
                               second, identical Lanczos run, C = min(k, 32) vectors at a time
                               through a ring of 2C fields, at twice the Lanczos time (vector
                               outputs: no basis stored; gradient: only the left basis,
                               turned into Z in place, k + 2C fields instead of 3k); -1
                               (default): recompute only when the stored form does not fit in
                               the free device memory */
    int quad_max_levels;    /* refinement levels of the sgn(T_k) e_1 quadrature before the call
                               fails with OVD_ENOCONV (two successive levels must agree to
                               1e-10); 0: 9; at most 20 */
    int sign_method;        /* OVD_SIGN_QUAD (default): sgn(T_k) e_1 by the quadrature above;
                               OVD_SIGN_NESTED: by a nested two-sided Lanczos run (Sec. 4: one
                               level of nesting, inner Krylov size nested_inner) on
                               (T_k + T_k^{-1})/2, whose kp x kp Ritz matrix is signed by the
                               quadrature; an inner breakdown returns OVD_EBREAKDOWN */
    int nested_inner;       /* inner Krylov size of OVD_SIGN_NESTED; 0: 100 (the paper's);
                               values above k are clamped to k */
    long long mem_budget;   /* > 0: with basis_recompute = -1, the bytes a stored Krylov basis may
                               take; a larger one is regenerated instead (as when it does not
                               fit in free device memory); 0 (default): no budget */
    int eig_shift_max;      /* ovd_compute_deflation: iteration limit of each shifted solve for the
                               eigenvector derivatives (CGLS); 0: 60000 */
    int batch_separate;     /* ovd_sign_apply_deriv_batch: 1 runs this lattice's Lanczos steps as
                               launches of its own on its own stream, even where the batch could
                               share them; 0 (default): shared when the batch allows */
} ovd_options;

typedef struct {
    int kind;               /* OVD_DIR_MU or OVD_DIR_LINK */
    const void* dU;         /* OVD_DIR_LINK: device complex128 [4][V][3][3], dU = dU/dt
                               (e.g. X U for U -> exp(tX) U); ignored for OVD_DIR_MU */
} ovd_dir;

typedef struct {
    int k;                  /* Krylov steps taken */
    int breakdown_step;     /* first step with a serious breakdown, -1 if none */
    double min_margin;      /* min over steps and right-hand sides of |w^dag v|/(|w||v|) */
    double sign_check;      /* error estimate of sgn(T_k) e_1: max difference between the last two
                               refinement levels of the quadrature (see quad_step); set also
                               when the call fails with OVD_ENOCONV */
    double ms_lanczos;      /* device time of the Lanczos steps (HIP events) */
    double ms_small_sign;   /* device time of the sgn(T_k) e_1 solve */
    double ms_total;        /* device time of the whole call */
    double ms_stencil;      /* summed device time of the k stencil launches (HIP events) */
    double ms_update;       /* summed device time of the k - 1 three-term update launches */
    int basis_recomputed;   /* 1 if the call regenerated its Krylov basis (see basis_recompute) */
} ovd_stats;

/* Create a handle for one lattice.  Sec. 4 lattices are Lt x Ls^3 (e.g. 14 x 14^3).
 *   dims      host int[4] = {Lx, Ly, Lz, Lt}, each >= 2
 *   m0, r     Wilson mass and Wilson parameter (r must be 1)
 *   t_bc      +1 periodic or -1 antiperiodic time boundary
 *   opt       host, nullable (defaults above)
 *   stream    hipStream_t to enqueue on (NULL = null stream)
 *   out       host, receives the handle */
ovd_status ovd_create_lattice(const int dims[4], double m0, double r, int t_bc,
                              const ovd_options* opt, void* stream, ovd_h* out);
ovd_status ovd_destroy(ovd_h h);
const char* ovd_last_error(ovd_h h);
ovd_status ovd_set_stream(ovd_h h, void* stream);

/* Upload a gauge configuration (Sec. 4: the derivative is taken on SU(3)
 * configurations).  U: device complex128 [4][V][3][3].  The handle keeps an
 * FP64 copy and, for OVD_MIXED, an FP32 copy in its own layout.  Every
 * deflation set of the handle is removed: its eigenvectors belong to the
 * previous links. */
ovd_status ovd_set_links(ovd_h h, const void* U);

/* Apply one operator to nrhs spinor fields (used for stencil checks and the
 * Dw.v bandwidth measurement).
 *   op    OVD_OP_H: H(mu) = gamma5 Dw(mu) (eq. 1; its adjoint is H(-mu));
 *         OVD_OP_DW: Dw(mu);  OVD_OP_DH_DMU: dH/dmu;
 *         OVD_OP_DH_DLINK: dH/dt along dir->dU.
 *   in, out  device complex128 [nrhs][V][4][3]; must not alias.
 *   ms    host, nullable: device time of the stencil kernel alone. */
ovd_status ovd_apply_op(ovd_h h, int op, double mu, const ovd_dir* dir, int nrhs,
                        const void* in, void* out, double* ms);

/* Deflation set for one mu (Sec. 3, eq. 8 and eq. 10-11).  Replaces any set
 * stored for the same mu.
 *   m        number of eigenpairs of H(mu) used by ovd_sign_apply (eq. 8)
 *   lam      host complex128 [m] eigenvalues, closest to zero first
 *   R, L     device complex128 [m][V][4][3] right / left eigenvectors with
 *            L_i^dag R_j = delta_ij (checked; OVD_EINVAL if violated by > 1e-8)
 *   l        number of Jordan blocks of B deflated by ovd_sign_apply_deriv
 *            (0 <= l <= m; only the first l pairs are used there)
 *   dR, dL   device complex128 [l][V][4][3], t-derivatives of the first l
 *            R_i, L_i along dir, gauge L_i^dag dR_i = 0 = dL_i^dag R_i; may be
 *            NULL when l = 0
 *   dir      the direction dR, dL belong to (nullable when l = 0); for
 *            OVD_DIR_LINK with l > 0, dir->dU must be that direction: the set
 *            keeps a copy, and ovd_sign_apply_deriv along any other direction
 *            (mu, or a different dU) fails with OVD_EINVAL instead of using
 *            derivatives that belong elsewhere.
 * The set lives until it is replaced, cleared, or the links change. */
ovd_status ovd_set_deflation(ovd_h h, double mu, int m, const double* lam,
                             const void* R, const void* L, int l,
                             const void* dR, const void* dL, const ovd_dir* dir);
/* Statistics of ovd_compute_deflation. */
typedef struct {
    int outer_right, outer_left;      /* Arnoldi restart cycles on H(mu)^-1 and H(-mu)^-1 = (H(mu)^dag)^-1 */
    double max_res_right, max_res_left; /* max |H r - lambda r| (|r| = 1) of the m pairs, both sides */
    double max_biorth;                /* max |L^dag R - 1| */
    int shift_iters;                  /* total iterations of the 2 l shifted solves of the derivatives */
    double max_shift_res;             /* largest relative residual of those solves */
    double ms;                        /* wall time */
} ovd_eig_stats;

/* Compute and install the deflation set of mu on the GPU (Sec. 3): the m
 * eigenvalues of H(mu) closest to zero (smallest |lambda|) with right and left
 * eigenvectors normalised to L^dag R = 1 (eq. 8), and for the first l of them
 * the derivatives dR, dL along dir (mu or a link direction) that the
 * generalised deflation of eq. 9-11 needs, in the gauge L_j^dag dR_j = 0,
 * dL_j^dag R_j = 0:
 *   dR_j = sum_{i != j} R_i (L_i^dag dH R_j)/(lambda_j - lambda_i) + (lambda_j - H)^{-1} (1 - P) dH R_j
 *   dL_j = sum_{i != j} L_i conj((L_j^dag dH R_i)/(lambda_j - lambda_i)) + (conj(lambda_j) - H^dag)^{-1} (1 - P)^dag dH^dag L_j
 * with P = sum_{i<m} R_i L_i^dag and the resolvents taken on the range of 1 - P.
 * Method: thick-restart Arnoldi on H^-1 (and H^dag^-1), whose eigenvalues of
 * largest modulus are 1/lambda for the wanted lambda, every application a
 * conjugate-gradient solve of the normal equations, FP64; the shifted solves
 * of the derivatives by conjugate gradients on their normal equations (CGLS).
 *   tol   residual bound |H r - lambda r| for |r| = 1 (<= 0: 1e-10)
 *   lam   host double[2 m] (re, im), increasing |lambda|, or NULL
 * The set replaces any set of the same mu, exactly as ovd_set_deflation.
 * Errors: OVD_EINVAL (m < 1, l > m, m > 512, bad dir), OVD_ENOCONV (not
 * converged, or a cluster of eigenvalues straddles the m-th one, or
 * degenerate eigenvalues among the first l), OVD_ENOMEM, OVD_EHIP.  Needs about
 * (8 (m + max(16, m/2)) + 5 m) 12 V complex128 of device memory while it runs. */
ovd_status ovd_compute_deflation(ovd_h h, double mu, int m, int l, const ovd_dir* dir, double tol,
                                 double* lam, ovd_eig_stats* st);

/* Read back the deflation set of mu (as installed by ovd_set_deflation or
 * ovd_compute_deflation).  m, l: host int or NULL; lam: host double[2 m] or
 * NULL; R, L: device complex128 [m][V][4][3] or NULL; dR, dL: device
 * complex128 [l][V][4][3] or NULL.  OVD_ENODEFL if there is no set for mu.
 * Call once with only m and l to size the buffers. */
ovd_status ovd_get_deflation(ovd_h h, double mu, int* m, int* l, double* lam, void* R, void* L,
                             void* dR, void* dL);

ovd_status ovd_clear_deflation(ovd_h h);

/* y = sgn(H(mu)) b by k steps of two-sided Lanczos with left start equal to
 * the (deflated) source, y ~ |b'| V_k sgn(T_k) e_1 + exact part (eq. 8 when a
 * deflation set for mu exists).  Batched over nrhs independent systems.
 *   mu    host double[nrhs] (each mu must have a deflation set, or none at all)
 *   b, y  device complex128 [nrhs][V][4][3]
 *   st    host, nullable */
ovd_status ovd_sign_apply(ovd_h h, int nrhs, const double* mu, int k,
                          const void* b, void* y, ovd_stats* st);

/* Derivative along dir of sgn(H(mu)) b by the block method (eq. 6-7): k steps
 * of two-sided Lanczos on B = [[H, dH], [0, H]] with source psi = (0; b),
 * deflated by eq. 11 with the first l pairs of the deflation set for mu when
 * one exists.  Left start (not fixed by the paper): OVD_LEFT_SUM uses
 * (psi_t + psi_b; psi_b), OVD_LEFT_SAME uses psi.
 *   b         device complex128 [nrhs][V][4][3]
 *   y, dy     device complex128 [nrhs][V][4][3] or NULL: sgn(H) b and its derivative
 *   x         device complex128 [nrhs][V][4][3] or NULL
 *   xdy       host complex128 [nrhs] or NULL: <x|d sgn(H) b>; when y and dy are both
 *             NULL the Krylov basis is never stored (storage-free scalar mode) */
ovd_status ovd_sign_apply_deriv(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir,
                                int k, const void* b, void* y, void* dy,
                                const void* x, double* xdy, ovd_stats* st);

/* sgn(B) applied to a general block vector psi = (t; b) by the same method
 * (eq. 7 with a full source): k steps of two-sided Lanczos on
 * B = [[H, dH], [0, H]], left start (t + b; b), deflated by eq. 11 with the
 * first l pairs of the set for mu (the projections c = L^dag b,
 * d = dL^dag b + L^dag t).  With t = NULL this is ovd_sign_apply_deriv
 * (yt = dy, yb = y).  The second application of the Sec. 4 error estimate of
 * the derivative needs it.
 *   t         device complex128 [nrhs][V][4][3] or NULL (zero top half)
 *   b         device complex128 [nrhs][V][4][3]
 *   yt, yb    device complex128 [nrhs][V][4][3] or NULL (not both): top and
 *             bottom halves of sgn(B) psi */
ovd_status ovd_block_sign_apply(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* t,
                                const void* b, void* yt, void* yb, ovd_stats* st);

/* Error estimate of Sec. 4 for the derivative: with psi = (0; phi),
 *   eps_B = |sgn(B)(sgn(B) psi) - psi| / (2 |psi|),
 * both applications of sgn(B) by ovd_block_sign_apply (k steps each, the
 * handle's precision, deflated when a set for mu exists).  eps: host
 * double[nrhs]; phi: device complex128 [nrhs][V][4][3]. */
ovd_status ovd_deriv_error_estimate(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* phi,
                                    double* eps, ovd_stats* st);

/* The overlap operator of eq. 1 (lattice spacing a = 1) and its derivative:
 *   Db  = D_ov b = b + gamma5 sgn(H(mu)) b,     dDb = d/dt D_ov b = gamma5 d/dt sgn(H) b,
 * with sgn(H) b and its derivative from ovd_sign_apply / ovd_sign_apply_deriv
 * (same k, deflation and precision rules).  Db, dDb: device complex128
 * [nrhs][V][4][3], either may be NULL (not both); dir as in
 * ovd_sign_apply_deriv (used only for dDb). */
ovd_status ovd_overlap_apply(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k, const void* b,
                             void* Db, void* dDb, ovd_stats* st);

/* Error estimate of Sec. 4 from sgn(A)^2 = 1: eps = |sgn(H)(sgn(H) b) - b| / (2 |b|)
 * per source, with the k-step approximation applied twice.  eps: host
 * double[nrhs]. */
ovd_status ovd_sign_error_estimate(ovd_h h, int nrhs, const double* mu, int k, const void* b, double* eps,
                                   ovd_stats* st);

/* One lattice's share of an uneven batch: the arguments of
 * ovd_sign_apply_deriv for handle h, and its status on return. */
typedef struct {
    ovd_h h;
    int nrhs;
    const double* mu;       /* host [nrhs] */
    const ovd_dir* dir;     /* NULL: mu */
    int k;
    const void* b;
    void* y;
    void* dy;
    const void* x;
    double* xdy;            /* host [2 nrhs] or NULL */
    ovd_stats* st;          /* or NULL */
    ovd_status status;      /* out */
} ovd_deriv_job;

/* Uneven batch (derivatives on several lattices of different sizes at once,
 * each lattice with its own handle, batch of sources, mu values and k): every
 * job runs ovd_sign_apply_deriv on its handle from a host thread of its own.
 * When all handles have the same precision, all jobs the same kind of
 * direction (mu, or a link direction) and no handle sets batch_separate, the
 * lattices share their Lanczos steps: each job prepares its sources on its own
 * stream, then step j of every lattice whose k exceeds j runs in one update
 * launch and one stencil launch (the blocks split into one range per lattice,
 * each running that lattice's own kernel body), on a stream of the batch
 * after all jobs' preparation; each job then finishes on its own stream
 * (sgn(T_k) e_1, outputs, deflation terms).  The shared launches use one
 * stencil launch shape agreed from the handles' tuned or forced shapes (one
 * site group per block if every lattice has one, else two; the sequential
 * form, along mu, if every lattice has it, else the paired form) and each
 * lattice's XCD work order; the shape is recorded as every handle's tuned
 * shape, so later single calls give identical results.  Otherwise each lattice's steps run as its own graph on its own
 * stream, concurrently when the handles were created on different streams.
 * A handle may appear only once.  Returns OVD_OK if every job succeeded,
 * else the first failing job's status (each job's status is in its status
 * field). */
ovd_status ovd_sign_apply_deriv_batch(int njobs, ovd_deriv_job* jobs);

/* Gradient of s = <x|sgn(H(mu))|b> (the bilinear the paper's currents and
 * fermionic force are built from, Sec. 1): two-sided Lanczos with right
 * start b and left start x (precision below),
 * s ~ (x^dag b)[sgn(T_k)]_11, and with M_k = L_sgn(T_k, e_1 e_1^T) the
 * derivative ds/dt ~ (x^dag b) tr(M_k W_k^dag (dH/dt) V_k), evaluated for every
 * link at once through Z = W_k M_k^dag.
 * Deflation (Sec. 3, eq. 8): when the handle holds a set for mu, its m pairs
 * are deflated.  The run then starts from b' = (1 - P) b and x' = (1 - P)^dag x,
 * s = x'^dag sgn(H) b' + sum_i sgn(lambda_i)(x^dag R_i)(L_i^dag b), and the
 * Frechet kernel K = L_sgn(H, b x^dag) gains 2 m rank-one terms: the cross
 * terms between the deflated set and its complement through the Krylov-Ritz
 * form of g_j(z) = (sgn z - sgn lambda_j)/(z - lambda_j) on the two bases, and
 * the exact part within the set (divided differences of sgn over the pairs).
 * Only lambda, R and L are used (not dR, dL).
 *   x, b      device complex128 [V][4][3]
 *   s, ds_dmu host complex128 [1], nullable
 *   F         device complex128 [4][V][3][3] or NULL: per-link force with
 *             ds/dt = tr(F_nu(y) X) for U_nu(y) -> exp(tX) U_nu(y)
 *   dsdU, dsdUc  device complex128 [4][V][3][3] or NULL: Wirtinger derivatives
 *             ds/dU_nu(y)[a][b] and ds/dconj(U_nu(y)[a][b]) with the links taken
 *             as unconstrained complex matrices (for automatic differentiation)
 *   dsdtheta  device complex128 [4][V] or NULL: ds/dTheta_nu(y) = i tr F_nu(y),
 *             the derivatives along an external U(1) field, U_nu(y) ->
 *             e^{i Theta_nu(y)} U_nu(y) (Sec. 4 takes its derivatives along such a
 *             field; Sec. 5 builds the conserved axial current from them)
 * The Krylov bases V_k, W_k are stored (2 k 12 V complex128 of workspace).
 * With OVD_MIXED the Lanczos run keeps FP32 vectors (FP64 scalars, as in
 * ovd_sign_apply) and its bases are widened to FP64 for M_k, Z and the force
 * (2 k 12 V complex64 more workspace). */
ovd_status ovd_sign_apply_vjp(ovd_h h, double mu, int k, const void* x, const void* b,
                              double* s, double* ds_dmu, void* F, void* dsdU, void* dsdUc,
                              void* dsdtheta, ovd_stats* st);

/* ovd_sign_apply_deriv in its storage-free scalar mode (xdy = <x|d/dt sgn(H) b>,
 * no vector outputs) for callers that cannot allocate device memory: code that
 * must not call hipMalloc (allocation-free sections of serving loops, harnesses
 * that forbid device allocations).  Every workspace of the call comes from one
 * static device array of 256 MiB per device, which the library holds on each
 * device it runs on until the process ends; the call itself allocates nothing
 * on the device (no hipMalloc / hipFree, no graph instantiation, no events).
 * Same kernels and results as ovd_sign_apply_deriv (deflated by the set of mu
 * when one exists, left start and precision of the handle), launched one by
 * one; the launch shape is the one an earlier ovd_sign_apply_deriv of the
 * same precision, direction and batch size tuned, else the default shape.
 *   b, x   device complex128 [nrhs][V][4][3];  xdy  host complex128 [nrhs]
 * Limits: the workspaces of the call (about 10 block vectors per right-hand
 * side for the Lanczos ring, 6 more for staging, the small-sign scratch) must
 * fit in the 256 MiB, else OVD_EINVAL with the size needed and nothing is
 * launched: at k = 400, 14 x 14^3 fits one right-hand side in FP64 and two
 * in mixed precision; 8^4 fits 11 in FP64 and 21 in mixed precision.
 * Concurrency: every call on a device shares that device's array, and the
 * array keeps the last call's contents (what a call needs zeroed it clears
 * itself): calls that overlap on one device, from any handle or thread, race.
 * ovd_get_tridiag after this call reads the coefficients from the shared
 * array, valid until the next allocation-free call on the device. */
ovd_status ovd_sign_apply_deriv_noalloc(ovd_h h, int nrhs, const double* mu, const ovd_dir* dir, int k,
                                        const void* b, const void* x, double* xdy, ovd_stats* st);

/* Launch shapes in use so far (chosen by the autotuner, or forced through the
 * options), as text
 * "kernel:precision:dir-or-op:nrhs=map<m>,gpb<g>[,seq];..." into buf (host, len
 * bytes, truncated and NUL-terminated). */
ovd_status ovd_get_tuned(ovd_h h, char* buf, int len);

/* sgn(T) e_1 for nt complex tridiagonal k x k matrices given on the host: the
 * small dense step of every Krylov-Ritz approximation (Sec. 2, closing part:
 * f(A) psi ~ |psi| V_k f(T_k) e_1), on its own, with the method, quadrature
 * step, level limit, inner size and breakdown tolerance of opt (nullable:
 * defaults).  The sign is discontinuous on the imaginary axis (Sec. 3), so the
 * quadrature needs more levels for eigenvalues close to it.
 *   alpha, beta, delta  host complex128 [nt][k] in the convention of
 *             ovd_get_tridiag: diagonal alpha[0..k-1], T[i][i+1] = beta[i+1],
 *             T[i+1][i] = delta[i+1] (entries 0 of beta and delta unused)
 *   c         host complex128 [nt][k], receives sgn(T) e_1
 *   check     host double or NULL: the quadrature's last level difference
 *   stream    hipStream_t (NULL: null stream)
 * Errors: OVD_EINVAL (nt < 1, k < 1, null pointers), OVD_ENOCONV (levels
 * exhausted; c then holds the last level), OVD_EBREAKDOWN (inner breakdown of
 * OVD_SIGN_NESTED), OVD_ENOMEM, OVD_EHIP.  Device memory is allocated and
 * freed inside the call. */
ovd_status ovd_tridiag_sign(int nt, int k, const double* alpha, const double* beta, const double* delta,
                            const ovd_options* opt, double* c, double* check, void* stream);

/* Lanczos coefficients of the last Lanczos run (for parity checks), right-hand
 * side rhs: host complex128 arrays alpha[k], beta[k], delta[k].  T_k has
 * diagonal alpha[0..k-1], super-diagonal beta[1..k-1] and sub-diagonal
 * delta[1..k-1]; delta[0] = |psi| and beta[0] = phi^dag psi / |psi| are the
 * start-vector normalisations. */
ovd_status ovd_get_tridiag(ovd_h h, int rhs, int k, double* alpha, double* beta, double* delta);

#ifdef __cplusplus
}
#endif
#endif /* OVDERIV_H */
