/*
 * msv: modal-kernel tabulation, Mueller-Nystrom assembly and per-mode solves
 * for electromagnetic scattering from a penetrable body of revolution, on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Lai & O'Neil, "An FFT-accelerated direct solver for electromagnetic
 * scattering from penetrable axisymmetric objects".  Section numbers below
 * refer to that paper.
 *
 * Conventions shared by every call
 *  - Complex numbers are {re, im} pairs of doubles (msv_c128) or floats.
 *  - Pointers named h_* are host memory, d_* device memory.  The caller owns
 *    every buffer it passes; the library never frees them.  The plan owns its
 *    own device workspace and the LU factors until msv_plan_destroy.
 *  - `stream` is a hipStream_t passed as void*; every call except
 *    msv_plan_create and msv_plan_destroy is stream-ordered and returns before
 *    the work finishes.  Calls on one plan must use one stream at a time.
 *  - Every call returns an msv_status; on failure msv_last_error(plan) holds a
 *    message (msv_last_error(NULL) for a failed msv_plan_create).  A failed
 *    call leaves the plan usable unless it returned MSV_EHIP.
 *  - Units: omega = k0 / sqrt(eps0 mu0), k1 = omega sqrt(eps1 mu1) with
 *    Im k1 >= 0 (time dependence e^{-i omega t}, Section 1).
 */
#ifndef MSV_H
#define MSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } msv_c128;

typedef enum {
  MSV_OK = 0,
  MSV_EINVAL = 1,     /* invalid argument; nothing was launched */
  MSV_ENOMEM = 2,     /* device allocation failed */
  MSV_EHIP = 3,       /* a HIP runtime call failed; destroy the plan */
  MSV_ESINGULAR = 4,  /* zero pivot in a per-mode LU */
  MSV_ENOCONV = 5     /* iterative refinement did not reach the tolerance */
} msv_status;

typedef struct msv_plan msv_plan;

/* Discretized generating curve gamma(t) = (r, z) (Sections 3 and 5).
 * N = n_panels * order nodes, panel-major: node j = order*p + k lies at the k-th
 * Gauss-Legendre point (ascending) of panel p's local coordinate u in [-1, 1].
 * The curve runs counterclockwise in the (r, z) half-plane; an open curve
 * starts and ends on the axis (south pole to north pole).  Per node: r > 0, z,
 * the outward unit normal (nr, nz) = (z', -r') (' = d/ds), and ds/du > 0.
 * Panels p and p+1 are adjacent; for closed != 0 so are n_panels-1 and 0.
 * Adjacent panels must differ in arclength by at most a factor 2.2.
 * N <= 3072 (matrix order 4N <= 12288: an LU panel strip keeps its column in
 * the registers of one 1024-thread workgroup, 12 rows per thread). */
typedef struct {
  int32_t n_panels;
  int32_t order;            /* must be 16 */
  int32_t closed;
  const double *h_r, *h_z, *h_nr, *h_nz, *h_dsdu;  /* [N] each, host */
} msv_curve;

/* Near-panel quadrature rules (Section 5, eq_nyslike): for a target at
 * Gauss-Legendre node k of its panel, the panel itself is integrated with the
 * n_self nodes h_self_u[k*n_self + q] and weights h_self_w[...] (in u), and each
 * adjacent panel with the n_adj nodes/weights h_adj_u, h_adj_w.  Host arrays. */
typedef struct {
  int32_t n_self;
  const double *h_self_u, *h_self_w;   /* [order * n_self] */
  int32_t n_adj;
  const double *h_adj_u, *h_adj_w;     /* [n_adj] */
} msv_rules;

/* Physical and discretization parameters (Sections 1, 2.1, 4). */
typedef struct {
  double k0;                 /* exterior wavenumber, > 0 (omega -> 0 excluded) */
  msv_c128 eps0, mu0;        /* exterior: real and positive */
  msv_c128 eps1, mu1;        /* interior: Re > 0, Im >= 0 (eq. materials) */
  int32_t m_max;             /* M: modes |m| <= M are assembled and solved */
  int32_t fft_len;           /* L: azimuthal FFT length, a power of two in
                                [8, 1024]; the
                                plan refuses L too short for M and k (the
                                discrete convolution of eq. discA needs
                                M + 1 + N_f <= L/2 - 1) */
  int32_t precision;         /* 0: complex128 LU; 1: complex64 LU with
                                complex128 iterative refinement */
  double ir_tol;             /* precision 1: stop when ||b - A x|| <= ir_tol ||b|| */
  int32_t ir_max_iter;       /* precision 1: at most this many refinement steps */
  int32_t formulation;       /* 0: the direct system (eq. mullerrep), whose
                                currents are J = n x H, M = n x E; 1: the
                                indirect system (eq. dualmullrep, Section 2.2),
                                whose currents generate the exterior field by
                                eq. exteriorfield and the interior one by
                                eq. interior_dual.  Rows 4j, 4j+1 of every
                                right-hand side carry i w mu0 (n x H_inc)
                                (direct) or i w eps0 (n x H_inc) (indirect),
                                rows 4j+2, 4j+3 i w eps0 (n x E_inc) or
                                i w mu0 (n x E_inc), in (t, e_theta) components */
} msv_desc;

/* Device memory for the library's own buffers (plan geometry and workspace,
 * LU factors and inverses, solve workspace, batch lists).  By default the
 * library calls hipMalloc and hipFree.  A caller that runs its own pool of
 * device memory (a framework's caching allocator, a serving process that
 * recycles the memory of evicted bodies instead of returning it to the
 * driver) passes `alloc` and `free_fn`: alloc(bytes, device, ctx) returns
 * device memory of at least `bytes` on `device` (the current device), or
 * NULL when it cannot (the call then fails with MSV_ENOMEM);
 * free_fn(ptr, device, ctx) takes it back.  Inside a stream-ordered call
 * (storage regrown for more modes) the library waits for the device, as
 * hipFree does, before it hands a buffer back.  msv_plan_destroy does not
 * wait: with a pool the caller must have waited for the plan's last call
 * (synchronized its stream) before destroying it, so that destroying one
 * plan does not stall work on other streams.  Both hooks or neither
 * (NULL, NULL restores hipMalloc / hipFree); they may be changed only while
 * no plan or batch exists (MSV_EINVAL otherwise), and they are called from
 * the thread that makes the msv call.  Not part of the paper's method: the
 * memory management of a long-running process. */
typedef void *(*msv_alloc_fn)(size_t bytes, int32_t device, void *ctx);
typedef void (*msv_free_fn)(void *ptr, int32_t device, void *ctx);
msv_status msv_set_allocator(msv_alloc_fn alloc, msv_free_fn free_fn, void *ctx);

/* Validate the inputs, upload the geometry, build the near-panel support
 * nodes and the pair classification.  Synchronizes `stream` once. */
msv_status msv_plan_create(msv_plan **out, const msv_curve *curve, const msv_rules *rules,
                           const msv_desc *desc, void *stream);
void msv_plan_destroy(msv_plan *plan);
const char *msv_last_error(const msv_plan *plan);

/* Sizes: N nodes, S support slots per target (n_self + 2 n_adj), the number
 * of complex entries of the modal-kernel table, and the 4N x 4N matrix order. */
int32_t msv_num_nodes(const msv_plan *plan);
int32_t msv_num_support(const msv_plan *plan);
size_t msv_table_entries(const msv_plan *plan);
int32_t msv_matrix_order(const msv_plan *plan);

/* Device memory owned by a plan (not the caller's table, matrices, right-hand
 * sides or solutions).  msv_workspace_bytes is an upper bound, computable
 * before any plan exists, on what a plan of n_nodes nodes, n_support support
 * slots and FFT length fft_len holds once n_modes modes are factored
 * (msv_factor) and a solve of n_solve_vectors (mode, right-hand side) vectors
 * at once has run: geometry, the near pairs' spectra scratch (at most 262144
 * pairs x (fft_len/2 + 1) x 16 bytes), pivots, LU workspace, complex64 factors
 * (precision 1), diagonal-block inverses and the solve workspace.  It counts
 * the near-pair list and the spectra scratch as if every pair were near, so it
 * exceeds the real footprint by at most 8 N (N + S) bytes plus that scratch's
 * unused part, one 72-byte batch record per factored mode and 256 bytes of
 * alignment.  Returns 0 for invalid arguments.  msv_plan_device_bytes is what
 * the plan holds now.  Neither touches the device. */
size_t msv_workspace_bytes(int32_t n_nodes, int32_t n_support, int32_t fft_len, int32_t n_modes,
                           int32_t n_solve_vectors, int32_t precision);
size_t msv_plan_device_bytes(const msv_plan *plan);

/* Modal Green's functions (Section 4): for every target node t, every source
 * point s (the N nodes, then the S support nodes of t) and every mode
 * m = 0..M+1, the nine quantities
 *   0 g^{k0}            1 d_r g^{k0}              2 d_z g^{k0}
 *   3 g^{k0}-g^{k1}     4 d_r (g^{k0}-g^{k1})     5 d_z (g^{k0}-g^{k1})
 *   6 d_rr(g^{k0}-g^{k1})  7 d_rz(g^{k0}-g^{k1})  8 d_zz(g^{k0}-g^{k1})
 * with g^k_m = int_0^{2pi} e^{ik rho}/(4 pi rho) e^{-i m phi} dphi (eq. green11)
 * and derivatives with respect to the target coordinates.  The interior
 * kernels enter the Mueller system only through differences with the exterior
 * ones (eq. mullerrep: K^{k0} - K^{k1}, mu0 N^{k0} - mu1 N^{k1}); types 3-5 are
 * those differences, evaluated from analytic differences of the integrands so
 * that nothing cancels when the two kernels are close (g^{k1} = type 0 - type 3).
 * d_kern: device, [M+2][9][N][N+S] complex128, written in full (coincident
 * pairs t = s and unused support slots are 0).  kern_elems must equal
 * msv_table_entries(plan). */
msv_status msv_tabulate(msv_plan *plan, msv_c128 *d_kern, size_t kern_elems, void *stream);

/* The same table for the target rows t0 .. t0+nt-1 only (0 <= t0, 1 <= nt,
 * t0 + nt <= N): d_kern is [M+2][9][nt][N+S] complex128 and kern_elems must be
 * (M+2) * 9 * nt * (N+S).  Every pair is tabulated exactly as by
 * msv_tabulate, so row blocks of any size reproduce its table bit for bit.
 * A row block is all the assembly of those targets' equations reads (see
 * msv_assemble_rows), so a caller can stream a body whose whole table does not
 * fit beside its matrices (Section 5: the table is 9 (M+2) N (N+S) entries). */
msv_status msv_tabulate_rows(msv_plan *plan, int32_t t0, int32_t nt, msv_c128 *d_kern, size_t kern_elems,
                             void *stream);

/* Per-mode Mueller-Nystrom matrices (eq. mullerrep with Lemma 1 and the N, K
 * expansions of Section 3; quadrature of Section 5) for 0 <= m_lo <= m <= m_hi
 * <= M, from a table written by msv_tabulate on this plan.
 * d_A: device, [m_hi-m_lo+1][4N][4N] complex128, row-major.  Row 4i+a is the
 * equation at node i: a = 0,1 the t and theta components of the magnetic
 * equation, a = 2,3 of the electric one; column 4j+b the unknown at node j:
 * b = 0..3 for J^1, J^2, M^1, M^2 (J = n x H, M = n x E in (t, e_theta)).
 * The stored matrix is the L^2-weighted one, sqrt(w_i/w_j) A_ij (Section 6). */
msv_status msv_assemble(msv_plan *plan, const msv_c128 *d_kern, int32_t m_lo, int32_t m_hi,
                        msv_c128 *d_A, void *stream);

/* The equations (rows 4 t0 .. 4(t0+nt)-1 of every matrix) of targets
 * t0 .. t0+nt-1 only, from the row block d_kern written by msv_tabulate_rows
 * with the same t0, nt.  d_A is the full [m_hi-m_lo+1][4N][4N] array; the
 * other rows are not touched.  Bitwise the same rows as msv_assemble. */
msv_status msv_assemble_rows(msv_plan *plan, const msv_c128 *d_kern, int32_t t0, int32_t nt, int32_t m_lo,
                             int32_t m_hi, msv_c128 *d_A, void *stream);

/* The per-mode direct solve of Section 6: the discretized Mueller system of
 * each azimuthal mode (eq. mullerrep after the separation of variables of
 * Section 3) is a dense 4N x 4N system, factored once by LU with partial
 * pivoting so that further right-hand sides cost only triangular solves.
 * msv_factor factors each matrix of d_A (as written by msv_assemble for the
 * same m_lo..m_hi).  precision 0: complex128, in place in d_A; precision 1: the
 * plan keeps complex64 factors and d_A is left intact for the refinement
 * residual of msv_solve.  The plan keeps the pivots (and remembers d_A, which
 * must stay valid and unchanged until the last msv_solve).  A zero pivot is
 * recorded on the device and reported as MSV_ESINGULAR by the next msv_solve
 * (the first solve after a factorization reads the flags, which waits for the
 * factorization).  The plan allocates its factor storage on the first call
 * and whenever the mode count grows; while a batch holds the plan (see below)
 * it refuses, with MSV_EINVAL, a mode count larger than the batch's.
 * Streams: two or more modes of an order above 4096 are factored in two
 * halves, the second on a stream the plan owns, each of its panels after the
 * same panel of the first half (one half's panel factorization overlaps the
 * other's trailing update).  That stream waits for the work queued on
 * `stream` before the call, and `stream` for all of it after, so the call is
 * ordered on `stream` like any other; the factors are bitwise those of one
 * mode per call. */
msv_status msv_factor(msv_plan *plan, msv_c128 *d_A, int32_t m_lo, int32_t m_hi, void *stream);

/* Solve A_m x = b for modes m in [m_lo, m_hi] with -M <= m, |m| factored:
 * the surface currents J, M of each mode (Section 2.1, eq. mullerrep; the
 * further right-hand sides of Section 6 reuse the factors).
 * Negative modes use A_{-m} = D A_m D, D = diag(1, -1, -1, 1) per node.
 * d_rhs, d_x: device, [m_hi-m_lo+1][n_rhs][4N] complex128 in physical
 * (unweighted) form; rows as above: i w mu0 (n x H_inc)_{t,theta} then
 * i w eps0 (n x E_inc)_{t,theta}, Fourier modes (1/2pi) int f e^{-i m theta}.
 * d_x may not alias d_rhs.  precision 0: triangular solves with the complex128
 * factors, stream-ordered.  precision 1: x <- x + LU32^{-1}(b - A x) with the
 * residual in complex128 from the caller's matrices, until
 * max_v ||b - A x||_inf / ||b||_inf <= ir_tol; the steps the plan's previous
 * converged solve needed are queued without waiting, after which each step's
 * residual is read on the host, so the call returns once the stream reaches
 * the converged step.  MSV_ENOCONV if ir_max_iter steps do not converge (x
 * then holds the last iterate).  The solve workspace is allocated on the
 * first call and whenever the vector count grows. */
msv_status msv_solve(msv_plan *plan, int32_t m_lo, int32_t m_hi, int32_t n_rhs,
                     const msv_c128 *d_rhs, msv_c128 *d_x, void *stream);

/* msv_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, bit for bit, but its workspace is a static device array of the
 * library, msv_solve_noalloc_max_bytes() = 192 MiB, of which each device the
 * library runs on holds one copy until the process ends.  It calls no
 * hipMalloc or hipFree (the plan's factors must already exist: msv_factor
 * allocates).  A solve whose workspace would exceed the array -- 48 bytes
 * per element of the (mode, right-hand side) vectors, 64 with precision 1:
 * 257 modes of order 8192 with one right-hand side (135 MB) fit, with two
 * they do not -- returns MSV_EINVAL; solve fewer modes or right-hand sides
 * per call.  Every call on one device shares that
 * device's array and leaves its contents behind (nothing in it is assumed to
 * start at zero): calls that overlap on one device, on any streams or plans,
 * race and must be serialized by the caller. */
msv_status msv_solve_noalloc(msv_plan *plan, int32_t m_lo, int32_t m_hi, int32_t n_rhs,
                             const msv_c128 *d_rhs, msv_c128 *d_x, void *stream);
size_t msv_solve_noalloc_max_bytes(void);

/* Fields from the currents of msv_solve (Sections 2.1, 2.2 and 6).  d_x holds
 * the modes m_lo..m_hi (-M <= m_lo <= m_hi <= M) of n_vec solutions,
 * [m - m_lo][v][4N] as msv_solve returns them (J^1, J^2, M^1, M^2 per node).
 * Both calls synthesize the currents on a surface grid -- the N nodes times T
 * equispaced azimuths, weighted by the Gauss-Legendre arclength weights and
 * the trapezoid rule in theta -- in a stream-ordered workspace of
 * n_vec * N * T * 64 + T * 16 bytes allocated and freed by the call
 * (hipMallocAsync; MSV_ENOMEM if that fails), then reduce one sum over the
 * grid per output on the device.  Outputs are complex, device, row-major.
 *
 * msv_far_field: the far-field pattern of the exterior field (eq.
 * farfieldform, derived from eq. exteriorfield as |x| -> infinity, with the M
 * term that the printed form leaves out):
 *   E_inf(xhat) = (1/(4 pi)) [i k0 xhat x Mt - i omega mu0 xhat x (xhat x Jt)],
 *   Jt = int_Gamma e^{-i k0 xhat.y} J(y) da(y), Mt likewise,
 * so that the scattered field is e^{i k0 |x|}/|x| E_inf(x/|x|) + O(|x|^-2).
 * d_dirs [n_dirs][3] unit vectors; d_out [n_vec][n_dirs][3].
 * T = floor(2 (max |m| + k0 r_max) + 64).
 *
 * msv_fields: E and H at points off the surface.  region 0: points outside
 * the body, the scattered field of eq. exteriorfield; region 1: points inside,
 * the field of eq. interiorfield (direct system) or eq. interior_dual
 * (indirect system, msv_desc.formulation).  The caller states the region;
 * the rule along the curve loses accuracy for points whose distance to the
 * surface is small against the nearby panels, so with upsample = U in [2, 8]
 * each panel's current modes, r, z, dr/du and dz/du are first interpolated
 * (Legendre interpolation from its 16 nodes) to U sub-panels of 16
 * Gauss-Legendre nodes (the grid then has N U nodes and the workspace holds
 * the interpolated modes too).  The first call with a new U synchronizes
 * `stream` and uploads that sub-panel geometry, (5 N U + 256 U) * 8 bytes kept
 * by the plan (counted by msv_plan_device_bytes).  d_points [n_points][3];
 * d_E, d_H [n_vec][n_points][3].  T = floor(4 (max |m| + |k| r_max) + 128)
 * with k the region's wavenumber. */
msv_status msv_far_field(msv_plan *plan, int32_t m_lo, int32_t m_hi, int32_t n_vec, const msv_c128 *d_x,
                         int32_t n_dirs, const double *d_dirs, msv_c128 *d_out, void *stream);
msv_status msv_fields(msv_plan *plan, int32_t m_lo, int32_t m_hi, int32_t n_vec, const msv_c128 *d_x,
                      int32_t n_points, const double *d_points, int32_t region, int32_t upsample,
                      msv_c128 *d_E, msv_c128 *d_H, void *stream);

/* Iterations used by the last precision-1 msv_solve (max over modes). */
int32_t msv_last_ir_iterations(const msv_plan *plan);

/* ---------------------------------------------------------------------------
 * Batching form.  The paper factors the modes of one body at a time, with the
 * modes spread over threads (Section 6).  Here the per-mode systems of several
 * bodies, of different orders, are factored by one shared sequence of launches.
 * That sequence is captured once in a HIP graph and replayed.
 *
 * msv_batch_create: plans[i] (precision 1, distinct) with its matrices
 * d_A[i] = [m_hi-m_lo+1][4N_i][4N_i] from msv_assemble(plans[i], .., m_lo,
 * m_hi, ..).  The matrices must stay alive and unchanged while the batch is
 * used.  Creation allocates each plan's factor storage.  It then times the
 * outer panel widths 64, 128, 256 and 512 columns on the batch itself, keeps
 * the fastest graph, and leaves every plan factored as by msv_factor.  128,
 * 256 and 512 are candidates only when every order below the largest is a
 * multiple of them.
 * It synchronizes `stream` and returns MSV_EINVAL for bad arguments, MSV_ENOMEM
 * and MSV_EHIP otherwise (message: msv_batch_last_error(NULL)).
 *
 * msv_batch_factor: refactors the batch from the current contents of d_A,
 * ordered on `stream` (the graph runs on the batch's own stream, joined by
 * events).  Afterwards msv_solve works on each plan.  Factorizations of the
 * same plan outside the batch overwrite its factors.
 *
 * The captured launches hold the plans' factor storage by address, so a batch
 * pins its plans: msv_factor on a pinned plan may not grow that storage
 * (MSV_EINVAL), and msv_plan_destroy of a pinned plan only marks it; the last
 * msv_batch_destroy that holds it frees it.  msv_batch_destroy waits for the
 * batch's stream.
 * ------------------------------------------------------------------------- */
typedef struct msv_batch msv_batch;
msv_status msv_batch_create(msv_batch **out, msv_plan *const *plans, msv_c128 *const *d_A, int32_t n_plans,
                            int32_t m_lo, int32_t m_hi, void *stream);
msv_status msv_batch_factor(msv_batch *batch, void *stream);
void msv_batch_destroy(msv_batch *batch);
const char *msv_batch_last_error(const msv_batch *batch);
/* The autotuner chooses the tiling in two stages: the outer panel width (64,
 * 128, 256 or 512 columns, with trailing updates of at least 256 rows and
 * columns on 128 x 128 bf16 tiles), then at that width the smallest update
 * that goes to the 128 x 128 tiles (256, 512 or 1024; smaller updates use
 * 64 x 64 tiles).  The choice is kept per size class (device, largest order
 * and matrix count each rounded up to a power of two, and the panel widths
 * the orders allow); a later batch of a known class is captured with it
 * untimed. */
/* outer panel width the autotuner chose (64, 128, 256 or 512) */
int32_t msv_batch_panel(const msv_batch *batch);
/* smallest trailing update (rows and columns) on 128 x 128 tiles: 256, 512 or 1024 */
int32_t msv_batch_plane_min(const msv_batch *batch);
/* the timed duration in ms of one batched factorization with panel width 64,
 * 128, 256 or 512 (-1 if that candidate was not run) */
float msv_batch_tuned_ms(const msv_batch *batch, int32_t panel);
/* the same with the chosen panel width and plane_min 256, 512 or 1024 */
float msv_batch_tuned_plane_ms(const msv_batch *batch, int32_t plane_min);
/* 1 if the tiling came from the table of an earlier batch of the same size
 * class (only the chosen configuration was timed), 0 if tuned here */
int32_t msv_batch_tuned_from_table(const msv_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* MSV_H */
