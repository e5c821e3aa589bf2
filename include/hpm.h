/*
 * hpm.h -- C ABI of the Hierarchical Particle-Mesh (HPM) library for AMD Instinct MI355X
 * (gfx950). HPM (Gnedin, "Hierarchical Particle-Mesh: an FFT-accelerated Fast Multipole
 * Method", arXiv:1906.10734) is an FMM in which each oct-tree cell carries a gridlet of N_g^3
 * effective masses whose Cartesian multipoles match the cell's (Sec. 2.2), and in which the
 * interaction-zone step is one zero-padded (8 N_g)^3 FFT convolution with the exact Green
 * function (Sec. 2.1).
 *
 * Problem statement (Sec. 1, Sec. 2.1, Sec. 4): particles with positions and masses in a cubic,
 * non-periodic box; the softened point-mass Green function g(r) = -G (r^2 + eps^2)^{-1/2};
 * a gridlet order N_g and a tree rule. Output: potential phi_i and acceleration a_i = -grad phi_i
 * of every particle, with the self term excluded.
 *
 * Conventions shared by every entry point:
 *   - Arrays named "device" are HIP device pointers to structure-of-arrays data, one element
 *     per particle, of the dtype given by hpm_problem.precision (float for HPM_F32, double for
 *     HPM_F64). Arrays named "host" are ordinary host memory.
 *   - The caller owns every array it passes; the library never frees or retains them. The
 *     library owns plans and contexts and the device memory inside them.
 *   - "stream" is a hipStream_t passed as void* (NULL is the legacy default stream). Compute
 *     calls enqueue on it; results are valid once the caller has synchronised the stream.
 *   - Calls return an hpm_status. Scalar arguments are checked on the host before any work.
 *     hpm_plan_create reads back a device status word and fails with HPM_ERR_OUT_OF_BOX or
 *     HPM_ERR_NONFINITE if any position is outside [box_lo, box_lo + box_size] or not finite
 *     (a position on the upper face belongs to the last cell). On failure nothing is written to
 *     the caller's output arrays and *out pointers are set to NULL. hpm_last_error() returns a
 *     thread-local message about the last failure.
 *   - A plan is used by one host thread at a time; distinct plans may be used from distinct
 *     threads. A server (below) may be called from several host threads.
 */
#ifndef HPM_H
#define HPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPM_ABI_VERSION 6

typedef enum {
  HPM_OK = 0,
  HPM_ERR_INVALID_ARG = 1,
  HPM_ERR_OUT_OF_BOX = 2,
  HPM_ERR_NONFINITE = 3,
  HPM_ERR_NO_MEMORY = 4,
  HPM_ERR_DEVICE = 5,
  HPM_ERR_UNSUPPORTED = 6,
  HPM_ERR_NOT_READY = 7
} hpm_status;

typedef enum { HPM_F64 = 0, HPM_F32 = 1 } hpm_precision;

/*
 * Interaction kernel: the potential g of a unit point mass at distance r, with the softened
 * distance s = (r^2 + eps^2)^{1/2}. The method is kernel independent (Abstract; Sec. 4): the
 * kernel enters the lattice Green function of the source-to-target step (Eq. 1 with g in place
 * of 1/r) and the near-zone pair sum; the gridlet fit, the translations and the interpolation
 * do not depend on it.
 *   HPM_KERNEL_NEWTON   g = -G / s                    (eps = 0: the bare 1/r kernel)
 *   HPM_KERNEL_YUKAWA   g = -G exp(-s / lam) / s      (screened; lam = screening > 0)
 */
typedef enum { HPM_KERNEL_NEWTON = 0, HPM_KERNEL_YUKAWA = 1 } hpm_kernel;

/*
 * Route of the source-to-target step (both compute the same sums, Sec. 2.1 and Sec. 2.5):
 *   HPM_M2L_GRID   one zero-padded (8 N_g)^3 convolution per target over its whole interaction
 *                  zone (the method);
 *   HPM_M2L_CELLS  cell-by-cell: each source cube's gridlet zero-padded to (2 N_g)^3 and
 *                  transformed once per solve, multiplied per (target, source) pair by the
 *                  transform of the Green function at that pair's cube offset, the products
 *                  summed and transformed back once per target (the alternative the paper
 *                  weighs in Sec. 2.5; kept for comparison).
 *   HPM_M2L_SHARED one zero-padded (8 N_g)^3 convolution per split parent, shared by its children:
 *                  the 152 cubes of the parent's 6^3 block outside its central 4^3 lie in the
 *                  interaction zone of all 8 children, so their transform is taken once and
 *                  read out at every child's window; the other 37 cubes of each child's zone
 *                  (the central 4^3 minus its 27 near cubes) are added cell by cell as in
 *                  HPM_M2L_CELLS. The two sets partition the zone, so nothing is subtracted
 *                  (the sharing of transforms among siblings that Sec. 2.1 leaves open).
 *                  N_g in {2, 3, 4, 6}; no extended gridlet.
 */
typedef enum { HPM_M2L_GRID = 0, HPM_M2L_CELLS = 1, HPM_M2L_SHARED = 2 } hpm_m2l_mode;

/*
 * Problem description.
 *   ng             gridlet points per axis (Sec. 2): 2, 3, 4, 6 or 8 (the FFT edge 8 N_g must
 *                  factor into 2s and 3s). N_g = 8 accepts at most 65536 particles (a plan for
 *                  more, or a rebuild or server request with more, returns HPM_ERR_UNSUPPORTED:
 *                  a 2^18-particle solve at N_g = 8 faulted in an earlier version of the library
 *                  and no cause has been shown). The padded-grid route only (the cell-by-cell
 *                  and shared routes go up to N_g = 6). Other values give HPM_ERR_UNSUPPORTED.
 *   precision      HPM_F32 or HPM_F64: dtype of all particle/output arrays and of the arithmetic
 *                  of the path. Constant tables (fit matrix, child-to-parent matrices, Green
 *                  function transforms) are always built in double and rounded once.
 *   uniform_depth  > 0: every cell is split down to this level (1..10); 0: adaptive rule.
 *   leaf_capacity  adaptive rule: a cell at level l is split while it holds more than
 *   max_depth      leaf_capacity particles and l < max_depth (1..10).
 *   softening      Plummer softening eps >= 0 of g(r) (eps = 0: the bare 1/r kernel).
 *   gconst         G > 0.
 *   box_lo, box_size  the cubic root cell (level 0), box_size > 0 (Sec. 1).
 *   kernel         an hpm_kernel value.
 *   m2l_mode       an hpm_m2l_mode value.
 *   screening      lam > 0 of HPM_KERNEL_YUKAWA (ignored for HPM_KERNEL_NEWTON).
 *   extended       0 or 1. 1: target gridlets widened by one node on every side (Sec. 2.5), so
 *                  the source-to-target output, parent-to-child and leaf interpolation use
 *                  (N_g + 2)^3 nodes at the same spacing; sources keep N_g^3 effective masses.
 *                  On the padded grid the target window is [(2 + c) N_g - 1, (3 + c) N_g + 1)
 *                  per axis, still exact with n = 8 N_g. Built on the cell-by-cell route
 *                  (N_g <= 6) and on the padded-grid route (N_g = 4 and 6); with
 *                  HPM_M2L_SHARED, or another order on the padded grid, it returns
 *                  HPM_ERR_UNSUPPORTED.
 *   reserved       must be 0.
 */
typedef struct {
  int32_t abi;
  int32_t ng;
  int32_t precision;
  int32_t uniform_depth;
  int32_t leaf_capacity;
  int32_t max_depth;
  double softening;
  double gconst;
  double box_lo[3];
  double box_size;
  int32_t kernel;
  int32_t m2l_mode;
  double screening;
  int32_t extended;
  int32_t reserved;
} hpm_problem;

/* Per-solve statistics filled by hpm_plan_info (host struct owned by the caller). */
typedef struct {
  int32_t n_levels;             /* levels 0..n_levels-1 hold real cells */
  int32_t ng;
  int64_t n_particles;
  int64_t n_cells;              /* real cells over all levels */
  int64_t n_leaves;
  int64_t n_targets;            /* cells at level >= 2: one source-to-target FFT each */
  int64_t cells_per_level[11];
  int64_t p2p_pairs;            /* near-zone pairs (including i == j slots), 0 until computed */
  int64_t device_bytes;         /* device memory the plan holds (buffers and tables) */
} hpm_plan_info;

typedef struct hpm_plan_s hpm_plan;

const char* hpm_status_string(hpm_status s);
const char* hpm_last_error(void);
int32_t hpm_abi_version(void);

/*
 * Tree construction (Sec. 1): Morton keys of the n positions, a stable key sort (ties by input
 * index), the levels of real cells by the tree rule, each cell's 27 cube neighbours, and the
 * leaf list. All of it runs on the device; the host reads back the counts per level. Positions
 * are copied into the plan in sorted order, so the caller may reuse x, y, z afterwards. The
 * plan holds every buffer hpm_plan_execute needs, sized for this tree.
 *   problem  host; n >= 1; x, y, z device arrays of n elements.
 *   *out     receives the plan (NULL on failure).
 * Errors: HPM_ERR_INVALID_ARG, HPM_ERR_UNSUPPORTED, HPM_ERR_OUT_OF_BOX, HPM_ERR_NONFINITE,
 * HPM_ERR_NO_MEMORY, HPM_ERR_DEVICE. The call synchronises "stream" once, when the counts that
 * size the tree are read back (x, y, z are no longer read after that); the last few kernels of
 * the build are enqueued after it, so work that uses the plan on another stream must wait for
 * "stream".
 */
hpm_status hpm_plan_create(const hpm_problem* problem, int64_t n, const void* x, const void* y,
                           const void* z, void* stream, hpm_plan** out);

/*
 * One HPM evaluation on the plan's tree with masses m (device, n elements, input order):
 *   P2M   Cartesian-moment fit of every leaf at level >= 2 (Eq. 2-5), here with Legendre
 *         moments and the equivalent fit matrix, as one batched dense GEMM on the matrix cores;
 *   M2M   child-to-parent translation T^C, deepest level first (Sec. 2.3);
 *   M2L   for every cell at level >= 2: the 189-cube interaction zone in one zero-padded
 *         (8 N_g)^3 FFT, times the transform of the exact lattice Green function, inverse FFT,
 *         target gridlet read out (Sec. 2.1, Eq. 1);
 *   L2L   parent-to-child via Eq. (6)-(7) evaluated at the child nodes (Sec. 2.4);
 *   L2P + P2P  Eq. (7) and its gradient at each particle plus the near-zone direct sum over
 *         the 27 neighbouring cubes (Sec. 1), combined with compensated addition.
 * Outputs phi, ax, ay, az (device, n elements, input order, caller-allocated) are overwritten.
 * Enqueued on "stream" without host synchronisation, allocation or memory set, so a caller may
 * capture it in a HIP graph and replay it for new masses on the same tree. For n >= 2^16 the
 * near-zone sums run on a stream the plan owns, forked from "stream" before the source-to-target
 * step and joined back before the leaf pass, so the call is ordered on "stream" as a whole.
 * Errors: HPM_ERR_INVALID_ARG (NULL pointer), HPM_ERR_DEVICE (launch failure).
 */
hpm_status hpm_plan_execute(hpm_plan* plan, const void* m, void* phi, void* ax, void* ay,
                            void* az, void* stream);

/*
 * Rebuilds the plan's tree for n new positions (same problem), reusing the plan's device
 * buffers; they grow when the new tree needs more. Same checks, errors and synchronisation as
 * hpm_plan_create; on failure the plan must not be executed until a rebuild succeeds.
 */
hpm_status hpm_plan_rebuild(hpm_plan* plan, int64_t n, const void* x, const void* y,
                            const void* z, void* stream);

/*
 * Per-stage timing with HIP events recorded on the caller's stream (off by default).
 * hpm_plan_enable_timing(plan, 1) clears the totals and starts recording; 0 stops it.
 * hpm_plan_stage_times waits for every recorded execution and returns accumulated
 * milliseconds in ms[7] (host): [0] tree build (create/rebuild), [1] P2M (moments + fit GEMM,
 * with the mass gather), [2] M2M, [3] M2L, [4] L2L, [5] leaves (L2P and the combination with
 * the near zone, plus the wait for the near-zone sums when they ran on the plan's second
 * stream), [6] the near-zone sums themselves (P2P, timed on the stream that ran them, beside
 * [3] and [4] from 2^16 particles on); *n_exec and *n_build (host, may be NULL) receive the
 * number of executions and builds timed.
 */
hpm_status hpm_plan_enable_timing(hpm_plan* plan, int32_t on);
hpm_status hpm_plan_stage_times(hpm_plan* plan, double* ms, int64_t* n_exec, int64_t* n_build);

/*
 * Source-to-target route of the plan's later evaluations (an hpm_m2l_mode). All three routes
 * compute the same sums (Sec. 2.1, Sec. 2.5); they differ in speed. A plan made with
 * HPM_M2L_GRID can only use that route, since the others need the cell spectra and their Green
 * tables; a plan made with HPM_M2L_CELLS or HPM_M2L_SHARED can use all three, except with
 * extended gridlets (HPM_M2L_CELLS, and HPM_M2L_GRID at N_g = 4 and 6).
 * Errors: HPM_ERR_INVALID_ARG (NULL plan, unknown mode), HPM_ERR_UNSUPPORTED (route not built).
 */
hpm_status hpm_plan_set_route(hpm_plan* plan, int32_t m2l_mode);

/*
 * Where the near-zone sums of later evaluations run: on = 1 (the default) puts them on a second
 * stream of the plan beside the source-to-target step from 2^16 particles on (they need only the
 * tree and the masses), on = 0 keeps them in line on the caller's stream after it. The results
 * are the same either way; in line, the near-zone time of hpm_plan_stage_times is that of the
 * kernel alone.
 * Errors: HPM_ERR_INVALID_ARG (NULL plan, on not 0 or 1).
 */
hpm_status hpm_plan_set_overlap(hpm_plan* plan, int32_t on);

/*
 * FP32 arithmetic throughout the padded-grid route's source-to-target step: on = 1 makes the
 * kernel form its inverse x sums (Sec. 2.1, the last inverse transform, pruned to the target's
 * nodes) and each target's mean in float-float arithmetic (pairs of floats, error-free sums and
 * FMA products, twiddles as float pairs from the FP64-built tables) instead of double, and L2L
 * (Sec. 2.4) add the local constants in float-float; on = 0 (the default) uses double there.
 * Other routes are unchanged. The results agree with the default to FP32 rounding of the inverse
 * transforms' inputs.
 * Errors: HPM_ERR_INVALID_ARG (NULL plan, on not 0 or 1), HPM_ERR_UNSUPPORTED (an FP64 plan, or
 * N_g other than 4 and 6).
 */
hpm_status hpm_plan_set_fp32_strict(hpm_plan* plan, int32_t on);

/*
 * Chooses the route by measurement: for every route the plan can use, one untimed evaluation
 * and then reps (1..1000) timed ones with masses m (device, n elements), outputs overwritten
 * (device, as hpm_plan_execute), HIP events on "stream"; keeps the fastest for later
 * evaluations. *mode (host, may be NULL) receives it, ms (host, 3 doubles, may be NULL) the mean
 * milliseconds per evaluation of HPM_M2L_GRID, _CELLS and _SHARED (-1 for a route the plan
 * cannot use). Synchronises "stream". On failure the plan keeps its previous route.
 */
hpm_status hpm_plan_autotune(hpm_plan* plan, const void* m, void* phi, void* ax, void* ay,
                             void* az, int32_t reps, void* stream, int32_t* mode, double* ms);

/* Releases the plan and all its device memory (NULL is ignored). Synchronises the device. */
void hpm_plan_destroy(hpm_plan* plan);

/* One-shot solve: hpm_plan_create + hpm_plan_execute + hpm_plan_destroy. Synchronises. */
hpm_status hpm_solve(const hpm_problem* problem, int64_t n, const void* x, const void* y,
                     const void* z, const void* m, void* phi, void* ax, void* ay, void* az,
                     void* stream);

/*
 * hpm_solve for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same steps and arguments as hpm_solve, but
 * every device buffer of the solve (particles in key order, tree, gridlets, local potentials,
 * near-zone work items, constant tables, the words the tree build reads back) is carved from a
 * fixed 64 MiB device region of the library, one per device, which each device holds from its
 * first call until the process ends. The call makes no hipMalloc, hipFree, hipHostMalloc, stream
 * or event creation; the near-zone sums run in line on "stream".
 * Limit: the estimate of hpm_plan_bytes_estimate for (problem, n) must fit the 64 MiB region (for
 * instance 4096 particles at any order, or 2^15 at N_g <= 6 in FP32); a larger problem returns
 * HPM_ERR_NO_MEMORY before any device work, and so does a tree that outgrows the region while it
 * is built (the outputs are then unspecified).
 * Calls on one device share the region and it keeps the last call's contents (every buffer is
 * written before it is read). Calls from threads of this process are serialised by the library,
 * and each call synchronises "stream" before it returns; any other overlapping use of the region
 * races.
 * Errors: those of hpm_plan_create and hpm_plan_execute.
 */
hpm_status hpm_solve_noalloc(const hpm_problem* problem, int64_t n, const void* x, const void* y,
                             const void* z, const void* m, void* phi, void* ax, void* ay,
                             void* az, void* stream);

/* Tree and size statistics of a plan (info: host, caller-owned). */
hpm_status hpm_plan_info_get(const hpm_plan* plan, hpm_plan_info* info);

/*
 * Inspection of a plan's device state, copied to host memory (synchronous on "stream").
 * These exist so that each step can be compared with an independent implementation.
 *   hpm_plan_copy_perm     perm[n] (int32): input index of the particle in each sorted slot.
 *   hpm_plan_copy_cells    for level l, count = cells_per_level[l] cells in Morton order:
 *                          coords[3*count] (int32, cube coordinates at level l), pb/pe[count]
 *                          (int32, sorted-slot range), split[count] (int32, 1 if internal),
 *                          parent[count] (int32, index within level l-1, -1 at level 0).
 *                          Any output pointer may be NULL.
 *   hpm_plan_copy_gridlets effective masses of level l cells after the last execute,
 *                          count * N_g^3 values of the plan's dtype, node index
 *                          i + N_g (j + N_g k) fastest in x (Sec. 2.2). Defined for l >= 2.
 *   hpm_plan_copy_locals   gridlet part dPhi of the local potentials of level l cells after the
 *                          last execute, same layout with N_g + 2 nodes per axis when
 *                          problem.extended is 1 (node i at (i - 1/2)/N_g - 1/2), l >= 2. The local potential (far field
 *                          from source-to-target plus parent-to-child, Sec. 2.1 and 2.4) of cell
 *                          i is c_i + dPhi_i, with the per-cell constant c_i (double, count
 *                          values) from hpm_plan_copy_local_offsets.
 * Errors: HPM_ERR_INVALID_ARG for a NULL plan or a level without cells.
 */
hpm_status hpm_plan_copy_perm(const hpm_plan* plan, int32_t* perm);
hpm_status hpm_plan_copy_cells(const hpm_plan* plan, int32_t level, int32_t* coords, int32_t* pb,
                               int32_t* pe, int32_t* split, int32_t* parent);
hpm_status hpm_plan_copy_gridlets(const hpm_plan* plan, int32_t level, void* host);
hpm_status hpm_plan_copy_locals(const hpm_plan* plan, int32_t level, void* host);
hpm_status hpm_plan_copy_local_offsets(const hpm_plan* plan, int32_t level, double* host);

/*
 * Direct sum of the kernel (the force-error reference of Sec. 3.2's accuracy measure), on the
 * device in double precision regardless of "precision" of the inputs:
 *   phi_t = sum_{j != i_t} m_j g(r_tj),  a_t = -grad phi_t
 * (for HPM_KERNEL_NEWTON: phi_t = -G sum m_j (r^2+eps^2)^{-1/2}, a_t = -G sum m_j r_tj (r^2+eps^2)^{-3/2})
 * for n_targets input indices "targets" (device int32) against all n sources.
 *   precision   dtype of x, y, z, m (HPM_F32 or HPM_F64);
 *   kernel, screening  as in hpm_problem;
 *   phi, ax, ay, az  device double arrays of n_targets elements (outputs).
 */
hpm_status hpm_direct_sum(int32_t precision, int64_t n, const void* x, const void* y,
                          const void* z, const void* m, int64_t n_targets, const int32_t* targets,
                          double gconst, double softening, int32_t kernel, double screening,
                          double* phi, double* ax, double* ay, double* az, void* stream);

/*
 * Estimated device memory of a plan for n particles of this problem (the admission measure of
 * the server below), made before the tree is known: 10 n / leaf_capacity + 64 cells (a uniform
 * density whose leaves hold just over an eighth of the capacity gives about 9.2 n /
 * leaf_capacity), or every cell of a uniform tree; one virtual cube per cell; four near-zone
 * work items per cell; and the Green tables of every level. It is an estimate: trees with many
 * particles at the deepest level, or leaves next to much denser regions, can need more. *bytes:
 * host.
 * Errors: HPM_ERR_INVALID_ARG, HPM_ERR_UNSUPPORTED (the checks of hpm_plan_create).
 */
hpm_status hpm_plan_bytes_estimate(const hpm_problem* problem, int64_t n, int64_t* bytes);

/*
 * Serving: many independent solves (each the whole method above on its own particle set) in
 * flight on one device at once.
 *
 * A server owns "slots" host worker threads. Each has its own HIP stream (default priority)
 * and runs one request at a time: tree, then one evaluation, then a synchronisation of its
 * stream. Requests wait in one first-in-first-out queue. The request at the head is admitted
 * when a worker is free and its memory fits: the estimate of hpm_plan_bytes_estimate beyond
 * what the plan it will use already holds, plus the memory that all plans hold, must stay
 * within hbm_budget. Plans stay resident between requests, keyed by the whole hpm_problem: a
 * request with a problem seen before rebuilds an idle plan of that problem (no table build,
 * no allocation once the plan is large enough). When the head does not fit, idle plans are
 * released, least recently used first; if it still does not fit and nothing else runs, the
 * request fails with HPM_ERR_NO_MEMORY. The estimate can be below what a clumped set's tree
 * needs; once the tree is built (before the evaluation buffers are sized) the request fails
 * with HPM_ERR_NO_MEMORY if its plan would hold more than its reservation plus the budget left
 * free at admission. Once a plan has served a request, its measured size replaces the estimate
 * in the total. Requests in flight on different workers overlap on the
 * device; each result is the one the same problem and particles give alone (the kernels do
 * not depend on what else runs).
 *
 * Buffers of a request (x, y, z, m, phi, ax, ay, az: device, n elements, the problem's
 * dtype, input order) are owned by the caller. Their contents must be complete on the device
 * when hpm_server_submit is called (synchronise the stream that wrote them), and they must
 * stay allocated, and the inputs unchanged, until the request has finished. The outputs are
 * valid once hpm_server_poll or hpm_server_wait reports the request.
 */
typedef struct {
  int32_t abi;          /* HPM_ABI_VERSION */
  int32_t slots;        /* 1..16 requests in flight at once */
  int64_t hbm_budget;   /* bytes of device memory the server's plans may hold; 0: no limit */
  int32_t reserved[4];  /* must be 0 */
} hpm_server_config;

/* What a finished request reports (host struct owned by the caller). */
typedef struct {
  int32_t status;       /* hpm_status of the solve */
  int32_t slot;         /* worker that ran it, -1 if it never ran */
  int64_t n;
  double submit_ms;     /* host clock, milliseconds since the server was created */
  double start_ms;      /* admitted: tree build starts */
  double done_ms;       /* outputs complete on the device */
  int64_t plan_bytes;   /* device memory of the plan that served it (after the solve) */
  int64_t estimate_bytes;  /* hpm_plan_bytes_estimate of the request */
} hpm_request_info;

/* Counters of a server (host struct owned by the caller). */
typedef struct {
  int64_t submitted, completed, failed;
  int32_t queued, running;
  int64_t plans;            /* resident plans */
  int64_t held_bytes;       /* device memory the plans hold, with reservations of running ones */
  int64_t peak_held_bytes;
  int64_t plans_created, plans_released;
} hpm_server_stats;

typedef struct hpm_server_s hpm_server;

/*
 * Starts a server on the calling thread's current device. cfg: host.
 * Errors: HPM_ERR_INVALID_ARG (abi, slots, negative budget, reserved != 0), HPM_ERR_DEVICE.
 */
hpm_status hpm_server_create(const hpm_server_config* cfg, hpm_server** out);

/*
 * Queues one solve and returns its ticket (host) at once. The problem is checked here, as by
 * hpm_plan_create (HPM_ERR_INVALID_ARG, HPM_ERR_UNSUPPORTED); the other errors of a solve
 * (out of box, non-finite, memory, device) arrive with the request's result.
 */
hpm_status hpm_server_submit(hpm_server* server, const hpm_problem* problem, int64_t n,
                             const void* x, const void* y, const void* z, const void* m,
                             void* phi, void* ax, void* ay, void* az, uint64_t* ticket);

/*
 * Result of a ticket. poll returns HPM_ERR_NOT_READY while the request is queued or running;
 * wait blocks until it has finished. Once finished, either returns the request's own status and
 * fills *info (host, may be NULL); that releases the ticket, and a later call on it returns
 * HPM_ERR_INVALID_ARG, as does an unknown ticket.
 */
hpm_status hpm_server_poll(hpm_server* server, uint64_t ticket, hpm_request_info* info);
hpm_status hpm_server_wait(hpm_server* server, uint64_t ticket, hpm_request_info* info);

/*
 * A batch of independent solves: submits count requests (host arrays of problems, sizes and
 * device pointers, one entry per solve), the largest first, and waits for all of them.
 * status (host, count entries, may be NULL) receives each solve's status. Returns HPM_OK when
 * every solve succeeded, else the status of the first failed solve in index order.
 */
hpm_status hpm_server_run_batch(hpm_server* server, int32_t count, const hpm_problem* problems,
                                const int64_t* n, const void* const* x, const void* const* y,
                                const void* const* z, const void* const* m, void* const* phi,
                                void* const* ax, void* const* ay, void* const* az,
                                int32_t* status);

hpm_status hpm_server_stats_get(hpm_server* server, hpm_server_stats* stats);

/*
 * Finishes every queued and running request, then stops the workers and releases the plans
 * (NULL is ignored). Tickets not yet reported are released with it. No other call on the same
 * server may run concurrently with it or follow it (every poll and wait must have returned).
 */
void hpm_server_destroy(hpm_server* server);

#ifdef __cplusplus
}
#endif

#endif /* HPM_H */
