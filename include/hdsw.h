/*
 * hdsw -- trace-transfer diagonal sweeping DDM for the Helmholtz equation
 * with PML, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Leng & Ju, "Trace transfer-based diagonal sweeping DDM for the
 * Helmholtz equation: algorithms and convergence analysis",
 * arXiv:2003.02585 -- Algorithm 2.1 (2D), Algorithm 4.1 (3D), used as a
 * preconditioner of an FP64 Krylov iteration as in Sec. 5.2.
 *
 * Problem (Sec. 2.1, eq. (helm), (radiation), (PML)): Delta u + k(x)^2 u = f
 * in R^d with the radiation condition, replaced by a uniaxial PML outside
 * the box B = [0, n_x h] x [0, n_y h] (x [0, n_z h]).  The library
 * discretizes eq. (PML) with the second-order 5-point (2D) / 7-point (3D)
 * stencil on cell-centred nodes x_p = (p + 1/2) h, W layer nodes per side,
 * quadratic profile sigma(t) = sigma0 (t / (W h))^2, alpha = 1 + i sigma,
 * sigma0 = 3 ln(1/pml_R) / (min k * W h), Dirichlet ghosts beyond the layer.
 * The J-scaled discrete operator S is complex symmetric.  The layer's
 * wavenumber is that of the nearest interior node (eq. (wave_number)).
 *
 * Partition (Sec. 2.3 / Sec. 4): nsub[a] equal boxes per axis; each
 * subdomain is extended by its own W-node PML and its wavenumber by the
 * nearest point of the subdomain.
 *
 * Conventions for every entry point:
 *  - All arrays are C order with x the fastest index.  Interior grids are
 *    [n_z][n_y][n_x]; "global" grids (interior plus layer) are
 *    [M_z][M_y][M_x] with M_a = n_a + 2 W.  Batches of right-hand sides are
 *    the slowest index: [nrhs][grid].
 *  - Device pointers must come from hipMalloc (or a caching allocator on
 *    top of it) on the context's device; they stay owned by the caller and
 *    must stay valid until the call returns.  Every entry point checks each
 *    array with hipPointerGetAttributes before any kernel runs: host memory
 *    (pinned or not), another device's memory, or an allocation too small
 *    for the stated nrhs (checked against the allocation that contains the
 *    pointer) returns HDSW_EINVAL and leaves the context usable.
 *  - Every call is ordered on the context's stream and returns when its
 *    work is complete.  One host thread per context; separate contexts may
 *    be used concurrently on separate streams and host threads.  The
 *    library's runtime calls that may wait on other streams (allocation,
 *    free, blocking copies, creation of streams, events and graphs) and its
 *    recording of a DDM application as a graph hold one process-wide lock,
 *    so one thread may factor a context while another records and replays
 *    applications of a different one.
 *  - Nothing throws or aborts across this interface; every function that
 *    can fail returns an hdsw_status.  HDSW_EDEVICE is sticky: the context
 *    must be destroyed.
 */
#ifndef HDSW_H
#define HDSW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdsw_ctx hdsw_ctx;

typedef struct { double re, im; } hdsw_c128;

typedef enum {
  HDSW_OK = 0,
  HDSW_EINVAL = 1,        /* invalid argument (shape, value, pointer)          */
  HDSW_ENOMEM = 2,        /* device allocation or HBM budget exceeded          */
  HDSW_EDEVICE = 3,       /* HIP runtime error (sticky)                        */
  HDSW_ENOTFACTORED = 4,  /* solve / apply before hdsw_factor                  */
  HDSW_ENOCONV = 5,       /* iteration limit reached; last iterate returned    */
  HDSW_EBUSY = 6          /* context in use                                     */
} hdsw_status;

enum { HDSW_FP64 = 0, HDSW_MIXED = 1 };

typedef struct {
  int dim;        /* 2 or 3                                                  */
  int n[3];       /* interior nodes per axis (x, y, z); n[2] ignored in 2D    */
  double h;       /* mesh width; B = [0, n[a] h] per axis                     */
} hdsw_grid;

typedef struct {
  int nsub[3];    /* subdomains per axis; n[a] % nsub[a] == 0              */
} hdsw_partition;

typedef struct {
  int precision;  /* HDSW_FP64: factors and sweeps in complex128.
                     HDSW_MIXED: factors and sweeps in complex64; the global
                     residual, the update and the Krylov iteration in FP64 */
  int rounds;     /* rounds of the 2^d sweeps per DDM application (>= 1);
                     2 = one extra round (Thm 3.10, Sec. 4)                  */
  double pml_R;   /* nominal layer attenuation giving sigma0 (> 0, < 1)      */
  double tol;     /* stop when ||b - S x||_2 / ||b||_2 <= tol, per RHS       */
  int max_iter;   /* iteration limit of hdsw_solve                           */
  int gmres_m;    /* 0: iterative refinement x += M^{-1}(b - S x);
                     m > 0: right-preconditioned GMRES(m), FP64 Arnoldi     */
  int dedup;      /* share factors between identical subdomain operators    */
  int graphs;     /* 1: a DDM application applied twice with the same
                     arrays and column count is captured as a HIP graph and
                     replayed from then on (same kernels, same results bit
                     for bit); 0: every launch is issued eagerly             */
  size_t hbm_budget; /* bytes for factors plus workspaces; 0 = no limit      */
  /* Device allocator hooks (both or neither; NULL = hipMalloc / hipFree).
   * Every device allocation of the context -- factors, interface responses,
   * workspaces -- is made by dev_alloc(bytes, alloc_ctx), which returns
   * device memory of the context's device usable on the context's stream,
   * aligned to 256 bytes, or NULL (the call then returns HDSW_ENOMEM); each
   * is released by dev_free(ptr, alloc_ctx), at the latest in hdsw_destroy.
   * Lets a framework's caching allocator own the memory pool.  The hooks are
   * called from the calling thread only, and must not call into the
   * library. */
  void* (*dev_alloc)(size_t bytes, void* alloc_ctx);
  void (*dev_free)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
} hdsw_options;

typedef struct {
  int iters;            /* iterations until this RHS met tol (or max_iter)  */
  double rel_residual;  /* final ||b - S x|| / ||b|| in FP64                */
} hdsw_solve_info;

/* Fills *opt with the defaults: HDSW_MIXED, rounds 1, pml_R 1e-16,
 * tol 1e-10, max_iter 30, gmres_m 0, dedup 1, graphs 1, no budget, no
 * allocator hooks. */
void hdsw_default_options(hdsw_options* opt);

/* Validates the problem, builds the partition, the per-subdomain layer
 * profiles and wavenumbers (eq. (sigma), eq. (wave_number)), the sweep
 * schedule (eq. (Sorder2D)/(Sorder3D), eq. (step_subd)/(step_subd3)) and the
 * trace routing (Rules 2.4/2.5, 4.1/4.2 applied over rounds * 2^d sweeps),
 * groups identical subdomain operators when opt->dedup, and allocates all
 * device state on the current device.
 *   kappa_host : host array [n_z][n_y][n_x] of real k > 0, finite; copied.
 *   pml_width  : W >= 1 layer nodes per side (global and subdomain layers).
 *   stream     : hipStream_t to order all work on (NULL = default stream).
 *   out        : receives the context; unchanged on failure.
 * Errors: EINVAL (dim not 2/3, n % nsub != 0, nonpositive sizes, W < 1,
 * non-finite or nonpositive k, h <= 0, bad options, only one allocator
 * hook, NULL pointers; in 2D an extended subdomain line n_x / P_x + 2 W of
 * more than 384 nodes, or more than 256 with HDSW_FP64, whose block solve
 * would not keep its vectors and register tiles on chip; in 3D an
 * interface response beyond 32-bit offsets), ENOMEM (budget or
 * allocation), EDEVICE. */
hdsw_status hdsw_setup(const hdsw_grid* grid, const double* kappa_host,
                       const hdsw_partition* part, int pml_width,
                       const hdsw_options* opt, void* stream, hdsw_ctx** out);

/* Factors every distinct subdomain operator once (the paper factors each
 * subdomain problem once with a sparse direct solver, Sec. 5): block
 * tridiagonal LU over grid lines (2D) or planes (3D),
 *   D_1 = A_1,  D_k = A_k - B_k D_{k-1}^{-1} B_k,  X_k = D_k^{-1},
 * each D_k inverted by Gauss-Jordan elimination with partial pivoting, and
 * (2D) the interface-to-interface response of each subdomain operator.
 * Idempotent.  Errors: EDEVICE, ENOMEM. */
hdsw_status hdsw_factor(hdsw_ctx* ctx);

/* Solves S x = b, b = h^2 J f, for nrhs sources:
 *   f_dev : device complex128 [nrhs][n_z][n_y][n_x], source on the interior
 *           nodes of B (zero in the layer, f supported in B, Sec. 2.1).
 *   x_dev : device complex128 [nrhs][n_z][n_y][n_x], receives u on the
 *           interior nodes.
 *   info  : host array of nrhs entries, or NULL.
 * Iterates (refinement or GMRES(m), FP64 residual on the device) with the
 * DDM of Algorithm 2.1 / 4.1 as preconditioner until every RHS meets tol.
 * Errors: EINVAL, ENOTFACTORED, ENOCONV (x holds the last iterate, info the
 * residuals), ENOMEM (nrhs too large for the budget), EDEVICE. */
hdsw_status hdsw_solve(hdsw_ctx* ctx, const hdsw_c128* f_dev,
                       hdsw_c128* x_dev, int nrhs, hdsw_solve_info* info);

/* One application of the DDM (opts.rounds rounds of Algorithm 2.1 / 4.1)
 * to global-grid right-hand sides:
 *   r_dev : device complex128 [nrhs][M_z][M_y][M_x], the b-space vector
 *           (for example a residual b - S x; nonzero in the layer allowed).
 *   z_dev : device complex128 [nrhs][M_z][M_y][M_x], receives u_DDM (sum of
 *           the local solutions on owned nodes, Algorithm 2.1's last line).
 * Computes in complex64 when precision == HDSW_MIXED.
 * Errors: EINVAL, ENOTFACTORED, ENOMEM, EDEVICE. */
hdsw_status hdsw_apply_precond(hdsw_ctx* ctx, const hdsw_c128* r_dev,
                               hdsw_c128* z_dev, int nrhs);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * DDM application as hdsw_apply_precond, with the same arguments and the
 * same results bit for bit, that allocates nothing.  Its per-call
 * workspaces come from a fixed 64 MiB array per device, held by the library
 * from its first load on that device until the process ends; nrhs is
 * processed in passes of as many columns as fit (at the 1024^2, 8 x 8
 * complex64 scale about 3 columns per pass).  Every call on one device
 * shares that array: calls that overlap on one device (several contexts on
 * several streams, or threads) race and must be serialized by the caller.
 * The context's own workspaces are not touched, so it may hold batch slots.
 * Errors: EINVAL (arguments, pointers as for every entry point),
 * ENOTFACTORED, ENOMEM (one column's workspace exceeds the 64 MiB array --
 * a refusal, not an allocation failure), EDEVICE (the array's address could
 * not be looked up, or a kernel failed). */
hdsw_status hdsw_apply_precond_noalloc(hdsw_ctx* ctx, const hdsw_c128* r_dev,
                                       hdsw_c128* z_dev, int nrhs);

/* Global residual r = b - S x on the global grid in FP64 (b on the global
 * grid, both [nrhs][M_z][M_y][M_x] complex128 on the device), and per-RHS
 * norms ||r||_2 written to rnorm_host (nrhs doubles, may be NULL).  r must
 * not overlap b or x (HDSW_EINVAL). */
hdsw_status hdsw_residual(hdsw_ctx* ctx, const hdsw_c128* b_dev,
                          const hdsw_c128* x_dev, hdsw_c128* r_dev, int nrhs,
                          double* rnorm_host);

/* Sizes: factor bytes, number of distinct subdomain operators, workspace
 * bytes currently allocated; any pointer may be NULL. */
hdsw_status hdsw_query(const hdsw_ctx* ctx, size_t* factor_bytes,
                       int* n_distinct_ops, size_t* workspace_bytes);

/* Kernel timing: HIP events bracket every launch of the enabled kernel
 * classes (0 = batched block solve, 1 = sweep step, 2 = block
 * factorization, 3 = FP64 residual, 4 = the source-driven 2D block solve of
 * a DDM application, which skips (subdomain, 8-column) pairs whose
 * right-hand side is zero; class 0 then holds the other block solves) on
 * the context's stream.  `enable` is a bit mask of classes (bit k enables
 * class k, 0 disables timing); events add a few microseconds between
 * launches, so time only what is needed.  hdsw_timing_get returns the
 * accumulated milliseconds, launch count and the algorithmic flops and
 * bytes of those launches (0 for class 4, whose work depends on the
 * data), then resets them. */
hdsw_status hdsw_timing_enable(hdsw_ctx* ctx, int enable);
hdsw_status hdsw_timing_get(hdsw_ctx* ctx, int which, double* total_ms,
                            long long* launches, double* flops, double* bytes);

/* Continuous batching (for a request loop): the context holds `capacity`
 * right-hand-side slots; solves join and leave between iterations.
 *   hdsw_batch_reserve : allocate workspaces for `capacity` columns; no
 *       slot may be occupied.  Errors: ENOTFACTORED, EINVAL, EBUSY, ENOMEM.
 *   hdsw_batch_add     : f_dev complex128 [nrhs][n_z][n_y][n_x] (interior
 *       sources, caller-owned, read before return); the column starts at
 *       x = 0, r = b; the slot ids are written to slots[nrhs] (host).
 *       EBUSY if fewer than nrhs slots are free.
 *   hdsw_batch_step    : enqueue one refinement iteration for every occupied
 *       slot: x += M^{-1} r (M^{-1} = the DDM of Algorithm 2.1), then the
 *       FP64 residual r = b - S x; returns without waiting, so steps of
 *       several contexts on separate streams overlap on the device.
 *   hdsw_batch_wait    : wait for the step; rel_residual (host, capacity
 *       entries, nullable) receives ||b - S x|| / ||b|| of each occupied
 *       slot's updated iterate, -1 for free slots and for slots added after
 *       the step was enqueued.
 *   hdsw_batch_ready   : non-blocking: HDSW_OK if the last step has
 *       finished (or none is in flight), HDSW_EBUSY while it runs.
 *   hdsw_batch_take    : copy the slot's iterate on the interior nodes to
 *       x_dev (complex128 [n_z][n_y][n_x], nullable) and free the slot;
 *       call it after hdsw_batch_wait.  The other slots keep their ids.
 * A column's arithmetic does not depend on the other columns.  While any
 * slot is occupied, hdsw_solve, hdsw_apply_precond and hdsw_residual on the
 * same context return HDSW_EBUSY (the slots own the workspaces). */
hdsw_status hdsw_batch_reserve(hdsw_ctx* ctx, int capacity);
hdsw_status hdsw_batch_add(hdsw_ctx* ctx, const hdsw_c128* f_dev, int nrhs, int* slots);
hdsw_status hdsw_batch_step(hdsw_ctx* ctx);
hdsw_status hdsw_batch_wait(hdsw_ctx* ctx, double* rel_residual);
hdsw_status hdsw_batch_ready(hdsw_ctx* ctx);
hdsw_status hdsw_batch_take(hdsw_ctx* ctx, int slot, hdsw_c128* x_dev);

/* Launch parameters of the kernels (the autotuner's search space; not a
 * passage of the paper: they choose how the method's block solves and sweep
 * steps are laid out on the GPU, never what they compute).  0 in a field
 * selects the library's built-in rule.
 *   solve_ng    : complex64 2D block solve, 1 = 8 or 2 = 16 right-hand sides
 *                 per workgroup (the columns of a product are independent:
 *                 results do not change).
 *   sweep_rw    : 2D sweep step, 2 or 4 row tiles of 16 per workgroup (sets
 *                 how a sum is split in parts, so results change at the
 *                 rounding level; fixed per context, never per call).
 *   sweep_kb    : 2D sweep step, 4-deep slices of the interface response
 *                 per register batch: 6, 8 or 10 (complex64), 3, 4, 5
 *                 or 6 (complex128); results do not change.
 *   gemm_skinny : 3D products with at most 8 columns per operator, 1 =
 *                 stream the matrix through the skinny kernel, 2 = tiled
 *                 kernel (order of the sum differs at the rounding level).
 *   sweep_nw    : 2D sweep step, 8 waves per workgroup (one workgroup per
 *                 CU, long face chunks staged at once) or 4 (two per CU,
 *                 shorter chunks); with sweep_rw it sets how a sum is
 *                 split in parts (results change at the rounding level).
 *   sweep_sched : 2D sweep steps, 1 = one launch per step in sweep order,
 *                 2 = the steps of one level of the slot dependences (a
 *                 subdomain's sweep after every trace its slot receives and
 *                 after its previous sweep) share a launch; every slot
 *                 still receives its additions in sweep order, so results
 *                 do not change.
 * hdsw_tuning_set validates every field (EINVAL for values outside the
 * lists above) and drops captured graphs; hdsw_tuning_get returns the
 * fields as set. */
typedef struct {
  int solve_ng;
  int sweep_rw;
  int sweep_kb;
  int gemm_skinny;
  int sweep_nw;
  int sweep_sched;
} hdsw_tuning;
hdsw_status hdsw_tuning_set(hdsw_ctx* ctx, const hdsw_tuning* t);
hdsw_status hdsw_tuning_get(const hdsw_ctx* ctx, hdsw_tuning* t);

void hdsw_destroy(hdsw_ctx* ctx);
const char* hdsw_status_str(hdsw_status s);

#ifdef __cplusplus
}
#endif

#endif /* HDSW_H */
