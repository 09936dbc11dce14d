/* rbf.h -- C ABI of the MI355X Gaussian radial-basis-function interpolation
 * library: cell binning, cutoff-truncated Gaussian matvec, restricted additive
 * Schwarz (RASM) preconditioner with dense local Cholesky solves, and
 * right-preconditioned restarted GMRES, in plain FP64 or FP32-inner/FP64-outer
 * mixed precision, all on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Yokota, Barba and Knepley, "PetRBF -- A parallel O(N)
 * algorithm for radial basis function interpolation":
 *   - the interpolation problem and its linear system: Section 2.1, eqs. rbf1
 *     and rbf2 (the Gaussian needs no polynomial block);
 *   - the normalised 2-D Gaussian A_ij = exp(-|x_i-x_j|^2/(2 sigma^2)) /
 *     (2 pi sigma^2) and the matvec that neglects distant pairs: Section 2.3;
 *   - RASM, z = sum_i Rt_i^T A_i^{-1} R_i v, used as a preconditioner for
 *     GMRES: Section 2.2, eq. rasm and the matrix M^{-1} that follows it.
 *
 * Conventions for every function:
 *   - extern "C", no exceptions cross the boundary, nothing aborts or exits;
 *     every failure is a status code, with detail in rbf_last_error().
 *   - Points are 2-D, passed as n x 2 row-major doubles (x0, y0, x1, y1, ...).
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory of the current device.  The caller owns every buffer it passes in;
 *     the library owns everything reachable from an rbf_problem handle.
 *   - Vectors indexed by point are in the caller's ORIGINAL point order unless
 *     an argument says RBF_ORDER_SORTED (the library's cell-binned order,
 *     sorted by (cell index, original index)).
 *   - stream: a hipStream_t passed as void*; NULL means the default stream.
 *     Calls that take host buffers synchronise that stream before returning.
 *   - A handle is not thread-safe; distinct handles may be used concurrently.
 */
#ifndef RBF_H
#define RBF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbf_problem rbf_problem;   /* opaque; created by rbf_setup* */

typedef enum {
    RBF_OK = 0,
    RBF_EINVAL = 1,       /* bad argument: n < 1, sigma/cutoff <= 0 or non-finite,
                             overlap < 0, NaN/Inf in points or values, NULL pointer */
    RBF_EDUPLICATE = 2,   /* two bit-identical points: the Gaussian matrix is then
                             singular (Section 2.1 needs distinct nodes) */
    RBF_ENOMEM = 3,       /* device allocation failed or max_device_bytes exceeded */
    RBF_EDEVICE = 4,      /* a HIP runtime error */
    RBF_ENOTPD = 5,       /* a local block failed its Cholesky factorisation */
    RBF_ENOCONV = 6,      /* iteration limit reached, or (RBF_MIXED) refinement
                             stalled; the last accepted iterate is returned */
    RBF_EBREAKDOWN = 7,   /* Arnoldi breakdown with a residual above tolerance */
    RBF_ENAN = 8,         /* a NaN or Inf appeared in an iterate */
    RBF_ESTATE = 9,       /* call out of order (e.g. evaluate before a solve) */
    RBF_ELIMIT = 10       /* problem exceeds a documented size limit (a cell with
                             more points than RBF_MAX_CELL_POINTS, or a local
                             block larger than RBF_MAX_BLOCK) */
} rbf_status;

/* RBF_FP64: every step in FP64.  RBF_MIXED: FP32 matvec and FP32 local
 * factors inside inner GMRES solves, FP64 outer residual, Arnoldi and update
 * (iterative refinement).  RBF_FP64_PC32: the FP64 method (FP64 matvec,
 * Arnoldi, residual and update) right-preconditioned with the FP32 local
 * factors' centre rows, applied to the FP64 vector with FP64 sums: a fixed
 * linear preconditioner, so the solve and its stopping test are the FP64
 * method's, with half the preconditioner's bytes. */
typedef enum { RBF_FP64 = 0, RBF_MIXED = 1, RBF_FP64_PC32 = 2 } rbf_precision;
typedef enum { RBF_ORDER_ORIGINAL = 0, RBF_ORDER_SORTED = 1 } rbf_order;

#define RBF_MAX_BLOCK 1536          /* largest overlapping-subdomain size */
#define RBF_MAX_CELL_POINTS 1536    /* largest number of points in one cell */

typedef struct {
    int restart;            /* GMRES restart length m (default 30) */
    int max_iters;          /* total Arnoldi steps over all cycles (default 10000) */
    double rtol;            /* stop when ||f - A lambda||_2 / ||f||_2 <= rtol, with
                               A the cutoff-truncated matrix (default 1e-10) */
    rbf_precision precision;
    double inner_rtol;      /* RBF_MIXED: inner GMRES relative tolerance (default 1e-4) */
    int max_outer;          /* RBF_MIXED: outer refinement steps (default 60); an
                               outer step that does not lower the FP64 residual is
                               undone and the solve ends with RBF_ENOCONV */
    size_t max_device_bytes;/* 0 = no limit; else fail with RBF_ENOMEM beyond it */
    void* stream;           /* hipStream_t for every launch of the call */
    int stall_cycles;       /* RBF_FP64 and RBF_FP64_PC32: 0 (default) = off; k > 0 ends
                               the solve with RBF_ENOCONV (and its last iterate) when
                               the true residual at the start of a cycle is above half
                               of what it was k cycles earlier -- for callers such as a
                               serving loop that would rather give up on a stagnating
                               system (GMRES(m) restarted on a system beyond the
                               preconditioner, e.g. h/sigma < 0.7 with the 6 sigma
                               cutoff) than spend max_iters on it */
} rbf_solve_opts;

typedef struct {
    int iterations;         /* Arnoldi steps (inner steps in RBF_MIXED) */
    int outer_iterations;   /* refinement steps (RBF_MIXED), else 0 */
    int restarts;           /* GMRES cycles completed */
    double rel_residual;    /* final true relative residual, FP64 */
    /* phase seconds, named after the paper's time breakdown (Section 4.2):
       t_init is the handle's set-up (binning, sorting, neighbour lists; the
       same figure for every solve on one handle), t_pcsetup the local
       factorisations this call made (0 if they were already built) */
    double t_init, t_pcsetup, t_matmult, t_matsolve, t_vecmdot, t_other;
    long long interactions_per_matvec;  /* in-cutoff ordered pairs, i = j included
                                           (with a box truncation the pairs of the
                                           box squares); -1 until rbf_neighbor_counts
                                           has run or a truncation side was set */
    int matvecs64;          /* FP64 matvec applications in this call */
    int matvecs32;          /* FP32 matvec applications (RBF_MIXED inner solves) */
    int precond_applies;    /* RASM applications */
    size_t device_bytes;    /* bytes the handle holds on the device */
    int history_len;        /* entries in history (valid until the next call) */
    const double* history;  /* true relative residual at each cycle start and end */
    int shifted_blocks;     /* RBF_MIXED, RBF_FP64_PC32: local blocks factored with a diagonal
                               shift (FP32 Cholesky breakdown), else 0 */
} rbf_solve_info;

/* Set opts to the defaults listed above. */
void rbf_default_opts(rbf_solve_opts* opts);

/* Build a problem from host arrays (Section 2.1: points x_j, data f_j):
 * bins the points into square cells of side `cutoff` (the non-overlapping
 * subdomains), sorts them by cell, and checks them.  `overlap` is the number of
 * cell layers added around a cell to form its overlapping subdomain (1 gives the
 * 3x3 block of cells).  sigma is the Gaussian width; pairs farther apart than
 * `cutoff` are dropped from the matvec.  values may be NULL (then solve needs a
 * right-hand side through rbf_set_values).  Inputs are copied; they may be
 * freed on return.  Errors: RBF_EINVAL, RBF_EDUPLICATE, RBF_ENOMEM, RBF_EDEVICE,
 * RBF_ELIMIT. */
rbf_status rbf_setup(const double* points, const double* values, long long n,
                     double sigma, double cutoff, int overlap, rbf_problem** out);

/* As rbf_setup, with device arrays read on `stream`. */
rbf_status rbf_setup_device(const double* d_points, const double* d_values, long long n,
                            double sigma, double cutoff, int overlap, void* stream,
                            rbf_problem** out);

/* Replace the right-hand side f (n values, original order, device or host). */
rbf_status rbf_set_values(rbf_problem* p, const double* values, int values_on_device,
                          void* stream);

/* Subdomains in lengths (Section 3.1, Fig. 3): the non-overlapping subdomains
 * become boxes of side `box` (B) on a grid anchored at the minimum point
 * coordinates (box index floor((x - x_min) / B), clamped to the grid), and the
 * overlapping subdomain of a box its own points and every point within half
 * of `overlap` (D >= B) of the box's centre x_min + (b + 1/2) B along both
 * axes; members in the cell-sorted order with the box's own points last.
 * The paper's measured optimum is B = 5 sigma, D = 1.9 B.
 * With truncation = 0 the product keeps its radial cutoff.  With a truncation
 * side T >= B it is truncated by boxes instead (Section 3.1): a point keeps
 * the sources inside the square of side T centred on its own box (the same
 * |x - centre| <= T/2 test along both axes), so the matrix is no longer
 * symmetric; the paper takes T = B + 4 sigma (B + 6 sigma at h/sigma = 0.8),
 * which on the paper's iteration counts reads as the box widened by 4 sigma
 * (6 sigma) on every side: T = B + 8 sigma (B + 12 sigma).  Every product,
 * residual, count and evaluation of the handle then uses the box truncation;
 * it runs in FP64 only (rbf_solve with RBF_MIXED and rbf_matvec_device with
 * RBF_MIXED fail with RBF_EINVAL; RBF_FP64_PC32 is allowed), and the serving
 * engine does not pack such handles.  A per-box list of the square's points
 * is kept on the device (4 bytes per (box, point) pair).
 * Replaces the cell subdomains set up by rbf_setup (and drops any
 * preconditioner built on them); rbf_precond_block then indexes boxes, row by
 * row.  Errors: RBF_EINVAL (NULL, B <= 0, D < B, T neither 0 nor >= B,
 * non-finite, too many boxes), RBF_ELIMIT (a truncation side with 2^24 boxes
 * or more), RBF_ENOMEM (the boxes may then be set with the radial product); a
 * box whose square holds more than RBF_MAX_BLOCK points makes the next
 * rbf_precond_setup fail with RBF_ELIMIT. */
typedef struct {
    double box;         /* B: side of the non-overlapping subdomains */
    double overlap;     /* D: side of the overlapping square around each one */
    double truncation;  /* T: side of the product's square per box, 0 = radial cutoff */
} rbf_geometry;
rbf_status rbf_set_geometry(rbf_problem* p, const rbf_geometry* geo, void* stream);

/* Factor every local block (Section 2.2: A_i on the overlapping subdomain,
 * untruncated Gaussian, dense Cholesky) and keep the centre rows of its inverse.
 * precisions RBF_MIXED and RBF_FP64_PC32 store them in FP32 (one FP32 set serves
 * both).  rbf_solve calls this when needed;
 * calling it first separates its time.  Errors: RBF_ENOTPD, RBF_ENOMEM. */
rbf_status rbf_precond_setup(rbf_problem* p, rbf_precision precision, void* stream);

/* Solve A lambda = f (Section 2.1) by GMRES(m) right-preconditioned with RASM
 * (Section 2.2).  lambda0: initial guess, original order, host, or NULL for 0.
 * lambda_out: n host doubles, original order.  info may be NULL.
 * On RBF_ENOCONV lambda_out holds the last iterate and info its residual. */
rbf_status rbf_solve(rbf_problem* p, const rbf_solve_opts* opts, const double* lambda0,
                     double* lambda_out, rbf_solve_info* info);

/* As rbf_solve with device buffers (original order). */
rbf_status rbf_solve_device(rbf_problem* p, const rbf_solve_opts* opts,
                            const double* d_lambda0, double* d_lambda_out,
                            rbf_solve_info* info);

/* Interpolant s(x) = sum_j lambda_j phi(|x - x_j|) (eq. rbf1 without the
 * polynomial part) at m targets (m x 2 host doubles) with the weights of the
 * last successful solve, over sources within the cutoff (with a box
 * truncation, over the square of the box the target falls in).  Targets
 * outside the point set's grid are clamped to the border cells (boxes).
 * Errors: RBF_ESTATE if no solve has succeeded. */
rbf_status rbf_evaluate(const rbf_problem* p, const double* targets, long long m,
                        double* out);
rbf_status rbf_evaluate_device(const rbf_problem* p, const double* d_targets, long long m,
                               double* d_out, void* stream);

/* The interpolant on a regular lattice of targets, t(a, b) = (x0 + a hx,
 * y0 + b hy) for a < nx, b < ny (remeshing onto a lattice, the use the paper's
 * Sections 1 and 5 name): out[b nx + a], the same sums as rbf_evaluate at those
 * coordinates (each computed as x0 + a * hx, one rounding per operation), with
 * the lattice's separable structure used for speed.  hx, hy > 0; x0, y0 and the
 * far corner finite.  out: nx * ny doubles, host (rbf_evaluate_lattice) or
 * device on `stream` (rbf_evaluate_lattice_device), caller-owned.  nx or ny = 0
 * writes nothing.  Errors: RBF_ESTATE (no successful solve), RBF_EINVAL (NULL
 * output, negative sizes, non-finite origin or extent, spacing <= 0),
 * RBF_ELIMIT (a side above 2^31, more than 2^40 targets, or more than 2^26
 * tiles of 8 x 8 targets within one cell each), RBF_ENOMEM. */
rbf_status rbf_evaluate_lattice(const rbf_problem* p, double x0, double y0, double hx, double hy,
                                long long nx, long long ny, double* out);
rbf_status rbf_evaluate_lattice_device(const rbf_problem* p, double x0, double y0, double hx,
                                       double hy, long long nx, long long ny, double* d_out,
                                       void* stream);

/* The number of sources the interpolant sums at each of m targets (device
 * arrays: targets m x 2, counts m ints, original target order): the in-cutoff
 * neighbours of eq. rbf1's truncated sum, found as rbf_evaluate_device finds
 * them (target cells clamped to the grid).  Needs no solve.  Errors:
 * RBF_EINVAL (NULL, m < 0, NaN or Inf in the targets). */
rbf_status rbf_target_counts_device(const rbf_problem* p, const double* d_targets, long long m,
                                    int* d_counts, void* stream);

/* Release everything the handle owns (NULL is ignored).  Waits for the work
 * that the handle's calls enqueued and no other work, through an event
 * recorded on the stream of the handle's last call, which must therefore
 * still exist; the handle's device buffers go to the library's block cache
 * (below). */
void rbf_destroy(rbf_problem* p);

/* Device block cache.  Buffers a handle gives back (on rbf_destroy, or
 * scratch freed inside a call) are kept by the library and handed to later
 * allocations of about the same size on the same device (a block at most
 * 1/8 larger than asked), so that a stream of problems of varying sizes
 * neither maps fresh memory per call nor waits for the whole device on each
 * free.  A block is handed out again only after the work that last used it
 * has finished.  Idle blocks are returned to the runtime when an allocation
 * fails, when they exceed a quarter of the device memory, or here.
 *   device      device ordinal, or -1 for every device
 *   trim        non-zero: return the idle blocks of `device` to the runtime
 *   idle_bytes  out (may be NULL): idle bytes held before trimming
 * Thread-safe.  Budgets (max_device_bytes) count the block sizes actually
 * held, which are rounded up to 2 MiB (powers of two below 1 MiB). */
rbf_status rbf_block_cache(int device, int trim, size_t* idle_bytes);

/* ---- single steps of the method, for measurement and parity checks -------- */

/* Grid: out4 = {x0, y0, L, 1/L} (origin = minimum coordinates, side L = cutoff),
 * ncxy = {ncx, ncy}. */
rbf_status rbf_grid(const rbf_problem* p, double* out4, long long* ncxy);

/* Binning (host outputs, any may be NULL): cell_of[i] for each original point,
 * perm[s] = original index of the s-th sorted point, cell_start[c] for
 * c = 0..ncx*ncy (ncx*ncy + 1 entries, int32). */
rbf_status rbf_binning(const rbf_problem* p, int* cell_of, int* perm, int* cell_start);

/* Number of in-cutoff sources of every point (original order, host), and the
 * total (the interactions of one matvec); with a box truncation, the points
 * of the square of each point's box. */
rbf_status rbf_neighbor_counts(rbf_problem* p, int* nnb, long long* total);

/* y = A w (Section 2.3, truncated normalised Gaussian) on device vectors in the
 * given order; precision RBF_MIXED runs the FP32 kernel (FP64 in and out;
 * RBF_EINVAL under a box truncation); RBF_FP64_PC32 is not a matvec precision
 * (RBF_EINVAL). */
rbf_status rbf_matvec_device(rbf_problem* p, const double* d_w, double* d_y,
                             rbf_precision precision, rbf_order order, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of rbf_matvec_device in the caller's ORIGINAL order, with the sorted-order
 * staging of w and y in a fixed device array that the library holds on every
 * device it runs on (two vectors of RBF_NOALLOC_MAX_POINTS doubles, 64 MiB)
 * instead of blocks it allocates.  The call allocates nothing and does not
 * wait; it enqueues three kernels on `stream`.  d_w and d_y are n device
 * doubles in original order (caller-owned; they may not overlap).  The array
 * is shared by every call on one device and keeps the last call's contents:
 * calls that overlap in time on one device (concurrent streams or threads)
 * race on it and must be serialised by the caller.  Errors: RBF_EINVAL (NULL
 * argument, bad precision), RBF_ELIMIT (more than RBF_NOALLOC_MAX_POINTS
 * points), RBF_EDEVICE (the array's address could not be read). */
#define RBF_NOALLOC_MAX_POINTS 4194304
rbf_status rbf_matvec_device_noalloc(rbf_problem* p, const double* d_w, double* d_y,
                                     rbf_precision precision, void* stream);

/* z = M^{-1} v, RASM (Section 2.2, eq. rasm), on device vectors; builds the
 * preconditioner of that precision first if needed.  RBF_MIXED applies the
 * FP32 centre rows in FP32 (v rounded to FP32, Kahan sums); RBF_FP64_PC32
 * applies the same FP32 centre rows to the FP64 v with FP64 sums. */
rbf_status rbf_precond_apply_device(rbf_problem* p, const double* d_v, double* d_z,
                                    rbf_precision precision, rbf_order order,
                                    void* stream);

/* Members of subdomain c's overlapping subdomain (original indices; for cells
 * the neighbour cells in (dy, dx) order first, for boxes the cell-sorted order;
 * the subdomain's own points last) and the stored centre
 * rows Z_c of the inverse of its local matrix, row-major ncentre x nomega, as
 * doubles.  Pass NULL to query the sizes only. */
rbf_status rbf_precond_block(rbf_problem* p, long long c, rbf_precision precision,
                             long long* members, double* z_rows, int* nomega,
                             int* ncentre);

/* Kernels of the local factorisations (rbf_precond_setup), by kind. */
typedef enum {
    RBF_K_ASSEMBLE = 0,   /* local matrices and their first 64x64 diagonal factor */
    RBF_K_CHOL_STEP = 1,  /* 64-column block-column update and panel solve, one launch each */
    RBF_K_CHOL_DIAG = 2,  /* next diagonal block: product and 64x64 Cholesky */
    RBF_K_FORWARD = 3,    /* forward solve L W = E_C on the trailing rows */
    RBF_K_BACK = 4,       /* back solve L^T X = W, one launch per 32-row block row */
    RBF_K_SETUP_KINDS = 5
} rbf_setup_kernel;

/* Event timing of the local factorisations.  With enable != 0, later
 * rbf_precond_setup calls on this handle record a HIP event pair around every
 * kernel launch they make (on their stream) and add up the elapsed time per
 * kind; profiling costs two event records per launch.  rbf_setup_kernel_times
 * gives, for the last profiled setup of the given precision, the total
 * milliseconds ms[k] and launch count launches[k] of each kind k
 * (RBF_K_SETUP_KINDS entries each, caller-owned host arrays).
 * Errors: RBF_EINVAL (NULL argument), RBF_ESTATE (no profiled setup yet). */
rbf_status rbf_set_profiling(rbf_problem* p, int enable);

/* Graph launches of the Arnoldi step (Section 2.2's GMRES iteration; the
 * Gram-Schmidt work of step j -- two classical passes, the norm, the
 * normalisation and the read-back of the Hessenberg column -- captured once per
 * j as a HIP graph -- when step j comes round a second time on the handle --
 * and replayed on the solve's stream).  enable != 0 uses them; enable == 0
 * (the default: on ROCm 7 one graph launch of these few kernels costs more
 * than launching them back to back) launches the same kernels one by one.
 * The results are bit-identical either way.  A handle whose capture fails
 * falls back to single launches by itself.  Errors: RBF_EINVAL (NULL handle). */
rbf_status rbf_set_graphs(rbf_problem* p, int enable);
rbf_status rbf_setup_kernel_times(const rbf_problem* p, rbf_precision precision, double* ms,
                                  int* launches);

/* ---- serving: a request loop over many problems (continuous batching) ---- */

/* Requests are admitted in arrival order whenever fewer than max_active are
 * on the device and their predicted device footprint fits what the budget has
 * left (a request larger than the whole budget is admitted alone); each
 * admitted request runs its setup and preconditioner on its own HIP stream
 * from a worker thread, so requests that arrive while others run join as
 * slots and memory free up and their kernels overlap on the device.  Its solve
 * then joins a packed engine at the next step boundary (packed > 0, up to
 * pack_max_points points): an engine thread advances every solve it holds by
 * one GMRES step per engine step, each kernel of the step (the RASM applies, the matvecs, the
 * Gram-Schmidt passes) launched once for all requests over a (request, unit)
 * job table, the step captured as a HIP graph per set of requests; with
 * packed = 0 each request solves alone on its worker's stream.  Either way a
 * request's arithmetic is that of a lone rbf_solve_device call, with the same
 * per-request reductions: its weights do not depend on the mix. */
typedef struct rbf_server rbf_server;   /* opaque; created by rbf_server_create */

typedef struct {
    int max_active;            /* requests on the device at once, 1..64 (default 8) */
    size_t max_device_bytes;   /* admission budget; 0 = 90% of the device memory free
                                  at creation */
    int packed;                /* engines, 0..8 (default 2): each engine advances the
                                  solves it holds together, each engine step one
                                  Arnoldi step (or cycle end) of every one of them,
                                  every kernel of the step launched once for all;
                                  new solves go to the engine holding the fewest, so
                                  one engine's host work overlaps the others' steps;
                                  0: each request solves alone on its worker's stream */
    int graphs;                /* packed: capture a step's launches once per set of
                                  active requests as a HIP graph and replay it
                                  (default 1) */
    long long pack_max_points; /* packed: requests with more points solve alone on
                                  their worker's stream (their kernels fill the
                                  device by themselves, and in lockstep they would
                                  hold the small ones back); 0 = no limit
                                  (default 65536) */
} rbf_server_opts;

typedef struct {
    rbf_status status;         /* of the request's setup + preconditioner + solve */
    rbf_solve_info info;       /* as rbf_solve_device fills it (history NULL) */
    double t_queue;            /* seconds from submission to admission */
    double t_run;              /* seconds from admission to completion */
    double latency;            /* t_queue + t_run */
    size_t predicted_bytes;    /* footprint charged against the budget */
    char message[256];         /* rbf_last_error of the failing call, or "" */
} rbf_request_result;

void rbf_server_default_opts(rbf_server_opts* opts);
/* Starts the dispatcher and max_active worker threads on the current device.
 * Errors: RBF_EINVAL, RBF_ENOMEM, RBF_EDEVICE. */
rbf_status rbf_server_create(const rbf_server_opts* opts, rbf_server** out);
/* Queue one interpolation problem (arguments as rbf_setup, host arrays copied
 * on the call, options as rbf_solve with their stream ignored); returns at
 * once with the request's id.  Errors: RBF_EINVAL, RBF_ESTATE (server
 * stopping). */
rbf_status rbf_server_submit(rbf_server* s, const double* points, const double* values,
                             long long n, double sigma, double cutoff, int overlap,
                             const rbf_solve_opts* opts, long long* id);
/* Block until request id has finished; copy its weights (n host doubles,
 * original order; also on RBF_ENOCONV) to lambda_out if not NULL and its
 * result to *result if not NULL.  Returns the request's status; each request
 * is collected once (RBF_EINVAL for an unknown or collected id). */
rbf_status rbf_server_wait(rbf_server* s, long long id, double* lambda_out,
                           rbf_request_result* result);
/* Counters: requests submitted and finished so far, on the device, queued, and
 * the bytes their predicted footprints currently charge.  NULL fields skipped. */
rbf_status rbf_server_stats(rbf_server* s, long long* submitted, long long* finished,
                            int* active, int* queued, size_t* bytes_charged);
/* Finish every submitted request, then stop the threads and free the server
 * (uncollected results are dropped). */
void rbf_server_destroy(rbf_server* s);

const char* rbf_status_string(rbf_status s);
const char* rbf_last_error(void);   /* detail of the calling thread's last error */

#ifdef __cplusplus
}
#endif
#endif
