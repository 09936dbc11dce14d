/* rbf_oracle.h -- plain CPU FP64 reference of Gaussian RBF interpolation solved
 * by GMRES with a restricted additive Schwarz preconditioner (Yokota, Barba and
 * Knepley, "PetRBF -- A parallel O(N) algorithm for radial basis function
 * interpolation").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against an independent, obviously correct computation.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no source, header, table or constant with the GPU library.
 *
 * All arrays passed in or out are in the caller's original point order unless a
 * comment says "sorted order" (the order of the cell-binned points).
 */
#ifndef RBF_ORACLE_H
#define RBF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_EINVAL = 1,
    ORC_EDUPLICATE = 2,
    ORC_ENOMEM = 3,
    ORC_ENOTPD = 5,
    ORC_ENOCONV = 6,
    ORC_EBREAKDOWN = 7,
    ORC_ENAN = 8,
    ORC_ESTATE = 9
};

typedef struct orc_problem orc_problem;

typedef struct {
    int iterations;           /* Arnoldi steps taken, over all restarts        */
    int restarts;             /* GMRES cycles completed                        */
    double rel_residual;      /* final true ||f - A x|| / ||f||                */
    int history_len;          /* entries written to history                    */
} orc_info;

/* Validate inputs, build the cell grid, bin and sort the points.
 * points: n x 2 row-major (x0, y0, x1, y1, ...).  Copies what it needs. */
int orc_create(const double* points, long long n, double sigma, double cutoff,
               int overlap, orc_problem** out);
void orc_destroy(orc_problem* p);

/* Grid: out4 = {x0, y0, L, invL}, ncxy = {ncx, ncy}. */
int orc_grid(const orc_problem* p, double* out4, long long* ncxy);

/* Binning artefacts: cell_of[i] (original order), perm[s] = original index of the
 * s-th sorted point, cell_start[c] for c = 0..ncells (ncells + 1 entries). */
int orc_binning(const orc_problem* p, int* cell_of, int* perm, long long* cell_start);

/* y = A w with A the cutoff-truncated normalised Gaussian matrix.
 * nnb (may be NULL): number of in-cutoff sources of each target, i = j included. */
int orc_matvec(const orc_problem* p, const double* w, double* y, int* nnb);

/* out[t] = sum_j lambda_j phi(|target_t - x_j|) over sources within the cutoff. */
int orc_evaluate(const orc_problem* p, const double* lambda, const double* targets,
                 long long m, double* out);
/* As orc_evaluate, and nnb[t] (may be NULL) = the number of sources summed for
 * target t (the target's in-cutoff neighbours). */
int orc_evaluate_counts(const orc_problem* p, const double* lambda, const double* targets,
                        long long m, double* out, int* nnb);

/* RASM: factor every local block (dense Cholesky), then z = M^{-1} v. */
int orc_rasm_setup(orc_problem* p);
int orc_rasm_apply(const orc_problem* p, const double* v, double* z);

/* Local block of cell c: members[k] = original index of the k-th member
 * (neighbour cells first, centre cell last), nomega, ncentre; L (may be NULL,
 * else nomega*nomega, column-major) = its Cholesky factor, upper part zero. */
int orc_rasm_block(const orc_problem* p, long long c, long long* members,
                   int* nomega, int* ncentre, double* L);
/* Member count of cell c's local block (to size the buffers above). */
int orc_rasm_block_size(const orc_problem* p, long long c, int* nomega, int* ncentre);

/* Subdomain geometry in lengths (Section 3.1, Fig. 3): the non-overlapping
 * subdomains become boxes of side B on a grid anchored at the minimum point
 * coordinates (box index by the cell rule with side B), the overlapping
 * subdomain of a box its own points and every point of the square of side
 * D >= B centred on it, and T > 0 (T >= B) replaces the radial cutoff of the
 * matvec by the square of side T centred on the target's box (T = 0 keeps the
 * radial cutoff).  Drops any RASM factors; the subdomain functions then index
 * boxes. */
int orc_set_geometry(orc_problem* p, double B, double D, double T);
/* Subdomains along x and y: boxes with a geometry set, else cells. */
int orc_subdomains(const orc_problem* p, long long* nxy);

/* Right-preconditioned restarted GMRES(m) on A x = f.  x0 may be NULL (zero).
 * history (may be NULL, capacity history_cap): true relative residual at the
 * start of every cycle and at the end. */
int orc_gmres(orc_problem* p, const double* f, int restart, double rtol, int max_iters,
              const double* x0, double* x, orc_info* info, double* history,
              int history_cap);

/* ||f - A x||_2 / ||f||_2 with the truncated matrix. */
int orc_rel_residual(const orc_problem* p, const double* f, const double* x, double* out);

/* Number of OpenMP threads the oracle runs with; set it (n > 0) for the
 * calls that follow on the calling thread. */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
