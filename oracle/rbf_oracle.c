/* rbf_oracle.c -- plain, slow, obviously correct CPU FP64 reference of Gaussian
 * radial-basis-function interpolation solved by right-preconditioned GMRES with
 * a restricted additive Schwarz (RASM) preconditioner.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg to check and time the GPU library.  It shares no
 * code with it.  Build: gcc -O2 -ffp-contract=off -fopenmp (no FMA contraction:
 * the one fused multiply-add below is written out with fma()).
 *
 * What it computes, step by step, with the passage of the paper it follows:
 *  - The interpolation problem (Section 2.1, eqs. rbf1-rbf2): find lambda with
 *    sum_j lambda_j phi(|x_i - x_j|) = f_i.  The Gaussian is positive definite
 *    on its own, so no polynomial block.
 *  - phi is the normalised 2-D Gaussian of Section 2.3:
 *    A_ij = exp(-|x_i - x_j|^2 / (2 sigma^2)) / (2 pi sigma^2), and the matvec
 *    drops pairs farther apart than a cutoff r_c (Section 2.3: the matrix is
 *    treated as banded, sparse with controllable accuracy).
 *  - Square cells of side r_c form the non-overlapping subdomains; the
 *    overlapping subdomain of a cell is the (2*overlap+1)^2 block of cells
 *    around it (Section 2.2, Fig. 1).
 *  - RASM (Section 2.2, eq. rasm and the preconditioner M^{-1} after it):
 *    z = sum_i Rt_i^T A_i^{-1} R_i v: solve the dense local system on every
 *    overlapping subdomain and keep only the values of its own cell.  The local
 *    matrices are dense and factored directly (Section 2.4: dense sub-matrices,
 *    direct local solves); here by Cholesky, as they are symmetric positive
 *    definite.
 *  - GMRES (Section 2.2, last paragraph; Saad's textbook), restarted, right
 *    preconditioned, modified Gram-Schmidt Arnoldi, Givens rotations for the
 *    small least-squares problem.
 *  - The paper's parametric geometry (Section 3.1, Fig. 3), on request
 *    (orc_set_geometry): non-overlapping subdomains are boxes of side B,
 *    overlapping ones the squares of side D centred on them, and optionally
 *    the matvec of a target keeps only the sources in the square of side T
 *    centred on its box.
 *
 * Readings where the paper does not fix a detail (each applied identically by
 * the GPU library):
 *  - grid origin = the minimum point coordinates, cell side L = r_c exactly,
 *    cell index cx = floor((x - x0) * (1/L)) clamped to [0, ncx-1];
 *  - sorted order = stable sort of the points by cell index;
 *  - a pair is in the cutoff iff fma(dx, dx, dy*dy) <= r_c*r_c, i = j included;
 *  - local matrices use the untruncated Gaussian (always SPD for distinct
 *    points), ordered neighbour cells by (dy, dx) ascending, the centre last;
 *  - stop on the true relative residual ||f - A x|| / ||f|| <= rtol;
 *  - boxes: index floor((x - x0) * (1/B)) clamped, centre x0 + (b + 1/2) B,
 *    a point is in a square of side S around a centre iff |x - c| <= S/2
 *    along both axes; a box's members are its own points and the points of
 *    its D-square, the others first, each part in sorted order.
 */
#include "rbf_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_problem {
    long long n;
    double sigma, cutoff;
    int overlap;
    /* subdomain geometry in lengths (Section 3.1, Fig. 3), geo = 1 once set:
     * boxes of side B on a grid anchored at (x0, y0), overlapping squares of
     * side D, truncation square of side T (T = 0: the radial cutoff) */
    int geo;
    double B, D, T, invB;
    long long nbx, nby;
    /* grid */
    double x0, y0, L, invL;
    long long ncx, ncy, ncells;
    /* binning */
    int* cell_of;          /* n, original order */
    int* perm;             /* n, sorted -> original */
    long long* cell_start; /* ncells + 1 */
    double* xs;            /* n, sorted order */
    double* ys;
    /* RASM factors */
    int rasm_ready;
    long long* blk_off;    /* ncells: offset of the cell's factor in lstore */
    int* blk_n;            /* ncells: members of the overlapping subdomain */
    int* blk_nc;           /* ncells: members of the cell itself */
    double* lstore;        /* sum of blk_n^2 doubles, column-major factors */
};

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---- the kernel phi (Section 2.3) ------------------------------------------ */

static double gauss_norm(double sigma) { return 1.0 / (2.0 * M_PI * sigma * sigma); }

static double phi_of_d2(double d2, double sigma) {
    return exp(-d2 / (2.0 * sigma * sigma)) * gauss_norm(sigma);
}

/* squared distance, rounded as one fused multiply-add on top of dy*dy */
static double dist2(double xa, double ya, double xb, double yb) {
    double dx = xa - xb;
    double dy = ya - yb;
    return fma(dx, dx, dy * dy);
}

/* ---- grid and binning ------------------------------------------------------- */

static long long cell_coord(double v, double v0, double invL, long long nc) {
    double t = floor((v - v0) * invL);
    if (!(t >= 0.0)) t = 0.0;              /* also catches NaN */
    if (t > (double)(nc - 1)) t = (double)(nc - 1);
    return (long long)t;
}

static long long cell_index(const orc_problem* p, double x, double y, long long* cx,
                            long long* cy) {
    *cx = cell_coord(x, p->x0, p->invL, p->ncx);
    *cy = cell_coord(y, p->y0, p->invL, p->ncy);
    return (*cy) * p->ncx + (*cx);
}

int orc_create(const double* points, long long n, double sigma, double cutoff,
               int overlap, orc_problem** out) {
    if (!out) return ORC_EINVAL;
    *out = NULL;
    if (!points || n < 1 || !(sigma > 0.0) || !isfinite(sigma) || !(cutoff > 0.0) ||
        !isfinite(cutoff) || overlap < 0 || n > 2000000000LL)
        return ORC_EINVAL;
    for (long long i = 0; i < 2 * n; ++i)
        if (!isfinite(points[i])) return ORC_EINVAL;

    orc_problem* p = (orc_problem*)calloc(1, sizeof(orc_problem));
    if (!p) return ORC_ENOMEM;
    p->n = n;
    p->sigma = sigma;
    p->cutoff = cutoff;
    p->overlap = overlap;

    double xmin = points[0], xmax = points[0], ymin = points[1], ymax = points[1];
    for (long long i = 1; i < n; ++i) {
        double x = points[2 * i], y = points[2 * i + 1];
        if (x < xmin) xmin = x;
        if (x > xmax) xmax = x;
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    p->x0 = xmin;
    p->y0 = ymin;
    p->L = cutoff;
    p->invL = 1.0 / cutoff;
    double fx = floor((xmax - xmin) * p->invL), fy = floor((ymax - ymin) * p->invL);
    if (!(fx < 1e9) || !(fy < 1e9) || (fx + 1.0) * (fy + 1.0) > 1e9) {
        free(p);
        return ORC_EINVAL;
    }
    p->ncx = (long long)fx + 1;
    p->ncy = (long long)fy + 1;
    p->ncells = p->ncx * p->ncy;

    p->cell_of = (int*)malloc(sizeof(int) * n);
    p->perm = (int*)malloc(sizeof(int) * n);
    p->cell_start = (long long*)calloc(p->ncells + 1, sizeof(long long));
    p->xs = (double*)malloc(sizeof(double) * n);
    p->ys = (double*)malloc(sizeof(double) * n);
    if (!p->cell_of || !p->perm || !p->cell_start || !p->xs || !p->ys) {
        orc_destroy(p);
        return ORC_ENOMEM;
    }
    /* stable counting sort by cell index */
    for (long long i = 0; i < n; ++i) {
        long long cx, cy;
        long long c = cell_index(p, points[2 * i], points[2 * i + 1], &cx, &cy);
        p->cell_of[i] = (int)c;
        p->cell_start[c + 1] += 1;
    }
    for (long long c = 0; c < p->ncells; ++c) p->cell_start[c + 1] += p->cell_start[c];
    long long* fill = (long long*)malloc(sizeof(long long) * p->ncells);
    if (!fill) {
        orc_destroy(p);
        return ORC_ENOMEM;
    }
    memcpy(fill, p->cell_start, sizeof(long long) * p->ncells);
    for (long long i = 0; i < n; ++i) {
        long long s = fill[p->cell_of[i]]++;
        p->perm[s] = (int)i;
        p->xs[s] = points[2 * i];
        p->ys[s] = points[2 * i + 1];
    }
    free(fill);

    /* distinct nodes are needed for a positive-definite Gaussian matrix
     * (Section 2.1); identical points always share a cell */
    int dup = 0;
    for (long long c = 0; c < p->ncells && !dup; ++c)
        for (long long a = p->cell_start[c]; a < p->cell_start[c + 1] && !dup; ++a)
            for (long long b = a + 1; b < p->cell_start[c + 1]; ++b)
                if (p->xs[a] == p->xs[b] && p->ys[a] == p->ys[b]) {
                    dup = 1;
                    break;
                }
    if (dup) {
        orc_destroy(p);
        return ORC_EDUPLICATE;
    }
    *out = p;
    return ORC_OK;
}

void orc_destroy(orc_problem* p) {
    if (!p) return;
    free(p->cell_of);
    free(p->perm);
    free(p->cell_start);
    free(p->xs);
    free(p->ys);
    free(p->blk_off);
    free(p->blk_n);
    free(p->blk_nc);
    free(p->lstore);
    free(p);
}

int orc_grid(const orc_problem* p, double* out4, long long* ncxy) {
    if (!p || !out4 || !ncxy) return ORC_EINVAL;
    out4[0] = p->x0;
    out4[1] = p->y0;
    out4[2] = p->L;
    out4[3] = p->invL;
    ncxy[0] = p->ncx;
    ncxy[1] = p->ncy;
    return ORC_OK;
}

int orc_binning(const orc_problem* p, int* cell_of, int* perm, long long* cell_start) {
    if (!p) return ORC_EINVAL;
    if (cell_of) memcpy(cell_of, p->cell_of, sizeof(int) * p->n);
    if (perm) memcpy(perm, p->perm, sizeof(int) * p->n);
    if (cell_start) memcpy(cell_start, p->cell_start, sizeof(long long) * (p->ncells + 1));
    return ORC_OK;
}

/* ---- truncated matvec (Section 2.3) ------------------------------------------ */

/* ---- subdomain boxes (Section 3.1, Fig. 3) ---------------------------------- */

/* box of a point: the cell rule with side B, clamped to the box grid */
static long long box_index(const orc_problem* p, double x, double y, long long* bx, long long* by) {
    *bx = cell_coord(x, p->x0, p->invB, p->nbx);
    *by = cell_coord(y, p->y0, p->invB, p->nby);
    return (*by) * p->nbx + (*bx);
}

/* centre of box (bx, by) */
static void box_centre(const orc_problem* p, long long bx, long long by, double* cx, double* cy) {
    *cx = p->x0 + ((double)bx + 0.5) * p->B;
    *cy = p->y0 + ((double)by + 0.5) * p->B;
}

/* the cells that hold every point of the square [cx - h, cx + h] x [cy - h, cy + h]:
 * the cells of its corners, widened by one (rounding at the edges), clamped */
static void cells_of_square(const orc_problem* p, double cx, double cy, double h, long long* xa,
                            long long* xb, long long* ya, long long* yb) {
    *xa = cell_coord(cx - h, p->x0, p->invL, p->ncx) - 1;
    *xb = cell_coord(cx + h, p->x0, p->invL, p->ncx) + 1;
    *ya = cell_coord(cy - h, p->y0, p->invL, p->ncy) - 1;
    *yb = cell_coord(cy + h, p->y0, p->invL, p->ncy) + 1;
    if (*xa < 0) *xa = 0;
    if (*ya < 0) *ya = 0;
    if (*xb > p->ncx - 1) *xb = p->ncx - 1;
    if (*yb > p->ncy - 1) *yb = p->ncy - 1;
}

/* box truncation of the matvec (Section 3.1): the sources in the square of
 * side T centred on the target's box, in cell order then sorted order */
static double box_sum(const orc_problem* p, double x, double y, const double* wsorted, int* count) {
    long long bx, by, xa, xb, ya, yb;
    double cx, cy;
    box_index(p, x, y, &bx, &by);
    box_centre(p, bx, by, &cx, &cy);
    const double h = 0.5 * p->T;
    cells_of_square(p, cx, cy, h, &xa, &xb, &ya, &yb);
    double s = 0.0;
    int cnt = 0;
    for (long long ny = ya; ny <= yb; ++ny)
        for (long long nx = xa; nx <= xb; ++nx) {
            long long c = ny * p->ncx + nx;
            for (long long j = p->cell_start[c]; j < p->cell_start[c + 1]; ++j)
                if (fabs(p->xs[j] - cx) <= h && fabs(p->ys[j] - cy) <= h) {
                    s += wsorted[j] * phi_of_d2(dist2(x, y, p->xs[j], p->ys[j]), p->sigma);
                    ++cnt;
                }
        }
    if (count) *count = cnt;
    return s;
}

/* sum over the sources of the 3x3 block of cells around (cx, cy), in (dy, dx)
 * order then sorted order, of wsorted_j * phi for pairs within the cutoff
 * (or, with a truncation square T set, over the sources in that square). */
static double cell_sum(const orc_problem* p, double x, double y, long long cx, long long cy,
                       const double* wsorted, int* count) {
    if (p->geo && p->T > 0.0) return box_sum(p, x, y, wsorted, count);
    double rc2 = p->cutoff * p->cutoff;
    double s = 0.0;
    int cnt = 0;
    for (long long dy = -1; dy <= 1; ++dy) {
        long long ny = cy + dy;
        if (ny < 0 || ny >= p->ncy) continue;
        for (long long dx = -1; dx <= 1; ++dx) {
            long long nx = cx + dx;
            if (nx < 0 || nx >= p->ncx) continue;
            long long c = ny * p->ncx + nx;
            for (long long j = p->cell_start[c]; j < p->cell_start[c + 1]; ++j) {
                double d2 = dist2(x, y, p->xs[j], p->ys[j]);
                if (d2 <= rc2) {
                    s += wsorted[j] * phi_of_d2(d2, p->sigma);
                    ++cnt;
                }
            }
        }
    }
    if (count) *count = cnt;
    return s;
}

int orc_matvec(const orc_problem* p, const double* w, double* y, int* nnb) {
    if (!p || !w || !y) return ORC_EINVAL;
    long long n = p->n;
    double* ws = (double*)malloc(sizeof(double) * n);
    if (!ws) return ORC_ENOMEM;
    for (long long s = 0; s < n; ++s) ws[s] = w[p->perm[s]];
#pragma omp parallel for schedule(dynamic, 256)
    for (long long s = 0; s < n; ++s) {
        long long cx, cy;
        cell_index(p, p->xs[s], p->ys[s], &cx, &cy);
        int cnt;
        double v = cell_sum(p, p->xs[s], p->ys[s], cx, cy, ws, &cnt);
        y[p->perm[s]] = v;
        if (nnb) nnb[p->perm[s]] = cnt;
    }
    free(ws);
    return ORC_OK;
}

int orc_evaluate(const orc_problem* p, const double* lambda, const double* targets,
                 long long m, double* out) {
    return orc_evaluate_counts(p, lambda, targets, m, out, NULL);
}

int orc_evaluate_counts(const orc_problem* p, const double* lambda, const double* targets,
                        long long m, double* out, int* nnb) {
    if (!p || !lambda || (m > 0 && (!targets || !out)) || m < 0) return ORC_EINVAL;
    for (long long t = 0; t < 2 * m; ++t)
        if (!isfinite(targets[t])) return ORC_EINVAL;
    long long n = p->n;
    double* ws = (double*)malloc(sizeof(double) * n);
    if (!ws) return ORC_ENOMEM;
    for (long long s = 0; s < n; ++s) ws[s] = lambda[p->perm[s]];
#pragma omp parallel for schedule(dynamic, 256)
    for (long long t = 0; t < m; ++t) {
        long long cx, cy;
        double x = targets[2 * t], y = targets[2 * t + 1];
        cell_index(p, x, y, &cx, &cy);
        int cnt;
        out[t] = cell_sum(p, x, y, cx, cy, ws, &cnt);
        if (nnb) nnb[t] = cnt;
    }
    free(ws);
    return ORC_OK;
}

/* ---- RASM (Section 2.2, eq. rasm) ------------------------------------------- */

/* members of the overlapping subdomain of box b (geometry set): the points
 * of the square of side D centred on the box, in sorted order, with the box's
 * own points moved last (still in sorted order). */
static int box_members(const orc_problem* p, long long b, long long* sorted_idx, int* ncentre) {
    long long bx = b % p->nbx, by = b / p->nbx, xa, xb, ya, yb, ox, oy;
    double cx, cy;
    box_centre(p, bx, by, &cx, &cy);
    const double h = 0.5 * p->D;
    cells_of_square(p, cx, cy, h, &xa, &xb, &ya, &yb);
    int k = 0, kc = 0;
    for (int own = 0; own <= 1; ++own)
        for (long long ny = ya; ny <= yb; ++ny)
            for (long long nx = xa; nx <= xb; ++nx) {
                long long c = ny * p->ncx + nx;
                for (long long j = p->cell_start[c]; j < p->cell_start[c + 1]; ++j) {
                    const int mine = box_index(p, p->xs[j], p->ys[j], &ox, &oy) == b;
                    const int inside = fabs(p->xs[j] - cx) <= h && fabs(p->ys[j] - cy) <= h;
                    if (own ? mine : (inside && !mine)) {
                        if (sorted_idx) sorted_idx[k] = j;
                        ++k;
                        kc += own;
                    }
                }
            }
    if (ncentre) *ncentre = kc;
    return k;
}

/* members of the overlapping subdomain of cell c, as sorted-order indices:
 * neighbour cells in (dy, dx) ascending order, then the cell itself. */
static int block_members(const orc_problem* p, long long c, long long* sorted_idx,
                         int* ncentre) {
    if (p->geo) return box_members(p, c, sorted_idx, ncentre);
    long long cx = c % p->ncx, cy = c / p->ncx;
    int ov = p->overlap, k = 0;
    for (long long dy = -ov; dy <= ov; ++dy) {
        long long ny = cy + dy;
        if (ny < 0 || ny >= p->ncy) continue;
        for (long long dx = -ov; dx <= ov; ++dx) {
            long long nx = cx + dx;
            if (nx < 0 || nx >= p->ncx || (dx == 0 && dy == 0)) continue;
            long long nc = ny * p->ncx + nx;
            for (long long j = p->cell_start[nc]; j < p->cell_start[nc + 1]; ++j) {
                if (sorted_idx) sorted_idx[k] = j;
                ++k;
            }
        }
    }
    int kc = 0;
    for (long long j = p->cell_start[c]; j < p->cell_start[c + 1]; ++j) {
        if (sorted_idx) sorted_idx[k] = j;
        ++k;
        ++kc;
    }
    if (ncentre) *ncentre = kc;
    return k;
}

/* textbook right-looking Cholesky of the n x n column-major matrix a (lower
 * part), in place; returns 0, or k+1 if the k-th pivot is not positive. */
static int cholesky_lower(double* a, int n) {
    for (int k = 0; k < n; ++k) {
        double piv = a[(long long)k * n + k];
        if (!(piv > 0.0)) return k + 1;
        double lkk = sqrt(piv);
        a[(long long)k * n + k] = lkk;
        for (int i = k + 1; i < n; ++i) a[(long long)k * n + i] /= lkk;
        for (int j = k + 1; j < n; ++j) {
            double ljk = a[(long long)k * n + j];
            for (int i = j; i < n; ++i) a[(long long)j * n + i] -= a[(long long)k * n + i] * ljk;
        }
    }
    for (int j = 1; j < n; ++j)
        for (int i = 0; i < j; ++i) a[(long long)j * n + i] = 0.0;
    return 0;
}

/* number of subdomains: boxes once a geometry is set, else cells */
static long long n_subdomains(const orc_problem* p) { return p->geo ? p->nbx * p->nby : p->ncells; }

int orc_rasm_setup(orc_problem* p) {
    if (!p) return ORC_EINVAL;
    if (p->rasm_ready) return ORC_OK;
    long long nc = n_subdomains(p);
    p->blk_off = (long long*)malloc(sizeof(long long) * nc);
    p->blk_n = (int*)malloc(sizeof(int) * nc);
    p->blk_nc = (int*)malloc(sizeof(int) * nc);
    if (!p->blk_off || !p->blk_n || !p->blk_nc) return ORC_ENOMEM;
    long long tot = 0;
    for (long long c = 0; c < nc; ++c) {
        int kc;
        int k = block_members(p, c, NULL, &kc);
        p->blk_n[c] = k;
        p->blk_nc[c] = kc;
        p->blk_off[c] = tot;
        if (kc > 0) tot += (long long)k * k;   /* empty cells own no unknowns */
    }
    p->lstore = (double*)malloc(sizeof(double) * (tot > 0 ? tot : 1));
    if (!p->lstore) return ORC_ENOMEM;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (long long c = 0; c < nc; ++c) {
        int k = p->blk_n[c];
        if (p->blk_nc[c] == 0) continue;
        long long* mem = (long long*)malloc(sizeof(long long) * k);
        if (!mem) {
            bad |= 2;
            continue;
        }
        block_members(p, c, mem, NULL);
        double* a = p->lstore + p->blk_off[c];
        /* untruncated Gaussian on the subdomain's points */
        for (int q = 0; q < k; ++q)
            for (int r = 0; r < k; ++r)
                a[(long long)q * k + r] = phi_of_d2(
                    dist2(p->xs[mem[r]], p->ys[mem[r]], p->xs[mem[q]], p->ys[mem[q]]),
                    p->sigma);
        if (cholesky_lower(a, k)) bad |= 1;
        free(mem);
    }
    if (bad & 2) return ORC_ENOMEM;
    if (bad & 1) return ORC_ENOTPD;
    p->rasm_ready = 1;
    return ORC_OK;
}

int orc_rasm_apply(const orc_problem* p, const double* v, double* z) {
    if (!p || !v || !z) return ORC_EINVAL;
    if (!p->rasm_ready) return ORC_ESTATE;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (long long c = 0; c < n_subdomains(p); ++c) {
        int k = p->blk_n[c], kc = p->blk_nc[c];
        if (kc == 0) continue;
        long long* mem = (long long*)malloc(sizeof(long long) * k);
        double* t = (double*)malloc(sizeof(double) * k);
        if (!mem || !t) {
            free(mem);
            free(t);
            err = 1;
            continue;
        }
        block_members(p, c, mem, NULL);
        for (int r = 0; r < k; ++r) t[r] = v[p->perm[mem[r]]];   /* R_i v */
        const double* l = p->lstore + p->blk_off[c];
        /* forward substitution L t' = t */
        for (int j = 0; j < k; ++j) {
            t[j] /= l[(long long)j * k + j];
            for (int i = j + 1; i < k; ++i) t[i] -= l[(long long)j * k + i] * t[j];
        }
        /* back substitution L^T x = t' on the trailing (centre) block only:
         * the centre rows of the solution depend on nothing else */
        int c0 = k - kc;
        for (int i = k - 1; i >= c0; --i) {
            double s = t[i];
            for (int j = i + 1; j < k; ++j) s -= l[(long long)i * k + j] * t[j];
            t[i] = s / l[(long long)i * k + i];
        }
        /* restricted prolongation: only the cell's own values are kept */
        for (int i = c0; i < k; ++i) z[p->perm[mem[i]]] = t[i];
        free(mem);
        free(t);
    }
    return err ? ORC_ENOMEM : ORC_OK;
}

int orc_rasm_block_size(const orc_problem* p, long long c, int* nomega, int* ncentre) {
    if (!p || c < 0 || c >= n_subdomains(p)) return ORC_EINVAL;
    int kc;
    int k = block_members(p, c, NULL, &kc);
    if (nomega) *nomega = k;
    if (ncentre) *ncentre = kc;
    return ORC_OK;
}

int orc_rasm_block(const orc_problem* p, long long c, long long* members, int* nomega,
                   int* ncentre, double* L) {
    if (!p || c < 0 || c >= n_subdomains(p)) return ORC_EINVAL;
    int kc;
    int k = block_members(p, c, NULL, &kc);
    if (nomega) *nomega = k;
    if (ncentre) *ncentre = kc;
    if (members) {
        long long* mem = (long long*)malloc(sizeof(long long) * (k > 0 ? k : 1));
        if (!mem) return ORC_ENOMEM;
        block_members(p, c, mem, NULL);
        for (int r = 0; r < k; ++r) members[r] = p->perm[mem[r]];
        free(mem);
    }
    if (L) {
        if (!p->rasm_ready || kc == 0) return ORC_ESTATE;
        memcpy(L, p->lstore + p->blk_off[c], sizeof(double) * (long long)k * k);
    }
    return ORC_OK;
}

static void drop_factors(orc_problem* p) {
    free(p->blk_off);
    free(p->blk_n);
    free(p->blk_nc);
    free(p->lstore);
    p->blk_off = NULL;
    p->blk_n = NULL;
    p->blk_nc = NULL;
    p->lstore = NULL;
    p->rasm_ready = 0;
}

int orc_set_geometry(orc_problem* p, double B, double D, double T) {
    if (!p || !(B > 0.0) || !isfinite(B) || !(D >= B) || !isfinite(D) || !(T >= 0.0) ||
        !isfinite(T) || (T > 0.0 && T < B))
        return ORC_EINVAL;
    double xmax = p->xs[0], ymax = p->ys[0];
    for (long long i = 1; i < p->n; ++i) {
        if (p->xs[i] > xmax) xmax = p->xs[i];
        if (p->ys[i] > ymax) ymax = p->ys[i];
    }
    const double invB = 1.0 / B;
    const double fx = floor((xmax - p->x0) * invB), fy = floor((ymax - p->y0) * invB);
    if (!(fx < 1e9) || !(fy < 1e9) || (fx + 1.0) * (fy + 1.0) > 1e9) return ORC_EINVAL;
    drop_factors(p);
    p->geo = 1;
    p->B = B;
    p->D = D;
    p->T = T;
    p->invB = invB;
    p->nbx = (long long)fx + 1;
    p->nby = (long long)fy + 1;
    return ORC_OK;
}

int orc_subdomains(const orc_problem* p, long long* nxy) {
    if (!p || !nxy) return ORC_EINVAL;
    nxy[0] = p->geo ? p->nbx : p->ncx;
    nxy[1] = p->geo ? p->nby : p->ncy;
    return ORC_OK;
}

/* ---- GMRES (Section 2.2; Saad) ---------------------------------------------- */

static double dot(const double* a, const double* b, long long n) {
    double s = 0.0;
    for (long long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

int orc_rel_residual(const orc_problem* p, const double* f, const double* x, double* out) {
    if (!p || !f || !x || !out) return ORC_EINVAL;
    long long n = p->n;
    double* r = (double*)malloc(sizeof(double) * n);
    if (!r) return ORC_ENOMEM;
    int rc = orc_matvec(p, x, r, NULL);
    if (rc) {
        free(r);
        return rc;
    }
    for (long long i = 0; i < n; ++i) r[i] = f[i] - r[i];
    double fn = sqrt(dot(f, f, n));
    double rn = sqrt(dot(r, r, n));
    *out = fn > 0.0 ? rn / fn : rn;
    free(r);
    return ORC_OK;
}

int orc_gmres(orc_problem* p, const double* f, int restart, double rtol, int max_iters,
              const double* x0, double* x, orc_info* info, double* history,
              int history_cap) {
    if (!p || !f || !x || restart < 1 || !(rtol >= 0.0) || max_iters < 0) return ORC_EINVAL;
    int rc = orc_rasm_setup(p);
    if (rc) return rc;
    long long n = p->n;
    int m = restart;
    double* V = (double*)malloc(sizeof(double) * (size_t)n * (m + 1));
    double* w = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* g = (double*)malloc(sizeof(double) * (m + 1));
    double* yv = (double*)malloc(sizeof(double) * m);
    if (!V || !w || !z || !H || !cs || !sn || !g || !yv) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (long long i = 0; i < n; ++i) x[i] = x0 ? x0[i] : 0.0;
    double fnorm = sqrt(dot(f, f, n));
    int iters = 0, cycles = 0, hl = 0;
    double rel = 0.0;
    if (fnorm == 0.0) {
        for (long long i = 0; i < n; ++i) x[i] = 0.0;
        rc = ORC_OK;
        goto report;
    }
    for (;;) {
        /* true residual r = f - A x */
        rc = orc_matvec(p, x, w, NULL);
        if (rc) goto done;
        for (long long i = 0; i < n; ++i) w[i] = f[i] - w[i];
        double beta = sqrt(dot(w, w, n));
        rel = beta / fnorm;
        if (history && hl < history_cap) history[hl++] = rel;
        if (!isfinite(rel)) {
            rc = ORC_ENAN;
            goto report;
        }
        if (rel <= rtol) {
            rc = ORC_OK;
            goto report;
        }
        if (iters >= max_iters) {
            rc = ORC_ENOCONV;
            goto report;
        }
        for (long long i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0, breakdown = 0;
        for (int j = 0; j < m; ++j) {
            double* vj = V + (size_t)j * n;
            rc = orc_rasm_apply(p, vj, z);          /* z = M^{-1} v_j */
            if (rc) goto done;
            rc = orc_matvec(p, z, w, NULL);         /* w = A z */
            if (rc) goto done;
            for (int i = 0; i <= j; ++i) {          /* modified Gram-Schmidt */
                double* vi = V + (size_t)i * n;
                double hij = dot(w, vi, n);
                H[i * m + j] = hij;
                for (long long t = 0; t < n; ++t) w[t] -= hij * vi[t];
            }
            double hn = sqrt(dot(w, w, n));
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {           /* earlier rotations */
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double rho = hypot(a, b);
            if (!isfinite(rho)) {
                rc = ORC_ENAN;
                goto report;
            }
            cs[j] = rho > 0.0 ? a / rho : 1.0;
            sn[j] = rho > 0.0 ? b / rho : 0.0;
            H[j * m + j] = rho;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            k = j + 1;
            if (hn == 0.0) {
                breakdown = 1;
                break;
            }
            if (fabs(g[j + 1]) <= rtol * fnorm || iters >= max_iters) break;
            double* vn = V + (size_t)(j + 1) * n;
            for (long long t = 0; t < n; ++t) vn[t] = w[t] / hn;
        }
        /* y = H^{-1} g (upper triangular k x k) */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * yv[j];
            yv[i] = s / H[i * m + i];
        }
        /* x += M^{-1} (V y) */
        for (long long t = 0; t < n; ++t) w[t] = 0.0;
        for (int i = 0; i < k; ++i) {
            const double* vi = V + (size_t)i * n;
            for (long long t = 0; t < n; ++t) w[t] += yv[i] * vi[t];
        }
        rc = orc_rasm_apply(p, w, z);
        if (rc) goto done;
        for (long long t = 0; t < n; ++t) x[t] += z[t];
        ++cycles;
        if (breakdown) {
            rc = orc_rel_residual(p, f, x, &rel);
            if (rc) goto done;
            if (history && hl < history_cap) history[hl++] = rel;
            rc = rel <= rtol ? ORC_OK : ORC_EBREAKDOWN;
            goto report;
        }
    }
report:
    if (info) {
        info->iterations = iters;
        info->restarts = cycles;
        info->rel_residual = rel;
        info->history_len = hl;
    }
done:
    free(V);
    free(w);
    free(z);
    free(H);
    free(cs);
    free(sn);
    free(g);
    free(yv);
    return rc;
}
