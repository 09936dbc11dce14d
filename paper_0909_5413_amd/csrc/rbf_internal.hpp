// rbf_internal.hpp -- launchers shared between the gfx950 kernels and the host
// driver.  Every launcher enqueues on `st` and returns hipSuccess or the launch
// error; none synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

struct rbf_problem;
#include "../../include/rbf.h"

namespace rbf {

struct Grid {
    double x0, y0, L, invL;
    int ncx, ncy;
    long long ncells() const { return (long long)ncx * ncy; }
};

// ---- binning (binning.hip) --------------------------------------------------
// Reduce min/max of x and y over n interleaved points and flag non-finite
// points or values.  out4 = {xmin, ymin, xmax, ymax}; bad = 1 if any NaN/Inf.
// work must hold 4 * kReduceBlocks doubles.
constexpr int kReduceBlocks = 512;
hipError_t launch_minmax(const double* pts, const double* vals, long long n, double* work,
                         double* out4, int* bad, hipStream_t st);
// cell_of[i], slot[i] = arrival rank within the cell, counts[c] += 1.
hipError_t launch_cell_count(const double* pts, long long n, Grid g, int* cell_of,
                             int* slot, int* counts, hipStream_t st);
// Exclusive scan of n ints into out (n + 1 entries, out[n] = total).
// work must hold scan_work_ints(n) ints.
long long scan_work_ints(long long n);
hipError_t launch_exclusive_scan(const int* in, int* out, long long n, int* work,
                                 hipStream_t st);
// tmp[cell_start[cell_of[i]] + slot[i]] = i
hipError_t launch_scatter(const int* cell_of, const int* slot, const int* cell_start,
                          long long n, int* tmp, hipStream_t st);
// perm[cell range] = tmp[cell range] sorted ascending, for every cell.
// Also counts cells with more than max_pts points into *overflow.
hipError_t launch_sort_cells(const int* tmp, const int* cell_start, long long ncells,
                             int* perm, int max_pts, int* overflow, hipStream_t st);
// Gather sorted coordinates / values and the FP32 cell-centre-relative scaled
// coordinates (scale sc) used by the FP32 kernels.
hipError_t launch_gather(const double* pts, const double* vals, const int* perm,
                         const int* cell_of, long long n, Grid g, double sc, double* xs,
                         double* ys, double* fs, float* xr, float* yr, hipStream_t st);
// Flag bit-identical points within a cell.
hipError_t launch_dup_check(const double* xs, const double* ys, const int* cell_start,
                            long long ncells, int* dup, hipStream_t st);
// dst[perm[s]] = src[s] (to original order) or dst[s] = src[perm[s]] (to sorted).
hipError_t launch_unpermute(const double* src, const int* perm, long long n, double* dst,
                            hipStream_t st);
hipError_t launch_permute(const double* src, const int* perm, long long n, double* dst,
                          hipStream_t st);
hipError_t launch_unpermute_int(const int* src, const int* perm, long long n, int* dst,
                                hipStream_t st);

// ---- matvec (matvec.hip) ----------------------------------------------------
struct MatvecArgs {
    const double* sx;       // sources, sorted order
    const double* sy;
    const int* scell;       // source cell_start, ncells + 1
    const double* tx;       // targets, target-sorted order
    const double* ty;
    const int* tcell;       // target cell_start
    Grid g;
    double rc2;             // cutoff^2
    double mk;              // -1 / (2 sigma^2)
    double beta;            // -32 / (2 sigma^2 ln2): exp(mk d2) = 2^(beta d2 / 32)
    double norm;            // 1 / (2 pi sigma^2)
    const double* etab;     // e^{-n/128}, n < ntab, or NULL (no table)
    int ntab;
    const double* t32;      // 2^(j/32), j < 32
};
// entries of the exponential table held in LDS (covers cutoffs up to ~6.3 sigma)
constexpr int kExpTableMax = 2560;
// y[t] = norm * sum_{s in 3x3 cells, d2 <= rc2} w[s] exp(mk d2); nnb may be NULL.
hipError_t launch_matvec64(const MatvecArgs& a, const double* w, double* y, int* nnb,
                           hipStream_t st);
// FP32 form: coordinates are the FP32 cell-centre-relative scaled ones, with the
// exponent folded in (e = 2^-(d_s^2)); weights read as FP64 and rounded; Kahan
// FP32 accumulation; FP64 output.
struct Matvec32Args {
    const float* sx;
    const float* sy;
    const int* scell;
    Grid g;
    float Ls;               // cell side in scaled units
    float rc2s;             // cutoff^2 in scaled units
    double norm;
};
// w32: n floats of workspace (the weights rounded to FP32)
hipError_t launch_matvec32(const Matvec32Args& a, const double* w, float* w32, double* y,
                           long long n, hipStream_t st);

// ---- neighbour lists (matvec.hip) --------------------------------------------
// A group is a run of consecutive cells cxa..cxb of one cell row cy together
// with a range [t0, t1) of their targets (all of them unless one cell alone is
// split over several groups); one workgroup serves it.  The group stages once
// the sources of the rows dy = -1, 0, 1 around its cells, each row the
// contiguous sorted range from the column left of cxa to the column right of
// cxb, concatenated in that order (n_span sources).  Its targets are cut into
// units of 64 consecutive targets, one per wave (lane = target).  A unit's
// list holds, per lane, the target's in-cutoff sources (those of its own 3x3
// block with d2 <= rc2) in local order (rows, then sorted order) as 16 * their
// index in the staging, padded to the unit's longest list (a multiple of 4)
// with 16 * n_span, a null source; entry k of lane l sits at
// off[u] + 256 (k / 4) + 4 l + k % 4, so one 8-byte load fetches four entries.
struct ListGroup {
    int u0, nu;                // first unit, units
    int cy, cxa, cxb;          // cell row and columns
    int t0, t1;                // targets (sorted order)
    int pad;
};
struct NeighborLists {
    const ListGroup* group;
    const long long* off;      // per unit, entries
    const int* len;            // per unit, padded list length
    const unsigned short* idx;
    int nunits, ngroups;
    int gunits;                // most units in one group (waves per workgroup)
    int max_nb;                // largest n_span over the groups
};
// Sources one 3x3 block may hold for the lists to be built (16-bit entries of
// 16 * index, LDS), the staged sources and cell columns a group grows to, and
// the units (waves) of one group.
constexpr int kListMaxNb = 2047;
constexpr int kGroupSpan = 2047;
constexpr int kGroupCells = 8;
constexpr int kGroupMaxUnits = 8;
// len[u] = the unit's padded list length (max in-cutoff count over its lanes,
// rounded up to 4); nb[u] = its group's n_span.
hipError_t launch_list_count(const MatvecArgs& a, const NeighborLists& nl, int* len,
                             hipStream_t st);
hipError_t launch_list_fill(const MatvecArgs& a, const NeighborLists& nl, unsigned short* idx,
                            hipStream_t st);
// The same products as launch_matvec64 / launch_matvec32 (targets = sources),
// driven by the lists: every evaluated pair is an interaction.
hipError_t launch_matvec64_lists(const MatvecArgs& a, const NeighborLists& nl, const double* w,
                                 double* y, hipStream_t st);
hipError_t launch_matvec32_lists(const Matvec32Args& a, const NeighborLists& nl, const double* w,
                                 double* y, hipStream_t st);

// ---- preconditioner (precond.hip) --------------------------------------------
struct PrecondArgs {
    const double* xs;       // sorted coordinates
    const double* ys;
    const int* cell_start;
    Grid g;
    int overlap;
    double mk, norm;        // Gaussian: norm * exp(mk d2)
    const long long* zoff;  // per cell offset of Z_c (elements)
    int np_max;             // padded block size bound (multiple of 64)
    int nc_max;             // largest number of points in one cell
    long long ncells;
    double2* xy;            // setup only: per batch slot, np_max member coordinates
                            // (padded order; the padding rows unused)
    // Subdomain boxes (NULL: the subdomains are the cells with `overlap`
    // layers): members of subdomain c are mem[moff[c] .. moff[c + 1]) (sorted-
    // order indices), the last nown[c] of them its own points.
    const int* mem;
    const long long* moff;
    const int* nown;
};
// Subdomain boxes in lengths (Section 3.1, Fig. 3): boxes of side B on the grid
// anchored at (x0, y0), box index by the cell rule with 1/B, the overlapping
// subdomain of a box its own points and every point within half of D of its
// centre along both axes.
struct BoxGeometry {
    double x0, y0, B, invB, halfD;
    int nbx, nby;
};
// Members of every box, in sorted order with the box's own points moved last:
// counts (n_omega[b], n_own[b]) with mem == NULL, else the indices at
// mem[moff[b] ..].  One wave per box.
hipError_t launch_box_members(const PrecondArgs& a, const BoxGeometry& bg, int* n_omega,
                              int* n_own, const long long* moff, int* mem, hipStream_t st);
// Build Z_c (centre rows of the inverse of the local matrix) for all cells, in
// batches of nslots cells.  a.xy holds 8 * ceil(nslots / 8) * np_max entries,
// scratch nslots * slot_elems64(np_max) elements, meta and lvl 8 * ceil(nslots / 8) entries, lt 2 * 2048 * 8 *
// ceil(nslots / 8) elements.  status[c]: 0 ok, -k after the k-th diagonal
// shift level (FP32 only), > 0 the failing pivot (1-based).
__host__ __device__ inline long long slot_elems64(int np_max) {
    const long long b = np_max / 32;
    return 512LL * b * (b + 1);
}
// Optional event timing of the setup launches: (kind, start, stop) per launch,
// kinds as rbf_setup_kernel; the caller reads and destroys the events after
// the stream has finished.
struct SetupProfile {
    struct Rec {
        int kind;
        hipEvent_t start, stop;
    };
    std::vector<Rec> recs;
};
// One lane of the batched setup: a stream and the per-slot buffers of one
// batch in flight (factor scratch, member coordinates, slot records, shift
// levels, the two ping-pong diagonal-block buffers).  Batches go to the lanes
// in turn; with two lanes, two batches advance together on two streams.
template <typename T>
struct SetupLane {
    hipStream_t st;
    T* scratch;
    double2* xy;
    int4* meta;
    T* lt;
    int* lvl;
};
hipError_t launch_precond_setup64(const PrecondArgs& a, double* Z, int nslots,
                                  const SetupLane<double>* lanes, int nlanes, int* status,
                                  hipStream_t st, SetupProfile* prof);
hipError_t launch_precond_setup32(const PrecondArgs& a, float* Z, int nslots,
                                  const SetupLane<float>* lanes, int nlanes, int* status,
                                  hipStream_t st, SetupProfile* prof);
// z[own points of c] = Z_c v[members of c], every cell.
hipError_t launch_rasm_apply64(const PrecondArgs& a, const double* Z, const double* v,
                               double* z, hipStream_t st);
hipError_t launch_rasm_apply32(const PrecondArgs& a, const float* Z, const double* v,
                               double* z, hipStream_t st);
// FP32-stored Z applied to FP64 v with FP64 sums (the FP64 method with FP32
// local inverses)
hipError_t launch_rasm_apply32x64(const PrecondArgs& a, const float* Z, const double* v,
                                  double* z, hipStream_t st);

// ---- box truncation of the product (boxtrunc.hip) ---------------------------
// With subdomain boxes (Section 3.1), a target keeps the sources inside the
// square of side T centred on its own box.  The points of box b's square are
// src[soff[b] .. soff[b + 1]) (sorted-order indices, ascending); its targets
// are its own points, the last nown[b] entries of mem[moff[b] .. moff[b + 1]).
struct BoxTrunc {
    BoxGeometry bg;
    double halfT;
    double d2max;           // d2 cap: keeps the exponential's argument above -690
    long long nbox;
    const int* src;
    const long long* soff;
    const int* mem;
    const long long* moff;
    const int* nown;
};
// nsrc[b] for every box (src == NULL), else the lists at src[soff[b] ..].
hipError_t launch_box_square(const MatvecArgs& a, const BoxTrunc& bt, int* nsrc, int* src,
                             hipStream_t st);
// y[t] = norm * sum over the square of t's box of w[s] exp(mk d2), every point
// t (sorted order); one workgroup per box.
hipError_t launch_matvec64_box(const MatvecArgs& a, const BoxTrunc& bt, const double* w,
                               double* y, hipStream_t st);
// The same sum at m targets (tx, ty) of any position (the box by the clamped
// box rule); nnb[i] = the size of that square, when nnb is not NULL.
hipError_t launch_evaluate_box(const MatvecArgs& a, const BoxTrunc& bt, const double* tx,
                               const double* ty, long long m, const double* w, double* y,
                               int* nnb, hipStream_t st);

// ---- evaluation on a regular lattice of targets (lattice.hip) ---------------
// Targets (x0 + a hx, y0 + b hy), a < nx, b < ny, output at b nx + a.  Along
// each axis the lattice indices are grouped by the cell the cell rule gives
// their coordinate (a contiguous run, the rule being monotone) and cut into
// chunks of at most kLatticeChunk; one wave serves each (column chunk, row
// chunk) pair, workgroup i + ncol j for column chunk i and row chunk j.
constexpr int kLatticeChunk = 8;
struct LatticeChunk {
    long long t0;            // first lattice index
    int c;                   // the cell column (row) of all of them
    int nt;                  // indices in the chunk, 1 .. kLatticeChunk
};
struct LatticeArgs {
    double x0, y0, hx, hy;
    long long nx;
    const LatticeChunk* col;
    const LatticeChunk* row;
    int ncol, nrow;
};
// out[b nx + a] = norm * sum over the target's 3x3 block of w[s] exp(mk d2),
// d2 <= rc2 (the cell-binned product at lattice targets)
hipError_t launch_evaluate_lattice(const MatvecArgs& a, const LatticeArgs& L, const double* w,
                                   double* out, hipStream_t st);
// the lattice's coordinates, target b nx + a at tx[b nx + a], ty[b nx + a]
hipError_t launch_lattice_points(const LatticeArgs& L, long long ny, double* tx, double* ty,
                                 hipStream_t st);

// Batches of a handle's local factorisations in flight together (1 or 2; 2 by
// default).  The serving loop keeps its requests to one: they already overlap
// one another on the device, and its admission counts one batch of scratch.
void set_setup_lanes(rbf_problem* p, int lanes);

// ---- errors (capi.cpp) ---------------------------------------------------------
// Sets the calling thread's rbf_last_error message and returns s.
rbf_status set_error(rbf_status s, const char* fmt, ...);

// ---- device block cache (capi.cpp) -------------------------------------------
// Allocation from, and return to, the library's cache of device blocks (see
// rbf_block_cache); *got is the size actually held.  cached_free takes a
// block back once the work enqueued on st before the call has finished.
hipError_t cached_alloc(int dev, size_t bytes, void** out, size_t* got);
void cached_free(int dev, void* p, size_t bytes, hipStream_t st);

// ---- allocation-free entry point (noalloc.hip) -------------------------------
// Points the fixed device scratch serves: two vectors of this many doubles.
constexpr long long kNoAllocMaxPoints = 1LL << 22;
// Device address of the scratch array on `device` (2 * kNoAllocMaxPoints
// doubles), looked up with hipGetSymbolAddress on the first call per device.
hipError_t noalloc_scratch(int device, double** out);

// ---- the packed solve engine (capi.cpp) --------------------------------------
// Advances the GMRES solves of several problems together in packed launches
// on one stream (see capi.cpp).  Not thread-safe: one thread drives an engine.
class Engine;
struct EngineDone {
    void* tag;
    rbf_status status;
    std::string message;
};
Engine* engine_create(hipStream_t st, int capacity, bool graphs);
void engine_destroy(Engine* e);
// p's preconditioner of o.precision must be built; the weights go to d_lam_out
// (device, original order) when the solve ends; the problem joins at the next
// step.  RBF_ELIMIT when the engine is full or p cannot be packed (no lists).
rbf_status engine_add(Engine* e, rbf_problem* p, const rbf_solve_opts& o, double* d_lam_out,
                      void* tag);
int engine_active(const Engine* e);
// One step of every active problem; the problems that ended are appended to
// done (their weights written, their stream work enqueued and finished).
rbf_status engine_step(Engine* e, std::vector<EngineDone>* done);
// The solve information of a problem that ended (as rbf_solve_device fills it).
void engine_info(const rbf_problem* p, rbf_solve_info* info);

// ---- Krylov vector operations (krylov.hip) -----------------------------------
constexpr int kDotBlocks = 1024;
// out[k] = <V_k, w> for k < nv (V column k at V + k*ldv), deterministic
// two-stage reduction; partial must hold kDotBlocks * nv doubles.
hipError_t launch_multidot(const double* V, long long ldv, int nv, const double* w,
                           long long n, double* partial, double* out, hipStream_t st);
// w -= sum_k h[k] V_k (h on device), nv <= 64
hipError_t launch_multi_axpy(const double* V, long long ldv, int nv, const double* h,
                             double* w, long long n, double sign, hipStream_t st);
// dst = src / sqrt(*nrm2)   (the squared norm on device)
hipError_t launch_scale_by_inv(const double* src, const double* nrm2, double* dst,
                               long long n, hipStream_t st);
// r = f - y
hipError_t launch_sub(const double* f, const double* y, double* r, long long n,
                      hipStream_t st);
// x += a * z (a host scalar)
hipError_t launch_axpy(double a, const double* z, double* x, long long n, hipStream_t st);
hipError_t launch_fill(double* x, double v, long long n, hipStream_t st);
// flag = 1 if any x is NaN/Inf
hipError_t launch_check_finite(const double* x, long long n, int* flag, hipStream_t st);
// in-place block sum helpers used by the driver
hipError_t launch_sum_counts(const int* nnb, long long n, long long* partial_out,
                             hipStream_t st);

// ---- packed launches: the same operation for many problems at once ----------
// Each launch takes a device table of jobs and the workgroup offsets of the
// jobs (block0[j] .. block0[j + 1] serve job j, block0[njobs] = nblocks); a
// job's workgroups run exactly the computation of the single-problem launch
// (its block count is the single-problem grid), so results are bit-identical.
// Blocks of the single-problem launches, for sizing the packed ones.
int dot_blocks(long long n);   // launch_multidot's grid
int vec_blocks(long long n);   // the element-wise kernels' grid
struct VecJob {
    enum : int { kSub = 0, kAxpy = 1, kFill = 2, kScaleByInv = 3, kMultiAxpy = 4, kNop = 5,
                 kAxpyKeep = 6 };
    int op;                  // y = a - b | y += a | y = 0 | y = a / sqrt(den[0]) |
                             // y = sign * sum_k coef[k] a[k * ld ..] + (overwrite ? 0 : y) | none |
                             // b = y, then y += a (b written: the old y kept)
    int nv;                  // multi-axpy: vectors (<= 64)
    int overwrite;
    long long n, ld;
    const double* a;
    const double* b;
    const double* den;
    const double* coef;      // multi-axpy coefficients (device)
    double* y;
    double* keep;            // kAxpyKeep: where the old y goes
    double sign;
};
struct DotJob {              // out[k] = <V_k, w>, k < nv, partials in partial (nv = 0: none)
    const double* V;
    long long ldv;
    int nv, nb;              // nb: dot_blocks(n)
    const double* w;
    long long n;
    double* partial;         // kDotBlocks * nv
    double* out;
};
hipError_t launch_vec_packed(const VecJob* jobs, const int* block0, int njobs, int nblocks,
                             hipStream_t st);
// partials of every DotJob (block counts nb each), then their sums (nv blocks each)
hipError_t launch_multidot_packed(const DotJob* jobs, const int* block0, int njobs, int nblocks,
                                  hipStream_t st);
hipError_t launch_reduce_packed(const DotJob* jobs, const int* block0, int njobs, int nblocks,
                                hipStream_t st);
struct MatvecJob {           // y = A w by the lists (prec 0: FP64, 1: FP32)
    MatvecArgs a;
    Matvec32Args a32;
    NeighborLists nl;
    const double* w;
    double* y;
    int prec, skip;
};
// workgroups: nl.ngroups per job; threads: 64 * the largest nl.gunits
hipError_t launch_matvec_lists_packed(const MatvecJob* jobs, const int* block0, int njobs,
                                      int nblocks, int threads, hipStream_t st);
struct RasmJob {             // z = M^-1 v (prec 0: FP64 Z; 1: FP32 Z, FP32 sums; 2: FP32 Z, FP64 sums)
    PrecondArgs a;
    const void* Z;
    const double* v;
    double* z;
    int prec, skip;
};
// workgroups: a.ncells per job
hipError_t launch_rasm_packed(const RasmJob* jobs, const int* block0, int njobs, int nblocks,
                              hipStream_t st);

}  // namespace rbf
