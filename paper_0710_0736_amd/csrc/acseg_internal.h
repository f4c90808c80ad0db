// acseg_internal.h -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "acseg_device.hpp"

namespace acseg {

// Per-step convergence record; two alternate between consecutive steps so
// that the end of one step can re-arm the slot of the step after next while
// the kernels of the next step read theirs.
struct StepSlot {
    int done;    // a cycle kernel found the step converged before `cycles` cycles
    int cycles;
    float resid;
    int pad;
};

// Control block in device memory, one per call.  Between time steps `cur`
// names the iterate buffer holding the current field; within a step the
// cycle kernels derive their input from it and their launch index, and never
// write it.  k_step_end resolves the step, moves `cur` and folds the
// statistics.  No kernel communicates across workgroups within a launch:
// partial results are plain stores consumed by a later kernel.
struct Ctl {
    StepSlot step[2];
    int cur;
    int steps_done;
    int empty_steps;
    int nonfinite;
    int steps_unconv;
    int cycles_total;
    int cycles_max;
    int empty_now;       // the last colour-means pass found an empty phase
    float resid;         // natural residual at the end of the last step
    float max_resid;     // largest end-of-step residual
    double alpha;        // line-search step of the current coarse correction
    int pad[12];
};
static_assert(sizeof(Ctl) <= 256, "control block must fit in 256 bytes");

// Three iterate buffers: [0] and [1] alternate as outputs, [2] may hold a
// read-only initial iterate.  A launch reading buffer c writes out_of(c).
struct Bufs {
    const float* b[3];
};

__host__ __device__ __forceinline__ int out_of(int cur) { return cur == 0 ? 1 : 0; }

// Buffer holding the iterate after k buffer-flipping launches from `start`.
__host__ __device__ __forceinline__ int iterate_buf(int start, int k) {
    if (k <= 0) return start;
    const int first = out_of(start);
    return ((k - 1) & 1) ? out_of(first) : first;
}

// Fine-level constants for the right-hand side (float64).
struct RhsCoef {
    double wd[4];   // w / D per node class
    double a;       // 1/tau + 2/eps
    double lambda;
    float wda[4];   // (w / D)(1/tau + 2/eps) per node class (< 1 when eps > 0.71 h)
};

constexpr int kCmeansBlocks = 1024;  // workgroups of the colour-mean pass (every CU busy)
constexpr int kRhsBlocks = 512;     // workgroups of the right-hand-side pass

// ---- launchers (kernels_fine.hip) ----------------------------------------

hipError_t launch_project(int N, int64_t count, const float* y, float* x, hipStream_t s);

// Colour-mean partial sums of bufs[ctl->cur] (or `u` when non-NULL):
// partials[cmeans_blocks][cmeans_width] float64.
int cmeans_width(int N, int C);
int cmeans_blocks(int W, int H);
hipError_t launch_cmeans(int N, int C, int W, int H, const float* image, const float* u,
                         Bufs bufs, const Ctl* ctl, double* partials, hipStream_t s);

// The colour means of fields[first .. first+count-1] (float[N][H][W] each,
// count <= kCmeansFields) in
// three launches: the sums of every field (partials: count x cmeans_blocks x
// cmeans_width doubles), their totals into tot[field][kCmeansMaxM], then the
// means into c64[field][kNC] in field order, an empty phase keeping the
// previous field's mean (field 0: the mean image colour).
hipError_t launch_cmeans_fields(int N, int C, int W, int H, const float* image, const float* fields,
                                int first, int count, double* partials, double* tot, double* c64, Ctl* ctl,
                                hipStream_t s);

// One block: the reduced sums tot[cmeans_width] (may be NULL), c64 (float64
// [N][C]) and c_out (float, may be NULL) from the partials; empty phases keep
// c_prev64 (NULL: mean image colour).
hipError_t launch_cmeans_finish(int N, int C, int W, int H, const double* partials, Ctl* ctl,
                                const double* c_prev64, double* c64, float* c_out, double* tot,
                                hipStream_t s);

// ---- launchers (kernels_cycle.hip) ---------------------------------------

// ---- smoothing cycles and the end of a step (kernels_cycle.hip) -----------

constexpr int kXcd = 8;  // XCDs of an MI355X: workgroup id mod 8 selects the XCD
constexpr int kStrip = 8;  // tile columns per strip of a single-image cycle launch
constexpr int kCmeansMaxM = 8 * 4 + 8 + 4 + 2;  // colour-mean sums per set, N <= 8, C <= 4
constexpr int kCmeansFields = 64;                // most fields of one launch_cmeans_fields
constexpr int kNC = 8 * 4;                       // stride of one set of means

// Per image, constant over a solve.
struct CycleArgs {
    Bufs bufs;
    Ctl* ctl;
    const float* image;       // [C][H][W]
    double* tot;              // colour-mean sums, two sets [2][kCmeansMaxM]
    double* c64;              // colour means, three sets [3][kNC]
    float* c_out;             // out (float) by the step's first launch, or NULL
    float* rhs;               // rhs' [N][H][W]: written by the first launch if store_rhs, else read
    float* res_part;          // [2][part_stride]        row = cycle & 1
    double* cm_part;          // [2][M][part_stride]     row = cycle & 1
    int part_stride;
    LevelCoef coef;
    RhsCoef rc;
    float tol;
    int W, H;
    int tiles_x, ntiles, tiles_per_xcd;
    int tiles_y, rows_per_xcd;  // tile rows; tile rows per XCD band (single-image launch order)
    float omega;                // over-relaxation of the smoothing sweeps (1: Gauss-Seidel; single image)
    // the truncated coarse correction's direction w and its line-search partials
    // (pairs <g~, w>, <w, H w>), applied by the launch after it (CycleStep::mg_update);
    // NULL without a truncated multigrid
    const float* mg_w;
    const double* mg_part;
    int mg_parts;
};

// Per launch.
struct CycleStep {
    int slot;       // control slot of this step (step index & 1)
    int cycle;      // cycle index within the step
    int first;      // this launch opens the cycle
    int launch;     // launch index within the step (buffer parity)
    int fixed;      // no convergence checks
    int store_rhs;
    int cm;         // closing launch accumulates colour-mean partials
    int tot_sel;    // sums of u^n in tot set tot_sel; the step's end writes set tot_sel ^ 1
    int c64_sel;    // the step's first launch writes the means of u^n to c64 set c64_sel
    int prev_sel;   // previous means (empty phases) in c64 set prev_sel, or -1
    int fixed_c;    // the means of every step are c64 set prev_sel (not recomputed)
    int mg_update;  // stage u as max(u + alpha w, 0): the coarse correction's update (not in a step's first launch)
};

// What a run of smoothing launches is within its step and cycle.
struct CycleRole {
    bool step_first;  // the first launch opens the step: it builds the right-hand side
    bool opens;       // the first launch opens the cycle: convergence check
    bool closes;      // the last launch closes the cycle: residual and colour-mean partials
    bool mg_update;   // the first launch applies the truncated coarse correction's update
};

// Where a launch's tiles come from: one image (descs == NULL) or a batch.
struct CycleGrid {
    const CycleArgs* descs;
    const int2* work;
    int nwork;
    int sor;  // batched launch with over-relaxed sweeps (omega from each descriptor)
};

// The iterate after a step of `cycles` cycles is the one left by
// cycles * launches_per_cycle + launch_offset smoothing launches.
struct StepEndArgs {
    int max_cycles, launches_per_cycle, launch_offset;
};

// A cycle's tiles are 64 x cycle_tile_rows(N) nodes.
int cycle_tile_rows(int N);
int cycle_launches(int sweeps);
int cycle_tiles(int N, int W, int H);
// Fill the lattice / tiling fields of a (W, H, tiles_x, ntiles, tiles_per_xcd).
void cycle_tiling(int N, int W, int H, CycleArgs* a);

// `sweeps` red-black projected block Gauss-Seidel sweeps of the current time
// step (launches of at most two).  The step's first launch builds the
// right-hand side from u^n (= bufs[ctl->cur]), the image and the colour-mean
// sums (stored to `rhs` when later launches need it); a closing launch writes
// per-tile residual partials and, with `cm`, colour-mean partials of its
// output.  Unless `fixed`, a cycle's first launch checks the previous cycle's
// residual and the rest of the step is skipped once it is <= tol.
hipError_t launch_cycle(int N, int C, int sweeps, const CycleArgs& a, const CycleStep& st,
                        const CycleGrid& g, CycleRole role, hipStream_t s);

// Convergence test after `cycles` cycles of the step in control slot `slot`.
hipError_t launch_step_check(const CycleArgs& a, int slot, int cycles, hipStream_t s);

// End of a time step: the reduced colour-mean sums of the new iterate into tot
// set st.tot_sel ^ 1, the step's residual and cycle count, the buffer holding
// the iterate, statistics; re-arms control slot st.slot ^ 1.  With descs, for
// the images imgs[0..nimg) of a batch.
hipError_t launch_step_end(int N, int C, const CycleArgs& a, const CycleStep& st,
                           const StepEndArgs& e, const CycleArgs* descs, const int* imgs, int nimg,
                           hipStream_t s);

// One workgroup: colour means from reduced sums tot (empty phases keep
// c_prev64) into c64 / c_out, flags in ctl.
hipError_t launch_means_from_tot(int N, int C, const double* tot, const double* c_prev64,
                                 Ctl* ctl, double* c64, float* c_out, hipStream_t s);

// ---- launchers (kernels_mg.hip): the truncated multigrid correction -------

constexpr int kMgBlocks = 1024;    // most workgroups of a pass with per-workgroup partials
constexpr int kTailSide = 64;      // levels with both sides <= this may run in the LDS tail
constexpr int kTailLds = 64 * 1024;   // LDS bytes the tail may use
constexpr int kCoarseSweeps = 8;   // most red-black sweeps on the coarsest level
constexpr int kMaxLevels = 16;     // lattice levels of a hierarchy (sides up to 2^15)

// Tiles of the multigrid passes.
constexpr int kDrTX = 32, kDrTY = 8;    // defect + restriction: level-1 nodes per workgroup
constexpr int kDnTX = 32, kDnTY = 16;   // down-leg of level l: level-(l+1) nodes per workgroup
constexpr int kUpTX = 64, kUpTY = 16;   // up-leg of level l: level-l nodes per workgroup
constexpr int kDirTX = 64, kDirTY = 8;  // direction and line-search partials: fine nodes
constexpr int kDirBlocks = 2048;        // most workgroups of one image's direction pass

// One coarse level l >= 1 of one image.  The level's correction problem is
// H_l v = r (componentwise, H_l rediscretised at spacing 2^l h); v holds the
// correction after the down-leg (pre-smoothing from zero), v2 after the
// up-leg (prolongation of the next coarser level and post-smoothing), or the
// result of the LDS tail or of the coarsest level's sweeps.
struct MgLevel {
    float* r;     // [N][H][W]
    float* v;     // [N][H][W]
    float* v2;    // [N][H][W]
    LevelCoef coef;
    int W, H;
    int pad[2];
};

// One image's truncated multigrid correction, constant over a solve.  The
// iterate is bufs[iterate_buf(ctl->cur, launch)], updated in place.  Levels
// 1..tail-1 are processed by tiled global-memory passes, levels tail..L-1 by
// the LDS tail (tail == L: none; the coarsest level is then a global pass).
struct MgImage {
    Bufs bufs;
    Ctl* ctl;
    const float* rhs;   // stored right-hand side [N][H][W]
    float* gt;          // direction w [N][H][W]
    double* part;       // line-search partials [dir_blocks][2]
    int N, W, H;        // finest level
    int L, tail;
    int dir_blocks;     // workgroups of the direction pass (partials to reduce)
    int coarse_sweeps;  // red-black sweeps on the coarsest level
    // the convergence test that opens a cycle (MgStep::check): the residual
    // partials of the smoothing launches, one per tile, in two sets by cycle parity
    const float* res_part;
    int part_stride, ntiles;
    float tol;
    LevelCoef fine;
    MgLevel lv[kMaxLevels];  // lv[1..L-1]
};

// Per launch.
struct MgStep {
    int slot, fixed, launch;
    int level;    // the level a coarse pass works on
    int sweeps;   // red-black sweeps of a coarse pass
    int zero;     // up-leg pass starts from v = 0 without a prolongation (coarsest global level)
    int nu_pre, nu_post;
    int check;    // > 0: the defect pass first tests whether cycle check - 1 converged
};

// Where a multigrid launch's workgroups come from: one image (descs == NULL:
// workgroup x is tile x of `single`, at st.level) or a batch (work[x] =
// (image, tile, level, zero): an up pass item with zero set starts from v = 0
// with the image's coarse_sweeps sweeps, the coarsest level of an image
// without an LDS tail).  blockIdx.y selects the component of componentwise passes.
struct MgGrid {
    const MgImage* descs;
    const int4* work;
    int nwork;
};

enum MgPass { kMgDefectRestrict = 0, kMgDown, kMgTail, kMgUp, kMgDir };

// Workgroups of pass `op` on level st.level of one image (single-image grid).
int mg_pass_tiles(int op, const MgImage& m, int level);
// Dynamic LDS bytes of pass `op` (down / up: `sweeps` red-black sweeps; tail:
// the hierarchy from m.tail).
size_t mg_pass_lds(int op, const MgImage& m, int sweeps);
// LDS bytes of the tail from level t of an image with level sides W[], H[].
size_t mg_tail_lds(const int* W, const int* H, int t, int L);
// Dynamic LDS bytes of a down / up pass with nu sweeps.
size_t mg_lds_down(int nu);
size_t mg_lds_up(int nu);

// Enqueue one multigrid pass.  Fine-level passes (defect + restriction,
// direction, update) are instantiated per N and need one N per launch (`N`);
// coarse passes are componentwise (grid.y = largest N of the launch).
hipError_t launch_mg(int op, int N, int ncomp, const MgImage& single, const MgGrid& g, const MgStep& st,
                     size_t lds, hipStream_t s);

// One launch of the subspace correction over the basis functions of one coarse
// level: level lattice Wc x Hc, spacing 2^sh finest nodes, the functions whose
// node (X, Y) has X % 2 == colour & 1 and Y % 2 == colour >> 1.  In place on
// the iterate left by `launch` smoothing launches of the step.  With `part`
// the supports are cut into chunks of `rows` box rows over two launches.
struct SscArgs {
    Bufs bufs;
    const Ctl* ctl;
    const float* rhs;   // stored right-hand side [N][H][W]
    LevelCoef coef;     // finest level
    int W, H;
    int Wc, Hc, sh, colour;
    int slot, fixed, launch;
    double* part;       // non-NULL: two launches, per-chunk partials [functions * chunks][2N+1]
    int rows, chunks;   // box rows per chunk, chunks per function
};

hipError_t launch_ssc(int N, const SscArgs& a, hipStream_t s);


// Prolongation (dir 0: dst[planes][Hf][Wf] = P src) or restriction (dir 1:
// dst[planes][Hc][Wc] = P^T src) between a Wf x Hf lattice and its coarse
// lattice of ceil(Wf/2) x ceil(Hf/2) nodes.
hipError_t launch_transfer(int planes, int dir, const float* src, float* dst, int Wf, int Hf,
                           hipStream_t s);

// ---- data on refined lattices, colour spaces (kernels_data.hip) -----------
hipError_t launch_refine(int planes, int W, int H, int r, const float* src, float* dst, hipStream_t s);
hipError_t launch_sample(int planes, int W, int H, int r, const float* src, float* dst, hipStream_t s);
hipError_t launch_lab(int ab_only, int64_t count, const float* rgb, float* dst, hipStream_t s);
hipError_t launch_mass_avg(int planes, int W, int H, const float* src, float* dst, int simplex, hipStream_t s);

// ---- launchers (kernels_adjoint.hip): gradients through the time steps ------

struct AdjCtl {
    int done;         // the current adjoint solve converged
    int sweeps;       // after this many sweeps
    float omega;      // over-relaxation factor of the current solve, set at sweep kAdjOmegaSweep
    int fin_done;     // the solve's outcome as the accumulation pass found it
    int fin_sweeps;   // and its sweeps
    int short_steps;  // steps whose enqueued sweeps, below the cap, did not converge
    int pad[2];
};

enum AdjOp { kAdjSweep = 0, kAdjCheck, kAdjAccum, kAdjReduce, kAdjFinal };

constexpr int kAdjAccBlocks = 256;  // most workgroups (partial rows) of the accumulation pass

// Step s backwards: u0 = u^s, u1 = u^{s+1}, ub = dL/du^{s+1}; out: ub_out =
// dL/du^s; accumulated: Ibar, grads (lambda, eps, tau); cbar of the step.
struct AdjArgs {
    Ctl* ctl;
    AdjCtl* actl;
    const float* image;
    const float* u0;
    const float* u1;
    const float* ub;
    float* ub_out;
    float* z;             // [N][H][W], z of the sweeps of one parity
    float* z2;            // [N][H][W], the other parity
    float* Ibar;          // [C][H][W]
    double* grads;        // [3]
    const double* c64;    // means of u^s [N][C]
    const double* tot;    // colour-mean sums of u^s (mass-weight units)
    double* cbar64;       // [N][C]
    float* cbar_out;      // [N][C] or NULL
    int cbar_accumulate;  // add cbar to cbar_out (fixed means) instead of storing it
    float* part_f;        // [6 (sweep mod 6)][2][kMgBlocks]: max |dz|, max |z| per workgroup
    double* part_d;       // [kMgBlocks][3 + N C]
    LevelCoef coef;       // finest level
    float diagA[4];       // stiffness diagonal per node class
    float inv_h2, rtol;
    float omega;          // largest over-relaxation factor of the sweeps (from the coupling bound)
    double h2, eps, tau, lambda;
    int W, H, nblocks, nblocks_acc, max_sweeps;
    int budget;  // sweeps enqueued for the current step (a multiple of the sweeps per launch)
    // the colour means share of the step after this one, applied by this
    // step's sweeps (to ub) and accumulation (to Ibar): its cbar [N][C], means
    // and sums; cm_cbar NULL: none
    const double* cm_cbar;
    const double* cm_c64;
    const double* cm_tot;
};

int adj_sweep_blocks(int W, int H);
int adj_accum_blocks(int N, int C, int W, int H);
int adj_sweeps_per_launch();
hipError_t launch_adj(int N, int C, int op, const AdjArgs& a, int sweep, hipStream_t s);
hipError_t launch_adj_init(AdjCtl* ac, double* grads, hipStream_t s);

// Initialise a control block (cur = initial buffer index).
hipError_t launch_ctl_init(Ctl* ctl, int cur, hipStream_t s);

// Copy bufs[ctl->cur] to dst unless it already is dst (count floats).
hipError_t launch_copy_current(Bufs bufs, const Ctl* ctl, float* dst, int64_t count,
                               hipStream_t s);

hipError_t launch_labels(int N, int C, int W, int H, const float* u, const float* c,
                         uint8_t* labels, float* composite, float* rounded, hipStream_t s);

// Energy parts of eq. E with c64 the colour means of u; energy[0..3].
// partials: at least kCmeansBlocks * 3 doubles.
hipError_t launch_energy(int N, int C, int W, int H, const float* image, const float* u,
                         const double* c64, double eps, double lambda, double h,
                         double* partials, double* energy, hipStream_t s);

// dst[t] = (double)src[t] for t < count.
hipError_t launch_widen(const float* src, double* dst, int count, hipStream_t s);

// Fill a float array with a value (graph-capture friendly; no memset nodes).
hipError_t launch_fill(float* p, int64_t count, float v, hipStream_t s);

}  // namespace acseg
