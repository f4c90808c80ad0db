// acseg_internal.h -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "acseg_device.hpp"

namespace acseg {

// Per-step / per-solve control block in device memory.  Kernels read `cur`
// (which of the three iterate buffers holds the current iterate) and `done`
// (the current step has converged or spent its cycle budget); the last block
// of each cycle kernel updates them.  Statistics accumulate over a solve.
struct Ctl {
    int cur;
    int done;
    int cycles;          // cycles run in the current step
    int steps_done;
    unsigned arrive;     // last-block counter (cycle kernels)
    unsigned arrive2;    // last-block counter (reductions)
    unsigned arrive3;    // last-block counter (line search)
    int empty_steps;
    int nonfinite;
    int steps_unconv;
    int cycles_total;
    int cycles_max;
    float resid;         // natural residual after the last cycle
    float max_resid;     // largest end-of-step residual
    double alpha;        // line-search step of the current coarse correction
    int empty_now;       // the last colour-means pass found an empty phase
    int pad[7];
};
static_assert(sizeof(Ctl) <= 256, "control block must fit in 256 bytes");

// Three iterate buffers: [0] and [1] alternate as cycle outputs, [2] may hold
// a read-only initial iterate.  The output of a cycle reading buffer `cur` is
// buffer (cur == 0 ? 1 : 0).
struct Bufs {
    const float* b[3];
};

__device__ __forceinline__ int out_of(int cur) { return cur == 0 ? 1 : 0; }

// Fine-level constants for the right-hand side (float64).
struct RhsCoef {
    double wd[4];   // w / D per node class
    double a;       // 1/tau + 2/eps
    double lambda;
};

// ---- launchers (kernels_fine.hip) ----------------------------------------

hipError_t launch_project(int N, int64_t count, const float* y, float* x, hipStream_t s);

// colour-mean partial sums of buffer bufs[ctl->cur] (or `u` when non-NULL);
// the last block writes c64 (float64 [N][C]) using c_prev64 for empty phases
// (c_prev64 may be NULL: mean image colour), and c_out (float, may be NULL).
hipError_t launch_cmeans(int N, int C, int W, int H, const float* image, const float* u,
                         Bufs bufs, Ctl* ctl, const double* c_prev64, double* c64,
                         float* c_out, double* partials, int max_blocks, hipStream_t s);

// rhs' = w[(1/tau+2/eps) u - lambda F(c)] / D, shifted per node so that its
// largest component is 0; resets the per-step control fields.
hipError_t launch_rhs(int N, int C, int W, int H, const float* image, Bufs bufs, Ctl* ctl,
                      const double* c64, RhsCoef rc, float* rhs, hipStream_t s);

// One smoothing cycle: `sweeps` red-black projected block Gauss-Seidel sweeps
// from bufs[cur] into bufs[out_of(cur)]; with `resid`, also the natural
// residual of the result, the done flag and the statistics (last block).
hipError_t launch_smooth(int N, int W, int H, int sweeps, bool resid, Bufs bufs, Ctl* ctl,
                         const float* rhs, LevelCoef coef, float tol, int max_cycles,
                         float* partials, hipStream_t s);

// Upper bound on the number of workgroups of one smoothing launch.
int smooth_max_tiles(int W, int H);

// End of a step: fold the step's counters into the solve statistics.
hipError_t launch_step_end(Ctl* ctl, float tol, hipStream_t s);

// Initialise a control block (cur = initial buffer index).
hipError_t launch_ctl_init(Ctl* ctl, int cur, hipStream_t s);

// Copy bufs[ctl->cur] to dst unless it already is dst (count floats).
hipError_t launch_copy_current(Bufs bufs, Ctl* ctl, float* dst, int64_t count, hipStream_t s);

hipError_t launch_labels(int N, int C, int W, int H, const float* u, const float* c,
                         uint8_t* labels, float* composite, float* rounded, hipStream_t s);

// Energy parts of eq. E with c64 the colour means of u; energy[0..3].
hipError_t launch_energy(int N, int C, int W, int H, const float* image, const float* u,
                         const double* c64, double eps, double lambda, double h,
                         double* partials, int max_blocks, Ctl* ctl, double* energy,
                         hipStream_t s);

// dst[t] = (double)src[t] for t < count.
hipError_t launch_widen(const float* src, double* dst, int count, hipStream_t s);

// Fill a float array with a value (graph-capture friendly; no memset nodes).
hipError_t launch_fill(float* p, int64_t count, float v, hipStream_t s);

}  // namespace acseg
