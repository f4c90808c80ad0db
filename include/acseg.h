/*
 * acseg.h -- C ABI of the MI355X (gfx950) solver for the vector-valued
 * Allen-Cahn phase-field colour segmentation of Kay & Tomasi
 * ("Colour Image Segmentation by the Vector-valued Allen-Cahn Phase-field
 * Model: a Multigrid Solution").
 *
 * The model (Section "A modified vector-valued Allen-Cahn equation"): an image
 * I with C channels on a W x H pixel lattice is segmented by N phase fields
 * u_1..u_N that stay on the Gibbs simplex (sum_i u_i = 1, u_i >= 0) at every
 * node, evolving by the gradient flow of the energy of eq. E with the colour
 * fitting term of eq. VV_fidelity.  Discretisation (Section "Discretisation
 * and Numerical Solution"): P1 finite elements with one node per pixel, every
 * lattice cell split along its (x,y)-(x+1,y+1) diagonal, lumped mass, natural
 * boundary conditions; backward Euler with the diffusion and the simplex
 * constraint implicit and the concave term -(2/eps) u and the fitting term
 * at the old time level (eq. alpha, read with the stiffness entering with a
 * positive sign and the time step multiplying the whole bracket).  Each time
 * step is a strictly convex quadratic program over a product of simplices,
 * solved by red-black projected block Gauss-Seidel (the per-node simplex
 * correction of Section "Gibbs Space Constraint Pseudocode") with truncated
 * multigrid corrections (Section "Multigrid Solution") until the natural
 * residual max_{p,i} |Pi(y_p(u)) - u_p,i| is at most `tol`.
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers on the context's device,
 *     contiguous, 4-byte aligned, owned by the caller; the library never
 *     allocates, frees or retains them.  Results are undefined if input and
 *     output arrays overlap unless stated otherwise.
 *   - Layout is structure-of-arrays, row major: an image is float[C][H][W], a
 *     phase field float[N][H][W]; node (x, y) has flat index y*W + x.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it and the call returns without waiting, except where an
 *     `acseg_stats*` output is non-NULL: then the call waits for the stream
 *     and fills it.
 *   - Return value: ACSEG_OK (0) or a negative error code.  Argument errors
 *     are detected on the host before anything is enqueued and leave the
 *     outputs untouched.  Conditions found on the device (not converged,
 *     empty phase, non-finite image values) are reported through
 *     acseg_stats.status, which may carry a positive warning code.
 *   - The workspace `ws` is caller-allocated device memory of at least
 *     acseg_workspace_size() bytes, 256-byte aligned; it must not be used by
 *     two calls that can run concurrently.
 */
#ifndef ACSEG_H
#define ACSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t acseg_status;

#define ACSEG_OK 0
#define ACSEG_ERR_INVALID_ARG (-1)  /* bad sizes or parameters, NULL where not allowed */
#define ACSEG_ERR_NONFINITE (-2)    /* the image holds NaN or Inf (device-detected) */
#define ACSEG_ERR_WORKSPACE (-3)    /* ws is NULL, misaligned or smaller than required */
#define ACSEG_ERR_HIP (-4)          /* a HIP runtime call failed */
#define ACSEG_ERR_UNSUPPORTED (-5)  /* N or C outside the compiled range */
#define ACSEG_ERR_TOO_LARGE (-6)    /* acseg_solve_no_alloc: the problem needs more than its scratch */
#define ACSEG_WARN_NOT_CONVERGED 1  /* some step hit max_cycles with residual > tol */
#define ACSEG_WARN_EMPTY_PHASE 2    /* some phase had no mass; its colour mean was kept */

/* Compiled ranges */
#define ACSEG_MIN_N 2
#define ACSEG_MAX_N 8
#define ACSEG_MAX_C 4

/* acseg_problem.flags */
#define ACSEG_FLAG_STORE_CHECKPOINTS 1u  /* acseg_solve writes u^0..u^steps */
/*
 * Every time step runs exactly max_cycles cycles instead of stopping at the
 * first cycle whose residual is <= tol.  The residual after the last cycle
 * still decides whether the step counts as converged (stats).  Without this
 * flag a step stops at convergence (see ACSEG_FLAG_NO_HOST_WAIT).
 * With this flag and stats == NULL, acseg_solve enqueues only kernels and
 * device-to-device copies on its stream (no host reads, no memsets), so the
 * call can be captured in a HIP graph and replayed.  acseg_solve_batched
 * uploads host-built descriptor tables on every call; with
 * ACSEG_FLAG_REUSE_TABLES it does not, and is capturable too.
 */
#define ACSEG_FLAG_FIXED_CYCLES 2u
/*
 * The colour means are an input, the same in every time step, instead of the
 * means of u^n (eq. VV_fidelity): acseg_solve reads them from c_out (which it
 * then does not write), acseg_solve_batched from c_outs[b], acseg_step from
 * c_prev (copied to c_out); all of them must be non-NULL.  acseg_backward
 * then takes them as c_fixed and returns dL/dc_fixed in grad_c ([N][C]).
 */
#define ACSEG_FLAG_FIXED_C 4u
/*
 * Adaptive schedules (no ACSEG_FLAG_FIXED_CYCLES) enqueue the cycles of a time
 * step in chunks (the first as long as the previous step needed, then growing)
 * and read the step's convergence flag back between chunks, so acseg_step and
 * acseg_solve wait for the stream while they run.  With this flag they instead
 * enqueue all max_cycles cycles of every step at once, which exit on the
 * device after convergence (no host wait; each skipped launch still costs a
 * few microseconds).  acseg_solve_batched always works this way.  With this
 * flag and stats == NULL, acseg_solve enqueues only kernels and device copies,
 * so it can be captured in a HIP graph whose converged cycles exit on the device.
 */
#define ACSEG_FLAG_NO_HOST_WAIT 8u
/*
 * The coarse correction of a multigrid cycle (levels >= 2) is the paper's own
 * successive subspace correction (Section "Multigrid Solution", with the
 * constraint handling of Section "Gibbs Space Constraint Pseudocode") instead
 * of the truncated correction: after the pre-smoothing sweeps, every basis
 * function of every coarse level, from the coarsest level to the finest,
 * moves u by the multiple alpha (one value per phase, summing to zero) of
 * itself that minimises the step's objective while every node stays on its
 * simplex, then the post-smoothing sweeps follow.  Same fixed point, usually
 * many more cycles: a coarse function's step stops where any node of its
 * support reaches zero.  No effect with one level.
 */
#define ACSEG_FLAG_SSC 16u
/*
 * acseg_solve_batched only: the workspace already holds the descriptor tables
 * of an earlier acseg_solve_batched call with the same B, problems (flags
 * aside), images, us, c_outs and workspace, and nothing has written to the
 * workspace's table region since; the call then builds no tables on the device
 * side and uploads nothing.  With ACSEG_FLAG_FIXED_CYCLES as well and stats ==
 * NULL, the call enqueues kernels only and can be captured in a HIP graph.  The
 * call still builds the tables on the host and returns ACSEG_ERR_INVALID_ARG,
 * enqueueing nothing, unless they equal the last tables this context uploaded
 * and went to the same workspace address.  That the workspace still holds them
 * (nothing else wrote there, the memory was not handed to another owner) is
 * the caller's responsibility.  Ignored by the other entry points.
 */
#define ACSEG_FLAG_REUSE_TABLES 32u
/*
 * The smoothing sweeps are over-relaxed, u_p <- Pi_G(u_p + omega (y_p - u_p)) with
 * y_p the node's Gauss-Seidel value, omega = 2 / (1 + sqrt(1 - q^2)) from the
 * bound q = max_p kappa_p sum_q c_pq of the block-Jacobi radius (Young's
 * factor; about 1.67 in pixel units, 1.00 at the unit scale).  Each update is
 * a projected step of length omega / D_p along the node's own block, which
 * for 0 < omega < 2 never raises the step's objective, so the minimiser is
 * the same.  The launch that measures the residual keeps its last black
 * half-sweep plain, so the residual is the natural one.  Also for
 * acseg_solve_batched (all problems of a batch share their flags).
 */
#define ACSEG_FLAG_SOR 64u

/*
 * One segmentation problem.  Parameters follow eq. E and eq. alpha:
 *   H, W    lattice rows and columns; each >= 2 and W * H <= 2^30
 *   C, N    image channels (1..ACSEG_MAX_C) and phases (ACSEG_MIN_N..ACSEG_MAX_N)
 *   h       lattice spacing (node (x,y) sits at (x h, y h)); > 0
 *   eps     interface parameter epsilon; > 0
 *   lambda  fitting weight; >= 0
 *   tau     time step (delta t of eq. alpha); > 0
 *   steps   number of time steps for acseg_solve; >= 0
 *   levels  lattice levels of the multigrid hierarchy including the finest:
 *           1 = Gauss-Seidel only; 0 = automatic (halve the sides, rounding
 *           up, while the longer side exceeds 15 and the shorter is >= 3);
 *           at most the automatic count (ACSEG_ERR_INVALID_ARG otherwise)
 *   nu_pre, nu_post  smoothing sweeps before / after the coarse correction
 *           (multigrid) -- with levels == 1, nu_pre + nu_post red-black
 *           sweeps form one cycle; each >= 0, sum >= 1.  With two or more
 *           levels both must be >= 1 (ACSEG_ERR_UNSUPPORTED otherwise); the
 *           coarse levels use the same counts; the coarsest level runs as
 *           many red-black sweeps from zero as its Jacobi contraction bound
 *           needs for FP32 rounding, at most 8.  With nu_pre = nu_post = 1 a
 *           cycle ends with the next cycle's pre-smoothing sweep (one launch
 *           of two sweeps), and the convergence test follows both: a step's
 *           first cycle is pre-smoothing, correction, two sweeps, every later
 *           one correction, two sweeps
 *   max_cycles  cycle budget per time step; >= 1
 *   tol     natural-residual tolerance (max norm, absolute); >= 0
 */
typedef struct acseg_problem {
    int32_t H, W, C, N;
    double h, eps, lambda, tau;
    int32_t steps;
    int32_t levels;
    int32_t nu_pre, nu_post;
    int32_t max_cycles;
    uint32_t flags;
    double tol;
} acseg_problem;

/* Filled (after waiting for the stream) when a non-NULL pointer is passed. */
typedef struct acseg_stats {
    int32_t status;              /* ACSEG_OK, a warning (>0) or ACSEG_ERR_NONFINITE */
    int32_t steps_done;
    int32_t cycles_total;        /* over all steps */
    int32_t cycles_max;          /* largest count in one step */
    int32_t steps_not_converged;
    int32_t empty_phase_steps;
    double final_residual;       /* natural residual after the last step */
    double max_residual;         /* largest end-of-step residual */
} acseg_stats;

typedef struct acseg_ctx acseg_ctx;

/* Library version as major*10000 + minor*100 + patch. */
int32_t acseg_version(void);

/* Human-readable text for a status code (static storage). */
const char *acseg_status_string(acseg_status s);

/*
 * Create a context bound to HIP device `device` (it becomes current for the
 * calling thread).  The context holds device properties and small pinned
 * host buffers for statistics; it holds no problem data.  One context per
 * host thread.  *out is set to NULL on failure.
 */
acseg_status acseg_create(int device, acseg_ctx **out);

/* Destroy a context created by acseg_create (NULL is allowed). */
acseg_status acseg_destroy(acseg_ctx *ctx);

/* Workspace bytes needed by acseg_step / acseg_solve / acseg_energy for p. */
acseg_status acseg_workspace_size(const acseg_problem *p, size_t *bytes);

/*
 * Euclidean projection onto the Gibbs simplex of `count` vectors of length N
 * (Section "Gibbs Space Constraint Pseudocode"): y and x are float[N][count]
 * (component-major).  x may equal y.  2 <= N <= ACSEG_MAX_N.
 */
acseg_status acseg_project_simplex(acseg_ctx *ctx, int32_t N, int64_t count, const float *y,
                                   float *x, void *stream);

/*
 * Transfer operators of the multigrid hierarchy (Section "Multigrid
 * Solution"): the coarse lattice of a Wf x Hf lattice has ceil(Wf/2) x
 * ceil(Hf/2) nodes, coarse node (X, Y) sitting on fine node (2X, 2Y).  The
 * prolongation P interpolates the coarse P1 function at the fine nodes (every
 * cell split along its (x,y)-(x+1,y+1) diagonal: a fine node halfway between
 * two coarse nodes along a lattice line or that diagonal takes their mean); a
 * fine node past the last coarse row or column (even side) takes the value of
 * that row or column.  direction 0: dst[planes][Hf][Wf] = P src, with src
 * [planes][Hc][Wc]; direction 1: dst[planes][Hc][Wc] = P^T src, with src
 * [planes][Hf][Wf].  src and dst must not overlap.  Wf, Hf >= 2.
 */
acseg_status acseg_transfer(acseg_ctx *ctx, int32_t direction, int32_t planes, int32_t Wf,
                            int32_t Hf, const float *src, float *dst, void *stream);

/*
 * Image data on a refined lattice (Section "Data Projection"; the refinement
 * of the pixel grid in Section "Determination of Natural Scales"): r uniform
 * refinements of a W x H pixel lattice give Wf = (W - 1) 2^r + 1 by Hf = (H - 1) 2^r + 1
 * nodes of spacing h / 2^r, pixel (x, y) sitting on node (x 2^r, y 2^r).
 * Every node that a refinement creates takes the value of one of its
 * neighbours, never an interpolated one (no new gradients): here the value of
 * the pixel at or below-left of it, so node (X, Y) holds pixel
 * (X >> r, Y >> r).  The automatic multigrid hierarchy of the refined lattice
 * passes through the pixel lattice.
 *   src  float[planes][H][W] (device), dst float[planes][Hf][Wf] (device);
 *        they must not overlap.
 *   0 <= r <= 8, W, H >= 2, Wf * Hf <= 2^30; ACSEG_ERR_INVALID_ARG otherwise.
 */
acseg_status acseg_refine(acseg_ctx *ctx, int32_t planes, int32_t W, int32_t H, int32_t r,
                          const float *src, float *dst, void *stream);

/*
 * The values of a field on the refined lattice of acseg_refine at the pixel
 * nodes: dst[c][y][x] = src[c][y 2^r][x 2^r], src float[planes][Hf][Wf], dst
 * float[planes][H][W] (device, not overlapping).  Same limits as acseg_refine.
 * Sampling the phase fields and taking their labels gives the segmentation at
 * the pixels.
 */
acseg_status acseg_sample(acseg_ctx *ctx, int32_t planes, int32_t W, int32_t H, int32_t r,
                          const float *src, float *dst, void *stream);

/*
 * The image as the standard (consistent) mass matrix sees it (Section "Data
 * Projection": fidelity terms assembled with M_pq = (eta_p, eta_q) instead of
 * the lumped mass):  dst_p = (M I)_p / m_p per channel, m_p = sum_q M_pq, on
 * the lattice of the solver (cells split along (x,y)-(x+1,y+1)).  Inside the
 * lattice this is I_p / 2 plus 1/12 of the six neighbours sharing a triangle.
 * With consistent-mass fitting, the right-hand side of every phase at node p
 * differs from the lumped one on dst by a term that is the same for all
 * phases, and the colour means equal the lumped means on dst; so the solver
 * run on dst computes the consistent-mass segmentation.
 *   src, dst  float[planes][H][W] (device), not overlapping; W, H >= 2,
 *   W * H <= 2^30, planes >= 1 (ACSEG_ERR_INVALID_ARG otherwise).
 */
acseg_status acseg_mass_average(acseg_ctx *ctx, int32_t planes, int32_t W, int32_t H,
                                const float *src, float *dst, void *stream);

/*
 * The image as "projection by simplex" sees it (Section "Data Projection": the
 * image enters the fidelity terms only through its integral over each
 * element).  Each triangle carries one value, the mean of its three vertex
 * values (the integral of the P1 interpolant over it divided by its area);
 * the load (M I)_p = sum over the triangles at p of that value times |T|/3,
 * and dst_p = (M I)_p / m_p, the mean of the values of the triangles at p
 * (cells split along (x,y)-(x+1,y+1)).  Inside the lattice this is I_p / 3
 * plus 1/9 of the six neighbours sharing a triangle.  Fitting with the
 * element values is the lumped solver run on dst: the right-hand sides differ
 * per node by a term common to all phases and the colour means agree.
 *   src, dst  float[planes][H][W] (device), not overlapping; W, H >= 2,
 *   W * H <= 2^30, planes >= 1 (ACSEG_ERR_INVALID_ARG otherwise).
 */
acseg_status acseg_simplex_average(acseg_ctx *ctx, int32_t planes, int32_t W, int32_t H,
                                   const float *src, float *dst, void *stream);

/*
 * Colour-space pre-pass (Section "Two Dimensional Examples", multi-channel
 * data: the model takes any colour space and number of channels, and L*a*b*
 * with the luminosity ignored is suggested in place of RGB).  rgb
 * float[3][count] holds sRGB values in [0, 1] (IEC 61966-2-1 transfer curve
 * and primaries, D65 white); dst gets CIE 1976 L*a*b* divided by 100:
 *   ACSEG_LAB  dst float[3][count] = (L*, a*, b*) / 100, so the first channel lies in [0, 1];
 *   ACSEG_AB   dst float[2][count] = (a*, b*) / 100 (luminosity dropped).
 * The white point is the image of RGB (1, 1, 1), so white and every grey
 * map to a* = b* = 0.  Device pointers; rgb and dst must not overlap.
 * ACSEG_ERR_INVALID_ARG for count < 0 or an unknown kind.
 */
#define ACSEG_LAB 0
#define ACSEG_AB 1
acseg_status acseg_colour_space(acseg_ctx *ctx, int32_t kind, int64_t count, const float *rgb,
                                float *dst, void *stream);

/*
 * Colour means of eq. VV_fidelity with the lumped mass (one node per pixel):
 *   c_ik = sum_p M_p u_pi I_pk / sum_p M_p u_pi,   c: float[N][C].
 * A phase whose mass is below 1e-12 of the domain area keeps c_prev[i] (if
 * c_prev is non-NULL) or gets the mean image colour; this is reported as
 * ACSEG_WARN_EMPTY_PHASE.  Uses the workspace.
 */
acseg_status acseg_colour_means(acseg_ctx *ctx, const acseg_problem *p, const float *image,
                                const float *u, const float *c_prev, float *c_out,
                                acseg_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * One time step (eq. alpha): c = colour means of u_in (c_prev for empty
 * phases, may be NULL), then u_out = the minimiser over the simplices of
 *   sum_i [ u_i.(M/tau + eps A) u_i / 2 - b_i.u_i ],
 *   b_pi = M_p [ (1/tau + 2/eps) u_in_pi - lambda F_pi(c) ],
 * starting from u_in, to residual <= tol or max_cycles cycles.  c_out
 * (float[N][C], may be NULL) receives the means used.  u_in and u_out must
 * not overlap.
 */
acseg_status acseg_step(acseg_ctx *ctx, const acseg_problem *p, const float *image,
                        const float *u_in, float *u_out, const float *c_prev, float *c_out,
                        acseg_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * p->steps time steps.  u: float[N][H][W], holds u^0 on entry and u^steps on
 * return.  c_out (float[N][C], may be NULL) receives the colour means of the
 * returned u.  With ACSEG_FLAG_STORE_CHECKPOINTS, checkpoints (float[steps+1]
 * [N][H][W]) receives u^0..u^steps; otherwise it may be NULL.
 */
acseg_status acseg_solve(acseg_ctx *ctx, const acseg_problem *p, const float *image, float *u,
                         float *c_out, float *checkpoints, acseg_stats *stats, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * acseg_solve without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  The call runs the kernels of acseg_solve with the
 * same arguments and results, on a scratch array that the library holds in
 * static device memory: ACSEG_NO_ALLOC_SCRATCH_BYTES (80 MiB) on every device
 * the library runs on, reserved when the library's code is loaded there and
 * held until the process ends.  It calls no device or host allocator.
 * Problems whose workspace (acseg_workspace_size) exceeds the scratch are
 * refused with ACSEG_ERR_TOO_LARGE before anything is enqueued; 1024 x 1024 at
 * N = 4 fits with its full multigrid hierarchy.  Every call on one device
 * uses that device's one scratch array and leaves its contents behind (each
 * call initialises what it reads): calls that can overlap on one device --
 * other streams, other threads, other contexts -- race and must be
 * serialised by the caller.  Kernel timing (acseg_timing_enable) does not
 * record these calls.
 */
#define ACSEG_NO_ALLOC_SCRATCH_BYTES 83886080u
acseg_status acseg_solve_no_alloc(acseg_ctx *ctx, const acseg_problem *p, const float *image,
                                  float *u, float *c_out, float *checkpoints, acseg_stats *stats,
                                  void *stream);

/*
 * B independent segmentations in one time loop: the solve of acseg_solve
 * (eq. alpha, time steps of Section "Multigrid Solution") for images[b] with
 * ps[b], u^0 in us[b] (overwritten with u^steps) and, when c_outs and
 * c_outs[b] are non-NULL, the colour means of the result in c_outs[b].  The
 * images may differ in size, N, C and every model parameter; they must agree
 * on steps, nu_pre, nu_post, max_cycles and flags (ACSEG_ERR_INVALID_ARG
 * otherwise) and not ask for checkpoints; the subspace correction
 * (ACSEG_FLAG_SSC with two or more levels) is refused with
 * ACSEG_ERR_UNSUPPORTED.  The images are grouped by N, C and cycle kind
 * (Gauss-Seidel or multigrid).  Each smoothing launch covers the tiles of all
 * images of a group; each pass of a multigrid correction (defect and
 * restriction, one down and one up pass per large level, the LDS tail,
 * direction, update) is one launch over the images of the group that have
 * that level, whatever their sizes.  Each image keeps its own convergence
 * control, so the result for every image is identical to acseg_solve's.
 * images, us, c_outs and stats are HOST arrays of B entries (device pointers
 * / statistics); stats may be NULL.
 * 1 <= B <= 4096.  The workspace size comes from acseg_batch_workspace_size.
 */
acseg_status acseg_batch_workspace_size(int32_t B, const acseg_problem *ps, size_t *bytes);
acseg_status acseg_solve_batched(acseg_ctx *ctx, int32_t B, const acseg_problem *ps,
                                 const float *const *images, float *const *us,
                                 float *const *c_outs, acseg_stats *stats, void *ws,
                                 size_t ws_bytes, void *stream);

/*
 * Post-processing of Section "Post-processing": labels[p] = argmax_i u_pi
 * (lowest index on ties), composite_kp = sum_i c_ik u_pi, rounded composite
 * rounded_kp = c_{labels[p],k}.  labels: uint8[H][W]; composite, rounded:
 * float[C][H][W]; each output may be NULL.  c: float[N][C].
 */
acseg_status acseg_labels(acseg_ctx *ctx, const acseg_problem *p, const float *u, const float *c,
                          uint8_t *labels, float *composite, float *rounded, void *stream);

/*
 * Discrete energy of eq. E on the P1 space with the lumped mass, with c the
 * colour means of u itself: energy[0] = eps/2 sum_i u_i.A u_i (interface),
 * energy[1] = 1/eps sum_{p,i} M_p u_pi (1 - u_pi) (concave potential),
 * energy[2] = lambda sum_{p,i} M_p u_pi F_pi (fitting), energy[3] = total.
 * energy: device double[4].  Uses the workspace.
 */
acseg_status acseg_energy(acseg_ctx *ctx, const acseg_problem *p, const float *image,
                          const float *u, double *energy, void *ws, size_t ws_bytes,
                          void *stream);

/*
 * Gradients of a loss L(u^steps) through a solve (the derivative of the
 * discrete time steps of eq. alpha; the paper does not differentiate them).
 * checkpoints: float[steps+1][N][H][W], u^0..u^steps of an acseg_solve of p
 * (ACSEG_FLAG_STORE_CHECKPOINTS); grad_uT: float[N][H][W] = dL/du^steps.
 * Outputs (device): grad_image float[C][H][W] = dL/dI; grad_u0
 * float[N][H][W] = dL/du^0 (may be NULL); grad_params double[3] = dL/dlambda,
 * dL/deps at fixed tau, dL/dtau; grad_c float[steps][N][C] = dL/dc^n, the
 * gradient at the colour means used by step n (may be NULL).  With
 * ACSEG_FLAG_FIXED_C, c_fixed (float[N][C]) are the means of the solve and
 * grad_c is float[N][C] = dL/dc_fixed; otherwise c_fixed is ignored.  Each step's
 * derivative holds the free sets {i : u^{n+1}_pi > 0} fixed (components at 0
 * count as active) and treats the kept mean of an empty phase as a constant.
 * The per-step linear solves are over-relaxed red-black sweeps, two per
 * launch, stopped after the first pair of sweeps that follows a sweep whose
 * change dz, with r the observed contraction per sweep (the ratio of the last
 * two changes, at least omega - 1, at most 0.999), satisfies
 * dz <= max(tol, 2e-7) max|z| (1 - r), so that the distance to the solution,
 * at most dz r / (1 - r), is below that relative tolerance, or
 * dz <= 8 ulp(max|z|) (float32 rounding sets such changes); at most
 * max(4, 2 max_cycles) sweeps, rounded up to even (stats count steps that hit
 * the cap as not converged, and the sweeps as cycles).  The first call for a
 * problem enqueues the sweeps in chunks of 4, 8, ... 64 and waits for the
 * stream between chunks to read the convergence flag.  The context then
 * remembers, per problem (all fields of p), the most sweeps a step took; a
 * later call gives every step that many sweeps without waiting (launches
 * after convergence do nothing), and runs again in chunks if a step did not
 * converge within them.  Either way the call waits for the stream once at
 * the end, so it returns with the work done.
 * Workspace from acseg_backward_workspace_size.
 */
acseg_status acseg_backward_workspace_size(const acseg_problem *p, size_t *bytes);
acseg_status acseg_backward(acseg_ctx *ctx, const acseg_problem *p, const float *image,
                            const float *checkpoints, const float *c_fixed,
                            const float *grad_uT, float *grad_image, float *grad_u0,
                            double *grad_params, float *grad_c, acseg_stats *stats, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * Kernel timing (profiling aid).  While enabled on a context, the calls
 * acseg_step and acseg_solve bracket each kernel family they enqueue with HIP
 * events on the call's stream; acseg_timing_read waits for those events, adds
 * up the elapsed times per family into out[0..*count-1] (at most max entries)
 * and forgets them.  Families: "cmeans", "rhs", "smooth" (one smoothing
 * cycle, or one launch of it when a cycle needs several), the passes of the
 * truncated multigrid correction ("mg_restrict": fine defect and first
 * restriction, "mg_down", "mg_tail": the coarsest levels in one workgroup
 * per component, "mg_up", "mg_dir": prolongated direction and line-search
 * partials; the step length and update count with the post-smoothing under
 * "smooth"), "ssc" (the subspace correction), "adj_sweep" (adjoint sweeps),
 * "other".
 */
typedef struct acseg_kernel_time {
    char name[16];
    int64_t launches;
    double total_ms;
} acseg_kernel_time;

acseg_status acseg_timing_enable(acseg_ctx *ctx, int32_t enable);
acseg_status acseg_timing_read(acseg_ctx *ctx, acseg_kernel_time *out, int32_t max,
                               int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* ACSEG_H */
