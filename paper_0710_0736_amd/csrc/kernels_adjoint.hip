// kernels_adjoint.hip -- gradients of a segmentation through its time steps.
//
// The paper does not differentiate its scheme; this is the derivative of the
// discrete step map of eq. alpha.  With the free sets I_p = {i : u^{n+1}_pi > 0}
// held fixed, u^{n+1} minimises the step's quadratic over
// {u_pi = 0 outside I_p, sum_{I_p} u_pi = 1}, so for a loss gradient ubar at
// u^{n+1} the gradient at the right-hand side b is z = (T H T)^+ T ubar, T the
// node-wise tangent projection (zero outside I_p, minus the mean over I_p;
// zero when |I_p| <= 1).  z is found by red-black block Gauss-Seidel on
//     z_p = T_p (ubar_p / (h^2 D_p) + kappa_p sum_q c_pq z_q)
// (the nodal minimiser of z.H z / 2 - ubar.z on the range of T_p, in the
// scaled units of the smoother), over-relaxed: z_p <- z_p + omega (that - z_p),
// which stays in the range of T_p.  The system is symmetric positive definite
// and red-black ordered (two-cyclic), so the sweeps converge for 0 < omega < 2
// and Young's optimum is 2 / (1 + sqrt(1 - rho^2)) with rho the block-Jacobi
// radius.  The first kAdjOmegaSweep sweeps of a solve are plain Gauss-Seidel
// (omega = 1); their successive changes shrink by its contraction rho^2, whose
// estimate, the ratio of the last two changes, then fixes omega for the rest
// of the solve, capped by
// the value for the bound rho <= q = max_p kappa_p sum_q c_pq (the T_p only
// shrink the coupling).  An early estimate errs low (fast transients), which
// under-relaxes: still faster than Gauss-Seidel.  For a contraction by r per
// sweep, the distance to the solution after a sweep that changed z by dz is
// at most dz r / (1 - r); so the solve stops when dz <= rtol max|z| (1 - r),
// with r the larger of the ratio of the last two changes and omega - 1 (the
// contraction of over-relaxed sweeps cannot be smaller), at most 0.999, or
// when dz has fallen to a few units of float32 rounding of max|z|.  The
// chain rule then runs through
//     b_pi = M_p [(1/tau + 2/eps) un_pi - lambda F_pi],  F_pi = sum_k (I_pk - c_ik)^2,
//     c_ik = S_ik / S_i,  H = M/tau + eps A,
// with M_p = h^2 w_p; an empty phase's (kept) mean is a constant.
#include <algorithm>

#include "acseg_internal.h"

namespace acseg {

namespace {

// Weighted neighbour sum of node p = y W + x of one plane (32-bit offsets
// from the plane's base; the lattice holds at most 2^30 nodes).
__device__ __forceinline__ float nbs(const float* __restrict__ v, int W, int H, int x, int y, uint32_t p) {
    const float h = (x > 0 ? gload(v, p - 1) : 0.f) + (x < W - 1 ? gload(v, p + 1) : 0.f);
    const float vv = (y > 0 ? gload(v, p - W) : 0.f) + (y < H - 1 ? gload(v, p + W) : 0.f);
    return edge_w_h(y, H) * h + edge_w_v(x, W) * vv;
}

// Maxima of V values over a workgroup of T threads, with one barrier: every
// thread returns them in v.
template <int V, int T>
__device__ __forceinline__ void block_max_v(float (&v)[V]) {
    __shared__ float sh[T / kWave][V];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = wave_max(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < V; ++j) sh[wid][j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < V; ++j) {
        float r = sh[0][j];
        for (int w = 1; w < T / kWave; ++w) r = fmaxf(r, sh[w][j]);
        v[j] = r;
    }
}

// Column sums of part[nb][M] into tot[M] by a workgroup of T threads.
template <int M, int T>
__device__ void reduce_rows_t(const double* __restrict__ part, int nb, double* tot, double (*sh)[M]) {
    double acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    for (int b = threadIdx.x; b < nb; b += T)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] += part[(int64_t)b * M + m];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const double v = wave_sum(acc[m]);
        if (lane == 0) sh[wid][m] = v;
    }
    __syncthreads();
    if (threadIdx.x < M) {
        double t = 0.0;
        for (int w = 0; w < T / kWave; ++w) t += sh[w][threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
}

// Threads of a workgroup of the node-parallel passes (accumulation, means):
// 1024, or 256 where the 3 + N C float64 partial sums would not fit the
// registers of a thread of a 1024-thread workgroup.
__host__ __device__ constexpr int adj_threads(int N, int C) { return N * C <= 12 ? 1024 : kBlock; }

// Two red-black sweeps of the adjoint solve per launch, tile by tile in LDS.
// A tile of 64 x 8 nodes stages z, the scaled loss gradient ubar_p / (h^2 D_p)
// and the free sets with a halo of 4.  Half-sweep k of the launch (k = 0..3:
// red, black, red, black) updates the nodes of its colour within distance
// 4 - 1 - k of the tile from the values the previous half-sweep left in LDS,
// so the tile's own nodes end as two global red-black sweeps leave them.  The
// launch that starts at sweep s reads z from buffer (s / 2) & 1 (a.z, a.z2)
// and writes the other, so tiles never see each other's new values.  Each
// sweep leaves per-workgroup partials (max |dz| over the tile's black nodes,
// max |z|) in the set of its index mod 6, so a launch never overwrites a set
// it reads.  Every launch after the first evaluates the stopping rule on the
// partials of the sweeps before it and skips the rest of the solve once the
// rule holds.  Per node the arithmetic is that of one half-sweep of a global
// red-black sweep.
constexpr int kAdjK = 2;  // sweeps per launch
constexpr int kAdjTX = 64, kAdjTY = 8, kAdjR = 2 * kAdjK;
constexpr int kAdjSlots = 6;
constexpr int kAdjOmegaSweep = 6;  // the sweep that fixes omega from the Gauss-Seidel contraction
constexpr float kAdjUlps = 8.f;    // changes this close to float32 rounding of max|z| stop the solve
constexpr int kAdjLX = kAdjTX + 2 * kAdjR, kAdjLY = kAdjTY + 2 * kAdjR;
static_assert(kAdjOmegaSweep % kAdjK == 0, "omega is fixed at the start of a launch");
static_assert(kAdjSlots >= kAdjK + 3, "a launch writes kAdjK sets and reads the three before them");

__host__ __device__ inline int adj_tiles(int W, int H) {
    return ((W + kAdjTX - 1) / kAdjTX) * ((H + kAdjTY - 1) / kAdjTY);
}

// Weighted neighbour sum of staged node (lx, ly) = lattice node (x, y).
__device__ __forceinline__ float nbs_tile(const float (&zl)[kAdjLY][kAdjLX], int W, int H, int x, int y, int lx,
                                          int ly) {
    const float h = (x > 0 ? zl[ly][lx - 1] : 0.f) + (x < W - 1 ? zl[ly][lx + 1] : 0.f);
    const float vv = (y > 0 ? zl[ly - 1][lx] : 0.f) + (y < H - 1 ? zl[ly + 1][lx] : 0.f);
    return edge_w_h(y, H) * h + edge_w_v(x, W) * vv;
}

// The stopping rule after `sweeps` sweeps, evaluated by a whole workgroup
// (every workgroup that evaluates it reads the same partials and reaches the
// same result).  For a sweep t >= 2: with dz_t the largest change of sweep
// t - 1 and r the contraction per sweep (the ratio of the last two changes;
// sweep 0 compared its black values with zero, so it gives none), never
// below omega - 1 of the sweep, at most 0.999, the rule holds at t when
// dz_t <= rtol max|z| (1 - r), or when dz_t is within kAdjUlps units in the
// last place of max|z|: there float32 rounding, not the contraction, sets
// the changes, and further sweeps do not bring z closer.  The solve stops
// after `sweeps` sweeps when the rule holds at `sweeps` or at `sweeps` - 1
// (the sweep in between only brings z closer).  `ratio` is the ratio at
// `sweeps`, for the choice of omega.
struct AdjRule {
    bool stop;
    float ratio;
};

template <int T = kBlock>
__device__ AdjRule adj_rule(const AdjArgs& a, int sweeps) {
    auto set = [&](int t) { return a.part_f + (((t % kAdjSlots) + kAdjSlots) % kAdjSlots) * 2 * kMgBlocks; };
    const float *p1 = set(sweeps - 1), *p2 = set(sweeps - 2), *p3 = set(sweeps - 3);
    float dz1 = 0.f, zm1 = 0.f, dz2 = 0.f, zm2 = 0.f, dz3 = 0.f;
    for (int b = threadIdx.x; b < a.nblocks; b += T) {
        dz1 = fmaxf(dz1, p1[b]);
        zm1 = fmaxf(zm1, p1[kMgBlocks + b]);
        dz2 = fmaxf(dz2, p2[b]);
        zm2 = fmaxf(zm2, p2[kMgBlocks + b]);
        dz3 = fmaxf(dz3, p3[b]);
    }
    float m[5] = {dz1, zm1, dz2, zm2, dz3};
    block_max_v<5, T>(m);
    dz1 = m[0];
    zm1 = m[1];
    dz2 = m[2];
    zm2 = m[3];
    dz3 = m[4];
    const float omega = a.actl->omega;
    auto holds = [&](int t, float dz, float zm, float dzp) {
        const float ratio = t > 2 ? (dzp > 0.f ? dz / dzp : 0.f) : 1.f;
        const float om = t - 1 >= kAdjOmegaSweep ? omega : 1.f;
        const float r = fminf(fmaxf(ratio, om - 1.f), 0.999f);
        return !(dz > fmaxf(a.rtol * (1.f - r), kAdjUlps * 0x1p-24f) * zm);
    };
    const float ratio = sweeps > 2 ? (dz2 > 0.f ? dz1 / dz2 : 0.f) : 1.f;
    const bool stop = holds(sweeps, dz1, zm1, dz2) || (sweeps - 1 >= 2 && holds(sweeps - 1, dz2, zm2, dz3));
    return {stop, ratio};
}

__device__ __forceinline__ float mass_wf(int cls) {
    return cls == 0 ? 1.f : (cls == 1 ? 0.5f : (cls == 2 ? (1.f / 3.f) : (1.f / 6.f)));
}

// The colour means' share of a step's gradient (c_ik = S_ik / S_i), applied
// one launch later: for the step whose cbar, means and sums a.cm_* point to,
// A_ik = cbar_ik / S_i (0 for an empty phase, whose kept mean is a constant)
// and B_i = sum_k A_ik c_ik; then dL/du^n_pi gains w_p (sum_k A_ik I_pk - B_i)
// and dL/dI_pk gains w_p sum_i A_ik u^n_pi.  Threads i < N fill A[N*C], B[N].
template <int N, int C>
__device__ void means_share(const AdjArgs& a, float* A, float* B) {
    if (threadIdx.x >= N) return;
    const int i = threadIdx.x;
    const double* tot = a.cm_tot;
    const double S = tot[N * C + i], area = tot[N * C + N + C];
    double b = 0.0;
    for (int k = 0; k < C; ++k) {
        const double Aik = S > 1e-12 * area ? a.cm_cbar[i * C + k] / S : 0.0;
        A[i * C + k] = (float)Aik;
        b += Aik * a.cm_c64[i * C + k];
    }
    B[i] = (float)b;
}

// The buffer that holds z after `sweeps` sweeps (a multiple of kAdjK).
__device__ __forceinline__ const float* adj_z_after(const AdjArgs& a, int sweeps) {
    return ((sweeps / kAdjK) & 1) ? a.z2 : a.z;
}

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_adj_sweep(AdjArgs a, int s0) {
    static_assert(N <= 8, "free sets are bytes");
    constexpr int kStageP = N <= 4 ? (kAdjLX * kAdjLY + kBlock - 1) / kBlock : 20 / N;
    __shared__ float zl[N][kAdjLY][kAdjLX];
    __shared__ float bl[N][kAdjLY][kAdjLX];  // ubar_p / (h^2 D_p)
    __shared__ uint8_t fl[kAdjLY][kAdjLX];   // bit i: phase i free at u^{n+1}
    __shared__ float cmA[N * C], cmB[N];
    AdjCtl* ac = a.actl;
    if (ac->done) return;
    const bool share = a.cm_cbar != nullptr;  // ubar = a.ub plus the later step's means share
    if (share) means_share<N, C>(a, cmA, cmB);  // read after the tile loop's first barrier
    float omega = 1.f;  // of both sweeps of the launch
    if (s0 >= 2) {
        const AdjRule rule = adj_rule(a, s0);
        if (rule.stop) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                ac->done = 1;
                ac->sweeps = s0;
            }
            return;
        }
        if (s0 == kAdjOmegaSweep) {
            // Gauss-Seidel so far: the ratio estimates rho^2
            const float rho2 = fminf(rule.ratio, 0.99f);
            omega = fminf(a.omega, fmaxf(1.f, 2.f / (1.f + sqrtf(1.f - rho2))));
            if (blockIdx.x == 0 && threadIdx.x == 0) ac->omega = omega;  // read by later launches
        } else if (s0 > kAdjOmegaSweep) {
            omega = ac->omega;
        }
    }
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    const float* zin = adj_z_after(a, s0);
    float* zout = const_cast<float*>(adj_z_after(a, s0 + kAdjK));
    const int tiles_x = (W + kAdjTX - 1) / kAdjTX;
    const int ntiles = adj_tiles(W, H);
    float dzm[kAdjK], zmax[kAdjK];
#pragma unroll
    for (int j = 0; j < kAdjK; ++j) dzm[j] = zmax[j] = 0.f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % tiles_x) * kAdjTX - kAdjR, y0 = (tile / tiles_x) * kAdjTY - kAdjR;
        __syncthreads();  // the previous tile's reads of the staged arrays are done
        // every load of a chunk of kStageP positions per thread is issued
        // before the first LDS store, so the chunk waits for memory once
        for (int q0 = 0; q0 < kAdjLX * kAdjLY; q0 += kStageP * kBlock) {
            float zv[kStageP][N], bv[kStageP][N], uv[kStageP][N], iv[kStageP][C];
            uint32_t gq[kStageP];
#pragma unroll
            for (int pp = 0; pp < kStageP; ++pp) {
                const int q = q0 + pp * kBlock + (int)threadIdx.x;
                const int ly = q / kAdjLX, lx = q - ly * kAdjLX;
                const int gx = x0 + lx, gy = y0 + ly;
                const bool in = q < kAdjLX * kAdjLY && gx >= 0 && gx < W && gy >= 0 && gy < H;
                gq[pp] = in ? (uint32_t)(gy * W + gx) : 0xffffffffu;
                const uint32_t g = in ? gq[pp] : 0u;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    zv[pp][i] = gload(zin + i * n, g);
                    bv[pp][i] = gload(a.ub + i * n, g);
                    uv[pp][i] = gload(a.u1 + i * n, g);
                }
#pragma unroll
                for (int k = 0; k < C; ++k) iv[pp][k] = share ? gload(a.image + k * n, g) : 0.f;
            }
#pragma unroll
            for (int pp = 0; pp < kStageP; ++pp) {
                const int q = q0 + pp * kBlock + (int)threadIdx.x;
                if (q >= kAdjLX * kAdjLY) break;
                const int ly = q / kAdjLX, lx = q - ly * kAdjLX;
                const bool in = gq[pp] != 0xffffffffu;
                const int cls = node_class(x0 + lx, y0 + ly, W, H);
                const float rs = in ? sel4(a.coef.inv_d, cls) * a.inv_h2 : 0.f;
                const float wv = mass_wf(cls);
                uint32_t f = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    float b = bv[pp][i];
                    if (share) {
                        float t = -cmB[i];
#pragma unroll
                        for (int k = 0; k < C; ++k) t = fmaf(cmA[i * C + k], iv[pp][k], t);
                        b = fmaf(wv, t, b);
                    }
                    zl[i][ly][lx] = (in && s0 > 0) ? zv[pp][i] : 0.f;
                    bl[i][ly][lx] = b * rs;
                    f |= (uv[pp][i] > 0.f ? 1u : 0u) << i;
                }
                fl[ly][lx] = (uint8_t)(in ? f : 0u);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2 * kAdjK; ++k) {
            const int j = k / 2, colour = k % 2, sweep = s0 + j;
            const bool last = j == kAdjK - 1;
            // the nodes of this colour within distance d of the tile: rows of
            // kAdjTX + 2 d nodes, half of them of each colour
            const int d = 2 * kAdjK - 1 - k;
            const int lo = kAdjR - d;
            const int per_row = (kAdjTX + 2 * d) / 2;
            const int rows = kAdjTY + 2 * d;
            for (int q = threadIdx.x; q < per_row * rows; q += kBlock) {
                const int r = q / per_row, m = q - r * per_row;
                const int ly = lo + r, gy = y0 + ly;
                const int gx0 = x0 + lo;
                const int gx = gx0 + 2 * m + ((gx0 + gy + colour) & 1);
                const int lx = gx - x0;
                if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
                const float kap = sel4(a.coef.kappa, node_class(gx, gy, W, H));
                const uint32_t f = fl[ly][lx];
                float yv[N];
                int kf = 0;
                float sum = 0.f;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    float v = bl[i][ly][lx];
                    if (!(sweep == 0 && colour == 0)) v += kap * nbs_tile(zl[i], W, H, gx, gy, lx, ly);
                    yv[i] = v;
                    if ((f >> i) & 1u) {
                        sum += v;
                        ++kf;
                    }
                }
                const float mean = kf > 0 ? sum / (float)kf : 0.f;
                const bool own = lx >= kAdjR && lx < kAdjR + kAdjTX && ly >= kAdjR && ly < kAdjR + kAdjTY;
                const uint32_t p = (uint32_t)(gy * W + gx);
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const float zo = zl[i][ly][lx];  // this node's value before the half-sweep (0 at sweep 0)
                    const float zg = (kf >= 2 && ((f >> i) & 1u)) ? yv[i] - mean : 0.f;
                    const float zn = fmaf(omega, zg - zo, zo);
                    if (colour == 1 && own) {
                        dzm[j] = fmaxf(dzm[j], fabsf(zn - zo));
                        zmax[j] = fmaxf(zmax[j], fabsf(zn));
                    }
                    if (!(last && colour == 1)) zl[i][ly][lx] = zn;  // read by the next half-sweep
                    if (own && last) gstore(zout + i * n, p, zn);
                }
            }
            __syncthreads();
        }
    }
    float m[2 * kAdjK];
#pragma unroll
    for (int j = 0; j < kAdjK; ++j) {
        m[2 * j] = dzm[j];
        m[2 * j + 1] = zmax[j];
    }
    block_max_v<2 * kAdjK, kBlock>(m);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < kAdjK; ++j) {
            float* cur = a.part_f + ((s0 + j) % kAdjSlots) * 2 * kMgBlocks;
            cur[blockIdx.x] = m[2 * j];
            cur[kMgBlocks + blockIdx.x] = m[2 * j + 1];
        }
}

// One workgroup: the stopping rule after `sweeps` sweeps, for a caller that
// reads the convergence flag between chunks of sweep launches.
__global__ __launch_bounds__(kBlock) void k_adj_check(AdjArgs a, int sweeps) {
    AdjCtl* ac = a.actl;
    if (ac->done) return;
    if (adj_rule(a, sweeps).stop && threadIdx.x == 0) {
        ac->done = 1;
        ac->sweeps = sweeps;
    }
}

// The black half-sweep's change bounds the sweep's residual: the red values
// of the sweep were computed from the previous black ones, so with those
// reproduced to |dz| the red nodes are consistent to kappa-weighted |dz|.

// Direct terms of the chain rule at every node, in float32, summed in
// float64 into block partials of dL/dlambda, dL/deps, dL/dtau and cbar_ik;
// with the later step's means share of dL/dI (u^{n+1} is that step's u^n).
// The solve ended either where a sweep launch found the stopping rule met,
// or after the a.budget sweeps the caller enqueued: then every workgroup
// evaluates the rule there itself, and workgroup 0 records the outcome for
// the step's bookkeeping.  Partial q: 0 sum z M F, 1 sum z (-2/eps^2 M u^n -
// A u^{n+1}), 2 sum z M (u^{n+1} - u^n), 3 + iC + k sum 2 lambda M z (I - c);
// k_adj_reduce applies the signs and 1/tau^2.
template <int N, int C>
__global__ __launch_bounds__(adj_threads(N, C)) void k_adj_accum(AdjArgs a) {
    constexpr int Q = 3 + N * C;
    constexpr int kAdjT = adj_threads(N, C);
    __shared__ double sh[kAdjT / kWave][Q];
    __shared__ float cmA[N * C], cmB[N];
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    AdjCtl* ac = a.actl;
    const bool share = a.cm_cbar != nullptr;
    if (share) means_share<N, C>(a, cmA, cmB);  // read after adj_rule's (or the next) barrier
    int sweeps = a.budget;
    bool conv = ac->done != 0;
    if (conv)
        sweeps = ac->sweeps;
    else if (sweeps >= 2)
        conv = adj_rule<kAdjT>(a, sweeps).stop;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ac->fin_done = conv ? 1 : 0;
        ac->fin_sweeps = sweeps;
    }
    const float* zf = adj_z_after(a, sweeps);
    float c[N * C];
#pragma unroll
    for (int q = 0; q < N * C; ++q) c[q] = (float)a.c64[q];
    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    const float h2 = (float)a.h2, ce = (float)(-2.0 / (a.eps * a.eps)), lam2 = (float)(2.0 * a.lambda);
    const float aa = (float)(1.0 / a.tau + 2.0 / a.eps);
    for (int t = blockIdx.x * kAdjT + threadIdx.x; t < (int)n; t += gridDim.x * kAdjT) {
        const int y = t / W, x = t - y * W;
        const uint32_t p = (uint32_t)t;
        const int cls = node_class(x, y, W, H);
        const float w = mass_wf(cls), Mp = h2 * w;
        const float ast = sel4(a.diagA, cls);
        // every load of the node before its first store (the stores could
        // alias later loads, which would then wait for them)
        float Ik[C], ib[C], zv[N], unv[N], u1v[N], nbv[N];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            Ik[k] = gload(a.image + k * n, p);
            ib[k] = gload(a.Ibar + k * n, p);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            zv[i] = gload(zf + i * n, p);
            unv[i] = gload(a.u0 + i * n, p);
            u1v[i] = gload(a.u1 + i * n, p);
            nbv[i] = nbs(a.u1 + i * n, W, H, x, y, p);
        }
        float tq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) tq[q] = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float z = zv[i], un = unv[i], u1 = u1v[i];
            const float Au1 = ast * u1 - nbv[i];
            const float zM = z * Mp;
            float F = 0.f;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const float d = Ik[k] - c[i * C + k];
                F = fmaf(d, d, F);
                const float g = lam2 * zM * d;
                tq[3 + i * C + k] += g;
                ib[k] -= g;
                if (share) ib[k] = fmaf(w * cmA[i * C + k], u1, ib[k]);
            }
            gstore(a.ub_out + i * n, p, aa * zM);
            tq[0] = fmaf(zM, F, tq[0]);
            tq[1] += z * fmaf(ce * Mp, un, -Au1);
            tq[2] = fmaf(zM, u1 - un, tq[2]);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] += (double)tq[q];
#pragma unroll
        for (int k = 0; k < C; ++k) gstore(a.Ibar + k * n, p, ib[k]);
    }
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) sh[wid][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < Q) {
        double t = 0.0;
        for (int w = 0; w < kAdjT / kWave; ++w) t += sh[w][threadIdx.x];
        a.part_d[(int64_t)blockIdx.x * Q + threadIdx.x] = t;
    }
}

// The step's totals tot[Q] (reduced from k_adj_accum's partials): into grads
// (accumulated) and cbar of the step, plus the solve's bookkeeping.  One
// thread.
template <int N, int C>
__device__ void adj_finish_step(const AdjArgs& a, const double* tot) {
    // every load before the first store (a store could alias a later load,
    // which would then wait for it)
    AdjCtl* ac = a.actl;
    Ctl* ctl = a.ctl;
    const int sw = ac->fin_sweeps, fin_done = ac->fin_done, short_steps = ac->short_steps;
    const int c_total = ctl->cycles_total, c_max = ctl->cycles_max, unconv = ctl->steps_unconv,
              done = ctl->steps_done;
    const double g0 = a.grads[0], g1 = a.grads[1], g2 = a.grads[2];
    float cb[N * C];
    for (int q = 0; q < N * C; ++q) cb[q] = (a.cbar_out && a.cbar_accumulate) ? a.cbar_out[q] : 0.f;
    a.grads[0] = g0 - tot[0];
    a.grads[1] = g1 + tot[1];
    a.grads[2] = g2 + tot[2] / (a.tau * a.tau);
    for (int q = 0; q < N * C; ++q) {
        a.cbar64[q] = tot[3 + q];
        if (a.cbar_out) a.cbar_out[q] = cb[q] + (float)tot[3 + q];
    }
    ctl->cycles_total = c_total + sw;
    ctl->cycles_max = sw > c_max ? sw : c_max;
    if (!fin_done) {
        // a budget below the cap was the caller's guess, not the solve's limit
        if (a.budget < a.max_sweeps)
            ac->short_steps = short_steps + 1;
        else
            ctl->steps_unconv = unconv + 1;
    }
    ctl->steps_done = done + 1;
    ac->done = 0;
    ac->sweeps = 0;
}

// One workgroup: the step's totals from k_adj_accum's partials.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_adj_reduce(AdjArgs a) {
    constexpr int Q = 3 + N * C;
    __shared__ double sh[kBlock / kWave][Q];
    __shared__ double tot[Q];
    reduce_rows<Q>(a.part_d, a.nblocks_acc, tot, sh);
    if (threadIdx.x == 0) adj_finish_step<N, C>(a, tot);
}

// The means share of the first step (the one left after the last
// accumulation pass): grad_u0 = a.ub + that share (when a.ub_out is set) and
// dL/dI gains its part, with u^n = a.u0.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_adj_final(AdjArgs a) {
    __shared__ float cmA[N * C], cmB[N];
    means_share<N, C>(a, cmA, cmB);
    __syncthreads();
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < (int)n; t += gridDim.x * kBlock) {
        const int y = t / W, x = t - y * W;
        const uint32_t p = (uint32_t)t;
        const float w = mass_wf(node_class(x, y, W, H));
        float Ik[C], ib[C], unv[N], ubv[N];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            Ik[k] = gload(a.image + k * n, p);
            ib[k] = gload(a.Ibar + k * n, p);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            unv[i] = gload(a.u0 + i * n, p);
            ubv[i] = a.ub_out ? gload(a.ub + i * n, p) : 0.f;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float du = -cmB[i];
#pragma unroll
            for (int k = 0; k < C; ++k) {
                du = fmaf(cmA[i * C + k], Ik[k], du);
                ib[k] = fmaf(w * cmA[i * C + k], unv[i], ib[k]);
            }
            if (a.ub_out) gstore(a.ub_out + i * n, p, fmaf(w, du, ubv[i]));
        }
#pragma unroll
        for (int k = 0; k < C; ++k) gstore(a.Ibar + k * n, p, ib[k]);
    }
}

__global__ void k_adj_init(AdjCtl* ac, double* grads) {
    if (threadIdx.x == 0) {
        AdjCtl c = {};
        *ac = c;
        grads[0] = grads[1] = grads[2] = 0.0;
    }
}

// Workgroups of a node-parallel pass, one node per thread of `threads`, at
// most `cap`.
int adj_blocks(int64_t n, int threads, int cap) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, cap));
}

template <int N, int C>
hipError_t adj_nc(int op, const AdjArgs& a, int sweep, hipStream_t s) {
    const int64_t n = (int64_t)a.W * a.H;
    switch (op) {
        case kAdjSweep:
            hipLaunchKernelGGL((k_adj_sweep<N, C>), dim3(a.nblocks), dim3(kBlock), 0, s, a, sweep);
            break;
        case kAdjCheck: hipLaunchKernelGGL(k_adj_check, dim3(1), dim3(kBlock), 0, s, a, sweep); break;
        case kAdjAccum:
            hipLaunchKernelGGL((k_adj_accum<N, C>), dim3(a.nblocks_acc), dim3(adj_threads(N, C)), 0, s, a);
            break;
        case kAdjReduce: hipLaunchKernelGGL((k_adj_reduce<N, C>), dim3(1), dim3(kBlock), 0, s, a); break;
        case kAdjFinal:
            hipLaunchKernelGGL((k_adj_final<N, C>), dim3(adj_blocks(n, kBlock, kMgBlocks)), dim3(kBlock), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int N>
hipError_t adj_n(int C, int op, const AdjArgs& a, int sweep, hipStream_t s) {
    switch (C) {
        case 1: return adj_nc<N, 1>(op, a, sweep, s);
        case 2: return adj_nc<N, 2>(op, a, sweep, s);
        case 3: return adj_nc<N, 3>(op, a, sweep, s);
        case 4: return adj_nc<N, 4>(op, a, sweep, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int adj_sweep_blocks(int W, int H) { return std::min(adj_tiles(W, H), kMgBlocks); }
int adj_accum_blocks(int N, int C, int W, int H) {
    return adj_blocks((int64_t)W * H, adj_threads(N, C), kAdjAccBlocks);
}
int adj_sweeps_per_launch() { return kAdjK; }

hipError_t launch_adj(int N, int C, int op, const AdjArgs& a, int sweep, hipStream_t s) {
    switch (N) {
        case 2: return adj_n<2>(C, op, a, sweep, s);
        case 3: return adj_n<3>(C, op, a, sweep, s);
        case 4: return adj_n<4>(C, op, a, sweep, s);
        case 5: return adj_n<5>(C, op, a, sweep, s);
        case 6: return adj_n<6>(C, op, a, sweep, s);
        case 7: return adj_n<7>(C, op, a, sweep, s);
        case 8: return adj_n<8>(C, op, a, sweep, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adj_init(AdjCtl* ac, double* grads, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_init, dim3(1), dim3(kWave), 0, s, ac, grads);
    return hipGetLastError();
}

}  // namespace acseg
