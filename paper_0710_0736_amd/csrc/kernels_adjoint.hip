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
// contraction of over-relaxed sweeps cannot be smaller), at most 0.999.  The
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

__device__ __forceinline__ float block_max_f(float v, float* sh) {
    v = wave_max(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = sh[0];
    for (int w = 1; w < kBlock / kWave; ++w) r = fmaxf(r, sh[w]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// One red-black sweep of the adjoint solve per launch, tile by tile in LDS.
// A tile of 64 x 8 nodes stages z with a halo of 2: the red nodes within
// distance 1 of the tile are updated from the staged (old) black values, then
// the tile's black nodes from those reds, so the tile ends as one global
// red-black sweep leaves it.  Sweep s reads z from buffer s & 1 (a.z, a.z2)
// and writes the other, so tiles never see each other's new values.  Every
// sweep after the second first checks the partials of the two sweeps before
// it (max |dz| over its black nodes, max |z|; three sets, by sweep mod 3, so
// that no workgroup of a launch overwrites a set another one may still read)
// and skips the rest of the solve once the stopping rule holds.  Per node the
// arithmetic is that of the two half-sweeps it replaces.
constexpr int kAdjTX = 64, kAdjTY = 8, kAdjR = 2;
constexpr int kAdjOmegaSweep = 6;  // the sweep that fixes omega from the Gauss-Seidel contraction
constexpr int kAdjLX = kAdjTX + 2 * kAdjR, kAdjLY = kAdjTY + 2 * kAdjR;

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

template <int N>
__global__ __launch_bounds__(kBlock) void k_adj_sweep(AdjArgs a, int sweep) {
    __shared__ float sh[kBlock / kWave];
    __shared__ float zl[N][kAdjLY][kAdjLX];
    AdjCtl* ac = a.actl;
    if (ac->done) return;
    float omega = 1.f;
    if (sweep > 1) {  // sweep 0 compared its black values with unset memory
        const float* prev = a.part_f + ((sweep - 1) % 3) * 2 * kMgBlocks;
        const float* pp = a.part_f + ((sweep - 2) % 3) * 2 * kMgBlocks;
        float dz = 0.f, zm = 0.f, dz2 = 0.f;
        for (int b = threadIdx.x; b < a.nblocks; b += kBlock) {
            dz = fmaxf(dz, prev[b]);
            zm = fmaxf(zm, prev[kMgBlocks + b]);
            dz2 = fmaxf(dz2, pp[b]);
        }
        dz = block_max_f(dz, sh);
        zm = block_max_f(zm, sh);
        dz2 = block_max_f(dz2, sh);
        // contraction per sweep: the ratio of the last two changes (sweep - 2
        // >= 1 compared real values), never below omega - 1 of the last sweep
        const float ratio = sweep > 2 ? (dz2 > 0.f ? dz / dz2 : 0.f) : 1.f;
        const float om_prev = sweep - 1 >= kAdjOmegaSweep ? ac->omega : 1.f;
        const float r = fminf(fmaxf(ratio, om_prev - 1.f), 0.999f);
        if (!(dz > a.rtol * zm * (1.f - r))) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                ac->done = 1;
                ac->sweeps = sweep;
            }
            return;
        }
        if (sweep == kAdjOmegaSweep) {
            // Gauss-Seidel so far: the ratio estimates rho^2
            const float rho2 = fminf(ratio, 0.99f);
            omega = fminf(a.omega, fmaxf(1.f, 2.f / (1.f + sqrtf(1.f - rho2))));
            if (blockIdx.x == 0 && threadIdx.x == 0) ac->omega = omega;  // read by later sweeps
        } else if (sweep > kAdjOmegaSweep) {
            omega = ac->omega;
        }
    }
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    const float* zin = (sweep & 1) ? a.z2 : a.z;
    float* zout = (sweep & 1) ? a.z : a.z2;
    const int tiles_x = (W + kAdjTX - 1) / kAdjTX;
    const int ntiles = adj_tiles(W, H);
    float dzm = 0.f, zmax = 0.f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % tiles_x) * kAdjTX - kAdjR, y0 = (tile / tiles_x) * kAdjTY - kAdjR;
        __syncthreads();  // the previous tile's reads of zl are done
        for (int q = threadIdx.x; q < kAdjLX * kAdjLY; q += kBlock) {
            const int ly = q / kAdjLX, lx = q - ly * kAdjLX;
            const int gx = x0 + lx, gy = y0 + ly;
            const bool in = sweep > 0 && gx >= 0 && gx < W && gy >= 0 && gy < H;
            const uint32_t g = in ? (uint32_t)(gy * W + gx) : 0u;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float t = gload(zin + i * n, g);
                zl[i][ly][lx] = in ? t : 0.f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int colour = 0; colour < 2; ++colour) {
            // red: the nodes within distance 1 of the tile, 33 per staged row;
            // black: the tile's own nodes, 32 per row
            const int lo = colour == 0 ? 1 : kAdjR;
            const int per_row = colour == 0 ? (kAdjTX + 2) / 2 : kAdjTX / 2;
            const int rows = colour == 0 ? kAdjTY + 2 : kAdjTY;
            for (int q = threadIdx.x; q < per_row * rows; q += kBlock) {
                const int r = q / per_row, k = q - r * per_row;
                const int ly = lo + r, gy = y0 + ly;
                const int gx0 = x0 + lo;
                const int gx = gx0 + 2 * k + ((gx0 + gy + colour) & 1);
                const int lx = gx - x0;
                if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
                const uint32_t p = (uint32_t)(gy * W + gx);
                const int cls = node_class(gx, gy, W, H);
                const float kap = sel4(a.coef.kappa, cls), rs = sel4(a.coef.inv_d, cls) * a.inv_h2;
                float yv[N];
                bool fr[N];
                int kf = 0;
                float sum = 0.f;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    float v = gload(a.ub + i * n, p) * rs;
                    if (!(sweep == 0 && colour == 0)) v += kap * nbs_tile(zl[i], W, H, gx, gy, lx, ly);
                    yv[i] = v;
                    fr[i] = gload(a.u1 + i * n, p) > 0.f;
                    if (fr[i]) {
                        sum += v;
                        ++kf;
                    }
                }
                const float mean = kf > 0 ? sum / (float)kf : 0.f;
                const bool own = lx >= kAdjR && lx < kAdjR + kAdjTX && ly >= kAdjR && ly < kAdjR + kAdjTY;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const float zo = zl[i][ly][lx];  // this node's value before the sweep (0 at sweep 0)
                    const float zg = (kf >= 2 && fr[i]) ? yv[i] - mean : 0.f;
                    const float zn = fmaf(omega, zg - zo, zo);
                    if (colour == 1) {
                        dzm = fmaxf(dzm, fabsf(zn - zo));
                        zmax = fmaxf(zmax, fabsf(zn));
                    } else {
                        zl[i][ly][lx] = zn;  // reds are read only by the black half
                    }
                    if (own) gstore(zout + i * n, p, zn);
                }
            }
            __syncthreads();
        }
    }
    const float d = block_max_f(dzm, sh);
    const float m = block_max_f(zmax, sh);
    if (threadIdx.x == 0) {
        float* cur = a.part_f + (sweep % 3) * 2 * kMgBlocks;
        cur[blockIdx.x] = d;
        cur[kMgBlocks + blockIdx.x] = m;
    }
}

// The black half-sweep's change bounds the sweep's residual: the red values
// of the sweep were computed from the previous black ones, so with those
// reproduced to |dz| the red nodes are consistent to kappa-weighted |dz|.

// Direct terms of the chain rule at every node; block partials of
// dL/dlambda, dL/deps, dL/dtau and cbar_ik.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_adj_accum(AdjArgs a) {
    constexpr int Q = 3 + N * C;
    __shared__ double sh[kBlock / kWave];
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    const double* c = a.c64;
    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    const double h2 = a.h2, tau = a.tau, eps = a.eps, lam = a.lambda;
    const double aa = 1.0 / tau + 2.0 / eps;
    // z after the last completed sweep: sweep s wrote buffer (s + 1) & 1
    const int done_sweeps = a.actl->done ? a.actl->sweeps : a.max_sweeps;
    const float* zf = (done_sweeps & 1) ? a.z2 : a.z;
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < (int)n; t += gridDim.x * kBlock) {
        const int y = t / W, x = t - y * W;
        const uint32_t p = (uint32_t)t;
        const int cls = node_class(x, y, W, H);
        const double Mp = h2 * mass_w(cls);
        const float ast = sel4(a.diagA, cls);
        float Ik[C];
#pragma unroll
        for (int k = 0; k < C; ++k) Ik[k] = gload(a.image + k * n, p);
        float ib[C];
#pragma unroll
        for (int k = 0; k < C; ++k) ib[k] = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double z = gload(zf + i * n, p);
            const double un = gload(a.u0 + i * n, p);
            const double u1 = gload(a.u1 + i * n, p);
            const double Au1 = (double)ast * u1 - (double)nbs(a.u1 + i * n, W, H, x, y, p);
            double F = 0.0;
            double d[C];
#pragma unroll
            for (int k = 0; k < C; ++k) {
                d[k] = (double)Ik[k] - c[i * C + k];
                F += d[k] * d[k];
            }
            gstore(a.ub_out + i * n, p, (float)(aa * Mp * z));
            acc[0] += z * (-Mp * F);
            acc[1] += z * (-2.0 / (eps * eps)) * Mp * un - z * Au1;
            acc[2] += (-z * Mp * un + z * Mp * u1) / (tau * tau);
            const double Fbar = -lam * Mp * z;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                ib[k] += (float)(2.0 * Fbar * d[k]);
                acc[3 + i * C + k] += -2.0 * Fbar * d[k];
            }
        }
#pragma unroll
        for (int k = 0; k < C; ++k) gstore(a.Ibar + k * n, p, gload(a.Ibar + k * n, p) + ib[k]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double t = block_sum(acc[q], sh);
        if (threadIdx.x == 0) a.part_d[(int64_t)blockIdx.x * Q + q] = t;
    }
}

// One workgroup: the partials into grads (accumulated) and cbar of the step.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_adj_reduce(AdjArgs a) {
    constexpr int Q = 3 + N * C;
    __shared__ double sh[kBlock / kWave][Q];
    __shared__ double tot[Q];
    reduce_rows<Q>(a.part_d, a.nblocks_acc, tot, sh);
    if (threadIdx.x < 3) a.grads[threadIdx.x] += tot[threadIdx.x];
    if (threadIdx.x < N * C) {
        a.cbar64[threadIdx.x] = tot[3 + threadIdx.x];
        if (a.cbar_out) {
            if (a.cbar_accumulate)
                a.cbar_out[threadIdx.x] += (float)tot[3 + threadIdx.x];
            else
                a.cbar_out[threadIdx.x] = (float)tot[3 + threadIdx.x];
        }
    }
    if (threadIdx.x == 0) {
        AdjCtl* ac = a.actl;
        Ctl* ctl = a.ctl;
        const int sw = ac->done ? ac->sweeps : a.max_sweeps;
        ctl->cycles_total += sw;
        ctl->cycles_max = sw > ctl->cycles_max ? sw : ctl->cycles_max;
        if (!ac->done) ctl->steps_unconv += 1;
        ctl->steps_done += 1;
        ac->done = 0;
        ac->sweeps = 0;
    }
}

// The colour means' share: c_ik = S_ik / S_i.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_adj_means(AdjArgs a) {
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    constexpr int NC = N * C;
    const double* tot = a.tot;  // S_ik [N*C], S_i [N], sum w I [C], area, flag (mass-weight units)
    const double area = tot[NC + N + C];
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < (int)n; t += gridDim.x * kBlock) {
        const int y = t / W, x = t - y * W;
        const uint32_t p = (uint32_t)t;
        const double w = mass_w(node_class(x, y, W, H));
        double ib[C];
#pragma unroll
        for (int k = 0; k < C; ++k) ib[k] = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double S = tot[NC + i];
            if (!(S > 1e-12 * area)) continue;
            const double un = gload(a.u0 + i * n, p);
            double du = 0.0;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const double cb = a.cbar64[i * C + k];
                ib[k] += cb * w * un / S;
                du += cb * w * ((double)gload(a.image + k * n, p) - a.c64[i * C + k]) / S;
            }
            gstore(a.ub_out + i * n, p, gload(a.ub_out + i * n, p) + (float)du);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) gstore(a.Ibar + k * n, p, gload(a.Ibar + k * n, p) + (float)ib[k]);
    }
}

__global__ void k_adj_init(AdjCtl* ac, double* grads) {
    if (threadIdx.x == 0) {
        ac->done = 0;
        ac->sweeps = 0;
        grads[0] = grads[1] = grads[2] = 0.0;
    }
}

int adj_blocks(int64_t work) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((work + kBlock - 1) / kBlock, kMgBlocks));
}

template <int N, int C>
hipError_t adj_nc(int op, const AdjArgs& a, int colour, int sweep, hipStream_t s) {
    const int64_t n = (int64_t)a.W * a.H;
    switch (op) {
        case kAdjSweep:
            hipLaunchKernelGGL((k_adj_sweep<N>), dim3(a.nblocks), dim3(kBlock), 0, s, a, sweep);
            break;
        case kAdjAccum:
            hipLaunchKernelGGL((k_adj_accum<N, C>), dim3(a.nblocks_acc), dim3(kBlock), 0, s, a);
            break;
        case kAdjReduce: hipLaunchKernelGGL((k_adj_reduce<N, C>), dim3(1), dim3(kBlock), 0, s, a); break;
        case kAdjMeans:
            hipLaunchKernelGGL((k_adj_means<N, C>), dim3(adj_blocks(n)), dim3(kBlock), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int N>
hipError_t adj_n(int C, int op, const AdjArgs& a, int colour, int sweep, hipStream_t s) {
    switch (C) {
        case 1: return adj_nc<N, 1>(op, a, colour, sweep, s);
        case 2: return adj_nc<N, 2>(op, a, colour, sweep, s);
        case 3: return adj_nc<N, 3>(op, a, colour, sweep, s);
        case 4: return adj_nc<N, 4>(op, a, colour, sweep, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int adj_sweep_blocks(int W, int H) { return std::min(adj_tiles(W, H), kMgBlocks); }
int adj_accum_blocks(int W, int H) { return adj_blocks((int64_t)W * H); }

hipError_t launch_adj(int N, int C, int op, const AdjArgs& a, int colour, int sweep, hipStream_t s) {
    switch (N) {
        case 2: return adj_n<2>(C, op, a, colour, sweep, s);
        case 3: return adj_n<3>(C, op, a, colour, sweep, s);
        case 4: return adj_n<4>(C, op, a, colour, sweep, s);
        case 5: return adj_n<5>(C, op, a, colour, sweep, s);
        case 6: return adj_n<6>(C, op, a, colour, sweep, s);
        case 7: return adj_n<7>(C, op, a, colour, sweep, s);
        case 8: return adj_n<8>(C, op, a, colour, sweep, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adj_init(AdjCtl* ac, double* grads, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_init, dim3(1), dim3(kWave), 0, s, ac, grads);
    return hipGetLastError();
}

}  // namespace acseg
