// kernels_fine.hip -- finest-level kernels of the Allen-Cahn segmentation step.
//
//   k_project   simplex projection of independent vectors
//   k_cmeans    colour means c_ik (eq. VV_fidelity, lumped mass), float64 sums
//   k_rhs       per-step right-hand side of eq. alpha in u units
//   k_smooth    red-black projected block Gauss-Seidel on LDS tiles
//   k_labels    argmax labels, composite and rounded composite
//   k_energy    discrete energy of eq. E
#include "acseg_internal.h"

namespace acseg {

// ---------------------------------------------------------------------------
// Projection of independent vectors (component-major [N][count])
// ---------------------------------------------------------------------------

template <int N>
__global__ __launch_bounds__(kBlock) void k_project(const float* y, float* x, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= count) return;
    float v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = y[i * count + t];
    project_simplex<N>(v);
#pragma unroll
    for (int i = 0; i < N; ++i) x[i * count + t] = v[i];
}

// ---------------------------------------------------------------------------
// Colour means: S_ik = sum_p w_p u_pi I_pk, S_i = sum_p w_p u_pi,
// SI_k = sum_p w_p I_pk, Sw = sum_p w_p; c_ik = S_ik / S_i.
// ---------------------------------------------------------------------------

struct CmeansArgs {
    const float* image;
    const float* u;  // explicit field, or NULL: bufs.b[ctl->cur]
    Bufs bufs;
    Ctl* ctl;
    const double* c_prev64;
    double* c64;
    float* c_out;
    double* partials;
    int W, H;
};

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_cmeans(CmeansArgs a) {
    constexpr int M = N * C + N + C + 2;  // S_ik, S_i, SI_k, Sw, non-finite count
    __shared__ double sh[kBlock / kWave][M];
    __shared__ double tot[M];
    __shared__ int flag;
    const float* u = a.u ? a.u : a.bufs.b[a.ctl->cur];
    const int64_t n = (int64_t)a.W * a.H;
    double acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / a.W), x = (int)(p - (int64_t)y * a.W);
        const double w = mass_w(node_class(x, y, a.W, a.H));
        float I[C];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            I[k] = a.image[k * n + p];
            bad |= !isfinite(I[k]);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double wu = w * (double)u[i * n + p];
            acc[N * C + i] += wu;
#pragma unroll
            for (int k = 0; k < C; ++k) acc[i * C + k] += wu * (double)I[k];
        }
#pragma unroll
        for (int k = 0; k < C; ++k) acc[N * C + N + k] += w * (double)I[k];
        acc[N * C + N + C] += w;
        acc[M - 1] += bad ? 1.0 : 0.0;
    }
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const double v = wave_sum(acc[m]);
        if (lane == 0) sh[wid][m] = v;
    }
    __syncthreads();
    if (threadIdx.x < M) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sh[w][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * M + threadIdx.x] = s;
    }
    if (!arrive_last(&a.ctl->arrive2, &flag)) return;
    if (threadIdx.x < M) {
        double s = 0.0;  // fixed order over blocks: deterministic
        for (int b = 0; b < (int)gridDim.x; ++b) s += a.partials[(int64_t)b * M + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double area = tot[N * C + N + C];
        int empty = 0;
        for (int i = 0; i < N; ++i) {
            const double S = tot[N * C + i];
            const bool has_mass = S > 1e-12 * area;
            empty |= has_mass ? 0 : 1;
            for (int k = 0; k < C; ++k) {
                double c;
                if (has_mass)
                    c = tot[i * C + k] / S;
                else if (a.c_prev64)
                    c = a.c_prev64[i * C + k];
                else
                    c = tot[N * C + N + k] / area;
                a.c64[i * C + k] = c;
                if (a.c_out) a.c_out[i * C + k] = (float)c;
            }
        }
        a.ctl->empty_now = empty;
        if (tot[M - 1] > 0.0) a.ctl->nonfinite = 1;
    }
}

// ---------------------------------------------------------------------------
// Right-hand side in u units: rhs'_pi = w_p [(1/tau + 2/eps) un_pi - lambda F_pi] / D_p,
// F_pi = sum_k (I_pk - c_ik)^2, evaluated in float64 and shifted per node so
// that max_i rhs'_pi = 0 (the simplex projection ignores per-node shifts).
// ---------------------------------------------------------------------------

struct RhsArgs {
    const float* image;
    Bufs bufs;
    Ctl* ctl;
    const double* c64;
    RhsCoef rc;
    float* rhs;
    int W, H;
};

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_rhs(RhsArgs a) {
    __shared__ double cs[N * C];
    if (threadIdx.x < N * C) cs[threadIdx.x] = a.c64[threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl->done = 0;
        a.ctl->cycles = 0;
    }
    __syncthreads();
    const float* u = a.bufs.b[a.ctl->cur];
    const int64_t n = (int64_t)a.W * a.H;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / a.W), x = (int)(p - (int64_t)y * a.W);
        const double wd = sel4d(a.rc.wd, node_class(x, y, a.W, a.H));
        double I[C];
#pragma unroll
        for (int k = 0; k < C; ++k) I[k] = (double)a.image[k * n + p];
        double r[N];
        double rmax = -1e300;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double F = 0.0;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const double d = I[k] - cs[i * C + k];
                F += d * d;
            }
            r[i] = wd * (a.rc.a * (double)u[i * n + p] - a.rc.lambda * F);
            rmax = fmax(rmax, r[i]);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) a.rhs[i * n + p] = (float)(r[i] - rmax);
    }
}

// ---------------------------------------------------------------------------
// Red-black projected block Gauss-Seidel on LDS tiles.
//
// A workgroup owns a TX x TY tile of the output and stages the tile plus a
// halo of R = 2K (+1 for the residual) nodes of every phase plane in LDS.  A
// half-sweep updates the nodes of one colour ((x+y) even = red) inside a
// region that shrinks by one node per half-sweep, so after K red/black sweeps
// the tile holds exactly what K global red-black sweeps produce.  Each node
// update is the exact minimisation of the step objective over the node's
// simplex block: y_p = rhs'_p + kappa_p sum_q c_pq u_q, u_p = Pi(y_p) (the
// block Hessian is D_p times the identity, so u_p's old value is not used).
// With RESID, one more red evaluation (not written) gives the natural
// residual of the output: black nodes have just been set from the final red
// values, so their residual is zero.
//
// LDS holds each row split into its even-x and odd-x halves, so a half-sweep
// touches consecutive LDS words across a wavefront.
// ---------------------------------------------------------------------------

struct SmoothArgs {
    Bufs bufs;
    Ctl* ctl;
    const float* rhs;
    float* partials;
    LevelCoef coef;
    float tol;
    int max_cycles;
    int W, H;
    int tiles_x;
};

template <int N, int K>
struct SmoothTile {
    static constexpr int TX = 64;
    static constexpr int R = 2 * K + 1;  // halo incl. the residual layer
    static constexpr int TY = (N <= 3) ? 32 : ((N * (TX + 2 * R) * (16 + 2 * R) * 4 <= 65536) ? 16 : 8);
    static constexpr int LX = TX + 2 * R;
    static constexpr int LY = TY + 2 * R;
    static constexpr int LDS_BYTES = N * LX * LY * 4;
    static_assert(LDS_BYTES <= 65536, "tile does not fit in 64 KiB of LDS");
};

template <int N, int K, bool RESID>
__global__ __launch_bounds__(kBlock) void k_smooth(SmoothArgs a) {
    using T = SmoothTile<N, K>;
    constexpr int TX = T::TX, TY = T::TY;
    constexpr int R = 2 * K + (RESID ? 1 : 0);
    constexpr int LX = TX + 2 * R, LY = TY + 2 * R, LXH = LX / 2, PL = LX * LY;
    extern __shared__ float lds[];
    __shared__ float red[kBlock / kWave];
    __shared__ int flag;

    Ctl* ctl = a.ctl;
    if (ctl->done) return;  // uniform: the step has converged
    const int cur = ctl->cur;
    const float* __restrict__ src = a.bufs.b[cur];
    float* __restrict__ dst = const_cast<float*>(a.bufs.b[out_of(cur)]);
    const float* __restrict__ rhs = a.rhs;
    const int W = a.W, H = a.H;
    const int64_t P = (int64_t)W * H;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int x0 = tx * TX - R, y0 = ty * TY - R;  // LDS origin; x0 + y0 is even

    for (int idx = threadIdx.x; idx < PL; idx += kBlock) {
        const int ly = idx / LX, lx = idx - ly * LX;
        const int gx = x0 + lx, gy = y0 + ly;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const int li = ly * LX + (lx & 1) * LXH + (lx >> 1);
        const int64_t g = (int64_t)gy * W + gx;
#pragma unroll
        for (int i = 0; i < N; ++i) lds[i * PL + li] = in ? src[i * P + g] : 0.f;
    }

    float res = 0.f;
    constexpr int NHALF = 2 * K + (RESID ? 1 : 0);
    for (int s = 0; s < NHALF; ++s) {
        const int colour = s & 1;
        const int r = R - 1 - s;
        __syncthreads();
        for (int pi = threadIdx.x; pi < LXH * LY; pi += kBlock) {
            const int ly = pi / LXH, j = pi - ly * LXH;
            const int par = (ly + colour) & 1;  // parity of lx for this colour
            const int lx = 2 * j + par;
            if (lx < R - r || lx >= R + TX + r || ly < R - r || ly >= R + TY + r) continue;
            const int gx = x0 + lx, gy = y0 + ly;
            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
            const float kap = sel4(a.coef.kappa, node_class(gx, gy, W, H));
            const float ch = edge_w_h(gy, H), cv = edge_w_v(gx, W);
            const int row = ly * LX;
            const int iL = par ? row + j : row + LXH + j - 1;
            const int iR = par ? row + j + 1 : row + LXH + j;
            const int iC = row + par * LXH + j;
            const int iU = iC - LX, iD = iC + LX;
            const int64_t g = (int64_t)gy * W + gx;
            float v[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float* L = lds + i * PL;
                const float S = ch * (L[iL] + L[iR]) + cv * (L[iU] + L[iD]);
                v[i] = rhs[i * P + g] + kap * S;
            }
            project_simplex<N>(v);
            if (RESID && s == NHALF - 1) {
#pragma unroll
                for (int i = 0; i < N; ++i) res = fmaxf(res, fabsf(v[i] - lds[i * PL + iC]));
            } else {
#pragma unroll
                for (int i = 0; i < N; ++i) lds[i * PL + iC] = v[i];
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < TX * TY; idx += kBlock) {
        const int oy = idx / TX, ox = idx - oy * TX;
        const int gx = x0 + R + ox, gy = y0 + R + oy;
        if (gx >= W || gy >= H) continue;
        const int lx = R + ox, ly = R + oy;
        const int li = ly * LX + (lx & 1) * LXH + (lx >> 1);
        const int64_t g = (int64_t)gy * W + gx;
#pragma unroll
        for (int i = 0; i < N; ++i) dst[i * P + g] = lds[i * PL + li];
    }

    const float bm = block_max(res, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = bm;
    if (!arrive_last(&ctl->arrive, &flag)) return;
    float rho = 0.f;
    if (RESID) {
        for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) rho = fmaxf(rho, a.partials[b]);
        rho = block_max(rho, red);
    }
    if (threadIdx.x == 0) {
        ctl->cur = out_of(cur);
        if (RESID) {
            ctl->resid = rho;
            const int c = ctl->cycles + 1;
            ctl->cycles = c;
            if (!(rho > a.tol) || c >= a.max_cycles) ctl->done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Control-block helpers
// ---------------------------------------------------------------------------

__global__ void k_ctl_init(Ctl* ctl, int cur) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctl c = {};
        c.cur = cur;
        *ctl = c;
    }
}

__global__ void k_step_end(Ctl* ctl, float tol) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int c = ctl->cycles;
    ctl->cycles_total += c;
    ctl->cycles_max = c > ctl->cycles_max ? c : ctl->cycles_max;
    if (ctl->resid > tol) ctl->steps_unconv += 1;
    ctl->max_resid = fmaxf(ctl->max_resid, ctl->resid);
    ctl->steps_done += 1;
    if (ctl->empty_now) ctl->empty_steps += 1;
}

__global__ __launch_bounds__(kBlock) void k_copy_current(Bufs bufs, Ctl* ctl, float* dst,
                                                         int64_t count) {
    const float* src = bufs.b[ctl->cur];
    if (src == dst) return;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * kBlock)
        dst[t] = src[t];
}

__global__ void k_widen(const float* src, double* dst, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = (double)src[t];
}

__global__ __launch_bounds__(kBlock) void k_fill(float* p, int64_t count, float v) {
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * kBlock)
        p[t] = v;
}

// ---------------------------------------------------------------------------
// Post-processing
// ---------------------------------------------------------------------------

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_labels(const float* u, const float* c, uint8_t* labels,
                                                   float* composite, float* rounded, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    float v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = u[i * n + p];
    int best = 0;
#pragma unroll
    for (int i = 1; i < N; ++i)
        if (v[i] > v[best]) best = i;
    if (labels) labels[p] = (uint8_t)best;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        if (composite) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < N; ++i) s += c[i * C + k] * v[i];
            composite[k * n + p] = s;
        }
        if (rounded) rounded[k * n + p] = c[best * C + k];
    }
}

// ---------------------------------------------------------------------------
// Energy of eq. E: interface eps/2 sum_edges c_e (u_p - u_q)^2, concave
// (h^2/eps) sum w u (1 - u), fitting lambda h^2 sum w u F(c).
// ---------------------------------------------------------------------------

struct EnergyArgs {
    const float* image;
    const float* u;
    const double* c64;
    double* partials;
    Ctl* ctl;
    double* energy;
    double eps, lambda, h;
    int W, H;
};

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a) {
    __shared__ double cs[N * C];
    __shared__ double sh[kBlock / kWave][3];
    __shared__ int flag;
    if (threadIdx.x < N * C) cs[threadIdx.x] = a.c64[threadIdx.x];
    __syncthreads();
    const int64_t n = (int64_t)a.W * a.H;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / a.W), x = (int)(p - (int64_t)y * a.W);
        const double w = mass_w(node_class(x, y, a.W, a.H));
        const double chh = (y == 0 || y == a.H - 1) ? 0.5 : 1.0;  // edge (x,y)-(x+1,y)
        const double cvv = (x == 0 || x == a.W - 1) ? 0.5 : 1.0;  // edge (x,y)-(x,y+1)
        double I[C];
#pragma unroll
        for (int k = 0; k < C; ++k) I[k] = (double)a.image[k * n + p];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double v = (double)a.u[i * n + p];
            if (x + 1 < a.W) {
                const double d = v - (double)a.u[i * n + p + 1];
                e0 += chh * d * d;
            }
            if (y + 1 < a.H) {
                const double d = v - (double)a.u[i * n + p + a.W];
                e0 += cvv * d * d;
            }
            e1 += w * v * (1.0 - v);
            double F = 0.0;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const double d = I[k] - cs[i * C + k];
                F += d * d;
            }
            e2 += w * v * F;
        }
    }
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    e0 = wave_sum(e0);
    e1 = wave_sum(e1);
    e2 = wave_sum(e2);
    if (lane == 0) {
        sh[wid][0] = e0;
        sh[wid][1] = e1;
        sh[wid][2] = e2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sh[w][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * 3 + threadIdx.x] = s;
    }
    if (!arrive_last(&a.ctl->arrive2, &flag)) return;
    if (threadIdx.x == 0) {
        double t[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < (int)gridDim.x; ++b)
            for (int m = 0; m < 3; ++m) t[m] += a.partials[(int64_t)b * 3 + m];
        const double h2 = a.h * a.h;
        a.energy[0] = 0.5 * a.eps * t[0];
        a.energy[1] = h2 / a.eps * t[1];
        a.energy[2] = a.lambda * h2 * t[2];
        a.energy[3] = a.energy[0] + a.energy[1] + a.energy[2];
    }
}

// ---------------------------------------------------------------------------
// Launchers: runtime N, C -> template instances
// ---------------------------------------------------------------------------

static int grid_for(int64_t n, int max_blocks) {
    int64_t b = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

hipError_t launch_project(int N, int64_t count, const float* y, float* x, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, y, x, count);
        return hipGetLastError();
    };
    switch (N) {
        case 2: return go(k_project<2>);
        case 3: return go(k_project<3>);
        case 4: return go(k_project<4>);
        case 5: return go(k_project<5>);
        case 6: return go(k_project<6>);
        case 7: return go(k_project<7>);
        case 8: return go(k_project<8>);
        default: return hipErrorInvalidValue;
    }
}

template <int N, int C>
static hipError_t run_cmeans(const CmeansArgs& a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cmeans<N, C>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int N>
static hipError_t cmeans_c(int C, const CmeansArgs& a, int blocks, hipStream_t s) {
    switch (C) {
        case 1: return run_cmeans<N, 1>(a, blocks, s);
        case 2: return run_cmeans<N, 2>(a, blocks, s);
        case 3: return run_cmeans<N, 3>(a, blocks, s);
        case 4: return run_cmeans<N, 4>(a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cmeans(int N, int C, int W, int H, const float* image, const float* u,
                         Bufs bufs, Ctl* ctl, const double* c_prev64, double* c64,
                         float* c_out, double* partials, int max_blocks, hipStream_t s) {
    CmeansArgs a{image, u, bufs, ctl, c_prev64, c64, c_out, partials, W, H};
    const int blocks = grid_for((int64_t)W * H, max_blocks);
    switch (N) {
        case 2: return cmeans_c<2>(C, a, blocks, s);
        case 3: return cmeans_c<3>(C, a, blocks, s);
        case 4: return cmeans_c<4>(C, a, blocks, s);
        case 5: return cmeans_c<5>(C, a, blocks, s);
        case 6: return cmeans_c<6>(C, a, blocks, s);
        case 7: return cmeans_c<7>(C, a, blocks, s);
        case 8: return cmeans_c<8>(C, a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N, int C>
static hipError_t run_rhs(const RhsArgs& a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_rhs<N, C>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int N>
static hipError_t rhs_c(int C, const RhsArgs& a, int blocks, hipStream_t s) {
    switch (C) {
        case 1: return run_rhs<N, 1>(a, blocks, s);
        case 2: return run_rhs<N, 2>(a, blocks, s);
        case 3: return run_rhs<N, 3>(a, blocks, s);
        case 4: return run_rhs<N, 4>(a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rhs(int N, int C, int W, int H, const float* image, Bufs bufs, Ctl* ctl,
                      const double* c64, RhsCoef rc, float* rhs, hipStream_t s) {
    RhsArgs a{image, bufs, ctl, c64, rc, rhs, W, H};
    const int blocks = grid_for((int64_t)W * H, 4096);
    switch (N) {
        case 2: return rhs_c<2>(C, a, blocks, s);
        case 3: return rhs_c<3>(C, a, blocks, s);
        case 4: return rhs_c<4>(C, a, blocks, s);
        case 5: return rhs_c<5>(C, a, blocks, s);
        case 6: return rhs_c<6>(C, a, blocks, s);
        case 7: return rhs_c<7>(C, a, blocks, s);
        case 8: return rhs_c<8>(C, a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N, int K, bool RESID>
static hipError_t run_smooth(SmoothArgs a, hipStream_t s) {
    using T = SmoothTile<N, K>;
    constexpr int R = 2 * K + (RESID ? 1 : 0);
    constexpr int lds = N * (T::TX + 2 * R) * (T::TY + 2 * R) * 4;
    a.tiles_x = (a.W + T::TX - 1) / T::TX;
    const int tiles_y = (a.H + T::TY - 1) / T::TY;
    hipLaunchKernelGGL((k_smooth<N, K, RESID>), dim3(a.tiles_x * tiles_y), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

template <int N>
static hipError_t smooth_n(int sweeps, bool resid, const SmoothArgs& a, hipStream_t s) {
    // split the sweeps into launches of at most 2 sweeps; only the last one
    // evaluates the residual and closes the cycle
    hipError_t e = hipSuccess;
    while (sweeps > 0 && e == hipSuccess) {
        const int k = sweeps >= 2 ? 2 : 1;
        sweeps -= k;
        const bool last = sweeps == 0 && resid;
        if (k == 2)
            e = last ? run_smooth<N, 2, true>(a, s) : run_smooth<N, 2, false>(a, s);
        else
            e = last ? run_smooth<N, 1, true>(a, s) : run_smooth<N, 1, false>(a, s);
    }
    return e;
}

hipError_t launch_smooth(int N, int W, int H, int sweeps, bool resid, Bufs bufs, Ctl* ctl,
                         const float* rhs, LevelCoef coef, float tol, int max_cycles,
                         float* partials, hipStream_t s) {
    SmoothArgs a{bufs, ctl, rhs, partials, coef, tol, max_cycles, W, H, 0};
    switch (N) {
        case 2: return smooth_n<2>(sweeps, resid, a, s);
        case 3: return smooth_n<3>(sweeps, resid, a, s);
        case 4: return smooth_n<4>(sweeps, resid, a, s);
        case 5: return smooth_n<5>(sweeps, resid, a, s);
        case 6: return smooth_n<6>(sweeps, resid, a, s);
        case 7: return smooth_n<7>(sweeps, resid, a, s);
        case 8: return smooth_n<8>(sweeps, resid, a, s);
        default: return hipErrorInvalidValue;
    }
}

int smooth_max_tiles(int W, int H) {
    // upper bound on the smoother's grid (smallest tile: 64 x 8)
    return ((W + 63) / 64) * ((H + 7) / 8);
}

hipError_t launch_step_end(Ctl* ctl, float tol, hipStream_t s) {
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, s, ctl, tol);
    return hipGetLastError();
}

hipError_t launch_ctl_init(Ctl* ctl, int cur, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, cur);
    return hipGetLastError();
}

hipError_t launch_copy_current(Bufs bufs, Ctl* ctl, float* dst, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_current, dim3(grid_for(count, 4096)), dim3(kBlock), 0, s, bufs, ctl,
                       dst, count);
    return hipGetLastError();
}

hipError_t launch_widen(const float* src, double* dst, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, dim3((count + 63) / 64), dim3(64), 0, s, src, dst, count);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t count, float v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count, 4096)), dim3(kBlock), 0, s, p, count, v);
    return hipGetLastError();
}

template <int N>
static hipError_t labels_c(int C, const float* u, const float* c, uint8_t* l, float* comp,
                           float* rnd, int64_t n, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    switch (C) {
        case 1: hipLaunchKernelGGL((k_labels<N, 1>), dim3(blocks), dim3(kBlock), 0, s, u, c, l, comp, rnd, n); break;
        case 2: hipLaunchKernelGGL((k_labels<N, 2>), dim3(blocks), dim3(kBlock), 0, s, u, c, l, comp, rnd, n); break;
        case 3: hipLaunchKernelGGL((k_labels<N, 3>), dim3(blocks), dim3(kBlock), 0, s, u, c, l, comp, rnd, n); break;
        case 4: hipLaunchKernelGGL((k_labels<N, 4>), dim3(blocks), dim3(kBlock), 0, s, u, c, l, comp, rnd, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_labels(int N, int C, int W, int H, const float* u, const float* c,
                         uint8_t* labels, float* composite, float* rounded, hipStream_t s) {
    const int64_t n = (int64_t)W * H;
    switch (N) {
        case 2: return labels_c<2>(C, u, c, labels, composite, rounded, n, s);
        case 3: return labels_c<3>(C, u, c, labels, composite, rounded, n, s);
        case 4: return labels_c<4>(C, u, c, labels, composite, rounded, n, s);
        case 5: return labels_c<5>(C, u, c, labels, composite, rounded, n, s);
        case 6: return labels_c<6>(C, u, c, labels, composite, rounded, n, s);
        case 7: return labels_c<7>(C, u, c, labels, composite, rounded, n, s);
        case 8: return labels_c<8>(C, u, c, labels, composite, rounded, n, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t energy_c(int C, const EnergyArgs& a, int blocks, hipStream_t s) {
    switch (C) {
        case 1: hipLaunchKernelGGL((k_energy<N, 1>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_energy<N, 2>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_energy<N, 3>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_energy<N, 4>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_energy(int N, int C, int W, int H, const float* image, const float* u,
                         const double* c64, double eps, double lambda, double h,
                         double* partials, int max_blocks, Ctl* ctl, double* energy,
                         hipStream_t s) {
    EnergyArgs a{image, u, c64, partials, ctl, energy, eps, lambda, h, W, H};
    const int blocks = grid_for((int64_t)W * H, max_blocks);
    switch (N) {
        case 2: return energy_c<2>(C, a, blocks, s);
        case 3: return energy_c<3>(C, a, blocks, s);
        case 4: return energy_c<4>(C, a, blocks, s);
        case 5: return energy_c<5>(C, a, blocks, s);
        case 6: return energy_c<6>(C, a, blocks, s);
        case 7: return energy_c<7>(C, a, blocks, s);
        case 8: return energy_c<8>(C, a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace acseg
