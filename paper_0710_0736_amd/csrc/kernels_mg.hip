// kernels_mg.hip -- the truncated multigrid correction of a time step
// (Section "Multigrid Solution"; truncation as motivated in Section "Gibbs
// Space Constraint Pseudocode": coarse corrections must not move components
// that sit on the constraint).
//
// One correction, between the pre- and post-smoothing sweeps of a cycle:
//   1. truncated defect  g~_p = T_I (b_p - (H u)_p) on the finest level, with
//      I_p = {i : u_pi > 0} and T_I zeroing the components outside I and
//      removing the mean over I from the others (0 when |I| <= 1);
//   2. r_1 = P^T g~ (transpose of the P1 prolongation of the nested lattices);
//   3. coarse levels: an approximate solve of the componentwise linear
//      problems H_l v = r_l (H_l rediscretised at spacing 2^l h) by a V-cycle
//      of red-black Gauss-Seidel sweeps; the levels whose longer side is at
//      most kTailSide run in one workgroup per component, entirely in LDS;
//   4. direction w_p = Pi(u_p + T_I (P v_1)_p) - u_p (feasible, since the
//      simplex is convex), and the exact line search on the step's quadratic
//      along w: alpha = clamp(<g~, w> / <w, H w>, 0, 1), u += alpha w.
//      w vanishes on the active components and sums to zero over the free
//      ones at every node, so <g, w> = <g~, w>; the truncated form keeps the
//      per-node multiplier of the sum constraint out of the dot product.
//
// Units: every level is scaled by 1/h^2 of the finest spacing; the defect is
// D_p (y_p - u_p) with y_p the nodal map of the smoother.  The stored
// right-hand side is shifted per node by a constant vector, which T_I removes.
#include <algorithm>

#include "acseg_internal.h"

namespace acseg {

constexpr int kTailThreads = 1024;

// ---------------------------------------------------------------------------
// Transfer operators of the nested lattices.  Coarse node (X, Y) coincides
// with fine node (2X, 2Y); every fine cell pair is split along the same
// (x,y)-(x+1,y+1) diagonal, so a fine node between two coarse nodes
// (horizontally, vertically or along that diagonal) takes the mean of the two.
// A fine node past the last coarse row / column (even fine side) takes the
// values of that row / column.  In "half coordinates" a = min(x, 2 Wc - 2).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float prolong_at(const float* __restrict__ vc, int Wc, int Hc, int x, int y) {
    const int a = min(x, 2 * Wc - 2), b = min(y, 2 * Hc - 2);
    const int X = a >> 1, Y = b >> 1;
    const float* r0 = vc + (int64_t)Y * Wc + X;
    const int ao = a & 1, bo = b & 1;
    if (!ao && !bo) return r0[0];
    if (ao && !bo) return 0.5f * (r0[0] + r0[1]);
    if (!ao && bo) return 0.5f * (r0[0] + r0[Wc]);
    return 0.5f * (r0[0] + r0[Wc + 1]);
}

// Visit the fine nodes that prolong_at lets coarse node (X, Y) reach, with
// their weights: f(x, y, weight).  The transpose of the prolongation is the
// weighted sum of a fine field over these visits.
template <class F>
__device__ __forceinline__ void for_restrict(int Wf, int Hf, int Wc, int Hc, int X, int Y, F&& f) {
#pragma unroll
    for (int db = -1; db <= 1; ++db) {
        const int b = 2 * Y + db;
        if (b < 0 || b > 2 * Hc - 2) continue;
        const int yn = (b == 2 * Hc - 2 && b + 1 < Hf) ? 2 : 1;
#pragma unroll
        for (int da = -1; da <= 1; ++da) {
            const int a = 2 * X + da;
            if (a < 0 || a > 2 * Wc - 2) continue;
            if (da != 0 && db != 0 && da != db) continue;  // not a neighbour along the split diagonal
            const float wt = (da == 0 && db == 0) ? 1.f : 0.5f;
            const int xn = (a == 2 * Wc - 2 && a + 1 < Wf) ? 2 : 1;
            for (int yy = 0; yy < yn; ++yy)
                for (int xx = 0; xx < xn; ++xx) f(a + xx, b + yy, wt);
        }
    }
}

// (P^T rf) at coarse node (X, Y).
__device__ __forceinline__ float restrict_at(const float* __restrict__ rf, int Wf, int Hf, int Wc,
                                             int Hc, int X, int Y) {
    float s = 0.f;
    for_restrict(Wf, Hf, Wc, Hc, X, Y, [&](int x, int y, float wt) { s += wt * rf[(int64_t)y * Wf + x]; });
    return s;
}

// Sum of the lattice neighbours of node (x, y) weighted by the edge weights
// c_pq (1/2 along the boundary), 0 for neighbours outside the lattice.
__device__ __forceinline__ float nb_sum(const float* __restrict__ v, int W, int H, int x, int y, int64_t p) {
    const float h = (x > 0 ? v[p - 1] : 0.f) + (x < W - 1 ? v[p + 1] : 0.f);
    const float vv = (y > 0 ? v[p - W] : 0.f) + (y < H - 1 ? v[p + W] : 0.f);
    return edge_w_h(y, H) * h + edge_w_v(x, W) * vv;
}

// nb_sum of v + P vc (vc on the coarse lattice Wc x Hc of this one).
__device__ __forceinline__ float nb_sum_prolonged(const float* __restrict__ v, const float* __restrict__ vc,
                                                  int W, int H, int Wc, int Hc, int x, int y, int64_t p) {
    const float l = x > 0 ? v[p - 1] + prolong_at(vc, Wc, Hc, x - 1, y) : 0.f;
    const float r = x < W - 1 ? v[p + 1] + prolong_at(vc, Wc, Hc, x + 1, y) : 0.f;
    const float d = y > 0 ? v[p - W] + prolong_at(vc, Wc, Hc, x, y - 1) : 0.f;
    const float u = y < H - 1 ? v[p + W] + prolong_at(vc, Wc, Hc, x, y + 1) : 0.f;
    return edge_w_h(y, H) * (l + r) + edge_w_v(x, W) * (d + u);
}

// The truncated defect g~_p = T_I (D (y_p(u) - u_p)) of node (x, y), N values.
template <int N>
__device__ __forceinline__ void trunc_defect(const MgArgs& a, const float* __restrict__ u, int x, int y,
                                             float (&g)[N]) {
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H, p = (int64_t)y * W + x;
    const int cls = node_class(x, y, W, H);
    const float kap = sel4(a.coef.kappa, cls), D = sel4(a.coef.d, cls);
    bool fr[N];
    float s = 0.f;
    int k = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float* ui = u + i * n;
        const float uc = ui[p];
        const float yv = a.rhs[i * n + p] + kap * nb_sum(ui, W, H, x, y, p);
        g[i] = D * (yv - uc);
        fr[i] = uc > 0.f;
        if (fr[i]) {
            s += g[i];
            ++k;
        }
    }
    const float mean = k > 0 ? s / (float)k : 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) g[i] = (k >= 2 && fr[i]) ? g[i] - mean : 0.f;
}

__device__ __forceinline__ bool step_done(const MgArgs& a) {
    return !a.fixed && a.ctl->step[a.slot].done;
}

__device__ __forceinline__ double block_sum_d(double v, double* sh /* kBlock/kWave */) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / kWave; ++w) r += sh[w];
    return r;
}

// ---------------------------------------------------------------------------
// Finest level
// ---------------------------------------------------------------------------

// 1-2. r_1 = P^T g~, coarse node by coarse node (the defect of a fine node is
// recomputed for each coarse node it reaches).
template <int N>
__global__ __launch_bounds__(kBlock) void k_mg_defect_restrict(MgArgs a) {
    if (step_done(a)) return;
    const float* __restrict__ u = a.bufs.b[__builtin_amdgcn_readfirstlane(iterate_buf(a.ctl->cur, a.launch))];
    const int Wc = a.Wc, Hc = a.Hc;
    const int64_t nc = (int64_t)Wc * Hc;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nc; p += (int64_t)gridDim.x * kBlock) {
        const int Y = (int)(p / Wc), X = (int)(p - (int64_t)Y * Wc);
        float r[N];
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = 0.f;
        for_restrict(a.W, a.H, Wc, Hc, X, Y, [&](int x, int y, float wt) {
            float g[N];
            trunc_defect<N>(a, u, x, y, g);
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] += wt * g[i];
        });
#pragma unroll
        for (int i = 0; i < N; ++i) a.r1[i * nc + p] = r[i];
    }
}

// 4a. w = Pi(u + T_I P v_1) - u into a.gt, block partials of <g~, w> (g~ recomputed).
template <int N>
__global__ __launch_bounds__(kBlock) void k_mg_dir(MgArgs a) {
    __shared__ double sh[kBlock / kWave];
    if (step_done(a)) return;
    const float* __restrict__ u = a.bufs.b[__builtin_amdgcn_readfirstlane(iterate_buf(a.ctl->cur, a.launch))];
    const int W = a.W, H = a.H, Wc = a.Wc, Hc = a.Hc;
    const int64_t n = (int64_t)W * H, nc = (int64_t)Wc * Hc;
    double gw = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        float uc[N], v[N];
        int k = 0;
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            uc[i] = u[i * n + p];
            v[i] = prolong_at(a.v1 + i * nc, Wc, Hc, x, y);
            if (uc[i] > 0.f) {
                s += v[i];
                ++k;
            }
        }
        float g[N];
        trunc_defect<N>(a, u, x, y, g);
        float w[N];
        if (k >= 2) {
            const float mean = s / (float)k;
            float xv[N];
#pragma unroll
            for (int i = 0; i < N; ++i) xv[i] = uc[i] + (uc[i] > 0.f ? v[i] - mean : 0.f);
            project_simplex<N>(xv);
#pragma unroll
            for (int i = 0; i < N; ++i) w[i] = xv[i] - uc[i];
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) w[i] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            gw += (double)g[i] * (double)w[i];
            a.gt[i * n + p] = w[i];
        }
    }
    const double t = block_sum_d(gw, sh);
    if (threadIdx.x == 0) a.part[blockIdx.x] = t;
}

// 4b. block partials of <w, H w>.
template <int N>
__global__ __launch_bounds__(kBlock) void k_mg_whw(MgArgs a) {
    __shared__ double sh[kBlock / kWave];
    if (step_done(a)) return;
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const float D = sel4(a.coef.d, node_class(x, y, W, H));
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float* wi = a.gt + i * n;
            const float wc = wi[p];
            const float hw = D * wc - a.coef.e2 * nb_sum(wi, W, H, x, y, p);
            acc += (double)wc * (double)hw;
        }
    }
    const double t = block_sum_d(acc, sh);
    if (threadIdx.x == 0) a.part[kMgBlocks + blockIdx.x] = t;
}

// 4c. alpha from the partials (one workgroup, fixed order).
__global__ __launch_bounds__(kBlock) void k_mg_alpha(MgArgs a) {
    __shared__ double sh[kBlock / kWave];
    if (step_done(a)) return;
    double g = 0.0, q = 0.0;
    for (int b = threadIdx.x; b < a.nblocks; b += kBlock) {
        g += a.part[b];
        q += a.part[kMgBlocks + b];
    }
    const double gt = block_sum_d(g, sh);
    __syncthreads();
    const double qt = block_sum_d(q, sh);
    if (threadIdx.x == 0) a.ctl->alpha = (qt > 0.0 && gt > 0.0) ? fmin(gt / qt, 1.0) : 0.0;
}

// 4d. u += alpha w (in place: the iterate buffer of the cycle).
template <int N>
__global__ __launch_bounds__(kBlock) void k_mg_update(MgArgs a) {
    if (step_done(a)) return;
    const float alpha = (float)a.ctl->alpha;
    if (alpha == 0.f) return;
    float* __restrict__ u = const_cast<float*>(a.bufs.b[__builtin_amdgcn_readfirstlane(iterate_buf(a.ctl->cur, a.launch))]);
    const int64_t total = (int64_t)N * a.W * a.H;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock)
        u[t] = fmaxf(u[t] + alpha * a.gt[t], 0.f);
}

// ---------------------------------------------------------------------------
// Coarse levels in global memory (levels too large for the LDS tail)
// ---------------------------------------------------------------------------

// dst (coarse) = P^T src (fine), N planes.
template <int N>
__global__ __launch_bounds__(kBlock) void k_restrict(CoarseArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    const int64_t nf = (int64_t)a.Wf * a.Hf, nc = (int64_t)a.W * a.H;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nc; p += (int64_t)gridDim.x * kBlock) {
        const int Y = (int)(p / a.W), X = (int)(p - (int64_t)Y * a.W);
#pragma unroll
        for (int i = 0; i < N; ++i) a.dst[i * nc + p] = restrict_at(a.src + i * nf, a.Wf, a.Hf, a.W, a.H, X, Y);
    }
}

// v (fine level of the pair) += P vc, N planes.
template <int N>
__global__ __launch_bounds__(kBlock) void k_prolong_add(CoarseArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    const int64_t nf = (int64_t)a.Wf * a.Hf, nc = (int64_t)a.W * a.H;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nf; p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / a.Wf), x = (int)(p - (int64_t)y * a.Wf);
#pragma unroll
        for (int i = 0; i < N; ++i) a.dst[i * nf + p] += prolong_at(a.src + i * nc, a.W, a.H, x, y);
    }
}

// One red (colour 0) or black (colour 1) half-sweep of linear Gauss-Seidel on
// H_l v = r: v_p = r_p / D_p + kappa_p sum_q c_pq v_q.  With `zero` the other
// colour is taken as 0 (the first half-sweep from v = 0).
template <int N>
__global__ __launch_bounds__(kBlock) void k_lin_half(CoarseArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    const int W = a.W, H = a.H, hw = (W + 1) / 2;
    const int64_t n = (int64_t)W * H, nh = (int64_t)hw * H;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nh; t += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(t / hw), j = (int)(t - (int64_t)y * hw);
        const int x = 2 * j + ((y + a.colour) & 1);
        if (x >= W) continue;
        const int64_t p = (int64_t)y * W + x;
        const int cls = node_class(x, y, W, H);
        const float kap = sel4(a.coef.kappa, cls), invd = sel4(a.coef.inv_d, cls);
        const int Wc = (W + 1) / 2, Hc = (H + 1) / 2;
        const int64_t nc = (int64_t)Wc * Hc;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float s = a.src[i * n + p] * invd;
            if (a.aux)  // the neighbours' values plus the prolonged coarse correction
                s += kap * nb_sum_prolonged(a.dst + i * n, a.aux + i * nc, W, H, Wc, Hc, x, y, p);
            else if (!a.zero)
                s += kap * nb_sum(a.dst + i * n, W, H, x, y, p);
            a.dst[i * n + p] = s;
        }
    }
}

// res = r - H_l v.
template <int N>
__global__ __launch_bounds__(kBlock) void k_lin_resid(CoarseArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    const int W = a.W, H = a.H;
    const int64_t n = (int64_t)W * H;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const float D = sel4(a.coef.d, node_class(x, y, W, H));
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float* v = a.aux + i * n;
            a.res[i * n + p] = a.src[i * n + p] - (D * v[p] - a.coef.e2 * nb_sum(v, W, H, x, y, p));
        }
    }
}

// dst (level of (W, H)) = P^T (r - H v) of the finer level (Wf, Hf): src = r,
// aux = v of the finer level, coef of the finer level in a.coef.
template <int N>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(CoarseArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    const int Wf = a.Wf, Hf = a.Hf;
    const int64_t nf = (int64_t)Wf * Hf, nc = (int64_t)a.W * a.H;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nc; p += (int64_t)gridDim.x * kBlock) {
        const int Y = (int)(p / a.W), X = (int)(p - (int64_t)Y * a.W);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float* v = a.aux + i * nf;
            const float* r = a.src + i * nf;
            float s = 0.f;
            for_restrict(Wf, Hf, a.W, a.H, X, Y, [&](int x, int y, float wt) {
                const int64_t q = (int64_t)y * Wf + x;
                const float D = sel4(a.coef.d, node_class(x, y, Wf, Hf));
                s += wt * (r[q] - (D * v[q] - a.coef.e2 * nb_sum(v, Wf, Hf, x, y, q)));
            });
            a.dst[i * nc + p] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// LDS tail: the V-cycle over levels t0..L-1 (longer side <= kTailSide), one
// workgroup per component.  r_{t0} is read from and v_{t0} written to global
// memory; every other array lives in LDS.
// ---------------------------------------------------------------------------

__device__ void tail_half(float* v, const float* r, int W, int H, const LevelCoef& c, int colour, bool zero) {
    const int hw = (W + 1) / 2, nh = hw * H;
    for (int t = threadIdx.x; t < nh; t += kTailThreads) {
        const int y = t / hw, j = t - y * hw;
        const int x = 2 * j + ((y + colour) & 1);
        if (x >= W) continue;
        const int p = y * W + x;
        const int cls = node_class(x, y, W, H);
        float s = r[p] * sel4(c.inv_d, cls);
        if (!zero) s += sel4(c.kappa, cls) * nb_sum(v, W, H, x, y, p);
        v[p] = s;
    }
    __syncthreads();
}

__device__ void tail_sweeps(float* v, const float* r, int W, int H, const LevelCoef& c, int sweeps, bool zero) {
    for (int s = 0; s < sweeps; ++s) {
        tail_half(v, r, W, H, c, 0, zero && s == 0);
        tail_half(v, r, W, H, c, 1, false);
    }
}

__global__ __launch_bounds__(kTailThreads) void k_coarse_tail(TailArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int i = blockIdx.x;  // component
    const TailLevel* lv = a.lv;
    float* res = lds + a.off_res;
    {
        const int n0 = lv[0].W * lv[0].H;
        const float* src = a.r_in + (int64_t)i * n0;
        for (int t = threadIdx.x; t < n0; t += kTailThreads) lds[lv[0].off_r + t] = src[t];
        __syncthreads();
    }
    for (int l = 0; l + 1 < a.nl; ++l) {  // down
        const int W = lv[l].W, H = lv[l].H;
        float* v = lds + lv[l].off_v;
        const float* r = lds + lv[l].off_r;
        tail_sweeps(v, r, W, H, a.coef[l], a.nu_pre, true);
        for (int p = threadIdx.x; p < W * H; p += kTailThreads) {
            const int y = p / W, x = p - y * W;
            const float D = sel4(a.coef[l].d, node_class(x, y, W, H));
            res[p] = r[p] - (D * v[p] - a.coef[l].e2 * nb_sum(v, W, H, x, y, p));
        }
        __syncthreads();
        const int Wc = lv[l + 1].W, Hc = lv[l + 1].H;
        float* rc = lds + lv[l + 1].off_r;
        for (int p = threadIdx.x; p < Wc * Hc; p += kTailThreads) {
            const int Y = p / Wc, X = p - Y * Wc;
            rc[p] = restrict_at(res, W, H, Wc, Hc, X, Y);
        }
        __syncthreads();
    }
    {
        const int l = a.nl - 1;
        tail_sweeps(lds + lv[l].off_v, lds + lv[l].off_r, lv[l].W, lv[l].H, a.coef[l], a.coarse_sweeps, true);
    }
    for (int l = a.nl - 2; l >= 0; --l) {  // up
        const int W = lv[l].W, H = lv[l].H, Wc = lv[l + 1].W, Hc = lv[l + 1].H;
        float* v = lds + lv[l].off_v;
        const float* vc = lds + lv[l + 1].off_v;
        for (int p = threadIdx.x; p < W * H; p += kTailThreads) {
            const int y = p / W, x = p - y * W;
            v[p] += prolong_at(vc, Wc, Hc, x, y);
        }
        __syncthreads();
        tail_sweeps(v, lds + lv[l].off_r, W, H, a.coef[l], a.nu_post, false);
    }
    const int n0 = lv[0].W * lv[0].H;
    float* dst = a.v_out + (int64_t)i * n0;
    for (int t = threadIdx.x; t < n0; t += kTailThreads) dst[t] = lds[lv[0].off_v + t];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

namespace {

int grid_for(int64_t work) {
    const int64_t b = (work + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMgBlocks));
}

template <int N>
hipError_t mg_fine(int op, const MgArgs& a, hipStream_t s) {
    const int g = a.nblocks;
    switch (op) {
        case kMgDefectRestrict:
            hipLaunchKernelGGL((k_mg_defect_restrict<N>), dim3(grid_for((int64_t)a.Wc * a.Hc)), dim3(kBlock), 0, s, a);
            break;
        case kMgDir: hipLaunchKernelGGL((k_mg_dir<N>), dim3(g), dim3(kBlock), 0, s, a); break;
        case kMgWhw: hipLaunchKernelGGL((k_mg_whw<N>), dim3(g), dim3(kBlock), 0, s, a); break;
        case kMgAlpha: hipLaunchKernelGGL(k_mg_alpha, dim3(1), dim3(kBlock), 0, s, a); break;
        case kMgUpdate: hipLaunchKernelGGL((k_mg_update<N>), dim3(grid_for((int64_t)N * a.W * a.H)), dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int N>
hipError_t mg_coarse(int op, const CoarseArgs& a, hipStream_t s) {
    switch (op) {
        case kCoarseRestrict:
            hipLaunchKernelGGL((k_restrict<N>), dim3(grid_for((int64_t)a.W * a.H)), dim3(kBlock), 0, s, a);
            break;
        case kCoarseProlongAdd:
            hipLaunchKernelGGL((k_prolong_add<N>), dim3(grid_for((int64_t)a.Wf * a.Hf)), dim3(kBlock), 0, s, a);
            break;
        case kCoarseHalf:
            hipLaunchKernelGGL((k_lin_half<N>), dim3(grid_for((int64_t)(a.W + 1) / 2 * a.H)), dim3(kBlock), 0, s, a);
            break;
        case kCoarseResid:
            hipLaunchKernelGGL((k_lin_resid<N>), dim3(grid_for((int64_t)a.W * a.H)), dim3(kBlock), 0, s, a);
            break;
        case kCoarseResidRestrict:
            hipLaunchKernelGGL((k_resid_restrict<N>), dim3(grid_for((int64_t)a.W * a.H)), dim3(kBlock), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int mg_blocks(int W, int H) { return grid_for((int64_t)W * H); }

hipError_t launch_mg_fine(int N, int op, const MgArgs& a, hipStream_t s) {
    switch (N) {
        case 2: return mg_fine<2>(op, a, s);
        case 3: return mg_fine<3>(op, a, s);
        case 4: return mg_fine<4>(op, a, s);
        case 5: return mg_fine<5>(op, a, s);
        case 6: return mg_fine<6>(op, a, s);
        case 7: return mg_fine<7>(op, a, s);
        case 8: return mg_fine<8>(op, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mg_coarse(int N, int op, const CoarseArgs& a, hipStream_t s) {
    switch (N) {
        case 2: return mg_coarse<2>(op, a, s);
        case 3: return mg_coarse<3>(op, a, s);
        case 4: return mg_coarse<4>(op, a, s);
        case 5: return mg_coarse<5>(op, a, s);
        case 6: return mg_coarse<6>(op, a, s);
        case 7: return mg_coarse<7>(op, a, s);
        case 8: return mg_coarse<8>(op, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_coarse_tail(int N, const TailArgs& a, size_t lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_tail, dim3(N), dim3(kTailThreads), lds_bytes, s, a);
    return hipGetLastError();
}

// Transfer operators on their own (no control block), `planes` plane sets.
namespace {
__global__ __launch_bounds__(kBlock) void k_transfer(int dir, int planes, const float* src, float* dst,
                                                      int Wf, int Hf, int Wc, int Hc) {
    const int64_t nf = (int64_t)Wf * Hf, nc = (int64_t)Wc * Hc;
    const int64_t n = dir == 0 ? nf : nc;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) {
        for (int i = 0; i < planes; ++i) {
            if (dir == 0) {
                const int y = (int)(p / Wf), x = (int)(p - (int64_t)y * Wf);
                dst[i * nf + p] = prolong_at(src + i * nc, Wc, Hc, x, y);
            } else {
                const int Y = (int)(p / Wc), X = (int)(p - (int64_t)Y * Wc);
                dst[i * nc + p] = restrict_at(src + i * nf, Wf, Hf, Wc, Hc, X, Y);
            }
        }
    }
}
}  // namespace

hipError_t launch_transfer(int planes, int dir, const float* src, float* dst, int Wf, int Hf, hipStream_t s) {
    const int Wc = (Wf + 1) / 2, Hc = (Hf + 1) / 2;
    const int64_t n = dir == 0 ? (int64_t)Wf * Hf : (int64_t)Wc * Hc;
    if (n == 0 || planes < 1) return hipSuccess;
    hipLaunchKernelGGL(k_transfer, dim3(grid_for(n)), dim3(kBlock), 0, s, dir, planes, src, dst, Wf, Hf, Wc, Hc);
    return hipGetLastError();
}

}  // namespace acseg
