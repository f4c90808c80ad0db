// kernels_ssc.hip -- the paper's own multilevel iteration (Section "Multigrid
// Solution"): successive subspace correction over the basis functions of every
// coarse level, seen on the finest lattice, from the coarsest level to the
// finest, each correction kept on the Gibbs simplices as in Section "Gibbs
// Space Constraint Pseudocode".  No truncation: a coarse function moves every
// node of its support, so its step is bounded by the node that reaches zero
// first.
//
// One correction along eta (node (X, Y) of a level of spacing s = 2^sh finest
// nodes): u <- u + alpha eta with
//   g_i = sum_p eta_p (b - H u_i)_p,    Q = eta.H eta,
//   m_i = min_{eta_p > 0} u_pi / eta_p,
//   alpha = the point of {sum alpha = 0, alpha_i >= -m_i} nearest to g / Q,
// the exact minimiser of the step objective along eta over the feasible alpha
// (the objective is isotropic in alpha).  With beta = alpha + m that is the
// projection of g / Q + m onto {beta >= 0, sum beta = sum m}.
//
// Functions of one level whose nodes differ by 2 in x or y have supports at
// least two finest nodes apart, so no node of one is a 5-point neighbour of a
// node of the other: the four parity classes of (X, Y) are four launches, and
// the functions of one launch update in place without touching each other's
// reads.  The lanes serving a function stride over its support's bounding
// box, reduce, and all apply the same alpha.  By support size:
//   * small (levels 1-3): a group of 16 or 64 lanes per function, several
//     functions per workgroup, xor-butterfly reductions inside the group;
//   * medium (level 4): one workgroup per function;
//   * large (coarsest levels): a class holds few functions, so a function's
//     box is cut into chunks of rows: one launch writes each chunk's partial
//     sums, a second one recomputes alpha from all partials of the function
//     (the same order in every workgroup) and updates the chunk.
//
// Units as the multigrid path: the level is scaled by 1/h^2 of the finest
// spacing, the residual is D_p (y_p - u_p) with y_p the smoother's nodal map,
// and the stored right-hand side carries a per-node shift common to all
// phases, which moves g by a multiple of (1, ..., 1) and so leaves alpha
// unchanged.
#include <algorithm>

#include "acseg_internal.h"

namespace acseg {

namespace {

// eta of node (X, Y) of a level with Wc x Hc nodes and spacing 2^sh, at finest
// node (x, y): the P1 hat of that level's lattice, cells split along the
// (x,y)-(x+1,y+1) diagonal, so 1 - max(|dx|, |dy|) / s where dx and dy share
// a sign and 1 - (|dx| + |dy|) / s where they do not.  Finest nodes past the
// last row / column of the level take the value on it.  Exact in FP32.
__device__ __forceinline__ float hat_at(int x, int y, int X, int Y, int sh, int Wc, int Hc, float inv_s) {
    int dx = x - (X << sh), dy = y - (Y << sh);
    if (X == Wc - 1 && dx > 0) dx = 0;
    if (Y == Hc - 1 && dy > 0) dy = 0;
    const int ax = abs(dx), ay = abs(dy);
    const int t = ((dx >= 0) == (dy >= 0)) ? max(ax, ay) : ax + ay;
    const int s = 1 << sh;
    return t >= s ? 0.f : (float)(s - t) * inv_s;
}

// Butterflies inside a row of 16 lanes by DPP moves: quad_perm [1,0,3,2] and
// [2,3,0,1] (lane xor 1, xor 2), row_half_mirror (quads 0-1 and 2-3 swap) and
// row_mirror (the row's halves swap).  Each step adds the partner's value, so
// every lane of the row ends with the same sum (addition is commutative).
template <int CTRL>
__device__ __forceinline__ float dpp_row_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_row_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_row_d<0xB1>(v);
    v += dpp_row_d<0x4E>(v);
    v += dpp_row_d<0x141>(v);
    v += dpp_row_d<0x140>(v);
    return v;
}
__device__ __forceinline__ float row_min(float v) {
    v = fminf(v, dpp_row_f<0xB1>(v));
    v = fminf(v, dpp_row_f<0x4E>(v));
    v = fminf(v, dpp_row_f<0x141>(v));
    v = fminf(v, dpp_row_f<0x140>(v));
    return v;
}
// Minimum over the wave: the rows' minima, then the four rows read back (the
// minimum does not depend on the order).
__device__ __forceinline__ float wave_min_f(float v) {
    v = row_min(v);
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fminf(fminf(a, b), fminf(c, d));
}

// beta <- its projection onto {beta >= 0, sum beta = M} (M > 0): sort, then
// the largest threshold (S_k - M) / k over the k largest values.
template <int N>
__device__ __forceinline__ void project_scaled(float (&v)[N], float M) {
    float s[N];
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = v[i];
#pragma unroll
    for (int c = 0; c < SortNet<N>::n; ++c) {
        const int i = SortNet<N>::p[c][0], j = SortNet<N>::p[c][1];
        const float a = s[i], b = s[j];
        s[i] = fmaxf(a, b);
        s[j] = fminf(a, b);
    }
    float T = s[0] - M, thr = T;
#pragma unroll
    for (int k = 2; k <= N; ++k) {
        T += s[k - 1];
        thr = fmaxf(thr, T * (1.0f / (float)k));
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = fmaxf(v[i] - thr, 0.f);
}

// Function f of the launch's parity class and the bounding box of its support.
struct FunBox {
    int X, Y, x0, x1, y0, y1, bw;
};

__device__ __forceinline__ int class_count_x(const SscArgs& a) { return (a.Wc - (a.colour & 1) + 1) >> 1; }
__device__ __forceinline__ int class_count(const SscArgs& a) {
    return class_count_x(a) * ((a.Hc - (a.colour >> 1) + 1) >> 1);
}

__device__ __forceinline__ FunBox fun_box(const SscArgs& a, int f) {
    const int nx = class_count_x(a), fy = f / nx, sh = a.sh;
    FunBox b;
    b.X = (a.colour & 1) + 2 * (f - fy * nx);
    b.Y = (a.colour >> 1) + 2 * fy;
    b.x0 = max(0, ((b.X - 1) << sh) + 1);
    b.x1 = min(a.W - 1, ((b.X + 1) << sh) - 1);
    b.y0 = max(0, ((b.Y - 1) << sh) + 1);
    b.y1 = min(a.H - 1, ((b.Y + 1) << sh) - 1);
    b.bw = b.x1 - b.x0 + 1;
    return b;
}

__device__ __forceinline__ float* iterate_of(const SscArgs& a) {
    return const_cast<float*>(a.bufs.b[__builtin_amdgcn_readfirstlane(iterate_buf(a.ctl->cur, a.launch))]);
}

// A lane's share (box nodes t0, t0 + stride, ...) of g, Q = eta.H eta and m
// over box rows [ya, yb].
template <int N>
__device__ __forceinline__ void accumulate(const SscArgs& a, const float* u, const FunBox& b, int ya, int yb,
                                           double (&g)[N], double& q, float (&m)[N], int t0, int stride) {
    const int W = a.W, H = a.H, sh = a.sh, Wc = a.Wc, Hc = a.Hc;
    const uint32_t n = (uint32_t)W * (uint32_t)H;
    const float inv_s = 1.f / (float)(1 << sh);
    const int nbox = b.bw * (yb - ya + 1);
    for (int k = t0; k < nbox; k += stride) {
        const int yy = k / b.bw;
        const int y = ya + yy, x = b.x0 + (k - yy * b.bw);
        const float e = hat_at(x, y, b.X, b.Y, sh, Wc, Hc, inv_s);
        if (e <= 0.f) continue;
        const int cls = node_class(x, y, W, H);
        const float D = sel4(a.coef.d, cls), kap = sel4(a.coef.kappa, cls);
        const float wh = edge_w_h(y, H), wv = edge_w_v(x, W);
        const float ne = wh * ((x > 0 ? hat_at(x - 1, y, b.X, b.Y, sh, Wc, Hc, inv_s) : 0.f) +
                               (x < W - 1 ? hat_at(x + 1, y, b.X, b.Y, sh, Wc, Hc, inv_s) : 0.f)) +
                         wv * ((y > 0 ? hat_at(x, y - 1, b.X, b.Y, sh, Wc, Hc, inv_s) : 0.f) +
                               (y < H - 1 ? hat_at(x, y + 1, b.X, b.Y, sh, Wc, Hc, inv_s) : 0.f));
        q += (double)e * (double)(D * e - a.coef.e2 * ne);
        const uint32_t p = (uint32_t)y * (uint32_t)W + (uint32_t)x;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float* ui = u + (size_t)i * n;
            const float uc = gload(ui, p);
            const float nb = wh * ((x > 0 ? gload(ui, p - 1) : 0.f) + (x < W - 1 ? gload(ui, p + 1) : 0.f)) +
                             wv * ((y > 0 ? gload(ui, p - W) : 0.f) + (y < H - 1 ? gload(ui, p + W) : 0.f));
            const float yv = gload(a.rhs + (size_t)i * n, p) + kap * nb;
            g[i] += (double)e * (double)(D * (yv - uc));
            m[i] = fminf(m[i], uc / e);
        }
    }
}

// Workgroup reduction in a fixed order; every thread returns the same sums.
template <int N, int T>
__device__ __forceinline__ void reduce(double (&g)[N], double& q, float (&m)[N], double (*sh_g)[N + 1],
                                       float (*sh_m)[N]) {
    constexpr int kW = T / kWave;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    q = wave_sum(q);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        g[i] = wave_sum(g[i]);
        m[i] = wave_min_f(m[i]);
    }
    if (lane == 0) {
        sh_g[wid][N] = q;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            sh_g[wid][i] = g[i];
            sh_m[wid][i] = m[i];
        }
    }
    __syncthreads();
    q = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        g[i] = 0.0;
        m[i] = INFINITY;
    }
    for (int w = 0; w < kW; ++w) {
        q += sh_g[w][N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] += sh_g[w][i];
            m[i] = fminf(m[i], sh_m[w][i]);
        }
    }
    __syncthreads();  // the shared partials are reused
}

// alpha from the reduced sums; false when only alpha = 0 is feasible.
template <int N>
__device__ __forceinline__ bool step_of(const double (&g)[N], double q, const float (&m)[N], float (&al)[N]) {
    float M = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        al[i] = (float)(g[i] / q) + m[i];
        M += m[i];
    }
    if (!(M > 0.f) || !(q > 0.0)) return false;
    project_scaled<N>(al, M);
#pragma unroll
    for (int i = 0; i < N; ++i) al[i] -= m[i];
    return true;
}

// u += alpha eta over box rows [ya, yb] (a lane's share, as in accumulate).
template <int N>
__device__ __forceinline__ void apply(const SscArgs& a, float* u, const FunBox& b, int ya, int yb,
                                      const float (&al)[N], int t0, int stride) {
    const uint32_t n = (uint32_t)a.W * (uint32_t)a.H;
    const float inv_s = 1.f / (float)(1 << a.sh);
    const int nbox = b.bw * (yb - ya + 1);
    for (int k = t0; k < nbox; k += stride) {
        const int yy = k / b.bw;
        const int y = ya + yy, x = b.x0 + (k - yy * b.bw);
        const float e = hat_at(x, y, b.X, b.Y, a.sh, a.Wc, a.Hc, inv_s);
        if (e <= 0.f) continue;
        const uint32_t p = (uint32_t)y * (uint32_t)a.W + (uint32_t)x;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float* ui = u + (size_t)i * n;
            gstore(ui, p, fmaxf(fmaf(al[i], e, gload(ui, p)), 0.f));  // a bound met exactly may round below 0
        }
    }
}

// One workgroup per function: sums, alpha and update in one launch.
template <int N, int T>
__global__ __launch_bounds__(T) void k_ssc(SscArgs a) {
    __shared__ double sh_g[T / kWave][N + 1];
    __shared__ float sh_m[T / kWave][N];
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    float* u = iterate_of(a);
    const int nfun = class_count(a);
    for (int f = blockIdx.x; f < nfun; f += gridDim.x) {
        const FunBox b = fun_box(a, f);
        double g[N], q = 0.0;
        float m[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            m[i] = INFINITY;
        }
        accumulate<N>(a, u, b, b.y0, b.y1, g, q, m, threadIdx.x, T);
        reduce<N, T>(g, q, m, sh_g, sh_m);
        float al[N];
        if (!step_of<N>(g, q, m, al)) continue;
        apply<N>(a, u, b, b.y0, b.y1, al, threadIdx.x, T);
    }
}

// Large supports, two launches.  Item = (function, chunk of a.rows box rows),
// a.chunks chunks per function.  Partials per item: g[N], Q, m[N] (doubles).
template <int N, int T>
__global__ __launch_bounds__(T) void k_ssc_part(SscArgs a) {
    __shared__ double sh_g[T / kWave][N + 1];
    __shared__ float sh_m[T / kWave][N];
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    const float* u = iterate_of(a);
    const int items = class_count(a) * a.chunks;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int f = it / a.chunks, ch = it - f * a.chunks;
        const FunBox b = fun_box(a, f);
        const int ya = b.y0 + ch * a.rows, yb = min(b.y1, ya + a.rows - 1);
        double g[N], q = 0.0;
        float m[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            m[i] = INFINITY;
        }
        if (ya <= yb) accumulate<N>(a, u, b, ya, yb, g, q, m, threadIdx.x, T);
        reduce<N, T>(g, q, m, sh_g, sh_m);
        if (threadIdx.x == 0) {
            double* o = a.part + (size_t)it * (2 * N + 1);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                o[i] = g[i];
                o[N + 1 + i] = (double)m[i];
            }
            o[N] = q;
        }
    }
}

template <int N, int T>
__global__ __launch_bounds__(T) void k_ssc_apply(SscArgs a) {
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    float* u = iterate_of(a);
    const int items = class_count(a) * a.chunks;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int f = it / a.chunks, ch = it - f * a.chunks;
        const FunBox b = fun_box(a, f);
        const int ya = b.y0 + ch * a.rows, yb = min(b.y1, ya + a.rows - 1);
        if (ya > yb) continue;
        double g[N], q = 0.0;
        float m[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            m[i] = INFINITY;
        }
        const double* o = a.part + (size_t)f * a.chunks * (2 * N + 1);
        for (int c = 0; c < a.chunks; ++c, o += 2 * N + 1) {  // the function's chunks in order
            q += o[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                g[i] += o[i];
                m[i] = fminf(m[i], (float)o[N + 1 + i]);
            }
        }
        float al[N];
        if (!step_of<N>(g, q, m, al)) continue;
        apply<N>(a, u, b, ya, yb, al, threadIdx.x, T);
    }
}

// Small supports: G lanes per function (16: a DPP row, 64: the wave), 256 / G
// functions per workgroup, reduced inside the lane group so that each lane
// ends with the same sums.  The loop over functions is uniform across the
// workgroup so every lane takes part in the moves; lanes past the last
// function only contribute zeros.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 16 || G == 64, "a row or the wave");
    return G == 16 ? row_sum(v) : wave_sum(v);
}
template <int G>
__device__ __forceinline__ float group_min(float v) {
    static_assert(G == 16 || G == 64, "a row or the wave");
    return G == 16 ? row_min(v) : wave_min_f(v);
}

template <int N, int G>
__global__ __launch_bounds__(256) void k_ssc_small(SscArgs a) {
    constexpr int kPer = 256 / G;
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    float* u = iterate_of(a);
    const int nfun = class_count(a);
    const int grp = threadIdx.x / G, gl = threadIdx.x % G;
    for (int f0 = blockIdx.x * kPer; f0 < nfun; f0 += gridDim.x * kPer) {
        const int f = f0 + grp;
        const bool valid = f < nfun;
        const FunBox b = fun_box(a, valid ? f : f0);
        double g[N], q = 0.0;
        float m[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            m[i] = INFINITY;
        }
        if (valid) accumulate<N>(a, u, b, b.y0, b.y1, g, q, m, gl, G);
        q = group_sum<G>(q);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] = group_sum<G>(g[i]);
            m[i] = group_min<G>(m[i]);
        }
        float al[N];
        if (!valid || !step_of<N>(g, q, m, al)) continue;
        apply<N>(a, u, b, b.y0, b.y1, al, gl, G);
    }
}

template <int N>
hipError_t ssc_launch(const SscArgs& a, hipStream_t s) {
    const int cx = a.colour & 1, cy = a.colour >> 1;
    const int nfun = ((a.Wc - cx + 1) >> 1) * ((a.Hc - cy + 1) >> 1);
    if (nfun <= 0) return hipSuccess;
    if (a.part) {
        const int items = nfun * a.chunks;
        const int blocks = std::min(items, 1 << 20);
        hipLaunchKernelGGL((k_ssc_part<N, 256>), dim3(blocks), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_ssc_apply<N, 256>), dim3(blocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // box side 2^(sh+1) - 1: 3, 7, 15 nodes for sh = 1, 2, 3
    if (a.sh == 1) {
        hipLaunchKernelGGL((k_ssc_small<N, 16>), dim3(std::min((nfun + 15) / 16, 1 << 20)), dim3(256), 0, s, a);
    } else if (a.sh <= 3) {
        hipLaunchKernelGGL((k_ssc_small<N, 64>), dim3(std::min((nfun + 3) / 4, 1 << 20)), dim3(256), 0, s, a);
    } else {
        const int blocks = std::min(nfun, 1 << 20);
        if (a.sh == 4)
            hipLaunchKernelGGL((k_ssc<N, 256>), dim3(blocks), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_ssc<N, 1024>), dim3(blocks), dim3(1024), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ssc(int N, const SscArgs& a, hipStream_t s) {
    switch (N) {
        case 2: return ssc_launch<2>(a, s);
        case 3: return ssc_launch<3>(a, s);
        case 4: return ssc_launch<4>(a, s);
        case 5: return ssc_launch<5>(a, s);
        case 6: return ssc_launch<6>(a, s);
        case 7: return ssc_launch<7>(a, s);
        case 8: return ssc_launch<8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace acseg
