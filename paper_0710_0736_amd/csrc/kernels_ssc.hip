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
// reads.  One workgroup per function; its threads stride over the support's
// bounding box, reduce, and every thread applies the same alpha.
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

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
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

template <int N, int T>
__global__ __launch_bounds__(T) void k_ssc(SscArgs a) {
    constexpr int kW = T / kWave;
    __shared__ double sh_g[kW][N + 1];
    __shared__ float sh_m[kW][N];
    if (!a.fixed && a.ctl->step[a.slot].done) return;
    float* u = const_cast<float*>(a.bufs.b[__builtin_amdgcn_readfirstlane(iterate_buf(a.ctl->cur, a.launch))]);
    const int W = a.W, H = a.H, Wc = a.Wc, Hc = a.Hc, sh = a.sh;
    const uint32_t n = (uint32_t)W * (uint32_t)H;
    const int s = 1 << sh;
    const float inv_s = 1.f / (float)s;
    const int cx = a.colour & 1, cy = a.colour >> 1;
    const int nx = (Wc - cx + 1) >> 1, ny = (Hc - cy + 1) >> 1;
    const int nfun = nx * ny;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    for (int f = blockIdx.x; f < nfun; f += gridDim.x) {
        const int fy = f / nx;
        const int X = cx + 2 * (f - fy * nx), Y = cy + 2 * fy;
        const int x0 = max(0, ((X - 1) << sh) + 1), x1 = min(W - 1, ((X + 1) << sh) - 1);
        const int y0 = max(0, ((Y - 1) << sh) + 1), y1 = min(H - 1, ((Y + 1) << sh) - 1);
        const int bw = x1 - x0 + 1, nbox = bw * (y1 - y0 + 1);
        double g[N], q = 0.0;
        float m[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            m[i] = INFINITY;
        }
        for (int k = threadIdx.x; k < nbox; k += T) {
            const int yy = k / bw;
            const int y = y0 + yy, x = x0 + (k - yy * bw);
            const float e = hat_at(x, y, X, Y, sh, Wc, Hc, inv_s);
            if (e <= 0.f) continue;
            const int cls = node_class(x, y, W, H);
            const float D = sel4(a.coef.d, cls), kap = sel4(a.coef.kappa, cls);
            const float wh = edge_w_h(y, H), wv = edge_w_v(x, W);
            const float ne = wh * ((x > 0 ? hat_at(x - 1, y, X, Y, sh, Wc, Hc, inv_s) : 0.f) +
                                   (x < W - 1 ? hat_at(x + 1, y, X, Y, sh, Wc, Hc, inv_s) : 0.f)) +
                             wv * ((y > 0 ? hat_at(x, y - 1, X, Y, sh, Wc, Hc, inv_s) : 0.f) +
                                   (y < H - 1 ? hat_at(x, y + 1, X, Y, sh, Wc, Hc, inv_s) : 0.f));
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
        // workgroup reduction in a fixed order: every thread gets the same sums
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
        __syncthreads();  // the shared partials are reused by the next function
        float al[N], M = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            al[i] = (float)(g[i] / q) + m[i];
            M += m[i];
        }
        if (!(M > 0.f) || !(q > 0.0)) continue;  // only alpha = 0 is feasible
        project_scaled<N>(al, M);
#pragma unroll
        for (int i = 0; i < N; ++i) al[i] -= m[i];
        for (int k = threadIdx.x; k < nbox; k += T) {
            const int yy = k / bw;
            const int y = y0 + yy, x = x0 + (k - yy * bw);
            const float e = hat_at(x, y, X, Y, sh, Wc, Hc, inv_s);
            if (e <= 0.f) continue;
            const uint32_t p = (uint32_t)y * (uint32_t)W + (uint32_t)x;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float* ui = u + (size_t)i * n;
                gstore(ui, p, fmaxf(fmaf(al[i], e, gload(ui, p)), 0.f));  // a bound met exactly may round below 0
            }
        }
    }
}

template <int N>
hipError_t ssc_launch(const SscArgs& a, hipStream_t s) {
    const int cx = a.colour & 1, cy = a.colour >> 1;
    const int nfun = ((a.Wc - cx + 1) >> 1) * ((a.Hc - cy + 1) >> 1);
    if (nfun <= 0) return hipSuccess;
    const int blocks = std::min(nfun, 1 << 20);
    if (a.sh <= 2)
        hipLaunchKernelGGL((k_ssc<N, 64>), dim3(blocks), dim3(64), 0, s, a);
    else if (a.sh <= 4)
        hipLaunchKernelGGL((k_ssc<N, 256>), dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_ssc<N, 1024>), dim3(blocks), dim3(1024), 0, s, a);
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
