// kernels_fine.hip -- finest-level kernels of the Allen-Cahn segmentation step.
//
//   k_project   simplex projection of independent vectors
//   k_cmeans    colour means c_ik (eq. VV_fidelity, lumped mass), float64 sums
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
    const Ctl* ctl;
    double* partials;  // [gridDim.y][gridDim.x][cmeans_width(N, C)]
    int W, H;
    int64_t u_stride;  // floats from one explicit field to the next (grid row y: u + y u_stride)
};

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_cmeans(CmeansArgs a) {
    constexpr int M = N * C + N + C + 2;  // S_ik, S_i, SI_k, Sw, non-finite count
    __shared__ double sh[kBlock / kWave][M];
    const float* u = a.u ? a.u + blockIdx.y * a.u_stride : a.bufs.b[__builtin_amdgcn_readfirstlane(a.ctl->cur)];
    a.partials += (int64_t)blockIdx.y * gridDim.x * M;
    const int64_t n = (int64_t)a.W * a.H;
    double acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    // no stores in the loop: unrolled, the loads of several nodes issue together
#pragma unroll 4
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
}

struct CmeansFinArgs {
    const double* partials;
    int nb;
    Ctl* ctl;
    const double* c_prev64;
    double* c64;
    float* c_out;
    double* tot_out;  // reduced sums, or NULL
};

// One block: finish the colour means from k_cmeans' partials.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_cmeans_finish(CmeansFinArgs a) {
    constexpr int M = N * C + N + C + 2;
    __shared__ double sh[kBlock / kWave][M];
    __shared__ double tot[M];
    reduce_rows<M>(a.partials, a.nb, tot, sh);
    if (a.tot_out && threadIdx.x < M) a.tot_out[threadIdx.x] = tot[threadIdx.x];
    if (threadIdx.x == 0) {
        double c[N * C];
        const int empty = finish_means<N, C>(tot, a.c_prev64, c);
        for (int m = 0; m < N * C; ++m) {
            a.c64[m] = c[m];
            if (a.c_out) a.c_out[m] = (float)c[m];
        }
        a.ctl->empty_now = empty;
        if (tot[M - 1] > 0.0) a.ctl->nonfinite = 1;
    }
}

// One workgroup per field of a k_cmeans launch over several fields: its
// reduced sums into tot[y][kCmeansMaxM].
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_cmeans_tot(const double* partials, int nb, double* tot) {
    constexpr int M = N * C + N + C + 2;
    __shared__ double sh[kBlock / kWave][M];
    __shared__ double t[M];
    reduce_rows<M>(partials + (int64_t)blockIdx.x * nb * M, nb, t, sh);
    if (threadIdx.x < M) tot[(int64_t)blockIdx.x * kCmeansMaxM + threadIdx.x] = t[threadIdx.x];
}

// One thread: the means of fields first..first+count-1 from their reduced
// sums, in order, an empty phase keeping the previous field's mean (the first
// field's previous means: c64 of field first - 1, or the mean image colour
// when first is 0).
// (The sums and means pass through LDS: the one thread that walks the
// fields then waits on no memory.)  count <= kCmeansFields.
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_cmeans_chain(const double* tot, int first, int count, Ctl* ctl,
                                                         double* c64) {
    constexpr int M = N * C + N + C + 2;
    __shared__ double ts[kCmeansFields][M];
    __shared__ double cs[kCmeansFields + 1][N * C];
    for (int q = threadIdx.x; q < count * M; q += kBlock) {
        const int f = q / M, m = q - f * M;
        ts[f][m] = tot[(int64_t)(first + f) * kCmeansMaxM + m];
    }
    if (first > 0 && threadIdx.x < N * C) cs[0][threadIdx.x] = c64[(int64_t)(first - 1) * kNC + threadIdx.x];
    __syncthreads();
    // thread i C + k follows c_ik through the fields (a phase's chain does
    // not depend on the other phases)
    if (threadIdx.x < N * C) {
        const int i = threadIdx.x / C, k = threadIdx.x - i * C;
        for (int f = 0; f < count; ++f) {
            const double* t = ts[f];
            const double area = t[N * C + N + C], S = t[N * C + i];
            cs[f + 1][threadIdx.x] = S > 1e-12 * area
                                         ? t[i * C + k] / S
                                         : ((first + f) > 0 ? cs[f][threadIdx.x] : t[N * C + N + k] / area);
        }
    }
    if (threadIdx.x == 0) {
        const double* t = ts[count - 1];
        int empty = 0, bad = 0;
        for (int i = 0; i < N; ++i) empty |= t[N * C + i] > 1e-12 * t[N * C + N + C] ? 0 : 1;
        for (int f = 0; f < count; ++f) bad |= ts[f][M - 1] > 0.0 ? 1 : 0;
        ctl->empty_now = empty;
        if (bad) ctl->nonfinite = 1;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < count * N * C; q += kBlock) {
        const int f = q / (N * C), m = q - f * (N * C);
        c64[(int64_t)(first + f) * kNC + m] = cs[f + 1][m];
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

__global__ __launch_bounds__(kBlock) void k_copy_current(Bufs bufs, const Ctl* ctl, float* dst,
                                                         int64_t count) {
    const float* src = bufs.b[__builtin_amdgcn_readfirstlane(ctl->cur)];
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
    double* partials;  // [gridDim.x][3]
    int W, H;
};

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a) {
    __shared__ double cs[N * C];
    __shared__ double sh[kBlock / kWave][3];
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
}

// One block: energy parts from k_energy's partials.
__global__ __launch_bounds__(kBlock) void k_energy_finish(const double* partials, int nb,
                                                          double eps, double lambda, double h,
                                                          double* energy) {
    __shared__ double sh[kBlock / kWave][3];
    __shared__ double tot[3];
    reduce_rows<3>(partials, nb, tot, sh);
    if (threadIdx.x == 0) {
        const double h2 = h * h;
        energy[0] = 0.5 * eps * tot[0];
        energy[1] = h2 / eps * tot[1];
        energy[2] = lambda * h2 * tot[2];
        energy[3] = energy[0] + energy[1] + energy[2];
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

// Runtime N (2..8) and C (1..4) to template instances.
template <template <int, int> class F, class... A>
static hipError_t dispatch_nc(int N, int C, A&&... args) {
#define ACSEG_NC(n)                                          \
    case n:                                                  \
        switch (C) {                                         \
            case 1: return F<n, 1>::run(args...);            \
            case 2: return F<n, 2>::run(args...);            \
            case 3: return F<n, 3>::run(args...);            \
            case 4: return F<n, 4>::run(args...);            \
            default: return hipErrorInvalidValue;            \
        }
    switch (N) {
        ACSEG_NC(2) ACSEG_NC(3) ACSEG_NC(4) ACSEG_NC(5) ACSEG_NC(6) ACSEG_NC(7) ACSEG_NC(8)
        default: return hipErrorInvalidValue;
    }
#undef ACSEG_NC
}

template <template <int> class F, class... A>
static hipError_t dispatch_n(int N, A&&... args) {
    switch (N) {
        case 2: return F<2>::run(args...);
        case 3: return F<3>::run(args...);
        case 4: return F<4>::run(args...);
        case 5: return F<5>::run(args...);
        case 6: return F<6>::run(args...);
        case 7: return F<7>::run(args...);
        case 8: return F<8>::run(args...);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
struct ProjectRun {
    static hipError_t run(int64_t count, const float* y, float* x, hipStream_t s) {
        const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_project<N>, dim3(blocks), dim3(kBlock), 0, s, y, x, count);
        return hipGetLastError();
    }
};

hipError_t launch_project(int N, int64_t count, const float* y, float* x, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    return dispatch_n<ProjectRun>(N, count, y, x, s);
}

int cmeans_width(int N, int C) { return N * C + N + C + 2; }

int cmeans_blocks(int W, int H) { return grid_for((int64_t)W * H, kCmeansBlocks); }

template <int N, int C>
struct CmeansRun {
    static hipError_t run(const CmeansArgs& a, int blocks, hipStream_t s) {
        hipLaunchKernelGGL((k_cmeans<N, C>), dim3(blocks), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
};

hipError_t launch_cmeans(int N, int C, int W, int H, const float* image, const float* u,
                         Bufs bufs, const Ctl* ctl, double* partials, hipStream_t s) {
    const CmeansArgs a{image, u, bufs, ctl, partials, W, H, 0};
    return dispatch_nc<CmeansRun>(N, C, a, cmeans_blocks(W, H), s);
}

template <int N, int C>
struct CmeansFieldsRun {
    static hipError_t run(const CmeansArgs& a, int first, int count, double* tot, double* c64, Ctl* ctl,
                          hipStream_t s) {
        const int nb = cmeans_blocks(a.W, a.H);
        hipLaunchKernelGGL((k_cmeans<N, C>), dim3(nb, count), dim3(kBlock), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cmeans_tot<N, C>), dim3(count), dim3(kBlock), 0, s, a.partials, nb,
                           tot + (int64_t)first * kCmeansMaxM);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cmeans_chain<N, C>), dim3(1), dim3(kBlock), 0, s, tot, first, count, ctl, c64);
        return hipGetLastError();
    }
};

hipError_t launch_cmeans_fields(int N, int C, int W, int H, const float* image, const float* fields,
                                int first, int count, double* partials, double* tot, double* c64, Ctl* ctl,
                                hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (count > kCmeansFields) return hipErrorInvalidValue;
    const int64_t stride = (int64_t)N * W * H;
    const CmeansArgs a{image, fields + first * stride, Bufs{}, ctl, partials, W, H, stride};
    return dispatch_nc<CmeansFieldsRun>(N, C, a, first, count, tot, c64, ctl, s);
}

template <int N, int C>
struct CmeansFinishRun {
    static hipError_t run(const CmeansFinArgs& a, hipStream_t s) {
        hipLaunchKernelGGL((k_cmeans_finish<N, C>), dim3(1), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
};

hipError_t launch_cmeans_finish(int N, int C, int W, int H, const double* partials, Ctl* ctl,
                                const double* c_prev64, double* c64, float* c_out, double* tot,
                                hipStream_t s) {
    const CmeansFinArgs a{partials, cmeans_blocks(W, H), ctl, c_prev64, c64, c_out, tot};
    return dispatch_nc<CmeansFinishRun>(N, C, a, s);
}

// One block: colour means from already reduced sums.
template <int N, int C>
__global__ void k_means_from_tot(const double* tot, const double* c_prev64, Ctl* ctl, double* c64,
                                 float* c_out) {
    constexpr int M = N * C + N + C + 2;
    if (threadIdx.x != 0) return;
    double c[N * C];
    const int empty = finish_means<N, C>(tot, c_prev64, c);
    for (int q = 0; q < N * C; ++q) {
        if (c64) c64[q] = c[q];
        if (c_out) c_out[q] = (float)c[q];
    }
    ctl->empty_now = empty;
    if (tot[M - 1] > 0.0) ctl->nonfinite = 1;
}

template <int N, int C>
struct MeansFromTotRun {
    static hipError_t run(const double* tot, const double* c_prev64, Ctl* ctl, double* c64,
                          float* c_out, hipStream_t s) {
        hipLaunchKernelGGL((k_means_from_tot<N, C>), dim3(1), dim3(64), 0, s, tot, c_prev64, ctl, c64,
                           c_out);
        return hipGetLastError();
    }
};

hipError_t launch_means_from_tot(int N, int C, const double* tot, const double* c_prev64,
                                 Ctl* ctl, double* c64, float* c_out, hipStream_t s) {
    return dispatch_nc<MeansFromTotRun>(N, C, tot, c_prev64, ctl, c64, c_out, s);
}

hipError_t launch_ctl_init(Ctl* ctl, int cur, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, cur);
    return hipGetLastError();
}

hipError_t launch_copy_current(Bufs bufs, const Ctl* ctl, float* dst, int64_t count,
                               hipStream_t s) {
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

template <int N, int C>
struct LabelsRun {
    static hipError_t run(const float* u, const float* c, uint8_t* l, float* comp, float* rnd,
                          int64_t n, hipStream_t s) {
        const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_labels<N, C>), dim3(blocks), dim3(kBlock), 0, s, u, c, l, comp, rnd, n);
        return hipGetLastError();
    }
};

hipError_t launch_labels(int N, int C, int W, int H, const float* u, const float* c,
                         uint8_t* labels, float* composite, float* rounded, hipStream_t s) {
    return dispatch_nc<LabelsRun>(N, C, u, c, labels, composite, rounded, (int64_t)W * H, s);
}

template <int N, int C>
struct EnergyRun {
    static hipError_t run(const EnergyArgs& a, int blocks, hipStream_t s) {
        hipLaunchKernelGGL((k_energy<N, C>), dim3(blocks), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
};

hipError_t launch_energy(int N, int C, int W, int H, const float* image, const float* u,
                         const double* c64, double eps, double lambda, double h,
                         double* partials, double* energy, hipStream_t s) {
    const EnergyArgs a{image, u, c64, partials, W, H};
    const int blocks = grid_for((int64_t)W * H, kCmeansBlocks);
    hipError_t e = dispatch_nc<EnergyRun>(N, C, a, blocks, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(kBlock), 0, s, partials, blocks, eps, lambda,
                       h, energy);
    return hipGetLastError();
}

}  // namespace acseg
