// acseg_device.hpp -- device-side building blocks shared by the gfx950 kernels.
//
// Discrete setting (Section "Finite Element Notation" of Kay & Tomasi): P1
// elements on the W x H pixel lattice, every cell split along its
// (x,y)-(x+1,y+1) diagonal, lumped mass, natural boundary conditions.  On this
// mesh the stiffness matrix is the 5-point stencil with weight 1 on interior
// lattice edges and 1/2 on edges lying on the boundary, and the lumped mass is
// M_p = h^2 w_p with w_p = 1 (interior), 1/2 (edge), 1/3 at the corners (0,0)
// and (W-1,H-1) (two triangles) and 1/6 at (W-1,0) and (0,H-1) (one triangle).
// No per-node coefficient arrays are stored: a node's class follows from its
// coordinates.
//
// Every level works in units scaled by 1/h^2 of the finest spacing h: the
// diagonal of H = M/tau + eps A at level l (spacing 2^l h) is
// D_p = 4^l w_p / tau + (eps/h^2) a_pp, the off-diagonal coupling to a lattice
// neighbour q is -(eps/h^2) c_pq with c_pq in {1, 1/2}.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acseg {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)
constexpr int kWave = 64;

// Global memory through address space 1.  A pointer read from a descriptor
// table is generic, and an access through it becomes a flat instruction with
// a 64-bit vector address of its own (two VALU operations per access, and a
// count on the LDS counter too).  Through these helpers the access is a
// global instruction addressed as a uniform base in scalar registers plus a
// 32-bit byte offset, which all planes of a field share.  Element index
// i < 2^30 (the lattice limit).
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ float gload(const float* base, uint32_t i) {
    return *(const gfloat*)((const gchar*)base + (i << 2));
}
__device__ __forceinline__ void gstore(float* base, uint32_t i, float v) {
    *(gfloat*)((gchar*)base + (i << 2)) = v;
}

// Node class: 0 interior, 1 edge, 2 corner (0,0)/(W-1,H-1), 3 corner (W-1,0)/(0,H-1).
__device__ __forceinline__ int node_class(int x, int y, int W, int H) {
    const int bx = (x == 0) | (x == W - 1);
    const int by = (y == 0) | (y == H - 1);
    const int k = bx + by;
    if (k < 2) return k;
    return ((x == 0) == (y == 0)) ? 2 : 3;
}

// Per-level coefficients of the scaled nodal system, by node class.
struct LevelCoef {
    float kappa[4];  // (eps/h^2) / D
    float inv_d[4];  // 1 / D
    float d[4];      // D
    float e2;        // eps / h^2
    float pad[3];
};

// Uniform values forced into scalar registers: a per-lane select among them
// is then a register select, not a select of kernel-argument addresses
// followed by a dependent load.
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float sel4(const float (&a)[4], int k) {
    const float a0 = uniform_f(a[0]), a1 = uniform_f(a[1]), a2 = uniform_f(a[2]), a3 = uniform_f(a[3]);
    return k == 0 ? a0 : (k == 1 ? a1 : (k == 2 ? a2 : a3));
}

__device__ __forceinline__ double sel4d(const double (&a)[4], int k) {
    const double a0 = uniform_d(a[0]), a1 = uniform_d(a[1]), a2 = uniform_d(a[2]), a3 = uniform_d(a[3]);
    return k == 0 ? a0 : (k == 1 ? a1 : (k == 2 ? a2 : a3));
}

// Horizontal / vertical edge weights of node (x,y): 1/2 along the boundary line.
__device__ __forceinline__ float edge_w_h(int y, int H) { return (y == 0 || y == H - 1) ? 0.5f : 1.0f; }
__device__ __forceinline__ float edge_w_v(int x, int W) { return (x == 0 || x == W - 1) ? 0.5f : 1.0f; }

// Lumped-mass weight w_p (M_p / h^2 on its own level).
__device__ __forceinline__ double mass_w(int cls) {
    return cls == 0 ? 1.0 : (cls == 1 ? 0.5 : (cls == 2 ? (1.0 / 3.0) : (1.0 / 6.0)));
}

// Sorting networks (descending), N <= 8: pairs (i, j), i < j, after which
// s[i] >= s[j].  Each was checked exhaustively on 0/1 inputs.
template <int N> struct SortNet;
template <> struct SortNet<2> { static constexpr int n = 1; static constexpr int p[1][2] = {{0, 1}}; };
template <> struct SortNet<3> { static constexpr int n = 3; static constexpr int p[3][2] = {{0, 2}, {0, 1}, {1, 2}}; };
template <> struct SortNet<4> {
    static constexpr int n = 5;
    static constexpr int p[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
};
template <> struct SortNet<5> {
    static constexpr int n = 9;
    static constexpr int p[9][2] = {{0, 1}, {3, 4}, {2, 4}, {2, 3}, {0, 3}, {0, 2}, {1, 4}, {1, 3}, {1, 2}};
};
template <> struct SortNet<6> {
    static constexpr int n = 12;
    static constexpr int p[12][2] = {{1, 2}, {4, 5}, {0, 2}, {3, 5}, {0, 1}, {3, 4},
                                     {2, 5}, {0, 3}, {1, 4}, {2, 4}, {1, 3}, {2, 3}};
};
template <> struct SortNet<7> {
    static constexpr int n = 16;
    static constexpr int p[16][2] = {{1, 2}, {3, 4}, {5, 6}, {0, 2}, {3, 5}, {4, 6}, {0, 1}, {4, 5},
                                     {2, 6}, {0, 4}, {1, 5}, {0, 3}, {2, 5}, {1, 3}, {2, 4}, {2, 3}};
};
template <> struct SortNet<8> {
    static constexpr int n = 19;
    static constexpr int p[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6},
                                     {3, 7}, {0, 1}, {2, 3}, {4, 5}, {6, 7}, {2, 4}, {3, 5},
                                     {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
};

// Euclidean projection of v onto the Gibbs simplex, in registers.
//
// The correction loop of Section "Gibbs Space Constraint Pseudocode" ends at
// x_i = max(v_i - theta, 0) with theta the common shift that makes the free
// components sum to one.  Here theta is found without the loop, by the
// sort-based characterisation of the same projection (Held, Wolfe & Crowder
// 1974; Duchi et al. 2008): with s the values sorted in descending order and
// S_k the sum of the k largest, theta = max_k (S_k - 1) / k (each candidate
// is a lower bound of theta, and the one at the number of free components is
// theta itself).  Two phases have the closed form x_0 = (1 + v_0 - v_1) / 2
// clipped to [0, 1], x_1 = 1 - x_0.
//
// CENTRED: the sums are taken relative to the largest value, which keeps
// them well conditioned for inputs of any magnitude.  The sweep of the solver
// calls it with CENTRED = false: its largest component is of order one (the
// right-hand side, shifted per node so that its largest component lies in
// [0, (w/D)(1/tau + 2/eps)], plus neighbour terms in [0, 1)), so every
// component that can be free lies within one of it, and the plain sums are
// as well conditioned.
// Components of the result lie in [0, 1], so max(v_i - theta, 0) is a clamp
// to [0, 1], which folds into the subtraction.
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 1.f); }

template <int N, bool CENTRED = true>
__device__ __forceinline__ void project_simplex(float (&v)[N]) {
    if constexpr (N == 2) {
        const float x0 = clamp01(fmaf(v[0] - v[1], 0.5f, 0.5f));
        v[0] = x0;
        v[1] = 1.f - x0;
        return;
    } else {
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
        float thr;
        if constexpr (CENTRED) {
            const float vmax = s[0];
            float S = 0.f, theta = -1.0f;  // k = 1: the largest value alone
#pragma unroll
            for (int k = 2; k <= N; ++k) {
                S += s[k - 1] - vmax;
                theta = fmaxf(theta, fmaf(S, 1.0f / (float)k, -1.0f / (float)k));
            }
            thr = vmax + theta;  // the shift in the original values
        } else {
            float T = s[0] - 1.f;  // S_k - 1, accumulated
            thr = T;
#pragma unroll
            for (int k = 2; k <= N; ++k) {
                T += s[k - 1];
                thr = fmaxf(thr, T * (1.0f / (float)k));
            }
        }
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = clamp01(v[i] - thr);
    }
}

// ---------------------------------------------------------------------------
// Wave / block reductions (wave64)
// ---------------------------------------------------------------------------

// Maximum over the 64 lanes of a wave (DPP moves as in wave_sum_last, lanes
// a move does not reach keeping their own value), read back from lane 63:
// every lane returns it.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_keep_f(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_keep_f<0xB1, 0xF>(v));
    v = fmaxf(v, dpp_keep_f<0x4E, 0xF>(v));
    v = fmaxf(v, dpp_keep_f<0x124, 0xF>(v));
    v = fmaxf(v, dpp_keep_f<0x128, 0xF>(v));
    v = fmaxf(v, dpp_keep_f<0x142, 0xA>(v));
    v = fmaxf(v, dpp_keep_f<0x143, 0xC>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over the 64 lanes of a wave in a fixed order (data-parallel-primitive
// moves: within quads, rotations within rows of 16, then row broadcasts); the
// total is exact in lane 63 only.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
__device__ __forceinline__ float wave_sum_last(float v) {
    v += dpp_f<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]: every lane holds its quad's sum
    v += dpp_f<0x124, 0xF>(v);  // row_ror:4
    v += dpp_f<0x128, 0xF>(v);  // row_ror:8: every lane holds its row's sum
    v += dpp_f<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum over the 4 lanes of each quad (every lane of the quad holds it).
__device__ __forceinline__ float quad_sum(float v) {
    v += dpp_f<0xB1, 0xF>(v);
    v += dpp_f<0x4E, 0xF>(v);
    return v;
}

// Sum over each half-wave (32 lanes) in a fixed order; exact in lanes 31 and 63.
__device__ __forceinline__ float half_wave_sum_last(float v) {
    v += dpp_f<0xB1, 0xF>(v);
    v += dpp_f<0x4E, 0xF>(v);
    v += dpp_f<0x124, 0xF>(v);
    v += dpp_f<0x128, 0xF>(v);
    v += dpp_f<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    return v;
}

// Sum over the 64 lanes of a wave in the fixed order of wave_sum_last (each
// DPP move on both 32-bit halves), read back from lane 63: every lane
// returns the total.  All lanes of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1, 0xF>(v);
    v += dpp_d<0x4E, 0xF>(v);
    v += dpp_d<0x124, 0xF>(v);
    v += dpp_d<0x128, 0xF>(v);
    v += dpp_d<0x142, 0xA>(v);
    v += dpp_d<0x143, 0xC>(v);
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// This thread's share (t, t + kBlock, ...) of a sum / max over n values, with
// four independent accumulators combined in a fixed order: deterministic, and
// four loads in flight per thread instead of one dependent chain.
__device__ __forceinline__ double strided_sum4(const double* __restrict__ v, int n) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * kBlock < n; b += 4 * kBlock) {
        t0 += v[b];
        t1 += v[b + kBlock];
        t2 += v[b + 2 * kBlock];
        t3 += v[b + 3 * kBlock];
    }
    for (; b < n; b += kBlock) t0 += v[b];
    return (t0 + t1) + (t2 + t3);
}
__device__ __forceinline__ float strided_max4(const float* __restrict__ v, int n) {
    float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f;
    int b = threadIdx.x;
    for (; b + 3 * kBlock < n; b += 4 * kBlock) {
        r0 = fmaxf(r0, v[b]);
        r1 = fmaxf(r1, v[b + kBlock]);
        r2 = fmaxf(r2, v[b + 2 * kBlock]);
        r3 = fmaxf(r3, v[b + 3 * kBlock]);
    }
    for (; b < n; b += kBlock) r0 = fmaxf(r0, v[b]);
    return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// Block-wide max over kBlock threads; result valid in thread 0.
__device__ __forceinline__ float block_max(float v, float* sh /* >= kBlock/kWave */) {
    v = wave_max(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = 0.f;
    if (threadIdx.x == 0) {
        r = sh[0];
        for (int w = 1; w < kBlock / kWave; ++w) r = fmaxf(r, sh[w]);
    }
    __syncthreads();
    return r;
}

// Double wave sum over a block's kBlock threads is done per value; this
// helper sums partial rows [nb][M] in a fixed order into tot[M] (LDS) so that
// every caller obtains bit-identical results.  sh: LDS [kBlock/kWave][M].
template <int M>
__device__ void reduce_rows(const double* __restrict__ part, int nb, double* tot,
                            double (*sh)[M]) {
    double acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock)
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
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sh[w][threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

// c_ik = S_ik / S_i from the reduced sums; empty phases keep c_prev64 (or the
// mean image colour).  Runs in every thread (cheap); returns the empty flag.
template <int N, int C>
__device__ int finish_means(const double* tot, const double* c_prev64, double* c) {
    const double area = tot[N * C + N + C];
    int empty = 0;
    for (int i = 0; i < N; ++i) {
        const double S = tot[N * C + i];
        const bool has_mass = S > 1e-12 * area;
        empty |= has_mass ? 0 : 1;
        for (int k = 0; k < C; ++k)
            c[i * C + k] = has_mass ? tot[i * C + k] / S
                                    : (c_prev64 ? c_prev64[i * C + k] : tot[N * C + N + k] / area);
    }
    return empty;
}

}  // namespace acseg
