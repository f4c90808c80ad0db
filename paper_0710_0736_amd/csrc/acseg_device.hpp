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

__device__ __forceinline__ float sel4(const float (&a)[4], int k) {
    // select without dynamic indexing of a kernel-argument array
    return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}

__device__ __forceinline__ double sel4d(const double (&a)[4], int k) {
    return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}

// Horizontal / vertical edge weights of node (x,y): 1/2 along the boundary line.
__device__ __forceinline__ float edge_w_h(int y, int H) { return (y == 0 || y == H - 1) ? 0.5f : 1.0f; }
__device__ __forceinline__ float edge_w_v(int x, int W) { return (x == 0 || x == W - 1) ? 0.5f : 1.0f; }

// Lumped-mass weight w_p (M_p / h^2 on its own level).
__device__ __forceinline__ double mass_w(int cls) {
    return cls == 0 ? 1.0 : (cls == 1 ? 0.5 : (cls == 2 ? (1.0 / 3.0) : (1.0 / 6.0)));
}

// Euclidean projection of v onto the Gibbs simplex, in registers.
//
// The correction loop of Section "Gibbs Space Constraint Pseudocode" in
// threshold form: all free components are shifted by one common theta chosen
// so that they sum to one; every free component that would go negative is
// fixed at zero and leaves the free set; repeat.  At most N rounds.  Values
// are taken relative to the largest component (which never leaves the free
// set) so that the threshold arithmetic stays well conditioned in FP32.
template <int N>
__device__ __forceinline__ void project_simplex(float (&v)[N]) {
    float vmax = v[0];
#pragma unroll
    for (int i = 1; i < N; ++i) vmax = fmaxf(vmax, v[i]);
    int imax = N - 1;
#pragma unroll
    for (int i = N - 1; i >= 0; --i)
        if (v[i] == vmax) imax = i;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] -= vmax;
    unsigned freem = (1u << N) - 1u;
    float theta = 0.f;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        float s = 0.f;
        int k = 0;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if ((freem >> i) & 1u) {
                s += v[i];
                ++k;
            }
        theta = (s - 1.0f) / (float)k;
        unsigned out = 0u;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (((freem >> i) & 1u) && i != imax && v[i] < theta) out |= 1u << i;
        if (out == 0u) break;
        freem &= ~out;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = ((freem >> i) & 1u) ? fmaxf(v[i] - theta, 0.f) : 0.f;
}

// ---------------------------------------------------------------------------
// Wave / block reductions (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
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

// Last-block detection: every block calls this once after writing its partial
// results; it returns true in all threads of the block that arrives last, and
// that block then sees every other block's partials.  Each thread publishes
// its own writes with a device-scope fence before the barrier; the last block
// fences again before reading.  The counter is reset by the last block.
__device__ __forceinline__ bool arrive_last(unsigned* counter, int* sh_flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(counter, 1u);
        *sh_flag = (prev == gridDim.x * gridDim.y * gridDim.z - 1u) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *sh_flag != 0;
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return last;
}

}  // namespace acseg
