// cycle_impl.hpp -- one smoothing cycle of a time step, on LDS tiles, and the
// end-of-step reduction.  Instantiated per phase count in cycle_n*.hip.
//
// A cycle is `sweeps` red-black sweeps of projected block Gauss-Seidel over the
// nodal sub-problems of the step (Section "Finite Element Notation": one
// exact block minimisation per node, the nodes of one colour at a time), then
// the natural residual of the result.  The first launch of a step also builds
// the right-hand side of eq. alpha from u^n and the image while it stages the
// tile, so a one-cycle step touches each node's data once:
//     read u^n (N floats) and I (C floats), write u^{n+1} (N floats).
// The closing launch of a cycle leaves, per tile, the largest residual and
// the colour-mean partial sums of its output (the means of the next step).
//
// Tiles: a workgroup owns a TX x TY block of the lattice and stages it with a
// halo of R = 2K (+1 for the residual) nodes in LDS, every row split into its
// even-x and odd-x halves.  Half-sweep s updates one colour inside a region
// that shrinks by one node per half-sweep, so the tile ends up exactly as K
// global red-black sweeps leave it.
//
// Work split: each thread owns fixed horizontal node pairs of the staged
// region, chosen so that the first node of every pair is red ((x+y) even) and
// the second black: a half-sweep updates the same node of every pair, with
// no per-lane colour selection.  Per pair the thread keeps in registers the
// LDS slots of both nodes, their coupling weights kappa*c_pq, their distance
// outside the tile interior, and the right-hand side of both nodes.  Tiles
// are assigned so that the workgroups of one XCD (workgroup id mod 8) own a
// contiguous band of tile rows and share halos in their L2.
#pragma once

#include "acseg_internal.h"

namespace acseg {

__host__ __device__ constexpr int cycle_ty(int N) { return N <= 3 ? 32 : 16; }
constexpr int kTX = 64;


constexpr int kCycT = 512;  // threads of a cycle workgroup (8 wave64)

// LDS holds the staged field node-major: the N components of a node are
// contiguous, padded to NP(N) floats so that a node is read or written with
// one to three vector accesses (float4 for N = 4 and 8). N = 3 takes a
// 3-float stride with dword accesses, 2% faster than a 16-byte stride.
__host__ __device__ constexpr int node_pad(int N) {
    return N <= 2 ? 2 : (N == 3 ? 3 : (N <= 4 ? 4 : (N <= 6 ? 6 : 8)));
}

// Lower bound on waves per SIMD asked of the register allocator. N = 6 sits
// just above the 80-VGPR line of six waves; the bound brings it under
// (+10% throughput). Elsewhere it spills or gains nothing.
__host__ __device__ constexpr int cycle_min_waves(int N) { return N == 6 ? 6 : 1; }

template <int N>
__device__ __forceinline__ void lds_ld(const float* __restrict__ p, float (&v)[N]) {
    constexpr int P = node_pad(N);
    if constexpr (P % 2 == 1) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = p[k];
    } else if constexpr (P % 4 == 0) {
#pragma unroll
        for (int k = 0; k < P / 4; ++k) {
            const float4 t = reinterpret_cast<const float4*>(p)[k];
            if (4 * k + 0 < N) v[4 * k + 0] = t.x;
            if (4 * k + 1 < N) v[4 * k + 1] = t.y;
            if (4 * k + 2 < N) v[4 * k + 2] = t.z;
            if (4 * k + 3 < N) v[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < P / 2; ++k) {
            const float2 t = reinterpret_cast<const float2*>(p)[k];
            if (2 * k + 0 < N) v[2 * k + 0] = t.x;
            if (2 * k + 1 < N) v[2 * k + 1] = t.y;
        }
    }
}

template <int N>
__device__ __forceinline__ void lds_st(float* __restrict__ p, const float (&v)[N]) {
    constexpr int P = node_pad(N);
    if constexpr (P % 2 == 1) {
#pragma unroll
        for (int k = 0; k < N; ++k) p[k] = v[k];
    } else if constexpr (P % 4 == 0) {
#pragma unroll
        for (int k = 0; k < P / 4; ++k) {
            float4 t;
            t.x = 4 * k + 0 < N ? v[4 * k + 0] : 0.f;
            t.y = 4 * k + 1 < N ? v[4 * k + 1] : 0.f;
            t.z = 4 * k + 2 < N ? v[4 * k + 2] : 0.f;
            t.w = 4 * k + 3 < N ? v[4 * k + 3] : 0.f;
            reinterpret_cast<float4*>(p)[k] = t;
        }
    } else {
#pragma unroll
        for (int k = 0; k < P / 2; ++k) {
            float2 t;
            t.x = 2 * k + 0 < N ? v[2 * k + 0] : 0.f;
            t.y = 2 * k + 1 < N ? v[2 * k + 1] : 0.f;
            reinterpret_cast<float2*>(p)[k] = t;
        }
    }
}

template <int N>
__device__ __forceinline__ void lds_get(const float* __restrict__ L, int slot, float (&v)[N]) {
    lds_ld<N>(L + slot * node_pad(N), v);
}

template <int N>
__device__ __forceinline__ void lds_put(float* __restrict__ L, int slot, const float (&v)[N]) {
    lds_st<N>(L + slot * node_pad(N), v);
}

// Dynamic LDS of one cycle launch: the staged field.
template <int N, int K, bool RESID>
__host__ __device__ constexpr int cycle_lds_bytes() {
    constexpr int R = 2 * K + (RESID ? 1 : 0);
    return node_pad(N) * (cycle_ty(N) + 2 * R) * ((kTX + 2 * R) / 2 + 1) * 2 * 4;
}

template <int T>
__device__ __forceinline__ float block_max_t(float v, float* sh /* >= T/kWave */) {
    v = wave_max(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = 0.f;
    if (threadIdx.x == 0) {
        r = sh[0];
        for (int w = 1; w < T / kWave; ++w) r = fmaxf(r, sh[w]);
    }
    __syncthreads();
    return r;
}

// One cycle launch on one tile.  The convergence check (a cycle's first
// launch, adaptive schedules) is done by every workgroup of the image; the
// one owning tile 0 records it.
// INT: the staged region lies strictly inside the image, so every staged node
// is an interior node (class 0, unit edge weights) and no bounds test is needed.
// SOR: the writing half-sweeps are over-relaxed, u_p <- Pi(u_p + omega (y_p - u_p)).  The launch that measures the residual keeps
// its last black half-sweep plain, so the black residual is zero again and the
// red residual half-sweep still measures the natural residual.
template <int N, int C, int K, bool FIRST, bool RESID, bool INT, bool SOR = false>
__device__ __forceinline__ void cycle_tile(const CycleArgs& a, const CycleStep& st, int tile) {
    constexpr int T = kCycT;
    constexpr int TX = kTX, TY = cycle_ty(N);
    constexpr int R = 2 * K + (RESID ? 1 : 0);
    constexpr int LX = TX + 2 * R, LY = TY + 2 * R;
    constexpr int LXH = LX / 2;    // pairs per row
    constexpr int HL = LXH + 1;    // half-row length in LDS (one spare slot)
    constexpr int RW = 2 * HL;     // LDS row stride
    constexpr int NP = LXH * LY;   // pairs in the staged region
    constexpr int MP = (NP + T - 1) / T;
    constexpr int NO = TX * TY / T;  // output nodes per thread
    static_assert(TX * TY % T == 0, "output tile must split evenly");
    static_assert(LY / 2 <= T, "straggler column must fit one pass");
    constexpr int M = N * C + N + C + 2;
    constexpr int NHALF = 2 * K + (RESID ? 1 : 0);
    constexpr int kOut = 255;      // "radius" of a node outside the image: never updated
    // 16-byte aligned: the staged field is read and written with b128 accesses,
    // and the static arrays before it need not end on a 16-byte boundary
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ float red[T / kWave];
    __shared__ double cs[N * C];  // 2 lambda c_ik (first launch of a step)
    __shared__ double cs2[N];     // -lambda |c_i|^2
    constexpr int MD = N * C + N;  // colour-mean sums that change with u
    __shared__ double tsh[M + N * C];
    __shared__ int flag;

    Ctl* ctl = a.ctl;
    StepSlot* slot = &ctl->step[st.slot];
    if (!st.fixed) {
        if (slot->done) return;  // uniform: an earlier cycle of this step converged
        if (st.first && st.cycle > 0) {
            const float* prev = a.res_part + ((st.cycle - 1) & 1) * a.part_stride;
            float r = 0.f;
            for (int b = threadIdx.x; b < a.ntiles; b += T) r = fmaxf(r, prev[b]);
            r = block_max_t<T>(r, red);
            if (threadIdx.x == 0) flag = !(r > a.tol);
            __syncthreads();
            if (flag) {
                if (tile == 0 && threadIdx.x == 0) {
                    slot->done = 1;
                    slot->cycles = st.cycle;
                    slot->resid = r;
                }
                return;
            }
        }
    }
    // uniform: the plane bases then live in scalar registers
    const int cur = __builtin_amdgcn_readfirstlane(iterate_buf(ctl->cur, st.launch));
    const int W = a.W, H = a.H;
    const int64_t P = (int64_t)W * H;
    // per-plane base pointers (uniform), 32-bit node indices
    const float* __restrict__ srcp[N];
    float* __restrict__ dstp[N];
    const float* __restrict__ rhsp[N];
    const float* __restrict__ imgp[C];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        srcp[i] = a.bufs.b[cur] + i * P;
        dstp[i] = const_cast<float*>(a.bufs.b[out_of(cur)]) + i * P;
        rhsp[i] = a.rhs + i * P;
    }
#pragma unroll
    for (int k = 0; k < C; ++k) imgp[k] = a.image + k * P;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int x0 = tx * TX - R, y0 = ty * TY - R;  // LDS origin; x0 + y0 is even

    // ---- one burst of global loads: u of the staged region in row order
    //      (coalesced), and the image (first launch) or stored right-hand side
    //      of the owned pairs
    constexpr int NS = (LX * LY + T - 1) / T;
    float ust[NS][N];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int idx = threadIdx.x + q * T;
        const int ly = idx / LX, lx = idx - ly * LX;
        const int gx = x0 + lx, gy = y0 + ly;
        const bool in = idx < LX * LY && (INT || (gx >= 0 && gx < W && gy >= 0 && gy < H));
        const uint32_t g = in ? (uint32_t)(gy * W + gx) : 0u;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float t = gload(srcp[i], g);
            ust[q][i] = in ? t : 0.f;
        }
    }
    constexpr int NV = FIRST ? C : N;
    float pv0[MP][NV], pv1[MP][NV];
    // LDS addresses of each owned pair, so that every access of a sweep is an
    // immediate offset from one of them: the red node sits at yr + RW, its
    // neighbours at xr + {0, 1} (left, right) and yr + {0, 2 RW} (up, down);
    // the black node sits at zb + RW, its neighbours at yr + RW + {0, 1} and
    // zb + {0, 2 RW} (in slots of NPD floats; the rows beyond the staged
    // region that the outermost ring points to are never accessed)
    constexpr int NPD = node_pad(N);
    float* xr[MP];
    float* yr[MP];
    float* zb[MP];
    int pk[MP];      // rad0 | rad1 << 8
    float kh0[MP], kv0[MP], kh1[MP], kv1[MP];
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        const int pi = threadIdx.x + m * T;
        const int ly = pi / LXH, j = pi - ly * LXH;
        const int odd = ly & 1;
        const int c0 = ly * RW + odd * HL + j;       // red node
        const int cb = c0 + (odd ? 1 - HL : HL);     // black node
        xr[m] = lds + (cb - 1) * NPD;
        yr[m] = lds + (c0 - RW) * NPD;
        zb[m] = lds + (cb - RW) * NPD;
        int packed = 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int lx = 2 * j + odd + e;
            const int gx = x0 + lx, gy = y0 + ly;
            const bool in = pi < NP && lx < LX && (INT || (gx >= 0 && gx < W && gy >= 0 && gy < H));
            const int dx = max(max(R - lx, lx - (R + TX - 1)), 0);
            const int dy = max(max(R - ly, ly - (R + TY - 1)), 0);
            const int rad = in ? max(dx, dy) : kOut;
            const bool need = rad <= R - 1;  // some half-sweep updates this node
            const uint32_t g = need ? (uint32_t)(gy * W + gx) : 0u;
            // unconditional loads (index 0 is always valid): no branch between
            // the loads of the burst
            // (read only for nodes that a half-sweep updates: no mask)
            float v[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] = gload(FIRST ? imgp[q] : rhsp[q], g);
            float kh = 0.f, kv = 0.f;
            if (INT) {
                kh = kv = in ? uniform_f(a.coef.kappa[0]) : 0.f;
            } else if (in) {
                const float kap = sel4(a.coef.kappa, node_class(gx, gy, W, H));
                kh = kap * edge_w_h(gy, H);
                kv = kap * edge_w_v(gx, W);
            }
            packed |= rad << (8 * e);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                if (e == 0) pv0[m][q] = v[q]; else pv1[m][q] = v[q];
            }
            if (e == 0) {
                kh0[m] = kh;
                kv0[m] = kv;
            } else {
                kh1[m] = kh;
                kv1[m] = kv;
            }
        }
        pk[m] = packed;
    }

    // the colour-mean sums of u^n (and the previous means, for empty phases)
    // join the burst: one value per thread of the first wave
    constexpr int NT = M + N * C;
    const double* tot = a.tot + st.tot_sel * kCmeansMaxM;
    const double* c_prev64 = st.prev_sel >= 0 ? a.c64 + st.prev_sel * kNC : nullptr;
    if (FIRST && threadIdx.x < NT) {
        const int t = threadIdx.x;
        const bool prev = t >= M;
        const double* src = prev ? (c_prev64 ? c_prev64 : tot) : tot;
        tsh[t] = src[prev ? t - M : t];
    }

    // ---- u into LDS
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int idx = threadIdx.x + q * T;
        if (idx >= LX * LY) continue;
        const int ly = idx / LX, lx = idx - ly * LX;
        const int li = ly * RW + (lx & 1) * HL + (lx >> 1);
        lds_put<N>(lds, li, ust[q]);
    }
    // After a truncated coarse correction this launch applies
    // u = max(u + alpha w, 0), alpha = clamp(<g~,w>/<w,Hw>, 0, 1) from the
    // direction pass's partials (every workgroup sums them in the same order).
    // In the one-sweep launches (the multigrid's post-smoothing) the partial
    // sums and w at the thread's staged nodes are loaded here, into the
    // registers u has left, so their latency overlaps the barrier; the
    // two-sweep launches keep their register allocation and load them after it.
    constexpr bool kEarly = K == 1;
    [[maybe_unused]] float wst[kEarly ? NS : 1][N];
    [[maybe_unused]] double ga = 0.0, qa = 0.0;
    if constexpr (!FIRST && kEarly) {
        if (st.mg_update) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int idx = threadIdx.x + q * T;
                const int ly = idx / LX, lx = idx - ly * LX;
                const int gx = x0 + lx, gy = y0 + ly;
                const bool in = idx < LX * LY && (INT || (gx >= 0 && gx < W && gy >= 0 && gy < H));
                const uint32_t g = in ? (uint32_t)(gy * W + gx) : 0u;
#pragma unroll
                for (int i = 0; i < N; ++i) wst[q][i] = gload(a.mg_w + i * P, g);
            }
            for (int k = threadIdx.x; k < a.mg_parts; k += T) {
                ga += a.mg_part[2 * k];
                qa += a.mg_part[2 * k + 1];
            }
        }
    }
    __syncthreads();  // u and the sums staged
    if constexpr (!FIRST) {
        if (st.mg_update) {
            __shared__ double mgs[2 * (T / kWave)];
            if constexpr (!kEarly) {
                for (int k = threadIdx.x; k < a.mg_parts; k += T) {
                    ga += a.mg_part[2 * k];
                    qa += a.mg_part[2 * k + 1];
                }
            }
            ga = wave_sum(ga);
            qa = wave_sum(qa);
            if (threadIdx.x % kWave == 0) {
                mgs[2 * (threadIdx.x / kWave)] = ga;
                mgs[2 * (threadIdx.x / kWave) + 1] = qa;
            }
            __syncthreads();
            ga = qa = 0.0;
            for (int w = 0; w < T / kWave; ++w) {
                ga += mgs[2 * w];
                qa += mgs[2 * w + 1];
            }
            const float alpha = (qa > 0.0 && ga > 0.0) ? (float)fmin(ga / qa, 1.0) : 0.f;
            if (tile == 0 && threadIdx.x == 0) ctl->alpha = alpha;  // for inspection
            if constexpr (kEarly) {
                // each thread updates the nodes it staged
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int idx = threadIdx.x + q * T;
                    const int ly = idx / LX, lx = idx - ly * LX;
                    const int gx = x0 + lx, gy = y0 + ly;
                    if (!(idx < LX * LY && (INT || (gx >= 0 && gx < W && gy >= 0 && gy < H)))) continue;
                    float* slot = lds + (ly * RW + (lx & 1) * HL + (lx >> 1)) * NPD;
                    float uv[N];
                    lds_ld<N>(slot, uv);
#pragma unroll
                    for (int i = 0; i < N; ++i) uv[i] = fmaxf(fmaf(alpha, wst[q][i], uv[i]), 0.f);
                    lds_st<N>(slot, uv);
                }
            } else {
                for (int idx = threadIdx.x; idx < LX * LY; idx += T) {
                    const int ly = idx / LX, lx = idx - ly * LX;
                    const int gx = x0 + lx, gy = y0 + ly;
                    if (!(INT || (gx >= 0 && gx < W && gy >= 0 && gy < H))) continue;
                    const uint32_t g = (uint32_t)(gy * W + gx);
                    float wv[N], uv[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) wv[i] = gload(a.mg_w + i * P, g);
                    float* slot = lds + (ly * RW + (lx & 1) * HL + (lx >> 1)) * NPD;
                    lds_ld<N>(slot, uv);
#pragma unroll
                    for (int i = 0; i < N; ++i) uv[i] = fmaxf(fmaf(alpha, wv[i], uv[i]), 0.f);
                    lds_st<N>(slot, uv);
                }
            }
            __syncthreads();
        }
    }
    if (FIRST) {
        // colour means of u^n (identical in every workgroup): lane i < N of
        // the first wave finishes phase i
        if (threadIdx.x < kWave) {
            const int i = threadIdx.x;
            bool empty = false;
            if (i < N) {
                const double area = tsh[N * C + N + C];
                const double S = tsh[N * C + i];
                // fixed means: the caller's, in the previous-means slot
                const bool has_mass = !st.fixed_c && S > 1e-12 * area;
                empty = !st.fixed_c && !has_mass;
                double q2 = 0.0;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const double c = has_mass ? tsh[i * C + k] / S
                                              : (c_prev64 ? tsh[M + i * C + k]
                                                          : tsh[N * C + N + k] / area);
                    cs[i * C + k] = 2.0 * a.rc.lambda * c;  // 2 lambda c_ik
                    q2 += c * c;
                    if (tile == 0) {
                        a.c64[st.c64_sel * kNC + i * C + k] = c;
                        if (a.c_out) a.c_out[i * C + k] = (float)c;
                    }
                }
                cs2[i] = -a.rc.lambda * q2;  // -lambda |c_i|^2
            }
            const bool any_empty = __any(empty);
            if (tile == 0 && i == 0) {
                if (any_empty) ctl->empty_steps += 1;
                if (tsh[M - 1] > 0.0) ctl->nonfinite = 1;
            }
        }
        __syncthreads();  // means known
    }

    // ---- right-hand side of the owned nodes (registers)
    float rr0[MP][N], rr1[MP][N];
#pragma unroll
    for (int m = 0; m < MP; ++m) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            float rv[N];
            const int rad = (pk[m] >> (8 * e)) & 255;
            if (FIRST) {
                // rhs'_i = (w/D)[(1/tau + 2/eps) u_i - lambda F_i(c)] with
                // F_i = |I|^2 - 2 c_i.I + |c_i|^2, up to a constant per node (which
                // leaves the projection unchanged): the colour part
                // g_i = lambda (2 c_i.I - |c_i|^2) in float64, shifted by its largest
                // value (its terms, of size lambda |c|^2, cancel), plus the mass part
                // (w/D)(1/tau + 2/eps) u_i in float32.  The largest component of rhs'
                // lies in [0, (w/D)(1/tau + 2/eps)], below one when eps > 0.71 h.
                if (rad <= R - 1) {
                    const int pi = threadIdx.x + m * T;
                    const int ly = pi / LXH, j = pi - ly * LXH;
                    const int gx = x0 + 2 * j + (ly & 1) + e, gy = y0 + ly;
                    const int cls = INT ? 0 : node_class(gx, gy, W, H);
                    const double wd = INT ? uniform_d(a.rc.wd[0]) : sel4d(a.rc.wd, cls);
                    const float wda = INT ? uniform_f(a.rc.wda[0]) : sel4(a.rc.wda, cls);
                    double Ik[C];
#pragma unroll
                    for (int k = 0; k < C; ++k) Ik[k] = (double)(e == 0 ? pv0[m][k] : pv1[m][k]);
                    double gc[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        double t = cs2[i];
#pragma unroll
                        for (int k = 0; k < C; ++k) t = fma(cs[i * C + k], Ik[k], t);
                        gc[i] = t;
                    }
                    double gmax = gc[0];
#pragma unroll
                    for (int i = 1; i < N; ++i) gmax = fmax(gmax, gc[i]);
                    const double off = -wd * gmax;
                    float un[N];
                    lds_ld<N>((e == 0 ? yr[m] : zb[m]) + RW * NPD, un);
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        rv[i] = fmaf(wda, un[i], (float)fma(wd, gc[i], off));
                        if (st.store_rhs && rad == 0) gstore(const_cast<float*>(rhsp[i]), (uint32_t)(gy * W + gx), rv[i]);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < N; ++i) rv[i] = 0.f;
                }
            } else {
#pragma unroll
                for (int i = 0; i < N; ++i) rv[i] = e == 0 ? pv0[m][i] : pv1[m][i];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if (e == 0)
                    rr0[m][i] = rv[i];
                else
                    rr1[m][i] = rv[i];
            }
        }
    }

    float Io[NO][C];  // image of the owned output nodes (closing launch), loaded before the last half-sweep
    bool on[NO];

    // ---- red-black half-sweeps on the shrinking region
    float res = 0.f;
    const float om = SOR ? uniform_f(a.omega) : 1.f;
    for (int s = 0; s < NHALF; ++s) {
        const int r = R - 1 - s;
        if (RESID && s == NHALF - 1) {
#pragma unroll
            for (int q = 0; q < NO; ++q) {
                const int idx = threadIdx.x + q * T;
                const int oy = idx / TX, ox = idx - oy * TX;
                const int gx = x0 + R + ox, gy = y0 + R + oy;
                on[q] = st.cm && (INT || (gx < W && gy < H));
                const uint32_t g = on[q] ? (uint32_t)(gy * W + gx) : 0u;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const float t = gload(imgp[k], g);
                    Io[q][k] = on[q] ? t : 0.f;
                }
            }
        }
        __syncthreads();
        if ((s & 1) == 0) {  // red: the first node of every pair
#pragma unroll
            for (int m = 0; m < MP; ++m) {
                if ((pk[m] & 255) > r) continue;
                float v[N], a0[N], a1[N], a2[N], a3[N];
                lds_ld<N>(xr[m], a0);
                lds_ld<N>(xr[m] + NPD, a1);
                lds_ld<N>(yr[m], a2);
                lds_ld<N>(yr[m] + 2 * RW * NPD, a3);
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = rr0[m][i] + kh0[m] * (a0[i] + a1[i]) + kv0[m] * (a2[i] + a3[i]);
                if constexpr (SOR) {
                    if (!(RESID && s == NHALF - 1)) {
                        float o[N];
                        lds_ld<N>(yr[m] + RW * NPD, o);
#pragma unroll
                        for (int i = 0; i < N; ++i) v[i] = fmaf(om, v[i] - o[i], o[i]);
                    }
                }
                project_simplex<N, false>(v);
                if (RESID && s == NHALF - 1) {
                    float o[N];
                    lds_ld<N>(yr[m] + RW * NPD, o);
#pragma unroll
                    for (int i = 0; i < N; ++i) res = fmaxf(res, fabsf(v[i] - o[i]));
                } else {
                    lds_st<N>(yr[m] + RW * NPD, v);
                }
            }
        } else {  // black: the second node of every pair
#pragma unroll
            for (int m = 0; m < MP; ++m) {
                if (((pk[m] >> 8) & 255) > r) continue;
                float v[N], a0[N], a1[N], a2[N], a3[N];
                lds_ld<N>(yr[m] + RW * NPD, a0);
                lds_ld<N>(yr[m] + (RW + 1) * NPD, a1);
                lds_ld<N>(zb[m], a2);
                lds_ld<N>(zb[m] + 2 * RW * NPD, a3);
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = rr1[m][i] + kh1[m] * (a0[i] + a1[i]) + kv1[m] * (a2[i] + a3[i]);
                if constexpr (SOR) {
                    if (!(RESID && s == NHALF - 2)) {
                        float o[N];
                        lds_ld<N>(zb[m] + RW * NPD, o);
#pragma unroll
                        for (int i = 0; i < N; ++i) v[i] = fmaf(om, v[i] - o[i], o[i]);
                    }
                }
                project_simplex<N, false>(v);
                lds_st<N>(zb[m] + RW * NPD, v);
            }
        }
    }
    __syncthreads();

    // ---- the tile's interior: global stores (coalesced rows)
    float uo[NO][N];
#pragma unroll
    for (int q = 0; q < NO; ++q) {
        const int idx = threadIdx.x + q * T;
        const int oy = idx / TX, ox = idx - oy * TX;
        const int gx = x0 + R + ox, gy = y0 + R + oy;
        const int lx = R + ox, ly = R + oy;
        const int li = ly * RW + (lx & 1) * HL + (lx >> 1);
        const bool o = INT || (gx < W && gy < H);
        const uint32_t g = o ? (uint32_t)(gy * W + gx) : 0u;
        lds_get<N>(lds, li, uo[q]);
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (o) gstore(dstp[i], g, uo[q][i]);
    }
    if (!RESID) return;

    // ---- per-tile residual and colour-mean partials of the output
    const int row = st.cycle & 1;
    const float bm = block_max_t<T>(res, red);
    if (threadIdx.x == 0) a.res_part[row * a.part_stride + tile] = bm;
    if (!st.cm) return;
    // the sums that depend on u: S_ik = sum w u_i I_k and S_i = sum w u_i (the
    // image-only ones do not change from step to step)
    float acc[MD];
#pragma unroll
    for (int q = 0; q < MD; ++q) acc[q] = 0.f;
#pragma unroll
    for (int q = 0; q < NO; ++q) {
        const int idx = threadIdx.x + q * T;
        const int oy = idx / TX, ox = idx - oy * TX;
        const float w = on[q] ? (INT ? 1.f : (float)mass_w(node_class(x0 + R + ox, y0 + R + oy, W, H))) : 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float wu = w * uo[q][i];
            acc[N * C + i] += wu;
#pragma unroll
            for (int k = 0; k < C; ++k) acc[i * C + k] += wu * Io[q][k];
        }
    }
    // block sum in a fixed order, in FP32: quads first (data-parallel moves),
    // one lane per quad into LDS (the staging area is free: the residual's
    // block reduction has synchronised the reads of the field), then 32 lanes
    // per sum add four quad sums each and reduce across their half-wave
    constexpr int NQ = T / 4;  // quads per workgroup
    static_assert(MD * NQ * 4 <= cycle_lds_bytes<N, K, RESID>(), "quad sums must fit in the staging area");
    static_assert(NQ == 32 * 4, "a half-wave of lanes covers the quads of one sum");
    float* qs = lds;  // [MD][NQ]
#pragma unroll
    for (int q = 0; q < MD; ++q) {
        const float t = quad_sum(acc[q]);
        if ((threadIdx.x & 3) == 0) qs[q * NQ + (threadIdx.x >> 2)] = t;
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < (MD * 32 + T - 1) / T; ++pass) {
        const int t = threadIdx.x + pass * T;
        const int q = t >> 5, seg = t & 31;  // sum q, quads 4 seg .. 4 seg + 3
        float v = 0.f;
        if (q < MD) {
            const float* r4 = qs + q * NQ + 4 * seg;
            v = (r4[0] + r4[1]) + (r4[2] + r4[3]);
        }
        v = half_wave_sum_last(v);
        if (seg == 31 && q < MD) a.cm_part[((int64_t)row * MD + q) * a.part_stride + tile] = (double)v;
    }
}

// One image: tiles in XCD-aware order (the workgroups of one XCD, id mod 8,
// own a contiguous band of tiles).
// Whether the staged region of a tile lies strictly inside the image.
template <int N, int K, bool RESID>
__device__ __forceinline__ bool tile_interior(const CycleArgs& a, int tile) {
    constexpr int R = 2 * K + (RESID ? 1 : 0);
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int x0 = tx * kTX - R, y0 = ty * cycle_ty(N) - R;
    return x0 >= 1 && y0 >= 1 && x0 + kTX + 2 * R <= a.W - 1 && y0 + cycle_ty(N) + 2 * R <= a.H - 1;
}

template <int N, int C, int K, bool FIRST, bool RESID, bool SOR = false>
__device__ __forceinline__ void cycle_tile_any(const CycleArgs& a, const CycleStep& st, int tile) {
    if (tile_interior<N, K, RESID>(a, tile))
        cycle_tile<N, C, K, FIRST, RESID, true, SOR>(a, st, tile);
    else
        cycle_tile<N, C, K, FIRST, RESID, false, SOR>(a, st, tile);
}

// Tile of workgroup b in a single-image launch, -1 for none.  XCD x = b mod 8
// owns a band of whole tile rows.  Inside the band the tiles go down strips of
// kStrip tile columns, row by row within a strip, so the tile above a tile ran
// about kStrip tiles earlier on the same XCD and the halo rows they share are
// still in that XCD's L2.  In plain row-major order a whole tile row runs in
// between, which on a wide lattice (64 tiles of about 85 KB each at 4096 nodes
// and N = 8) no longer fits in the 4 MB L2.
__device__ __forceinline__ int tile_of_block(const CycleArgs& a, int b) {
    const int x = b % kXcd, j = b / kXcd;
    const int r0 = x * a.rows_per_xcd;
    const int rows = min(a.rows_per_xcd, a.tiles_y - r0);
    if (rows <= 0) return -1;
    const int per_strip = rows * kStrip;
    const int g = j / per_strip;
    const int c0 = g * kStrip;
    if (c0 >= a.tiles_x) return -1;
    const int w = min(kStrip, a.tiles_x - c0);  // the last strip may be narrower
    const int rem = j - g * per_strip;
    const int r = rem / w, c = rem - r * w;
    if (r >= rows) return -1;
    return (r0 + r) * a.tiles_x + c0 + c;
}

template <int N, int C, int K, bool FIRST, bool RESID, bool SOR>
__global__ __launch_bounds__(kCycT, cycle_min_waves(N)) void k_cycle(CycleArgs a, CycleStep st) {
    const int tile = tile_of_block(a, blockIdx.x);
    if (tile < 0) return;
    cycle_tile_any<N, C, K, FIRST, RESID, SOR>(a, st, tile);
}

// A batch of images with the same N and C: work[] lists (image, tile) of
// every tile of the batch, already in XCD-aware order (image -1: nothing to
// do); the per-image constants are read from the descriptor table.
template <int N, int C, int K, bool FIRST, bool RESID, bool SOR>
__global__ __launch_bounds__(kCycT, cycle_min_waves(N)) void k_cycle_batch(const CycleArgs* __restrict__ descs,
                                                       const int2* __restrict__ work, int nwork,
                                                       CycleStep st) {
    if ((int)blockIdx.x >= nwork) return;
    const int2 wv = work[blockIdx.x];
    if (wv.x < 0) return;
    cycle_tile_any<N, C, K, FIRST, RESID, SOR>(descs[wv.x], st, wv.y);
}

// ---------------------------------------------------------------------------
// End of a time step, MD + 1 workgroups (MD = N C + N).  Workgroup q < MD
// sums row q of the last cycle's colour-mean partials over the tiles (fixed
// order, so the result is deterministic) into the next set of sums: those of
// the new iterate.  Workgroup MD carries the image-only sums over, takes the
// step's residual (the last cycle's, unless a cycle kernel found convergence
// earlier), moves `cur` to the buffer holding the iterate, folds the
// statistics and re-arms the other control slot for the step after next.
// ---------------------------------------------------------------------------

template <int N, int C>
__device__ __forceinline__ void step_end(const CycleArgs& a, const CycleStep& st, const StepEndArgs& e) {
    constexpr int M = N * C + N + C + 2;
    constexpr int MD = N * C + N;  // rows reduced; the image-only sums are carried over
    __shared__ float red[kBlock / kWave];
    __shared__ double shd[kBlock / kWave];
    Ctl* ctl = a.ctl;
    StepSlot* slot = &ctl->step[st.slot];
    const int done = slot->done;
    const int cycles = done ? slot->cycles : e.max_cycles;
    if ((int)blockIdx.x < MD) {
        const int q = blockIdx.x;
        const double* row = a.cm_part + ((int64_t)((cycles - 1) & 1) * MD + q) * a.part_stride;
        double t = strided_sum4(row, a.ntiles);
        t = wave_sum(t);
        if (threadIdx.x % kWave == 0) shd[threadIdx.x / kWave] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += shd[w];
            a.tot[(st.tot_sel ^ 1) * kCmeansMaxM + q] = s;
        }
        return;
    }
    if (threadIdx.x < M - MD)  // sum w I_k, sum w and the image flag: constants of the solve
        a.tot[(st.tot_sel ^ 1) * kCmeansMaxM + MD + threadIdx.x] = a.tot[st.tot_sel * kCmeansMaxM + MD + threadIdx.x];
    float resid;
    if (done) {
        resid = slot->resid;
    } else {
        const float* last = a.res_part + ((e.max_cycles - 1) & 1) * a.part_stride;
        resid = block_max(strided_max4(last, a.ntiles), red);
    }
    if (threadIdx.x != 0) return;
    ctl->cur = iterate_buf(ctl->cur, cycles * e.launches_per_cycle + e.launch_offset);
    ctl->resid = resid;
    ctl->cycles_total += cycles;
    ctl->cycles_max = cycles > ctl->cycles_max ? cycles : ctl->cycles_max;
    if (resid > a.tol) ctl->steps_unconv += 1;
    ctl->max_resid = fmaxf(ctl->max_resid, resid);
    ctl->steps_done += 1;
    StepSlot* next = &ctl->step[st.slot ^ 1];
    next->done = 0;
    next->cycles = 0;
    next->resid = 0.f;
}

template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_step_end(CycleArgs a, CycleStep st, StepEndArgs e) {
    step_end<N, C>(a, st, e);
}

// blockIdx.y: position in imgs[] (the images of one batch group)
template <int N, int C>
__global__ __launch_bounds__(kBlock) void k_step_end_batch(const CycleArgs* __restrict__ descs,
                                                           const int* __restrict__ imgs, CycleStep st,
                                                           StepEndArgs e) {
    step_end<N, C>(descs[imgs[blockIdx.y]], st, e);
}

int cycle_launches(int sweeps);

template <int N, int C, int K, bool FIRST, bool RESID>
hipError_t run_cycle(const CycleArgs& a, const CycleStep& st, const CycleGrid& g, hipStream_t s) {
    constexpr int lds = cycle_lds_bytes<N, K, RESID>();
    static_assert(lds <= 65536, "tile does not fit in 64 KiB of LDS");
    if (g.descs && g.sor)
        hipLaunchKernelGGL((k_cycle_batch<N, C, K, FIRST, RESID, true>), dim3(g.nwork), dim3(kCycT), lds, s,
                           g.descs, g.work, g.nwork, st);
    else if (g.descs)
        hipLaunchKernelGGL((k_cycle_batch<N, C, K, FIRST, RESID, false>), dim3(g.nwork), dim3(kCycT), lds, s,
                           g.descs, g.work, g.nwork, st);
    else if (a.omega != 1.f)
        hipLaunchKernelGGL((k_cycle<N, C, K, FIRST, RESID, true>), dim3(a.tiles_per_xcd * kXcd), dim3(kCycT),
                           lds, s, a, st);
    else
        hipLaunchKernelGGL((k_cycle<N, C, K, FIRST, RESID, false>), dim3(a.tiles_per_xcd * kXcd), dim3(kCycT),
                           lds, s, a, st);
    return hipGetLastError();
}

// `sweeps` sweeps in launches of at most two.
template <int N, int C>
hipError_t run_cycle_nc(int sweeps, const CycleArgs& a, CycleStep st, const CycleGrid& g, CycleRole role,
                        hipStream_t s) {
    const int nl = cycle_launches(sweeps);
    const int base = st.launch;
    hipError_t e = hipSuccess;
    for (int k = 0; k < nl && e == hipSuccess; ++k) {
        const int kk = (k < nl - 1 || sweeps % 2 == 0) ? 2 : 1;
        const bool last = role.closes && k == nl - 1;
        const bool first = role.step_first && k == 0;
        st.first = role.opens && k == 0;
        st.launch = base + k;
        st.mg_update = (role.mg_update && k == 0) ? 1 : 0;
        if (kk == 2) {
            if (first)
                e = last ? run_cycle<N, C, 2, true, true>(a, st, g, s) : run_cycle<N, C, 2, true, false>(a, st, g, s);
            else
                e = last ? run_cycle<N, C, 2, false, true>(a, st, g, s) : run_cycle<N, C, 2, false, false>(a, st, g, s);
        } else {
            if (first)
                e = last ? run_cycle<N, C, 1, true, true>(a, st, g, s) : run_cycle<N, C, 1, true, false>(a, st, g, s);
            else
                e = last ? run_cycle<N, C, 1, false, true>(a, st, g, s) : run_cycle<N, C, 1, false, false>(a, st, g, s);
        }
    }
    return e;
}

template <int N, int C>
hipError_t run_step_end_nc(const CycleArgs& a, const CycleStep& st, const StepEndArgs& e,
                           const CycleArgs* descs, const int* imgs, int nimg, hipStream_t s) {
    constexpr int MD = N * C + N;
    if (descs)
        hipLaunchKernelGGL((k_step_end_batch<N, C>), dim3(MD + 1, nimg), dim3(kBlock), 0, s, descs, imgs, st, e);
    else
        hipLaunchKernelGGL((k_step_end<N, C>), dim3(MD + 1), dim3(kBlock), 0, s, a, st, e);
    return hipGetLastError();
}

// Per-N entry points, each instantiated in its own translation unit.
template <int N>
hipError_t cycle_for_n(int C, int sweeps, const CycleArgs& a, const CycleStep& st, const CycleGrid& g,
                       CycleRole role, hipStream_t s) {
    switch (C) {
        case 1: return run_cycle_nc<N, 1>(sweeps, a, st, g, role, s);
        case 2: return run_cycle_nc<N, 2>(sweeps, a, st, g, role, s);
        case 3: return run_cycle_nc<N, 3>(sweeps, a, st, g, role, s);
        case 4: return run_cycle_nc<N, 4>(sweeps, a, st, g, role, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t step_end_for_n(int C, const CycleArgs& a, const CycleStep& st, const StepEndArgs& e,
                          const CycleArgs* descs, const int* imgs, int nimg, hipStream_t s) {
    switch (C) {
        case 1: return run_step_end_nc<N, 1>(a, st, e, descs, imgs, nimg, s);
        case 2: return run_step_end_nc<N, 2>(a, st, e, descs, imgs, nimg, s);
        case 3: return run_step_end_nc<N, 3>(a, st, e, descs, imgs, nimg, s);
        case 4: return run_step_end_nc<N, 4>(a, st, e, descs, imgs, nimg, s);
        default: return hipErrorInvalidValue;
    }
}

#define ACSEG_CYCLE_EXTERN(n)                                                                  \
    extern template hipError_t cycle_for_n<n>(int, int, const CycleArgs&, const CycleStep&,      \
                                              const CycleGrid&, CycleRole, hipStream_t);         \
    extern template hipError_t step_end_for_n<n>(int, const CycleArgs&, const CycleStep&,        \
                                                 const StepEndArgs&, const CycleArgs*, const int*, \
                                                 int, hipStream_t);
ACSEG_CYCLE_EXTERN(2)
ACSEG_CYCLE_EXTERN(3)
ACSEG_CYCLE_EXTERN(4)
ACSEG_CYCLE_EXTERN(5)
ACSEG_CYCLE_EXTERN(6)
ACSEG_CYCLE_EXTERN(7)
ACSEG_CYCLE_EXTERN(8)
#undef ACSEG_CYCLE_EXTERN

}  // namespace acseg
