// stream_impl.hpp -- the smoothing cycle of a time step (two red-black sweeps,
// the natural residual and the colour-mean partials), streamed down a column
// of the lattice instead of tiled.
//
// The cycle is the same computation as the tiled kernel (cycle_impl.hpp): on
// every node of one colour at a time the nodal map y_p = rhs_p + kappa_p sum_q
// c_pq u_q and its projection onto the Gibbs simplex (Section "Finite Element
// Notation", Section "Gibbs Space Constraint Pseudocode"), two sweeps, then a
// non-writing red half-sweep whose largest change is the natural residual.
// What differs is the order.  A workgroup owns a column of kSOut = 54 output
// nodes and S output rows and walks down its rows once.  With the five
// half-sweeps as pipeline levels k = 1..5 (red, black, red, black, residual),
// level k processes row i - 2k while row i is staged: a node's update needs
// its row and the rows above and below at the previous level, which the
// previous level finished one and three steps earlier, and no two levels
// touch the same row in a step.  So each row of the column is staged, given
// its right-hand side and updated once per level, and only the horizontal
// halo (R = 5 nodes each side: level k updates the nodes within R - k of the
// output columns) and R rows above and below a segment are recomputed.  The
// tiled kernel recomputes its halo on all four sides of a 64 x 16 tile.
//
// A workgroup runs rows + 5 steps: level 5 reaches the last output row four
// steps after it is staged plus one.  A 64-node row is one wave wide.  Wave 0 stages rows (prefetched kSPd rows
// ahead) and builds their right-hand side; wave 1 runs levels 1 and 2 (one per
// half-wave), wave 2 levels 3 and 4, wave 3 the residual level and then
// writes the finished row and adds it to the colour-mean partials.  One
// barrier per row step.  The rows live in an LDS ring of kSRing rows, each
// split into its even-x and odd-x halves, so the 32 lanes of a level read and
// write consecutive nodes.
#pragma once

#include "acseg_internal.h"

namespace acseg {

constexpr int kSR = 5;                   // halo: 2 sweeps + the residual half-sweep
constexpr int kSLX = 64;                 // staged row width (one wave)
constexpr int kSOut = kSLX - 2 * kSR;    // output columns per workgroup
constexpr int kSB = 1;                   // rows per step and role
constexpr int kSD = kSB + 1;             // level k works kSD k rows behind the staging
constexpr int kSRing = 6 * kSB + 6;      // rows in flight: staged rows down to the residual's upper row
constexpr int kSPd = 3;                  // steps of rows prefetched ahead of staging
constexpr int kST = 256;                 // threads (4 waves)

template <int N>
__host__ __device__ constexpr int stream_lds_bytes() {
    return kSRing * kSLX * (node_pad(N) + N) * 4;
}

// Ring slot of staged row i >= 0.
__device__ __forceinline__ int ring_of(int i) { return i % kSRing; }
__device__ __forceinline__ int ring_add(int s, int d) {  // (s + d) mod kSRing, |d| < kSRing
    s += d;
    return s >= kSRing ? s - kSRing : (s < 0 ? s + kSRing : s);
}

// The roles of a streamed workgroup's waves (see the file comment), kSB rows
// per step each.  INT: every staged node is an interior node of the lattice.
template <int N, int C, bool FIRST, bool INT>
__device__ __forceinline__ void stream_roles(const CycleArgs& a, const CycleStep& st, int item, int X0, int Y0,
                                             int S, int rows, int wave, int lane, const float* __restrict__ src,
                                             float* __restrict__ dst, float* __restrict__ ur, float* __restrict__ rr,
                                             const double* cs, const double* cs2) {
    constexpr int NPD = node_pad(N);
    constexpr int MD = N * C + N;
    constexpr int RS = kSLX * NPD;  // floats per ring row (u)
    constexpr int RN = kSLX * N;    // floats per ring row (rhs)
    constexpr int B = kSB;
    const int W = a.W, H = a.H;
    const int64_t P = (int64_t)W * H;
    // steps until the residual level has passed the last output row
    const int nsteps = (rows - 6 + 5 * kSD + B) / B;
    // node lx of a ring row: slot index (even-x half first)
    auto nidx = [](int lx) { return (lx & 1) * (kSLX / 2) + (lx >> 1); };

    if (wave == 0) {
        // ---- stager: rows B t .. B t + B - 1 at step t, prefetched kSPd steps ahead
        const int lx = lane, gx = X0 - kSR + lx;
        const bool xin = INT || (gx >= 0 && gx < W);
        const int radx = max(max(kSR - lx, lx - (kSR + kSOut - 1)), 0);
        const int cls_x = (gx == 0) | (gx == W - 1);
        constexpr int NV = FIRST ? C : N;  // image (rhs built here) or stored rhs
        const int ni = nidx(lx);
        float pu[kSPd][B][N], pv[kSPd][B][NV];
        auto fetch = [&](int i, float (&u)[N], float (&v)[NV]) {
            const int gy = Y0 - kSR + i;
            const bool ok = i < rows && xin && (INT || (gy >= 0 && gy < H));
            const uint32_t g = ok ? (uint32_t)(gy * W + gx) : 0u;
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const float t = gload(src + c * P, g);
                u[c] = ok ? t : 0.f;
            }
#pragma unroll
            for (int c = 0; c < NV; ++c) v[c] = gload(FIRST ? a.image + c * P : a.rhs + c * P, g);
        };
#pragma unroll
        for (int d = 0; d < kSPd; ++d)
#pragma unroll
            for (int b = 0; b < B; ++b) fetch(B * d + b, pu[d][b], pv[d][b]);
        const double wd0 = uniform_d(a.rc.wd[0]);
        const float wda0 = uniform_f(a.rc.wda[0]);
        int sl = 0;
        for (int t = 0; t < nsteps; ++t) {
            if (B * t < rows) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int i = B * t + b;
                    const int gy = Y0 - kSR + i;
                    const int rady = max(max(kSR - i, i - (kSR + S - 1)), 0);
                    const int rad = max(radx, rady);
                    float rv[N];
                    if (FIRST) {
                        double wd = wd0;
                        float wda = wda0;
                        if (!INT) {
                            const int cls = cls_x + ((gy == 0) | (gy == H - 1));
                            const int klass = cls < 2 ? cls : (((gx == 0) == (gy == 0)) ? 2 : 3);
                            wd = sel4d(a.rc.wd, klass);
                            wda = sel4(a.rc.wda, klass);
                        }
                        double gc[N];
#pragma unroll
                        for (int c = 0; c < N; ++c) {
                            double t2 = cs2[c];
#pragma unroll
                            for (int k = 0; k < C; ++k) t2 = fma(cs[c * C + k], (double)pv[0][b][k], t2);
                            gc[c] = t2;
                        }
                        double gmax = gc[0];
#pragma unroll
                        for (int c = 1; c < N; ++c) gmax = fmax(gmax, gc[c]);
                        const double off = -wd * gmax;
#pragma unroll
                        for (int c = 0; c < N; ++c) rv[c] = fmaf(wda, pu[0][b][c], (float)fma(wd, gc[c], off));
                        if (st.store_rhs && rad == 0 && i < rows && (INT || (xin && gy >= 0 && gy < H)))
#pragma unroll
                            for (int c = 0; c < N; ++c)
                                gstore(const_cast<float*>(a.rhs + c * P), (uint32_t)(gy * W + gx), rv[c]);
                    } else {
#pragma unroll
                        for (int c = 0; c < N; ++c) rv[c] = pv[0][b][c];
                    }
                    const int slb = ring_add(sl, b);
                    lds_st<N>(ur + slb * RS + ni * NPD, pu[0][b]);
                    float* rp = rr + slb * RN + ni * N;
#pragma unroll
                    for (int c = 0; c < N; ++c) rp[c] = rv[c];
                }
                sl = ring_add(sl, B);
                // the next rows
#pragma unroll
                for (int d = 0; d + 1 < kSPd; ++d)
#pragma unroll
                    for (int b = 0; b < B; ++b) {
#pragma unroll
                        for (int c = 0; c < N; ++c) pu[d][b][c] = pu[d + 1][b][c];
#pragma unroll
                        for (int c = 0; c < NV; ++c) pv[d][b][c] = pv[d + 1][b][c];
                    }
#pragma unroll
                for (int b = 0; b < B; ++b) fetch(B * (t + kSPd) + b, pu[kSPd - 1][b], pv[kSPd - 1][b]);
            }
            __syncthreads();
        }
        return;
    }

    // ---- node updates.  Waves 1, 2: levels 1..4 (level k = 2 (wave - 1) + 1 +
    // half, half-sweep k - 1, writing); wave 3 lanes 0..31: level 5 (the
    // residual, a non-writing red half-sweep).  At step t level k works on rows
    // B t - kSD k .. + B - 1, its lane j on the node of its colour at column
    // k + parity + 2 j of each.
    const bool upd = wave < 3 || lane < 32;
    const int half = lane >> 5, j = lane & 31;
    const int k = wave < 3 ? 2 * (wave - 1) + 1 + half : 5;
    const int colour = (k - 1) & 1;
    // parity of the first node of the colour in staged row i: p0 ^ (i & 1)
    const int p0 = ((X0 - kSR + k) + (Y0 - kSR) + colour) & 1;
    int oc[2], ol[2], orr[2];  // node offsets in a ring row by parity: centre, left, right
    bool lok[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int lx = k + q + 2 * j;
        const int lxc = min(lx, kSLX - 2);  // clamp idle lanes into the row
        oc[q] = nidx(lxc);
        ol[q] = nidx(lxc - 1);
        orr[q] = nidx(lxc + 1);
        const int gx = X0 - kSR + lx;
        lok[q] = upd && lx <= kSLX - 1 - k && (INT || (gx >= 0 && gx < W));
    }
    const float kap0 = uniform_f(a.coef.kappa[0]);
    float res = 0.f;
    float acc[MD];
#pragma unroll
    for (int q = 0; q < MD; ++q) acc[q] = 0.f;
    constexpr int DS = 4 * kSD + B;  // the output rows trail the staging by DS rows
    for (int t = 0; t < nsteps; ++t) {
        const int i0 = B * t - kSD * k;
        // load every row's operands first, then update (independent rows)
        float v[B][N], o[B][N];
        bool act[B];
        int slv[B], qv[B], gyv[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            const int gy = Y0 - kSR + i;
            const int q = p0 ^ (i & 1);
            act[b] = i >= k && i <= rows - 1 - k && lok[q] && (INT || (gy >= 0 && gy < H));
            const int sl = act[b] ? ring_of(i) : 0;
            const int su = ring_add(sl, -1), sd = ring_add(sl, 1);
            slv[b] = sl;
            qv[b] = q;
            gyv[b] = gy;
            if (act[b]) {
                float a0[N], a1[N], a2[N], a3[N];
                lds_ld<N>(ur + sl * RS + ol[q] * NPD, a0);
                lds_ld<N>(ur + sl * RS + orr[q] * NPD, a1);
                lds_ld<N>(ur + su * RS + oc[q] * NPD, a2);
                lds_ld<N>(ur + sd * RS + oc[q] * NPD, a3);
                const float* rp = rr + sl * RN + oc[q] * N;
                float kh = kap0, kv = kap0;
                if (!INT) {
                    const int gx = X0 - kSR + k + q + 2 * j;
                    const int bx = (gx == 0) | (gx == W - 1), by = (gy == 0) | (gy == H - 1);
                    const int cls = bx + by;
                    const int klass = cls < 2 ? cls : (((gx == 0) == (gy == 0)) ? 2 : 3);
                    const float kap = sel4(a.coef.kappa, klass);
                    kh = by ? 0.5f * kap : kap;
                    kv = bx ? 0.5f * kap : kap;
                }
#pragma unroll
                for (int c = 0; c < N; ++c) v[b][c] = rp[c] + kh * (a0[c] + a1[c]) + kv * (a2[c] + a3[c]);
                if (k == 5) lds_ld<N>(ur + sl * RS + oc[q] * NPD, o[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            project_simplex<N, false>(v[b]);
            if (k == 5) {
#pragma unroll
                for (int c = 0; c < N; ++c) res = fmaxf(res, fabsf(v[b][c] - o[b][c]));
            } else {
                lds_st<N>(ur + slv[b] * RS + oc[qv[b]] * NPD, v[b]);
            }
        }
        (void)gyv;
        if (wave == 3) {
            // rows B t - DS .. + B - 1: finished (level 4 passed them last step)
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int io = B * t - DS + b;
                if (io < kSR || io >= kSR + S) continue;
                const int gy = Y0 - kSR + io, gx = X0 + lane;
                if (lane < kSOut && (INT || (gy < H && gx < W))) {
                    float uo[N];
                    lds_ld<N>(ur + ring_of(io) * RS + nidx(lane + kSR) * NPD, uo);
                    const uint32_t g = (uint32_t)(gy * W + gx);
#pragma unroll
                    for (int c = 0; c < N; ++c) gstore(dst + c * P, g, uo[c]);
                    if (st.cm) {
                        float w = 1.f;
                        if (!INT) {
                            const int bx = (gx == 0) | (gx == W - 1), by = (gy == 0) | (gy == H - 1);
                            const int cls = bx + by;
                            const int klass = cls < 2 ? cls : (((gx == 0) == (gy == 0)) ? 2 : 3);
                            w = (float)mass_w(klass);
                        }
                        float Ik[C];
#pragma unroll
                        for (int kk = 0; kk < C; ++kk) Ik[kk] = gload(a.image + kk * P, g);
#pragma unroll
                        for (int c = 0; c < N; ++c) {
                            const float wu = w * uo[c];
                            acc[N * C + c] += wu;
#pragma unroll
                            for (int kk = 0; kk < C; ++kk) acc[c * C + kk] += wu * Ik[kk];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (wave == 3) {
        // per-workgroup residual and colour-mean partials (this wave only, fixed order)
        const int row = st.cycle & 1;
        res = wave_max(res);
        if (lane == 0) a.res_part[row * a.part_stride + item] = res;
        if (st.cm) {
#pragma unroll
            for (int q = 0; q < MD; ++q) {
                const float v = wave_sum_last(acc[q]);
                if (lane == kWave - 1) a.cm_part[((int64_t)row * MD + q) * a.part_stride + item] = (double)v;
            }
        }
    }
}

template <int N, int C, bool FIRST>
__device__ __forceinline__ void stream_column(const CycleArgs& a, const CycleStep& st, int item) {
    constexpr int NPD = node_pad(N);
    constexpr int M = N * C + N + C + 2;
    constexpr int NT = M + N * C;
    extern __shared__ __attribute__((aligned(16))) float lds[];
    float* ur = lds;                                // u ring [kSRing][kSLX][NPD]
    float* rr = lds + kSRing * kSLX * NPD;          // rhs ring [kSRing][kSLX][N]
    __shared__ float red[kST / kWave];
    __shared__ double cs[N * C];  // 2 lambda c_ik (first launch of a step)
    __shared__ double cs2[N];     // -lambda |c_i|^2
    __shared__ double tsh[NT];
    __shared__ int flag;

    Ctl* ctl = a.ctl;
    StepSlot* slot = &ctl->step[st.slot];
    if (!st.fixed) {
        if (slot->done) return;  // uniform: an earlier cycle of this step converged
        if (st.first && st.cycle > 0) {
            const float* prev = a.res_part + ((st.cycle - 1) & 1) * a.part_stride;
            float r = 0.f;
            for (int b = threadIdx.x; b < a.ntiles; b += kST) r = fmaxf(r, prev[b]);
            r = wave_max(r);
            if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = r;
            __syncthreads();
            if (threadIdx.x == 0) {
                float m = red[0];
                for (int w = 1; w < kST / kWave; ++w) m = fmaxf(m, red[w]);
                flag = !(m > a.tol);
                if (flag && item == 0) {
                    slot->done = 1;
                    slot->cycles = st.cycle;
                    slot->resid = m;
                }
            }
            __syncthreads();
            if (flag) return;
        }
    }
    const int cur = __builtin_amdgcn_readfirstlane(iterate_buf(ctl->cur, st.launch));
    const int W = a.W, H = a.H, S = a.seg_rows;
    const int col = item / a.ssegs, seg = item - col * a.ssegs;
    const int X0 = col * kSOut, Y0 = seg * S;
    const int rows = S + 2 * kSR;  // staged rows Y0 - R .. Y0 + S + R - 1
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;

    // colour means of u^n (identical in every workgroup)
    const double* tot = a.tot + st.tot_sel * kCmeansMaxM;
    const double* c_prev64 = st.prev_sel >= 0 ? a.c64 + st.prev_sel * kNC : nullptr;
    if (FIRST) {
        if (threadIdx.x < NT) {
            const int t = threadIdx.x;
            const bool prev = t >= M;
            const double* src = prev ? (c_prev64 ? c_prev64 : tot) : tot;
            tsh[t] = src[prev ? t - M : t];
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
            const int i = threadIdx.x;
            bool empty = false;
            if (i < N) {
                const double area = tsh[N * C + N + C];
                const double Sm = tsh[N * C + i];
                const bool has_mass = !st.fixed_c && Sm > 1e-12 * area;
                empty = !st.fixed_c && !has_mass;
                double q2 = 0.0;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const double c = has_mass ? tsh[i * C + k] / Sm
                                              : (c_prev64 ? tsh[M + i * C + k] : tsh[N * C + N + k] / area);
                    cs[i * C + k] = 2.0 * a.rc.lambda * c;
                    q2 += c * c;
                    if (item == 0) {
                        a.c64[st.c64_sel * kNC + i * C + k] = c;
                        if (a.c_out) a.c_out[i * C + k] = (float)c;
                    }
                }
                cs2[i] = -a.rc.lambda * q2;
            }
            const bool any_empty = __any(empty);
            if (item == 0 && i == 0) {
                if (any_empty) ctl->empty_steps += 1;
                if (tsh[M - 1] > 0.0) ctl->nonfinite = 1;
            }
        }
        __syncthreads();
    }

    const float* __restrict__ src = a.bufs.b[cur];
    float* __restrict__ dst = const_cast<float*>(a.bufs.b[out_of(cur)]);
    // the whole staged block strictly inside the lattice: one node class, no bounds
    const bool in = X0 - kSR >= 1 && Y0 - kSR >= 1 && X0 - kSR + kSLX <= W - 1 && Y0 - kSR + rows <= H - 1;
    if (in)
        stream_roles<N, C, FIRST, true>(a, st, item, X0, Y0, S, rows, wave, lane, src, dst, ur, rr, cs, cs2);
    else
        stream_roles<N, C, FIRST, false>(a, st, item, X0, Y0, S, rows, wave, lane, src, dst, ur, rr, cs, cs2);
}

// Workgroup b of a single-image launch: XCD x = b mod 8 takes a contiguous
// range of items, column by column with the segments of a column in order,
// so a segment's upper neighbour (which shares its halo rows) ran just
// before it on the same XCD.
__device__ __forceinline__ int stream_item_of_block(const CycleArgs& a, int b) {
    const int x = b % kXcd, j = b / kXcd;
    const int it = x * a.sitems_per_xcd + j;
    return (j < a.sitems_per_xcd && it < a.ntiles) ? it : -1;
}

template <int N, int C, bool FIRST>
__global__ __launch_bounds__(kST) void k_stream(CycleArgs a, CycleStep st) {
    const int item = stream_item_of_block(a, blockIdx.x);
    if (item < 0) return;
    stream_column<N, C, FIRST>(a, st, item);
}

template <int N, int C, bool FIRST>
__global__ __launch_bounds__(kST) void k_stream_batch(const CycleArgs* __restrict__ descs,
                                                       const int2* __restrict__ work, int nwork, CycleStep st) {
    if ((int)blockIdx.x >= nwork) return;
    const int2 wv = work[blockIdx.x];
    if (wv.x < 0) return;
    stream_column<N, C, FIRST>(descs[wv.x], st, wv.y);
}

template <int N, int C, bool FIRST>
hipError_t run_stream(const CycleArgs& a, const CycleStep& st, const CycleGrid& g, hipStream_t s) {
    constexpr int lds = stream_lds_bytes<N>();
    if (g.descs)
        hipLaunchKernelGGL((k_stream_batch<N, C, FIRST>), dim3(g.nwork), dim3(kST), lds, s, g.descs, g.work,
                           g.nwork, st);
    else
        hipLaunchKernelGGL((k_stream<N, C, FIRST>), dim3(a.sitems_per_xcd * kXcd), dim3(kST), lds, s, a, st);
    return hipGetLastError();
}

}  // namespace acseg
