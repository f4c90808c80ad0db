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
//      of red-black Gauss-Seidel sweeps.  Each large level is one tiled pass
//      down (sweeps from zero, residual, restriction) and one up
//      (prolongation, sweeps), every tile staged in LDS with the halo its
//      sweeps need; the small levels (sides <= kTailSide) run as one V-cycle
//      in one workgroup per component;
//   4. direction w_p = Pi(u_p + T_I (P v_1)_p) - u_p (feasible, since the
//      simplex is convex), and the exact line search on the step's quadratic
//      along w: alpha = clamp(<g~, w> / <w, H w>, 0, 1), u += alpha w.  Each
//      workgroup of the direction pass leaves its partial sums of the two
//      dot products; the post-smoothing launch reduces them to alpha and
//      applies the update as it stages u.
//      w vanishes on the active components and sums to zero over the free
//      ones at every node, so <g, w> = <g~, w>; the truncated form keeps the
//      per-node multiplier of the sum constraint out of the dot product.
//
// Units: every level is scaled by 1/h^2 of the finest spacing; the defect is
// D_p (y_p - u_p) with y_p the nodal map of the smoother.  The stored
// right-hand side is shifted per node by a constant vector, which T_I removes.
#include <algorithm>
#include <atomic>

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
    // the second coarse node: right, below, or along the diagonal (itself on a coarse node)
    const float r1 = r0[ao * (bo ? Wc + 1 : 1) + (ao ? 0 : bo * Wc)];
    return (ao | bo) ? 0.5f * (r0[0] + r1) : r0[0];
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

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------

// floor(q / d) for 0 <= q < 2^20 and 1 <= d < 2^20, with inv = 1.0f / d: the
// quotient of q + 1/2 lies at least 1/(2d) from an integer, further than the
// rounding error of the product (below 2^-3 / d for q < 2^20).
__device__ __forceinline__ int fdiv(int q, float inv) { return (int)(((float)q + 0.5f) * inv); }

__device__ __forceinline__ double block_sum_d(double v, double* sh /* kBlock/kWave */) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// The step's state for a pass, loaded in one round: whether the step has
// converged (the pass then does nothing) and the buffer holding the iterate.
struct MgState {
    bool skip;
    float* u;  // bufs[iterate_buf(ctl->cur, launch)]
};

__device__ __forceinline__ MgState mg_state(const MgImage& d, const MgStep& st) {
    const Ctl* ctl = d.ctl;
    const int done = ctl->step[st.slot].done;
    const int cur = ctl->cur;
    MgState m;
    m.skip = !st.fixed && __builtin_amdgcn_readfirstlane(done) != 0;
    m.u = const_cast<float*>(d.bufs.b[__builtin_amdgcn_readfirstlane(iterate_buf(cur, st.launch))]);
    return m;
}

__device__ __forceinline__ bool mg_skip(const MgImage& d, const MgStep& st) { return mg_state(d, st).skip; }

// Red-black half-sweep of linear Gauss-Seidel for H v = r on a block of a
// level held in LDS (row pitch SX, origin (sx0, sy0) in level coordinates):
// the nodes of `colour` ((x + y) & 1) strictly inside the block and inside the
// W x H lattice get v = r / D + kappa sum_q c_pq v_q.  Nodes outside the
// lattice hold 0 and are never updated, which makes the sum over the lattice
// neighbours only.  INT: the whole block lies inside the lattice's interior
// (one node class, unit edge weights, no bounds).  T threads.
template <int T, bool INT>
__device__ __forceinline__ void block_half(float* __restrict__ v, const float* __restrict__ r, int SX, int SY,
                                           int sx0, int sy0, int W, int H, const LevelCoef& c, int colour) {
    const int hw = (SX - 1) / 2;  // nodes of one colour per block row, at most
    const float inv = 1.0f / (float)hw;
    const int total = hw * (SY - 2);
    const float k0 = uniform_f(c.kappa[0]), i0 = uniform_f(c.inv_d[0]);
    for (int q = threadIdx.x; q < total; q += T) {
        const int row = fdiv(q, inv), j = q - row * hw;
        const int ly = row + 1, gy = sy0 + ly;
        const int lx0 = 1 + ((sx0 + 1 + gy + colour) & 1);  // first node of the colour in the row
        const int lx = lx0 + 2 * j, gx = sx0 + lx;
        if (lx > SX - 2) continue;
        const int p = ly * SX + lx;
        if (INT) {
            v[p] = fmaf(k0, (v[p - 1] + v[p + 1]) + (v[p - SX] + v[p + SX]), r[p] * i0);
        } else {
            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
            const int cls = node_class(gx, gy, W, H);
            const float nb = edge_w_h(gy, H) * (v[p - 1] + v[p + 1]) + edge_w_v(gx, W) * (v[p - SX] + v[p + SX]);
            v[p] = fmaf(sel4(c.kappa, cls), nb, r[p] * sel4(c.inv_d, cls));
        }
    }
}

// Whether a block of SX x SY level nodes at (sx0, sy0) lies strictly inside the lattice.
__device__ __forceinline__ bool block_interior(int sx0, int sy0, int SX, int SY, int W, int H) {
    return sx0 >= 1 && sy0 >= 1 && sx0 + SX <= W - 1 && sy0 + SY <= H - 1;
}

// (r - H v) at level node (gx, gy), block position p (lattice neighbours in the block).
__device__ __forceinline__ float block_resid(const float* __restrict__ v, const float* __restrict__ r, int SX,
                                             int p, int gx, int gy, int W, int H, const LevelCoef& c) {
    const float nb = edge_w_h(gy, H) * (v[p - 1] + v[p + 1]) + edge_w_v(gx, W) * (v[p - SX] + v[p + SX]);
    return r[p] - (sel4(c.d, node_class(gx, gy, W, H)) * v[p] - c.e2 * nb);
}

// Stage N planes of a field on an SX x SY block at (sx0, sy0) into LDS
// dst[N][SY][SX] (0 outside the lattice): every load of a thread issued before
// any store, so their latencies overlap.
template <int N, int SX, int SY>
__device__ __forceinline__ void stage_planes(float* __restrict__ dst, const float* __restrict__ src, uint32_t n,
                                             int sx0, int sy0, int W, int H) {
    constexpr int Q = (SX * SY + kBlock - 1) / kBlock;
    float t[Q][N];
    bool ok[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int q = threadIdx.x + c * kBlock;
        const int ly = q / SX, lx = q - ly * SX;
        const int gx = sx0 + lx, gy = sy0 + ly;
        ok[c] = q < SX * SY && gx >= 0 && gx < W && gy >= 0 && gy < H;
        const uint32_t g = ok[c] ? (uint32_t)(gy * W + gx) : 0u;
#pragma unroll
        for (int i = 0; i < N; ++i) t[c][i] = gload(src + i * n, g);
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int q = threadIdx.x + c * kBlock;
        if (q < SX * SY) {
#pragma unroll
            for (int i = 0; i < N; ++i) dst[i * SX * SY + q] = ok[c] ? t[c][i] : 0.f;
        }
    }
}

// ---------------------------------------------------------------------------
// 1-2. Truncated defect of the finest level, restricted to level 1: one
// workgroup per kDrTX x kDrTY level-1 nodes.  The fine nodes those reach
// (2X0-1 .. 2X0+2 kDrTX-1) get their truncated defect once, from u staged
// with a halo of one.
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ void mg_defect_restrict(const MgImage& d, int tile, const MgStep& st) {
    constexpr int SX = 2 * kDrTX + 3, SY = 2 * kDrTY + 3;
    constexpr int FX = 2 * kDrTX + 1, FY = 2 * kDrTY + 1;
    static_assert(kDrTX * kDrTY == kBlock, "one level-1 node per thread");
    __shared__ float us[N][SY][SX];
    __shared__ float gs[N][FY][FX];
    const MgLevel c = d.lv[1];
    const int W = d.W, H = d.H, Wc = c.W, Hc = c.H;
    const MgState ms = mg_state(d, st);
    if (ms.skip) return;
    if (st.check > 0 && !st.fixed) {
        // The test that opens cycle st.check when one launch smooths both after
        // the previous correction and before this one: the residual that launch
        // left.  Every workgroup reduces the same partials, so all take the
        // same decision; workgroup 0 records it.
        __shared__ float red[kBlock / kWave];
        __shared__ int stop;
        const float* prev = d.res_part + ((st.check - 1) & 1) * d.part_stride;
        float r = 0.f;
        for (int b = threadIdx.x; b < d.ntiles; b += kBlock) r = fmaxf(r, prev[b]);
        r = block_max(r, red);
        if (threadIdx.x == 0) {
            stop = !(r > d.tol);
            if (stop && tile == 0) {
                StepSlot* slot = &d.ctl->step[st.slot];
                slot->done = 1;
                slot->cycles = st.check;
                slot->resid = r;
            }
        }
        __syncthreads();
        if (stop) return;
    }
    const int tx = (Wc + kDrTX - 1) / kDrTX;
    const int X0 = (tile % tx) * kDrTX, Y0 = (tile / tx) * kDrTY;
    const int sx0 = 2 * X0 - 2, sy0 = 2 * Y0 - 2;
    const uint32_t n = (uint32_t)W * H, nc = (uint32_t)Wc * Hc;
    const float* u = ms.u;
    stage_planes<N, SX, SY>(&us[0][0][0], u, n, sx0, sy0, W, H);
    __syncthreads();
    for (int q = threadIdx.x; q < FX * FY; q += kBlock) {
        const int fy = q / FX, fx = q - fy * FX;
        const int gx = sx0 + 1 + fx, gy = sy0 + 1 + fy;
        if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;  // never restricted
        const int lx = fx + 1, ly = fy + 1;
        const int cls = node_class(gx, gy, W, H);
        const float kap = sel4(d.fine.kappa, cls), D = sel4(d.fine.d, cls);
        const float ewh = edge_w_h(gy, H), ewv = edge_w_v(gx, W);
        const uint32_t p = (uint32_t)(gy * W + gx);
        float g[N];
        bool fr[N];
        float sum = 0.f;
        int k = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float uc = us[i][ly][lx];
            const float nb = ewh * (us[i][ly][lx - 1] + us[i][ly][lx + 1]) + ewv * (us[i][ly - 1][lx] + us[i][ly + 1][lx]);
            const float yv = gload(d.rhs + i * n, p) + kap * nb;
            g[i] = D * (yv - uc);
            fr[i] = uc > 0.f;
            if (fr[i]) {
                sum += g[i];
                ++k;
            }
        }
        const float mean = k > 0 ? sum / (float)k : 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) gs[i][fy][fx] = (k >= 2 && fr[i]) ? g[i] - mean : 0.f;
    }
    __syncthreads();
    const int X = X0 + threadIdx.x % kDrTX, Y = Y0 + threadIdx.x / kDrTX;
    if (X >= Wc || Y >= Hc) return;
    float r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = 0.f;
    for_restrict(W, H, Wc, Hc, X, Y, [&](int x, int y, float wt) {
        const int fx = x - (sx0 + 1), fy = y - (sy0 + 1);
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] += wt * gs[i][fy][fx];
    });
#pragma unroll
    for (int i = 0; i < N; ++i) gstore(c.r + i * nc, (uint32_t)(Y * Wc + X), r[i]);
}

// ---------------------------------------------------------------------------
// 3a. Down-leg of level l (1 <= l < tail): nu red-black sweeps of H_l v = r_l
// from v = 0, then r_{l+1} = P^T (r_l - H_l v).  One workgroup per kDnTX x
// kDnTY level-(l+1) nodes and component.  The level-l nodes that restriction
// reaches (2X0-1 .. 2X0+2 kDnTX-1) need v with a halo of one; v after the
// sweeps is exact on the block less 2 nu nodes at its rim (the first
// half-sweep from zero reads no neighbour, every later one loses a ring, and
// the rim itself is never updated), so the block is that region plus
// 2 nu + 1.  The workgroup writes v of the level-l nodes 2X0 .. 2X0+2 kDnTX-1.
// ---------------------------------------------------------------------------

__host__ __device__ inline int down_halo(int nu) { return 2 * nu + 1; }
__host__ __device__ inline int down_sx(int nu) { return 2 * kDnTX + 1 + 2 * down_halo(nu); }
__host__ __device__ inline int down_sy(int nu) { return 2 * kDnTY + 1 + 2 * down_halo(nu); }

template <int T>
__device__ __forceinline__ void mg_down(const MgImage& d, int tile, const MgStep& st, int comp) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int l = st.level, nu = st.sweeps;
    const MgLevel f = d.lv[l];
    const MgLevel c = d.lv[l + 1];
    if (comp >= d.N || mg_skip(d, st)) return;
    const int W = f.W, H = f.H, Wc = c.W, Hc = c.H;
    const int tx = (Wc + kDnTX - 1) / kDnTX;
    const int X0 = (tile % tx) * kDnTX, Y0 = (tile / tx) * kDnTY;
    const int hal = down_halo(nu), SX = down_sx(nu), SY = down_sy(nu);
    const int sx0 = 2 * X0 - 1 - hal, sy0 = 2 * Y0 - 1 - hal;
    const uint32_t n = (uint32_t)W * H, nc = (uint32_t)Wc * Hc;
    float* rs = lds;
    float* vs = lds + SX * SY;
    const float* r = f.r + comp * n;
    const float inv = 1.0f / (float)SX;
    constexpr int CH = T >= 1024 ? 4 : 8;  // loads in flight per thread (one or two rounds for nu <= 2)
    for (int base = 0; base < SX * SY; base += CH * T) {
        float t[CH];
        bool ok[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int q = base + k * T + threadIdx.x;
            const int ly = fdiv(q, inv), lx = q - ly * SX;
            const int gx = sx0 + lx, gy = sy0 + ly;
            ok[k] = q < SX * SY && gx >= 0 && gx < W && gy >= 0 && gy < H;
            t[k] = gload(r, ok[k] ? (uint32_t)(gy * W + gx) : 0u);
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int q = base + k * T + threadIdx.x;
            if (q < SX * SY) {
                rs[q] = ok[k] ? t[k] : 0.f;
                vs[q] = 0.f;
            }
        }
    }
    const bool in = block_interior(sx0, sy0, SX, SY, W, H);
    for (int h = 0; h < 2 * nu; ++h) {
        __syncthreads();
        if (in)
            block_half<T, true>(vs, rs, SX, SY, sx0, sy0, W, H, f.coef, h & 1);
        else
            block_half<T, false>(vs, rs, SX, SY, sx0, sy0, W, H, f.coef, h & 1);
    }
    __syncthreads();
    // r_{l+1} = P^T (r - H v) on this workgroup's level-(l+1) nodes
    for (int q = threadIdx.x; q < kDnTX * kDnTY; q += T) {
        const int X = X0 + q % kDnTX, Y = Y0 + q / kDnTX;
        if (X >= Wc || Y >= Hc) continue;
        float sum = 0.f;
        for_restrict(W, H, Wc, Hc, X, Y, [&](int x, int y, float wt) {
            sum += wt * block_resid(vs, rs, SX, (y - sy0) * SX + (x - sx0), x, y, W, H, f.coef);
        });
        gstore(c.r + comp * nc, (uint32_t)(Y * Wc + X), sum);
    }
    // v of the owned level-l nodes
    float* v = f.v + comp * n;
    for (int q = threadIdx.x; q < 4 * kDnTX * kDnTY; q += T) {
        const int ox = q % (2 * kDnTX), oy = q / (2 * kDnTX);
        const int gx = 2 * X0 + ox, gy = 2 * Y0 + oy;
        if (gx >= W || gy >= H) continue;
        gstore(v, (uint32_t)(gy * W + gx), vs[(gy - sy0) * SX + (gx - sx0)]);
    }
}

// ---------------------------------------------------------------------------
// 3c. Up-leg of level l: v = v_down + P v2_{l+1} (or v = 0 on the coarsest
// level when no LDS tail solves it), then nu red-black sweeps of H_l v = r_l;
// the result goes to v2.  One workgroup per kUpTX x kUpTY level-l nodes and
// component, staged with a halo of 2 nu: each half-sweep, which updates the
// block less its rim, loses one ring of exact values.
// ---------------------------------------------------------------------------

__host__ __device__ inline int up_sx(int nu) { return kUpTX + 4 * nu; }
__host__ __device__ inline int up_sy(int nu) { return kUpTY + 4 * nu; }
// the coarser level's block that the prolongation reads for the staged nodes
__host__ __device__ inline int up_cx(int nu) { return up_sx(nu) / 2 + 2; }
__host__ __device__ inline int up_cy(int nu) { return up_sy(nu) / 2 + 2; }

template <int T>
__device__ __forceinline__ void mg_up(const MgImage& d, int tile, const MgStep& st, int comp) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int l = st.level, nu = st.sweeps;
    const MgLevel f = d.lv[l];
    const bool zero = st.zero != 0;
    const MgLevel c = d.lv[zero ? l : l + 1];
    if (comp >= d.N || mg_skip(d, st)) return;
    const int W = f.W, H = f.H;
    const int tx = (W + kUpTX - 1) / kUpTX;
    const int x0 = (tile % tx) * kUpTX, y0 = (tile / tx) * kUpTY;
    const int SX = up_sx(nu), SY = up_sy(nu);
    const int sx0 = x0 - 2 * nu, sy0 = y0 - 2 * nu;
    const uint32_t n = (uint32_t)W * H;
    float* rs = lds;
    float* vs = lds + SX * SY;
    float* cs = lds + 2 * SX * SY;  // the coarser block, CX x CY
    const float* r = f.r + comp * n;
    const float* vd = f.v + comp * n;
    const float* vc = c.v2 + (size_t)comp * c.W * c.H;
    const int CX = up_cx(nu), CY = up_cy(nu);
    const int cx0 = max(sx0, 0) >> 1, cy0 = max(sy0, 0) >> 1;
    if (!zero) {
        for (int q = threadIdx.x; q < CX * CY; q += T) {
            const int qy = q / CX, qx = q - qy * CX;
            const int X = cx0 + qx, Y = cy0 + qy;
            const bool ok = X < c.W && Y < c.H;
            const float t = gload(vc, ok ? (uint32_t)(Y * c.W + X) : 0u);
            cs[q] = ok ? t : 0.f;
        }
        __syncthreads();
    }
    const float inv = 1.0f / (float)SX;
    constexpr int CH = T >= 1024 ? 2 : 4;  // staged nodes in flight per thread (one or two rounds for nu <= 2)
    for (int base = 0; base < SX * SY; base += CH * T) {
        float t[CH], v[CH];
        bool ok[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int q = base + k * T + threadIdx.x;
            const int ly = fdiv(q, inv), lx = q - ly * SX;
            const int gx = sx0 + lx, gy = sy0 + ly;
            ok[k] = q < SX * SY && gx >= 0 && gx < W && gy >= 0 && gy < H;
            const uint32_t g = ok[k] ? (uint32_t)(gy * W + gx) : 0u;
            t[k] = gload(r, g);
            v[k] = (ok[k] && !zero) ? gload(vd, g) : 0.f;
            if (ok[k] && !zero) {
                // P v2 at (gx, gy) from the staged block (as prolong_at)
                const int pa = min(gx, 2 * c.W - 2), pb = min(gy, 2 * c.H - 2);
                const int o = ((pb >> 1) - cy0) * CX + ((pa >> 1) - cx0);
                const int dxo = pa & 1, dyo = pb & 1;
                const float c00 = cs[o];
                v[k] += dxo ? 0.5f * (c00 + cs[o + dyo * CX + 1]) : (dyo ? 0.5f * (c00 + cs[o + CX]) : c00);
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int q = base + k * T + threadIdx.x;
            if (q < SX * SY) {
                rs[q] = ok[k] ? t[k] : 0.f;
                vs[q] = v[k];
            }
        }
    }
    const bool in = block_interior(sx0, sy0, SX, SY, W, H);
    for (int h = 0; h < 2 * nu; ++h) {
        __syncthreads();
        if (in)
            block_half<T, true>(vs, rs, SX, SY, sx0, sy0, W, H, f.coef, h & 1);
        else
            block_half<T, false>(vs, rs, SX, SY, sx0, sy0, W, H, f.coef, h & 1);
    }
    __syncthreads();
    float* v2 = f.v2 + comp * n;
    for (int q = threadIdx.x; q < kUpTX * kUpTY; q += T) {
        const int gx = x0 + q % kUpTX, gy = y0 + q / kUpTX;
        if (gx >= W || gy >= H) continue;
        gstore(v2, (uint32_t)(gy * W + gx), vs[(gy - sy0) * SX + (gx - sx0)]);
    }
}

// ---------------------------------------------------------------------------
// 3b. LDS tail: the V-cycle over levels t = tail .. L-1 (sides <= kTailSide)
// of one component in one workgroup of kTailThreads, v and r of every level
// in LDS.  A restriction first writes the fine level's residual to an LDS
// scratch, then every coarse node gathers from it.  The levels' sizes,
// coefficients and LDS offsets are copied to LDS once, so the dozens of
// steps that follow read them there instead of waiting on scalar loads of the
// descriptor.  The result v_t goes to v2 of level t.
// ---------------------------------------------------------------------------

struct TailLevel {
    LevelCoef coef;
    int W, H, off;  // off: float offset of v in the LDS field area (r follows v)
    int pad;
};

// A level's coefficients per node class, read once into wave-uniform registers.
struct TailCoef {
    float kappa[4], inv_d[4], d[4], e2;
};

__device__ __forceinline__ TailCoef tail_coef(const LevelCoef& c) {
    TailCoef t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        t.kappa[k] = uniform_f(c.kappa[k]);
        t.inv_d[k] = uniform_f(c.inv_d[k]);
        t.d[k] = uniform_f(c.d[k]);
    }
    t.e2 = uniform_f(c.e2);
    return t;
}

__device__ __forceinline__ float pick4(const float (&a)[4], int k) {
    return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}

// sum_q c_pq v_q over the lattice neighbours of node (x, y) at p, without
// branches: a missing neighbour's read takes the node itself (in bounds) and a
// select drops it, so the waves that hold boundary nodes do not diverge.
__device__ __forceinline__ float lattice_nb(const float* __restrict__ v, int W, int H, int x, int y, int p) {
    const bool lf = x > 0, rt = x < W - 1, up = y > 0, dn = y < H - 1;
    const float a = v[lf ? p - 1 : p], b = v[rt ? p + 1 : p];
    const float c = v[up ? p - W : p], e = v[dn ? p + W : p];
    return edge_w_h(y, H) * ((lf ? a : 0.f) + (rt ? b : 0.f)) + edge_w_v(x, W) * ((up ? c : 0.f) + (dn ? e : 0.f));
}

// The nodes of `colour` ((x + y) & 1) of a W x H level: v = r / D + kappa
// sum_q c_pq v_q (zero: v is 0 beforehand, so v = r / D).  Lanes `lane`,
// lane + T, ... of the T threads that take part.
template <int T>
__device__ __forceinline__ void tail_half(float* __restrict__ v, const float* __restrict__ r, int W, int H,
                                          const TailCoef& c, int colour, bool zero, int lane) {
    const int hw = (W + 1) / 2;
    const float inv = 1.0f / (float)hw;
    for (int q = lane; q < hw * H; q += T) {
        const int y = fdiv(q, inv), j = q - y * hw;
        const int x = 2 * j + ((y + colour) & 1);
        if (x >= W) continue;
        const int p = y * W + x;
        const int cls = node_class(x, y, W, H);
        const float rd = r[p] * pick4(c.inv_d, cls);
        if (zero)
            v[p] = rd;
        else
            v[p] = fmaf(pick4(c.kappa, cls), lattice_nb(v, W, H, x, y, p), rd);
    }
}

__device__ __forceinline__ void tail_sweeps(float* v, const float* r, int W, int H, const TailCoef& c, int sweeps,
                                            bool zero) {
    for (int s = 0; s < sweeps; ++s) {
        tail_half<kTailThreads>(v, r, W, H, c, 0, zero && s == 0, threadIdx.x);
        __syncthreads();
        tail_half<kTailThreads>(v, r, W, H, c, 1, false, threadIdx.x);
        __syncthreads();
    }
}

// The same sweeps on a small level by wavefront 0 alone.  The LDS accesses of
// one wavefront take effect in the order it issues them, so its half-sweeps
// need no workgroup barrier between them, only a fence that keeps the compiler
// from moving LDS accesses across.
constexpr int kTailWaveNodes = 256;

__device__ __forceinline__ void tail_sweeps_wave(float* v, const float* r, int W, int H, const TailCoef& c,
                                                 int sweeps, bool zero) {
    if (threadIdx.x < kWave) {
        for (int s = 0; s < sweeps; ++s) {
            tail_half<kWave>(v, r, W, H, c, 0, zero && s == 0, threadIdx.x);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            tail_half<kWave>(v, r, W, H, c, 1, false, threadIdx.x);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
    }
    __syncthreads();
}

// rc = P^T (r - H v) from level (W, H) to (Wc, Hc): the residual of every fine
// node goes to s, then every coarse node sums its weighted fine nodes from s.
__device__ __forceinline__ void tail_resid_restrict(const float* __restrict__ v, const float* __restrict__ r,
                                                    int W, int H, const TailCoef& c, float* __restrict__ rc,
                                                    int Wc, int Hc, float* __restrict__ s) {
    const float inv = 1.0f / (float)W;
    for (int q = threadIdx.x; q < W * H; q += kTailThreads) {
        const int y = fdiv(q, inv), x = q - y * W;
        s[q] = r[q] - (pick4(c.d, node_class(x, y, W, H)) * v[q] - c.e2 * lattice_nb(v, W, H, x, y, q));
    }
    __syncthreads();
    const float invc = 1.0f / (float)Wc;
    for (int q = threadIdx.x; q < Wc * Hc; q += kTailThreads) {
        const int Y = fdiv(q, invc), X = q - Y * Wc;
        rc[q] = restrict_at(s, W, H, Wc, Hc, X, Y);
    }
    __syncthreads();
}

__device__ __forceinline__ void tail_prolong_add(float* __restrict__ v, int W, int H, const float* __restrict__ vc,
                                                 int Wc, int Hc) {
    const float inv = 1.0f / (float)W;
    for (int q = threadIdx.x; q < W * H; q += kTailThreads) {
        const int y = fdiv(q, inv), x = q - y * W;
        v[q] += prolong_at(vc, Wc, Hc, x, y);
    }
    __syncthreads();
}

// Level t's r is read into registers before anything else (the workgroup's
// kTailPre loads per thread overlap the convergence check and the descriptor
// copy); levels tail..L-1 then follow in LDS, then the residual scratch s.
constexpr int kTailPre = (kTailSide * kTailSide + kTailThreads - 1) / kTailThreads;

__device__ __forceinline__ void mg_tail(const MgImage& d, const MgStep& st, int comp) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ TailLevel tl[kMaxLevels];
    if (comp >= d.N) return;
    const int t = d.tail, L = d.L;
    const int Wt = d.lv[t].W, Ht = d.lv[t].H;
    const uint32_t nt = (uint32_t)Wt * Ht;
    float pre[kTailPre];
    {
        const float* rt = d.lv[t].r + comp * nt;
#pragma unroll
        for (int k = 0; k < kTailPre; ++k) {
            const uint32_t q = threadIdx.x + k * kTailThreads;
            pre[k] = q < nt ? gload(rt, q) : 0.f;
        }
    }
    if (mg_skip(d, st)) return;
    int off = 0;
    for (int l = t; l < L; ++l) {
        if (threadIdx.x == 0) {
            tl[l].coef = d.lv[l].coef;
            tl[l].W = d.lv[l].W;
            tl[l].H = d.lv[l].H;
            tl[l].off = off;
        }
        off += 2 * d.lv[l].W * d.lv[l].H;
    }
    float* const s = lds + off;
    {
        float* r0 = lds + nt;  // level t's v starts at offset 0
#pragma unroll
        for (int k = 0; k < kTailPre; ++k) {
            const uint32_t q = threadIdx.x + k * kTailThreads;
            if (q < nt) r0[q] = pre[k];
        }
        __syncthreads();
    }
    for (int l = t; l < L; ++l) {  // down
        const TailLevel& g = tl[l];
        const TailCoef c = tail_coef(g.coef);
        float* v = lds + g.off;
        float* r = v + g.W * g.H;
        if (l == L - 1) {
            if (g.W * g.H <= kTailWaveNodes)
                tail_sweeps_wave(v, r, g.W, g.H, c, d.coarse_sweeps, true);
            else
                tail_sweeps(v, r, g.W, g.H, c, d.coarse_sweeps, true);
        } else {
            tail_sweeps(v, r, g.W, g.H, c, st.nu_pre, true);
            const TailLevel& n = tl[l + 1];
            tail_resid_restrict(v, r, g.W, g.H, c, lds + n.off + n.W * n.H, n.W, n.H, s);
        }
    }
    for (int l = L - 2; l >= t; --l) {  // up
        const TailLevel& g = tl[l];
        const TailLevel& n = tl[l + 1];
        const TailCoef c = tail_coef(g.coef);
        float* v = lds + g.off;
        tail_prolong_add(v, g.W, g.H, lds + n.off, n.W, n.H);
        tail_sweeps(v, v + g.W * g.H, g.W, g.H, c, st.nu_post, false);
    }
    float* out = d.lv[t].v2 + comp * nt;
    for (int q = threadIdx.x; q < (int)nt; q += kTailThreads) gstore(out, (uint32_t)q, lds[q]);
}

// ---------------------------------------------------------------------------
// 4a. Direction w = Pi(u + T_I P v2_1) - u and the line-search partials
// <g~, w>, <w, H w>: workgroup b of an image takes the kDirTX x kDirTY fine
// tiles b, b + dir_blocks, ...; per tile w on the tile and a ring of one (for
// H w) from u staged with that ring, g~ on the tile.  Each workgroup leaves
// its two sums; the smoothing launch after the correction reduces them to the
// step length and applies the update as it stages u.
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ void mg_dir(const MgImage& d, int blk, const MgStep& st) {
    constexpr int SX = kDirTX + 2, SY = kDirTY + 2;
    // the level-1 nodes the prolongation reads for the staged fine nodes
    // (x0 - 1 .. x0 + kDirTX, and the right / lower neighbour of each)
    constexpr int CX = kDirTX / 2 + 3, CY = kDirTY / 2 + 3;
    __shared__ float us[N][SY][SX];
    __shared__ float ws[N][SY][SX];
    __shared__ float vcs[N][CY][CX];
    __shared__ double sh[kBlock / kWave];
    const int W = d.W, H = d.H;
    const MgLevel c = d.lv[1];
    const MgState ms = mg_state(d, st);
    if (ms.skip) return;
    const int tx = (W + kDirTX - 1) / kDirTX;
    const int ntiles = tx * ((H + kDirTY - 1) / kDirTY);
    const uint32_t n = (uint32_t)W * H, nc = (uint32_t)c.W * c.H;
    const float* u = ms.u;
    double gw = 0.0, whw = 0.0;
    for (int tile = blk; tile < ntiles; tile += d.dir_blocks) {
        const int x0 = (tile % tx) * kDirTX, y0 = (tile / tx) * kDirTY;
        const int sx0 = x0 - 1, sy0 = y0 - 1;
        const int cx0 = max(sx0, 0) >> 1, cy0 = max(sy0, 0) >> 1;
        __syncthreads();  // the previous tile's reads of us / ws / vcs are done
        stage_planes<N, CX, CY>(&vcs[0][0][0], c.v2, nc, cx0, cy0, c.W, c.H);
        stage_planes<N, SX, SY>(&us[0][0][0], u, n, sx0, sy0, W, H);
        __syncthreads();
#pragma unroll
        for (int q = threadIdx.x; q < SX * SY; q += kBlock) {
            const int ly = q / SX, lx = q - ly * SX;
            const int gx = sx0 + lx, gy = sy0 + ly;
            float w[N];
#pragma unroll
            for (int i = 0; i < N; ++i) w[i] = 0.f;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                float uc[N], v[N];
                int k = 0;
                float s = 0.f;
                // P v2_1 at (gx, gy) from the staged level-1 block (as prolong_at)
                const int pa = min(gx, 2 * c.W - 2), pb = min(gy, 2 * c.H - 2);
                const int cxl = (pa >> 1) - cx0, cyl = (pb >> 1) - cy0;
                const int dxo = pa & 1, dyo = pb & 1;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    uc[i] = us[i][ly][lx];
                    const float v00 = vcs[i][cyl][cxl];
                    v[i] = dxo ? 0.5f * (v00 + vcs[i][cyl + dyo][cxl + 1])
                               : (dyo ? 0.5f * (v00 + vcs[i][cyl + 1][cxl]) : v00);
                    if (uc[i] > 0.f) {
                        s += v[i];
                        ++k;
                    }
                }
                if (k >= 2) {
                    const float mean = s / (float)k;
                    float xv[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) xv[i] = uc[i] + (uc[i] > 0.f ? v[i] - mean : 0.f);
                    project_simplex<N>(xv);
#pragma unroll
                    for (int i = 0; i < N; ++i) w[i] = xv[i] - uc[i];
                }
            }
#pragma unroll
            for (int i = 0; i < N; ++i) ws[i][ly][lx] = w[i];
        }
        __syncthreads();
#pragma unroll
        for (int q = threadIdx.x; q < kDirTX * kDirTY; q += kBlock) {
            const int ox = q % kDirTX, oy = q / kDirTX;
            const int gx = x0 + ox, gy = y0 + oy;
            if (gx >= W || gy >= H) continue;
            const int lx = ox + 1, ly = oy + 1;
            const int cls = node_class(gx, gy, W, H);
            const float kap = sel4(d.fine.kappa, cls), D = sel4(d.fine.d, cls);
            const float ewh = edge_w_h(gy, H), ewv = edge_w_v(gx, W);
            const uint32_t p = (uint32_t)(gy * W + gx);
            float g[N];
            bool fr[N];
            float sum = 0.f;
            int k = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float uc = us[i][ly][lx];
                const float nb = ewh * (us[i][ly][lx - 1] + us[i][ly][lx + 1]) + ewv * (us[i][ly - 1][lx] + us[i][ly + 1][lx]);
                g[i] = D * (gload(d.rhs + i * n, p) + kap * nb - uc);
                fr[i] = uc > 0.f;
                if (fr[i]) {
                    sum += g[i];
                    ++k;
                }
            }
            const float mean = k > 0 ? sum / (float)k : 0.f;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float gt = (k >= 2 && fr[i]) ? g[i] - mean : 0.f;
                const float wc = ws[i][ly][lx];
                const float nbw = ewh * (ws[i][ly][lx - 1] + ws[i][ly][lx + 1]) + ewv * (ws[i][ly - 1][lx] + ws[i][ly + 1][lx]);
                const float hw = D * wc - d.fine.e2 * nbw;
                gw += (double)gt * (double)wc;
                whw += (double)wc * (double)hw;
                gstore(d.gt + i * n, p, wc);
            }
        }
    }
    const double tg = block_sum_d(gw, sh);
    const double tq = block_sum_d(whw, sh);
    if (threadIdx.x == 0) {
        d.part[2 * blk] = tg;
        d.part[2 * blk + 1] = tq;
    }
}

// ---------------------------------------------------------------------------
// Kernels: one image (its descriptor by value, workgroup x = tile x) or a
// batch (descriptor table and work list).
// ---------------------------------------------------------------------------

// Each pass has two kernels.  One image: its descriptor is the kernel
// argument (constant offsets into the argument segment, loaded together) and
// workgroup x is tile x.  A batch: descriptor table and work list.
#define ACSEG_MG_KERNELS(TPL, NAME, BOUND, BODY)                                             \
    TPL __global__ __launch_bounds__(BOUND) void NAME(MgImage d, MgStep st) {                \
        const int tile = blockIdx.x;                                                         \
        BODY;                                                                                \
    }                                                                                        \
    TPL __global__ __launch_bounds__(BOUND) void NAME##_b(const MgImage* __restrict__ descs, \
                                                          const int4* __restrict__ work,     \
                                                          int nwork, MgStep sb) {            \
        if ((int)blockIdx.x >= nwork) return;                                                \
        const int4 wv = work[blockIdx.x];                                                    \
        if (wv.x < 0) return;                                                                \
        const MgImage& d = descs[wv.x];                                                      \
        const int tile = wv.y;                                                               \
        MgStep st = sb;                                                                      \
        st.level = wv.z;                                                                     \
        st.zero = wv.w;                                                                      \
        if (wv.w) st.sweeps = d.coarse_sweeps;                                               \
        BODY;                                                                                \
    }

#define ACSEG_TPL_N template <int N>
#define ACSEG_TPL_NONE
#define ACSEG_TPL_T template <int T>
ACSEG_MG_KERNELS(ACSEG_TPL_N, k_mg_defect_restrict, kBlock, mg_defect_restrict<N>(d, tile, st))
ACSEG_MG_KERNELS(ACSEG_TPL_T, k_mg_down, T, mg_down<T>(d, tile, st, blockIdx.y))
ACSEG_MG_KERNELS(ACSEG_TPL_T, k_mg_up, T, mg_up<T>(d, tile, st, blockIdx.y))
ACSEG_MG_KERNELS(ACSEG_TPL_NONE, k_mg_tail, kTailThreads, (void)tile; mg_tail(d, st, blockIdx.y))
ACSEG_MG_KERNELS(ACSEG_TPL_N, k_mg_dir, kBlock, mg_dir<N>(d, tile, st))
#undef ACSEG_TPL_N
#undef ACSEG_TPL_NONE
#undef ACSEG_TPL_T
#undef ACSEG_MG_KERNELS

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

namespace {

int grid_for(int64_t work) {
    const int64_t b = (work + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMgBlocks));
}

int tiles_of(int W, int H, int TX, int TY) { return ((W + TX - 1) / TX) * ((H + TY - 1) / TY); }

// One launch of a pass: the single-image kernel K1 or the batch kernel KB.
template <class K1, class KB>
hipError_t mg_launch(K1 k1, KB kb, dim3 grid, int threads, size_t lds, const MgImage& m, const MgGrid& g,
                     const MgStep& st, hipStream_t s) {
    if (g.descs)
        hipLaunchKernelGGL(kb, grid, dim3(threads), lds, s, g.descs, g.work, g.nwork, st);
    else
        hipLaunchKernelGGL(k1, grid, dim3(threads), lds, s, m, st);
    return hipGetLastError();
}

template <int N>
hipError_t mg_fine(int op, const MgImage& m, const MgGrid& g, const MgStep& st, dim3 grid, hipStream_t s) {
    switch (op) {
        case kMgDefectRestrict:
            return mg_launch(k_mg_defect_restrict<N>, k_mg_defect_restrict_b<N>, grid, kBlock, 0, m, g, st, s);
        case kMgDir: return mg_launch(k_mg_dir<N>, k_mg_dir_b<N>, grid, kBlock, 0, m, g, st, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int mg_pass_tiles(int op, const MgImage& m, int level) {
    switch (op) {
        case kMgDefectRestrict: return tiles_of(m.lv[1].W, m.lv[1].H, kDrTX, kDrTY);
        case kMgDown: return tiles_of(m.lv[level + 1].W, m.lv[level + 1].H, kDnTX, kDnTY);
        case kMgUp: return tiles_of(m.lv[level].W, m.lv[level].H, kUpTX, kUpTY);
        case kMgTail: return 1;
        case kMgDir: return m.dir_blocks;
        default: return 0;
    }
}

size_t mg_tail_lds(const int* W, const int* H, int t, int L) {
    if (t >= L) return 0;
    size_t f = (size_t)W[t] * H[t];  // residual scratch
    for (int l = t; l < L; ++l) f += (size_t)W[l] * H[l] * 2;
    return f * sizeof(float);
}

size_t mg_lds_down(int nu) { return (size_t)2 * down_sx(nu) * down_sy(nu) * sizeof(float); }
size_t mg_lds_up(int nu) { return ((size_t)2 * up_sx(nu) * up_sy(nu) + (size_t)up_cx(nu) * up_cy(nu)) * sizeof(float); }

size_t mg_pass_lds(int op, const MgImage& m, int sweeps) {
    switch (op) {
        case kMgDown: return (size_t)2 * down_sx(sweeps) * down_sy(sweeps) * sizeof(float);
        case kMgUp: return mg_lds_up(sweeps);
        case kMgTail: {
            int W[kMaxLevels], H[kMaxLevels];
            for (int l = 1; l < m.L; ++l) {
                W[l] = m.lv[l].W;
                H[l] = m.lv[l].H;
            }
            return mg_tail_lds(W, H, m.tail, m.L);
        }
        default: return 0;
    }
}

// Compute units of the current device, queried once per device.
static int device_cus() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

hipError_t launch_mg(int op, int N, int ncomp, const MgImage& single, const MgGrid& g, const MgStep& st,
                     size_t lds, hipStream_t s) {
    const int items = g.descs ? g.nwork : mg_pass_tiles(op, single, st.level);
    if (items <= 0) return hipSuccess;
    // A down / up pass's tile stages 1.4-2.8k nodes; more threads take fewer of
    // them at a time in every phase.  The most that lets all of the pass's
    // workgroups fit on the device at once (2048 threads per CU) is taken.
    const int64_t fit = 2048 * (int64_t)device_cus() / ((int64_t)items * ncomp);
    const int T = fit >= 1024 ? 1024 : (fit >= 512 ? 512 : kBlock);
    const dim3 cg(items, ncomp);  // componentwise passes
    switch (op) {
        case kMgDown:
            if (T == 1024) return mg_launch(k_mg_down<1024>, k_mg_down_b<1024>, cg, T, lds, single, g, st, s);
            if (T == 512) return mg_launch(k_mg_down<512>, k_mg_down_b<512>, cg, T, lds, single, g, st, s);
            return mg_launch(k_mg_down<kBlock>, k_mg_down_b<kBlock>, cg, T, lds, single, g, st, s);
        case kMgUp:
            if (T == 1024) return mg_launch(k_mg_up<1024>, k_mg_up_b<1024>, cg, T, lds, single, g, st, s);
            if (T == 512) return mg_launch(k_mg_up<512>, k_mg_up_b<512>, cg, T, lds, single, g, st, s);
            return mg_launch(k_mg_up<kBlock>, k_mg_up_b<kBlock>, cg, T, lds, single, g, st, s);
        case kMgTail: return mg_launch(k_mg_tail, k_mg_tail_b, cg, kTailThreads, lds, single, g, st, s);
        default: break;
    }
    const dim3 grid(items);
    switch (N) {
        case 2: return mg_fine<2>(op, single, g, st, grid, s);
        case 3: return mg_fine<3>(op, single, g, st, grid, s);
        case 4: return mg_fine<4>(op, single, g, st, grid, s);
        case 5: return mg_fine<5>(op, single, g, st, grid, s);
        case 6: return mg_fine<6>(op, single, g, st, grid, s);
        case 7: return mg_fine<7>(op, single, g, st, grid, s);
        case 8: return mg_fine<8>(op, single, g, st, grid, s);
        default: return hipErrorInvalidValue;
    }
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
