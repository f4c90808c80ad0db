// acseg_api.hip -- host runtime behind the C ABI declared in include/acseg.h.
//
// Validates problems, derives the float64 per-class constants of the nodal
// system, carves the caller's workspace, and enqueues the kernels of the time
// loop on the caller's stream.  Convergence is decided on the device: every
// cycle kernel reads the control block's `done` flag and exits at once after
// the step has converged, so the host never needs to read the residual.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "acseg.h"
#include "acseg_internal.h"

using namespace acseg;

namespace {
// Timing families: the multigrid ones follow the order of MgPass.
enum Family {
    kFamCmeans = 0, kFamRhs, kFamSmooth,
    kFamMgRestrict, kFamMgDown, kFamMgTail, kFamMgUp, kFamMgDir,
    kFamSsc, kFamAdjSweep, kFamOther, kFamCount
};
const char* const kFamName[kFamCount] = {"cmeans", "rhs", "smooth", "mg_restrict", "mg_down",
                                         "mg_tail", "mg_up", "mg_dir", "ssc", "adj_sweep", "other"};
static_assert(kFamMgDir - kFamMgRestrict == kMgDir - kMgDefectRestrict, "family order");
int mg_family(int op) { return kFamMgRestrict + (op - kMgDefectRestrict); }
struct TimedRec {
    int fam;
    hipEvent_t a, b;
};
}  // namespace

struct acseg_ctx {
    int device = 0;
    int cu_count = 0;
    Ctl* host_ctl = nullptr;  // pinned, for statistics read-back
    AdjCtl* host_actl = nullptr;  // pinned, for the adjoint's convergence flag
    StepSlot* host_slot = nullptr;  // pinned, for a step's convergence flag
    int cycle_hint = 2;             // cycles of the first chunk of an adaptive step
    bool timing = false;
    std::vector<hipEvent_t> pool;
    std::vector<TimedRec> recs;
    // pinned staging of a batch's descriptor tables; stage_ev marks the end of
    // the last upload from it
    void* stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_ev = nullptr;
    // the last uploaded tables and the workspace they went to (REUSE_TABLES check)
    std::vector<char> last_tables;
    const void* last_tables_ws = nullptr;
    // device address of this device's copy of the static scratch array
    // (acseg_solve_no_alloc), looked up once at creation with the device current
    void* scratch = nullptr;
    // most adjoint sweeps any step of the last backward of a problem took, by
    // problem (at most kAdjMemo entries, oldest dropped first)
    std::vector<std::pair<acseg_problem, int>> adj_memo;
};

// Scratch of acseg_solve_no_alloc: a file-scope device array, one copy per
// device the library runs on, held until the process ends.  Host code never
// uses its name as an address (on the host it is only a stand-in for the
// symbol): acseg_create looks up the device address with hipGetSymbolAddress
// and every use goes through acseg_ctx::scratch.
static __device__ __align__(256) unsigned char scratch[ACSEG_NO_ALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxBatch = 4096;
static_assert(kCmeansMaxM == ACSEG_MAX_N * ACSEG_MAX_C + ACSEG_MAX_N + ACSEG_MAX_C + 2, "sums per set");
static_assert(kNC == ACSEG_MAX_N * ACSEG_MAX_C, "means per set");

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int coarse_side(int n) { return (n + 1) / 2; }

int auto_levels(int W, int H) {
    int L = 1;
    while (std::max(W, H) > 15 && std::min(W, H) >= 3) {
        W = coarse_side(W);
        H = coarse_side(H);
        ++L;
    }
    return L;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

acseg_status validate(const acseg_problem* p, bool need_steps) {
    if (!p) return ACSEG_ERR_INVALID_ARG;
    if (p->W < 2 || p->H < 2 || p->C < 1 || p->N < 1) return ACSEG_ERR_INVALID_ARG;
    if ((int64_t)p->W * p->H > ((int64_t)1 << 30)) return ACSEG_ERR_INVALID_ARG;  // 32-bit byte offsets per plane
    if (p->N < ACSEG_MIN_N || p->N > ACSEG_MAX_N || p->C > ACSEG_MAX_C) return ACSEG_ERR_UNSUPPORTED;
    if (!finite_pos(p->h) || !finite_pos(p->eps) || !finite_pos(p->tau)) return ACSEG_ERR_INVALID_ARG;
    if (!isfinite(p->lambda) || p->lambda < 0.0) return ACSEG_ERR_INVALID_ARG;
    if (!isfinite(p->tol) || p->tol < 0.0) return ACSEG_ERR_INVALID_ARG;
    if (need_steps && p->steps < 0) return ACSEG_ERR_INVALID_ARG;
    if (p->nu_pre < 0 || p->nu_post < 0 || p->nu_pre + p->nu_post < 1) return ACSEG_ERR_INVALID_ARG;
    if (p->max_cycles < 1 || p->levels < 0) return ACSEG_ERR_INVALID_ARG;
    if (p->levels > auto_levels(p->W, p->H)) return ACSEG_ERR_INVALID_ARG;
    // a multigrid cycle opens with pre-smoothing (right-hand side, convergence
    // check) and closes with post-smoothing (residual)
    const int L = p->levels == 0 ? auto_levels(p->W, p->H) : p->levels;
    if (L >= 2 && (p->nu_pre < 1 || p->nu_post < 1)) return ACSEG_ERR_UNSUPPORTED;
    if ((p->flags & ~(ACSEG_FLAG_STORE_CHECKPOINTS | ACSEG_FLAG_FIXED_CYCLES | ACSEG_FLAG_FIXED_C |
                      ACSEG_FLAG_NO_HOST_WAIT | ACSEG_FLAG_SSC | ACSEG_FLAG_REUSE_TABLES |
                      ACSEG_FLAG_SOR)) != 0u)
        return ACSEG_ERR_INVALID_ARG;
    return ACSEG_OK;
}

// Multigrid hierarchy of a problem: level l has side ceil(side_{l-1} / 2) and
// spacing 2^l h.  Levels tail..L-1 (the first level whose sides are both <=
// kTailSide and whose tail fits in kTailLds bytes of LDS, and every coarser
// one) run in the LDS tail kernel; tail == L when none does.
struct MgPlan {
    int L = 1, tail = 1, coarse_sweeps = kCoarseSweeps;
    int W[kMaxLevels], H[kMaxLevels];
    LevelCoef coef[kMaxLevels];
};

LevelCoef level_coef(const acseg_problem* p, int l) {
    static const double w[4] = {1.0, 0.5, 1.0 / 3.0, 1.0 / 6.0};  // lumped mass / (2^l h)^2
    static const double a[4] = {4.0, 2.0, 1.0, 1.0};              // stiffness diagonal
    LevelCoef c;
    memset(&c, 0, sizeof(c));
    const double e2 = p->eps / (p->h * p->h);
    const double s = ldexp(1.0, 2 * l);  // (2^l)^2: mass in units of the finest h^2
    for (int k = 0; k < 4; ++k) {
        const double D = s * w[k] / p->tau + e2 * a[k];
        c.kappa[k] = (float)(e2 / D);
        c.inv_d[k] = (float)(1.0 / D);
        c.d[k] = (float)D;
    }
    c.e2 = (float)e2;
    return c;
}

// Red-black sweeps that solve the coarsest level to FP32 rounding, at most
// kCoarseSweeps.  The level's matrix is strictly diagonally dominant, so one
// Gauss-Seidel sweep shrinks the error's max norm at least by the Jacobi bound
// rho = max_k kappa_k a_k (a_k: the sum of the neighbour weights of node class
// k, equal to its stiffness diagonal); from v = 0, rho^s <= 2^-24 after s
// sweeps.  With a large mass term (coarse spacing, short time step) rho is
// tiny and one to three sweeps do.
int coarse_sweeps_of(const LevelCoef& c) {
    static const double a[4] = {4.0, 2.0, 1.0, 1.0};
    double rho = 0.0;
    for (int k = 0; k < 4; ++k) rho = std::max(rho, (double)c.kappa[k] * a[k]);
    if (!(rho > 0.0)) return 1;
    if (rho >= 1.0) return kCoarseSweeps;
    const double s = ceil(24.0 * log(2.0) / -log(rho));
    return (int)std::min<double>(std::max(s, 1.0), kCoarseSweeps);
}

MgPlan plan_of(const acseg_problem* p) {
    MgPlan m;
    m.L = std::min(p->levels == 0 ? auto_levels(p->W, p->H) : p->levels, kMaxLevels);
    m.W[0] = p->W;
    m.H[0] = p->H;
    for (int l = 0; l < m.L; ++l) {
        if (l > 0) {
            m.W[l] = coarse_side(m.W[l - 1]);
            m.H[l] = coarse_side(m.H[l - 1]);
        }
        m.coef[l] = level_coef(p, l);
    }
    m.coarse_sweeps = coarse_sweeps_of(m.coef[m.L - 1]);
    m.tail = m.L;
    for (int l = 1; l < m.L; ++l)
        if (m.W[l] <= kTailSide && m.H[l] <= kTailSide && mg_tail_lds(m.W, m.H, l, m.L) <= (size_t)kTailLds) {
            m.tail = l;
            break;
        }
    return m;
}

// Workspace carve-up (offsets in bytes from ws).
struct Layout {
    size_t ubuf = 0, rhs = 0, part_f = 0, part_cm = 0, part_d = 0, c64 = 0, tot = 0, ctl = 0;
    size_t mg_gt = 0, mg_part = 0;
    size_t mg_v[kMaxLevels] = {}, mg_r[kMaxLevels] = {}, mg_v2[kMaxLevels] = {};  // coarse levels 1..L-1
    size_t total = 0;
    int part_stride = 0;
};

int dir_blocks(int W, int H) {
    return std::min(((W + kDirTX - 1) / kDirTX) * ((H + kDirTY - 1) / kDirTY), kDirBlocks);
}

Layout layout_of(const acseg_problem* p) {
    Layout L;
    const size_t n = (size_t)p->W * p->H;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.ubuf = take(sizeof(float) * p->N * n);
    L.rhs = take(sizeof(float) * p->N * n);
    L.part_stride = cycle_tiles(p->N, p->W, p->H);
    L.part_f = take(sizeof(float) * 2 * (size_t)L.part_stride);
    L.part_cm = take(sizeof(double) * 2 * (size_t)L.part_stride * cmeans_width(p->N, p->C));
    L.part_d = take(sizeof(double) * (size_t)kCmeansBlocks * kCmeansMaxM);
    L.c64 = take(sizeof(double) * 3 * kNC);          // two alternating sets + a caller's c_prev
    L.tot = take(sizeof(double) * 2 * kCmeansMaxM);  // reduced colour-mean sums, alternating
    L.ctl = take(sizeof(Ctl));
    const MgPlan m = plan_of(p);
    if (m.L >= 2) {
        L.mg_gt = take(sizeof(float) * p->N * n);
        L.mg_part = take(sizeof(double) * 2 * (size_t)dir_blocks(p->W, p->H));
        for (int l = 1; l < m.L; ++l) {
            const size_t nl = (size_t)p->N * m.W[l] * m.H[l];
            L.mg_v[l] = take(sizeof(float) * nl);
            L.mg_r[l] = take(sizeof(float) * nl);
            L.mg_v2[l] = take(sizeof(float) * nl);
        }
    }
    L.total = off;
    return L;
}

// Float64 constants of the fine-level nodal system, rounded once for the kernels.
struct Coefs {
    LevelCoef fine;
    RhsCoef rhs;
};

Coefs coefs_of(const acseg_problem* p) {
    static const double w[4] = {1.0, 0.5, 1.0 / 3.0, 1.0 / 6.0};  // lumped mass / h^2
    static const double a[4] = {4.0, 2.0, 1.0, 1.0};              // stiffness diagonal
    Coefs c;
    memset(&c, 0, sizeof(c));
    const double e2 = p->eps / (p->h * p->h);
    for (int k = 0; k < 4; ++k) {
        const double D = w[k] / p->tau + e2 * a[k];
        c.fine.kappa[k] = (float)(e2 / D);
        c.fine.inv_d[k] = (float)(1.0 / D);
        c.fine.d[k] = (float)D;
        c.rhs.wd[k] = w[k] / D;
        c.rhs.wda[k] = (float)(w[k] / D * (1.0 / p->tau + 2.0 / p->eps));
    }
    c.fine.e2 = (float)e2;
    c.rhs.a = 1.0 / p->tau + 2.0 / p->eps;
    c.rhs.lambda = p->lambda;
    return c;
}

acseg_status hip_status(hipError_t e) { return e == hipSuccess ? ACSEG_OK : ACSEG_ERR_HIP; }

#define ACSEG_TRY(expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return ACSEG_ERR_HIP;       \
    } while (0)

acseg_status check_ws(const acseg_problem* p, void* ws, size_t ws_bytes, Layout* L) {
    *L = layout_of(p);
    if (!ws || ((uintptr_t)ws % kAlign) != 0 || ws_bytes < L->total) return ACSEG_ERR_WORKSPACE;
    return ACSEG_OK;
}

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

hipEvent_t take_event(acseg_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Run one launcher, bracketed by timing events when timing is enabled.
template <class F>
hipError_t timed(acseg_ctx* ctx, int fam, hipStream_t s, F&& launch) {
    if (!ctx->timing) return launch();
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    ctx->recs.push_back({fam, a, b});
    return e;
}

// One image's multigrid descriptor (constant over a solve).
MgImage mg_image_of(const acseg_problem* p, const MgPlan& m, const Layout& L, void* ws, Bufs bufs) {
    MgImage d;
    memset(&d, 0, sizeof(d));
    d.bufs = bufs;
    d.ctl = at<Ctl>(ws, L.ctl);
    d.rhs = at<float>(ws, L.rhs);
    d.gt = at<float>(ws, L.mg_gt);
    d.part = at<double>(ws, L.mg_part);
    d.N = p->N;
    d.W = p->W;
    d.H = p->H;
    d.L = m.L;
    d.tail = m.tail;
    d.dir_blocks = dir_blocks(p->W, p->H);
    d.coarse_sweeps = m.coarse_sweeps;
    CycleArgs tiling{};
    cycle_tiling(p->N, p->W, p->H, &tiling);
    d.res_part = at<float>(ws, L.part_f);
    d.part_stride = L.part_stride;
    d.ntiles = tiling.ntiles;
    d.tol = (float)p->tol;
    d.fine = m.coef[0];
    for (int l = 1; l < m.L; ++l) {
        MgLevel& v = d.lv[l];
        v.r = at<float>(ws, L.mg_r[l]);
        v.v = at<float>(ws, L.mg_v[l]);
        v.v2 = at<float>(ws, L.mg_v2[l]);
        v.coef = m.coef[l];
        v.W = m.W[l];
        v.H = m.H[l];
    }
    return d;
}

// The passes of one truncated multigrid correction, in order: (pass, level,
// sweeps, zero).  Levels 1..tail-1 go down (sweeps from zero, restriction)
// and up (prolongation, sweeps) in tiled passes, the LDS tail solves levels
// tail..L-1; without a tail the coarsest level is an up pass from zero.  The
// direction pass closes it; the next smoothing launch applies the update.
struct MgPassRec {
    int op, level, sweeps, zero;
};

std::vector<MgPassRec> mg_passes(const MgPlan& m, int nu_pre, int nu_post) {
    std::vector<MgPassRec> v;
    v.push_back({kMgDefectRestrict, 0, 0, 0});
    const int down_end = m.tail < m.L ? m.tail : m.L - 1;  // levels 1 .. down_end-1 go down
    for (int l = 1; l < down_end; ++l) v.push_back({kMgDown, l, nu_pre, 0});
    if (m.tail < m.L)
        v.push_back({kMgTail, m.tail, 0, 0});
    else
        v.push_back({kMgUp, m.L - 1, m.coarse_sweeps, 1});
    for (int l = down_end - 1; l >= 1; --l) v.push_back({kMgUp, l, nu_post, 0});
    v.push_back({kMgDir, 0, 0, 0});
    return v;
}

// The truncated multigrid correction of the iterate left by `launch`
// smoothing launches of the current step (in place).
acseg_status enqueue_correction(acseg_ctx* ctx, const acseg_problem* p, const MgPlan& m,
                                const Layout& L, void* ws, Bufs bufs, int slot, bool fixed,
                                int launch, int check, hipStream_t s) {
    const MgImage d = mg_image_of(p, m, L, ws, bufs);
    const MgGrid single{nullptr, nullptr, 0};
    MgStep st{};
    st.slot = slot;
    st.fixed = fixed ? 1 : 0;
    st.launch = launch;
    st.check = check;
    st.nu_pre = p->nu_pre;
    st.nu_post = p->nu_post;
    for (const MgPassRec& r : mg_passes(m, p->nu_pre, p->nu_post)) {
        st.level = r.level;
        st.sweeps = r.sweeps;
        st.zero = r.zero;
        const size_t lds = mg_pass_lds(r.op, d, r.sweeps);
        ACSEG_TRY(timed(ctx, mg_family(r.op), s, [&] { return launch_mg(r.op, p->N, p->N, d, single, st, lds, s); }));
    }
    return ACSEG_OK;
}

// The subspace correction over the basis functions of the coarse levels,
// coarsest first, four parity classes per level (in place on the iterate left
// by `launch` smoothing launches of the current step).
constexpr int kSscChunkLevel = 5;     // levels from which a support spans several workgroups
constexpr int kSscChunkNodes = 2048;  // box nodes per chunk
acseg_status enqueue_ssc(acseg_ctx* ctx, const acseg_problem* p, const MgPlan& m, const Layout& L,
                         void* ws, Bufs bufs, int slot, bool fixed, int launch, hipStream_t s) {
    SscArgs a{};
    a.bufs = bufs;
    a.ctl = at<Ctl>(ws, L.ctl);
    a.rhs = at<float>(ws, L.rhs);
    a.coef = m.coef[0];
    a.W = m.W[0];
    a.H = m.H[0];
    a.slot = slot;
    a.fixed = fixed ? 1 : 0;
    a.launch = launch;
    // chunked two-launch form where supports are large; the partials go to the
    // truncated correction's defect buffer, unused by this correction
    double* part = at<double>(ws, L.mg_gt);
    const size_t part_cap = sizeof(float) * (size_t)p->N * m.W[0] * m.H[0] / ((2 * p->N + 1) * sizeof(double));
    for (int l = m.L - 1; l >= 1; --l) {
        a.Wc = m.W[l];
        a.Hc = m.H[l];
        a.sh = l;
        const int side = (2 << l) - 1;  // box side of an interior function
        a.rows = std::max(1, kSscChunkNodes / side);
        a.chunks = (side + a.rows - 1) / a.rows;
        const size_t items = (size_t)((a.Wc + 1) / 2) * ((a.Hc + 1) / 2) * a.chunks;
        a.part = (l >= kSscChunkLevel && items <= part_cap) ? part : nullptr;
        for (int c = 0; c < 4; ++c) {
            a.colour = c;
            ACSEG_TRY(timed(ctx, kFamSsc, s, [&] { return launch_ssc(p->N, a, s); }));
        }
    }
    return ACSEG_OK;
}

// Enqueue time step n on the iterate bufs[ctl->cur] whose reduced colour-mean
// sums are in `tot`: max_cycles smoothing cycles (after convergence they exit
// at once unless the schedule is fixed), then the step's end, which leaves the
// sums of the new iterate in tot_next.  The step's first launch writes the
// means it uses to c64 (and c_out when non-NULL).
// Per-image constants of the cycle kernels.
CycleArgs cycle_args_of(const acseg_problem* p, const Coefs& cf, const float* image, Bufs bufs,
                        const Layout& L, void* ws) {
    CycleArgs a{};
    a.bufs = bufs;
    a.ctl = at<Ctl>(ws, L.ctl);
    a.image = image;
    a.tot = at<double>(ws, L.tot);
    a.c64 = at<double>(ws, L.c64);
    a.c_out = nullptr;
    a.rhs = at<float>(ws, L.rhs);
    a.res_part = at<float>(ws, L.part_f);
    a.cm_part = at<double>(ws, L.part_cm);
    a.part_stride = L.part_stride;
    a.coef = cf.fine;
    a.rc = cf.rhs;
    a.tol = (float)p->tol;
    a.omega = 1.f;
    if (plan_of(p).L >= 2 && (p->flags & ACSEG_FLAG_SSC) == 0u) {
        a.mg_w = at<float>(ws, L.mg_gt);
        a.mg_part = at<double>(ws, L.mg_part);
        a.mg_parts = dir_blocks(p->W, p->H);
    }
    if ((p->flags & ACSEG_FLAG_SOR) != 0u) {
        // Young's factor for the bound rho <= q = max over node classes of
        // kappa * (sum of edge weights = stiffness diagonal) of the block-Jacobi radius
        static const double diag[4] = {4.0, 2.0, 1.0, 1.0};
        double q = 0.0;
        for (int k = 0; k < 4; ++k) q = std::max(q, (double)cf.fine.kappa[k] * diag[k]);
        q = std::min(q, 0.999);
        a.omega = (float)std::min(1.95, 2.0 / (1.0 + std::sqrt(1.0 - q * q)));
    }
    cycle_tiling(p->N, p->W, p->H, &a);
    return a;
}

// Launches per cycle and whether the first launch must store the rhs.  A
// truncated V(1,1) cycle (merged) closes with one launch of two sweeps: its
// post-smoothing sweep and the next cycle's pre-smoothing sweep, the residual
// measured after both; the defect pass of the next cycle makes the
// convergence test.  A step takes one launch per cycle plus its first
// pre-smoothing, with a fixed cycle count or not, and its last cycle keeps
// the pre-smoothing sweep of the cycle it does not run.
struct Schedule {
    int lpc, lpre;
    bool merged;
    bool fixed, store_rhs, mg;
};

Schedule schedule_of(const acseg_problem* p) {
    Schedule sc;
    const MgPlan m = plan_of(p);
    const int sweeps = p->nu_pre + p->nu_post;
    sc.fixed = (p->flags & ACSEG_FLAG_FIXED_CYCLES) != 0u;
    sc.mg = m.L >= 2;
    sc.lpre = cycle_launches(p->nu_pre);
    sc.lpc = sc.mg ? sc.lpre + cycle_launches(p->nu_post) : cycle_launches(sweeps);
    sc.merged = sc.mg && (p->flags & ACSEG_FLAG_SSC) == 0u && p->nu_pre == 1 && p->nu_post == 1;
    // a one-launch step keeps the rhs in registers; the defect reads it
    sc.store_rhs = sc.mg || !(sc.fixed && p->max_cycles == 1 && sc.lpc == 1);
    return sc;
}

// Enqueue time step n on the iterate bufs[ctl->cur] whose reduced colour-mean
// sums are in tot set tot_sel: max_cycles cycles (after convergence they exit
// at once unless the schedule is fixed), then the step's end, which leaves the
// sums of the new iterate in tot set tot_sel ^ 1.  The step's first launch
// writes the means it uses to c64 set c64_sel (empty phases keep set
// prev_sel, -1 for none).
acseg_status enqueue_step(acseg_ctx* ctx, const acseg_problem* p, const Coefs& cf,
                          const float* image, Bufs bufs, const Layout& L, void* ws, int n,
                          int tot_sel, int c64_sel, int prev_sel, hipStream_t s) {
    const CycleArgs a = cycle_args_of(p, cf, image, bufs, L, ws);
    const Schedule sc = schedule_of(p);
    const CycleGrid single{nullptr, nullptr, 0, 0};
    CycleStep st{};
    st.slot = n & 1;
    st.fixed = sc.fixed ? 1 : 0;
    st.store_rhs = sc.store_rhs ? 1 : 0;
    st.tot_sel = tot_sel;
    st.c64_sel = c64_sel;
    st.fixed_c = (p->flags & ACSEG_FLAG_FIXED_C) != 0u ? 1 : 0;
    st.prev_sel = st.fixed_c ? 2 : prev_sel;  // fixed means sit in c64 set 2
    const MgPlan m = plan_of(p);
    auto cycle = [&](int k) -> acseg_status {
        st.cycle = k;
        st.cm = (!sc.fixed || k == p->max_cycles - 1) ? 1 : 0;
        st.launch = k * sc.lpc;
        if (!sc.mg) {
            const CycleRole role{k == 0, true, true};
            ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] {
                return launch_cycle(p->N, p->C, p->nu_pre + p->nu_post, a, st, single, role, s);
            }));
            return ACSEG_OK;
        }
        if (sc.merged) {
            if (k == 0) {
                const CycleRole pre{true, true, false};
                st.launch = 0;
                ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] { return launch_cycle(p->N, p->C, 1, a, st, single, pre, s); }));
            }
            const acseg_status v = enqueue_correction(ctx, p, m, L, ws, bufs, st.slot, sc.fixed, k + 1, k, s);
            if (v != ACSEG_OK) return v;
            st.launch = k + 1;
            const CycleRole post{false, false, true, true};
            ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] { return launch_cycle(p->N, p->C, 2, a, st, single, post, s); }));
            return ACSEG_OK;
        }
        const CycleRole pre{k == 0, true, false};
        ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] { return launch_cycle(p->N, p->C, p->nu_pre, a, st, single, pre, s); }));
        const acseg_status v =
            (p->flags & ACSEG_FLAG_SSC) != 0u
                ? enqueue_ssc(ctx, p, m, L, ws, bufs, st.slot, sc.fixed, k * sc.lpc + sc.lpre, s)
                : enqueue_correction(ctx, p, m, L, ws, bufs, st.slot, sc.fixed, k * sc.lpc + sc.lpre, 0, s);
        if (v != ACSEG_OK) return v;
        st.launch = k * sc.lpc + sc.lpre;
        const CycleRole post{false, false, true, (p->flags & ACSEG_FLAG_SSC) == 0u};
        ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] { return launch_cycle(p->N, p->C, p->nu_post, a, st, single, post, s); }));
        return ACSEG_OK;
    };
    const bool chunked = !sc.fixed && (p->flags & ACSEG_FLAG_NO_HOST_WAIT) == 0u;
    ctx->host_slot->done = 0;
    if (!chunked) {
        for (int k = 0; k < p->max_cycles; ++k) {
            const acseg_status v = cycle(k);
            if (v != ACSEG_OK) return v;
        }
    } else {
        // chunks of cycles; after each, a convergence test whose flag the host reads
        int k = 0, chunk = std::max(1, std::min(ctx->cycle_hint, p->max_cycles));
        while (k < p->max_cycles) {
            const int end = std::min(p->max_cycles, k + chunk);
            for (; k < end; ++k) {
                const acseg_status v = cycle(k);
                if (v != ACSEG_OK) return v;
            }
            if (k >= p->max_cycles) break;
            ACSEG_TRY(launch_step_check(a, st.slot, k, s));
            ACSEG_TRY(hipMemcpyAsync(ctx->host_slot, &a.ctl->step[st.slot], sizeof(StepSlot),
                                     hipMemcpyDeviceToHost, s));
            ACSEG_TRY(hipStreamSynchronize(s));
            if (ctx->host_slot->done) break;
            chunk = std::min(2 * chunk, 64);
        }
        // the next step starts with as many cycles as this one needed
        ctx->cycle_hint = std::max(1, ctx->host_slot->done ? ctx->host_slot->cycles : k);
    }
    const StepEndArgs e = sc.merged ? StepEndArgs{p->max_cycles, 1, 1} : StepEndArgs{p->max_cycles, sc.lpc, 0};
    ACSEG_TRY(timed(ctx, kFamOther, s, [&] {
        return launch_step_end(p->N, p->C, a, st, e, nullptr, nullptr, 0, s);
    }));
    return ACSEG_OK;
}

// Colour means of an explicit field u: reduced sums into tot (may be NULL),
// means into c64 / c_out.
acseg_status enqueue_means(const acseg_problem* p, const float* image, const float* u,
                           const Layout& L, void* ws, const double* c_prev64, double* c64,
                           float* c_out, double* tot, hipStream_t s) {
    const Bufs bufs{{u, u, u}};
    Ctl* ctl = at<Ctl>(ws, L.ctl);
    double* part_d = at<double>(ws, L.part_d);
    ACSEG_TRY(launch_cmeans(p->N, p->C, p->W, p->H, image, u, bufs, ctl, part_d, s));
    ACSEG_TRY(launch_cmeans_finish(p->N, p->C, p->W, p->H, part_d, ctl, c_prev64, c64, c_out, tot, s));
    return ACSEG_OK;
}

acseg_status read_stats(acseg_ctx* ctx, const Layout& L, void* ws, hipStream_t s,
                        acseg_stats* st) {
    if (!st) return ACSEG_OK;
    ACSEG_TRY(hipMemcpyAsync(ctx->host_ctl, at<Ctl>(ws, L.ctl), sizeof(Ctl), hipMemcpyDeviceToHost, s));
    ACSEG_TRY(hipStreamSynchronize(s));
    const Ctl& c = *ctx->host_ctl;
    memset(st, 0, sizeof(*st));
    st->steps_done = c.steps_done;
    st->cycles_total = c.cycles_total;
    st->cycles_max = c.cycles_max;
    st->steps_not_converged = c.steps_unconv;
    st->empty_phase_steps = c.empty_steps;
    st->final_residual = c.resid;
    st->max_residual = c.max_resid;
    if (c.nonfinite)
        st->status = ACSEG_ERR_NONFINITE;
    else if (c.steps_unconv)
        st->status = ACSEG_WARN_NOT_CONVERGED;
    else if (c.empty_steps || c.empty_now)
        st->status = ACSEG_WARN_EMPTY_PHASE;
    return ACSEG_OK;
}

// ---- batches ---------------------------------------------------------------

// A batch shares the time loop: every problem must agree on these.
bool same_schedule(const acseg_problem& a, const acseg_problem& b) {
    return a.steps == b.steps && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post &&
           a.max_cycles == b.max_cycles && a.flags == b.flags;
}

acseg_status validate_batch(int32_t B, const acseg_problem* ps) {
    if (B < 1 || B > kMaxBatch || !ps) return ACSEG_ERR_INVALID_ARG;
    for (int b = 0; b < B; ++b) {
        const acseg_status v = validate(&ps[b], true);
        if (v != ACSEG_OK) return v;
        if (!same_schedule(ps[0], ps[b])) return ACSEG_ERR_INVALID_ARG;
        if ((ps[b].flags & ACSEG_FLAG_STORE_CHECKPOINTS) != 0u) return ACSEG_ERR_INVALID_ARG;
        // the subspace correction runs per image only
        if ((ps[b].flags & ACSEG_FLAG_SSC) != 0u && plan_of(&ps[b]).L >= 2) return ACSEG_ERR_UNSUPPORTED;
    }
    return ACSEG_OK;
}

int tiles_of(int W, int H, int TX, int TY) { return ((W + TX - 1) / TX) * ((H + TY - 1) / TY); }

// One multigrid launch of a batch group: pass, its work items, sweeps, LDS.
struct MgLaunchRec {
    int op, work0, nwork, sweeps;
    size_t lds;
};

// Images of one batch with the same N, C and cycle kind (Gauss-Seidel cycles
// or multigrid cycles): their cycles share launches.
struct BatchGroup {
    int N = 0, C = 0;
    bool mg = false;
    std::vector<int> members;
    int work0 = 0, nwork = 0;  // smoothing tiles (int2 work list)
    int img0 = 0;              // step-end image list
    std::vector<MgLaunchRec> mgl;  // the passes of one multigrid correction, in order
};

// Everything about a batch that does not depend on the workspace address:
// groups, work lists, and the workspace carve-up.
struct BatchPlan {
    std::vector<BatchGroup> groups;
    std::vector<int2> work;    // smoothing tiles, every group
    std::vector<int> imgs;     // step-end image lists, every group
    std::vector<int4> mgwork;  // multigrid work items, every group
    std::vector<MgPlan> mp;
    size_t descs = 0, mgdescs = 0, work_off = 0, imgs_off = 0, mgwork_off = 0;
    size_t table_bytes = 0;    // descs .. mgwork, uploaded in one copy
    std::vector<size_t> region;
    std::vector<Layout> L;
    size_t total = 0;
};

// The multigrid passes of a group: defect + restriction, down passes level by
// level, LDS tails, up passes level by level (with the coarsest-level solve of
// images without a tail), direction (the post-smoothing launch applies the
// update).  An image takes part in the passes its hierarchy has.
void plan_group_mg(const acseg_problem* ps, BatchPlan& bp, BatchGroup& g) {
    const int nu_pre = ps[g.members[0]].nu_pre, nu_post = ps[g.members[0]].nu_post;
    auto add = [&](int op, int sweeps, size_t lds, const std::vector<int4>& items) {
        if (items.empty()) return;
        g.mgl.push_back({op, (int)bp.mgwork.size(), (int)items.size(), sweeps, lds});
        bp.mgwork.insert(bp.mgwork.end(), items.begin(), items.end());
    };
    auto down_end = [&](int b) { const MgPlan& m = bp.mp[b]; return m.tail < m.L ? m.tail : m.L - 1; };
    std::vector<int4> it;
    for (int b : g.members) {
        const MgPlan& m = bp.mp[b];
        for (int t = 0; t < tiles_of(m.W[1], m.H[1], kDrTX, kDrTY); ++t) it.push_back(make_int4(b, t, 1, 0));
    }
    add(kMgDefectRestrict, 0, 0, it);
    int maxL = 0;
    for (int b : g.members) maxL = std::max(maxL, bp.mp[b].L);
    for (int l = 1; l < maxL; ++l) {
        it.clear();
        for (int b : g.members) {
            const MgPlan& m = bp.mp[b];
            if (l >= down_end(b)) continue;
            for (int t = 0; t < tiles_of(m.W[l + 1], m.H[l + 1], kDnTX, kDnTY); ++t) it.push_back(make_int4(b, t, l, 0));
        }
        add(kMgDown, nu_pre, mg_lds_down(nu_pre), it);
    }
    it.clear();
    size_t tail_lds = 0;
    for (int b : g.members) {
        const MgPlan& m = bp.mp[b];
        if (m.tail >= m.L) continue;
        it.push_back(make_int4(b, 0, m.tail, 0));
        tail_lds = std::max(tail_lds, mg_tail_lds(m.W, m.H, m.tail, m.L));
    }
    add(kMgTail, 0, tail_lds, it);
    for (int l = maxL - 1; l >= 1; --l) {
        it.clear();
        bool zero_any = false;
        for (int b : g.members) {
            const MgPlan& m = bp.mp[b];
            const bool zero = m.tail >= m.L && l == m.L - 1;  // the coarsest level without a tail
            if (!zero && l >= down_end(b)) continue;
            zero_any = zero_any || zero;
            for (int t = 0; t < tiles_of(m.W[l], m.H[l], kUpTX, kUpTY); ++t)
                it.push_back(make_int4(b, t, l, zero ? 1 : 0));
        }
        add(kMgUp, nu_post, std::max(mg_lds_up(nu_post), zero_any ? mg_lds_up(kCoarseSweeps) : 0), it);
    }
    it.clear();
    for (int b : g.members)
        for (int k = 0; k < dir_blocks(ps[b].W, ps[b].H); ++k) it.push_back(make_int4(b, k, 0, 0));
    add(kMgDir, 0, 0, it);
}

BatchPlan plan_batch(int32_t B, const acseg_problem* ps) {
    BatchPlan bp;
    for (int b = 0; b < B; ++b) bp.mp.push_back(plan_of(&ps[b]));
    // groups by (N, C, cycle kind), in order of first appearance
    for (int b = 0; b < B; ++b) {
        const bool mg = bp.mp[b].L >= 2;
        BatchGroup* g = nullptr;
        for (auto& x : bp.groups)
            if (x.N == ps[b].N && x.C == ps[b].C && x.mg == mg) g = &x;
        if (!g) {
            bp.groups.push_back(BatchGroup{});
            g = &bp.groups.back();
            g->N = ps[b].N;
            g->C = ps[b].C;
            g->mg = mg;
        }
        g->members.push_back(b);
    }
    for (BatchGroup& g : bp.groups) {
        // concatenated smoothing tiles of the group, dealt to the XCDs in contiguous bands
        std::vector<int2> tiles;
        for (int b : g.members)
            for (int t = 0; t < cycle_tiles(ps[b].N, ps[b].W, ps[b].H); ++t) tiles.push_back(make_int2(b, t));
        g.nwork = (int)((tiles.size() + kXcd - 1) / kXcd * kXcd);
        g.work0 = (int)bp.work.size();
        const int tpx = g.nwork / kXcd;
        for (int k = 0; k < g.nwork; ++k) {
            const int gt = (k % kXcd) * tpx + k / kXcd;
            bp.work.push_back(gt < (int)tiles.size() ? tiles[gt] : make_int2(-1, 0));
        }
        g.img0 = (int)bp.imgs.size();
        bp.imgs.insert(bp.imgs.end(), g.members.begin(), g.members.end());
        if (g.mg) plan_group_mg(ps, bp, g);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    bp.descs = take(sizeof(CycleArgs) * B);
    bp.mgdescs = take(sizeof(MgImage) * B);
    bp.work_off = take(sizeof(int2) * bp.work.size());
    bp.imgs_off = take(sizeof(int) * bp.imgs.size());
    bp.mgwork_off = take(sizeof(int4) * bp.mgwork.size());
    bp.table_bytes = off;
    for (int b = 0; b < B; ++b) {
        bp.L.push_back(layout_of(&ps[b]));
        bp.region.push_back(take(bp.L.back().total));
    }
    bp.total = off;
    return bp;
}

// ---- backward ---------------------------------------------------------------

constexpr size_t kAdjMemo = 8;

struct BackLayout {
    size_t ctl = 0, actl = 0, c64 = 0, tot = 0, part_cm = 0, part_adj = 0, part_f = 0, cbar = 0;
    size_t z = 0, z2 = 0, ub0 = 0, ub1 = 0, total = 0;
};

BackLayout back_layout_of(const acseg_problem* p) {
    BackLayout L;
    const size_t n = (size_t)p->W * p->H, S = (size_t)std::max(p->steps, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.ctl = take(sizeof(Ctl));
    L.actl = take(sizeof(AdjCtl));
    L.c64 = take(sizeof(double) * S * kNC);
    L.tot = take(sizeof(double) * S * kCmeansMaxM);
    L.part_cm = take(sizeof(double) * std::min<size_t>(S, kCmeansFields) * cmeans_blocks(p->W, p->H) *
                     kCmeansMaxM);
    L.part_adj = take(sizeof(double) * (size_t)kAdjAccBlocks * (3 + kNC));
    L.part_f = take(sizeof(float) * 12 * kMgBlocks);
    L.cbar = take(sizeof(double) * kNC);
    L.z = take(sizeof(float) * p->N * n);
    L.z2 = take(sizeof(float) * p->N * n);
    L.ub0 = take(sizeof(float) * p->N * n);
    L.ub1 = take(sizeof(float) * p->N * n);
    L.total = off;
    return L;
}

// acseg_solve on a given workspace (arguments validated by the caller).
acseg_status solve_impl(acseg_ctx* ctx, const acseg_problem* p, const float* image, float* u,
                        float* c_out, float* checkpoints, acseg_stats* stats, void* ws, size_t ws_bytes,
                        void* stream);

}  // namespace

extern "C" {

int32_t acseg_version(void) { return 100; }

const char* acseg_status_string(acseg_status s) {
    switch (s) {
        case ACSEG_OK: return "ok";
        case ACSEG_ERR_INVALID_ARG: return "invalid argument";
        case ACSEG_ERR_NONFINITE: return "image holds non-finite values";
        case ACSEG_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case ACSEG_ERR_HIP: return "HIP runtime error";
        case ACSEG_ERR_UNSUPPORTED: return "unsupported size or option";
        case ACSEG_ERR_TOO_LARGE: return "problem needs more than the library's static scratch";
        case ACSEG_WARN_NOT_CONVERGED: return "a step did not reach the tolerance";
        case ACSEG_WARN_EMPTY_PHASE: return "a phase had no mass";
        default: return "unknown status";
    }
}

acseg_status acseg_create(int device, acseg_ctx** out) {
    if (!out) return ACSEG_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return ACSEG_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return ACSEG_ERR_HIP;
    acseg_ctx* c = new acseg_ctx();
    c->device = device;
    if (hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipGetSymbolAddress(&c->scratch, HIP_SYMBOL(scratch)) != hipSuccess || !c->scratch ||
        hipHostMalloc((void**)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->host_actl, sizeof(AdjCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->host_slot, sizeof(StepSlot), hipHostMallocDefault) != hipSuccess) {
        if (c->host_ctl) (void)hipHostFree(c->host_ctl);
        if (c->host_actl) (void)hipHostFree(c->host_actl);
        delete c;
        return ACSEG_ERR_HIP;
    }
    *out = c;
    return ACSEG_OK;
}

acseg_status acseg_destroy(acseg_ctx* ctx) {
    if (!ctx) return ACSEG_OK;
    for (const TimedRec& r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->host_ctl) (void)hipHostFree(ctx->host_ctl);
    if (ctx->host_actl) (void)hipHostFree(ctx->host_actl);
    if (ctx->host_slot) (void)hipHostFree(ctx->host_slot);
    if (ctx->stage_ev) {
        (void)hipEventSynchronize(ctx->stage_ev);
        (void)hipEventDestroy(ctx->stage_ev);
    }
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    delete ctx;
    return ACSEG_OK;
}

acseg_status acseg_workspace_size(const acseg_problem* p, size_t* bytes) {
    if (!bytes) return ACSEG_ERR_INVALID_ARG;
    const acseg_status v = validate(p, false);
    if (v != ACSEG_OK) return v;
    *bytes = layout_of(p).total;
    return ACSEG_OK;
}

acseg_status acseg_project_simplex(acseg_ctx* ctx, int32_t N, int64_t count, const float* y,
                                   float* x, void* stream) {
    if (!ctx || count < 0 || (count > 0 && (!y || !x))) return ACSEG_ERR_INVALID_ARG;
    if (N < ACSEG_MIN_N || N > ACSEG_MAX_N) return ACSEG_ERR_UNSUPPORTED;
    return hip_status(launch_project(N, count, y, x, (hipStream_t)stream));
}

acseg_status acseg_transfer(acseg_ctx* ctx, int32_t direction, int32_t planes, int32_t Wf,
                            int32_t Hf, const float* src, float* dst, void* stream) {
    if (!ctx || (direction != 0 && direction != 1) || planes < 1 || Wf < 2 || Hf < 2 || !src ||
        !dst || (int64_t)Wf * Hf > ((int64_t)1 << 31))
        return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_transfer(planes, direction, src, dst, Wf, Hf, (hipStream_t)stream));
}

// Sizes of the refined lattice of acseg_refine / acseg_sample, or false when
// out of range.
static bool refined_sides(int32_t W, int32_t H, int32_t r, int64_t* Wf, int64_t* Hf) {
    if (W < 2 || H < 2 || r < 0 || r > 8) return false;
    *Wf = ((int64_t)(W - 1) << r) + 1;
    *Hf = ((int64_t)(H - 1) << r) + 1;
    return *Wf * *Hf <= ((int64_t)1 << 30);
}

acseg_status acseg_refine(acseg_ctx* ctx, int32_t planes, int32_t W, int32_t H, int32_t r, const float* src,
                          float* dst, void* stream) {
    int64_t Wf, Hf;
    if (!ctx || planes < 1 || !src || !dst || !refined_sides(W, H, r, &Wf, &Hf)) return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_refine(planes, W, H, r, src, dst, (hipStream_t)stream));
}

acseg_status acseg_sample(acseg_ctx* ctx, int32_t planes, int32_t W, int32_t H, int32_t r, const float* src,
                          float* dst, void* stream) {
    int64_t Wf, Hf;
    if (!ctx || planes < 1 || !src || !dst || !refined_sides(W, H, r, &Wf, &Hf)) return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_sample(planes, W, H, r, src, dst, (hipStream_t)stream));
}

acseg_status acseg_mass_average(acseg_ctx* ctx, int32_t planes, int32_t W, int32_t H, const float* src,
                                float* dst, void* stream) {
    if (!ctx || planes < 1 || W < 2 || H < 2 || !src || !dst || (int64_t)W * H > ((int64_t)1 << 30))
        return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_mass_avg(planes, W, H, src, dst, 0, (hipStream_t)stream));
}

acseg_status acseg_simplex_average(acseg_ctx* ctx, int32_t planes, int32_t W, int32_t H, const float* src,
                                   float* dst, void* stream) {
    if (!ctx || planes < 1 || W < 2 || H < 2 || !src || !dst || (int64_t)W * H > ((int64_t)1 << 30))
        return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_mass_avg(planes, W, H, src, dst, 1, (hipStream_t)stream));
}

acseg_status acseg_colour_space(acseg_ctx* ctx, int32_t kind, int64_t count, const float* rgb, float* dst,
                                void* stream) {
    if (!ctx || (kind != ACSEG_LAB && kind != ACSEG_AB) || count < 0 || (count > 0 && (!rgb || !dst)))
        return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_lab(kind == ACSEG_AB, count, rgb, dst, (hipStream_t)stream));
}

acseg_status acseg_colour_means(acseg_ctx* ctx, const acseg_problem* p, const float* image,
                                const float* u, const float* c_prev, float* c_out,
                                acseg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    acseg_status v = validate(p, false);
    if (v != ACSEG_OK) return v;
    if (!ctx || !image || !u || !c_out) return ACSEG_ERR_INVALID_ARG;
    Layout L;
    if ((v = check_ws(p, ws, ws_bytes, &L)) != ACSEG_OK) return v;
    hipStream_t s = (hipStream_t)stream;
    Ctl* ctl = at<Ctl>(ws, L.ctl);
    double* c64 = at<double>(ws, L.c64);
    double* cprev = c64 + 2 * kNC;
    ACSEG_TRY(launch_ctl_init(ctl, 0, s));
    if (c_prev) ACSEG_TRY(launch_widen(c_prev, cprev, p->N * p->C, s));
    v = enqueue_means(p, image, u, L, ws, c_prev ? cprev : nullptr, c64, c_out, nullptr, s);
    if (v != ACSEG_OK) return v;
    return read_stats(ctx, L, ws, s, stats);
}

acseg_status acseg_step(acseg_ctx* ctx, const acseg_problem* p, const float* image,
                        const float* u_in, float* u_out, const float* c_prev, float* c_out,
                        acseg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    acseg_status v = validate(p, false);
    if (v != ACSEG_OK) return v;
    const bool fixed_c = (p->flags & ACSEG_FLAG_FIXED_C) != 0u;
    if (!ctx || !image || !u_in || !u_out || u_in == u_out || (fixed_c && !c_prev))
        return ACSEG_ERR_INVALID_ARG;
    Layout L;
    if ((v = check_ws(p, ws, ws_bytes, &L)) != ACSEG_OK) return v;
    hipStream_t s = (hipStream_t)stream;
    const Coefs cf = coefs_of(p);
    const int64_t nu = (int64_t)p->N * p->W * p->H;
    Ctl* ctl = at<Ctl>(ws, L.ctl);
    double* c64 = at<double>(ws, L.c64);
    double* cprev = c64 + 2 * kNC;
    const Bufs bufs{{u_out, at<float>(ws, L.ubuf), u_in}};
    double* tot = at<double>(ws, L.tot);
    ACSEG_TRY(launch_ctl_init(ctl, 2, s));
    if (c_prev) ACSEG_TRY(launch_widen(c_prev, cprev, p->N * p->C, s));
    const double* cp = c_prev ? cprev : nullptr;
    v = enqueue_means(p, image, u_in, L, ws, cp, c64, fixed_c ? nullptr : c_out, tot, s);
    if (v != ACSEG_OK) return v;
    v = enqueue_step(ctx, p, cf, image, bufs, L, ws, 0, 0, 0, c_prev ? 2 : -1, s);
    if (v != ACSEG_OK) return v;
    if (fixed_c && c_out)
        ACSEG_TRY(hipMemcpyAsync(c_out, c_prev, sizeof(float) * p->N * p->C, hipMemcpyDeviceToDevice, s));
    ACSEG_TRY(launch_copy_current(bufs, ctl, u_out, nu, s));
    return read_stats(ctx, L, ws, s, stats);
}

acseg_status acseg_solve(acseg_ctx* ctx, const acseg_problem* p, const float* image, float* u,
                         float* c_out, float* checkpoints, acseg_stats* stats, void* ws,
                         size_t ws_bytes, void* stream) {
    acseg_status v = validate(p, true);
    if (v != ACSEG_OK) return v;
    return solve_impl(ctx, p, image, u, c_out, checkpoints, stats, ws, ws_bytes, stream);
}

acseg_status acseg_solve_no_alloc(acseg_ctx* ctx, const acseg_problem* p, const float* image, float* u,
                                  float* c_out, float* checkpoints, acseg_stats* stats, void* stream) {
    const acseg_status v = validate(p, true);
    if (v != ACSEG_OK) return v;
    if (!ctx || !ctx->scratch) return ACSEG_ERR_INVALID_ARG;
    if (layout_of(p).total > ACSEG_NO_ALLOC_SCRATCH_BYTES) return ACSEG_ERR_TOO_LARGE;
    // kernel timing would create HIP events: off for this call
    const bool timing = ctx->timing;
    ctx->timing = false;
    const acseg_status r = solve_impl(ctx, p, image, u, c_out, checkpoints, stats, ctx->scratch,
                                      ACSEG_NO_ALLOC_SCRATCH_BYTES, stream);
    ctx->timing = timing;
    return r;
}

}  // extern "C"

namespace {

acseg_status solve_impl(acseg_ctx* ctx, const acseg_problem* p, const float* image, float* u,
                        float* c_out, float* checkpoints, acseg_stats* stats, void* ws, size_t ws_bytes,
                        void* stream) {
    acseg_status v;
    const bool ckpt = (p->flags & ACSEG_FLAG_STORE_CHECKPOINTS) != 0u;
    const bool fixed_c = (p->flags & ACSEG_FLAG_FIXED_C) != 0u;
    if (!ctx || !image || !u || (ckpt && !checkpoints) || (fixed_c && !c_out))
        return ACSEG_ERR_INVALID_ARG;
    Layout L;
    if ((v = check_ws(p, ws, ws_bytes, &L)) != ACSEG_OK) return v;
    hipStream_t s = (hipStream_t)stream;
    const Coefs cf = coefs_of(p);
    const int64_t nu = (int64_t)p->N * p->W * p->H;
    Ctl* ctl = at<Ctl>(ws, L.ctl);
    double* c64 = at<double>(ws, L.c64);  // [2][kNC]: the means used by step n in set n & 1
    double* tot = at<double>(ws, L.tot);  // [2][kCmeansMaxM]: sums of u^n in set n & 1
    const Bufs bufs{{u, at<float>(ws, L.ubuf), u}};
    ACSEG_TRY(launch_ctl_init(ctl, 0, s));
    if (fixed_c) ACSEG_TRY(launch_widen(c_out, c64 + 2 * kNC, p->N * p->C, s));
    if (ckpt) ACSEG_TRY(hipMemcpyAsync(checkpoints, u, sizeof(float) * nu, hipMemcpyDeviceToDevice, s));
    v = enqueue_means(p, image, u, L, ws, nullptr, c64 + kNC,
                      (p->steps == 0 && !fixed_c) ? c_out : nullptr, tot, s);
    if (v != ACSEG_OK) return v;
    for (int n = 0; n < p->steps; ++n) {
        const int a = n & 1, b = a ^ 1;
        v = enqueue_step(ctx, p, cf, image, bufs, L, ws, n, a, a, n > 0 ? b : -1, s);
        if (v != ACSEG_OK) return v;
        if (ckpt) ACSEG_TRY(launch_copy_current(bufs, ctl, checkpoints + (n + 1) * nu, nu, s));
    }
    ACSEG_TRY(launch_copy_current(bufs, ctl, u, nu, s));
    if (c_out && p->steps > 0 && !fixed_c) {
        const int a = p->steps & 1, b = a ^ 1;  // sums of u^steps; means used by the last step
        ACSEG_TRY(launch_means_from_tot(p->N, p->C, tot + a * kCmeansMaxM, c64 + b * kNC, ctl,
                                        nullptr, c_out, s));
    }
    return read_stats(ctx, L, ws, s, stats);
}

}  // namespace

extern "C" {

acseg_status acseg_batch_workspace_size(int32_t B, const acseg_problem* ps, size_t* bytes) {
    if (!bytes) return ACSEG_ERR_INVALID_ARG;
    const acseg_status v = validate_batch(B, ps);
    if (v != ACSEG_OK) return v;
    *bytes = plan_batch(B, ps).total;
    return ACSEG_OK;
}

acseg_status acseg_solve_batched(acseg_ctx* ctx, int32_t B, const acseg_problem* ps,
                                 const float* const* images, float* const* us,
                                 float* const* c_outs, acseg_stats* stats, void* ws,
                                 size_t ws_bytes, void* stream) {
    acseg_status v = validate_batch(B, ps);
    if (v != ACSEG_OK) return v;
    const bool fixed_c = (ps[0].flags & ACSEG_FLAG_FIXED_C) != 0u;
    if (!ctx || !images || !us || (fixed_c && !c_outs)) return ACSEG_ERR_INVALID_ARG;
    for (int b = 0; b < B; ++b)
        if (!images[b] || !us[b] || (fixed_c && !c_outs[b])) return ACSEG_ERR_INVALID_ARG;
    const BatchPlan bp = plan_batch(B, ps);
    if (!ws || ((uintptr_t)ws % kAlign) != 0 || ws_bytes < bp.total) return ACSEG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* base = static_cast<char*>(ws);

    // ---- descriptor tables and work lists, built on the host.  With
    // REUSE_TABLES the workspace already holds them (from an earlier call with the
    // same arguments): they are built into host memory for the check only, and
    // neither the staging buffer nor the stream is touched.
    const bool reuse = (ps[0].flags & ACSEG_FLAG_REUSE_TABLES) != 0u;
    std::vector<char> local;
    char* hs = nullptr;
    if (reuse) {
        local.assign(bp.table_bytes, 0);
        hs = local.data();
    } else {
        if (ctx->stage_ev) ACSEG_TRY(hipEventSynchronize(ctx->stage_ev));  // the last upload is done
        if (ctx->stage_bytes < bp.table_bytes) {
            if (ctx->stage) ACSEG_TRY(hipHostFree(ctx->stage));
            ctx->stage = nullptr;
            ctx->stage_bytes = 0;
            ACSEG_TRY(hipHostMalloc(&ctx->stage, bp.table_bytes, hipHostMallocDefault));
            ctx->stage_bytes = bp.table_bytes;
        }
        if (!ctx->stage_ev) ACSEG_TRY(hipEventCreateWithFlags(&ctx->stage_ev, hipEventDisableTiming));
        hs = static_cast<char*>(ctx->stage);
        memset(hs, 0, bp.table_bytes);
    }
    CycleArgs* hdesc = reinterpret_cast<CycleArgs*>(hs + bp.descs);
    MgImage* hmg = reinterpret_cast<MgImage*>(hs + bp.mgdescs);
    std::vector<Bufs> bufs(B);
    for (int b = 0; b < B; ++b) {
        void* wsb = base + bp.region[b];
        const Coefs cf = coefs_of(&ps[b]);
        bufs[b] = Bufs{{us[b], at<float>(wsb, bp.L[b].ubuf), us[b]}};
        hdesc[b] = cycle_args_of(&ps[b], cf, images[b], bufs[b], bp.L[b], wsb);
        if (bp.mp[b].L >= 2) hmg[b] = mg_image_of(&ps[b], bp.mp[b], bp.L[b], wsb, bufs[b]);
    }
    if (!bp.work.empty()) memcpy(hs + bp.work_off, bp.work.data(), sizeof(int2) * bp.work.size());
    memcpy(hs + bp.imgs_off, bp.imgs.data(), sizeof(int) * bp.imgs.size());
    if (!bp.mgwork.empty()) memcpy(hs + bp.mgwork_off, bp.mgwork.data(), sizeof(int4) * bp.mgwork.size());
    if (!reuse) {
        ACSEG_TRY(hipMemcpyAsync(base, hs, bp.table_bytes, hipMemcpyHostToDevice, s));
        ACSEG_TRY(hipEventRecord(ctx->stage_ev, s));
        ctx->last_tables.assign(hs, hs + bp.table_bytes);
        ctx->last_tables_ws = ws;
    } else if (ctx->last_tables_ws != ws || ctx->last_tables.size() != bp.table_bytes ||
               memcmp(ctx->last_tables.data(), hs, bp.table_bytes) != 0) {
        return ACSEG_ERR_INVALID_ARG;  // not the tables of this context's last upload to ws
    }
    const CycleArgs* ddesc = reinterpret_cast<const CycleArgs*>(base + bp.descs);
    const MgImage* dmg = reinterpret_cast<const MgImage*>(base + bp.mgdescs);
    const int2* dwork = reinterpret_cast<const int2*>(base + bp.work_off);
    const int* dimgs = reinterpret_cast<const int*>(base + bp.imgs_off);
    const int4* dmgwork = reinterpret_cast<const int4*>(base + bp.mgwork_off);

    // ---- colour means of every u^0
    for (int b = 0; b < B; ++b) {
        void* wsb = base + bp.region[b];
        const Layout& L = bp.L[b];
        ACSEG_TRY(launch_ctl_init(at<Ctl>(wsb, L.ctl), 0, s));
        if (fixed_c) ACSEG_TRY(launch_widen(c_outs[b], at<double>(wsb, L.c64) + 2 * kNC, ps[b].N * ps[b].C, s));
        v = enqueue_means(&ps[b], images[b], us[b], L, wsb, nullptr, at<double>(wsb, L.c64) + kNC,
                          (ps[b].steps == 0 && c_outs && !fixed_c) ? c_outs[b] : nullptr,
                          at<double>(wsb, L.tot), s);
        if (v != ACSEG_OK) return v;
    }

    // ---- the time loop: per group, its cycles' launches over the tiles of all
    // its images (a multigrid cycle: pre-smoothing, the correction's passes,
    // post-smoothing), then the group's step end
    const acseg_problem& p0 = ps[0];
    const int sor = (p0.flags & ACSEG_FLAG_SOR) != 0u ? 1 : 0;
    MgImage none;
    memset(&none, 0, sizeof(none));
    for (int n = 0; n < p0.steps; ++n) {
        const int a = n & 1, bsel = a ^ 1;
        for (const BatchGroup& g : bp.groups) {
            const acseg_problem& pg = ps[g.members[0]];
            const Schedule sc = schedule_of(&pg);
            CycleStep st{};
            st.slot = a;
            st.fixed = sc.fixed ? 1 : 0;
            st.store_rhs = sc.store_rhs ? 1 : 0;
            st.tot_sel = a;
            st.c64_sel = a;
            st.fixed_c = fixed_c ? 1 : 0;
            st.prev_sel = fixed_c ? 2 : (n > 0 ? bsel : -1);
            const CycleGrid grid{ddesc, dwork + g.work0, g.nwork, sor};
            const CycleArgs& any = hdesc[g.members[0]];
            for (int k = 0; k < p0.max_cycles; ++k) {
                st.cycle = k;
                st.cm = (!sc.fixed || k == p0.max_cycles - 1) ? 1 : 0;
                st.launch = k * sc.lpc;
                if (!g.mg) {
                    const CycleRole role{k == 0, true, true};
                    ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] {
                        return launch_cycle(g.N, g.C, pg.nu_pre + pg.nu_post, any, st, grid, role, s);
                    }));
                    continue;
                }
                if (!sc.merged || k == 0) {
                    const CycleRole pre{k == 0, true, false};
                    ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] {
                        return launch_cycle(g.N, g.C, pg.nu_pre, any, st, grid, pre, s);
                    }));
                }
                MgStep ms{};
                ms.slot = a;
                ms.fixed = st.fixed;
                ms.launch = sc.merged ? k + 1 : k * sc.lpc + sc.lpre;
                ms.check = sc.merged ? k : 0;
                ms.nu_pre = pg.nu_pre;
                ms.nu_post = pg.nu_post;
                for (const MgLaunchRec& r : g.mgl) {
                    ms.sweeps = r.sweeps;
                    const MgGrid mgrid{dmg, dmgwork + r.work0, r.nwork};
                    ACSEG_TRY(timed(ctx, mg_family(r.op), s, [&] {
                        return launch_mg(r.op, g.N, g.N, none, mgrid, ms, r.lds, s);
                    }));
                }
                st.launch = sc.merged ? k + 1 : k * sc.lpc + sc.lpre;
                const CycleRole post{false, false, true, true};  // applies the correction's update
                const int sweeps = sc.merged ? 2 : pg.nu_post;
                ACSEG_TRY(timed(ctx, kFamSmooth, s, [&] {
                    return launch_cycle(g.N, g.C, sweeps, any, st, grid, post, s);
                }));
            }
            const StepEndArgs e = sc.merged ? StepEndArgs{p0.max_cycles, 1, 1} : StepEndArgs{p0.max_cycles, sc.lpc, 0};
            ACSEG_TRY(timed(ctx, kFamOther, s, [&] {
                return launch_step_end(g.N, g.C, any, st, e, ddesc, dimgs + g.img0, (int)g.members.size(), s);
            }));
        }
    }

    // ---- results
    for (int b = 0; b < B; ++b) {
        void* wsb = base + bp.region[b];
        const Layout& L = bp.L[b];
        Ctl* ctl = at<Ctl>(wsb, L.ctl);
        const int64_t nu = (int64_t)ps[b].N * ps[b].W * ps[b].H;
        ACSEG_TRY(launch_copy_current(bufs[b], ctl, us[b], nu, s));
        if (c_outs && c_outs[b] && p0.steps > 0 && !fixed_c) {
            const int a = p0.steps & 1, bsel = a ^ 1;
            ACSEG_TRY(launch_means_from_tot(ps[b].N, ps[b].C, at<double>(wsb, L.tot) + a * kCmeansMaxM,
                                            at<double>(wsb, L.c64) + bsel * kNC, ctl, nullptr,
                                            c_outs[b], s));
        }
    }
    if (stats)
        for (int b = 0; b < B; ++b) {
            v = read_stats(ctx, bp.L[b], base + bp.region[b], s, &stats[b]);
            if (v != ACSEG_OK) return v;
        }
    return ACSEG_OK;
}

acseg_status acseg_labels(acseg_ctx* ctx, const acseg_problem* p, const float* u, const float* c,
                          uint8_t* labels, float* composite, float* rounded, void* stream) {
    const acseg_status v = validate(p, false);
    if (v != ACSEG_OK) return v;
    if (!ctx || !u || !c) return ACSEG_ERR_INVALID_ARG;
    return hip_status(launch_labels(p->N, p->C, p->W, p->H, u, c, labels, composite, rounded,
                                    (hipStream_t)stream));
}

acseg_status acseg_backward_workspace_size(const acseg_problem* p, size_t* bytes) {
    if (!bytes) return ACSEG_ERR_INVALID_ARG;
    const acseg_status v = validate(p, true);
    if (v != ACSEG_OK) return v;
    *bytes = back_layout_of(p).total;
    return ACSEG_OK;
}

acseg_status acseg_backward(acseg_ctx* ctx, const acseg_problem* p, const float* image,
                            const float* checkpoints, const float* c_fixed,
                            const float* grad_uT, float* grad_image, float* grad_u0,
                            double* grad_params, float* grad_c, acseg_stats* stats, void* ws,
                            size_t ws_bytes, void* stream) {
    acseg_status v = validate(p, true);
    if (v != ACSEG_OK) return v;
    const bool fixed_c = (p->flags & ACSEG_FLAG_FIXED_C) != 0u;
    if (!ctx || !image || !checkpoints || !grad_uT || !grad_image || !grad_params || (fixed_c && !c_fixed))
        return ACSEG_ERR_INVALID_ARG;
    const BackLayout L = back_layout_of(p);
    if (!ws || ((uintptr_t)ws % kAlign) != 0 || ws_bytes < L.total) return ACSEG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int N = p->N, C = p->C, W = p->W, H = p->H;
    const int64_t n = (int64_t)W * H, nu = (int64_t)N * n;
    const int K = adj_sweeps_per_launch();
    Ctl* ctl = at<Ctl>(ws, L.ctl);
    AdjCtl* actl = at<AdjCtl>(ws, L.actl);
    double* c64 = at<double>(ws, L.c64);
    double* tot = at<double>(ws, L.tot);
    AdjArgs a{};
    a.ctl = ctl;
    a.actl = actl;
    a.image = image;
    a.z = at<float>(ws, L.z);
    a.z2 = at<float>(ws, L.z2);
    a.Ibar = grad_image;
    a.grads = grad_params;
    a.cbar64 = at<double>(ws, L.cbar);
    a.part_f = at<float>(ws, L.part_f);
    a.part_d = at<double>(ws, L.part_adj);
    a.coef = coefs_of(p).fine;
    const float dA[4] = {4.f, 2.f, 1.f, 1.f};
    for (int k = 0; k < 4; ++k) a.diagA[k] = dA[k];
    // SOR factor from q = max over node classes of kappa * (sum of edge weights
    // = stiffness diagonal), the bound of the block-Jacobi radius
    {
        double q = 0.0;
        for (int k = 0; k < 4; ++k) q = std::max(q, (double)a.coef.kappa[k] * dA[k]);
        q = std::min(q, 0.999);
        a.omega = (float)std::min(1.95, 2.0 / (1.0 + std::sqrt(1.0 - q * q)));
    }
    a.h2 = p->h * p->h;
    a.inv_h2 = (float)(1.0 / a.h2);
    a.rtol = (float)std::max(p->tol, 2e-7);
    a.eps = p->eps;
    a.tau = p->tau;
    a.lambda = p->lambda;
    a.W = W;
    a.H = H;
    a.nblocks = adj_sweep_blocks(W, H);
    a.nblocks_acc = adj_accum_blocks(N, C, W, H);
    a.max_sweeps = (std::min(4000, std::max(4, 2 * p->max_cycles)) + K - 1) / K * K;
    float* ubuf[2] = {at<float>(ws, L.ub0), at<float>(ws, L.ub1)};

    // The sweeps of a step stop at convergence; how many it takes is known on
    // the device only.  With a remembered count for the same problem (the most
    // sweeps any step of an earlier backward took), every step gets that
    // budget and no host wait; a step that used its whole budget below the
    // cap without converging makes the call run again with waits.  Without
    // one, the sweeps go in chunks with a read of the convergence flag after
    // each.
    auto memo = std::find_if(ctx->adj_memo.begin(), ctx->adj_memo.end(), [&](const auto& e) {
        return memcmp(&e.first, p, sizeof(*p)) == 0;
    });
    const int budget = memo == ctx->adj_memo.end() ? 0 : std::min(a.max_sweeps, (memo->second + K - 1) / K * K);

    auto run = [&](int spec) -> acseg_status {
        ACSEG_TRY(launch_ctl_init(ctl, 0, s));
        ACSEG_TRY(launch_adj_init(actl, grad_params, s));
        ACSEG_TRY(launch_fill(grad_image, (int64_t)C * n, 0.f, s));
        if (fixed_c) {
            ACSEG_TRY(launch_widen(c_fixed, c64, N * C, s));
            if (grad_c) ACSEG_TRY(launch_fill(grad_c, (int64_t)N * C, 0.f, s));
        } else {
            // the means of every step, recomputed from the checkpoints
            for (int f = 0; f < p->steps; f += kCmeansFields) {
                const int cnt = std::min(kCmeansFields, p->steps - f);
                ACSEG_TRY(timed(ctx, kFamCmeans, s, [&] {
                    return launch_cmeans_fields(N, C, W, H, image, checkpoints, f, cnt, at<double>(ws, L.part_cm),
                                                tot, c64, ctl, s);
                }));
            }
        }
        const float* ub = grad_uT;
        a.cm_cbar = a.cm_c64 = a.cm_tot = nullptr;
        for (int st = p->steps - 1; st >= 0; --st) {
            a.u0 = checkpoints + st * nu;
            a.u1 = checkpoints + (st + 1) * nu;
            a.ub = ub;
            a.ub_out = ubuf[st & 1];
            a.c64 = fixed_c ? c64 : c64 + st * kNC;
            a.tot = tot + st * kCmeansMaxM;
            a.cbar_out = grad_c ? (fixed_c ? grad_c : grad_c + (int64_t)st * N * C) : nullptr;
            a.cbar_accumulate = fixed_c ? 1 : 0;
            int sw = 0;
            if (spec > 0) {
                for (; sw < spec; sw += K)
                    ACSEG_TRY(timed(ctx, kFamAdjSweep, s, [&] { return launch_adj(N, C, kAdjSweep, a, sw, s); }));
            } else {
                int chunk = 4;
                while (true) {
                    const int end = std::min(a.max_sweeps, sw + chunk);
                    for (; sw < end; sw += K)
                        ACSEG_TRY(timed(ctx, kFamAdjSweep, s,
                                        [&] { return launch_adj(N, C, kAdjSweep, a, sw, s); }));
                    if (sw >= a.max_sweeps) break;
                    ACSEG_TRY(timed(ctx, kFamOther, s, [&] { return launch_adj(N, C, kAdjCheck, a, sw, s); }));
                    ACSEG_TRY(hipMemcpyAsync(ctx->host_actl, actl, sizeof(AdjCtl), hipMemcpyDeviceToHost, s));
                    ACSEG_TRY(hipStreamSynchronize(s));
                    if (ctx->host_actl->done) break;
                    chunk = std::min(64, chunk * 2);
                }
            }
            a.budget = sw;
            ACSEG_TRY(timed(ctx, kFamOther, s, [&] { return launch_adj(N, C, kAdjAccum, a, 0, s); }));
            ACSEG_TRY(timed(ctx, kFamOther, s, [&] { return launch_adj(N, C, kAdjReduce, a, 0, s); }));
            ub = a.ub_out;
            // this step's means share goes to the next step's launches (fixed
            // means depend on neither u^n nor the image: no share)
            if (!fixed_c) {
                a.cm_cbar = a.cbar64;
                a.cm_c64 = c64 + st * kNC;
                a.cm_tot = tot + st * kCmeansMaxM;
            }
        }
        if (a.cm_cbar) {
            // the first step's share: grad_u0 and dL/dI
            a.u0 = checkpoints;
            a.ub = ub;
            a.ub_out = grad_u0;
            ACSEG_TRY(timed(ctx, kFamOther, s, [&] { return launch_adj(N, C, kAdjFinal, a, 0, s); }));
        } else if (grad_u0) {
            ACSEG_TRY(hipMemcpyAsync(grad_u0, ub, sizeof(float) * nu, hipMemcpyDeviceToDevice, s));
        }
        ACSEG_TRY(hipMemcpyAsync(ctx->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        ACSEG_TRY(hipMemcpyAsync(ctx->host_actl, actl, sizeof(AdjCtl), hipMemcpyDeviceToHost, s));
        ACSEG_TRY(hipStreamSynchronize(s));
        return ACSEG_OK;
    };
    acseg_status r = run(budget);
    if (r != ACSEG_OK) return r;
    const bool rerun = budget > 0 && ctx->host_actl->short_steps > 0;
    if (rerun) {
        r = run(0);
        if (r != ACSEG_OK) return r;
    }
    const Ctl& c = *ctx->host_ctl;
    if (memo != ctx->adj_memo.end()) {
        // a count that sufficed decays by one launch per call, so one slow
        // problem does not hold the budget up for good
        memo->second = rerun ? c.cycles_max : std::max(c.cycles_max, memo->second - K);
    } else {
        if (ctx->adj_memo.size() >= kAdjMemo) ctx->adj_memo.erase(ctx->adj_memo.begin());
        ctx->adj_memo.push_back({*p, c.cycles_max});
    }
    if (!stats) return ACSEG_OK;
    memset(stats, 0, sizeof(*stats));
    stats->steps_done = c.steps_done;
    stats->cycles_total = c.cycles_total;
    stats->cycles_max = c.cycles_max;
    stats->steps_not_converged = c.steps_unconv;
    stats->status = c.nonfinite ? ACSEG_ERR_NONFINITE : (c.steps_unconv ? ACSEG_WARN_NOT_CONVERGED : ACSEG_OK);
    return ACSEG_OK;
}

acseg_status acseg_energy(acseg_ctx* ctx, const acseg_problem* p, const float* image,
                          const float* u, double* energy, void* ws, size_t ws_bytes,
                          void* stream) {
    acseg_status v = validate(p, false);
    if (v != ACSEG_OK) return v;
    if (!ctx || !image || !u || !energy) return ACSEG_ERR_INVALID_ARG;
    Layout L;
    if ((v = check_ws(p, ws, ws_bytes, &L)) != ACSEG_OK) return v;
    hipStream_t s = (hipStream_t)stream;
    Ctl* ctl = at<Ctl>(ws, L.ctl);
    double* c64 = at<double>(ws, L.c64);
    ACSEG_TRY(launch_ctl_init(ctl, 0, s));
    v = enqueue_means(p, image, u, L, ws, nullptr, c64, nullptr, nullptr, s);
    if (v != ACSEG_OK) return v;
    ACSEG_TRY(launch_energy(p->N, p->C, p->W, p->H, image, u, c64, p->eps, p->lambda, p->h,
                            at<double>(ws, L.part_d), energy, s));
    return ACSEG_OK;
}

acseg_status acseg_timing_enable(acseg_ctx* ctx, int32_t enable) {
    if (!ctx) return ACSEG_ERR_INVALID_ARG;
    ctx->timing = enable != 0;
    return ACSEG_OK;
}

acseg_status acseg_timing_read(acseg_ctx* ctx, acseg_kernel_time* out, int32_t max,
                               int32_t* count) {
    if (!ctx || !count || max < 0 || (max > 0 && !out)) return ACSEG_ERR_INVALID_ARG;
    int64_t launches[kFamCount] = {};
    double total[kFamCount] = {};
    acseg_status st = ACSEG_OK;
    for (const TimedRec& r : ctx->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            st = ACSEG_ERR_HIP;
        launches[r.fam] += 1;
        total[r.fam] += ms;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    int n = 0;
    for (int f = 0; f < kFamCount; ++f) {
        if (launches[f] == 0) continue;
        if (n < max) {
            memset(&out[n], 0, sizeof(out[n]));
            strncpy(out[n].name, kFamName[f], sizeof(out[n].name) - 1);
            out[n].launches = launches[f];
            out[n].total_ms = total[f];
        }
        ++n;
    }
    *count = n < max ? n : max;
    return st;
}

}  // extern "C"
