/*
 * acseg_oracle.c -- plain FP64 CPU oracle for the vector-valued Allen-Cahn
 * phase-field segmentation of Kay & Tomasi ("Colour Image Segmentation by the
 * Vector-valued Allen-Cahn Phase-field Model: a Multigrid Solution").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP implementation; it is slow
 * on purpose and written so that each function can be checked against the
 * paper by eye.
 *
 * What is computed, by section of the paper:
 *   - the P1 finite-element space on the pixel lattice, its lumped mass
 *     M_p = <eta_p, 1> and stiffness A_pq = <grad eta_p, grad eta_q>
 *     (Section "Finite Element Notation"), assembled triangle by triangle;
 *   - colour means c_ij = int u_i I_j / int u_i and fitting
 *     F_i = sum_j (I_j - c_ij)^2 (eq. VV_fidelity and its multichannel form in
 *     Section "Two Dimensional Examples"), with the lumped-mass quadrature
 *     ("projection by node", Section "Data Projection");
 *   - one backward-Euler time step of the discrete variational inequality
 *     (eq. E_fe, eq. alpha): the diffusion and the simplex constraint are
 *     implicit, the concave part -(2/eps) u and the fitting term are taken at
 *     the old time level.  Readings: the stiffness enters with a positive sign
 *     (it comes from eps |grad u|^2 / 2 in eq. E), and the time step multiplies
 *     the whole bracket of eq. alpha;
 *   - the Gibbs-simplex constraint of Section "Gibbs Space Constraint
 *     Pseudocode" as the exact Euclidean projection onto the simplex
 *     (Michelot's finite algorithm, the procedure the section describes);
 *   - a lexicographic projected block Gauss-Seidel sweep over the nodal
 *     sub-problems (Section "Finite Element Notation") and a truncated
 *     multigrid correction with an exact line search (Section "Multigrid
 *     Solution"; truncation as motivated at the start of the Gibbs-constraint
 *     section), iterated until the natural residual meets the tolerance;
 *   - the paper's own multilevel iteration (Section "Multigrid Solution"):
 *     successive subspace correction over the basis functions of every level,
 *     seen on the finest lattice, from the coarsest level to the finest, each
 *     correction kept on the simplices by the Gibbs correction with the
 *     function's own lower bound;
 *   - the discrete energy of eq. E and the composite / rounded composite of
 *     Section "Post-processing".
 *
 * Data layout: node (x, y) of a W x H lattice has flat index p = y*W + x;
 * phase fields are [N][H*W], images [C][H*W], all double.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_N 64

typedef struct {
    int32_t H, W, C, N;
    double h, eps, lambda, tau;
    int32_t levels;        /* lattice levels incl. the finest; 1 = Gauss-Seidel only, 0 = auto */
    int32_t nu_pre, nu_post;
    int32_t coarse_sweeps; /* Gauss-Seidel sweeps on the coarsest level */
    int32_t max_cycles;
    int32_t ssc;           /* 1: cycles are the paper's subspace correction over all basis functions */
    double tol;            /* on the natural residual (max norm) */
} orc_params;

typedef struct {
    int32_t cycles;
    int32_t converged;
    int32_t empty_phase;
    int32_t nonmonotone;   /* coarse corrections that raised the step objective */
    double residual;
    double objective;
} orc_stats;

/* ------------------------------------------------------------------------ */
/* Finite-element space on the lattice                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int W, H;
    double h;
    double *mass;   /* [H*W]   lumped mass <eta_p, 1> */
    double *stiff;  /* [H*W*9] A_pq for q = p + (dx, dy), slot (dy+1)*3 + (dx+1) */
} grid_t;

static int slot(int dx, int dy) { return (dy + 1) * 3 + (dx + 1); }

/* Add the contributions of one P1 triangle with lattice vertices v[3][2]. */
static void add_triangle(grid_t *g, const int v[3][2])
{
    double X[3], Y[3];
    for (int a = 0; a < 3; ++a) {
        X[a] = v[a][0] * g->h;
        Y[a] = v[a][1] * g->h;
    }
    /* twice the signed area */
    double two_area = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
    double area = fabs(two_area) / 2.0;
    /* gradients of the three barycentric (hat) functions on this triangle */
    double gx[3], gy[3];
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        gx[a] = (Y[b] - Y[c]) / two_area;
        gy[a] = (X[c] - X[b]) / two_area;
    }
    for (int a = 0; a < 3; ++a) {
        int pa = v[a][1] * g->W + v[a][0];
        g->mass[pa] += area / 3.0;  /* integral of a hat function over the triangle */
        for (int b = 0; b < 3; ++b) {
            int dx = v[b][0] - v[a][0], dy = v[b][1] - v[a][1];
            g->stiff[(size_t)pa * 9 + slot(dx, dy)] += area * (gx[a] * gx[b] + gy[a] * gy[b]);
        }
    }
}

/* Every lattice cell is split along its diagonal (x,y)-(x+1,y+1). */
static int grid_init(grid_t *g, int W, int H, double h)
{
    g->W = W;
    g->H = H;
    g->h = h;
    g->mass = calloc((size_t)W * H, sizeof(double));
    g->stiff = calloc((size_t)W * H * 9, sizeof(double));
    if (!g->mass || !g->stiff) return -1;
    for (int cy = 0; cy + 1 < H; ++cy)
        for (int cx = 0; cx + 1 < W; ++cx) {
            const int t1[3][2] = {{cx, cy}, {cx + 1, cy}, {cx + 1, cy + 1}};
            const int t2[3][2] = {{cx, cy}, {cx + 1, cy + 1}, {cx, cy + 1}};
            add_triangle(g, t1);
            add_triangle(g, t2);
        }
    return 0;
}

static void grid_free(grid_t *g)
{
    free(g->mass);
    free(g->stiff);
    g->mass = g->stiff = NULL;
}

/* (A v)_p for one scalar field v on grid g */
static double stiff_apply(const grid_t *g, const double *v, int x, int y)
{
    double s = 0.0;
    int p = y * g->W + x;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int qx = x + dx, qy = y + dy;
            if (qx < 0 || qy < 0 || qx >= g->W || qy >= g->H) continue;
            s += g->stiff[(size_t)p * 9 + slot(dx, dy)] * v[qy * g->W + qx];
        }
    return s;
}

/* sum over q != p of A_pq v_q */
static double stiff_offdiag(const grid_t *g, const double *v, int x, int y)
{
    int p = y * g->W + x;
    return stiff_apply(g, v, x, y) - g->stiff[(size_t)p * 9 + slot(0, 0)] * v[p];
}

/* ------------------------------------------------------------------------ */
/* Gibbs-simplex projection                                                  */
/* ------------------------------------------------------------------------ */

/*
 * Euclidean projection of y onto the Gibbs simplex {x : sum_i x_i = 1,
 * x_i >= 0}, the nodal constraint of Section "Gibbs Space Constraint
 * Pseudocode", by Michelot's finite algorithm (C. Michelot, J. Optim. Theory
 * Appl. 50, 1986).  With F the current free set, the projection onto the
 * affine set {sum_{i in F} x_i = 1, x_i = 0 outside F} shifts every free
 * component by the same theta = (sum_{i in F} y_i - 1) / |F|.  Components
 * that come out negative leave F for good and the projection onto the
 * smaller affine set is taken again from y; once none is negative, x is the
 * projection onto the simplex.  F shrinks every round but never empties (its
 * values sum to one), so there are at most N rounds.  Returns the number of
 * rounds (>= 1).
 */
int orc_project(int N, const double *y, double *x)
{
    unsigned char in_f[ORC_MAX_N];
    if (N < 1 || N > ORC_MAX_N) return -1;
    for (int i = 0; i < N; ++i) in_f[i] = 1;
    int size = N, rounds = 0;
    for (;;) {
        ++rounds;
        double s = 0.0;
        for (int i = 0; i < N; ++i)
            if (in_f[i]) s += y[i];
        const double theta = (s - 1.0) / size;
        int left = 0;
        for (int i = 0; i < N; ++i) {
            x[i] = in_f[i] ? y[i] - theta : 0.0;
            if (in_f[i] && x[i] < 0.0) {
                in_f[i] = 0;
                ++left;
            }
        }
        if (left == 0) return rounds;
        size -= left;
    }
}

/* ------------------------------------------------------------------------ */
/* Colour means, fitting term, right-hand side                               */
/* ------------------------------------------------------------------------ */

/*
 * c_ij = sum_p M_p u_pi I_pj / sum_p M_p u_pi.  A phase whose mass is below
 * 1e-12 of the domain area has no mean; it keeps c_prev (or, without c_prev,
 * the mean colour of the whole image).  Returns 1 if some phase was empty.
 */
static int colour_means(const grid_t *g, int N, int C, const double *I, const double *u,
                        const double *c_prev, double *c)
{
    size_t n = (size_t)g->W * g->H;
    double area = 0.0;
    for (size_t p = 0; p < n; ++p) area += g->mass[p];
    int empty = 0;
    for (int i = 0; i < N; ++i) {
        double S = 0.0;
        for (size_t p = 0; p < n; ++p) S += g->mass[p] * u[i * n + p];
        if (S > 1e-12 * area) {
            for (int k = 0; k < C; ++k) {
                double Sk = 0.0;
                for (size_t p = 0; p < n; ++p) Sk += g->mass[p] * u[i * n + p] * I[k * n + p];
                c[i * C + k] = Sk / S;
            }
        } else {
            empty = 1;
            for (int k = 0; k < C; ++k) {
                if (c_prev) {
                    c[i * C + k] = c_prev[i * C + k];
                } else {
                    double Sk = 0.0;
                    for (size_t p = 0; p < n; ++p) Sk += g->mass[p] * I[k * n + p];
                    c[i * C + k] = Sk / area;
                }
            }
        }
    }
    return empty;
}

static double fitting(int C, const double *I, size_t n, size_t p, const double *ci)
{
    double F = 0.0;
    for (int k = 0; k < C; ++k) {
        double d = I[k * n + p] - ci[k];
        F += d * d;
    }
    return F;
}

/* b_pi = M_p [ (1/tau + 2/eps) un_pi - lambda F_pi(c) ] */
static void rhs(const grid_t *g, const orc_params *P, const double *I, const double *un,
                const double *c, double *b)
{
    size_t n = (size_t)g->W * g->H;
    for (int i = 0; i < P->N; ++i)
        for (size_t p = 0; p < n; ++p)
            b[i * n + p] = g->mass[p] * ((1.0 / P->tau + 2.0 / P->eps) * un[i * n + p]
                                         - P->lambda * fitting(P->C, I, n, p, c + i * P->C));
}

/* ------------------------------------------------------------------------ */
/* The step problem: minimise J(u) = sum_i [ u_i.H u_i / 2 - b_i.u_i ]       */
/* over the product of simplices, H = M/tau + eps A.                          */
/* ------------------------------------------------------------------------ */

static double diag_H(const grid_t *g, const orc_params *P, size_t p)
{
    return g->mass[p] / P->tau + P->eps * g->stiff[p * 9 + slot(0, 0)];
}

/* Unconstrained nodal minimiser y_p of J in the block of node p (N values). */
static void nodal_trial(const grid_t *g, const orc_params *P, const double *b, const double *u,
                        int x, int y, double *yv)
{
    size_t n = (size_t)g->W * g->H, p = (size_t)y * g->W + x;
    double d = diag_H(g, P, p);
    for (int i = 0; i < P->N; ++i)
        yv[i] = (b[i * n + p] - P->eps * stiff_offdiag(g, u + i * n, x, y)) / d;
}

/* One lexicographic (row-major) sweep of projected block Gauss-Seidel. */
static void gs_sweep(const grid_t *g, const orc_params *P, const double *b, double *u)
{
    size_t n = (size_t)g->W * g->H;
    double yv[ORC_MAX_N], xv[ORC_MAX_N];
    for (int y = 0; y < g->H; ++y)
        for (int x = 0; x < g->W; ++x) {
            nodal_trial(g, P, b, u, x, y, yv);
            orc_project(P->N, yv, xv);
            for (int i = 0; i < P->N; ++i) u[i * n + (size_t)y * g->W + x] = xv[i];
        }
}

/* Natural residual max_{p,i} |Pi(y_p(u)) - u_p|, every node evaluated at u. */
static double natural_residual(const grid_t *g, const orc_params *P, const double *b,
                               const double *u)
{
    size_t n = (size_t)g->W * g->H;
    double yv[ORC_MAX_N], xv[ORC_MAX_N], r = 0.0;
    for (int y = 0; y < g->H; ++y)
        for (int x = 0; x < g->W; ++x) {
            nodal_trial(g, P, b, u, x, y, yv);
            orc_project(P->N, yv, xv);
            for (int i = 0; i < P->N; ++i) {
                double d = fabs(xv[i] - u[i * n + (size_t)y * g->W + x]);
                if (d > r) r = d;
            }
        }
    return r;
}

static double objective(const grid_t *g, const orc_params *P, const double *b, const double *u)
{
    size_t n = (size_t)g->W * g->H;
    double J = 0.0;
    for (int i = 0; i < P->N; ++i)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                size_t p = (size_t)y * g->W + x;
                double Hu = g->mass[p] / P->tau * u[i * n + p] + P->eps * stiff_apply(g, u + i * n, x, y);
                J += 0.5 * u[i * n + p] * Hu - b[i * n + p] * u[i * n + p];
            }
    return J;
}

/* ------------------------------------------------------------------------ */
/* Lattice hierarchy and transfers                                           */
/* ------------------------------------------------------------------------ */

/* Coarse node j sits on fine node 2j, so a side of n nodes coarsens to ceil(n/2). */
static int coarse_side(int n) { return (n + 1) / 2; }

int orc_auto_levels(int W, int H)
{
    int L = 1;
    while ((W > H ? W : H) > 15 && (W < H ? W : H) >= 3) {
        W = coarse_side(W);
        H = coarse_side(H);
        ++L;
    }
    return L;
}

/*
 * Prolongation: the fine value at node (x, y) is the coarse P1 function
 * evaluated at the fine node's position, (x/2, y/2) in coarse lattice units,
 * clamped into the coarse lattice (a fine node past the last coarse row or
 * column takes the value on that row or column).  The coarse cell is split
 * along the same diagonal as the fine ones.  Emits up to 3 (coarse index,
 * weight) pairs and returns their count.
 */
static int prolong_weights(int x, int y, int Wc, int Hc, int *q, double *wt)
{
    double X = 0.5 * x, Y = 0.5 * y;
    if (X > Wc - 1) X = Wc - 1;
    if (Y > Hc - 1) Y = Hc - 1;
    int i0 = (int)floor(X), j0 = (int)floor(Y);
    int i1 = i0 + 1 < Wc ? i0 + 1 : i0, j1 = j0 + 1 < Hc ? j0 + 1 : j0;
    double s = X - i0, t = Y - j0;
    int m = 0;
    /* barycentric coordinates on the lower (s >= t) or upper (s < t) triangle */
    if (s >= t) {
        q[m] = j0 * Wc + i0; wt[m++] = 1.0 - s;
        q[m] = j0 * Wc + i1; wt[m++] = s - t;
        q[m] = j1 * Wc + i1; wt[m++] = t;
    } else {
        q[m] = j0 * Wc + i0; wt[m++] = 1.0 - t;
        q[m] = j1 * Wc + i0; wt[m++] = t - s;
        q[m] = j1 * Wc + i1; wt[m++] = s;
    }
    return m;
}

/* vf (fine, N planes) = P vc */
static void prolong(const grid_t *f, const grid_t *cg, int N, const double *vc, double *vf)
{
    size_t nf = (size_t)f->W * f->H, nc = (size_t)cg->W * cg->H;
    int q[3];
    double wt[3];
    for (int y = 0; y < f->H; ++y)
        for (int x = 0; x < f->W; ++x) {
            int m = prolong_weights(x, y, cg->W, cg->H, q, wt);
            for (int i = 0; i < N; ++i) {
                double s = 0.0;
                for (int k = 0; k < m; ++k) s += wt[k] * vc[i * nc + q[k]];
                vf[i * nf + (size_t)y * f->W + x] = s;
            }
        }
}

/* rc (coarse, N planes) = P^T rf */
static void restrict_T(const grid_t *f, const grid_t *cg, int N, const double *rf, double *rc)
{
    size_t nf = (size_t)f->W * f->H, nc = (size_t)cg->W * cg->H;
    int q[3];
    double wt[3];
    memset(rc, 0, sizeof(double) * N * nc);
    for (int y = 0; y < f->H; ++y)
        for (int x = 0; x < f->W; ++x) {
            int m = prolong_weights(x, y, cg->W, cg->H, q, wt);
            for (int i = 0; i < N; ++i)
                for (int k = 0; k < m; ++k)
                    rc[i * nc + q[k]] += wt[k] * rf[i * nf + (size_t)y * f->W + x];
        }
}

/* ------------------------------------------------------------------------ */
/* Linear coarse-level correction (componentwise, untruncated operator)       */
/* ------------------------------------------------------------------------ */

static void lin_gs_sweep(const grid_t *g, const orc_params *P, const double *r, double *v)
{
    size_t n = (size_t)g->W * g->H;
    for (int y = 0; y < g->H; ++y)
        for (int x = 0; x < g->W; ++x) {
            size_t p = (size_t)y * g->W + x;
            double d = diag_H(g, P, p);
            for (int i = 0; i < P->N; ++i)
                v[i * n + p] = (r[i * n + p] - P->eps * stiff_offdiag(g, v + i * n, x, y)) / d;
        }
}

/* res = r - H v */
static void lin_residual(const grid_t *g, const orc_params *P, const double *r, const double *v,
                         double *res)
{
    size_t n = (size_t)g->W * g->H;
    for (int i = 0; i < P->N; ++i)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                size_t p = (size_t)y * g->W + x;
                res[i * n + p] = r[i * n + p] - (g->mass[p] / P->tau * v[i * n + p]
                                                 + P->eps * stiff_apply(g, v + i * n, x, y));
            }
}

/* Approximate solve of H_l v = r on level l (0 = finest) with a V-cycle, v from 0. */
static void coarse_vcycle(const grid_t *G, int L, int l, const orc_params *P, const double *r,
                          double *v)
{
    const grid_t *g = &G[l];
    size_t n = (size_t)g->W * g->H;
    memset(v, 0, sizeof(double) * P->N * n);
    if (l == L - 1) {
        for (int s = 0; s < P->coarse_sweeps; ++s) lin_gs_sweep(g, P, r, v);
        return;
    }
    for (int s = 0; s < P->nu_pre; ++s) lin_gs_sweep(g, P, r, v);
    const grid_t *c = &G[l + 1];
    size_t nc = (size_t)c->W * c->H;
    double *res = malloc(sizeof(double) * P->N * n);
    double *rc = malloc(sizeof(double) * P->N * nc);
    double *vc = malloc(sizeof(double) * P->N * nc);
    double *e = malloc(sizeof(double) * P->N * n);
    lin_residual(g, P, r, v, res);
    restrict_T(g, c, P->N, res, rc);
    coarse_vcycle(G, L, l + 1, P, rc, vc);
    prolong(g, c, P->N, vc, e);
    for (size_t k = 0; k < (size_t)P->N * n; ++k) v[k] += e[k];
    for (int s = 0; s < P->nu_post; ++s) lin_gs_sweep(g, P, r, v);
    free(res);
    free(rc);
    free(vc);
    free(e);
}

/*
 * T_I x: zero the components outside the free set I = {i : u_i > 0} and
 * remove the mean over I from the others (the tangent projection restricted to
 * the free components).  With one free component or fewer the result is 0.
 */
static void tangent_free(int N, const double *up, const double *xin, double *xout)
{
    int k = 0;
    double s = 0.0;
    for (int i = 0; i < N; ++i)
        if (up[i] > 0.0) {
            ++k;
            s += xin[i];
        }
    for (int i = 0; i < N; ++i) xout[i] = (k >= 2 && up[i] > 0.0) ? xin[i] - s / k : 0.0;
}

/*
 * One truncated multigrid cycle on the step problem:
 *   pre-smooth; defect g = b - H u; truncate it node by node with T_I;
 *   restrict; approximately solve the componentwise linear coarse problems;
 *   prolong, truncate again, make it feasible (w = Pi(u + v) - u, a feasible
 *   direction because the simplex is convex); exact line search on J along w
 *   with the step clamped to [0, 1]; post-smooth.
 * Returns 1 if the coarse correction raised J (never expected).
 */
static int mg_cycle(const grid_t *G, int L, const orc_params *P, const double *b, double *u)
{
    const grid_t *g = &G[0];
    const grid_t *c = &G[1];
    int N = P->N;
    size_t n = (size_t)g->W * g->H, nc = (size_t)c->W * c->H;
    for (int s = 0; s < P->nu_pre; ++s) gs_sweep(g, P, b, u);

    double *gd = malloc(sizeof(double) * N * n);
    double *gt = malloc(sizeof(double) * N * n);
    double *rc = malloc(sizeof(double) * N * nc);
    double *vc = malloc(sizeof(double) * N * nc);
    double *v = malloc(sizeof(double) * N * n);
    double *w = malloc(sizeof(double) * N * n);
    double up[ORC_MAX_N], xi[ORC_MAX_N], xo[ORC_MAX_N];

    /* defect g = b - H u (the negative gradient of J) */
    for (int i = 0; i < N; ++i)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                size_t p = (size_t)y * g->W + x;
                gd[i * n + p] = b[i * n + p] - (g->mass[p] / P->tau * u[i * n + p]
                                                + P->eps * stiff_apply(g, u + i * n, x, y));
            }
    for (size_t p = 0; p < n; ++p) {
        for (int i = 0; i < N; ++i) {
            up[i] = u[i * n + p];
            xi[i] = gd[i * n + p];
        }
        tangent_free(N, up, xi, xo);
        for (int i = 0; i < N; ++i) gt[i * n + p] = xo[i];
    }
    restrict_T(g, c, N, gt, rc);
    coarse_vcycle(G, L, 1, P, rc, vc);
    prolong(g, c, N, vc, v);

    /* feasible direction */
    for (size_t p = 0; p < n; ++p) {
        for (int i = 0; i < N; ++i) {
            up[i] = u[i * n + p];
            xi[i] = v[i * n + p];
        }
        tangent_free(N, up, xi, xo);
        for (int i = 0; i < N; ++i) xi[i] = up[i] + xo[i];
        orc_project(N, xi, xo);
        for (int i = 0; i < N; ++i) w[i * n + p] = xo[i] - up[i];
    }
    /*
     * Exact line search: J(u + a w) = J(u) - a <g,w> + a^2 <w,Hw> / 2.  The
     * direction w is zero on the active components and sums to zero over the
     * free ones at every node, so <g,w> = <T_I g, w>; the truncated defect is
     * used because the full one carries the per-node multiplier of the sum
     * constraint, whose round-off would swamp <g,w> near convergence.
     */
    double gw = 0.0, wHw = 0.0;
    for (int i = 0; i < N; ++i)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                size_t p = (size_t)y * g->W + x;
                gw += gt[i * n + p] * w[i * n + p];
                wHw += w[i * n + p] * (g->mass[p] / P->tau * w[i * n + p]
                                       + P->eps * stiff_apply(g, w + i * n, x, y));
            }
    int bad = 0;
    if (wHw > 0.0 && gw > 0.0) {
        double a = gw / wHw;
        if (a > 1.0) a = 1.0;
        double J0 = objective(g, P, b, u);
        for (size_t k = 0; k < (size_t)N * n; ++k) u[k] += a * w[k];
        double J1 = objective(g, P, b, u);
        if (J1 > J0 + 1e-12 * fabs(J0)) bad = 1;
    }
    free(gd);
    free(gt);
    free(rc);
    free(vc);
    free(v);
    free(w);
    for (int s = 0; s < P->nu_post; ++s) gs_sweep(g, P, b, u);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Successive subspace correction over the basis functions of every level     */
/* (Section "Multigrid Solution"; Gibbs correction of Section "Gibbs Space    */
/* Constraint Pseudocode")                                                    */
/* ------------------------------------------------------------------------ */

/* A basis function of some level seen on the finest lattice: its nonzero values. */
typedef struct {
    int count;
    int *idx;     /* finest-lattice node indices where eta > 0 */
    double *val;  /* eta at those nodes */
} basis_fn;

/*
 * eta for node q of level l (0 = finest): the unit vector of node q prolonged
 * level by level down to level 0 (all basis functions of all levels are
 * projected onto the finest grid).
 */
static int basis_build(const grid_t *G, int l, int q, basis_fn *f)
{
    size_t m = (size_t)G[l].W * G[l].H;
    double *a = calloc(m, sizeof(double));
    if (!a) return -1;
    a[q] = 1.0;
    for (int k = l; k > 0; --k) {
        size_t mf = (size_t)G[k - 1].W * G[k - 1].H;
        double *fine = malloc(sizeof(double) * mf);
        if (!fine) {
            free(a);
            return -1;
        }
        prolong(&G[k - 1], &G[k], 1, a, fine);
        free(a);
        a = fine;
        m = mf;
    }
    f->count = 0;
    for (size_t p = 0; p < m; ++p) f->count += a[p] > 0.0;
    f->idx = malloc(sizeof(int) * (f->count ? f->count : 1));
    f->val = malloc(sizeof(double) * (f->count ? f->count : 1));
    if (!f->idx || !f->val) {
        free(a);
        return -1;
    }
    int k = 0;
    for (size_t p = 0; p < m; ++p)
        if (a[p] > 0.0) {
            f->idx[k] = (int)p;
            f->val[k] = a[p];
            ++k;
        }
    free(a);
    return 0;
}

typedef struct {
    int L;
    int count[32];     /* functions per level */
    basis_fn *fn[32];  /* [level][node of that level, row-major] */
} basis_set;

static void basis_set_free(basis_set *B)
{
    for (int l = 0; l < B->L; ++l) {
        if (!B->fn[l]) continue;
        for (int q = 0; q < B->count[l]; ++q) {
            free(B->fn[l][q].idx);
            free(B->fn[l][q].val);
        }
        free(B->fn[l]);
        B->fn[l] = NULL;
    }
}

static int basis_set_init(const grid_t *G, int L, basis_set *B)
{
    memset(B, 0, sizeof(*B));
    B->L = L;
    for (int l = 0; l < L; ++l) {
        B->count[l] = G[l].W * G[l].H;
        B->fn[l] = calloc((size_t)B->count[l], sizeof(basis_fn));
        if (!B->fn[l]) {
            basis_set_free(B);
            return -1;
        }
        for (int q = 0; q < B->count[l]; ++q)
            if (basis_build(G, l, q, &B->fn[l][q])) {
                basis_set_free(B);
                return -1;
            }
    }
    return 0;
}

/*
 * alpha = the point of {sum alpha = 0, alpha_i >= -m_i} nearest to a (the
 * Gibbs correction with lower bounds): start from a made to sum to zero; raise
 * every component below its bound to the bound, take the total raise equally
 * from the components not yet fixed, and repeat until none is below.  Each
 * round recomputes the free components from a with the one common shift that
 * makes the total zero, which is the same as subtracting the raises round by
 * round but keeps the sum exactly zero.
 */
static void bounded_correction(int N, const double *a, const double *m, double *alpha)
{
    unsigned char free_[ORC_MAX_N];
    for (int i = 0; i < N; ++i) free_[i] = 1;
    for (;;) {
        double s = 0.0;
        int nfree = 0;
        for (int i = 0; i < N; ++i) {
            if (free_[i]) {
                s += a[i];
                ++nfree;
            } else {
                s -= m[i];
            }
        }
        for (int i = 0; i < N; ++i) alpha[i] = free_[i] ? a[i] - s / nfree : -m[i];
        int nlow = 0;
        for (int i = 0; i < N; ++i)
            if (free_[i] && alpha[i] < -m[i]) {
                free_[i] = 0;
                ++nlow;
            }
        if (nlow == 0 || nlow == nfree) break;
    }
    for (int i = 0; i < N; ++i)
        if (alpha[i] < -m[i]) alpha[i] = -m[i];
}

/*
 * One subspace correction along basis function eta (eq. alpha, with the
 * stiffness sign and time step as read above): u <- u + alpha eta with alpha
 * minimising J(u + alpha eta) over the alpha that keep every node on its
 * simplex.  J is isotropic in alpha (curvature eta.H eta for every phase), so
 * that minimiser is the nearest feasible point to the unconstrained one
 * g / (eta.H eta), g_i = eta.(b_i - H u_i); feasibility is sum alpha = 0 and
 * u_pi + alpha_i eta_p >= 0 on the support, i.e. alpha_i >= -m_i with
 * m_i = min_p u_pi / eta_p (the bound at which the lowest value becomes
 * zero).  `scratch` is a zeroed [H*W] field, left zeroed.  Returns 1 if J
 * rose (never expected).
 */
static int ssc_update(const grid_t *g, const orc_params *P, const double *b, double *u,
                      const basis_fn *f, double *scratch)
{
    const int N = P->N;
    const size_t n = (size_t)g->W * g->H;
    double gi[ORC_MAX_N], mi[ORC_MAX_N], a[ORC_MAX_N], alpha[ORC_MAX_N];
    for (int k = 0; k < f->count; ++k) scratch[f->idx[k]] = f->val[k];
    double D = 0.0;
    for (int k = 0; k < f->count; ++k) {
        int p = f->idx[k], x = p % g->W, y = p / g->W;
        D += f->val[k] * (g->mass[p] / P->tau * f->val[k] + P->eps * stiff_apply(g, scratch, x, y));
    }
    for (int k = 0; k < f->count; ++k) scratch[f->idx[k]] = 0.0;
    for (int i = 0; i < N; ++i) {
        const double *ui = u + i * n;
        gi[i] = 0.0;
        mi[i] = INFINITY;
        for (int k = 0; k < f->count; ++k) {
            int p = f->idx[k], x = p % g->W, y = p / g->W;
            double r = b[i * n + p] - (g->mass[p] / P->tau * ui[p] + P->eps * stiff_apply(g, ui, x, y));
            gi[i] += f->val[k] * r;
            double q = ui[p] / f->val[k];
            if (q < mi[i]) mi[i] = q;
        }
        a[i] = gi[i] / D;
    }
    bounded_correction(N, a, mi, alpha);
    /* J(u + alpha eta) - J(u); alpha is the projection of g / D onto a convex
       set holding 0, so exactly it is at most -D |alpha|^2 / 2.  The slack
       covers the rounding of alpha (a few ulps of |a|) times |g|. */
    double dJ = 0.0, scale = 0.0, gs = 0.0, as = 0.0;
    for (int i = 0; i < N; ++i) {
        dJ += 0.5 * D * alpha[i] * alpha[i] - gi[i] * alpha[i];
        scale += 0.5 * D * alpha[i] * alpha[i] + fabs(gi[i] * alpha[i]);
        gs += fabs(gi[i]);
        as += fabs(a[i]) + mi[i];
        for (int k = 0; k < f->count; ++k) {
            double v = u[i * n + f->idx[k]] + alpha[i] * f->val[k];
            u[i * n + f->idx[k]] = v > 0.0 ? v : 0.0;  /* a bound met exactly may round below 0 */
        }
    }
    return dJ > 1e-10 * scale + 8.0 * N * DBL_EPSILON * gs * as;
}

/*
 * One iteration: every basis function of every level, from the coarsest level
 * to the finest, each level's nodes in row-major order.  On the finest level
 * the functions are the nodal ones, and the update is the projected block
 * Gauss-Seidel update of that node.  Returns the number of updates that
 * raised J.
 */
static int ssc_iteration(const grid_t *G, const basis_set *B, const orc_params *P, const double *b,
                         double *u, double *scratch)
{
    int bad = 0;
    for (int l = B->L - 1; l >= 0; --l)
        for (int q = 0; q < B->count[l]; ++q) bad += ssc_update(&G[0], P, b, u, &B->fn[l][q], scratch);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Public oracle entry points                                                */
/* ------------------------------------------------------------------------ */

static int hierarchy_init(const orc_params *P, grid_t *G, int *L_out)
{
    int L = P->levels > 0 ? P->levels : orc_auto_levels(P->W, P->H);
    int W = P->W, H = P->H;
    double h = P->h;
    for (int l = 0; l < L; ++l) {
        if (l > 0) {
            W = coarse_side(W);
            H = coarse_side(H);
            h *= 2.0;
        }
        if (W < 2 || H < 2) return -1;
        if (grid_init(&G[l], W, H, h)) return -1;
    }
    *L_out = L;
    return 0;
}

static void hierarchy_free(grid_t *G, int L)
{
    for (int l = 0; l < L; ++l) grid_free(&G[l]);
}

/* Assembled lumped mass [H*W] and stiffness stencils [H*W*9] of a W x H lattice. */
int orc_assemble(int W, int H, double h, double *mass, double *stiff)
{
    grid_t g;
    if (grid_init(&g, W, H, h)) return -1;
    memcpy(mass, g.mass, sizeof(double) * W * H);
    memcpy(stiff, g.stiff, sizeof(double) * W * H * 9);
    grid_free(&g);
    return 0;
}

int orc_prolong(int Wf, int Hf, int N, const double *vc, double *vf)
{
    grid_t f = {Wf, Hf, 1.0, NULL, NULL}, c = {coarse_side(Wf), coarse_side(Hf), 2.0, NULL, NULL};
    prolong(&f, &c, N, vc, vf);
    return 0;
}

int orc_restrict(int Wf, int Hf, int N, const double *vf, double *vc)
{
    grid_t f = {Wf, Hf, 1.0, NULL, NULL}, c = {coarse_side(Wf), coarse_side(Hf), 2.0, NULL, NULL};
    restrict_T(&f, &c, N, vf, vc);
    return 0;
}

int orc_colour_means(const orc_params *P, const double *I, const double *u, const double *c_prev,
                     double *c)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1;
    int e = colour_means(&g, P->N, P->C, I, u, c_prev, c);
    grid_free(&g);
    return e;
}

int orc_rhs(const orc_params *P, const double *I, const double *un, const double *c, double *b)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1;
    rhs(&g, P, I, un, c, b);
    grid_free(&g);
    return 0;
}

double orc_residual(const orc_params *P, const double *b, const double *u)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1.0;
    double r = natural_residual(&g, P, b, u);
    grid_free(&g);
    return r;
}

double orc_objective(const orc_params *P, const double *b, const double *u)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return NAN;
    double J = objective(&g, P, b, u);
    grid_free(&g);
    return J;
}

/* out = H v per component, H = M/tau + eps A on the W x H lattice of spacing h */
int orc_apply_H(const orc_params *P, const double *v, double *out)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1;
    size_t n = (size_t)P->W * P->H;
    for (int i = 0; i < P->N; ++i)
        for (int y = 0; y < P->H; ++y)
            for (int x = 0; x < P->W; ++x) {
                size_t p = (size_t)y * P->W + x;
                out[i * n + p] = g.mass[p] / P->tau * v[i * n + p] + P->eps * stiff_apply(&g, v + i * n, x, y);
            }
    grid_free(&g);
    return 0;
}

/*
 * Solve the step problem for a given right-hand side b, starting from u
 * (overwritten with the result).  Cycles are multigrid cycles when the
 * hierarchy has two or more levels, single Gauss-Seidel sweeps otherwise, or
 * with P->ssc the subspace-correction iterations over all levels; they repeat
 * until the natural residual is <= tol or max_cycles is reached.
 */
static int solve_rhs(const grid_t *G, int L, const orc_params *P, const double *b, double *u,
                     orc_stats *st)
{
    int cycles = 0, bad = 0;
    double r;
    basis_set B;
    double *scratch = NULL;
    if (P->ssc) {
        if (basis_set_init(G, L, &B)) return -1;
        scratch = calloc((size_t)G[0].W * G[0].H, sizeof(double));
        if (!scratch) {
            basis_set_free(&B);
            return -1;
        }
        /* The corrections sum to zero, so they keep every node's sum: the
           start must lie on the simplices.  A start read from float32 misses
           them by rounding; project it node by node (a no-op on the simplices). */
        size_t n = (size_t)G[0].W * G[0].H;
        double yv[ORC_MAX_N], xv[ORC_MAX_N];
        for (size_t p = 0; p < n; ++p) {
            for (int i = 0; i < P->N; ++i) yv[i] = u[i * n + p];
            orc_project(P->N, yv, xv);
            for (int i = 0; i < P->N; ++i) u[i * n + p] = xv[i];
        }
    }
    do {
        if (P->ssc)
            bad += ssc_iteration(G, &B, P, b, u, scratch);
        else if (L >= 2)
            bad += mg_cycle(G, L, P, b, u);
        else
            gs_sweep(&G[0], P, b, u);
        ++cycles;
        r = natural_residual(&G[0], P, b, u);
    } while (r > P->tol && cycles < P->max_cycles);
    if (P->ssc) {
        basis_set_free(&B);
        free(scratch);
    }
    if (st) {
        st->cycles = cycles;
        st->converged = r <= P->tol;
        st->nonmonotone = bad;
        st->residual = r;
        st->objective = objective(&G[0], P, b, u);
    }
    return 0;
}

/* Solve the step problem for a caller-supplied b (u: initial iterate in, result out). */
int orc_solve_qp(const orc_params *P, const double *b, double *u, orc_stats *st)
{
    grid_t G[32];
    int L;
    if (hierarchy_init(P, G, &L)) return -1;
    int e = solve_rhs(G, L, P, b, u, st);
    hierarchy_free(G, L);
    return e;
}

/*
 * One time step: c = colour means of un (c_prev for empty phases), b from un
 * and c, then u_out = argmin J over the simplices, starting from un.
 * c_out receives the means used in this step.  Returns 0, or -1 on bad input.
 */
int orc_step(const orc_params *P, const double *I, const double *un, const double *c_prev,
             double *u_out, double *c_out, orc_stats *st)
{
    grid_t G[32];
    int L;
    if (hierarchy_init(P, G, &L)) return -1;
    size_t n = (size_t)P->W * P->H;
    double *b = malloc(sizeof(double) * P->N * n);
    int empty = colour_means(&G[0], P->N, P->C, I, un, c_prev, c_out);
    rhs(&G[0], P, I, un, c_out, b);
    memcpy(u_out, un, sizeof(double) * P->N * n);
    solve_rhs(G, L, P, b, u_out, st);
    if (st) st->empty_phase = empty;
    free(b);
    hierarchy_free(G, L);
    return 0;
}

/*
 * `steps` time steps from u0.  traj (optional) receives u^0..u^steps
 * ([steps+1][N][H*W]), c_traj (optional) the means used in each step
 * ([steps][N][C]), stats (optional) one record per step.  u_out gets u^steps.
 */
int orc_solve(const orc_params *P, int steps, const double *I, const double *u0, double *u_out,
              double *traj, double *c_traj, orc_stats *stats)
{
    grid_t G[32];
    int L;
    if (hierarchy_init(P, G, &L)) return -1;
    size_t n = (size_t)P->W * P->H, nu = (size_t)P->N * n;
    double *b = malloc(sizeof(double) * nu);
    double *cur = malloc(sizeof(double) * nu);
    double *nxt = malloc(sizeof(double) * nu);
    double *c = malloc(sizeof(double) * P->N * P->C);
    double *cp = malloc(sizeof(double) * P->N * P->C);
    memcpy(cur, u0, sizeof(double) * nu);
    if (traj) memcpy(traj, u0, sizeof(double) * nu);
    for (int s = 0; s < steps; ++s) {
        int empty = colour_means(&G[0], P->N, P->C, I, cur, s > 0 ? cp : NULL, c);
        rhs(&G[0], P, I, cur, c, b);
        memcpy(nxt, cur, sizeof(double) * nu);
        orc_stats st;
        solve_rhs(G, L, P, b, nxt, &st);
        st.empty_phase = empty;
        if (stats) stats[s] = st;
        if (c_traj) memcpy(c_traj + (size_t)s * P->N * P->C, c, sizeof(double) * P->N * P->C);
        if (traj) memcpy(traj + (size_t)(s + 1) * nu, nxt, sizeof(double) * nu);
        memcpy(cp, c, sizeof(double) * P->N * P->C);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(u_out, cur, sizeof(double) * nu);
    free(b);
    free(cur);
    free(nxt);
    free(c);
    free(cp);
    hierarchy_free(G, L);
    return 0;
}

/*
 * As orc_solve, with the colour means fixed to c_fixed ([N][C]) in every step
 * instead of recomputed from u^n.
 */
int orc_solve_c(const orc_params *P, int steps, const double *I, const double *u0,
                const double *c_fixed, double *u_out, double *traj, orc_stats *stats)
{
    grid_t G[32];
    int L;
    if (hierarchy_init(P, G, &L)) return -1;
    size_t n = (size_t)P->W * P->H, nu = (size_t)P->N * n;
    double *b = malloc(sizeof(double) * nu);
    double *cur = malloc(sizeof(double) * nu);
    double *nxt = malloc(sizeof(double) * nu);
    memcpy(cur, u0, sizeof(double) * nu);
    if (traj) memcpy(traj, u0, sizeof(double) * nu);
    for (int s = 0; s < steps; ++s) {
        rhs(&G[0], P, I, cur, c_fixed, b);
        memcpy(nxt, cur, sizeof(double) * nu);
        orc_stats st;
        solve_rhs(G, L, P, b, nxt, &st);
        st.empty_phase = 0;
        if (stats) stats[s] = st;
        if (traj) memcpy(traj + (size_t)(s + 1) * nu, nxt, sizeof(double) * nu);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(u_out, cur, sizeof(double) * nu);
    free(b);
    free(cur);
    free(nxt);
    hierarchy_free(G, L);
    return 0;
}

/*
 * Discrete energy of eq. E on the P1 space with the lumped mass:
 *   parts[0] = eps/2 sum_i u_i.A u_i                       (interface)
 *   parts[1] = 1/eps sum_i sum_p M_p u_pi (1 - u_pi)         (concave potential)
 *   parts[2] = lambda sum_i sum_p M_p u_pi F_pi(c(u))        (fitting)
 * with c(u) the colour means of u itself (c_prev for an empty phase).
 * Returns the total.
 */
double orc_energy(const orc_params *P, const double *I, const double *u, const double *c_prev,
                  double *parts)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return NAN;
    size_t n = (size_t)P->W * P->H;
    double *c = malloc(sizeof(double) * P->N * P->C);
    colour_means(&g, P->N, P->C, I, u, c_prev, c);
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int i = 0; i < P->N; ++i)
        for (int y = 0; y < P->H; ++y)
            for (int x = 0; x < P->W; ++x) {
                size_t p = (size_t)y * P->W + x;
                double v = u[i * n + p];
                e0 += 0.5 * P->eps * v * stiff_apply(&g, u + i * n, x, y);
                e1 += g.mass[p] * v * (1.0 - v) / P->eps;
                e2 += P->lambda * g.mass[p] * v * fitting(P->C, I, n, p, c + i * P->C);
            }
    if (parts) {
        parts[0] = e0;
        parts[1] = e1;
        parts[2] = e2;
    }
    free(c);
    grid_free(&g);
    return e0 + e1 + e2;
}

/*
 * Post-processing: label_p = the phase with the largest u_pi (lowest index on
 * ties); composite_kp = sum_i c_ik u_pi; rounded composite_kp = c_{label_p,k}.
 * composite / rounded may be NULL.
 */
void orc_labels(int N, int C, int H, int W, const double *u, const double *c, uint8_t *labels,
                double *composite, double *rounded)
{
    size_t n = (size_t)W * H;
    for (size_t p = 0; p < n; ++p) {
        int best = 0;
        for (int i = 1; i < N; ++i)
            if (u[i * n + p] > u[best * n + p]) best = i;
        labels[p] = (uint8_t)best;
        for (int k = 0; k < C; ++k) {
            if (composite) {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s += c[i * C + k] * u[i * n + p];
                composite[k * n + p] = s;
            }
            if (rounded) rounded[k * n + p] = c[best * C + k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the time step (derived; the paper does not differentiate)      */
/* ------------------------------------------------------------------------ */

/*
 * Derivative of the step map.  With the free sets I_p = {i : u^{n+1}_pi > 0}
 * held fixed, u^{n+1} minimises J(u) = sum_i [u_i.H u_i / 2 - b_i.u_i] over
 * the affine set {u_pi = 0 for i outside I_p, sum_{i in I_p} u_pi = 1}, so a
 * change db moves it by du = T (T H T)^+ T db, where T applies tangent_free
 * node by node (H is symmetric).  For a loss with gradient ubar at u^{n+1},
 * the gradient at b is therefore z = (T H T)^+ T ubar (z = T z): solved here
 * by conjugate gradients on the range of T.  Components with u = 0 count as
 * active whatever their multiplier.
 *
 * The rest is the chain rule through eq. alpha and eq. VV_fidelity:
 *   b_pi = M_p [(1/tau + 2/eps) un_pi - lambda F_pi],
 *   F_pi = sum_k (I_pk - c_ik)^2,  c_ik = S_ik / S_i,
 *   S_ik = sum_p M_p un_pi I_pk,   S_i = sum_p M_p un_pi,
 *   H = M/tau + eps A.
 * An empty phase's mean is the kept previous mean: treated as a constant.
 */

/* out = T(v) node by node, the free sets taken from u */
static void tangent_field(size_t n, int N, const double *u, const double *v, double *out)
{
    double up[ORC_MAX_N], xi[ORC_MAX_N], xo[ORC_MAX_N];
    for (size_t p = 0; p < n; ++p) {
        for (int i = 0; i < N; ++i) {
            up[i] = u[i * n + p];
            xi[i] = v[i * n + p];
        }
        tangent_free(N, up, xi, xo);
        for (int i = 0; i < N; ++i) out[i * n + p] = xo[i];
    }
}

/* out = H v, componentwise */
static void apply_H_field(const grid_t *g, const orc_params *P, const double *v, double *out)
{
    size_t n = (size_t)g->W * g->H;
    for (int i = 0; i < P->N; ++i)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                size_t p = (size_t)y * g->W + x;
                out[i * n + p] = g->mass[p] / P->tau * v[i * n + p] + P->eps * stiff_apply(g, v + i * n, x, y);
            }
}

static double dotn(size_t m, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t k = 0; k < m; ++k) s += a[k] * b[k];
    return s;
}

/* z = (T H T)^+ T rhs by conjugate gradients; returns the iteration count */
static int adjoint_solve(const grid_t *g, const orc_params *P, const double *unext, const double *rv,
                         double *z, double rtol)
{
    size_t n = (size_t)g->W * g->H, m = (size_t)P->N * n;
    double *r = malloc(sizeof(double) * m), *d = malloc(sizeof(double) * m);
    double *q = malloc(sizeof(double) * m), *t = malloc(sizeof(double) * m);
    memset(z, 0, sizeof(double) * m);
    tangent_field(n, P->N, unext, rv, r);
    memcpy(d, r, sizeof(double) * m);
    double rr = dotn(m, r, r), r0 = sqrt(rr);
    int it = 0;
    while (sqrt(rr) > rtol * r0 && rr > 0.0 && it < 100000) {
        apply_H_field(g, P, d, t);
        tangent_field(n, P->N, unext, t, q);
        double a = rr / dotn(m, d, q);
        for (size_t k = 0; k < m; ++k) {
            z[k] += a * d[k];
            r[k] -= a * q[k];
        }
        double rr1 = dotn(m, r, r);
        double beta = rr1 / rr;
        rr = rr1;
        for (size_t k = 0; k < m; ++k) d[k] = r[k] + beta * d[k];
        ++it;
    }
    free(r);
    free(d);
    free(q);
    free(t);
    return it;
}

/*
 * One step backwards.  Inputs: un = u^n, unext = u^{n+1} (the converged
 * step), c_prev (the previous step's means, for empty phases; may be NULL),
 * ubar_next = dL/du^{n+1}.  Outputs: ubar_n = dL/du^n through this step,
 * z (optional, the gradient at b), cbar = dL/dc^n [N][C]; accumulated:
 * Ibar += dL/dI, grads[0..2] += dL/dlambda, dL/deps (tau fixed), dL/dtau.
 */
static int adjoint_step(const grid_t *g, const orc_params *P, const double *I, const double *un,
                        const double *c_prev, const double *c_fixed, const double *unext,
                        const double *ubar_next, double *ubar_n, double *Ibar, double *grads,
                        double *cbar, double *z_out)
{
    const int N = P->N, C = P->C;
    size_t n = (size_t)g->W * g->H, m = (size_t)N * n;
    double c[ORC_MAX_N * 4];
    double S[ORC_MAX_N];
    unsigned char nonempty[ORC_MAX_N];
    if (C > 4) return -1;
    if (c_fixed)
        memcpy(c, c_fixed, sizeof(double) * N * C);
    else
        colour_means(g, N, C, I, un, c_prev, c);
    double area = 0.0;
    for (size_t p = 0; p < n; ++p) area += g->mass[p];
    for (int i = 0; i < N; ++i) {
        S[i] = 0.0;
        for (size_t p = 0; p < n; ++p) S[i] += g->mass[p] * un[i * n + p];
        nonempty[i] = !c_fixed && S[i] > 1e-12 * area;  /* fixed means depend on nothing */
    }
    double *z = malloc(sizeof(double) * m);
    adjoint_solve(g, P, unext, ubar_next, z, 1e-14);
    if (z_out) memcpy(z_out, z, sizeof(double) * m);

    const double a = 1.0 / P->tau + 2.0 / P->eps;
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < C; ++k) cbar[i * C + k] = 0.0;
    double gl = 0.0, ge = 0.0, gt = 0.0;
    for (int i = 0; i < N; ++i)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                size_t p = (size_t)y * g->W + x;
                double zp = z[i * n + p], Mp = g->mass[p];
                double F = fitting(C, I, n, p, c + i * C);
                /* db/du^n */
                ubar_n[i * n + p] = a * Mp * zp;
                /* b depends on lambda, eps, tau; H on eps, tau */
                gl += zp * (-Mp * F);
                ge += zp * (-2.0 / (P->eps * P->eps)) * Mp * un[i * n + p]
                      - zp * stiff_apply(g, unext + i * n, x, y);
                gt += -zp * Mp * un[i * n + p] / (P->tau * P->tau)
                      + zp * Mp * unext[i * n + p] / (P->tau * P->tau);
                /* F: direct image term and the means */
                double Fbar = -P->lambda * Mp * zp;
                for (int k = 0; k < C; ++k) {
                    double d = I[k * n + p] - c[i * C + k];
                    Ibar[k * n + p] += 2.0 * Fbar * d;
                    cbar[i * C + k] += -2.0 * Fbar * d;
                }
            }
    /* c_ik = S_ik / S_i */
    for (int i = 0; i < N; ++i) {
        if (!nonempty[i]) continue;
        for (size_t p = 0; p < n; ++p) {
            double Mp = g->mass[p];
            for (int k = 0; k < C; ++k) {
                Ibar[k * n + p] += cbar[i * C + k] * Mp * un[i * n + p] / S[i];
                ubar_n[i * n + p] += cbar[i * C + k] * Mp * (I[k * n + p] - c[i * C + k]) / S[i];
            }
        }
    }
    grads[0] += gl;
    grads[1] += ge;
    grads[2] += gt;
    free(z);
    return 0;
}

int orc_backward_c(const orc_params *P, int steps, const double *I, const double *traj,
                   const double *c_fixed, const double *ubar_T, double *Ibar, double *grads,
                   double *cbar, double *ubar0);

/* The gradient at b of one step: z = (T H T)^+ T ubar, free sets from unext. */
int orc_adjoint_solve(const orc_params *P, const double *unext, const double *ubar, double *z)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1;
    int it = adjoint_solve(&g, P, unext, ubar, z, 1e-14);
    grid_free(&g);
    return it;
}

int orc_adjoint_step(const orc_params *P, const double *I, const double *un, const double *c_prev,
                     const double *unext, const double *ubar_next, double *ubar_n, double *Ibar,
                     double *grads, double *cbar)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1;
    int r = adjoint_step(&g, P, I, un, c_prev, NULL, unext, ubar_next, ubar_n, Ibar, grads, cbar, NULL);
    grid_free(&g);
    return r;
}

/*
 * Backwards through `steps` steps of a trajectory traj = u^0..u^steps
 * ([steps+1][N][H*W]) for dL/du^steps = ubar_T.  Ibar [C][H*W] and
 * grads[3] (lambda, eps at fixed tau, tau) are overwritten; cbar
 * ([steps][N][C], optional) receives dL/dc^n of every step; ubar0
 * (optional) dL/du^0.  The means are recomputed from the trajectory.
 */
int orc_backward(const orc_params *P, int steps, const double *I, const double *traj,
                 const double *ubar_T, double *Ibar, double *grads, double *cbar, double *ubar0)
{
    return orc_backward_c(P, steps, I, traj, NULL, ubar_T, Ibar, grads, cbar, ubar0);
}

/*
 * As orc_backward; with c_fixed ([N][C], non-NULL) every step used those
 * means (no colour-mean update), and cbar ([N][C]) receives dL/dc_fixed,
 * the sum over the steps.
 */
int orc_backward_c(const orc_params *P, int steps, const double *I, const double *traj,
                   const double *c_fixed, const double *ubar_T, double *Ibar, double *grads,
                   double *cbar, double *ubar0)
{
    grid_t g;
    if (grid_init(&g, P->W, P->H, P->h)) return -1;
    const int N = P->N, C = P->C;
    size_t n = (size_t)P->W * P->H, m = (size_t)N * n;
    double *cs = malloc(sizeof(double) * (size_t)(steps > 0 ? steps : 1) * N * C);
    for (int s = 0; s < steps; ++s)
        colour_means(&g, N, C, I, traj + (size_t)s * m, s > 0 ? cs + (size_t)(s - 1) * N * C : NULL,
                     cs + (size_t)s * N * C);
    double *ub = malloc(sizeof(double) * m), *ub2 = malloc(sizeof(double) * m);
    double cb[ORC_MAX_N * 4];
    memcpy(ub, ubar_T, sizeof(double) * m);
    memset(Ibar, 0, sizeof(double) * C * n);
    grads[0] = grads[1] = grads[2] = 0.0;
    int r = 0;
    if (c_fixed && cbar) memset(cbar, 0, sizeof(double) * N * C);
    for (int s = steps - 1; s >= 0 && r == 0; --s) {
        r = adjoint_step(&g, P, I, traj + (size_t)s * m, s > 0 ? cs + (size_t)(s - 1) * N * C : NULL,
                         c_fixed, traj + (size_t)(s + 1) * m, ub, ub2, Ibar, grads, cb, NULL);
        if (cbar && c_fixed)
            for (int q = 0; q < N * C; ++q) cbar[q] += cb[q];
        else if (cbar)
            memcpy(cbar + (size_t)s * N * C, cb, sizeof(double) * N * C);
        double *t = ub;
        ub = ub2;
        ub2 = t;
    }
    if (ubar0) memcpy(ubar0, ub, sizeof(double) * m);
    free(cs);
    free(ub);
    free(ub2);
    grid_free(&g);
    return r;
}

/*
 * The basis function of node q of level l seen on the finest lattice, written
 * densely into eta ([H*W] of the finest lattice).  Returns 0, or -1.
 */
int orc_basis(const orc_params *P, int l, int q, double *eta)
{
    grid_t G[32];
    int L;
    if (hierarchy_init(P, G, &L)) return -1;
    int e = -1;
    if (l >= 0 && l < L && q >= 0 && q < G[l].W * G[l].H) {
        basis_fn f;
        if (!basis_build(G, l, q, &f)) {
            memset(eta, 0, sizeof(double) * P->W * P->H);
            for (int k = 0; k < f.count; ++k) eta[f.idx[k]] = f.val[k];
            free(f.idx);
            free(f.val);
            e = 0;
        }
    }
    hierarchy_free(G, L);
    return e;
}

/*
 * One subspace correction of u ([N][H*W], in place) along the basis function
 * of node q of level l, for the step problem with right-hand side b.
 * Returns 0, 1 if J rose, or -1.
 */
int orc_ssc_update(const orc_params *P, int l, int q, const double *b, double *u)
{
    grid_t G[32];
    int L;
    if (hierarchy_init(P, G, &L)) return -1;
    int e = -1;
    double *scratch = calloc((size_t)P->W * P->H, sizeof(double));
    if (scratch && l >= 0 && l < L && q >= 0 && q < G[l].W * G[l].H) {
        basis_fn f;
        if (!basis_build(G, l, q, &f)) {
            e = ssc_update(&G[0], P, b, u, &f, scratch);
            free(f.idx);
            free(f.val);
        }
    }
    free(scratch);
    hierarchy_free(G, L);
    return e;
}
