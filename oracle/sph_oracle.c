/*
 * FP64 CPU oracle for the semi-implicit SPH viscous solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code.  It shares no source with the
 * HIP library: it is a plain, slow, directly readable transcription of what
 * the paper defines, compiled with contraction off (-ffp-contract=off) so
 * every product is rounded on its own, as the paper's appendix on symmetry
 * pitfalls (fused multiply-add) requires.
 *
 * Contents, each citing the passage it follows:
 *   - Wendland psi_{3,1} kernel w(q), f(q) and the truncated Gaussian (k = 3)
 *                                                 Section "Smoothing kernel choice"
 *   - neighbour sets: brute force and a cell grid Section "Smoothing kernel choice"
 *                                                 (support radius 2h), appendix on
 *                                                 relative positions (minimum image)
 *   - the viscous matrix A(dt), matrix-free and dense
 *                                                 eqs. kab, implicit-system-base, diag,
 *                                                 offdiag, implicit-system-dummy-full
 *   - the same matrix assembled on the neighbour pattern (stored entries,
 *     for solves of systems of millions of rows) eqs. diag, offdiag,
 *                                                 implicit-system-dummy-full
 *   - Jacobi scaling                              appendix "Implementation notes"
 *   - Kahan's compensated FP32 sums and inner products (the paper's
 *     single-precision arithmetic)                appendix "Implementation notes"
 *   - robust (restructured) BiCGSTAB and the textbook BiCGSTAB, three systems
 *     sharing one matrix, with the three-state stopping rule; the loop is
 *     organised in the phases direction update, first half-step, second
 *     half-step, close-out; FP64 inner products are summed in fixed blocks
 *     (the same result for any thread count)
 *                                                 Section "Restructuring the stabilized
 *                                                 biconjugate gradient method"
 *   - the rotated Conjugate Gradient for the symmetric case (dynamic walls,
 *     uniform mass)                               Section "Restructuring the Conjugate
 *                                                 Gradient", Section "Linear system
 *                                                 properties and resolution"
 *   - the Papanastasiou viscosity from the velocity field: velocity gradient,
 *     shear rate, its second invariant and the regularised yield term with
 *     its truncated Maclaurin branch              Section "Non-Newtonian viscosity",
 *                                                 eq. papa
 *
 * Readings of passages that are ambiguous or inconsistent in the paper:
 *   - Sign of K (eq. kab): the Wendland F is <= 0, so the printed K would be
 *     >= 0 and the printed diagonal 1 - dt sum K could not be strictly
 *     diagonally dominant, contradicting the paper's own claim.  We take the
 *     physically diffusive reading: pair weight w = -2 mubar m_a F/(rho_a rho_b)
 *     >= 0, A_bb = 1 + dt sum w, A_ba = -dt w (i.e. K = -w in eqs. diag/offdiag).
 *   - tau^2 floor: "lower bound" -> tau^2 = max(eps^2 b.b, floor).
 *   - gamma_1 = r0.r0 for the first iteration of the robust variant.
 *   - a zero or non-finite delta, omega or gamma' marks the component stalled
 *     and zeroes the dependent coefficients; the iteration still completes.
 *   - converged components keep iterating while any component progresses;
 *     "converged" takes precedence over "stalled" in the state.
 *   - convergence is checked before the first iteration (0 iterations when
 *     every component already meets its threshold).
 *   - true residual: every `true_res_period` iterations and whenever no
 *     component is progressing, r_true = b - A x is recomputed; a component
 *     marked converged whose true residual fails the threshold is restarted
 *     from r_true (r0hat = r_true, alpha' = beta = 0) and made progressing;
 *     after three such restarts it is reported stalled instead.  Optionally
 *     (restart_drop > 0) a progressing component whose true r.r at a periodic
 *     check has fallen below restart_drop times its r.r at the last (re)start
 *     restarts the same way.
 *   - textbook variant: when the half-step residual s already meets the
 *     threshold the component takes omega = 0 (x = x + alpha p, r = s).
 *   - CG with the Jacobi scaling: the paper divides the system by its
 *     diagonal for both solvers.  D^-1 A is not symmetric, but it is
 *     self-adjoint in the inner product <u, v>_D = sum_i D_i u_i v_i when A
 *     is symmetric, so the CG takes its inner products in that product
 *     (Jacobi-preconditioned CG written for the scaled system); without
 *     scaling D = 1 and it is the printed rotated CG.  The stopping rule
 *     uses the Euclidean r.r of the scaled residual, as the BiCGSTAB does.
 *   - CG and the wall rows: with dynamic walls A is symmetric only on the
 *     fluid rows (fluid rows see wall columns, wall rows are identity), so
 *     the start takes the exact value b on every wall row; the wall entries
 *     of r and p then stay zero and the iteration runs on the symmetric
 *     fluid block, the paper's reduced system.  Dummy walls break the
 *     symmetry for good: the CG refuses them.
 *   - CG stall: alpha = 0 in finite precision (or a zero or non-finite
 *     p.Ap) while r.r is above the threshold marks the component stalled;
 *     the iteration completes (a no-op update) and beta is taken as 0.
 *   - velocity gradient: the printed sum, with r_ab = r_a - r_b and
 *     u_ab = u_a - u_b over all neighbours a of b (fluid and wall, with the
 *     velocities given for them), is minus the usual SPH gradient (F <= 0);
 *     only its symmetric part enters D quadratically, so the sign does not
 *     matter and the printed form is kept.
 *   - second invariant: D = sqrt(2 S:S) with S the symmetric part, the norm
 *     that equals the shear rate in simple shear (u = (G y, 0, 0) gives D = G
 *     in the continuum), as the yield law needs.
 *   - Maclaurin threshold: the printed switch "D >= m" cannot be meant (for
 *     m = 1000 the 8-term series would run at m D up to 1e6); the branch is
 *     taken for x = m D below x0 = (9! 2^-23)^(1/8) = 0.675..., where the
 *     first omitted term x^8/9! equals single-precision epsilon, the
 *     accuracy the paper states for its choice.
 *   - wall particles keep their given viscosity; only fluid rows are updated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FLUID 0
#define ORC_WALL 1
#define ORC_WALL_DYNAMIC 0
#define ORC_WALL_DUMMY 1
#define ORC_AVG_ARITH 0
#define ORC_AVG_HARMONIC 1

#define ORC_CONVERGED 0
#define ORC_STALLED 1
#define ORC_PROGRESSING 2

#define ORC_OK 0
#define ORC_STATUS_STALLED 1
#define ORC_NOT_CONVERGED 2
#define ORC_E_ARG (-1)
#define ORC_E_NONFINITE (-5)

/* loops over particles run in parallel only from this length on (small systems
 * would spend more on the thread team than on the loop) */
#define ORC_PAR_MIN 65536

static const double ORC_PI = 3.14159265358979323846;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Wendland psi_{3,1} kernel, radius 2 (Section "Smoothing kernel choice"):   */
/*   W(r,h) = w(r/h)/h^3,  w(q) = 21/(16 pi) (1 - q/2)^4 (2q + 1),  q <= 2     */
/*   F(r,h) = f(r/h)/h^5,  f(q) = 105/(128 pi) (q - 2)^3,           q <= 2     */
/* with F = (1/r) dW/dr (Section "Spatial discretization").                  */
/* ------------------------------------------------------------------------ */
double orc_wendland_w(double q) {
    if (!(q < 2.0)) return 0.0;
    double a = 1.0 - 0.5 * q;
    return 21.0 / (16.0 * ORC_PI) * (a * a * a * a) * (2.0 * q + 1.0);
}

double orc_wendland_f(double q) {
    if (!(q < 2.0)) return 0.0;
    double a = q - 2.0;
    return 105.0 / (128.0 * ORC_PI) * (a * a * a);
}

/* ------------------------------------------------------------------------ */
/* Normalised truncated Gaussian of radius k = 3 (Section "Smoothing kernel  */
/* choice"):  w(q) = (e^{-q^2} - e^{-k^2}) / w_G for q < k, with            */
/*   w_G = pi^{3/2} erf(k) - (2 pi/3) e^{-k^2} k (3 + 2 k^2),               */
/* and f(q) = w'(q)/q = -2 e^{-q^2} / w_G for q < k (the printed f has the  */
/* opposite sign; F = (1/r) dW/dr is kept, as for the Wendland kernel).     */
/* ------------------------------------------------------------------------ */
#define ORC_GAUSS_K 3.0
static double orc_gauss_norm(void) {
    const double k = ORC_GAUSS_K;
    return pow(ORC_PI, 1.5) * erf(k) - 2.0 * ORC_PI / 3.0 * exp(-k * k) * k * (3.0 + 2.0 * k * k);
}

double orc_gauss_w(double q) {
    if (!(q < ORC_GAUSS_K)) return 0.0;
    return (exp(-q * q) - exp(-ORC_GAUSS_K * ORC_GAUSS_K)) / orc_gauss_norm();
}

double orc_gauss_f(double q) {
    if (!(q < ORC_GAUSS_K)) return 0.0;
    return -2.0 * exp(-q * q) / orc_gauss_norm();
}

/* Displacement r_i - r_j on one axis, minimum image when the axis is periodic. */
static double orc_disp(double xi, double xj, double period) {
    double d = xi - xj;
    if (period > 0.0) {
        double k = nearbyint(d / period);
        d = d - period * k;
    }
    return d;
}

/* Squared distance, summed as (dx^2 + dy^2) + dz^2. */
static double orc_dist2(const double *x, const double *y, const double *z, int64_t i, int64_t j,
                        const double period[3], double *dx, double *dy, double *dz) {
    double a = orc_disp(x[i], x[j], period[0]);
    double b = orc_disp(y[i], y[j], period[1]);
    double c = orc_disp(z[i], z[j], period[2]);
    if (dx) { *dx = a; *dy = b; *dz = c; }
    return (a * a + b * b) + c * c;
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets N(i) = { j != i : |r_i - r_j|^2 < s^2 }, s the kernel's     */
/* support radius (2h Wendland, 3h Gaussian).                                 */
/* CSR by row, columns ascending.  Returns total nnz; cols is written only     */
/* up to `cap` entries (the caller re-calls with enough room).                */
/* ------------------------------------------------------------------------ */
int64_t orc_neighbors_brute(int64_t n, const double *x, const double *y, const double *z,
                            const double *period, double s, int64_t *row_ptr, int32_t *cols,
                            int64_t cap) {
    double cut2 = s * s;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && orc_dist2(x, y, z, i, j, period, 0, 0, 0) < cut2) ++c;
        cnt[i] = c;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t nnz = row_ptr[n];
    if (nnz <= cap) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t k = row_ptr[i];
            for (int64_t j = 0; j < n; ++j)
                if (j != i && orc_dist2(x, y, z, i, j, period, 0, 0, 0) < cut2) cols[k++] = (int32_t)j;
        }
    }
    free(cnt);
    return nnz;
}

static int orc_cmp_i32(const void *a, const void *b) {
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* Cell-grid search: particles are binned into cells no smaller than 2h along
 * each axis (the bounding box of the data on non-periodic axes, the period on
 * periodic ones); each particle tests the particles of the (deduplicated)
 * 3x3x3 block of cells around its own.  Same predicate as the brute force. */
typedef struct {
    int nc[3];
    double org[3], cs[3];
    int64_t *start; /* [ncell + 1] */
    int64_t *items; /* particle ids grouped by cell, ascending inside a cell */
    int32_t *cell_of;
} orc_grid;

static int orc_cell_axis(double v, double org, double cs, int nc, int periodic) {
    double u = floor((v - org) / cs);
    long c = (long)u;
    if (periodic) {
        c %= nc;
        if (c < 0) c += nc;
    } else {
        if (c < 0) c = 0;
        if (c >= nc) c = nc - 1;
    }
    return (int)c;
}

static void orc_grid_build(orc_grid *g, int64_t n, const double *x, const double *y,
                           const double *z, const double *lo, const double *period, double s) {
    const double *p[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        double ext;
        if (period[a] > 0.0) {
            g->org[a] = lo[a];
            ext = period[a];
        } else {
            double mn = p[a][0], mx = p[a][0];
            for (int64_t i = 1; i < n; ++i) {
                if (p[a][i] < mn) mn = p[a][i];
                if (p[a][i] > mx) mx = p[a][i];
            }
            g->org[a] = mn;
            ext = mx - mn;
        }
        int nc = (int)floor(ext / s);
        if (nc < 1) nc = 1;
        if (period[a] <= 0.0 && ext <= 0.0) ext = 1.0;
        g->nc[a] = nc;
        g->cs[a] = ext / nc;
        if (period[a] <= 0.0 && nc == 1) g->cs[a] = ext > 0.0 ? ext * 2.0 : 1.0;
    }
    int64_t ncell = (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    g->cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int c0 = orc_cell_axis(x[i], g->org[0], g->cs[0], g->nc[0], period[0] > 0.0);
        int c1 = orc_cell_axis(y[i], g->org[1], g->cs[1], g->nc[1], period[1] > 0.0);
        int c2 = orc_cell_axis(z[i], g->org[2], g->cs[2], g->nc[2], period[2] > 0.0);
        int64_t c = ((int64_t)c2 * g->nc[1] + c1) * g->nc[0] + c0;
        g->cell_of[i] = (int32_t)c;
        g->start[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) { /* ascending i => ascending inside each cell */
        int64_t c = g->cell_of[i];
        g->items[g->start[c] + fill[c]++] = i;
    }
    free(fill);
}

static void orc_grid_free(orc_grid *g) {
    free(g->start);
    free(g->items);
    free(g->cell_of);
}

/* Distinct neighbour cells of cell c (at most 27). */
static int orc_grid_stencil(const orc_grid *g, int64_t c, const double *period, int64_t *out) {
    int cc[3];
    cc[0] = (int)(c % g->nc[0]);
    cc[1] = (int)((c / g->nc[0]) % g->nc[1]);
    cc[2] = (int)(c / ((int64_t)g->nc[0] * g->nc[1]));
    int m = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int d[3] = {dx, dy, dz}, q[3], ok = 1;
                for (int a = 0; a < 3; ++a) {
                    q[a] = cc[a] + d[a];
                    if (period[a] > 0.0) {
                        q[a] %= g->nc[a];
                        if (q[a] < 0) q[a] += g->nc[a];
                    } else if (q[a] < 0 || q[a] >= g->nc[a]) {
                        ok = 0;
                    }
                }
                if (!ok) continue;
                int64_t id = ((int64_t)q[2] * g->nc[1] + q[1]) * g->nc[0] + q[0];
                int dup = 0;
                for (int k = 0; k < m; ++k) dup |= (out[k] == id);
                if (!dup) out[m++] = id;
            }
    return m;
}

int64_t orc_neighbors_grid(int64_t n, const double *x, const double *y, const double *z,
                           const double *lo, const double *period, double s, int64_t *row_ptr,
                           int32_t *cols, int64_t cap) {
    orc_grid g;
    orc_grid_build(&g, n, x, y, z, lo, period, s);
    double cut2 = s * s;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t st[27];
        int m = orc_grid_stencil(&g, g.cell_of[i], period, st);
        int64_t c = 0;
        for (int k = 0; k < m; ++k)
            for (int64_t t = g.start[st[k]]; t < g.start[st[k] + 1]; ++t) {
                int64_t j = g.items[t];
                if (j != i && orc_dist2(x, y, z, i, j, period, 0, 0, 0) < cut2) ++c;
            }
        cnt[i] = c;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t nnz = row_ptr[n];
    if (nnz <= cap) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t st[27];
            int m = orc_grid_stencil(&g, g.cell_of[i], period, st);
            int64_t k0 = row_ptr[i], k = k0;
            for (int q = 0; q < m; ++q)
                for (int64_t t = g.start[st[q]]; t < g.start[st[q] + 1]; ++t) {
                    int64_t j = g.items[t];
                    if (j != i && orc_dist2(x, y, z, i, j, period, 0, 0, 0) < cut2) cols[k++] = (int32_t)j;
                }
            qsort(cols + k0, (size_t)(k - k0), sizeof(int32_t), orc_cmp_i32);
        }
    }
    free(cnt);
    orc_grid_free(&g);
    return nnz;
}

/* Neighbour lists of the listed rows only (every other row gets an empty
 * list): the cell-grid search and predicate of orc_neighbors_grid, for checks
 * of single rows of systems too large for full lists.  rows[] ascending and
 * distinct, each in [0, n); row_ptr has n + 1 entries. */
int64_t orc_neighbors_grid_rows(int64_t n, const double *x, const double *y, const double *z,
                                const double *lo, const double *period, double s,
                                const int64_t *rows, int64_t nrows, int64_t *row_ptr,
                                int32_t *cols, int64_t cap) {
    orc_grid g;
    orc_grid_build(&g, n, x, y, z, lo, period, s);
    double cut2 = s * s;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        int64_t st[27];
        int m = orc_grid_stencil(&g, g.cell_of[i], period, st);
        int64_t c = 0;
        for (int q = 0; q < m; ++q)
            for (int64_t t = g.start[st[q]]; t < g.start[st[q] + 1]; ++t) {
                int64_t j = g.items[t];
                if (j != i && orc_dist2(x, y, z, i, j, period, 0, 0, 0) < cut2) ++c;
            }
        cnt[i] = c;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t nnz = row_ptr[n];
    if (nnz <= cap) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < nrows; ++k) {
            int64_t i = rows[k];
            int64_t st[27];
            int m = orc_grid_stencil(&g, g.cell_of[i], period, st);
            int64_t k0 = row_ptr[i], kk = k0;
            for (int q = 0; q < m; ++q)
                for (int64_t t = g.start[st[q]]; t < g.start[st[q] + 1]; ++t) {
                    int64_t j = g.items[t];
                    if (j != i && orc_dist2(x, y, z, i, j, period, 0, 0, 0) < cut2) cols[kk++] = (int32_t)j;
                }
            qsort(cols + k0, (size_t)(kk - k0), sizeof(int32_t), orc_cmp_i32);
        }
    }
    free(cnt);
    orc_grid_free(&g);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* The viscous matrix A(dt) (Section "From explicit to semi-implicit").       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *cols;
    const double *x, *y, *z;
    double period[3];
    double h;
    const double *mass, *rho, *mu;
    const uint8_t *type;
    double dt;
    int32_t wall;   /* ORC_WALL_DYNAMIC / ORC_WALL_DUMMY */
    int32_t avg;    /* ORC_AVG_ARITH / ORC_AVG_HARMONIC */
    int32_t jacobi; /* 1: rows scaled by 1/A_bb (appendix "Implementation notes") */
    int32_t kernel; /* ORC_KERNEL_WENDLAND / ORC_KERNEL_GAUSSIAN */
    /* Optional assembled form (orc_assemble_csr): the matrix entries on the
     * neighbour pattern, a_diag[b] = A_bb and a_off[k] = A_b,cols[k] (Jacobi
     * scaled when jacobi is set).  When a_off is non-null orc_apply forms
     * y = A x from these stored entries instead of re-evaluating them. */
    const double *a_diag;
    const double *a_off;
} orc_op;

#define ORC_KERNEL_WENDLAND 0
#define ORC_KERNEL_GAUSSIAN 1

static double orc_kernel_w(const orc_op *op, double q) {
    return op->kernel == ORC_KERNEL_GAUSSIAN ? orc_gauss_w(q) : orc_wendland_w(q);
}
static double orc_kernel_f(const orc_op *op, double q) {
    return op->kernel == ORC_KERNEL_GAUSSIAN ? orc_gauss_f(q) : orc_wendland_f(q);
}

/* 2 * mubar_ab: arithmetic mean (mu_a + mu_b)/2 or harmonic 2 mu_a mu_b/(mu_a + mu_b)
 * (Section "Discretized equations"). */
static double orc_two_mubar(double ma, double mb, int avg) {
    if (avg == ORC_AVG_HARMONIC) {
        double s = ma + mb;
        return s > 0.0 ? 4.0 * (ma * mb) / s : 0.0;
    }
    return ma + mb;
}

/* Pair weight w_ba = -2 mubar_ab m_a F_ab / (rho_a rho_b) >= 0 for row b and
 * neighbour a (eq. kab with the diffusive sign reading). */
static double orc_pair_w(const orc_op *op, int64_t b, int64_t a) {
    double r2 = orc_dist2(op->x, op->y, op->z, b, a, op->period, 0, 0, 0);
    double q = sqrt(r2) / op->h;
    double h2 = op->h * op->h;
    double F = orc_kernel_f(op, q) / (h2 * h2 * op->h);
    double tm = orc_two_mubar(op->mu[a], op->mu[b], op->avg);
    return -(tm * op->mass[a] * F) / (op->rho[a] * op->rho[b]);
}

/* Kernel value W_ba used by the dummy-wall rows (eq. dummyvel). */
static double orc_pair_W(const orc_op *op, int64_t b, int64_t a) {
    double r2 = orc_dist2(op->x, op->y, op->z, b, a, op->period, 0, 0, 0);
    double q = sqrt(r2) / op->h;
    return orc_kernel_w(op, q) / (op->h * op->h * op->h);
}

/* Diagonal A_bb: 1 + dt sum_a w_ba for fluid rows (eq. diag), 1 for wall rows. */
static double orc_row_diag(const orc_op *op, int64_t b) {
    if (op->type[b] != ORC_FLUID) return 1.0;
    double sw = 0.0;
    for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) sw += orc_pair_w(op, b, op->cols[k]);
    return 1.0 + op->dt * sw;
}

void orc_diag(const orc_op *op, double *d) {
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < op->n; ++b) d[b] = orc_row_diag(op, b);
}

/* y = A x (or D^-1 A x with Jacobi) for the three components, matrix-free.
 *   fluid row b:        y_b = (1 + dt sum w_ba) x_b - dt sum w_ba x_a   (eq. implicit-system-base)
 *   dynamic wall row b: y_b = x_b                                       (eq. implicit-system-dyn-full)
 *   dummy wall row b:   y_b = x_b + sum_{a in F} W_ba x_a / sum_{a in F} W_ba
 *                       (identity when no fluid neighbour)              (eq. implicit-system-dummy-full) */
void orc_apply(const orc_op *op, const double *const *xin, double *const *yout) {
    if (op->a_off) {
        /* y_b = A_bb x_b + sum_k A_b,cols[k] x_cols[k] over the stored entries */
        #pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < op->n; ++b) {
            double d = op->a_diag[b];
            double y0 = d * xin[0][b], y1 = d * xin[1][b], y2 = d * xin[2][b];
            for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
                double e = op->a_off[k];
                int64_t a = op->cols[k];
                y0 += e * xin[0][a];
                y1 += e * xin[1][a];
                y2 += e * xin[2][a];
            }
            yout[0][b] = y0;
            yout[1][b] = y1;
            yout[2][b] = y2;
        }
        return;
    }
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < op->n; ++b) {
        double y0, y1, y2;
        if (op->type[b] == ORC_FLUID) {
            double sw = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
                int64_t a = op->cols[k];
                double w = orc_pair_w(op, b, a);
                sw += w;
                s0 += w * xin[0][a];
                s1 += w * xin[1][a];
                s2 += w * xin[2][a];
            }
            double diag = 1.0 + op->dt * sw;
            y0 = diag * xin[0][b] - op->dt * s0;
            y1 = diag * xin[1][b] - op->dt * s1;
            y2 = diag * xin[2][b] - op->dt * s2;
            if (op->jacobi) {
                y0 /= diag;
                y1 /= diag;
                y2 /= diag;
            }
        } else if (op->wall == ORC_WALL_DUMMY) {
            double sW = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
                int64_t a = op->cols[k];
                if (op->type[a] != ORC_FLUID) continue;
                double W = orc_pair_W(op, b, a);
                sW += W;
                s0 += W * xin[0][a];
                s1 += W * xin[1][a];
                s2 += W * xin[2][a];
            }
            y0 = xin[0][b];
            y1 = xin[1][b];
            y2 = xin[2][b];
            if (sW > 0.0) {
                y0 += s0 / sW;
                y1 += s1 / sW;
                y2 += s2 / sW;
            }
        } else {
            y0 = xin[0][b];
            y1 = xin[1][b];
            y2 = xin[2][b];
        }
        yout[0][b] = y0;
        yout[1][b] = y1;
        yout[2][b] = y2;
    }
}

/* Dense row-major n x n assembly of A (or D^-1 A), entry by entry from eqs.
 * diag / offdiag and the dummy-wall row. */
void orc_assemble_dense(const orc_op *op, double *A) {
    int64_t n = op->n;
    memset(A, 0, sizeof(double) * (size_t)(n * n));
    for (int64_t b = 0; b < n; ++b) {
        double *row = A + b * n;
        if (op->type[b] == ORC_FLUID) {
            double diag = orc_row_diag(op, b);
            double scale = op->jacobi ? 1.0 / diag : 1.0;
            row[b] = op->jacobi ? 1.0 : diag;
            for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
                int64_t a = op->cols[k];
                row[a] += -op->dt * orc_pair_w(op, b, a) * scale;
            }
        } else if (op->wall == ORC_WALL_DUMMY) {
            double sW = 0.0;
            for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
                int64_t a = op->cols[k];
                if (op->type[a] == ORC_FLUID) sW += orc_pair_W(op, b, a);
            }
            row[b] = 1.0;
            if (sW > 0.0)
                for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
                    int64_t a = op->cols[k];
                    if (op->type[a] == ORC_FLUID) row[a] += orc_pair_W(op, b, a) / sW;
                }
        } else {
            row[b] = 1.0;
        }
    }
}

/* The entries of A (or D^-1 A) on the neighbour pattern, by the same
 * expressions as the dense assembly: a_diag[b] = A_bb, a_off[k] = A_b,a with
 * a = cols[k] (0 for the wall neighbours of a dummy-wall row and for every
 * neighbour of an identity row).  a_off has row_ptr[n] entries. */
void orc_assemble_csr(const orc_op *op, double *a_diag, double *a_off) {
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < op->n; ++b) {
        int64_t k0 = op->row_ptr[b], k1 = op->row_ptr[b + 1];
        for (int64_t k = k0; k < k1; ++k) a_off[k] = 0.0;
        if (op->type[b] == ORC_FLUID) {
            double diag = orc_row_diag(op, b);
            double scale = op->jacobi ? 1.0 / diag : 1.0;
            a_diag[b] = op->jacobi ? 1.0 : diag;
            for (int64_t k = k0; k < k1; ++k) a_off[k] = -op->dt * orc_pair_w(op, b, op->cols[k]) * scale;
        } else if (op->wall == ORC_WALL_DUMMY) {
            double sW = 0.0;
            for (int64_t k = k0; k < k1; ++k)
                if (op->type[op->cols[k]] == ORC_FLUID) sW += orc_pair_W(op, b, op->cols[k]);
            a_diag[b] = 1.0;
            if (sW > 0.0)
                for (int64_t k = k0; k < k1; ++k)
                    if (op->type[op->cols[k]] == ORC_FLUID) a_off[k] = orc_pair_W(op, b, op->cols[k]) / sW;
        } else {
            a_diag[b] = 1.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Single-precision compensated sums (appendix "Implementation notes": every */
/* multi-term sum in single precision uses Kahan's compensated summation).   */
/* ------------------------------------------------------------------------ */

/* Kahan's compensated sum of v[0..n) in FP32, in index order. */
float orc_kahan_sum_f32(int64_t n, const float *v) {
    float s = 0.0f, c = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        float y = v[i] - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    return s;
}

/* sum_i w_i a_i b_i in FP32: each product rounded to FP32 ((w_i a_i) b_i
 * when w is given, else a_i b_i), the products added in index order with
 * Kahan's compensation. */
float orc_kahan_dot_f32(int64_t n, const float *w, const float *a, const float *b) {
    float s = 0.0f, c = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        float p = w ? (w[i] * a[i]) * b[i] : a[i] * b[i];
        float y = p - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    return s;
}

/* out[b] = Kahan's FP32 sum of v[row_ptr[b] .. row_ptr[b+1]) in order, its
 * zero terms skipped. */
void orc_kahan_rows_f32(int64_t n, const int64_t *row_ptr, const float *v, float *out) {
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int64_t b = 0; b < n; ++b) {
        float s = 0.0f, c = 0.0f;
        for (int64_t k = row_ptr[b]; k < row_ptr[b + 1]; ++k) {
            if (v[k] == 0.0f) continue;
            float y = v[k] - c;
            float t = s + y;
            c = (t - s) - y;
            s = t;
        }
        out[b] = s;
    }
}

/* The single-precision gemv: y_b = A_bb x_b + sum_k A_b,cols[k] x_cols[k],
 * every product rounded to FP32, the terms (diagonal first, then the stored
 * entries in order, zero entries skipped) summed with Kahan's compensation. */
void orc_kahan_gemv_f32(int64_t n, const int64_t *row_ptr, const int32_t *cols, const float *diag,
                        const float *off, const float *x, float *y) {
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int64_t b = 0; b < n; ++b) {
        float s = 0.0f, c = 0.0f;
        float terms0 = diag[b] * x[b];
        {
            float yy = terms0 - c;
            float t = s + yy;
            c = (t - s) - yy;
            s = t;
        }
        for (int64_t k = row_ptr[b]; k < row_ptr[b + 1]; ++k) {
            if (off[k] == 0.0f) continue;
            float p = off[k] * x[cols[k]];
            float yy = p - c;
            float t = s + yy;
            c = (t - s) - yy;
            s = t;
        }
        y[b] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* BiCGSTAB for d = 3 systems sharing one matrix.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t iters;
    int32_t status;
    int32_t state[3];
    int32_t stall_count[3];
    double rr[3];       /* final recursive r.r (scaled system) */
    double bb[3];       /* b.b of the scaled right-hand side */
    double tau2[3];
    double true_rr[3];  /* final (b - A x).(b - A x) of the scaled system */
    int32_t n_true_checks;
    int32_t n_replaced;
    int32_t history_len;
} orc_report;

#define ORC_ROBUST 0
#define ORC_STANDARD 1
#define ORC_MAX_RESTARTS 3

/* Inner products are summed in fixed blocks of ORC_DOT_BLOCK terms and the
 * block sums then in block order, so the result does not depend on the
 * thread count (for n <= ORC_DOT_BLOCK it is the plain sequential sum). */
#define ORC_DOT_BLOCK 16384

static double orc_dot(int64_t n, const double *a, const double *b) {
    int64_t nblk = (n + ORC_DOT_BLOCK - 1) / ORC_DOT_BLOCK;
    if (nblk <= 1) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
        return s;
    }
    double *part = (double *)malloc(sizeof(double) * (size_t)nblk);
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int64_t k = 0; k < nblk; ++k) {
        int64_t i1 = (k + 1) * ORC_DOT_BLOCK < n ? (k + 1) * ORC_DOT_BLOCK : n;
        double s = 0.0;
        for (int64_t i = k * ORC_DOT_BLOCK; i < i1; ++i) s += a[i] * b[i];
        part[k] = s;
    }
    double s = 0.0;
    for (int64_t k = 0; k < nblk; ++k) s += part[k];
    free(part);
    return s;
}

static int orc_finite(double v) { return isfinite(v); }

/* r = bh - Ah x for all three components. */
static void orc_residual(const orc_op *op, double *const *bh, double *const *x, double *const *r,
                         double *const *tmp) {
    orc_apply(op, (const double *const *)x, tmp);
    for (int c = 0; c < 3; ++c) {
        #pragma omp parallel for schedule(static) if (op->n >= ORC_PAR_MIN)
        for (int64_t i = 0; i < op->n; ++i) r[c][i] = bh[c][i] - tmp[c][i];
    }
}

/* State of one BiCGSTAB solve: vectors and per-component scalars. */
typedef struct {
    const orc_op *op;
    int32_t variant;
    int64_t n;
    double *bh[3], *r[3], *rh0[3], *p[3], *Ap[3], *s[3], *As[3], *tmp[3];
    double *const *x;
    /* robust form: gamma_i, alpha'_{i-1}, beta_{i-1}; textbook form:
     * gamma_{i-1}, alpha_{i-1}, omega_{i-1} (in gamma_prev, alpha, omega) */
    double gamma[3], gamma_prev[3], alpha[3], alphap[3], beta[3], omega[3], delta[3];
    double tau2[3], rr[3], rr_ref[3];
    int state[3], restarts[3], stall[3];
} orc_bicg;

static void orc_bicg_fresh_direction(orc_bicg *S, int c) {
    /* the next direction is built from r alone */
    S->alphap[c] = 0.0;
    S->beta[c] = 0.0;
    S->gamma_prev[c] = 1.0;
    S->alpha[c] = 1.0;
    S->omega[c] = 1.0;
}

/* Direction update.  Robust form: p = r + beta p - alpha' A p, a term with
 * a zero coefficient skipped so that p and A p need not be defined at the
 * first iteration.  Textbook form: gamma = r0hat . r, beta =
 * (gamma / gamma_prev)(alpha / omega), p = r + beta (p - omega A p), and a
 * zero gamma is a breakdown. */
static void orc_bicg_direction(orc_bicg *S) {
    int64_t n = S->n;
    for (int c = 0; c < 3; ++c) {
        double *p = S->p[c];
        const double *r = S->r[c], *Ap = S->Ap[c];
        if (S->variant == ORC_ROBUST) {
            double bt = S->beta[c], ap = S->alphap[c];
            #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) {
                double v = r[i];
                if (bt != 0.0) v += bt * p[i];
                if (ap != 0.0) v -= ap * Ap[i];
                p[i] = v;
            }
        } else {
            double g = orc_dot(n, S->rh0[c], r);
            double bt = 0.0;
            if (S->gamma_prev[c] != 0.0 && S->omega[c] != 0.0)
                bt = (g / S->gamma_prev[c]) * (S->alpha[c] / S->omega[c]);
            if (!orc_finite(bt)) bt = 0.0;
            if (g == 0.0) S->stall[c] = 1;
            S->gamma[c] = g;
            S->beta[c] = bt;
            double om = S->omega[c];
            #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) {
                double v = r[i];
                if (bt != 0.0) v += bt * (p[i] - om * Ap[i]);
                p[i] = v;
            }
        }
    }
}

/* First half-step: A p, delta = r0hat . A p, alpha = gamma / delta (a zero
 * or non-finite delta or alpha is a breakdown, alpha = 0), and the
 * intermediate residual s = r - alpha A p. */
static void orc_bicg_half1(orc_bicg *S, int it, int32_t force_stall_iter, int32_t force_stall_comp) {
    int64_t n = S->n;
    orc_apply(S->op, (const double *const *)S->p, S->Ap);
    for (int c = 0; c < 3; ++c) {
        double d = orc_dot(n, S->rh0[c], S->Ap[c]);
        if (it == force_stall_iter && c == force_stall_comp) d = 0.0;
        double a = 0.0;
        if (d != 0.0 && orc_finite(d)) a = S->gamma[c] / d;
        if (!orc_finite(a) || d == 0.0 || !orc_finite(d)) {
            a = 0.0;
            S->stall[c] = 1;
        }
        S->delta[c] = d;
        S->alpha[c] = a;
        double *sv = S->s[c];
        const double *r = S->r[c], *Ap = S->Ap[c];
        #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
        for (int64_t i = 0; i < n; ++i) sv[i] = r[i] - a * Ap[i];
    }
}

/* Second half-step: A s, omega = (s . A s)/(A s . A s) (zero: breakdown);
 * the textbook form also checks s itself and takes omega = 0 when s . s
 * already meets the threshold; then x = x + alpha p + omega s and
 * r = s - omega A s. */
static void orc_bicg_half2(orc_bicg *S) {
    int64_t n = S->n;
    orc_apply(S->op, (const double *const *)S->s, S->As);
    for (int c = 0; c < 3; ++c) {
        double tt = orc_dot(n, S->As[c], S->As[c]);
        double ts = orc_dot(n, S->As[c], S->s[c]);
        double w = 0.0;
        if (tt != 0.0) w = ts / tt;
        if (!orc_finite(w)) w = 0.0;
        if (w == 0.0) S->stall[c] = 1;
        if (S->variant == ORC_STANDARD && orc_dot(n, S->s[c], S->s[c]) < S->tau2[c]) w = 0.0;
        S->omega[c] = w;
        double a = S->alpha[c];
        double *x = S->x[c], *r = S->r[c];
        const double *p = S->p[c], *sv = S->s[c], *As = S->As[c];
        #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
        for (int64_t i = 0; i < n; ++i) {
            double xv = x[i] + a * p[i];
            x[i] = xv + w * sv[i];
            r[i] = sv[i] - w * As[i];
        }
    }
}

/* Close-out.  Robust form: gamma' = r0hat . r, alpha' = gamma'/delta,
 * beta = alpha'/omega (both 0 after a breakdown; a zero gamma' is one);
 * textbook form: keep gamma for the next beta.  Then r . r and the state:
 * converged when r . r < tau^2 (taking precedence), stalled after a
 * breakdown, progressing otherwise. */
static void orc_bicg_close(orc_bicg *S, orc_report *rep) {
    int64_t n = S->n;
    for (int c = 0; c < 3; ++c) {
        if (S->variant == ORC_ROBUST) {
            double g = orc_dot(n, S->rh0[c], S->r[c]);
            double ap = 0.0, bt = 0.0;
            if (!S->stall[c]) {
                ap = g / S->delta[c];
                if (!orc_finite(ap)) ap = 0.0;
                bt = ap / S->omega[c];
                if (!orc_finite(bt)) bt = 0.0;
            }
            if (g == 0.0) S->stall[c] = 1;
            S->gamma[c] = g;
            S->alphap[c] = ap;
            S->beta[c] = bt;
        } else {
            S->gamma_prev[c] = S->gamma[c];
        }
        S->rr[c] = orc_dot(n, S->r[c], S->r[c]);
        if (S->stall[c]) rep->stall_count[c]++;
        S->state[c] = S->rr[c] < S->tau2[c] ? ORC_CONVERGED : (S->stall[c] ? ORC_STALLED : ORC_PROGRESSING);
    }
}

/* True residual check: r_true = bh - Ah x; a component the recursion calls
 * converged but r_true does not is restarted from r_true (at most
 * ORC_MAX_RESTARTS times, then reported stalled); with restart_drop > 0 a
 * progressing component whose true r.r fell below restart_drop times its
 * r.r at the last (re)start restarts the same way.  A restart takes
 * r = r0hat = r_true and a fresh direction. */
static void orc_bicg_check(orc_bicg *S, double restart_drop, orc_report *rep) {
    int64_t n = S->n;
    rep->n_true_checks++;
    orc_residual(S->op, S->bh, S->x, S->tmp, S->s);
    for (int c = 0; c < 3; ++c) {
        double trr = orc_dot(n, S->tmp[c], S->tmp[c]);
        int restart = 0;
        if (S->state[c] == ORC_CONVERGED && !(trr < S->tau2[c])) {
            if (S->restarts[c] >= ORC_MAX_RESTARTS) {
                S->state[c] = ORC_STALLED; /* precision cannot reach the tolerance */
            } else {
                S->restarts[c]++;
                restart = 1;
            }
        } else if (S->state[c] == ORC_PROGRESSING && trr < restart_drop * S->rr_ref[c]) {
            restart = 1; /* residual far below the shadow vector: fresh start */
        }
        if (restart) {
            memcpy(S->r[c], S->tmp[c], sizeof(double) * (size_t)n);
            memcpy(S->rh0[c], S->tmp[c], sizeof(double) * (size_t)n);
            S->rr[c] = trr;
            S->gamma[c] = orc_dot(n, S->rh0[c], S->r[c]);
            orc_bicg_fresh_direction(S, c);
            memset(S->p[c], 0, sizeof(double) * (size_t)n);
            memset(S->Ap[c], 0, sizeof(double) * (size_t)n);
            S->state[c] = trr < S->tau2[c] ? ORC_CONVERGED : ORC_PROGRESSING;
            S->rr_ref[c] = trr;
            rep->n_replaced++;
        }
    }
}

static int orc_bicg_any_progressing(const orc_bicg *S) {
    int any = 0;
    for (int c = 0; c < 3; ++c) any |= (S->state[c] == ORC_PROGRESSING);
    return any;
}

/*
 * Solve A V = B for the three columns of B by the restructured ("robust")
 * BiCGSTAB or the textbook BiCGSTAB (Section "Restructuring the stabilized
 * biconjugate gradient method"), each component with its own scalars and
 * the stopping rule of that Section.  With op->jacobi the system is
 * left-scaled: Ah = D^-1 A, bh = D^-1 b (appendix "Implementation notes"),
 * and every threshold refers to the scaled residual.
 *
 * b, x: three component arrays of length n; x holds the initial guess on
 * entry and the solution on exit.  history (optional) receives r.r per
 * component at the end of every iteration, history[3*it + c], it = 0 being
 * the initial residual.
 *
 * force_stall_iter / force_stall_comp: host-forced breakdown used by the
 * failure-handling tests -- at that iteration that component's delta is
 * treated as zero.  Pass -1 to disable.
 */
int orc_bicgstab(const orc_op *op, int32_t variant, const double *const *b, double *const *x,
                 double tol, int32_t max_iter, double floor_, int32_t true_res_period,
                 double restart_drop, int32_t force_stall_iter, int32_t force_stall_comp,
                 orc_report *rep, double *history, int32_t history_cap) {
    int64_t n = op->n;
    memset(rep, 0, sizeof(*rep));
    double *buf = (double *)calloc((size_t)(n > 0 ? n : 1) * 3 * 9, sizeof(double));
    orc_bicg S;
    memset(&S, 0, sizeof(S));
    S.op = op;
    S.variant = variant;
    S.n = n;
    S.x = x;
    double *D = buf + 8 * 3 * n;
    for (int c = 0; c < 3; ++c) {
        S.bh[c] = buf + (0 * 3 + c) * n;
        S.r[c] = buf + (1 * 3 + c) * n;
        S.rh0[c] = buf + (2 * 3 + c) * n;
        S.p[c] = buf + (3 * 3 + c) * n;
        S.Ap[c] = buf + (4 * 3 + c) * n;
        S.s[c] = buf + (5 * 3 + c) * n;
        S.As[c] = buf + (6 * 3 + c) * n;
        S.tmp[c] = buf + (7 * 3 + c) * n;
    }
    /* Jacobi: D = diag(A); bh = b / D. */
    if (op->jacobi) orc_diag(op, D);
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) S.bh[c][i] = op->jacobi ? b[c][i] / D[i] : b[c][i];
    for (int c = 0; c < 3; ++c) {
        rep->bb[c] = orc_dot(n, S.bh[c], S.bh[c]);
        if (!orc_finite(rep->bb[c])) {
            free(buf);
            rep->status = ORC_E_NONFINITE;
            return ORC_E_NONFINITE;
        }
    }
    /* r0 = bh - Ah x0; r0hat = r0; tau^2 = max(eps^2 bh.bh, floor); the
     * robust form starts with gamma_1 = r0hat . r0 */
    orc_residual(op, S.bh, x, S.r, S.tmp);
    for (int c = 0; c < 3; ++c) {
        memcpy(S.rh0[c], S.r[c], sizeof(double) * (size_t)n);
        S.tau2[c] = tol * tol * rep->bb[c];
        if (S.tau2[c] < floor_) S.tau2[c] = floor_;
        S.rr[c] = orc_dot(n, S.r[c], S.r[c]);
        S.rr_ref[c] = S.rr[c];
        S.gamma[c] = orc_dot(n, S.rh0[c], S.r[c]);
        orc_bicg_fresh_direction(&S, c);
        S.delta[c] = 0.0;
        S.state[c] = S.rr[c] < S.tau2[c] ? ORC_CONVERGED : ORC_PROGRESSING;
        if (history && history_cap > 0) history[c] = S.rr[c];
    }
    int hl = 1;
    int it = 0;
    for (;;) {
        int periodic_check = (it > 0 && true_res_period > 0 && it % true_res_period == 0);
        if (!orc_bicg_any_progressing(&S) || periodic_check) orc_bicg_check(&S, restart_drop, rep);
        if (!orc_bicg_any_progressing(&S) || it >= max_iter) break;
        ++it;
        for (int c = 0; c < 3; ++c) S.stall[c] = 0;
        orc_bicg_direction(&S);
        orc_bicg_half1(&S, it, force_stall_iter, force_stall_comp);
        orc_bicg_half2(&S);
        orc_bicg_close(&S, rep);
        if (history && hl < history_cap)
            for (int c = 0; c < 3; ++c) history[3 * hl + c] = S.rr[c];
        ++hl;
    }
    /* final true residual for the report */
    orc_residual(op, S.bh, x, S.tmp, S.s);
    int any_prog = 0, any_stall = 0;
    for (int c = 0; c < 3; ++c) {
        rep->true_rr[c] = orc_dot(n, S.tmp[c], S.tmp[c]);
        rep->rr[c] = S.rr[c];
        rep->tau2[c] = S.tau2[c];
        rep->state[c] = S.state[c];
        any_prog |= S.state[c] == ORC_PROGRESSING;
        any_stall |= S.state[c] == ORC_STALLED;
    }
    rep->iters = it;
    rep->history_len = hl < history_cap ? hl : history_cap;
    rep->status = any_prog ? ORC_NOT_CONVERGED : (any_stall ? ORC_STATUS_STALLED : ORC_OK);
    free(buf);
    return rep->status;
}

/* ------------------------------------------------------------------------ */
/* Rotated CG for d = 3 symmetric systems sharing one matrix (Section       */
/* "Restructuring the Conjugate Gradient"): p update first, beta last.      */
/* ------------------------------------------------------------------------ */

/* <a, b>_D = sum_i D_i a_i b_i (D = NULL: the Euclidean product). */
static double orc_dot_w(int64_t n, const double *D, const double *a, const double *b) {
    /* blocked like orc_dot: the same result for any thread count */
    int64_t nblk = (n + ORC_DOT_BLOCK - 1) / ORC_DOT_BLOCK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nblk > 0 ? nblk : 1));
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int64_t k = 0; k < nblk; ++k) {
        int64_t i1 = (k + 1) * ORC_DOT_BLOCK < n ? (k + 1) * ORC_DOT_BLOCK : n;
        double s = 0.0;
        for (int64_t i = k * ORC_DOT_BLOCK; i < i1; ++i) s += (D ? D[i] : 1.0) * a[i] * b[i];
        part[k] = s;
    }
    double s = 0.0;
    for (int64_t k = 0; k < nblk; ++k) s += part[k];
    free(part);
    return s;
}

/*
 * Arguments and report as orc_bicgstab (restart_drop does not apply: the CG
 * has no shadow vector).  Returns ORC_E_ARG for dummy walls.
 *
 * Per component c, with Ah = D^-1 A, bh = D^-1 b under op->jacobi (D = 1
 * otherwise) and <,> the D-weighted product:
 *   x_w = bh_w on wall rows;  r_0 = bh - Ah x_0;  rho_0 = <r_0, r_0>;  beta_0 = 0
 *   iteration i >= 0:
 *     p_i     = r_i + beta_i p_{i-1}          (p_{i-1} unread when beta_i = 0)
 *     alpha_i = rho_i / <p_i, Ah p_i>
 *     r_{i+1} = r_i - alpha_i Ah p_i,  x_{i+1} = x_i + alpha_i p_i
 *     beta_{i+1} = rho_{i+1} / rho_i,  rho_{i+1} = <r_{i+1}, r_{i+1}>
 *   converged when r.r < tau^2 (Euclidean, scaled residual).
 */
int orc_cg(const orc_op *op, const double *const *b, double *const *x, double tol, int32_t max_iter,
           double floor_, int32_t true_res_period, int32_t force_stall_iter, int32_t force_stall_comp,
           orc_report *rep, double *history, int32_t history_cap) {
    int64_t n = op->n;
    memset(rep, 0, sizeof(*rep));
    if (op->wall == ORC_WALL_DUMMY) {
        rep->status = ORC_E_ARG;
        return ORC_E_ARG;
    }
    double *buf = (double *)calloc((size_t)(n > 0 ? n : 1) * (3 * 5 + 1), sizeof(double));
    double *bh[3], *r[3], *p[3], *Ap[3], *tmp[3];
    for (int c = 0; c < 3; ++c) {
        bh[c] = buf + (0 * 3 + c) * n;
        r[c] = buf + (1 * 3 + c) * n;
        p[c] = buf + (2 * 3 + c) * n;
        Ap[c] = buf + (3 * 3 + c) * n;
        tmp[c] = buf + (4 * 3 + c) * n;
    }
    double *D = NULL;
    if (op->jacobi) {
        D = buf + 15 * n;
        orc_diag(op, D);
    }
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) bh[c][i] = D ? b[c][i] / D[i] : b[c][i];
    for (int c = 0; c < 3; ++c) {
        rep->bb[c] = orc_dot(n, bh[c], bh[c]);
        if (!orc_finite(rep->bb[c])) {
            free(buf);
            rep->status = ORC_E_NONFINITE;
            return ORC_E_NONFINITE;
        }
    }
    /* wall rows are identity rows: start them at their solution */
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i)
            if (op->type[i] != ORC_FLUID) x[c][i] = bh[c][i];
    orc_residual(op, bh, x, r, tmp);
    double rho[3], beta[3], tau2[3], rr[3];
    int state[3], restarts[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        tau2[c] = tol * tol * rep->bb[c];
        if (tau2[c] < floor_) tau2[c] = floor_;
        rr[c] = orc_dot(n, r[c], r[c]);
        rho[c] = orc_dot_w(n, D, r[c], r[c]);
        beta[c] = 0.0;
        state[c] = rr[c] < tau2[c] ? ORC_CONVERGED : ORC_PROGRESSING;
        if (history && history_cap > 0) history[c] = rr[c];
    }
    int hl = 1;
    int it = 0;
    for (;;) {
        int any_prog = 0;
        for (int c = 0; c < 3; ++c) any_prog |= (state[c] == ORC_PROGRESSING);
        int periodic_check = (it > 0 && true_res_period > 0 && it % true_res_period == 0);
        if (!any_prog || periodic_check) {
            /* true residual; a converged component that fails it restarts
             * from r_true with beta = 0 (at most ORC_MAX_RESTARTS times) */
            rep->n_true_checks++;
            orc_residual(op, bh, x, tmp, Ap);
            for (int c = 0; c < 3; ++c) {
                double trr = orc_dot(n, tmp[c], tmp[c]);
                if (state[c] == ORC_CONVERGED && !(trr < tau2[c])) {
                    if (restarts[c] >= ORC_MAX_RESTARTS) {
                        state[c] = ORC_STALLED;
                    } else {
                        restarts[c]++;
                        memcpy(r[c], tmp[c], sizeof(double) * (size_t)n);
                        rr[c] = trr;
                        rho[c] = orc_dot_w(n, D, r[c], r[c]);
                        beta[c] = 0.0;
                        state[c] = trr < tau2[c] ? ORC_CONVERGED : ORC_PROGRESSING;
                        rep->n_replaced++;
                    }
                }
            }
            any_prog = 0;
            for (int c = 0; c < 3; ++c) any_prog |= (state[c] == ORC_PROGRESSING);
        }
        if (!any_prog || it >= max_iter) break;
        ++it;
        int stall[3] = {0, 0, 0};
        /* direction update (beta = 0: the direction restarts from r) */
        for (int c = 0; c < 3; ++c) {
            double bt = beta[c];
            double *pc = p[c];
            const double *rc = r[c];
            #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) pc[i] = bt != 0.0 ? rc[i] + bt * pc[i] : rc[i];
        }
        orc_apply(op, (const double *const *)p, Ap);
        for (int c = 0; c < 3; ++c) {
            double pap = orc_dot_w(n, D, p[c], Ap[c]);
            if (it == force_stall_iter && c == force_stall_comp) pap = 0.0;
            double a = 0.0;
            if (pap != 0.0 && orc_finite(pap)) a = rho[c] / pap;
            if (!orc_finite(a) || a == 0.0) {
                a = 0.0;
                stall[c] = 1;
            }
            double *xc = x[c], *rc = r[c];
            const double *pc = p[c], *apc = Ap[c];
            #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t i = 0; i < n; ++i) {
                xc[i] = xc[i] + a * pc[i];
                rc[i] = rc[i] - a * apc[i];
            }
            double rho_new = orc_dot_w(n, D, r[c], r[c]);
            double bt = 0.0;
            if (!stall[c] && rho[c] != 0.0) bt = rho_new / rho[c];
            if (!orc_finite(bt)) bt = 0.0;
            beta[c] = bt;
            rho[c] = rho_new;
            rr[c] = orc_dot(n, r[c], r[c]);
            if (stall[c]) rep->stall_count[c]++;
            state[c] = rr[c] < tau2[c] ? ORC_CONVERGED : (stall[c] ? ORC_STALLED : ORC_PROGRESSING);
            if (history && hl < history_cap) history[3 * hl + c] = rr[c];
        }
        ++hl;
    }
    orc_residual(op, bh, x, tmp, Ap);
    int any_prog = 0, any_stall = 0;
    for (int c = 0; c < 3; ++c) {
        rep->true_rr[c] = orc_dot(n, tmp[c], tmp[c]);
        rep->rr[c] = rr[c];
        rep->tau2[c] = tau2[c];
        rep->state[c] = state[c];
        any_prog |= state[c] == ORC_PROGRESSING;
        any_stall |= state[c] == ORC_STALLED;
    }
    rep->iters = it;
    rep->history_len = hl < history_cap ? hl : history_cap;
    rep->status = any_prog ? ORC_NOT_CONVERGED : (any_stall ? ORC_STATUS_STALLED : ORC_OK);
    free(buf);
    return rep->status;
}

/* ------------------------------------------------------------------------ */
/* Papanastasiou viscosity (Section "Non-Newtonian viscosity", eq. papa).    */
/* ------------------------------------------------------------------------ */

/* Ybar(D) = (1 - exp(-m D))/D for m D >= x0, else m T(m D) with T the
 * Maclaurin series of (1 - e^-x)/x truncated after 8 terms, in Horner form:
 * T(x) = 1 - x/2 (1 - x/3 (1 - x/4 (1 - x/5 (1 - x/6 (1 - x/7 (1 - x/8)))))). */
double orc_ybar(double D, double m) {
    const double x0 = pow(362880.0 * ldexp(1.0, -23), 0.125);
    double x = m * D;
    if (x >= x0) return (1.0 - exp(-x)) / D;
    double t = 1.0;
    for (int k = 8; k >= 2; --k) t = 1.0 - x / (double)k * t;
    return m * t;
}

/* Per particle b: G = sum_a (m_a/rho_a) F(r_ab) r_ab u_ab^T (r_ab = r_a - r_b
 * by minimum image, u_ab = u_a - u_b), S = (G + G^T)/2, D_b = sqrt(2 S:S);
 * fluid rows: mu_b = tau0 Ybar(D_b) + mu0, wall rows keep op->mu.  u: three
 * component arrays; D_out may be NULL. */
void orc_papanastasiou(const orc_op *op, const double *const *u, double tau0, double m, double mu0,
                       double *mu_out, double *D_out) {
    const double h = op->h;
    const double h5 = h * h * h * h * h;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < op->n; ++b) {
        double G[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (int64_t k = op->row_ptr[b]; k < op->row_ptr[b + 1]; ++k) {
            int64_t a = op->cols[k];
            double r[3];
            r[0] = orc_disp(op->x[a], op->x[b], op->period[0]);
            r[1] = orc_disp(op->y[a], op->y[b], op->period[1]);
            r[2] = orc_disp(op->z[a], op->z[b], op->period[2]);
            double d = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
            double F = orc_kernel_f(op, d / h) / h5;
            double vf = op->mass[a] / op->rho[a] * F;
            double du[3];
            for (int j = 0; j < 3; ++j) du[j] = u[j][a] - u[j][b];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) G[i][j] += vf * r[i] * du[j];
        }
        double ss = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double sij = 0.5 * (G[i][j] + G[j][i]);
                ss += sij * sij;
            }
        double D = sqrt(2.0 * ss);
        if (D_out) D_out[b] = D;
        mu_out[b] = op->type[b] == ORC_FLUID ? tau0 * orc_ybar(D, m) + mu0 : op->mu[b];
    }
}
