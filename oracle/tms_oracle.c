/*
 * tms_oracle.c -- plain FP64 CPU oracle for the Gaussian-surface adaptive
 * partition-and-estimation method of Liu, Chen & Lu, "Efficient and Qualified
 * Mesh Generation for Gaussian Molecular Surface Using Piecewise Trilinear
 * Polynomial Approximation" (arXiv:1611.03474).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * Everything is computed in double precision, step by step, in the order the
 * paper gives, with no blocking or fusion beyond what the definitions state.
 * The only acceleration structure is a uniform bin grid used to enumerate a
 * superset of the atoms that pass the neighbourhood predicate; the predicate
 * itself decides membership.
 *
 * Readings of the paper that this file takes (the paper is silent or garbled
 * there) are marked "Reading:" in the comments.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -o libtms_oracle.so tms_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameters                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double D;        /* decay rate of the Gaussian kernel (Section 1, eq. Gaussian1) */
    double c;        /* isovalue (Section 1) */
    double tau;      /* bound on the higher-order coefficients (Section 2.2, Step 3) */
    double h0;       /* edge of the initial coarse grid cubes (Section 2.2) */
    double h_min;    /* edge of the finest cubes allowed */
    double pad;      /* padding of the initial grid around the atoms */
    double eps_cut;  /* truncation level of a single Gaussian term */
    int32_t uniform; /* 1: plain method, every cube of an h0 grid is a leaf */
    int32_t nthreads;/* OpenMP threads (0: library default) */
    int32_t conf;    /* conformation id written into edge keys */
    int32_t gl_nodes;/* Gauss-Legendre nodes for the 1-D projections (0: 32) */
    int32_t degree;  /* degree n of the 1-D Legendre series, 1..3 (0: 3, the
                        paper's choice; Section 2.2.1) */
    int32_t reexpand;/* 0: a child's tensor is projected from the atoms again;
                        1: it is the parent's polynomial written in the child's
                        Legendre basis (eq. childtensor), no atom loop below the
                        roots */
} or_params;

enum { OR_REASON_UNIFORM = 0, OR_REASON_CONVERGED = 1, OR_REASON_HMIN = 2 };
enum { OR_CLS_OUTSIDE = 0, OR_CLS_SURFACE = 1, OR_CLS_INSIDE = 2 };

#define OR_MAXLEV 8
#define OR_TIE 1e-9
#define OR_TIE_LIST 1024

/* ------------------------------------------------------------------------ */
/* Legendre polynomials L0..L3 and Gauss-Legendre quadrature                  */
/* ------------------------------------------------------------------------ */

static void legendre4(double t, double L[4])
{
    L[0] = 1.0;
    L[1] = t;
    L[2] = 0.5 * (3.0 * t * t - 1.0);
    L[3] = 0.5 * (5.0 * t * t * t - 3.0 * t);
}

/* n-point Gauss-Legendre nodes and weights on [-1,1]: the nodes are the roots
 * of the degree-n Legendre polynomial, found by Newton's method from the
 * asymptotic guess cos(pi (i - 1/4) / (n + 1/2)); the weight of a node t is
 * 2 / ((1 - t^2) P_n'(t)^2).  P_n and P_n' come from Bonnet's recurrence. */
void or_gauss_legendre(int n, double *t, double *w)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            /* p1 = P_n(x), p0 = P_{n-1}(x) */
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17)
                break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* ------------------------------------------------------------------------ */
/* One-dimensional degree-3 Legendre projection with C0 endpoint correction   */
/* (Section 2.2.1: eqs. poly2_1..poly2_3, the alpha_j integrals, eqs. poly3,  */
/* condition1, alpha).                                                        */
/*                                                                            */
/* Reading: the alpha_j integral is printed with normalisation 2/(b-a) and   */
/* integrand "phi(local coordinate)"; it is taken as the standard Legendre    */
/* projection of the one-dimensional factor f of the Gaussian, i.e.           */
/*   alpha_j = (2j+1)/2 * int_{-1}^{1} f(t) L_j(t) dt,                        */
/* the only reading for which the paper's least-squares remark holds.         */
/* ------------------------------------------------------------------------ */

typedef double (*or_fun1)(double t, void *ctx);

/* Generic projection of a function f on [-1,1] given its values at the ends;
 * exposed so that the tests can feed polynomials through it. */
static double gl_t[65][64], gl_w[65][64];
static volatile int gl_ready[65];

static void gl_nodes(int n, const double **t, const double **w)
{
    if (!gl_ready[n]) {
#ifdef _OPENMP
#pragma omp critical(or_gl_init)
#endif
        {
            if (!gl_ready[n]) {
                or_gauss_legendre(n, gl_t[n], gl_w[n]);
                gl_ready[n] = 1;
            }
        }
    }
    *t = gl_t[n];
    *w = gl_w[n];
}

/* Degree-n series (n = 1..3) of f on [-1,1] with the endpoint correction of
 * eqs. poly3, condition1 and alpha; coefficients above n are zero. */
void or_project_fn_deg(or_fun1 f, void *ctx, int nodes, int degree, double alpha[4])
{
    const double *t, *w;
    if (nodes <= 0 || nodes > 64)
        nodes = 32;
    const int n = (degree >= 1 && degree <= 3) ? degree : 3;
    gl_nodes(nodes, &t, &w);
    double a[4] = {0, 0, 0, 0};
    for (int q = 0; q < nodes; ++q) {
        double L[4];
        legendre4(t[q], L);
        double fq = f(t[q], ctx);
        for (int j = 0; j <= n; ++j)
            a[j] += w[q] * fq * L[j];
    }
    for (int j = 0; j <= n; ++j)
        a[j] *= (2.0 * j + 1.0) / 2.0;
    /* eq. condition1: the corrected polynomial must equal f at both ends.
     * With P(1) = sum_j a_j and P(-1) = sum_j (-1)^j a_j, the corrections
     * e0 (on L_{n-1}) and e1 (on L_n) satisfy, since L_j(+-1) = (+-1)^j,
     *   e0 + e1 = f(1) - P(1) =: ep,
     *   (-1)^(n-1) e0 + (-1)^n e1 = f(-1) - P(-1) =: em.
     * n odd: e0 - e1 = em; n even: -e0 + e1 = em. */
    double fp = f(1.0, ctx), fm = f(-1.0, ctx);
    double Pp = 0.0, Pm = 0.0;
    for (int j = 0; j <= n; ++j) {
        Pp += a[j];
        Pm += (j & 1) ? -a[j] : a[j];
    }
    double ep = fp - Pp, em = fm - Pm;
    double e0, e1;
    if (n & 1) {
        e0 = 0.5 * (ep + em);
        e1 = 0.5 * (ep - em);
    } else {
        e0 = 0.5 * (ep - em);
        e1 = 0.5 * (ep + em);
    }
    for (int j = 0; j < 4; ++j)
        alpha[j] = j <= n ? a[j] : 0.0;
    alpha[n - 1] += e0; /* eq. alpha, j = n-1 */
    alpha[n] += e1;     /* eq. alpha, j = n */
}

void or_project_fn(or_fun1 f, void *ctx, int nodes, double alpha[4])
{
    or_project_fn_deg(f, ctx, nodes, 3, alpha);
}

typedef struct {
    double D, s, delta;
} gauss1_ctx;

/* the one-dimensional factor exp(-D (x - x_i)^2) with x = m + s t and
 * delta = m - x_i (eq. Gaussian2, written with D carried explicitly). */
static double gauss1(double t, void *vctx)
{
    const gauss1_ctx *g = (const gauss1_ctx *)vctx;
    double u = g->s * t + g->delta;
    return exp(-g->D * u * u);
}

/* Projection of the factor of atom coordinate xi on the interval [lo,hi],
 * series of degree n (1..3). */
void or_project_deg(double D, double lo, double hi, double xi, int nodes, int degree,
                    double alpha[4])
{
    gauss1_ctx g;
    g.D = D;
    g.s = 0.5 * (hi - lo);
    g.delta = 0.5 * (lo + hi) - xi;
    or_project_fn_deg(gauss1, &g, nodes, degree, alpha);
}

void or_project(double D, double lo, double hi, double xi, int nodes, double alpha[4])
{
    or_project_deg(D, lo, hi, xi, nodes, 3, alpha);
}

/* ------------------------------------------------------------------------ */
/* Atom bins: a superset enumerator for the neighbourhood predicates.         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const double *xyzr; /* [n][4] */
    double lo[3];       /* bin grid origin */
    double bs;          /* bin size */
    int64_t nb[3];
    int64_t *start;     /* [nbins+1] */
    int64_t *idx;       /* atom indices, bin-major, ascending inside a bin */
} or_bins;

static int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

static void bins_build(or_bins *b, const double *xyzr, int64_t n, double bs)
{
    b->n = n;
    b->xyzr = xyzr;
    b->bs = bs;
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        mn[a] = n ? xyzr[a] : 0.0;
        mx[a] = mn[a];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = xyzr[4 * i + a];
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    int64_t tot = 1;
    for (int a = 0; a < 3; ++a) {
        b->lo[a] = mn[a];
        b->nb[a] = (int64_t)floor((mx[a] - mn[a]) / bs) + 1;
        tot *= b->nb[a];
    }
    b->start = (int64_t *)calloc((size_t)tot + 1, sizeof(int64_t));
    b->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = clampi((int64_t)floor((xyzr[4 * i + a] - b->lo[a]) / bs), 0, b->nb[a] - 1);
        key[i] = (c[2] * b->nb[1] + c[1]) * b->nb[0] + c[0];
        b->start[key[i] + 1]++;
    }
    for (int64_t k = 0; k < tot; ++k)
        b->start[k + 1] += b->start[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)tot);
    memcpy(fill, b->start, sizeof(int64_t) * (size_t)tot);
    for (int64_t i = 0; i < n; ++i)
        b->idx[fill[key[i]]++] = i;
    free(fill);
    free(key);
}

static void bins_free(or_bins *b)
{
    free(b->start);
    free(b->idx);
}

/* Visit every atom whose bin overlaps the box [lo-R, hi+R]. */
#define BINS_FOREACH(b, blo, bhi, R, i_var, ...)                                          \
    do {                                                                                  \
        int64_t c0_[3], c1_[3];                                                           \
        for (int a_ = 0; a_ < 3; ++a_) {                                                  \
            c0_[a_] = clampi((int64_t)floor(((blo)[a_] - (R) - (b)->lo[a_]) / (b)->bs), 0, \
                             (b)->nb[a_] - 1);                                            \
            c1_[a_] = clampi((int64_t)floor(((bhi)[a_] + (R) - (b)->lo[a_]) / (b)->bs), 0, \
                             (b)->nb[a_] - 1);                                            \
        }                                                                                 \
        for (int64_t z_ = c0_[2]; z_ <= c1_[2]; ++z_)                                     \
            for (int64_t y_ = c0_[1]; y_ <= c1_[1]; ++y_)                                 \
                for (int64_t x_ = c0_[0]; x_ <= c1_[0]; ++x_) {                           \
                    int64_t k_ = (z_ * (b)->nb[1] + y_) * (b)->nb[0] + x_;                \
                    for (int64_t p_ = (b)->start[k_]; p_ < (b)->start[k_ + 1]; ++p_) {    \
                        int64_t i_var = (b)->idx[p_];                                     \
                        __VA_ARGS__                                                       \
                    }                                                                     \
                }                                                                         \
    } while (0)

/* Reading: the paper only says that the sum is taken over the atoms near the
 * cube (Section 2.2.1, after eq. polynew).  Here an atom belongs to the
 * neighbourhood of a closed box iff its squared distance to the box is at
 * most R_c^2 = r_max^2 + ln(1/eps_cut)/D, so every dropped term of phi is
 * below eps_cut.  A point is a box with lo = hi. */
static double box_dist2(const double *x, const double lo[3], const double hi[3])
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = 0.0;
        if (x[a] < lo[a]) d = lo[a] - x[a];
        else if (x[a] > hi[a]) d = x[a] - hi[a];
        d2 += d * d;
    }
    return d2;
}

double or_cutoff2(const double *xyzr, int64_t n, double D, double eps_cut)
{
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (xyzr[4 * i + 3] > rmax) rmax = xyzr[4 * i + 3];
    return rmax * rmax + log(1.0 / eps_cut) / D;
}

/* ------------------------------------------------------------------------ */
/* phi and its gradient (Section 1, eq. Gaussian1)                            */
/*   phi(p)  = sum_i exp(-D(|p-x_i|^2 - r_i^2))                               */
/*   grad(p) = sum_i -2D (p - x_i) exp(-D(|p-x_i|^2 - r_i^2))                 */
/* over the atoms with |p - x_i|^2 <= R_c^2.                                  */
/* ------------------------------------------------------------------------ */

static void phi_point(const or_bins *b, double D, double rc2, const double *p, double *phi,
                      double *grad)
{
    const double *xyzr = b->xyzr;
    double R = sqrt(rc2);
    double s = 0.0, g[3] = {0, 0, 0};
    BINS_FOREACH(b, p, p, R, i, {
        const double *x = xyzr + 4 * i;
        double d[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (d2 <= rc2) {
            double term = exp(-D * (d2 - x[3] * x[3]));
            s += term;
            for (int a = 0; a < 3; ++a)
                g[a] += -2.0 * D * d[a] * term;
        }
    });
    *phi = s;
    if (grad)
        for (int a = 0; a < 3; ++a)
            grad[a] = g[a];
}

void or_phi(const double *xyzr, int64_t n, double D, double eps_cut, const double *pts,
            int64_t m, double *phi, double *grad, int nthreads)
{
    double rc2 = or_cutoff2(xyzr, n, D, eps_cut);
    or_bins b;
    bins_build(&b, xyzr, n, sqrt(rc2));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t k = 0; k < m; ++k)
        phi_point(&b, D, rc2, pts + 3 * k, phi + k, grad ? grad + 3 * k : NULL);
    bins_free(&b);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of phi: derivative of eq. Gaussian1 with respect to the atom       */
/* centres and radii.  For weights wbar_p at points p,                        */
/*   out[i] = sum_p wbar_p d phi(p) / d(x_i, y_i, z_i, r_i)                   */
/*          = sum_p wbar_p term_ip (2D (p - x_i), 2D r_i),                    */
/*   term_ip = exp(-D(|p - x_i|^2 - r_i^2)),                                  */
/* over the pairs inside the cut-off.  Reading: the cut-off radius is a       */
/* truncation level, not part of the model, so it is held fixed (its own     */
/* derivative would only move terms below eps_cut).  Atom-major loop over a   */
/* bin grid of the points; each atom's sum is independent.                    */
/* ------------------------------------------------------------------------ */

void or_phi_adjoint(const double *xyzr, int64_t n, double D, double eps_cut, const double *pts,
                    int64_t m, const double *wbar, double *out, int nthreads)
{
    double rc2 = or_cutoff2(xyzr, n, D, eps_cut);
    double R = sqrt(rc2);
    /* points with their weights in the [m][4] layout the bin grid takes */
    double *pw = (double *)malloc(sizeof(double) * 4 * (size_t)(m ? m : 1));
    for (int64_t k = 0; k < m; ++k) {
        for (int a = 0; a < 3; ++a)
            pw[4 * k + a] = pts[3 * k + a];
        pw[4 * k + 3] = wbar[k];
    }
    or_bins b;
    bins_build(&b, pw, m, R);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const double *x = xyzr + 4 * i;
        double acc[4] = {0, 0, 0, 0};
        if (m > 0)
            BINS_FOREACH(&b, x, x, R, k, {
                const double *p = pw + 4 * k;
                double d[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
                double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (d2 <= rc2) {
                    double f = p[3] * exp(-D * (d2 - x[3] * x[3]));
                    for (int a = 0; a < 3; ++a)
                        acc[a] += f * 2.0 * D * d[a];
                    acc[3] += f * 2.0 * D * x[3];
                }
            });
        for (int a = 0; a < 4; ++a)
            out[4 * i + a] = acc[a];
    }
    bins_free(&b);
    free(pw);
}

/* ------------------------------------------------------------------------ */
/* Coefficient tensor of one cube (eqs. polynew, tensor1, tensor2)            */
/*   A[j][k][l] = sum_{i in N(Q)} exp(D r_i^2) a~x_j a~y_k a~z_l               */
/* j: x-degree, k: y-degree, l: z-degree; flat index 16 j + 4 k + l.          */
/* ------------------------------------------------------------------------ */

static int64_t cube_tensor(const or_bins *b, double D, double rc2, int nodes, int degree,
                           const double lo[3], const double hi[3], double A[64])
{
    const double *xyzr = b->xyzr;
    double R = sqrt(rc2);
    int64_t cnt = 0;
    for (int e = 0; e < 64; ++e)
        A[e] = 0.0;
    BINS_FOREACH(b, lo, hi, R, i, {
        const double *x = xyzr + 4 * i;
        if (box_dist2(x, lo, hi) <= rc2) {
            double ax[4], ay[4], az[4];
            or_project_deg(D, lo[0], hi[0], x[0], nodes, degree, ax);
            or_project_deg(D, lo[1], hi[1], x[1], nodes, degree, ay);
            or_project_deg(D, lo[2], hi[2], x[2], nodes, degree, az);
            double w = exp(D * x[3] * x[3]);
            for (int j = 0; j < 4; ++j)
                for (int k = 0; k < 4; ++k)
                    for (int l = 0; l < 4; ++l)
                        A[16 * j + 4 * k + l] += w * ax[j] * ay[k] * az[l];
            ++cnt;
        }
    });
    return cnt;
}

void or_cube_tensor(const double *xyzr, int64_t n, double D, double eps_cut, int nodes,
                    const double lo[3], const double hi[3], double A[64], int64_t *n_nb)
{
    double rc2 = or_cutoff2(xyzr, n, D, eps_cut);
    or_bins b;
    bins_build(&b, xyzr, n, sqrt(rc2));
    int64_t c = cube_tensor(&b, D, rc2, nodes, 3, lo, hi, A);
    if (n_nb) *n_nb = c;
    bins_free(&b);
}

/* Value of the tensor polynomial at local coordinates (eq. tensor1). */
double or_tensor_eval(const double A[64], double x, double y, double z)
{
    double Lx[4], Ly[4], Lz[4], s = 0.0;
    legendre4(x, Lx);
    legendre4(y, Ly);
    legendre4(z, Lz);
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l)
                s += A[16 * j + 4 * k + l] * Lx[j] * Ly[k] * Lz[l];
    return s;
}

/* The parent's polynomial written in the Legendre basis of one of its eight
 * children (eq. childtensor).  Child `octant` (bit 0: x, 1: y, 2: z; a set
 * bit is the upper half) covers parent coordinates u = (t + s) / 2 with
 * t in [-1,1] the child's coordinate and s = -1 or +1.  Along one axis the
 * child coefficients of a parent basis polynomial L_i are its Legendre
 * projection on the child,
 *   M[j][i] = (2j+1)/2 int_{-1}^{1} L_i((t + s)/2) L_j(t) dt,
 * computed by Gauss-Legendre quadrature with 8 nodes (exact: the integrand
 * has degree <= 6); then A'[j][k][l] = sum over (i, i', i'') of
 * Mx[j][i] My[k][i'] Mz[l][i''] A[i][i'][i''].  The child polynomial equals
 * the parent's on the child exactly (degree <= 3 both). */
void or_child_tensor(const double Ap[64], int octant, double Ac[64])
{
    const double *t, *w;
    gl_nodes(8, &t, &w);
    double M[3][4][4];
    for (int a = 0; a < 3; ++a) {
        const double s = ((octant >> a) & 1) ? 1.0 : -1.0;
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i) {
                double acc = 0.0;
                for (int q = 0; q < 8; ++q) {
                    double Lu[4], Lt[4];
                    legendre4(0.5 * (t[q] + s), Lu);
                    legendre4(t[q], Lt);
                    acc += w[q] * Lu[i] * Lt[j];
                }
                M[a][j][i] = 0.5 * (2.0 * j + 1.0) * acc;
            }
    }
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l) {
                double acc = 0.0;
                for (int i = 0; i < 4; ++i)
                    for (int i2 = 0; i2 < 4; ++i2)
                        for (int i3 = 0; i3 < 4; ++i3)
                            acc += M[0][j][i] * M[1][k][i2] * M[2][l][i3] *
                                   Ap[16 * i + 4 * i2 + i3];
                Ac[16 * j + 4 * k + l] = acc;
            }
}

/* Reading of Step 3's stopping rule (the coefficients beyond the linear
 * terms must fall under a user bound): the absolute l1 mass of the 56
 * entries with max(j,k,l) >= 2. */
double or_higher_mass(const double A[64])
{
    double e = 0.0;
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l)
                if (j >= 2 || k >= 2 || l >= 2)
                    e += fabs(A[16 * j + 4 * k + l]);
    return e;
}

/* ------------------------------------------------------------------------ */
/* Singular value decomposition of a small m x n matrix (m <= n <= 16) by     */
/* one-sided (Hestenes) Jacobi rotations on the columns of M^T.               */
/*   M = U diag(s) Vt, s descending; U is m x m, Vt is m x n (row-major).     */
/* ------------------------------------------------------------------------ */

void or_svd(int m, int n, const double *M, double *s, double *U, double *Vt)
{
    double B[16][16]; /* B = M^T, n x m: column q of B is row q of M */
    double W[16][16]; /* accumulated rotations, m x m */
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < m; ++q)
            B[i][q] = M[q * n + i];
    for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q)
            W[p][q] = (p == q) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 80; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < n; ++i) {
                    al += B[i][p] * B[i][p];
                    be += B[i][q] * B[i][q];
                    ga += B[i][p] * B[i][q];
                }
                if (ga == 0.0 || fabs(ga) <= 1e-16 * sqrt(al * be))
                    continue;
                rotated = 1;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < n; ++i) {
                    double bp = B[i][p], bq = B[i][q];
                    B[i][p] = cs * bp - sn * bq;
                    B[i][q] = sn * bp + cs * bq;
                }
                for (int i = 0; i < m; ++i) {
                    double wp = W[i][p], wq = W[i][q];
                    W[i][p] = cs * wp - sn * wq;
                    W[i][q] = sn * wp + cs * wq;
                }
            }
        if (!rotated)
            break;
    }
    /* M^T W = B has orthogonal columns; with sigma_q = |B_q| and
     * v_q = B_q / sigma_q this gives M = W diag(sigma) V^T. */
    double sig[16];
    int ord[16];
    for (int q = 0; q < m; ++q) {
        double nn = 0.0;
        for (int i = 0; i < n; ++i)
            nn += B[i][q] * B[i][q];
        sig[q] = sqrt(nn);
        ord[q] = q;
    }
    for (int a = 0; a < m; ++a) /* selection sort, descending */
        for (int b2 = a + 1; b2 < m; ++b2)
            if (sig[ord[b2]] > sig[ord[a]]) {
                int t = ord[a];
                ord[a] = ord[b2];
                ord[b2] = t;
            }
    for (int a = 0; a < m; ++a) {
        int q = ord[a];
        s[a] = sig[q];
        for (int i = 0; i < m; ++i)
            U[i * m + a] = W[i][q];
        for (int i = 0; i < n; ++i)
            Vt[a * n + i] = sig[q] > 0.0 ? B[i][q] / sig[q] : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Range of a one-dimensional degree-3 Legendre series on [-1,1].             */
/* Reading: the paper asks for the lower and upper bounds of the cubics       */
/* (Section 2.2.2) without saying how; the exact extremes are taken, over     */
/* the end points and the real critical points inside the interval.           */
/* ------------------------------------------------------------------------ */

static double series_eval(const double q[4], double t)
{
    double L[4];
    legendre4(t, L);
    return q[0] * L[0] + q[1] * L[1] + q[2] * L[2] + q[3] * L[3];
}

void or_cubic_range(const double q[4], double *lo, double *hi)
{
    /* derivative of q0 + q1 t + q2 (3t^2-1)/2 + q3 (5t^3-3t)/2:
     * (15/2 q3) t^2 + 3 q2 t + (q1 - 3/2 q3) */
    double a = 7.5 * q[3], b = 3.0 * q[2], c = q[1] - 1.5 * q[3];
    double cand[4];
    int nc = 0;
    cand[nc++] = -1.0;
    cand[nc++] = 1.0;
    if (a == 0.0) {
        if (b != 0.0) cand[nc++] = -c / b;
    } else {
        double disc = b * b - 4.0 * a * c;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double qq = -0.5 * (b + (b >= 0.0 ? sq : -sq));
            if (qq != 0.0) {
                cand[nc++] = qq / a;
                cand[nc++] = c / qq;
            } else {
                cand[nc++] = 0.0; /* b = 0 and disc = 0: double root at 0 */
            }
        }
    }
    double mn = series_eval(q, -1.0), mx = mn;
    for (int i = 0; i < nc; ++i) {
        double t = cand[i];
        if (!(t >= -1.0 && t <= 1.0))
            continue;
        double v = series_eval(q, t);
        if (v < mn) mn = v;
        if (v > mx) mx = v;
    }
    *lo = mn;
    *hi = mx;
}

static void interval_mul(double a0, double a1, double b0, double b1, double *lo, double *hi)
{
    double p[4] = {a1 * b1, a1 * b0, a0 * b1, a0 * b0};
    double mn = p[0], mx = p[0];
    for (int i = 1; i < 4; ++i) {
        if (p[i] < mn) mn = p[i];
        if (p[i] > mx) mx = p[i];
    }
    *lo = mn;
    *hi = mx;
}

/* Smallest r with sum_{i<=r} s_i >= 0.99 sum_{i<=4} s_i (eq. SVD3 and its
 * inner counterpart); 0 when every s_i is zero.  *margin receives the
 * relative distance of that decision from a tie. */
static int rank99(const double s[4], double *margin)
{
    double tot = s[0] + s[1] + s[2] + s[3];
    *margin = 1.0;
    if (!(tot > 0.0))
        return 0;
    double target = 0.99 * tot, cum = 0.0;
    int r = 4;
    for (int i = 0; i < 4; ++i) {
        double prev = cum;
        cum += s[i];
        if (cum >= target) {
            r = i + 1;
            double m1 = (cum - target) / tot;
            double m0 = (i > 0) ? (target - prev) / tot : 1.0;
            *margin = m1 < m0 ? m1 : m0;
            break;
        }
    }
    return r;
}

/* ------------------------------------------------------------------------ */
/* Lower and upper bound of the tensor polynomial on its cube                 */
/* (Section 2.2.2: eqs. matrix1, SVD1..SVD7, poly5..poly7, Sxyz, bound1..3).  */
/*                                                                            */
/* Reading (unfolding): the rows of the 4 x 16 unfolding carry the x-degree   */
/* j and the columns the pair (k,l) as 4k+l, so that u_i multiplies the       */
/* x-Legendre vector as in eq. Sxyz; V_i[k][l] = v_i[4k+l].                   */
/* Reading (residual): |T| <= sum |R_ijk| (the form eqs. bound2/3 use).       */
/*                                                                            */
/* out[0] = L, out[1] = U, out[2] = rho (residual l1 mass), out[3] = outer    */
/* rank r, out[4] = smallest decision margin of the rank rules and singular   */
/* value gaps that shape the main part (a near-tie indicator).                */
/* ------------------------------------------------------------------------ */

void or_bound(const double A[64], double out[5])
{
    double sig[4], U[16], Vt[64];
    or_svd(4, 16, A, sig, U, Vt);
    double tie = 1.0, mr;
    int r = rank99(sig, &mr);
    if (mr < tie) tie = mr;
    for (int i = 0; i < r; ++i) {
        double g = (sig[0] > 0.0) ? (sig[i] - (i + 1 < 4 ? sig[i + 1] : 0.0)) / sig[0] : 1.0;
        if (i + 1 < 4 && g < tie) tie = g;
    }

    double At[64];
    for (int e = 0; e < 64; ++e)
        At[e] = 0.0;
    double Msum = 0.0, msum = 0.0;
    for (int i = 0; i < r; ++i) {
        double Vi[16], d[4], Wi[16], Zt[16];
        for (int e = 0; e < 16; ++e)
            Vi[e] = Vt[i * 16 + e];
        or_svd(4, 4, Vi, d, Wi, Zt);
        double mi;
        int ri = rank99(d, &mi);
        if (mi < tie) tie = mi;
        for (int k = 0; k < ri; ++k) {
            double g = (d[0] > 0.0) ? (d[k] - (k + 1 < 4 ? d[k + 1] : 0.0)) / d[0] : 1.0;
            if (k + 1 < 4 && g < tie) tie = g;
        }
        double u[4];
        for (int j = 0; j < 4; ++j)
            u[j] = U[j * 4 + i];
        double Myz = 0.0, myz = 0.0;
        for (int k = 0; k < ri; ++k) {
            double w[4], z[4];
            for (int a = 0; a < 4; ++a) {
                w[a] = Wi[a * 4 + k];
                z[a] = Zt[k * 4 + a];
            }
            /* main part: sigma_i u_i (x) d_k w_k (x) z_k  (eq. SVD7) */
            for (int j = 0; j < 4; ++j)
                for (int kk = 0; kk < 4; ++kk)
                    for (int l = 0; l < 4; ++l)
                        At[16 * j + 4 * kk + l] += sig[i] * u[j] * d[k] * w[kk] * z[l];
            double wy0, wy1, zz0, zz1, p0, p1;
            or_cubic_range(w, &wy0, &wy1);
            or_cubic_range(z, &zz0, &zz1);
            interval_mul(wy0, wy1, zz0, zz1, &p0, &p1); /* m_k^yz, M_k^yz */
            Myz += d[k] * p1;
            myz += d[k] * p0;
        }
        double ux0, ux1, q0, q1;
        or_cubic_range(u, &ux0, &ux1);
        interval_mul(ux0, ux1, myz, Myz, &q0, &q1); /* m_i, M_i */
        Msum += sig[i] * q1;
        msum += sig[i] * q0;
    }
    double rho = 0.0;
    for (int e = 0; e < 64; ++e)
        rho += fabs(A[e] - At[e]);
    out[0] = msum - rho; /* eq. bound3 */
    out[1] = Msum + rho; /* eq. bound2 */
    out[2] = rho;
    out[3] = (double)r;
    out[4] = tie;
}

/* ------------------------------------------------------------------------ */
/* Adaptive partition and estimation (Section 2.2, Steps 1-3), leaf           */
/* classification against the trilinear interpolant (eq. linear1) and the    */
/* edge intersection points (eq. intersection).                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n_leaves;
    int32_t *ijk;       /* [n_leaves][3] cube index at its level */
    uint8_t *level;     /* [n_leaves] */
    uint8_t *reason;    /* [n_leaves] OR_REASON_* */
    uint8_t *mask;      /* [n_leaves] bit v = dx + 2 dy + 4 dz set iff phi >= c */
    uint8_t *cls;       /* [n_leaves] OR_CLS_* */
    double *corner_phi; /* [n_leaves][8] */
    int64_t n_vert;
    uint64_t *vkey;     /* [n_vert] */
    double *vt;         /* [n_vert] */
    double *vxyz;       /* [n_vert][3] */
    double origin[3];
    int64_t dims[3];
    int32_t K;
    int32_t status;     /* 0 ok, <0 invalid input */
    double rc2;
    int64_t n_est[OR_MAXLEV], n_disc[OR_MAXLEV], n_refine[OR_MAXLEV];
    int64_t n_conv[OR_MAXLEV], n_hmin[OR_MAXLEV];
    int64_t n_pairs;      /* cube-atom pairs inside the cut-off */
    int64_t n_corners;    /* unique leaf corners */
    int64_t tie_cube;     /* cube decisions with a margin below OR_TIE */
    int64_t tie_corner;   /* corner signs with |phi-c|/c below OR_TIE */
    int64_t n_tie_list;   /* entries used in tie_list */
    int32_t tie_list[4 * OR_TIE_LIST]; /* (level, ix, iy, iz) of near-tie cubes */
    uint64_t tie_corner_keys[OR_TIE_LIST]; /* finest-lattice keys of near-tie corners */
} or_result;

static int is_pow2_ratio(double a, double b, int *k)
{
    double r = a / b;
    for (int i = 0; i < OR_MAXLEV; ++i)
        if (r == (double)(1 << i)) {
            *k = i;
            return 1;
        }
    return 0;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static const uint64_t *sort_keys_ctx;
static int cmp_by_key(const void *a, const void *b)
{
    uint64_t x = sort_keys_ctx[*(const int64_t *)a], y = sort_keys_ctx[*(const int64_t *)b];
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int64_t find_u64(const uint64_t *v, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (v[mid] == key) return mid;
        if (v[mid] < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* lattice point key: finest-lattice coordinates, 16 bits each */
static uint64_t point_key(int64_t X, int64_t Y, int64_t Z)
{
    return ((uint64_t)X << 32) | ((uint64_t)Y << 16) | (uint64_t)Z;
}

/* edge key: conf(11) | level(3) | axis(2) | X(16) | Y(16) | Z(16), X,Y,Z the
 * finest-lattice coordinates of the edge's lower end */
static uint64_t edge_key(int conf, int level, int axis, int64_t X, int64_t Y, int64_t Z)
{
    return ((uint64_t)conf << 53) | ((uint64_t)level << 50) | ((uint64_t)axis << 48) |
           ((uint64_t)X << 32) | ((uint64_t)Y << 16) | (uint64_t)Z;
}

void or_free(or_result *r)
{
    if (!r) return;
    free(r->ijk);
    free(r->level);
    free(r->reason);
    free(r->mask);
    free(r->cls);
    free(r->corner_phi);
    free(r->vkey);
    free(r->vt);
    free(r->vxyz);
    free(r);
}

typedef struct {
    int32_t i[3];
} cube3;

/* Edge intersection points (eq. intersection) of the SURFACE leaves of R
 * (ijk, level, mask, cls and corner values filled in), into R's vertex
 * arrays.  hmin: the finest lattice spacing (the unit of the edge keys). */
static void or_extract_edges(or_result *R, double c, double h0, double hmin, int conf)
{
    const int64_t nl = R->n_leaves;
    /* ---- edge intersections (eq. intersection) ----------------------------
     * g restricted to a cube edge is linear in the edge coordinate, so the
     * root of g = c on an edge whose end signs differ is
     * t = (c - phi0) / (phi1 - phi0), measured from the lower end.  Edges are
     * visited leaf by leaf (leaf order), edge by edge (axis-major; inside an
     * axis the two other offsets with the lower axis first); an edge key that
     * was already emitted is skipped.  The list is finally sorted by key. */
    int64_t vcap = 1024, nv = 0;
    R->vkey = (uint64_t *)malloc(sizeof(uint64_t) * vcap);
    R->vt = (double *)malloc(sizeof(double) * vcap);
    R->vxyz = (double *)malloc(sizeof(double) * 3 * vcap);
    /* seen-set: open addressing on the edge key */
    int64_t hcap = 1024;
    while (hcap < 24 * (nl + 1)) hcap *= 2;
    uint64_t *hset = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)hcap);
    for (int64_t i = 0; i < hcap; ++i)
        hset[i] = ~(uint64_t)0;
    for (int64_t q = 0; q < nl; ++q) {
        if (R->cls[q] != OR_CLS_SURFACE) continue;
        int lev = R->level[q], sh = R->K - lev;
        double h = h0 / (double)(1 << lev);
        for (int axis = 0; axis < 3; ++axis)
            for (int ab = 0; ab < 4; ++ab) {
                int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
                int lowo = o1 < o2 ? o1 : o2, higho = o1 < o2 ? o2 : o1;
                int off[3] = {0, 0, 0};
                off[lowo] = ab & 1;
                off[higho] = (ab >> 1) & 1;
                int v0 = off[0] + 2 * off[1] + 4 * off[2];
                int v1 = v0 + (1 << axis);
                int b0 = (R->mask[q] >> v0) & 1, b1 = (R->mask[q] >> v1) & 1;
                if (b0 == b1) continue;
                int64_t X = ((int64_t)R->ijk[3 * q + 0] + off[0]) << sh;
                int64_t Y = ((int64_t)R->ijk[3 * q + 1] + off[1]) << sh;
                int64_t Z = ((int64_t)R->ijk[3 * q + 2] + off[2]) << sh;
                uint64_t key = edge_key(conf, lev, axis, X, Y, Z);
                uint64_t hsh = key * 0x9E3779B97F4A7C15ull;
                int64_t slot = (int64_t)(hsh >> 17) & (hcap - 1);
                int found = 0;
                while (hset[slot] != ~(uint64_t)0) {
                    if (hset[slot] == key) { found = 1; break; }
                    slot = (slot + 1) & (hcap - 1);
                }
                if (found) continue;
                hset[slot] = key;
                double f0 = R->corner_phi[8 * q + v0], f1 = R->corner_phi[8 * q + v1];
                double t = (c - f0) / (f1 - f0);
                if (nv == vcap) {
                    vcap *= 2;
                    R->vkey = (uint64_t *)realloc(R->vkey, sizeof(uint64_t) * vcap);
                    R->vt = (double *)realloc(R->vt, sizeof(double) * vcap);
                    R->vxyz = (double *)realloc(R->vxyz, sizeof(double) * 3 * vcap);
                }
                R->vkey[nv] = key;
                R->vt[nv] = t;
                double p0[3] = {R->origin[0] + (double)X * hmin, R->origin[1] + (double)Y * hmin,
                                R->origin[2] + (double)Z * hmin};
                p0[axis] += t * h;
                for (int a = 0; a < 3; ++a)
                    R->vxyz[3 * nv + a] = p0[a];
                ++nv;
            }
    }
    free(hset);
    R->n_vert = nv;
    /* canonical order of the vertex list: ascending edge key */
    {
        int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv ? nv : 1));
        for (int64_t i = 0; i < nv; ++i)
            ord[i] = i;
        sort_keys_ctx = R->vkey;
        qsort(ord, (size_t)nv, sizeof(int64_t), cmp_by_key);
        uint64_t *k2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nv ? nv : 1));
        double *t2 = (double *)malloc(sizeof(double) * (size_t)(nv ? nv : 1));
        double *x2 = (double *)malloc(sizeof(double) * 3 * (size_t)(nv ? nv : 1));
        for (int64_t i = 0; i < nv; ++i) {
            k2[i] = R->vkey[ord[i]];
            t2[i] = R->vt[ord[i]];
            for (int a = 0; a < 3; ++a)
                x2[3 * i + a] = R->vxyz[3 * ord[i] + a];
        }
        free(R->vkey);
        free(R->vt);
        free(R->vxyz);
        R->vkey = k2;
        R->vt = t2;
        R->vxyz = x2;
        free(ord);
    }
}

or_result *or_partition(const double *xyzr, int64_t n, const or_params *P)
{
    or_result *R = (or_result *)calloc(1, sizeof(or_result));
    int K = 0;
    if (!(P->D > 0) || !(P->c > 0) || !(P->h0 > 0) || !(P->h_min > 0) || !(P->eps_cut > 0) ||
        !(P->eps_cut < 1) || !(P->pad >= 0) || n < 0 || P->degree < 0 || P->degree > 3 ||
        (P->reexpand != 0 && P->reexpand != 1) ||
        (!P->uniform && (!(P->tau > 0) || !is_pow2_ratio(P->h0, P->h_min, &K)))) {
        R->status = -1;
        return R;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 4; ++a)
            if (!isfinite(xyzr[4 * i + a]) || (a == 3 && !(xyzr[4 * i + 3] > 0))) {
                R->status = -1;
                return R;
            }
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    if (P->uniform) K = 0;
    R->K = K;
    const double D = P->D, c = P->c, h0 = P->h0;
    const int nodes = P->gl_nodes > 0 ? P->gl_nodes : 32;
    const int degree = P->degree > 0 ? P->degree : 3;
    const int reexpand = P->reexpand;

    /* Initial coarse grid (Section 2.2): reading -- the origin is snapped to
     * a multiple of h0 below the padded atom box, and the grid covers the
     * padded box. */
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        mn[a] = n ? xyzr[a] : 0.0;
        mx[a] = mn[a];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = xyzr[4 * i + a];
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    for (int a = 0; a < 3; ++a) {
        R->origin[a] = h0 * floor((mn[a] - P->pad) / h0);
        R->dims[a] = (int64_t)ceil((mx[a] + P->pad - R->origin[a]) / h0);
        if (R->dims[a] < 1) R->dims[a] = 1;
        if ((R->dims[a] << K) > 65535) {
            R->status = -2;
            return R;
        }
    }
    double rc2 = or_cutoff2(xyzr, n, D, P->eps_cut);
    R->rc2 = rc2;
    double Rc = sqrt(rc2);
    or_bins bins;
    bins_build(&bins, xyzr, n, Rc);

    /* ---- leaves --------------------------------------------------------- */
    int64_t cap = 1024, nl = 0;
    cube3 *lijk = (cube3 *)malloc(sizeof(cube3) * cap);
    uint8_t *llev = (uint8_t *)malloc(cap), *lrea = (uint8_t *)malloc(cap);
#define PUSH_LEAF(I0, I1, I2, LEV, REA)                                   \
    do {                                                                  \
        if (nl == cap) {                                                  \
            cap *= 2;                                                     \
            lijk = (cube3 *)realloc(lijk, sizeof(cube3) * cap);           \
            llev = (uint8_t *)realloc(llev, cap);                         \
            lrea = (uint8_t *)realloc(lrea, cap);                         \
        }                                                                 \
        lijk[nl].i[0] = (I0); lijk[nl].i[1] = (I1); lijk[nl].i[2] = (I2); \
        llev[nl] = (uint8_t)(LEV); lrea[nl] = (uint8_t)(REA);             \
        ++nl;                                                             \
    } while (0)

    if (P->uniform) {
        for (int64_t z = 0; z < R->dims[2]; ++z)
            for (int64_t y = 0; y < R->dims[1]; ++y)
                for (int64_t x = 0; x < R->dims[0]; ++x)
                    PUSH_LEAF((int32_t)x, (int32_t)y, (int32_t)z, 0, OR_REASON_UNIFORM);
    } else {
        /* Q_0: the root cubes in raster order (x fastest) whose neighbourhood
         * holds at least one atom; an empty neighbourhood gives A = 0 and
         * the bound [0,0], which excludes c > 0, so such a root is dropped
         * without being estimated. */
        int64_t nroot = R->dims[0] * R->dims[1] * R->dims[2];
        uint8_t *occ = (uint8_t *)calloc((size_t)nroot, 1);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
        for (int64_t k = 0; k < nroot; ++k) {
            int64_t x = k % R->dims[0], y = (k / R->dims[0]) % R->dims[1],
                    z = k / (R->dims[0] * R->dims[1]);
            double lo[3] = {R->origin[0] + x * h0, R->origin[1] + y * h0, R->origin[2] + z * h0};
            double hi[3] = {lo[0] + h0, lo[1] + h0, lo[2] + h0};
            int hit = 0;
            BINS_FOREACH(&bins, lo, hi, Rc, i, {
                if (!hit && box_dist2(xyzr + 4 * i, lo, hi) <= rc2) hit = 1;
            });
            occ[k] = (uint8_t)hit;
        }
        int64_t nq = 0, qcap = 1024;
        cube3 *Q = (cube3 *)malloc(sizeof(cube3) * qcap);
        for (int64_t k = 0; k < nroot; ++k)
            if (occ[k]) {
                if (nq == qcap) {
                    qcap *= 2;
                    Q = (cube3 *)realloc(Q, sizeof(cube3) * qcap);
                }
                Q[nq].i[0] = (int32_t)(k % R->dims[0]);
                Q[nq].i[1] = (int32_t)((k / R->dims[0]) % R->dims[1]);
                Q[nq].i[2] = (int32_t)(k / (R->dims[0] * R->dims[1]));
                ++nq;
            }
        free(occ);

        /* with re-expansion: the tensors of the previous level's queue, and
         * for each cube of the current queue its parent and octant */
        double *Aprev = NULL;
        int64_t *par = NULL;
        uint8_t *oct = NULL;
        for (int lev = 0; lev <= K; ++lev) {
            double h = h0 / (double)(1 << lev);
            R->n_est[lev] = nq;
            /* decision per cube: 0 discard, 1 refine, 2 converged leaf, 3 h_min leaf */
            uint8_t *dec = (uint8_t *)malloc((size_t)(nq ? nq : 1));
            double *Acur = reexpand ? (double *)malloc(sizeof(double) * 64 * (size_t)(nq ? nq : 1))
                                    : NULL;
            int64_t pairs = 0, ties = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pairs, ties)
#endif
            for (int64_t q = 0; q < nq; ++q) {
                double lo[3], hi[3], A[64];
                for (int a = 0; a < 3; ++a) {
                    lo[a] = R->origin[a] + Q[q].i[a] * h;
                    hi[a] = lo[a] + h;
                }
                /* Step 1: the tensor polynomial of the cube -- projected from
                 * the atoms, or (re-expansion, below the roots) the parent's
                 * polynomial in the child's basis (eq. childtensor) */
                if (reexpand && lev >= 1)
                    or_child_tensor(Aprev + 64 * par[q], oct[q], A);
                else
                    pairs += cube_tensor(&bins, D, rc2, nodes, degree, lo, hi, A);
                if (Acur) memcpy(Acur + 64 * q, A, sizeof(double) * 64);
                double E = or_higher_mass(A);
                double tie = 1.0;
                /* Step 3 for a child cube: higher-order mass under the
                 * user bound -> trilinear leaf (2E bounds |P - g|). */
                if (lev >= 1) {
                    double m = fabs(2.0 * E - P->tau) / P->tau;
                    if (m < tie) tie = m;
                }
                if (lev >= 1 && 2.0 * E <= P->tau) {
                    dec[q] = 2;
                } else {
                    /* Step 2: keep the cube iff L <= c <= U */
                    double b[5];
                    or_bound(A, b);
                    double scale = 0.0;
                    for (int e = 0; e < 64; ++e)
                        scale += fabs(A[e]);
                    if (scale > 0.0) {
                        double m = fmin(fabs(b[0] - c), fabs(b[1] - c)) / scale;
                        if (m < tie) tie = m;
                        if (b[4] < tie) tie = b[4];
                    }
                    if (c < b[0] || c > b[1]) dec[q] = 0;
                    else if (lev == K) dec[q] = 3;
                    else dec[q] = 1;
                }
                if (tie < OR_TIE) {
                    ++ties;
#ifdef _OPENMP
#pragma omp critical(or_tie)
#endif
                    {
                        if (R->n_tie_list < OR_TIE_LIST) {
                            int32_t *t4 = R->tie_list + 4 * R->n_tie_list++;
                            t4[0] = lev;
                            t4[1] = Q[q].i[0];
                            t4[2] = Q[q].i[1];
                            t4[3] = Q[q].i[2];
                        }
                    }
                }
            }
            R->n_pairs += pairs;
            R->tie_cube += ties;
            /* ordered compaction: leaves in queue order, children of each
             * refined cube in octant order (bit 0: x, bit 1: y, bit 2: z) */
            int64_t nn = 0;
            for (int64_t q = 0; q < nq; ++q) {
                if (dec[q] == 0) R->n_disc[lev]++;
                else if (dec[q] == 1) { R->n_refine[lev]++; nn += 8; }
                else if (dec[q] == 2) { R->n_conv[lev]++; PUSH_LEAF(Q[q].i[0], Q[q].i[1], Q[q].i[2], lev, OR_REASON_CONVERGED); }
                else { R->n_hmin[lev]++; PUSH_LEAF(Q[q].i[0], Q[q].i[1], Q[q].i[2], lev, OR_REASON_HMIN); }
            }
            cube3 *Qn = (cube3 *)malloc(sizeof(cube3) * (size_t)(nn ? nn : 1));
            int64_t *parn = reexpand ? (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn ? nn : 1)) : NULL;
            uint8_t *octn = reexpand ? (uint8_t *)malloc((size_t)(nn ? nn : 1)) : NULL;
            int64_t w = 0;
            for (int64_t q = 0; q < nq; ++q)
                if (dec[q] == 1)
                    for (int o = 0; o < 8; ++o) {
                        Qn[w].i[0] = 2 * Q[q].i[0] + (o & 1);
                        Qn[w].i[1] = 2 * Q[q].i[1] + ((o >> 1) & 1);
                        Qn[w].i[2] = 2 * Q[q].i[2] + ((o >> 2) & 1);
                        if (reexpand) {
                            parn[w] = q;
                            octn[w] = (uint8_t)o;
                        }
                        ++w;
                    }
            free(dec);
            free(Q);
            free(Aprev);
            free(par);
            free(oct);
            Aprev = Acur;
            par = parn;
            oct = octn;
            Q = Qn;
            nq = nn;
        }
        free(Aprev);
        free(par);
        free(oct);
        free(Q);
    }

    /* ---- corners: phi once per unique finest-lattice point --------------- */
    R->n_leaves = nl;
    R->ijk = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(nl ? nl : 1));
    R->level = llev;
    R->reason = lrea;
    for (int64_t q = 0; q < nl; ++q)
        for (int a = 0; a < 3; ++a)
            R->ijk[3 * q + a] = lijk[q].i[a];
    free(lijk);
    R->mask = (uint8_t *)malloc((size_t)(nl ? nl : 1));
    R->cls = (uint8_t *)malloc((size_t)(nl ? nl : 1));
    R->corner_phi = (double *)malloc(sizeof(double) * 8 * (size_t)(nl ? nl : 1));
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * 8 * (size_t)(nl ? nl : 1));
    for (int64_t q = 0; q < nl; ++q) {
        int sh = K - R->level[q];
        for (int v = 0; v < 8; ++v) {
            int64_t X = ((int64_t)R->ijk[3 * q + 0] + (v & 1)) << sh;
            int64_t Y = ((int64_t)R->ijk[3 * q + 1] + ((v >> 1) & 1)) << sh;
            int64_t Z = ((int64_t)R->ijk[3 * q + 2] + ((v >> 2) & 1)) << sh;
            keys[8 * q + v] = point_key(X, Y, Z);
        }
    }
    int64_t nk = 8 * nl;
    uint64_t *uk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nk ? nk : 1));
    memcpy(uk, keys, sizeof(uint64_t) * (size_t)nk);
    qsort(uk, (size_t)nk, sizeof(uint64_t), cmp_u64);
    int64_t nu = 0;
    for (int64_t i = 0; i < nk; ++i)
        if (i == 0 || uk[i] != uk[i - 1]) uk[nu++] = uk[i];
    R->n_corners = nu;
    double *uphi = (double *)malloc(sizeof(double) * (size_t)(nu ? nu : 1));
    double hmin = P->uniform ? h0 : P->h_min;
    int64_t cties = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < nu; ++i) {
        double p[3] = {R->origin[0] + (double)(int64_t)((uk[i] >> 32) & 0xFFFF) * hmin,
                       R->origin[1] + (double)(int64_t)((uk[i] >> 16) & 0xFFFF) * hmin,
                       R->origin[2] + (double)(int64_t)(uk[i] & 0xFFFF) * hmin};
        phi_point(&bins, D, rc2, p, uphi + i, NULL);
    }
    for (int64_t i = 0; i < nu; ++i)
        if (fabs(uphi[i] - c) / c < OR_TIE) {
            if (cties < OR_TIE_LIST) R->tie_corner_keys[cties] = uk[i];
            ++cties;
        }
    R->tie_corner = cties;
    /* classification against c through the sign pattern of the trilinear
     * interpolant's corner values (eq. linear1): g is a convex combination
     * of the corner values, so g = c meets the closed cube iff
     * min <= c <= max over the corners. */
    for (int64_t q = 0; q < nl; ++q) {
        uint8_t m = 0;
        for (int v = 0; v < 8; ++v) {
            int64_t u = find_u64(uk, nu, keys[8 * q + v]);
            double f = uphi[u];
            R->corner_phi[8 * q + v] = f;
            if (f >= c) m |= (uint8_t)(1u << v);
        }
        R->mask[q] = m;
        R->cls[q] = (m == 0) ? OR_CLS_OUTSIDE : (m == 0xFF ? OR_CLS_INSIDE : OR_CLS_SURFACE);
    }
    free(uphi);
    free(uk);
    free(keys);

    or_extract_edges(R, c, h0, hmin, P->conf);
    bins_free(&bins);
    return R;
#undef PUSH_LEAF
}

/* ------------------------------------------------------------------------ */
/* Stage 2 points of a leaf's trilinear surface g = c (Section 2.3).          */
/*                                                                            */
/* The leaf is mapped to [-1,1]^3 as in eq. linear1; corner v = dx + 2dy +    */
/* 4dz sits at (2dx - 1, 2dy - 1, 2dz - 1) and holds the value f[v].          */
/*                                                                            */
/*  - extreme points on the face alpha = a (eq. curve): g = c, alpha = a and  */
/*    dg/dalpha = 0, alpha in {x, y, z}, a in {-1, 1};                        */
/*  - fold curves along alpha (eq. fold1): g = c and dg/dalpha = 0.  g is     */
/*    linear in alpha, so dg/dalpha does not depend on alpha and, where it    */
/*    vanishes, neither does g: the fold curve is a set of full segments      */
/*    parallel to the alpha axis, each joining an extreme point of the face   */
/*    alpha = -1 to one of the face alpha = +1 (the paper's remark that the   */
/*    trilinear fold curves are straight segments ending at extreme points);  */
/*  - critical points (eq. critical): g = c, dg/dalpha = 0, dg/dbeta = 0 for  */
/*    a pair alpha != beta.                                                   */
/*                                                                            */
/* Reading: only SURFACE leaves are processed (the corner values straddle c,  */
/* so g = c meets the closed cube); points on the boundary of the closed      */
/* cube count.  A configuration with infinitely many solutions (g constant    */
/* along alpha, or the two equations sharing a factor) is reported as         */
/* degenerate and contributes no points.                                       */
/*                                                                            */
/* Each record: kind 0 = fold segment along `axis` (its lower end, the        */
/* extreme point on the face axis = -1, is stored; the upper end, on the face */
/* axis = +1, is the same point moved by the cube edge along the axis), kind  */
/* 1 = critical point of the pair of axes other than `axis`.  Solutions of    */
/* one (kind, axis) are numbered by `root` in ascending order of their first  */
/* free coordinate (fold: the lower of the two other axes; critical: the      */
/* coordinate along `axis`).                                                  */
/* ------------------------------------------------------------------------ */

#define OR_S2_MAX 12

typedef struct {
    int32_t leaf;
    uint8_t kind, axis, root, pad;
    double p[3];
} or_s2pt;

/* bilinear function on [-1,1]^2 from its corner values F[k] at
 * (2(k&1) - 1, 2(k>>1) - 1): b[0] + b[1] u + b[2] v + b[3] u v */
static void bilinear_coeffs(const double F[4], double b[4])
{
    b[0] = (F[0] + F[1] + F[2] + F[3]) / 4.0;
    b[1] = (-F[0] + F[1] - F[2] + F[3]) / 4.0;
    b[2] = (-F[0] - F[1] + F[2] + F[3]) / 4.0;
    b[3] = (F[0] - F[1] - F[2] + F[3]) / 4.0;
}

/* Real roots of q0 + q1 t + q2 t^2 (ascending); returns their number, or -1
 * when every coefficient is zero.  *dmargin receives the relative distance
 * of the discriminant from zero (1 when linear or constant). */
static int quad_roots(double q0, double q1, double q2, double t[2], double *dmargin)
{
    *dmargin = 1.0;
    if (q2 == 0.0) {
        if (q1 == 0.0) return (q0 == 0.0) ? -1 : 0;
        t[0] = -q0 / q1;
        return 1;
    }
    double disc = q1 * q1 - 4.0 * q2 * q0;
    double den = q1 * q1 + 4.0 * fabs(q2 * q0);
    if (den > 0.0) *dmargin = fabs(disc) / den;
    if (disc < 0.0) return 0;
    if (disc == 0.0) {
        t[0] = -q1 / (2.0 * q2);
        return 1;
    }
    double sq = sqrt(disc);
    double q = -0.5 * (q1 + (q1 >= 0.0 ? sq : -sq));
    double a = q / q2, b = (q != 0.0) ? q0 / q : a;
    t[0] = a < b ? a : b;
    t[1] = a < b ? b : a;
    return 2;
}

static double range_margin(double u)
{
    return fmin(fabs(u - 1.0), fabs(u + 1.0));
}

/* Whether two linear functions p0 + p1 t and q0 + q1 t have a common real
 * zero (both identically zero included). */
static int linear_common_zero(double p0, double p1, double q0, double q1)
{
    if (p1 == 0.0 && q1 == 0.0) return p0 == 0.0 && q0 == 0.0;
    return p0 * q1 - p1 * q0 == 0.0;
}

/* Extreme points of g = c on the face axis = a (eq. curve) in the local
 * coordinates (u, v) of the two other axes (u the lower axis).  Returns the
 * number of points (ascending u), or -1 when the equations have infinitely
 * many real solutions (degenerate). */
static int face_extremes(const double f[8], double c, int axis, int a, double uv[2][2],
                         double *margin)
{
    int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
    int ax_u = o1 < o2 ? o1 : o2, ax_v = o1 < o2 ? o2 : o1;
    double FG[4], FH[4];
    for (int k = 0; k < 4; ++k) {
        int d[3] = {0, 0, 0};
        d[ax_u] = k & 1;
        d[ax_v] = k >> 1;
        d[axis] = (a > 0) ? 1 : 0;
        int vf = d[0] + 2 * d[1] + 4 * d[2];
        d[axis] = 0;
        int v0 = d[0] + 2 * d[1] + 4 * d[2];
        int v1 = v0 + (1 << axis);
        FG[k] = f[vf] - c;             /* g - c restricted to the face (eq. linear1) */
        FH[k] = (f[v1] - f[v0]) / 2.0; /* dg/dalpha: half the edge differences      */
    }
    double g[4], h[4];
    bilinear_coeffs(FG, g);
    bilinear_coeffs(FH, h);
    /* dg/dalpha identically zero: g does not depend on alpha and every point
     * of the surface (which meets a SURFACE leaf) solves the system */
    if (FH[0] == 0.0 && FH[1] == 0.0 && FH[2] == 0.0 && FH[3] == 0.0) return -1;
    /* G = (g0 + g1 u) + (g2 + g3 u) v,  H = (h0 + h1 u) + (h2 + h3 u) v: a
     * common v exists iff the resultant in v vanishes */
    double r0 = g[0] * h[2] - g[2] * h[0];
    double r1 = g[0] * h[3] + g[1] * h[2] - g[2] * h[1] - g[3] * h[0];
    double r2 = g[1] * h[3] - g[3] * h[1];
    double sg = fabs(g[0]) + fabs(g[1]) + fabs(g[2]) + fabs(g[3]);
    double sh = fabs(h[0]) + fabs(h[1]) + fabs(h[2]) + fabs(h[3]);
    double sr = fabs(r0) + fabs(r1) + fabs(r2);
    if (sg * sh > 0.0 && sr / (sg * sh) < *margin) *margin = sr / (sg * sh);
    double t[2], dm;
    int nr = quad_roots(r0, r1, r2, t, &dm);
    if (nr < 0) {
        /* resultant identically zero: if neither equation involves v, both
         * are linear in u and share a zero (a whole line along v) or have no
         * common solution; otherwise they share a factor (a curve) */
        if (g[2] == 0.0 && g[3] == 0.0 && h[2] == 0.0 && h[3] == 0.0)
            return linear_common_zero(g[0], g[1], h[0], h[1]) ? -1 : 0;
        return -1;
    }
    if (dm < *margin) *margin = dm;
    /* a root at which both equations vanish for every v: a line of solutions */
    for (int i = 0; i < nr; ++i) {
        double u = t[i];
        double AG = g[0] + g[1] * u, BG = g[2] + g[3] * u;
        double AH = h[0] + h[1] * u, BH = h[2] + h[3] * u;
        if (BG == 0.0 && BH == 0.0 && AG == 0.0 && AH == 0.0) return -1;
    }
    int n = 0;
    for (int i = 0; i < nr; ++i) {
        double u = t[i];
        double m = range_margin(u);
        if (m < *margin) *margin = m;
        if (u < -1.0 || u > 1.0) continue;
        double AG = g[0] + g[1] * u, BG = g[2] + g[3] * u;
        double AH = h[0] + h[1] * u, BH = h[2] + h[3] * u;
        double bmax = fmax(fabs(BG), fabs(BH));
        if (bmax == 0.0) {
            /* no v solves both unless both constant terms vanish too */
            double am = fmax(fabs(AG), fabs(AH)) / (sg + sh);
            if (am < *margin) *margin = am;
            continue;
        }
        double v = (fabs(BG) >= fabs(BH)) ? -AG / BG : -AH / BH;
        m = range_margin(v);
        if (m < *margin) *margin = m;
        if (v < -1.0 || v > 1.0) continue;
        uv[n][0] = u;
        uv[n][1] = v;
        ++n;
    }
    return n;
}

/* monomial coefficients of g (eq. linear1): g = sum_e m[e] prod_{i in e} x_i
 * over the subsets e of {x, y, z} (bit 0 x, bit 1 y, bit 2 z) */
static void trilinear_monomials(const double f[8], double m[8])
{
    for (int e = 0; e < 8; ++e) {
        double s = 0.0;
        for (int v = 0; v < 8; ++v) {
            double sg = 1.0;
            for (int i = 0; i < 3; ++i)
                if ((e >> i) & 1) sg *= ((v >> i) & 1) ? 1.0 : -1.0;
            s += sg * f[v];
        }
        m[e] = s / 8.0;
    }
}

/* Critical points (eq. critical) of the pair of axes other than gamma, in
 * local coordinates, ascending along gamma.  Returns their number, or -1
 * when the equations have infinitely many real solutions (degenerate). */
static int critical_points(const double f[8], double c, int gamma, double xyz[2][3],
                           double *margin)
{
    int o1 = (gamma + 1) % 3, o2 = (gamma + 2) % 3;
    int al = o1 < o2 ? o1 : o2, be = o1 < o2 ? o2 : o1;
    int A = 1 << al, B = 1 << be, G = 1 << gamma;
    double m[8];
    trilinear_monomials(f, m);
    /* at fixed gamma: g = k + P alpha + Q beta + S alpha beta, with k, P, Q, S
     * linear in gamma; dg/dalpha = P + S beta, dg/dbeta = Q + S alpha; where
     * both vanish (S != 0), g = k - P Q / S, so g = c iff (k - c) S - P Q = 0 */
    double k0 = m[0] - c, k1 = m[G];
    double P0 = m[A], P1 = m[A | G], Q0 = m[B], Q1 = m[B | G];
    double S0 = m[A | B], S1 = m[A | B | G];
    double w0 = k0 * S0 - P0 * Q0;
    double w1 = k0 * S1 + k1 * S0 - P0 * Q1 - P1 * Q0;
    double w2 = k1 * S1 - P1 * Q1;
    double sc = 0.0;
    for (int e = 0; e < 8; ++e)
        sc += fabs(e == 0 ? m[0] - c : m[e]);
    double sw = fabs(w0) + fabs(w1) + fabs(w2);
    if (sc > 0.0 && sw / (sc * sc) < *margin) *margin = sw / (sc * sc);
    double t[2], dm;
    int nr = quad_roots(w0, w1, w2, t, &dm);
    if (nr < 0) {
        /* identically zero.  With S not identically zero every slice's
         * stationary point lies on the surface: a curve.  With S = 0 the
         * slices are g = k + P alpha + Q beta: a solution needs P = Q = 0 and
         * k = c at one gamma (then the whole slice solves it) */
        if (S0 != 0.0 || S1 != 0.0) return -1;
        double a[3] = {P0, Q0, k0}, b[3] = {P1, Q1, k1};
        int rank1 = 1, anyb = 0, anya = 0;
        for (int i = 0; i < 3; ++i) {
            if (b[i] != 0.0) anyb = 1;
            if (a[i] != 0.0) anya = 1;
            for (int j = i + 1; j < 3; ++j)
                if (a[i] * b[j] - a[j] * b[i] != 0.0) rank1 = 0;
        }
        return (rank1 && (anyb || !anya)) ? -1 : 0;
    }
    if (dm < *margin) *margin = dm;
    /* a root at which a whole slice solves the system */
    for (int i = 0; i < nr; ++i) {
        double gm = t[i];
        if (S0 + S1 * gm == 0.0 && P0 + P1 * gm == 0.0 && Q0 + Q1 * gm == 0.0 &&
            k0 + k1 * gm == 0.0)
            return -1;
    }
    int n = 0;
    for (int i = 0; i < nr; ++i) {
        double gm = t[i];
        double mg = range_margin(gm);
        if (mg < *margin) *margin = mg;
        if (gm < -1.0 || gm > 1.0) continue;
        double S = S0 + S1 * gm, P = P0 + P1 * gm, Q = Q0 + Q1 * gm;
        if (S == 0.0) {
            /* the slice is g = k + P alpha + Q beta with P Q = 0: no isolated
             * stationary point on it */
            double pm = fmax(fabs(P), fabs(Q));
            if (pm == 0.0) pm = fabs(k0 + k1 * gm);
            if (sc > 0.0 && pm / sc < *margin) *margin = pm / sc;
            continue;
        }
        double a = -Q / S, b = -P / S;
        mg = fmin(range_margin(a), range_margin(b));
        if (mg < *margin) *margin = mg;
        if (a < -1.0 || a > 1.0 || b < -1.0 || b > 1.0) continue;
        xyz[n][al] = a;
        xyz[n][be] = b;
        xyz[n][gamma] = gm;
        ++n;
    }
    return n;
}

/* Every Stage 2 point of one cube (local coordinates).  Returns the number
 * of records written (<= OR_S2_MAX); *margin receives the smallest relative
 * distance of a discrete decision from a tie (1 if none), *ndeg the number
 * of degenerate (kind, axis) configurations, *mismatch the number of fold
 * segments whose extreme points on the faces -1 and +1 differ by more than
 * 1e-9 (they coincide in exact arithmetic). */
int or_stage2_cube(const double f[8], double c, double loc[OR_S2_MAX][3], uint8_t *kind,
                   uint8_t *axis, uint8_t *root, double *margin, int *ndeg, int *mismatch)
{
    int n = 0;
    *margin = 1.0;
    *ndeg = 0;
    *mismatch = 0;
    for (int al = 0; al < 3; ++al) {
        double lo[2][2], hi[2][2];
        int nl = face_extremes(f, c, al, -1, lo, margin);
        int nh = face_extremes(f, c, al, +1, hi, margin);
        if (nl < 0 || nh < 0) {
            ++*ndeg;
            continue;
        }
        if (nl != nh) ++*mismatch;
        for (int k = 0; k < nl; ++k) {
            if (k < nh && (fabs(lo[k][0] - hi[k][0]) > 1e-9 || fabs(lo[k][1] - hi[k][1]) > 1e-9))
                ++*mismatch;
            int o1 = (al + 1) % 3, o2 = (al + 2) % 3;
            int au = o1 < o2 ? o1 : o2, av = o1 < o2 ? o2 : o1;
            loc[n][al] = -1.0;
            loc[n][au] = lo[k][0];
            loc[n][av] = lo[k][1];
            kind[n] = 0;
            axis[n] = (uint8_t)al;
            root[n] = (uint8_t)k;
            ++n;
        }
    }
    for (int gm = 0; gm < 3; ++gm) {
        double p[2][3];
        int nc = critical_points(f, c, gm, p, margin);
        if (nc < 0) {
            ++*ndeg;
            continue;
        }
        for (int k = 0; k < nc; ++k) {
            for (int a = 0; a < 3; ++a)
                loc[n][a] = p[k][a];
            kind[n] = 1;
            axis[n] = (uint8_t)gm;
            root[n] = (uint8_t)k;
            ++n;
        }
    }
    return n;
}

/* Stage 2 points of every SURFACE leaf of a partition result, in world
 * coordinates: leaf q's cube is origin + (ijk + [0,1]) h0 / 2^level, local
 * u in [-1,1] maps to lo + (u + 1) h / 2.  Records come out by leaf, then
 * in the order of or_stage2_cube.  leaf_margin[q] receives the cube's
 * margin (1 for leaves that are not processed). */
typedef struct {
    int64_t n;
    or_s2pt *pts;
    double *leaf_margin;
    int64_t n_degenerate;
    int64_t n_mismatch;
} or_s2result;

or_s2result *or_stage2_points(const int32_t *ijk, const uint8_t *level, const uint8_t *cls,
                              const double *corner_phi, int64_t nl, double c, const double origin[3],
                              double h0, int nthreads)
{
    or_s2result *R = (or_s2result *)calloc(1, sizeof(or_s2result));
    int32_t *cnt = (int32_t *)calloc((size_t)(nl ? nl : 1), sizeof(int32_t));
    or_s2pt *tmp = (or_s2pt *)malloc(sizeof(or_s2pt) * OR_S2_MAX * (size_t)(nl ? nl : 1));
    R->leaf_margin = (double *)malloc(sizeof(double) * (size_t)(nl ? nl : 1));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t ndeg = 0, nmis = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : ndeg, nmis)
#endif
    for (int64_t q = 0; q < nl; ++q) {
        R->leaf_margin[q] = 1.0;
        if (cls[q] != OR_CLS_SURFACE) continue;
        double loc[OR_S2_MAX][3], margin;
        uint8_t kind[OR_S2_MAX], axis[OR_S2_MAX], root[OR_S2_MAX];
        int nd, mis;
        int n = or_stage2_cube(corner_phi + 8 * q, c, loc, kind, axis, root, &margin, &nd, &mis);
        R->leaf_margin[q] = margin;
        ndeg += nd;
        nmis += mis;
        double h = h0 / (double)(1 << level[q]);
        for (int k = 0; k < n; ++k) {
            or_s2pt *o = tmp + OR_S2_MAX * q + k;
            o->leaf = (int32_t)q;
            o->kind = kind[k];
            o->axis = axis[k];
            o->root = root[k];
            o->pad = 0;
            for (int a = 0; a < 3; ++a)
                o->p[a] = origin[a] + (double)ijk[3 * q + a] * h + (loc[k][a] + 1.0) * h / 2.0;
        }
        cnt[q] = n;
    }
    int64_t tot = 0;
    for (int64_t q = 0; q < nl; ++q)
        tot += cnt[q];
    R->pts = (or_s2pt *)malloc(sizeof(or_s2pt) * (size_t)(tot ? tot : 1));
    int64_t w = 0;
    for (int64_t q = 0; q < nl; ++q)
        for (int k = 0; k < cnt[q]; ++k)
            R->pts[w++] = tmp[OR_S2_MAX * q + k];
    R->n = tot;
    R->n_degenerate = ndeg;
    R->n_mismatch = nmis;
    free(tmp);
    free(cnt);
    return R;
}

void or_stage2_free(or_s2result *R)
{
    if (!R) return;
    free(R->pts);
    free(R->leaf_margin);
    free(R);
}

/* Edge intersection points (eq. intersection) of a caller's leaf list: leaf
 * q is the cube origin + (ijk + [0,1]) h0 / 2^level with corner values
 * corner_phi[8 q + v]; its corner mask and class against c follow eq.
 * linear1 (bit v set iff the value is >= c).  K: the finest level (edge keys
 * count in units of h0 / 2^K).  Vertices come out in ascending key order, as
 * in or_partition.  Free with or_free. */
or_result *or_extract(const int32_t *ijk, const uint8_t *level, const double *corner_phi,
                      int64_t nl, double c, const double origin[3], double h0, int K, int conf)
{
    or_result *R = (or_result *)calloc(1, sizeof(or_result));
    R->n_leaves = nl;
    R->K = K;
    for (int a = 0; a < 3; ++a)
        R->origin[a] = origin[a];
    size_t m = (size_t)(nl ? nl : 1);
    R->ijk = (int32_t *)malloc(sizeof(int32_t) * 3 * m);
    R->level = (uint8_t *)malloc(m);
    R->reason = (uint8_t *)calloc(m, 1);
    R->mask = (uint8_t *)malloc(m);
    R->cls = (uint8_t *)malloc(m);
    R->corner_phi = (double *)malloc(sizeof(double) * 8 * m);
    memcpy(R->ijk, ijk, sizeof(int32_t) * 3 * (size_t)nl);
    memcpy(R->level, level, (size_t)nl);
    memcpy(R->corner_phi, corner_phi, sizeof(double) * 8 * (size_t)nl);
    for (int64_t q = 0; q < nl; ++q) {
        uint8_t mk = 0;
        for (int v = 0; v < 8; ++v)
            if (corner_phi[8 * q + v] >= c) mk |= (uint8_t)(1u << v);
        R->mask[q] = mk;
        R->cls[q] = (mk == 0) ? OR_CLS_OUTSIDE : (mk == 0xFF ? OR_CLS_INSIDE : OR_CLS_SURFACE);
    }
    or_extract_edges(R, c, h0, h0 / (double)(1 << K), conf);
    return R;
}
