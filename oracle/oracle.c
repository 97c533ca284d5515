/*
 * Reference ("oracle") implementation of the DG Helmholtz-type pressure
 * operator -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 C.  It evaluates the quadrature-defined bilinear form
 * directly: at every quadrature point it evaluates all basis functions by the
 * Lagrange product formula, with no sum factorisation, blocking or fusion.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no code with
 * the HIP library.
 *
 * What is computed (paper section 2, the Helmholtz equation for the pressure,
 * linearised with frozen coefficients, and section 3.1, the matrix S~ whose
 * volume terms are a mass term plus a dt-scaled enthalpy-weighted stiffness):
 *
 *   a(u,v) = sum_K sum_q w_q detJ_q [alpha_q u v + beta_q grad u . grad v]
 *          + sum_F sum_q ds_q [ -1/2 (b- dn u- + b+ dn u+) [v]
 *                               -1/2 (b- dn v- + b+ dn v+) [u]
 *                               + sigma_F 1/2 (b- + b+) [u][v] ]
 *
 * on conforming hexahedral meshes mapped by a tensor-product Lagrange map of
 * degree g through equispaced reference nodes;  the DG space is the
 * tensor-product Lagrange basis on (k+1) Gauss-Lobatto points (section 2);
 * quadrature is (k+1)-point Gauss-Legendre per direction, the rule of the
 * fast block-diagonal evaluation (section 3.3);  [w] = w- - w+, n is the unit
 * normal of the minus cell (the cell whose +d face it is), ds and n are taken
 * from the minus side for both sides, the plus-side point has the same
 * tangential reference coordinates;
 *   sigma_F = P (k+1)^2 max(|F|/|K-|, |F|/|K+|);
 * boundary faces (neighbour -1) contribute nothing (natural Neumann).
 *
 * Non-conforming meshes (section 3: the paper's second mesh refines part of
 * the domain, so faces between a coarse cell and four finer ones appear):
 * each quarter of a coarse face that meets a fine cell is a face of the same
 * form, integrated with the fine face's Gauss rule; the coarse side is
 * evaluated at the images of those points on its face, ds and n come from
 * the fine side, the minus cell is the one whose +d face it is, and
 * sigma = P (k+1)^2 max(|S|/|K_fine|, |S|/|K_coarse|) with |S| the quarter's
 * area.
 *
 * The separable cell-block preconditioner Ahat_K (the tensor-product
 * structure used for the fast inverse of block-diagonal operators, section
 * 3.3) is built here by explicit Kronecker sums and solved densely.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define MAXN 10          /* max (k+1) and (g+1) */

/* ------------------------------------------------------------------------ */
/* 1-D rules on [0,1]                                                        */
/* ------------------------------------------------------------------------ */

/* Legendre P_n(x) and its derivative on [-1,1] by the three-term recurrence. */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
        p0 = p1; p1 = p2;
    }
    *p = p1;
    /* (x^2 - 1) P_n' = n (x P_n - P_{n-1}) */
    if (fabs(x) < 1.0)
        *dp = n * (x * p1 - p0) / (x * x - 1.0);
    else
        *dp = 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
}

/* n-point Gauss-Legendre: roots of P_n by Newton from Chebyshev guesses. */
void or_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double t = -cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, t, &p, &dp);
            double dt = p / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double p, dp;
        legendre(n, t, &p, &dp);
        x[i] = 0.5 * (t + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

/* n-point Gauss-Lobatto: the endpoints and the roots of P'_{n-1}.
 * Newton on q(x) = P'_{n-1}(x) using q' = (2x q - m(m+1) P_m)/(1-x^2), m = n-1. */
void or_gauss_lobatto(int n, double *x, double *w)
{
    int m = n - 1;
    x[0] = 0.0; x[n - 1] = 1.0;
    w[0] = w[n - 1] = 0.5 * 2.0 / (n * (n - 1.0));
    for (int i = 1; i < n - 1; ++i) {
        double t = -cos(M_PI * i / m);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(m, t, &p, &dp);
            double ddp = (2.0 * t * dp - m * (m + 1.0) * p) / (1.0 - t * t);
            double dt = dp / ddp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double p, dp;
        legendre(m, t, &p, &dp);
        x[i] = 0.5 * (t + 1.0);
        w[i] = 0.5 * 2.0 / (n * (n - 1.0) * p * p);
    }
}

/* Lagrange basis through nodes[0..n-1]: values and derivatives at t,
 * straight from the product formula. */
void or_lagrange(int n, const double *nodes, double t, double *val, double *der)
{
    for (int i = 0; i < n; ++i) {
        double v = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != i) v *= (t - nodes[m]) / (nodes[i] - nodes[m]);
        val[i] = v;
        double d = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == i) continue;
            double prod = 1.0 / (nodes[i] - nodes[m]);
            for (int l = 0; l < n; ++l)
                if (l != i && l != m) prod *= (t - nodes[l]) / (nodes[i] - nodes[l]);
            d += prod;
        }
        der[i] = d;
    }
}

/* ------------------------------------------------------------------------ */
/* reference data                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, nd;               /* k+1, (k+1)^3 */
    int ng, ngn;             /* g+1, (g+1)^3 */
    double xq[MAXN], wq[MAXN];   /* GL on [0,1] */
    double xl[MAXN], wl[MAXN];   /* GLL on [0,1] (dof nodes) */
    double xe[MAXN];             /* equispaced geometry nodes */
} ref_t;

static void ref_init(ref_t *r, int k, int g)
{
    r->n = k + 1; r->nd = r->n * r->n * r->n;
    r->ng = g + 1; r->ngn = r->ng * r->ng * r->ng;
    or_gauss_legendre(r->n, r->xq, r->wq);
    or_gauss_lobatto(r->n, r->xl, r->wl);
    for (int a = 0; a <= g; ++a) r->xe[a] = (double)a / g;
}

/* all nd basis functions and reference gradients at reference point xi */
static void basis_at(const ref_t *r, const double xi[3], double *phi, double (*dphi)[3])
{
    double v[3][MAXN], d[3][MAXN];
    for (int c = 0; c < 3; ++c) or_lagrange(r->n, r->xl, xi[c], v[c], d[c]);
    int n = r->n;
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int a = i + n * (j + n * l);
                phi[a] = v[0][i] * v[1][j] * v[2][l];
                dphi[a][0] = d[0][i] * v[1][j] * v[2][l];
                dphi[a][1] = v[0][i] * d[1][j] * v[2][l];
                dphi[a][2] = v[0][i] * v[1][j] * d[2][l];
            }
}

/* physical position and Jacobian J[r][d] = d x_r / d xi_d of one cell */
static void geom_at(const ref_t *r, const double *X, const double xi[3],
                    double x[3], double J[3][3])
{
    double v[3][MAXN], d[3][MAXN];
    for (int c = 0; c < 3; ++c) or_lagrange(r->ng, r->xe, xi[c], v[c], d[c]);
    int ng = r->ng;
    for (int a = 0; a < 3; ++a) { x[a] = 0.0; J[a][0] = J[a][1] = J[a][2] = 0.0; }
    for (int c = 0; c < ng; ++c)
        for (int b = 0; b < ng; ++b)
            for (int a = 0; a < ng; ++a) {
                const double *P = X + 3 * (a + ng * (b + ng * c));
                double s = v[0][a] * v[1][b] * v[2][c];
                double s0 = d[0][a] * v[1][b] * v[2][c];
                double s1 = v[0][a] * d[1][b] * v[2][c];
                double s2 = v[0][a] * v[1][b] * d[2][c];
                for (int q = 0; q < 3; ++q) {
                    x[q] += s * P[q];
                    J[q][0] += s0 * P[q];
                    J[q][1] += s1 * P[q];
                    J[q][2] += s2 * P[q];
                }
            }
}

static double det3(double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* inverse transpose K = J^{-T} (so that grad = K * grad_ref) */
static void inv_transpose(double J[3][3], double det, double K[3][3])
{
    double C[3][3];   /* cofactor matrix */
    C[0][0] =  (J[1][1] * J[2][2] - J[1][2] * J[2][1]);
    C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
    C[0][2] =  (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
    C[1][1] =  (J[0][0] * J[2][2] - J[0][2] * J[2][0]);
    C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
    C[2][0] =  (J[0][1] * J[1][2] - J[0][2] * J[1][1]);
    C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
    C[2][2] =  (J[0][0] * J[1][1] - J[0][1] * J[1][0]);
    /* J^{-1} = C^T / det  =>  J^{-T} = C / det */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K[a][b] = C[a][b] / det;
}

static void matvec3(double K[3][3], const double v[3], double out[3])
{
    for (int a = 0; a < 3; ++a) out[a] = K[a][0] * v[0] + K[a][1] * v[1] + K[a][2] * v[2];
}

static const double *cell_nodes(const or_prob *p, const ref_t *r, long c)
{
    return p->nodes + (size_t)c * r->ngn * 3;
}

/* cell volume |K| = sum_q w_q detJ_q */
static double cell_volume(const or_prob *p, const ref_t *r, long c)
{
    int n = r->n;
    double vol = 0.0;
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xi[3] = {r->xq[i], r->xq[j], r->xq[l]}, x[3], J[3][3];
                geom_at(r, cell_nodes(p, r, c), xi, x, J);
                vol += r->wq[i] * r->wq[j] * r->wq[l] * det3(J);
            }
    return vol;
}

/* reference point on the (+d or -d) face of a cell, tangential GL (a,b) */
static void face_point(const ref_t *r, int d, int plus, int a, int b, double xi[3])
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    xi[d] = plus ? 1.0 : 0.0;
    xi[t1] = r->xq[a];
    xi[t2] = r->xq[b];
}

/* minus-side normal and surface element at one face point of the +d face */
static void face_normal(const ref_t *r, const double *Xm, int d, int a, int b,
                        double nrm[3], double *ds)
{
    double xi[3], x[3], J[3][3], K[3][3];
    face_point(r, d, 1, a, b, xi);
    geom_at(r, Xm, xi, x, J);
    double det = det3(J);
    inv_transpose(J, det, K);
    double e[3] = {0, 0, 0}, m[3];
    e[d] = 1.0;
    matvec3(K, e, m);
    double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    for (int q = 0; q < 3; ++q) nrm[q] = m[q] / len;
    *ds = r->wq[a] * r->wq[b] * det * len;
}

/* |F| of the +d face of cell c (minus side) */
static double face_area(const or_prob *p, const ref_t *r, long c, int d)
{
    double area = 0.0, nrm[3], ds;
    for (int b = 0; b < r->n; ++b)
        for (int a = 0; a < r->n; ++a) {
            face_normal(r, cell_nodes(p, r, c), d, a, b, nrm, &ds);
            area += ds;
        }
    return area;
}

/* penalty of the +d face of cell c (c is the minus cell), -1 if boundary */
static double face_sigma(const or_prob *p, const ref_t *r, long c, int d)
{
    long nb = p->nbr[6 * c + 2 * d + 1];
    if (nb < 0) return -1.0;
    double area = face_area(p, r, c, d);
    double vm = cell_volume(p, r, c), vp = cell_volume(p, r, nb);
    double s = area / vm > area / vp ? area / vm : area / vp;
    return p->P * (double)(r->n * r->n) * s;
}

void or_face_sigma(const or_prob *p, double *sigma)
{
    ref_t r; ref_init(&r, p->k, p->g);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < p->n_cells; ++c)
        for (int d = 0; d < 3; ++d) sigma[3 * c + d] = face_sigma(p, &r, c, d);
}

void or_cell_volumes(const or_prob *p, double *vol)
{
    ref_t r; ref_init(&r, p->k, p->g);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < p->n_cells; ++c) vol[c] = cell_volume(p, &r, c);
}

/* ------------------------------------------------------------------------ */
/* mesh check                                                                */
/* ------------------------------------------------------------------------ */

int or_mesh_check(const or_prob *p)
{
    ref_t r; ref_init(&r, p->k, p->g);
    int bad = 0;
    for (long c = 0; c < p->n_cells; ++c) {
        for (int f = 0; f < 6; ++f) {
            long nb = p->nbr[6 * c + f];
            if (nb < (p->n_hang > 0 ? -2 : -1) || nb >= p->n_cells) return 2;
            if (nb >= 0 && p->nbr[6 * nb + (f ^ 1)] != c) return 2;
        }
    }
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (long c = 0; c < p->n_cells; ++c) {
        int n = r.n;
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3];
                    geom_at(&r, cell_nodes(p, &r, c), xi, x, J);
                    if (!(det3(J) > 0.0)) bad |= 1;
                }
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* coordinates and load vectors                                              */
/* ------------------------------------------------------------------------ */

void or_dof_coords(const or_prob *p, double *xyz)
{
    ref_t r; ref_init(&r, p->k, p->g);
    long ndofs = p->n_cells * r.nd;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < p->n_cells; ++c) {
        int n = r.n;
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double xi[3] = {r.xl[i], r.xl[j], r.xl[l]}, x[3], J[3][3];
                    geom_at(&r, cell_nodes(p, &r, c), xi, x, J);
                    long dof = c * r.nd + i + n * (j + n * l);
                    for (int q = 0; q < 3; ++q) xyz[q * ndofs + dof] = x[q];
                }
    }
}

void or_quad_data(const or_prob *p, double *xyz, double *wdet)
{
    ref_t r; ref_init(&r, p->k, p->g);
    long nq = p->n_cells * r.nd;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < p->n_cells; ++c) {
        int n = r.n;
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3];
                    geom_at(&r, cell_nodes(p, &r, c), xi, x, J);
                    long q = c * r.nd + i + n * (j + n * l);
                    for (int a = 0; a < 3; ++a) xyz[a * nq + q] = x[a];
                    wdet[q] = r.wq[i] * r.wq[j] * r.wq[l] * det3(J);
                }
    }
}

/* b_i = sum_q w_q detJ_q f(x_q) phi_i(x_q), with f given at the GL points */
void or_load_vector(const or_prob *p, const double *fq, double *b)
{
    ref_t r; ref_init(&r, p->k, p->g);
#pragma omp parallel
    {
        double *phi = malloc(sizeof(double) * r.nd);
        double (*dphi)[3] = malloc(sizeof(double) * 3 * r.nd);
#pragma omp for schedule(static)
        for (long c = 0; c < p->n_cells; ++c) {
            int n = r.n;
            double *bc = b + c * r.nd;
            for (int a = 0; a < r.nd; ++a) bc[a] = 0.0;
            for (int l = 0; l < n; ++l)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3];
                        geom_at(&r, cell_nodes(p, &r, c), xi, x, J);
                        double wd = r.wq[i] * r.wq[j] * r.wq[l] * det3(J);
                        basis_at(&r, xi, phi, dphi);
                        double fv = fq[c * r.nd + i + n * (j + n * l)];
                        for (int a = 0; a < r.nd; ++a) bc[a] += wd * fv * phi[a];
                    }
        }
        free(phi); free(dphi);
    }
}

/* ------------------------------------------------------------------------ */
/* operator action                                                           */
/* ------------------------------------------------------------------------ */

/* value of a DG field (nodal coefficients f of cell c) at reference point */
static double field_at(const double *phi, const double *fc, int nd)
{
    double s = 0.0;
    for (int a = 0; a < nd; ++a) s += phi[a] * fc[a];
    return s;
}

typedef struct {
    double *phi;            /* [nd] */
    double (*dphi)[3];      /* [nd][3] */
} scratch_t;

static void hang_apply_cell(const or_prob *p, const ref_t *r, long c, const double *xv, double *yc);

/* (A x) restricted to the test functions of cell c, written to yc[nd] */
static void apply_one_cell(const or_prob *p, int flags, long c, const double *xv, double *yc)
{
    ref_t r; ref_init(&r, p->k, p->g);
    const int nd = r.nd, n = r.n;
    double *phi = malloc(sizeof(double) * nd), *phiB = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    double (*dphiB)[3] = malloc(sizeof(double) * 3 * nd);
    const double *xc = xv + c * nd;
    for (int a = 0; a < nd; ++a) yc[a] = 0.0;
    const double *X = cell_nodes(p, &r, c);
    /* ---- cell integral ---- */
    if (flags & OR_CELL) {
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3], K[3][3];
                    geom_at(&r, X, xi, x, J);
                    double det = det3(J);
                    inv_transpose(J, det, K);
                    double w = r.wq[i] * r.wq[j] * r.wq[l] * det;
                    basis_at(&r, xi, phi, dphi);
                    double al = field_at(phi, p->alpha + c * nd, nd);
                    double be = field_at(phi, p->beta + c * nd, nd);
                    double u = 0.0, gr[3] = {0, 0, 0};
                    for (int a = 0; a < nd; ++a) {
                        u += phi[a] * xc[a];
                        for (int q = 0; q < 3; ++q) gr[q] += dphi[a][q] * xc[a];
                    }
                    double gu[3];
                    matvec3(K, gr, gu);
                    for (int a = 0; a < nd; ++a) {
                        double gv[3];
                        matvec3(K, dphi[a], gv);
                        yc[a] += w * (al * u * phi[a]
                                      + be * (gu[0] * gv[0] + gu[1] * gv[1] + gu[2] * gv[2]));
                    }
                }
    }
    /* ---- face integrals, test functions of cell c only ---- */
    if (flags & OR_FACE) {
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                /* side 1: the +d face of c (c is the minus cell);
                   side 0: the -d face of c (c is the plus cell) */
                long nb = p->nbr[6 * c + 2 * d + side];
                if (nb < 0) continue;
                long km = side ? c : nb, kp = side ? nb : c;
                double sigma = face_sigma(p, &r, km, d);
                const double *Xm = cell_nodes(p, &r, km), *Xp = cell_nodes(p, &r, kp);
                const double *xm = xv + km * nd, *xp = xv + kp * nd;
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        double nrm[3], ds;
                        face_normal(&r, Xm, d, a, b, nrm, &ds);
                        double xim[3], xip[3], pos[3], Jm[3][3], Jp[3][3], Km[3][3], Kp[3][3];
                        face_point(&r, d, 1, a, b, xim);
                        face_point(&r, d, 0, a, b, xip);
                        geom_at(&r, Xm, xim, pos, Jm);
                        geom_at(&r, Xp, xip, pos, Jp);
                        inv_transpose(Jm, det3(Jm), Km);
                        inv_transpose(Jp, det3(Jp), Kp);
                        basis_at(&r, xim, phi, dphi);      /* minus side */
                        basis_at(&r, xip, phiB, dphiB);    /* plus side */
                        double bm = field_at(phi, p->beta + km * nd, nd);
                        double bp = field_at(phiB, p->beta + kp * nd, nd);
                        double um = 0, up = 0, gm[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
                        for (int e = 0; e < nd; ++e) {
                            um += phi[e] * xm[e];
                            up += phiB[e] * xp[e];
                            for (int q = 0; q < 3; ++q) {
                                gm[q] += dphi[e][q] * xm[e];
                                gp[q] += dphiB[e][q] * xp[e];
                            }
                        }
                        double Gm[3], Gp[3];
                        matvec3(Km, gm, Gm);
                        matvec3(Kp, gp, Gp);
                        double dnm = nrm[0] * Gm[0] + nrm[1] * Gm[1] + nrm[2] * Gm[2];
                        double dnp = nrm[0] * Gp[0] + nrm[1] * Gp[1] + nrm[2] * Gp[2];
                        double flux = bm * dnm + bp * dnp;
                        double jump = um - up;
                        double pen = sigma * 0.5 * (bm + bp);
                        /* own test functions */
                        const double *tphi = side ? phi : phiB;
                        double (*tdphi)[3] = side ? dphi : dphiB;
                        double (*Kown)[3] = side ? Km : Kp;
                        double bown = side ? bm : bp;
                        double sgn = side ? 1.0 : -1.0;
                        for (int e = 0; e < nd; ++e) {
                            double gv[3];
                            matvec3(Kown, tdphi[e], gv);
                            double dnv = nrm[0] * gv[0] + nrm[1] * gv[1] + nrm[2] * gv[2];
                            double jv = sgn * tphi[e];
                            yc[e] += ds * (-0.5 * flux * jv - 0.5 * bown * dnv * jump
                                           + pen * jump * jv);
                        }
                    }
            }
        hang_apply_cell(p, &r, c, xv, yc);
    }
    free(phi); free(phiB); free(dphi); free(dphiB);
}

/* ------------------------------------------------------------------------ */
/* non-conforming faces                                                      */
/* ------------------------------------------------------------------------ */

/* reference points of the fine face's Gauss point (a, b) on the fine cell
 * (xiF) and on the coarse cell (xiC) for the hanging record h */
static void hang_points(const ref_t *r, const long *h, int a, int b, double xiF[3], double xiC[3])
{
    const int fc = (int)h[1], d = fc >> 1, s = (int)h[3];
    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    face_point(r, d, (fc ^ 1) & 1, a, b, xiF);
    xiC[d] = (fc & 1) ? 1.0 : 0.0;
    xiC[t1] = 0.5 * ((s & 1) + r->xq[a]);
    xiC[t2] = 0.5 * ((s >> 1) + r->xq[b]);
}

/* unit normal n (the +d direction, i.e. the minus cell's outward normal) and
 * surface element at the fine face's point (a, b), from the fine side */
static void hang_normal(const or_prob *p, const ref_t *r, const long *h, int a, int b,
                        double nrm[3], double *ds)
{
    double xiF[3], xiC[3], x[3], J[3][3], K[3][3];
    const int d = (int)(h[1] >> 1);
    hang_points(r, h, a, b, xiF, xiC);
    geom_at(r, cell_nodes(p, r, h[2]), xiF, x, J);
    double det = det3(J);
    inv_transpose(J, det, K);
    double e[3] = {0, 0, 0}, m[3];
    e[d] = 1.0;
    matvec3(K, e, m);
    double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    for (int q = 0; q < 3; ++q) nrm[q] = m[q] / len;
    *ds = r->wq[a] * r->wq[b] * det * len;
}

/* penalty of the quarter face of record h */
static double hang_sigma(const or_prob *p, const ref_t *r, const long *h)
{
    double area = 0.0, nrm[3], ds;
    for (int b = 0; b < r->n; ++b)
        for (int a = 0; a < r->n; ++a) {
            hang_normal(p, r, h, a, b, nrm, &ds);
            area += ds;
        }
    double vf = cell_volume(p, r, h[2]), vc = cell_volume(p, r, h[0]);
    double s = area / vf > area / vc ? area / vf : area / vc;
    return p->P * (double)(r->n * r->n) * s;
}

void or_hang_sigma(const or_prob *p, double *sigma)
{
    ref_t r; ref_init(&r, p->k, p->g);
#pragma omp parallel for schedule(static)
    for (long h = 0; h < p->n_hang; ++h) sigma[h] = hang_sigma(p, &r, p->hang + 4 * h);
}

/* values, physical gradients and beta of both sides at the fine face's point
 * (a, b) of record h; side 0 = coarse, 1 = fine */
typedef struct {
    double *phi[2];
    double (*dphi[2])[3];
    double K[2][3][3];
    double beta[2];
} hang_pt;

static void hang_eval(const or_prob *p, const ref_t *r, const long *h, int a, int b, hang_pt *hp)
{
    double xi[2][3], x[3], J[3][3];
    const int nd = r->nd;
    hang_points(r, h, a, b, xi[1], xi[0]);
    for (int side = 0; side < 2; ++side) {
        const long c = side ? h[2] : h[0];
        geom_at(r, cell_nodes(p, r, c), xi[side], x, J);
        inv_transpose(J, det3(J), hp->K[side]);
        basis_at(r, xi[side], hp->phi[side], hp->dphi[side]);
        hp->beta[side] = field_at(hp->phi[side], p->beta + c * nd, nd);
    }
}

/* contributions of the quarter face of record h to the test functions of its
 * coarse (own = 0) or fine (own = 1) cell, added to yc[nd] */
static void hang_apply(const or_prob *p, const ref_t *r, const long *h, int own, const double *xv,
                       double *yc, hang_pt *hp)
{
    const int nd = r->nd, n = r->n;
    const int minus = (h[1] & 1) ? 0 : 1;   /* the coarse cell is minus on its own +d face */
    const double sigma = hang_sigma(p, r, h);
    const double *xs[2] = {xv + h[0] * nd, xv + h[2] * nd};
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            double nrm[3], ds;
            hang_normal(p, r, h, a, b, nrm, &ds);
            hang_eval(p, r, h, a, b, hp);
            double u[2], dn[2];
            for (int side = 0; side < 2; ++side) {
                double gr[3] = {0, 0, 0}, g[3];
                u[side] = 0.0;
                for (int e = 0; e < nd; ++e) {
                    u[side] += hp->phi[side][e] * xs[side][e];
                    for (int q = 0; q < 3; ++q) gr[q] += hp->dphi[side][e][q] * xs[side][e];
                }
                matvec3(hp->K[side], gr, g);
                dn[side] = nrm[0] * g[0] + nrm[1] * g[1] + nrm[2] * g[2];
            }
            const int plus = 1 - minus;
            double flux = hp->beta[minus] * dn[minus] + hp->beta[plus] * dn[plus];
            double jump = u[minus] - u[plus];
            double pen = sigma * 0.5 * (hp->beta[minus] + hp->beta[plus]);
            double sgn = own == minus ? 1.0 : -1.0;
            for (int e = 0; e < nd; ++e) {
                double gv[3];
                matvec3(hp->K[own], hp->dphi[own][e], gv);
                double dnv = nrm[0] * gv[0] + nrm[1] * gv[1] + nrm[2] * gv[2];
                double jv = sgn * hp->phi[own][e];
                yc[e] += ds * (-0.5 * flux * jv - 0.5 * hp->beta[own] * dnv * jump + pen * jump * jv);
            }
        }
}

static void hang_alloc(hang_pt *hp, int nd)
{
    for (int s = 0; s < 2; ++s) {
        hp->phi[s] = malloc(sizeof(double) * nd);
        hp->dphi[s] = malloc(sizeof(double) * 3 * nd);
    }
}

static void hang_free(hang_pt *hp)
{
    for (int s = 0; s < 2; ++s) { free(hp->phi[s]); free(hp->dphi[s]); }
}

/* the non-conforming face terms on the test functions of cell c */
static void hang_apply_cell(const or_prob *p, const ref_t *r, long c, const double *xv, double *yc)
{
    if (p->n_hang <= 0) return;
    hang_pt hp;
    hang_alloc(&hp, r->nd);
    for (long h = 0; h < p->n_hang; ++h) {
        const long *rec = p->hang + 4 * h;
        if (rec[0] == c) hang_apply(p, r, rec, 0, xv, yc, &hp);
        if (rec[2] == c) hang_apply(p, r, rec, 1, xv, yc, &hp);
    }
    hang_free(&hp);
}

/* ------------------------------------------------------------------------ */
/* consistent integration (section 3.3: 2r+1 Gauss points per direction)     */
/* ------------------------------------------------------------------------ */

#define MAXQ 20

/* (A x) on the test functions of cell c with an nq-point Gauss rule per
 * direction on cells and faces; the same form as apply_one_cell, whose rule
 * is the (k+1)-point one.  The penalty sigma_F keeps its geometric
 * definition. */
static void apply_one_cell_q(const or_prob *p, int nq, int flags, long c, const double *xv,
                             double *yc)
{
    ref_t r; ref_init(&r, p->k, p->g);
    const int nd = r.nd;
    double xg[MAXQ], wg[MAXQ];
    or_gauss_legendre(nq, xg, wg);
    double *phi = malloc(sizeof(double) * nd), *phiB = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    double (*dphiB)[3] = malloc(sizeof(double) * 3 * nd);
    const double *xc = xv + c * nd;
    for (int a = 0; a < nd; ++a) yc[a] = 0.0;
    const double *X = cell_nodes(p, &r, c);
    if (flags & OR_CELL) {
        for (int l = 0; l < nq; ++l)
            for (int j = 0; j < nq; ++j)
                for (int i = 0; i < nq; ++i) {
                    double xi[3] = {xg[i], xg[j], xg[l]}, x[3], J[3][3], K[3][3];
                    geom_at(&r, X, xi, x, J);
                    double det = det3(J);
                    inv_transpose(J, det, K);
                    double w = wg[i] * wg[j] * wg[l] * det;
                    basis_at(&r, xi, phi, dphi);
                    double al = field_at(phi, p->alpha + c * nd, nd);
                    double be = field_at(phi, p->beta + c * nd, nd);
                    double u = 0.0, gr[3] = {0, 0, 0};
                    for (int a = 0; a < nd; ++a) {
                        u += phi[a] * xc[a];
                        for (int q = 0; q < 3; ++q) gr[q] += dphi[a][q] * xc[a];
                    }
                    double gu[3];
                    matvec3(K, gr, gu);
                    for (int a = 0; a < nd; ++a) {
                        double gv[3];
                        matvec3(K, dphi[a], gv);
                        yc[a] += w * (al * u * phi[a]
                                      + be * (gu[0] * gv[0] + gu[1] * gv[1] + gu[2] * gv[2]));
                    }
                }
    }
    if (flags & OR_FACE) {
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                long nb = p->nbr[6 * c + 2 * d + side];
                if (nb < 0) continue;
                long km = side ? c : nb, kp = side ? nb : c;
                double sigma = face_sigma(p, &r, km, d);
                const double *Xm = cell_nodes(p, &r, km), *Xp = cell_nodes(p, &r, kp);
                const double *xm = xv + km * nd, *xp = xv + kp * nd;
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                for (int b = 0; b < nq; ++b)
                    for (int a = 0; a < nq; ++a) {
                        double xim[3], xip[3], pos[3], Jm[3][3], Jp[3][3], Km[3][3], Kp[3][3];
                        xim[d] = 1.0; xip[d] = 0.0;
                        xim[t1] = xip[t1] = xg[a];
                        xim[t2] = xip[t2] = xg[b];
                        geom_at(&r, Xm, xim, pos, Jm);
                        geom_at(&r, Xp, xip, pos, Jp);
                        double detm = det3(Jm);
                        inv_transpose(Jm, detm, Km);
                        inv_transpose(Jp, det3(Jp), Kp);
                        /* minus-side unit normal J^-T e_d / |.| and surface element */
                        double e[3] = {0, 0, 0}, mv[3], nrm[3];
                        e[d] = 1.0;
                        matvec3(Km, e, mv);
                        double len = sqrt(mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2]);
                        for (int q = 0; q < 3; ++q) nrm[q] = mv[q] / len;
                        double ds = wg[a] * wg[b] * detm * len;
                        basis_at(&r, xim, phi, dphi);
                        basis_at(&r, xip, phiB, dphiB);
                        double bm = field_at(phi, p->beta + km * nd, nd);
                        double bp = field_at(phiB, p->beta + kp * nd, nd);
                        double um = 0, up = 0, gm[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
                        for (int q2 = 0; q2 < nd; ++q2) {
                            um += phi[q2] * xm[q2];
                            up += phiB[q2] * xp[q2];
                            for (int q = 0; q < 3; ++q) {
                                gm[q] += dphi[q2][q] * xm[q2];
                                gp[q] += dphiB[q2][q] * xp[q2];
                            }
                        }
                        double Gm[3], Gp[3];
                        matvec3(Km, gm, Gm);
                        matvec3(Kp, gp, Gp);
                        double dnm = nrm[0] * Gm[0] + nrm[1] * Gm[1] + nrm[2] * Gm[2];
                        double dnp = nrm[0] * Gp[0] + nrm[1] * Gp[1] + nrm[2] * Gp[2];
                        double flux = bm * dnm + bp * dnp;
                        double jump = um - up;
                        double pen = sigma * 0.5 * (bm + bp);
                        const double *tphi = side ? phi : phiB;
                        double (*tdphi)[3] = side ? dphi : dphiB;
                        double (*Kown)[3] = side ? Km : Kp;
                        double bown = side ? bm : bp;
                        double sgn = side ? 1.0 : -1.0;
                        for (int q2 = 0; q2 < nd; ++q2) {
                            double gv[3];
                            matvec3(Kown, tdphi[q2], gv);
                            double dnv = nrm[0] * gv[0] + nrm[1] * gv[1] + nrm[2] * gv[2];
                            double jv = sgn * tphi[q2];
                            yc[q2] += ds * (-0.5 * flux * jv - 0.5 * bown * dnv * jump
                                            + pen * jump * jv);
                        }
                    }
            }
    }
    free(phi); free(phiB); free(dphi); free(dphiB);
}

/* y = A x with the nq-point rule (nq = 2k+1: consistent integration) */
void or_apply_q(const or_prob *p, int nq, int flags, const double *xv, double *yv)
{
    int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (long c = 0; c < p->n_cells; ++c) apply_one_cell_q(p, nq, flags, c, xv, yv + c * nd);
}

/* the same restricted to listed cells: out[s][nd] */
void or_apply_q_cells(const or_prob *p, int nq, int flags, const long *cells, long m,
                      const double *xv, double *out)
{
    int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < m; ++s) apply_one_cell_q(p, nq, flags, cells[s], xv, out + s * nd);
}

/* Diagonal of the volume part of the form (section 3.1: the paper's
 * "Helmholtz preconditioner" is the inverse of the diagonal of S~, whose
 * entries are volume integrals only; its "internal-energy" variant keeps the
 * mass term alone):
 *   d_i = sum_q w_q detJ_q [alpha_q phi_i^2 + beta_q |J^-T grad phi_i|^2]
 * with the stiffness term only if `stiff` is nonzero. */
void or_cell_diagonal(const or_prob *p, int stiff, double *diag)
{
    const int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (long c = 0; c < p->n_cells; ++c) {
        ref_t r; ref_init(&r, p->k, p->g);
        const int n = r.n;
        double *phi = malloc(sizeof(double) * nd);
        double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
        double *dc = diag + c * nd;
        for (int a = 0; a < nd; ++a) dc[a] = 0.0;
        const double *X = cell_nodes(p, &r, c);
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3], K[3][3];
                    geom_at(&r, X, xi, x, J);
                    double det = det3(J);
                    inv_transpose(J, det, K);
                    double w = r.wq[i] * r.wq[j] * r.wq[l] * det;
                    basis_at(&r, xi, phi, dphi);
                    double al = field_at(phi, p->alpha + c * nd, nd);
                    double be = field_at(phi, p->beta + c * nd, nd);
                    for (int a = 0; a < nd; ++a) {
                        double v = al * phi[a] * phi[a];
                        if (stiff) {
                            double gv[3];
                            matvec3(K, dphi[a], gv);
                            v += be * (gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
                        }
                        dc[a] += w * v;
                    }
                }
        free(phi); free(dphi);
    }
}

/* y = A x: each cell accumulates a(x, phi_i) for its own test functions. */
void or_apply(const or_prob *p, int flags, const double *xv, double *yv)
{
    int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (long c = 0; c < p->n_cells; ++c) apply_one_cell(p, flags, c, xv, yv + c * nd);
}

/* y restricted to the listed cells: out[m*nd + a] = (A x)_{cells[m]*nd + a}.
 * Same arithmetic as or_apply, for spot checks on large meshes. */
void or_apply_cells(const or_prob *p, int flags, const long *cells, long m,
                    const double *xv, double *out)
{
    int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
    or_prob sub = *p;
    (void)sub;
#pragma omp parallel
    {
        double *tmp = malloc(sizeof(double) * nd);
#pragma omp for schedule(dynamic, 1)
        for (long s = 0; s < m; ++s) {
            apply_one_cell(p, flags, cells[s], xv, tmp);
            for (int a = 0; a < nd; ++a) out[s * nd + a] = tmp[a];
        }
        free(tmp);
    }
}


/* values of a DG field at the cell GL points, uq[c*nd + q] */
void or_eval_quad(const or_prob *p, const double *u, double *uq)
{
    ref_t r; ref_init(&r, p->k, p->g);
#pragma omp parallel
    {
        double *phi = malloc(sizeof(double) * r.nd);
        double (*dphi)[3] = malloc(sizeof(double) * 3 * r.nd);
#pragma omp for schedule(static)
        for (long c = 0; c < p->n_cells; ++c) {
            int n = r.n;
            for (int l = 0; l < n; ++l)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        double xi[3] = {r.xq[i], r.xq[j], r.xq[l]};
                        basis_at(&r, xi, phi, dphi);
                        uq[c * r.nd + i + n * (j + n * l)] = field_at(phi, u + c * r.nd, r.nd);
                    }
        }
        free(phi); free(dphi);
    }
}

/* ------------------------------------------------------------------------ */
/* dense assembly (a second, independent route: explicit matrix entries)    */
/* ------------------------------------------------------------------------ */

void or_assemble_dense(const or_prob *p, int flags, double *A)
{
    ref_t r; ref_init(&r, p->k, p->g);
    const int nd = r.nd, n = r.n;
    const long N = p->n_cells * nd;
    memset(A, 0, sizeof(double) * (size_t)N * N);
    double *phi = malloc(sizeof(double) * nd), *phi2 = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    double (*dphi2)[3] = malloc(sizeof(double) * 3 * nd);
    double (*gphys)[3] = malloc(sizeof(double) * 3 * nd);
    double (*gphys2)[3] = malloc(sizeof(double) * 3 * nd);
    /* element matrices */
    if (flags & OR_CELL) {
        for (long c = 0; c < p->n_cells; ++c) {
            const double *X = cell_nodes(p, &r, c);
            for (int l = 0; l < n; ++l)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3], K[3][3];
                        geom_at(&r, X, xi, x, J);
                        double det = det3(J);
                        inv_transpose(J, det, K);
                        double w = r.wq[i] * r.wq[j] * r.wq[l] * det;
                        basis_at(&r, xi, phi, dphi);
                        double al = 0, be = 0;
                        for (int a = 0; a < nd; ++a) {
                            al += phi[a] * p->alpha[c * nd + a];
                            be += phi[a] * p->beta[c * nd + a];
                            matvec3(K, dphi[a], gphys[a]);
                        }
                        for (int ti = 0; ti < nd; ++ti)
                            for (int tj = 0; tj < nd; ++tj) {
                                double s = al * phi[ti] * phi[tj]
                                    + be * (gphys[ti][0] * gphys[tj][0] + gphys[ti][1] * gphys[tj][1]
                                            + gphys[ti][2] * gphys[tj][2]);
                                A[(size_t)(c * nd + ti) * N + c * nd + tj] += w * s;
                            }
                    }
        }
    }
    /* interior faces, each once, all four blocks */
    if (flags & OR_FACE) {
        for (long km = 0; km < p->n_cells; ++km)
            for (int d = 0; d < 3; ++d) {
                long kp = p->nbr[6 * km + 2 * d + 1];
                if (kp < 0) continue;
                double sigma = face_sigma(p, &r, km, d);
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        double nrm[3], ds, xim[3], xip[3], pos[3], Jm[3][3], Jp[3][3], Km[3][3], Kp[3][3];
                        face_normal(&r, cell_nodes(p, &r, km), d, a, b, nrm, &ds);
                        face_point(&r, d, 1, a, b, xim);
                        face_point(&r, d, 0, a, b, xip);
                        geom_at(&r, cell_nodes(p, &r, km), xim, pos, Jm);
                        geom_at(&r, cell_nodes(p, &r, kp), xip, pos, Jp);
                        inv_transpose(Jm, det3(Jm), Km);
                        inv_transpose(Jp, det3(Jp), Kp);
                        basis_at(&r, xim, phi, dphi);
                        basis_at(&r, xip, phi2, dphi2);
                        double bm = 0, bp = 0;
                        for (int e = 0; e < nd; ++e) {
                            bm += phi[e] * p->beta[km * nd + e];
                            bp += phi2[e] * p->beta[kp * nd + e];
                            matvec3(Km, dphi[e], gphys[e]);
                            matvec3(Kp, dphi2[e], gphys2[e]);
                        }
                        double pen = sigma * 0.5 * (bm + bp);
                        /* side s in {0: minus, 1: plus}: value, normal derivative, beta, sign */
                        for (int st = 0; st < 2; ++st)        /* test side */
                            for (int su = 0; su < 2; ++su) {  /* trial side */
                                long ct = st ? kp : km, cu = su ? kp : km;
                                const double *vt = st ? phi2 : phi, *vu = su ? phi2 : phi;
                                double (*gt)[3] = st ? gphys2 : gphys;
                                double (*gu)[3] = su ? gphys2 : gphys;
                                double bt = st ? bp : bm, bu = su ? bp : bm;
                                double zt = st ? -1.0 : 1.0, zu = su ? -1.0 : 1.0;
                                for (int ti = 0; ti < nd; ++ti) {
                                    double dnt = nrm[0] * gt[ti][0] + nrm[1] * gt[ti][1] + nrm[2] * gt[ti][2];
                                    for (int tj = 0; tj < nd; ++tj) {
                                        double dnu = nrm[0] * gu[tj][0] + nrm[1] * gu[tj][1] + nrm[2] * gu[tj][2];
                                        double s = -0.5 * bu * dnu * zt * vt[ti]
                                                   - 0.5 * bt * dnt * zu * vu[tj]
                                                   + pen * zu * vu[tj] * zt * vt[ti];
                                        A[(size_t)(ct * nd + ti) * N + cu * nd + tj] += ds * s;
                                    }
                                }
                            }
                    }
            }
    }
    /* non-conforming quarter faces, each once, all four blocks */
    if ((flags & OR_FACE) && p->n_hang > 0) {
        hang_pt hp;
        hang_alloc(&hp, nd);
        for (long h = 0; h < p->n_hang; ++h) {
            const long *rec = p->hang + 4 * h;
            const long cells[2] = {rec[0], rec[2]};
            const int minus = (rec[1] & 1) ? 0 : 1;
            const double sigma = hang_sigma(p, &r, rec);
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    double nrm[3], ds;
                    hang_normal(p, &r, rec, a, b, nrm, &ds);
                    hang_eval(p, &r, rec, a, b, &hp);
                    for (int side = 0; side < 2; ++side)
                        for (int e = 0; e < nd; ++e)
                            matvec3(hp.K[side], hp.dphi[side][e], side ? gphys2[e] : gphys[e]);
                    double pen = sigma * 0.5 * (hp.beta[0] + hp.beta[1]);
                    for (int st = 0; st < 2; ++st)
                        for (int su = 0; su < 2; ++su) {
                            double (*gt)[3] = st ? gphys2 : gphys, (*gu)[3] = su ? gphys2 : gphys;
                            const double *vt = hp.phi[st], *vu = hp.phi[su];
                            double zt = st == minus ? 1.0 : -1.0, zu = su == minus ? 1.0 : -1.0;
                            for (int ti = 0; ti < nd; ++ti) {
                                double dnt = nrm[0] * gt[ti][0] + nrm[1] * gt[ti][1] + nrm[2] * gt[ti][2];
                                for (int tj = 0; tj < nd; ++tj) {
                                    double dnu = nrm[0] * gu[tj][0] + nrm[1] * gu[tj][1] + nrm[2] * gu[tj][2];
                                    double s = -0.5 * hp.beta[su] * dnu * zt * vt[ti]
                                               - 0.5 * hp.beta[st] * dnt * zu * vu[tj]
                                               + pen * zu * vu[tj] * zt * vt[ti];
                                    A[(size_t)(cells[st] * nd + ti) * N + cells[su] * nd + tj] += ds * s;
                                }
                            }
                        }
                }
        }
        hang_free(&hp);
    }
    free(phi); free(phi2); free(dphi); free(dphi2); free(gphys); free(gphys2);
}

/* ------------------------------------------------------------------------ */
/* separable cell-block preconditioner                                      */
/* ------------------------------------------------------------------------ */

/* per-cell data of the separable block: lengths l_d (mean over GL points of
 * the column norms |J e_d|), volume-weighted means of alpha and beta, and the
 * penalties at the two ends of each direction (-1 where the end is a
 * boundary). */
void or_bj_cell_data(const or_prob *p, long c, double ell[3], double *abar,
                     double *bbar, double sig[3][2])
{
    ref_t r; ref_init(&r, p->k, p->g);
    int n = r.n, nd = r.nd;
    double *phi = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    double vol = 0, sa = 0, sb = 0;
    ell[0] = ell[1] = ell[2] = 0.0;
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3];
                geom_at(&r, cell_nodes(p, &r, c), xi, x, J);
                double w = r.wq[i] * r.wq[j] * r.wq[l] * det3(J);
                basis_at(&r, xi, phi, dphi);
                vol += w;
                sa += w * field_at(phi, p->alpha + c * nd, nd);
                sb += w * field_at(phi, p->beta + c * nd, nd);
                for (int d = 0; d < 3; ++d)
                    ell[d] += sqrt(J[0][d] * J[0][d] + J[1][d] * J[1][d] + J[2][d] * J[2][d]);
            }
    for (int d = 0; d < 3; ++d) {
        ell[d] /= nd;
        long lo = p->nbr[6 * c + 2 * d];
        sig[d][0] = lo >= 0 ? face_sigma(p, &r, lo, d) : -1.0;
        sig[d][1] = face_sigma(p, &r, c, d);
        /* a non-conforming end: the penalty of the fine cell's quarter face,
           or the area-weighted mean over the four quarters of a coarse face */
        for (int e = 0; e < 2; ++e) {
            if (p->nbr[6 * c + 2 * d + e] != -2) continue;
            double ssum = 0.0, asum = 0.0;
            for (long h = 0; h < p->n_hang; ++h) {
                const long *rec = p->hang + 4 * h;
                int f = rec[0] == c ? (int)rec[1] : (rec[2] == c ? (int)(rec[1] ^ 1) : -1);
                if (f != 2 * d + e) continue;
                double area = 0.0, nrm[3], ds;
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        hang_normal(p, &r, rec, a, b, nrm, &ds);
                        area += ds;
                    }
                ssum += area * hang_sigma(p, &r, rec);
                asum += area;
            }
            sig[d][e] = asum > 0.0 ? ssum / asum : -1.0;
        }
    }
    *abar = sa / vol;
    *bbar = sb / vol;
    free(phi); free(dphi);
}

/* 1-D reference mass and SIP blocks on [0,1] for one direction of a cell */
static void one_d_blocks(const ref_t *r, double ell, const double sig[2],
                         double M[MAXN][MAXN], double L[MAXN][MAXN])
{
    int n = r->n;
    double v[MAXN], d[MAXN], ve[2][MAXN], de[2][MAXN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) M[i][j] = L[i][j] = 0.0;
    for (int q = 0; q < n; ++q) {
        or_lagrange(n, r->xl, r->xq[q], v, d);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                M[i][j] += r->wq[q] * v[i] * v[j];
                L[i][j] += r->wq[q] * d[i] * d[j];
            }
    }
    or_lagrange(n, r->xl, 0.0, ve[0], de[0]);
    or_lagrange(n, r->xl, 1.0, ve[1], de[1]);
    for (int e = 0; e < 2; ++e) {
        if (sig[e] < 0) continue;
        double nh = e ? 1.0 : -1.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                L[i][j] += -0.5 * nh * (de[e][i] * ve[e][j] + ve[e][i] * de[e][j])
                           + sig[e] * ell * ve[e][i] * ve[e][j];
    }
}

/* dense Ahat_K = abar lx ly lz M(x)M(x)M + bbar [ (ly lz/lx) M(x)M(x)Lx + ... ],
 * the x factor acting on the fastest local index */
void or_bj_sep_block(const or_prob *p, long c, double *Ab)
{
    ref_t r; ref_init(&r, p->k, p->g);
    int n = r.n, nd = r.nd;
    double ell[3], abar, bbar, sig[3][2];
    or_bj_cell_data(p, c, ell, &abar, &bbar, sig);
    double M[3][MAXN][MAXN], L[3][MAXN][MAXN];
    for (int d = 0; d < 3; ++d) one_d_blocks(&r, ell[d], sig[d], M[d], L[d]);
    double cm = abar * ell[0] * ell[1] * ell[2];
    double cx = bbar * ell[1] * ell[2] / ell[0];
    double cy = bbar * ell[0] * ell[2] / ell[1];
    double cz = bbar * ell[0] * ell[1] / ell[2];
    for (int l = 0; l < n; ++l) for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i)
        for (int l2 = 0; l2 < n; ++l2) for (int j2 = 0; j2 < n; ++j2) for (int i2 = 0; i2 < n; ++i2) {
            int row = i + n * (j + n * l), col = i2 + n * (j2 + n * l2);
            double mx = M[0][i][i2], my = M[1][j][j2], mz = M[2][l][l2];
            Ab[row * nd + col] = cm * mx * my * mz + cx * L[0][i][i2] * my * mz
                               + cy * mx * L[1][j][j2] * mz + cz * mx * my * L[2][l][l2];
        }
}

/* in-place Cholesky solve of a dense SPD system (row-major A, overwritten) */
static int chol_solve(int nd, double *A, double *x)
{
    for (int j = 0; j < nd; ++j) {
        double s = A[j * nd + j];
        for (int m = 0; m < j; ++m) s -= A[j * nd + m] * A[j * nd + m];
        if (!(s > 0.0)) return 1;
        double ljj = sqrt(s);
        A[j * nd + j] = ljj;
        for (int i = j + 1; i < nd; ++i) {
            double t = A[i * nd + j];
            for (int m = 0; m < j; ++m) t -= A[i * nd + m] * A[j * nd + m];
            A[i * nd + j] = t / ljj;
        }
    }
    for (int i = 0; i < nd; ++i) {
        double t = x[i];
        for (int m = 0; m < i; ++m) t -= A[i * nd + m] * x[m];
        x[i] = t / A[i * nd + i];
    }
    for (int i = nd - 1; i >= 0; --i) {
        double t = x[i];
        for (int m = i + 1; m < nd; ++m) t -= A[m * nd + i] * x[m];
        x[i] = t / A[i * nd + i];
    }
    return 0;
}

int or_bj_sep_apply(const or_prob *p, const double *rv, double *zv)
{
    int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
    int bad = 0;
#pragma omp parallel reduction(|:bad)
    {
        double *Ab = malloc(sizeof(double) * nd * nd);
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < p->n_cells; ++c) {
            or_bj_sep_block(p, c, Ab);
            for (int a = 0; a < nd; ++a) zv[c * nd + a] = rv[c * nd + a];
            bad |= chol_solve(nd, Ab, zv + c * nd);
        }
        free(Ab);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* cell mass blocks (the block-diagonal matrix whose fast inverse section 3.3 */
/* builds from 1-D factors)                                                  */
/* ------------------------------------------------------------------------ */

/* M_K[i][j] = sum_q w_q detJ_q alpha_q phi_i phi_j, by direct quadrature */
void or_mass_block(const or_prob *p, long c, double *Mb)
{
    ref_t r; ref_init(&r, p->k, p->g);
    const int nd = r.nd, n = r.n;
    double *phi = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    for (int a = 0; a < nd * nd; ++a) Mb[a] = 0.0;
    const double *X = cell_nodes(p, &r, c);
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3];
                geom_at(&r, X, xi, x, J);
                double w = r.wq[i] * r.wq[j] * r.wq[l] * det3(J);
                basis_at(&r, xi, phi, dphi);
                double al = field_at(phi, p->alpha + c * nd, nd);
                for (int a = 0; a < nd; ++a)
                    for (int b = 0; b < nd; ++b) Mb[a * nd + b] += w * al * phi[a] * phi[b];
            }
    free(phi); free(dphi);
}

/* z = M_K^{-1} r on every cell (dense Cholesky); nonzero if a block is not
 * positive definite */
int or_mass_block_apply(const or_prob *p, const double *rv, double *zv)
{
    int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
    int bad = 0;
#pragma omp parallel reduction(|:bad)
    {
        double *Mb = malloc(sizeof(double) * nd * nd);
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < p->n_cells; ++c) {
            or_mass_block(p, c, Mb);
            for (int a = 0; a < nd; ++a) zv[c * nd + a] = rv[c * nd + a];
            bad |= chol_solve(nd, Mb, zv + c * nd);
        }
        free(Mb);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* velocity-pressure coupling of the IMEX stage (section 2: the discrete     */
/* momentum and energy equations A U + B P = F, C U + D P = G, and the       */
/* pressure system D P + C A^-1 (F - B P) = G).  The paper names these       */
/* matrices without giving them; they are read here from the stage           */
/* equations with central fluxes:                                            */
/*   (B p)_{c,i} = tau [ -sum_K int_K p d_c phi_i                            */
/*                       + sum_K int_dK p^ phi_i n_{K,c} ],                  */
/*     p^ = {p} on interior faces, the own trace on boundary faces;          */
/*   (C u)_i = tau [ -sum_K int_K hr u . grad Psi_i                          */
/*                   + sum_F interior int_F {hr u . n} [Psi_i] ],            */
/*     no flux through boundary faces;                                       */
/* hr is the nodal field of h rho (enthalpy times density), tau = a_ll dt.   */
/* Velocity vectors are component-major: u3[c * n_dofs + dof].               */
/* ------------------------------------------------------------------------ */

/* outward unit normal and surface element of a cell on its own (d, plus)
 * face at tangential GL point (a, b), from the cell's own map */
static void face_normal_own(const ref_t *r, const double *X, int d, int plus, int a, int b,
                            double nrm[3], double *ds)
{
    double xi[3], x[3], J[3][3], K[3][3];
    face_point(r, d, plus, a, b, xi);
    geom_at(r, X, xi, x, J);
    double det = det3(J);
    inv_transpose(J, det, K);
    double e[3] = {0, 0, 0}, m[3];
    e[d] = 1.0;
    matvec3(K, e, m);
    double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    double s = plus ? 1.0 : -1.0;
    for (int q = 0; q < 3; ++q) nrm[q] = s * m[q] / len;
    *ds = r->wq[a] * r->wq[b] * det * len;
}

/* (B p) on the test functions of cell c: yc[3][nd] */
static void grad_one_cell(const or_prob *p, double tau, long c, const double *pv, double *yc)
{
    ref_t r; ref_init(&r, p->k, p->g);
    const int nd = r.nd, n = r.n;
    double *phi = malloc(sizeof(double) * nd), *phiB = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    double (*dphiB)[3] = malloc(sizeof(double) * 3 * nd);
    for (int a = 0; a < 3 * nd; ++a) yc[a] = 0.0;
    const double *X = cell_nodes(p, &r, c);
    /* cell term: -int_K p grad phi_i */
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3], K[3][3];
                geom_at(&r, X, xi, x, J);
                double det = det3(J);
                inv_transpose(J, det, K);
                double w = r.wq[i] * r.wq[j] * r.wq[l] * det;
                basis_at(&r, xi, phi, dphi);
                double pq = field_at(phi, pv + c * nd, nd);
                for (int a = 0; a < nd; ++a) {
                    double gv[3];
                    matvec3(K, dphi[a], gv);
                    for (int cc = 0; cc < 3; ++cc) yc[cc * nd + a] -= tau * w * pq * gv[cc];
                }
            }
    /* face terms: int_dK p^ phi_i n_K */
    for (int d = 0; d < 3; ++d)
        for (int side = 0; side < 2; ++side) {
            long nb = p->nbr[6 * c + 2 * d + side];
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    double nrm[3], ds, ph, xi[3];
                    const double *tphi;
                    if (nb < 0) {
                        face_normal_own(&r, X, d, side, a, b, nrm, &ds);
                        face_point(&r, d, side, a, b, xi);
                        basis_at(&r, xi, phi, dphi);
                        ph = field_at(phi, pv + c * nd, nd);
                        tphi = phi;
                    } else {
                        long km = side ? c : nb, kp = side ? nb : c;
                        double xim[3], xip[3];
                        face_normal(&r, cell_nodes(p, &r, km), d, a, b, nrm, &ds);
                        face_point(&r, d, 1, a, b, xim);
                        face_point(&r, d, 0, a, b, xip);
                        basis_at(&r, xim, phi, dphi);
                        basis_at(&r, xip, phiB, dphiB);
                        ph = 0.5 * (field_at(phi, pv + km * nd, nd) + field_at(phiB, pv + kp * nd, nd));
                        tphi = side ? phi : phiB;
                        if (!side)
                            for (int q = 0; q < 3; ++q) nrm[q] = -nrm[q];   /* outward for c */
                    }
                    for (int e = 0; e < nd; ++e)
                        for (int cc = 0; cc < 3; ++cc)
                            yc[cc * nd + e] += tau * ds * ph * tphi[e] * nrm[cc];
                }
        }
    free(phi); free(phiB); free(dphi); free(dphiB);
}

void or_grad_apply(const or_prob *p, double tau, const double *pv, double *u3)
{
    const int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
    const long nt = p->n_cells * nd;
#pragma omp parallel
    {
        double *tmp = malloc(sizeof(double) * 3 * nd);
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < p->n_cells; ++c) {
            grad_one_cell(p, tau, c, pv, tmp);
            for (int cc = 0; cc < 3; ++cc)
                for (int a = 0; a < nd; ++a) u3[cc * nt + c * nd + a] = tmp[cc * nd + a];
        }
        free(tmp);
    }
}

/* (C u) on the test functions of cell c: yc[nd] */
static void div_one_cell(const or_prob *p, double tau, const double *hr, long c,
                         const double *u3, double *yc)
{
    ref_t r; ref_init(&r, p->k, p->g);
    const int nd = r.nd, n = r.n;
    const long nt = p->n_cells * nd;
    double *phi = malloc(sizeof(double) * nd), *phiB = malloc(sizeof(double) * nd);
    double (*dphi)[3] = malloc(sizeof(double) * 3 * nd);
    double (*dphiB)[3] = malloc(sizeof(double) * 3 * nd);
    for (int a = 0; a < nd; ++a) yc[a] = 0.0;
    const double *X = cell_nodes(p, &r, c);
    /* cell term: -int_K hr u . grad Psi_i */
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xi[3] = {r.xq[i], r.xq[j], r.xq[l]}, x[3], J[3][3], K[3][3];
                geom_at(&r, X, xi, x, J);
                double det = det3(J);
                inv_transpose(J, det, K);
                double w = r.wq[i] * r.wq[j] * r.wq[l] * det;
                basis_at(&r, xi, phi, dphi);
                double hq = field_at(phi, hr + c * nd, nd);
                double uq[3];
                for (int cc = 0; cc < 3; ++cc) uq[cc] = field_at(phi, u3 + cc * nt + c * nd, nd);
                for (int a = 0; a < nd; ++a) {
                    double gv[3];
                    matvec3(K, dphi[a], gv);
                    yc[a] -= tau * w * hq * (uq[0] * gv[0] + uq[1] * gv[1] + uq[2] * gv[2]);
                }
            }
    /* interior faces: int_F {hr u . n} [Psi_i], n the minus-side normal */
    for (int d = 0; d < 3; ++d)
        for (int side = 0; side < 2; ++side) {
            long nb = p->nbr[6 * c + 2 * d + side];
            if (nb < 0) continue;
            long km = side ? c : nb, kp = side ? nb : c;
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    double nrm[3], ds, xim[3], xip[3];
                    face_normal(&r, cell_nodes(p, &r, km), d, a, b, nrm, &ds);
                    face_point(&r, d, 1, a, b, xim);
                    face_point(&r, d, 0, a, b, xip);
                    basis_at(&r, xim, phi, dphi);
                    basis_at(&r, xip, phiB, dphiB);
                    double fm = 0.0, fp = 0.0;
                    for (int cc = 0; cc < 3; ++cc) {
                        fm += field_at(phi, u3 + cc * nt + km * nd, nd) * nrm[cc];
                        fp += field_at(phiB, u3 + cc * nt + kp * nd, nd) * nrm[cc];
                    }
                    fm *= field_at(phi, hr + km * nd, nd);
                    fp *= field_at(phiB, hr + kp * nd, nd);
                    const double avg = 0.5 * (fm + fp);
                    const double *tphi = side ? phi : phiB;
                    const double sgn = side ? 1.0 : -1.0;
                    for (int e = 0; e < nd; ++e) yc[e] += tau * ds * avg * sgn * tphi[e];
                }
        }
    free(phi); free(phiB); free(dphi); free(dphiB);
}

void or_div_apply(const or_prob *p, double tau, const double *hr, const double *u3, double *qv)
{
    const int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (long c = 0; c < p->n_cells; ++c) div_one_cell(p, tau, hr, c, u3, qv + c * nd);
}

/* the same restricted to listed cells: out[s][3][nd] = (B p) on cells[s] */
void or_grad_apply_cells(const or_prob *p, double tau, const long *cells, long m, const double *pv,
                         double *out)
{
    const int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < m; ++s) grad_one_cell(p, tau, cells[s], pv, out + s * 3 * nd);
}

/* out[s][nd] = (C u) on cells[s]; u3 is read on the listed cells and their
 * face neighbours only */
void or_div_apply_cells(const or_prob *p, double tau, const double *hr, const long *cells, long m,
                        const double *u3, double *out)
{
    const int nd = (p->k + 1) * (p->k + 1) * (p->k + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < m; ++s) div_one_cell(p, tau, hr, cells[s], u3, out + s * nd);
}
