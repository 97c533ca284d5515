// Geometry and coefficient set-up (FP64): cell metric terms, face normals,
// surface elements and penalties, merged per-quadrature-point operator data,
// the separable block-Jacobi eigen-tables and dof coordinates.
//
// Everything here runs once per mesh (setup_mesh) or once per coefficient
// update (set_coefficients, redone each fixed-point iteration of the paper's
// pressure solve, section 3.1), so it favours clarity over speed.
#include "common.hpp"

#include <cmath>

namespace hx {
namespace {

// Lagrange basis through the equispaced nodes a/g, a = 0..g (the geometry
// nodes of the mesh format): values and derivatives at t.
__device__ inline void lag_equi(int ng, double t, double *v, double *d)
{
    const double g = ng - 1;
    for (int i = 0; i < ng; ++i) {
        const double xi = i / g;
        double val = 1.0, der = 0.0;
        for (int m = 0; m < ng; ++m) {
            if (m == i) continue;
            const double xm = m / g;
            const double f = (t - xm) / (xi - xm);
            der = der * f + val / (xi - xm);
            val *= f;
        }
        v[i] = val;
        d[i] = der;
    }
}

// x(xi) and J = dx/dxi of one cell from its geometry nodes X[(g+1)^3][3].
__device__ inline void cell_map(const double *__restrict__ X, int ng, const double xi[3],
                                double x[3], double J[3][3])
{
    double v[3][MAXG + 1], d[3][MAXG + 1];
    for (int c = 0; c < 3; ++c) lag_equi(ng, xi[c], v[c], d[c]);
    for (int r = 0; r < 3; ++r) x[r] = J[r][0] = J[r][1] = J[r][2] = 0.0;
    for (int cz = 0; cz < ng; ++cz)
        for (int cy = 0; cy < ng; ++cy) {
            const double vyz = v[1][cy] * v[2][cz], dyz = d[1][cy] * v[2][cz], yzd = v[1][cy] * d[2][cz];
            for (int cx = 0; cx < ng; ++cx) {
                const double *P = X + 3 * (cx + ng * (cy + ng * cz));
                const double s = v[0][cx] * vyz, s0 = d[0][cx] * vyz, s1 = v[0][cx] * dyz,
                             s2 = v[0][cx] * yzd;
                for (int r = 0; r < 3; ++r) {
                    const double p = P[r];
                    x[r] += s * p;
                    J[r][0] += s0 * p;
                    J[r][1] += s1 * p;
                    J[r][2] += s2 * p;
                }
            }
        }
}

__device__ inline double det3(const double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Ji = J^{-1}
__device__ inline void inv3(const double J[3][3], double det, double Ji[3][3])
{
    const double id = 1.0 / det;
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
}

__device__ inline int lidx(int n, int i, int j, int l) { return i + n * (j + n * l); }

// local index of the point with coordinate m along d and tangential (p, r),
// t1 < t2 the other two directions
__device__ inline int layer_idx(int n, int d, int m, int p, int r)
{
    int c[3];
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    c[d] = m;
    c[t1] = p;
    c[t2] = r;
    return lidx(n, c[0], c[1], c[2]);
}

__device__ inline void face_xi(const RefTab64 *T, int d, int plus, int a, int b, double xi[3])
{
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    xi[d] = plus ? 1.0 : 0.0;
    xi[t1] = T->xq[a];
    xi[t2] = T->xq[b];
}

// -------------------------------------------------------------------------
// per cell: volume, mean column lengths l_d, minimum detJ (thread per cell)
// -------------------------------------------------------------------------
__global__ void k_cell_geometry(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                                const RefTab64 *__restrict__ T, double *vol, double *ell,
                                double *mindet)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const double *X = nodes + c * (int64_t)ng * ng * ng * 3;
    double v = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0, md = 1e300;
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xi[3] = {T->xq[i], T->xq[j], T->xq[l]}, x[3], J[3][3];
                cell_map(X, ng, xi, x, J);
                const double det = det3(J);
                md = fmin(md, det);
                v += T->wq[i] * T->wq[j] * T->wq[l] * det;
                e0 += sqrt(J[0][0] * J[0][0] + J[1][0] * J[1][0] + J[2][0] * J[2][0]);
                e1 += sqrt(J[0][1] * J[0][1] + J[1][1] * J[1][1] + J[2][1] * J[2][1]);
                e2 += sqrt(J[0][2] * J[0][2] + J[1][2] * J[1][2] + J[2][2] * J[2][2]);
            }
    const double inv = 1.0 / (n * n * n);
    vol[c] = v;
    ell[3 * c + 0] = e0 * inv;
    ell[3 * c + 1] = e1 * inv;
    ell[3 * c + 2] = e2 * inv;
    mindet[c] = md;
}

// -------------------------------------------------------------------------
// penalty of the +d face of each cell (thread per (cell, d))
// -------------------------------------------------------------------------
__global__ void k_face_sigma(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                             const int32_t *__restrict__ nbr, const RefTab64 *__restrict__ T,
                             const double *__restrict__ vol, double P, double *sigma)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n_cells) return;
    const int64_t c = t / 3;
    const int d = (int)(t % 3);
    const int32_t nb = nbr[6 * c + 2 * d + 1];
    if (nb < 0) {
        sigma[t] = -1.0;
        return;
    }
    const double *X = nodes + c * (int64_t)ng * ng * ng * 3;
    double area = 0.0;
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            double xi[3], x[3], J[3][3], Ji[3][3];
            face_xi(T, d, 1, a, b, xi);
            cell_map(X, ng, xi, x, J);
            const double det = det3(J);
            inv3(J, det, Ji);
            // |J^{-T} e_d| = norm of row d of J^{-1}
            const double len = sqrt(Ji[d][0] * Ji[d][0] + Ji[d][1] * Ji[d][1] + Ji[d][2] * Ji[d][2]);
            area += T->wq[a] * T->wq[b] * det * len;
        }
    const double r = fmax(area / vol[c], area / vol[nb]);
    sigma[t] = P * (double)(n * n) * r;
}

// -------------------------------------------------------------------------
// generalised eigenproblems of the separable block (thread per (cell, d)):
// L_d s = lambda M s with L_d the 1-D SIP block of the cell in direction d.
// -------------------------------------------------------------------------
template <int N>
__device__ void jacobi_eig(double (&A)[N][N], double (&V)[N][N])
{
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                tot += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-34 * tot) break;
        for (int p = 0; p < N - 1; ++p)
            for (int q = p + 1; q < N; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < N; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < N; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < N; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq;
                    V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
}

template <int N>
__global__ void k_bj_eigen(int64_t n_cells, const int32_t *__restrict__ nbr,
                           const RefTab64 *__restrict__ T, const double *__restrict__ ell,
                           const double *__restrict__ sigma, const double *__restrict__ endsig,
                           double *S64, float *S32, double *L64, float *L32)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n_cells) return;
    const int64_t c = t / 3;
    const int d = (int)(t % 3);
    const double l = ell[3 * c + d];
    const int32_t lo = nbr[6 * c + 2 * d], hi = nbr[6 * c + 2 * d + 1];
    // a non-conforming end (neighbour -2) takes its penalty from endsig
    const double sig_lo = lo >= 0 ? sigma[3 * (int64_t)lo + d] : (lo == -2 ? endsig[6 * c + 2 * d] : -1.0);
    const double sig_hi = hi >= 0 ? sigma[3 * c + d] : (hi == -2 ? endsig[6 * c + 2 * d + 1] : -1.0);
    double L[N][N];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) L[i][j] = T->L0[i * N + j];
    // end terms; the GLL basis is 1 at its own end node and 0 at the others
    if (sig_lo >= 0.0) {   // end 0, outward reference normal -1
        for (int i = 0; i < N; ++i) {
            L[i][0] += 0.5 * T->DL[0][i];
            L[0][i] += 0.5 * T->DL[0][i];
        }
        L[0][0] += sig_lo * l;
    }
    if (sig_hi >= 0.0) {   // end 1, outward reference normal +1
        for (int i = 0; i < N; ++i) {
            L[i][N - 1] -= 0.5 * T->DL[1][i];
            L[N - 1][i] -= 0.5 * T->DL[1][i];
        }
        L[N - 1][N - 1] += sig_hi * l;
    }
    // C = Cinv L Cinv^T
    double A[N][N], tmp[N][N], V[N][N];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int r = 0; r < N; ++r) s += T->Cinv[i * N + r] * L[r][j];
            tmp[i][j] = s;
        }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int r = 0; r < N; ++r) s += tmp[i][r] * T->Cinv[j * N + r];
            A[i][j] = s;
        }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < i; ++j) A[i][j] = A[j][i] = 0.5 * (A[i][j] + A[j][i]);
    jacobi_eig<N>(A, V);
    // S = Cinv^T V, stored row-major S[i][m]
    double *S = S64 + t * N * N;
    float *Sf = S32 + t * N * N;
    for (int i = 0; i < N; ++i)
        for (int m = 0; m < N; ++m) {
            double s = 0.0;
            for (int r = 0; r < N; ++r) s += T->Cinv[r * N + i] * V[r][m];
            S[i * N + m] = s;
            Sf[i * N + m] = (float)s;
        }
    for (int m = 0; m < N; ++m) {
        L64[t * N + m] = A[m][m];
        L32[t * N + m] = (float)A[m][m];
    }
}

// -------------------------------------------------------------------------
// Geometric factors, once per mesh (block per cell / thread per face point).
// Cell quadrature point q:   cg[0] = w detJ,
//                            cg[1..6] = w detJ (J^-1 J^-T)_{xx,xy,xz,yy,yz,zz}.
// Point (a, b) of the +d face of a cell (a, b along the first and second
// tangential direction, stored at b + n a):
//                            fg[0..2] = ds J-^{-1} n,  fg[3..5] = ds J+^{-1} n
// (components in the face's own order: normal direction d, first, second
// tangential), fg[6] = ds / 2, with n and ds from the minus cell; zero on
// boundary faces.  Coefficients multiply these in k_set_cell / k_set_face.
// -------------------------------------------------------------------------
__global__ void k_cell_geofac(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                              const RefTab64 *__restrict__ T, double *cellgeo)
{
    const int nd = n * n * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_cells * nd) return;
    const int64_t c = t / nd;
    const int q = (int)(t % nd);
    const int i = q % n, j = (q / n) % n, l = q / (n * n);
    double xi[3] = {T->xq[i], T->xq[j], T->xq[l]}, x[3], J[3][3], Ji[3][3];
    cell_map(nodes + c * (int64_t)ng * ng * ng * 3, ng, xi, x, J);
    const double det = det3(J);
    inv3(J, det, Ji);
    const double w = T->wq[i] * T->wq[j] * T->wq[l] * det;
    double *dst = cellgeo + c * 7 * nd + q;
    dst[0] = w;
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int s = 0; s < 6; ++s) {
        const int A = pa[s], Bq = pb[s];
        dst[(1 + s) * nd] = w * (Ji[A][0] * Ji[Bq][0] + Ji[A][1] * Ji[Bq][1] + Ji[A][2] * Ji[Bq][2]);
    }
}

__global__ void k_face_geofac(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                              const int32_t *__restrict__ nbr, const RefTab64 *__restrict__ T,
                              double *facegeo)
{
    const int nf = n * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n_cells * nf) return;
    const int pt = (int)(t % nf);
    const int64_t cd = t / nf;
    const int64_t c = cd / 3;
    const int d = (int)(cd % 3);
    const int b = pt % n, a = pt / n;
    double *dst = facegeo + cd * 7 * nf + pt;
    const int32_t nb = nbr[6 * c + 2 * d + 1];
    if (nb < 0) {
        for (int s = 0; s < 7; ++s) dst[s * nf] = 0.0;
        return;
    }
    double xim[3], xip[3], x[3], Jm[3][3], Jp[3][3], Jmi[3][3], Jpi[3][3];
    face_xi(T, d, 1, a, b, xim);
    face_xi(T, d, 0, a, b, xip);
    const int64_t gsz = (int64_t)ng * ng * ng * 3;
    cell_map(nodes + c * gsz, ng, xim, x, Jm);
    cell_map(nodes + (int64_t)nb * gsz, ng, xip, x, Jp);
    const double detm = det3(Jm), detp = det3(Jp);
    inv3(Jm, detm, Jmi);
    inv3(Jp, detp, Jpi);
    // J^{-T} e_d is row d of J^{-1}
    double nv[3] = {Jmi[d][0], Jmi[d][1], Jmi[d][2]};
    const double len = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int r = 0; r < 3; ++r) nv[r] /= len;
    const double ds = T->wq[a] * T->wq[b] * detm * len;
    const int dir[3] = {d, d == 0 ? 1 : 0, d == 2 ? 1 : 2};
    for (int k = 0; k < 3; ++k) {
        const int r = dir[k];
        dst[k * nf] = ds * (Jmi[r][0] * nv[0] + Jmi[r][1] * nv[1] + Jmi[r][2] * nv[2]);
        dst[(3 + k) * nf] = ds * (Jpi[r][0] * nv[0] + Jpi[r][1] * nv[1] + Jpi[r][2] * nv[2]);
    }
    dst[6 * nf] = 0.5 * ds;
}

// -------------------------------------------------------------------------
// Affine cells (thread per cell): the geometry nodes are the image of the
// reference nodes under x0 + A xi, A from the three edges at the first corner,
// to 1e-14 of the longest edge.  Their Jacobian is constant, so the operator
// may read one J^-1 J^-T per cell and the coefficients at the points instead
// of the seven merged values per point.  The per-cell constants are taken
// from the general geometric factors of the first Gauss point:
// kk = (w detJ J^-1 J^-T) / (w detJ), and detJ.
// -------------------------------------------------------------------------
__global__ void k_affine_detect(const double *__restrict__ nodes, int ng, int nd, int64_t n_cells,
                                const RefTab64 *__restrict__ T, const double *__restrict__ cellgeo,
                                uint8_t *ctype, double *kk64, float *kk32)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const double *X = nodes + c * (int64_t)ng * ng * ng * 3;
    const int g = ng - 1;
    const int corner[3] = {g, g * ng, g * ng * ng};
    double A[3][3], diam = 0.0;
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int r = 0; r < 3; ++r) {
            A[r][d] = X[3 * corner[d] + r] - X[r];
            s += A[r][d] * A[r][d];
        }
        diam = fmax(diam, sqrt(s));
    }
    double dev = 0.0;
    for (int az = 0; az < ng; ++az)
        for (int ay = 0; ay < ng; ++ay)
            for (int ax = 0; ax < ng; ++ax) {
                const double xi[3] = {(double)ax / g, (double)ay / g, (double)az / g};
                const double *P = X + 3 * (ax + ng * (ay + ng * az));
                for (int r = 0; r < 3; ++r) {
                    const double pr = X[r] + A[r][0] * xi[0] + A[r][1] * xi[1] + A[r][2] * xi[2];
                    dev = fmax(dev, fabs(P[r] - pr));
                }
            }
    ctype[c] = dev <= 1e-14 * diam ? 1 : 0;
    const double *geo = cellgeo + c * 7 * nd;
    const double w0 = geo[0];
    for (int s = 0; s < 6; ++s) {
        const double v = geo[(1 + s) * nd] / w0;
        kk64[8 * c + s] = v;
        kk32[8 * c + s] = (float)v;
    }
    const double det = w0 / (T->wq[0] * T->wq[0] * T->wq[0]);
    kk64[8 * c + 6] = det;
    kk32[8 * c + 6] = (float)det;
    kk64[8 * c + 7] = 0.0;
    kk32[8 * c + 7] = 0.0f;
}

// -------------------------------------------------------------------------
// merged cell data from the coefficients (block per cell, thread per point):
//   m = alpha_q w detJ,  G = beta_q w detJ J^-1 J^-T  (alpha_q, beta_q: the
// nodal fields at the Gauss point), plus the cell means of the separable
// block (volume-weighted alpha, beta) and the network's coefficient feature
// -------------------------------------------------------------------------
__global__ void k_set_cell(int n, const RefTab64 *__restrict__ T, const double *__restrict__ alpha,
                           const double *__restrict__ beta, const double *__restrict__ ell,
                           const double *__restrict__ cellgeo, double *cell64, float *cell32,
                           double *bjC64, float *bjC32, double *coef_feat,
                           const uint8_t *__restrict__ ctype, double *acell64, float *acell32)
{
    const int64_t c = blockIdx.x;
    const int nd = n * n * n;
    const int q = threadIdx.x;
    double sw = 0.0, sa = 0.0, sb = 0.0;
    if (q < nd) {
        const int i = q % n, j = (q / n) % n, l = q / (n * n);
        const double *ac = alpha + c * nd, *bc = beta + c * nd;
        double aq = 0.0, bq = 0.0;
        for (int l2 = 0; l2 < n; ++l2)
            for (int j2 = 0; j2 < n; ++j2) {
                const double byz = T->B[j * n + j2] * T->B[l * n + l2];
                for (int i2 = 0; i2 < n; ++i2) {
                    const double wgt = T->B[i * n + i2] * byz;
                    const int e = lidx(n, i2, j2, l2);
                    aq += wgt * ac[e];
                    bq += wgt * bc[e];
                }
            }
        const double *g = cellgeo + c * 7 * nd + q;
        double *dst = cell64 + c * 7 * nd + q;
        float *dstf = cell32 + c * 7 * nd + q;
        const double w = g[0];
        dst[0] = aq * w;
        dstf[0] = (float)(aq * w);
        for (int s = 1; s < 7; ++s) {
            const double v = bq * g[s * nd];
            dst[s * nd] = v;
            dstf[s * nd] = (float)v;
        }
        if (ctype[c]) {
            // affine cell: alpha w detJ and beta w detJ (G = beta w detJ J^-1 J^-T)
            const double am = aq * w, bm = bq * w;
            acell64[c * 2 * nd + q] = am;
            acell64[c * 2 * nd + nd + q] = bm;
            acell32[c * 2 * nd + q] = (float)am;
            acell32[c * 2 * nd + nd + q] = (float)bm;
        }
        sw = w;
        sa = w * aq;
        sb = w * bq;
    }
    // block reduction (fixed order)
    __shared__ double red[3][512];
    red[0][threadIdx.x] = sw;
    red[1][threadIdx.x] = sa;
    red[2][threadIdx.x] = sb;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int r = 0; r < 3; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double vol = red[0][0];
        const double ab = red[1][0] / vol, bb = red[2][0] / vol;
        const double lx = ell[3 * c], ly = ell[3 * c + 1], lz = ell[3 * c + 2];
        const double cc[4] = {ab * lx * ly * lz, bb * ly * lz / lx, bb * lx * lz / ly, bb * lx * ly / lz};
        for (int r = 0; r < 4; ++r) {
            bjC64[4 * c + r] = cc[r];
            bjC32[4 * c + r] = (float)cc[r];
        }
        const double l2 = cbrt(lx * ly * lz);
        coef_feat[c] = log(bb / (ab * l2 * l2));
    }
}

// -------------------------------------------------------------------------
// merged face data of the +d face of every cell (thread per face point),
// [cell][d][component][a][b] with a, b the first and second tangential index:
//   g- = beta- ds J-^{-1} n,  g+ = beta+ ds J+^{-1} n,  s = sigma 1/2 (b- + b+) ds
// with n and ds from the minus cell; the three components of g are stored in
// the order (d, first tangential, second tangential) so that the operator
// pairs them with its reference derivatives without a per-lane selection.
// -------------------------------------------------------------------------
__global__ void k_set_face(int n, int64_t n_cells, const int32_t *__restrict__ nbr,
                           const RefTab64 *__restrict__ T, const double *__restrict__ beta,
                           const double *__restrict__ sigma, const double *__restrict__ facegeo,
                           double *face64, float *face32, const uint8_t *__restrict__ ctype,
                           double *aface64, float *aface32, double *fc64, float *fc32)
{
    const int nf = n * n, nd = nf * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n_cells * nf) return;
    const int pt = (int)(t % nf);
    const int64_t cd = t / nf;
    const int64_t c = cd / 3;
    const int d = (int)(cd % 3);
    const int b = pt % n, a = pt / n;
    double *dst = face64 + cd * 7 * nf + pt;
    float *dstf = face32 + cd * 7 * nf + pt;
    const double *g = facegeo + cd * 7 * nf + pt;
    const int32_t nb = nbr[6 * c + 2 * d + 1];
    if (nb < 0) {
        for (int s = 0; s < 7; ++s) {
            dst[s * nf] = 0.0;
            dstf[s * nf] = 0.0f;
        }
        return;
    }
    double bm = 0.0, bp = 0.0;
    for (int r = 0; r < n; ++r)
        for (int p = 0; p < n; ++p) {
            const double wgt = T->B[a * n + p] * T->B[b * n + r];
            bm += wgt * beta[c * nd + layer_idx(n, d, n - 1, p, r)];
            bp += wgt * beta[(int64_t)nb * nd + layer_idx(n, d, 0, p, r)];
        }
    double out[7];
    for (int k = 0; k < 3; ++k) {
        out[k] = bm * g[k * nf];
        out[3 + k] = bp * g[(3 + k) * nf];
    }
    out[6] = sigma[3 * c + d] * (bm + bp) * g[6 * nf];
    for (int s = 0; s < 7; ++s) {
        dst[s * nf] = out[s];
        dstf[s * nf] = (float)out[s];
    }
    if (ctype[c] && ctype[nb]) {
        // face between two affine cells: g- = (beta- w) v-, g+ = (beta+ w) v+,
        // s = sd ((beta- w) + (beta+ w)) with w the face weight, v = ds0 J^-1 n
        // and sd = sigma ds0 / 2 constant over the face (ds = w ds0)
        const double wab = T->wq[a] * T->wq[b];
        aface64[cd * 2 * nf + pt] = bm * wab;
        aface64[cd * 2 * nf + nf + pt] = bp * wab;
        aface32[cd * 2 * nf + pt] = (float)(bm * wab);
        aface32[cd * 2 * nf + nf + pt] = (float)(bp * wab);
        if (pt == 0) {
            double v[8];
            for (int k = 0; k < 6; ++k) v[k] = g[k * nf] / wab;
            v[6] = sigma[3 * c + d] * g[6 * nf] / wab;
            v[7] = 0.0;
            for (int k = 0; k < 8; ++k) {
                fc64[cd * 8 + k] = v[k];
                fc32[cd * 8 + k] = (float)v[k];
            }
        }
    }
}

// -------------------------------------------------------------------------
// dof coordinates (thread per dof)
// -------------------------------------------------------------------------
__global__ void k_dof_coords(const double *__restrict__ nodes, int ng, int n, int64_t n_dofs,
                             const RefTab64 *__restrict__ T, double *xyz)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_dofs) return;
    const int nd = n * n * n;
    const int64_t c = t / nd;
    const int q = (int)(t % nd);
    double xi[3] = {T->xl[q % n], T->xl[(q / n) % n], T->xl[q / (n * n)]}, x[3], J[3][3];
    cell_map(nodes + c * (int64_t)ng * ng * ng * 3, ng, xi, x, J);
    xyz[t] = x[0];
    xyz[n_dofs + t] = x[1];
    xyz[2 * n_dofs + t] = x[2];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_cell_geometry(hx_ctx *c)
{
    hipLaunchKernelGGL(k_cell_geometry, dim3(nblk(c->n_cells, 64)), dim3(64), 0, c->stream,
                       c->nodes, c->g + 1, c->n, c->n_cells, c->ref, c->vol, c->ell, c->mindet);
    return hipGetLastError();
}

hipError_t launch_face_sigma(hx_ctx *c)
{
    hipLaunchKernelGGL(k_face_sigma, dim3(nblk(3 * c->n_cells, 64)), dim3(64), 0, c->stream,
                       c->nodes, c->g + 1, c->n, c->n_cells, c->nbr, c->ref, c->vol, c->P,
                       c->sigma);
    return hipGetLastError();
}

template <int N>
static hipError_t bj_eigen_n(hx_ctx *c)
{
    hipLaunchKernelGGL(k_bj_eigen<N>, dim3(nblk(3 * c->n_cells, 64)), dim3(64), 0, c->stream,
                       c->n_cells, c->nbr, c->ref, c->ell, c->sigma, c->endsig, c->bjS64, c->bjS32,
                       c->bjL64, c->bjL32);
    return hipGetLastError();
}

hipError_t launch_bj_eigen(hx_ctx *c)
{
    switch (c->n) {
    case 2: return bj_eigen_n<2>(c);
    case 3: return bj_eigen_n<3>(c);
    case 4: return bj_eigen_n<4>(c);
    case 5: return bj_eigen_n<5>(c);
    case 6: return bj_eigen_n<6>(c);
    case 7: return bj_eigen_n<7>(c);
    case 8: return bj_eigen_n<8>(c);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_geofac(hx_ctx *c)
{
    hipLaunchKernelGGL(k_cell_geofac, dim3(nblk(c->n_cells * c->nd, 128)), dim3(128), 0, c->stream,
                       c->nodes, c->g + 1, c->n, c->n_cells, c->ref, c->cellgeo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nt = 3 * c->n_cells * c->nf;
    hipLaunchKernelGGL(k_face_geofac, dim3(nblk(nt, 128)), dim3(128), 0, c->stream, c->nodes,
                       c->g + 1, c->n, c->n_cells, c->nbr, c->ref, c->facegeo);
    return hipGetLastError();
}

hipError_t launch_affine_detect(hx_ctx *c)
{
    hipLaunchKernelGGL(k_affine_detect, dim3(nblk(c->n_cells, 128)), dim3(128), 0, c->stream, c->nodes,
                       c->g + 1, c->nd, c->n_cells, c->ref, c->cellgeo, c->ctype, c->kk64, c->kk32);
    return hipGetLastError();
}

hipError_t launch_set_coefficients(hx_ctx *c, const double *alpha, const double *beta)
{
    int threads = 64;                     // power of two for the tree reduction
    while (threads < c->nd) threads *= 2;
    hipLaunchKernelGGL(k_set_cell, dim3((unsigned)c->n_cells), dim3(threads), 0, c->stream, c->n,
                       c->ref, alpha, beta, c->ell, c->cellgeo, c->cell64, c->cell32, c->bjC64,
                       c->bjC32, c->coef_feat, c->ctype, c->acell64, c->acell32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nt = 3 * c->n_cells * c->nf;
    hipLaunchKernelGGL(k_set_face, dim3(nblk(nt, 128)), dim3(128), 0, c->stream, c->n, c->n_cells,
                       c->nbr, c->ref, beta, c->sigma, c->facegeo, c->face64, c->face32, c->ctype,
                       c->aface64, c->aface32, c->fc64, c->fc32);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (c->n_hang) {
        e = launch_hang_coefficients(c, beta);
        if (e != hipSuccess) return e;
    }
    return launch_cell_diag(c);
}

// -------------------------------------------------------------------------
// Volume diagonals from the merged cell data (block per cell):
//   d_i = sum_q [ m_q phi_i(q)^2 + grad phi_i(q)^T G_q grad phi_i(q) ],
// phi_i(q) = B(qx,a) B(qy,b) B(qz,l), reference gradient from BD.  Every
// term is a tensor contraction of one quadrature field with products of
// 1-D tables, P0 = B B, P1 = B BD, P2 = BD BD, e.g. the Gxy term is
// 2 sum_q Gxy P1(qx,a) P1(qy,b) P0(qz,l); the kernel contracts z, then y,
// then x, merging terms that share their remaining tables (N^4 work per
// sweep instead of N^6 per cell).  Stored as inverses: dg[0] of mass plus
// stiffness (the paper's Helmholtz preconditioner, section 3.1), dg[1] of
// the mass alone (its internal-energy variant).
// -------------------------------------------------------------------------
__device__ __forceinline__ double ptab(const RefTab64 *T, int n, int kind, int q, int a)
{
    const double bv = T->B[q * n + a], dv = T->BD[q * n + a];
    return kind == 0 ? bv * bv : (kind == 1 ? bv * dv : dv * dv);
}

__global__ void k_cell_diag(int n, int64_t n_cells, const RefTab64 *__restrict__ T,
                            const double *__restrict__ cell, double *dg64, float *dg32)
{
    extern __shared__ double sd[];           // F [7][nd], then A [7][nd]
    const int nd = n * n * n;
    const int64_t c = blockIdx.x;
    const double *cd = cell + c * 7 * nd;
    double *F = sd, *A = sd + 7 * nd;
    for (int e = threadIdx.x; e < 7 * nd; e += blockDim.x) F[e] = cd[e];
    __syncthreads();
    const int t = threadIdx.x;
    const bool on = t < nd;
    const int i0 = t % n, i1 = (t / n) % n, i2 = t / (n * n);
    // z: thread (qx, qy, l); fields m, Gxx, Gxy, Gxz, Gyy, Gyz, Gzz
    if (on) {
        double tm = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
        for (int qz = 0; qz < n; ++qz) {
            const int q = i0 + n * (i1 + n * qz);
            const double p0 = ptab(T, n, 0, qz, i2), p1 = ptab(T, n, 1, qz, i2),
                         p2 = ptab(T, n, 2, qz, i2);
            tm += p0 * F[q];
            txx += p0 * F[nd + q];
            txy += p0 * F[2 * nd + q];
            txz += p1 * F[3 * nd + q];
            tyy += p0 * F[4 * nd + q];
            tyz += p1 * F[5 * nd + q];
            tzz += p2 * F[6 * nd + q];
        }
        // groups by their remaining (x, y) tables:
        // 0 mass (P0,P0), 1 m + Gzz (P0,P0), 2 Gxx (P2,P0), 3 Gyy (P0,P2),
        // 4 2Gxy (P1,P1), 5 2Gxz (P1,P0), 6 2Gyz (P0,P1)
        A[t] = tm;
        A[nd + t] = tm + tzz;
        A[2 * nd + t] = txx;
        A[3 * nd + t] = tyy;
        A[4 * nd + t] = 2.0 * txy;
        A[5 * nd + t] = 2.0 * txz;
        A[6 * nd + t] = 2.0 * tyz;
    }
    __syncthreads();
    // y: thread (qx, b, l); results by their x table: mass P0, P0, P2, P1
    double cm = 0, c0 = 0, c2 = 0, c1 = 0;
    if (on) {
        for (int qy = 0; qy < n; ++qy) {
            const int q = i0 + n * (qy + n * i2);
            const double p0 = ptab(T, n, 0, qy, i1), p1 = ptab(T, n, 1, qy, i1),
                         p2 = ptab(T, n, 2, qy, i1);
            cm += p0 * A[q];
            c0 += p0 * A[nd + q] + p2 * A[3 * nd + q] + p1 * A[6 * nd + q];
            c2 += p0 * A[2 * nd + q];
            c1 += p1 * A[4 * nd + q] + p0 * A[5 * nd + q];
        }
    }
    __syncthreads();
    if (on) {
        F[t] = cm;
        F[nd + t] = c0;
        F[2 * nd + t] = c2;
        F[3 * nd + t] = c1;
    }
    __syncthreads();
    // x: thread (a, b, l)
    if (!on) return;
    double dm = 0, dt = 0;
    for (int qx = 0; qx < n; ++qx) {
        const int q = qx + n * (i1 + n * i2);
        const double p0 = ptab(T, n, 0, qx, i0), p1 = ptab(T, n, 1, qx, i0),
                     p2 = ptab(T, n, 2, qx, i0);
        dm += p0 * F[q];
        dt += p0 * F[nd + q] + p2 * F[2 * nd + q] + p1 * F[3 * nd + q];
    }
    const int64_t o = c * nd + t, nt = n_cells * nd;
    const double ih = 1.0 / dt, im = 1.0 / dm;
    dg64[o] = ih;
    dg64[nt + o] = im;
    dg32[o] = (float)ih;
    dg32[nt + o] = (float)im;
}

hipError_t launch_cell_diag(hx_ctx *c)
{
    int threads = 64;
    while (threads < c->nd) threads *= 2;
    hipLaunchKernelGGL(k_cell_diag, dim3((unsigned)c->n_cells), dim3(threads),
                       sizeof(double) * 14 * c->nd, c->stream, c->n, c->n_cells, c->ref, c->cell64,
                       c->dg64, c->dg32);
    return hipGetLastError();
}

hipError_t launch_dof_coords(hx_ctx *c, double *xyz)
{
    hipLaunchKernelGGL(k_dof_coords, dim3(nblk(c->n_dofs, 128)), dim3(128), 0, c->stream,
                       c->nodes, c->g + 1, c->n, c->n_dofs, c->ref, xyz);
    return hipGetLastError();
}

}  // namespace hx

namespace hx {
namespace {

// -------------------------------------------------------------------------
// Data of the pressure system of one IMEX stage (section 2: A U + B P = F,
// C U + D P = G).  At cell Gauss point q of cell c:
//   W[c][3d+e][q]  = w detJ (J^-1)_{de}   (so that (grad phi)_e = sum_d W ... / (w detJ))
//   WC[c][3d+e][q] = hr_q W[c][3d+e][q]   (hr = h rho formed at the nodes, interpolated)
//   mr[c][q] = rho_q w detJ,  md[c][q] = w detJ / (gamma - 1);
// at Gauss point (a, b) of the cell's own face f = 2d + s:
//   fn[c][f][e][a + N b] = ds n_e (outward),  fh[c][f][a + N b] = hr.
// -------------------------------------------------------------------------
__global__ void k_press_cell(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                             const RefTab64 *__restrict__ T, const double *__restrict__ rho,
                             const double *__restrict__ h, double inv_gm1, double *W, double *WC,
                             double *mr, double *md)
{
    const int nd = n * n * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_cells * nd) return;
    const int64_t c = t / nd;
    const int q = (int)(t % nd);
    const int i = q % n, j = (q / n) % n, l = q / (n * n);
    double xi[3] = {T->xq[i], T->xq[j], T->xq[l]}, x[3], J[3][3], Ji[3][3];
    cell_map(nodes + c * (int64_t)ng * ng * ng * 3, ng, xi, x, J);
    const double det = det3(J);
    inv3(J, det, Ji);
    const double w = T->wq[i] * T->wq[j] * T->wq[l] * det;
    double rq = 0.0, hq = 0.0;
    const double *rc = rho + c * nd, *hc = h + c * nd;
    for (int l2 = 0; l2 < n; ++l2)
        for (int j2 = 0; j2 < n; ++j2) {
            const double byz = T->B[j * n + j2] * T->B[l * n + l2];
            for (int i2 = 0; i2 < n; ++i2) {
                const double wgt = T->B[i * n + i2] * byz;
                const int e = lidx(n, i2, j2, l2);
                rq += wgt * rc[e];
                hq += wgt * (hc[e] * rc[e]);
            }
        }
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) {
            const double v = w * Ji[d][e];
            W[(c * 9 + 3 * d + e) * nd + q] = v;
            WC[(c * 9 + 3 * d + e) * nd + q] = hq * v;
        }
    mr[c * nd + q] = rq * w;
    md[c * nd + q] = w * inv_gm1;
}

__global__ void k_press_face(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                             const RefTab64 *__restrict__ T, const double *__restrict__ rho,
                             const double *__restrict__ h, double *fn, double *fh)
{
    const int nf = n * n, nd = nf * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_cells * 6 * nf) return;
    const int pt = (int)(t % nf);
    const int64_t cf = t / nf;
    const int64_t c = cf / 6;
    const int f = (int)(cf % 6), d = f >> 1, s = f & 1;
    const int a = pt % n, b = pt / n;
    double xi[3], x[3], J[3][3], Ji[3][3];
    face_xi(T, d, s, a, b, xi);
    cell_map(nodes + c * (int64_t)ng * ng * ng * 3, ng, xi, x, J);
    const double det = det3(J);
    inv3(J, det, Ji);
    // ds n = +-w_a w_b detJ J^-T e_d (row d of J^-1), outward
    const double sw = (s ? 1.0 : -1.0) * T->wq[a] * T->wq[b] * det;
    for (int e = 0; e < 3; ++e) fn[(cf * 3 + e) * nf + pt] = sw * Ji[d][e];
    // trace of hr: the face layer of GLL nodes interpolated to the point
    const int m = s ? n - 1 : 0;
    double hv = 0.0;
    for (int e2 = 0; e2 < n; ++e2)
        for (int e1 = 0; e1 < n; ++e1) {
            const int64_t e = c * nd + layer_idx(n, d, m, e1, e2);
            hv += T->B[a * n + e1] * T->B[b * n + e2] * (h[e] * rho[e]);
        }
    fh[cf * nf + pt] = hv;
}

}  // namespace

hipError_t launch_press_setup(hx_ctx *c, const double *rho, const double *h, double gamma)
{
    const int64_t nt = c->n_cells * c->nd;
    hipLaunchKernelGGL(k_press_cell, dim3(nblk(nt, 128)), dim3(128), 0, c->stream, c->nodes, c->g + 1,
                       c->n, c->n_cells, c->ref, rho, h, 1.0 / (gamma - 1.0), c->psW, c->psWC,
                       c->psMr, c->psMd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nf = c->n_cells * 6 * c->nf;
    hipLaunchKernelGGL(k_press_face, dim3(nblk(nf, 128)), dim3(128), 0, c->stream, c->nodes, c->g + 1,
                       c->n, c->n_cells, c->ref, rho, h, c->psFn, c->psFh);
    return hipGetLastError();
}

}  // namespace hx

namespace hx {
namespace {

// -------------------------------------------------------------------------
// Consistent integration (section 3.3: 2r+1 Gauss points per direction):
// the merged cell and face data of the operator at the nq-point rule, the
// same quantities as k_cell_geofac / k_set_cell and k_face_geofac /
// k_set_face, with alpha and beta interpolated from the nodes to the points.
// Cell point index qx + nq (qy + nq qz); face point a + nq b (a along t1).
// -------------------------------------------------------------------------
__global__ void k_q_cell(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                         const RefTabQ *__restrict__ Q, const double *__restrict__ alpha,
                         const double *__restrict__ beta, double *qcell)
{
    const int nq = Q->nq, nq3 = nq * nq * nq, nd = n * n * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_cells * nq3) return;
    const int64_t c = t / nq3;
    const int q = (int)(t % nq3);
    const int i = q % nq, j = (q / nq) % nq, l = q / (nq * nq);
    double xi[3] = {Q->xq[i], Q->xq[j], Q->xq[l]}, x[3], J[3][3], Ji[3][3];
    cell_map(nodes + c * (int64_t)ng * ng * ng * 3, ng, xi, x, J);
    const double det = det3(J);
    inv3(J, det, Ji);
    const double w = Q->wq[i] * Q->wq[j] * Q->wq[l] * det;
    double aq = 0.0, bq = 0.0;
    const double *ac = alpha + c * nd, *bc = beta + c * nd;
    for (int l2 = 0; l2 < n; ++l2)
        for (int j2 = 0; j2 < n; ++j2) {
            const double byz = Q->B[j * n + j2] * Q->B[l * n + l2];
            for (int i2 = 0; i2 < n; ++i2) {
                const double wgt = Q->B[i * n + i2] * byz;
                const int e = lidx(n, i2, j2, l2);
                aq += wgt * ac[e];
                bq += wgt * bc[e];
            }
        }
    double *dst = qcell + c * 7 * nq3 + q;
    dst[0] = aq * w;
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int s = 0; s < 6; ++s) {
        const int A = pa[s], Bq = pb[s];
        dst[(1 + s) * nq3] =
            bq * w * (Ji[A][0] * Ji[Bq][0] + Ji[A][1] * Ji[Bq][1] + Ji[A][2] * Ji[Bq][2]);
    }
}

__global__ void k_q_face(const double *__restrict__ nodes, int ng, int n, int64_t n_cells,
                         const int32_t *__restrict__ nbr, const RefTabQ *__restrict__ Q,
                         const double *__restrict__ beta, const double *__restrict__ sigma,
                         double *qface)
{
    const int nq = Q->nq, nq2 = nq * nq, nd = n * n * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n_cells * nq2) return;
    const int pt = (int)(t % nq2);
    const int64_t cd = t / nq2;
    const int64_t c = cd / 3;
    const int d = (int)(cd % 3);
    const int a = pt % nq, b = pt / nq;
    double *dst = qface + cd * 7 * nq2 + pt;
    const int32_t nb = nbr[6 * c + 2 * d + 1];
    if (nb < 0) {
        for (int s = 0; s < 7; ++s) dst[s * nq2] = 0.0;
        return;
    }
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    double xim[3], xip[3], x[3], Jm[3][3], Jp[3][3], Jmi[3][3], Jpi[3][3];
    xim[d] = 1.0;
    xip[d] = 0.0;
    xim[t1] = xip[t1] = Q->xq[a];
    xim[t2] = xip[t2] = Q->xq[b];
    const int64_t gsz = (int64_t)ng * ng * ng * 3;
    cell_map(nodes + c * gsz, ng, xim, x, Jm);
    cell_map(nodes + (int64_t)nb * gsz, ng, xip, x, Jp);
    const double detm = det3(Jm), detp = det3(Jp);
    inv3(Jm, detm, Jmi);
    inv3(Jp, detp, Jpi);
    double nv[3] = {Jmi[d][0], Jmi[d][1], Jmi[d][2]};
    const double len = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int r = 0; r < 3; ++r) nv[r] /= len;
    const double ds = Q->wq[a] * Q->wq[b] * detm * len;
    // beta on both sides: the face layers interpolated to the point
    double bm = 0.0, bp = 0.0;
    for (int e2 = 0; e2 < n; ++e2)
        for (int e1 = 0; e1 < n; ++e1) {
            const double wgt = Q->B[a * n + e1] * Q->B[b * n + e2];
            bm += wgt * beta[c * nd + layer_idx(n, d, n - 1, e1, e2)];
            bp += wgt * beta[(int64_t)nb * nd + layer_idx(n, d, 0, e1, e2)];
        }
    const int dir[3] = {d, t1, t2};
    for (int k = 0; k < 3; ++k) {
        const int r = dir[k];
        dst[k * nq2] = bm * ds * (Jmi[r][0] * nv[0] + Jmi[r][1] * nv[1] + Jmi[r][2] * nv[2]);
        dst[(3 + k) * nq2] = bp * ds * (Jpi[r][0] * nv[0] + Jpi[r][1] * nv[1] + Jpi[r][2] * nv[2]);
    }
    dst[6 * nq2] = sigma[3 * c + d] * 0.5 * (bm + bp) * ds;
}

}  // namespace

hipError_t launch_q_setup(hx_ctx *c, const double *alpha, const double *beta)
{
    const int nq = c->nq;
    const int64_t nt = c->n_cells * nq * nq * nq;
    hipLaunchKernelGGL(k_q_cell, dim3(nblk(nt, 128)), dim3(128), 0, c->stream, c->nodes, c->g + 1, c->n,
                       c->n_cells, c->refq, alpha, beta, c->qcell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nf = 3 * c->n_cells * nq * nq;
    hipLaunchKernelGGL(k_q_face, dim3(nblk(nf, 128)), dim3(128), 0, c->stream, c->nodes, c->g + 1, c->n,
                       c->n_cells, c->nbr, c->refq, beta, c->sigma, c->qface);
    return hipGetLastError();
}

}  // namespace hx
