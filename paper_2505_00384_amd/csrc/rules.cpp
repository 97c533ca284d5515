// Host-side 1-D reference data of the library: Gauss-Legendre and
// Gauss-Lobatto rules by the Golub-Welsch eigenvalue method, Lagrange
// bases in barycentric form, and the per-degree tables of the set-up and
// block-Jacobi kernels (the operator's copies are generated from the same
// rules at build time).
//
// Dof nodes are the (k+1) Gauss-Lobatto points (section 2 of the paper);
// quadrature is (k+1)-point Gauss-Legendre (section 3.3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace hx {

// Cyclic Jacobi eigenvalue iteration for a small symmetric matrix (row-major
// a[n*n], destroyed); eigenvalues to w, eigenvectors as columns of v.
void sym_eig(int n, double *a, double *w, double *v)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a[i * n + j] * a[i * n + j];
                if (i != j) off += a[i * n + j] * a[i * n + j];
            }
        if (off <= 1e-34 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a[p * n + q];
                if (apq == 0.0) continue;
                double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {      // columns p, q
                    double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = cs * akp - sn * akq;
                    a[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {      // rows p, q
                    double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = cs * apk - sn * aqk;
                    a[q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = v[k * n + p], vkq = v[k * n + q];
                    v[k * n + p] = cs * vkp - sn * vkq;
                    v[k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = a[i * n + i];
}

// Legendre P_m at x by recurrence, with P_{m-1}.
static void legendre_pair(int m, double x, double &pm, double &pm1)
{
    double a = 1.0, b = x;
    if (m == 0) { pm = 1.0; pm1 = 0.0; return; }
    for (int j = 2; j <= m; ++j) {
        double c = ((2.0 * j - 1.0) * x * b - (j - 1.0) * a) / j;
        a = b; b = c;
    }
    pm = b; pm1 = a;
}

// Eigen-decomposition of a symmetric tridiagonal Jacobi matrix with zero
// diagonal; sorted nodes and first eigenvector components.
static void golub_welsch(int n, const std::vector<double> &offd, std::vector<double> &x,
                         std::vector<double> &v0sq)
{
    std::vector<double> a(n * n, 0.0), w(n), v(n * n);
    for (int i = 0; i + 1 < n; ++i) a[i * n + i + 1] = a[(i + 1) * n + i] = offd[i];
    sym_eig(n, a.data(), w.data(), v.data());
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (w[idx[j]] < w[idx[i]]) std::swap(idx[i], idx[j]);
    x.resize(n); v0sq.resize(n);
    for (int i = 0; i < n; ++i) {
        x[i] = w[idx[i]];
        v0sq[i] = v[0 * n + idx[i]] * v[0 * n + idx[i]];
    }
}

void rule_gauss_legendre(int n, double *x01, double *w01)
{
    std::vector<double> off(n > 1 ? n - 1 : 0), x, v0;
    for (int k = 1; k < n; ++k) off[k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
    golub_welsch(n, off, x, v0);
    for (int i = 0; i < n; ++i) {
        double t = x[i];
        // one Newton polish on P_n
        for (int it = 0; it < 2; ++it) {
            double p, pm1;
            legendre_pair(n, t, p, pm1);
            double dp = n * (t * p - pm1) / (t * t - 1.0);
            t -= p / dp;
        }
        double p, pm1;
        legendre_pair(n, t, p, pm1);
        double dp = n * (t * p - pm1) / (t * t - 1.0);
        x01[i] = 0.5 * (t + 1.0);
        w01[i] = 1.0 / ((1.0 - t * t) * dp * dp);   // (2/((1-t^2) P'^2)) / 2
    }
}

void rule_gauss_lobatto(int n, double *x01, double *w01)
{
    // interior nodes: zeros of the Jacobi polynomial P^(1,1)_{n-2}
    x01[0] = 0.0; x01[n - 1] = 1.0;
    w01[0] = w01[n - 1] = 1.0 / (n * (n - 1.0));
    int m = n - 2;
    if (m <= 0) return;
    std::vector<double> off(m > 1 ? m - 1 : 0), x, v0;
    for (int k = 1; k < m; ++k)
        off[k - 1] = std::sqrt(k * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)));
    golub_welsch(m, off, x, v0);
    for (int i = 0; i < m; ++i) {
        double t = x[i], p, pm1;
        legendre_pair(n - 1, t, p, pm1);
        x01[i + 1] = 0.5 * (t + 1.0);
        w01[i + 1] = 1.0 / (n * (n - 1.0) * p * p);
    }
}

// Lagrange basis through nodes (barycentric form), values and derivatives at t.
void lagrange_eval(int n, const double *nodes, double t, double *val, double *der)
{
    std::vector<double> lam(n);
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= nodes[j] - nodes[k];
        lam[j] = 1.0 / p;
    }
    int hit = -1;
    for (int j = 0; j < n; ++j)
        if (t == nodes[j]) hit = j;
    if (hit >= 0) {
        for (int j = 0; j < n; ++j) {
            val[j] = (j == hit) ? 1.0 : 0.0;
            if (j != hit) {
                der[j] = (lam[j] / lam[hit]) / (nodes[hit] - nodes[j]);
            } else {
                double s = 0.0;
                for (int k = 0; k < n; ++k)
                    if (k != hit) s += 1.0 / (nodes[hit] - nodes[k]);
                der[j] = s;
            }
        }
        return;
    }
    double l = 1.0;
    for (int k = 0; k < n; ++k) l *= t - nodes[k];
    for (int j = 0; j < n; ++j) {
        val[j] = l * lam[j] / (t - nodes[j]);
        double s = 0.0;
        for (int k = 0; k < n; ++k)
            if (k != j) s += 1.0 / (t - nodes[k]);
        der[j] = val[j] * s;
    }
}

void build_ref_tables(int n, RefTab64 &t)
{
    std::memset(&t, 0, sizeof(t));
    double xq[MAXN], wq[MAXN], xl[MAXN], wl[MAXN];
    rule_gauss_legendre(n, xq, wq);
    rule_gauss_lobatto(n, xl, wl);
    double v[MAXN], d[MAXN];
    for (int q = 0; q < n; ++q) {
        t.xq[q] = xq[q];
        t.wq[q] = wq[q];
        t.xl[q] = xl[q];
        lagrange_eval(n, xl, xq[q], v, d);
        for (int i = 0; i < n; ++i) {
            t.B[q * n + i] = v[i];
            t.BD[q * n + i] = d[i];
        }
    }
    for (int e = 0; e < 2; ++e) {
        lagrange_eval(n, xl, e ? 1.0 : 0.0, v, d);
        for (int i = 0; i < n; ++i) t.DL[e][i] = d[i];
    }
    // the basis at the nodes of either half of the interval (the embedding of
    // a parent cell's polynomial into its children)
    for (int o = 0; o < 2; ++o)
        for (int i = 0; i < n; ++i) {
            lagrange_eval(n, xl, 0.5 * (o + xl[i]), v, d);
            for (int j = 0; j < n; ++j) t.Eh[o][i * n + j] = v[j];
        }
    // 1-D reference mass and stiffness with GL quadrature
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double m = 0.0, s = 0.0;
            for (int q = 0; q < n; ++q) {
                m += wq[q] * t.B[q * n + i] * t.B[q * n + j];
                s += wq[q] * t.BD[q * n + i] * t.BD[q * n + j];
            }
            t.M[i * n + j] = m;
            t.L0[i * n + j] = s;
        }
    // Cholesky M = C C^T and its inverse (lower triangular), for the
    // generalised eigenproblems of the block preconditioner
    double C[MAXN * MAXN] = {0};
    for (int j = 0; j < n; ++j) {
        double s = t.M[j * n + j];
        for (int k = 0; k < j; ++k) s -= C[j * n + k] * C[j * n + k];
        C[j * n + j] = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double r = t.M[i * n + j];
            for (int k = 0; k < j; ++k) r -= C[i * n + k] * C[j * n + k];
            C[i * n + j] = r / C[j * n + j];
        }
    }
    for (int col = 0; col < n; ++col)
        for (int i = 0; i < n; ++i) {
            double r = (i == col) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) r -= C[i * n + k] * t.Cinv[k * n + col];
            t.Cinv[i * n + col] = r / C[i * n + i];
        }
    // Binv = B^{-1} (B maps nodal values to the n Gauss points, so it is
    // square): Gauss-Jordan elimination with partial pivoting
    double W[MAXN][2 * MAXN];
    for (int q = 0; q < n; ++q)
        for (int i = 0; i < 2 * n; ++i) W[q][i] = i < n ? t.B[q * n + i] : (i - n == q ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(W[r][col]) > std::fabs(W[piv][col])) piv = r;
        if (piv != col)
            for (int i = 0; i < 2 * n; ++i) std::swap(W[col][i], W[piv][i]);
        const double d = W[col][col];
        for (int i = 0; i < 2 * n; ++i) W[col][i] /= d;
        for (int r = 0; r < n; ++r)
            if (r != col) {
                const double f = W[r][col];
                for (int i = 0; i < 2 * n; ++i) W[r][i] -= f * W[col][i];
            }
    }
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < n; ++q) t.Binv[i * n + q] = W[i][n + q];
}

void build_q_tables(int n, int nq, RefTabQ &t)
{
    t.nq = nq;
    double xl[MAXN], wl[MAXN], v[MAXN], d[MAXN];
    rule_gauss_lobatto(n, xl, wl);
    rule_gauss_legendre(nq, t.xq, t.wq);
    for (int q = 0; q < nq; ++q) {
        lagrange_eval(n, xl, t.xq[q], v, d);
        for (int i = 0; i < n; ++i) {
            t.B[q * n + i] = v[i];
            t.BD[q * n + i] = d[i];
        }
    }
}

}  // namespace hx
