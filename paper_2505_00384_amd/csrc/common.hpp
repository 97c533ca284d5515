// Internal declarations of the helmdg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/helmdg.h"

namespace hx {

constexpr int MAXK = 7;             // highest supported polynomial degree
constexpr int MAXN = MAXK + 1;      // points per direction
constexpr int MAXG = 8;             // highest geometry degree
constexpr int NXCD = 8;             // accelerator complex dies of the MI355X

// Reference data of one degree (host side, FP64).
struct RefTab64 {
    double xq[MAXN], wq[MAXN], xl[MAXN];   // GL points/weights, GLL nodes on [0,1]
    double B[MAXN * MAXN];                 // B[q*n+i]  = l_i(xq_q)   (GLL basis at GL points)
    double BD[MAXN * MAXN];                // BD[q*n+i] = l_i'(xq_q)
    double DL[2][MAXN];                    // DL[e][i]  = l_i'(e), e = 0, 1
    double M[MAXN * MAXN];                 // 1-D reference mass
    double L0[MAXN * MAXN];                // 1-D reference stiffness
    double Cinv[MAXN * MAXN];              // inverse Cholesky factor of M (lower)
    double Binv[MAXN * MAXN];              // Binv[i*n+q]: inverse of B (n points = n nodes)
    double Eh[2][MAXN * MAXN];             // Eh[o][i*n+j] = l_j((o + xl_i)/2): the basis at the
                                           // nodes of the lower (o = 0) or upper half interval
};

void sym_eig(int n, double *a, double *w, double *v);
void rule_gauss_legendre(int n, double *x01, double *w01);
void rule_gauss_lobatto(int n, double *x01, double *w01);
void lagrange_eval(int n, const double *nodes, double t, double *val, double *der);
void build_ref_tables(int n, RefTab64 &t);

// tables of an nq-point Gauss rule for the n-node GLL basis (consistent
// integration uses nq = 2k+1 = 2n-1)
constexpr int MAXQ = 2 * MAXK + 1;
struct RefTabQ {
    int nq = 0;
    double xq[MAXQ], wq[MAXQ];           // GL on [0,1]
    double B[MAXQ * MAXN];               // B[q*n+i]  = l_i(xq_q)
    double BD[MAXQ * MAXN];              // BD[q*n+i] = l_i'(xq_q)
};
void build_q_tables(int n, int nq, RefTabQ &t);

struct MlpState;   // learned preconditioner (mlp.hip)

}  // namespace hx

struct hx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // mesh
    int k = 0, n = 0, nd = 0, nf = 0, g = 0;
    int64_t n_cells = 0, n_dofs = 0;
    bool has_mesh = false, has_coef = false;
    double P = 2.0;

    double *nodes = nullptr;      // [n_cells][(g+1)^3][3]
    int32_t *nbr = nullptr;       // [n_cells][6]
    int32_t *visit = nullptr;     // [n_cells][8] operator traversal: {cell, 6 neighbours, 0}
    hx::RefTab64 *ref = nullptr;  // device copy of the tables of degree k
    hx::RefTab64 ref_host{};
    double *vol = nullptr;        // [n_cells]
    double *ell = nullptr;        // [n_cells][3]
    double *mindet = nullptr;     // [n_cells]
    double *sigma = nullptr;      // [n_cells][3]

    // merged operator data
    double *cell64 = nullptr;     // [n_cells][7][nd]
    float *cell32 = nullptr;
    double *cellgeo = nullptr;    // [n_cells][7][nd] geometric factors of the cell data
    double *facegeo = nullptr;    // [n_cells][3][7][nf] geometric factors of the face data
    double *face64 = nullptr;     // [n_cells][3][7][N (1st tangential)][N (2nd)]
    float *face32 = nullptr;
    // compressed data of affine cells (one Jacobian per cell): the operator
    // reads these instead of cell64/face64 for affine cells and for faces
    // between two affine cells (bits of the traversal record's last word)
    int compress = 1;             // 1: use the compressed data where it applies
    int64_t n_affine = 0;         // affine cells
    int64_t n_iface = 0;          // interior faces (each once)
    int64_t n_cface = 0;          // interior faces between two affine cells
    uint8_t *ctype = nullptr;     // [n_cells] 1 = affine
    std::vector<int32_t> *order_h = nullptr;   // host: the traversal order of all cells
    std::vector<int32_t> *nbr_h = nullptr;     // host copy of the neighbour table
    int64_t n_vis_op = 0;         // records in visit (with padding)
    int vis_mode = 0;             // 0 general cells only, 1 affine only, 2 both, interleaved by wave
    int32_t *visitp = nullptr;    // [n_cells][8] plain traversal records (no padding, mask 0)
    std::vector<uint8_t> *ctype_h = nullptr;   // host copy of ctype
    double *acell64 = nullptr;    // [n_cells][2][nd]  alpha w detJ, beta w detJ (affine cells)
    float *acell32 = nullptr;
    double *kk64 = nullptr;       // [n_cells][8]      J^-1 J^-T (6 unique entries), detJ, 0
    float *kk32 = nullptr;
    double *aface64 = nullptr;    // [n_cells][3][2][nf] beta- w, beta+ w on the +d face (affine pair)
    float *aface32 = nullptr;
    double *fc64 = nullptr;       // [n_cells][3][8]   v- (3), v+ (3), sigma ds0 / 2, 0 of the +d face
    float *fc32 = nullptr;
    // non-conforming (2:1) quarter faces: records {C, fc, F, s} (face fc of
    // the coarse cell C, face fc ^ 1 of the fine cell F, quarter s)
    int64_t n_hang = 0;
    int32_t *hang = nullptr;      // [n_hang][4]
    double *hgeo = nullptr;       // [n_hang][7][nf] ds J_C^-1 n, ds J_F^-1 n, ds / 2
    double *hsig = nullptr;       // [n_hang] penalty
    double *harea = nullptr;      // [n_hang] area
    double *hdata64 = nullptr;    // [n_hang][7][nf] beta_C ds J_C^-1 n, beta_F ds J_F^-1 n, s
    float *hdata32 = nullptr;
    double *hcontrib64 = nullptr; // [n_hang][2][nd] staged contributions (coarse, fine side)
    float *hcontrib32 = nullptr;
    int64_t n_hcell = 0;          // cells with quarter faces
    int32_t *hcells = nullptr;    // [n_hcell]
    int32_t *hptr = nullptr;      // [n_hcell + 1]
    int32_t *hlist = nullptr;     // [2 n_hang] record * 2 + side, by cell
    double *endsig = nullptr;     // [n_cells][6] block-Jacobi penalty of non-conforming ends
    double *dg64 = nullptr;       // [2][n_dofs] inverse volume diagonals: mass + stiffness, mass
    float *dg32 = nullptr;
    double *cgpart = nullptr;     // [2][n_cells + 1] per-block partial sums of the fused CG steps
    double *pqpart = nullptr;     // [2 (n_cells + 1)] the operator's per-workgroup partial sums of p.q
    // pressure system of the IMEX stage (A U + B P = F, C U + D P = G)
    bool has_press = false;
    double ps_tau = 0.0;
    double *psW = nullptr;        // [n_cells][9][nd]  w detJ J^-1
    double *psWC = nullptr;       // [n_cells][9][nd]  h rho w detJ J^-1
    double *psMr = nullptr;       // [n_cells][nd]     rho w detJ (velocity mass)
    double *psMd = nullptr;       // [n_cells][nd]     w detJ / (gamma - 1) (internal-energy mass)
    double *psFn = nullptr;       // [n_cells][6][3][nf] outward ds n on the own faces
    double *psFh = nullptr;       // [n_cells][6][nf]  h rho on the own faces
    double *psWork = nullptr;     // [7][n_dofs]       velocity temporaries and C A^-1 B x
    // Chebyshev preconditioner: degree and interval of M^-1 A (M = block Jacobi)
    int cheb_deg = 0;
    double cheb_lo = 0.0, cheb_hi = 0.0;
    double *chebw = nullptr;      // [2][n_dofs] residual and step direction
    float *chebw32 = nullptr;     // [2][n_dofs] the same in FP32
    // consistent integration: the operator with nq = 2k+1 Gauss points
    bool has_q = false;
    int nq = 0;
    hx::RefTabQ *refq = nullptr;  // device tables
    double *qcell = nullptr;      // [n_cells][7][nq^3]   m, Gxx, Gxy, Gxz, Gyy, Gyz, Gzz
    double *qface = nullptr;      // [n_cells][3][7][nq^2] g-(3), g+(3), s of the +d face
    // geometric multigrid: the next coarser level (not owned), the children of
    // each of its cells, and the level vectors
    hx_ctx *mg_coarse = nullptr;
    int64_t mg_nc = 0;            // cells of the coarser level when linked
    int32_t *mg_cptr = nullptr;   // [mg_nc + 1] children of coarse cell j: mg_clist[cptr[j]..cptr[j+1])
    int32_t *mg_clist = nullptr;  // [n_cells] child cell * 8 + octant, grouped by parent
    int32_t *mg_child8 = nullptr; // [mg_nc][8] child in octant o, when every coarse cell has all eight
    double *mgw = nullptr;        // [3][n_dofs] b, x (as a coarse level), r
    float *mgw32 = nullptr;       // [3][n_dofs] the same in FP32 (the mixed-precision V-cycle)

    // separable block-Jacobi data
    double *bjS64 = nullptr;      // [n_cells][3][n][n]  eigenvectors S_d
    float *bjS32 = nullptr;
    double *bjL64 = nullptr;      // [n_cells][3][n]     eigenvalues
    float *bjL32 = nullptr;
    double *bjC64 = nullptr;      // [n_cells][4]        c0, cx, cy, cz
    float *bjC32 = nullptr;
    double *coef_feat = nullptr;  // [n_cells] log(bbar / (abar l^2))

    // reductions
    double *red = nullptr;        // partial sums
    double *red_host = nullptr;   // pinned
    double *dpart = nullptr;      // [128][1024] partial block dots of blas_dcgs
    // pinned, device-mapped: the scalars of the two FGMRES steps in flight,
    // written by the kernels themselves (FG_SLOT doubles per step)
    double *pin_host = nullptr;
    double *pin_dev = nullptr;
    int red_blocks = 0;

    // solver work space (allocated on first use, grown as needed)
    double *work64 = nullptr;
    size_t work64_len = 0;
    float *work32 = nullptr;
    size_t work32_len = 0;

    hx::MlpState *mlp = nullptr;
};

namespace hx {

hx_status fail(hx_ctx *c, hx_status s, const char *fmt, ...);

#define HX_HIP(c, call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::hx::fail((c), HX_ERR_DEVICE, "%s failed: %s", #call,            \
                              hipGetErrorString(e_));                                \
    } while (0)

hx_status dalloc(hx_ctx *c, void **p, size_t bytes);
void build_traversal(const int32_t *nbr, int64_t n_cells, int32_t *order);
void dfree(void **p);

// ---- kernel launchers (defined in the .hip translation units) ----------
// geometry / coefficients
hipError_t launch_cell_geometry(hx_ctx *c);                 // vol, ell, mindet
hipError_t launch_face_sigma(hx_ctx *c);                    // sigma
hipError_t launch_bj_eigen(hx_ctx *c);                      // bjS, bjL
hipError_t launch_set_coefficients(hx_ctx *c, const double *alpha, const double *beta);
hipError_t launch_dof_coords(hx_ctx *c, double *xyz);
hipError_t launch_geofac(hx_ctx *c);
// affine cells (geometry nodes an affine image of the reference nodes) and
// their per-cell constants J^-1 J^-T, detJ
hipError_t launch_affine_detect(hx_ctx *c);
hipError_t launch_cell_diag(hx_ctx *c);
hipError_t launch_diag64(hx_ctx *c, int which, const double *r, double *z);
hipError_t launch_diag32(hx_ctx *c, int which, const float *r, float *z);
// z = M^{-1} r, M the block-diagonal alpha-weighted mass matrix (fast
// tensor-product inverse)
hipError_t launch_massinv64(hx_ctx *c, const double *r, double *z);
// z = M r (inv = 0) or M^{-1} r (inv = 1) for the block-diagonal mass matrix
// with quadrature weights wgt[cell * wstride + q] (FP64)
hipError_t launch_mass64(hx_ctx *c, const double *wgt, int64_t wstride, int inv, const double *r,
                         double *z);
// pressure system: set-up from nodal rho and h; B p (3 components),
// C u, and y = S x or y = b - S x with S = D - C A^-1 B
hipError_t launch_press_setup(hx_ctx *c, const double *rho, const double *h, double gamma);
hipError_t launch_grad(hx_ctx *c, const double *p, double *u3);
hipError_t launch_div(hx_ctx *c, const double *u3, double *q);
hipError_t press_apply64(hx_ctx *c, const double *x, double *y, const double *b);
// consistent integration: quadrature data from nodal alpha, beta (device), and
// y = A_q x
hipError_t launch_q_setup(hx_ctx *c, const double *alpha, const double *beta);
hipError_t launch_apply_q(hx_ctx *c, const double *x, double *y);
// one Chebyshev step around block Jacobi (FP64): d = ca M^-1 r + cb d
// (cb used if read_d), then x += d (accum) or x = d
hipError_t launch_bj_cheb64(hx_ctx *c, const double *r, double *d, double *x, double ca, double cb,
                            int read_d, int accum);
hipError_t launch_bj_cheb32(hx_ctx *c, const float *r, float *d, float *x, double ca, double cb,
                            int read_d, int accum);
// z = p(M^-1 A) M^-1 r, the Chebyshev polynomial preconditioner (FP64)
hipError_t cheb_apply64(hx_ctx *c, const double *r, double *z);
// the same Chebyshev iteration for A x = b from the given x (x_zero: from
// zero, x is then only written): x <- x + p(M^-1 A) M^-1 (b - A x)
hipError_t cheb_iterate64(hx_ctx *c, const double *b, double *x, bool x_zero);
hipError_t cheb_iterate32(hx_ctx *c, const float *b, float *x, bool x_zero);
// geometric multigrid: x = V b, one V-cycle from the level c down (FP64);
// restriction of a fine dual vector to the next coarser level (overwrites
// b_coarse) and prolongation of a coarse vector added to x_fine
hipError_t mg_vcycle64(hx_ctx *c, const double *b, double *x);
hipError_t mg_restrict64(hx_ctx *c, const double *r_fine, double *b_coarse);
hipError_t mg_prolong_add64(hx_ctx *c, const double *x_coarse, double *x_fine);
// the same V-cycle in FP32 throughout (FP32 operator, smoother, transfers and
// level vectors) for an FP64 residual r: z = (double) V32 (float) r
hipError_t mg_vcycle_mixed(hx_ctx *c, const double *r, double *z);
// the same FP32 cycle from the finest level's FP32 input vector mgw32[0, n)
// to its output mgw32[n, 2n)
hipError_t mg_vcycle32_resident(hx_ctx *c);
// HX_OK if the chain of levels below c is usable by the V-cycle
hx_status mg_check(hx_ctx *c);
// h = gamma p / ((gamma - 1) rho) at the nodes
hipError_t launch_enthalpy(hx_ctx *c, const double *p, const double *rho, double gamma, double *h);
hipError_t launch_massinv32(hx_ctx *c, const float *r, float *z);
hipError_t launch_cg_massinv64(hx_ctx *c, double *x, double *r, const double *p, const double *q,
                               double *z, const double *sc, int *nblk, const double *pqp, int npq);
hipError_t launch_cg_massinv32(hx_ctx *c, float *x, float *r, const float *p, const float *q,
                               float *z, const double *sc, int *nblk, const double *pqp, int npq);

// operator: y = A x, or y = b - A x when b != nullptr
hipError_t launch_apply64(hx_ctx *c, const double *x, double *y, const double *b);
hipError_t launch_apply32(hx_ctx *c, const float *x, float *y, const float *b);
// non-conforming faces: geometry and penalties, merged data from nodal
// beta, and y += (y -= with residual) the quarter faces' terms of A x
hipError_t launch_hang_geometry(hx_ctx *c);
hipError_t launch_hang_coefficients(hx_ctx *c, const double *beta);
hipError_t launch_hang_apply64(hx_ctx *c, const double *x, double *y, bool residual);
hipError_t launch_hang_apply32(hx_ctx *c, const float *x, float *y, bool residual);
// cells per wave of the operator kernel at n points per direction
int op_cells_per_wave(int n);
// one part of A x: part 1 the cell integrals only, part 2 the face terms only
hipError_t launch_apply_part64(hx_ctx *c, int part, const double *x, double *y);
hipError_t launch_apply_part32(hx_ctx *c, int part, const float *x, float *y);
// y = A x and x.(A x) in FP64 (CG's p.q), summed in a fixed order.  With
// npq given and at most PQ_MAX per-workgroup partial sums, the partial sums
// stay in c->pqpart for the next fused CG step to sum (*npq = their count);
// otherwise dst = their sum (*npq = 0).
constexpr int PQ_MAX = 8192;
hipError_t launch_apply64_dot(hx_ctx *c, const double *x, double *y, double *dst,
                              int *npq = nullptr);
hipError_t launch_apply32_dot(hx_ctx *c, const float *x, float *y, double *dst,
                              int *npq = nullptr);
// dst = sum of part[0..n) in a fixed order (two stages)
hipError_t reduce_parts(hx_ctx *c, const double *part, int64_t n, double *dst);

// separable block Jacobi: z = Ahat^{-1} r
hipError_t launch_bj64(hx_ctx *c, const double *r, double *z);
hipError_t launch_bj32(hx_ctx *c, const float *r, float *z);

// BLAS-1 / block kernels (blas.hip); results of reductions stay on device
// in c->red[slot] unless copied.
hipError_t blas_dot(hx_ctx *c, int64_t n, const double *x, const double *y, double *dst);
hipError_t blas_dot32(hx_ctx *c, int64_t n, const float *x, const float *y, double *dst);
hipError_t blas_mdot(hx_ctx *c, int64_t n, int m, const double *V, int64_t ldv,
                     const double *w, double *dst /*[m]*/);
// One step of delayed classical Gram-Schmidt (blas.hip).  host_out (device
// view of a pinned slot, may be null) receives the step's scalars in the
// layout of sc and, from FG_PART, the nb partial sums of |w|^2 (*nb_out);
// with scale the normalised w goes to V[j+1] (else a later kernel does it).
hipError_t blas_dcgs(hx_ctx *c, int64_t n, int j, double *V, int64_t ldv, double *w, double *sc,
                     double *host_out, bool scale, int *nb_out);
constexpr int DCGS_S = 364;   // device scalars of blas_dcgs: 1/rho, hj/rho, rho, hj, flag
constexpr int FG_PART = 512;  // offset of the |w|^2 partial sums in a pinned slot
// c->red: stage-1 partial sums from 0, the |w|^2 partial sums of blas_dcgs
// at RED_WPART (at most 1024), solver scalars from 66 Ki
constexpr int64_t RED_WPART = 65536;
constexpr int FG_SLOT = 1536; // doubles per pinned slot
// v = w / |w| with |w|^2 the fixed-order sum (sum256) of part[0..nb), and
// z = block Jacobi of v, in one launch (FP64)
hipError_t launch_bj64_scaled(hx_ctx *c, const double *w, const double *part, int nb, double *v,
                              double *z);
// host repetition of the device's sum256 order
double host_sum256(const double *p, int nb);

hipError_t blas_mupdate(hx_ctx *c, int64_t n, int m, const double *V, int64_t ldv,
                        const double *h /*device [m]*/, double sign, double *w);
hipError_t blas_axpby(hx_ctx *c, int64_t n, double a, const double *x, double b, double *y);
hipError_t blas_scale_copy(hx_ctx *c, int64_t n, const double *s_dev, int inv,
                           const double *x, double *y);
hipError_t blas_cast64to32(hx_ctx *c, int64_t n, const double *x, float *y, const double *s_dev);
hipError_t blas_cast32to64(hx_ctx *c, int64_t n, const float *x, double *y, const double *s_dev);
hipError_t blas_copy(hx_ctx *c, int64_t n, const double *x, double *y);
hipError_t blas_fill(hx_ctx *c, int64_t n, double v, double *y);
hipError_t blas_fill32(hx_ctx *c, int64_t n, float v, float *y);
// fused CG steps on device scalars (no host round trip)
hipError_t cg32_init(hx_ctx *c, int64_t n, float *r, float *z, float *p, double *sc);
hipError_t cg32_step_x(hx_ctx *c, int64_t n, float *x, float *r, const float *p,
                       const float *q, double *sc, const double *pqp, int npq);
hipError_t cg32_step_p(hx_ctx *c, int64_t n, const float *z, float *p, double *sc);
// fused CG steps (scalars in sc[0..3], see blas.hip); p.q is the sum256 of
// pqp[0..npq) when pqp is given, else sc[1]
hipError_t launch_cg_bj64(hx_ctx *c, double *x, double *r, const double *p, const double *q,
                          double *z, const double *sc, int *nblk, const double *pqp, int npq);
hipError_t launch_cg_bj32(hx_ctx *c, float *x, float *r, const float *p, const float *q, float *z,
                          const double *sc, int *nblk, const double *pqp, int npq);
// flags of a fused CG step: the direction coefficient is in sc[5] and the
// new r.z already in sc[0] (no shift needed); r.r was written (or, deferred,
// will be written by the direction update) to host_rr; deferred: the
// direction update sums r.z and r.r itself
constexpr int CG_BETA_READY = 1, CG_RR_ON_HOST = 2, CG_DEFERRED = 4;
// A CG loop's state between its fused step and its direction update: the
// slot of sc (0 or 2) that holds the current r.z (with the deferred sums the
// direction update reads it and writes the new r.z to the other slot, so no
// workgroup overwrites a value others still read), the step's partial-sum
// count and the host slot for r.r.
struct CgLoop {
    int cur = 0;
    int nb = 0;
    double *host = nullptr;
};
hipError_t cg_step_pc64(hx_ctx *c, int pc, double *x, double *r, const double *p, const double *q,
                        double *z, double *sc, double *host_rr, int *flags, int npq, CgLoop *lp);
hipError_t cg_step_pc32(hx_ctx *c, int pc, float *x, float *r, const float *p, const float *q,
                        float *z, double *sc, int *flags, int npq, CgLoop *lp);
hipError_t cg_step_p64(hx_ctx *c, const double *z, double *p, double *sc, int flags, CgLoop *lp);
hipError_t cg_step_p32(hx_ctx *c, const float *z, float *p, double *sc, int flags, CgLoop *lp);
hipError_t cg32_step_p_dot(hx_ctx *c, int64_t n, const float *r, const float *z, double *sc);
hipError_t blas_lincomb(hx_ctx *c, int64_t n, int m, const double *Z, int64_t ldz,
                        const double *y_dev, double *x);

// learned preconditioner (mlp.hip)
hx_status mlp_create(hx_ctx *c);
void mlp_destroy(hx_ctx *c);
int64_t mlp_param_count(const hx_ctx *c);
hx_status mlp_set(hx_ctx *c, const float *w, int64_t n);
hx_status mlp_get(const hx_ctx *c, float *w, int64_t n);
hx_status mlp_features(hx_ctx *c, const double *r, float *feats, float *scale);
hx_status mlp_forward(hx_ctx *c, const float *feats, int64_t batch, float *out);
// the same forward pass with its work buffers in a static device array
hx_status noalloc_init(hx_ctx *c);
int64_t mlp_noalloc_max_batch(const hx_ctx *c);
hx_status mlp_forward_noalloc(hx_ctx *c, const float *feats, int64_t batch, float *out);
hx_status mlp_train(hx_ctx *c, const float *feats, const float *targets, int64_t batch,
                    float lr, float *loss_out, float *grad_out);
hx_status mlp_precondition(hx_ctx *c, const double *r, double *z);
hx_status mlp_precondition_batched(hx_ctx *c, const double *r, double *z);
hx_status mlp_trace(hx_ctx *c, int what, float *host_buf, int64_t count);
// z = BJ(v) + w_K net(features(v))_K with v = w / |w| (|w|^2 the sum256 of
// part[0..nbp); v written to vout) or v = w when part is null, in one launch
hx_status mlp_apply_fused(hx_ctx *c, const double *w, const double *part, int nbp, double *vout,
                          double *z);
hx_status mlp_training_pair(hx_ctx *c, const double *b, const double *xs, const double *xj,
                            float clip, float *feats, float *targets);

}  // namespace hx
