/*
 * helmdg -- matrix-free DG Helmholtz-type pressure operator and its
 * preconditioned Krylov solve on one AMD Instinct MI355X (gfx950).
 *
 * The operator is the implicit pressure step of an IMEX-DG compressible-Euler
 * solver (Orlando, Benacchio, Bonaventura, "Improving the scalability of a
 * high-order atmospheric dynamics solver based on the deal.II library",
 * arXiv:2505.00384): the Helmholtz-type equation for the pressure (section 2),
 * linearised with frozen coefficients, whose volume terms are the mass term
 * plus the dt-scaled, enthalpy-weighted stiffness of the matrix S~
 * (section 3.1, entries of the Helmholtz preconditioner), discretised by
 * symmetric interior-penalty DG with the tensor-product Lagrange basis on
 * (k+1) Gauss-Lobatto points (section 2) and (k+1)-point Gauss-Legendre
 * quadrature per direction (section 3.3):
 *
 *   a(u,v) = sum_K sum_q w_q detJ_q [alpha u v + beta grad u . grad v]
 *          + sum_F sum_q ds_q [ -1/2 (b- dn u- + b+ dn u+)[v]
 *                               -1/2 (b- dn v- + b+ dn v+)[u]
 *                               + sigma_F 1/2 (b- + b+)[u][v] ],
 *   sigma_F = P (k+1)^2 max(|F|/|K-|, |F|/|K+|),
 *
 * with [w] = w- - w+, n the unit normal of the minus cell (the cell whose +d
 * face it is), ds and n taken from the minus side, and natural Neumann
 * boundaries.  The operator is never assembled; only its action is computed
 * (section 3.1).
 *
 * Conventions for every call
 * --------------------------
 * - Vectors are cell-major; inside a cell the (k+1)^3 nodal values are in
 *   lexicographic Gauss-Lobatto order with x fastest:
 *   dof = cell*(k+1)^3 + i + (k+1)*(j + (k+1)*l).
 * - Vector arguments of apply/residual/preconditioner/solve are DEVICE
 *   pointers owned by the caller (e.g. torch tensors); the library never frees
 *   them.  FP64 vectors are double, FP32 vectors float.  They must not alias
 *   unless stated.
 * - Host arrays are copied during the call and may be freed afterwards.
 * - A context is bound at creation to one device and one HIP stream; every
 *   kernel of the context runs on that stream, so apply_* calls are
 *   asynchronous with respect to the host.  hx_solve returns after the solve
 *   has finished.  One context must not be used by two host threads at once.
 * - Every call returns an hx_status and never aborts; hx_last_error() gives a
 *   message for the last failed call of the context.
 */
#ifndef HELMDG_H
#define HELMDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hx_ctx hx_ctx;

typedef enum {
    HX_OK = 0,
    HX_ERR_ARG = 1,        /* invalid argument (null pointer, size, degree) */
    HX_ERR_STATE = 2,      /* call order: e.g. apply before mesh/coefficients */
    HX_ERR_DEVICE = 3,     /* a HIP runtime call failed */
    HX_ERR_OOM = 4,        /* device allocation failed */
    HX_ERR_MESH = 5,       /* detJ <= 0, or inconsistent neighbour table */
    HX_ERR_NOCONV = 6,     /* solver did not reach the tolerance */
    HX_FALLBACK_USED = 7   /* converged, after the fallback preconditioner took over */
} hx_status;

typedef enum { HX_F64 = 0, HX_F32 = 1 } hx_prec;

typedef enum {
    HX_PC_NONE = 0,
    HX_PC_BLOCK_JACOBI = 1,   /* separable cell block, fast-diagonalisation inverse */
    HX_PC_LEARNED = 2,        /* block Jacobi + per-cell network correction */
    HX_PC_HELMHOLTZ_DIAG = 3, /* inverse diagonal of the volume terms (mass + stiffness) */
    HX_PC_MASS_DIAG = 4,      /* inverse diagonal of the mass term alone */
    HX_PC_MASS_BLOCK = 5,     /* exact inverse of the alpha-weighted cell mass blocks */
    HX_PC_CHEBYSHEV = 6,      /* Chebyshev polynomial in M^-1 A, M = block Jacobi (FP64) */
    HX_PC_MULTIGRID = 7,      /* one geometric multigrid V-cycle (FP64, hx_set_multigrid) */
    HX_PC_MULTIGRID_MIXED = 8 /* the same V-cycle in FP32 for FP64 residuals */
} hx_pc;

/* Create a context on `device` (HIP ordinal) whose kernels run on
 * `hip_stream` (a hipStream_t; NULL = the null stream). */
hx_status hx_create(hx_ctx **out, int device, void *hip_stream);
/* Free every device buffer the context owns.  Accepts NULL. */
hx_status hx_destroy(hx_ctx *c);
/* Message of the last failed call (never NULL; "" if none). */
const char *hx_last_error(const hx_ctx *c);
/* Highest polynomial degree the library supports. */
int hx_max_degree(void);

/* ---------------------------------------------------------------------- */
/* setup: geometry of the mapped hexahedra (section 2, the DG space on the  */
/* mesh; section 3.3, J = detJ x quadrature weight at the Gauss points)    */
/* ---------------------------------------------------------------------- */

/* Upload a conforming hexahedral mesh and compute its geometry data.
 *   degree      polynomial degree k of the DG space, 1 <= k <= hx_max_degree()
 *   n_cells     number of cells (>= 1, < 2^31)
 *   geo_degree  g >= 1, degree of the cell map
 *   geo_nodes   HOST [n_cells][(g+1)^3][3]: node a + (g+1)*(b + (g+1)*c) is
 *               the image of the reference point (a/g, b/g, c/g); the cell map
 *               is the tensor-product Lagrange interpolant through them
 *   neighbours  HOST [n_cells][6]: cell across the -x,+x,-y,+y,-z,+z faces, -1
 *               for a boundary face; the +d face of a cell must be the -d face
 *               of its +d neighbour (conforming, standard orientation; a cell
 *               may be its own neighbour in a periodic direction)
 * Fails with HX_ERR_MESH if the table is inconsistent or detJ <= 0 at any
 * quadrature point.  Invalidates coefficients set before. */
hx_status hx_setup_mesh(hx_ctx *c, int degree, int64_t n_cells, int geo_degree,
                        const double *geo_nodes, const int64_t *neighbours);

/* The same for a non-conforming mesh with 2:1 faces (section 3: the paper's
 * second mesh refines part of its domain).  A face of a coarse cell C that
 * meets four finer cells is marked -2 in neighbours, on C and on each fine
 * cell, and described by n_hang records hang (HOST [n_hang][4]) =
 * {C, fc, F, s}: face fc (0..5 = -x, +x, -y, +y, -z, +z) of C, of which the
 * face fc ^ 1 of the fine cell F is quarter s = s1 + 2 s2 (s1, s2 the half
 * along the first and second of the two tangential directions, in the
 * direction order x, y, z; the fine cell's tangential axes run parallel to
 * the coarse cell's).  Each quarter carries the interior-penalty terms
 * integrated with the fine face's Gauss rule, the coarse side evaluated at
 * the images of those points, ds and n from the fine side, penalty
 * P (k+1)^2 max(|S|/|K_fine|, |S|/|K_coarse|).  Fails with HX_ERR_MESH unless
 * every face marked -2 is listed once (fine side) or with its four quarters
 * (coarse side).  The separable block Jacobi, the volume diagonals, the mass
 * blocks, Chebyshev and every solve accept such meshes; the geometric
 * multigrid, the pressure system and consistent integration return
 * HX_ERR_STATE on them. */
hx_status hx_setup_mesh_hanging(hx_ctx *c, int degree, int64_t n_cells, int geo_degree,
                                const double *geo_nodes, const int64_t *neighbours,
                                int64_t n_hang, const int64_t *hang);

/* Physical coordinates of every dof (Gauss-Lobatto node images), written to
 * the DEVICE array xyz [3][n_dofs] (all x, then all y, then all z). */
hx_status hx_dof_coordinates(hx_ctx *c, double *xyz);

/* Number of dofs, (k+1)^3 * n_cells, or -1 without a mesh. */
int64_t hx_num_dofs(const hx_ctx *c);

/* ---------------------------------------------------------------------- */
/* coefficients (section 3.1: the entries of S~, rebuilt each fixed-point */
/* iteration from the previous pressure)                                  */
/* ---------------------------------------------------------------------- */

/* Set the mass coefficient alpha and the stiffness coefficient beta (the
 * dt-scaled enthalpy weight) as DG nodal fields [n_dofs] (FP64), and the
 * penalty factor P (> 0; 2 is the usual choice).  Pointers are device
 * pointers if on_device != 0, host pointers otherwise.  Builds the merged
 * per-quadrature-point data of the operator in FP64 and FP32 and the
 * separable block-Jacobi data.  In the fixed-point iteration of the paper
 * (section 3.1) this is redone each outer iteration with the new pressure. */
hx_status hx_set_coefficients(hx_ctx *c, const double *alpha, const double *beta,
                              double penalty_factor, int on_device);

/* ---------------------------------------------------------------------- */
/* operator action (section 2: the Helmholtz-type equation for the       */
/* pressure; section 3.1: matrix-free evaluation)                          */
/* ---------------------------------------------------------------------- */

/* y = A x (y overwritten).  prec selects FP64 (double*) or FP32 (float*)
 * vectors and arithmetic; the FP32 form uses an FP32 copy of the merged
 * geometry and accumulates in FP32.  x and y must not alias. */
hx_status hx_apply_operator(hx_ctx *c, hx_prec prec, const void *x, void *y);

/* r = b - A x in FP64.  r must not alias b or x. */
hx_status hx_residual(hx_ctx *c, const double *b, const double *x, double *r);

/* One part of y = A x (y overwritten): HX_PART_CELL the cell integrals
 * (mass and stiffness volume terms), HX_PART_FACE the interior-penalty face
 * terms; their sum is hx_apply_operator.  For measurement and checks. */
#define HX_PART_CELL 1
#define HX_PART_FACE 2
hx_status hx_apply_operator_part(hx_ctx *c, hx_prec prec, int part, const void *x, void *y);

/* Affine cells (geometry nodes an affine image of the reference nodes, to
 * 1e-14 of the cell size) have a constant Jacobian; the operator then reads
 * J^-1 J^-T once per cell and alpha w detJ, beta w detJ at the points (2
 * values per point instead of 7), and on faces between two affine cells
 * beta- w, beta+ w per point plus 7 constants per face (instead of 7 values
 * per point).  on = 1 (the default after hx_setup_mesh) uses this compressed
 * data; on = 0 makes every cell and face read the general data.  The results
 * agree to rounding. */
hx_status hx_set_cell_compression(hx_ctx *c, int on);

/* Counts of the mesh as the operator sees it, counts[4] (HOST, may be NULL)
 * = {cells, affine cells, interior faces, interior faces between two affine
 * cells}, and *bytes (HOST, may be NULL) = the bytes one application in the
 * precision prec must move at the least: x and y, and each cell's and each
 * interior face's data once, compressed where it applies. */
hx_status hx_operator_info(const hx_ctx *c, int prec, int64_t *counts, double *bytes);

/* ---------------------------------------------------------------------- */
/* preconditioners (section 3.1: the Helmholtz and internal-energy        */
/* diagonals; section 3.3: tensor-product inverses of cell blocks)        */
/* ---------------------------------------------------------------------- */

/* z = M^{-1} r.  HX_PC_BLOCK_JACOBI: inverse of the separable approximation
 * of each cell block,
 *   Ahat_K = abar lx ly lz M(x)M(x)M + bbar [ (ly lz/lx) L_x(x)M(x)M + ... ],
 * applied by fast diagonalisation (S_z(x)S_y(x)S_x) D^{-1} (S_z(x)S_y(x)S_x)^T
 * with S^T M S = I, S^T L S = Lambda -- the tensor-product inverse of
 * block-diagonal operators of section 3.3, with the 1-D SIP blocks in place of
 * the mass.  HX_PC_LEARNED (FP64 only; needs hx_set_network): block Jacobi
 * plus the per-cell network correction w_K net(features(r))_K, with w_K the
 * RMS of the block-Jacobi output on cell K.  HX_PC_HELMHOLTZ_DIAG: the
 * paper's "Helmholtz preconditioner" (section 3.1), the inverse of the
 * diagonal of the volume terms of the form,
 *   d_i = sum_q w_q detJ_q [alpha_q phi_i^2 + beta_q |J^-T grad phi_i|^2],
 * face terms left out; HX_PC_MASS_DIAG: its "internal-energy" variant, the
 * inverse of the mass diagonal alone.  Both diagonals are formed by
 * hx_set_coefficients.  HX_PC_MASS_BLOCK: the exact inverse of the
 * block-diagonal mass matrix with entries sum_q w_q detJ_q alpha_q phi_i phi_j
 * (curved cells and variable alpha included), by the tensor-product form of
 * section 3.3, M_K^{-1} = B3^{-1} diag(1/(w detJ alpha)) B3^{-T} with B3 the
 * square interpolation from the (k+1)^3 nodes to the (k+1)^3 Gauss points;
 * it reads the first component of the merged cell data.  HX_PC_NONE copies
 * r.  r and z must not alias. */
hx_status hx_apply_preconditioner(hx_ctx *c, hx_pc kind, hx_prec prec,
                                  const void *r, void *z);

/* ---------------------------------------------------------------------- */
/* solve (section 3.1: preconditioned CG for the SPD systems, GMRES with  */
/* a Jacobi-type preconditioner for the pressure system)                  */
/* ---------------------------------------------------------------------- */

typedef struct {
    int method;          /* 0 = preconditioned CG, 1 = flexible GMRES(restart) */
    int restart;         /* FGMRES restart length, 1..63 (30) */
    double rtol;         /* stop when ||b - A x||_2 <= rtol ||b||_2 */
    int max_iter;        /* total iteration cap */
    int pc;              /* hx_pc of the iteration; with mixed = 1, of the inner FP32 CG
                            (HX_PC_LEARNED is not allowed there) */
    int mixed;           /* 0: FP64 throughout; 1: outer FP64 FGMRES, preconditioner =
                            inner FP32 CG; 2 (minimal form): FP64 FGMRES vectors and
                            orthogonalisation, the operator and the preconditioner pc
                            (block Jacobi, a diagonal kind, the mass blocks or none)
                            applied once per step in FP32; the FP64 residual at each
                            restart refines (Helmholtz-type system only) */
    int inner_iters;     /* inner FP32 CG iterations per outer step (mixed; 32) */
    double inner_rtol;   /* not used: the inner FP32 CG runs inner_iters iterations with its
                            scalars on the device, so it has no stopping test */
    int x0_mode;         /* 0: start from zero, 1: x holds the initial guess */
    int stall_window;    /* FGMRES stall rule window (10); 0 disables it */
    double stall_ratio;  /* stall if estimate > ratio * estimate window ago (0.99) */
    int orth;            /* FGMRES orthogonalisation, both classical Gram-Schmidt twice:
                            0 = two block-dot/update pairs per step (four passes over
                            the basis), 1 = second pass delayed by one step and fused
                            with the next step's (two passes; default) */
    int system;          /* 0 = the Helmholtz-type operator A (default); 1 = the pressure
                            system S = D - C A^-1 B of hx_set_pressure_system (FGMRES
                            only: S is not symmetric); the preconditioners, the inner
                            FP32 CG of the mixed form included, act with the
                            Helmholtz-type operator set by hx_set_pressure_system;
                            2 = the operator with consistent integration of
                            hx_set_consistent (CG or FGMRES), preconditioned by the
                            preconditioners of the (k+1)-point operator (block
                            Jacobi, the mass-block inverse, Chebyshev, multigrid,
                            the inner FP32 CG) */
} hx_solve_params;

typedef struct {
    int iters;           /* outer iterations */
    int restarts;        /* FGMRES cycles */
    int status;          /* hx_status of the solve */
    int fallback_used;   /* 1 if the learned preconditioner was replaced by BJ */
    int inner_iters;     /* total inner (FP32) iterations, mixed form */
    double true_rel_res; /* ||b - A x||_2 / ||b||_2 in FP64, recomputed at the end */
    double ms_total;     /* wall time of the solve (host clock) */
    double ms_op, ms_pc, ms_orth;  /* device time per phase (HIP events): operator,
                                      preconditioner, orthogonalisation (FGMRES) or
                                      vector updates and dot products (CG) */
    double *history;     /* optional HOST buffer: residual estimate per iteration */
    int history_len;     /* in: capacity of history; out: entries written */
} hx_solve_info;

/* Fill p with the defaults (CG, restart 30, rtol 1e-8, max_iter 10000, block
 * Jacobi, FP64, inner 12 iterations, zero initial guess, stall 10/0.99). */
void hx_default_params(hx_solve_params *p);

/* Solve A x = b.  b, x: DEVICE FP64 [n_dofs]; x is the initial guess if
 * x0_mode = 1 and always receives the best iterate.  info is always written.
 * Returns HX_OK, HX_FALLBACK_USED (converged after the learned preconditioner
 * stalled or produced a non-finite value and block Jacobi took over) or
 * HX_ERR_NOCONV. */
hx_status hx_solve(hx_ctx *c, const hx_solve_params *prm, const double *b,
                   double *x, hx_solve_info *info);

/* Chebyshev polynomial preconditioner (section 3.1 names it for the
 * symmetric positive-definite systems: a polynomial that damps the eigenvalue
 * range of the preconditioned operator, the range estimated by the Lanczos
 * process).  HX_PC_CHEBYSHEV applies z = p(M^-1 A) M^-1 r: `degree` steps of
 * the Chebyshev iteration for A z = r from z = 0 on the interval [lo, hi] of
 * the eigenvalues of M^-1 A, M the block Jacobi preconditioner; each step
 * costs one operator and one block-Jacobi application.  The result is a
 * fixed SPD operator when lo is at most the smallest eigenvalue, so CG may
 * use it.  hx_set_chebyshev stores degree (1..64) and 0 < lo < hi.
 * hx_estimate_eigenvalues runs `iters` (1..200) steps of CG with block
 * Jacobi on A x = b (b DEVICE FP64 [n_dofs], e.g. random) and returns the
 * extreme Ritz values of M^-1 A (HOST) from the Lanczos tridiagonal matrix of
 * the CG coefficients: lo from above, hi from below. */
hx_status hx_set_chebyshev(hx_ctx *c, int degree, double lo, double hi);
hx_status hx_estimate_eigenvalues(hx_ctx *c, const double *b, int iters, double *lo, double *hi);

/* Geometric multigrid (section 3.1: CG preconditioned by geometric multigrid
 * for the SPD systems, smoothed by Chebyshev polynomials).  Each level is a
 * context of its own with its mesh, coefficients (the operator is
 * re-discretised on every level) and Chebyshev polynomial (hx_set_chebyshev:
 * the smoother, typically on [hi/15, 1.1 hi] of the level's estimated range;
 * on the coarsest level it replaces the coarse solve, typically over the
 * whole range with a higher degree).  hx_set_multigrid(c, coarse, ...) makes
 * `coarse` the next coarser level of c; calling it on every level but the
 * coarsest builds the hierarchy.  The levels must share the device, the
 * stream and the degree, and the fine mesh must be a refinement of the
 * coarse one: parent[f] (HOST int32 [n_cells of c]) is the coarse cell that
 * holds fine cell f and octant[f] = ox + 2 oy + 4 oz (0..7) the octant of its
 * reference cube that f fills, with the same axis orientation; no two cells
 * may fill the same octant of one parent.  Prolongation writes the parent's
 * polynomial in the child's basis (exact embedding of the spaces), and
 * restriction is its transpose.  HX_PC_MULTIGRID then applies x = V r, one
 * V-cycle: the level's Chebyshev polynomial from zero, the restricted
 * residual handed to the next level's V-cycle and its prolongation added,
 * and the same polynomial on the updated residual; it is a fixed symmetric
 * operator, so CG may use it.  HX_PC_MULTIGRID_MIXED runs the same cycle in
 * FP32 throughout (FP32 operator, smoother, transfers and level vectors) on
 * the FP64 residual rounded to FP32 and returns it widened to FP64: about
 * half the bytes per cycle, at the price of a preconditioner that is linear
 * and symmetric only up to FP32 rounding (CG tolerates that in practice,
 * FGMRES by construction).  coarse = NULL removes the link.  c does not
 * own `coarse`: keep it alive while linked; set up its mesh again and the
 * link must be set again.  Errors: HX_ERR_ARG for bad maps, a degree,
 * device or stream mismatch or a cycle of links; HX_ERR_STATE before
 * hx_setup_mesh; a failed call leaves c without a coarser level.  Working
 * memory: 3 n_dofs doubles and 3 n_dofs floats on each linked level (and 2
 * of each per level for its Chebyshev polynomial).
 *
 * hx_mg_transfer applies one transfer of the link (DEVICE FP64 vectors):
 * dir 0 restricts `in` ([n_dofs of c]) into `out` ([n_dofs of the coarse
 * level], overwritten); dir 1 adds the prolongation of `in` (coarse) to
 * `out` (fine).  in and out must not alias. */
hx_status hx_set_multigrid(hx_ctx *c, hx_ctx *coarse, const int32_t *parent, const int32_t *octant);
hx_status hx_mg_transfer(hx_ctx *c, int dir, const double *in, double *out);

/* ---------------------------------------------------------------------- */
/* consistent integration                                                   */
/* ---------------------------------------------------------------------- */

/* Section 3.3 contrasts the fast evaluation with (r+1) Gauss points per
 * direction (exact for mass matrices, aliasing for products of three
 * polynomials such as variable-coefficient terms) with consistent
 * integration by 2r+1 points.  hx_set_consistent builds the quadrature data
 * of the same form (cell and face terms, penalty of hx_set_coefficients)
 * with nq = 2k+1 points from nodal alpha, beta ([n_dofs], HOST, or DEVICE
 * with on_device = 1): 7 nq^3 numbers per cell and 21 nq^2 per cell for the
 * faces (for k = 4, 5.4x the data of the fast form).  Requires
 * hx_set_coefficients (for the penalty).  hx_apply_consistent: y = A_q x,
 * x, y DEVICE FP64 [n_dofs], distinct. */
hx_status hx_set_consistent(hx_ctx *c, const double *alpha, const double *beta, int on_device);
hx_status hx_apply_consistent(hx_ctx *c, const double *x, double *y);

/* ---------------------------------------------------------------------- */
/* pressure system of one IMEX stage                                        */
/* ---------------------------------------------------------------------- */

/* Section 2 writes the stage as the discrete momentum and energy equations
 *   A U + B P = F,   C U + D P = G,
 * and solves D P + C A^-1 (F - B P) = G for the pressure, i.e.
 *   S P = (D - C A^-1 B) P = G - C A^-1 F.
 * The paper does not give the matrices; from the stage equations with
 * central fluxes (velocity: three DG fields of the pressure space,
 * component-major [3][n_dofs]):
 *   (B p)_{e,i} = tau [ -int_K p d_e phi_i + int_dK p^ phi_i n_e ],
 *                 p^ = {p} inside, the own trace on boundary faces;
 *   (C u)_i     = tau [ -int_K h rho u . grad Psi_i + int_dK {h rho u . n} Psi_i ],
 *                 no flux through boundary faces;
 *   A = rho-weighted velocity mass (one block per cell and component),
 *   D = mass / (gamma - 1) (internal energy of an ideal gas),
 * all with the (k+1)-point Gauss rules of the operator, so A^-1 is the exact
 * tensor-product inverse of section 3.3.  tau = a_ll dt.
 *
 * Set-up: rho, h (specific enthalpy) nodal fields [n_dofs] (HOST, or DEVICE
 * with on_device = 1), gamma > 1, tau > 0.  It also calls
 * hx_set_coefficients with alpha = 1/(gamma - 1) and beta = tau^2 h: the
 * Helmholtz-type operator whose volume diagonal is the paper's Helmholtz
 * preconditioner (section 3.1) and which preconditions S.  Requires
 * setup_mesh; may be called again with new fields (the fixed-point loop). */
hx_status hx_set_pressure_system(hx_ctx *c, const double *rho, const double *h, double gamma,
                                 double tau, double penalty_factor, int on_device);

typedef enum {
    HX_PS_GRAD = 0,       /* out[3][n] = B in[n] */
    HX_PS_DIV = 1,        /* out[n] = C in[3][n] */
    HX_PS_VMASS_INV = 2,  /* out[3][n] = A^-1 in[3][n] */
    HX_PS_DMASS = 3,      /* out[n] = D in[n] */
    HX_PS_SYSTEM = 4      /* out[n] = S in[n] */
} hx_ps_part;

/* Apply one part of the pressure system; in, out DEVICE FP64, distinct. */
hx_status hx_apply_pressure_part(hx_ctx *c, int part, const double *in, double *out);

/* rhs[n] = G - C A^-1 F (F DEVICE [3][n], G DEVICE [n]). */
hx_status hx_pressure_rhs(hx_ctx *c, const double *F, const double *G, double *rhs);

/* U[3][n] = A^-1 (F - B P): the velocity of the stage once P is known. */
hx_status hx_pressure_velocity(hx_ctx *c, const double *F, const double *P, double *U);

/* Fixed-point solve of the pressure system (section 2; the coefficients of
 * the system and of its Helmholtz preconditioner are re-evaluated from the
 * previous iterate, section 3.1).  For m = 0, 1, ...: h = gamma p_m /
 * ((gamma - 1) rho) at the nodes (ideal gas), hx_set_pressure_system(rho, h),
 * p_{m+1} = solution of S(h) p = G - C(h) A^-1 F by hx_solve with prm
 * (system 1 and the previous iterate as initial guess are imposed); stop when
 * ||p_{m+1} - p_m|| <= fp_tol ||p_{m+1}|| or after max_fp_iters iterations.
 * rho [n], F [3][n], G [n], p [n] DEVICE FP64; p holds p_0 and receives the
 * last iterate.  *fp_iters, *fp_change (HOST, may be NULL): iterations done and
 * the last relative change; info: the last linear solve.  Returns HX_OK or
 * HX_ERR_NOCONV (fixed point or linear solve not converged). */
hx_status hx_solve_pressure_fixed_point(hx_ctx *c, const double *rho, const double *F,
                                        const double *G, double *p, double gamma, double tau,
                                        double penalty_factor, const hx_solve_params *prm,
                                        int max_fp_iters, double fp_tol, int *fp_iters,
                                        double *fp_change, hx_solve_info *info);

/* ---------------------------------------------------------------------- */
/* BLAS-1 helpers on the context stream (Krylov scalars), FP64 vectors    */
/* ---------------------------------------------------------------------- */

/* *out (HOST) = x . y, deterministic two-stage reduction. */
hx_status hx_dot(hx_ctx *c, int64_t n, const double *x, const double *y, double *out);

/* ---------------------------------------------------------------------- */
/* learned preconditioner (not in the paper: a per-cell network added to  */
/* block Jacobi inside flexible GMRES)                                    */
/* ---------------------------------------------------------------------- */

/* Network: n_in = (k+1)^3 + 6 (k+1)^2 + 1 -> 256 -> 256 -> (k+1)^3, ReLU,
 * parameters flat [W1, b1, W2, b2, W3, b3], W row-major [out][in].  BF16
 * weights and activations, FP32 accumulation on MFMA; FP32 master weights
 * and Adam moments live in the context. */
int64_t hx_network_size(const hx_ctx *c);

/* Load FP32 master weights (HOST, n = hx_network_size) and reset Adam. */
hx_status hx_set_network(hx_ctx *c, const float *master_weights, int64_t n);
/* Copy the FP32 master weights to the HOST buffer. */
hx_status hx_get_network(const hx_ctx *c, float *master_weights, int64_t n);

/* Features of every cell from the FP64 residual r (DEVICE [n_dofs]):
 * feats DEVICE float [n_cells][n_in] (r_K, the six neighbour face layers, the
 * coefficient feature log(bbar/(abar l^2)), all but the last divided by
 * s = RMS(r_K)), scale DEVICE float [n_cells] (s). */
hx_status hx_gather_features(hx_ctx *c, const double *r, float *feats, float *scale);

/* Training pair of every cell from an iterate x_j of a solve of A x = b whose
 * converged solution is x_star (all DEVICE FP64 [n_dofs]): with r = b - A x_j
 * and e = x_star - x_j, feats = features(r) as in hx_gather_features and
 * targets DEVICE float [n_cells][n_out] = (e_K - BJ(r)_K) / w_K, w_K = RMS(BJ(r)_K):
 * the part of the error that block Jacobi misses, in the network's output
 * scaling; with clip > 0 each target is limited to [-clip, clip] (0: none;
 * negative: HX_ERR_ARG). */
hx_status hx_training_pair(hx_ctx *c, const double *b, const double *x_star, const double *x_j,
                           float clip, float *feats, float *targets);

/* out DEVICE float [batch][n_out] = network(feats DEVICE float [batch][n_in]). */
hx_status hx_network_forward(hx_ctx *c, const float *feats, int64_t batch, float *out);

/* The same forward pass for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or allocating library routine.
 * Its work buffers (packed BF16 inputs and both hidden layers, 2 (ldx + 512)
 * bytes per row, ldx = n_in rounded up to 32) live in one 16 MiB static
 * device array per GPU, held until the process ends; batch may not exceed
 * hx_network_noalloc_max_batch (10,485 rows at Q4), else HX_ERR_ARG and no
 * launch.  Arguments and layout as hx_network_forward; the result is the
 * same bit for bit.  All calls on one GPU share the array: calls that
 * overlap on one GPU (several streams or threads) race.  Asynchronous on the
 * context's stream. */
hx_status hx_network_forward_noalloc(hx_ctx *c, const float *feats, int64_t batch, float *out);
/* Largest batch of hx_network_forward_noalloc for this context's degree
 * (-1 before hx_setup_mesh). */
int64_t hx_network_noalloc_max_batch(const hx_ctx *c);

/* One Adam step on the MSE loss mean((net(feats) - targets)^2): forward,
 * backward and update on the GPU.  feats DEVICE float [batch][n_in], targets
 * DEVICE float [batch][n_out]; *loss_out (HOST, may be NULL) = loss before
 * the step.  With grad_out (DEVICE float [hx_network_size], may be NULL) the
 * gradient is also returned and, if lr == 0, no update is made. */
hx_status hx_train_step(hx_ctx *c, const float *feats, const float *targets,
                        int64_t batch, float lr, float *loss_out, float *grad_out);

/* Intermediates of the last hx_train_step, for checking each layer on the
 * operands the GPU actually used.  what (all FP32, row-major, batch rows):
 *   HX_TRACE_INPUT  [batch][n_in]  the BF16-rounded inputs;
 *   HX_TRACE_H1/H2  [batch][256]   hidden layer 1/2 after bias and ReLU,
 *                                  before the BF16 rounding of the next product;
 *   HX_TRACE_OUT    [batch][n_out] the network output;
 *   HX_TRACE_DOUT   [batch][n_out] d loss / d output, before BF16 rounding;
 *   HX_TRACE_DH2/DH1 [batch][256]  d loss / d pre-activation of hidden layer
 *                                  2/1 (ReLU mask applied), before BF16 rounding.
 * count = the number of floats of the HOST buffer and must equal the size
 * above (HX_ERR_ARG otherwise); HX_ERR_STATE when no step has been taken or
 * a call that shares the step's work buffers (hx_network_forward,
 * hx_training_pair) has run since.  Synchronous. */
enum {
    HX_TRACE_INPUT = 0, HX_TRACE_H1 = 1, HX_TRACE_H2 = 2, HX_TRACE_OUT = 3,
    HX_TRACE_DOUT = 4, HX_TRACE_DH2 = 5, HX_TRACE_DH1 = 6
};
hx_status hx_network_trace(hx_ctx *c, int what, float *host_buf, int64_t count);

/* ---------------------------------------------------------------------- */
/* inspection                                                              */
/* ---------------------------------------------------------------------- */

enum {
    HX_EXPORT_CELL_DATA = 0,   /* FP64 [n_cells][7][(k+1)^3]: m, Gxx, Gxy, Gxz, Gyy, Gyz, Gzz */
    HX_EXPORT_FACE_DATA = 1,   /* FP64 [n_cells][3][7][(k+1)][(k+1)]: g-(3), g+(3), s of the +d face;
                                  g components in the order normal direction d, first, second
                                  tangential direction; points [first][second tangential] */
    HX_EXPORT_SIGMA = 2,       /* FP64 [n_cells][3]: penalty of the +d face (-1: boundary) */
    HX_EXPORT_VOLUME = 3,      /* FP64 [n_cells] */
    HX_EXPORT_BJ_SCALARS = 4,  /* FP64 [n_cells][4]: abar lx ly lz, bbar ly lz/lx, ... */
    HX_EXPORT_INV_DIAG = 5     /* FP64 [2][n_dofs]: inverse volume diagonals, mass + stiffness
                                  (HX_PC_HELMHOLTZ_DIAG) then mass alone (HX_PC_MASS_DIAG) */
};
/* Copy internal data to a HOST buffer of `bytes` bytes (for tests). */
hx_status hx_debug_export(hx_ctx *c, int what, void *host_buf, int64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* HELMDG_H */
