/* Oracle (test infrastructure only): plain FP64 reference of the DG
 * Helmholtz-type pressure operator and its separable cell-block
 * preconditioner.  Not part of the product library. */
#ifndef HELM_ORACLE_H
#define HELM_ORACLE_H

#define OR_CELL 1
#define OR_FACE 2

typedef struct {
    int k;                 /* polynomial degree of the DG space */
    int g;                 /* degree of the geometry map */
    long n_cells;
    const double *nodes;   /* [n_cells][(g+1)^3][3], equispaced reference nodes */
    const long *nbr;       /* [n_cells][6]: -x,+x,-y,+y,-z,+z; -1 = boundary */
    const double *alpha;   /* [n_cells*(k+1)^3] DG nodal field */
    const double *beta;    /* [n_cells*(k+1)^3] DG nodal field */
    double P;              /* penalty factor */
    long n_hang;           /* non-conforming (2:1) subfaces, 0 on a conforming mesh */
    const long *hang;      /* [n_hang][4] = {coarse cell C, its face fc, fine cell F, quarter s}:
                              face fc^1 of F is quarter s = s1 + 2 s2 of face fc of C
                              (s1, s2: halves along the first, second tangential
                              direction); both faces are marked -2 in nbr */
} or_prob;

void or_gauss_legendre(int n, double *x, double *w);
void or_gauss_lobatto(int n, double *x, double *w);
void or_lagrange(int n, const double *nodes, double t, double *val, double *der);

int  or_mesh_check(const or_prob *p);
void or_dof_coords(const or_prob *p, double *xyz);
void or_quad_data(const or_prob *p, double *xyz, double *wdet);
void or_load_vector(const or_prob *p, const double *fq, double *b);
void or_cell_volumes(const or_prob *p, double *vol);
void or_face_sigma(const or_prob *p, double *sigma);
void or_hang_sigma(const or_prob *p, double *sigma);
void or_eval_quad(const or_prob *p, const double *u, double *uq);
void or_apply(const or_prob *p, int flags, const double *x, double *y);
void or_apply_cells(const or_prob *p, int flags, const long *cells, long m,
                    const double *x, double *out);
void or_apply_q(const or_prob *p, int nq, int flags, const double *x, double *y);
void or_apply_q_cells(const or_prob *p, int nq, int flags, const long *cells, long m,
                      const double *x, double *out);
void or_assemble_dense(const or_prob *p, int flags, double *A);
void or_cell_diagonal(const or_prob *p, int stiff, double *diag);
void or_bj_cell_data(const or_prob *p, long c, double ell[3], double *abar,
                     double *bbar, double sig[3][2]);
void or_bj_sep_block(const or_prob *p, long c, double *Ab);
int  or_bj_sep_apply(const or_prob *p, const double *r, double *z);
void or_mass_block(const or_prob *p, long c, double *Mb);
int  or_mass_block_apply(const or_prob *p, const double *r, double *z);
void or_grad_apply(const or_prob *p, double tau, const double *pv, double *u3);
void or_div_apply(const or_prob *p, double tau, const double *hr, const double *u3, double *q);
void or_grad_apply_cells(const or_prob *p, double tau, const long *cells, long m, const double *pv,
                         double *out);
void or_div_apply_cells(const or_prob *p, double tau, const double *hr, const long *cells, long m,
                        const double *u3, double *out);

#endif
