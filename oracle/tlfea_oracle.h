/*
 * tlfea_oracle.h -- plain FP64 CPU oracle for the internal force f_int and the
 * tangent stiffness K of the total-Lagrangian finite element method of
 * arXiv 2604.10357 (Part II), Sec. 4.1-4.4.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant with the library.
 *
 * Every function computes the plain definition in double precision with
 * natural loop order: no blocking, no fusion, no reordering.
 *
 * Conventions (shared with the library only through the written contract):
 *   DOF index = 3*coef + d.  T10 coef = node.  ANCF3443 coef = 4*node + k,
 *   k in (r, r_x, r_y, r_z).  CSR rows are sorted ascending; all entries of a
 *   3x3 block are stored.
 *
 * Readings where the paper is silent (it defers the formulas to Part I):
 *   SVK:  S = lambda tr(E) I + 2 mu E,  P = F S.
 *   MR:   W = mu10 (J^-2/3 I1 - 3) + mu01 (J^-4/3 I2 - 3) + kappa/2 (J-1)^2.
 *   KV:   S_v = 2 eta Edot + lambda_v tr(Edot) I,  P_v = F S_v.
 *   tangent(alpha, beta) = alpha dP/dF + beta dP/dFdot, contracted per Eq.
 *   (tangent_block), so (alpha, beta) = (h, 1) is d f_int(q_n + h v, v)/dv.
 */
#ifndef TLFEA_ORACLE_H
#define TLFEA_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_T10 1
#define ORC_ANCF3443 2
#define ORC_ANCF3243 3
#define ORC_SVK 1
#define ORC_MR 2

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EDEGENERATE -3
#define ORC_ENOTFOUND -7

typedef struct {
  int kind;         /* ORC_SVK: p = {E, nu, -}; ORC_MR: p = {mu10, mu01, kappa} */
  double p[3];
  double eta;       /* Kelvin-Voigt */
  double lam_v;
} orc_material;

typedef struct {
  int elem_type;      /* ORC_T10, ORC_ANCF3443 or ORC_ANCF3243 */
  int n_coef;         /* number of coefficient vectors (rows of X) */
  int n_elem;
  const int* conn;    /* T10: n_elem*10 node ids; ANCF3443: n_elem*4, ANCF3243: n_elem*2 physical node ids */
  const double* X;    /* n_coef*3 reference coefficients */
  int gl[3];          /* ANCF Gauss-Legendre points per parent direction */
  double thickness;   /* ANCF3443 shell thickness; ANCF3243 cross-section height (z) */
  double width;       /* ANCF3243 cross-section width (y) */
} orc_mesh;

/* quadrature: returns the number of points (pts: nq*3 parent coords, w: nq) */
int orc_quadrature(int elem_type, const int gl[3], double* pts, double* w);
int orc_gauss_legendre(int n, double* x, double* w);

/* shape functions and parent gradients */
void orc_t10_shape(const double xi[3], double N[10], double dN[30]);
int orc_ancf3443_shape(const double xi[3], double lx, double ly, double H,
                       double S[16], double dS[48]);
int orc_ancf3243_shape(const double xi[3], double L, double W, double H, double S[8], double dS[24]);

/* pointwise constitutive law; Hd = F - I (displacement gradient), Fdot */
double orc_energy_density(const orc_material* m, const double Hd[9]);
void orc_pk1(const orc_material* m, const double Hd[9], const double Fdot[9], double P[9]);
void orc_tangent(const orc_material* m, const double Hd[9], const double Fdot[9],
                 double alpha, double beta, double A[81]);

/* per element: dV[q] and physical gradients g[q][a][J] */
int orc_element_geometry(const orc_mesh* mesh, int e, double* dV, double* g);
int orc_n_en(int elem_type);
int orc_n_qp(const orc_mesh* mesh);

/* element force (3*n_en) and stiffness ((3 n_en)^2, row-major, may be NULL) */
int orc_element(const orc_mesh* mesh, const orc_material* mat, int e, const double* q,
                const double* qdot, double alpha, double beta, double* fe, double* Ke);

/* CSR pattern of the DOF-level matrix; returns nnz (or <0 on error).
 * With row_off == NULL only the count is returned. */
long long orc_csr_build(const orc_mesh* mesh, int* row_off, int* cols);

/* accumulate (+=) f and CSR values over the listed elements (elems == NULL: all).
 * f or vals may be NULL. */
int orc_assemble(const orc_mesh* mesh, const orc_material* mat, const double* q,
                 const double* qdot, double alpha, double beta, const int* elems,
                 int n_list, double* f, const int* row_off, const int* cols, double* vals);

/* canonical slot map for elements [e0, e0+ne): (3 n_en)^2 CSR positions each */
int orc_slot_map(const orc_mesh* mesh, const int* row_off, const int* cols, int e0, int ne,
                 int* slots);

/* vector-Jacobian products: gq = (df/dq)^T w, gqdot = (df/dqdot)^T w,
 * gparams[5] = d(w.f)/d(p0, p1, p2, eta, lam_v).  Outputs accumulate (+=). */
int orc_vjp(const orc_mesh* mesh, const orc_material* mat, const double* q, const double* qdot,
            const double* w, double* gq, double* gqdot, double* gparams);

/* consistent element mass m_ab = int rho N_a N_b dV (n_en x n_en; Sec. 4.1):
 * T10 exact on straight-sided elements (ORC_EINVAL if curved), ANCF3443 by
 * Gauss-Legendre 4x4x2 */
int orc_element_mass(const orc_mesh* mesh, int e, double rho, double* m);
/* accumulate (+=) M = [m_ab I_3] into CSR values of the mesh pattern */
int orc_mass_assemble(const orc_mesh* mesh, double rho, const int* row_off, const int* cols,
                      double* vals);
/* g = M (v - v_prev) / h + f_int - f_ext (Sec. 4.4.1, Eq. grad_L, no constraints) */
void orc_gradient(int n_dof, const int* row_off, const int* cols, const double* mvals, const double* v,
                  const double* v_prev, const double* f_int, const double* f_ext, double h, double* g);
/* total elastic energy sum_e sum_q dV W(F) */
double orc_energy(const orc_mesh* mesh, const orc_material* mat, const double* q);

#ifdef __cplusplus
}
#endif
#endif
