/*
 * tlfea_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * What it computes, and where the paper defines it (arXiv 2604.10357, Part II):
 *   - reference-configuration constants: quadrature, parent gradients, J0,
 *     det J0, physical gradients (Sec. 4.1);
 *   - deformation gradient F = sum_a x_a (x) grad N_a (Sec. 4.3, Eq. F_assembly),
 *     evaluated in the equivalent displacement form I + sum_a (x_a - X_a) (x) g_a;
 *   - PK1 stress P = P_el + P_vis (Sec. 4.3, Stage 1);
 *   - element force f_a = sum_q P g_a J0 w_q (Sec. 4.3, Eq. fint_local) and its
 *     scatter (Eqs. fint_global, atomic_scatter), here a serial +=;
 *   - tangent blocks K_ab = sum_q A g_a g_b J0 w_q (Sec. 4.4.2, Eq. tangent_block);
 *   - the DOF-level CSR pattern built from coefficient adjacency lifted to 3x3
 *     blocks (Sec. 4.2; Sec. 4.4.2);
 *   - vector-Jacobian products and the energy used by the tests.
 *
 * The paper defers the constitutive formulas to Part I; the textbook forms used
 * here are listed in tlfea_oracle.h.  No line of this file is shared with the
 * GPU library.
 */
#include "tlfea_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* 3x3 helpers (row-major, M[3*i + j])                                        */
/* ------------------------------------------------------------------------- */

static double det3(const double* M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
         M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* inverse through the adjugate; returns the determinant */
static double inv3(const double* M, double* R) {
  double d = det3(M);
  R[0] = (M[4] * M[8] - M[5] * M[7]) / d;
  R[1] = (M[2] * M[7] - M[1] * M[8]) / d;
  R[2] = (M[1] * M[5] - M[2] * M[4]) / d;
  R[3] = (M[5] * M[6] - M[3] * M[8]) / d;
  R[4] = (M[0] * M[8] - M[2] * M[6]) / d;
  R[5] = (M[2] * M[3] - M[0] * M[5]) / d;
  R[6] = (M[3] * M[7] - M[4] * M[6]) / d;
  R[7] = (M[1] * M[6] - M[0] * M[7]) / d;
  R[8] = (M[0] * M[4] - M[1] * M[3]) / d;
  return d;
}

static double kron(int i, int j) { return i == j ? 1.0 : 0.0; }

/* ------------------------------------------------------------------------- */
/* Quadrature (Sec. 4.1: tabulated once per element type and order; Sec. 4.3   */
/* names the 5-point Keast rule for T10 and Gauss-Legendre products for ANCF)  */
/* ------------------------------------------------------------------------- */

int orc_gauss_legendre(int n, double* x, double* w) {
  /* textbook Gauss-Legendre nodes and weights on [-1, 1] */
  switch (n) {
    case 1:
      x[0] = 0.0; w[0] = 2.0;
      return 1;
    case 2:
      x[0] = -1.0 / sqrt(3.0); x[1] = -x[0];
      w[0] = w[1] = 1.0;
      return 2;
    case 3:
      x[0] = -sqrt(0.6); x[1] = 0.0; x[2] = sqrt(0.6);
      w[0] = w[2] = 5.0 / 9.0; w[1] = 8.0 / 9.0;
      return 3;
    case 4: {
      double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
      double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
      double wa = (18.0 + sqrt(30.0)) / 36.0, wb = (18.0 - sqrt(30.0)) / 36.0;
      x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
      w[0] = wb; w[1] = wa; w[2] = wa; w[3] = wb;
      return 4;
    }
    case 5: {
      double a = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
      double b = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
      double wa = (322.0 + 13.0 * sqrt(70.0)) / 900.0, wb = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
      x[0] = -b; x[1] = -a; x[2] = 0.0; x[3] = a; x[4] = b;
      w[0] = wb; w[1] = wa; w[2] = 128.0 / 225.0; w[3] = wa; w[4] = wb;
      return 5;
    }
    default:
      return ORC_EINVAL;
  }
}

int orc_quadrature(int elem_type, const int gl[3], double* pts, double* w) {
  if (elem_type == ORC_T10) {
    /* Keast 5-point rule on the unit tetrahedron {xi, eta, zeta >= 0,
     * xi + eta + zeta <= 1}: the centroid with weight -4/5 and the four points
     * with barycentric coordinates (1/2, 1/6, 1/6, 1/6) and permutations with
     * weight 9/20, all scaled by the reference volume 1/6.  Parent coordinates
     * are the barycentric coordinates L1, L2, L3. */
    double bary[5][4] = {{0.25, 0.25, 0.25, 0.25},
                         {0.5, 1.0 / 6, 1.0 / 6, 1.0 / 6},
                         {1.0 / 6, 0.5, 1.0 / 6, 1.0 / 6},
                         {1.0 / 6, 1.0 / 6, 0.5, 1.0 / 6},
                         {1.0 / 6, 1.0 / 6, 1.0 / 6, 0.5}};
    for (int qp = 0; qp < 5; ++qp) {
      pts[3 * qp + 0] = bary[qp][1];
      pts[3 * qp + 1] = bary[qp][2];
      pts[3 * qp + 2] = bary[qp][3];
      w[qp] = (qp == 0 ? -4.0 / 5.0 : 9.0 / 20.0) / 6.0;
    }
    return 5;
  }
  if (elem_type == ORC_ANCF3443 || elem_type == ORC_ANCF3243) {
    double x0[8], w0[8], x1[8], w1[8], x2[8], w2[8];
    int n0 = orc_gauss_legendre(gl[0], x0, w0);
    int n1 = orc_gauss_legendre(gl[1], x1, w1);
    int n2 = orc_gauss_legendre(gl[2], x2, w2);
    if (n0 < 0 || n1 < 0 || n2 < 0) return ORC_EINVAL;
    int k = 0;
    for (int i = 0; i < n0; ++i)
      for (int j = 0; j < n1; ++j)
        for (int l = 0; l < n2; ++l) {
          pts[3 * k + 0] = x0[i];
          pts[3 * k + 1] = x1[j];
          pts[3 * k + 2] = x2[l];
          w[k] = w0[i] * w1[j] * w2[l];
          ++k;
        }
    return k;
  }
  return ORC_EINVAL;
}

/* ------------------------------------------------------------------------- */
/* Shape functions (Sec. 4.1: s_i(u_q) and their parent gradients)             */
/* ------------------------------------------------------------------------- */

void orc_t10_shape(const double xi[3], double N[10], double dN[30]) {
  /* quadratic tetrahedron in barycentric coordinates L0 = 1 - xi - eta - zeta,
   * L1 = xi, L2 = eta, L3 = zeta: corner c has N = L_c (2 L_c - 1), the node on
   * edge (c, d) has N = 4 L_c L_d. */
  static const int edges[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
  double L[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
  double dL[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int c = 0; c < 4; ++c) {
    N[c] = L[c] * (2.0 * L[c] - 1.0);
    for (int m = 0; m < 3; ++m) dN[3 * c + m] = (4.0 * L[c] - 1.0) * dL[c][m];
  }
  for (int k = 0; k < 6; ++k) {
    int c = edges[k][0], d = edges[k][1];
    N[4 + k] = 4.0 * L[c] * L[d];
    for (int m = 0; m < 3; ++m) dN[3 * (4 + k) + m] = 4.0 * (L[c] * dL[d][m] + L[d] * dL[c][m]);
  }
}

/* in-plane ANCF3443 basis: the 12-term incomplete bicubic polynomial space */
static const int ancf_pow[12][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2},
                                    {3, 0}, {2, 1}, {1, 2}, {0, 3}, {3, 1}, {1, 3}};
static const double ancf_corner[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};

static double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

/* value and parent derivatives of monomial k at (s, t) */
static void monomial(int k, double s, double t, double* v, double* ds, double* dt) {
  int a = ancf_pow[k][0], b = ancf_pow[k][1];
  *v = ipow(s, a) * ipow(t, b);
  *ds = a > 0 ? a * ipow(s, a - 1) * ipow(t, b) : 0.0;
  *dt = b > 0 ? b * ipow(s, a) * ipow(t, b - 1) : 0.0;
}

/* Gauss-Jordan inverse with partial pivoting, n <= 12 */
static int invert(int n, double* A, double* R) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) R[i * n + j] = kron(i, j);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return ORC_EDEGENERATE;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        double t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t;
        t = R[c * n + j]; R[c * n + j] = R[piv * n + j]; R[piv * n + j] = t;
      }
    double d = A[c * n + c];
    for (int j = 0; j < n; ++j) { A[c * n + j] /= d; R[c * n + j] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[c * n + j]; R[r * n + j] -= f * R[c * n + j]; }
    }
  }
  return ORC_OK;
}

int orc_ancf3443_shape(const double xi[3], double lx, double ly, double H, double S[16],
                       double dS[48]) {
  /* ANCF3443 shell (4 nodes x {r, r_x, r_y, r_z}).  The paper takes the element
   * from Part I / Yamashita et al. without printing its shape functions; this
   * reading fixes them by their defining interpolation conditions: for each
   * corner p the three in-plane functions (for r, r_x, r_y) lie in the 12-term
   * incomplete bicubic space and interpolate value, d/dx and d/dy at the four
   * corners, with x = lx xi / 2 and y = ly eta / 2; the transverse function is
   * z * (1 + xi_p xi)(1 + eta_p eta) / 4 with z = H zeta / 2. */
  double V[144], Vinv[144];
  for (int p = 0; p < 4; ++p)
    for (int k = 0; k < 12; ++k) {
      double v, ds, dt;
      monomial(k, ancf_corner[p][0], ancf_corner[p][1], &v, &ds, &dt);
      V[(3 * p + 0) * 12 + k] = v;
      V[(3 * p + 1) * 12 + k] = ds * 2.0 / lx;
      V[(3 * p + 2) * 12 + k] = dt * 2.0 / ly;
    }
  if (invert(12, V, Vinv) != ORC_OK) return ORC_EDEGENERATE;
  /* function r has coefficients C[r][k] with C V^T = I, i.e. C = (V^-1)^T */
  double s = xi[0], t = xi[1], zeta = xi[2];
  double mv[12], ms[12], mt[12];
  for (int k = 0; k < 12; ++k) monomial(k, s, t, &mv[k], &ms[k], &mt[k]);
  for (int p = 0; p < 4; ++p) {
    for (int kind = 0; kind < 3; ++kind) {
      int r = 3 * p + kind;
      double v = 0, ds = 0, dt = 0;
      for (int k = 0; k < 12; ++k) {
        double c = Vinv[k * 12 + r];
        v += c * mv[k];
        ds += c * ms[k];
        dt += c * mt[k];
      }
      S[4 * p + kind] = v;
      dS[3 * (4 * p + kind) + 0] = ds;
      dS[3 * (4 * p + kind) + 1] = dt;
      dS[3 * (4 * p + kind) + 2] = 0.0;
    }
    double sp = ancf_corner[p][0], tp = ancf_corner[p][1];
    double b = 0.25 * (1.0 + sp * s) * (1.0 + tp * t);
    double z = 0.5 * H * zeta;
    S[4 * p + 3] = z * b;
    dS[3 * (4 * p + 3) + 0] = z * 0.25 * sp * (1.0 + tp * t);
    dS[3 * (4 * p + 3) + 1] = z * 0.25 * tp * (1.0 + sp * s);
    dS[3 * (4 * p + 3) + 2] = 0.5 * H * b;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Constitutive law (Sec. 4.3, Stage 1: P = P_el(F) + P_vis(F, Fdot))          */
/* ------------------------------------------------------------------------- */

/* SVK Lame constants from (E, nu) */
static void lame(double E, double nu, double* lam, double* mu) {
  *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  *mu = E / (2.0 * (1.0 + nu));
}

/* internal parametrisation: SVK by (lambda, mu); MR by (mu10, mu01, kappa) */
typedef struct {
  int kind;
  double c0, c1, c2;   /* SVK: lambda, mu, -; MR: mu10, mu01, kappa */
  double eta, lam_v;
} mat_int;

static mat_int to_internal(const orc_material* m) {
  mat_int r;
  r.kind = m->kind;
  if (m->kind == ORC_SVK) {
    lame(m->p[0], m->p[1], &r.c0, &r.c1);
    r.c2 = 0.0;
  } else {
    r.c0 = m->p[0]; r.c1 = m->p[1]; r.c2 = m->p[2];
  }
  r.eta = m->eta;
  r.lam_v = m->lam_v;
  return r;
}

/* J - 1 = det(I + Hd) - 1 via the invariants of Hd (no cancellation near J=1) */
static double det_minus_one(const double* H) {
  double tr = H[0] + H[4] + H[8];
  double trH2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trH2 += H[3 * i + j] * H[3 * j + i];
  return tr + 0.5 * (tr * tr - trH2) + det3(H);
}

typedef struct {
  double F[9], C[9], B[9], G[9], FC[9];
  double J, Jm1, I1, I2;
} kin;

static void kinematics(const double* Hd, kin* k) {
  for (int i = 0; i < 9; ++i) k->F[i] = Hd[i] + ((i % 4) == 0 ? 1.0 : 0.0);
  const double* F = k->F;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double c = 0, b = 0;
      for (int m = 0; m < 3; ++m) {
        c += F[3 * m + i] * F[3 * m + j];
        b += F[3 * i + m] * F[3 * j + m];
      }
      k->C[3 * i + j] = c;
      k->B[3 * i + j] = b;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += F[3 * i + m] * k->C[3 * m + j];
      k->FC[3 * i + j] = s;
    }
  k->Jm1 = det_minus_one(Hd);
  k->J = 1.0 + k->Jm1;
  double Finv[9];
  inv3(F, Finv);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) k->G[3 * i + j] = Finv[3 * j + i]; /* G = F^-T */
  k->I1 = k->C[0] + k->C[4] + k->C[8];
  double trC2 = 0;
  for (int i = 0; i < 9; ++i) trC2 += k->C[i] * k->C[i];
  k->I2 = 0.5 * (k->I1 * k->I1 - trC2);
}

static double energy_int(const mat_int* m, const double* Hd) {
  kin k;
  kinematics(Hd, &k);
  if (m->kind == ORC_SVK) {
    /* W = lambda/2 tr(E)^2 + mu E:E with E = (Hd + Hd^T + Hd^T Hd) / 2 */
    double E[9], trE = 0, EE = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = Hd[3 * i + j] + Hd[3 * j + i];
        for (int m2 = 0; m2 < 3; ++m2) s += Hd[3 * m2 + i] * Hd[3 * m2 + j];
        E[3 * i + j] = 0.5 * s;
      }
    for (int i = 0; i < 3; ++i) trE += E[4 * i];
    for (int i = 0; i < 9; ++i) EE += E[i] * E[i];
    return 0.5 * m->c0 * trE * trE + m->c1 * EE;
  }
  double a = pow(k.J, -2.0 / 3.0), b = pow(k.J, -4.0 / 3.0);
  return m->c0 * (a * k.I1 - 3.0) + m->c1 * (b * k.I2 - 3.0) + 0.5 * m->c2 * k.Jm1 * k.Jm1;
}

double orc_energy_density(const orc_material* m, const double Hd[9]) {
  mat_int mi = to_internal(m);
  return energy_int(&mi, Hd);
}

static void pk1_int(const mat_int* m, const double* Hd, const double* Fd, double* P) {
  kin k;
  kinematics(Hd, &k);
  const double* F = k.F;
  for (int i = 0; i < 9; ++i) P[i] = 0.0;
  /* Green strain E = (C - I) / 2 = (Hd + Hd^T + Hd^T Hd) / 2: of the size of the
   * strain, with no rounded O(1) term left in it when Hd itself is small */
  double E[9], S[9], trE = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = Hd[3 * i + j] + Hd[3 * j + i];
      for (int m2 = 0; m2 < 3; ++m2) s += Hd[3 * m2 + i] * Hd[3 * m2 + j];
      E[3 * i + j] = 0.5 * s;
    }
  for (int i = 0; i < 3; ++i) trE += E[4 * i];
  if (m->kind == ORC_SVK) {
    /* S = lambda tr(E) I + 2 mu E, P = F S */
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[3 * i + j] = m->c0 * trE * kron(i, j) + 2.0 * m->c1 * E[3 * i + j];
  } else {
    /* S = 2 dW/dC = 2 mu10 J^-2/3 (I - I1/3 C^-1) + 2 mu01 J^-4/3 (I1 I - C - 2/3 I2 C^-1)
     *     + kappa J (J - 1) C^-1.
     * With C = I + 2E the two brackets are C^-1 times
     *   C - I1/3 I = 2 dev(E)   and
     *   I1 C - C^2 - 2/3 I2 I = 2 dev(E) + 4 tr(E) E - 4 E^2 + 4/3 (E:E - tr(E)^2) I,
     * so S is formed from E alone, without the difference of O(1) numbers that
     * the first form takes at small strain. */
    double a = pow(k.J, -2.0 / 3.0), b = pow(k.J, -4.0 / 3.0);
    double EE[9], ee = 0.0, T[9], C[9], Ci[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int m2 = 0; m2 < 3; ++m2) s += E[3 * i + m2] * E[3 * m2 + j];
        EE[3 * i + j] = s;
        ee += E[3 * i + j] * E[3 * i + j];
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double dev = E[3 * i + j] - trE / 3.0 * kron(i, j);
        double b1 = 2.0 * dev;
        double b2 = 2.0 * dev + 4.0 * trE * E[3 * i + j] - 4.0 * EE[3 * i + j] +
                    4.0 / 3.0 * (ee - trE * trE) * kron(i, j);
        T[3 * i + j] = 2.0 * m->c0 * a * b1 + 2.0 * m->c1 * b * b2 + m->c2 * k.J * k.Jm1 * kron(i, j);
        C[3 * i + j] = kron(i, j) + 2.0 * E[3 * i + j];
      }
    inv3(C, Ci);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int m2 = 0; m2 < 3; ++m2) s += Ci[3 * i + m2] * T[3 * m2 + j];
        S[3 * i + j] = s;
      }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int m2 = 0; m2 < 3; ++m2) P[3 * i + j] += F[3 * i + m2] * S[3 * m2 + j];
  if (m->eta != 0.0 || m->lam_v != 0.0) {
    /* Edot = (Fdot^T F + F^T Fdot) / 2, S_v = 2 eta Edot + lam_v tr(Edot) I, P_v = F S_v */
    double Ed[9], Sv[9], trEd = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int m2 = 0; m2 < 3; ++m2) s += Fd[3 * m2 + i] * F[3 * m2 + j] + F[3 * m2 + i] * Fd[3 * m2 + j];
        Ed[3 * i + j] = 0.5 * s;
      }
    for (int i = 0; i < 3; ++i) trEd += Ed[4 * i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Sv[3 * i + j] = 2.0 * m->eta * Ed[3 * i + j] + m->lam_v * trEd * kron(i, j);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int m2 = 0; m2 < 3; ++m2) P[3 * i + j] += F[3 * i + m2] * Sv[3 * m2 + j];
  }
}

void orc_pk1(const orc_material* m, const double Hd[9], const double Fdot[9], double P[9]) {
  mat_int mi = to_internal(m);
  pk1_int(&mi, Hd, Fdot, P);
}

#define A4(i, J, k, L) A[27 * (i) + 9 * (J) + 3 * (k) + (L)]

/* A = alpha dP/dF + beta dP/dFdot, A[i][J][k][L] = d P_iJ / d F_kL */
static void tangent_int(const mat_int* m, const double* Hd, const double* Fd, double alpha,
                        double beta, double* A) {
  kin k;
  kinematics(Hd, &k);
  const double *F = k.F, *G = k.G, *C = k.C, *B = k.B, *FC = k.FC;
  double S[9];
  memset(A, 0, 81 * sizeof(double));
  if (m->kind == ORC_SVK) {
    double E[9], trE = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = Hd[3 * i + j] + Hd[3 * j + i];
        for (int m2 = 0; m2 < 3; ++m2) s += Hd[3 * m2 + i] * Hd[3 * m2 + j];
        E[3 * i + j] = 0.5 * s;
      }
    for (int i = 0; i < 3; ++i) trE += E[4 * i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[3 * i + j] = m->c0 * trE * kron(i, j) + 2.0 * m->c1 * E[3 * i + j];
    /* dP/dF = d_ik S_JL + lambda F_iJ F_kL + mu (F_iL F_kJ + (F F^T)_ik d_JL) */
    for (int i = 0; i < 3; ++i)
      for (int J = 0; J < 3; ++J)
        for (int kk = 0; kk < 3; ++kk)
          for (int L = 0; L < 3; ++L)
            A4(i, J, kk, L) += alpha * (kron(i, kk) * S[3 * J + L] + m->c0 * F[3 * i + J] * F[3 * kk + L] +
                                        m->c1 * (F[3 * i + L] * F[3 * kk + J] + B[3 * i + kk] * kron(J, L)));
  } else {
    double a = pow(k.J, -2.0 / 3.0), b = pow(k.J, -4.0 / 3.0);
    double I1 = k.I1, I2 = k.I2, J = k.J, Jm1 = k.Jm1;
    double mu10 = m->c0, mu01 = m->c1, kap = m->c2;
    for (int i = 0; i < 3; ++i)
      for (int JJ = 0; JJ < 3; ++JJ)
        for (int kk = 0; kk < 3; ++kk)
          for (int L = 0; L < 3; ++L) {
            double dikJL = kron(i, kk) * kron(JJ, L);
            double FiJ = F[3 * i + JJ], FkL = F[3 * kk + L], GiJ = G[3 * i + JJ], GkL = G[3 * kk + L];
            double GiL = G[3 * i + L], GkJ = G[3 * kk + JJ];
            /* d/dF of 2 mu10 J^-2/3 (F - I1/3 G) */
            double t1 = 2.0 * mu10 * a *
                        (dikJL - 2.0 / 3.0 * (FiJ * GkL + GiJ * FkL) + 2.0 / 9.0 * I1 * GiJ * GkL +
                         I1 / 3.0 * GiL * GkJ);
            /* d/dF of 2 mu01 J^-4/3 (I1 F - F C - 2/3 I2 G) */
            double Q = I1 * FiJ - FC[3 * i + JJ] - 2.0 / 3.0 * I2 * GiJ;
            double dQ = 2.0 * FkL * FiJ + I1 * dikJL -
                        (kron(i, kk) * C[3 * L + JJ] + F[3 * i + L] * F[3 * kk + JJ] + B[3 * i + kk] * kron(JJ, L)) -
                        4.0 / 3.0 * (I1 * FkL - FC[3 * kk + L]) * GiJ + 2.0 / 3.0 * I2 * GiL * GkJ;
            double t2 = 2.0 * mu01 * b * (-4.0 / 3.0 * GkL * Q + dQ);
            /* d/dF of kappa J (J - 1) G */
            double t3 = kap * J * (2.0 * J - 1.0) * GiJ * GkL - kap * J * Jm1 * GiL * GkJ;
            A4(i, JJ, kk, L) += alpha * (t1 + t2 + t3);
          }
  }
  if (m->eta != 0.0 || m->lam_v != 0.0) {
    double Ed[9], Sv[9], trEd = 0, FFd[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0, t = 0;
        for (int m2 = 0; m2 < 3; ++m2) {
          s += Fd[3 * m2 + i] * F[3 * m2 + j] + F[3 * m2 + i] * Fd[3 * m2 + j];
          t += F[3 * i + m2] * Fd[3 * j + m2];
        }
        Ed[3 * i + j] = 0.5 * s;
        FFd[3 * i + j] = t; /* F Fdot^T */
      }
    for (int i = 0; i < 3; ++i) trEd += Ed[4 * i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Sv[3 * i + j] = 2.0 * m->eta * Ed[3 * i + j] + m->lam_v * trEd * kron(i, j);
    for (int i = 0; i < 3; ++i)
      for (int J = 0; J < 3; ++J)
        for (int kk = 0; kk < 3; ++kk)
          for (int L = 0; L < 3; ++L) {
            /* dP_v/dF = d_ik S_v,JL + eta ((F Fdot^T)_ik d_JL + F_iL Fdot_kJ) + lam_v F_iJ Fdot_kL */
            double dF = kron(i, kk) * Sv[3 * J + L] +
                        m->eta * (FFd[3 * i + kk] * kron(J, L) + F[3 * i + L] * Fd[3 * kk + J]) +
                        m->lam_v * F[3 * i + J] * Fd[3 * kk + L];
            /* dP_v/dFdot = eta (F_iL F_kJ + (F F^T)_ik d_JL) + lam_v F_iJ F_kL */
            double dFd = m->eta * (F[3 * i + L] * F[3 * kk + J] + B[3 * i + kk] * kron(J, L)) +
                         m->lam_v * F[3 * i + J] * F[3 * kk + L];
            A4(i, J, kk, L) += alpha * dF + beta * dFd;
          }
  }
}

void orc_tangent(const orc_material* m, const double Hd[9], const double Fdot[9], double alpha,
                 double beta, double A[81]) {
  mat_int mi = to_internal(m);
  tangent_int(&mi, Hd, Fdot, alpha, beta, A);
}

/* ------------------------------------------------------------------------- */
/* Element geometry and kinematics (Sec. 4.1; Sec. 4.3, Eq. F_assembly)        */
/* ------------------------------------------------------------------------- */

int orc_n_en(int elem_type) {
  return elem_type == ORC_T10 ? 10 : (elem_type == ORC_ANCF3443 ? 16 : (elem_type == ORC_ANCF3243 ? 8 : 0));
}

/* physical nodes per element (T10: 10, ANCF3443: 4, ANCF3243: 2) */
static int nodes_per_elem(const orc_mesh* m) {
  return m->elem_type == ORC_T10 ? 10 : (m->elem_type == ORC_ANCF3243 ? 2 : 4);
}

/* ANCF3243 beam (two nodes, coefficients r, r_x, r_y, r_z each): with
 * xi = (1 + u)/2 along the axis (x = L xi), y = W v / 2, z = H w / 2,
 *   node 0:  1 - 3 xi^2 + 2 xi^3,  L (xi - 2 xi^2 + xi^3),  y (1 - xi),  z (1 - xi)
 *   node 1:  3 xi^2 - 2 xi^3,      L (xi^3 - xi^2),          y xi,        z xi
 * (cubic Hermite interpolation of position and axial slope, linear
 * interpolation of the cross-section gradients).  dS: parent gradients d/du,
 * d/dv, d/dw. */
int orc_ancf3243_shape(const double xi3[3], double L, double W, double H, double S[8], double dS[24]) {
  if (!(L > 0.0) || !(W > 0.0) || !(H > 0.0)) return ORC_EINVAL;
  const double t = 0.5 * (1.0 + xi3[0]), y = 0.5 * W * xi3[1], z = 0.5 * H * xi3[2];
  const double dt = 0.5, dy = 0.5 * W, dz = 0.5 * H;  /* d xi/du, dy/dv, dz/dw */
  S[0] = 1.0 - 3.0 * t * t + 2.0 * t * t * t;
  S[1] = L * (t - 2.0 * t * t + t * t * t);
  S[2] = y * (1.0 - t);
  S[3] = z * (1.0 - t);
  S[4] = 3.0 * t * t - 2.0 * t * t * t;
  S[5] = L * (t * t * t - t * t);
  S[6] = y * t;
  S[7] = z * t;
  const double dSdt[8] = {-6.0 * t + 6.0 * t * t, L * (1.0 - 4.0 * t + 3.0 * t * t), -y, -z,
                          6.0 * t - 6.0 * t * t, L * (3.0 * t * t - 2.0 * t), y, z};
  const double dSdy[8] = {0, 0, 1.0 - t, 0, 0, 0, t, 0};
  const double dSdz[8] = {0, 0, 0, 1.0 - t, 0, 0, 0, t};
  for (int a = 0; a < 8; ++a) {
    dS[3 * a + 0] = dSdt[a] * dt;
    dS[3 * a + 1] = dSdy[a] * dy;
    dS[3 * a + 2] = dSdz[a] * dz;
  }
  return ORC_OK;
}

int orc_n_qp(const orc_mesh* mesh) {
  if (mesh->elem_type == ORC_T10) return 5;
  return mesh->gl[0] * mesh->gl[1] * mesh->gl[2];
}

/* global coefficient of local shape function a of element e */
static int coef_of(const orc_mesh* mesh, int e, int a) {
  if (mesh->elem_type == ORC_T10) return mesh->conn[10 * e + a];
  const int npn = nodes_per_elem(mesh);
  return 4 * mesh->conn[npn * e + a / 4] + a % 4;
}

/* 1 if local shape function a carries a position (value) coefficient: every
 * T10 node, and coefficient k = 0 of each ANCF node */
static int is_position(const orc_mesh* mesh, int a) {
  return mesh->elem_type == ORC_T10 ? 1 : (a % 4 == 0);
}

/* parent gradients of all shape functions at qp; returns n_en */
static int parent_gradients(const orc_mesh* mesh, int e, const double* xi, double* dN) {
  if (mesh->elem_type == ORC_T10) {
    double N[10];
    orc_t10_shape(xi, N, dN);
    return 10;
  }
  if (mesh->elem_type == ORC_ANCF3243) {
    const double* X = mesh->X;
    int n0 = mesh->conn[2 * e], n1 = mesh->conn[2 * e + 1];
    double L = 0;
    for (int d = 0; d < 3; ++d) {
      double a = X[3 * (4 * n1) + d] - X[3 * (4 * n0) + d];
      L += a * a;
    }
    double S[8];
    if (orc_ancf3243_shape(xi, sqrt(L), mesh->width, mesh->thickness, S, dN) != ORC_OK) return -1;
    return 8;
  }
  /* element in-plane sizes from the reference positions of its corners */
  const double* X = mesh->X;
  int n0 = mesh->conn[4 * e], n1 = mesh->conn[4 * e + 1], n3 = mesh->conn[4 * e + 3];
  double lx = 0, ly = 0;
  for (int d = 0; d < 3; ++d) {
    double a = X[3 * (4 * n1) + d] - X[3 * (4 * n0) + d];
    double b = X[3 * (4 * n3) + d] - X[3 * (4 * n0) + d];
    lx += a * a;
    ly += b * b;
  }
  double S[16];
  if (orc_ancf3443_shape(xi, sqrt(lx), sqrt(ly), mesh->thickness, S, dN) != ORC_OK) return -1;
  return 16;
}

/* dV and physical gradients g[a][J] = sum_m Jinv[m][J] dN[a][m] at one qp */
static int qp_geometry(const orc_mesh* mesh, int e, const double* xi, double wq, double* dV,
                       double* g) {
  double dN[48];
  int nen = parent_gradients(mesh, e, xi, dN);
  if (nen < 0) return ORC_EDEGENERATE;
  /* J0 = sum_a X_a (x) dN_a, with the first position coefficient taken out of
   * every position coefficient (their parent gradients sum to zero): the same
   * sum, with terms of the element's size however far it lies from the origin */
  double J0[9] = {0};
  const double* X0 = mesh->X + 3 * coef_of(mesh, e, 0);
  for (int a = 0; a < nen; ++a) {
    const double* Xa = mesh->X + 3 * coef_of(mesh, e, a);
    const int pos = is_position(mesh, a);
    for (int i = 0; i < 3; ++i) {
      const double xa = Xa[i] - (pos ? X0[i] : 0.0);
      for (int m = 0; m < 3; ++m) J0[3 * i + m] += xa * dN[3 * a + m];
    }
  }
  double Jinv[9];
  double det = inv3(J0, Jinv);
  if (!(det > 0.0)) return ORC_EDEGENERATE;
  for (int a = 0; a < nen; ++a)
    for (int J = 0; J < 3; ++J) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += Jinv[3 * m + J] * dN[3 * a + m];
      g[3 * a + J] = s;
    }
  *dV = det * wq;
  return ORC_OK;
}

int orc_element_geometry(const orc_mesh* mesh, int e, double* dV, double* g) {
  double pts[3 * 128], w[128];
  int nq = orc_quadrature(mesh->elem_type, mesh->gl, pts, w);
  if (nq < 0) return nq;
  int nen = orc_n_en(mesh->elem_type);
  for (int qp = 0; qp < nq; ++qp) {
    int rc = qp_geometry(mesh, e, pts + 3 * qp, w[qp], dV + qp, g + 3 * nen * qp);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

/* element force and stiffness with an internal material (accumulates) */
static int element_int(const orc_mesh* mesh, const mat_int* mat, int e, const double* q,
                       const double* qdot, double alpha, double beta, double* fe, double* Ke) {
  double pts[3 * 128], w[128];
  int nq = orc_quadrature(mesh->elem_type, mesh->gl, pts, w);
  if (nq < 0) return nq;
  int nen = orc_n_en(mesh->elem_type);
  int nd = 3 * nen;
  double g[48], A[81], P[9];
  for (int qp = 0; qp < nq; ++qp) {
    double dV;
    int rc = qp_geometry(mesh, e, pts + 3 * qp, w[qp], &dV, g);
    if (rc != ORC_OK) return rc;
    /* Hd = sum_a (x_a - X_a) (x) g_a, Fdot = sum_a xdot_a (x) g_a.  The
     * position shape functions sum to one, so their gradients sum to zero:
     * taking the displacement and velocity of the element's first position
     * coefficient out of every position coefficient leaves both sums unchanged,
     * and keeps their terms of the size of the element's own deformation under
     * a large rigid motion (otherwise |x - X| / h digits are lost). */
    double Hd[9] = {0}, Fd[9] = {0}, u0[3], v0[3];
    const int c0 = coef_of(mesh, e, 0);
    for (int i = 0; i < 3; ++i) {
      u0[i] = q[3 * c0 + i] - mesh->X[3 * c0 + i];
      v0[i] = qdot ? qdot[3 * c0 + i] : 0.0;
    }
    for (int a = 0; a < nen; ++a) {
      int c = coef_of(mesh, e, a);
      const int pos = is_position(mesh, a);
      for (int i = 0; i < 3; ++i) {
        double u = q[3 * c + i] - mesh->X[3 * c + i] - (pos ? u0[i] : 0.0);
        double v = (qdot ? qdot[3 * c + i] : 0.0) - (pos ? v0[i] : 0.0);
        for (int J = 0; J < 3; ++J) {
          Hd[3 * i + J] += u * g[3 * a + J];
          Fd[3 * i + J] += v * g[3 * a + J];
        }
      }
    }
    if (fe) {
      pk1_int(mat, Hd, Fd, P);
      /* Eq. fint_local: f_a += P g_a J0 w_q */
      for (int a = 0; a < nen; ++a)
        for (int i = 0; i < 3; ++i) {
          double s = 0;
          for (int J = 0; J < 3; ++J) s += P[3 * i + J] * g[3 * a + J];
          fe[3 * a + i] += s * dV;
        }
    }
    if (Ke) {
      tangent_int(mat, Hd, Fd, alpha, beta, A);
      /* Eq. tangent_block: [K_ab]_ik += A_iJkL g_aJ g_bL J0 w_q */
      for (int a = 0; a < nen; ++a)
        for (int i = 0; i < 3; ++i)
          for (int b = 0; b < nen; ++b)
            for (int kk = 0; kk < 3; ++kk) {
              double s = 0;
              for (int J = 0; J < 3; ++J)
                for (int L = 0; L < 3; ++L) s += A4(i, J, kk, L) * g[3 * a + J] * g[3 * b + L];
              Ke[(3 * a + i) * nd + 3 * b + kk] += s * dV;
            }
    }
  }
  return ORC_OK;
}

int orc_element(const orc_mesh* mesh, const orc_material* mat, int e, const double* q,
                const double* qdot, double alpha, double beta, double* fe, double* Ke) {
  int nd = 3 * orc_n_en(mesh->elem_type);
  if (nd == 0 || e < 0 || e >= mesh->n_elem) return ORC_EINVAL;
  if (fe) memset(fe, 0, nd * sizeof(double));
  if (Ke) memset(Ke, 0, (size_t)nd * nd * sizeof(double));
  mat_int mi = to_internal(mat);
  return element_int(mesh, &mi, e, q, qdot, alpha, beta, fe, Ke);
}

/* ------------------------------------------------------------------------- */
/* CSR pattern (Sec. 4.2; Sec. 4.4.2: coefficient adjacency from connectivity, */
/* each adjacent pair a 3x3 block, DOF = 3 coef + d)                           */
/* ------------------------------------------------------------------------- */

static int cmp_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

/* nodes shared by elements: T10 node = coefficient; ANCF physical node holds 4 */
static int pattern_nodes_per_elem(const orc_mesh* m) { return nodes_per_elem(m); }
static int coefs_per_pattern_node(const orc_mesh* m) { return m->elem_type == ORC_T10 ? 1 : 4; }

long long orc_csr_build(const orc_mesh* mesh, int* row_off, int* cols) {
  int npe = pattern_nodes_per_elem(mesh), mc = coefs_per_pattern_node(mesh);
  int nn = mesh->n_coef / mc;
  /* incidence lists node -> elements */
  int* cnt = (int*)calloc((size_t)nn + 1, sizeof(int));
  for (long long i = 0; i < (long long)mesh->n_elem * npe; ++i) {
    int n = mesh->conn[i];
    if (n < 0 || n >= nn) { free(cnt); return ORC_EINVAL; }
    cnt[n + 1]++;
  }
  for (int i = 0; i < nn; ++i) cnt[i + 1] += cnt[i];
  int* inc = (int*)malloc(sizeof(int) * (size_t)(cnt[nn] > 0 ? cnt[nn] : 1));
  int* fill = (int*)calloc((size_t)nn, sizeof(int));
  for (int e = 0; e < mesh->n_elem; ++e)
    for (int a = 0; a < npe; ++a) {
      int n = mesh->conn[(long long)e * npe + a];
      inc[cnt[n] + fill[n]++] = e;
    }
  /* adjacency of every node: sorted unique nodes of its incident elements */
  long long nnz = 0;
  int* buf = NULL;
  size_t cap = 0;
  if (row_off) row_off[0] = 0;
  for (int I = 0; I < nn; ++I) {
    size_t need = (size_t)(cnt[I + 1] - cnt[I]) * npe;
    if (need > cap) { cap = need; buf = (int*)realloc(buf, cap * sizeof(int)); }
    size_t k = 0;
    for (int t = cnt[I]; t < cnt[I + 1]; ++t)
      for (int a = 0; a < npe; ++a) buf[k++] = mesh->conn[(long long)inc[t] * npe + a];
    qsort(buf, k, sizeof(int), cmp_int);
    size_t u = 0;
    for (size_t t = 0; t < k; ++t)
      if (u == 0 || buf[t] != buf[u - 1]) buf[u++] = buf[t];
    long long rowlen = 3LL * mc * (long long)u;
    for (int c = 0; c < mc; ++c)
      for (int i = 0; i < 3; ++i) {
        long long r = 3LL * ((long long)mc * I + c) + i;
        if (row_off) {
          long long pos = nnz;
          for (size_t t = 0; t < u; ++t)
            for (int c2 = 0; c2 < mc; ++c2)
              for (int kk = 0; kk < 3; ++kk) cols[pos++] = 3 * (mc * buf[t] + c2) + kk;
          row_off[r + 1] = (int)(nnz + rowlen);
        }
        nnz += rowlen;
      }
  }
  free(buf);
  free(fill);
  free(inc);
  free(cnt);
  return nnz;
}

static long long find_col(const int* row_off, const int* cols, int r, int c) {
  int lo = row_off[r], hi = row_off[r + 1] - 1;
  while (lo <= hi) {
    int mid = lo + (hi - lo) / 2;
    if (cols[mid] == c) return mid;
    if (cols[mid] < c) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int orc_assemble(const orc_mesh* mesh, const orc_material* mat, const double* q,
                 const double* qdot, double alpha, double beta, const int* elems, int n_list,
                 double* f, const int* row_off, const int* cols, double* vals) {
  int nen = orc_n_en(mesh->elem_type);
  int nd = 3 * nen;
  mat_int mi = to_internal(mat);
  double* fe = (double*)malloc(sizeof(double) * nd);
  double* Ke = vals ? (double*)malloc(sizeof(double) * nd * nd) : NULL;
  int n = elems ? n_list : mesh->n_elem;
  int rc = ORC_OK;
  for (int t = 0; t < n && rc == ORC_OK; ++t) {
    int e = elems ? elems[t] : t;
    memset(fe, 0, sizeof(double) * nd);
    if (Ke) memset(Ke, 0, sizeof(double) * nd * nd);
    rc = element_int(mesh, &mi, e, q, qdot, alpha, beta, f ? fe : NULL, Ke);
    if (rc != ORC_OK) break;
    for (int a = 0; a < nen; ++a) {
      int ca = coef_of(mesh, e, a);
      for (int i = 0; i < 3; ++i) {
        if (f) f[3 * ca + i] += fe[3 * a + i];
        if (!Ke) continue;
        for (int b = 0; b < nen; ++b) {
          int cb = coef_of(mesh, e, b);
          for (int kk = 0; kk < 3; ++kk) {
            long long pos = find_col(row_off, cols, 3 * ca + i, 3 * cb + kk);
            if (pos < 0) { rc = ORC_ENOTFOUND; break; }
            vals[pos] += Ke[(3 * a + i) * nd + 3 * b + kk];
          }
        }
      }
    }
  }
  free(fe);
  free(Ke);
  return rc;
}

int orc_slot_map(const orc_mesh* mesh, const int* row_off, const int* cols, int e0, int ne,
                 int* slots) {
  int nen = orc_n_en(mesh->elem_type), nd = 3 * nen;
  for (int e = e0; e < e0 + ne; ++e)
    for (int a = 0; a < nen; ++a)
      for (int i = 0; i < 3; ++i)
        for (int b = 0; b < nen; ++b)
          for (int kk = 0; kk < 3; ++kk) {
            long long pos = find_col(row_off, cols, 3 * coef_of(mesh, e, a) + i, 3 * coef_of(mesh, e, b) + kk);
            if (pos < 0) return ORC_ENOTFOUND;
            slots[(long long)(e - e0) * nd * nd + (3 * a + i) * nd + 3 * b + kk] = (int)pos;
          }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Vector-Jacobian products and energy                                          */
/* ------------------------------------------------------------------------- */

/* w . f over all elements for one internal material (P linear in its constants) */
static double w_dot_f(const orc_mesh* mesh, const mat_int* m, const double* q, const double* qdot,
                      const double* w) {
  int nen = orc_n_en(mesh->elem_type);
  double fe[48], s = 0;
  for (int e = 0; e < mesh->n_elem; ++e) {
    memset(fe, 0, sizeof(fe));
    if (element_int(mesh, m, e, q, qdot, 1.0, 0.0, fe, NULL) != ORC_OK) return NAN;
    for (int a = 0; a < nen; ++a) {
      int c = coef_of(mesh, e, a);
      for (int i = 0; i < 3; ++i) s += w[3 * c + i] * fe[3 * a + i];
    }
  }
  return s;
}

int orc_vjp(const orc_mesh* mesh, const orc_material* mat, const double* q, const double* qdot,
            const double* w, double* gq, double* gqdot, double* gparams) {
  int nen = orc_n_en(mesh->elem_type), nd = 3 * nen;
  mat_int mi = to_internal(mat);
  double* Ke = (double*)malloc(sizeof(double) * nd * nd);
  for (int e = 0; e < mesh->n_elem; ++e) {
    for (int pass = 0; pass < 2; ++pass) {
      double* out = pass == 0 ? gq : gqdot;
      if (!out) continue;
      memset(Ke, 0, sizeof(double) * nd * nd);
      int rc = element_int(mesh, &mi, e, q, qdot, pass == 0 ? 1.0 : 0.0, pass == 0 ? 0.0 : 1.0, NULL, Ke);
      if (rc != ORC_OK) { free(Ke); return rc; }
      /* out_b,k += sum_{a,i} K[(a,i),(b,k)] w_a,i  (transpose product) */
      for (int b = 0; b < nen; ++b) {
        int cb = coef_of(mesh, e, b);
        for (int kk = 0; kk < 3; ++kk) {
          double s = 0;
          for (int a = 0; a < nen; ++a) {
            int ca = coef_of(mesh, e, a);
            for (int i = 0; i < 3; ++i) s += Ke[(3 * a + i) * nd + 3 * b + kk] * w[3 * ca + i];
          }
          out[3 * cb + kk] += s;
        }
      }
    }
  }
  free(Ke);
  if (gparams) {
    /* f is linear in (lambda, mu) | (mu10, mu01, kappa) and in (eta, lam_v):
     * d(w.f)/d theta_i = w . f(theta = e_i) */
    mat_int u = mi;
    u.c0 = u.c1 = u.c2 = u.eta = u.lam_v = 0.0;
    mat_int m0 = u, m1 = u, m2 = u, me = u, ml = u;
    m0.c0 = 1.0; m1.c1 = 1.0; m2.c2 = 1.0; me.eta = 1.0; ml.lam_v = 1.0;
    double d0 = w_dot_f(mesh, &m0, q, qdot, w);
    double d1 = w_dot_f(mesh, &m1, q, qdot, w);
    double d2 = mat->kind == ORC_MR ? w_dot_f(mesh, &m2, q, qdot, w) : 0.0;
    double de = w_dot_f(mesh, &me, q, qdot, w);
    double dl = w_dot_f(mesh, &ml, q, qdot, w);
    if (mat->kind == ORC_SVK) {
      /* chain rule from (lambda, mu) to (E, nu) */
      double E = mat->p[0], nu = mat->p[1];
      double dlam_dE = nu / ((1 + nu) * (1 - 2 * nu)), dmu_dE = 1.0 / (2 * (1 + nu));
      double dlam_dnu = E * (1 + 2 * nu * nu) / ((1 + nu) * (1 + nu) * (1 - 2 * nu) * (1 - 2 * nu));
      double dmu_dnu = -E / (2 * (1 + nu) * (1 + nu));
      gparams[0] += dlam_dE * d0 + dmu_dE * d1;
      gparams[1] += dlam_dnu * d0 + dmu_dnu * d1;
    } else {
      gparams[0] += d0;
      gparams[1] += d1;
      gparams[2] += d2;
    }
    gparams[3] += de;
    gparams[4] += dl;
  }
  return ORC_OK;
}

double orc_energy(const orc_mesh* mesh, const orc_material* mat, const double* q) {
  double pts[3 * 128], w[128], g[48];
  int nq = orc_quadrature(mesh->elem_type, mesh->gl, pts, w);
  int nen = orc_n_en(mesh->elem_type);
  mat_int mi = to_internal(mat);
  double total = 0;
  for (int e = 0; e < mesh->n_elem; ++e)
    for (int qp = 0; qp < nq; ++qp) {
      double dV;
      if (qp_geometry(mesh, e, pts + 3 * qp, w[qp], &dV, g) != ORC_OK) return NAN;
      /* the displacement gradient as in element_int (first position coefficient taken out) */
      double Hd[9] = {0};
      const int c0 = coef_of(mesh, e, 0);
      for (int a = 0; a < nen; ++a) {
        int c = coef_of(mesh, e, a);
        const int pos = is_position(mesh, a);
        for (int i = 0; i < 3; ++i) {
          const double u = q[3 * c + i] - mesh->X[3 * c + i] - (pos ? q[3 * c0 + i] - mesh->X[3 * c0 + i] : 0.0);
          for (int J = 0; J < 3; ++J) Hd[3 * i + J] += u * g[3 * a + J];
        }
      }
      total += dV * energy_int(&mi, Hd);
    }
  return total;
}

/* ------------------------------------------------------------------------- */
/* Mass, gradient (Sec. 4.1: m_ij = int rho s_i s_j dV, M_e = [m_ij I_3];     */
/* Sec. 4.4.1, Eq. grad_L; Sec. 4.4.2, Eq. hessian)                           */
/* ------------------------------------------------------------------------- */

static long long factorial(int n) {
  long long f = 1;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

/* T10 shape function a as a homogeneous quadratic in the barycentric
 * coordinates (using L0 + L1 + L2 + L3 = 1): N_a = sum_ij Q[i][j] L_i L_j */
static void t10_quadratic(int a, double Q[4][4]) {
  static const int edges[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Q[i][j] = 0.0;
  if (a < 4) {
    /* L_c (2 L_c - 1) = 2 L_c^2 - L_c sum_k L_k */
    for (int k = 0; k < 4; ++k) {
      Q[a][k] -= 0.5;
      Q[k][a] -= 0.5;
    }
    Q[a][a] += 2.0;
  } else {
    int c = edges[a - 4][0], d = edges[a - 4][1];
    Q[c][d] = 2.0;
    Q[d][c] = 2.0;
  }
}

/* consistent element mass (scalar m_ab, n_en x n_en).  T10: exact integral over
 * a straight-sided tetrahedron, int L0^a0 L1^a1 L2^a2 L3^a3 dV = det J0 a0! a1!
 * a2! a3! / (a0+a1+a2+a3+3)!; curved elements are rejected.  ANCF3443: Gauss-
 * Legendre 4 x 4 x 2 in the parent box (exact for the element's polynomial
 * products on an affine reference geometry). */
int orc_element_mass(const orc_mesh* mesh, int e, double rho, double* m) {
  int nen = orc_n_en(mesh->elem_type);
  if (nen == 0) return ORC_EINVAL;
  for (int t = 0; t < nen * nen; ++t) m[t] = 0.0;
  if (mesh->elem_type == ORC_T10) {
    double g[30], det0, det1;
    const double c0[3] = {0.25, 0.25, 0.25}, c1[3] = {0.1, 0.2, 0.3};
    int rc = qp_geometry(mesh, e, c0, 1.0, &det0, g);
    if (rc != ORC_OK) return rc;
    rc = qp_geometry(mesh, e, c1, 1.0, &det1, g);
    if (rc != ORC_OK) return rc;
    if (fabs(det1 - det0) > 1e-12 * fabs(det0)) return ORC_EINVAL;  /* not straight-sided */
    double Q[10][4][4];
    for (int a = 0; a < 10; ++a) t10_quadratic(a, Q[a]);
    for (int a = 0; a < 10; ++a)
      for (int b = 0; b < 10; ++b) {
        double sum = 0.0;
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k)
              for (int l = 0; l < 4; ++l) {
                double c = Q[a][i][j] * Q[b][k][l];
                if (c == 0.0) continue;
                int al[4] = {0, 0, 0, 0};
                al[i]++; al[j]++; al[k]++; al[l]++;
                sum += c * (double)(factorial(al[0]) * factorial(al[1]) * factorial(al[2]) * factorial(al[3])) /
                       (double)factorial(7);
              }
        m[10 * a + b] = rho * det0 * sum;
      }
    return ORC_OK;
  }
  if (mesh->elem_type == ORC_ANCF3243) {
    /* Gauss-Legendre 4 x 2 x 2: exact for the cubic x linear products */
    double x4[4], w4[4], x2[2], w2[2];
    orc_gauss_legendre(4, x4, w4);
    orc_gauss_legendre(2, x2, w2);
    const double* X = mesh->X;
    int n0 = mesh->conn[2 * e], n1 = mesh->conn[2 * e + 1];
    double L = 0;
    for (int d = 0; d < 3; ++d) {
      double a = X[3 * (4 * n1) + d] - X[3 * (4 * n0) + d];
      L += a * a;
    }
    L = sqrt(L);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
          double xi[3] = {x4[i], x2[j], x2[k]}, S[8], dS[24], g[24], dV;
          if (orc_ancf3243_shape(xi, L, mesh->width, mesh->thickness, S, dS) != ORC_OK) return ORC_EDEGENERATE;
          int rc = qp_geometry(mesh, e, xi, w4[i] * w2[j] * w2[k], &dV, g);
          if (rc != ORC_OK) return rc;
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) m[8 * a + b] += rho * S[a] * S[b] * dV;
        }
    return ORC_OK;
  }
  /* ANCF3443 */
  double x4[4], w4[4], x2[2], w2[2];
  orc_gauss_legendre(4, x4, w4);
  orc_gauss_legendre(2, x2, w2);
  const double* X = mesh->X;
  int n0 = mesh->conn[4 * e], n1 = mesh->conn[4 * e + 1], n3 = mesh->conn[4 * e + 3];
  double lx = 0, ly = 0;
  for (int d = 0; d < 3; ++d) {
    double a = X[3 * (4 * n1) + d] - X[3 * (4 * n0) + d];
    double b = X[3 * (4 * n3) + d] - X[3 * (4 * n0) + d];
    lx += a * a;
    ly += b * b;
  }
  lx = sqrt(lx);
  ly = sqrt(ly);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 2; ++k) {
        double xi[3] = {x4[i], x4[j], x2[k]}, S[16], dS[48], g[48], dV;
        if (orc_ancf3443_shape(xi, lx, ly, mesh->thickness, S, dS) != ORC_OK) return ORC_EDEGENERATE;
        int rc = qp_geometry(mesh, e, xi, w4[i] * w4[j] * w2[k], &dV, g);
        if (rc != ORC_OK) return rc;
        for (int a = 0; a < 16; ++a)
          for (int b = 0; b < 16; ++b) m[16 * a + b] += rho * S[a] * S[b] * dV;
      }
  return ORC_OK;
}

/* accumulate (+=) the DOF-level mass M_e = [m_ab I_3] of every element into
 * CSR values on the mesh pattern (off-diagonal entries of a 3x3 block get 0) */
int orc_mass_assemble(const orc_mesh* mesh, double rho, const int* row_off, const int* cols,
                      double* vals) {
  int nen = orc_n_en(mesh->elem_type);
  double* m = (double*)malloc(sizeof(double) * nen * nen);
  int rc = ORC_OK;
  for (int e = 0; e < mesh->n_elem && rc == ORC_OK; ++e) {
    rc = orc_element_mass(mesh, e, rho, m);
    if (rc != ORC_OK) break;
    for (int a = 0; a < nen; ++a)
      for (int b = 0; b < nen; ++b)
        for (int d = 0; d < 3; ++d) {
          long long pos = find_col(row_off, cols, 3 * coef_of(mesh, e, a) + d, 3 * coef_of(mesh, e, b) + d);
          if (pos < 0) { rc = ORC_ENOTFOUND; break; }
          vals[pos] += m[nen * a + b];
        }
  }
  free(m);
  return rc;
}

/* Eq. grad_L without constraint terms: g = M (v - v_prev) / h + f_int - f_ext,
 * M given as DOF-level CSR values (f_ext may be NULL); overwrites g */
void orc_gradient(int n_dof, const int* row_off, const int* cols, const double* mvals, const double* v,
                  const double* v_prev, const double* f_int, const double* f_ext, double h, double* g) {
  for (int r = 0; r < n_dof; ++r) {
    double s = 0.0;
    for (int k = row_off[r]; k < row_off[r + 1]; ++k) s += mvals[k] * (v[cols[k]] - v_prev[cols[k]]);
    g[r] = s / h + f_int[r] - (f_ext ? f_ext[r] : 0.0);
  }
}

