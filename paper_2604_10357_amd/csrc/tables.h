// tables.h -- compile-time element tables for the gfx950 kernels.
//
// Sec. 4.1 of the paper: shape-function parent gradients and quadrature
// nodes/weights depend only on the element type and the rule, so they are
// tabulated once.  Here they are built by constexpr code, which lets the
// kernels index them with compile-time quadrature/node indices and fold the
// values (and skip the zeros) inside fully unrolled loops.  A copy with
// internal linkage in __constant__ memory serves run-time indices.
#pragma once

namespace tlfea {

// ---------------------------------------------------------------------------
// T10: 10-node quadratic tetrahedron, parent coordinates = barycentric
// (L1, L2, L3), L0 = 1 - L1 - L2 - L3.  Corner c: N = L_c (2 L_c - 1); node on
// edge (c, d): N = 4 L_c L_d.  Edge order (0,1),(1,2),(0,2),(0,3),(1,3),(2,3).
// Rule: 5-point Keast (degree 3) -- centroid weight -4/5, the four points with
// one barycentric coordinate 1/2 and the others 1/6 weight 9/20, times 1/6.
// ---------------------------------------------------------------------------
struct T10Table {
  double dN[5][10][3];  // parent gradient of N_a at point q
  double w[5];          // weights (sum 1/6)
};

constexpr T10Table make_t10_table() {
  T10Table t{};
  const double sixth = 1.0 / 6.0;
  const double bary[5][4] = {{0.25, 0.25, 0.25, 0.25},
                             {0.5, sixth, sixth, sixth},
                             {sixth, 0.5, sixth, sixth},
                             {sixth, sixth, 0.5, sixth},
                             {sixth, sixth, sixth, 0.5}};
  const double dL[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const int ed[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
  for (int q = 0; q < 5; ++q) {
    const double* L = bary[q];
    for (int c = 0; c < 4; ++c)
      for (int m = 0; m < 3; ++m) t.dN[q][c][m] = (4.0 * L[c] - 1.0) * dL[c][m];
    for (int k = 0; k < 6; ++k) {
      int c = ed[k][0], d = ed[k][1];
      for (int m = 0; m < 3; ++m) t.dN[q][4 + k][m] = 4.0 * (L[c] * dL[d][m] + L[d] * dL[c][m]);
    }
    t.w[q] = (q == 0 ? -0.8 : 0.45) / 6.0;
  }
  return t;
}

inline constexpr T10Table kT10 = make_t10_table();

// ---------------------------------------------------------------------------
// ANCF3443 shell: per corner p (parent (sp, tp) in {(-1,-1),(1,-1),(1,1),(-1,1)})
// and s0 = sp*xi, t0 = tp*eta the functions are
//   value  : (1+s0)(1+t0)(2 + s0 + t0 - xi^2 - eta^2) / 8
//   r_x    : (lx/2) * sp (1+s0)^2 (s0-1)(1+t0) / 8
//   r_y    : (ly/2) * tp (1+t0)^2 (t0-1)(1+s0) / 8
//   r_z    : (H/2)  * zeta (1+s0)(1+t0) / 4
// i.e. the incomplete-bicubic functions that interpolate value and physical
// slopes at the corners (x = lx xi / 2, y = ly eta / 2), and the bilinear
// transverse-gradient function.  The table stores the gradients WITHOUT the
// element scale factors (1, lx/2, ly/2, H/2), which the kernels apply.
// ---------------------------------------------------------------------------
constexpr double kCornerS[4] = {-1, 1, 1, -1};
constexpr double kCornerT[4] = {-1, -1, 1, 1};

// textbook Gauss-Legendre nodes / weights (n = 2, 3, 4)
constexpr double gl_node(int n, int i) {
  if (n == 2) return i == 0 ? -0.57735026918962576451 : 0.57735026918962576451;
  if (n == 3) return i == 0 ? -0.77459666924148337704 : (i == 1 ? 0.0 : 0.77459666924148337704);
  // n == 4
  return i == 0 ? -0.86113631159405257522
                : (i == 1 ? -0.33998104358485626480 : (i == 2 ? 0.33998104358485626480 : 0.86113631159405257522));
}
constexpr double gl_weight(int n, int i) {
  if (n == 2) return 1.0;
  if (n == 3) return i == 1 ? 8.0 / 9.0 : 5.0 / 9.0;
  return (i == 1 || i == 2) ? 0.65214515486254614263 : 0.34785484513745385737;
}

template <int NX, int NY, int NZ>
struct AncfTable {
  static constexpr int NQ = NX * NY * NZ;
  double dS[NQ][16][3];  // unit-scaled parent gradients
  double w[NQ];
};

template <int NX, int NY, int NZ>
constexpr AncfTable<NX, NY, NZ> make_ancf_table() {
  AncfTable<NX, NY, NZ> t{};
  int q = 0;
  for (int i = 0; i < NX; ++i)
    for (int j = 0; j < NY; ++j)
      for (int k = 0; k < NZ; ++k) {
        const double s = gl_node(NX, i), r = gl_node(NY, j), z = gl_node(NZ, k);
        t.w[q] = gl_weight(NX, i) * gl_weight(NY, j) * gl_weight(NZ, k);
        for (int p = 0; p < 4; ++p) {
          const double sp = kCornerS[p], tp = kCornerT[p];
          const double s0 = sp * s, t0 = tp * r;
          const double A = 1.0 + s0, B = 1.0 + t0, C = 2.0 + s0 + t0 - s * s - r * r;
          // value function
          t.dS[q][4 * p + 0][0] = B * (sp * C + A * (sp - 2.0 * s)) / 8.0;
          t.dS[q][4 * p + 0][1] = A * (tp * C + B * (tp - 2.0 * r)) / 8.0;
          t.dS[q][4 * p + 0][2] = 0.0;
          // x-slope function (unit scale)
          t.dS[q][4 * p + 1][0] = A * B * (3.0 * s0 - 1.0) / 8.0;
          t.dS[q][4 * p + 1][1] = sp * tp * A * A * (s0 - 1.0) / 8.0;
          t.dS[q][4 * p + 1][2] = 0.0;
          // y-slope function (unit scale)
          t.dS[q][4 * p + 2][0] = sp * tp * B * B * (t0 - 1.0) / 8.0;
          t.dS[q][4 * p + 2][1] = A * B * (3.0 * t0 - 1.0) / 8.0;
          t.dS[q][4 * p + 2][2] = 0.0;
          // transverse function zeta * b_p (unit scale)
          t.dS[q][4 * p + 3][0] = z * sp * B / 4.0;
          t.dS[q][4 * p + 3][1] = z * tp * A / 4.0;
          t.dS[q][4 * p + 3][2] = A * B / 4.0;
        }
        ++q;
      }
  return t;
}

inline constexpr AncfTable<3, 3, 2> kAncf332 = make_ancf_table<3, 3, 2>();
inline constexpr AncfTable<4, 4, 3> kAncf443 = make_ancf_table<4, 4, 3>();

// ---------------------------------------------------------------------------
// ANCF3243 beam: nodes 0, 1 at parent u = -1, 1 with coefficients r, r_x, r_y,
// r_z.  With t = (1 + u)/2 along the axis and the parent cross-section
// coordinates v, w (y = W v / 2, z = H w / 2) the functions of node 0 / node 1 are
//   value : 1 - 3t^2 + 2t^3          / 3t^2 - 2t^3
//   r_x   : L (t - 2t^2 + t^3)       / L (t^3 - t^2)
//   r_y   : (W/2) v (1 - t)          / (W/2) v t
//   r_z   : (H/2) w (1 - t)          / (H/2) w t
// (cubic Hermite functions along the axis, cross-section gradients
// interpolated linearly).  As for the shell, the table holds the gradients
// without the element scales (1, L, W/2, H/2).
// ---------------------------------------------------------------------------
template <int NX, int NY, int NZ>
struct BeamTable {
  static constexpr int NQ = NX * NY * NZ;
  double dS[NQ][8][3];  // unit-scaled parent gradients
  double w[NQ];
};

template <int NX, int NY, int NZ>
constexpr BeamTable<NX, NY, NZ> make_beam_table() {
  BeamTable<NX, NY, NZ> t{};
  int q = 0;
  for (int i = 0; i < NX; ++i)
    for (int j = 0; j < NY; ++j)
      for (int k = 0; k < NZ; ++k) {
        const double u = gl_node(NX, i), v = gl_node(NY, j), z = gl_node(NZ, k);
        const double tt = 0.5 * (1.0 + u);
        t.w[q] = gl_weight(NX, i) * gl_weight(NY, j) * gl_weight(NZ, k);
        for (int a = 0; a < 8; ++a)
          for (int m = 0; m < 3; ++m) t.dS[q][a][m] = 0.0;
        // d/du = (1/2) d/dt
        t.dS[q][0][0] = 0.5 * (6.0 * tt * tt - 6.0 * tt);
        t.dS[q][1][0] = 0.5 * (1.0 - 4.0 * tt + 3.0 * tt * tt);
        t.dS[q][2][0] = -0.5 * v;
        t.dS[q][2][1] = 1.0 - tt;
        t.dS[q][3][0] = -0.5 * z;
        t.dS[q][3][2] = 1.0 - tt;
        t.dS[q][4][0] = 0.5 * (6.0 * tt - 6.0 * tt * tt);
        t.dS[q][5][0] = 0.5 * (3.0 * tt * tt - 2.0 * tt);
        t.dS[q][6][0] = 0.5 * v;
        t.dS[q][6][1] = tt;
        t.dS[q][7][0] = 0.5 * z;
        t.dS[q][7][2] = tt;
        ++q;
      }
  return t;
}

inline constexpr BeamTable<3, 2, 2> kBeam322 = make_beam_table<3, 2, 2>();

}  // namespace tlfea
