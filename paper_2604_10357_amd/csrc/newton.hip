// newton.hip -- the pieces of a Newton step around the assembly:
//   the consistent mass matrix, built once (Sec. 4.1: m_ij = int rho s_i s_j
//   dV, M_e = [m_ij I_3]), stored per pair of adjacent pattern nodes in
//   adjacency order (T10: one value; ANCF: the 4 x 4 block of the two nodes'
//   coefficient pairs);
//   the Newton matrix H = M/h + h K_t on the CSR pattern of K (Sec. 4.4.2,
//   Eq. hessian, without constraint terms), the mass term entering pass 2's
//   LDS segment so that H leaves in the same single write as K;
//   the gradient g = M (v - v_prev)/h + f_int - f_ext (Sec. 4.4.1, Eq.
//   grad_L, without constraint terms), eight lanes per node over its mass row.
#include <cmath>

#include "tlfea_internal.h"

using tlfea::Mesh;

namespace tlfea {
namespace {

// reference integrals int N_a N_b dxi over the unit tetrahedron (volume 1/6)
struct T10MassTable {
  double c[10][10];
};

// T10 shape values at a parent point (corners L (2 L - 1), edge (c, d) nodes
// 4 L_c L_d, node order: corners, then edges 01, 12, 02, 03, 13, 23)
void t10_values(double x, double y, double z, double* N) {
  const double L[4] = {1.0 - x - y - z, x, y, z};
  static const int edge[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
  for (int c = 0; c < 4; ++c) N[c] = L[c] * (2.0 * L[c] - 1.0);
  for (int k = 0; k < 6; ++k) N[4 + k] = 4.0 * L[edge[k][0]] * L[edge[k][1]];
}

// Products of two quadratics are quartic: a 4 x 4 x 4 Gauss-Legendre product
// rule on the cube, mapped onto the tetrahedron by x = u, y = v (1 - u),
// z = w (1 - u)(1 - v) (Jacobian (1 - u)^2 (1 - v)), integrates them exactly.
T10MassTable t10_mass_table() {
  const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
  const double gx[4] = {-b, -a, a, b}, gw[4] = {wb, wa, wa, wb};
  T10MassTable t{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 4; ++k) {
        const double u = 0.5 * (gx[i] + 1.0), v = 0.5 * (gx[j] + 1.0), w = 0.5 * (gx[k] + 1.0);
        const double wt = 0.125 * gw[i] * gw[j] * gw[k] * (1.0 - u) * (1.0 - u) * (1.0 - v);
        double N[10];
        t10_values(u, v * (1.0 - u), w * (1.0 - u) * (1.0 - v), N);
        for (int p = 0; p < 10; ++p)
          for (int q = 0; q < 10; ++q) t.c[p][q] += wt * N[p] * N[q];
      }
  return t;
}

// ANCF: reference integrals int S~_a S~_b dxi over the parent cube [-1, 1]^3
// of the unit-scaled shape functions (the kind scales 1, l_1, l_2, l_3 of the
// coefficients are applied per element).  Shell (per corner p, parent corner
// (sp, tp), s0 = sp xi, t0 = tp eta): value (1+s0)(1+t0)(2+s0+t0-xi^2-eta^2)/8,
// x-slope sp (1+s0)^2 (s0-1)(1+t0)/8, y-slope tp (1+t0)^2 (t0-1)(1+s0)/8,
// transverse zeta (1+s0)(1+t0)/4.  Beam (t = (1+xi)/2): 1-3t^2+2t^3,
// t-2t^2+t^3, eta (1-t), zeta (1-t), 3t^2-2t^3, t^3-t^2, eta t, zeta t.
struct AncfMassTable {
  double c[16][16];
};

void shell_values(double xi, double eta, double zeta, double* S) {
  static const double cs[4] = {-1, 1, 1, -1}, ct[4] = {-1, -1, 1, 1};
  for (int p = 0; p < 4; ++p) {
    const double s0 = cs[p] * xi, t0 = ct[p] * eta, A = 1.0 + s0, B = 1.0 + t0;
    S[4 * p] = A * B * (2.0 + s0 + t0 - xi * xi - eta * eta) / 8.0;
    S[4 * p + 1] = cs[p] * A * A * (s0 - 1.0) * B / 8.0;
    S[4 * p + 2] = ct[p] * B * B * (t0 - 1.0) * A / 8.0;
    S[4 * p + 3] = zeta * A * B / 4.0;
  }
}

void beam_values(double xi, double eta, double zeta, double* S) {
  const double t = 0.5 * (1.0 + xi);
  S[0] = 1.0 - 3.0 * t * t + 2.0 * t * t * t;
  S[1] = t - 2.0 * t * t + t * t * t;
  S[2] = eta * (1.0 - t);
  S[3] = zeta * (1.0 - t);
  S[4] = 3.0 * t * t - 2.0 * t * t * t;
  S[5] = t * t * t - t * t;
  S[6] = eta * t;
  S[7] = zeta * t;
}

// Products of the value functions are at most cubic x cubic in each in-plane
// (shell) or axial (beam) direction and linear x linear across: Gauss-Legendre
// 4 points there and 2 across integrate them exactly.
AncfMassTable ancf_mass_table(bool beam) {
  const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
  const double x4[4] = {-b, -a, a, b}, w4[4] = {wb, wa, wa, wb};
  const double x2[2] = {-1.0 / std::sqrt(3.0), 1.0 / std::sqrt(3.0)};
  const int ny = beam ? 2 : 4, nen = beam ? 8 : 16;
  AncfMassTable t{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < ny; ++j)
      for (int k = 0; k < 2; ++k) {
        const double eta = beam ? x2[j] : x4[j], wy = beam ? 1.0 : w4[j];
        double S[16];
        if (beam) beam_values(x4[i], eta, x2[k], S);
        else shell_values(x4[i], eta, x2[k], S);
        const double wt = w4[i] * wy;  // the 2-point weights are 1
        for (int p = 0; p < nen; ++p)
          for (int q = 0; q < nen; ++q) t.c[p][q] += wt * S[p] * S[q];
      }
  return t;
}

// a lane per (element, node a): m_ab = rho det J0 c_ab added at the adjacency
// entry of (node a, node b) (one-time build; float64 atomics)
__global__ void k_mass_t10(const int32_t* conn, const double* geo, const uint8_t* rank, const int32_t* adj_off,
                           int64_t n_elem, double rho, T10MassTable tab, double* mass) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_elem * 10) return;
  const int64_t e = t / 10;
  const int a = (int)(t - 10 * e);
  const double s = rho * geo[10 * e + 9];
  const int32_t k0 = adj_off[conn[t]];
  const uint8_t* rk = rank + t * rank_stride(10);
  for (int b = 0; b < 10; ++b) atomicAdd(mass + k0 + rk[b], s * tab.c[a][b]);
}

// ANCF (NPN pattern nodes of four coefficients): a lane per (element,
// coefficient a); the affine element's mass is rho det J0 sc_a sc_b c_ab, added
// at entry (ka, kb) of the 4 x 4 block of the adjacency entry (node a, node b)
template <int NPN>
__global__ void k_mass_ancf(const int32_t* conn, const double* geo, const double* escale, double half_h,
                            const uint8_t* rank, const int32_t* adj_off, int64_t n_elem, double rho,
                            AncfMassTable tab, double* mass) {
  constexpr int NEN = 4 * NPN;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_elem * NEN) return;
  const int64_t e = t / NEN;
  const int a = (int)(t - NEN * e), pa = a >> 2, ka = a & 3;
  const double sc[4] = {1.0, escale[2 * e], escale[2 * e + 1], half_h};
  const double s = rho * geo[10 * e + 9] * sc[ka];
  const int32_t k0 = adj_off[conn[e * NPN + pa]];
  const uint8_t* rk = rank + (e * NPN + pa) * rank_stride(NPN);
  for (int b = 0; b < NEN; ++b) {
    const int pb = b >> 2, kb = b & 3;
    atomicAdd(mass + 16 * (int64_t)(k0 + rk[pb]) + 4 * ka + kb, s * sc[kb] * tab.c[a][b]);
  }
}

// DOF-level CSR values of M: row 3(mc I + k) + d holds M_(I,k)(J,l) at column
// 3(mc J + l) + d and 0 at the other columns of the 3 x 3 block
__global__ void k_mass_values(const int32_t* adj_off, const int32_t* row_off, const double* mass, int64_t n_nodes,
                              int mc, double* vals) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n_nodes) return;
  const int32_t k0 = adj_off[I], k1 = adj_off[I + 1];
  for (int k = 0; k < mc; ++k)
    for (int d = 0; d < 3; ++d) {
      double* row = vals + row_off[3 * (mc * I + k) + d];
      for (int32_t x = k0; x < k1; ++x)
        for (int l = 0; l < mc; ++l)
          for (int c = 0; c < 3; ++c)
            row[3 * mc * (x - k0) + 3 * l + c] = c == d ? mass[(int64_t)mc * mc * x + mc * k + l] : 0.0;
    }
}

// g = M (v - v_prev) / h + f_int - f_ext: LANES lanes per pattern node split
// its mass row (consecutive entries: coalesced loads), UNR entries per lane
// and step in flight, and sum their parts with a fixed butterfly of shuffles;
// the group's lanes then write the node's 3 MC rows of g, lane j taking rows
// j, j + LANES, ...  T10 nodes have about 28 neighbours (8 lanes), ANCF nodes
// 3 (beam) or 9 (shell) (4 lanes).
#ifndef TLFEA_GRAD_UNROLL
#define TLFEA_GRAD_UNROLL 2
#endif
template <int MC>
constexpr int grad_lanes() { return MC == 1 ? 8 : 4; }
__global__ void k_vdiff(const double* v, const double* vp, int64_t n, double* dv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dv[i] = v[i] - vp[i];
}

// T10 (about 28 neighbours per node) gathers v - v_prev formed once per DOF
// (dv, vp null); ANCF (3 or 9) forms the difference at each gather.
template <int MC>
__global__ __launch_bounds__(256) void k_gradient(const int32_t* adj_off, const int32_t* adj, const double* mass,
                                                  int64_t n_nodes, const double* dv, const double* vp,
                                                  const double* fint, const double* fext, double inv_h, double* g) {
  constexpr int NR = 3 * MC;  // rows per node: (coefficient k, component d) at 3 k + d
  constexpr int LANES = grad_lanes<MC>(), UNR = TLFEA_GRAD_UNROLL;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t I = t / LANES;
  const int sub = (int)(t % LANES);
  double s[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) s[j] = 0.0;
  if (I < n_nodes) {
    const int32_t x1 = adj_off[I + 1];
    for (int32_t x0 = adj_off[I] + sub; x0 < x1; x0 += LANES * UNR) {
      int64_t J[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) J[u] = x0 + u * LANES < x1 ? adj[x0 + u * LANES] : -1;
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (J[u] < 0) continue;
        const double* mx = mass + (int64_t)MC * MC * (x0 + u * LANES);
#pragma unroll
        for (int l = 0; l < MC; ++l) {
          const int64_t c = 3 * (MC * J[u] + l);
          double d0 = dv[c], d1 = dv[c + 1], d2 = dv[c + 2];
          if constexpr (MC != 1) {
            d0 -= vp[c];
            d1 -= vp[c + 1];
            d2 -= vp[c + 2];
          }
#pragma unroll
          for (int k = 0; k < MC; ++k) {
            const double m = mx[MC * k + l];
            s[3 * k] += m * d0;
            s[3 * k + 1] += m * d1;
            s[3 * k + 2] += m * d2;
          }
        }
      }
    }
  }
  // butterfly over the group: every lane ends with the full sums (all lanes
  // take part; groups never straddle a wave)
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1)
#pragma unroll
    for (int j = 0; j < NR; ++j) s[j] += __shfl_xor(s[j], o, LANES);
  if (I < n_nodes) {
#pragma unroll
    for (int j = 0; j < NR; ++j)
      if (j % LANES == sub) {
        const int64_t r = NR * I + j;
        g[r] = s[j] * inv_h + fint[r] - (fext ? fext[r] : 0.0);
      }
  }
}

int blocks_of(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace
}  // namespace tlfea

static int mass_ready(tlfea_mesh_t mesh) {
  if (!mesh) return TLFEA_ERR_INVALID;
  if (!mesh->m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (!mesh->m.d_mass) return TLFEA_ERR_INVALID;
  if (hipSetDevice(mesh->m.device) != hipSuccess) return TLFEA_ERR_HIP;
  return TLFEA_OK;
}

TLFEA_API int tlfea_build_mass(tlfea_mesh_t mesh, double density) {
  if (!mesh || !(density > 0.0) || !std::isfinite(density)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (!m.affine) return TLFEA_ERR_UNSUPPORTED;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  int32_t n_adj = 0;
  TLFEA_HIP_CHECK(hipMemcpy(&n_adj, m.d_adj_off + m.n_pnodes, sizeof(int32_t), hipMemcpyDeviceToHost));
  const size_t n_val = (size_t)m.mc * m.mc * (n_adj > 0 ? n_adj : 1);
  double* d = nullptr;
  if (hipMalloc(&d, sizeof(double) * n_val) != hipSuccess) {
    (void)hipGetLastError();
    return TLFEA_ERR_NOMEM;
  }
  hipError_t e1 = hipMemset(d, 0, sizeof(double) * n_val);
  const int grid = tlfea::blocks_of(m.n_elem * m.n_en, 256);
  if (e1 == hipSuccess && m.n_elem > 0) {
    if (m.elem_type == TLFEA_T10)
      hipLaunchKernelGGL(tlfea::k_mass_t10, dim3(grid), dim3(256), 0, nullptr, m.d_conn, m.d_geo, m.d_rank,
                         m.d_adj_off, m.n_elem, density, tlfea::t10_mass_table(), d);
    else if (m.elem_type == TLFEA_ANCF3243)
      hipLaunchKernelGGL(tlfea::k_mass_ancf<2>, dim3(grid), dim3(256), 0, nullptr, m.d_conn, m.d_geo, m.d_escale,
                         0.5 * m.thickness, m.d_rank, m.d_adj_off, m.n_elem, density, tlfea::ancf_mass_table(true),
                         d);
    else
      hipLaunchKernelGGL(tlfea::k_mass_ancf<4>, dim3(grid), dim3(256), 0, nullptr, m.d_conn, m.d_geo, m.d_escale,
                         0.5 * m.thickness, m.d_rank, m.d_adj_off, m.n_elem, density, tlfea::ancf_mass_table(false),
                         d);
  }
  hipError_t e2 = hipGetLastError();
  hipError_t e3 = hipDeviceSynchronize();
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    (void)hipFree(d);
    return TLFEA_ERR_HIP;
  }
  (void)hipFree(m.d_mass);
  m.d_mass = d;
  m.density = density;
  return TLFEA_OK;
}

TLFEA_API int tlfea_get_mass(tlfea_mesh_t mesh, double* d_vals, void* stream) {
  int rc = mass_ready(mesh);
  if (rc) return rc;
  if (!d_vals) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (m.n_pnodes > 0)
    hipLaunchKernelGGL(tlfea::k_mass_values, dim3(tlfea::blocks_of(m.n_pnodes, 256)), dim3(256), 0,
                       (hipStream_t)stream, m.d_adj_off, m.d_row_off, m.d_mass, m.n_pnodes, m.mc, d_vals);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

TLFEA_API int tlfea_newton_gradient(tlfea_mesh_t mesh, const double* d_v, const double* d_v_prev,
                                    const double* d_f_int, const double* d_f_ext, double h, double* d_g,
                                    void* stream) {
  int rc = mass_ready(mesh);
  if (rc) return rc;
  if (!d_v || !d_v_prev || !d_f_int || !d_g || !(h > 0.0) || !std::isfinite(h)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (m.n_pnodes == 0) return TLFEA_OK;
  const auto s = (hipStream_t)stream;
  if (m.mc == 1) {
    // v - v_prev once per DOF, so that the neighbour gathers read one vector
    if (!m.d_dv) {
      if (hipMalloc(&m.d_dv, sizeof(double) * m.n_dof) != hipSuccess) {
        (void)hipGetLastError();
        m.d_dv = nullptr;
        return TLFEA_ERR_NOMEM;
      }
    }
    hipLaunchKernelGGL(tlfea::k_vdiff, dim3(tlfea::blocks_of(m.n_dof, 256)), dim3(256), 0, s, d_v, d_v_prev,
                       m.n_dof, m.d_dv);
    hipLaunchKernelGGL(tlfea::k_gradient<1>, dim3(tlfea::blocks_of(m.n_pnodes * tlfea::grad_lanes<1>(), 256)),
                       dim3(256), 0, s, m.d_adj_off, m.d_adj, m.d_mass, m.n_pnodes, m.d_dv, nullptr, d_f_int,
                       d_f_ext, 1.0 / h, d_g);
  } else {
    hipLaunchKernelGGL(tlfea::k_gradient<4>, dim3(tlfea::blocks_of(m.n_pnodes * tlfea::grad_lanes<4>(), 256)),
                       dim3(256), 0, s, m.d_adj_off, m.d_adj, m.d_mass, m.n_pnodes, d_v, d_v_prev, d_f_int,
                       d_f_ext, 1.0 / h, d_g);
  }
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

TLFEA_API int tlfea_assemble_newton(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                                    double* d_f, double* d_vals, void* stream) {
  int rc = mass_ready(mesh);
  if (rc) return rc;
  if (!d_q || !d_vals || !(h > 0.0) || !std::isfinite(h)) return TLFEA_ERR_INVALID;
  // pass 1 with (alpha, beta) = (h, 1), then pass 2 with the mass term
  if ((rc = tlfea_assemble_points(mesh, d_q, d_qdot, h, 1.0, 1, stream))) return rc;
  Mesh& m = mesh->m;
  tlfea::GatherOptions mt;
  mt.mass = m.d_mass;
  mt.inv_h = 1.0 / h;
  return tlfea::launch_nodes(m, d_f, d_vals, false, (hipStream_t)stream, mt);
}

TLFEA_API int tlfea_assemble_newton_upper(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                                          double* d_f, double* d_vals_upper, void* stream) {
  int rc = mass_ready(mesh);
  if (rc) return rc;
  if (!d_q || !d_vals_upper || !(h > 0.0) || !std::isfinite(h)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (!m.d_row_off_u) return TLFEA_ERR_INVALID;
  // M/h + h df/dq is symmetric for the hyperelastic laws; the Kelvin-Voigt part is not
  if (m.kv_eta != 0.0 || m.kv_lambda != 0.0) return TLFEA_ERR_UNSUPPORTED;
  if ((rc = tlfea_assemble_points(mesh, d_q, d_qdot, h, 1.0, 1, stream))) return rc;
  tlfea::GatherOptions mt;
  mt.mass = m.d_mass;
  mt.inv_h = 1.0 / h;
  mt.row_off_u = m.d_row_off_u;
  return tlfea::launch_nodes(m, d_f, d_vals_upper, false, (hipStream_t)stream, mt);
}
