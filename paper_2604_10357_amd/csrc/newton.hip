// newton.hip -- the pieces of a Newton step around the assembly (T10):
//   the consistent mass matrix, built once (Sec. 4.1: m_ij = int rho s_i s_j
//   dV, M_e = [m_ij I_3]), stored per coefficient pair in adjacency order;
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

// DOF-level CSR values of M: row 3I+d holds M_IJ at column 3J+d, 0 elsewhere
__global__ void k_mass_values(const int32_t* adj_off, const int32_t* row_off, const double* mass, int64_t n_nodes,
                              double* vals) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n_nodes) return;
  const int32_t k0 = adj_off[I], k1 = adj_off[I + 1];
  for (int d = 0; d < 3; ++d) {
    double* row = vals + row_off[3 * I + d];
    for (int32_t k = k0; k < k1; ++k)
      for (int c = 0; c < 3; ++c) row[3 * (k - k0) + c] = c == d ? mass[k] : 0.0;
  }
}

// g = M (v - v_prev) / h + f_int - f_ext: kGradLanes lanes per node split its
// mass row (consecutive entries: coalesced loads) and sum their parts with a
// fixed butterfly of shuffles; lanes 0, 1, 2 of the group write g_I
constexpr int kGradLanes = 8;
__global__ __launch_bounds__(256) void k_gradient(const int32_t* adj_off, const int32_t* adj, const double* mass,
                                                  int64_t n_nodes, const double* v, const double* vp,
                                                  const double* fint, const double* fext, double inv_h, double* g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t I = t / kGradLanes;
  const int sub = (int)(t % kGradLanes);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (I < n_nodes) {
    for (int32_t k = adj_off[I] + sub; k < adj_off[I + 1]; k += kGradLanes) {
      const int64_t J = adj[k];
      const double m = mass[k];
      s0 += m * (v[3 * J] - vp[3 * J]);
      s1 += m * (v[3 * J + 1] - vp[3 * J + 1]);
      s2 += m * (v[3 * J + 2] - vp[3 * J + 2]);
    }
  }
  // butterfly over the group: every lane ends with the full sums (all lanes
  // take part; groups never straddle a wave)
#pragma unroll
  for (int o = kGradLanes / 2; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, kGradLanes);
    s1 += __shfl_xor(s1, o, kGradLanes);
    s2 += __shfl_xor(s2, o, kGradLanes);
  }
  if (I < n_nodes && sub < 3) {
    const double s = sub == 0 ? s0 : sub == 1 ? s1 : s2;
    const int64_t r = 3 * I + sub;
    g[r] = s * inv_h + fint[r] - (fext ? fext[r] : 0.0);
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
  if (m.elem_type != TLFEA_T10 || !m.affine) return TLFEA_ERR_UNSUPPORTED;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  int32_t n_adj = 0;
  TLFEA_HIP_CHECK(hipMemcpy(&n_adj, m.d_adj_off + m.n_pnodes, sizeof(int32_t), hipMemcpyDeviceToHost));
  double* d = nullptr;
  if (hipMalloc(&d, sizeof(double) * (n_adj > 0 ? n_adj : 1)) != hipSuccess) {
    (void)hipGetLastError();
    return TLFEA_ERR_NOMEM;
  }
  hipError_t e1 = hipMemset(d, 0, sizeof(double) * (n_adj > 0 ? n_adj : 1));
  if (e1 == hipSuccess && m.n_elem > 0)
    hipLaunchKernelGGL(tlfea::k_mass_t10, dim3(tlfea::blocks_of(m.n_elem * 10, 256)), dim3(256), 0, nullptr,
                       m.d_conn, m.d_geo, m.d_rank, m.d_adj_off, m.n_elem, density, tlfea::t10_mass_table(), d);
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
                       (hipStream_t)stream, m.d_adj_off, m.d_row_off, m.d_mass, m.n_pnodes, d_vals);
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
  if (m.n_pnodes > 0)
    hipLaunchKernelGGL(tlfea::k_gradient, dim3(tlfea::blocks_of(m.n_pnodes * tlfea::kGradLanes, 256)), dim3(256), 0,
                       (hipStream_t)stream, m.d_adj_off, m.d_adj, m.d_mass, m.n_pnodes, d_v, d_v_prev, d_f_int,
                       d_f_ext, 1.0 / h, d_g);
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
