// mesh.hip -- mesh handles, reference-geometry precompute and the C ABI entry points.
//
// Sec. 4.1 of the paper: everything that depends only on the reference
// configuration is computed once and cached in device memory.  Here that is,
// per element and quadrature point, J0 = sum_a X_a (x) dN_a, det J0 and J0^-1
// (computed by a kernel), kept once per element when the element is affine
// (straight-sided T10, flat rectangular ANCF) and per point otherwise.
#include <cmath>
#include <cstring>
#include <new>

#include "rules.h"
#include "tlfea_internal.h"

namespace tlfea {
namespace {

// J0 at every (element, point); ANCF element scales from the reference nodes
// (shell: half edge lengths; beam: length L and half width)
template <class Rule>
__global__ void k_geometry(const int32_t* conn, const double* X, int64_t n_elem, double half_h, double half_w,
                           double* geo, double* escale, uint32_t* err) {
  constexpr int NQ = Rule::NQ;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_elem * NQ) return;
  const int64_t e = t / NQ;
  const int q = (int)(t % NQ);
  const int32_t* ce = conn + e * Rule::NPN;
  double sc[4] = {1.0, 1.0, 1.0, 1.0};
  if constexpr (Rule::MC == 4 && Rule::NPN == 2) {
    const double* x0 = X + 3 * (4 * (int64_t)ce[0]);
    const double* x1 = X + 3 * (4 * (int64_t)ce[1]);
    sc[1] = sqrt((x1[0] - x0[0]) * (x1[0] - x0[0]) + (x1[1] - x0[1]) * (x1[1] - x0[1]) +
                 (x1[2] - x0[2]) * (x1[2] - x0[2]));
    sc[2] = half_w;
    sc[3] = half_h;
    if (q == 0) {
      escale[2 * e] = sc[1];
      escale[2 * e + 1] = sc[2];
    }
  } else if constexpr (Rule::MC == 4) {
    const double* x0 = X + 3 * (4 * (int64_t)ce[0]);
    const double* x1 = X + 3 * (4 * (int64_t)ce[1]);
    const double* x3 = X + 3 * (4 * (int64_t)ce[3]);
    const double lx = sqrt((x1[0] - x0[0]) * (x1[0] - x0[0]) + (x1[1] - x0[1]) * (x1[1] - x0[1]) +
                           (x1[2] - x0[2]) * (x1[2] - x0[2]));
    const double ly = sqrt((x3[0] - x0[0]) * (x3[0] - x0[0]) + (x3[1] - x0[1]) * (x3[1] - x0[1]) +
                           (x3[2] - x0[2]) * (x3[2] - x0[2]));
    sc[1] = 0.5 * lx;
    sc[2] = 0.5 * ly;
    sc[3] = half_h;
    if (q == 0) {
      escale[2 * e] = sc[1];
      escale[2 * e + 1] = sc[2];
    }
  }
  // The position functions (T10: all; ANCF: the value functions) sum to one,
  // so their gradients sum to zero and J0 may be formed from positions taken
  // relative to the element's first node: the same J0, without the
  // cancellation that absolute coordinates far from the origin (a long chain)
  // would cost.
  double J0[9], x_ref[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) J0[k] = 0.0;
  {
    const int64_t c0 = Rule::MC == 1 ? (int64_t)ce[0] : 4 * (int64_t)ce[0];
#pragma unroll
    for (int i = 0; i < 3; ++i) x_ref[i] = X[3 * c0 + i];
  }
  for (int a = 0; a < Rule::NEN; ++a) {
    int64_t c;
    if constexpr (Rule::MC == 1) c = ce[a]; else c = 4 * (int64_t)ce[a >> 2] + (a & 3);
    const double s = sc[a % 4];
    const bool position = Rule::MC == 1 || (a & 3) == 0;
    const double d0 = Rule::dN_rt(q, a, 0) * s, d1 = Rule::dN_rt(q, a, 1) * s, d2 = Rule::dN_rt(q, a, 2) * s;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double x = position ? X[3 * c + i] - x_ref[i] : X[3 * c + i];
      J0[3 * i] += x * d0;
      J0[3 * i + 1] += x * d1;
      J0[3 * i + 2] += x * d2;
    }
  }
  const double c00 = J0[4] * J0[8] - J0[5] * J0[7];
  const double c01 = J0[5] * J0[6] - J0[3] * J0[8];
  const double c02 = J0[3] * J0[7] - J0[4] * J0[6];
  const double det = J0[0] * c00 + J0[1] * c01 + J0[2] * c02;
  double* rec = geo + 10 * t;
  if (!(det > 0.0) || !isfinite(det)) {
    atomicOr(err, 1u);
    for (int k = 0; k < 10; ++k) rec[k] = 0.0;
    return;
  }
  const double id = 1.0 / det;
  // inverse = adj / det, row-major [m][J]
  rec[0] = c00 * id;
  rec[1] = (J0[2] * J0[7] - J0[1] * J0[8]) * id;
  rec[2] = (J0[1] * J0[5] - J0[2] * J0[4]) * id;
  rec[3] = c01 * id;
  rec[4] = (J0[0] * J0[8] - J0[2] * J0[6]) * id;
  rec[5] = (J0[2] * J0[3] - J0[0] * J0[5]) * id;
  rec[6] = c02 * id;
  rec[7] = (J0[1] * J0[6] - J0[0] * J0[7]) * id;
  rec[8] = (J0[0] * J0[4] - J0[1] * J0[3]) * id;
  rec[9] = det;
}

// flag elements whose J0 differs between points (relative 1e-13)
__global__ void k_affine_check(const double* geo, int64_t n_elem, int nq, uint32_t* err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  const double* r0 = geo + 10 * e * nq;
  double scale = 0.0;
  for (int k = 0; k < 9; ++k) scale = fmax(scale, fabs(r0[k]));
  for (int q = 1; q < nq; ++q) {
    const double* r = r0 + 10 * q;
    bool same = fabs(r[9] - r0[9]) <= 1e-13 * fabs(r0[9]);
    for (int k = 0; k < 9; ++k) same = same && (fabs(r[k] - r0[k]) <= 1e-13 * scale);
    if (!same) {
      atomicOr(err, 2u);
      return;
    }
  }
}

__global__ void k_compact(const double* full, int64_t n_elem, int nq, double* geo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_elem * 10) return;
  geo[t] = full[(t / 10) * 10 * nq + t % 10];
}

int grid_of(int64_t n, int b) { return (int)((n + b - 1) / b); }

void free_mesh(Mesh& m) {
  (void)hipFree(m.d_conn);
  (void)hipFree(m.d_X);
  (void)hipFree(m.d_geo);
  (void)hipFree(m.d_escale);
  (void)hipFree(m.d_flags);
  (void)hipFree(m.d_mp);
  (void)hipFree(m.d_row_off);
  (void)hipFree(m.d_cols);
  (void)hipFree(m.d_adj_off);
  (void)hipFree(m.d_adj);
  (void)hipFree(m.d_rank);
  (void)hipFree(m.d_inc_off);
  (void)hipFree(m.d_inc);
  (void)hipFree(m.d_ranges);
  (void)hipFree(m.d_incpos);
  (void)hipFree(m.d_rank_inc);
  (void)hipFree(m.d_mass);
  (void)hipFree(m.d_solver);
  (void)hipFree(m.d_dv);
  (void)hipFree(m.d_row_off_u);
  (void)hipFree(m.d_cols_u);
  (void)hipFree(m.d_stage);
  m = Mesh{};
}

bool valid_material(int material, const double* params, double eta, double lam_v) {
  if (material == TLFEA_SVK) {
    if (!(params[1] > -1.0 && params[1] < 0.5)) return false;
  } else if (material != TLFEA_MOONEY_RIVLIN) {
    return false;
  }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(params[k])) return false;
  return std::isfinite(eta) && std::isfinite(lam_v);
}

int check_call(tlfea_mesh_t mesh, const double* q, bool need_pattern) {
  if (!mesh || !q) return TLFEA_ERR_INVALID;
  if (need_pattern && !mesh->m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (hipSetDevice(mesh->m.device) != hipSuccess) return TLFEA_ERR_HIP;
  return TLFEA_OK;
}

}  // namespace

MatParams make_params(int material, const double* params, double eta, double lam_v) {
  MatParams mp{};
  mp.kind = material;
  if (material == TLFEA_SVK) {
    const double E = params[0], nu = params[1];
    mp.c0 = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    mp.c1 = E / (2.0 * (1.0 + nu));
    mp.c2 = 0.0;
  } else {
    mp.c0 = params[0];
    mp.c1 = params[1];
    mp.c2 = params[2];
  }
  mp.eta = eta;
  mp.lam_v = lam_v;
  return mp;
}

int precompute_geometry(Mesh& m) {
  const int nq = m.n_qp;
  const int64_t nrec = m.n_elem * nq;
  double* full = nullptr;
  TLFEA_HIP_CHECK(hipMalloc(&full, sizeof(double) * 10 * (nrec > 0 ? nrec : 1)));
  uint32_t* err = nullptr;
  if (hipMalloc(&err, sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(full);
    return TLFEA_ERR_NOMEM;
  }
  (void)hipMemset(err, 0, sizeof(uint32_t));
  if (nrec > 0) {
    const double hh = 0.5 * m.thickness, hw = 0.5 * m.width;
    if (m.elem_type == TLFEA_T10)
      hipLaunchKernelGGL(k_geometry<RuleT10>, dim3(grid_of(nrec, 256)), dim3(256), 0, 0, m.d_conn, m.d_X,
                         m.n_elem, hh, hw, full, m.d_escale, err);
    else if (m.elem_type == TLFEA_ANCF3243)
      hipLaunchKernelGGL(k_geometry<RuleBeam>, dim3(grid_of(nrec, 256)), dim3(256), 0, 0, m.d_conn, m.d_X,
                         m.n_elem, hh, hw, full, m.d_escale, err);
    else if (m.gl[0] == 3)
      hipLaunchKernelGGL((k_geometry<RuleAncf<3, 3, 2>>), dim3(grid_of(nrec, 256)), dim3(256), 0, 0, m.d_conn,
                         m.d_X, m.n_elem, hh, hw, full, m.d_escale, err);
    else
      hipLaunchKernelGGL((k_geometry<RuleAncf<4, 4, 3>>), dim3(grid_of(nrec, 256)), dim3(256), 0, 0, m.d_conn,
                         m.d_X, m.n_elem, hh, hw, full, m.d_escale, err);
    hipLaunchKernelGGL(k_affine_check, dim3(grid_of(m.n_elem, 256)), dim3(256), 0, 0, full, m.n_elem, nq, err);
  }
  uint32_t h = 0;
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipMemcpy(&h, err, sizeof(uint32_t), hipMemcpyDeviceToHost);
  (void)hipFree(err);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    (void)hipFree(full);
    return TLFEA_ERR_HIP;
  }
  if (h & 1u) {
    (void)hipFree(full);
    return TLFEA_ERR_DEGENERATE;
  }
  if (!(h & 2u) && m.n_elem > 0) {
    double* geo = nullptr;
    if (hipMalloc(&geo, sizeof(double) * 10 * m.n_elem) != hipSuccess) {
      (void)hipFree(full);
      return TLFEA_ERR_NOMEM;
    }
    hipLaunchKernelGGL(k_compact, dim3(grid_of(m.n_elem * 10, 256)), dim3(256), 0, 0, full, m.n_elem, nq, geo);
    hipError_t e3 = hipDeviceSynchronize();
    (void)hipFree(full);
    if (e3 != hipSuccess) {
      (void)hipFree(geo);
      return TLFEA_ERR_HIP;
    }
    m.d_geo = geo;
    m.affine = true;
  } else {
    m.d_geo = full;
    m.affine = false;
  }
  return TLFEA_OK;
}

AsmArgs make_args(const Mesh& m, const double* q, const double* qdot, double* f, double* vals, double alpha,
                  double beta) {
  AsmArgs a{};
  a.conn = m.d_conn;
  a.X = m.d_X;
  a.geo = m.d_geo;
  a.escale = m.d_escale;
  a.half_h = 0.5 * m.thickness;
  a.affine = m.affine ? 1 : 0;
  a.n_elem = m.n_elem;
  a.q = q;
  a.qdot = qdot;
  a.f = f;
  a.vals = vals;
  a.row_off = m.d_row_off;
  a.rank = m.d_rank;
  a.mp = m.mp;
  a.alpha = alpha;
  a.beta = beta;
  a.flags = m.d_flags;
  a.mp_dev = nullptr;
  return a;
}

}  // namespace tlfea

using tlfea::Mesh;

TLFEA_API const char* tlfea_status_string(int status) {
  switch (status) {
    case TLFEA_OK: return "ok";
    case TLFEA_ERR_INVALID: return "invalid argument";
    case TLFEA_ERR_UNSUPPORTED: return "unsupported element, material, rule or mesh feature";
    case TLFEA_ERR_DEGENERATE: return "degenerate reference element (det J0 <= 0)";
    case TLFEA_ERR_HIP: return "HIP runtime error";
    case TLFEA_ERR_NOMEM: return "device out of memory";
    case TLFEA_ERR_NO_PATTERN: return "CSR pattern not built";
    case TLFEA_ERR_TOO_LARGE:
      return "size exceeds int32 indexing, or the fixed work area of an allocation-free call";
    default: return "unknown status";
  }
}

TLFEA_API int tlfea_version(void) { return 100; }

TLFEA_API int tlfea_mesh_create(const tlfea_mesh_desc* d, tlfea_mesh_t* out) {
  if (!out) return TLFEA_ERR_INVALID;
  *out = nullptr;
  if (!d || d->n_elem < 0 || d->n_coef < 0 || (d->n_elem > 0 && (!d->h_conn || !d->h_X))) return TLFEA_ERR_INVALID;
  Mesh m;
  m.elem_type = d->elem_type;
  if (d->elem_type == TLFEA_T10) {
    m.n_en = 10; m.n_pn = 10; m.mc = 1; m.n_qp = 5;
    m.n_pnodes = d->n_coef;
  } else if (d->elem_type == TLFEA_ANCF3443) {
    const bool r332 = d->gl[0] == 3 && d->gl[1] == 3 && d->gl[2] == 2;
    const bool r443 = d->gl[0] == 4 && d->gl[1] == 4 && d->gl[2] == 3;
    if (!r332 && !r443) return TLFEA_ERR_UNSUPPORTED;
    if (d->n_coef % 4 != 0 || !(d->thickness > 0.0)) return TLFEA_ERR_INVALID;
    m.n_en = 16; m.n_pn = 4; m.mc = 4; m.n_qp = d->gl[0] * d->gl[1] * d->gl[2];
    m.gl[0] = d->gl[0]; m.gl[1] = d->gl[1]; m.gl[2] = d->gl[2];
    m.thickness = d->thickness;
    m.n_pnodes = d->n_coef / 4;
  } else if (d->elem_type == TLFEA_ANCF3243) {
    if (d->gl[0] != 3 || d->gl[1] != 2 || d->gl[2] != 2) return TLFEA_ERR_UNSUPPORTED;
    if (d->n_coef % 4 != 0 || !(d->thickness > 0.0) || !(d->width > 0.0) || !std::isfinite(d->thickness) ||
        !std::isfinite(d->width))
      return TLFEA_ERR_INVALID;
    m.n_en = 8; m.n_pn = 2; m.mc = 4; m.n_qp = 12;
    m.gl[0] = 3; m.gl[1] = 2; m.gl[2] = 2;
    m.thickness = d->thickness;
    m.width = d->width;
    m.n_pnodes = d->n_coef / 4;
  } else {
    return TLFEA_ERR_UNSUPPORTED;
  }
  if (d->material != TLFEA_SVK && d->material != TLFEA_MOONEY_RIVLIN) return TLFEA_ERR_UNSUPPORTED;
  if (!tlfea::valid_material(d->material, d->params, d->kv_eta, d->kv_lambda)) return TLFEA_ERR_INVALID;
  if (d->precision != TLFEA_FP64 && d->precision != TLFEA_MIXED) return TLFEA_ERR_INVALID;
  if (3 * d->n_coef + 1 > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  // host-side argument validation: connectivity ids in range
  const int64_t nconn = d->n_elem * m.n_pn;
  for (int64_t i = 0; i < nconn; ++i)
    if (d->h_conn[i] < 0 || d->h_conn[i] >= m.n_pnodes) return TLFEA_ERR_INVALID;
  for (int64_t i = 0; i < 3 * d->n_coef; ++i)
    if (!std::isfinite(d->h_X[i])) return TLFEA_ERR_INVALID;
  m.n_elem = d->n_elem;
  m.n_coef = d->n_coef;
  m.n_dof = 3 * d->n_coef;
  m.precision = d->precision;
  m.material = d->material;
  std::memcpy(m.params, d->params, sizeof(m.params));
  m.kv_eta = d->kv_eta;
  m.kv_lambda = d->kv_lambda;
  m.mp = tlfea::make_params(d->material, d->params, d->kv_eta, d->kv_lambda);
  if (hipGetDevice(&m.device) != hipSuccess) return TLFEA_ERR_HIP;

  auto fail = [&](int rc) {
    tlfea::free_mesh(m);
    return rc;
  };
  if (hipMalloc(&m.d_conn, sizeof(int32_t) * (nconn > 0 ? nconn : 1)) != hipSuccess ||
      hipMalloc(&m.d_X, sizeof(double) * (m.n_dof > 0 ? m.n_dof : 1)) != hipSuccess ||
      hipMalloc(&m.d_flags, sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&m.d_mp, sizeof(double) * 5) != hipSuccess ||
      (m.mc == 4 && hipMalloc(&m.d_escale, sizeof(double) * 2 * (m.n_elem > 0 ? m.n_elem : 1)) != hipSuccess)) {
    (void)hipGetLastError();
    return fail(TLFEA_ERR_NOMEM);
  }
  if ((nconn > 0 && hipMemcpy(m.d_conn, d->h_conn, sizeof(int32_t) * nconn, hipMemcpyHostToDevice) != hipSuccess) ||
      (m.n_dof > 0 && hipMemcpy(m.d_X, d->h_X, sizeof(double) * m.n_dof, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemset(m.d_flags, 0, sizeof(uint32_t)) != hipSuccess)
    return fail(TLFEA_ERR_HIP);
  int rc = tlfea::precompute_geometry(m);
  if (rc) return fail(rc);
  auto* h = new (std::nothrow) tlfea_mesh_s;
  if (!h) return fail(TLFEA_ERR_NOMEM);
  h->m = m;
  *out = h;
  return TLFEA_OK;
}

TLFEA_API int tlfea_mesh_destroy(tlfea_mesh_t mesh) {
  if (!mesh) return TLFEA_OK;
  (void)hipSetDevice(mesh->m.device);
  (void)hipDeviceSynchronize();
  tlfea::free_mesh(mesh->m);
  delete mesh;
  return TLFEA_OK;
}

TLFEA_API int tlfea_mesh_info(tlfea_mesh_t mesh, int64_t* n_dof, int64_t* n_elem, int64_t* nnz, int32_t* n_en,
                              int32_t* n_qp) {
  if (!mesh) return TLFEA_ERR_INVALID;
  const Mesh& m = mesh->m;
  if (n_dof) *n_dof = m.n_dof;
  if (n_elem) *n_elem = m.n_elem;
  if (nnz) *nnz = m.has_pattern ? m.nnz : -1;
  if (n_en) *n_en = m.n_en;
  if (n_qp) *n_qp = m.n_qp;
  return TLFEA_OK;
}

TLFEA_API int tlfea_mesh_set_material(tlfea_mesh_t mesh, int32_t material, const double params[3], double kv_eta,
                                      double kv_lambda) {
  if (!mesh || !params) return TLFEA_ERR_INVALID;
  if (material != TLFEA_SVK && material != TLFEA_MOONEY_RIVLIN) return TLFEA_ERR_UNSUPPORTED;
  if (!tlfea::valid_material(material, params, kv_eta, kv_lambda)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  m.material = material;
  std::memcpy(m.params, params, sizeof(m.params));
  m.kv_eta = kv_eta;
  m.kv_lambda = kv_lambda;
  m.mp = tlfea::make_params(material, params, kv_eta, kv_lambda);
  ++m.generation;
  return TLFEA_OK;
}

TLFEA_API int tlfea_mesh_set_precision(tlfea_mesh_t mesh, int32_t precision) {
  if (!mesh || (precision != TLFEA_FP64 && precision != TLFEA_MIXED)) return TLFEA_ERR_INVALID;
  if (mesh->m.precision != precision) ++mesh->m.generation;
  mesh->m.precision = precision;
  return TLFEA_OK;
}

TLFEA_API int tlfea_build_csr_pattern(tlfea_mesh_t mesh, int64_t* nnz_out) {
  if (!mesh) return TLFEA_ERR_INVALID;
  if (hipSetDevice(mesh->m.device) != hipSuccess) return TLFEA_ERR_HIP;
  ++mesh->m.generation;  // the old pattern's arrays are released even when the build fails
  int rc = tlfea::build_pattern(mesh->m);
  if (rc) return rc;
  if (nnz_out) *nnz_out = mesh->m.nnz;
  return TLFEA_OK;
}

TLFEA_API int tlfea_get_csr_pattern(tlfea_mesh_t mesh, int32_t* row_offsets, int32_t* col_indices,
                                    int32_t on_device, void* stream) {
  if (!mesh || !row_offsets || (!col_indices && mesh->m.nnz > 0)) return TLFEA_ERR_INVALID;
  const Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  auto s = (hipStream_t)stream;
  if (on_device) {
    TLFEA_HIP_CHECK(hipMemcpyAsync(row_offsets, m.d_row_off, sizeof(int32_t) * (m.n_dof + 1),
                                   hipMemcpyDeviceToDevice, s));
    if (m.nnz > 0)
      TLFEA_HIP_CHECK(hipMemcpyAsync(col_indices, m.d_cols, sizeof(int32_t) * m.nnz, hipMemcpyDeviceToDevice, s));
  } else {
    TLFEA_HIP_CHECK(hipMemcpy(row_offsets, m.d_row_off, sizeof(int32_t) * (m.n_dof + 1), hipMemcpyDeviceToHost));
    if (m.nnz > 0)
      TLFEA_HIP_CHECK(hipMemcpy(col_indices, m.d_cols, sizeof(int32_t) * m.nnz, hipMemcpyDeviceToHost));
  }
  return TLFEA_OK;
}

TLFEA_API int tlfea_get_slot_map(tlfea_mesh_t mesh, int64_t elem_begin, int64_t elem_count, int32_t* slots,
                                 int32_t on_device, void* stream) {
  if (!mesh || !slots || elem_begin < 0 || elem_count < 0 || elem_begin + elem_count > mesh->m.n_elem)
    return TLFEA_ERR_INVALID;
  const Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  auto s = (hipStream_t)stream;
  if (on_device) return tlfea::export_slot_map(m, elem_begin, elem_count, slots, s);
  const size_t bytes = sizeof(int32_t) * (size_t)elem_count * 9 * m.n_en * m.n_en;
  if (bytes == 0) return TLFEA_OK;
  int32_t* tmp = nullptr;
  TLFEA_HIP_CHECK(hipMalloc(&tmp, bytes));
  int rc = tlfea::export_slot_map(m, elem_begin, elem_count, tmp, s);
  hipError_t e1 = hipStreamSynchronize(s);
  hipError_t e2 = rc ? hipSuccess : hipMemcpy(slots, tmp, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(tmp);
  if (rc) return rc;
  TLFEA_HIP_CHECK(e1);
  TLFEA_HIP_CHECK(e2);
  return TLFEA_OK;
}

namespace tlfea {
int ensure_stage(Mesh& m, size_t need) {
  if (m.stage_cap >= need) return TLFEA_OK;
  (void)hipFree(m.d_stage);  // synchronises with work that may still read it
  m.d_stage = nullptr;
  m.stage_cap = 0;
  m.staged = 0;
  TLFEA_HIP_CHECK(hipMalloc(&m.d_stage, need));
  m.stage_cap = need;
  return TLFEA_OK;
}
}  // namespace tlfea

// pass 1 of an assembly: per-point records in the mesh's work buffer
static int run_points(tlfea_mesh_t mesh, const double* q, const double* qdot, double alpha, double beta, bool want_k,
                      void* stream) {
  int rc = tlfea::check_call(mesh, q, true);
  if (rc) return rc;
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  auto s = (hipStream_t)stream;
  m.last_stream = s;
  if ((rc = tlfea::ensure_stage(m, tlfea::stage_bytes(m, want_k)))) return rc;
  tlfea::AsmArgs a = tlfea::make_args(m, q, qdot, nullptr, nullptr, alpha, beta);
  rc = tlfea::launch_points(m, a, want_k, s);
  m.staged = rc ? 0 : (want_k ? (tlfea::use_rows(m, true) ? 3 : 2) : (tlfea::use_force_blocks(m, false) ? 4 : 1));
  m.staged_precision = m.precision;
  m.staged_sym = m.staged == 2 && tlfea::point_records_sym(m, true);
  return rc;
}

// pass 2: per-node reduction of the records into f and / or the CSR values
static int run_nodes(tlfea_mesh_t mesh, double* f, double* vals, bool accumulate, void* stream) {
  if (!mesh || (!f && !vals)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (m.staged == 0 || (vals && (m.staged < 2 || m.staged > 3)) || m.staged_precision != m.precision)
    return TLFEA_ERR_INVALID;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  m.last_stream = (hipStream_t)stream;
  return tlfea::launch_nodes(m, f, vals, accumulate, (hipStream_t)stream);
}

static int run_assembly(tlfea_mesh_t mesh, const double* q, const double* qdot, double alpha, double beta,
                        double* f, double* vals, void* stream, bool accumulate = false) {
  if (!f && !vals) return TLFEA_ERR_INVALID;
  int rc = run_points(mesh, q, qdot, alpha, beta, vals != nullptr, stream);
  if (rc) return rc;
  return run_nodes(mesh, f, vals, accumulate, stream);
}

TLFEA_API int tlfea_assemble_points(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                                    double beta, int32_t want_tangent, void* stream) {
  return run_points(mesh, d_q, d_qdot, alpha, beta, want_tangent != 0, stream);
}

TLFEA_API int tlfea_assemble_nodes(tlfea_mesh_t mesh, double* d_f, double* d_vals, int32_t accumulate,
                                   void* stream) {
  return run_nodes(mesh, d_f, d_vals, accumulate != 0, stream);
}

TLFEA_API int tlfea_internal_force(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double* d_f,
                                   void* stream) {
  if (!d_f) return TLFEA_ERR_INVALID;
  return run_assembly(mesh, d_q, d_qdot, 1.0, 0.0, d_f, nullptr, stream);
}

TLFEA_API int tlfea_internal_force_noalloc(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double* d_f,
                                           void* stream) {
  int rc = tlfea::check_call(mesh, d_q, true);
  if (rc) return rc;
  if (!d_f) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  m.last_stream = (hipStream_t)stream;
  tlfea::AsmArgs a = tlfea::make_args(m, d_q, d_qdot, nullptr, nullptr, 1.0, 0.0);
  return tlfea::launch_force_noalloc(m, a, d_f, (hipStream_t)stream);
}

// A null values pointer stands for the empty output of a pattern without
// entries (a mesh without elements); otherwise the values are required.
static bool vals_given(tlfea_mesh_t mesh, const double* d_vals) {
  return d_vals || (mesh && mesh->m.has_pattern && mesh->m.nnz == 0);
}

static int run_tangent(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha, double beta,
                       double* d_vals, void* stream) {
  if (!vals_given(mesh, d_vals)) return TLFEA_ERR_INVALID;
  if (!d_vals) return tlfea::check_call(mesh, d_q, true);  // nothing to compute
  return run_assembly(mesh, d_q, d_qdot, alpha, beta, nullptr, d_vals, stream);
}

TLFEA_API int tlfea_tangent(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h, double* d_vals,
                            void* stream) {
  return run_tangent(mesh, d_q, d_qdot, h, 1.0, d_vals, stream);
}

TLFEA_API int tlfea_tangent_ex(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                               double beta, double* d_vals, void* stream) {
  return run_tangent(mesh, d_q, d_qdot, alpha, beta, d_vals, stream);
}

TLFEA_API int tlfea_assemble(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h, double* d_f,
                             double* d_vals, void* stream) {
  if (!d_f || !vals_given(mesh, d_vals)) return TLFEA_ERR_INVALID;
  return run_assembly(mesh, d_q, d_qdot, h, 1.0, d_f, d_vals, stream);
}

TLFEA_API int tlfea_assemble_ex(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                                double beta, double* d_f, double* d_vals, void* stream) {
  if (!d_f || !vals_given(mesh, d_vals)) return TLFEA_ERR_INVALID;
  return run_assembly(mesh, d_q, d_qdot, alpha, beta, d_f, d_vals, stream);
}

TLFEA_API int tlfea_assemble_accumulate(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                                        double beta, double* d_f, double* d_vals, void* stream) {
  return run_assembly(mesh, d_q, d_qdot, alpha, beta, d_f, d_vals, stream, true);
}

TLFEA_API int tlfea_internal_force_vjp(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot,
                                       const double* d_w, double* d_gq, double* d_gqdot, double* d_gparam,
                                       void* stream) {
  int rc = tlfea::check_call(mesh, d_q, false);
  if (rc) return rc;
  if (!d_w || (!d_gq && !d_gqdot && !d_gparam)) return TLFEA_ERR_INVALID;
  if (!mesh->m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  mesh->m.last_stream = (hipStream_t)stream;
  return tlfea::launch_vjp(mesh->m, d_q, d_qdot, d_w, d_gq, d_gqdot, d_gparam, (hipStream_t)stream);
}

TLFEA_API int tlfea_internal_force_p(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot,
                                     const double* d_params, double* d_f, void* stream) {
  int rc = tlfea::check_call(mesh, d_q, true);
  if (rc) return rc;
  if (!d_params || !d_f) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  auto s = (hipStream_t)stream;
  m.last_stream = s;
  if ((rc = tlfea::launch_params(m, d_params, s))) return rc;
  tlfea::AsmArgs a = tlfea::make_args(m, d_q, d_qdot, nullptr, nullptr, 1.0, 0.0);
  a.mp_dev = m.d_mp;
  return tlfea::launch_force_blocks(m, a, d_f, s);
}

TLFEA_API int tlfea_internal_force_vjp_p(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot,
                                         const double* d_params, const double* d_w, double* d_gq, double* d_gqdot,
                                         double* d_gparam, void* stream) {
  int rc = tlfea::check_call(mesh, d_q, true);
  if (rc) return rc;
  if (!d_params || !d_w || (!d_gq && !d_gqdot && !d_gparam)) return TLFEA_ERR_INVALID;
  mesh->m.last_stream = (hipStream_t)stream;
  return tlfea::launch_vjp(mesh->m, d_q, d_qdot, d_w, d_gq, d_gqdot, d_gparam, (hipStream_t)stream, d_params);
}

TLFEA_API int tlfea_get_runtime_flags(tlfea_mesh_t mesh, uint32_t* flags) {
  if (!mesh || !flags) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  TLFEA_HIP_CHECK(hipStreamSynchronize(m.last_stream));
  TLFEA_HIP_CHECK(hipMemcpy(flags, m.d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost));
  TLFEA_HIP_CHECK(hipMemset(m.d_flags, 0, sizeof(uint32_t)));
  return TLFEA_OK;
}

static tlfea::GatherTuning shape_in(const tlfea_gather_shape& s) {
  return tlfea::GatherTuning{s.waves, s.range_tasks, s.range_values};
}

static void shape_out(const tlfea::GatherTuning& t, tlfea_gather_shape* s) {
  if (!s) return;
  s->waves = t.waves;
  s->range_tasks = t.range_tasks;
  s->range_values = t.range_values;
}

TLFEA_API int tlfea_mesh_set_gather_shape(tlfea_mesh_t mesh, const tlfea_gather_shape* shape) {
  if (!mesh || !shape) return TLFEA_ERR_INVALID;
  return tlfea::set_gather_shape(mesh->m, shape_in(*shape));
}

TLFEA_API int tlfea_mesh_get_gather_shape(tlfea_mesh_t mesh, tlfea_gather_shape* shape, int64_t* n_ranges) {
  if (!mesh || (!shape && !n_ranges)) return TLFEA_ERR_INVALID;
  if (!mesh->m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  shape_out(mesh->m.tune, shape);
  if (n_ranges) *n_ranges = mesh->m.n_ranges;
  return TLFEA_OK;
}

TLFEA_API int tlfea_mesh_autotune(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                                  double* d_f, double* d_vals, int32_t reps, void* stream,
                                  tlfea_gather_shape* chosen, float* ms_per_call) {
  int rc = tlfea::check_call(mesh, d_q, true);
  if (rc) return rc;
  if (!d_f || !d_vals || !std::isfinite(h)) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  const tlfea::GatherTuning current = m.tune;
  tlfea::GatherTuning best = current;
  float ms = 0.0f;
  rc = tlfea::autotune_shape(
      current, [&](const tlfea::GatherTuning& t) { return tlfea::set_gather_shape(m, t); },
      [&]() { return run_assembly(mesh, d_q, d_qdot, h, 1.0, d_f, d_vals, stream); }, reps,
      (hipStream_t)stream, best, ms);
  if (rc) return rc;
  shape_out(best, chosen);
  if (ms_per_call) *ms_per_call = ms;
  return TLFEA_OK;
}

TLFEA_API int tlfea_build_upper_pattern(tlfea_mesh_t mesh, int64_t* nnz_upper) {
  if (!mesh) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  const int rc = tlfea::build_upper_pattern(m);
  if (!rc && nnz_upper) *nnz_upper = m.nnz_u;
  return rc;
}

TLFEA_API int tlfea_get_csr_pattern_upper(tlfea_mesh_t mesh, int32_t* row_offsets, int32_t* col_indices,
                                          int32_t on_device, void* stream) {
  if (!mesh || !row_offsets) return TLFEA_ERR_INVALID;
  const Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (!m.d_row_off_u) return TLFEA_ERR_INVALID;
  if (!col_indices && m.nnz_u > 0) return TLFEA_ERR_INVALID;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  const auto kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (on_device) {
    TLFEA_HIP_CHECK(hipMemcpyAsync(row_offsets, m.d_row_off_u, sizeof(int32_t) * (m.n_dof + 1), kind,
                                   (hipStream_t)stream));
    if (m.nnz_u > 0)
      TLFEA_HIP_CHECK(hipMemcpyAsync(col_indices, m.d_cols_u, sizeof(int32_t) * m.nnz_u, kind, (hipStream_t)stream));
  } else {
    TLFEA_HIP_CHECK(hipMemcpy(row_offsets, m.d_row_off_u, sizeof(int32_t) * (m.n_dof + 1), kind));
    if (m.nnz_u > 0) TLFEA_HIP_CHECK(hipMemcpy(col_indices, m.d_cols_u, sizeof(int32_t) * m.nnz_u, kind));
  }
  return TLFEA_OK;
}

TLFEA_API int tlfea_assemble_upper(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                                   double beta, double* d_f, double* d_vals_upper, void* stream) {
  if (!mesh || !d_vals_upper) return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (!m.d_row_off_u) return TLFEA_ERR_INVALID;
  // dP/dF of the hyperelastic laws is symmetric; the Kelvin-Voigt part is not
  if (m.kv_eta != 0.0 || m.kv_lambda != 0.0) return TLFEA_ERR_UNSUPPORTED;
  int rc = run_points(mesh, d_q, d_qdot, alpha, beta, true, stream);
  if (rc) return rc;
  tlfea::GatherOptions opt;
  opt.row_off_u = m.d_row_off_u;
  return tlfea::launch_nodes(m, d_f, d_vals_upper, false, (hipStream_t)stream, opt);
}

