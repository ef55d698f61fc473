// vjp.hip -- reverse-mode products of the internal force for autograd.
//
// For a cotangent w the library returns, without forming K:
//   gq     = (df/dq)^T w     : per point Z_kL = sum_iJ W_iJ dP_iJ/dF_kL with
//                              W = sum_a w_a (x) g_a, then gq_b = sum dV Z g_b
//   gqdot  = (df/dqdot)^T w  : the same with dP/dFdot
//   gparam = d(w . f)/dtheta : P is linear in every material constant, so the
//                              partial is dV W : P(theta = e_i), reduced over
//                              the grid; SVK (E, nu) follow by the chain rule
//                              through the Lame constants.
// f itself follows Sec. 4.3 (Eqs. F_assembly, fint_local) of the paper; the
// VJP is the transpose of the Sec. 4.4.2 tangent (Eq. tangent_block) applied
// element by element.  Runs in float64.
//
// The per-node sums have exactly the form of f_int with the stress replaced by
// Z: pass 1 (k_vjp_stage, one lane per element x point) stores
// Zhat = dV Z J0^-T as a force-type record, and pass 2 is the force gather of
// the assembly (per node range, LDS sums, plain stores; no global atomics).
#include "kernel_common.h"

namespace tlfea {
namespace {

constexpr int kVjpThreads = 256;
constexpr int kZRec = 12;  // force-type record: Zhat_km at 4 k + m

template <class Rule>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_stage(AsmArgs a, const double* w, double* zq, double* zqd,
                                                          double* gacc) {
  constexpr int NQ = Rule::NQ;
  __shared__ double red[kVjpThreads / 64][5];
  const int64_t p = (int64_t)blockIdx.x * kVjpThreads + threadIdx.x;
  double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (p < a.n_elem * NQ) {
    const int64_t ge = p / NQ;
    const int q = (int)(p % NQ);
    double Hd[9], Fd[9], Jinv[9], det, sc[4], Wg[9];
    load_kinematics<Rule>(a, ge, q, Hd, Fd, Jinv, det);
    element_scales<Rule>(a, ge, sc);
    field_gradient<Rule>(a, ge, q, sc, w, nullptr, Jinv, Wg);
    const double dV = det * Rule::w_rt(q);
    for (int pass = 0; pass < 2; ++pass) {
      double* out = pass == 0 ? zq : zqd;
      if (!out) continue;
      PointOut<double> o;
      (void)point_update<double, true>(a.mp, Hd, Fd, dV, pass == 0 ? 1.0 : 0.0, pass == 0 ? 0.0 : 1.0, o);
      double Z[9];
      cotangent_contract(o, Wg, Z);
      // parent-coordinate form Z J0^-T, rows padded to 4
      double* rec = out + p * kZRec;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
          rec[4 * k + m] = Z[3 * k] * Jinv[3 * m] + Z[3 * k + 1] * Jinv[3 * m + 1] + Z[3 * k + 2] * Jinv[3 * m + 2];
        rec[4 * k + 3] = 0.0;
      }
    }
    if (gacc) {
      for (int th = 0; th < 5; ++th) {
        if (th == 2 && a.mp.kind == 1) continue;
        MatParams u{};
        u.kind = a.mp.kind;
        if (th == 0) u.c0 = 1.0;
        if (th == 1) u.c1 = 1.0;
        if (th == 2) u.c2 = 1.0;
        if (th == 3) u.eta = 1.0;
        if (th == 4) u.lam_v = 1.0;
        PointOut<double> o;
        (void)point_update<double, false>(u, Hd, Fd, dV, 1.0, 0.0, o);
        double c = 0.0;
#pragma unroll
        for (int t = 0; t < 9; ++t) c += Wg[t] * o.P[t];
        part[th] = c;
      }
    }
  }
  if (!gacc) return;
  // workgroup sums of the five partials: one float64 atomic per partial and workgroup
#pragma unroll
  for (int th = 0; th < 5; ++th) {
    double v = part[th];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][th] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double v = 0.0;
    for (int wv = 0; wv < kVjpThreads / 64; ++wv) v += red[wv][threadIdx.x];
    atomicAdd(gacc + threadIdx.x, v);
  }
}

__global__ void k_zero5(double* p) {
  if (threadIdx.x < 5) p[threadIdx.x] = 0.0;
}

// internal partials (c0, c1, c2, eta, lam_v) -> user parameters
__global__ void k_vjp_finalize(const double* gacc, int kind, double E, double nu, double* gparam) {
  if (threadIdx.x != 0) return;
  if (kind == 1) {
    const double dlam_dE = nu / ((1 + nu) * (1 - 2 * nu)), dmu_dE = 1.0 / (2 * (1 + nu));
    const double dlam_dnu = E * (1 + 2 * nu * nu) / ((1 + nu) * (1 + nu) * (1 - 2 * nu) * (1 - 2 * nu));
    const double dmu_dnu = -E / (2 * (1 + nu) * (1 + nu));
    gparam[0] = dlam_dE * gacc[0] + dmu_dE * gacc[1];
    gparam[1] = dlam_dnu * gacc[0] + dmu_dnu * gacc[1];
    gparam[2] = 0.0;
  } else {
    gparam[0] = gacc[0];
    gparam[1] = gacc[1];
    gparam[2] = gacc[2];
  }
  gparam[3] = gacc[3];
  gparam[4] = gacc[4];
}

template <class Rule>
int launch_vjp_stage(const AsmArgs& a, const double* w, double* zq, double* zqd, double* gacc, hipStream_t s) {
  const int64_t npts = a.n_elem * Rule::NQ;
  const int64_t blocks = (npts + kVjpThreads - 1) / kVjpThreads;
  if (blocks > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  if (blocks > 0)
    hipLaunchKernelGGL((k_vjp_stage<Rule>), dim3((unsigned)blocks), dim3(kVjpThreads), 0, s, a, w, zq, zqd, gacc);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

}  // namespace

int launch_vjp(Mesh& m, const double* q, const double* qdot, const double* w, double* gq, double* gqdot,
               double* gparam, hipStream_t s) {
  AsmArgs a = make_args(m, q, qdot, nullptr, nullptr, 1.0, 0.0);
  int rc;
  const size_t set = (size_t)m.n_elem * m.n_qp * kZRec * sizeof(double);
  // the Zhat records live in the mesh's work buffer: it no longer holds assembly records
  if ((gq || gqdot) && (rc = ensure_stage(m, set * ((gq ? 1 : 0) + (gqdot ? 1 : 0))))) return rc;
  m.staged = 0;
  double* zq = gq ? (double*)m.d_stage : nullptr;
  double* zqd = gqdot ? (double*)m.d_stage + (gq ? set / sizeof(double) : 0) : nullptr;
  double* gacc = gparam ? m.d_vjp_acc : nullptr;
  if (gacc) {
    hipLaunchKernelGGL(k_zero5, dim3(1), dim3(64), 0, s, gacc);
    TLFEA_HIP_CHECK(hipGetLastError());
  }
  if (m.elem_type == TLFEA_T10) rc = launch_vjp_stage<RuleT10>(a, w, zq, zqd, gacc, s);
  else if (m.elem_type == TLFEA_ANCF3243) rc = launch_vjp_stage<RuleBeam>(a, w, zq, zqd, gacc, s);
  else if (m.gl[0] == 3) rc = launch_vjp_stage<RuleAncf<3, 3, 2>>(a, w, zq, zqd, gacc, s);
  else rc = launch_vjp_stage<RuleAncf<4, 4, 3>>(a, w, zq, zqd, gacc, s);
  if (rc) return rc;
  if (gq && (rc = launch_force_gather_f64(m, zq, gq, s))) return rc;
  if (gqdot && (rc = launch_force_gather_f64(m, zqd, gqdot, s))) return rc;
  if (gparam) {
    hipLaunchKernelGGL(k_vjp_finalize, dim3(1), dim3(64), 0, s, gacc, m.material, m.params[0], m.params[1], gparam);
    TLFEA_HIP_CHECK(hipGetLastError());
  }
  return TLFEA_OK;
}

}  // namespace tlfea
