// vjp.hip -- reverse-mode products of the internal force for autograd.
//
// For a cotangent w the kernel returns, without forming K:
//   gq     = (df/dq)^T w     : per point Z_kL = sum_iJ W_iJ dP_iJ/dF_kL with
//                              W = sum_a w_a (x) g_a, then gq_b += dV Z g_b
//   gqdot  = (df/dqdot)^T w  : the same with dP/dFdot
//   gparam = d(w . f)/dtheta : P is linear in every material constant, so the
//                              partial is dV W : P(theta = e_i), reduced over
//                              the grid; SVK (E, nu) follow by the chain rule
//                              through the Lame constants.
// f itself follows Sec. 4.3 (Eqs. F_assembly, fint_local) of the paper; the
// VJP is the transpose of the Sec. 4.4.2 tangent (Eq. tangent_block) applied
// element by element.  Runs in float64.
#include "kernel_common.h"

namespace tlfea {
namespace {

template <class Rule, int TE>
__global__ __launch_bounds__(64) void k_vjp(AsmArgs a, const double* w, double* gq, double* gqd, double* gacc) {
  constexpr int NEN = Rule::NEN, NQ = Rule::NQ;
  __shared__ double lds[TE * NQ * 24];
  __shared__ double red[5];
  const int lane = threadIdx.x;
  const int tile = remap_tile(blockIdx.x, gridDim.x);
  const int64_t e0 = (int64_t)tile * TE;
  if (lane < 5) red[lane] = 0.0;
  __syncthreads();
  for (int p = lane; p < TE * NQ; p += 64) {
    const int el = p / NQ, q = p % NQ;
    const int64_t ge = e0 + el;
    if (ge >= a.n_elem) continue;
    double Hd[9], Fd[9], Jinv[9], det, sc[4], Wg[9];
    load_kinematics<Rule>(a, ge, q, Hd, Fd, Jinv, det);
    element_scales<Rule>(a, ge, sc);
    field_gradient<Rule>(a, ge, q, sc, w, nullptr, Jinv, Wg);
    const double dV = det * Rule::w_rt(q);
    double* s = lds + p * 24;
    for (int pass = 0; pass < 2; ++pass) {
      if ((pass == 0 && !gq) || (pass == 1 && !gqd)) continue;
      PointOut<double> o;
      (void)point_update<double, true>(a.mp, Hd, Fd, dV, pass == 0 ? 1.0 : 0.0, pass == 0 ? 0.0 : 1.0, o);
      double Z[9];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int L = 0; L < 3; ++L) {
          double z = 0.0;
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int J = 0; J < 3; ++J) z += Wg[3 * i + J] * tangent_entry(o, i, J, k, L);
          Z[3 * k + L] = z;
        }
      // parent-coordinate form Z J0^-T, rows padded to 4
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m)
          s[12 * pass + 4 * k + m] = Z[3 * k] * Jinv[3 * m] + Z[3 * k + 1] * Jinv[3 * m + 1] + Z[3 * k + 2] * Jinv[3 * m + 2];
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
        atomicAdd(&red[th], c);
      }
    }
  }
  __syncthreads();
  for (int t = lane; t < TE * NEN; t += 64) {
    const int el = t / NEN, al = t % NEN;
    const int64_t ge = e0 + el;
    if (ge >= a.n_elem) continue;
    double scd[4];
    element_scales<Rule>(a, ge, scd);
    const int64_t c = coef_of<Rule>(a.conn + ge * Rule::NPN, al);
    for (int pass = 0; pass < 2; ++pass) {
      double* out = pass == 0 ? gq : gqd;
      if (!out) continue;
      double g0 = 0.0, g1 = 0.0, g2 = 0.0;
      sfor<0, NQ>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        const double* s = lds + (el * NQ + q) * 24 + 12 * pass;
        const double d0 = Rule::dN_rt(q, al, 0), d1 = Rule::dN_rt(q, al, 1), d2 = Rule::dN_rt(q, al, 2);
        g0 += s[0] * d0 + s[1] * d1 + s[2] * d2;
        g1 += s[4] * d0 + s[5] * d1 + s[6] * d2;
        g2 += s[8] * d0 + s[9] * d1 + s[10] * d2;
      });
      const double sa = scd[al % 4];
      unsafeAtomicAdd(out + 3 * c, g0 * sa);
      unsafeAtomicAdd(out + 3 * c + 1, g1 * sa);
      unsafeAtomicAdd(out + 3 * c + 2, g2 * sa);
    }
  }
  if (gacc && lane < 5) unsafeAtomicAdd(gacc + lane, red[lane]);
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

template <class Rule, int TE>
int launch_vjp_rule(const AsmArgs& a0, const double* w, double* gq, double* gqd, double* gacc, hipStream_t s) {
  AsmArgs a = a0;
  const int64_t tiles = (a.n_elem + TE - 1) / TE;
  if (tiles > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  a.n_tiles = (int)tiles;
  if (tiles > 0) hipLaunchKernelGGL((k_vjp<Rule, TE>), dim3(a.n_tiles), dim3(64), 0, s, a, w, gq, gqd, gacc);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

}  // namespace

int launch_vjp(const Mesh& m, const double* q, const double* qdot, const double* w, double* gq, double* gqdot,
               double* gparam, hipStream_t s) {
  AsmArgs a = make_args(m, q, qdot, nullptr, nullptr, 1.0, 0.0);
  int rc;
  if (gq && (rc = launch_zero(gq, m.n_dof, s))) return rc;
  if (gqdot && (rc = launch_zero(gqdot, m.n_dof, s))) return rc;
  double* gacc = gparam ? m.d_vjp_acc : nullptr;
  if (gacc) {
    hipLaunchKernelGGL(k_zero5, dim3(1), dim3(64), 0, s, gacc);
    TLFEA_HIP_CHECK(hipGetLastError());
  }
  if (m.elem_type == TLFEA_T10) rc = launch_vjp_rule<RuleT10, 12>(a, w, gq, gqdot, gacc, s);
  else if (m.gl[0] == 3) rc = launch_vjp_rule<RuleAncf<3, 3, 2>, 3>(a, w, gq, gqdot, gacc, s);
  else rc = launch_vjp_rule<RuleAncf<4, 4, 3>, 1>(a, w, gq, gqdot, gacc, s);
  if (rc) return rc;
  if (gparam) {
    hipLaunchKernelGGL(k_vjp_finalize, dim3(1), dim3(64), 0, s, gacc, m.material, m.params[0], m.params[1], gparam);
    TLFEA_HIP_CHECK(hipGetLastError());
  }
  return TLFEA_OK;
}

}  // namespace tlfea
