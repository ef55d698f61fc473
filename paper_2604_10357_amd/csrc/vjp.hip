// vjp.hip -- reverse-mode products of the internal force for autograd.
//
// For a cotangent w the library returns, without forming K:
//   gq     = (df/dq)^T w     : per point Z_kL = sum_iJ W_iJ dP_iJ/dF_kL with
//                              W = sum_a w_a (x) g_a, then gq_b = sum dV Z g_b
//   gqdot  = (df/dqdot)^T w  : the same with dP/dFdot
//   gparam = d(w . f)/dtheta : P is linear in every material constant, so the
//                              partial is sum dV W : P_i with P_i the stress per
//                              unit constant; SVK (E, nu) follow by the chain
//                              rule through the Lame constants.
// f itself follows Sec. 4.3 (Eqs. F_assembly, fint_local) of the paper; the
// VJP is the transpose of the Sec. 4.4.2 tangent (Eq. tangent_block) applied
// element by element.  Runs in float64.
//
// Shaped like the force-only path: one workgroup holds whole elements, their
// nodal values (u, qdot, w) go to LDS once, gathered in one pass, a lane per
// point runs one reverse-mode stress product (stress_vjp) for the products and
// the parameter parts, the points' Zhat = dV Z J0^-T stay in LDS, and a lane
// per (element, coefficient) sums them against the parent gradients into one
// block per incidence.  The qdot product is formed only when it is asked for.
// The per-node sums then run in a fixed order (the force path's pass 2), and
// the parameter partials are reduced per workgroup and then in a fixed order:
// repeated calls give the same bits.
#include "kernel_common.h"

namespace tlfea {
namespace {

constexpr int kVjpThreads = 256;
template <class Rule>
constexpr int vjp_elems() { return kVjpThreads / Rule::NQ; }

// QD: the qdot product is formed too (bqd non-null)
template <class Rule, bool QD>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_elem(AsmArgs a, const double* __restrict__ w,
                                                         const int32_t* __restrict__ incpos, double* __restrict__ bq,
                                                         double* __restrict__ bqd, double* __restrict__ gpart) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN, MC = Rule::MC, EB = vjp_elems<Rule>();
  constexpr int ZS = QD ? 18 : 9;  // LDS values per point: Zhat of q, then of qdot
  constexpr size_t NOD = (size_t)EB * NEN * 9 * sizeof(double), ZB = (size_t)EB * NQ * ZS * sizeof(double);
  __shared__ __align__(16) unsigned char smem[NOD > ZB ? NOD : ZB];
  __shared__ double dn[NQ * NEN * 3];  // unit-scaled parent gradients, dN_a(q)_m at 3 (NEN q + a) + m
  __shared__ double red[kVjpThreads / 64][5];
  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * EB;
  const int ne = (int)(a.n_elem - e0 < EB ? a.n_elem - e0 : EB);
  double* nod = reinterpret_cast<double*>(smem);  // 6 per coefficient (u, qdot)
  double* wn = nod + EB * NEN * 6;                // 3 per coefficient (w)
  // u = q - X, qdot and w of every (element, coefficient), all loads of one
  // coefficient issued together
  for (int idx = tid; idx < ne * NEN; idx += kVjpThreads) {
    const int le = idx / NEN, al = idx - le * NEN;
    const int64_t c = coef_of<Rule>(a.conn + (e0 + le) * NPN, al);
    double v[12];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = a.q[3 * c + i];
      v[3 + i] = a.X[3 * c + i];
      v[6 + i] = a.qdot ? a.qdot[3 * c + i] : 0.0;
      v[9 + i] = w[3 * c + i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      nod[6 * idx + i] = v[i] - v[3 + i];
      nod[6 * idx + 3 + i] = v[6 + i];
      wn[3 * idx + i] = v[9 + i];
    }
  }
  for (int idx = tid; idx < NQ * NEN * 3; idx += kVjpThreads) {
    const int q = idx / (3 * NEN), r = idx - 3 * NEN * q;
    dn[idx] = Rule::dN_rt(q, r / 3, r % 3);
  }
  __syncthreads();
  const bool act = tid < ne * NQ;
  const int pl = act ? tid : 0;  // idle lanes evaluate point 0 and store nothing
  const int el = pl / NQ, q = pl - el * NQ;
  double Jinv[9], det, Hd[9], Fd[9], Wg[9];
  tile_kinematics<Rule, true>(a, nod + 6 * NEN * el, e0 + el, q, Jinv, det, Hd, Fd);
  {
    // W = sum_a w_a (x) g_a, the first position coefficient's value taken out
    // of every position coefficient (the position gradients sum to zero)
    double sc[4], D[9];
    element_scales<Rule>(a, e0 + el, sc);
    const double* we = wn + 3 * NEN * el;
    const double r0[3] = {we[0], we[1], we[2]};
#pragma unroll
    for (int t = 0; t < 9; ++t) D[t] = 0.0;
    for (int al = 0; al < NEN; ++al) {
      const double s = sc[al % 4];
      const bool position = MC == 1 || (al & 3) == 0;
      const double* d = dn + 3 * (NEN * q + al);
      const double w0 = d[0] * s, w1 = d[1] * s, w2 = d[2] * s;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double v = we[3 * al + i] - (position ? r0[i] : 0.0);
        D[3 * i] += v * w0;
        D[3 * i + 1] += v * w1;
        D[3 * i + 2] += v * w2;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int J = 0; J < 3; ++J)
        Wg[3 * i + J] = D[3 * i] * Jinv[J] + D[3 * i + 1] * Jinv[3 + J] + D[3 * i + 2] * Jinv[6 + J];
  }
  __syncthreads();  // the nodal values are consumed: the LDS holds Zhat from here on
  const double dV = det * Rule::w_rt(q);
  double Zq[9], Zd[9], part[5];
  stress_vjp(launch_material(a), Hd, Fd, Wg, Zq, Zd, part);
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    Zq[t] *= dV;
    Zd[t] *= dV;
  }
#pragma unroll
  for (int th = 0; th < 5; ++th) part[th] = act ? dV * part[th] : 0.0;
  double* zr = reinterpret_cast<double*>(smem);  // Zhat of q at ZS p, of qdot at ZS p + 9
  if (act) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        zr[ZS * pl + 3 * k + m] = Zq[3 * k] * Jinv[3 * m] + Zq[3 * k + 1] * Jinv[3 * m + 1] + Zq[3 * k + 2] * Jinv[3 * m + 2];
        if constexpr (QD)
          zr[ZS * pl + 9 + 3 * k + m] =
              Zd[3 * k] * Jinv[3 * m] + Zd[3 * k + 1] * Jinv[3 * m + 1] + Zd[3 * k + 2] * Jinv[3 * m + 2];
      }
  }
  // workgroup sums of the five partials, in a fixed order
  if (gpart) {
#pragma unroll
    for (int th = 0; th < 5; ++th) {
      double v = part[th];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) red[tid >> 6][th] = v;
    }
  }
  __syncthreads();
  if (gpart && tid < 5) {
    double v = 0.0;
    for (int wv = 0; wv < kVjpThreads / 64; ++wv) v += red[wv][tid];
    gpart[5 * (int64_t)blockIdx.x + tid] = v;
  }
  for (int t = tid; t < ne * NEN; t += kVjpThreads) {
    const int le = t / NEN, al = t - le * NEN;
    double g[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int qq = 0; qq < NQ; ++qq) {
      const double* z = zr + ZS * (le * NQ + qq);
      const double* d = dn + 3 * (NEN * qq + al);
      const double d0 = d[0], d1 = d[1], d2 = d[2];
#pragma unroll
      for (int h = 0; h < (QD ? 2 : 1); ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) g[h][k] += z[9 * h + 3 * k] * d0 + z[9 * h + 3 * k + 1] * d1 + z[9 * h + 3 * k + 2] * d2;
    }
    double sc[4];
    element_scales<Rule>(a, e0 + le, sc);
    const double s = sc[al % 4];
    const int64_t pos = incpos[(e0 + le) * NPN + al / MC];
    double* oq = bq + pos * (3 * MC) + 3 * (al % MC);
#pragma unroll
    for (int k = 0; k < 3; ++k) oq[k] = g[0][k] * s;
    if constexpr (QD) {
      double* od = bqd + pos * (3 * MC) + 3 * (al % MC);
#pragma unroll
      for (int k = 0; k < 3; ++k) od[k] = g[1][k] * s;
    }
  }
}

// internal partials (c0, c1, c2, eta, lam_v), summed over the workgroups in a
// fixed order, -> user parameters.  The partials lie flat, five per workgroup;
// lane t of kFinGroups * 5 sums every kFinGroups * 5-th value from t on (one
// parameter each, four loads in flight), then a tree over the groups.
constexpr int kFinGroups = 204, kFinThreads = 1024, kFinTree = 256;
__global__ __launch_bounds__(kFinThreads) void k_vjp_finalize(const double* __restrict__ gpart, int64_t n_blocks,
                                                              int kind, double E, double nu,
                                                              const double* __restrict__ d_params, double* gparam) {
  constexpr int S = 5 * kFinGroups;
  __shared__ double red[kFinTree][5];
  const int t = threadIdx.x;
  const int64_t n = 5 * n_blocks;
  double s = 0.0;
  if (t < S) {
    int64_t i = t;
    for (; i + 3 * S < n; i += 4 * S) {
      const double v0 = gpart[i], v1 = gpart[i + S], v2 = gpart[i + 2 * S], v3 = gpart[i + 3 * S];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; i < n; i += S) s += gpart[i];
  }
  for (int k = t; k < 5 * kFinTree; k += kFinThreads) red[k / 5][k % 5] = k == t ? s : 0.0;  // zero past S
  __syncthreads();
  for (int half = kFinTree / 2; half > 0; half >>= 1) {
    if (t < 5 * half) red[t / 5][t % 5] += red[t / 5 + half][t % 5];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double* g = red[0];
  if (d_params) {
    E = d_params[0];
    nu = d_params[1];
  }
  if (kind == 1) {
    const double dlam_dE = nu / ((1 + nu) * (1 - 2 * nu)), dmu_dE = 1.0 / (2 * (1 + nu));
    const double dlam_dnu = E * (1 + 2 * nu * nu) / ((1 + nu) * (1 + nu) * (1 - 2 * nu) * (1 - 2 * nu));
    const double dmu_dnu = -E / (2 * (1 + nu) * (1 + nu));
    gparam[0] = dlam_dE * g[0] + dmu_dE * g[1];
    gparam[1] = dlam_dnu * g[0] + dmu_dnu * g[1];
    gparam[2] = 0.0;
  } else {
    gparam[0] = g[0];
    gparam[1] = g[1];
    gparam[2] = g[2];
  }
  gparam[3] = g[3];
  gparam[4] = g[4];
}

template <class Rule>
int64_t vjp_blocks(int64_t n_elem) {
  return (n_elem + vjp_elems<Rule>() - 1) / vjp_elems<Rule>();
}

template <class Rule>
int launch_vjp_elem(const AsmArgs& a, const double* w, const int32_t* incpos, double* bq, double* bqd,
                    double* gpart, hipStream_t s) {
  const int64_t blocks = vjp_blocks<Rule>(a.n_elem);
  if (blocks > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  if (blocks > 0) {
    if (bqd)
      hipLaunchKernelGGL((k_vjp_elem<Rule, true>), dim3((unsigned)blocks), dim3(kVjpThreads), 0, s, a, w, incpos, bq,
                         bqd, gpart);
    else
      hipLaunchKernelGGL((k_vjp_elem<Rule, false>), dim3((unsigned)blocks), dim3(kVjpThreads), 0, s, a, w, incpos,
                         bq, bqd, gpart);
  }
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

}  // namespace

int launch_vjp(Mesh& m, const double* q, const double* qdot, const double* w, double* gq, double* gqdot,
               double* gparam, hipStream_t s, const double* d_params) {
  if (!m.d_incpos) return TLFEA_ERR_NO_PATTERN;
  AsmArgs a = make_args(m, q, qdot, nullptr, nullptr, 1.0, 0.0);
  if (d_params) {
    if (int rc = launch_params(m, d_params, s)) return rc;
    a.mp_dev = m.d_mp;
  }
  int64_t blocks;
  if (m.elem_type == TLFEA_T10) blocks = vjp_blocks<RuleT10>(m.n_elem);
  else if (m.elem_type == TLFEA_ANCF3243) blocks = vjp_blocks<RuleBeam>(m.n_elem);
  else if (m.gl[0] == 3) blocks = vjp_blocks<RuleAncf<3, 3, 2>>(m.n_elem);
  else blocks = vjp_blocks<RuleAncf<4, 4, 3>>(m.n_elem);
  // the mesh's work buffer: the q blocks (always formed), the qdot blocks and the
  // per-workgroup partials; it no longer holds assembly records afterwards
  const size_t set = (size_t)m.n_elem * m.n_pn * 3 * m.mc;  // doubles per block set
  const size_t need = sizeof(double) * (set * (gqdot ? 2 : 1) + 5 * (size_t)blocks + 1);
  int rc;
  if ((rc = ensure_stage(m, need))) return rc;
  m.staged = 0;
  double* bq = (double*)m.d_stage;
  double* bqd = gqdot ? bq + set : nullptr;
  double* gpart = gparam ? bq + set * (gqdot ? 2 : 1) : nullptr;
  if (m.elem_type == TLFEA_T10) rc = launch_vjp_elem<RuleT10>(a, w, m.d_incpos, bq, bqd, gpart, s);
  else if (m.elem_type == TLFEA_ANCF3243) rc = launch_vjp_elem<RuleBeam>(a, w, m.d_incpos, bq, bqd, gpart, s);
  else if (m.gl[0] == 3) rc = launch_vjp_elem<RuleAncf<3, 3, 2>>(a, w, m.d_incpos, bq, bqd, gpart, s);
  else rc = launch_vjp_elem<RuleAncf<4, 4, 3>>(a, w, m.d_incpos, bq, bqd, gpart, s);
  if (rc) return rc;
  if (gq && (rc = launch_block_sum(m, bq, gq, s))) return rc;
  if (gqdot && (rc = launch_block_sum(m, bqd, gqdot, s))) return rc;
  if (gparam) {
    hipLaunchKernelGGL(k_vjp_finalize, dim3(1), dim3(kFinThreads), 0, s, gpart, blocks, m.material, m.params[0],
                       m.params[1], d_params, gparam);
    TLFEA_HIP_CHECK(hipGetLastError());
  }
  return TLFEA_OK;
}

}  // namespace tlfea
