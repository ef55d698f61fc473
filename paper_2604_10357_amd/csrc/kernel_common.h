// kernel_common.h -- device helpers shared by the element kernels: tile
// remapping, coefficient lookup, reference geometry and field gradients.
#pragma once

#include "rules.h"
#include "tlfea_internal.h"

namespace tlfea {
namespace {

// Workgroup b is dispatched to XCD b % 8; hand each XCD a contiguous tile range
// so the CSR rows a tile touches are shared with its neighbours in one L2.
__device__ __forceinline__ int remap_tile(int bid, int nblocks) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nblocks >> 3, extra = nblocks & 7;
  return xcd * per + (xcd < extra ? xcd : extra) + idx;
}

template <class Rule>
__device__ __forceinline__ int64_t coef_of(const int32_t* conn_e, int a) {
  if constexpr (Rule::MC == 1) return conn_e[a];
  else return 4 * (int64_t)conn_e[a >> 2] + (a & 3);
}

// element scale of each coefficient kind (ANCF: 1, lx/2, ly/2, H/2; T10: 1)
template <class Rule>
__device__ __forceinline__ void element_scales(const AsmArgs& a, int64_t ge, double* sc) {
  if constexpr (Rule::MC == 1) {
    sc[0] = sc[1] = sc[2] = sc[3] = 1.0;
  } else {
    sc[0] = 1.0;
    sc[1] = a.escale[2 * ge];
    sc[2] = a.escale[2 * ge + 1];
    sc[3] = a.half_h;
  }
}

template <class Rule>
__device__ __forceinline__ void load_geometry(const AsmArgs& a, int64_t ge, int q, double* Jinv, double& det) {
  const double* rec = a.geo + 10 * (a.affine ? ge : ge * Rule::NQ + q);
#pragma unroll
  for (int t = 0; t < 9; ++t) Jinv[t] = rec[t];
  det = rec[9];
}

// Gradient  sum_a (u_a - X_a) (x) g_a  (X may be null) of a nodal field u at point q.
// Formed as (sum_a u_a (x) dN_a) J0^-1: parent gradient first, then one 3x3 product.
// The gradients of the position functions sum to zero, so the value at the
// element's first coefficient is taken out of every position coefficient: the
// terms stay of the size of the element's own variation of the field.
template <class Rule>
__device__ __forceinline__ void field_gradient(const AsmArgs& a, int64_t ge, int q, const double* sc,
                                               const double* u, const double* X, const double* Jinv,
                                               double* out) {
  const int32_t* conn_e = a.conn + ge * Rule::NPN;
  double D[9], r0[3];
#pragma unroll
  for (int t = 0; t < 9; ++t) D[t] = 0.0;
  {
    const int64_t c0 = coef_of<Rule>(conn_e, 0);
#pragma unroll
    for (int i = 0; i < 3; ++i) r0[i] = X ? u[3 * c0 + i] - X[3 * c0 + i] : u[3 * c0 + i];
  }
#pragma unroll
  for (int al = 0; al < Rule::NEN; ++al) {
    const int64_t c = coef_of<Rule>(conn_e, al);
    const double s = sc[al % 4];
    const double w0 = Rule::dN_rt(q, al, 0) * s, w1 = Rule::dN_rt(q, al, 1) * s,
                 w2 = Rule::dN_rt(q, al, 2) * s;
    const bool position = Rule::MC == 1 || (al & 3) == 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double d = (X ? u[3 * c + i] - X[3 * c + i] : u[3 * c + i]) - (position ? r0[i] : 0.0);
      D[3 * i] += d * w0;
      D[3 * i + 1] += d * w1;
      D[3 * i + 2] += d * w2;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      out[3 * i + J] = D[3 * i] * Jinv[J] + D[3 * i + 1] * Jinv[3 + J] + D[3 * i + 2] * Jinv[6 + J];
}

// Nodal values of a workgroup's elements in LDS: 6 doubles per (element,
// coefficient), u = q - X then qdot (zero without qdot), for elements
// e_lo .. e_lo + ne - 1.
template <class Rule>
__device__ __forceinline__ void gather_nodal(const AsmArgs& a, int64_t e_lo, int ne, double* nod) {
  constexpr int NEN = Rule::NEN, NPN = Rule::NPN;
  for (int idx = threadIdx.x; idx < ne * NEN; idx += blockDim.x) {
    const int le = idx / NEN, al = idx - le * NEN;
    const int64_t e = e_lo + le;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (e < a.n_elem) {
      const int64_t c = coef_of<Rule>(a.conn + e * NPN, al);
#pragma unroll
      for (int i = 0; i < 3; ++i) v[i] = a.q[3 * c + i] - a.X[3 * c + i];
      if (a.qdot) {
#pragma unroll
        for (int i = 0; i < 3; ++i) v[3 + i] = a.qdot[3 * c + i];
      }
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) nod[6 * idx + t] = v[t];
  }
}

#ifndef TLFEA_KIN_UNROLL
#define TLFEA_KIN_UNROLL 4
#endif

// Displacement and velocity gradients at point q of element e from its nodal
// values in LDS (ne: 6 doubles per coefficient): Hd = sum_a u_a (x) g_a,
// Fd = sum_a qdot_a (x) g_a, with g_a = J0^-T dN_a (Sec. 4.3, Eq. F_assembly).
// The position functions sum to one, so their gradients sum to zero and the
// first coefficient's values may be taken out of every position coefficient:
// the terms then stay of the size of the element's own deformation instead of
// its rigid displacement (a body turned far from the origin keeps the digits
// of its strain).
// PART: coefficients in steps of TLFEA_KIN_UNROLL instead of all at once (a
// full unroll keeps every table load in flight; for the shell's 16
// coefficients that caps the kernels at one wave per SIMD).  Measured per
// kernel: steps for the four-coefficient elements (shell and beam) everywhere
// and for the T10 force and backward kernels, a full unroll for the T10
// element rows and point records.
template <class Rule, bool PART = (Rule::MC == 4 || Rule::NEN > 10)>
__device__ __forceinline__ void tile_kinematics(const AsmArgs& a, const double* ne, int64_t e, int q,
                                                double (&Jinv)[9], double& det, double (&Hd)[9], double (&Fd)[9]) {
  constexpr int NEN = Rule::NEN;
  double sc[4];
  load_geometry<Rule>(a, e, q, Jinv, det);
  element_scales<Rule>(a, e, sc);
  double Du[9], Dv[9], r0[6];
#pragma unroll
  for (int t = 0; t < 9; ++t) Du[t] = Dv[t] = 0.0;
#pragma unroll
  for (int t = 0; t < 6; ++t) r0[t] = ne[t];
  auto add = [&](int al) __attribute__((always_inline)) {
    const double s = sc[al % 4];
    const double w0 = Rule::dN_rt(q, al, 0) * s, w1 = Rule::dN_rt(q, al, 1) * s, w2 = Rule::dN_rt(q, al, 2) * s;
    const bool position = Rule::MC == 1 || (al & 3) == 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u = ne[6 * al + i] - (position ? r0[i] : 0.0);
      const double v = ne[6 * al + 3 + i] - (position ? r0[3 + i] : 0.0);
      Du[3 * i] += u * w0;
      Du[3 * i + 1] += u * w1;
      Du[3 * i + 2] += u * w2;
      Dv[3 * i] += v * w0;
      Dv[3 * i + 1] += v * w1;
      Dv[3 * i + 2] += v * w2;
    }
  };
  if constexpr (PART) {
#pragma unroll TLFEA_KIN_UNROLL
    for (int al = 0; al < NEN; ++al) add(al);
  } else {
#pragma unroll
    for (int al = 0; al < NEN; ++al) add(al);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      Hd[3 * i + J] = Du[3 * i] * Jinv[J] + Du[3 * i + 1] * Jinv[3 + J] + Du[3 * i + 2] * Jinv[6 + J];
      Fd[3 * i + J] = Dv[3 * i] * Jinv[J] + Dv[3 * i + 1] * Jinv[3 + J] + Dv[3 * i + 2] * Jinv[6 + J];
    }
}

// material constants of a launch: the host copy, or the device vector when given
__device__ __forceinline__ MatParams launch_material(const AsmArgs& a) {
  MatParams mp = a.mp;
  if (a.mp_dev) {
    mp.c0 = a.mp_dev[0];
    mp.c1 = a.mp_dev[1];
    mp.c2 = a.mp_dev[2];
    mp.eta = a.mp_dev[3];
    mp.lam_v = a.mp_dev[4];
  }
  return mp;
}

// Hd = F - I and Fdot at point q of element ge (float64).
template <class Rule>
__device__ __forceinline__ void load_kinematics(const AsmArgs& a, int64_t ge, int q, double* Hd, double* Fd,
                                                double* Jinv, double& det) {
  load_geometry<Rule>(a, ge, q, Jinv, det);
  double sc[4];
  element_scales<Rule>(a, ge, sc);
  field_gradient<Rule>(a, ge, q, sc, a.q, a.X, Jinv, Hd);
  if (a.qdot) {
    field_gradient<Rule>(a, ge, q, sc, a.qdot, nullptr, Jinv, Fd);
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t) Fd[t] = 0.0;
  }
}

// the assembly arguments of body `bi` of a batch
__device__ __forceinline__ AsmArgs body_args(const BatchArgs& b, const BatchBody& B, int bi) {
  AsmArgs a;
  a.conn = B.conn;
  a.X = B.X;
  a.geo = B.geo;
  a.escale = B.escale;
  a.half_h = B.half_h;
  a.affine = B.affine;
  a.n_elem = B.n_elem;
  a.n_tiles = 0;
  a.q = b.q + B.dof_off;
  a.qdot = b.qdot ? b.qdot + B.dof_off : nullptr;
  a.f = nullptr;
  a.vals = nullptr;
  a.row_off = B.row_off;
  a.rank = B.rank;
  a.mp = B.mp;
  a.alpha = b.h[bi];
  a.beta = 1.0;
  a.flags = b.flags;
  a.mp_dev = nullptr;
  return a;
}

}  // namespace
}  // namespace tlfea
