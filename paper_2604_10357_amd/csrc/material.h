// material.h -- quadrature-point constitutive update for the gfx950 kernels.
//
// Sec. 4.3, Stage 1: P = P_el(F) + P_vis(F, Fdot).  Sec. 4.4.2: the material
// tangent A_iJkL = dP_iJ / dF_kL enters Eq. tangent_block.  The paper leaves
// the formulas to Part I; the library uses the textbook forms
//   SVK : S = lambda tr(E) I + 2 mu E, P = F S
//   MR  : W = mu10 (J^-2/3 I1 - 3) + mu01 (J^-4/3 I2 - 3) + kappa/2 (J - 1)^2
//   KV  : S_v = 2 eta Edot + lam_v tr(Edot) I, P_v = F S_v
// and evaluates the combined tangent  alpha dP/dF + beta dP/dFdot  in the
// factored form
//   A_iJkL = d_ik M_JL + N_ik d_JL + F_iJ W_kL + F_iL Y_kJ
//            + [MR] U_iJ G_kL + G_iJ V_kL + c_gx G_iL G_kJ,   G = F^-T,
// whose 3x3 factors are formed once per point; each of the 81 entries then
// costs a handful of FMAs.
//
// Precision: the displacement gradient Hd = F - I arrives in float64.  The
// Green strain E = (Hd + Hd^T + Hd^T Hd) / 2 is formed from it in float64,
// so it carries no rounded O(1) term even when the strain is small and the
// element has turned through a large rotation; J - 1 is formed in float64 from
// the invariants of Hd (no cancellation near J = 1), and J^-2/3, J^-4/3 and the
// volumetric coefficients kappa J (J-1), kappa J (2J-1) stay float64.  The
// stresses are written in E alone:
//   SVK : S = lambda tr(E) I + 2 mu E,                       P = F S
//   MR  : S = 2 dW/dC = C^-1 T with C = I + 2E and
//         T = 2 mu10 J^-2/3 (2 dev E)
//           + 2 mu01 J^-4/3 (2 dev E + 4 tr(E) E - 4 E^2 + 4/3 (E:E - tr(E)^2) I)
//           + kappa J (J - 1) I,                             P = F C^-1 T = F^-T T
// (the two brackets are C - I1/3 I and I1 C - C^2 - 2/3 I2 I rewritten with
// C = I + 2E), so no stress is a difference of O(1) numbers.  Everything after
// the cast of E runs in R (float64 for the FP64 path, float32 for the mixed
// path); the tangent factors are O(1) combinations and are formed from F in R.
#pragma once

#include <hip/hip_runtime.h>

namespace tlfea {

struct MatParams {
  int kind;          // 1 = SVK, 2 = Mooney-Rivlin
  double c0, c1, c2; // SVK: lambda, mu, -; MR: mu10, mu01, kappa
  double eta, lam_v; // Kelvin-Voigt
};

__device__ __forceinline__ double det3d(const double* M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
         M[2] * (M[3] * M[7] - M[4] * M[6]);
}

// J - 1 = det(I + H) - 1 = tr H + ((tr H)^2 - tr(H^2)) / 2 + det H
__device__ __forceinline__ double jm1_of(const double* H) {
  double tr = H[0] + H[4] + H[8];
  double trH2 = H[0] * H[0] + H[4] * H[4] + H[8] * H[8] +
                2.0 * (H[1] * H[3] + H[2] * H[6] + H[5] * H[7]);
  return tr + 0.5 * (tr * tr - trH2) + det3d(H);
}

// Output of the constitutive update: P (row-major) and the factors of A,
// both already multiplied by the quadrature volume dV.
template <typename R>
struct PointOut {
  R F[9];                    // deformation gradient in R
  R P[9];
  R M[9], N[9], W[9], Y[9];  // see the factored form above
  R U[9], V[9], G[9];        // MR only
  R cgx;                     // MR only
  bool mr;
};

// Constitutive update at one point.  Hd, Fd in float64; returns flags bits.
template <typename R, bool WANT_A>
__device__ __forceinline__ unsigned point_update(const MatParams& mp, const double* Hd,
                                                 const double* Fd64, double dV, double alpha,
                                                 double beta, PointOut<R>& o) {
  unsigned flags = 0;
  R Fd[9], E[9];
  R* F = o.F;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    F[t] = (R)Hd[t] + ((t % 4) == 0 ? R(1) : R(0));
    Fd[t] = (R)Fd64[t];
  }
  // Green strain in float64, then cast
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double e = 0.5 * (Hd[3 * i + j] + Hd[3 * j + i] + Hd[i] * Hd[j] + Hd[3 + i] * Hd[3 + j] +
                              Hd[6 + i] * Hd[6 + j]);
      E[3 * i + j] = (R)e;
      E[3 * j + i] = (R)e;
    }
  const R trE = E[0] + E[4] + E[8];
  const bool kv = (mp.eta != 0.0) || (mp.lam_v != 0.0);
  const R a_ = (R)alpha, b_ = (R)beta, sdv = (R)dV;
  R S[9];  // total second Piola-Kirchhoff stress of the S-type terms (SVK + KV)
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    S[t] = R(0);
    o.M[t] = R(0);
    o.N[t] = R(0);
    o.W[t] = R(0);
    o.Y[t] = R(0);
  }
  R B[9];  // F F^T
  if (WANT_A) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        B[3 * i + j] = F[3 * i] * F[3 * j] + F[3 * i + 1] * F[3 * j + 1] + F[3 * i + 2] * F[3 * j + 2];
  }

  double jm1 = jm1_of(Hd);
  double J = 1.0 + jm1;
  if (!(J > 0.0)) flags |= 1u;

  o.mr = (mp.kind == 2);
  R Pel[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) Pel[t] = R(0);
  if (mp.kind == 1) {
    // SVK
    const R lam = (R)mp.c0, mu = (R)mp.c1;
#pragma unroll
    for (int t = 0; t < 9; ++t) S[t] = R(2) * mu * E[t] + ((t % 4) == 0 ? lam * trE : R(0));
    if (WANT_A) {
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        o.M[t] = a_ * S[t];
        o.N[t] = a_ * mu * B[t];
        o.W[t] = a_ * lam * F[t];
        o.Y[t] = a_ * mu * F[t];
      }
    }
  } else {
    // Mooney-Rivlin with decoupled invariants and (kappa/2)(J-1)^2
    const double cbJ = cbrt(J);
    const double a = 1.0 / (cbJ * cbJ);  // J^-2/3
    const double b = a * a;              // J^-4/3
    // G = F^-T = cof(F) / J
    const R invJ = (R)(1.0 / J);
    R* G = o.G;
    G[0] = (F[4] * F[8] - F[5] * F[7]) * invJ;
    G[1] = (F[5] * F[6] - F[3] * F[8]) * invJ;
    G[2] = (F[3] * F[7] - F[4] * F[6]) * invJ;
    G[3] = (F[2] * F[7] - F[1] * F[8]) * invJ;
    G[4] = (F[0] * F[8] - F[2] * F[6]) * invJ;
    G[5] = (F[1] * F[6] - F[0] * F[7]) * invJ;
    G[6] = (F[1] * F[5] - F[2] * F[4]) * invJ;
    G[7] = (F[2] * F[3] - F[0] * F[5]) * invJ;
    G[8] = (F[0] * F[4] - F[1] * F[3]) * invJ;
    const double mu10 = mp.c0, mu01 = mp.c1, kap = mp.c2;
    const double vol1 = kap * J * jm1;  // kappa J (J - 1)
    {
      // T (symmetric) from E, then P_el = G T
      R EE[9], ee = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          EE[3 * i + j] = E[3 * i] * E[j] + E[3 * i + 1] * E[3 + j] + E[3 * i + 2] * E[6 + j];
          ee += E[3 * i + j] * E[3 * i + j];
        }
      const R p1 = (R)(2.0 * mu10 * a), p2 = (R)(2.0 * mu01 * b), pv = (R)vol1;
      const R tr3 = trE / R(3), diag2 = R(4) / R(3) * (ee - trE * trE);
      R T[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const R dev2 = R(2) * (E[t] - ((t % 4) == 0 ? tr3 : R(0)));
        T[t] = p1 * dev2 + p2 * (dev2 + R(4) * trE * E[t] - R(4) * EE[t] + ((t % 4) == 0 ? diag2 : R(0))) +
               ((t % 4) == 0 ? pv : R(0));
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          Pel[3 * i + j] = G[3 * i] * T[j] + G[3 * i + 1] * T[3 + j] + G[3 * i + 2] * T[6 + j];
    }
    if (WANT_A) {
      R C[9];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          C[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
      R FC[9];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          FC[3 * i + j] = F[3 * i] * C[j] + F[3 * i + 1] * C[3 + j] + F[3 * i + 2] * C[6 + j];
      const R I1 = C[0] + C[4] + C[8];
      R trC2 = R(0);
#pragma unroll
      for (int t = 0; t < 9; ++t) trC2 += C[t] * C[t];
      const R I2 = R(0.5) * (I1 * I1 - trC2);
      const double I1d = (double)I1, I2d = (double)I2;
      const double vol2 = kap * J * (2.0 * J - 1.0);  // kappa J (2J - 1)
      const R cdd = (R)(alpha * (2.0 * mu10 * a + 2.0 * mu01 * b * I1d));
      const R cmc = (R)(alpha * (-2.0 * mu01 * b));
      const R cfg = (R)(alpha * (-4.0 / 3.0 * mu10 * a - 8.0 / 3.0 * mu01 * b * I1d));
      const R ccg = (R)(alpha * (8.0 / 3.0 * mu01 * b));
      const R cgg = (R)(alpha * (4.0 / 9.0 * mu10 * a * I1d + 16.0 / 9.0 * mu01 * b * I2d + vol2));
      const R cgx = (R)(alpha * (2.0 / 3.0 * mu10 * a * I1d + 4.0 / 3.0 * mu01 * b * I2d - vol1));
      const R cff = (R)(alpha * 4.0 * mu01 * b);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        o.M[t] = cmc * C[t] + ((t % 4) == 0 ? cdd : R(0));
        o.N[t] = cmc * B[t];
        o.W[t] = cff * F[t];
        o.Y[t] = cmc * F[t];
        o.V[t] = cfg * F[t] + ccg * FC[t];
        o.U[t] = o.V[t] + cgg * G[t];
      }
      o.cgx = cgx * sdv;
    }
  }
  if (kv) {
    // Edot = (Fdot^T F + F^T Fdot) / 2, S_v = 2 eta Edot + lam_v tr(Edot) I
    const R eta = (R)mp.eta, lv = (R)mp.lam_v;
    R Ed[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        R s = R(0);
#pragma unroll
        for (int m = 0; m < 3; ++m) s += Fd[3 * m + i] * F[3 * m + j] + F[3 * m + i] * Fd[3 * m + j];
        Ed[3 * i + j] = R(0.5) * s;
      }
    const R trEd = Ed[0] + Ed[4] + Ed[8];
    R Sv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) Sv[t] = R(2) * eta * Ed[t] + ((t % 4) == 0 ? lv * trEd : R(0));
#pragma unroll
    for (int t = 0; t < 9; ++t) S[t] += Sv[t];
    if (WANT_A) {
      R FFd[9];  // F Fdot^T
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          FFd[3 * i + j] = F[3 * i] * Fd[3 * j] + F[3 * i + 1] * Fd[3 * j + 1] + F[3 * i + 2] * Fd[3 * j + 2];
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        o.M[t] += a_ * Sv[t];
        o.N[t] += a_ * eta * FFd[t] + b_ * eta * B[t];
        o.W[t] += a_ * lv * Fd[t] + b_ * lv * F[t];
        o.Y[t] += a_ * eta * Fd[t] + b_ * eta * F[t];
      }
    }
  }
  // P = Pel + F S  (Pel: the Mooney-Rivlin stress; S: the SVK and/or viscous stress)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      R p = Pel[3 * i + j] + F[3 * i] * S[j] + F[3 * i + 1] * S[3 + j] + F[3 * i + 2] * S[6 + j];
      o.P[3 * i + j] = p * sdv;
      if (!isfinite((double)p)) flags |= 2u;
    }
  if (WANT_A) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      o.M[t] *= sdv;
      o.N[t] *= sdv;
      o.W[t] *= sdv;
      o.Y[t] *= sdv;
      if (o.mr) {
        o.U[t] *= sdv;
        o.V[t] *= sdv;
      }
    }
  }
  return flags;
}

// 3x3 helpers (row-major) for the reverse-mode product below
__device__ __forceinline__ void mm3(const double* A, const double* B, double* C) {  // C = A B
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
__device__ __forceinline__ void mtm3(const double* A, const double* B, double* C) {  // C = A^T B
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}
__device__ __forceinline__ double ddot3(const double* A, const double* B) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 9; ++t) s += A[t] * B[t];
  return s;
}

// Reverse-mode product of the stress at one point, in float64.  For the
// cotangent gradient Wc:
//   Zq_kL = sum_iJ Wc_iJ dP_iJ / dF_kL,   Zd_kL = sum_iJ Wc_iJ dP_iJ / dFdot_kL,
//   parts[i] = Wc : P_i, P_i the stress per unit value of constant i (P is
//   linear in every constant: SVK (lambda, mu), MR (mu10, mu01, kappa), then
//   KV (eta, lam_v), formed even when the law's constant is zero).
// The adjoints of the E-based forms of point_update, with Y = F^T Wc,
// Ym = sym(G^T Wc), G = F^-T, sym(A) = (A + A^T) / 2:
//   SVK : P = F S                 Zq = Wc S + F (lambda tr(Y) I + 2 mu sym(Y))
//   KV  : P = F S_v               Zq += Wc S_v + Fdot Sh,  Zd = F Sh,
//                                 Sh = 2 eta sym(Y) + lam_v tr(Y) I
//   MR  : P = G T(E, J)           Zq = -G T Wc^T G + F (2 mu10 a D1 + 2 mu01 b D2) + c G,
//     D1 = 2 dev(Ym)   (the adjoint of T's first bracket 2 dev E),
//     D2 = 2 dev(Ym) + 4 (Ym:E) I + 4 tr(E) Ym - 4 (Ym E + E Ym)
//          + 8/3 tr(Ym) (E - tr(E) I)   (that of the second bracket B2),
//     c  = -4/3 mu10 a (Ym : 2 dev E) - 8/3 mu01 b (Ym : B2) + kappa J (2J - 1) tr(Ym)
//          (the J-dependence of J^-2/3, J^-4/3 and the volumetric term, dJ = J G : dF).
__device__ __forceinline__ void stress_vjp(const MatParams& mp, const double* Hd, const double* Fd, const double* Wc,
                                           double* Zq, double* Zd, double* parts) {
  double F[9], E[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) F[t] = Hd[t] + ((t % 4) == 0 ? 1.0 : 0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      E[3 * i + j] = 0.5 * (Hd[3 * i + j] + Hd[3 * j + i] + Hd[i] * Hd[j] + Hd[3 + i] * Hd[3 + j] + Hd[6 + i] * Hd[6 + j]);
  const double trE = E[0] + E[4] + E[8];
  double Y[9];  // F^T Wc
  mtm3(F, Wc, Y);
  const double trY = Y[0] + Y[4] + Y[8];
  double YE = 0.0;  // sym(Y) : E = Y : E
#pragma unroll
  for (int t = 0; t < 9; ++t) YE += Y[t] * E[t];
  if (mp.kind == 1) {
    const double lam = mp.c0, mu = mp.c1;
    parts[0] = trE * trY;
    parts[1] = 2.0 * YE;
    parts[2] = 0.0;
    double S[9], Sh[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const bool d = i == j;
        S[3 * i + j] = 2.0 * mu * E[3 * i + j] + (d ? lam * trE : 0.0);
        Sh[3 * i + j] = mu * (Y[3 * i + j] + Y[3 * j + i]) + (d ? lam * trY : 0.0);
      }
    double A[9], B[9];
    mm3(Wc, S, A);
    mm3(F, Sh, B);
#pragma unroll
    for (int t = 0; t < 9; ++t) Zq[t] = A[t] + B[t];
  } else {
    const double mu10 = mp.c0, mu01 = mp.c1, kap = mp.c2;
    const double jm1 = jm1_of(Hd), J = 1.0 + jm1;
    const double cbJ = cbrt(J), a = 1.0 / (cbJ * cbJ), b = a * a, invJ = 1.0 / J;
    double G[9];
    G[0] = (F[4] * F[8] - F[5] * F[7]) * invJ;
    G[1] = (F[5] * F[6] - F[3] * F[8]) * invJ;
    G[2] = (F[3] * F[7] - F[4] * F[6]) * invJ;
    G[3] = (F[2] * F[7] - F[1] * F[8]) * invJ;
    G[4] = (F[0] * F[8] - F[2] * F[6]) * invJ;
    G[5] = (F[1] * F[6] - F[0] * F[7]) * invJ;
    G[6] = (F[1] * F[5] - F[2] * F[4]) * invJ;
    G[7] = (F[2] * F[3] - F[0] * F[5]) * invJ;
    G[8] = (F[0] * F[4] - F[1] * F[3]) * invJ;
    double EE[9];
    mm3(E, E, EE);
    const double ee = ddot3(E, E);
    double Ym[9], dev2[9], B2[9];
    {
      double T0[9];
      mtm3(G, Wc, T0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Ym[3 * i + j] = 0.5 * (T0[3 * i + j] + T0[3 * j + i]);
    }
    const double trYm = Ym[0] + Ym[4] + Ym[8];
    const double diag2 = 4.0 / 3.0 * (ee - trE * trE);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const bool d = (t % 4) == 0;
      dev2[t] = 2.0 * (E[t] - (d ? trE / 3.0 : 0.0));
      B2[t] = dev2[t] + 4.0 * trE * E[t] - 4.0 * EE[t] + (d ? diag2 : 0.0);
    }
    const double y_dev2 = ddot3(Ym, dev2), y_b2 = ddot3(Ym, B2), ymE = ddot3(Ym, E);
    parts[0] = 2.0 * a * y_dev2;
    parts[1] = 2.0 * b * y_b2;
    parts[2] = J * jm1 * trYm;
    // -G T Wc^T G
    double GT[9], M1[9], M2[9];
    {
      double T[9];
#pragma unroll
      for (int t = 0; t < 9; ++t)
        T[t] = 2.0 * mu10 * a * dev2[t] + 2.0 * mu01 * b * B2[t] + ((t % 4) == 0 ? kap * J * jm1 : 0.0);
      mm3(G, T, GT);
    }
    {
      double WtG[9];  // Wc^T G
      mtm3(Wc, G, WtG);
      mm3(GT, WtG, M1);
    }
    double D[9];
    {
      double YE2[9], EY[9];
      mm3(Ym, E, YE2);
      mm3(E, Ym, EY);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const bool d = (t % 4) == 0;
        const double dv = 2.0 * (Ym[t] - (d ? trYm / 3.0 : 0.0));
        const double d2 = dv + (d ? 4.0 * ymE : 0.0) + 4.0 * trE * Ym[t] - 4.0 * (YE2[t] + EY[t]) +
                          8.0 / 3.0 * trYm * (E[t] - (d ? trE : 0.0));
        D[t] = 2.0 * mu10 * a * dv + 2.0 * mu01 * b * d2;
      }
    }
    mm3(F, D, M2);
    const double c = -4.0 / 3.0 * mu10 * a * y_dev2 - 8.0 / 3.0 * mu01 * b * y_b2 + kap * J * (2.0 * J - 1.0) * trYm;
#pragma unroll
    for (int t = 0; t < 9; ++t) Zq[t] = M2[t] - M1[t] + c * G[t];
  }
  // Kelvin-Voigt
  double Ed[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) s += Fd[3 * m + i] * F[3 * m + j] + F[3 * m + i] * Fd[3 * m + j];
      Ed[3 * i + j] = 0.5 * s;
    }
  const double trEd = Ed[0] + Ed[4] + Ed[8];
  parts[3] = 2.0 * ddot3(Y, Ed);
  parts[4] = trEd * trY;
  const double eta = mp.eta, lv = mp.lam_v;
  if (eta != 0.0 || lv != 0.0) {
    double Sv[9], Sh[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const bool d = i == j;
        Sv[3 * i + j] = 2.0 * eta * Ed[3 * i + j] + (d ? lv * trEd : 0.0);
        Sh[3 * i + j] = eta * (Y[3 * i + j] + Y[3 * j + i]) + (d ? lv * trY : 0.0);
      }
    double A[9], B[9];
    mm3(Wc, Sv, A);
    mm3(Fd, Sh, B);
#pragma unroll
    for (int t = 0; t < 9; ++t) Zq[t] += A[t] + B[t];
    mm3(F, Sh, Zd);
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t) Zd[t] = 0.0;
  }
}

// Z_kL = sum_iJ Wc_iJ A_iJkL (the tangent applied to a cotangent gradient Wc
// from the left), term by term from the factored form:
//   d_ik M_JL      -> (Wc M)_kL          N_ik d_JL  -> (N^T Wc)_kL
//   F_iJ W_kL      -> (Wc:F) W_kL        F_iL Y_kJ  -> (Y Wc^T F)_kL
//   U_iJ G_kL      -> (Wc:U) G_kL        G_iJ V_kL  -> (Wc:G) V_kL
//   c G_iL G_kJ    -> c (G Wc^T G)_kL
template <typename R>
__device__ __forceinline__ void cotangent_contract(const PointOut<R>& o, const R* Wc, R* Z) {
  R wf = R(0), wu = R(0), wg = R(0);
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    wf += Wc[t] * o.F[t];
    if (o.mr) {
      wu += Wc[t] * o.U[t];
      wg += Wc[t] * o.G[t];
    }
  }
  R T[9], S[9];  // Wc^T F and Wc^T G
#pragma unroll
  for (int J = 0; J < 3; ++J)
#pragma unroll
    for (int L = 0; L < 3; ++L) {
      T[3 * J + L] = Wc[J] * o.F[L] + Wc[3 + J] * o.F[3 + L] + Wc[6 + J] * o.F[6 + L];
      S[3 * J + L] = o.mr ? Wc[J] * o.G[L] + Wc[3 + J] * o.G[3 + L] + Wc[6 + J] * o.G[6 + L] : R(0);
    }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int L = 0; L < 3; ++L) {
      R z = wf * o.W[3 * k + L];
#pragma unroll
      for (int J = 0; J < 3; ++J)
        z += Wc[3 * k + J] * o.M[3 * J + L] + o.N[3 * J + k] * Wc[3 * J + L] + o.Y[3 * k + J] * T[3 * J + L];
      if (o.mr) {
        z += wu * o.G[3 * k + L] + wg * o.V[3 * k + L];
#pragma unroll
        for (int J = 0; J < 3; ++J) z += o.cgx * o.G[3 * k + J] * S[3 * J + L];
      }
      Z[3 * k + L] = z;
    }
}

// The same tangent and stress in parent coordinates, with dV folded in:
//   Ahat_imkn = sum_JL Jinv_mJ A_iJkL Jinv_nL,   Phat_im = sum_J P_iJ Jinv_mJ.
// Every factor of the decomposition transforms on its own:
//   d_ik M_JL   -> d_ik Mh_mn     Mh = Jinv M Jinv^T
//   N_ik d_JL   -> N_ik Ch_mn     Ch = Jinv Jinv^T
//   F_iJ W_kL   -> Fh_im Wh_kn    Xh = X Jinv^T for X in {F, W, Y, U, V, G}
//   F_iL Y_kJ   -> Fh_in Yh_km
//   U_iJ G_kL + G_iJ V_kL + c G_iL G_kJ -> Uh_im Gh_kn + Gh_im Vh_kn + c Gh_in Gh_km
template <typename R>
struct HatOut {
  R P[9], M[9], N[9], C[9], F[9], W[9], Y[9], U[9], V[9], G[9];
  R cgx;
  bool mr;
};

template <typename R>
__device__ __forceinline__ void rows_times_jinvT(const R* X, const R* Ji, R* out) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int m = 0; m < 3; ++m) out[3 * i + m] = X[3 * i] * Ji[3 * m] + X[3 * i + 1] * Ji[3 * m + 1] + X[3 * i + 2] * Ji[3 * m + 2];
}

template <typename R, bool WANT_A>
__device__ __forceinline__ void to_parent(const PointOut<R>& o, const double* Jinv64, HatOut<R>& h) {
  R Ji[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) Ji[t] = (R)Jinv64[t];
  rows_times_jinvT(o.P, Ji, h.P);
  if (!WANT_A) return;
  h.mr = o.mr;
  h.cgx = o.cgx;
  rows_times_jinvT(o.F, Ji, h.F);
  rows_times_jinvT(o.W, Ji, h.W);
  rows_times_jinvT(o.Y, Ji, h.Y);
  R T[9];
  rows_times_jinvT(o.M, Ji, T);  // M Jinv^T, then Jinv (M Jinv^T)
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      h.M[3 * m + n] = Ji[3 * m] * T[n] + Ji[3 * m + 1] * T[3 + n] + Ji[3 * m + 2] * T[6 + n];
      h.C[3 * m + n] = Ji[3 * m] * Ji[3 * n] + Ji[3 * m + 1] * Ji[3 * n + 1] + Ji[3 * m + 2] * Ji[3 * n + 2];
    }
#pragma unroll
  for (int t = 0; t < 9; ++t) h.N[t] = o.N[t];
  if (o.mr) {
    rows_times_jinvT(o.U, Ji, h.U);
    rows_times_jinvT(o.V, Ji, h.V);
    rows_times_jinvT(o.G, Ji, h.G);
  }
}

template <typename R>
__device__ __forceinline__ R hat_entry(const HatOut<R>& h, int i, int m, int k, int n) {
  R a = h.F[3 * i + m] * h.W[3 * k + n] + h.F[3 * i + n] * h.Y[3 * k + m] + h.N[3 * i + k] * h.C[3 * m + n];
  if (i == k) a += h.M[3 * m + n];
  if (h.mr)
    a += h.U[3 * i + m] * h.G[3 * k + n] + h.G[3 * i + m] * h.V[3 * k + n] + h.cgx * h.G[3 * i + n] * h.G[3 * k + m];
  return a;
}

}  // namespace tlfea
