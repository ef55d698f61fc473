// rules.h -- element rules (shape-function tables, quadrature) for the kernels.
//
// Each translation unit that includes this header gets its own __constant__
// copy of the tables (internal linkage) for run-time indexing; compile-time
// indexing goes through the constexpr tables of tables.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tables.h"

namespace tlfea {
namespace {

static __constant__ T10Table c_t10 = make_t10_table();
static __constant__ AncfTable<3, 3, 2> c_a332 = make_ancf_table<3, 3, 2>();
static __constant__ AncfTable<4, 4, 3> c_a443 = make_ancf_table<4, 4, 3>();
static __constant__ BeamTable<3, 2, 2> c_b322 = make_beam_table<3, 2, 2>();

template <int N>
struct Int {
  static constexpr int value = N;
};

template <int I, int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (I < N) {
    f(Int<I>{});
    sfor<I + 1, N>(f);
  }
}

// Parent gradients of one shape function at every point of the T10 rule,
// dN_a(q)_m at 3 q + m, padded to 16 values: one row per node, in the record
// precision, fetched by a lane with a few vector loads.
template <typename R>
struct alignas(16) T10Rows {
  R v[10][16];
};
template <typename R>
constexpr T10Rows<R> make_t10_rows() {
  T10Rows<R> t{};
  for (int a = 0; a < 10; ++a)
    for (int q = 0; q < 5; ++q)
      for (int m = 0; m < 3; ++m) t.v[a][3 * q + m] = (R)kT10.dN[q][a][m];
  return t;
}
static __constant__ T10Rows<float> c_t10_rows_f = make_t10_rows<float>();
static __constant__ T10Rows<double> c_t10_rows_d = make_t10_rows<double>();

struct RuleT10 {
  static constexpr int NEN = 10, NPN = 10, MC = 1, NQ = 5;
  template <typename R>
  __device__ static const R* rows(int a) {
    if constexpr (sizeof(R) == 4) return c_t10_rows_f.v[a];
    else return c_t10_rows_d.v[a];
  }
  static constexpr double dN(int q, int a, int m) { return kT10.dN[q][a][m]; }
  __device__ static double dN_rt(int q, int a, int m) { return c_t10.dN[q][a][m]; }
  __device__ static double w_rt(int q) { return c_t10.w[q]; }
};

// Float copies of the ANCF gradient tables (element-row kernels, float32
// arithmetic), read with a wave-uniform point index through the scalar cache.
template <int NQ, int NEN>
struct FloatGrad {
  float v[NQ][NEN][3];
};
template <int NQ, int NEN, class T>
constexpr FloatGrad<NQ, NEN> make_float_grad(const T& t) {
  FloatGrad<NQ, NEN> f{};
  for (int q = 0; q < NQ; ++q)
    for (int a = 0; a < NEN; ++a)
      for (int m = 0; m < 3; ++m) f.v[q][a][m] = (float)t.dS[q][a][m];
  return f;
}
static __constant__ FloatGrad<18, 16> c_a332_f = make_float_grad<18, 16>(kAncf332);
static __constant__ FloatGrad<48, 16> c_a443_f = make_float_grad<48, 16>(kAncf443);
static __constant__ FloatGrad<12, 8> c_b322_f = make_float_grad<12, 8>(kBeam322);

template <int NX, int NY, int NZ>
struct RuleAncf {
  static constexpr int NEN = 16, NPN = 4, MC = 4, NQ = NX * NY * NZ;
  static constexpr const AncfTable<NX, NY, NZ>& tab() {
    if constexpr (NX == 3) return kAncf332; else return kAncf443;
  }
  static constexpr double dN(int q, int a, int m) { return tab().dS[q][a][m]; }
  __device__ static const AncfTable<NX, NY, NZ>& ctab() {
    if constexpr (NX == 3) return c_a332; else return c_a443;
  }
  __device__ static double dN_rt(int q, int a, int m) { return ctab().dS[q][a][m]; }
  __device__ static double w_rt(int q) { return ctab().w[q]; }
  __device__ static float dNf_rt(int q, int a, int m) {
    if constexpr (NX == 3) return c_a332_f.v[q][a][m]; else return c_a443_f.v[q][a][m];
  }
};

// ANCF3243 beam, Gauss-Legendre 3 x 2 x 2 (two physical nodes of four coefficients)
struct RuleBeam {
  static constexpr int NEN = 8, NPN = 2, MC = 4, NQ = 12;
  static constexpr double dN(int q, int a, int m) { return kBeam322.dS[q][a][m]; }
  __device__ static double dN_rt(int q, int a, int m) { return c_b322.dS[q][a][m]; }
  __device__ static double w_rt(int q) { return c_b322.w[q]; }
  __device__ static float dNf_rt(int q, int a, int m) { return c_b322_f.v[q][a][m]; }
};

}  // namespace
}  // namespace tlfea
