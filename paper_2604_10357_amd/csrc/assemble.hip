// assemble.hip -- internal force and tangent stiffness for gfx950, in two passes
// that write every output value exactly once and use no global atomics.
//
// What is computed (arXiv 2604.10357, Part II):
//   F  = I + sum_a (x_a - X_a) (x) g_a,  Fdot = sum_a xdot_a (x) g_a   (Sec. 4.3, Eq. F_assembly)
//   P  = P_el(F) + P_vis(F, Fdot)                                     (Sec. 4.3, Stage 1)
//   f_a = sum_q P g_a J0 w_q, summed over the elements of each DOF    (Eqs. fint_local, fint_global)
//   K_ab = sum_q A g_a g_b J0 w_q, summed into the fixed CSR pattern  (Sec. 4.4.2, Eq. tangent_block)
//
// The paper scatters per entry with atomicAdd and names two-pass
// scatter/reduction as the way around atomic contention.  On MI355X scattered
// float64 atomics retire at roughly the rate of random read-modify-writes, so
// this library never issues them:
//
//   pass 1 (k_stage, one lane per element x quadrature point): gather the
//     element, form F and Fdot in float64, run the constitutive update and
//     store the point's tangent and stress in parent coordinates with the
//     quadrature volume folded in,
//        Ahat_imkn = dV sum_JL J0inv_mJ A_iJkL J0inv_nL,  Phat_im = dV sum_J P_iJ J0inv_mJ,
//     as one 96-value record: Ahat row i at [28 i, 28 i + 27), Phat row i at
//     [84 + 4 i, 84 + 4 i + 3), so that every row starts on 16 bytes.
//   pass 2 (k_gather, one workgroup per contiguous range of nodes): the CSR
//     rows of consecutive nodes form one contiguous segment, mirrored in LDS.
//     Each lane owns one (node, incident element, coefficient row) task and
//     contracts the records of that element,
//        t_kn = sum_m dN_a,m Ahat_imkn,   K[a i, b k] += sum_n t_kn dN_b,n,
//     where the parent gradients dN_b at each point are compile-time constants
//     (zeros skipped).  Results are added into the LDS segment in float64, and
//     the segment and the node forces are then written with plain coalesced
//     stores.  f_int comes out of the same pass from Phat.
//   Workgroups are remapped so each XCD walks a contiguous range of elements /
//   nodes, keeping the records a range reads in its own L2.
#include "kernel_common.h"

namespace tlfea {
namespace {

constexpr int kRecK = 96;  // record length with tangent: Ahat rows padded to 28, Phat rows padded to 4
constexpr int kRecF = 12;  // record length for the force only: Phat rows padded to 4
constexpr int kRowA = 28;  // Ahat row stride within a record
constexpr int kOffP = 84;  // Phat offset within a tangent record

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
template <class Rule, typename R, bool WANT_K>
__device__ __forceinline__ void stage_point(const AsmArgs& a, int64_t e, int q, R* rec) {
  double Hd[9], Fd[9], Jinv[9], det;
  load_kinematics<Rule>(a, e, q, Hd, Fd, Jinv, det);
  PointOut<R> o;
  const unsigned fl = point_update<R, WANT_K>(a.mp, Hd, Fd, det * Rule::w_rt(q), a.alpha, a.beta, o);
  if (fl) atomicOr(a.flags, fl);
  HatOut<R> h;
  to_parent<R, WANT_K>(o, Jinv, h);
  if constexpr (WANT_K) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int n = 0; n < 3; ++n) rec[kRowA * i + 9 * m + 3 * k + n] = hat_entry(h, i, m, k, n);
#pragma unroll
    for (int t = 0; t < 9; ++t) rec[kOffP + 4 * (t / 3) + t % 3] = h.P[t];
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t) rec[4 * (t / 3) + t % 3] = h.P[t];
  }
}

template <class Rule, typename R, bool WANT_K>
__global__ __launch_bounds__(256) void k_stage(AsmArgs a, R* stage) {
  constexpr int NQ = Rule::NQ;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_elem * NQ) return;
  stage_point<Rule, R, WANT_K>(a, p / NQ, (int)(p % NQ), stage + p * (WANT_K ? kRecK : kRecF));
}

// many bodies: the flat (element, point) index is resolved to a body by bisection
template <class Rule, typename R>
__global__ __launch_bounds__(256) void k_stage_batch(BatchArgs b) {
  constexpr int NQ = Rule::NQ;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.n_points) return;
  int lo = 0, hi = b.n_bodies - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.bodies[mid].point_off <= p) lo = mid; else hi = mid - 1;
  }
  const BatchBody& B = b.bodies[lo];
  const AsmArgs a = body_args(b, B, lo);
  const int64_t lp = p - B.point_off;
  stage_point<Rule, R, true>(a, lp / NQ, (int)(lp % NQ), (R*)b.stage + p * kRecK);
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
template <typename R, bool WANT_K>
struct RowBuf {
  R a[WANT_K ? kRowA : 4];  // Ahat row (27 used)
  R p[4];                    // Phat row (3 used)
};

template <typename T>
struct Vec4 { using type = float4; };
template <>
struct Vec4<double> { using type = double2; };

// one record row with 16-byte vector loads
template <typename R, bool WANT_K>
__device__ __forceinline__ void load_row(const R* rec, int i, RowBuf<R, WANT_K>& b) {
  using V = typename Vec4<R>::type;
  constexpr int per = sizeof(V) / sizeof(R);
  if constexpr (WANT_K) {
    const V* src = reinterpret_cast<const V*>(rec + kRowA * i);
#pragma unroll
    for (int t = 0; t < kRowA / per; ++t) *reinterpret_cast<V*>(b.a + per * t) = src[t];
    const V* sp = reinterpret_cast<const V*>(rec + kOffP + 4 * i);
#pragma unroll
    for (int t = 0; t < 4 / per; ++t) *reinterpret_cast<V*>(b.p + per * t) = sp[t];
  } else {
    const V* sp = reinterpret_cast<const V*>(rec + 4 * i);
#pragma unroll
    for (int t = 0; t < 4 / per; ++t) *reinterpret_cast<V*>(b.p + per * t) = sp[t];
  }
}
template <class Rule, typename R, bool WANT_F, bool WANT_K, bool ACCUM>
__device__ __forceinline__ void gather_range(const GatherArgs& g, int32_t I0, int32_t I1, double* lds,
                                             int32_t* pre) {
  constexpr int NEN = Rule::NEN, NQ = Rule::NQ, NPN = Rule::NPN, MC = Rule::MC;
  constexpr int TPI = 3 * MC;  // tasks (coefficient rows) per incidence
  constexpr int REC = WANT_K ? kRecK : kRecF;
  constexpr int NB = WANT_K ? NEN : 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nn = I1 - I0;
  const int64_t row0 = (int64_t)TPI * I0, row1 = (int64_t)TPI * I1;
  const int64_t seg0 = WANT_K ? g.row_off[row0] : 0, seg1 = WANT_K ? g.row_off[row1] : 0;
  const int nseg = (int)(seg1 - seg0);
  const int nrow = (int)(row1 - row0);
  double* lf = lds + nseg;
  for (int t = tid; t < nseg + nrow; t += nthr) lds[t] = 0.0;
  // the incidence offsets are already a prefix sum: task offsets of the
  // range's nodes follow from one parallel load
  const int32_t inc0 = g.inc_off[I0];
  for (int n = tid; n <= nn; n += nthr) pre[n] = TPI * (g.inc_off[I0 + n] - inc0);
  __syncthreads();
  const int ntask = pre[nn];
  for (int t = tid; t < ntask; t += nthr) {
    int n = 0, hi = nn - 1;  // last node whose first task is <= t
    while (n < hi) {
      const int mid = (n + hi + 1) >> 1;
      if (pre[mid] <= t) n = mid; else hi = mid - 1;
    }
    const int64_t I = I0 + n;
    const int tau = t - pre[n], j = tau / TPI, r = tau % TPI, c = r / 3, i = r % 3;
    const int32_t packed = g.inc[g.inc_off[I] + j];
    const int64_t e = packed >> 4;
    const int a = packed & 15;
    const int al = MC * a + c;
    double scd[4] = {1.0, 1.0, 1.0, 1.0};
    if constexpr (MC == 4) {
      scd[1] = g.escale[2 * e];
      scd[2] = g.escale[2 * e + 1];
      scd[3] = g.half_h;
    }
    const R sc_al = (R)scd[al % 4];
    R acc[NB][3];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b][0] = acc[b][1] = acc[b][2] = R(0);
    R facc = R(0);
    const R* recs = (const R*)g.stage + e * NQ * REC;
    // two-stage pipeline over the points: the row of point q + 1 is in flight
    // while point q is contracted
    RowBuf<R, WANT_K> cur, nxt;
    load_row<R, WANT_K>(recs, i, cur);
    sfor<0, NQ>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (q + 1 < NQ) load_row<R, WANT_K>(recs + (q + 1) * REC, i, nxt);
      const R d0 = (R)Rule::dN_rt(q, al, 0) * sc_al, d1 = (R)Rule::dN_rt(q, al, 1) * sc_al,
              d2 = (R)Rule::dN_rt(q, al, 2) * sc_al;
      if constexpr (WANT_F) facc += cur.p[0] * d0 + cur.p[1] * d1 + cur.p[2] * d2;
      if constexpr (WANT_K) {
        const R* Ar = cur.a;
        R tk[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int nq = 0; nq < 3; ++nq)
            tk[k][nq] = Ar[3 * k + nq] * d0 + Ar[9 + 3 * k + nq] * d1 + Ar[18 + 3 * k + nq] * d2;
        sfor<0, NEN>([&](auto bc) {
          constexpr int b = decltype(bc)::value;
          constexpr double c0 = Rule::dN(q, b, 0), c1 = Rule::dN(q, b, 1), c2 = Rule::dN(q, b, 2);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            R v = acc[b][k];
            if constexpr (c0 != 0.0) v += tk[k][0] * R(c0);
            if constexpr (c1 != 0.0) v += tk[k][1] * R(c1);
            if constexpr (c2 != 0.0) v += tk[k][2] * R(c2);
            acc[b][k] = v;
          }
        });
      }
      if constexpr (q + 1 < NQ) cur = nxt;
    });
    const int64_t row = (int64_t)TPI * I + 3 * c + i;
    if constexpr (WANT_F) atomicAdd(lf + (row - row0), (double)facc);
    if constexpr (WANT_K) {
      const int64_t base = g.row_off[row] - seg0;
      const uint8_t* rk = g.rank + (e * NPN + a) * NPN;
#pragma unroll
      for (int b = 0; b < NEN; ++b) {
        const int pb = (MC == 1) ? b : (b >> 2), cb = (MC == 1) ? 0 : (b & 3);
        double* dst = lds + base + 3 * (MC * (int)rk[pb] + cb);
        const double sb = scd[b % 4];
#pragma unroll
        for (int k = 0; k < 3; ++k) atomicAdd(dst + k, (double)acc[b][k] * sb);
      }
    }
  }
  __syncthreads();
  if constexpr (WANT_K) {
    double* out = g.vals + seg0;
    for (int t = tid; t < nseg; t += nthr) out[t] = ACCUM ? out[t] + lds[t] : lds[t];
  }
  if constexpr (WANT_F) {
    double* out = g.f + row0;
    for (int t = tid; t < nrow; t += nthr) out[t] = ACCUM ? out[t] + lf[t] : lf[t];
  }
}

template <class Rule, typename R, bool WANT_F, bool WANT_K, bool ACCUM>
__global__ __launch_bounds__(256) void k_gather(GatherArgs g) {
  extern __shared__ double lds[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  gather_range<Rule, R, WANT_F, WANT_K, ACCUM>(g, g.ranges[r], g.ranges[r + 1], lds, pre);
}

template <class Rule, typename R>
__global__ __launch_bounds__(256) void k_gather_batch(BatchArgs b) {
  extern __shared__ double lds[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  const BatchRange br = b.ranges[r];
  const BatchBody& B = b.bodies[br.body];
  GatherArgs g;
  g.ranges = nullptr;
  g.inc_off = B.inc_off;
  g.inc = B.inc;
  g.row_off = B.row_off;
  g.rank = B.rank;
  g.escale = B.escale;
  g.half_h = B.half_h;
  g.stage = (const R*)b.stage + B.point_off * kRecK;
  g.f = b.f + B.dof_off;
  g.vals = b.vals + B.nnz_off;
  gather_range<Rule, R, true, true, false>(g, br.I0, br.I1, lds, pre);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int grid_of(int64_t n, int b) { return (int)((n + b - 1) / b); }

template <class Rule, typename R>
int launch_points_rule(const Mesh& m, const AsmArgs& a, bool want_k, hipStream_t s) {
  const int64_t npts = m.n_elem * Rule::NQ;
  if (npts > (int64_t)INT32_MAX * 256) return TLFEA_ERR_TOO_LARGE;
  if (npts == 0) return TLFEA_OK;
  R* stage = (R*)m.d_stage;
  if (want_k)
    hipLaunchKernelGGL((k_stage<Rule, R, true>), dim3(grid_of(npts, 256)), dim3(256), 0, s, a, stage);
  else
    hipLaunchKernelGGL((k_stage<Rule, R, false>), dim3(grid_of(npts, 256)), dim3(256), 0, s, a, stage);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

template <class Rule, typename R>
int launch_nodes_rule(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s) {
  const bool want_f = f != nullptr, want_k = vals != nullptr;
  R* stage = (R*)m.d_stage;
  GatherArgs g{};
  g.ranges = m.d_ranges;
  g.inc_off = m.d_inc_off;
  g.inc = m.d_inc;
  g.row_off = m.d_row_off;
  g.rank = m.d_rank;
  g.escale = m.d_escale;
  g.half_h = 0.5 * m.thickness;
  g.stage = stage;
  g.f = f;
  g.vals = vals;
  const size_t lds = sizeof(double) * (want_k ? m.max_range_values : m.max_range_rows);
  const dim3 grid((unsigned)m.n_ranges), blk(256);
#define TLFEA_GATHER(F, K, A) hipLaunchKernelGGL((k_gather<Rule, R, F, K, A>), grid, blk, lds, s, g)
  if (want_k && want_f) {
    if (accum) TLFEA_GATHER(true, true, true); else TLFEA_GATHER(true, true, false);
  } else if (want_k) {
    if (accum) TLFEA_GATHER(false, true, true); else TLFEA_GATHER(false, true, false);
  } else {
    if (accum) TLFEA_GATHER(true, false, true); else TLFEA_GATHER(true, false, false);
  }
#undef TLFEA_GATHER
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

template <typename R>
int launch_points_prec(const Mesh& m, const AsmArgs& a, bool want_k, hipStream_t s) {
  if (m.elem_type == TLFEA_T10) return launch_points_rule<RuleT10, R>(m, a, want_k, s);
  if (m.gl[0] == 3) return launch_points_rule<RuleAncf<3, 3, 2>, R>(m, a, want_k, s);
  return launch_points_rule<RuleAncf<4, 4, 3>, R>(m, a, want_k, s);
}

template <typename R>
int launch_nodes_prec(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s) {
  if (m.elem_type == TLFEA_T10) return launch_nodes_rule<RuleT10, R>(m, f, vals, accum, s);
  if (m.gl[0] == 3) return launch_nodes_rule<RuleAncf<3, 3, 2>, R>(m, f, vals, accum, s);
  return launch_nodes_rule<RuleAncf<4, 4, 3>, R>(m, f, vals, accum, s);
}

template <class Rule, typename R>
int launch_batch_rule(const BatchArgs& b, int n_ranges, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_batch<Rule, R>), dim3(grid_of(b.n_points, 256)), dim3(256), 0, s, b);
  TLFEA_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_gather_batch<Rule, R>), dim3(n_ranges), dim3(256), lds, s, b);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

__global__ void k_zero(double* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

}  // namespace

size_t stage_bytes(const Mesh& m, bool want_k) {
  const size_t r = m.precision == TLFEA_MIXED ? sizeof(float) : sizeof(double);
  return (size_t)m.n_elem * m.n_qp * (want_k ? kRecK : kRecF) * r;
}

size_t stage_record_bytes(int precision) {
  return (size_t)kRecK * (precision == TLFEA_MIXED ? sizeof(float) : sizeof(double));
}

int launch_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return TLFEA_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

int launch_points(const Mesh& m, const AsmArgs& a, bool want_k, hipStream_t s) {
  if (m.precision == TLFEA_MIXED) return launch_points_prec<float>(m, a, want_k, s);
  return launch_points_prec<double>(m, a, want_k, s);
}

int launch_nodes(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s) {
  if (m.n_ranges == 0) {  // no nodes: only the (empty) outputs to clear
    if (accum) return TLFEA_OK;
    int rc = f ? launch_zero(f, m.n_dof, s) : TLFEA_OK;
    return (rc || !vals) ? rc : launch_zero(vals, m.nnz, s);
  }
  if (m.precision == TLFEA_MIXED) return launch_nodes_prec<float>(m, f, vals, accum, s);
  return launch_nodes_prec<double>(m, f, vals, accum, s);
}

int launch_batch(int elem_type, int gl0, int precision, const BatchArgs& b, int n_ranges, size_t lds,
                 hipStream_t s) {
  if (n_ranges == 0) return TLFEA_OK;
  const bool mixed = precision == TLFEA_MIXED;
  if (elem_type == TLFEA_T10)
    return mixed ? launch_batch_rule<RuleT10, float>(b, n_ranges, lds, s)
                 : launch_batch_rule<RuleT10, double>(b, n_ranges, lds, s);
  if (gl0 == 3)
    return mixed ? launch_batch_rule<RuleAncf<3, 3, 2>, float>(b, n_ranges, lds, s)
                 : launch_batch_rule<RuleAncf<3, 3, 2>, double>(b, n_ranges, lds, s);
  return mixed ? launch_batch_rule<RuleAncf<4, 4, 3>, float>(b, n_ranges, lds, s)
               : launch_batch_rule<RuleAncf<4, 4, 3>, double>(b, n_ranges, lds, s);
}

}  // namespace tlfea
