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
//   pass 1 (one lane per element x quadrature point): gather the element,
//     form F and Fdot in float64, run the constitutive update and store the
//     point's tangent and stress in parent coordinates with the quadrature
//     volume folded in,
//        Ahat_imkn = dV sum_JL J0inv_mJ A_iJkL J0inv_nL,  Phat_im = dV sum_J P_iJ J0inv_mJ,
//     as one record of nine 10-value slots: slot (i, k) holds Ahat_imkn at
//     3 m + n and Phat_ik at 9 (90 values, padded to 96).
//   pass 2 (one workgroup per contiguous range of nodes): the CSR rows of
//     consecutive nodes form one contiguous segment, mirrored in LDS.  Each
//     lane owns one (node, incident element, coefficient row i, component k)
//     task, reads slot (i, k) of the element's records at every point and forms
//        t_n = sum_m dN_a,m Ahat_imkn,   K[a i, b k] += sum_n t_n dN_b,n,
//     where the parent gradients dN_b at each point are compile-time constants
//     (zeros skipped).  Results are added into the LDS segment in float64, and
//     the segment and the node forces are then written with plain coalesced
//     stores.  f_int comes out of the same pass from Phat.
//   Workgroups are remapped so each XCD walks a contiguous range of elements /
//   nodes, keeping the records a range reads in its own L2.
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

#include "kernel_common.h"

// work area of the allocation-free force call, one copy per device
static __device__ __align__(256) unsigned char scratch[TLFEA_NOALLOC_SCRATCH_BYTES];

namespace tlfea {
namespace {

constexpr int kRecK = 96;  // tangent record: nine slots of kSlot values, padded
constexpr int kSlot = 10;  // slot (i, k): Ahat_imkn at 3 m + n, Phat_ik at 9
constexpr int kRecF = 12;  // force-only record: Phat_ik at 4 i + k

// 16-byte vectors as native clang vector types (HIP's struct vector types are
// not always promoted to registers)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Vec4 { using type = f32x4; };
template <>
struct Vec4<double> { using type = f64x2; };

// ordering of LDS accesses between the lanes of one wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
      for (int k = 0; k < 3; ++k) {
        R* slot = rec + kSlot * (3 * i + k);
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
          for (int n = 0; n < 3; ++n) slot[3 * m + n] = hat_entry(h, i, m, k, n);
        slot[9] = h.P[3 * i + k];
      }
#pragma unroll
    for (int t = 9 * kSlot; t < kRecK; ++t) rec[t] = R(0);
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

// Value W of a tangent record (W is a compile-time index into the layout above).
template <int W, typename R>
__device__ __forceinline__ R record_value(const HatOut<R>& h) {
  if constexpr (W < 9 * kSlot) {
    constexpr int slot = W / kSlot, x = W % kSlot, i = slot / 3, k = slot % 3;
    if constexpr (x < 9) return hat_entry(h, i, x / 3, k, x % 3);
    else return h.P[3 * i + k];
  } else {
    return R(0);
  }
}

// Undamped materials: the tangent has major symmetry, Ahat_imkn = Ahat_knim
// (every term of the factored form is symmetric under (i, m) <-> (k, n) once
// the viscous parts are zero), so slot (k, i) is slot (i, k) transposed.  An
// element-row record then holds the six slots with i <= k, in the order (0,0),
// (0,1), (0,2), (1,1), (1,2), (2,2), each as above (Ahat at 3 m + n, Phat_ik at
// 9), then Phat_10, Phat_20, Phat_21 and one pad: 64 values instead of 92.
constexpr int kRecS = 64;

template <int W, typename R>
__device__ __forceinline__ R record_value_sym(const HatOut<R>& h) {
  if constexpr (W < 6 * kSlot) {
    constexpr int sl = W / kSlot, x = W % kSlot;
    constexpr int i = sl < 3 ? 0 : sl < 5 ? 1 : 2, k = sl < 3 ? sl : sl < 5 ? sl - 2 : 2;
    if constexpr (x < 9) return hat_entry(h, i, x / 3, k, x % 3);
    else return h.P[3 * i + k];
  } else if constexpr (W < 6 * kSlot + 3) {
    constexpr int j = W - 6 * kSlot, i = j == 0 ? 1 : 2, k = j == 2 ? 1 : 0;
    return h.P[3 * i + k];
  } else {
    return R(0);
  }
}

// Where the slot (i, k) of a task lies in an element-row record (full or
// symmetric layout), and whether its Ahat block is read transposed.
struct SlotRef {
  int off;  // first Ahat value
  int p;    // Phat_ik
  bool tr;
};
template <bool SYM>
__device__ __forceinline__ SlotRef slot_ref(int i, int k) {
  if constexpr (!SYM) {
    return {kSlot * (3 * i + k), kSlot * (3 * i + k) + 9, false};
  } else {
    const int lo = i < k ? i : k, hi = i < k ? k : i;
    const int sl = lo == 0 ? hi : lo == 1 ? hi + 2 : 5;
    const bool tr = i > k;
    return {kSlot * sl, tr ? 6 * kSlot + i + k - 1 : kSlot * sl + 9, tr};
  }
}

// The ten values of a task's slot at one point of a record in LDS: Ahat_imkn
// at 3 m + n, then Phat_ik.
template <bool SYM>
__device__ __forceinline__ void read_slot(const float* r, const SlotRef& sr, float (&v)[10]) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  if constexpr (!SYM) {
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const f2 w = *reinterpret_cast<const f2*>(r + sr.off + 2 * x);
      v[2 * x] = w[0];
      v[2 * x + 1] = w[1];
    }
  } else {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const f2 w = *reinterpret_cast<const f2*>(r + sr.off + 2 * x);
      v[2 * x] = w[0];
      v[2 * x + 1] = w[1];
    }
    v[8] = r[sr.off + 8];
    v[9] = r[sr.p];
    const float a1 = v[1], a2 = v[2], a5 = v[5];
    v[1] = sr.tr ? v[3] : a1;
    v[3] = sr.tr ? a1 : v[3];
    v[2] = sr.tr ? v[6] : a2;
    v[6] = sr.tr ? a2 : v[6];
    v[5] = sr.tr ? v[7] : a5;
    v[7] = sr.tr ? a5 : v[7];
  }
}

// Pass 1 with the tangent, one workgroup per 256 consecutive (element, point)
// indices.  The nodal values of the workgroup's elements (u = q - X and qdot
// per coefficient) are gathered into LDS once instead of once per point, and
// the records leave through a per-wave LDS transpose: each 128-byte piece of
// the wave's 64 records is one cache line, stored by 8 lanes with 16-byte
// writes, so every store instruction writes 8 whole lines.
template <class Rule>
constexpr int stage_elems() { return (kStageThreads - 1) / Rule::NQ + 2; }

template <class Rule, typename R>
constexpr size_t stage_lds_bytes() {
  const size_t nodal = (size_t)stage_elems<Rule>() * Rule::NEN * 6 * sizeof(double);
  const size_t trans = (size_t)kStageThreads * (128 + 16);
  return nodal > trans ? nodal : trans;
}

template <class Rule, typename R, bool SYM = false>
__device__ __forceinline__ void stage_tile(const AsmArgs& a, R* stage, int64_t blk) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN;
  constexpr int REC = SYM ? kRecS : kRecK;  // record length (symmetric layout for undamped materials)
  constexpr int EB = stage_elems<Rule>();
  using V = typename Vec4<R>::type;
  constexpr int PER = (int)(sizeof(V) / sizeof(R));
  __shared__ __align__(16) unsigned char smem[stage_lds_bytes<Rule, R>()];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t npts = a.n_elem * NQ;
  const int64_t p0 = blk * kStageThreads;
  const int64_t e_lo = p0 / NQ;
  const int64_t p = p0 + tid;
  const bool act = p < npts;
  // 1. nodal values of the elements the block's points belong to
  double* nod = reinterpret_cast<double*>(smem);
  gather_nodal<Rule>(a, e_lo, EB, nod);
  __syncthreads();
  // 2. kinematics at the lane's point (lanes past the end evaluate the last
  //    point and store nothing)
  const int64_t pc = act ? p : npts - 1;
  const int64_t e = pc / NQ;
  const int q = (int)(pc - e * NQ);
  double Jinv[9], det, Hd[9], Fd[9];
  tile_kinematics<Rule>(a, nod + 6 * NEN * (int)(e - e_lo), e, q, Jinv, det, Hd, Fd);
  __syncthreads();  // the nodal values are consumed: the LDS becomes the transpose buffers
  PointOut<R> o;
  const unsigned fl = point_update<R, true>(a.mp, Hd, Fd, det * Rule::w_rt(q), a.alpha, a.beta, o);
  if (act && fl) atomicOr(a.flags, fl);
  HatOut<R> h;
  to_parent<R, true>(o, Jinv, h);
  // 3. records through the per-wave transpose, one 128-byte piece at a time
  constexpr int CW = 128 / (int)sizeof(R);       // values per piece
  constexpr int LS = CW + 16 / (int)sizeof(R);   // lane stride in the buffer (padded)
  R* tb = reinterpret_cast<R*>(smem) + wave * 64 * LS;
  const int64_t pw = p0 + 64 * wave;
  static_assert(REC % CW == 0, "records of whole 128-byte pieces");
  sfor<0, REC / CW>([&](auto cc) __attribute__((always_inline)) {
    constexpr int ch = decltype(cc)::value;
    wave_sync();
    sfor<0, CW / PER>([&](auto jc) __attribute__((always_inline)) {
      constexpr int j = decltype(jc)::value;
      V v;
      sfor<0, PER>([&](auto xc) __attribute__((always_inline)) {
        constexpr int x = decltype(xc)::value;
        if constexpr (SYM) v[x] = record_value_sym<ch * CW + j * PER + x>(h);
        else v[x] = record_value<ch * CW + j * PER + x>(h);
      });
      *reinterpret_cast<V*>(tb + lane * LS + j * PER) = v;
    });
    wave_sync();
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      const int r = 8 * s8 + (lane >> 3), j = lane & 7;
      if (pw + r < npts)
        *reinterpret_cast<V*>(stage + (pw + r) * REC + ch * CW + j * PER) =
            *reinterpret_cast<const V*>(tb + r * LS + j * PER);
    }
  });
}

template <class Rule, typename R, bool SYM>
__global__ __launch_bounds__(kStageThreads) void k_stage_tile(AsmArgs a, R* stage) {
  stage_tile<Rule, R, SYM>(a, stage, blockIdx.x);
}

// many bodies: every body starts on a block of its own, found by bisection
template <class Rule, typename R>
__global__ __launch_bounds__(kStageThreads) void k_stage_batch(BatchArgs b) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = b.n_bodies - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.bodies[mid].block_off <= blk) lo = mid; else hi = mid - 1;
  }
  const BatchBody& B = b.bodies[lo];
  const AsmArgs a = body_args(b, B, lo);
  stage_tile<Rule, R>(a, (R*)b.stage + B.point_off * kRecK, blk - B.block_off);
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
// Values one lane reads per point: its slot of a tangent record, or its Phat
// entry of a force record.
template <typename R, bool WANT_K>
struct Slot {
  static constexpr int N = WANT_K ? kSlot : 1;
  R v[N];
};

// read a slot from the wave's LDS copy of the records (8-byte aligned for
// float, 16-byte aligned for double)
template <typename R, bool WANT_K>
__device__ __forceinline__ void load_slot(const R* p, Slot<R, WANT_K>& s) {
  if constexpr (!WANT_K) {
    s.v[0] = *p;
  } else if constexpr (sizeof(R) == 8) {
#pragma unroll
    for (int t = 0; t < kSlot / 2; ++t) {
      const f64x2 x = reinterpret_cast<const f64x2*>(p)[t];
      s.v[2 * t] = x[0];
      s.v[2 * t + 1] = x[1];
    }
  } else {
#pragma unroll
    for (int t = 0; t < kSlot / 2; ++t) {
      const f32x2 x = reinterpret_cast<const f32x2*>(p)[t];
      s.v[2 * t] = x[0];
      s.v[2 * t + 1] = x[1];
    }
  }
}

// One point's contribution of a task (row i, component k of node a's
// coefficient al): with the slot of the task's element at point Q and the
// task's scaled parent gradient d = dN_al(Q) (times the coefficient scale),
//   t_n = sum_m d_m Ahat_imkn,  acc[b] += sum_n t_n dN_b,n(Q),  facc += Phat_ik d_k.
template <class Rule, typename R, bool WANT_F, bool WANT_K, int Q, int NB, bool KREC = WANT_K>
__device__ __forceinline__ void contract_point(const Slot<R, KREC>& s, R d0, R d1, R d2, int k, R (&acc)[NB],
                                               R& facc) {
  if constexpr (WANT_F) facc += (KREC ? s.v[9] : s.v[0]) * (k == 0 ? d0 : k == 1 ? d1 : d2);
  if constexpr (WANT_K) {
    R tn[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) tn[n] = s.v[n] * d0 + s.v[3 + n] * d1 + s.v[6 + n] * d2;
    sfor<0, Rule::NEN>([&](auto bc) __attribute__((always_inline)) {
      constexpr int b = decltype(bc)::value;
      constexpr double c0 = Rule::dN(Q, b, 0), c1 = Rule::dN(Q, b, 1), c2 = Rule::dN(Q, b, 2);
      R v = acc[b];
      if constexpr (c0 != 0.0) v += tn[0] * R(c0);
      if constexpr (c1 != 0.0) v += tn[1] * R(c1);
      if constexpr (c2 != 0.0) v += tn[2] * R(c2);
      acc[b] = v;
    });
  }
}

// Pass-2 records travel through LDS: the 64 tasks of a wave touch at most
// chunk_incidences() consecutive incidences, whose records are copied, one
// point at a time, into a wave-private LDS buffer with 16-byte loads of
// consecutive lanes (whole cache lines per instruction); each lane then reads
// its own slot from there.  The copies of the next points are in flight in
// registers while a point is contracted.
constexpr int chunk_incidences(int tpi) { return (tpi + 62) / tpi + 1; }

// Float32 tangent records of short rules can be read two ways: through the
// LDS copy, or by the lane itself (its 10-value slot always lies in three
// aligned 16-byte pieces of the record), for all points at once.  The first
// kStagedPoints points take the LDS copy; splitting the points between the two
// paths did not beat reading them all directly (the default, 0).
#ifndef TLFEA_STAGED_POINTS
#define TLFEA_STAGED_POINTS 0
#endif
constexpr int kStagedPoints = TLFEA_STAGED_POINTS;

template <class Rule, typename R, bool WANT_K>
constexpr bool direct_slots() {
  return WANT_K && sizeof(R) == 4 && Rule::NQ <= 6;
}
// points of a rule that go through the LDS copy
template <class Rule, typename R, bool WANT_K>
constexpr int staged_points() {
  return direct_slots<Rule, R, WANT_K>() ? (kStagedPoints < Rule::NQ ? kStagedPoints : Rule::NQ) : Rule::NQ;
}

template <class Rule, typename R, bool WANT_K, bool SYM = false>
constexpr size_t wave_buf_bytes() {
  return staged_points<Rule, R, WANT_K>() == 0
             ? 0
             : (size_t)chunk_incidences(9 * Rule::MC) * (WANT_K ? (SYM ? kRecS : kRecK) : kRecF) * sizeof(R);
}

// The same with a run-time point index q (long rules); q is uniform across the
// wave, so the gradients dN_b(q) come through the scalar cache.
template <class Rule, typename R, bool WANT_F, bool WANT_K, int NB, bool KREC = WANT_K>
__device__ __forceinline__ void contract_point_rt(const Slot<R, KREC>& s, int q, int al, int k, R sc_al,
                                                  R (&acc)[NB], R& facc) {
  const R d0 = (R)Rule::dN_rt(q, al, 0) * sc_al, d1 = (R)Rule::dN_rt(q, al, 1) * sc_al,
          d2 = (R)Rule::dN_rt(q, al, 2) * sc_al;
  if constexpr (WANT_F) facc += (KREC ? s.v[9] : s.v[0]) * (k == 0 ? d0 : k == 1 ? d1 : d2);
  if constexpr (WANT_K) {
    R tn[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) tn[n] = s.v[n] * d0 + s.v[3 + n] * d1 + s.v[6 + n] * d2;
#pragma unroll
    for (int b = 0; b < Rule::NEN; ++b)
      acc[b] += tn[0] * (R)Rule::dN_rt(q, b, 0) + tn[1] * (R)Rule::dN_rt(q, b, 1) + tn[2] * (R)Rule::dN_rt(q, b, 2);
  }
}

// The range's CSR values leave the LDS segment with plain coalesced stores:
// the whole segment, or (upper-triangle output) the suffix of every row from
// its diagonal on.  For the latter the range's upper row offsets are copied
// into LDS (after the force rows; the launch reserves the room), and groups of
// 16 lanes write a row each (one 128-byte line per store).  Called by every
// lane of the workgroup.
template <bool ACCUM>
__device__ __forceinline__ void write_segment(const GatherArgs& g, int64_t row0, int nrow, int nseg, int64_t seg0,
                                              double* lds, const int32_t* rowo) {
  if (!g.row_off_u) {
    double* out = g.vals + seg0;
    for (int t = threadIdx.x; t < nseg; t += blockDim.x) out[t] = ACCUM ? out[t] + lds[t] : lds[t];
    return;
  }
  int32_t* rowu = reinterpret_cast<int32_t*>(lds + nseg + nrow);
  const int32_t u_base = g.row_off_u[row0];
  for (int rr = threadIdx.x; rr <= nrow; rr += blockDim.x) rowu[rr] = g.row_off_u[row0 + rr] - u_base;
  __syncthreads();
  double* out = g.vals + u_base;
  constexpr int GL = 16;  // lanes per row
  const int sub = threadIdx.x % GL, groups = blockDim.x / GL;
  for (int rr = threadIdx.x / GL; rr < nrow; rr += groups) {
    const int u0 = rowu[rr], n = rowu[rr + 1] - u0;
    const int beg = (rr + 1 < nrow ? rowo[rr + 1] : nseg) - n;
    for (int j = sub; j < n; j += GL) out[u0 + j] = ACCUM ? out[u0 + j] + lds[beg + j] : lds[beg + j];
  }
}

// Newton matrix (Sec. 4.4.2, Eq. hessian): the LDS segment of a range starts
// from M_(I,k)(J,l) / h on the diagonal entries (d, d) of every 3x3 block
// ((I,k), (J,l)) of its rows (MC coefficients k per node; the segment is zero
// elsewhere).  Runs after the segment is cleared and before any contribution
// is added.  The range's mass entries (one MC x MC block per adjacent node
// pair) are contiguous in adjacency order, and a node's first entry within the
// range is rowo[3 MC n] / (9 MC^2) (each entry is one 3 x 3 MC piece of each
// of the node's 3 MC rows): a lane per entry finds its node by bisection.
template <int MC>
__device__ __forceinline__ void add_mass_term(const GatherArgs& g, int32_t I0, int nn, double* lds,
                                              const int32_t* rowo) {
  if (!g.mass) return;
  constexpr int RPN = 3 * MC, PER = 9 * MC * MC;
  const int32_t k0 = g.adj_off[I0];
  const int n_ent = g.adj_off[I0 + nn] - k0;
  for (int x = threadIdx.x; x < n_ent; x += blockDim.x) {
    int lo = 0, hi = nn - 1;  // last node whose first entry is <= x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rowo[RPN * mid] / PER <= x) lo = mid; else hi = mid - 1;
    }
    const int r = x - rowo[RPN * lo] / PER;
    const double* mx = g.mass + (int64_t)MC * MC * (k0 + x);
#pragma unroll
    for (int k = 0; k < MC; ++k)
#pragma unroll
      for (int l = 0; l < MC; ++l) {
        const double v = mx[MC * k + l] * g.inv_h;
#pragma unroll
        for (int d = 0; d < 3; ++d) lds[rowo[RPN * lo + 3 * k + d] + 3 * MC * r + 3 * l + d] = v;
      }
  }
}

// A slot read from a symmetric record: the lower slots (i > k) are the upper
// ones transposed, and Phat_ik of a lower slot lies after the six slots.
template <bool SYM, typename R, bool KREC>
__device__ __forceinline__ void sym_slot_fix(Slot<R, KREC>& sl, const R* recb, const SlotRef& sr) {
  if constexpr (SYM) {
    const R a1 = sl.v[1], a2 = sl.v[2], a5 = sl.v[5];
    sl.v[1] = sr.tr ? sl.v[3] : a1;
    sl.v[3] = sr.tr ? a1 : sl.v[3];
    sl.v[2] = sr.tr ? sl.v[6] : a2;
    sl.v[6] = sr.tr ? a2 : sl.v[6];
    sl.v[5] = sr.tr ? sl.v[7] : a5;
    sl.v[7] = sr.tr ? a5 : sl.v[7];
    sl.v[9] = recb[sr.p];
  }
}

// KREC: the records carry the tangent layout (a pass 1 with the tangent); the
// force alone can also be taken from them (WANT_K false).
// SYM: symmetric tangent records (float64 only; the lane's slot may be read
// transposed).
template <class Rule, typename R, bool WANT_F, bool WANT_K, bool ACCUM, bool KREC = WANT_K, bool SYM = false>
__device__ __forceinline__ void gather_range(const GatherArgs& g, int32_t I0, int32_t I1, unsigned char* smem,
                                             int32_t* pre, int32_t* rowo) {
  static_assert(KREC || !WANT_K, "the tangent needs tangent records");
  static_assert(!SYM || (KREC && sizeof(R) == 8), "symmetric records: float64 tangent records");
  constexpr int NQ = Rule::NQ, NPN = Rule::NPN, MC = Rule::MC, NEN = Rule::NEN;
  constexpr int RPN = 3 * MC;  // CSR rows per node
  constexpr int TPI = 3 * RPN; // tasks per incidence: (coefficient kind, row, component)
  constexpr int REC = KREC ? (SYM ? kRecS : kRecK) : kRecF;
  constexpr int NI = chunk_incidences(TPI);
  using V = typename Vec4<R>::type;
  constexpr int PER = (int)(sizeof(V) / sizeof(R));
  constexpr int NV = REC / PER;            // 16-byte pieces per record
  constexpr int KC = (NI * NV + 63) / 64;  // pieces each lane copies per point
  // short rules are unrolled over all points (gradients dN_b as compile-time
  // constants); long rules run over blocks of PB points
  constexpr bool UNROLL = NQ <= 6;
  constexpr int PB = UNROLL ? NQ : 3;
  static_assert(NQ % PB == 0, "point blocks must tile the rule");
  constexpr int PD = UNROLL ? (sizeof(R) == 4 ? NQ : 3) : PB;  // points whose pieces are in flight
  constexpr int NB = WANT_K ? NEN : 1;
  constexpr bool DIRECT = direct_slots<Rule, R, KREC>();
  constexpr int NS = staged_points<Rule, R, KREC>();  // points through the LDS copy (DIRECT: the first NS)
  constexpr int PDS = DIRECT ? (NS > 0 ? NS : 1) : PD;     // staged points in flight
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  // LDS: incidence -> node table, wave record buffers, CSR segment + forces
  uint8_t* incn = smem;
  R* wbuf = reinterpret_cast<R*>(smem + g.inc_cap) + wave * NI * REC;
  double* lds = reinterpret_cast<double*>(smem + g.inc_cap + nwave * wave_buf_bytes<Rule, R, KREC, SYM>());
  const int nn = I1 - I0;
  const int64_t row0 = (int64_t)RPN * I0, row1 = (int64_t)RPN * I1;
  const int64_t seg0 = WANT_K ? g.row_off[row0] : 0, seg1 = WANT_K ? g.row_off[row1] : 0;
  const int nseg = (int)(seg1 - seg0);
  const int nrow = (int)(row1 - row0);
  double* lf = lds + nseg;
  for (int t = tid; t < nseg + nrow; t += blockDim.x) lds[t] = 0.0;
  // the incidence offsets are already a prefix sum: task offsets of the
  // range's nodes follow from one parallel load
  const int32_t inc0 = g.inc_off[I0];
  for (int n = tid; n <= nn; n += blockDim.x) pre[n] = TPI * (g.inc_off[I0 + n] - inc0);
  // segment-relative offsets of the range's CSR rows
  if constexpr (WANT_K)
    for (int rr = tid; rr < nrow; rr += blockDim.x) rowo[rr] = (int32_t)(g.row_off[row0 + rr] - seg0);
  __syncthreads();
  // range-local node of every incidence (nodes < kMaxRangeNodes fit a byte)
  for (int n = tid; n < nn; n += blockDim.x)
    for (int j = pre[n] / TPI; j < pre[n + 1] / TPI; ++j) incn[j] = (uint8_t)n;
  if constexpr (WANT_K) add_mass_term<MC>(g, I0, nn, lds, rowo);
  __syncthreads();
  const int ntask = pre[nn];
  // Tasks are ordered (node, incidence, kind, row, component): task t belongs
  // to incidence inc0 + t / TPI of the range.  The wave's chunk of an
  // iteration starting at task t0 covers incidences j0 .. j0 + ni - 1; lanes
  // past the last task repeat it and store nothing, and copy pieces past the
  // chunk's end repeat its last piece (in bounds, same value written twice).
  auto chunk = [&](int t0_, int& j0_, int& ni_) __attribute__((always_inline)) {
    const int cw = min(t0_ + 64 * wave, ntask - 1);
    j0_ = cw / TPI;
    ni_ = min(cw + 63, ntask - 1) / TPI - j0_ + 1;
  };
  // the lane's copy pieces in a full chunk (record rr0, piece pp0); in a
  // short chunk, pieces past its end become its last piece (ni - 1, NV - 1)
  int rr0[KC], pp0[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    rr0[k] = (lane + 64 * k) / NV;
    pp0[k] = lane + 64 * k - rr0[k] * NV;
  }
  // record addresses in 16-byte units (32 bits: checked on the host)
  const V* stagev = reinterpret_cast<const V*>(g.stage);
  constexpr uint32_t VPP = REC / PER;  // 16-byte pieces per point record
  // incidence entries an iteration needs (its copy pieces' and the lane's
  // own), fetched one iteration ahead
  auto fetch_inc = [&](int t0_, int32_t (&icp)[KC], int32_t& ime) __attribute__((always_inline)) {
    int j0_, ni_;
    chunk(t0_, j0_, ni_);
    if constexpr (NS > 0) {
#pragma unroll
      for (int k = 0; k < KC; ++k) icp[k] = g.inc[inc0 + j0_ + min(rr0[k], ni_ - 1)];
    }
    ime = g.inc[inc0 + min(t0_ + tid, ntask - 1) / TPI];
  };
  int32_t icp[KC], ime;
  fetch_inc(0, icp, ime);
  for (int t0 = 0; t0 < ntask; t0 += blockDim.x) {  // uniform across the workgroup
    const bool act = t0 + tid < ntask;
    const int t = min(t0 + tid, ntask - 1);
    int j0, ni;
    chunk(t0, j0, ni);
    uint32_t src[KC];
    int dst[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const bool in = rr0[k] < ni;
      src[k] = (uint32_t)(icp[k] >> 4) * (NQ * VPP) + (uint32_t)(in ? pp0[k] : NV - 1);
      dst[k] = in ? rr0[k] * REC + pp0[k] * PER : ni * REC - PER;
    }
    V buf[PDS][KC];
    if constexpr (NS > 0) {
      sfor<0, PDS>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
#pragma unroll
        for (int k = 0; k < KC; ++k) buf[q][k] = stagev[src[k] + q * VPP];
      });
    }
    const int32_t packed = ime;
    if (t0 + (int)blockDim.x < ntask) fetch_inc(t0 + blockDim.x, icp, ime);
    const int n = incn[t / TPI];
    const int r = t % TPI, ca = r / 9, i = (r / 3) % 3, k = r % 3;  // pre[] holds multiples of TPI
    const int64_t e = packed >> 4;
    const int a = packed & 15;
    const int al = MC * a + ca;
    const SlotRef sr = slot_ref<SYM>(i, k);
    const R* recb = wbuf + (t / TPI - j0) * REC;  // the lane's record in the wave buffer
    const R* mine = recb + (KREC ? sr.off : 4 * i + k);
    // slot-map row of (e, a): one aligned vector load
    constexpr int RST = rank_stride(NPN);
    uint32_t rkw[RST / 4];
    if constexpr (WANT_K) {
      const uint32_t* rp = reinterpret_cast<const uint32_t*>(g.rank + (e * NPN + a) * RST);
      if constexpr (RST == 16) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 w = *reinterpret_cast<const u32x4*>(rp);
        rkw[0] = w[0];
        rkw[1] = w[1];
        rkw[2] = w[2];
        rkw[3] = w[3];
      } else {
        rkw[0] = rp[0];
      }
    }
    double scd[4] = {1.0, 1.0, 1.0, 1.0};
    if constexpr (MC == 4) {
      scd[1] = g.escale[2 * e];
      scd[2] = g.escale[2 * e + 1];
      scd[3] = g.half_h;
    }
    const R sc_al = (R)(ca == 0 ? scd[0] : ca == 1 ? scd[1] : ca == 2 ? scd[2] : scd[3]);
    R acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = R(0);
    R facc = R(0);
    // DIRECT: the lane's slot s = 3 i + k sits at value 10 s of each point
    // record, inside pieces floor(10 s / 4) .. + 2, shifted by 0 (s even) or 2
    V own[DIRECT && NQ > NS ? NQ - NS : 1][3];
    const bool odd_slot = (3 * i + k) & 1;
    if constexpr (DIRECT && NQ > NS) {
      const uint32_t p0 = (uint32_t)(packed >> 4) * (NQ * VPP) + (uint32_t)((kSlot * (3 * i + k)) >> 2);
#pragma unroll
      for (int q = NS; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < 3; ++j) own[q - NS][j] = stagev[p0 + q * VPP + j];
    }
    if constexpr (UNROLL) {
      // the task's parent gradients at all points: one row of the table
      R dna[16];
      {
        using V4 = typename Vec4<R>::type;
        constexpr int P4 = (int)(sizeof(V4) / sizeof(R));
        const V4* rowv = reinterpret_cast<const V4*>(Rule::template rows<R>(al));
#pragma unroll
        for (int t = 0; t < 16 / P4; ++t) {
          const V4 x = rowv[t];
#pragma unroll
          for (int u = 0; u < P4; ++u) dna[P4 * t + u] = x[u] * sc_al;
        }
      }
      sfor<0, NQ>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        Slot<R, KREC> sl;
        if constexpr (DIRECT && q >= NS) {
#pragma unroll
          for (int x = 0; x < kSlot; ++x) {
            const R lo = own[q - NS][x >> 2][x & 3], hi = own[q - NS][(x + 2) >> 2][(x + 2) & 3];
            sl.v[x] = odd_slot ? hi : lo;
          }
        } else {
          wave_sync();  // every lane is done with the previous point's records
#pragma unroll
          for (int kk = 0; kk < KC; ++kk) *reinterpret_cast<V*>(wbuf + dst[kk]) = buf[q % PDS][kk];
          wave_sync();
          if constexpr (q + PDS < NS) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk)
              buf[q % PDS][kk] = stagev[src[kk] + (q + PDS) * VPP];
          }
          load_slot<R, KREC>(mine, sl);
          sym_slot_fix<SYM>(sl, recb, sr);
        }
        contract_point<Rule, R, WANT_F, WANT_K, q, NB, KREC>(sl, dna[3 * q], dna[3 * q + 1], dna[3 * q + 2], k, acc,
                                                             facc);
      });
    } else {
#pragma unroll 1
      for (int qb = 0; qb < NQ; qb += PB) {
        sfor<0, PB>([&](auto xc) __attribute__((always_inline)) {
          constexpr int x = decltype(xc)::value;
          const int q = qb + x;
          wave_sync();
#pragma unroll
          for (int kk = 0; kk < KC; ++kk) *reinterpret_cast<V*>(wbuf + dst[kk]) = buf[x][kk];
          wave_sync();
          if (q + PB < NQ) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk)
              buf[x][kk] = stagev[src[kk] + (uint32_t)(q + PB) * VPP];
          }
          Slot<R, KREC> sl;
          load_slot<R, KREC>(mine, sl);
          sym_slot_fix<SYM>(sl, recb, sr);
          contract_point_rt<Rule, R, WANT_F, WANT_K, NB, KREC>(sl, q, al, k, sc_al, acc, facc);
        });
      }
    }
    if (act) {
      const int rl = RPN * n + 3 * ca + i;  // row within the range
      if constexpr (WANT_F) atomicAdd(lf + rl, (double)facc);
      if constexpr (WANT_K) {
        double* dstp = lds + rowo[rl] + k;
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
          const int pb = (MC == 1) ? b : (b >> 2), cb = (MC == 1) ? 0 : (b & 3);
          const int rank_b = (int)((rkw[pb >> 2] >> (8 * (pb & 3))) & 255u);
          atomicAdd(dstp + 3 * (MC * rank_b + cb), (double)acc[b] * scd[b % 4]);
        }
      }
    }
  }
  __syncthreads();
  if constexpr (WANT_K) write_segment<ACCUM>(g, row0, nrow, nseg, seg0, lds, rowo);
  if constexpr (WANT_F) {
    double* out = g.f + row0;
    for (int t = tid; t < nrow; t += blockDim.x) out[t] = ACCUM ? out[t] + lf[t] : lf[t];
  }
}

template <class Rule, typename R, bool WANT_F, bool WANT_K, bool ACCUM, bool KREC, bool SYM>
__global__ __launch_bounds__(512) void k_gather(GatherArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 3 * Rule::MC];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  gather_range<Rule, R, WANT_F, WANT_K, ACCUM, KREC, SYM>(g, g.ranges[r], g.ranges[r + 1], smem, pre, rowo);
}

template <class Rule, typename R>
__global__ __launch_bounds__(512) void k_gather_batch(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 3 * Rule::MC];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  const BatchRange br = b.ranges[r];
  const BatchBody& B = b.bodies[br.body];
  GatherArgs g{};
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
  g.inc_cap = b.inc_cap;
  gather_range<Rule, R, true, true, false>(g, br.I0, br.I1, smem, pre, rowo);
}

// ---------------------------------------------------------------------------
// element rows (T10, float32, with the tangent)
// ---------------------------------------------------------------------------
// Pass 1 reduces over the points itself.  A workgroup computes the records of
// kRowElems whole elements into LDS (a lane per point, as above), then a lane
// per task (element, node a, row i, component k) contracts the element's five
// records exactly as the gather does, giving the ten entries
// K_e[3a+i][3b+k], b = 0..9, summed over the points in float32 (Sec. 4.4.2,
// Eq. tangent_block), and its part P_ik dN_a,k of f_a,i (Eq. fint_local).
// Each (element, node) row block goes to the node's place in the node-sorted
// incidence list, so that pass 2 reads the blocks of a node range as one
// contiguous run, each block once, instead of re-reading per-point records
// for every range that shares an element.
constexpr int kRowBlk = 96;       // block: K entry (i, k, b) at 10 (3 i + k) + b, f_i at 90 + i
constexpr int kRowElems = 25;     // elements per pass-1 workgroup
constexpr int kRowThreads = 128;  // 125 point lanes
constexpr int kRecL = 92;         // LDS record stride in values (a 16-byte multiple)
constexpr int kRowStage = 7;      // incidences a wave contracts at a time (63 of its lanes)
constexpr int kDnL = 20;          // LDS stride of a node's gradient row (16 used; 20 keeps the rows
                                  // of the ten nodes on different banks)
constexpr int kStgL = 100;        // LDS stride of a staged row block (96 used; spreads the banks)

// Phase B of the element rows for a symmetric tangent (undamped materials):
// K_e^(ki)[b, a] = K_e^(ik)[a, b], so only the slots i <= k are contracted.
// A wave takes one element at a time, a lane per task (node a, slot i <= k):
// 60 lanes, each forming the ten entries K_e[3a+i][3b+k] over the points.  The
// lanes put them into the element's ten row blocks in the wave's LDS buffer,
// at (a, i, k, b) and, for i < k, transposed at (b, k, i, a); f_a,i is the sum
// of the parts Phat_ik dN_a,k of the node's lanes, in a fixed order.  Then the
// wave stores the ten blocks with 16-byte stores of consecutive lanes.  Two
// thirds of the multiply-adds of the full contraction.
template <class Rule, int EB>
__device__ __forceinline__ void elem_rows_sym_contract(const int32_t* __restrict__ incpos, float* __restrict__ rows,
                                                       int64_t e0, int ne, const float* rec, const float* dn,
                                                       float* stage_buf) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN;
  static_assert(6 * NEN <= 64, "a lane per (node, upper slot)");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* stg = stage_buf + wave * NEN * kStgL;
  const int tl = lane < 6 * NEN ? lane : 0;  // lanes past the tasks repeat task 0 and store nothing
  const int an = tl / 6, us = tl - 6 * an;
  const int i = us < 3 ? 0 : us < 5 ? 1 : 2, k = us < 3 ? us : us < 5 ? us - 2 : 2;
  const int so = kSlot * us, pt = 6 * kSlot + i + k - 1;  // the slot, Phat_ki (i < k)
  float dna[16];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const f32x4 x = reinterpret_cast<const f32x4*>(dn + kDnL * an)[u];
    dna[4 * u] = x[0];
    dna[4 * u + 1] = x[1];
    dna[4 * u + 2] = x[2];
    dna[4 * u + 3] = x[3];
  }
  for (int le = wave; le < ne; le += kRowThreads / 64) {  // uniform per wave
    const int32_t my_pos = lane < NEN ? incpos[(e0 + le) * NEN + lane] : 0;
    float acc[NEN], fd = 0.0f, ft = 0.0f;
#pragma unroll
    for (int b = 0; b < NEN; ++b) acc[b] = 0.0f;
    const float* base = rec + le * NQ * kRecS;
    sfor<0, NQ>([&](auto qc) __attribute__((always_inline)) {
      constexpr int qq = decltype(qc)::value;
      const float* r = base + qq * kRecS;
      Slot<float, true> sv;
#pragma unroll
      for (int x = 0; x < 5; ++x) {
        const f32x2 w = *reinterpret_cast<const f32x2*>(r + so + 2 * x);
        sv.v[2 * x] = w[0];
        sv.v[2 * x + 1] = w[1];
      }
      const float d0 = dna[3 * qq], d1 = dna[3 * qq + 1], d2 = dna[3 * qq + 2];
      contract_point<Rule, float, true, true, qq, NEN>(sv, d0, d1, d2, k, acc, fd);
      if (i < k) ft += r[pt] * (i == 0 ? d0 : d1);  // Phat_ki dN_a,i
    });
    wave_sync();  // the previous element's blocks have left the buffer
    if (lane < 6 * NEN) {
      float* own = stg + an * kStgL + kSlot * (3 * i + k);
#pragma unroll
      for (int u = 0; u < NEN / 2; ++u) {
        f32x2 v;
        v[0] = acc[2 * u];
        v[1] = acc[2 * u + 1];
        *reinterpret_cast<f32x2*>(own + 2 * u) = v;
      }
      if (i < k) {
#pragma unroll
        for (int b = 0; b < NEN; ++b) stg[b * kStgL + kSlot * (3 * k + i) + an] = acc[b];
      }
    }
    // f_a,0 = (0,0) + (0,1) + (0,2);  f_a,1 = (1,0) + (1,1) + (1,2);  f_a,2 = (2,0) + (2,1) + (2,2),
    // the (k, i) parts with k > i from the lanes of slot (i, k)
    const int l0 = 6 * an;
    const float d01 = __shfl(fd, l0 + 1, 64), d02 = __shfl(fd, l0 + 2, 64), d12 = __shfl(fd, l0 + 4, 64);
    const float t01 = __shfl(ft, l0 + 1, 64), t02 = __shfl(ft, l0 + 2, 64), t12 = __shfl(ft, l0 + 4, 64);
    const float d00 = __shfl(fd, l0, 64), d11 = __shfl(fd, l0 + 3, 64), d22 = __shfl(fd, l0 + 5, 64);
    if (lane < 6 * NEN && us < 3) {
      const float fv = us == 0 ? (d00 + d01) + d02 : us == 1 ? (t01 + d11) + d12 : (t02 + t12) + d22;
      stg[an * kStgL + 9 * kSlot + us] = fv;
      stg[an * kStgL + 9 * kSlot + 3 + us] = 0.0f;
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < (NEN * kRowBlk / 4 + 63) / 64; ++u) {
      const int pc = lane + 64 * u, bl = pc / (kRowBlk / 4), pi = pc - bl * (kRowBlk / 4);
      const int32_t pb = __shfl(my_pos, bl < NEN ? bl : 0, 64);
      if (bl < NEN)
        *reinterpret_cast<f32x4*>(rows + (int64_t)pb * kRowBlk + 4 * pi) =
            *reinterpret_cast<const f32x4*>(stg + bl * kStgL + 4 * pi);
    }
  }
}

template <class Rule, int EB = kRowElems, bool SYM = false>
__device__ __forceinline__ void elem_rows_tile(const AsmArgs& a, const int32_t* __restrict__ incpos,
                                               float* __restrict__ rows, int64_t blk) {
  static_assert(Rule::MC == 1 && Rule::NEN == 10, "element rows are built for T10");
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN;
  constexpr int REC = SYM ? kRecS : kRecL;  // LDS record stride
  static_assert(EB * NQ <= kRowThreads, "a lane per point");
  static_assert(kRowThreads % 64 == 0 && 9 * kRowStage <= 64, "a wave stages whole incidences");
  __shared__ __align__(16) float rec[EB * NQ * REC];
  __shared__ __align__(16) float dn[NEN * kDnL];  // parent gradients of every node at every point
  __shared__ int32_t pos[SYM ? 1 : EB * NEN];     // incidence position of every (element, node)
  __shared__ __align__(16) float stage_buf[(kRowThreads / 64) * (SYM ? NEN : kRowStage) * kStgL];  // per-wave blocks
  static_assert(EB * NEN * 6 * sizeof(double) <= sizeof(rec), "nodal values fit the record area");
  const int tid = threadIdx.x;
  const int64_t e0 = blk * EB;
  const int ne = (int)(a.n_elem - e0 < EB ? a.n_elem - e0 : EB);
  // 1. nodal values, the tables of the tasks, then each point's kinematics
  double* nod = reinterpret_cast<double*>(rec);
  gather_nodal<Rule>(a, e0, ne, nod);
  if constexpr (!SYM)
    for (int idx = tid; idx < ne * NEN; idx += kRowThreads) pos[idx] = incpos[e0 * NPN + idx];
  for (int idx = tid; idx < NEN * 16; idx += kRowThreads) dn[kDnL * (idx / 16) + idx % 16] = Rule::template rows<float>(idx / 16)[idx % 16];
  __syncthreads();
  const bool act = tid < ne * NQ;
  const int pl = act ? tid : 0;  // idle lanes evaluate point 0 and store nothing
  const int el = pl / NQ, q = pl - el * NQ;
  double Jinv[9], det, Hd[9], Fd[9];
  tile_kinematics<Rule>(a, nod + 6 * NEN * el, e0 + el, q, Jinv, det, Hd, Fd);
  __syncthreads();  // the nodal values are consumed: the LDS holds the records from here on
  // 2. the point's record (slot layout of the records above) into LDS
  PointOut<float> o;
  const unsigned fl = point_update<float, true>(a.mp, Hd, Fd, det * Rule::w_rt(q), a.alpha, a.beta, o);
  if (act && fl) atomicOr(a.flags, fl);
  HatOut<float> h;
  to_parent<float, true>(o, Jinv, h);
  if (act) {
    float* r = rec + pl * REC;
    sfor<0, REC / 4>([&](auto jc) __attribute__((always_inline)) {
      constexpr int j = decltype(jc)::value;
      f32x4 v;
      sfor<0, 4>([&](auto xc) __attribute__((always_inline)) {
        constexpr int x = decltype(xc)::value;
        if constexpr (SYM) v[x] = record_value_sym<4 * j + x>(h);
        else v[x] = record_value<4 * j + x>(h);
      });
      *reinterpret_cast<f32x4*>(r + 4 * j) = v;
    });
  }
  __syncthreads();
  if constexpr (SYM) {
    elem_rows_sym_contract<Rule, EB>(incpos, rows, e0, ne, rec, dn, stage_buf);
  } else {
  // 3. a lane per task: each wave takes 2 x 7 whole incidences at a time (63
  //    lanes, two tasks of the same slot each), contracts the element's
  //    points, and stages the row blocks, 7 at a time, in its LDS buffer; f_a,i
  //    is the sum of the three component lanes' parts, taken in a fixed order.
  //    The blocks leave with 16-byte stores of consecutive lanes (whole cache
  //    lines).
  const int lane = tid & 63, wave = tid >> 6;
  float* stg = stage_buf + wave * kRowStage * kStgL;
  const int li = lane / 9, sl = lane - 9 * li, i = sl / 3, k = sl - 3 * i;  // lane 63: li = 7, idle
  const int n_inc = ne * NEN;
  constexpr int kGroup = 2 * kRowStage;  // incidences per wave and iteration
  for (int c0 = kGroup * wave; c0 < n_inc; c0 += kGroup * (kRowThreads / 64)) {  // uniform per wave
    float acc[2][NEN], facc[2];
    sfor<0, 2>([&](auto hc) __attribute__((always_inline)) {
      constexpr int hh = decltype(hc)::value;
      const int ci = c0 + kRowStage * hh + li;
      const int cc = (li < kRowStage && ci < n_inc) ? ci : c0;  // idle lanes repeat a live incidence
      const int le = cc / NEN, an = cc - NEN * le;
      float dna[16];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const f32x4 x = reinterpret_cast<const f32x4*>(dn + kDnL * an)[u];
        dna[4 * u] = x[0];
        dna[4 * u + 1] = x[1];
        dna[4 * u + 2] = x[2];
        dna[4 * u + 3] = x[3];
      }
#pragma unroll
      for (int b = 0; b < NEN; ++b) acc[hh][b] = 0.0f;
      facc[hh] = 0.0f;
      const float* base = rec + le * NQ * REC;
      const SlotRef sr = slot_ref<SYM>(i, k);
      sfor<0, NQ>([&](auto qc) __attribute__((always_inline)) {
        constexpr int qq = decltype(qc)::value;
        Slot<float, true> sv;
        read_slot<SYM>(base + qq * REC, sr, sv.v);
        contract_point<Rule, float, true, true, qq, NEN>(sv, dna[3 * qq], dna[3 * qq + 1], dna[3 * qq + 2], k,
                                                         acc[hh], facc[hh]);
      });
    });
    sfor<0, 2>([&](auto hc) __attribute__((always_inline)) {
      constexpr int hh = decltype(hc)::value;
      const int g0 = c0 + kRowStage * hh;  // first incidence of this half
      const float f1 = __shfl_down(facc[hh], 1, 64), f2 = __shfl_down(facc[hh], 2, 64);
      wave_sync();  // the previous blocks have left the buffer
      if (li < kRowStage) {
        float* blk = stg + li * kStgL;
#pragma unroll
        for (int u = 0; u < NEN / 2; ++u) {
          f32x2 v;
          v[0] = acc[hh][2 * u];
          v[1] = acc[hh][2 * u + 1];
          *reinterpret_cast<f32x2*>(blk + kSlot * sl + 2 * u) = v;
        }
        if (k == 0) blk[9 * kSlot + i] = (facc[hh] + f1) + f2;
        if (sl < 3) blk[9 * kSlot + 3 + sl] = 0.0f;
      }
      wave_sync();
      const int nb = n_inc - g0 < kRowStage ? n_inc - g0 : kRowStage;  // blocks of this half (may be <= 0)
#pragma unroll
      for (int u = 0; u < (kRowStage * kRowBlk / 4 + 63) / 64; ++u) {
        const int pc = lane + 64 * u, bl = pc / (kRowBlk / 4), pi = pc - bl * (kRowBlk / 4);
        if (bl < nb)
          *reinterpret_cast<f32x4*>(rows + (int64_t)pos[g0 + bl] * kRowBlk + 4 * pi) =
              *reinterpret_cast<const f32x4*>(stg + bl * kStgL + 4 * pi);
      }
    });
  }
  }
}

template <class Rule, bool SYM>
__global__ __launch_bounds__(kRowThreads) void k_elem_rows(AsmArgs a, const int32_t* incpos, float* rows) {
  elem_rows_tile<Rule, kRowElems, SYM>(a, incpos, rows, blockIdx.x);
}

// many bodies: every body starts on a workgroup of its own, found by bisection
template <class Rule>
__global__ __launch_bounds__(kRowThreads) void k_elem_rows_batch(BatchArgs b) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = b.n_bodies - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.bodies[mid].rblock_off <= blk) lo = mid; else hi = mid - 1;
  }
  const BatchBody& B = b.bodies[lo];
  const AsmArgs a = body_args(b, B, lo);
  elem_rows_tile<Rule>(a, B.incpos, (float*)b.stage + B.blk_inc_off * kRowBlk, blk - B.rblock_off);
}

// Persistent form of the batch (the LPT schedule): a grid sized to what the
// GPU holds at once, whose workgroups take (body, tile) items from a counter
// in a list ordered longest first (full tiles of the largest bodies first,
// partial tiles last), EB elements per tile.
template <class Rule, int EB>
__global__ __launch_bounds__(kRowThreads) void k_elem_rows_batch_lpt(BatchArgs b, const int2* __restrict__ items,
                                                                    int n_items, unsigned* __restrict__ counter) {
  __shared__ int item;
  for (;;) {
    __syncthreads();  // the previous item's LDS and its item index are consumed
    if (threadIdx.x == 0) item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = item;
    if (it >= n_items) return;  // every wave of the workgroup leaves here together
    const int2 t = items[it];
    const BatchBody& B = b.bodies[t.x];
    const AsmArgs a = body_args(b, B, t.x);
    elem_rows_tile<Rule, EB>(a, B.incpos, (float*)b.stage + B.blk_inc_off * kRowBlk, t.y);
  }
}

__global__ void k_reset_counters(unsigned* counters) {
  if (threadIdx.x < 2) counters[threadIdx.x] = 0u;
}

// Pass 2 over the row blocks: a lane per (incidence, row i, component k) task
// of the range loads its ten K entries (three aligned 16-byte pieces of the
// block, shifted by 2 values for odd slots) and adds them into the range's
// LDS segment at row + 3 rank_b + k; lanes with k = 0 add the force entry.
template <bool WANT_F, bool WANT_K, bool ACCUM>
__device__ __forceinline__ void gather_rows(const GatherArgs& g, int32_t I0, int32_t I1, unsigned char* smem,
                                            int32_t* pre, int32_t* rowo) {
  constexpr int TPI = 9;
  const int tid = threadIdx.x;
  uint8_t* incn = smem;
  double* lds = reinterpret_cast<double*>(smem + g.inc_cap);
  const int nn = I1 - I0;
  const int64_t row0 = 3LL * I0, row1 = 3LL * I1;
  const int64_t seg0 = WANT_K ? g.row_off[row0] : 0, seg1 = WANT_K ? g.row_off[row1] : 0;
  const int nseg = (int)(seg1 - seg0);
  const int nrow = (int)(row1 - row0);
  double* lf = lds + nseg;
  for (int t = tid; t < nseg + nrow; t += blockDim.x) lds[t] = 0.0;
  const int32_t inc0 = g.inc_off[I0];
  for (int n = tid; n <= nn; n += blockDim.x) pre[n] = TPI * (g.inc_off[I0 + n] - inc0);
  if constexpr (WANT_K)
    for (int rr = tid; rr < nrow; rr += blockDim.x) rowo[rr] = (int32_t)(g.row_off[row0 + rr] - seg0);
  __syncthreads();
  for (int n = tid; n < nn; n += blockDim.x)
    for (int j = pre[n] / TPI; j < pre[n + 1] / TPI; ++j) incn[j] = (uint8_t)n;
  if constexpr (WANT_K) add_mass_term<1>(g, I0, nn, lds, rowo);
  __syncthreads();
  const int ntask = pre[nn];
  const float* blk = reinterpret_cast<const float*>(g.stage);
  const f32x4* blkv = reinterpret_cast<const f32x4*>(g.stage);
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  for (int t = tid; t < ntask; t += blockDim.x) {
    const int jl = t / TPI, sl = t - TPI * jl, i = sl / 3, k = sl - 3 * i;
    const uint32_t j = (uint32_t)(inc0 + jl);
    const int rl = 3 * incn[jl] + i;
    if constexpr (WANT_K) {
      // 16-byte units with 32-bit offsets (checked on the host)
      const uint32_t p0 = j * (uint32_t)(kRowBlk / 4) + (uint32_t)((kSlot * sl) >> 2);
      const f32x4 w[3] = {blkv[p0], blkv[p0 + 1], blkv[p0 + 2]};
      const u32x4 rw = *reinterpret_cast<const u32x4*>(g.rank + (size_t)j * 16);
      const bool odd = sl & 1;
      double* dstp = lds + rowo[rl] + k;
#pragma unroll
      for (int b = 0; b < 10; ++b) {
        const float lo = w[b >> 2][b & 3], hi = w[(b + 2) >> 2][(b + 2) & 3];
        const int rank_b = (int)((rw[b >> 2] >> (8 * (b & 3))) & 255u);
        atomicAdd(dstp + 3 * rank_b, (double)(odd ? hi : lo));
      }
    }
    if constexpr (WANT_F)
      if (k == 0) atomicAdd(lf + rl, (double)blk[(size_t)j * kRowBlk + 9 * kSlot + i]);
  }
  __syncthreads();
  if constexpr (WANT_K) write_segment<ACCUM>(g, row0, nrow, nseg, seg0, lds, rowo);
  if constexpr (WANT_F) {
    double* out = g.f + row0;
    for (int t = tid; t < nrow; t += blockDim.x) out[t] = ACCUM ? out[t] + lf[t] : lf[t];
  }
}

template <bool WANT_F, bool WANT_K, bool ACCUM>
__global__ __launch_bounds__(512) void k_gather_rows(GatherArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 3];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  gather_rows<WANT_F, WANT_K, ACCUM>(g, g.ranges[r], g.ranges[r + 1], smem, pre, rowo);
}

__global__ __launch_bounds__(512) void k_gather_rows_batch(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 3];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  const BatchRange br = b.ranges[r];
  const BatchBody& B = b.bodies[br.body];
  GatherArgs g{};
  g.inc_off = B.inc_off;
  g.row_off = B.row_off;
  g.rank = B.rank_inc;
  g.stage = (const float*)b.stage + B.blk_inc_off * kRowBlk;
  g.f = b.f + B.dof_off;
  g.vals = b.vals + B.nnz_off;
  g.inc_cap = b.inc_cap;
  gather_rows<true, true, false>(g, br.I0, br.I1, smem, pre, rowo);
}

// persistent form: ranges taken from a counter, largest first
__global__ __launch_bounds__(512) void k_gather_rows_batch_lpt(BatchArgs b, const int32_t* __restrict__ order,
                                                               int n_items, unsigned* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 3];
  __shared__ int item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = item;
    if (it >= n_items) return;
    const BatchRange br = b.ranges[order[it]];
    const BatchBody& B = b.bodies[br.body];
    GatherArgs g{};
    g.inc_off = B.inc_off;
    g.row_off = B.row_off;
    g.rank = B.rank_inc;
    g.stage = (const float*)b.stage + B.blk_inc_off * kRowBlk;
    g.f = b.f + B.dof_off;
    g.vals = b.vals + B.nnz_off;
    g.inc_cap = b.inc_cap;
    gather_rows<true, true, false>(g, br.I0, br.I1, smem, pre, rowo);
  }
}

// ---------------------------------------------------------------------------
// element rows for ANCF (four coefficient vectors per node; float32 tangent)
// ---------------------------------------------------------------------------
// The same split as for T10, for the shell and the beam: pass 1 contracts an
// element's points itself and leaves one block per (element, node) incidence
// at the node's place in the node-sorted incidence list; pass 2 reads every
// block once.  Block of an incidence: for row r = 3 c + i (coefficient kind c
// of the node, component i) and column component k, the NEN entries
// K_e[(a, i), (b, k)] over the element's coefficients b at (3 r + k) NEN + b,
// then the parts P^_ik dN_a,k s_a of f_a,i at 36 NEN + 3 r + k (the three
// parts of a row are added in pass 2).
constexpr int kRowsMcThreads = 128;
#ifndef TLFEA_ROWS_MC_UNROLL
#define TLFEA_ROWS_MC_UNROLL 2
#endif
constexpr int kRowsMcUnroll = TLFEA_ROWS_MC_UNROLL;  // points contracted per step (divides 12, 18 and 48)
template <class Rule>
constexpr int rows_mc_elems() { return kRowsMcThreads / Rule::NQ; }
template <int NEN>
constexpr int rows_mc_block() { return 36 * NEN + 36; }

// Phase B of the ANCF element rows for a symmetric tangent (undamped
// materials): only the slots i <= k are contracted, a lane per task (element,
// slot, coefficient a), coefficients fastest.  A task writes its NEN entries
// K_e[(a, i), (b, k)] as in the full form and, for i < k, the same values as
// the entries K_e[(b, k), (a, i)] of the blocks of the column coefficients'
// nodes (the lanes of consecutive a write consecutive values), plus the force
// parts of rows i and, for i < k, k.  Two thirds of the full form's tasks.
template <class Rule, int EB>
__device__ __forceinline__ void rows_mc_sym_contract(const AsmArgs& a, const int32_t* __restrict__ incpos,
                                                     float* __restrict__ rows, int64_t e0, int ne, const float* rec,
                                                     const float* dn) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN;
  constexpr int BLK = rows_mc_block<NEN>();
  const int tid = threadIdx.x;
  const int ntask = ne * NEN * 6;
  for (int t0 = 0; t0 < EB * NEN * 6; t0 += kRowsMcThreads) {
    const int t = t0 + tid;
    const bool on = t < ntask;
    const int tt = on ? t : ntask - 1;
    const int le = tt / (NEN * 6), r6 = tt - le * NEN * 6, us = r6 / NEN, al = r6 - us * NEN;
    const int i = us < 3 ? 0 : us < 5 ? 1 : 2, k = us < 3 ? us : us < 5 ? us - 2 : 2;
    const int so = kSlot * us, pt = 6 * kSlot + i + k - 1;  // the slot, Phat_ki (i < k)
    float acc[NEN];
#pragma unroll
    for (int b = 0; b < NEN; ++b) acc[b] = 0.0f;
    float facc = 0.0f, ft = 0.0f;
    const float* recp = rec + le * NQ * kRecS;
    static_assert(NQ % kRowsMcUnroll == 0, "point steps tile the rule");
#pragma unroll 1
    for (int q0 = 0; q0 < NQ; q0 += kRowsMcUnroll) {
      sfor<0, kRowsMcUnroll>([&](auto uc) __attribute__((always_inline)) {
        const int qq = q0 + decltype(uc)::value;
        const float* r = recp + qq * kRecS;
        float v[10];
#pragma unroll
        for (int x = 0; x < 5; ++x) {
          const f32x2 w = *reinterpret_cast<const f32x2*>(r + so + 2 * x);
          v[2 * x] = w[0];
          v[2 * x + 1] = w[1];
        }
        const float* d = dn + 3 * (NEN * qq + al);
        const float d0 = d[0], d1 = d[1], d2 = d[2];
        const float t0n = v[0] * d0 + v[3] * d1 + v[6] * d2;
        const float t1n = v[1] * d0 + v[4] * d1 + v[7] * d2;
        const float t2n = v[2] * d0 + v[5] * d1 + v[8] * d2;
        facc += v[9] * (k == 0 ? d0 : k == 1 ? d1 : d2);
        if (i < k) ft += r[pt] * (i == 0 ? d0 : d1);
#pragma unroll
        for (int b = 0; b < NEN; ++b)
          acc[b] += t0n * Rule::dNf_rt(qq, b, 0) + t1n * Rule::dNf_rt(qq, b, 1) + t2n * Rule::dNf_rt(qq, b, 2);
      });
    }
    if (on) {
      double sc[4];
      element_scales<Rule>(a, e0 + le, sc);
      const float s_a = (float)sc[al & 3];
      const int32_t* ip = incpos + (e0 + le) * NPN;
      const int c = al & 3, r = 3 * c + i;  // block row (kind, i)
      float* blk = rows + (int64_t)ip[al >> 2] * BLK;
      f32x4* outv = reinterpret_cast<f32x4*>(blk + (3 * r + k) * NEN);
#pragma unroll
      for (int u = 0; u < NEN / 4; ++u) {
        f32x4 w;
#pragma unroll
        for (int x = 0; x < 4; ++x) w[x] = acc[4 * u + x] * s_a * (float)sc[x];  // b = 4 u + x: kind x
        outv[u] = w;
      }
      blk[36 * NEN + 3 * r + k] = facc * s_a;
      if (i < k) {
        blk[36 * NEN + 3 * (3 * c + k) + i] = ft * s_a;
#pragma unroll
        for (int nb = 0; nb < NPN; ++nb) {
          float* ob = rows + (int64_t)ip[nb] * BLK;
#pragma unroll
          for (int x = 0; x < 4; ++x) ob[(3 * (3 * x + k) + i) * NEN + al] = acc[4 * nb + x] * s_a * (float)sc[x];
        }
      }
    }
  }
}

// Phase B of the shell's element rows on the matrix cores.  With
// D[(q,m), a] = dN_a,m(q) (the parent gradients, the same for every element)
// and T[(q,m), b] = sum_n Ahat_q,imkn dN_b,n(q), the slot (i, k) of K_e is the
// 16 x 16 product K^(ik) = D^T T over the 3 NQ values of (q, m): one MFMA tile,
// no padding in a or b (sixteen coefficients), the (q, m) axis padded to a
// multiple of four.  A wave takes one element at a time and runs the 16x16x4
// FP32 MFMA over the (q, m) axis in steps of four, for all the element's slots
// at once (independent accumulators, so the matrix-core chain of one slot
// overlaps the others); in each step lane l feeds D[(q,m), l % 16] and forms
// T[(q,m), l % 16] of every slot (three multiply-adds each from the LDS
// record), (q, m) = 4 step + l / 16.  Lane l then holds K^(ik)[4 (l / 16) +
// r][l % 16], r < 4, and stores them with the scales into the block of node
// l / 16 (rows of kind r); for a symmetric tangent (SYM: the six slots i <= k)
// a lane of a slot with i < k also stores its four values, consecutive in a,
// as K_e[(b, k), (a, i)] into the block of the column's node.  The force parts
// are spread over the four lane groups (a quarter of the points each) and
// summed in a fixed order.
template <bool SYM, int S>
struct McSlot {
  static constexpr int i = SYM ? (S < 3 ? 0 : S < 5 ? 1 : 2) : S / 3;
  static constexpr int k = SYM ? (S < 3 ? S : S < 5 ? S - 2 : 2) : S % 3;
  static constexpr int off = SYM ? kSlot * S : kSlot * (3 * i + k);
};

template <class Rule, int EB, bool SYM>
__device__ __forceinline__ void rows_mc_mfma_contract(const AsmArgs& a, const int32_t* __restrict__ incpos,
                                                      float* __restrict__ rows, int64_t e0, int ne, const float* rec,
                                                      const float* dn) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN, BLK = rows_mc_block<NEN>();
  static_assert(NEN == 16, "one 16 x 16 tile per slot");
  constexpr int RS = SYM ? kRecS : kRecL;
  constexpr int KK = 3 * NQ, NSTEP = (KK + 3) / 4, NSL = SYM ? 6 : 9, NW = kRowsMcThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  for (int le = wave; le < ne; le += NW) {  // uniform per wave
    const float* re = rec + le * NQ * RS;
    f32x4 acc[NSL];
#pragma unroll
    for (int t = 0; t < NSL; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 2
    for (int st = 0; st < NSTEP; ++st) {
      const int kk = 4 * st + g;
      const bool live = kk < KK;
      const int q = live ? kk / 3 : 0, m = kk - 3 * q;
      const float* d = dn + 3 * (NEN * q + c16);  // dN_c16(q)
      const float d0 = d[0], d1 = d[1], d2 = d[2];
      const float av = live ? (m == 0 ? d0 : m == 1 ? d1 : d2) : 0.0f;
      const float* r = re + q * RS + 3 * (live ? m : 0);
      sfor<0, NSL>([&](auto sc_) __attribute__((always_inline)) {
        constexpr int S = decltype(sc_)::value;
        constexpr int off = McSlot<SYM, S>::off;
        const float bv = r[off] * d0 + r[off + 1] * d1 + r[off + 2] * d2;
        acc[S] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[S], 0, 0, 0);
      });
    }
    // force parts of node c16: Phat_ik dN_c16,k (and Phat_ki dN_c16,i for i < k), a quarter of the points per group
    float fd[NSL], ft[3];
#pragma unroll
    for (int t = 0; t < NSL; ++t) fd[t] = 0.0f;
#pragma unroll
    for (int t = 0; t < 3; ++t) ft[t] = 0.0f;
    for (int q = g; q < NQ; q += 4) {
      const float* d = dn + 3 * (NEN * q + c16);
      const float* r = re + q * RS;
      sfor<0, NSL>([&](auto sc_) __attribute__((always_inline)) {
        constexpr int S = decltype(sc_)::value, i = McSlot<SYM, S>::i, k = McSlot<SYM, S>::k;
        fd[S] += r[McSlot<SYM, S>::off + 9] * d[k];
        if constexpr (SYM && i < k) ft[i + k - 1] += r[6 * kSlot + i + k - 1] * d[i];
      });
    }
#pragma unroll
    for (int t = 0; t < NSL; ++t)
      fd[t] = ((fd[t] + __shfl_down(fd[t], 16, 64)) + __shfl_down(fd[t], 32, 64)) + __shfl_down(fd[t], 48, 64);
#pragma unroll
    for (int t = 0; t < 3; ++t)
      ft[t] = ((ft[t] + __shfl_down(ft[t], 16, 64)) + __shfl_down(ft[t], 32, 64)) + __shfl_down(ft[t], 48, 64);
    double sc[4];
    element_scales<Rule>(a, e0 + le, sc);
    const int32_t* ip = incpos + (e0 + le) * NPN;
    const float sb = (float)sc[c16 & 3], sa = sb;  // column scale of b = c16; row scale of a = c16 (forces)
    float* blk = rows + (int64_t)ip[g] * BLK;      // node of the rows a = 4 g + r
    float* cb = rows + (int64_t)ip[c16 >> 2] * BLK;  // node of coefficient c16
    sfor<0, NSL>([&](auto sc_) __attribute__((always_inline)) {
      constexpr int S = decltype(sc_)::value, i = McSlot<SYM, S>::i, k = McSlot<SYM, S>::k;
#pragma unroll
      for (int r = 0; r < 4; ++r) blk[(3 * (3 * r + i) + k) * NEN + c16] = acc[S][r] * (float)sc[r] * sb;
      if (g == 0) {
        cb[36 * NEN + 3 * (3 * (c16 & 3) + i) + k] = fd[S] * sa;
        if constexpr (SYM && i < k) cb[36 * NEN + 3 * (3 * (c16 & 3) + k) + i] = ft[i + k - 1] * sa;
      }
      if constexpr (SYM && i < k) {
        f32x4 w;
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = acc[S][r] * (float)sc[r] * sb;
        *reinterpret_cast<f32x4*>(cb + (3 * (3 * (c16 & 3) + k) + i) * NEN + 4 * g) = w;
      }
    });
  }
}

template <class Rule, bool SYM, bool MF>
__device__ __forceinline__ void elem_rows_mc_tile(const AsmArgs& a, const int32_t* __restrict__ incpos,
                                                  float* __restrict__ rows, int64_t blk) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN, EB = rows_mc_elems<Rule>();
  constexpr int BLK = rows_mc_block<NEN>();
  constexpr int RS = SYM ? kRecS : kRecL;  // LDS record stride (symmetric layout for undamped materials)
  static_assert(Rule::MC == 4 && NEN % 4 == 0 && EB >= 1, "element rows of four-coefficient nodes");
  constexpr size_t NOD = (size_t)EB * NEN * 6 * sizeof(double), REC = (size_t)EB * NQ * RS * sizeof(float);
  __shared__ __align__(16) unsigned char smem[NOD > REC ? NOD : REC];
  __shared__ float dn[NQ * NEN * 3];  // unit-scaled parent gradients, dN_a(q)_m at 3 (NEN q + a) + m
  const int tid = threadIdx.x;
  const int64_t e0 = blk * EB;
  const int ne = (int)(a.n_elem - e0 < EB ? a.n_elem - e0 : EB);
  double* nod = reinterpret_cast<double*>(smem);
  gather_nodal<Rule>(a, e0, ne, nod);
  for (int idx = tid; idx < NQ * NEN * 3; idx += kRowsMcThreads) {
    const int q = idx / (3 * NEN), r = idx - 3 * NEN * q;
    dn[idx] = Rule::dNf_rt(q, r / 3, r % 3);
  }
  __syncthreads();
  // 1. a lane per point: kinematics, constitutive update, the point's record
  //    (the tangent-record layout of the point-record path) into LDS
  const bool act = tid < ne * NQ;
  const int pl = act ? tid : 0;  // idle lanes evaluate point 0 and store nothing
  const int el = pl / NQ, q = pl - el * NQ;
  double Jinv[9], det, Hd[9], Fd[9];
  tile_kinematics<Rule>(a, nod + 6 * NEN * el, e0 + el, q, Jinv, det, Hd, Fd);
  __syncthreads();  // the nodal values are consumed: the LDS holds the records from here on
  PointOut<float> o;
  const unsigned fl = point_update<float, true>(a.mp, Hd, Fd, det * Rule::w_rt(q), a.alpha, a.beta, o);
  if (act && fl) atomicOr(a.flags, fl);
  HatOut<float> h;
  to_parent<float, true>(o, Jinv, h);
  float* rec = reinterpret_cast<float*>(smem);
  if (act) {
    float* r = rec + pl * RS;
    sfor<0, RS / 4>([&](auto jc) __attribute__((always_inline)) {
      constexpr int j = decltype(jc)::value;
      f32x4 v;
      sfor<0, 4>([&](auto xc) __attribute__((always_inline)) {
        constexpr int x = decltype(xc)::value;
        if constexpr (SYM) v[x] = record_value_sym<4 * j + x>(h);
        else v[x] = record_value<4 * j + x>(h);
      });
      *reinterpret_cast<f32x4*>(r + 4 * j) = v;
    });
  }
  __syncthreads();
  if constexpr (MF) {
    rows_mc_mfma_contract<Rule, EB, SYM>(a, incpos, rows, e0, ne, rec, dn);
    return;
  }
  if constexpr (SYM) {
    rows_mc_sym_contract<Rule, EB>(a, incpos, rows, e0, ne, rec, dn);
    return;
  }
  // 2. a lane per task (element, coefficient a, row i, component k), tasks in
  //    block order; the point loop is uniform across the workgroup, so the
  //    gradients dN_b(q) of the columns come through the scalar cache
  const int ntask = ne * NEN * 9;
  for (int t0 = 0; t0 < EB * NEN * 9; t0 += kRowsMcThreads) {
    const int t = t0 + tid;
    const bool on = t < ntask;
    const int tt = on ? t : ntask - 1;
    const int le = tt / (NEN * 9), r9 = tt - le * NEN * 9, al = r9 / 9, s = r9 - 9 * al;  // s = 3 i + k
    const int k = s % 3;
    float acc[NEN];
#pragma unroll
    for (int b = 0; b < NEN; ++b) acc[b] = 0.0f;
    float facc = 0.0f;
    const float* recp = rec + le * NQ * RS;
    const SlotRef sr = slot_ref<SYM>(s / 3, k);
    static_assert(NQ % kRowsMcUnroll == 0, "point steps tile the rule");
#pragma unroll 1
    for (int q0 = 0; q0 < NQ; q0 += kRowsMcUnroll) {
      sfor<0, kRowsMcUnroll>([&](auto uc) __attribute__((always_inline)) {
        const int qq = q0 + decltype(uc)::value;
        float v[10];
        read_slot<SYM>(recp + qq * RS, sr, v);
        const float* d = dn + 3 * (NEN * qq + al);
        const float d0 = d[0], d1 = d[1], d2 = d[2];
        const float t0n = v[0] * d0 + v[3] * d1 + v[6] * d2;
        const float t1n = v[1] * d0 + v[4] * d1 + v[7] * d2;
        const float t2n = v[2] * d0 + v[5] * d1 + v[8] * d2;
        facc += v[9] * (k == 0 ? d0 : k == 1 ? d1 : d2);
#pragma unroll
        for (int b = 0; b < NEN; ++b)
          acc[b] += t0n * Rule::dNf_rt(qq, b, 0) + t1n * Rule::dNf_rt(qq, b, 1) + t2n * Rule::dNf_rt(qq, b, 2);
      });
    }
    if (on) {
      double sc[4];
      element_scales<Rule>(a, e0 + le, sc);
      const float s_a = (float)sc[al & 3];
      const int64_t pos = incpos[(e0 + le) * NPN + (al >> 2)];
      const int r = 3 * (al & 3) + s / 3;  // block row (kind, i)
      float* blk = rows + pos * BLK;
      f32x4* outv = reinterpret_cast<f32x4*>(blk + (3 * r + k) * NEN);
#pragma unroll
      for (int u = 0; u < NEN / 4; ++u) {
        f32x4 w;
#pragma unroll
        for (int x = 0; x < 4; ++x) w[x] = acc[4 * u + x] * s_a * (float)sc[x];  // b = 4 u + x: kind x
        outv[u] = w;
      }
      blk[36 * NEN + 3 * r + k] = facc * s_a;
    }
  }
}

template <class Rule, bool SYM, bool MF>
__global__ __launch_bounds__(kRowsMcThreads) void k_elem_rows_mc(AsmArgs a, const int32_t* __restrict__ incpos,
                                                                 float* __restrict__ rows) {
  elem_rows_mc_tile<Rule, SYM, MF>(a, incpos, rows, blockIdx.x);
}

// many bodies: every body starts on a workgroup of its own, found by bisection;
// the full tangent layout (the bodies' materials may differ)
template <class Rule, bool MF>
__global__ __launch_bounds__(kRowsMcThreads) void k_elem_rows_mc_batch(BatchArgs b) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = b.n_bodies - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.bodies[mid].rblock_off <= blk) lo = mid; else hi = mid - 1;
  }
  const BatchBody& B = b.bodies[lo];
  const AsmArgs a = body_args(b, B, lo);
  elem_rows_mc_tile<Rule, false, MF>(a, B.incpos, (float*)b.stage + B.blk_inc_off * rows_mc_block<Rule::NEN>(),
                                     blk - B.rblock_off);
}

// Pass 2 over the ANCF row blocks: a lane per (incidence, row r, component k)
// loads its NEN entries (16-byte pieces) and its element's rank row (4 bytes,
// element order), and adds them into the range's LDS segment at
// row + 3 (4 rank_b + c_b) + k; every lane adds its force part to the row.
template <class Rule, bool WANT_F, bool WANT_K, bool ACCUM>
__device__ __forceinline__ void gather_rows_mc(const GatherArgs& g, int32_t I0, int32_t I1, unsigned char* smem,
                                               int32_t* pre, int32_t* rowo) {
  constexpr int NEN = Rule::NEN, NPN = Rule::NPN, MC = 4, RPN = 3 * MC, TPI = 9 * MC;
  constexpr int BLK = rows_mc_block<NEN>();
  const int tid = threadIdx.x;
  uint8_t* incn = smem;
  double* lds = reinterpret_cast<double*>(smem + g.inc_cap);
  const int nn = I1 - I0;
  const int64_t row0 = (int64_t)RPN * I0, row1 = (int64_t)RPN * I1;
  const int64_t seg0 = WANT_K ? g.row_off[row0] : 0, seg1 = WANT_K ? g.row_off[row1] : 0;
  const int nseg = (int)(seg1 - seg0);
  const int nrow = (int)(row1 - row0);
  double* lf = lds + nseg;
  for (int t = tid; t < nseg + nrow; t += blockDim.x) lds[t] = 0.0;
  const int32_t inc0 = g.inc_off[I0];
  for (int n = tid; n <= nn; n += blockDim.x) pre[n] = TPI * (g.inc_off[I0 + n] - inc0);
  if constexpr (WANT_K)
    for (int rr = tid; rr < nrow; rr += blockDim.x) rowo[rr] = (int32_t)(g.row_off[row0 + rr] - seg0);
  __syncthreads();
  for (int n = tid; n < nn; n += blockDim.x)
    for (int j = pre[n] / TPI; j < pre[n + 1] / TPI; ++j) incn[j] = (uint8_t)n;
  if constexpr (WANT_K) add_mass_term<MC>(g, I0, nn, lds, rowo);
  __syncthreads();
  const int ntask = pre[nn];
  const float* blk = reinterpret_cast<const float*>(g.stage);
  for (int t = tid; t < ntask; t += blockDim.x) {
    const int jl = t / TPI, sl = t - TPI * jl, r = sl / 3, k = sl - 3 * r;
    const int64_t j = inc0 + jl;
    const int rl = RPN * incn[jl] + r;
    const float* bj = blk + j * BLK;
    if constexpr (WANT_K) {
      float val[NEN];
      const f32x4* p = reinterpret_cast<const f32x4*>(bj + (3 * r + k) * NEN);
#pragma unroll
      for (int u = 0; u < NEN / 4; ++u) {
        const f32x4 w = p[u];
#pragma unroll
        for (int x = 0; x < 4; ++x) val[4 * u + x] = w[x];
      }
      const int32_t v = g.inc[j];
      const int64_t ea = (int64_t)(v >> 4) * NPN + (v & 15);
      const uint32_t rw = *reinterpret_cast<const uint32_t*>(g.rank + ea * rank_stride(NPN));
      double* dstp = lds + rowo[rl] + k;
#pragma unroll
      for (int b = 0; b < NEN; ++b) {
        const int rank_b = (int)((rw >> (8 * (b >> 2))) & 255u);
        atomicAdd(dstp + 3 * (MC * rank_b + (b & 3)), (double)val[b]);
      }
    }
    if constexpr (WANT_F) atomicAdd(lf + rl, (double)bj[36 * NEN + 3 * r + k]);
  }
  __syncthreads();
  if constexpr (WANT_K) write_segment<ACCUM>(g, row0, nrow, nseg, seg0, lds, rowo);
  if constexpr (WANT_F) {
    double* out = g.f + row0;
    for (int t = tid; t < nrow; t += blockDim.x) out[t] = ACCUM ? out[t] + lf[t] : lf[t];
  }
}

template <class Rule, bool WANT_F, bool WANT_K, bool ACCUM>
__global__ __launch_bounds__(512) void k_gather_rows_mc(GatherArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 12];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  gather_rows_mc<Rule, WANT_F, WANT_K, ACCUM>(g, g.ranges[r], g.ranges[r + 1], smem, pre, rowo);
}

template <class Rule>
__global__ __launch_bounds__(512) void k_gather_rows_mc_batch(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t pre[kMaxRangeNodes + 1];
  __shared__ int32_t rowo[kMaxRangeNodes * 12];
  const int r = remap_tile(blockIdx.x, gridDim.x);
  const BatchRange br = b.ranges[r];
  const BatchBody& B = b.bodies[br.body];
  GatherArgs g{};
  g.inc_off = B.inc_off;
  g.inc = B.inc;
  g.row_off = B.row_off;
  g.rank = B.rank;
  g.stage = (const float*)b.stage + B.blk_inc_off * rows_mc_block<Rule::NEN>();
  g.f = b.f + B.dof_off;
  g.vals = b.vals + B.nnz_off;
  g.inc_cap = b.inc_cap;
  gather_rows_mc<Rule, true, true, false>(g, br.I0, br.I1, smem, pre, rowo);
}

// ---------------------------------------------------------------------------
// internal force alone (every element type)
// ---------------------------------------------------------------------------
// Pass 1 keeps each element's points in one workgroup: a lane per point forms
// Phat = dV P J0^-T (Sec. 4.3, Stage 1) into LDS, then a lane per (element,
// coefficient a) sums f_a = sum_q Phat_q dN_a(q) s_a over the element's points
// (Eq. fint_local, in the record precision) and writes the three values to the
// node-sorted incidence position of (element, node of a), 3 MC values per
// incidence.  Pass 2 adds each pattern node's incidence blocks in a fixed order,
// a lane per row of f, in float64: no atomics, the same sums on every call.
constexpr int kForceThreads = 256;
template <class Rule>
constexpr int force_elems() { return kForceThreads / Rule::NQ; }

template <class Rule, typename R>
__global__ __launch_bounds__(kForceThreads) void k_elem_force(AsmArgs a, const int32_t* __restrict__ incpos,
                                                             R* __restrict__ blocks) {
  constexpr int NQ = Rule::NQ, NEN = Rule::NEN, NPN = Rule::NPN, MC = Rule::MC, EB = force_elems<Rule>();
  constexpr size_t NOD = (size_t)EB * NEN * 6 * sizeof(double), PH = (size_t)EB * NQ * 9 * sizeof(R);
  __shared__ __align__(16) unsigned char smem[NOD > PH ? NOD : PH];
  __shared__ R dn[NQ * NEN * 3];  // unit-scaled parent gradients, dN_a(q)_m at 3 (NEN q + a) + m
  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * EB;
  const int ne = (int)(a.n_elem - e0 < EB ? a.n_elem - e0 : EB);
  double* nod = reinterpret_cast<double*>(smem);
  gather_nodal<Rule>(a, e0, ne, nod);
  for (int idx = tid; idx < NQ * NEN * 3; idx += kForceThreads) {
    const int q = idx / (3 * NEN), r = idx - 3 * NEN * q;
    dn[idx] = (R)Rule::dN_rt(q, r / 3, r % 3);
  }
  __syncthreads();
  const bool act = tid < ne * NQ;
  const int pl = act ? tid : 0;  // idle lanes evaluate point 0 and store nothing
  const int el = pl / NQ, q = pl - el * NQ;
  double Jinv[9], det, Hd[9], Fd[9];
  tile_kinematics<Rule, true>(a, nod + 6 * NEN * el, e0 + el, q, Jinv, det, Hd, Fd);
  __syncthreads();  // the nodal values are consumed: the LDS holds Phat from here on
  PointOut<R> o;
  const MatParams mp = launch_material(a);
  const unsigned fl = point_update<R, false>(mp, Hd, Fd, det * Rule::w_rt(q), a.alpha, a.beta, o);
  if (act && fl) atomicOr(a.flags, fl);
  HatOut<R> h;
  to_parent<R, false>(o, Jinv, h);
  R* ph = reinterpret_cast<R*>(smem);
  if (act) {
#pragma unroll
    for (int t = 0; t < 9; ++t) ph[9 * pl + t] = h.P[t];
  }
  __syncthreads();
  for (int t = tid; t < ne * NEN; t += kForceThreads) {
    const int le = t / NEN, al = t - le * NEN;
    R f0 = R(0), f1 = R(0), f2 = R(0);
    for (int qq = 0; qq < NQ; ++qq) {
      const R* p = ph + 9 * (le * NQ + qq);
      const R* d = dn + 3 * (NEN * qq + al);
      const R d0 = d[0], d1 = d[1], d2 = d[2];
      f0 += p[0] * d0 + p[1] * d1 + p[2] * d2;
      f1 += p[3] * d0 + p[4] * d1 + p[5] * d2;
      f2 += p[6] * d0 + p[7] * d1 + p[8] * d2;
    }
    double sc[4];
    element_scales<Rule>(a, e0 + le, sc);
    const R s = (R)sc[al % 4];
    const int64_t pos = incpos[(e0 + le) * NPN + al / MC];
    R* out = blocks + pos * (3 * MC) + 3 * (al % MC);
    out[0] = f0 * s;
    out[1] = f1 * s;
    out[2] = f2 * s;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_force_sum(const int32_t* __restrict__ inc_off, const R* __restrict__ blocks,
                                                   int64_t n_rows, int rpn, bool accum, double* __restrict__ f) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  const int64_t I = r / rpn;
  const int j = (int)(r - I * rpn);
  // four loads in flight, summed in incidence order
  double s = 0.0;
  int32_t x = inc_off[I];
  const int32_t x1 = inc_off[I + 1];
  for (; x + 4 <= x1; x += 4) {
    const R* b = blocks + (int64_t)x * rpn + j;
    const double v0 = (double)b[0], v1 = (double)b[rpn], v2 = (double)b[2 * rpn], v3 = (double)b[3 * rpn];
    s += v0;
    s += v1;
    s += v2;
    s += v3;
  }
  for (; x < x1; ++x) s += (double)blocks[(int64_t)x * rpn + j];
  f[r] = accum ? f[r] + s : s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int grid_of(int64_t n, int b) { return (int)((n + b - 1) / b); }

template <class Rule, typename R>
int launch_force_rule(const Mesh& m, const AsmArgs& a, void* blk, hipStream_t s) {
  constexpr int EB = force_elems<Rule>();
  const int64_t blocks = (m.n_elem + EB - 1) / EB;
  if (blocks > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  if (blocks > 0)
    hipLaunchKernelGGL((k_elem_force<Rule, R>), dim3((unsigned)blocks), dim3(kForceThreads), 0, s, a, m.d_incpos,
                       (R*)blk);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

template <typename R>
int launch_force_prec(const Mesh& m, const AsmArgs& a, void* blk, hipStream_t s) {
  if (m.elem_type == TLFEA_T10) return launch_force_rule<RuleT10, R>(m, a, blk, s);
  if (m.elem_type == TLFEA_ANCF3243) return launch_force_rule<RuleBeam, R>(m, a, blk, s);
  if (m.gl[0] == 3) return launch_force_rule<RuleAncf<3, 3, 2>, R>(m, a, blk, s);
  return launch_force_rule<RuleAncf<4, 4, 3>, R>(m, a, blk, s);
}

int launch_force_sum(const Mesh& m, const void* blk, double* f, bool accum, hipStream_t s) {
  const int rpn = 3 * m.mc;
  if (m.n_dof > 0) {
    if (m.precision == TLFEA_MIXED)
      hipLaunchKernelGGL(k_force_sum<float>, dim3(grid_of(m.n_dof, 256)), dim3(256), 0, s, m.d_inc_off,
                         (const float*)blk, m.n_dof, rpn, accum, f);
    else
      hipLaunchKernelGGL(k_force_sum<double>, dim3(grid_of(m.n_dof, 256)), dim3(256), 0, s, m.d_inc_off,
                         (const double*)blk, m.n_dof, rpn, accum, f);
  }
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

// Dynamic LDS beyond 64 KiB has to be allowed per kernel; the largest size
// granted so far is remembered per kernel (by address: kernels of one
// signature share a template instantiation here) and device.
template <typename Kernel>
int allow_lds(Kernel* kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return TLFEA_OK;
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> granted;
  int dev = 0, max_bytes = 0;
  TLFEA_HIP_CHECK(hipGetDevice(&dev));
  const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = granted.find(key);
  if (it != granted.end() && bytes <= it->second) return TLFEA_OK;
  TLFEA_HIP_CHECK(hipDeviceGetAttribute(&max_bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (bytes > (size_t)max_bytes) return TLFEA_ERR_UNSUPPORTED;
  TLFEA_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  granted[key] = bytes;
  return TLFEA_OK;
}

template <class Rule, typename R>
int launch_points_rule(const Mesh& m, const AsmArgs& a, bool want_k, hipStream_t s) {
  const int64_t npts = m.n_elem * Rule::NQ;
  if (npts > (int64_t)INT32_MAX * 256) return TLFEA_ERR_TOO_LARGE;
  if (npts == 0) return TLFEA_OK;
  R* stage = (R*)m.d_stage;
  if (want_k && point_records_sym(m, true))
    hipLaunchKernelGGL((k_stage_tile<Rule, R, sizeof(R) == 8>), dim3(grid_of(npts, kStageThreads)),
                       dim3(kStageThreads), 0, s, a, stage);
  else if (want_k)
    hipLaunchKernelGGL((k_stage_tile<Rule, R, false>), dim3(grid_of(npts, kStageThreads)), dim3(kStageThreads), 0,
                       s, a, stage);
  else
    hipLaunchKernelGGL((k_stage<Rule, R, false>), dim3(grid_of(npts, 256)), dim3(256), 0, s, a, stage);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

// LDS for a range's upper row offsets (upper-triangle output), 8-byte multiple
size_t upper_table_bytes(const Mesh& m) { return 8 * (size_t)((m.max_range_rows + 2) / 2); }

// pass 2 addresses records in 16-byte units with 32-bit offsets
template <class Rule, typename R>
bool records_addressable(int64_t n_elem, bool want_k) {
  const int64_t pieces = (int64_t)Rule::NQ * (want_k ? kRecK : kRecF) * (int64_t)sizeof(R) / 16;
  return n_elem * pieces < ((int64_t)1 << 32);
}

template <class Rule, typename R>
int launch_nodes_rule(const Mesh& m, const void* stage, double* f, double* vals, bool accum, hipStream_t s,
                      const GatherOptions& mt, bool tangent_records) {
  const bool want_f = f != nullptr, want_k = vals != nullptr;
  if (want_k && !tangent_records) return TLFEA_ERR_INVALID;
  const bool krec = tangent_records;
  const bool sym = krec && m.staged_sym;  // symmetric float64 records from pass 1
  if (!records_addressable<Rule, R>(m.n_elem, want_k)) return TLFEA_ERR_TOO_LARGE;
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
  g.mass = mt.mass;
  g.adj_off = m.d_adj_off;
  g.inv_h = mt.inv_h;
  g.row_off_u = mt.row_off_u;
  g.inc_cap = (int)((m.max_range_inc + 15) / 16 * 16);
  const size_t lds = sizeof(double) * (want_k ? m.max_range_values : m.max_range_rows) + g.inc_cap +
                     (size_t)m.tune.waves * (krec ? (sym ? wave_buf_bytes<Rule, R, true, sizeof(R) == 8>()
                                                         : wave_buf_bytes<Rule, R, true>())
                                                  : wave_buf_bytes<Rule, R, false>()) +
                     (mt.row_off_u ? upper_table_bytes(m) : 0);
  const dim3 grid((unsigned)m.n_ranges), blk(64 * m.tune.waves);
#define TLFEA_GATHER_S(F, K, A, KR, SY)                                              \
  do {                                                                               \
    if (int rc = allow_lds(k_gather<Rule, R, F, K, A, KR, SY>, lds)) return rc;      \
    hipLaunchKernelGGL((k_gather<Rule, R, F, K, A, KR, SY>), grid, blk, lds, s, g); \
  } while (0)
#define TLFEA_GATHER(F, K, A, KR)                                                            \
  do {                                                                                       \
    if (KR && sym) TLFEA_GATHER_S(F, K, A, KR, (KR && sizeof(R) == 8)); else TLFEA_GATHER_S(F, K, A, KR, false); \
  } while (0)
  if (want_k && want_f) {
    if (accum) TLFEA_GATHER(true, true, true, true); else TLFEA_GATHER(true, true, false, true);
  } else if (want_k) {
    if (accum) TLFEA_GATHER(false, true, true, true); else TLFEA_GATHER(false, true, false, true);
  } else if (krec) {  // the force alone from tangent records
    if (accum) TLFEA_GATHER(true, false, true, true); else TLFEA_GATHER(true, false, false, true);
  } else {
    if (accum) TLFEA_GATHER(true, false, true, false); else TLFEA_GATHER(true, false, false, false);
  }
#undef TLFEA_GATHER
#undef TLFEA_GATHER_S
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

// pass 2 over the element row blocks (addressed in 16-byte units with 32-bit offsets)
int launch_rows_nodes(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s, const GatherOptions& mt) {
  const bool want_f = f != nullptr, want_k = vals != nullptr;
  if (m.n_elem * m.n_pn * (int64_t)(kRowBlk / 4) >= ((int64_t)1 << 32)) return TLFEA_ERR_TOO_LARGE;
  GatherArgs g{};
  g.ranges = m.d_ranges;
  g.inc_off = m.d_inc_off;
  g.row_off = m.d_row_off;
  g.rank = m.d_rank_inc;
  g.stage = m.d_stage;
  g.f = f;
  g.vals = vals;
  g.mass = mt.mass;
  g.adj_off = m.d_adj_off;
  g.inv_h = mt.inv_h;
  g.row_off_u = mt.row_off_u;
  g.inc_cap = (int)((m.max_range_inc + 15) / 16 * 16);
  const size_t lds = sizeof(double) * (want_k ? m.max_range_values : m.max_range_rows) + g.inc_cap +
                     (mt.row_off_u ? upper_table_bytes(m) : 0);
  const dim3 grid((unsigned)m.n_ranges), blk(64 * m.tune.waves);
#define TLFEA_GATHER(F, K, A)                                              \
  do {                                                                     \
    if (int rc = allow_lds(k_gather_rows<F, K, A>, lds)) return rc;        \
    hipLaunchKernelGGL((k_gather_rows<F, K, A>), grid, blk, lds, s, g);   \
  } while (0)
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

// Undamped materials take the symmetric record layout in the element-row
// pass 1 (TLFEA_SYM_RECORDS=0 keeps the full layout, for comparisons).
bool sym_records(const Mesh& m) {
  static const bool on = [] {
    const char* v = std::getenv("TLFEA_SYM_RECORDS");
    return !(v && v[0] == '0');
  }();
  return on && m.mp.eta == 0.0 && m.mp.lam_v == 0.0;
}

// The shell's element-row contraction on the matrix cores (TLFEA_MC_MFMA=0
// keeps the vector form, for comparisons).
bool mc_mfma() {
  static const bool on = [] {
    const char* v = std::getenv("TLFEA_MC_MFMA");
    return !(v && v[0] == '0');
  }();
  return on;
}

template <class Rule>
int launch_rows_mc_points(const Mesh& m, const AsmArgs& a, hipStream_t s) {
  constexpr int EB = rows_mc_elems<Rule>();
  const int64_t blocks = (m.n_elem + EB - 1) / EB;
  if (blocks > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  // the shell's 16 x 16 slot tiles on the matrix cores (the beam's 8 x 8 slots
  // would fill half a tile: slower than its vector form, measured)
  constexpr bool MF = Rule::NEN == 16;
  if (blocks > 0) {
    if (sym_records(m) && mc_mfma())
      hipLaunchKernelGGL((k_elem_rows_mc<Rule, true, MF>), dim3((unsigned)blocks), dim3(kRowsMcThreads), 0, s,
                         a, m.d_incpos, (float*)m.d_stage);
    else if (sym_records(m))
      hipLaunchKernelGGL((k_elem_rows_mc<Rule, true, false>), dim3((unsigned)blocks), dim3(kRowsMcThreads), 0, s,
                         a, m.d_incpos, (float*)m.d_stage);
    else if (mc_mfma())
      hipLaunchKernelGGL((k_elem_rows_mc<Rule, false, MF>), dim3((unsigned)blocks), dim3(kRowsMcThreads), 0, s,
                         a, m.d_incpos, (float*)m.d_stage);
    else
      hipLaunchKernelGGL((k_elem_rows_mc<Rule, false, false>), dim3((unsigned)blocks), dim3(kRowsMcThreads), 0, s,
                         a, m.d_incpos, (float*)m.d_stage);
  }
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

template <class Rule>
int launch_rows_mc_nodes(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s, const GatherOptions& mt) {
  const bool want_f = f != nullptr, want_k = vals != nullptr;
  GatherArgs g{};
  g.ranges = m.d_ranges;
  g.inc_off = m.d_inc_off;
  g.inc = m.d_inc;
  g.row_off = m.d_row_off;
  g.rank = m.d_rank;
  g.stage = m.d_stage;
  g.f = f;
  g.vals = vals;
  g.mass = mt.mass;
  g.adj_off = m.d_adj_off;
  g.inv_h = mt.inv_h;
  g.row_off_u = mt.row_off_u;
  g.inc_cap = (int)((m.max_range_inc + 15) / 16 * 16);
  const size_t lds = sizeof(double) * (want_k ? m.max_range_values : m.max_range_rows) + g.inc_cap +
                     (mt.row_off_u ? upper_table_bytes(m) : 0);
  const dim3 grid((unsigned)m.n_ranges), blk(64 * m.tune.waves);
#define TLFEA_GATHER(F, K, A)                                                   \
  do {                                                                          \
    if (int rc = allow_lds(k_gather_rows_mc<Rule, F, K, A>, lds)) return rc;    \
    hipLaunchKernelGGL((k_gather_rows_mc<Rule, F, K, A>), grid, blk, lds, s, g); \
  } while (0)
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
  if (m.elem_type == TLFEA_ANCF3243) return launch_points_rule<RuleBeam, R>(m, a, want_k, s);
  if (m.gl[0] == 3) return launch_points_rule<RuleAncf<3, 3, 2>, R>(m, a, want_k, s);
  return launch_points_rule<RuleAncf<4, 4, 3>, R>(m, a, want_k, s);
}

template <typename R>
int launch_nodes_prec(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s, const GatherOptions& mt) {
  const bool kr = m.staged == 2;  // tangent records (else force records)
  if (m.elem_type == TLFEA_T10) return launch_nodes_rule<RuleT10, R>(m, m.d_stage, f, vals, accum, s, mt, kr);
  if (m.elem_type == TLFEA_ANCF3243)
    return launch_nodes_rule<RuleBeam, R>(m, m.d_stage, f, vals, accum, s, mt, kr);
  if (m.gl[0] == 3) return launch_nodes_rule<RuleAncf<3, 3, 2>, R>(m, m.d_stage, f, vals, accum, s, mt, kr);
  return launch_nodes_rule<RuleAncf<4, 4, 3>, R>(m, m.d_stage, f, vals, accum, s, mt, kr);
}

template <class Rule, typename R>
int launch_batch_rule(const GatherTuning& tu, const BatchArgs& b, int n_ranges, size_t lds, hipStream_t s) {
  if (b.n_blocks > 0)
    hipLaunchKernelGGL((k_stage_batch<Rule, R>), dim3((unsigned)b.n_blocks), dim3(kStageThreads), 0, s, b);
  TLFEA_HIP_CHECK(hipGetLastError());
  const size_t lds_all = lds + b.inc_cap + (size_t)tu.waves * wave_buf_bytes<Rule, R, true>();
  if (int rc = allow_lds(k_gather_batch<Rule, R>, lds_all)) return rc;
  hipLaunchKernelGGL((k_gather_batch<Rule, R>), dim3(n_ranges), dim3(64 * tu.waves), lds_all, s, b);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

__global__ void k_zero(double* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

}  // namespace

bool use_rows(const Mesh& m, bool want_k) {
  static const bool on = [] {
    const char* v = std::getenv("TLFEA_ELEMENT_ROWS");
    return !(v && v[0] == '0');
  }();
  return on && want_k && m.precision == TLFEA_MIXED && m.d_incpos && (m.elem_type != TLFEA_T10 || m.d_rank_inc);
}

// The float64 point records of a tangent pass take the symmetric layout for
// undamped materials (64 values instead of 96).
bool point_records_sym(const Mesh& m, bool want_k) {
  return want_k && m.precision == TLFEA_FP64 && sym_records(m);
}

bool use_force_blocks(const Mesh& m, bool want_k) {
  static const bool on = [] {
    const char* v = std::getenv("TLFEA_FORCE_BLOCKS");
    return !(v && v[0] == '0');
  }();
  return on && !want_k && m.d_incpos;
}

size_t stage_bytes(const Mesh& m, bool want_k) {
  if (use_rows(m, want_k))
    return (size_t)m.n_elem * m.n_pn * (m.elem_type == TLFEA_T10 ? kRowBlk : 36 * m.n_en + 36) * sizeof(float);
  const size_t r = m.precision == TLFEA_MIXED ? sizeof(float) : sizeof(double);
  if (use_force_blocks(m, want_k)) return (size_t)m.n_elem * m.n_pn * 3 * m.mc * r;
  return (size_t)m.n_elem * m.n_qp * (want_k ? kRecK : kRecF) * r;
}

size_t row_block_bytes() { return kRowBlk * sizeof(float); }
int row_elems() { return kRowElems; }

size_t row_block_bytes_for(int elem_type, int gl0) {
  if (elem_type == TLFEA_T10) return row_block_bytes();
  if (elem_type == TLFEA_ANCF3243) return rows_mc_block<RuleBeam::NEN>() * sizeof(float);
  return rows_mc_block<16>() * sizeof(float);
}
int row_elems_for(int elem_type, int gl0) {
  if (elem_type == TLFEA_T10) return kRowElems;
  if (elem_type == TLFEA_ANCF3243) return rows_mc_elems<RuleBeam>();
  return gl0 == 3 ? rows_mc_elems<RuleAncf<3, 3, 2>>() : rows_mc_elems<RuleAncf<4, 4, 3>>();
}

size_t stage_record_bytes(int precision) {
  return (size_t)kRecK * (precision == TLFEA_MIXED ? sizeof(float) : sizeof(double));
}

// Workgroups of the persistent batch kernels one CU holds at once (tile kernel
// for EB elements per tile; range kernel for the given shape and LDS bytes).
int batch_lpt_occupancy(int tile_elems, int waves, size_t lds_all, int* tiles_per_cu, int* ranges_per_cu) {
  int nt = 0, nr = 0;
  if (tile_elems == 16)
    TLFEA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nt, reinterpret_cast<const void*>(k_elem_rows_batch_lpt<RuleT10, 16>), kRowThreads, 0));
  else
    TLFEA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nt, reinterpret_cast<const void*>(k_elem_rows_batch_lpt<RuleT10, kRowElems>), kRowThreads, 0));
  if (int rc = allow_lds(k_gather_rows_batch_lpt, lds_all)) return rc;
  TLFEA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nr, reinterpret_cast<const void*>(k_gather_rows_batch_lpt), 64 * waves, lds_all));
  *tiles_per_cu = std::max(nt, 1);
  *ranges_per_cu = std::max(nr, 1);
  return TLFEA_OK;
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
  if (use_force_blocks(m, want_k))
    return m.precision == TLFEA_MIXED ? launch_force_prec<float>(m, a, m.d_stage, s)
                                     : launch_force_prec<double>(m, a, m.d_stage, s);
  if (use_rows(m, want_k) && m.elem_type != TLFEA_T10) {
    if (m.elem_type == TLFEA_ANCF3243) return launch_rows_mc_points<RuleBeam>(m, a, s);
    if (m.gl[0] == 3) return launch_rows_mc_points<RuleAncf<3, 3, 2>>(m, a, s);
    return launch_rows_mc_points<RuleAncf<4, 4, 3>>(m, a, s);
  }
  if (use_rows(m, want_k)) {
    const int64_t blocks = (m.n_elem + kRowElems - 1) / kRowElems;
    if (blocks > INT32_MAX) return TLFEA_ERR_TOO_LARGE;
    if (blocks > 0)
      if (sym_records(m))
        hipLaunchKernelGGL((k_elem_rows<RuleT10, true>), dim3((unsigned)blocks), dim3(kRowThreads), 0, s, a,
                           m.d_incpos, (float*)m.d_stage);
      else
        hipLaunchKernelGGL((k_elem_rows<RuleT10, false>), dim3((unsigned)blocks), dim3(kRowThreads), 0, s, a,
                           m.d_incpos, (float*)m.d_stage);
    TLFEA_HIP_CHECK(hipGetLastError());
    return TLFEA_OK;
  }
  if (m.precision == TLFEA_MIXED) return launch_points_prec<float>(m, a, want_k, s);
  return launch_points_prec<double>(m, a, want_k, s);
}

int launch_nodes(const Mesh& m, double* f, double* vals, bool accum, hipStream_t s, const GatherOptions& mt) {
  if (mt.mass && !vals) return TLFEA_ERR_INVALID;
  if (m.n_ranges == 0) {  // no nodes: only the (empty) outputs to clear
    if (accum) return TLFEA_OK;
    int rc = f ? launch_zero(f, m.n_dof, s) : TLFEA_OK;
    return (rc || !vals) ? rc : launch_zero(vals, mt.row_off_u ? m.nnz_u : m.nnz, s);
  }
  if (m.staged == 3 && m.elem_type == TLFEA_ANCF3243) return launch_rows_mc_nodes<RuleBeam>(m, f, vals, accum, s, mt);
  if (m.staged == 3 && m.elem_type == TLFEA_ANCF3443)
    return m.gl[0] == 3 ? launch_rows_mc_nodes<RuleAncf<3, 3, 2>>(m, f, vals, accum, s, mt)
                        : launch_rows_mc_nodes<RuleAncf<4, 4, 3>>(m, f, vals, accum, s, mt);
  if (m.staged == 3) return launch_rows_nodes(m, f, vals, accum, s, mt);
  if (m.staged == 4) return vals ? TLFEA_ERR_INVALID : launch_force_sum(m, m.d_stage, f, accum, s);
  if (m.precision == TLFEA_MIXED) return launch_nodes_prec<float>(m, f, vals, accum, s, mt);
  return launch_nodes_prec<double>(m, f, vals, accum, s, mt);
}

// Fixed work area of the allocation-free force call: the force blocks of one
// call (3 mc values per incidence).  The kernels take its device address,
// looked up once per device with that device current; the array's name in
// host code is only a host-side stand-in for the symbol.
int noalloc_scratch(void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  int dev = 0;
  TLFEA_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    TLFEA_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return TLFEA_ERR_HIP;
    it = addr.emplace(dev, p).first;
  }
  *out = it->second;
  return TLFEA_OK;
}

size_t noalloc_force_bytes(const Mesh& m) {
  return (size_t)m.n_elem * m.n_pn * 3 * m.mc * (m.precision == TLFEA_MIXED ? sizeof(float) : sizeof(double));
}

int launch_force_noalloc(const Mesh& m, const AsmArgs& a, double* f, hipStream_t s) {
  if (!m.d_incpos) return TLFEA_ERR_NO_PATTERN;
  if (noalloc_force_bytes(m) > kNoallocScratchBytes) return TLFEA_ERR_TOO_LARGE;
  void* blk = nullptr;
  if (int rc = noalloc_scratch(&blk)) return rc;
  // every incidence block is written by pass 1 before pass 2 reads it: nothing to clear
  int rc = m.precision == TLFEA_MIXED ? launch_force_prec<float>(m, a, blk, s) : launch_force_prec<double>(m, a, blk, s);
  if (rc) return rc;
  return launch_force_sum(m, blk, f, false, s);
}

int launch_force_blocks(Mesh& m, const AsmArgs& a, double* f, hipStream_t s) {
  if (!m.d_incpos) return TLFEA_ERR_NO_PATTERN;
  const size_t rsz = m.precision == TLFEA_MIXED ? sizeof(float) : sizeof(double);
  if (int rc = ensure_stage(m, (size_t)m.n_elem * m.n_pn * 3 * m.mc * rsz)) return rc;
  int rc = m.precision == TLFEA_MIXED ? launch_force_prec<float>(m, a, m.d_stage, s)
                                      : launch_force_prec<double>(m, a, m.d_stage, s);
  m.staged = rc ? 0 : 4;
  m.staged_precision = m.precision;
  if (rc) return rc;
  return launch_force_sum(m, m.d_stage, f, false, s);
}

__global__ void k_params(int kind, const double* __restrict__ p, double* __restrict__ mp) {
  if (threadIdx.x != 0) return;
  if (kind == TLFEA_SVK) {
    const double E = p[0], nu = p[1];
    mp[0] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    mp[1] = E / (2.0 * (1.0 + nu));
    mp[2] = 0.0;
  } else {
    mp[0] = p[0];
    mp[1] = p[1];
    mp[2] = p[2];
  }
  mp[3] = p[3];
  mp[4] = p[4];
}

int launch_params(const Mesh& m, const double* d_params, hipStream_t s) {
  hipLaunchKernelGGL(k_params, dim3(1), dim3(64), 0, s, m.material, d_params, m.d_mp);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

int launch_block_sum(const Mesh& m, const double* blk, double* out, hipStream_t s) {
  if (m.n_dof > 0)
    hipLaunchKernelGGL(k_force_sum<double>, dim3(grid_of(m.n_dof, 256)), dim3(256), 0, s, m.d_inc_off, blk, m.n_dof,
                       3 * m.mc, false, out);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

template <class Rule>
int launch_rows_mc_batch(const GatherTuning& tu, const BatchArgs& b, int n_ranges, size_t lds, hipStream_t s) {
  constexpr bool MF = Rule::NEN == 16;  // the shell's slot tiles on the matrix cores
  if (b.n_rblocks > 0) {
    if (mc_mfma())
      hipLaunchKernelGGL((k_elem_rows_mc_batch<Rule, MF>), dim3((unsigned)b.n_rblocks), dim3(kRowsMcThreads), 0, s,
                         b);
    else
      hipLaunchKernelGGL((k_elem_rows_mc_batch<Rule, false>), dim3((unsigned)b.n_rblocks), dim3(kRowsMcThreads), 0,
                         s, b);
  }
  TLFEA_HIP_CHECK(hipGetLastError());
  const size_t lds_all = lds + b.inc_cap;
  if (int rc = allow_lds(k_gather_rows_mc_batch<Rule>, lds_all)) return rc;
  hipLaunchKernelGGL(k_gather_rows_mc_batch<Rule>, dim3(n_ranges), dim3(64 * tu.waves), lds_all, s, b);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

int launch_batch(int elem_type, int gl0, int precision, const GatherTuning& tu, const BatchArgs& b,
                 int n_ranges, size_t lds, hipStream_t s, const BatchSchedule& sc) {
  if (n_ranges == 0) return TLFEA_OK;
  if (b.rows && sc.persistent) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, sc.counters);
    if (sc.n_tiles > 0) {
      if (sc.tile_elems == 16)
        hipLaunchKernelGGL((k_elem_rows_batch_lpt<RuleT10, 16>), dim3(sc.grid_tiles), dim3(kRowThreads), 0, s, b,
                           sc.tiles, sc.n_tiles, sc.counters);
      else
        hipLaunchKernelGGL((k_elem_rows_batch_lpt<RuleT10, kRowElems>), dim3(sc.grid_tiles), dim3(kRowThreads), 0, s,
                           b, sc.tiles, sc.n_tiles, sc.counters);
    }
    TLFEA_HIP_CHECK(hipGetLastError());
    const size_t lds_all = lds + b.inc_cap;
    if (int rc = allow_lds(k_gather_rows_batch_lpt, lds_all)) return rc;
    hipLaunchKernelGGL(k_gather_rows_batch_lpt, dim3(sc.grid_ranges), dim3(64 * tu.waves), lds_all, s, b,
                       sc.range_order, n_ranges, sc.counters + 1);
    TLFEA_HIP_CHECK(hipGetLastError());
    return TLFEA_OK;
  }
  if (b.rows && elem_type != TLFEA_T10) {
    if (elem_type == TLFEA_ANCF3243) return launch_rows_mc_batch<RuleBeam>(tu, b, n_ranges, lds, s);
    if (gl0 == 3) return launch_rows_mc_batch<RuleAncf<3, 3, 2>>(tu, b, n_ranges, lds, s);
    return launch_rows_mc_batch<RuleAncf<4, 4, 3>>(tu, b, n_ranges, lds, s);
  }
  if (b.rows) {
    if (b.n_rblocks > 0)
      hipLaunchKernelGGL(k_elem_rows_batch<RuleT10>, dim3((unsigned)b.n_rblocks), dim3(kRowThreads), 0, s, b);
    TLFEA_HIP_CHECK(hipGetLastError());
    const size_t lds_all = lds + b.inc_cap;
    if (int rc = allow_lds(k_gather_rows_batch, lds_all)) return rc;
    hipLaunchKernelGGL(k_gather_rows_batch, dim3(n_ranges), dim3(64 * tu.waves), lds_all, s, b);
    TLFEA_HIP_CHECK(hipGetLastError());
    return TLFEA_OK;
  }
  const bool mixed = precision == TLFEA_MIXED;
  if (elem_type == TLFEA_T10)
    return mixed ? launch_batch_rule<RuleT10, float>(tu, b, n_ranges, lds, s)
                 : launch_batch_rule<RuleT10, double>(tu, b, n_ranges, lds, s);
  if (elem_type == TLFEA_ANCF3243)
    return mixed ? launch_batch_rule<RuleBeam, float>(tu, b, n_ranges, lds, s)
                 : launch_batch_rule<RuleBeam, double>(tu, b, n_ranges, lds, s);
  if (gl0 == 3)
    return mixed ? launch_batch_rule<RuleAncf<3, 3, 2>, float>(tu, b, n_ranges, lds, s)
                 : launch_batch_rule<RuleAncf<3, 3, 2>, double>(tu, b, n_ranges, lds, s);
  return mixed ? launch_batch_rule<RuleAncf<4, 4, 3>, float>(tu, b, n_ranges, lds, s)
               : launch_batch_rule<RuleAncf<4, 4, 3>, double>(tu, b, n_ranges, lds, s);
}

}  // namespace tlfea
