// pattern.hip -- fixed CSR pattern and slot map, built once on the GPU.
//
// Sec. 4.2 of the paper: the coefficient-level adjacency comes from element
// connectivity, each adjacent pair of coefficients becomes a 3x3 DOF block
// (Sec. 4.4.2), and the structure never changes afterwards, so Newton
// iterations only rewrite values.  The paper sorts 64-bit pair keys on the
// device; this builder instead goes through node -> element incidence lists:
//   1. count and fill the incidence of every pattern node (atomics + scan);
//   2. one wavefront per node gathers the nodes of its incident elements into
//      LDS and ranks the distinct ones (sorted order, deterministic);
//   3. prefix sums give the adjacency offsets and the DOF row offsets;
//   4. columns are written per node; the slot map is stored as one byte per
//      (element, node a, node b): the rank of b in the sorted adjacency of a.
// A pattern node is a T10 node or an ANCF physical node (4 coefficients).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "tlfea_internal.h"

namespace tlfea {
namespace {

constexpr int kMaxCand = 4096;  // candidate neighbours per node held in LDS

__global__ void k_count_inc(const int32_t* conn, int64_t n, int32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(cnt + conn[i], 1);
}

__global__ void k_fill_inc(const int32_t* conn, int64_t n, int npn, const int32_t* off, int32_t* cursor,
                           int32_t* inc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t node = conn[i];
    const int32_t pos = atomicAdd(cursor + node, 1);
    inc[off[node] + pos] = (int32_t)(i / npn);
  }
}

// One wavefront per pattern node.  fill == 0: write the number of distinct
// neighbours to nadj[I]; fill == 1: write them, sorted, to adj[adj_off[I]..].
__global__ __launch_bounds__(64) void k_adjacency(const int32_t* conn, int npn, const int32_t* inc_off,
                                                  const int32_t* inc, int64_t n_nodes, int fill,
                                                  int32_t* nadj, const int32_t* adj_off, int32_t* adj,
                                                  uint32_t* err) {
  __shared__ int32_t cand[kMaxCand];
  __shared__ uint8_t first[kMaxCand];
  __shared__ int32_t count;
  const int64_t I = blockIdx.x;
  if (I >= n_nodes) return;
  const int lane = threadIdx.x;
  const int32_t b0 = inc_off[I], nin = inc_off[I + 1] - b0;
  const int nc = nin * npn;
  if (nc > kMaxCand) {
    if (lane == 0) {
      atomicOr(err, 1u);
      if (!fill) nadj[I] = 0;
    }
    return;
  }
  if (lane == 0) count = 0;
  for (int j = lane; j < nc; j += 64) cand[j] = conn[(int64_t)inc[b0 + j / npn] * npn + j % npn];
  __syncthreads();
  int mine = 0;
  for (int j = lane; j < nc; j += 64) {
    const int32_t v = cand[j];
    bool f = true;
    for (int k = 0; k < j; ++k)
      if (cand[k] == v) { f = false; break; }
    first[j] = f ? 1 : 0;
    mine += f ? 1 : 0;
  }
  __syncthreads();
  if (!fill) {
    if (mine) atomicAdd(&count, mine);
    __syncthreads();
    if (lane == 0) nadj[I] = count;
    return;
  }
  for (int j = lane; j < nc; j += 64) {
    if (!first[j]) continue;
    const int32_t v = cand[j];
    int r = 0;
    for (int k = 0; k < nc; ++k) r += (first[k] && cand[k] < v) ? 1 : 0;
    adj[adj_off[I] + r] = v;
  }
}

// per node: element id and the node's local index packed as (e << 4) | a,
// sorted by element (insertion sort of a short list)
__global__ void k_pack_inc(const int32_t* conn, int npn, const int32_t* inc_off, int32_t* inc, int64_t n_nodes) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n_nodes) return;
  const int32_t b0 = inc_off[I], b1 = inc_off[I + 1];
  for (int32_t s = b0; s < b1; ++s) {
    const int32_t e = inc[s];
    int a = 0;
    while (a < npn - 1 && conn[(int64_t)e * npn + a] != I) ++a;
    int32_t v = (e << 4) | a;
    int32_t t = s;
    while (t > b0 && inc[t - 1] > v) {
      inc[t] = inc[t - 1];
      --t;
    }
    inc[t] = v;
  }
}

// The position of every (element, local node) in the node-sorted incidence
// list (element blocks of the force path and the element-row path), and for
// the element-row path (T10, rank_inc non-null) that incidence's slot-map row
// copied into incidence order (16 bytes each).
__global__ void k_inc_tables(const int32_t* inc, int64_t ninc, int npn, const uint8_t* rank, int32_t* incpos,
                             uint8_t* rank_inc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ninc) return;
  const int32_t v = inc[j];
  const int64_t ea = (int64_t)(v >> 4) * npn + (v & 15);
  incpos[ea] = (int32_t)j;
  if (rank_inc) *reinterpret_cast<uint4*>(rank_inc + j * 16) = *reinterpret_cast<const uint4*>(rank + ea * 16);
}

// upper triangle: row r keeps its columns >= r, a suffix of the sorted row
__global__ void k_upper_len(const int32_t* row_off, const int32_t* cols, int64_t n_dof, int32_t* len) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n_dof) return;
  if (r == n_dof) {
    len[r] = 0;
    return;
  }
  int32_t lo = row_off[r], hi = row_off[r + 1];  // first column >= r
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (cols[mid] < r) lo = mid + 1; else hi = mid;
  }
  len[r] = row_off[r + 1] - lo;
}

__global__ void k_upper_cols(const int32_t* row_off, const int32_t* cols, const int32_t* row_off_u, int64_t n_dof,
                             int32_t* cols_u) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_dof) return;
  const int32_t u0 = row_off_u[r], n = row_off_u[r + 1] - u0, f0 = row_off[r + 1] - n;
  for (int32_t j = 0; j < n; ++j) cols_u[u0 + j] = cols[f0 + j];
}

__global__ void k_node_nnz(const int32_t* nadj, int64_t n, int64_t blk, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = blk * nadj[i];
}

// row offsets: row 3 (mc I + c) + i starts at node_off[I] + (3c + i) * 3 mc nadj[I]
__global__ void k_rows(const int64_t* node_off, const int32_t* nadj, int64_t n_nodes, int mc, int32_t* row_off,
                       int64_t n_dof) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I < n_nodes) {
    const int64_t len = 3LL * mc * nadj[I];
    for (int r = 0; r < 3 * mc; ++r) row_off[3LL * mc * I + r] = (int32_t)(node_off[I] + r * len);
  }
  if (I == 0) row_off[n_dof] = (int32_t)node_off[n_nodes];
}

// columns of all rows of node I, one wavefront per node
__global__ __launch_bounds__(64) void k_cols(const int32_t* adj_off, const int32_t* adj, const int32_t* row_off,
                                             int64_t n_nodes, int mc, int32_t* cols) {
  const int64_t I = blockIdx.x;
  if (I >= n_nodes) return;
  const int32_t a0 = adj_off[I], na = adj_off[I + 1] - a0;
  const int rl = 3 * mc * na;   // row length
  const int total = 3 * mc * rl;
  for (int t = threadIdx.x; t < total; t += 64) {
    const int r = t / rl, col = t % rl;           // local row (c, i), column position
    const int jr = col / (3 * mc), rest = col % (3 * mc);  // rank of neighbour, (c', k)
    const int64_t J = adj[a0 + jr];
    cols[(int64_t)row_off[3LL * mc * I + r] + col] = (int32_t)(3 * mc * J + rest);
  }
}

// rank[e][p][p'] = position of node conn[e][p'] in the sorted adjacency of
// conn[e][p]; rows of rank_stride(npn) bytes
__global__ void k_rank(const int32_t* conn, int64_t n_elem, int npn, const int32_t* adj_off,
                       const int32_t* adj, uint8_t* rank, uint32_t* err) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n_elem * npn * npn;
  if (t >= total) return;
  const int64_t e = t / (npn * npn);
  const int p = (int)((t / npn) % npn), pb = (int)(t % npn);
  const int32_t a = conn[e * npn + p], b = conn[e * npn + pb];
  uint8_t* out = rank + (e * npn + p) * rank_stride(npn) + pb;
  int lo = adj_off[a], hi = adj_off[a + 1] - 1;
  int found = -1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t v = adj[mid];
    if (v == b) { found = mid; break; }
    if (v < b) lo = mid + 1; else hi = mid - 1;
  }
  const int r = found - adj_off[a];
  if (found < 0 || r > 255) {
    atomicOr(err, 2u);
    *out = 0;
  } else {
    *out = (uint8_t)r;
  }
}

__global__ void k_slots(const int32_t* conn, int64_t e0, int64_t ne, int npn, int mc, int nen,
                        const int32_t* row_off, const uint8_t* rank, int32_t* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nd = 3 * nen;
  const int64_t total = ne * nd * nd;
  if (t >= total) return;
  const int64_t el = t / (nd * nd);
  const int r = (int)((t / nd) % nd), c = (int)(t % nd);
  const int64_t e = e0 + el;
  const int al = r / 3, i = r % 3, be = c / 3, k = c % 3;
  const int pa = al / mc, ca = al % mc, pb = be / mc, cb = be % mc;
  const int64_t coef_a = (int64_t)mc * conn[e * npn + pa] + ca;
  const int64_t base = row_off[3 * coef_a + i];
  out[t] = (int32_t)(base + 3 * (mc * (int64_t)rank[(e * npn + pa) * rank_stride(npn) + pb] + cb) + k);
}

int grid_of(int64_t n, int block) { return (int)((n + block - 1) / block); }

template <typename T>
int scan_exclusive(const T* in, T* out, int64_t n, hipStream_t s) {
  size_t bytes = 0;
  TLFEA_HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, s));
  void* tmp = nullptr;
  TLFEA_HIP_CHECK(hipMalloc(&tmp, bytes > 0 ? bytes : 1));
  hipError_t err = hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, (int)n, s);
  hipError_t err2 = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  TLFEA_HIP_CHECK(err);
  TLFEA_HIP_CHECK(err2);
  return TLFEA_OK;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

int build_pattern(Mesh& m) {
  hipStream_t s = nullptr;
  const int npn = m.n_pn, mc = m.mc;
  const int64_t nn = m.n_pnodes, ninc = m.n_elem * npn;
  if (nn + 1 > INT32_MAX || ninc > INT32_MAX || m.n_elem >= (1LL << 27)) return TLFEA_ERR_TOO_LARGE;
  DevBuf cnt, inc_off, cursor, inc, nadj, node_nnz, node_off, err;
  TLFEA_HIP_CHECK(hipMalloc(&cnt.p, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&inc_off.p, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&cursor.p, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&inc.p, sizeof(int32_t) * (ninc > 0 ? ninc : 1)));
  // ownership of the incidence lists passes to the mesh on success
  int32_t* d_inc_off = (int32_t*)inc_off.p;
  int32_t* d_inc = (int32_t*)inc.p;
  TLFEA_HIP_CHECK(hipMalloc(&nadj.p, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&node_nnz.p, sizeof(int64_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&node_off.p, sizeof(int64_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&err.p, sizeof(uint32_t)));
  TLFEA_HIP_CHECK(hipMemset(cnt.p, 0, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMemset(cursor.p, 0, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMemset(nadj.p, 0, sizeof(int32_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMemset(node_nnz.p, 0, sizeof(int64_t) * (nn + 1)));
  TLFEA_HIP_CHECK(hipMemset(err.p, 0, sizeof(uint32_t)));
  auto* d_cnt = (int32_t*)cnt.p;
  auto* d_nadj = (int32_t*)nadj.p;
  auto* d_err = (uint32_t*)err.p;

  if (ninc > 0)
    hipLaunchKernelGGL(k_count_inc, dim3(grid_of(ninc, 256)), dim3(256), 0, s, m.d_conn, ninc, d_cnt);
  TLFEA_HIP_CHECK(hipGetLastError());
  int rc = scan_exclusive<int32_t>(d_cnt, d_inc_off, nn + 1, s);
  if (rc) return rc;
  if (ninc > 0)
    hipLaunchKernelGGL(k_fill_inc, dim3(grid_of(ninc, 256)), dim3(256), 0, s, m.d_conn, ninc, npn, d_inc_off,
                       (int32_t*)cursor.p, d_inc);
  TLFEA_HIP_CHECK(hipGetLastError());

  if (nn > 0)
    hipLaunchKernelGGL(k_adjacency, dim3((unsigned)nn), dim3(64), 0, s, m.d_conn, npn, d_inc_off, d_inc, nn, 0,
                       d_nadj, nullptr, nullptr, d_err);
  TLFEA_HIP_CHECK(hipGetLastError());
  uint32_t herr = 0;
  TLFEA_HIP_CHECK(hipMemcpy(&herr, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (herr) return TLFEA_ERR_UNSUPPORTED;

  // adjacency offsets
  int32_t* d_adj_off = nullptr;
  TLFEA_HIP_CHECK(hipMalloc(&d_adj_off, sizeof(int32_t) * (nn + 1)));
  rc = scan_exclusive<int32_t>(d_nadj, d_adj_off, nn + 1, s);
  if (rc) { (void)hipFree(d_adj_off); return rc; }
  int32_t n_adj_total = 0;
  TLFEA_HIP_CHECK(hipMemcpy(&n_adj_total, d_adj_off + nn, sizeof(int32_t), hipMemcpyDeviceToHost));
  int32_t* d_adj = nullptr;
  TLFEA_HIP_CHECK(hipMalloc(&d_adj, sizeof(int32_t) * (n_adj_total > 0 ? n_adj_total : 1)));
  if (nn > 0)
    hipLaunchKernelGGL(k_adjacency, dim3((unsigned)nn), dim3(64), 0, s, m.d_conn, npn, d_inc_off, d_inc, nn, 1,
                       d_nadj, d_adj_off, d_adj, d_err);
  TLFEA_HIP_CHECK(hipGetLastError());

  // DOF rows: every neighbour contributes a (3 mc) x (3 mc) block
  const int64_t blk = 9LL * mc * mc;
  if (nn > 0)
    hipLaunchKernelGGL(k_node_nnz, dim3(grid_of(nn, 256)), dim3(256), 0, s, d_nadj, nn, blk,
                       (int64_t*)node_nnz.p);
  TLFEA_HIP_CHECK(hipGetLastError());
  rc = scan_exclusive<int64_t>((int64_t*)node_nnz.p, (int64_t*)node_off.p, nn + 1, s);
  if (rc) { (void)hipFree(d_adj_off); (void)hipFree(d_adj); return rc; }
  int64_t nnz = 0;
  TLFEA_HIP_CHECK(hipMemcpy(&nnz, (int64_t*)node_off.p + nn, sizeof(int64_t), hipMemcpyDeviceToHost));
  if (nnz > INT32_MAX) { (void)hipFree(d_adj_off); (void)hipFree(d_adj); return TLFEA_ERR_TOO_LARGE; }

  int32_t *d_row_off = nullptr, *d_cols = nullptr;
  uint8_t* d_rank = nullptr;
  if (hipMalloc(&d_row_off, sizeof(int32_t) * (m.n_dof + 1)) != hipSuccess ||
      hipMalloc(&d_cols, sizeof(int32_t) * (nnz > 0 ? nnz : 1)) != hipSuccess ||
      hipMalloc(&d_rank, (size_t)(m.n_elem > 0 ? m.n_elem * npn * rank_stride(npn) : 1)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(d_row_off); (void)hipFree(d_cols); (void)hipFree(d_rank);
    (void)hipFree(d_adj_off); (void)hipFree(d_adj);
    return TLFEA_ERR_NOMEM;
  }
  hipLaunchKernelGGL(k_rows, dim3(grid_of(nn > 0 ? nn : 1, 256)), dim3(256), 0, s, (int64_t*)node_off.p, d_nadj,
                     nn, mc, d_row_off, m.n_dof);
  if (nn > 0)
    hipLaunchKernelGGL(k_cols, dim3((unsigned)nn), dim3(64), 0, s, d_adj_off, d_adj, d_row_off, nn, mc, d_cols);
  const int64_t nrank = m.n_elem * npn * npn;
  if (nrank > 0) (void)hipMemsetAsync(d_rank, 0, (size_t)m.n_elem * npn * rank_stride(npn), s);  // padding bytes
  if (nrank > 0)
    hipLaunchKernelGGL(k_rank, dim3(grid_of(nrank, 256)), dim3(256), 0, s, m.d_conn, m.n_elem, npn, d_adj_off,
                       d_adj, d_rank, d_err);
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipDeviceSynchronize();
  uint32_t herr2 = 0;
  hipError_t e3 = hipMemcpy(&herr2, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || herr2) {
    (void)hipFree(d_row_off); (void)hipFree(d_cols); (void)hipFree(d_rank);
    (void)hipFree(d_adj_off); (void)hipFree(d_adj);
    if (herr2) return TLFEA_ERR_UNSUPPORTED;
    return TLFEA_ERR_HIP;
  }
  // packed, sorted incidence for pass 2
  if (nn > 0)
    hipLaunchKernelGGL(k_pack_inc, dim3(grid_of(nn, 128)), dim3(128), 0, s, m.d_conn, npn, d_inc_off, d_inc, nn);
  // incidence positions (every element type) and the incidence-ordered
  // slot-map rows of the element-row path (T10 only)
  DevBuf incpos, rank_inc;
  if (ninc > 0) {
    static_assert(rank_stride(10) == 16, "T10 slot-map rows are 16 bytes");
    const bool t10 = m.elem_type == TLFEA_T10;
    if (hipMalloc(&incpos.p, sizeof(int32_t) * ninc) != hipSuccess ||
        (t10 && hipMalloc(&rank_inc.p, 16 * ninc) != hipSuccess)) {
      (void)hipGetLastError();
      (void)hipFree(d_row_off); (void)hipFree(d_cols); (void)hipFree(d_rank);
      (void)hipFree(d_adj_off); (void)hipFree(d_adj);
      return TLFEA_ERR_NOMEM;
    }
    hipLaunchKernelGGL(k_inc_tables, dim3(grid_of(ninc, 256)), dim3(256), 0, s, d_inc, ninc, npn, d_rank,
                       (int32_t*)incpos.p, (uint8_t*)rank_inc.p);
  }
  std::vector<int32_t> h_inc_off(nn + 1), h_adj_off(nn + 1);
  hipError_t e4 = hipGetLastError();
  hipError_t e5 = hipMemcpy(h_inc_off.data(), d_inc_off, sizeof(int32_t) * (nn + 1), hipMemcpyDeviceToHost);
  hipError_t e6 = hipMemcpy(h_adj_off.data(), d_adj_off, sizeof(int32_t) * (nn + 1), hipMemcpyDeviceToHost);
  const GatherTuning tune = gather_tuning(m);
  RangePlan plan = plan_ranges(h_inc_off, h_adj_off, mc, tune);
  int32_t* d_ranges = nullptr;
  hipError_t e7 = hipMalloc(&d_ranges, sizeof(int32_t) * plan.ranges.size());
  hipError_t e8 = e7 == hipSuccess ? hipMemcpy(d_ranges, plan.ranges.data(), sizeof(int32_t) * plan.ranges.size(),
                                               hipMemcpyHostToDevice)
                                   : e7;
  // a range's LDS segment must fit next to the staging buffers (checked again at launch)
  const bool too_big = !plan_fits(plan);
  if (e4 != hipSuccess || e5 != hipSuccess || e6 != hipSuccess || e8 != hipSuccess || too_big) {
    (void)hipFree(d_row_off); (void)hipFree(d_cols); (void)hipFree(d_rank);
    (void)hipFree(d_adj_off); (void)hipFree(d_adj); (void)hipFree(d_ranges);
    return too_big ? TLFEA_ERR_UNSUPPORTED : TLFEA_ERR_HIP;
  }
  // replace a previous pattern, if any
  (void)hipFree(m.d_row_off); (void)hipFree(m.d_cols); (void)hipFree(m.d_rank);
  (void)hipFree(m.d_adj_off); (void)hipFree(m.d_adj); (void)hipFree(m.d_ranges);
  (void)hipFree(m.d_inc_off); (void)hipFree(m.d_inc);
  (void)hipFree(m.d_incpos); (void)hipFree(m.d_rank_inc);
  (void)hipFree(m.d_mass);  // indexed by the old adjacency
  m.d_mass = nullptr;
  m.density = 0.0;
  (void)hipFree(m.d_row_off_u);
  (void)hipFree(m.d_cols_u);
  m.d_row_off_u = m.d_cols_u = nullptr;
  m.nnz_u = -1;
  m.d_incpos = (int32_t*)incpos.p;
  m.d_rank_inc = (uint8_t*)rank_inc.p;
  incpos.p = rank_inc.p = nullptr;
  m.d_row_off = d_row_off;
  m.d_cols = d_cols;
  m.d_rank = d_rank;
  m.d_adj_off = d_adj_off;
  m.d_adj = d_adj;
  inc_off.p = nullptr;
  inc.p = nullptr;
  m.d_inc_off = d_inc_off;
  m.d_inc = d_inc;
  m.d_ranges = d_ranges;
  m.h_ranges = std::move(plan.ranges);
  m.n_ranges = (int)m.h_ranges.size() - 1;
  m.max_range_values = plan.max_values;
  m.max_range_rows = plan.max_rows;
  m.max_range_inc = plan.max_inc;
  m.tune = tune;
  m.h_inc_off = std::move(h_inc_off);
  m.h_adj_off = std::move(h_adj_off);
  m.nnz = nnz;
  m.has_pattern = true;
  return TLFEA_OK;
}

static int env_int(const char* name, int fallback, int lo, int hi) {
  const char* v = std::getenv(name);
  if (!v || !*v) return fallback;
  const long x = std::strtol(v, nullptr, 10);
  return (x < lo || x > hi) ? fallback : (int)x;
}

GatherTuning gather_tuning(const Mesh& m) {
  GatherTuning t;
  if (m.elem_type == TLFEA_T10 && m.precision == TLFEA_MIXED) t.range_values = 2048;
  t.waves = env_int("TLFEA_GATHER_WAVES", t.waves, 1, 8);
  t.range_tasks = env_int("TLFEA_RANGE_TASKS", t.range_tasks, 1, 1 << 20);
  t.range_values = env_int("TLFEA_RANGE_VALUES", t.range_values, 1, 12 * 1024);
  return t;
}

RangePlan plan_ranges(const std::vector<int32_t>& inc_off, const std::vector<int32_t>& adj_off, int mc,
                      const GatherTuning& t) {
  RangePlan p;
  const int64_t nn = (int64_t)inc_off.size() - 1;
  int64_t tasks = 0, vals = 0, rows = 0, nodes = 0, incs = 0;
  auto close = [&](int64_t end) {
    p.ranges.push_back((int32_t)end);
    p.max_values = std::max(p.max_values, vals);
    p.max_rows = std::max(p.max_rows, rows);
    p.max_inc = std::max(p.max_inc, incs);
    tasks = vals = rows = nodes = incs = 0;
  };
  for (int64_t I = 0; I < nn; ++I) {
    const int64_t nI = inc_off[I + 1] - inc_off[I];
    const int64_t tI = 9LL * mc * nI;                                     // tasks of the node
    const int64_t vI = 9LL * mc * mc * (adj_off[I + 1] - adj_off[I]) + 3LL * mc;  // its CSR values + force rows
    if (nodes > 0 && (tasks + tI > t.range_tasks || vals + vI > t.range_values || nodes >= kMaxRangeNodes)) close(I);
    incs += nI;
    tasks += tI;
    vals += vI;
    rows += 3LL * mc;
    ++nodes;
  }
  if (nodes > 0) close(nn);
  return p;
}

int build_upper_pattern(Mesh& m) {
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (m.d_row_off_u) return TLFEA_OK;
  const int64_t n = m.n_dof;
  DevBuf len;
  int32_t* d_ro = nullptr;
  TLFEA_HIP_CHECK(hipMalloc(&len.p, sizeof(int32_t) * (n + 1)));
  TLFEA_HIP_CHECK(hipMalloc(&d_ro, sizeof(int32_t) * (n + 1)));
  hipLaunchKernelGGL(k_upper_len, dim3(grid_of(n + 1, 256)), dim3(256), 0, nullptr, m.d_row_off, m.d_cols, n,
                     (int32_t*)len.p);
  hipError_t e0 = hipGetLastError();
  int rc = e0 == hipSuccess ? scan_exclusive<int32_t>((int32_t*)len.p, d_ro, n + 1, nullptr) : TLFEA_ERR_HIP;
  int32_t nnz_u = 0;
  if (!rc && hipMemcpy(&nnz_u, d_ro + n, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) rc = TLFEA_ERR_HIP;
  int32_t* d_cu = nullptr;
  if (!rc && hipMalloc(&d_cu, sizeof(int32_t) * (nnz_u > 0 ? nnz_u : 1)) != hipSuccess) {
    (void)hipGetLastError();
    rc = TLFEA_ERR_NOMEM;
  }
  if (!rc && n > 0)
    hipLaunchKernelGGL(k_upper_cols, dim3(grid_of(n, 256)), dim3(256), 0, nullptr, m.d_row_off, m.d_cols, d_ro, n,
                       d_cu);
  if (!rc && (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)) rc = TLFEA_ERR_HIP;
  if (rc) {
    (void)hipFree(d_ro);
    (void)hipFree(d_cu);
    return rc;
  }
  m.d_row_off_u = d_ro;
  m.d_cols_u = d_cu;
  m.nnz_u = nnz_u;
  return TLFEA_OK;
}

std::vector<GatherTuning> gather_candidates() {
  std::vector<GatherTuning> c;
  for (int w : {2, 4, 8})
    for (int t : {384, 768, 1536})
      for (int v : {2048, 4096, 8192}) c.push_back(GatherTuning{w, t, v});
  return c;
}

bool plan_fits(const RangePlan& p) { return p.max_values * (int64_t)sizeof(double) <= kMaxSegmentBytes; }

int set_gather_shape(Mesh& m, const GatherTuning& t) {
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (t.waves < 1 || t.waves > 8 || t.range_tasks < 1 || t.range_values < 1) return TLFEA_ERR_INVALID;
  RangePlan p = plan_ranges(m.h_inc_off, m.h_adj_off, m.mc, t);
  if (!plan_fits(p)) return TLFEA_ERR_UNSUPPORTED;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  int32_t* d = nullptr;
  if (hipMalloc(&d, sizeof(int32_t) * p.ranges.size()) != hipSuccess) {
    (void)hipGetLastError();
    return TLFEA_ERR_NOMEM;
  }
  if (hipMemcpy(d, p.ranges.data(), sizeof(int32_t) * p.ranges.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return TLFEA_ERR_HIP;
  }
  // the old ranges may still be read by queued work on the mesh's last stream
  if (m.d_ranges && hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(d);
    return TLFEA_ERR_HIP;
  }
  (void)hipFree(m.d_ranges);
  m.d_ranges = d;
  m.h_ranges = std::move(p.ranges);
  m.n_ranges = (int)m.h_ranges.size() - 1;
  m.max_range_values = p.max_values;
  m.max_range_rows = p.max_rows;
  m.max_range_inc = p.max_inc;
  m.tune = t;
  return TLFEA_OK;
}

int export_slot_map(const Mesh& m, int64_t e0, int64_t ne, int32_t* d_out, hipStream_t s) {
  const int64_t total = ne * 9LL * m.n_en * m.n_en;
  if (total <= 0) return TLFEA_OK;
  hipLaunchKernelGGL(k_slots, dim3(grid_of(total, 256)), dim3(256), 0, s, m.d_conn, e0, ne, m.n_pn, m.mc, m.n_en,
                     m.d_row_off, m.d_rank, d_out);
  TLFEA_HIP_CHECK(hipGetLastError());
  return TLFEA_OK;
}

}  // namespace tlfea
