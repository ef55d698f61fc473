// tlfea_internal.h -- private declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/tlfea.h"
#include "material.h"

#define TLFEA_API extern "C" __attribute__((visibility("default")))

#define TLFEA_HIP_CHECK(expr)                     \
  do {                                            \
    hipError_t err__ = (expr);                    \
    if (err__ != hipSuccess) {                    \
      (void)hipGetLastError();                    \
      return err__ == hipErrorOutOfMemory ? TLFEA_ERR_NOMEM : TLFEA_ERR_HIP; \
    }                                             \
  } while (0)

namespace tlfea {

constexpr int kStageThreads = 256;     // (element, point) indices per pass-1 workgroup
constexpr int kMaxRangeNodes = 64;      // nodes per pass-2 workgroup

// Bytes per (element, node) row of the slot map: padded so that a row is one
// aligned vector load (T10: 10 ranks in 16 bytes, ANCF: 4 ranks in 4 bytes).
constexpr int rank_stride(int npn) { return npn <= 4 ? 4 : 16; }

// Pass-2 launch shape.  Node ranges are cut so that a range has at most
// range_tasks tasks (lanes) and range_values LDS doubles (a single node may
// exceed both); a workgroup of `waves` waves processes one range.
struct GatherTuning {
  int waves = 4;
  int range_tasks = 768;
  int range_values = 4096;
};
// defaults ({4, 768, 2048} for T10 meshes created in mixed precision, whose
// tangent takes the element-row path, else {4, 768, 4096}), overridden by
// TLFEA_GATHER_WAVES / TLFEA_RANGE_TASKS / TLFEA_RANGE_VALUES when set
struct Mesh;
GatherTuning gather_tuning(const Mesh& m);
// a range's LDS segment (CSR values + force rows) must stay below this
constexpr int64_t kMaxSegmentBytes = 96 * 1024;

// Greedy cut of the pattern nodes 0 .. n-1, in order, into ranges of at most
// t.range_tasks tasks and t.range_values LDS doubles (a single node may exceed
// both; at most kMaxRangeNodes nodes).  inc_off / adj_off: node -> incident
// elements / adjacent nodes, n + 1 prefix offsets each.
struct RangePlan {
  std::vector<int32_t> ranges{0};  // n_ranges + 1 node boundaries
  int64_t max_values = 0, max_rows = 0, max_inc = 0;
};
RangePlan plan_ranges(const std::vector<int32_t>& inc_off, const std::vector<int32_t>& adj_off, int mc,
                      const GatherTuning& t);
bool plan_fits(const RangePlan& p);  // every segment below kMaxSegmentBytes

// Launch shapes the autotuners time: waves {2, 4, 8} x range_tasks {384, 768,
// 1536} x range_values {2048, 4096, 8192}.
std::vector<GatherTuning> gather_candidates();

// Autotuning loop shared by meshes and batches.  Every candidate that apply(t)
// accepts (TLFEA_ERR_UNSUPPORTED: skipped) is run() once to warm up and then
// `reps` times between two events on stream s.  The shape in use is timed
// first (after three warm-up calls) and again last, and keeps the lower of its
// two times, so that its place in the sweep does not count against it.  The
// fastest candidate replaces it only if it is at least kTuneMargin faster
// (shapes within a few percent trade places from run to run); the chosen shape
// is applied again and run() once more, so the outputs hold its result.  On an
// error the shape `current` is restored.  Synchronises the stream.
constexpr float kTuneMargin = 0.05f;
template <class Apply, class Run>
int autotune_shape(const GatherTuning& current, Apply&& apply, Run&& run, int reps, hipStream_t s,
                   GatherTuning& best, float& best_ms) {
  if (reps < 1 || reps > 1000) return TLFEA_ERR_INVALID;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipGetLastError();
    return TLFEA_ERR_HIP;
  }
  auto same = [](const GatherTuning& a, const GatherTuning& b) {
    return a.waves == b.waves && a.range_tasks == b.range_tasks && a.range_values == b.range_values;
  };
  std::vector<GatherTuning> cand{current};
  for (const GatherTuning& t : gather_candidates())
    if (!same(t, current)) cand.push_back(t);
  cand.push_back(current);
  best_ms = -1.0f;
  float current_ms = -1.0f;
  int rc = TLFEA_OK;
  for (size_t c = 0; c < cand.size(); ++c) {
    const GatherTuning& t = cand[c];
    rc = apply(t);
    if (rc == TLFEA_ERR_UNSUPPORTED) continue;
    for (int i = 0; !rc && i < (c == 0 ? 3 : 1); ++i) rc = run();
    if (rc == TLFEA_ERR_UNSUPPORTED) continue;  // more LDS than the device gives a workgroup
    for (int i = 0; !rc && i < reps; ++i) {
      if (i == 0 && hipEventRecord(e0, s) != hipSuccess) rc = TLFEA_ERR_HIP;
      if (!rc) rc = run();
    }
    float ms = 0.0f;
    if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = TLFEA_ERR_HIP;
    if (rc) break;
    ms /= (float)reps;
    if (same(t, current)) current_ms = current_ms < 0.0f ? ms : std::min(current_ms, ms);
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  if (!rc && current_ms >= 0.0f && best_ms > (1.0f - kTuneMargin) * current_ms) {
    best = current;  // not worth a change
    best_ms = current_ms;
  }
  if (!rc && best_ms < 0.0f) rc = TLFEA_ERR_UNSUPPORTED;  // no candidate fits
  if (!rc) {
    rc = apply(best);
    if (!rc) rc = run();
  }
  if (rc) (void)apply(current);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// Per-mesh state.  All d_* members are device allocations owned by the mesh.
struct Mesh {
  // bumped by every change a batch snapshots (pattern rebuild, material, precision)
  uint64_t generation = 0;
  int device = 0;
  int elem_type = 0;
  int n_en = 0;        // shape functions (coefficient vectors) per element
  int n_pn = 0;        // pattern nodes per element (T10: 10 nodes; ANCF shell: 4, beam: 2 physical nodes)
  int mc = 0;          // coefficient vectors per pattern node (T10: 1; ANCF: 4)
  int n_qp = 0;
  int gl[3] = {0, 0, 0};
  int64_t n_elem = 0, n_coef = 0, n_pnodes = 0, n_dof = 0;
  double thickness = 0.0;  // ANCF shell thickness; beam cross-section height
  double width = 0.0;      // beam cross-section width
  int precision = TLFEA_FP64;
  int material = 0;
  double params[3] = {0, 0, 0};
  double kv_eta = 0, kv_lambda = 0;
  MatParams mp{};

  int32_t* d_conn = nullptr;      // n_elem * n_pn
  double* d_X = nullptr;          // n_coef * 3
  double* d_geo = nullptr;        // records of {J0^-1 (9, row-major [m][J]), det J0}
  bool affine = false;            // true: one record per element; false: per (element, qp)
  double* d_escale = nullptr;     // ANCF: per element {lx/2, ly/2} (shell) or {L, W/2} (beam)
  uint32_t* d_flags = nullptr;    // runtime flags
  double* d_mp = nullptr;         // 5 material constants converted from a device parameter vector

  // pass-2 work partition: node ranges whose CSR rows form one contiguous segment
  int32_t* d_inc_off = nullptr;   // n_pnodes + 1, node -> incident elements
  int32_t* d_inc = nullptr;       // (element << 4) | local node index, sorted by element per node
  int32_t* d_ranges = nullptr;    // n_ranges + 1 node boundaries
  int32_t* d_incpos = nullptr;    // T10: incidence position of every (element, local node)
  uint8_t* d_rank_inc = nullptr;  // T10: slot-map rows in incidence order (16 bytes each)
  std::vector<int32_t> h_ranges;
  int n_ranges = 0;
  int64_t max_range_values = 0;   // largest LDS segment (CSR values + force rows), in doubles
  int64_t max_range_rows = 0;     // largest number of force rows of a range
  int64_t max_range_inc = 0;      // largest number of incidences of a range
  GatherTuning tune;              // launch shape the ranges were cut for
  std::vector<int32_t> h_inc_off; // host copies of inc_off / adj_off (range cuts)
  std::vector<int32_t> h_adj_off;
  void* d_stage = nullptr;        // pass-1 records
  size_t stage_cap = 0;
  int staged = 0;                 // what the last pass 1 left: 0 none, 1 force records, 2 force + tangent,
                                  // 3 element row blocks, 4 element force blocks
                                  // records, 3 element row blocks (force + tangent)
  int staged_precision = -1;
  bool staged_sym = false;        // point records of the last pass 1 in the symmetric float64 layout

  bool has_pattern = false;
  int64_t nnz = -1;
  int32_t* d_row_off = nullptr;   // n_dof + 1
  int32_t* d_cols = nullptr;      // nnz
  int32_t* d_adj_off = nullptr;   // n_pnodes + 1, pattern-node adjacency
  int32_t* d_adj = nullptr;
  uint8_t* d_rank = nullptr;      // n_elem * n_pn rows of rank_stride(n_pn) bytes: rank of node b in adj(node a)
  double* d_mass = nullptr;       // consistent mass: mc x mc block M_(I,k)(J,l) per adjacency entry (adj order)
  int32_t* d_row_off_u = nullptr; // upper-triangle CSR (columns >= row), built on request
  int32_t* d_cols_u = nullptr;
  int64_t nnz_u = -1;
  double density = 0.0;           // of the mass above (0: not built)
  double* d_solver = nullptr;     // first-order solver: iteration counter, bias corrections, norm partials, norms
  double* d_dv = nullptr;         // gradient: v - v_prev per DOF (allocated by the first call)
  hipStream_t last_stream = nullptr;
};

// Everything one assembly launch needs (passed by value to the kernels).
struct AsmArgs {
  const int32_t* conn;
  const double* X;
  const double* geo;
  const double* escale;
  double half_h;       // ANCF thickness / 2
  int affine;
  int64_t n_elem;
  int n_tiles;
  const double* q;
  const double* qdot;  // may be null
  double* f;           // may be null
  double* vals;        // may be null
  const int32_t* row_off;
  const uint8_t* rank;
  MatParams mp;
  const double* mp_dev;  // non-null: c0, c1, c2, eta, lam_v read from here instead of mp
  double alpha, beta;
  uint32_t* flags;
};


// Pass-2 arguments of one mesh.
struct GatherArgs {
  const int32_t* ranges;
  // Newton matrix: M_IJ / h added to the diagonal entries of each 3x3 block
  // (T10; mass == NULL: none)
  const double* mass;
  const int32_t* adj_off;
  double inv_h;
  // upper-triangle output: vals holds the values of the upper CSR (row
  // offsets row_off_u; a row's upper entries are the suffix of its full row)
  const int32_t* row_off_u;
  const int32_t* inc_off;
  const int32_t* inc;
  const int32_t* row_off;
  const uint8_t* rank;
  const double* escale;
  double half_h;
  const void* stage;
  double* f;
  double* vals;
  int inc_cap;  // LDS bytes for the range's incidence -> node table (multiple of 16)
};

// Batched launch: one descriptor per body; pass 1 runs over the concatenated
// (element, point) indices, pass 2 over the concatenated node ranges.
struct BatchBody {
  const int32_t* conn;
  const double* X;
  const double* geo;
  const double* escale;
  const int32_t* row_off;
  const uint8_t* rank;
  const int32_t* inc_off;
  const int32_t* inc;
  const int32_t* incpos;     // element-row path: incidence position of every (element, node)
  const uint8_t* rank_inc;   // element-row path: slot-map rows in incidence order
  int64_t n_elem, dof_off, nnz_off, point_off, block_off;
  int64_t blk_inc_off;       // element-row path: the body's first row block
  int64_t rblock_off;        // element-row path: the body's first pass-1 workgroup
  int affine;
  double half_h;
  MatParams mp;
};
struct BatchRange {
  int32_t body, I0, I1;
};
struct BatchArgs {
  const BatchBody* bodies;
  const BatchRange* ranges;
  int n_bodies;
  int64_t n_points, n_blocks;
  int64_t n_rblocks;  // pass-1 workgroups of the element-row path
  int rows;           // 1: element-row path (T10, mixed), 0: per-point records
  void* stage;
  const double* q;
  const double* qdot;
  const double* h;   // per body
  double* f;
  double* vals;
  uint32_t* flags;
  int inc_cap;  // LDS bytes for a range's incidence -> node table (multiple of 16)
};

// Schedule of a batched element-row launch.  persistent = 0: one workgroup per
// tile and per range (bodies found by bisection).  persistent = 1: fixed grids
// of grid_tiles / grid_ranges workgroups taking items from two device
// counters, tiles of tile_elems elements listed longest first, ranges ordered
// by decreasing work.
struct BatchSchedule {
  int persistent = 0;
  int tile_elems = 25;
  const int2* tiles = nullptr;
  int n_tiles = 0;
  const int32_t* range_order = nullptr;
  unsigned* counters = nullptr;
  int grid_tiles = 0, grid_ranges = 0;
};
int batch_lpt_occupancy(int tile_elems, int waves, size_t lds_all, int* tiles_per_cu, int* ranges_per_cu);

MatParams make_params(int material, const double* params, double eta, double lam_v);

// bytes of pass-1 records for a mesh / per record
// Element-row path: the tangent in mixed precision, every element type (the
// environment variable TLFEA_ELEMENT_ROWS=0 switches it off; batches take it
// for T10 only).  Pass 1 then leaves one row block per incidence instead of
// per-point records.
bool use_rows(const Mesh& m, bool want_k);
bool point_records_sym(const Mesh& m, bool want_k);
// Force-only path (every element type; TLFEA_FORCE_BLOCKS=0 switches it off):
// pass 1 leaves one float-or-double force block of 3 mc values per incidence.
bool use_force_blocks(const Mesh& m, bool want_k);
size_t stage_bytes(const Mesh& m, bool want_k);
size_t stage_record_bytes(int precision);
size_t row_block_bytes();  // element-row path: bytes per (element, node) row block
int row_elems();           // element-row path: elements per pass-1 workgroup
size_t row_block_bytes_for(int elem_type, int gl0);  // the same per element type
int row_elems_for(int elem_type, int gl0);
int launch_batch(int elem_type, int gl0, int precision, const GatherTuning& tune, const BatchArgs& b,
                 int n_ranges, size_t lds, hipStream_t s, const BatchSchedule& sc);

// kernel launchers (assemble.hip)
int launch_zero(double* p, int64_t n, hipStream_t s);
// pass 1: per-point records into m.d_stage; pass 2: per-node reduction into f / vals
int launch_points(const Mesh& m, const AsmArgs& a, bool want_k, hipStream_t s);
// Optional parts of pass 2: the Newton mass term, and output to the upper
// triangle only (row offsets of the upper CSR; vals is then its values).
struct GatherOptions {
  const double* mass = nullptr;  // mc x mc block per adjacency entry (Mesh::d_mass)
  double inv_h = 0.0;
  const int32_t* row_off_u = nullptr;
};
int launch_nodes(const Mesh& m, double* f, double* vals, bool accumulate, hipStream_t s,
                 const GatherOptions& mt = GatherOptions{});

// pattern builder (pattern.hip)
int build_pattern(Mesh& m);
// upper-triangle CSR of the mesh pattern (needs the pattern; synchronises)
int build_upper_pattern(Mesh& m);
// re-cut the mesh's node ranges for launch shape t (needs the pattern);
// TLFEA_ERR_UNSUPPORTED if a range would not fit, leaving the mesh unchanged
int set_gather_shape(Mesh& m, const GatherTuning& t);
int export_slot_map(const Mesh& m, int64_t e0, int64_t ne, int32_t* d_out, hipStream_t s);

// geometry precompute (mesh.hip)
int precompute_geometry(Mesh& m);

// work buffer of at least `bytes` (mesh.hip); reallocation synchronises
int ensure_stage(Mesh& m, size_t bytes);
// pass 2 over float64 force-type records (Phat_ik at 4 i + k, 12 per point)
// at `records`, written to `out` (n_dof); used by the VJP (assemble.hip)
// per-node sums, in incidence order, of float64 blocks of 3 mc values per
// (element, node) incidence at the node-sorted incidence positions -> out (n_dof)
int launch_block_sum(const Mesh& m, const double* blk, double* out, hipStream_t s);
constexpr size_t kNoallocScratchBytes = TLFEA_NOALLOC_SCRATCH_BYTES;
size_t noalloc_force_bytes(const Mesh& m);
int launch_force_noalloc(const Mesh& m, const AsmArgs& a, double* f, hipStream_t s);
// the force-block path with the mesh's work buffer (force only, pattern needed)
int launch_force_blocks(Mesh& m, const AsmArgs& a, double* f, hipStream_t s);
// material constants of a device parameter vector (p0, p1, p2, kv_eta, kv_lambda) -> m.d_mp
int launch_params(const Mesh& m, const double* d_params, hipStream_t s);

// VJP (vjp.hip)
int launch_vjp(Mesh& m, const double* q, const double* qdot, const double* w, double* gq,
               double* gqdot, double* gparam, hipStream_t s,
               const double* d_params = nullptr);

AsmArgs make_args(const Mesh& m, const double* q, const double* qdot, double* f, double* vals,
                  double alpha, double beta);

}  // namespace tlfea

struct tlfea_mesh_s {
  tlfea::Mesh m;
};
