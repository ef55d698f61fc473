// batch.hip -- many independent bodies assembled by one pair of launches.
//
// The paper runs one solver per body; for many small, uneven bodies a launch
// per body leaves most of the GPU idle.  Here every body keeps its own mesh,
// CSR pattern and slot map, and the batch concatenates their work: pass 1 runs
// over the concatenated (element, point) indices of all bodies, pass 2 over
// the concatenated node ranges, each workgroup writing into its body's slice
// of the concatenated q / f / CSR value arrays.  On a non-default stream the
// two launches are captured once into a HIP graph and replayed while the
// argument pointers stay the same.
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "tlfea_internal.h"

using tlfea::BatchArgs;
using tlfea::BatchBody;
using tlfea::BatchRange;

struct tlfea_batch_s {
  std::vector<tlfea_mesh_t> meshes;
  std::vector<uint64_t> generation;  // each member's generation when the batch copied its state
  int device = 0;
  int elem_type = 0, gl0 = 0, precision = TLFEA_FP64;
  std::vector<int64_t> dof_off, nnz_off;
  BatchBody* d_bodies = nullptr;
  BatchRange* d_ranges = nullptr;
  int n_ranges = 0;
  size_t ranges_cap = 0;             // BatchRange entries d_ranges holds
  tlfea::GatherTuning tune;          // pass-2 launch shape the ranges are cut for
  int64_t n_points = 0, n_blocks = 0;
  int rows = 0;                      // element-row path (mixed; persistent schedule for T10)
  int64_t n_inc = 0, n_rblocks = 0;  // its row blocks and pass-1 workgroups
  size_t lds = 0;
  int inc_cap = 0;
  void* d_stage = nullptr;
  uint32_t* d_flags = nullptr;
  // schedule of the element-row launches (persistent LPT form or one workgroup per item)
  tlfea::BatchSchedule sched;
  std::vector<BatchRange> h_ranges;  // the current range cut, host copy
  int2* d_tiles = nullptr;
  int32_t* d_range_order = nullptr;
  size_t tiles_cap = 0, order_cap = 0;
  unsigned* d_counters = nullptr;
  uint64_t signature = 0;  // of the member sizes, element type and precision (autotuner cache key)
  // graph cache, keyed by the argument pointers and the stream
  hipGraphExec_t exec = nullptr;
  const void* key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

static void drop_graph(tlfea_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  std::fill(b->key, b->key + 6, nullptr);
}

static void batch_free(tlfea_batch_s* b) {
  drop_graph(b);
  (void)hipFree(b->d_bodies);
  (void)hipFree(b->d_ranges);
  (void)hipFree(b->d_stage);
  (void)hipFree(b->d_flags);
  (void)hipFree(b->d_tiles);
  (void)hipFree(b->d_range_order);
  (void)hipFree(b->d_counters);
  delete b;
}

template <typename T>
static int upload(T*& d, size_t& cap, const std::vector<T>& h) {
  if (h.size() > cap || !d) {
    if (d && hipDeviceSynchronize() != hipSuccess) return TLFEA_ERR_HIP;  // queued work may read the old list
    T* nd = nullptr;
    if (hipMalloc(&nd, sizeof(T) * std::max<size_t>(1, h.size())) != hipSuccess) {
      (void)hipGetLastError();
      return TLFEA_ERR_NOMEM;
    }
    (void)hipFree(d);
    d = nd;
    cap = std::max<size_t>(1, h.size());
  } else if (hipDeviceSynchronize() != hipSuccess) {
    return TLFEA_ERR_HIP;
  }
  if (!h.empty() && hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice) != hipSuccess)
    return TLFEA_ERR_HIP;
  return TLFEA_OK;
}

// The persistent (LPT) schedule of the element-row batch: every body's tiles of
// tile_elems elements, full tiles of the largest bodies first and partial tiles
// last; the ranges by decreasing work (incidences, then rows); grids of as
// many workgroups as the GPU holds at once.
static int batch_plan_lpt(tlfea_batch_s* b, int tile_elems) {
  if (!b->rows || b->elem_type != TLFEA_T10) return TLFEA_ERR_UNSUPPORTED;
  if (tile_elems != 16 && tile_elems != tlfea::row_elems()) return TLFEA_ERR_INVALID;
  struct Tile {
    int64_t work, body_size;
    int body, tile;
  };
  std::vector<Tile> tiles;
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    const int64_t ne = b->meshes[i]->m.n_elem;
    for (int64_t t = 0; t * tile_elems < ne; ++t)
      tiles.push_back(Tile{std::min<int64_t>(tile_elems, ne - t * tile_elems), ne, (int)i, (int)t});
  }
  if (tiles.size() > (size_t)INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  std::stable_sort(tiles.begin(), tiles.end(), [](const Tile& x, const Tile& y) {
    return x.work != y.work ? x.work > y.work : x.body_size > y.body_size;
  });
  std::vector<int2> items(tiles.size());
  for (size_t k = 0; k < tiles.size(); ++k) items[k] = int2{tiles[k].body, tiles[k].tile};
  std::vector<int64_t> work(b->h_ranges.size());
  for (size_t r = 0; r < b->h_ranges.size(); ++r) {
    const BatchRange& br = b->h_ranges[r];
    const tlfea::Mesh& m = b->meshes[br.body]->m;
    work[r] = 16 * (int64_t)(m.h_inc_off[br.I1] - m.h_inc_off[br.I0]) + (br.I1 - br.I0);
  }
  std::vector<int32_t> order(b->h_ranges.size());
  for (size_t r = 0; r < order.size(); ++r) order[r] = (int32_t)r;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return work[x] > work[y]; });
  if (hipSetDevice(b->device) != hipSuccess) return TLFEA_ERR_HIP;
  int rc;
  if ((rc = upload(b->d_tiles, b->tiles_cap, items)) || (rc = upload(b->d_range_order, b->order_cap, order)))
    return rc;
  if (!b->d_counters && hipMalloc(&b->d_counters, 2 * sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    return TLFEA_ERR_NOMEM;
  }
  int cus = 0, per_tile = 1, per_range = 1;
  TLFEA_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  if ((rc = tlfea::batch_lpt_occupancy(tile_elems, b->tune.waves, b->lds + b->inc_cap, &per_tile, &per_range)))
    return rc;
  tlfea::BatchSchedule& sc = b->sched;
  sc.persistent = 1;
  sc.tile_elems = tile_elems;
  sc.tiles = b->d_tiles;
  sc.n_tiles = (int)items.size();
  sc.range_order = b->d_range_order;
  sc.counters = b->d_counters;
  sc.grid_tiles = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_tile, sc.n_tiles));
  sc.grid_ranges = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_range, b->n_ranges));
  drop_graph(b);
  return TLFEA_OK;
}

static int batch_set_schedule(tlfea_batch_s* b, int persistent, int tile_elems) {
  if (!persistent) {
    b->sched = tlfea::BatchSchedule{};
    drop_graph(b);
    return TLFEA_OK;
  }
  return batch_plan_lpt(b, tile_elems);
}

// Cut every body's nodes into ranges for launch shape t and upload the
// concatenated list (the bodies' own cuts are left alone).
static int batch_set_shape(tlfea_batch_s* b, const tlfea::GatherTuning& t) {
  if (t.waves < 1 || t.waves > 8 || t.range_tasks < 1 || t.range_values < 1) return TLFEA_ERR_INVALID;
  std::vector<BatchRange> ranges;
  int64_t max_vals = 0;
  int inc_cap = 0;
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    const tlfea::Mesh& m = b->meshes[i]->m;
    const tlfea::RangePlan p = tlfea::plan_ranges(m.h_inc_off, m.h_adj_off, m.mc, t);
    if (!tlfea::plan_fits(p)) return TLFEA_ERR_UNSUPPORTED;
    for (size_t r = 0; r + 1 < p.ranges.size(); ++r)
      ranges.push_back(BatchRange{(int)i, p.ranges[r], p.ranges[r + 1]});
    max_vals = std::max(max_vals, p.max_values);
    inc_cap = std::max(inc_cap, (int)((p.max_inc + 15) / 16 * 16));
  }
  if (ranges.size() > (size_t)INT32_MAX) return TLFEA_ERR_TOO_LARGE;
  if (hipSetDevice(b->device) != hipSuccess) return TLFEA_ERR_HIP;
  if (ranges.size() > b->ranges_cap || !b->d_ranges) {
    // queued launches may still read the old list
    if (b->d_ranges && hipDeviceSynchronize() != hipSuccess) return TLFEA_ERR_HIP;
    BatchRange* d = nullptr;
    const size_t cap = ranges.empty() ? 1 : ranges.size();
    if (hipMalloc(&d, sizeof(BatchRange) * cap) != hipSuccess) {
      (void)hipGetLastError();
      return TLFEA_ERR_NOMEM;
    }
    (void)hipFree(b->d_ranges);
    b->d_ranges = d;
    b->ranges_cap = cap;
  } else if (hipDeviceSynchronize() != hipSuccess) {
    return TLFEA_ERR_HIP;
  }
  if (!ranges.empty() &&
      hipMemcpy(b->d_ranges, ranges.data(), sizeof(BatchRange) * ranges.size(), hipMemcpyHostToDevice) != hipSuccess)
    return TLFEA_ERR_HIP;
  b->n_ranges = (int)ranges.size();
  b->lds = sizeof(double) * (size_t)max_vals;
  b->inc_cap = inc_cap;
  b->tune = t;
  b->h_ranges = std::move(ranges);
  drop_graph(b);  // the captured launches hold the old grid and LDS size
  return b->sched.persistent ? batch_plan_lpt(b, b->sched.tile_elems) : TLFEA_OK;
}

// Tuned choices of the autotuner, per batch signature, for the life of the process.
struct TunedChoice {
  tlfea::GatherTuning shape;
  int persistent = 0, tile_elems = 25;
};
static std::mutex g_tuned_mu;
static std::map<uint64_t, TunedChoice> g_tuned;

static uint64_t batch_signature(const tlfea_batch_s* b) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the sizes that decide the launches
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)b->elem_type);
  mix((uint64_t)b->gl0);
  mix((uint64_t)b->precision);
  mix((uint64_t)b->meshes.size());
  for (const tlfea_mesh_t mh : b->meshes) {
    mix((uint64_t)mh->m.n_elem);
    mix((uint64_t)mh->m.n_pnodes);
  }
  return h;
}

TLFEA_API int tlfea_batch_create(const tlfea_mesh_t* meshes, int32_t n_bodies, tlfea_batch_t* out) {
  if (!out) return TLFEA_ERR_INVALID;
  *out = nullptr;
  if (!meshes || n_bodies <= 0) return TLFEA_ERR_INVALID;
  for (int i = 0; i < n_bodies; ++i) {
    if (!meshes[i]) return TLFEA_ERR_INVALID;
    if (!meshes[i]->m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  }
  const tlfea::Mesh& m0 = meshes[0]->m;
  auto* b = new (std::nothrow) tlfea_batch_s;
  if (!b) return TLFEA_ERR_NOMEM;
  b->device = m0.device;
  b->elem_type = m0.elem_type;
  b->gl0 = m0.gl[0];
  b->precision = m0.precision;
  b->rows = 1;
  for (int i = 0; i < n_bodies; ++i)
    b->rows &= tlfea::use_rows(meshes[i]->m, true) ? 1 : 0;
  std::vector<BatchBody> bodies(n_bodies);
  b->dof_off.assign(n_bodies + 1, 0);
  b->nnz_off.assign(n_bodies + 1, 0);
  for (int i = 0; i < n_bodies; ++i) {
    const tlfea::Mesh& m = meshes[i]->m;
    if (m.elem_type != b->elem_type || m.gl[0] != b->gl0 || m.precision != b->precision || m.device != b->device) {
      delete b;
      return TLFEA_ERR_INVALID;
    }
    BatchBody& B = bodies[i];
    B.conn = m.d_conn;
    B.X = m.d_X;
    B.geo = m.d_geo;
    B.escale = m.d_escale;
    B.row_off = m.d_row_off;
    B.rank = m.d_rank;
    B.inc_off = m.d_inc_off;
    B.inc = m.d_inc;
    B.incpos = m.d_incpos;
    B.rank_inc = m.d_rank_inc;
    B.blk_inc_off = b->n_inc;
    B.rblock_off = b->n_rblocks;
    B.n_elem = m.n_elem;
    B.dof_off = b->dof_off[i];
    B.nnz_off = b->nnz_off[i];
    B.point_off = b->n_points;
    B.block_off = b->n_blocks;
    B.affine = m.affine ? 1 : 0;
    B.half_h = 0.5 * m.thickness;
    B.mp = m.mp;
    b->dof_off[i + 1] = b->dof_off[i] + m.n_dof;
    b->nnz_off[i + 1] = b->nnz_off[i] + m.nnz;
    b->n_points += m.n_elem * m.n_qp;
    b->n_blocks += (m.n_elem * m.n_qp + tlfea::kStageThreads - 1) / tlfea::kStageThreads;
    b->n_inc += m.n_elem * m.n_pn;
    const int reb = tlfea::row_elems_for(b->elem_type, b->gl0);
    b->n_rblocks += (m.n_elem + reb - 1) / reb;
    // pass 2 addresses a body's row blocks in 16-byte units with 32-bit offsets
    if (b->rows && b->elem_type == TLFEA_T10 &&
        m.n_elem * m.n_pn * (int64_t)(tlfea::row_block_bytes() / 16) >= ((int64_t)1 << 32)) {
      delete b;
      return TLFEA_ERR_TOO_LARGE;
    }
    // pass 2 addresses a body's records in 16-byte units with 32-bit offsets
    if (m.n_elem * m.n_qp * (int64_t)(tlfea::stage_record_bytes(b->precision) / 16) >= ((int64_t)1 << 32)) {
      delete b;
      return TLFEA_ERR_TOO_LARGE;
    }
    b->meshes.push_back(meshes[i]);
    b->generation.push_back(m.generation);
  }
  if (b->n_blocks > INT32_MAX || b->n_rblocks > INT32_MAX) { delete b; return TLFEA_ERR_TOO_LARGE; }
  const size_t stage = b->rows ? (size_t)b->n_inc * tlfea::row_block_bytes_for(b->elem_type, b->gl0)
                               : (size_t)b->n_points * tlfea::stage_record_bytes(b->precision);
  if (hipSetDevice(b->device) != hipSuccess) { delete b; return TLFEA_ERR_HIP; }
  if (hipMalloc(&b->d_bodies, sizeof(BatchBody) * bodies.size()) != hipSuccess ||
      hipMalloc(&b->d_stage, stage > 0 ? stage : 1) != hipSuccess ||
      hipMalloc(&b->d_flags, sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    batch_free(b);
    return TLFEA_ERR_NOMEM;
  }
  if (hipMemcpy(b->d_bodies, bodies.data(), sizeof(BatchBody) * bodies.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->d_flags, 0, sizeof(uint32_t)) != hipSuccess) {
    batch_free(b);
    return TLFEA_ERR_HIP;
  }
  b->signature = batch_signature(b);
  TunedChoice choice;
  bool tuned = false;
  {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    auto it = g_tuned.find(b->signature);
    if (it != g_tuned.end()) {
      choice = it->second;
      tuned = true;
    }
  }
  int rc = batch_set_shape(b, tuned ? choice.shape : m0.tune);
  if (!rc && tuned && choice.persistent) rc = batch_set_schedule(b, 1, choice.tile_elems);
  if (rc) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return TLFEA_OK;
}

TLFEA_API int tlfea_batch_destroy(tlfea_batch_t batch) {
  if (!batch) return TLFEA_OK;
  (void)hipSetDevice(batch->device);
  (void)hipDeviceSynchronize();
  batch_free(batch);
  return TLFEA_OK;
}

TLFEA_API int tlfea_batch_offsets(tlfea_batch_t batch, int64_t* dof_off, int64_t* nnz_off) {
  if (!batch) return TLFEA_ERR_INVALID;
  if (dof_off) std::copy(batch->dof_off.begin(), batch->dof_off.end(), dof_off);
  if (nnz_off) std::copy(batch->nnz_off.begin(), batch->nnz_off.end(), nnz_off);
  return TLFEA_OK;
}

// The batch holds copies of its members' device pointers, materials and
// precision: any later change to a member makes it stale.
static bool batch_current(tlfea_batch_t b) {
  for (size_t i = 0; i < b->meshes.size(); ++i)
    if (b->meshes[i]->m.generation != b->generation[i]) return false;
  return true;
}

static BatchArgs batch_args(tlfea_batch_t b, const double* d_q, const double* d_qdot, const double* d_h,
                            double* d_f, double* d_vals) {
  BatchArgs a{};
  a.bodies = b->d_bodies;
  a.ranges = b->d_ranges;
  a.n_bodies = (int)b->meshes.size();
  a.n_points = b->n_points;
  a.n_blocks = b->n_blocks;
  a.n_rblocks = b->n_rblocks;
  a.rows = b->rows;
  a.inc_cap = b->inc_cap;
  a.stage = b->d_stage;
  a.q = d_q;
  a.qdot = d_qdot;
  a.h = d_h;
  a.f = d_f;
  a.vals = d_vals;
  a.flags = b->d_flags;
  return a;
}

static int batch_enqueue(tlfea_batch_t b, const BatchArgs& a, hipStream_t s) {
  return tlfea::launch_batch(b->elem_type, b->gl0, b->precision, b->tune, a, b->n_ranges, b->lds, s, b->sched);
}

TLFEA_API int tlfea_batch_assemble(tlfea_batch_t b, const double* d_q, const double* d_qdot, const double* d_h,
                                   double* d_f, double* d_vals, void* stream) {
  if (!b || !d_q || !d_h || !d_f || !d_vals) return TLFEA_ERR_INVALID;
  if (!batch_current(b)) return TLFEA_ERR_INVALID;
  if (hipSetDevice(b->device) != hipSuccess) return TLFEA_ERR_HIP;
  const BatchArgs a = batch_args(b, d_q, d_qdot, d_h, d_f, d_vals);
  auto s = (hipStream_t)stream;
  if (!s) return batch_enqueue(b, a, s);  // the legacy stream cannot be captured
  const void* key[6] = {d_q, d_qdot, d_h, d_f, d_vals, stream};
  if (!b->exec || !std::equal(key, key + 6, b->key)) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    TLFEA_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = batch_enqueue(b, a, s);
    hipGraph_t g = nullptr;
    hipError_t e1 = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    TLFEA_HIP_CHECK(e1);
    hipError_t e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      b->exec = nullptr;
      (void)hipGetLastError();
      return TLFEA_ERR_HIP;
    }
    std::copy(key, key + 6, b->key);
  }
  TLFEA_HIP_CHECK(hipGraphLaunch(b->exec, s));
  return TLFEA_OK;
}

TLFEA_API int tlfea_batch_assemble_loop(tlfea_batch_t b, const double* d_q, const double* d_qdot,
                                        const double* d_h, double* d_f, double* d_vals, void* stream) {
  if (!b || !d_q || !d_h || !d_f || !d_vals) return TLFEA_ERR_INVALID;
  if (!batch_current(b)) return TLFEA_ERR_INVALID;
  if (hipSetDevice(b->device) != hipSuccess) return TLFEA_ERR_HIP;
  const size_t n = b->meshes.size();
  std::vector<double> h(n);
  auto s = (hipStream_t)stream;
  TLFEA_HIP_CHECK(hipMemcpyAsync(h.data(), d_h, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  TLFEA_HIP_CHECK(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i) {
    int rc = tlfea_assemble_ex(b->meshes[i], d_q + b->dof_off[i], d_qdot ? d_qdot + b->dof_off[i] : nullptr, h[i],
                               1.0, d_f + b->dof_off[i], d_vals + b->nnz_off[i], stream);
    if (rc) return rc;
  }
  return TLFEA_OK;
}

TLFEA_API int tlfea_batch_set_gather_shape(tlfea_batch_t b, const tlfea_gather_shape* shape) {
  if (!b || !shape) return TLFEA_ERR_INVALID;
  if (!batch_current(b)) return TLFEA_ERR_INVALID;
  return batch_set_shape(b, tlfea::GatherTuning{shape->waves, shape->range_tasks, shape->range_values});
}

TLFEA_API int tlfea_batch_get_gather_shape(tlfea_batch_t b, tlfea_gather_shape* shape, int64_t* n_ranges) {
  if (!b || (!shape && !n_ranges)) return TLFEA_ERR_INVALID;
  if (shape) {
    shape->waves = b->tune.waves;
    shape->range_tasks = b->tune.range_tasks;
    shape->range_values = b->tune.range_values;
  }
  if (n_ranges) *n_ranges = b->n_ranges;
  return TLFEA_OK;
}

TLFEA_API int tlfea_batch_set_schedule(tlfea_batch_t b, int32_t persistent, int32_t tile_elems) {
  if (!b || (persistent != 0 && persistent != 1)) return TLFEA_ERR_INVALID;
  if (!batch_current(b)) return TLFEA_ERR_INVALID;
  if (persistent && !(b->rows && b->elem_type == TLFEA_T10)) return TLFEA_ERR_UNSUPPORTED;
  if (hipSetDevice(b->device) != hipSuccess) return TLFEA_ERR_HIP;
  return batch_set_schedule(b, persistent, tile_elems);
}

TLFEA_API int tlfea_batch_get_schedule(tlfea_batch_t b, int32_t* persistent, int32_t* tile_elems,
                                       int32_t* grid_tiles, int32_t* grid_ranges) {
  if (!b) return TLFEA_ERR_INVALID;
  const tlfea::BatchSchedule& sc = b->sched;
  if (persistent) *persistent = sc.persistent;
  if (tile_elems) *tile_elems = sc.persistent ? sc.tile_elems : tlfea::row_elems_for(b->elem_type, b->gl0);
  if (grid_tiles) *grid_tiles = sc.persistent ? sc.grid_tiles : (int32_t)b->n_rblocks;
  if (grid_ranges) *grid_ranges = sc.persistent ? sc.grid_ranges : b->n_ranges;
  return TLFEA_OK;
}

TLFEA_API int tlfea_batch_autotune(tlfea_batch_t b, const double* d_q, const double* d_qdot, const double* d_h,
                                   double* d_f, double* d_vals, int32_t reps, void* stream,
                                   tlfea_gather_shape* chosen, float* ms_per_call) {
  if (!b || !d_q || !d_h || !d_f || !d_vals) return TLFEA_ERR_INVALID;
  if (!batch_current(b)) return TLFEA_ERR_INVALID;
  if (hipSetDevice(b->device) != hipSuccess) return TLFEA_ERR_HIP;
  const auto s = (hipStream_t)stream;
  // schedules: one workgroup per item; on the element-row path also the
  // persistent LPT form with tiles of 25 and of 16 elements
  struct Cand {
    int persistent, tile_elems;
  };
  std::vector<Cand> cands{{0, tlfea::row_elems()}};
  if (b->rows && b->elem_type == TLFEA_T10) {
    cands.push_back({1, tlfea::row_elems()});
    cands.push_back({1, 16});
  }
  const Cand cur{b->sched.persistent, b->sched.persistent ? b->sched.tile_elems : tlfea::row_elems()};
  const tlfea::GatherTuning cur_shape = b->tune;
  TunedChoice best, at_cur;
  float best_ms = -1.0f, cur_ms = -1.0f;
  for (const Cand& c : cands) {
    int rc = batch_set_shape(b, cur_shape);
    if (!rc) rc = batch_set_schedule(b, c.persistent, c.tile_elems);
    if (rc == TLFEA_ERR_UNSUPPORTED) continue;
    if (rc) return rc;
    tlfea::GatherTuning shape = cur_shape;
    float ms = 0.0f;
    // the launch pair itself, uncaptured: shapes change between the timings
    rc = tlfea::autotune_shape(
        cur_shape, [&](const tlfea::GatherTuning& t) { return batch_set_shape(b, t); },
        [&]() { return batch_enqueue(b, batch_args(b, d_q, d_qdot, d_h, d_f, d_vals), s); }, reps, s, shape, ms);
    if (rc == TLFEA_ERR_UNSUPPORTED) continue;
    if (rc) return rc;
    if (c.persistent == cur.persistent && c.tile_elems == cur.tile_elems) {
      cur_ms = ms;
      at_cur.shape = shape;
      at_cur.persistent = c.persistent;
      at_cur.tile_elems = c.tile_elems;
    }
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best.shape = shape;
      best.persistent = c.persistent;
      best.tile_elems = c.tile_elems;
    }
  }
  if (best_ms < 0.0f) return TLFEA_ERR_UNSUPPORTED;
  if (cur_ms >= 0.0f && best_ms > (1.0f - tlfea::kTuneMargin) * cur_ms) {
    best = at_cur;  // a schedule change must pay for itself
    best_ms = cur_ms;
  }
  int rc = batch_set_shape(b, best.shape);
  if (!rc) rc = batch_set_schedule(b, best.persistent, best.tile_elems);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    g_tuned[b->signature] = best;
  }
  if (chosen) {
    chosen->waves = best.shape.waves;
    chosen->range_tasks = best.shape.range_tasks;
    chosen->range_values = best.shape.range_values;
  }
  if (ms_per_call) *ms_per_call = best_ms;
  return TLFEA_OK;
}
