// plas_batch.cpp -- the batch engine of libplas.so (include/plas_batch.h):
// many sorts advanced together, one launch of each kernel kind per reorder
// covering every running sort, with optional HIP graph replay of whole
// chunks of reorders and a measured table of launch shapes.
//
// Each sort owns one device allocation (its three grids, permutation,
// grouping table, inverse counts, level table, trace and state) and a
// slot in the batch's descriptor array. Whenever the set of running sorts
// changes, the host rebuilds the launch plan -- the descriptors, the list of
// running slots and one block map per launch -- and uploads it in one copy.
// A chunk of reorders is then a fixed launch sequence: with graph replay it
// is captured once per plan and replayed until the next change. Between
// chunks the host reads (done, k) of every running sort.
#include "plas_batch.h"

#include <array>

#include "plas_host.h"

using namespace plas_host;

namespace {

constexpr int kDefaultWavesPerBlock = 2;  // as plas_sort
// Assignment blocks per sort when the tuning table names none (as a lone
// sort's launch).
constexpr int kBatchAssignBlocks = 4096;
constexpr int kMaxSlots = 1 << 16;     // grid index field of a block map entry
constexpr int kMaxLocalBlocks = 1 << 16;  // block index field

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

enum LaunchKind { kBlur = 1, kAssign = 2 };

// Byte offsets of one sort's buffers in its allocation.
struct SortLayout {
  size_t g, h, t, p, table, inv, levels, trace, state, bytes;
};

SortLayout sort_layout(int32_t w, int dp, int32_t storage, size_t nlevels, int64_t max_cells) {
  const size_t n = static_cast<size_t>(w) * w;
  const size_t grid_bytes = n * dp * storage_bytes(storage);
  SortLayout L{};
  size_t off = 0;
  L.g = off;
  off = align_up(off + grid_bytes);
  L.h = off;
  off = align_up(off + grid_bytes);
  L.t = off;
  off = align_up(off + grid_bytes);
  L.p = off;
  off = align_up(off + n * sizeof(int32_t));
  L.table = off;
  off = align_up(off + static_cast<size_t>(max_cells) * sizeof(int32_t));
  L.inv = off;
  off = align_up(off + static_cast<size_t>(w + 1) * sizeof(float));
  L.levels = off;
  off = align_up(off + nlevels * sizeof(LevelInfo));
  L.trace = off;
  off = align_up(off + nlevels * sizeof(plas_level_out));
  L.state = off;
  off = align_up(off + sizeof(DevState));
  L.bytes = off;
  return L;
}

struct Launch {
  int kind;
  int dp;
  int storage;
  int wpb;
  int large;       // blur: the running grids are a large working set (plas::blur_large_working_set)
  size_t map_off;  // byte offset of the block map in the plan
  int blocks;
};

// One sort of a batch.
struct Sort {
  plas_batch_item item{};
  int32_t w = 0, d = 0, dp = 0, storage = 0, s = 0;
  int64_t n = 0;
  std::vector<LevelInfo> levels;
  int64_t max_cells = 0, max_items = 0;
  DeviceBuffer mem;
  plas::BatchGrid grid{};
  int wpb = kDefaultWavesPerBlock;
  int assign_cap = 0;
  int slot = -1;
  bool running = false;
  int64_t slots = 0;  // reorder slots queued while running
  int64_t max_k = 0;
  double done_ms = 0.0;
  double submit_ms = 0.0;  // stats->total_ms counts from here
  int64_t tag = 0;  // caller's identifier (the server's job id)
  int64_t footprint = 0;
};

// Lines per block of a sort's blur launches (0 for the register kernel,
// which has one fixed shape).
int blur_wpb(const Sort& s) { return plas::staged_blur(s.dp, s.storage) ? s.wpb : 0; }

}  // namespace

struct plas_batch_state {
  hipStream_t stream = nullptr;  // the batch's own stream (capture needs a created stream)
  DeviceBuffer plan;             // descriptors | running list | block maps
  DeviceBuffer status;           // HostStatus per running sort
  void* plan_host = nullptr;     // pinned staging of the plan
  size_t plan_host_bytes = 0;
  void* status_host = nullptr;   // pinned HostStatus per running sort
  size_t status_host_bytes = 0;
  std::vector<hipEvent_t> events;
};

namespace {

void destroy_batch_state(plas_batch_state* b) {
  if (b == nullptr) return;
  if (b->stream != nullptr) (void)hipStreamSynchronize(b->stream);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  release(b->plan);
  release(b->status);
  if (b->plan_host != nullptr) (void)hipHostFree(b->plan_host);
  if (b->status_host != nullptr) (void)hipHostFree(b->status_host);
  if (b->stream != nullptr) (void)hipStreamDestroy(b->stream);
  delete b;
}

int32_t create_batch_state(plas_context* h, plas_batch_state** out) {
  plas_batch_state* b = new (std::nothrow) plas_batch_state();
  if (b == nullptr) return fail(h, PLAS_ERR_OUT_OF_MEMORY, "batch state");
  // Default priority (no priority argument).
  const hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(h, e, "hipStreamCreateWithFlags");
  }
  *out = b;
  return PLAS_OK;
}

int32_t ensure_batch_state(plas_context* h) {
  if (h->batch != nullptr) return PLAS_OK;
  return create_batch_state(h, &h->batch);
}

hipError_t reserve_pinned(void** p, size_t* cap, size_t bytes) {
  if (*p != nullptr && *cap >= bytes) return hipSuccess;
  if (*p != nullptr) {
    hipError_t e = hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipHostMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  *cap = bytes;
  return hipSuccess;
}

// Runs the library's helpers (which use h->stream) on another stream.
class StreamSwap {
 public:
  StreamSwap(plas_context* h, hipStream_t s) : h_(h), saved_(h->stream) { h->stream = s; }
  ~StreamSwap() { h_->stream = saved_; }

 private:
  plas_context* h_;
  hipStream_t saved_;
};

}  // namespace

void release_batch_state(plas_context* h) {
  if (h == nullptr || h->batch == nullptr) return;
  destroy_batch_state(h->batch);
  h->batch = nullptr;
}

// A batch in progress: sorts join (add), chunks of reorders run (chunk), and
// finished sorts are collected with their results written out.
class BatchRun {
 public:
  BatchRun(plas_context* h, plas_batch_state* b, const plas_sort_params& prm, const plas_batch_config& cfg,
           std::chrono::steady_clock::time_point t0)
      : h_(h), b_(b), prm_(prm), cfg_(cfg), t0_(t0) {
    chunk_ = cfg.reorders_per_sync > 0 ? cfg.reorders_per_sync : plas_host::kDefaultReordersPerSync;
    graph_ = cfg.graph != 0 && cfg.profile == 0;
    // Blur passes per axis (PLAS_FILTER_BOX3: three), through H and T in
    // turn, the last column pass writing T (as plas_sort does).
    const int passes = prm.filter == PLAS_FILTER_BOX3 ? 3 : 1;
    int src = 0;  // G
    for (int p = 0; p < passes; ++p) {
      const int dst = 1 + (p & 1);
      routes_.push_back(plas::blur_route(0, src, dst, p == 0));
      src = dst;
    }
    for (int p = 0; p < passes; ++p) {
      const int dst = p == passes - 1 ? 2 : 1 + ((passes + p) & 1);
      routes_.push_back(plas::blur_route(1, src, dst, 0));
      src = dst;
    }
  }
  ~BatchRun() {
    drop_graph();
    for (Sort& s : sorts_) release(s.mem);
  }

  int64_t graph_builds = 0, chunks = 0, slots = 0, launches = 0;
  double step_ms = 0.0, blur_ms = 0.0, assign_ms = 0.0;

  int running() const {
    int c = 0;
    for (const Sort& s : sorts_) c += s.running ? 1 : 0;
    return c;
  }

  // Validate, allocate and prepare one sort; it joins at the next chunk.
  int32_t add(const plas_batch_item& it, int64_t tag, double submit_ms = 0.0) {
    int32_t st = check_features(h_, it.features, it.n, it.d, it.side, it.layout, it.dtype);
    if (st != PLAS_OK) return st;
    if (it.perm_out == nullptr) return fail(h_, PLAS_ERR_INVALID_ARGUMENT, "item perm_out is NULL");
    if (!valid_storage(it.storage)) return fail(h_, PLAS_ERR_INVALID_ARGUMENT, "item storage is unknown");
    if (it.stats != nullptr && it.stats->struct_size != sizeof(plas_sort_stats))
      return fail(h_, PLAS_ERR_INVALID_ARGUMENT, "item stats->struct_size does not match this library");
    int slot = -1;
    for (size_t i = 0; i < sorts_.size(); ++i)
      if (!sorts_[i].running && sorts_[i].mem.ptr == nullptr) {
        slot = static_cast<int>(i);
        break;
      }
    if (slot < 0) {
      if (sorts_.size() >= static_cast<size_t>(kMaxSlots))
        return fail(h_, PLAS_ERR_INVALID_ARGUMENT, "too many sorts in one batch");
      sorts_.emplace_back();
      slot = static_cast<int>(sorts_.size() - 1);
    }
    Sort& s = sorts_[slot];
    s = Sort();
    s.slot = slot;
    s.tag = tag;
    s.submit_ms = submit_ms;
    s.item = it;
    s.w = it.side;
    s.d = it.d;
    s.n = it.n;
    s.dp = padded_channels(it.d);
    s.storage = it.storage;
    st = build_schedule(s.w, prm_.radius_decay, prm_.min_block, prm_.start_radius, &s.levels);
    if (st != PLAS_OK) return fail(h_, st, "bad schedule parameters");
    for (const LevelInfo& lv : s.levels) {
      s.max_cells = std::max<int64_t>(s.max_cells, static_cast<int64_t>(lv.beta) * lv.beta);
      s.max_items = std::max<int64_t>(s.max_items, lv.groups + lv.singles);
    }
    s.max_k = reorder_bound(s.levels.size(), prm_.inv_threshold);
    st = apply_tuning(s);
    if (st != PLAS_OK) return st;

    // One allocation for all of the sort's buffers.
    const SortLayout lay = sort_layout(s.w, s.dp, s.storage, s.levels.size(), s.max_cells);
    const size_t nl = s.levels.size();
    const size_t o_g = lay.g, o_h = lay.h, o_t = lay.t, o_p = lay.p, o_table = lay.table, o_inv = lay.inv,
                 o_levels = lay.levels, o_trace = lay.trace, o_state = lay.state;
    s.footprint = static_cast<int64_t>(lay.bytes);
    PLAS_HIP(h_, reserve(s.mem, lay.bytes));
    char* base = static_cast<char*>(s.mem.ptr);
    plas::BatchGrid& g = s.grid;
    g.G = base + o_g;
    g.H = base + o_h;
    g.T = base + o_t;
    g.P = reinterpret_cast<int32_t*>(base + o_p);
    g.table = reinterpret_cast<int32_t*>(base + o_table);
    g.inv = reinterpret_cast<const float*>(base + o_inv);
    g.levels = reinterpret_cast<const LevelInfo*>(base + o_levels);
    g.trace = reinterpret_cast<plas_level_out*>(base + o_trace);
    g.state = reinterpret_cast<DevState*>(base + o_state);
    g.w = s.w;
    g.blur_blocks = plas::batch_blur_blocks(s.w, s.dp, s.storage, s.wpb, s.max_cells);
    g.assign_blocks = plas::batch_assign_blocks(s.max_items, s.dp, s.storage,
                                                s.assign_cap > 0 ? s.assign_cap : kBatchAssignBlocks);

    // Features -> X in T, the start arrangement, G = X[P] (as plas_sort).
    hipStream_t stream = b_->stream;
    st = ingest_features(h_, it.features, it.dtype, s.n, s.d, it.layout, s.dp, s.storage, g.T, &s.s);
    if (st != PLAS_OK) return finish_failed(s, st);
    if (it.init_perm != nullptr) {
      st = check_permutation(h_, it.init_perm, s.n, static_cast<int32_t*>(g.H));
      if (st != PLAS_OK) return finish_failed(s, st);
      PLAS_HIP(h_, hipMemcpyAsync(g.P, it.init_perm, static_cast<size_t>(s.n) * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, stream));
    } else {
      const plas::Words4 k0 = plas::draw(it.seed, plas::kDrawStart, 0);
      PLAS_HIP(h_, plas::launch_start_perm(g.P, s.n, k0.v, stream));
    }
    PLAS_HIP(h_, plas::launch_gather(g.T, g.P, g.G, s.n, s.dp, s.storage, stream));
    const std::vector<float> inv = inverse_counts(s.w);
    PLAS_HIP(h_, hipMemcpyAsync(base + o_inv, inv.data(), inv.size() * sizeof(float), hipMemcpyHostToDevice,
                                stream));
    PLAS_HIP(h_, hipMemcpyAsync(base + o_levels, s.levels.data(), nl * sizeof(LevelInfo), hipMemcpyHostToDevice,
                                stream));
    PLAS_HIP(h_, hipMemsetAsync(base + o_trace, 0, nl * sizeof(plas_level_out), stream));
    DevState* S = h_->state_host;
    plas_sort_params prm = prm_;
    init_sort_state(S, s.w, s.s, s.levels, prm, it.seed);
    PLAS_HIP(h_, hipMemcpyAsync(g.state, S, sizeof(DevState), hipMemcpyHostToDevice, stream));
    // The host sources above are freed or reused at return.
    PLAS_HIP(h_, hipStreamSynchronize(stream));
    s.running = true;
    dirty_ = true;
    return PLAS_OK;
  }

  // Queue one chunk of reorders for every running sort and read their
  // status. Finished sorts are written out and leave the batch.
  int32_t chunk() {
    if (running() == 0) return PLAS_OK;
    if (dirty_) {
      int32_t st = rebuild();
      if (st != PLAS_OK) return st;
    }
    hipStream_t stream = b_->stream;
    const plas::BatchGrid* grids = static_cast<const plas::BatchGrid*>(b_->plan.ptr);
    if (graph_) {
      if (exec_ == nullptr) {
        PLAS_HIP(h_, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        const int32_t st = enqueue_reorders(false);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(stream, &graph);
        if (st != PLAS_OK) {
          if (graph != nullptr) (void)hipGraphDestroy(graph);
          return st;
        }
        if (e != hipSuccess) return hip_fail(h_, e, "hipStreamEndCapture");
        graph_obj_ = graph;
        PLAS_HIP(h_, hipGraphInstantiate(&exec_, graph_obj_, nullptr, nullptr, 0));
        ++graph_builds;
      }
      PLAS_HIP(h_, hipGraphLaunch(exec_, stream));
      launches += launches_per_chunk_;
    } else {
      const int32_t st = enqueue_reorders(cfg_.profile != 0);
      if (st != PLAS_OK) return st;
      launches += launches_per_chunk_;
    }
    ++chunks;
    slots += chunk_;
    const int nrun = static_cast<int>(run_list_.size());
    PLAS_HIP(h_, plas::launch_batch_status(grids, list_dev_, nrun, static_cast<HostStatus*>(b_->status.ptr),
                                           stream));
    PLAS_HIP(h_, hipMemcpyAsync(b_->status_host, b_->status.ptr, nrun * sizeof(HostStatus), hipMemcpyDeviceToHost,
                                stream));
    const HostStatus* status = static_cast<const HostStatus*>(b_->status_host);
    PLAS_HIP(h_, hipStreamSynchronize(stream));
    if (cfg_.profile) {
      for (int i = 0; i < chunk_; ++i) {
        float b = 0.0f, c = 0.0f;
        PLAS_HIP(h_, hipEventElapsedTime(&b, b_->events[3 * i + 0], b_->events[3 * i + 1]));
        PLAS_HIP(h_, hipEventElapsedTime(&c, b_->events[3 * i + 1], b_->events[3 * i + 2]));
        blur_ms += b;
        assign_ms += c;
      }
    }
    const double now = ms_since(t0_);
    for (int i = 0; i < nrun; ++i) {
      Sort& s = sorts_[run_list_[i]];
      s.slots += chunk_;
      const HostStatus hs = status[i];
      if (hs.done) {
        s.done_ms = now;
        const int32_t st = finish(s);
        if (st != PLAS_OK) return st;
        finished_.push_back(s.tag);
        continue;
      }
      // Every queued slot has run and been controlled by now.
      if (hs.k != s.slots || hs.k > s.max_k)
        return fail(h_, PLAS_ERR_HIP, "device controller made no progress");
    }
    return PLAS_OK;
  }

  // Tags of the sorts finished since the last call.
  std::vector<int64_t> take_finished() {
    std::vector<int64_t> out;
    out.swap(finished_);
    return out;
  }

  void drop_graph() {
    if (exec_ != nullptr) (void)hipGraphExecDestroy(exec_);
    if (graph_obj_ != nullptr) (void)hipGraphDestroy(graph_obj_);
    exec_ = nullptr;
    graph_obj_ = nullptr;
  }

 private:
  int32_t apply_tuning(Sort& s) {
    s.wpb = kDefaultWavesPerBlock;
    s.assign_cap = 0;
    for (int32_t i = 0; i < cfg_.tune_count; ++i) {
      const plas_tune_entry& e = cfg_.tune[i];
      if (s.w < e.side_lo || s.w > e.side_hi) continue;
      if (e.blur_waves_per_block != 0) s.wpb = e.blur_waves_per_block;
      s.assign_cap = e.assign_blocks;
      break;
    }
    if (s.wpb != 1 && s.wpb != 2 && s.wpb != 4)
      return fail(h_, PLAS_ERR_INVALID_ARGUMENT, "tune blur_waves_per_block must be 0, 1, 2 or 4");
    if (s.assign_cap < 0 || s.assign_cap >= kMaxLocalBlocks)
      return fail(h_, PLAS_ERR_INVALID_ARGUMENT, "tune assign_blocks must be in [0, 65535]");
    return PLAS_OK;
  }

  int32_t finish_failed(Sort& s, int32_t st) {
    release(s.mem);
    return st;
  }

  // Write a finished sort's permutation and stats and free its memory.
  int32_t finish(Sort& s) {
    hipStream_t stream = b_->stream;
    const DevState* Sd = s.grid.state;
    PLAS_HIP(h_, hipMemcpyAsync(s.item.perm_out, s.grid.P, static_cast<size_t>(s.n) * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, stream));
    DevState* S = h_->state_host;
    PLAS_HIP(h_, hipMemcpyAsync(S, Sd, sizeof(DevState), hipMemcpyDeviceToHost, stream));
    PLAS_HIP(h_, hipStreamSynchronize(stream));
    plas_sort_stats* stats = s.item.stats;
    if (stats != nullptr) {
      stats->levels = S->levels_run;
      stats->reorders = S->k;
      stats->energy_fixed = S->energy_last;
      stats->scale_shift = s.s;
      stats->energy = std::ldexp(static_cast<double>(S->energy_last), -s.s) / static_cast<double>(s.n);
      stats->trace_len = 0;
      if (stats->trace != nullptr && stats->trace_cap > 0) {
        const int32_t len = std::min(stats->trace_cap, S->levels_run);
        if (len > 0) {
          PLAS_HIP(h_, hipMemcpyAsync(stats->trace, s.grid.trace, static_cast<size_t>(len) * sizeof(plas_level_out),
                                      hipMemcpyDeviceToHost, stream));
          PLAS_HIP(h_, hipStreamSynchronize(stream));
        }
        stats->trace_len = len;
      }
      stats->blur_ms = 0.0;
      stats->blur_launches = 0;
      stats->assign_ms = 0.0;
      stats->assign_launches = 0;
      stats->total_ms = s.done_ms - s.submit_ms;
      if (stats->checkpoint != nullptr)
        fill_checkpoint(*S, static_cast<int32_t>(s.levels.size()), stats->checkpoint);
    }
    s.running = false;
    release(s.mem);
    dirty_ = true;
    return PLAS_OK;
  }

  // Descriptors of all slots, the running list and one block map per launch.
  int32_t rebuild() {
    drop_graph();
    run_list_.clear();
    for (const Sort& s : sorts_)
      if (s.running) run_list_.push_back(s.slot);
    const size_t nslots = sorts_.size();
    size_t off = align_up(nslots * sizeof(plas::BatchGrid));
    const size_t o_list = off;
    off = align_up(off + run_list_.size() * sizeof(int32_t));
    launches_.clear();
    std::vector<std::vector<uint32_t>> maps;
    auto add_launch = [&](int kind, int dp, int storage, int wpb, int regs, const std::vector<int>& members) {
      std::vector<uint32_t> map;
      for (int slot : members) {
        const plas::BatchGrid& g = sorts_[slot].grid;
        const int nb = kind == kBlur ? g.blur_blocks : g.assign_blocks;
        for (int b = 0; b < nb; ++b) map.push_back((static_cast<uint32_t>(slot) << 16) | static_cast<uint32_t>(b));
      }
      if (map.empty()) return;
      Launch L{kind, dp, storage, wpb, regs, off, static_cast<int>(map.size())};
      off = align_up(off + map.size() * sizeof(uint32_t));
      launches_.push_back(L);
      maps.push_back(std::move(map));
    };
    // Blur launches per (dp, storage, lines per block); assignment per (dp,
    // storage). The working set is the bytes of all running grids, which the
    // passes of a reorder stream through together.
    int64_t working_bytes = 0;
    for (int slot : run_list_) {
      const Sort& s = sorts_[slot];
      working_bytes += s.n * s.dp * (s.storage == plas::kStorageBF16 ? 2 : 4);
    }
    const int large = plas::blur_large_working_set(working_bytes) ? 1 : 0;
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<std::array<int, 4>> keys;
      auto key_of = [&](const Sort& s) -> std::array<int, 4> {
        return {s.dp, s.storage, pass == 0 ? blur_wpb(s) : 0, pass == 0 ? large : 0};
      };
      for (int slot : run_list_) {
        const std::array<int, 4> k = key_of(sorts_[slot]);
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
      }
      for (const auto& k : keys) {
        std::vector<int> members;
        for (int slot : run_list_)
          if (key_of(sorts_[slot]) == k) members.push_back(slot);
        add_launch(pass == 0 ? kBlur : kAssign, k[0], k[1], k[2], k[3], members);
      }
    }
    const size_t bytes = off;
    PLAS_HIP(h_, reserve(b_->plan, bytes));
    PLAS_HIP(h_, reserve_pinned(&b_->plan_host, &b_->plan_host_bytes, bytes));
    char* hb = static_cast<char*>(b_->plan_host);
    std::memset(hb, 0, bytes);
    for (size_t i = 0; i < nslots; ++i)
      std::memcpy(hb + i * sizeof(plas::BatchGrid), &sorts_[i].grid, sizeof(plas::BatchGrid));
    std::memcpy(hb + o_list, run_list_.data(), run_list_.size() * sizeof(int32_t));
    for (size_t i = 0; i < launches_.size(); ++i)
      std::memcpy(hb + launches_[i].map_off, maps[i].data(), maps[i].size() * sizeof(uint32_t));
    PLAS_HIP(h_, hipMemcpyAsync(b_->plan.ptr, hb, bytes, hipMemcpyHostToDevice, b_->stream));
    list_dev_ = reinterpret_cast<const int32_t*>(static_cast<char*>(b_->plan.ptr) + o_list);
    const size_t status_bytes = std::max<size_t>(1, run_list_.size()) * sizeof(HostStatus);
    PLAS_HIP(h_, reserve(b_->status, status_bytes));
    PLAS_HIP(h_, reserve_pinned(&b_->status_host, &b_->status_host_bytes, status_bytes));
    // Reorder launches: step, blur rows (each blur launch), blur columns, assignments.
    int per_reorder = 0;
    for (const Launch& L : launches_) per_reorder += L.kind == kBlur ? static_cast<int>(routes_.size()) : 1;
    launches_per_chunk_ = static_cast<int64_t>(per_reorder) * chunk_;
    if (cfg_.profile) {
      while (b_->events.size() < static_cast<size_t>(3 * chunk_)) {
        hipEvent_t e;
        PLAS_HIP(h_, hipEventCreate(&e));
        b_->events.push_back(e);
      }
    }
    dirty_ = false;
    return PLAS_OK;
  }

  // chunk_ reorders: blur rows (then each sort's grouping table), blur
  // columns, assignment (then each sort's control step), each over all
  // running sorts.
  int32_t enqueue_reorders(bool timed) {
    hipStream_t stream = b_->stream;
    const char* plan = static_cast<const char*>(b_->plan.ptr);
    const plas::BatchGrid* grids = reinterpret_cast<const plas::BatchGrid*>(plan);
    auto map_of = [&](const Launch& L) { return reinterpret_cast<const uint32_t*>(plan + L.map_off); };
    for (int i = 0; i < chunk_; ++i) {
      if (timed) PLAS_HIP(h_, hipEventRecord(b_->events[3 * i + 0], stream));
      for (const int route : routes_)
        for (const Launch& L : launches_)
          if (L.kind == kBlur)
            PLAS_HIP(h_, plas::launch_blur_batch(grids, map_of(L), L.blocks, L.dp, L.storage, L.wpb == 0 ? 4 : L.wpb,
                                                 route, L.large, stream));
      if (timed) PLAS_HIP(h_, hipEventRecord(b_->events[3 * i + 1], stream));
      for (const Launch& L : launches_)
        if (L.kind == kAssign)
          PLAS_HIP(h_, plas::launch_assign_batch(grids, map_of(L), L.blocks, L.dp, L.storage, stream));
      if (timed) PLAS_HIP(h_, hipEventRecord(b_->events[3 * i + 2], stream));
    }
    return PLAS_OK;
  }

  plas_context* h_;
  plas_batch_state* b_;
  plas_sort_params prm_;
  plas_batch_config cfg_;
  std::chrono::steady_clock::time_point t0_;
  int chunk_ = 32;
  std::vector<int> routes_;  // blur passes of a reorder, in order
  bool graph_ = false;
  bool dirty_ = true;
  std::vector<Sort> sorts_;
  std::vector<int> run_list_;
  std::vector<Launch> launches_;
  const int32_t* list_dev_ = nullptr;
  int64_t launches_per_chunk_ = 0;
  hipGraph_t graph_obj_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  std::vector<int64_t> finished_;
};

namespace {

int32_t check_config(plas_context* h, const plas_batch_config* config, plas_batch_config* cfg) {
  plas_batch_config_init(cfg);
  if (config != nullptr) {
    if (config->struct_size != sizeof(plas_batch_config))
      return fail(h, PLAS_ERR_INVALID_ARGUMENT, "config->struct_size does not match this library");
    *cfg = *config;
  }
  if (cfg->reorders_per_sync < 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "reorders_per_sync must be >= 0");
  if (cfg->tune_count < 0 || (cfg->tune_count > 0 && cfg->tune == nullptr))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "tune_count > 0 needs a tune table");
  return PLAS_OK;
}

// The sorts of items as one batch, to the end.
int32_t run_batch(plas_context* h, const plas_batch_item* items, int32_t count, const plas_sort_params& prm,
                  const plas_batch_config& cfg, plas_batch_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  plas_batch_state* b = h->batch;
  // Work the caller queued before this call (e.g. producing the features)
  // comes first.
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  StreamSwap swap(h, b->stream);
  BatchRun run(h, b, prm, cfg, t0);
  for (int32_t i = 0; i < count; ++i) {
    const int32_t st = run.add(items[i], i);
    if (st != PLAS_OK) return st;
  }
  const double prepare_ms = ms_since(t0);
  while (run.running() > 0) {
    const int32_t st = run.chunk();
    if (st != PLAS_OK) return st;
  }
  if (stats != nullptr) {
    stats->sorts = count;
    stats->chunks = run.chunks;
    stats->reorder_slots = run.slots;
    stats->graph_builds = run.graph_builds;
    stats->launches = run.launches;
    stats->prepare_ms = prepare_ms;
    stats->total_ms = ms_since(t0);
    stats->loop_ms = stats->total_ms - prepare_ms;
    stats->step_ms = run.step_ms;
    stats->blur_ms = run.blur_ms;
    stats->assign_ms = run.assign_ms;
  }
  return PLAS_OK;
}

int side_bucket(int32_t side) { return static_cast<int>(std::floor(2.0 * std::log2(static_cast<double>(side)))); }

}  // namespace

extern "C" {

int32_t plas_batch_config_init(plas_batch_config* c) {
  if (c == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  std::memset(c, 0, sizeof(*c));
  c->struct_size = sizeof(plas_batch_config);
  return PLAS_OK;
}

int32_t plas_sort_batch(plas_handle h, const plas_batch_item* items, int32_t count, const plas_sort_params* params,
                        const plas_batch_config* config, plas_batch_stats* stats) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  h->error.clear();
  if (count < 0 || (count > 0 && items == nullptr))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "items is NULL or count < 0");
  if (count >= kMaxSlots) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "too many sorts in one batch");
  if (stats != nullptr && stats->struct_size != sizeof(plas_batch_stats))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "stats->struct_size does not match this library");
  plas_sort_params prm;
  int32_t st = check_params(h, params, &prm);
  if (st == PLAS_OK && prm.resume != nullptr)
    st = fail(h, PLAS_ERR_INVALID_ARGUMENT, "batched sorts start from their items");
  if (st != PLAS_OK) return st;
  plas_batch_config cfg;
  st = check_config(h, config, &cfg);
  if (st != PLAS_OK) return st;
  {
    std::vector<const void*> outs(static_cast<size_t>(count));
    for (int32_t i = 0; i < count; ++i) outs[i] = items[i].perm_out;
    std::sort(outs.begin(), outs.end());
    if (std::adjacent_find(outs.begin(), outs.end()) != outs.end())
      return fail(h, PLAS_ERR_INVALID_ARGUMENT, "items share a perm_out buffer");
  }
  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  st = ensure_batch_state(h);
  if (st != PLAS_OK) return st;
  return run_batch(h, items, count, prm, cfg, stats);
}

int32_t plas_autotune_batch(plas_handle h, const plas_batch_item* items, int32_t count,
                            const plas_sort_params* params, int32_t graph, plas_tune_entry* table, int32_t cap,
                            int32_t* entries) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  h->error.clear();
  if (count < 1 || items == nullptr || table == nullptr || cap < 1 || entries == nullptr)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "bad autotune arguments");
  if (count >= kMaxSlots) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "too many sorts in one batch");
  plas_sort_params base;
  int32_t st = check_params(h, params, &base);
  if (st == PLAS_OK && base.resume != nullptr)
    st = fail(h, PLAS_ERR_INVALID_ARGUMENT, "batched sorts start from their items");
  if (st != PLAS_OK) return st;
  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  st = ensure_batch_state(h);
  if (st != PLAS_OK) return st;
  *entries = 0;

  std::vector<int> buckets;
  for (int32_t i = 0; i < count; ++i) {
    const int b = side_bucket(std::max(2, items[i].side));
    if (std::find(buckets.begin(), buckets.end(), b) == buckets.end()) buckets.push_back(b);
  }
  std::sort(buckets.begin(), buckets.end());
  if (static_cast<int32_t>(buckets.size()) > cap)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "tune table capacity below the number of side buckets");

  // Two truncated regimes: the first, coarsest level and the finest block
  // size (radius 15, beta 16).
  plas_sort_params coarse = base, fine = base;
  coarse.max_reorders = 6;
  fine.max_reorders = 6;
  fine.start_radius = 15.0;
  for (int b : buckets) {
    std::vector<plas_batch_item> sub;
    bool staged = false;
    for (int32_t i = 0; i < count; ++i)
      if (side_bucket(std::max(2, items[i].side)) == b) {
        plas_batch_item it = items[i];
        it.stats = nullptr;
        sub.push_back(it);
        staged = staged || plas::staged_blur(padded_channels(it.d), it.storage);
      }
    plas_tune_entry e{};
    e.side_lo = static_cast<int32_t>(std::ceil(std::pow(2.0, b / 2.0)));
    e.side_hi = static_cast<int32_t>(std::ceil(std::pow(2.0, (b + 1) / 2.0))) - 1;
    // Sides exactly on a bucket edge: make sure the range holds them.
    for (const plas_batch_item& it : sub) {
      e.side_lo = std::min(e.side_lo, it.side);
      e.side_hi = std::max(e.side_hi, it.side);
    }
    auto measure = [&](const plas_tune_entry& cand, double* ms) -> int32_t {
      plas_batch_config cfg;
      plas_batch_config_init(&cfg);
      cfg.graph = graph;
      cfg.tune = &cand;
      cfg.tune_count = 1;
      double best = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        double total = 0.0;
        for (const plas_sort_params* p : {&coarse, &fine}) {
          plas_batch_stats bs{};
          bs.struct_size = sizeof(bs);
          const int32_t r = run_batch(h, sub.data(), static_cast<int32_t>(sub.size()), *p, cfg, &bs);
          if (r != PLAS_OK) return r;
          total += bs.loop_ms;
        }
        best = std::min(best, total);
      }
      *ms = best;
      return PLAS_OK;
    };
    double best_ms = 1e300;
    e.blur_waves_per_block = kDefaultWavesPerBlock;
    e.assign_blocks = 0;
    for (int wpb : {2, 1, 4}) {
      if (!staged && wpb != kDefaultWavesPerBlock) continue;
      plas_tune_entry cand = e;
      cand.blur_waves_per_block = wpb;
      double ms = 0.0;
      st = measure(cand, &ms);
      if (st != PLAS_OK) return st;
      if (ms < best_ms) {
        best_ms = ms;
        e.blur_waves_per_block = wpb;
      }
    }
    for (int cap_blocks : {256, 1024, 16384}) {
      plas_tune_entry cand = e;
      cand.assign_blocks = cap_blocks;
      double ms = 0.0;
      st = measure(cand, &ms);
      if (st != PLAS_OK) return st;
      if (ms < best_ms) {
        best_ms = ms;
        e.assign_blocks = cap_blocks;
      }
    }
    table[(*entries)++] = e;
  }
  return PLAS_OK;
}

}  // extern "C"

// ================================================================== serving

namespace {

struct Job {
  int64_t id;
  plas_batch_item item;
  int64_t footprint;
  double submit_ms;
};

int64_t job_footprint(int32_t side, int32_t d, int32_t storage, const plas_sort_params& prm) {
  std::vector<LevelInfo> levels;
  if (build_schedule(side, prm.radius_decay, prm.min_block, prm.start_radius, &levels) != PLAS_OK) return -1;
  int64_t max_cells = 0;
  for (const LevelInfo& lv : levels) max_cells = std::max<int64_t>(max_cells, static_cast<int64_t>(lv.beta) * lv.beta);
  return static_cast<int64_t>(sort_layout(side, padded_channels(d), storage, levels.size(), max_cells).bytes);
}

}  // namespace

struct plas_server {
  plas_context* h = nullptr;
  plas_batch_state* b = nullptr;
  plas_sort_params prm{};
  plas_batch_config cfg{};
  std::vector<plas_tune_entry> tune;  // the server's copy of config->tune
  int64_t budget = 0;
  int64_t used = 0;
  int64_t next_id = 0;
  std::chrono::steady_clock::time_point t0;
  BatchRun* run = nullptr;
  std::vector<Job> waiting;                  // first come, first admitted
  std::vector<Job> running;                  // admitted, not finished
  std::vector<std::pair<int64_t, int32_t>> done;  // (id, status) not yet polled
  bool broken = false;
};

extern "C" {

int64_t plas_job_footprint(int32_t side, int32_t d, int32_t storage, const plas_sort_params* params) {
  plas_sort_params prm;
  plas_sort_params_init(&prm);
  if (params != nullptr) {
    if (params->struct_size != sizeof(plas_sort_params)) return PLAS_ERR_INVALID_ARGUMENT;
    prm = *params;
  }
  if (side < 2 || side > 46340 || d < 1 || d > PLAS_MAX_CHANNELS || !valid_storage(storage))
    return PLAS_ERR_INVALID_ARGUMENT;
  const int64_t f = job_footprint(side, d, storage, prm);
  return f < 0 ? PLAS_ERR_INVALID_ARGUMENT : f;
}

int32_t plas_server_create(plas_handle h, const plas_sort_params* params, const plas_batch_config* config,
                           int64_t memory_budget, plas_server_handle* out) {
  if (h == nullptr || out == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  h->error.clear();
  if (memory_budget <= 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "memory_budget must be > 0");
  plas_server* s = new (std::nothrow) plas_server();
  if (s == nullptr) return fail(h, PLAS_ERR_OUT_OF_MEMORY, "server");
  s->h = h;
  int32_t st = check_params(h, params, &s->prm);
  if (st == PLAS_OK && s->prm.resume != nullptr)
    st = fail(h, PLAS_ERR_INVALID_ARGUMENT, "served sorts start from their jobs");
  if (st == PLAS_OK) st = check_config(h, config, &s->cfg);
  if (st != PLAS_OK) {
    delete s;
    return st;
  }
  if (s->cfg.tune_count > 0) {
    s->tune.assign(s->cfg.tune, s->cfg.tune + s->cfg.tune_count);
    s->cfg.tune = s->tune.data();
  }
  s->budget = memory_budget;
  DeviceScope scope(h->device);
  if (!scope.ok()) {
    delete s;
    return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  }
  st = create_batch_state(h, &s->b);
  if (st != PLAS_OK) {
    delete s;
    return st;
  }
  s->t0 = std::chrono::steady_clock::now();
  s->run = new (std::nothrow) BatchRun(h, s->b, s->prm, s->cfg, s->t0);
  if (s->run == nullptr) {
    destroy_batch_state(s->b);
    delete s;
    return fail(h, PLAS_ERR_OUT_OF_MEMORY, "server");
  }
  *out = s;
  return PLAS_OK;
}

int32_t plas_server_submit(plas_server_handle s, const plas_batch_item* item, int64_t* job_id) {
  if (s == nullptr || item == nullptr || job_id == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  plas_context* h = s->h;
  h->error.clear();
  if (s->broken) return fail(h, PLAS_ERR_HIP, "the server failed earlier");
  int32_t st = check_features(h, item->features, item->n, item->d, item->side, item->layout, item->dtype);
  if (st != PLAS_OK) return st;
  if (item->perm_out == nullptr) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "item perm_out is NULL");
  if (!valid_storage(item->storage)) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "item storage is unknown");
  if (item->stats != nullptr && item->stats->struct_size != sizeof(plas_sort_stats))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "item stats->struct_size does not match this library");
  Job j;
  j.id = s->next_id++;
  j.item = *item;
  j.footprint = job_footprint(item->side, item->d, item->storage, s->prm);
  j.submit_ms = ms_since(s->t0);
  s->waiting.push_back(j);
  *job_id = j.id;
  return PLAS_OK;
}

int32_t plas_server_step(plas_server_handle s, int32_t* running, int32_t* waiting) {
  if (s == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  plas_context* h = s->h;
  h->error.clear();
  if (s->broken) return fail(h, PLAS_ERR_HIP, "the server failed earlier");
  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  // Work the caller queued before this call (e.g. producing features) comes first.
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  StreamSwap swap(h, s->b->stream);
  // Admission at this reorder boundary, first come first: a job enters when
  // its memory fits, or when nothing runs.
  size_t admitted = 0;
  while (admitted < s->waiting.size()) {
    const Job& j = s->waiting[admitted];
    if (!s->running.empty() && s->used + j.footprint > s->budget) break;
    const int32_t st = s->run->add(j.item, j.id, j.submit_ms);
    if (st == PLAS_OK) {
      s->running.push_back(j);
      s->used += j.footprint;
    } else if (st == PLAS_ERR_HIP || st == PLAS_ERR_OUT_OF_MEMORY) {
      s->broken = st == PLAS_ERR_HIP;
      if (st == PLAS_ERR_OUT_OF_MEMORY && !s->running.empty()) break;  // retry when memory frees up
      s->done.emplace_back(j.id, st);
    } else {
      s->done.emplace_back(j.id, st);  // this job's inputs are bad; the server goes on
    }
    ++admitted;
    if (s->broken) break;
  }
  s->waiting.erase(s->waiting.begin(), s->waiting.begin() + admitted);
  if (s->broken) return fail(h, PLAS_ERR_HIP, h->error.empty() ? "admission failed" : h->error);
  if (s->run->running() > 0) {
    const int32_t st = s->run->chunk();
    if (st != PLAS_OK) {
      s->broken = true;
      return st;
    }
    for (int64_t id : s->run->take_finished()) {
      for (size_t i = 0; i < s->running.size(); ++i)
        if (s->running[i].id == id) {
          s->used -= s->running[i].footprint;
          s->running.erase(s->running.begin() + i);
          break;
        }
      s->done.emplace_back(id, PLAS_OK);
    }
  }
  if (running) *running = static_cast<int32_t>(s->running.size());
  if (waiting) *waiting = static_cast<int32_t>(s->waiting.size());
  return PLAS_OK;
}

int32_t plas_server_poll(plas_server_handle s, int64_t* job_ids, int32_t* statuses, int32_t cap, int32_t* count) {
  if (s == nullptr || count == nullptr || cap < 0 || (cap > 0 && (job_ids == nullptr || statuses == nullptr)))
    return PLAS_ERR_INVALID_ARGUMENT;
  const int32_t n = std::min<int32_t>(cap, static_cast<int32_t>(s->done.size()));
  for (int32_t i = 0; i < n; ++i) {
    job_ids[i] = s->done[i].first;
    statuses[i] = s->done[i].second;
  }
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *count = n;
  return PLAS_OK;
}

int32_t plas_server_destroy(plas_server_handle s) {
  if (s == nullptr) return PLAS_OK;
  DeviceScope scope(s->h->device);
  if (s->b != nullptr && s->b->stream != nullptr) (void)hipStreamSynchronize(s->b->stream);
  delete s->run;
  destroy_batch_state(s->b);
  delete s;
  return PLAS_OK;
}

}  // extern "C"
