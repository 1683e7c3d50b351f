// plas_engine.cpp -- host side of libplas.so: argument checks, the device
// workspace, the schedule, the launch sequence of a sort, and the C ABI of
// include/plas.h and include/plas_stages.h.
//
// A sort runs entirely on the device. The host prepares the radius schedule
// (it depends only on the grid side), uploads the first reorder's
// parameters, and then queues reorders in chunks: blur rows (which then fill
// the grouping table), blur columns, assignment. The last block of each
// assignment runs the control step (stall test, new block shift, next
// radius), so the data-dependent control flow stays on the device and the
// host only reads a small status block between chunks to learn whether the
// device has finished; kernels queued after the end return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plas_host.h"
#include "plas_stages.h"

using namespace plas_host;

static_assert(sizeof(plas_level_out) == sizeof(plas_level_stat), "trace entry layout");


// ======================================================================== C ABI

extern "C" {

int32_t plas_get_abi_version(void) { return PLAS_ABI_VERSION; }

int32_t plas_sort_params_init(plas_sort_params* p) {
  if (p == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(plas_sort_params);
  p->inv_threshold = 10000;
  p->seed = 0x5EED;
  p->radius_decay = 0.95;
  p->start_radius = 0.0;
  p->max_reorders = 0;
  p->init_perm = nullptr;
  p->min_block = 16;
  p->profile = 0;
  p->reorders_per_sync = 0;
  p->storage = PLAS_STORAGE_F32;
  p->filter = PLAS_FILTER_BOX;
  return PLAS_OK;
}

const char* plas_status_string(int32_t status) {
  switch (status) {
    case PLAS_OK: return "ok";
    case PLAS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case PLAS_ERR_UNSUPPORTED: return "unsupported";
    case PLAS_ERR_OUT_OF_MEMORY: return "out of device memory";
    case PLAS_ERR_HIP: return "HIP runtime error";
    case PLAS_ERR_NONFINITE: return "non-finite feature value";
    default: return "unknown status";
  }
}

const char* plas_last_error(plas_handle h) { return h == nullptr ? "" : h->error.c_str(); }

int32_t plas_create(plas_handle* out, int32_t device) {
  if (out == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return PLAS_ERR_HIP;
  if (device < 0 || device >= count) return PLAS_ERR_INVALID_ARGUMENT;
  plas_context* h = new (std::nothrow) plas_context();
  if (h == nullptr) return PLAS_ERR_OUT_OF_MEMORY;
  h->device = device;
  DeviceScope scope(device);
  if (!scope.ok()) {
    delete h;
    return PLAS_ERR_HIP;
  }
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&h->status_host), sizeof(HostStatus)) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&h->range_host), (2 * 64 + 1) * sizeof(float)) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&h->u64_host), 16 * sizeof(unsigned long long)) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&h->state_host), sizeof(DevState)) == hipSuccess &&
            reserve(h->state, sizeof(DevState)) == hipSuccess &&
            reserve(h->stage_state, sizeof(DevState)) == hipSuccess &&
            reserve(h->scratch, 16 * sizeof(unsigned long long)) == hipSuccess;
  if (!ok) {
    plas_destroy(h);
    return PLAS_ERR_OUT_OF_MEMORY;
  }
  // The no-allocation energy query's scratch on this device (its address,
  // looked up once per device with the device current).
  if (plas::noalloc_scratch(device, &h->noalloc) != hipSuccess) {
    plas_destroy(h);
    return PLAS_ERR_HIP;
  }
  *out = h;
  return PLAS_OK;
}

int32_t plas_destroy(plas_handle h) {
  if (h == nullptr) return PLAS_OK;
  DeviceScope scope(h->device);
  if (h->stream != nullptr) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  release_batch_state(h);
  DeviceBuffer* bufs[] = {&h->grid_g, &h->grid_h, &h->grid_t, &h->perm, &h->table, &h->inv,
                          &h->range_part, &h->range_out, &h->levels, &h->trace, &h->state,
                          &h->stage_state, &h->scratch, &h->vad};
  for (DeviceBuffer* b : bufs) release(*b);
  if (h->status_host) (void)hipHostFree(h->status_host);
  if (h->range_host) (void)hipHostFree(h->range_host);
  if (h->u64_host) (void)hipHostFree(h->u64_host);
  if (h->state_host) (void)hipHostFree(h->state_host);
  delete h;
  return PLAS_OK;
}

int32_t plas_set_stream(plas_handle h, void* stream) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  h->stream = static_cast<hipStream_t>(stream);
  return PLAS_OK;
}

int32_t plas_sort(plas_handle h, const void* features, int64_t n, int32_t d, int32_t side,
                  int32_t layout, int32_t dtype, const plas_sort_params* params, int32_t* perm_out,
                  plas_sort_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  int32_t st = check_features(h, features, n, d, side, layout, dtype);
  if (st != PLAS_OK) return st;
  h->error.clear();
  if (perm_out == nullptr) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "perm_out is NULL");
  plas_sort_params prm;
  st = check_params(h, params, &prm);
  if (st != PLAS_OK) return st;
  if (stats != nullptr && stats->struct_size != sizeof(plas_sort_stats))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "stats->struct_size does not match this library");

  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  const int32_t w = side;
  const int dp = padded_channels(d);

  std::vector<LevelInfo> levels;
  st = build_schedule(w, prm.radius_decay, prm.min_block, prm.start_radius, &levels);
  if (st != PLAS_OK) return fail(h, st, "bad schedule parameters");
  int64_t max_cells = 0, max_items = 0;
  for (const LevelInfo& lv : levels) {
    max_cells = std::max<int64_t>(max_cells, static_cast<int64_t>(lv.beta) * lv.beta);
    max_items = std::max<int64_t>(max_items, lv.groups + lv.singles);
  }

  // Workspace.
  int32_t s = 0;
  const int32_t storage = prm.storage;
  st = prepare_features(h, features, dtype, n, d, layout, dp, storage, &s);
  if (st != PLAS_OK) return st;
  PLAS_HIP(h, reserve(h->perm, static_cast<size_t>(n) * sizeof(int32_t)));
  PLAS_HIP(h, reserve(h->table, static_cast<size_t>(max_cells) * sizeof(int32_t)));
  PLAS_HIP(h, reserve(h->levels, levels.size() * sizeof(LevelInfo)));
  PLAS_HIP(h, reserve(h->trace, levels.size() * sizeof(plas_level_out)));
  st = upload_inverse_counts(h, w);
  if (st != PLAS_OK) return st;
  PLAS_HIP(h, hipMemcpyAsync(h->levels.ptr, levels.data(), levels.size() * sizeof(LevelInfo),
                             hipMemcpyHostToDevice, h->stream));
  PLAS_HIP(h, hipMemsetAsync(h->trace.ptr, 0, levels.size() * sizeof(plas_level_out), h->stream));

  void* G = h->grid_g.ptr;
  void* H = h->grid_h.ptr;
  void* T = h->grid_t.ptr;  // holds X until the gather
  int32_t* P = as<int32_t>(h->perm);

  // Start arrangement: the caller's, or the keyed bijection of draw
  // (seed, 0, 0) (random positions, Sec. 3.1).
  if (prm.init_perm != nullptr) {
    st = check_permutation(h, prm.init_perm, n, as<int32_t>(h->grid_h));
    if (st != PLAS_OK) return st;
    PLAS_HIP(h, hipMemcpyAsync(P, prm.init_perm, static_cast<size_t>(n) * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, h->stream));
  } else {
    const plas::Words4 k0 = plas::draw(prm.seed, plas::kDrawStart, 0);
    PLAS_HIP(h, plas::launch_start_perm(P, n, k0.v, h->stream));
  }
  PLAS_HIP(h, plas::launch_gather(T, P, G, n, dp, storage, h->stream));

  // First reorder's state.
  DevState* S = h->state_host;
  init_sort_state(S, w, s, levels, prm, prm.seed);
  if (prm.resume != nullptr) {
    st = apply_checkpoint(h, S, *prm.resume, levels);
    if (st != PLAS_OK) return st;
  }
  // The state: the parameters of the next reorder and the controller. Each
  // reorder's assignment ends with the control step, run on it in place.
  DevState* Sd = as<DevState>(h->state);
  PLAS_HIP(h, hipMemcpyAsync(Sd, S, sizeof(DevState), hipMemcpyHostToDevice, h->stream));

  const LevelInfo* Ld = as<LevelInfo>(h->levels);
  plas_level_out* Td = as<plas_level_out>(h->trace);
  int32_t* table = as<int32_t>(h->table);
  const plas::TableArgs table_fill{table, max_cells};
  const plas::ControlArgs control{Ld, Td};
  const int chunk = prm.reorders_per_sync > 0 ? prm.reorders_per_sync : kDefaultReordersPerSync;
  const int passes = prm.filter == PLAS_FILTER_BOX3 ? 3 : 1;  // box passes per axis
  const bool profile = prm.profile != 0;
  if (profile) {
    st = ensure_events(h, static_cast<size_t>(chunk) * 3);
    if (st != PLAS_OK) return st;
  }
  const int64_t max_k = reorder_bound(levels.size(), prm.inv_threshold);
  double blur_ms = 0.0, assign_ms = 0.0;
  int64_t timed_reorders = 0;
  int64_t slots = 0;  // reorder slots queued so far; slot i runs reorder k0 + i unless the sort has ended
  const int64_t k0 = S->k;  // reorders done before this call (a resumed sort)
  for (;;) {
    for (int i = 0; i < chunk; ++i) {
      // Each axis takes `passes` box passes (PLAS_FILTER_BOX3: three),
      // through H and T in turn, the last column pass writing T: rows G -> H
      // [-> T -> H], columns [H -> T -> H ->] H -> T. The first row pass
      // fills the grouping table after its lines.
      const bool timed = profile && i % kProfileEvery == 0;
      if (timed) PLAS_HIP(h, hipEventRecord(h->events[3 * i + 0], h->stream));
      void* bufs[2] = {H, T};
      const void* src = G;
      for (int p = 0; p < passes; ++p) {
        void* dst = bufs[p & 1];
        PLAS_HIP(h, plas::launch_blur_pass(src, dst, w, dp, storage, Sd, 0, 0, as<float>(h->inv), h->stream,
                                           p == 0 ? &table_fill : nullptr));
        src = dst;
      }
      for (int p = 0; p < passes; ++p) {
        void* dst = p == passes - 1 ? T : bufs[(passes + p) & 1];
        PLAS_HIP(h, plas::launch_blur_pass(src, dst, w, dp, storage, Sd, 0, 1, as<float>(h->inv), h->stream));
        src = dst;
      }
      // One event ends the blur passes and starts the assignment.
      if (timed) PLAS_HIP(h, hipEventRecord(h->events[3 * i + 1], h->stream));
      PLAS_HIP(h, plas::launch_assign(G, T, P, table, Sd, dp, storage, max_items, h->stream, &control));
      if (timed) PLAS_HIP(h, hipEventRecord(h->events[3 * i + 2], h->stream));
    }
    const int64_t first_slot = slots;
    slots += chunk;
    PLAS_HIP(h, hipMemcpyAsync(h->status_host, &Sd->done, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    PLAS_HIP(h, hipMemcpyAsync(&h->status_host->k, &Sd->k, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
    PLAS_HIP(h, hipStreamSynchronize(h->stream));
    const bool done = h->status_host->done != 0;
    const int64_t k_now = h->status_host->k;
    if (profile) {
      // Slots at or after the end of the sort returned at once.
      const int64_t ran = done ? std::max<int64_t>(0, std::min<int64_t>(chunk, k_now - k0 - first_slot)) : chunk;
      for (int64_t i = 0; i < ran; i += kProfileEvery) {
        float a = 0.0f, b = 0.0f;
        PLAS_HIP(h, hipEventElapsedTime(&a, h->events[3 * i + 0], h->events[3 * i + 1]));
        PLAS_HIP(h, hipEventElapsedTime(&b, h->events[3 * i + 1], h->events[3 * i + 2]));
        blur_ms += a;
        assign_ms += b;
        ++timed_reorders;
      }
    }
    if (done) break;
    // Every queued slot has run and been controlled by now; if k falls short
    // the device state is broken. Also stop at the bound on reorders that
    // the stall test implies (energies strictly fall by at least 1/M per
    // improvement, two stalls end a level).
    if (k_now - k0 != slots || k_now > max_k)
      return fail(h, PLAS_ERR_HIP, "device controller made no progress");
  }

  PLAS_HIP(h, hipMemcpyAsync(perm_out, P, static_cast<size_t>(n) * sizeof(int32_t), hipMemcpyDeviceToDevice,
                             h->stream));
  PLAS_HIP(h, hipMemcpyAsync(S, Sd, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  if (stats != nullptr) {
    stats->levels = S->levels_run;
    stats->reorders = S->k;
    stats->energy_fixed = S->energy_last;
    stats->scale_shift = s;
    stats->energy = std::ldexp(static_cast<double>(S->energy_last), -s) / static_cast<double>(n);
    stats->trace_len = 0;
    if (stats->trace != nullptr && stats->trace_cap > 0) {
      const int32_t len = std::min(stats->trace_cap, S->levels_run);
      if (len > 0) {
        PLAS_HIP(h, hipMemcpyAsync(stats->trace, Td, static_cast<size_t>(len) * sizeof(plas_level_out),
                                   hipMemcpyDeviceToHost, h->stream));
        PLAS_HIP(h, hipStreamSynchronize(h->stream));
      }
      stats->trace_len = len;
    }
    stats->blur_ms = blur_ms;
    stats->blur_launches = 2 * passes * timed_reorders;
    stats->assign_ms = assign_ms;
    stats->assign_launches = timed_reorders;
    stats->total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats->checkpoint != nullptr) fill_checkpoint(*S, static_cast<int32_t>(levels.size()), stats->checkpoint);
  }
  return PLAS_OK;
}

int32_t plas_grid_energy(plas_handle h, const void* features, const int32_t* perm, int64_t n, int32_t d,
                         int32_t side, int32_t layout, int32_t dtype, int32_t storage, int32_t radius,
                         uint64_t* energy_fixed, int32_t* scale_shift_out, double* energy_mean) {
  int32_t st = check_features(h, features, n, d, side, layout, dtype);
  if (st != PLAS_OK) return st;
  h->error.clear();
  if (radius < 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "radius must be >= 0");
  if (!valid_storage(storage)) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "unknown storage");
  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  const int dp = padded_channels(d);
  int32_t s = 0;
  st = prepare_features(h, features, dtype, n, d, layout, dp, storage, &s);
  if (st != PLAS_OK) return st;
  if (perm != nullptr) {
    st = check_permutation(h, perm, n, as<int32_t>(h->grid_h));
    if (st != PLAS_OK) return st;
  }
  st = upload_inverse_counts(h, side);
  if (st != PLAS_OK) return st;
  void* G = h->grid_g.ptr;
  void* H = h->grid_h.ptr;
  void* T = h->grid_t.ptr;
  PLAS_HIP(h, plas::launch_gather(T, perm, G, n, dp, storage, h->stream));
  PLAS_HIP(h, plas::launch_blur_pass(G, H, side, dp, storage, nullptr, radius, 0, as<float>(h->inv), h->stream));
  PLAS_HIP(h, plas::launch_blur_pass(H, T, side, dp, storage, nullptr, radius, 1, as<float>(h->inv), h->stream));
  unsigned long long* acc = as<unsigned long long>(h->scratch);
  PLAS_HIP(h, hipMemsetAsync(acc, 0, sizeof(unsigned long long), h->stream));
  PLAS_HIP(h, plas::launch_energy(G, T, n, dp, storage, s, acc, h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->u64_host, acc, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  const uint64_t E = h->u64_host[0];
  if (energy_fixed) *energy_fixed = E;
  if (scale_shift_out) *scale_shift_out = s;
  if (energy_mean) *energy_mean = std::ldexp(static_cast<double>(E), -s) / static_cast<double>(n);
  return PLAS_OK;
}

int32_t plas_grid_energy_noalloc(plas_handle h, const void* features, const int32_t* perm, int64_t n, int32_t d,
                                 int32_t side, int32_t layout, int32_t dtype, int32_t storage, int32_t radius,
                                 uint64_t* energy_fixed, int32_t* scale_shift_out, double* energy_mean) {
  // plas_grid_energy's steps on the device's static scratch (no allocation,
  // no memset): ingest into T, range and scale, permutation check (counts in
  // H), 1/c table, gather into G, rows into H, columns into T, energy.
  using L = plas::NoAllocLayout;
  int32_t st = check_features(h, features, n, d, side, layout, dtype);
  if (st != PLAS_OK) return st;
  h->error.clear();
  if (radius < 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "radius must be >= 0");
  if (!valid_storage(storage)) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "unknown storage");
  if (n > plas::kNoAllocMaxCells)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "n above the no-allocation limit of 65536 cells (side 256)");
  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  char* base = static_cast<char*>(h->noalloc);
  void* G = base + L::kG;
  void* H = base + L::kH;
  void* T = base + L::kT;
  float* range_part = reinterpret_cast<float*>(base + L::kRangePart);
  float* range_out = reinterpret_cast<float*>(base + L::kRangeOut);
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(base + L::kFlags);
  int32_t* flag = reinterpret_cast<int32_t*>(base + L::kFlags + 8);
  float* inv = reinterpret_cast<float*>(base + L::kInv);
  const int dp = padded_channels(d);

  PLAS_HIP(h, plas::launch_ingest(features, dtype == PLAS_DTYPE_BF16, n, d, layout, dp, storage, T, h->stream));
  PLAS_HIP(h, plas::launch_range(T, n, d, dp, storage, range_part, range_out, h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->range_host, range_out, (2 * dp + 1) * sizeof(float), hipMemcpyDeviceToHost,
                             h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  if (h->range_host[2 * dp] != 0.0f) return fail(h, PLAS_ERR_NONFINITE, "features contain NaN or infinity");
  const int32_t s = scale_shift(h->range_host, h->range_host + dp, d, n);
  if (perm != nullptr) {
    int32_t* counts = static_cast<int32_t*>(H);
    PLAS_HIP(h, plas::launch_fill_u32(reinterpret_cast<uint32_t*>(counts), n, 0u, h->stream));
    PLAS_HIP(h, plas::launch_fill_u32(reinterpret_cast<uint32_t*>(flag), 1, 0u, h->stream));
    PLAS_HIP(h, plas::launch_check_perm(perm, n, counts, flag, h->stream));
    PLAS_HIP(h, hipMemcpyAsync(h->u64_host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    PLAS_HIP(h, hipStreamSynchronize(h->stream));
    int32_t bad = 0;
    std::memcpy(&bad, h->u64_host, sizeof(int32_t));
    if (bad != 0) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "permutation is not a bijection of [0, n)");
  }
  PLAS_HIP(h, plas::launch_inverse_counts(inv, side, h->stream));
  PLAS_HIP(h, plas::launch_gather(T, perm, G, n, dp, storage, h->stream));
  PLAS_HIP(h, plas::launch_blur_pass(G, H, side, dp, storage, nullptr, radius, 0, inv, h->stream));
  PLAS_HIP(h, plas::launch_blur_pass(H, T, side, dp, storage, nullptr, radius, 1, inv, h->stream));
  PLAS_HIP(h, plas::launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 2, 0u, h->stream));
  PLAS_HIP(h, plas::launch_energy(G, T, n, dp, storage, s, acc, h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->u64_host, acc, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  const uint64_t E = h->u64_host[0];
  if (energy_fixed) *energy_fixed = E;
  if (scale_shift_out) *scale_shift_out = s;
  if (energy_mean) *energy_mean = std::ldexp(static_cast<double>(E), -s) / static_cast<double>(n);
  return PLAS_OK;
}

int32_t plas_vad(plas_handle h, const void* features, const int32_t* perm, int64_t n, int32_t d, int32_t side,
                 int32_t layout, int32_t dtype, double* vad) {
  int32_t st = check_features(h, features, n, d, side, layout, dtype);
  if (st != PLAS_OK) return st;
  h->error.clear();
  if (vad == nullptr) return fail(h, PLAS_ERR_INVALID_ARGUMENT, "vad is NULL");
  DeviceScope scope(h->device);
  if (!scope.ok()) return fail(h, PLAS_ERR_HIP, "hipSetDevice failed");
  if (perm != nullptr) {
    PLAS_HIP(h, reserve(h->grid_h, static_cast<size_t>(n) * sizeof(int32_t)));
    st = check_permutation(h, perm, n, as<int32_t>(h->grid_h));
    if (st != PLAS_OK) return st;
  }
  const size_t parts = plas::vad_partial_doubles();
  PLAS_HIP(h, reserve(h->vad, (parts + 2) * sizeof(double)));
  double* part = as<double>(h->vad);
  double* out = part + parts;
  PLAS_HIP(h, plas::launch_vad(features, dtype == PLAS_DTYPE_BF16, perm, n, d, side, layout, part, out, h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->u64_host, out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  double v[2];
  std::memcpy(v, h->u64_host, sizeof(v));
  *vad = v[1];
  return PLAS_OK;
}

// ------------------------------------------------------------------ stages

static bool valid_dp(int32_t dp) { return dp == 4 || dp == 8 || dp == 16 || dp == 32 || dp == 64; }

int32_t plas_stage_blur(plas_handle h, const void* grid, void* target, int32_t side, int32_t dp, int32_t storage,
                        int32_t radius) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  if (grid == nullptr || target == nullptr || side < 1 || side > 46340 || !valid_dp(dp) || radius < 0 ||
      !valid_storage(storage))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "bad blur arguments");
  DeviceScope scope(h->device);
  const int64_t n = static_cast<int64_t>(side) * side;
  PLAS_HIP(h, reserve(h->grid_h, static_cast<size_t>(n) * dp * storage_bytes(storage)));
  int32_t st = upload_inverse_counts(h, side);
  if (st != PLAS_OK) return st;
  void* H = h->grid_h.ptr;
  PLAS_HIP(h, plas::launch_blur_pass(grid, H, side, dp, storage, nullptr, radius, 0, as<float>(h->inv), h->stream));
  PLAS_HIP(h, plas::launch_blur_pass(H, target, side, dp, storage, nullptr, radius, 1, as<float>(h->inv),
                                     h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  return PLAS_OK;
}

static int32_t upload_stage_state(plas_handle h, int32_t side, int32_t beta, int32_t dy, int32_t dx,
                                  const uint64_t keys[4], int32_t s) {
  DevState* S = h->state_host;
  std::memset(S, 0, sizeof(DevState));
  S->w = side;
  S->s = s;
  S->dy = dy;
  S->dx = dx;
  LevelInfo lv{};
  lv.phi = static_cast<double>(beta - 1);
  lv.r = beta - 1;
  lv.beta = beta;
  lv.nb = side / beta;
  const int64_t cells = static_cast<int64_t>(beta) * beta;
  lv.groups_per_block = cells / 4;
  lv.groups = static_cast<int64_t>(lv.nb) * lv.nb * lv.groups_per_block;
  const int64_t covered = static_cast<int64_t>(lv.nb) * beta;
  lv.singles = static_cast<int64_t>(side) * side - covered * covered +
               static_cast<int64_t>(lv.nb) * lv.nb * (cells % 4);
  fill_state_for_level(S, lv);
  for (int i = 0; i < 4; ++i) S->keys[i] = keys[i];
  PLAS_HIP(h, hipMemcpyAsync(h->stage_state.ptr, S, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  return PLAS_OK;
}

int32_t plas_stage_group_table(plas_handle h, int32_t beta, const uint64_t round_keys[4], int32_t* table) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  if (table == nullptr || round_keys == nullptr || beta < 1 || beta > 65535)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "bad group table arguments");
  DeviceScope scope(h->device);
  int32_t st = upload_stage_state(h, beta, beta, 0, 0, round_keys, 0);
  if (st != PLAS_OK) return st;
  PLAS_HIP(h, plas::launch_group_table(table, as<DevState>(h->stage_state),
                                       static_cast<int64_t>(beta) * beta, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  return PLAS_OK;
}

int32_t plas_stage_assign(plas_handle h, void* grid, const void* target, int32_t* perm, int32_t side,
                          int32_t dp, int32_t storage, int32_t beta, int32_t dy, int32_t dx,
                          const uint64_t round_keys[4], int32_t scale_shift_in, uint64_t* energy,
                          uint64_t* moved) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  if (grid == nullptr || target == nullptr || perm == nullptr || round_keys == nullptr || side < 2 ||
      side > 46340 || !valid_dp(dp) || !valid_storage(storage) || beta < 2 || beta > side || dy < 0 ||
      dy >= side || dx < 0 || dx >= side)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "bad assign arguments");
  DeviceScope scope(h->device);
  const int64_t cells = static_cast<int64_t>(beta) * beta;
  PLAS_HIP(h, reserve(h->table, static_cast<size_t>(cells) * sizeof(int32_t)));
  int32_t st = upload_stage_state(h, side, beta, dy, dx, round_keys, scale_shift_in);
  if (st != PLAS_OK) return st;
  DevState* Sd = as<DevState>(h->stage_state);
  PLAS_HIP(h, plas::launch_group_table(as<int32_t>(h->table), Sd, cells, h->stream));
  const int64_t items = h->state_host->groups + h->state_host->singles;
  PLAS_HIP(h, plas::launch_assign(grid, target, perm, as<int32_t>(h->table), Sd, dp, storage, items, h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->state_host, Sd, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  unsigned long long E = 0, M = 0;
  for (int i = 0; i < plas::kAccSlots; ++i) {
    E += h->state_host->energy_acc[i];
    M += h->state_host->moved_acc[i];
  }
  if (energy) *energy = E;
  if (moved) *moved = M;
  return PLAS_OK;
}

int32_t plas_stage_energy(plas_handle h, const void* grid, const void* target, int32_t side, int32_t dp,
                          int32_t storage, int32_t scale_shift_in, uint64_t* energy) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  if (grid == nullptr || target == nullptr || side < 1 || side > 46340 || !valid_dp(dp) || !valid_storage(storage))
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "bad energy arguments");
  DeviceScope scope(h->device);
  unsigned long long* acc = as<unsigned long long>(h->scratch);
  PLAS_HIP(h, hipMemsetAsync(acc, 0, sizeof(unsigned long long), h->stream));
  PLAS_HIP(h, plas::launch_energy(grid, target, static_cast<int64_t>(side) * side, dp, storage, scale_shift_in, acc,
                                  h->stream));
  PLAS_HIP(h, hipMemcpyAsync(h->u64_host, acc, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  if (energy) *energy = h->u64_host[0];
  return PLAS_OK;
}

int32_t plas_stage_bijection(plas_handle h, int64_t n, const uint64_t round_keys[4], int32_t* out) {
  if (h == nullptr) return PLAS_ERR_INVALID_ARGUMENT;
  if (out == nullptr || round_keys == nullptr || n < 1 || n > 2147483647LL)
    return fail(h, PLAS_ERR_INVALID_ARGUMENT, "bad bijection arguments");
  DeviceScope scope(h->device);
  PLAS_HIP(h, plas::launch_start_perm(out, n, round_keys, h->stream));
  PLAS_HIP(h, hipStreamSynchronize(h->stream));
  return PLAS_OK;
}

void plas_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  plas::Words4 x;
  for (int i = 0; i < 4; ++i) x.v[i] = ctr[i];
  const plas::Words4 y = plas::philox4x64_10(x, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = y.v[i];
}

void plas_draw(uint64_t seed, uint64_t purpose, uint64_t index, uint64_t out[4]) {
  const plas::Words4 y = plas::draw(seed, purpose, index);
  for (int i = 0; i < 4; ++i) out[i] = y.v[i];
}

int32_t plas_schedule(int32_t side, double decay, int32_t min_block, double start_radius, double* phi,
                      int32_t* r, int32_t* beta, int32_t cap) {
  std::vector<LevelInfo> levels;
  const int32_t st = build_schedule(side, decay, min_block, start_radius, &levels);
  if (st != PLAS_OK) return st;
  for (size_t i = 0; i < levels.size() && static_cast<int64_t>(i) < cap; ++i) {
    if (phi) phi[i] = levels[i].phi;
    if (r) r[i] = levels[i].r;
    if (beta) beta[i] = levels[i].beta;
  }
  return static_cast<int32_t>(levels.size());
}

int32_t plas_scale_shift_from_ranges(const float* mins, const float* maxs, int32_t d, int64_t n,
                                     int32_t* scale_shift_out) {
  if (mins == nullptr || maxs == nullptr || d < 1 || n < 1 || scale_shift_out == nullptr)
    return PLAS_ERR_INVALID_ARGUMENT;
  *scale_shift_out = scale_shift(mins, maxs, d, n);
  return PLAS_OK;
}

}  // extern "C"
