// rdx_engine.cpp -- device arena, run state, the runtime main loop of
// Algorithm 1 as planned sequences of window launches, HIP-graph replay and
// online tuning of the launch shape.
#include "rdx_engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace rdx {

namespace {

constexpr size_t kGranule = 256;
inline size_t align_up(size_t x) { return (x + kGranule - 1) & ~(kGranule - 1); }

#define RDX_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_error(RDX_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

template <typename T>
hipError_t dev_alloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

// The batch step index lives in an int32 on the device; it is brought back
// near zero (keeping its parity, which selects the worklist counter) before it
// could pass this.
constexpr int64_t kStepRebase = int64_t(1) << 30;

}  // namespace

// ------------------------------------------------------------------ arena ----
DeviceArena::~DeviceArena() {
  if (base_) (void)hipFree(base_);
}

hipError_t DeviceArena::reserve(size_t bytes) {
  bytes = align_up(bytes ? bytes : kGranule);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&base_), bytes);
  if (e != hipSuccess) {
    base_ = nullptr;
    return e;
  }
  cap_ = bytes;
  free_.clear();
  used_.clear();
  free_[0] = bytes;
  used_bytes_ = 0;
  return hipSuccess;
}

size_t DeviceArena::alloc(size_t bytes) {
  bytes = align_up(bytes ? bytes : kGranule);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, rest = it->second - bytes;
    free_.erase(it);
    if (rest) free_[off + bytes] = rest;
    used_[off] = bytes;
    used_bytes_ += bytes;
    return off;
  }
  return SIZE_MAX;
}

void DeviceArena::release(size_t off) {
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t start = off, size = u->second;
  used_bytes_ -= size;
  used_.erase(u);
  auto next = free_.lower_bound(start);
  if (next != free_.end() && next->first == start + size) {
    size += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == start) {
      start = prev->first;
      size += prev->second;
      free_.erase(prev);
    }
  }
  free_[start] = size;
}

size_t DeviceArena::largest_free() const {
  size_t m = 0;
  for (const auto& f : free_) m = std::max(m, f.second);
  return m;
}

// ------------------------------------------------------------------ model ----
void listing_pairs(const DevModel& m, int32_t pairs[32], int32_t* n_pairs, int32_t pair_of[32]) {
  int n = 0;
  for (int r = 0; r < 32; ++r) pair_of[r] = -1;
  for (int r = 0; r < m.R; ++r) {
    const int info = m.info[r];
    if ((info & 0xff) != 2) continue;
    const int a = (info >> 8) & 0xff, b = (info >> 16) & 0xff;
    const int key = a | (b << 8) | ((a == b ? 1 : 0) << 16);
    int p = 0;
    while (p < n && pairs[p] != key) ++p;
    if (p == n) pairs[n++] = key;
    pair_of[r] = p;
  }
  for (int p = n; p < 32; ++p) pairs[p] = 0;
  *n_pairs = n;
}

void listing_coefficients(const DevModel& m, const double* k, double* out) {
  int32_t pairs[32], pair_of[32], n_pairs = 0;
  listing_pairs(m, pairs, &n_pairs, pair_of);
  for (int j = 0; j < kLStride; ++j) out[j] = 0.0;
  for (int r = 0; r < m.R; ++r) {
    const int info = m.info[r];
    const int order = info & 0xff, a = (info >> 8) & 0xff, b = (info >> 16) & 0xff;
    if (order == 0) out[0] += k[r];
    else if (order == 1) out[1 + a] += k[r];
    else out[17 + pair_of[r]] += a == b ? 0.5 * k[r] : k[r];
  }
}

// Device image of a run's rate table: [kMaxRegions][32] constants, then
// [kMaxRegions][kLStride] listing coefficients, zero-padded.
static std::vector<double> rate_image(const DevModel& m, const HostInstance& I) {
  std::vector<double> kc((size_t)kMaxRegions * (32 + kLStride), 0.0);
  for (int reg = 0; reg < I.n_regions; ++reg) {
    for (int q = 0; q < I.R; ++q) kc[(size_t)reg * 32 + q] = I.kcst[(size_t)reg * I.R + q];
    listing_coefficients(m, &I.kcst[(size_t)reg * I.R], &kc[(size_t)kMaxRegions * 32 + (size_t)reg * kLStride]);
  }
  return kc;
}

DevModel make_dev_model(const HostInstance& I) {
  DevModel m;
  std::memset(&m, 0, sizeof m);
  m.S = I.S;
  m.R = I.R;
  const int S = I.S, R = I.R;
  for (int r = 0; r < R; ++r) {
    int order = 0, r0 = -1, r1 = -1;
    for (int s = 0; s < S; ++s) {
      const int nu = I.lhs[(size_t)r * S + s];
      order += nu;
      for (int c = 0; c < nu; ++c) {
        if (r0 < 0) r0 = s;
        else r1 = s;
      }
      m.delta[r][s] = (int8_t)(I.rhs[(size_t)r * S + s] - nu);
    }
    const int b0 = r0 < 0 ? 0xff : r0;
    const int b1 = (order == 2 && r1 >= 0) ? r1 : 0xff;
    m.info[r] = order | (b0 << 8) | (b1 << 16);
  }
  // deps(r): reactions whose propensity reads a species that r changes
  for (int r = 0; r < R; ++r) {
    unsigned long long mask = 0;
    for (int j = 0; j < R; ++j)
      for (int s = 0; s < S; ++s)
        if (m.delta[r][s] != 0 && I.lhs[(size_t)j * S + s] > 0) mask |= 1ull << j;
    m.deps[r] = mask;
  }
  return m;
}

// ----------------------------------------------------------------- engine ----
size_t Engine::run_bytes(const HostInstance& I) {
  const size_t T = (size_t)I.T, S = (size_t)I.S;
  size_t b = 2 * align_up(4 * S * T) + align_up(16 * T) + align_up(32 * T) + align_up(8 * T);
  if (I.n_regions > 1) b += align_up(T);
  b += align_up(sizeof(double) * kMaxRegions * (32 + kLStride));  // rate constants, listing coefficients
  b += align_up(sizeof(unsigned long long) * kTallyWords * kTallySlots + sizeof(int32_t));  // tallies, error flag
  return b;
}

size_t Engine::worklist_bytes_per_tet(int S) {
  (void)S;
  return 4 + 1;  // the tet index of its slot, and its share of the per-tile count and queue entry
}

void Engine::fence(hipStream_t stream) {
  for (auto& f : fences_)
    if (f.first == stream) {
      (void)hipEventRecord(f.second, stream);
      return;
    }
  hipEvent_t ev = nullptr;
  if (fences_.size() >= 16 || hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamSynchronize(stream);  // too many streams: wait for this one now
    return;
  }
  (void)hipEventRecord(ev, stream);
  fences_.emplace_back(stream, ev);
}

void Engine::drain() {
  for (auto& f : fences_) {
    (void)hipEventSynchronize(f.second);
    (void)hipEventDestroy(f.second);
  }
  fences_.clear();
}

namespace {
// Marks `stream` in the engine's fences when the enclosing method returns,
// whatever it enqueued before an early error return.
struct FenceOnExit {
  Engine* e;
  hipStream_t s;
  ~FenceOnExit() { e->fence(s); }
};
}  // namespace

Engine::~Engine() {
  drain();
  if (staged_) (void)hipEventSynchronize(staged_);
  free_graphs();
  if (capture_stream_) (void)hipStreamDestroy(capture_stream_);
  if (own_) (void)hipStreamDestroy(own_);
  for (hipEvent_t e : marks_) (void)hipEventDestroy(e);
  if (staged_) (void)hipEventDestroy(staged_);
  if (reset_staged_) {
    (void)hipEventSynchronize(reset_staged_);
    (void)hipEventDestroy(reset_staged_);
  }
  if (h_reset_) (void)hipHostFree(h_reset_);
  (void)hipFree(d_reset_);
  for (hipEvent_t e : tune_ev_)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(model_);
  (void)hipFree(d_runs_);
  (void)hipFree(d_tile_map_);
  (void)hipFree(d_n_tiles_);
  (void)hipFree(d_base_);
  (void)hipFree(wl_tile_count_);
  (void)hipFree(wl_mask_);
  (void)hipFree(evq_);
  (void)hipFree(evq_count_);
  (void)hipFree(wl_tet_);
  (void)hipFree(tile_ctr_);
  if (h_runs_) (void)hipHostFree(h_runs_);
  if (h_tile_map_) (void)hipHostFree(h_tile_map_);
  if (h_n_tiles_) (void)hipHostFree(h_n_tiles_);
}

void Engine::free_graphs() {
  for (auto& g : graphs_) (void)hipGraphExecDestroy(g.second);
  graphs_.clear();
}

rdx_status Engine::init(const HostInstance& proto, size_t arena_bytes, int max_runs, int64_t max_tets) {
  if (max_runs < 1 || max_tets < 1 || max_tets > (int64_t)INT32_MAX)
    return set_error(RDX_EINVAL, "engine capacity out of range");
  S_ = proto.S;
  R_ = proto.R;
  model_host_ = make_dev_model(proto);
  max_runs_ = max_runs;
  max_tets_ = max_tets;
  max_tiles_ = (max_tets + 63) / 64 + max_runs;
  if (max_tiles_ > (int64_t)INT32_MAX) return set_error(RDX_EINVAL, "too many tiles");
  if (64 * max_tiles_ > (int64_t)INT32_MAX) return set_error(RDX_EINVAL, "worklist too large");
  const size_t W = 64 * (size_t)max_tiles_;  // 64 worklist slots per tile
  bool ok = dev_alloc(&model_, 1) == hipSuccess && dev_alloc(&d_runs_, (size_t)max_runs) == hipSuccess &&
            dev_alloc(&d_tile_map_, (size_t)max_tiles_) == hipSuccess &&
            dev_alloc(&d_n_tiles_, 1) == hipSuccess && dev_alloc(&d_base_, 1) == hipSuccess &&
            dev_alloc(&wl_tile_count_, (size_t)max_tiles_) == hipSuccess && dev_alloc(&wl_mask_, (size_t)max_tiles_) == hipSuccess &&
            dev_alloc(&evq_, (size_t)kBins * kQueues * (size_t)((max_tiles_ + kQueues - 1) / kQueues)) == hipSuccess &&
            dev_alloc(&evq_count_, (size_t)2 * kBins * kQueues * kQueueStride) == hipSuccess &&
            dev_alloc(&wl_tet_, W) == hipSuccess && dev_alloc(&tile_ctr_, (size_t)2 * 8 * kClaimSubs * kCtrStride) == hipSuccess;
  if (ok && arena_bytes) ok = arena_.reserve(arena_bytes) == hipSuccess;
  if (ok) ok = hipHostMalloc(reinterpret_cast<void**>(&h_runs_), sizeof(RunDesc) * (size_t)max_runs) == hipSuccess;
  if (ok) ok = hipHostMalloc(reinterpret_cast<void**>(&h_tile_map_), sizeof(int2) * (size_t)max_tiles_) == hipSuccess;
  if (ok) ok = hipHostMalloc(reinterpret_cast<void**>(&h_n_tiles_), sizeof(int32_t)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return set_error(RDX_ENOMEM, "device allocation failed");
  }
  RDX_HIP(hipEventCreateWithFlags(&staged_, hipEventDisableTiming));
  RDX_HIP(hipEventCreate(&tune_ev_[0]));
  RDX_HIP(hipEventCreate(&tune_ev_[1]));
  RDX_HIP(hipStreamCreateWithFlags(&own_, hipStreamNonBlocking));
  RDX_HIP(hipMemcpyAsync(model_, &model_host_, sizeof model_host_, hipMemcpyHostToDevice, own_));
  RDX_HIP(hipMemsetAsync(d_n_tiles_, 0, sizeof(int32_t), own_));
  RDX_HIP(hipMemsetAsync(d_base_, 0, sizeof(int32_t), own_));
  RDX_HIP(hipMemsetAsync(wl_tile_count_, 0, sizeof(int32_t) * (size_t)max_tiles_, own_));
  RDX_HIP(hipMemsetAsync(evq_count_, 0, sizeof(unsigned long long) * 2 * kBins * kQueues * kQueueStride, own_));
  RDX_HIP(hipMemsetAsync(tile_ctr_, 0, sizeof(int32_t) * 2 * 8 * kClaimSubs * kCtrStride, own_));
  RDX_HIP(hipStreamSynchronize(own_));
  return RDX_OK;
}

bool Engine::compatible(const HostInstance& I) const {
  if (I.S != S_ || I.R != R_) return false;
  const DevModel m = make_dev_model(I);
  return std::memcmp(m.info, model_host_.info, sizeof m.info) == 0 &&
         std::memcmp(m.delta, model_host_.delta, sizeof m.delta) == 0 &&
         std::memcmp(m.deps, model_host_.deps, sizeof m.deps) == 0;
}

rdx_status Engine::add_run(Run* r, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  const HostInstance& I = r->host;
  if (!compatible(I)) return set_error(RDX_EINVAL, "run does not share the engine's species/reaction structure");
  if (resident_runs_ >= max_runs_ || resident_tets_ + I.T > max_tets_)
    return set_error(RDX_EBUDGET, "engine capacity reached");
  const size_t need = run_bytes(I);
  const size_t off = arena_.alloc(need);
  if (off == SIZE_MAX) return set_error(RDX_EBUDGET, "device arena cannot hold the run now");
  const size_t T = (size_t)I.T, S = (size_t)I.S;
  char* p = arena_.base() + off;
  auto carve = [&p](size_t bytes) {
    char* q = p;
    p += align_up(bytes);
    return q;
  };
  r->arena_off = off;
  r->cnt[0] = reinterpret_cast<int32_t*>(carve(4 * S * T));
  r->cnt[1] = reinterpret_cast<int32_t*>(carve(4 * S * T));
  r->nbr = reinterpret_cast<int32_t*>(carve(16 * T));
  r->geo = reinterpret_cast<double*>(carve(32 * T));
  r->nav = reinterpret_cast<double*>(carve(8 * T));
  r->region = I.n_regions > 1 ? reinterpret_cast<uint8_t*>(carve(T)) : nullptr;
  r->kcst = reinterpret_cast<double*>(carve(sizeof(double) * kMaxRegions * (32 + kLStride)));
  r->lcoef = r->kcst + kMaxRegions * 32;
  const size_t misc_bytes = sizeof(unsigned long long) * kTallyWords * kTallySlots + sizeof(int32_t);
  char* misc = carve(misc_bytes);
  r->tally = reinterpret_cast<unsigned long long*>(misc);
  r->err = reinterpret_cast<int32_t*>(misc + sizeof(unsigned long long) * kTallyWords * kTallySlots);

  // host images of the interleaved couplings and the padded rate table; the
  // copies are synchronous so the images can go when this returns
  std::vector<double> geo(4 * T);
  for (size_t i = 0; i < T; ++i) {
    geo[4 * i + 0] = I.G[i];
    geo[4 * i + 1] = I.cum[4 * i + 0];
    geo[4 * i + 2] = I.cum[4 * i + 1];
    geo[4 * i + 3] = I.cum[4 * i + 2];
  }
  const std::vector<double> kc = rate_image(model_host_, I);
  hipError_t e = hipMemcpyAsync(r->nbr, I.nbr.data(), 16 * T, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r->geo, geo.data(), 32 * T, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r->nav, I.nav.data(), 8 * T, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && r->region) e = hipMemcpyAsync(r->region, I.region.data(), T, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r->kcst, kc.data(), sizeof(double) * kc.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemsetAsync(r->cnt[0], 0, 4 * S * T, stream);
  if (e == hipSuccess) e = hipMemsetAsync(r->cnt[1], 0, 4 * S * T, stream);
  if (e == hipSuccess) e = hipMemsetAsync(misc, 0, misc_bytes, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    arena_.release(off);
    r->arena_off = SIZE_MAX;
    return set_error(RDX_EHIP, std::string("run upload: ") + hipGetErrorString(e));
  }
  r->t = 0.0;
  r->window = r->windows_run = r->voxel_steps = 0;
  resident_runs_ += 1;
  resident_tets_ += I.T;
  return RDX_OK;
}

void Engine::remove_run(Run* r, hipStream_t stream) {
  if (r->arena_off == SIZE_MAX) return;
  // the run's memory may only be reused once no launch can still touch it
  (void)hipStreamSynchronize(stream);
  arena_.release(r->arena_off);
  r->arena_off = SIZE_MAX;
  resident_runs_ -= 1;
  resident_tets_ -= r->host.T;
  tile_runs_.clear();  // the device tile map may name the run
}

rdx_status Engine::reset_run(Run* r, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  const size_t n = (size_t)r->host.S * (size_t)r->host.T;
  RDX_HIP(hipMemsetAsync(r->cnt[(r->window + 1) & 1], 0, sizeof(int32_t) * n, stream));
  RDX_HIP(hipMemsetAsync(r->tally, 0, sizeof(unsigned long long) * kTallyWords * kTallySlots, stream));
  RDX_HIP(hipMemsetAsync(r->err, 0, sizeof(int32_t), stream));
  return RDX_OK;
}

rdx_status Engine::reset_runs_device(Run* const* runs, size_t n, const int32_t* const* src, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  size_t n_chunks = 0;
  for (size_t j = 0; j < n; ++j) {
    const int64_t e = (int64_t)runs[j]->host.S * runs[j]->host.T;
    n_chunks += (size_t)std::max<int64_t>(1, (e + kResetChunk - 1) / kResetChunk);
  }
  if (n_chunks > (size_t)INT32_MAX) return set_error(RDX_EINVAL, "reset too large");
  if (!reset_staged_) RDX_HIP(hipEventCreateWithFlags(&reset_staged_, hipEventDisableTiming));
  RDX_HIP(hipEventSynchronize(reset_staged_));  // the pinned table may still be in flight
  if (n_chunks > reset_cap_) {
    if (h_reset_) RDX_HIP(hipHostFree(h_reset_));
    if (d_reset_) RDX_HIP(hipFree(d_reset_));
    h_reset_ = nullptr;
    d_reset_ = nullptr;
    reset_cap_ = 0;
    RDX_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_reset_), sizeof(ResetChunk) * n_chunks));
    RDX_HIP(hipMalloc(reinterpret_cast<void**>(&d_reset_), sizeof(ResetChunk) * n_chunks));
    reset_cap_ = n_chunks;
  }
  size_t c = 0;
  for (size_t j = 0; j < n; ++j) {
    Run* r = runs[j];
    if (r->arena_off == SIZE_MAX) return set_error(RDX_ESTATE, "run is not resident");
    r->t = 0.0;
    r->window = r->windows_run = r->voxel_steps = 0;
    const int64_t e = (int64_t)r->host.S * r->host.T;
    for (int64_t b = 0; b == 0 || b < e; b += kResetChunk) {
      ResetChunk& ch = h_reset_[c++];
      ch.src = src[j];
      ch.dst = r->cnt[0];
      ch.other = r->cnt[1];
      ch.tally = r->tally;
      ch.err = r->err;
      ch.begin = b;
      ch.end = std::min<int64_t>(b + kResetChunk, e);
    }
  }
  RDX_HIP(hipMemcpyAsync(d_reset_, h_reset_, sizeof(ResetChunk) * c, hipMemcpyHostToDevice, stream));
  RDX_HIP(hipEventRecord(reset_staged_, stream));
  const hipError_t e = launch_reset_chunks(d_reset_, (int64_t)c, stream);
  if (e != hipSuccess) return set_error(RDX_EHIP, std::string("reset launch: ") + hipGetErrorString(e));
  return RDX_OK;
}

rdx_status Engine::upload_counts(Run* r, const int32_t* counts, bool device, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  const size_t n = (size_t)r->host.S * (size_t)r->host.T;
  RDX_HIP(hipMemcpyAsync(r->cnt[r->window & 1], counts, sizeof(int32_t) * n,
                         device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, stream));
  if (!device) RDX_HIP(hipStreamSynchronize(stream));
  return RDX_OK;
}

rdx_status Engine::set_rates(Run* r, const double* kcst, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  const size_t n = (size_t)r->host.n_regions * (size_t)r->host.R;
  for (size_t i = 0; i < n; ++i)
    if (!(kcst[i] >= 0.0) || !std::isfinite(kcst[i]))
      return set_error(RDX_EINVAL, "rate constants must be finite and >= 0");
  std::vector<double> old(kcst, kcst + n);
  r->host.kcst.swap(old);
  const std::vector<double> kc = rate_image(model_host_, r->host);
  // stream-ordered: windows already enqueued keep the old constants; the
  // captured window graphs read the table through its pointer and need no
  // re-capture
  hipError_t e = hipMemcpyAsync(r->kcst, kc.data(), sizeof(double) * kc.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    r->host.kcst.swap(old);  // the host copy keeps describing the device table
    return set_error(RDX_EHIP, std::string("rate table upload: ") + hipGetErrorString(e));
  }
  return RDX_OK;
}

rdx_status Engine::region_counts(const Run* r, unsigned long long* scratch, unsigned long long* out,
                                 hipStream_t stream, bool mark) {
  RDX_HIP(launch_region_counts(r->cnt[r->window & 1], r->region, r->host.T, r->host.S, r->host.n_regions,
                               scratch, out, stream));
  if (mark) fence(stream);
  return RDX_OK;
}

rdx_status Engine::download_counts(const Run* r, int32_t* out, bool device, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  const size_t n = (size_t)r->host.S * (size_t)r->host.T;
  RDX_HIP(hipMemcpyAsync(out, r->cnt[r->window & 1], sizeof(int32_t) * n,
                         device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream));
  if (!device) RDX_HIP(hipStreamSynchronize(stream));
  return RDX_OK;
}

rdx_status Engine::plan_until(Run* r, double t_end, int64_t max_windows) {
  if (!std::isfinite(t_end)) return set_error(RDX_EINVAL, "t_end must be finite");
  const double tau = r->host.tau;
  double t = r->t;
  // the window index is a 32-bit field of the RNG counter: reject a horizon
  // that needs more windows than are left before counting them one by one
  const int64_t left = (int64_t)0xffffffffLL - r->window;
  const int64_t cap = max_windows < 0 ? left : std::min(max_windows, left + 1);
  if (t < t_end && (max_windows < 0 || max_windows > left)) {
    const double est = (t_end - t) / tau;  // windows to t_end, to within roundings
    if (!(est <= (double)left * (1.0 + 1e-9) + 2.0))
      return set_error(RDX_EINVAL, "window index exceeds the 32-bit RNG counter field");
  }
  int64_t steps = 0, full = 0;
  double tau_last = tau;
  while (t < t_end && steps <= cap && (max_windows < 0 || steps < max_windows)) {
    if (t + tau > t_end) {  // the last window is cut at t_end
      tau_last = t_end - t;
      t = t_end;
      steps += 1;
      break;
    }
    if (!(t + tau > t))  // tau below the resolution of t: the loop would not advance
      return set_error(RDX_EINVAL, "tau is below the floating-point resolution of t");
    t = t + tau;
    steps += 1;
    full += 1;
  }
  if (r->window + steps > (int64_t)0xffffffffLL)
    return set_error(RDX_EINVAL, "window index exceeds the 32-bit RNG counter field");
  r->plan_steps = steps;
  r->plan_full = full;
  r->plan_tau_last = tau_last;
  r->plan_t_after = t;
  return RDX_OK;
}

rdx_status Engine::plan_steps(Run* r, int64_t n) {
  if (n < 0) return set_error(RDX_EINVAL, "n_windows < 0");
  if (r->window + n > (int64_t)0xffffffffLL)
    return set_error(RDX_EINVAL, "window index exceeds the 32-bit RNG counter field");
  double t = r->t;
  for (int64_t k = 0; k < n; ++k) t = t + r->host.tau;
  r->plan_steps = n;
  r->plan_full = n;
  r->plan_tau_last = r->host.tau;
  r->plan_t_after = t;
  return RDX_OK;
}

namespace {
// Threshold of expected events (a0 tau_k) above which a listed tet goes to
// the heavy bin; with binning off every listed tet is light.
double heavy_events(const ExecShape& sh) { return sh.event_bins ? 1.0 : HUGE_VAL; }

// Fewest rounds of tiles `resident` blocks need, then the fewest blocks (a
// multiple of the 8 XCDs) that still finish in that many rounds.
int rounds_grid(int64_t n_tiles, int resident) {
  resident = std::max(8, resident);
  if (n_tiles < 1) return 1;
  const int64_t rounds = (n_tiles + resident - 1) / resident;
  int g = (int)((n_tiles + rounds - 1) / rounds);
  if (g >= 8) g = (g + 7) & ~7;
  if (g > resident) g = resident & ~7;
  return g > 0 ? g : 1;
}
}  // namespace

// Tile count rounded up to a coarse bucket (at most 1/8 above it): grids of
// engines whose set of runs changes between sequences (servers, batches
// whose runs finish at different times) then repeat, and so do the captured
// graphs keyed by them.  The kernels read the exact count from the device
// and leave surplus blocks idle.
static int64_t bucket_tiles(int64_t n) {
  if (n <= 64) return n;
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= n) ++lg;
  const int64_t g = int64_t(1) << (lg - 3);
  return (n + g - 1) / g * g;
}

void Engine::grids_for(int64_t n_tiles_exact, int div, int* detect, int* main) const {
  const int64_t n_tiles = max_runs_ > 1 ? bucket_tiles(n_tiles_exact) : n_tiles_exact;
  int rd = 0, rm = 0;
  grid_resident(S_, R_, &rd, &rm);
  // detect kernel: one block per tile (light blocks, many resident per SIMD,
  // so the latency of each tile's loads is hidden by the others)
  (void)rd;
  *detect = (int)std::max<int64_t>(1, std::min<int64_t>(n_tiles, 1 << 24));
  // main kernel: the diffusion blocks' grid plus room for the event blocks
  // (one per tile with listed tets, decided on the device), within what is
  // resident at once
  const int res = std::max(8, rm / std::max(1, div));
  const int reserve = std::min(256, std::max(8, res / 4));
  *main = std::max(2, std::min(res, rounds_grid(n_tiles, res) + reserve));
}

rdx_status Engine::upload_tables(const std::vector<Run*>& active, int64_t k0, hipStream_t stream,
                                 int64_t* n_tiles_out) {
  // the pinned images may still be in flight from the previous sequence
  RDX_HIP(hipEventSynchronize(staged_));
  const size_t n = active.size();
  for (size_t j = 0; j < n; ++j) {
    const Run* r = active[j];
    const HostInstance& I = r->host;
    RunDesc& d = h_runs_[j];
    std::memset(&d, 0, sizeof d);
    d.cnt[0] = r->cnt[0];
    d.cnt[1] = r->cnt[1];
    d.nbr = r->nbr;
    d.geo = r->geo;
    d.nav = r->nav;
    d.region = r->region;
    d.kcst = r->kcst;
    d.lcoef = r->lcoef;
    d.tally = r->tally;
    d.err = r->err;
    d.T = I.T;
    d.n_steps = (int32_t)(k0 + r->plan_steps);
    d.n_full = (int32_t)(k0 + r->plan_full);
    d.window0 = (uint32_t)((uint64_t)r->window - (uint64_t)k0);
    d.key0 = (uint32_t)(r->seed & 0xffffffffu);
    d.key1 = (uint32_t)(r->seed >> 32);
    d.tau = I.tau;
    d.tau_last = r->plan_tau_last;
    for (int s = 0; s < I.S; ++s) d.D[s] = I.D[s];
  }
  RDX_HIP(hipMemcpyAsync(d_runs_, h_runs_, sizeof(RunDesc) * n, hipMemcpyHostToDevice, stream));
  // tile map: rebuilt only when the set of runs changes
  bool same = tile_runs_.size() == n;
  for (size_t j = 0; same && j < n; ++j) same = tile_runs_[j] == active[j] && tile_run_T_[j] == active[j]->host.T;
  int64_t n_tiles = 0;
  for (const Run* r : active) n_tiles += (r->host.T + 63) / 64;
  if (n_tiles > max_tiles_) return set_error(RDX_EINVAL, "tile map capacity exceeded");
  if (!same) {
    int64_t t = 0;
    for (size_t j = 0; j < n; ++j)
      for (int32_t first = 0; first < active[j]->host.T; first += 64) h_tile_map_[t++] = make_int2((int)j, first);
    RDX_HIP(hipMemcpyAsync(d_tile_map_, h_tile_map_, sizeof(int2) * (size_t)n_tiles, hipMemcpyHostToDevice, stream));
    tile_runs_.assign(active.begin(), active.end());
    tile_run_T_.resize(n);
    for (size_t j = 0; j < n; ++j) tile_run_T_[j] = active[j]->host.T;
  }
  *h_n_tiles_ = (int32_t)n_tiles;
  RDX_HIP(hipMemcpyAsync(d_n_tiles_, h_n_tiles_, sizeof(int32_t), hipMemcpyHostToDevice, stream));
  *n_tiles_out = n_tiles;
  RDX_HIP(hipEventRecord(staged_, stream));
  return RDX_OK;
}

rdx_status Engine::launch_plain(const StepArgs& a0, int64_t K, hipStream_t stream) {
  StepArgs a = a0;
  for (int64_t k = 0; k < K; ++k) {
    a.k_rel = (int32_t)k;
    hipEvent_t* marks = nullptr;
    if (timing_) {
      while (marks_.size() < marks_used_ + 3) {
        hipEvent_t ev;
        RDX_HIP(hipEventCreate(&ev));
        marks_.push_back(ev);
      }
      marks = marks_.data() + marks_used_;
      marks_used_ += 3;
    }
    hipError_t e = launch_window(a, stream, marks);
    if (e != hipSuccess) return set_error(RDX_EHIP, std::string("window launch: ") + hipGetErrorString(e));
    if (rec_on_ && (k + 1) % rec_.every == 0) {
      // the counts after this window sit in buffer (window + k + 1) & 1 (the
      // run's window index advances when the sequence ends); the next window
      // clears that buffer only after this reduction in stream order
      const Run* r = rec_.run;
      const int64_t slot = (int64_t)r->host.n_regions * r->host.S;
      unsigned long long* out = rec_.ring + (rec_.records % rec_.slots) * slot;
      e = launch_region_counts(r->cnt[(r->window + k + 1) & 1], r->region, r->host.T, r->host.S,
                               r->host.n_regions, rec_.scratch, out, stream);
      if (e != hipSuccess) return set_error(RDX_EHIP, std::string("record launch: ") + hipGetErrorString(e));
      rec_.records += 1;
    }
  }
  if (K > 0) RDX_HIP(launch_advance_base(d_base_, (int32_t)K, stream));
  return RDX_OK;
}

rdx_status Engine::launch_graphs(const StepArgs& a0, int64_t reps, hipStream_t stream) {
  const int W = shape_.graph_windows;
  // everything of the arguments that can change between sequences is in the
  // key (pointers and tables are fixed for the engine's life)
  const long long shape_key = ((long long)a0.main_grid << 40) | ((long long)(a0.tile_claim ? 1 : 0) << 35) |
                              ((long long)a0.detect_grid << 9) |
                              ((long long)(a0.heavy_events < 1e300 ? 1 : 0) << 8) |
                              ((long long)a0.ev_group_max << 1) | (long long)a0.single_run;
  const auto key = std::make_pair(W, shape_key);
  auto it = graphs_.find(key);
  if (it == graphs_.end()) {
    if (graphs_.size() >= 16) free_graphs();
    if (!capture_stream_) RDX_HIP(hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking));
    // W windows and the step-base advance, captured once on a private stream
    StepArgs a = a0;
    RDX_HIP(hipStreamBeginCapture(capture_stream_, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < W && e == hipSuccess; ++k) {
      a.k_rel = k;
      e = launch_window(a, capture_stream_, nullptr);
    }
    if (e == hipSuccess) e = launch_advance_base(d_base_, W, capture_stream_);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(capture_stream_, &graph);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return set_error(RDX_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    it = graphs_.emplace(key, exec).first;
  }
  for (int64_t r = 0; r < reps; ++r) RDX_HIP(hipGraphLaunch(it->second, stream));
  return RDX_OK;
}

void Engine::set_autotune(bool on) {
  tuning_ = on;
  candidates_.clear();
  cand_ms_.clear();
  cand_next_ = 0;
  if (!on) return;
  // the first entry is a warm-up of the default shape and is not scored;
  // then every shape three times, in three passes, each scored by its best
  // pass, so that a drift of the per-window cost over the tuning windows (a
  // simulation relaxing from its initial counts) biases the choice less
  // (with two passes the batched ensemble settled on a shape 3.7% slower)
  const ExecShape shapes[] = {ExecShape{1, 1, 4},        ExecShape{2, 1, 4},       ExecShape{1, 8, 4},
                              ExecShape{2, 8, 4},        ExecShape{4, 8, 4},       ExecShape{1, 8, 8},
                              ExecShape{1, 8, 16},       ExecShape{1, 8, 64},      ExecShape{1, 1, 64},
                              ExecShape{1, 1, 4, 1, 1},  ExecShape{1, 8, 16, 1, 1}};
  candidates_.push_back(shapes[0]);
  for (int pass = 0; pass < 3; ++pass)
    for (const ExecShape& c : shapes) candidates_.push_back(c);
}

rdx_status Engine::sequence(const std::vector<Run*>& runs, hipStream_t stream) {
  FenceOnExit fence_on_exit{this, stream};
  std::vector<Run*> active;
  int64_t K = 0;
  for (Run* r : runs)
    if (r->plan_steps > 0) {
      if (r->arena_off == SIZE_MAX) return set_error(RDX_ESTATE, "run is not resident");
      active.push_back(r);
      K = std::max(K, r->plan_steps);
    }
  if (active.empty()) return RDX_OK;
  if ((int)active.size() > max_runs_) return set_error(RDX_EINVAL, "too many runs in one sequence");

  int64_t k0 = k_now_;
  if (k0 + K >= kStepRebase) {
    if (K >= kStepRebase) return set_error(RDX_EINVAL, "sequence too long");
    k0 = k_now_ & 1;  // keep the parity of the worklist counters
    RDX_HIP(launch_set_base(d_base_, (int32_t)k0, stream));
  }
  int64_t n_tiles = 0;
  rdx_status st = upload_tables(active, k0, stream, &n_tiles);
  if (st != RDX_OK) return st;

  StepArgs a;
  std::memset(&a, 0, sizeof a);
  a.runs = d_runs_;
  a.tile_map = d_tile_map_;
  a.n_tiles = d_n_tiles_;
  a.step_base = d_base_;
  a.S = S_;
  a.R = R_;
  a.wl_mask = wl_mask_;
  a.model = model_;
  std::memcpy(a.info, model_host_.info, sizeof a.info);
  {
    int32_t pair_of[32];
    listing_pairs(model_host_, a.pairs, &a.n_pairs, pair_of);
  }
  a.single_run = active.size() == 1 ? 1 : 0;
  a.wl_tile_count = wl_tile_count_;
  a.evq = evq_;
  a.evq_cap = (int32_t)((max_tiles_ + kQueues - 1) / kQueues);
  a.evq_count = evq_count_;
  a.wl_tet = wl_tet_;
  a.tile_ctr = tile_ctr_;

  auto run_chunk = [&](const ExecShape& sh, int64_t n) -> rdx_status {
    grids_for(n_tiles, sh.fast_grid_div, &a.detect_grid, &a.main_grid);
    a.ev_group_max = sh.event_group;
    a.heavy_events = heavy_events(sh);
    a.tile_claim = sh.tile_claim;
    const ExecShape keep = shape_;
    shape_ = sh;
    rdx_status r = RDX_OK;
    if (!timing_ && sh.graph_windows > 1 && n >= sh.graph_windows) {
      const int64_t reps = n / sh.graph_windows;
      r = launch_graphs(a, reps, stream);
      if (r == RDX_OK) r = launch_plain(a, n - reps * sh.graph_windows, stream);
    } else {
      r = launch_plain(a, n, stream);
    }
    shape_ = keep;
    return r;
  };

  int64_t done = 0;
  if (rec_on_) {  // records between windows: plain launches at the current shape
    grids_for(n_tiles, shape_.fast_grid_div, &a.detect_grid, &a.main_grid);
    a.ev_group_max = shape_.event_group;
    a.heavy_events = heavy_events(shape_);
    a.tile_claim = shape_.tile_claim;
    st = launch_plain(a, K, stream);
    if (st != RDX_OK) return st;
    done = K;
  }
  while (tuning_ && !timing_ && done < K && cand_next_ < candidates_.size()) {
    const ExecShape c = candidates_[cand_next_];
    const int64_t n = std::min<int64_t>(K - done, std::max(8, 2 * c.graph_windows));
    if (c.graph_windows > 1 && n >= c.graph_windows) {  // capture outside the timed span
      grids_for(n_tiles, c.fast_grid_div, &a.detect_grid, &a.main_grid);
      a.ev_group_max = c.event_group;
      a.heavy_events = heavy_events(c);
      a.tile_claim = c.tile_claim;
      const ExecShape keep = shape_;
      shape_ = c;
      st = launch_graphs(a, 0, stream);
      shape_ = keep;
      if (st != RDX_OK) return st;
    }
    RDX_HIP(hipEventRecord(tune_ev_[0], stream));
    st = run_chunk(c, n);
    if (st != RDX_OK) return st;
    RDX_HIP(hipEventRecord(tune_ev_[1], stream));
    RDX_HIP(hipEventSynchronize(tune_ev_[1]));
    float ms = 0.f;
    RDX_HIP(hipEventElapsedTime(&ms, tune_ev_[0], tune_ev_[1]));
    if (cand_next_ > 0) {
      const double per = (double)ms / (double)n;
      auto f = cand_ms_.find(c);
      cand_ms_[c] = f == cand_ms_.end() ? per : std::min(f->second, per);
    }
    done += n;
    cand_next_ += 1;
    if (cand_next_ == candidates_.size()) {
      ExecShape best = candidates_[0];
      double best_ms = 1e300;
      for (const auto& kv : cand_ms_)
        if (kv.second < best_ms) {
          best_ms = kv.second;
          best = kv.first;
        }
      shape_ = best;
      tuning_ = false;
    }
  }
  if (done < K) {
    st = run_chunk(shape_, K - done);
    if (st != RDX_OK) return st;
  }
  k_now_ = k0 + K;

  for (Run* r : active) {
    r->t = r->plan_t_after;
    r->window += r->plan_steps;
    r->windows_run += r->plan_steps;
    r->voxel_steps += r->plan_steps * (int64_t)r->host.T;
    r->plan_steps = r->plan_full = 0;
  }
  return RDX_OK;
}

rdx_status Engine::kernel_times(rdx_kernel_times* out, bool reset) {
  for (size_t k = 0; k + 3 <= marks_used_; k += 3) {
    RDX_HIP(hipEventSynchronize(marks_[k + 2]));
    float a = 0.f, b = 0.f;
    RDX_HIP(hipEventElapsedTime(&a, marks_[k], marks_[k + 1]));
    RDX_HIP(hipEventElapsedTime(&b, marks_[k + 1], marks_[k + 2]));
    detect_ms_ += a;
    main_ms_ += b;
    timed_windows_ += 1;
  }
  marks_used_ = 0;
  out->windows = timed_windows_;
  out->detect_ms = detect_ms_;
  out->main_ms = main_ms_;
  if (reset) {
    timed_windows_ = 0;
    detect_ms_ = main_ms_ = 0.0;
  }
  return RDX_OK;
}

rdx_status Engine::run_error(const Run* r) const {
  // on the engine's own stream: a copy on the legacy default stream is refused
  // while any other thread holds a blocking stream in graph capture
  int32_t flags = 0;
  RDX_HIP(hipMemcpyAsync(&flags, r->err, sizeof flags, hipMemcpyDeviceToHost, own_));
  RDX_HIP(hipStreamSynchronize(own_));
  if (flags & kErrOverflow) return set_error(RDX_EOVERFLOW, "a molecule count passed 2^30");
  if (flags & kErrEvents) return set_error(RDX_EEVENTS, "more than 2^22 SSA events in one tet window");
  return RDX_OK;
}

rdx_status Engine::read_run_async(const Run* r, Readout* out, hipStream_t stream) const {
  RDX_HIP(hipMemcpyAsync(&out->err, r->err, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  RDX_HIP(hipMemcpyAsync(out->slots, r->tally, sizeof out->slots, hipMemcpyDeviceToHost, stream));
  return RDX_OK;
}

rdx_status Engine::decode_readout(const Readout& in, unsigned long long tal[3]) {
  tal[0] = tal[1] = tal[2] = 0;
  for (int j = 0; j < kTallySlots; ++j)
    for (int q = 0; q < 3; ++q) tal[q] += in.slots[kTallyWords * j + q];
  if (in.err & kErrOverflow) return set_error(RDX_EOVERFLOW, "a molecule count passed 2^30");
  if (in.err & kErrEvents) return set_error(RDX_EEVENTS, "more than 2^22 SSA events in one tet window");
  return RDX_OK;
}

rdx_status Engine::run_tally(const Run* r, unsigned long long tal[3]) const {
  unsigned long long slots[kTallyWords * kTallySlots];
  RDX_HIP(hipMemcpyAsync(slots, r->tally, sizeof slots, hipMemcpyDeviceToHost, own_));
  RDX_HIP(hipStreamSynchronize(own_));
  tal[0] = tal[1] = tal[2] = 0;
  for (int j = 0; j < kTallySlots; ++j)
    for (int q = 0; q < 3; ++q) tal[q] += slots[kTallyWords * j + q];
  return RDX_OK;
}

}  // namespace rdx
