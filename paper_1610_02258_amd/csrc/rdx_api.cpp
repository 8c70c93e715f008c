// rdx_api.cpp -- the C ABI declared in include/rdx.h: simulation objects,
// device state, the runtime main loop of "Parallel STEPS" (Algorithm 1) as a
// host loop over window launches, checkpoints and error reporting.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rdx.h"
#include "rdx_internal.hpp"
#include "rdx_kernels.hpp"

namespace rdx {

namespace {
thread_local std::string g_last_error;
}

rdx_status set_error(rdx_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

}  // namespace rdx

using namespace rdx;

// Device state of one simulation.  Counts are double-buffered: the window
// reads (and zeroes) cnt[cur] and accumulates the new counts into cnt[1-cur].
struct rdx_sim {
  HostInstance host;
  int device = 0;
  uint64_t seed = 0;
  int32_t* cnt[2] = {nullptr, nullptr};
  int cur = 0;
  int32_t* nbr = nullptr;
  double* geo = nullptr;        // (G, cum0, cum1, cum2) per tet
  double* nav = nullptr;
  uint8_t* region = nullptr;
  DevModel* model = nullptr;
  unsigned long long* tally = nullptr;   // [2] events, moves
  int* err = nullptr;
  int32_t* wl_tet = nullptr;    // [T] tets with an SSA event in the current window
  int32_t* wl_cnt = nullptr;    // [S][T] their counts at the window start
  double* wl_nav = nullptr;     // [T] their N_A V[L]
  int32_t* wl_nbr = nullptr;    // [T][4] their neighbours
  double* wl_geo = nullptr;     // [T][4] their couplings
  int32_t* wl_count = nullptr;  // [2] list lengths, alternating by window parity
  KModel km;
  // per-kernel timing: three events per window, recycled after each read
  bool timing = false;
  std::vector<hipEvent_t> marks;
  size_t marks_used = 0;
  int64_t timed_windows = 0;
  double fast_ms = 0.0, event_ms = 0.0;
  double t = 0.0;
  int64_t window = 0;
  int64_t windows_run = 0;
  int64_t voxel_steps = 0;
  bool has_counts = false;
};

namespace {

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

void free_device(rdx_sim* s) {
  for (hipEvent_t e : s->marks) (void)hipEventDestroy(e);
  s->marks.clear();
  (void)hipFree(s->cnt[0]);
  (void)hipFree(s->cnt[1]);
  (void)hipFree(s->nbr);
  (void)hipFree(s->geo);
  (void)hipFree(s->nav);
  (void)hipFree(s->region);
  (void)hipFree(s->model);
  (void)hipFree(s->tally);
  (void)hipFree(s->err);
  (void)hipFree(s->wl_tet);
  (void)hipFree(s->wl_cnt);
  (void)hipFree(s->wl_count);
  (void)hipFree(s->wl_nav);
  (void)hipFree(s->wl_nbr);
  (void)hipFree(s->wl_geo);
}

DevModel make_dev_model(const HostInstance& I) {
  DevModel m;
  std::memset(&m, 0, sizeof m);
  m.S = I.S;
  m.R = I.R;
  m.n_regions = I.n_regions;
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
    for (int reg = 0; reg < I.n_regions; ++reg) m.kcst[reg][r] = I.kcst[(size_t)reg * R + r];
  }
  // deps(R): reactions whose propensity reads a species that r changes
  for (int r = 0; r < R; ++r) {
    unsigned long long mask = 0;
    for (int j = 0; j < R; ++j)
      for (int s = 0; s < S; ++s)
        if (m.delta[r][s] != 0 && I.lhs[(size_t)j * S + s] > 0) mask |= 1ull << j;
    m.deps[r] = mask;
  }
  return m;
}

rdx_status check_sim(const rdx_sim* s) {
  if (!s) return set_error(RDX_EINVAL, "null simulation handle");
  return RDX_OK;
}

rdx_status launch_one(rdx_sim* s, double tau_k, hipStream_t stream) {
  if (s->window > (int64_t)0xffffffffLL)
    return set_error(RDX_EINVAL, "window index exceeds the 32-bit RNG counter field");
  const HostInstance& I = s->host;
  WindowArgs a;
  std::memset(&a, 0, sizeof a);
  a.cnt_in = s->cnt[s->cur];
  a.cnt_out = s->cnt[1 - s->cur];
  a.nbr = s->nbr;
  a.geo = s->geo;
  a.nav = s->nav;
  a.region = I.n_regions > 1 ? s->region : nullptr;
  a.model = s->model;
  a.tally = s->tally;
  a.err = s->err;
  a.T = I.T;
  a.S = I.S;
  a.R = I.R;
  a.key0 = (uint32_t)(s->seed & 0xffffffffu);
  a.key1 = (uint32_t)(s->seed >> 32);
  a.window = (uint32_t)s->window;
  a.tau_k = tau_k;
  for (int sp = 0; sp < I.S; ++sp) a.tauD[sp] = tau_k * I.D[sp];
  a.wl_tet = s->wl_tet;
  a.wl_cnt = s->wl_cnt;
  a.wl_nav = s->wl_nav;
  a.wl_nbr = s->wl_nbr;
  a.wl_geo = s->wl_geo;
  a.wl_count = s->wl_count + (s->window & 1);
  a.wl_reset = s->wl_count + ((s->window + 1) & 1);
  a.event_blocks = std::max(1, std::min((I.T + 63) / 64, 1024));
  a.km = s->km;
  hipEvent_t* marks = nullptr;
  if (s->timing) {
    while (s->marks.size() < s->marks_used + 3) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return set_error(RDX_EHIP, "hipEventCreate failed");
      s->marks.push_back(ev);
    }
    marks = s->marks.data() + s->marks_used;
    s->marks_used += 3;
  }
  hipError_t e = launch_window(a, stream, marks);
  if (e != hipSuccess) return set_error(RDX_EHIP, std::string("window launch: ") + hipGetErrorString(e));
  s->cur = 1 - s->cur;
  s->window += 1;
  s->windows_run += 1;
  s->voxel_steps += I.T;
  return RDX_OK;
}

}  // namespace

extern "C" {

int32_t rdx_version(void) { return 100; }

const char* rdx_last_error(void) { return g_last_error.c_str(); }

rdx_status rdx_create(const rdx_mesh* mesh, const rdx_model* model, uint64_t seed,
                      double tau_override, rdx_sim** out) {
  clear_error();
  if (!out) return set_error(RDX_EINVAL, "null output handle");
  *out = nullptr;
  rdx_sim* s = new (std::nothrow) rdx_sim();
  if (!s) return set_error(RDX_ENOMEM, "host allocation failed");
  std::string err;
  rdx_status st = build_instance(mesh, model, tau_override, &s->host, &err);
  if (st != RDX_OK) {
    delete s;
    return set_error(st, err);
  }
  s->seed = seed;
  (void)hipGetDevice(&s->device);
  const HostInstance& I = s->host;
  const size_t T = (size_t)I.T, S = (size_t)I.S;
  std::vector<double> geo(4 * T);
  for (size_t i = 0; i < T; ++i) {
    geo[4 * i + 0] = I.G[i];
    geo[4 * i + 1] = I.cum[4 * i + 0];
    geo[4 * i + 2] = I.cum[4 * i + 1];
    geo[4 * i + 3] = I.cum[4 * i + 2];
  }
  DevModel dm = make_dev_model(I);
  std::memset(&s->km, 0, sizeof s->km);
  for (int r = 0; r < I.R; ++r) {
    s->km.info[r] = dm.info[r];
    s->km.kcst0[r] = dm.kcst[0][r];
  }
  bool ok = dev_alloc(&s->cnt[0], S * T) == hipSuccess && dev_alloc(&s->cnt[1], S * T) == hipSuccess &&
            dev_alloc(&s->nbr, 4 * T) == hipSuccess && dev_alloc(&s->geo, 4 * T) == hipSuccess &&
            dev_alloc(&s->nav, T) == hipSuccess && dev_alloc(&s->region, T) == hipSuccess &&
            dev_alloc(&s->model, 1) == hipSuccess && dev_alloc(&s->tally, 2) == hipSuccess &&
            dev_alloc(&s->err, 1) == hipSuccess && dev_alloc(&s->wl_tet, T) == hipSuccess &&
            dev_alloc(&s->wl_cnt, S * T) == hipSuccess && dev_alloc(&s->wl_count, 2) == hipSuccess &&
            dev_alloc(&s->wl_nav, T) == hipSuccess && dev_alloc(&s->wl_nbr, 4 * T) == hipSuccess &&
            dev_alloc(&s->wl_geo, 4 * T) == hipSuccess;
  if (!ok) {
    free_device(s);
    delete s;
    (void)hipGetLastError();
    return set_error(RDX_ENOMEM, "device allocation failed");
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(s->nbr, I.nbr.data(), sizeof(int32_t) * 4 * T, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->geo, geo.data(), sizeof(double) * 4 * T, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->nav, I.nav.data(), sizeof(double) * T, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->region, I.region.data(), T, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->model, &dm, sizeof dm, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(s->cnt[0], 0, sizeof(int32_t) * S * T);
  if (e == hipSuccess) e = hipMemset(s->cnt[1], 0, sizeof(int32_t) * S * T);
  if (e == hipSuccess) e = hipMemset(s->tally, 0, sizeof(unsigned long long) * 2);
  if (e == hipSuccess) e = hipMemset(s->err, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(s->wl_count, 0, 2 * sizeof(int32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_device(s);
    delete s;
    return set_error(RDX_EHIP, std::string("upload: ") + hipGetErrorString(e));
  }
  *out = s;
  return RDX_OK;
}

void rdx_destroy(rdx_sim* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  free_device(s);
  delete s;
}

rdx_status rdx_set_counts(rdx_sim* s, const int32_t* counts, int is_device_ptr, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!counts) return set_error(RDX_EINVAL, "null counts");
  (void)hipSetDevice(s->device);
  const size_t n = (size_t)s->host.S * (size_t)s->host.T;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (!is_device_ptr) {
    for (size_t x = 0; x < n; ++x)
      if (counts[x] < 0 || counts[x] > kCountCap)
        return set_error(RDX_EINVAL, "counts must lie in [0, 2^30]");
    RDX_HIP(hipMemcpyAsync(s->cnt[0], counts, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  } else {
    RDX_HIP(hipMemcpyAsync(s->cnt[0], counts, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  }
  RDX_HIP(hipMemsetAsync(s->cnt[1], 0, sizeof(int32_t) * n, st));
  RDX_HIP(hipMemsetAsync(s->tally, 0, sizeof(unsigned long long) * 2, st));
  RDX_HIP(hipMemsetAsync(s->err, 0, sizeof(int), st));
  RDX_HIP(hipMemsetAsync(s->wl_count, 0, 2 * sizeof(int32_t), st));
  if (!is_device_ptr) RDX_HIP(hipStreamSynchronize(st));
  s->cur = 0;
  s->t = 0.0;
  s->window = 0;
  s->windows_run = 0;
  s->voxel_steps = 0;
  s->has_counts = true;
  return RDX_OK;
}

rdx_status rdx_get_counts(rdx_sim* s, int32_t* out, int is_device_ptr, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null output");
  (void)hipSetDevice(s->device);
  const size_t n = (size_t)s->host.S * (size_t)s->host.T;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RDX_HIP(hipMemcpyAsync(out, s->cnt[s->cur], sizeof(int32_t) * n,
                         is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  if (!is_device_ptr) RDX_HIP(hipStreamSynchronize(st));
  return RDX_OK;
}

rdx_status rdx_run(rdx_sim* s, double t_end, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!std::isfinite(t_end)) return set_error(RDX_EINVAL, "t_end must be finite");
  (void)hipSetDevice(s->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const double tau = s->host.tau;
  while (s->t < t_end) {
    double tau_k = tau;
    bool truncated = false;
    if (s->t + tau_k > t_end) {
      tau_k = t_end - s->t;
      truncated = true;
    }
    rdx_status r = launch_one(s, tau_k, st);
    if (r != RDX_OK) return r;
    s->t = truncated ? t_end : s->t + tau_k;
  }
  return RDX_OK;
}

rdx_status rdx_step(rdx_sim* s, int64_t n_windows, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (n_windows < 0) return set_error(RDX_EINVAL, "n_windows < 0");
  (void)hipSetDevice(s->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int64_t k = 0; k < n_windows; ++k) {
    rdx_status r = launch_one(s, s->host.tau, st);
    if (r != RDX_OK) return r;
    s->t = s->t + s->host.tau;
  }
  return RDX_OK;
}

rdx_status rdx_sync(rdx_sim* s, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(s->device);
  RDX_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  int flags = 0;
  RDX_HIP(hipMemcpy(&flags, s->err, sizeof(int), hipMemcpyDeviceToHost));
  if (flags & kErrOverflow) return set_error(RDX_EOVERFLOW, "a molecule count passed 2^30");
  if (flags & kErrEvents) return set_error(RDX_EEVENTS, "more than 2^22 SSA events in one tet window");
  return RDX_OK;
}

rdx_status rdx_get_stats(rdx_sim* s, rdx_stats* out, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null stats");
  rdx_status st = rdx_sync(s, stream);
  unsigned long long tal[2] = {0, 0};
  RDX_HIP(hipMemcpy(tal, s->tally, sizeof tal, hipMemcpyDeviceToHost));
  out->windows = s->windows_run;
  out->voxel_steps = s->voxel_steps;
  out->ssa_events = (int64_t)tal[0];
  out->moves = (int64_t)tal[1];
  out->t = s->t;
  out->window_index = s->window;
  return st;
}

rdx_status rdx_get_tau(const rdx_sim* s, double* tau) {
  if (!s || !tau) return set_error(RDX_EINVAL, "null argument");
  *tau = s->host.tau;
  return RDX_OK;
}

rdx_status rdx_get_sizes(const rdx_sim* s, int32_t* n_tets, int32_t* n_species, int32_t* n_reactions) {
  if (!s) return set_error(RDX_EINVAL, "null simulation handle");
  if (n_tets) *n_tets = s->host.T;
  if (n_species) *n_species = s->host.S;
  if (n_reactions) *n_reactions = s->host.R;
  return RDX_OK;
}

rdx_status rdx_get_geometry(const rdx_sim* s, int32_t* nbr, double* g, double* G, double* cum,
                            double* nav) {
  if (!s) return set_error(RDX_EINVAL, "null simulation handle");
  const HostInstance& I = s->host;
  const size_t T = (size_t)I.T;
  if (nbr) std::memcpy(nbr, I.nbr.data(), sizeof(int32_t) * 4 * T);
  if (g) std::memcpy(g, I.g.data(), sizeof(double) * 4 * T);
  if (G) std::memcpy(G, I.G.data(), sizeof(double) * T);
  if (cum) std::memcpy(cum, I.cum.data(), sizeof(double) * 4 * T);
  if (nav) std::memcpy(nav, I.nav.data(), sizeof(double) * T);
  return RDX_OK;
}

rdx_status rdx_set_kernel_timing(rdx_sim* s, int enable) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  s->timing = enable != 0;
  return RDX_OK;
}

rdx_status rdx_get_kernel_times(rdx_sim* s, rdx_kernel_times* out, int reset) {
  clear_error();
  if (check_sim(s) != RDX_OK || !out) return set_error(RDX_EINVAL, "null argument");
  (void)hipSetDevice(s->device);
  for (size_t k = 0; k + 3 <= s->marks_used; k += 3) {
    RDX_HIP(hipEventSynchronize(s->marks[k + 2]));
    float a = 0.f, b = 0.f;
    RDX_HIP(hipEventElapsedTime(&a, s->marks[k], s->marks[k + 1]));
    RDX_HIP(hipEventElapsedTime(&b, s->marks[k + 1], s->marks[k + 2]));
    s->fast_ms += a;
    s->event_ms += b;
    s->timed_windows += 1;
  }
  s->marks_used = 0;
  out->windows = s->timed_windows;
  out->all_tets_ms = s->fast_ms;
  out->event_ms = s->event_ms;
  if (reset) {
    s->timed_windows = 0;
    s->fast_ms = s->event_ms = 0.0;
  }
  return RDX_OK;
}

rdx_status rdx_setup_geometry(const rdx_mesh* mesh, const rdx_model* model, double tau_override,
                              int32_t* nbr, double* g, double* G, double* cum, double* nav,
                              double* tau) {
  clear_error();
  HostInstance I;
  std::string err;
  rdx_status st = build_instance(mesh, model, tau_override, &I, &err);
  if (st != RDX_OK) return set_error(st, err);
  const size_t T = (size_t)I.T;
  if (nbr) std::memcpy(nbr, I.nbr.data(), sizeof(int32_t) * 4 * T);
  if (g) std::memcpy(g, I.g.data(), sizeof(double) * 4 * T);
  if (G) std::memcpy(G, I.G.data(), sizeof(double) * T);
  if (cum) std::memcpy(cum, I.cum.data(), sizeof(double) * 4 * T);
  if (nav) std::memcpy(nav, I.nav.data(), sizeof(double) * T);
  if (tau) *tau = I.tau;
  return RDX_OK;
}

namespace {
struct CheckpointHeader {
  char magic[8];
  int32_t version, T, S, pad;
  uint64_t seed;
  double t, tau;
  int64_t window, windows_run, voxel_steps, events, moves;
};
}  // namespace

rdx_status rdx_save(rdx_sim* s, void* buf, size_t* len, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK || !len) return set_error(RDX_EINVAL, "null argument");
  const size_t n = (size_t)s->host.S * (size_t)s->host.T;
  const size_t need = sizeof(CheckpointHeader) + sizeof(int32_t) * n;
  if (!buf) {
    *len = need;
    return RDX_OK;
  }
  if (*len < need) return set_error(RDX_EINVAL, "checkpoint buffer too small");
  rdx_stats stt;
  rdx_status st = rdx_get_stats(s, &stt, stream);
  if (st != RDX_OK) return st;
  CheckpointHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "RDXCKPT1", 8);
  h.version = rdx_version();
  h.T = s->host.T;
  h.S = s->host.S;
  h.seed = s->seed;
  h.t = s->t;
  h.tau = s->host.tau;
  h.window = s->window;
  h.windows_run = s->windows_run;
  h.voxel_steps = s->voxel_steps;
  h.events = stt.ssa_events;
  h.moves = stt.moves;
  std::memcpy(buf, &h, sizeof h);
  RDX_HIP(hipMemcpy(static_cast<char*>(buf) + sizeof h, s->cnt[s->cur], sizeof(int32_t) * n,
                    hipMemcpyDeviceToHost));
  *len = need;
  return RDX_OK;
}

rdx_status rdx_load(rdx_sim* s, const void* buf, size_t len, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK || !buf) return set_error(RDX_EINVAL, "null argument");
  CheckpointHeader h;
  if (len < sizeof h) return set_error(RDX_EINVAL, "checkpoint too short");
  std::memcpy(&h, buf, sizeof h);
  const size_t n = (size_t)s->host.S * (size_t)s->host.T;
  if (std::memcmp(h.magic, "RDXCKPT1", 8) != 0 || h.T != s->host.T || h.S != s->host.S ||
      h.seed != s->seed || h.tau != s->host.tau || len < sizeof h + sizeof(int32_t) * n)
    return set_error(RDX_EINVAL, "checkpoint does not match this simulation");
  rdx_status st = rdx_set_counts(s, reinterpret_cast<const int32_t*>(static_cast<const char*>(buf) + sizeof h),
                                 0, stream);
  if (st != RDX_OK) return st;
  unsigned long long tal[2] = {(unsigned long long)h.events, (unsigned long long)h.moves};
  RDX_HIP(hipMemcpy(s->tally, tal, sizeof tal, hipMemcpyHostToDevice));
  s->t = h.t;
  s->window = h.window;
  s->windows_run = h.windows_run;
  s->voxel_steps = h.voxel_steps;
  return RDX_OK;
}

rdx_status rdx_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n) {
  clear_error();
  if (!in || !out || n <= 0) return set_error(RDX_EINVAL, "bad arguments");
  uint32_t *din = nullptr, *dout = nullptr;
  RDX_HIP(hipMalloc(&din, sizeof(uint32_t) * 6 * n));
  if (hipMalloc(&dout, sizeof(uint32_t) * 4 * n) != hipSuccess) {
    (void)hipFree(din);
    return set_error(RDX_ENOMEM, "device allocation failed");
  }
  hipError_t e = hipMemcpy(din, in, sizeof(uint32_t) * 6 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_selftest_philox(din, dout, n, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost);
  (void)hipFree(din);
  (void)hipFree(dout);
  if (e != hipSuccess) return set_error(RDX_EHIP, hipGetErrorString(e));
  return RDX_OK;
}

rdx_status rdx_selftest_ln(const double* x, double* y, int64_t n) {
  clear_error();
  if (!x || !y || n <= 0) return set_error(RDX_EINVAL, "bad arguments");
  double *dx = nullptr, *dy = nullptr;
  RDX_HIP(hipMalloc(&dx, sizeof(double) * n));
  if (hipMalloc(&dy, sizeof(double) * n) != hipSuccess) {
    (void)hipFree(dx);
    return set_error(RDX_ENOMEM, "device allocation failed");
  }
  hipError_t e = hipMemcpy(dx, x, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_selftest_ln(dx, dy, n, nullptr);
  if (e == hipSuccess) e = hipMemcpy(y, dy, sizeof(double) * n, hipMemcpyDeviceToHost);
  (void)hipFree(dx);
  (void)hipFree(dy);
  if (e != hipSuccess) return set_error(RDX_EHIP, hipGetErrorString(e));
  return RDX_OK;
}

rdx_status rdx_selftest_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m, double p,
                              int64_t n, int64_t* out) {
  clear_error();
  if (!out || n <= 0 || m < 0 || !(p >= 0.0)) return set_error(RDX_EINVAL, "bad arguments");
  long long* d = nullptr;
  RDX_HIP(hipMalloc(&d, sizeof(long long) * n));
  hipError_t e = launch_selftest_binom(seed, stream_id, window, m, p, n, d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, d, sizeof(long long) * n, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return set_error(RDX_EHIP, hipGetErrorString(e));
  return RDX_OK;
}

rdx_status rdx_selftest_copy(int64_t bytes, int32_t reps, double* gbps) {
  clear_error();
  if (bytes < 16 || reps < 1 || !gbps) return set_error(RDX_EINVAL, "bad arguments");
  const int64_t n16 = bytes / 16;
  int4 *a = nullptr, *b = nullptr;
  RDX_HIP(hipMalloc(&a, sizeof(int4) * n16));
  if (hipMalloc(&b, sizeof(int4) * n16) != hipSuccess) {
    (void)hipFree(a);
    return set_error(RDX_ENOMEM, "device allocation failed");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemset(a, 1, sizeof(int4) * n16);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_copy(a, b, n16, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(a, b, n16, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return set_error(RDX_EHIP, hipGetErrorString(e));
  *gbps = 2.0 * 16.0 * (double)n16 * reps / (ms * 1e-3) / 1e9;
  return RDX_OK;
}

}  // extern "C"
