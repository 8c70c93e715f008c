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
#include "rdx_engine.hpp"
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

// One simulation: an engine holding a single run.
struct rdx_sim {
  Engine eng;
  Run run;
  int device = 0;
  unsigned long long* rec = nullptr;  // device staging of region sums for host output
};

// A batch: one engine holding every run; all runs advance in the same launches.
struct rdx_batch {
  Engine eng;
  std::vector<Run> runs;
  int device = 0;
  unsigned long long* rec = nullptr;
};

namespace {

#define RDX_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_error(RDX_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

rdx_status check_sim(const rdx_sim* s) {
  if (!s) return set_error(RDX_EINVAL, "null simulation handle");
  return RDX_OK;
}

constexpr size_t kRecStage = sizeof(unsigned long long) * kMaxRegions * kMaxSpecies;

rdx_status set_rates_of(Engine& eng, Run& r, const double* kcst, int64_t n, hipStream_t stream) {
  const int64_t want = (int64_t)r.host.n_regions * (int64_t)r.host.R;
  if (n != want)
    return set_error(RDX_EINVAL, "the rate table has n_regions*n_reactions = " + std::to_string(want) +
                                     " entries, got " + std::to_string(n));
  if (want == 0) return RDX_OK;
  if (!kcst) return set_error(RDX_EINVAL, "null rate constants");
  return eng.set_rates(&r, kcst, stream);
}

rdx_status region_counts_of(Engine& eng, const Run& r, int64_t* out, bool device, unsigned long long** rec,
                            hipStream_t stream) {
  if (!out) return set_error(RDX_EINVAL, "null output");
  // one device buffer per handle, made at the first call: the partial sums,
  // then a staging copy of the result for host output
  if (!*rec) RDX_HIP(hipMalloc(reinterpret_cast<void**>(rec), kRegionScratchBytes + kRecStage));
  unsigned long long* stage = *rec + kRegionScratchBytes / sizeof(unsigned long long);
  if (device) return eng.region_counts(&r, *rec, reinterpret_cast<unsigned long long*>(out), stream);
  const rdx_status q = eng.region_counts(&r, *rec, stage, stream);
  if (q != RDX_OK) return q;
  const size_t n = (size_t)r.host.n_regions * (size_t)r.host.S;
  RDX_HIP(hipMemcpyAsync(out, stage, sizeof(int64_t) * n, hipMemcpyDeviceToHost, stream));
  RDX_HIP(hipStreamSynchronize(stream));
  return RDX_OK;
}

rdx_status check_counts(const int32_t* counts, size_t n) {
  for (size_t x = 0; x < n; ++x)
    if (counts[x] < 0 || counts[x] > kCountCap) return set_error(RDX_EINVAL, "counts must lie in [0, 2^30]");
  return RDX_OK;
}

// Counts at t = 0: the run restarts at window 0 with zero tallies.
rdx_status start_run(Engine& eng, Run& r, const int32_t* counts, bool device, hipStream_t st) {
  if (!device) {
    rdx_status c = check_counts(counts, (size_t)r.host.S * (size_t)r.host.T);
    if (c != RDX_OK) return c;
  }
  r.t = 0.0;
  r.window = 0;
  r.windows_run = 0;
  r.voxel_steps = 0;
  rdx_status q = eng.reset_run(&r, st);
  if (q == RDX_OK) q = eng.upload_counts(&r, counts, device, st);
  return q;
}

rdx_status fill_stats(Engine& eng, const Run& r, rdx_stats* out) {
  unsigned long long tal[3] = {0, 0, 0};
  rdx_status st = eng.run_tally(&r, tal);
  if (st != RDX_OK) return st;
  out->windows = r.windows_run;
  out->voxel_steps = r.voxel_steps;
  out->ssa_events = (int64_t)tal[0];
  out->moves = (int64_t)tal[1];
  out->face_moves = (int64_t)tal[2];
  out->t = r.t;
  out->window_index = r.window;
  return RDX_OK;
}

rdx_status apply_options(Engine& eng, const rdx_exec_options* o) {
  if (!o) return set_error(RDX_EINVAL, "null options");
  if (!(o->fast_grid_div == 1 || o->fast_grid_div == 2 || o->fast_grid_div == 4) || o->graph_windows < 1 ||
      o->graph_windows > 256 || o->event_group < 0 || o->event_group > 64)
    return set_error(RDX_EINVAL,
                     "fast_grid_div must be 1, 2 or 4, graph_windows in [1, 256], event_group in [0, 64]");
  if (o->event_bins < 0 || o->event_bins > 1) return set_error(RDX_EINVAL, "event_bins must be 0 or 1");
  if (o->tile_claim < 0 || o->tile_claim > 1) return set_error(RDX_EINVAL, "tile_claim must be 0 or 1");
  eng.set_shape(ExecShape{o->fast_grid_div, o->graph_windows, o->event_group ? o->event_group : 4, o->event_bins,
                          o->tile_claim});
  if (o->autotune) eng.set_autotune(true);
  return RDX_OK;
}

void read_options(const Engine& eng, rdx_exec_options* o) {
  o->autotune = eng.tuning() ? 1 : 0;
  o->fast_grid_div = eng.shape().fast_grid_div;
  o->graph_windows = eng.shape().graph_windows;
  o->event_group = eng.shape().event_group;
  o->event_bins = eng.shape().event_bins;
  o->tile_claim = eng.shape().tile_claim;
}

}  // namespace

extern "C" {

int32_t rdx_version(void) { return RDX_ABI_VERSION; }

const char* rdx_last_error(void) { return g_last_error.c_str(); }

rdx_status rdx_create(const rdx_mesh* mesh, const rdx_model* model, uint64_t seed,
                      double tau_override, rdx_sim** out) {
  clear_error();
  if (!out) return set_error(RDX_EINVAL, "null output handle");
  *out = nullptr;
  rdx_sim* s = new (std::nothrow) rdx_sim();
  if (!s) return set_error(RDX_ENOMEM, "host allocation failed");
  std::string err;
  rdx_status st = build_instance(mesh, model, tau_override, &s->run.host, &err);
  if (st != RDX_OK) {
    delete s;
    return set_error(st, err);
  }
  s->run.seed = seed;
  (void)hipGetDevice(&s->device);
  st = s->eng.init(s->run.host, Engine::run_bytes(s->run.host), 1, s->run.host.T);
  if (st == RDX_OK) st = s->eng.add_run(&s->run, s->eng.own_stream());
  if (st != RDX_OK) {
    const std::string msg = rdx_last_error();
    delete s;
    return set_error(st == RDX_EBUDGET ? RDX_ENOMEM : st, msg);
  }
  *out = s;
  return RDX_OK;
}

void rdx_destroy(rdx_sim* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  s->eng.drain();  // every stream the simulation used, not the whole device
  if (s->rec) (void)hipFree(s->rec);
  delete s;
}

rdx_status rdx_set_rate_constants(rdx_sim* s, const double* kcst, int64_t n, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(s->device);
  return set_rates_of(s->eng, s->run, kcst, n, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_region_counts(rdx_sim* s, int64_t* out, int is_device_ptr, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(s->device);
  return region_counts_of(s->eng, s->run, out, is_device_ptr != 0, &s->rec, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_region_counts_static(rdx_sim* s, int64_t* out, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null output");
  (void)hipSetDevice(s->device);
  unsigned long long* scratch = nullptr;
  size_t cap = 0;
  RDX_HIP(static_region_scratch(&scratch, &cap));
  const size_t need = region_scratch_bytes(s->run.host.T, s->run.host.S);
  if (need > cap)
    return set_error(RDX_EINVAL, "the region sums need " + std::to_string(need) + " bytes of scratch, more than the " +
                                     std::to_string(cap) + "-byte static array");
  return s->eng.region_counts(&s->run, scratch, reinterpret_cast<unsigned long long*>(out),
                              reinterpret_cast<hipStream_t>(stream), false);
}

rdx_status rdx_set_counts(rdx_sim* s, const int32_t* counts, int is_device_ptr, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!counts) return set_error(RDX_EINVAL, "null counts");
  (void)hipSetDevice(s->device);
  return start_run(s->eng, s->run, counts, is_device_ptr != 0, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_get_counts(rdx_sim* s, int32_t* out, int is_device_ptr, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null output");
  (void)hipSetDevice(s->device);
  return s->eng.download_counts(&s->run, out, is_device_ptr != 0, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_run(rdx_sim* s, double t_end, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!std::isfinite(t_end)) return set_error(RDX_EINVAL, "t_end must be finite");
  (void)hipSetDevice(s->device);
  rdx_status st = Engine::plan_until(&s->run, t_end, -1);
  if (st != RDX_OK) return st;
  return s->eng.sequence({&s->run}, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_step(rdx_sim* s, int64_t n_windows, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(s->device);
  rdx_status st = Engine::plan_steps(&s->run, n_windows);
  if (st != RDX_OK) return st;
  return s->eng.sequence({&s->run}, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_step_recorded(rdx_sim* s, int64_t n_windows, int64_t every, int64_t* ring, int64_t ring_slots,
                             int64_t* n_records, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (n_records) *n_records = 0;
  if (n_windows < 0 || every <= 0 || ring_slots <= 0 || !ring)
    return set_error(RDX_EINVAL, "n_windows >= 0, every > 0, ring_slots > 0 and a device ring are required");
  (void)hipSetDevice(s->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (n_windows == 0) return RDX_OK;
  if (!s->rec) RDX_HIP(hipMalloc(reinterpret_cast<void**>(&s->rec), kRegionScratchBytes + kRecStage));
  // one sequence of n_windows plain windows with the reductions launched
  // between them (one table upload for the whole call)
  Engine::RecordHook hook;
  hook.run = &s->run;
  hook.every = every;
  hook.scratch = s->rec;
  hook.ring = reinterpret_cast<unsigned long long*>(ring);
  hook.slots = ring_slots;
  rdx_status q = Engine::plan_steps(&s->run, n_windows);
  if (q != RDX_OK) return q;
  s->eng.set_record_hook(&hook);
  q = s->eng.sequence({&s->run}, st);
  const int64_t written = s->eng.records_written();
  s->eng.set_record_hook(nullptr);
  if (n_records) *n_records = written;
  return q;
}

rdx_status rdx_sync(rdx_sim* s, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(s->device);
  RDX_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  return s->eng.run_error(&s->run);
}

rdx_status rdx_get_stats(rdx_sim* s, rdx_stats* out, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null stats");
  rdx_status st = rdx_sync(s, stream);
  const std::string msg = rdx_last_error();
  rdx_status q = fill_stats(s->eng, s->run, out);
  if (q != RDX_OK) return q;
  if (st != RDX_OK) set_error(st, msg);
  return st;
}

rdx_status rdx_set_exec_options(rdx_sim* s, const rdx_exec_options* o) {
  clear_error();
  if (check_sim(s) != RDX_OK) return RDX_EINVAL;
  return apply_options(s->eng, o);
}

rdx_status rdx_get_exec_options(const rdx_sim* s, rdx_exec_options* o) {
  clear_error();
  if (!s || !o) return set_error(RDX_EINVAL, "null argument");
  read_options(s->eng, o);
  return RDX_OK;
}

rdx_status rdx_get_tau(const rdx_sim* s, double* tau) {
  if (!s || !tau) return set_error(RDX_EINVAL, "null argument");
  *tau = s->run.host.tau;
  return RDX_OK;
}

rdx_status rdx_get_sizes(const rdx_sim* s, int32_t* n_tets, int32_t* n_species, int32_t* n_reactions) {
  if (!s) return set_error(RDX_EINVAL, "null simulation handle");
  if (n_tets) *n_tets = s->run.host.T;
  if (n_species) *n_species = s->run.host.S;
  if (n_reactions) *n_reactions = s->run.host.R;
  return RDX_OK;
}

rdx_status rdx_get_geometry(const rdx_sim* s, int32_t* nbr, double* g, double* G, double* cum,
                            double* nav) {
  if (!s) return set_error(RDX_EINVAL, "null simulation handle");
  const HostInstance& I = s->run.host;
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
  s->eng.set_timing(enable != 0);
  return RDX_OK;
}

rdx_status rdx_get_kernel_times(rdx_sim* s, rdx_kernel_times* out, int reset) {
  clear_error();
  if (check_sim(s) != RDX_OK || !out) return set_error(RDX_EINVAL, "null argument");
  (void)hipSetDevice(s->device);
  return s->eng.kernel_times(out, reset != 0);
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
  int64_t window, windows_run, voxel_steps, events, moves, face_moves;
};
}  // namespace

rdx_status rdx_save(rdx_sim* s, void* buf, size_t* len, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK || !len) return set_error(RDX_EINVAL, "null argument");
  const Run& r = s->run;
  const size_t n = (size_t)r.host.S * (size_t)r.host.T;
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
  std::memcpy(h.magic, "RDXCKPT2", 8);
  h.version = rdx_version();
  h.T = r.host.T;
  h.S = r.host.S;
  h.seed = r.seed;
  h.t = r.t;
  h.tau = r.host.tau;
  h.window = r.window;
  h.windows_run = r.windows_run;
  h.voxel_steps = r.voxel_steps;
  h.events = stt.ssa_events;
  h.moves = stt.moves;
  h.face_moves = stt.face_moves;
  std::memcpy(buf, &h, sizeof h);
  st = s->eng.download_counts(&r, reinterpret_cast<int32_t*>(static_cast<char*>(buf) + sizeof h), false,
                              reinterpret_cast<hipStream_t>(stream));
  if (st != RDX_OK) return st;
  *len = need;
  return RDX_OK;
}

rdx_status rdx_load(rdx_sim* s, const void* buf, size_t len, void* stream) {
  clear_error();
  if (check_sim(s) != RDX_OK || !buf) return set_error(RDX_EINVAL, "null argument");
  CheckpointHeader h;
  if (len < sizeof h) return set_error(RDX_EINVAL, "checkpoint too short");
  std::memcpy(&h, buf, sizeof h);
  Run& r = s->run;
  const size_t n = (size_t)r.host.S * (size_t)r.host.T;
  if (std::memcmp(h.magic, "RDXCKPT2", 8) != 0 || h.T != r.host.T || h.S != r.host.S || h.seed != r.seed ||
      h.tau != r.host.tau || h.window < 0 || h.window > (int64_t)0xffffffffLL || len < sizeof h + sizeof(int32_t) * n)
    return set_error(RDX_EINVAL, "checkpoint does not match this simulation");
  const int32_t* counts = reinterpret_cast<const int32_t*>(static_cast<const char*>(buf) + sizeof h);
  rdx_status st = check_counts(counts, n);
  if (st != RDX_OK) return st;
  (void)hipSetDevice(s->device);
  hipStream_t strm = reinterpret_cast<hipStream_t>(stream);
  // the counts go to the buffer of the restored window index
  r.window = h.window;
  st = s->eng.reset_run(&r, strm);
  if (st == RDX_OK) st = s->eng.upload_counts(&r, counts, false, strm);
  if (st != RDX_OK) return st;
  unsigned long long tal[3] = {(unsigned long long)h.events, (unsigned long long)h.moves,
                               (unsigned long long)h.face_moves};
  // into slot 0, behind the clearing of the tallies on the same stream
  RDX_HIP(hipMemcpyAsync(r.tally, tal, sizeof tal, hipMemcpyHostToDevice, strm));
  RDX_HIP(hipStreamSynchronize(strm));
  r.t = h.t;
  r.windows_run = h.windows_run;
  r.voxel_steps = h.voxel_steps;
  return RDX_OK;
}

// ------------------------------------------------------------------ batch ----
rdx_status rdx_batch_create(int32_t n_runs, const rdx_mesh* meshes, const rdx_model* models,
                            const uint64_t* seeds, const double* tau_overrides, rdx_batch** out) {
  clear_error();
  if (!out) return set_error(RDX_EINVAL, "null output handle");
  *out = nullptr;
  if (n_runs < 1 || !meshes || !models || !seeds) return set_error(RDX_EINVAL, "bad batch arguments");
  rdx_batch* b = new (std::nothrow) rdx_batch();
  if (!b) return set_error(RDX_ENOMEM, "host allocation failed");
  b->runs.resize((size_t)n_runs);
  size_t bytes = 0;
  int64_t tets = 0;
  for (int32_t i = 0; i < n_runs; ++i) {
    std::string err;
    rdx_status st = build_instance(&meshes[i], &models[i], tau_overrides ? tau_overrides[i] : 0.0,
                                   &b->runs[(size_t)i].host, &err);
    if (st != RDX_OK) {
      delete b;
      return set_error(st, "run " + std::to_string(i) + ": " + err);
    }
    b->runs[(size_t)i].seed = seeds[i];
    bytes += Engine::run_bytes(b->runs[(size_t)i].host);
    tets += b->runs[(size_t)i].host.T;
  }
  if (tets > (int64_t)INT32_MAX) {
    delete b;
    return set_error(RDX_EINVAL, "a batch holds at most 2^31 - 1 tets");
  }
  (void)hipGetDevice(&b->device);
  rdx_status st = b->eng.init(b->runs[0].host, bytes, n_runs, tets);
  for (int32_t i = 0; st == RDX_OK && i < n_runs; ++i)
    st = b->eng.add_run(&b->runs[(size_t)i], b->eng.own_stream());
  if (st != RDX_OK) {
    const std::string msg = rdx_last_error();
    delete b;
    return set_error(st == RDX_EBUDGET ? RDX_ENOMEM : st, msg);
  }
  b->eng.set_autotune(true);
  *out = b;
  return RDX_OK;
}

void rdx_batch_destroy(rdx_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  b->eng.drain();
  if (b->rec) (void)hipFree(b->rec);
  delete b;
}

static rdx_status check_batch_run(const rdx_batch* b, int32_t i) {
  if (!b) return set_error(RDX_EINVAL, "null batch handle");
  if (i < 0 || (size_t)i >= b->runs.size()) return set_error(RDX_EINVAL, "run index out of range");
  return RDX_OK;
}

rdx_status rdx_batch_set_rate_constants(rdx_batch* b, int32_t i, const double* kcst, int64_t n, void* stream) {
  clear_error();
  if (check_batch_run(b, i) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(b->device);
  return set_rates_of(b->eng, b->runs[(size_t)i], kcst, n, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_region_counts(rdx_batch* b, int32_t i, int64_t* out, int is_device_ptr, void* stream) {
  clear_error();
  if (check_batch_run(b, i) != RDX_OK) return RDX_EINVAL;
  (void)hipSetDevice(b->device);
  return region_counts_of(b->eng, b->runs[(size_t)i], out, is_device_ptr != 0, &b->rec,
                          reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_size(const rdx_batch* b, int32_t* n_runs) {
  clear_error();
  if (!b || !n_runs) return set_error(RDX_EINVAL, "null argument");
  *n_runs = (int32_t)b->runs.size();
  return RDX_OK;
}

rdx_status rdx_batch_get_run_info(const rdx_batch* b, int32_t i, int32_t* n_tets, double* tau) {
  clear_error();
  if (check_batch_run(b, i) != RDX_OK) return RDX_EINVAL;
  if (n_tets) *n_tets = b->runs[(size_t)i].host.T;
  if (tau) *tau = b->runs[(size_t)i].host.tau;
  return RDX_OK;
}

rdx_status rdx_batch_set_counts(rdx_batch* b, int32_t i, const int32_t* counts, int is_device_ptr,
                                void* stream) {
  clear_error();
  if (check_batch_run(b, i) != RDX_OK) return RDX_EINVAL;
  if (!counts) return set_error(RDX_EINVAL, "null counts");
  (void)hipSetDevice(b->device);
  return start_run(b->eng, b->runs[(size_t)i], counts, is_device_ptr != 0, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_set_counts_all(rdx_batch* b, const int32_t* const* counts, void* stream) {
  clear_error();
  if (!b || !counts) return set_error(RDX_EINVAL, "null argument");
  for (size_t i = 0; i < b->runs.size(); ++i)
    if (!counts[i]) return set_error(RDX_EINVAL, "null counts for run " + std::to_string(i));
  (void)hipSetDevice(b->device);
  std::vector<Run*> rs(b->runs.size());
  for (size_t i = 0; i < b->runs.size(); ++i) rs[i] = &b->runs[i];
  return b->eng.reset_runs_device(rs.data(), rs.size(), counts, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_get_counts(rdx_batch* b, int32_t i, int32_t* out, int is_device_ptr, void* stream) {
  clear_error();
  if (check_batch_run(b, i) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null output");
  (void)hipSetDevice(b->device);
  return b->eng.download_counts(&b->runs[(size_t)i], out, is_device_ptr != 0, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_run(rdx_batch* b, const double* t_end, void* stream) {
  clear_error();
  if (!b || !t_end) return set_error(RDX_EINVAL, "null argument");
  (void)hipSetDevice(b->device);
  std::vector<Run*> rs;
  rs.reserve(b->runs.size());
  for (size_t i = 0; i < b->runs.size(); ++i) {
    rdx_status st = Engine::plan_until(&b->runs[i], t_end[i], -1);
    if (st != RDX_OK) {
      for (Run& r : b->runs) r.plan_steps = r.plan_full = 0;
      return st;
    }
    rs.push_back(&b->runs[i]);
  }
  return b->eng.sequence(rs, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_step(rdx_batch* b, int64_t n_windows, void* stream) {
  clear_error();
  if (!b) return set_error(RDX_EINVAL, "null batch handle");
  (void)hipSetDevice(b->device);
  std::vector<Run*> rs;
  for (Run& r : b->runs) {
    rdx_status st = Engine::plan_steps(&r, n_windows);
    if (st != RDX_OK) {
      for (Run& q : b->runs) q.plan_steps = q.plan_full = 0;
      return st;
    }
    rs.push_back(&r);
  }
  return b->eng.sequence(rs, reinterpret_cast<hipStream_t>(stream));
}

rdx_status rdx_batch_sync(rdx_batch* b, void* stream) {
  clear_error();
  if (!b) return set_error(RDX_EINVAL, "null batch handle");
  (void)hipSetDevice(b->device);
  RDX_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  for (const Run& r : b->runs) {
    rdx_status st = b->eng.run_error(&r);
    if (st != RDX_OK) return st;
  }
  return RDX_OK;
}

rdx_status rdx_batch_get_stats(rdx_batch* b, int32_t i, rdx_stats* out, void* stream) {
  clear_error();
  if (check_batch_run(b, i) != RDX_OK) return RDX_EINVAL;
  if (!out) return set_error(RDX_EINVAL, "null stats");
  (void)hipSetDevice(b->device);
  RDX_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  const Run& r = b->runs[(size_t)i];
  rdx_status st = b->eng.run_error(&r);
  const std::string msg = rdx_last_error();
  rdx_status q = fill_stats(b->eng, r, out);
  if (q != RDX_OK) return q;
  if (st != RDX_OK) set_error(st, msg);
  return st;
}

rdx_status rdx_batch_set_exec_options(rdx_batch* b, const rdx_exec_options* o) {
  clear_error();
  if (!b) return set_error(RDX_EINVAL, "null batch handle");
  return apply_options(b->eng, o);
}

rdx_status rdx_batch_get_exec_options(const rdx_batch* b, rdx_exec_options* o) {
  clear_error();
  if (!b || !o) return set_error(RDX_EINVAL, "null argument");
  read_options(b->eng, o);
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
