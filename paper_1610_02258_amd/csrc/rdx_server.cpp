// rdx_server.cpp -- the served form: a request loop with continuous batching.
//
// Requests (a mesh, model parameters, seed, initial counts and t_end) are set
// up on the submitting thread (validation and the set-up step of section 2.1)
// and queued.  One worker thread owns the device side: it admits queued
// requests in arrival order while the device budget has room for their
// state, enqueues one tick -- up to `tick_windows` windows of every resident
// request, all in the same window launches -- and retires the requests that
// reached their t_end, which frees their memory for the next admissions.
// Requests therefore join and leave a running batch;
// each one's result is the one it would get alone, since every draw is
// addressed by (its seed, stream, tet, its window index).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rdx.h"
#include "rdx_engine.hpp"
#include "rdx_internal.hpp"

using namespace rdx;

namespace {

struct Request {
  int64_t ticket = 0;
  Run run;
  std::vector<int32_t> counts0;  // initial counts, then the result
  double t_end = 0.0;
  int32_t state = RDX_REQ_QUEUED;
  rdx_status status = RDX_OK;
  std::string error;
  bool cancel = false;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  rdx_stats stats{};
};

double quantile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest-rank quantile
  size_t k = (size_t)std::ceil(q * (double)v.size());
  if (k < 1) k = 1;
  if (k > v.size()) k = v.size();
  return v[k - 1];
}

}  // namespace

struct rdx_server {
  Engine eng;
  int device = 0;
  hipStream_t stream = nullptr;     // the ticks' launches
  hipStream_t up_stream = nullptr;  // admissions' uploads, retirements' reads
  hipEvent_t tick_begin[2] = {nullptr, nullptr}, tick_end[2] = {nullptr, nullptr};
  Engine::Readout* readout = nullptr;  // pinned, one per resident run
  int tick_windows = 8;
  int64_t capacity_tets = 0;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work;  // worker: something to do
  std::condition_variable cv_done;  // waiters: a request finished
  bool stop = false;
  int64_t next_ticket = 1;
  std::map<int64_t, std::unique_ptr<Request>> requests;
  std::deque<Request*> queue;
  std::vector<Request*> resident;  // touched by the worker only
  // statistics (under mu)
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, ticks = 0;
  int64_t voxel_steps = 0, ssa_events = 0, moves = 0;
  double gpu_busy_s = 0.0;  // device time of the retired ticks (HIP events)
  double host_s = 0.0;      // worker time spent on uploads, planning and launching
  std::vector<double> latencies;

  std::thread worker;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  ~rdx_server() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (up_stream) (void)hipStreamSynchronize(up_stream);
    for (int j = 0; j < 2; ++j) {
      if (tick_begin[j]) (void)hipEventDestroy(tick_begin[j]);
      if (tick_end[j]) (void)hipEventDestroy(tick_end[j]);
    }
    if (readout) (void)hipHostFree(readout);
    if (up_stream) (void)hipStreamDestroy(up_stream);
    if (stream) (void)hipStreamDestroy(stream);
  }
  void run_loop();
  void retire(std::vector<Request*>& leaving, int slot, rdx_status tick_st, const std::string& tick_err);
  void finish(Request* q, int32_t state, rdx_status st, const std::string& msg);
};

void rdx_server::finish(Request* q, int32_t state, rdx_status st, const std::string& msg) {
  // caller holds mu
  q->state = state;
  q->status = st;
  q->error = msg;
  q->t_done = now();
  if (state == RDX_REQ_DONE) {
    completed += 1;
    latencies.push_back(q->t_done - q->t_submit);
    voxel_steps += q->stats.voxel_steps;
    ssa_events += q->stats.ssa_events;
    moves += q->stats.moves;
  } else if (state == RDX_REQ_CANCELLED) {
    cancelled += 1;
  } else {
    failed += 1;
  }
  cv_done.notify_all();
}

void rdx_server::retire(std::vector<Request*>& leaving, int slot, rdx_status tick_st, const std::string& tick_err) {
  // every launch that can touch these runs is in tick `slot`, already enqueued
  // on `stream`: the reads go on the side stream behind that tick's end event,
  // so the tick enqueued after it keeps the device busy meanwhile.  With no
  // leavers the worker still waits for the tick's end, so that at most two
  // ticks are ever enqueued.
  if (leaving.empty()) {
    (void)hipEventSynchronize(tick_end[slot]);
    return;
  }
  if (hipStreamWaitEvent(up_stream, tick_end[slot], 0) != hipSuccess) {
    tick_st = RDX_EHIP;
    (void)hipStreamSynchronize(stream);
  }
  for (size_t j = 0; j < leaving.size(); ++j) {
    Request* q = leaving[j];
    const bool done = q->run.t >= q->t_end;
    rdx_status rs = tick_st;
    std::string msg = tick_err;
    if (rs == RDX_OK && done) {  // a finished request is delivered even if cancelled late
      Engine::Readout* ro = readout + j;
      rs = eng.read_run_async(&q->run, ro, up_stream);
      if (rs == RDX_OK) rs = eng.download_counts(&q->run, q->counts0.data(), false, up_stream);
      unsigned long long tal[3] = {0, 0, 0};
      if (rs == RDX_OK) {
        rs = Engine::decode_readout(*ro, tal);
        if (rs != RDX_OK) msg = rdx_last_error();
      } else {
        msg = rdx_last_error();
      }
      q->stats.windows = q->run.windows_run;
      q->stats.voxel_steps = q->run.voxel_steps;
      q->stats.ssa_events = (int64_t)tal[0];
      q->stats.moves = (int64_t)tal[1];
      q->stats.face_moves = (int64_t)tal[2];
      q->stats.t = q->run.t;
      q->stats.window_index = q->run.window;
    }
    // the side stream has passed the tick's end (and the reads): no launch
    // can still touch the run
    eng.remove_run(&q->run, up_stream);
    std::lock_guard<std::mutex> lk(mu);
    if (rs == RDX_OK && done) finish(q, RDX_REQ_DONE, RDX_OK, "");
    else if (rs == RDX_OK) finish(q, RDX_REQ_CANCELLED, RDX_ECANCELLED, "cancelled");
    else finish(q, RDX_REQ_FAILED, rs, msg);
  }
  leaving.clear();
}

void rdx_server::run_loop() {
  (void)hipSetDevice(device);
  // Two ticks are in the pipeline at once: while tick n runs on `stream`, the
  // worker uploads the next admissions on the side stream, enqueues tick n+1
  // behind tick n, and only then waits for tick n's end event to retire the
  // requests whose last windows were in it.  Requests leave the resident set
  // when their last windows are planned, so the tick after never names them.
  std::vector<Request*> leaving[2];  // per tick slot: retire once it has ended
  bool in_flight[2] = {false, false};
  int cur = 0;
  for (;;) {
    const int prev = cur ^ 1;
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      // queued cancellations end here; resident ones when their tick is planned
      for (auto it = queue.begin(); it != queue.end();) {
        if ((*it)->cancel || stop) {
          finish(*it, RDX_REQ_CANCELLED, RDX_ECANCELLED, "cancelled");
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
      // admission in arrival order while the budget has room
      int64_t tets = eng.resident_tets();
      int runs = eng.resident_runs();
      size_t free_bytes = eng.arena().capacity() - eng.arena().in_use();
      while (!stop && !queue.empty()) {
        Request* q = queue.front();
        const size_t need = Engine::run_bytes(q->run.host);
        if (tets + q->run.host.T > capacity_tets || runs + 1 > eng.max_runs() || need > free_bytes)
          break;
        tets += q->run.host.T;
        runs += 1;
        free_bytes -= need;
        queue.pop_front();
        admit.push_back(q);
      }
      const bool idle = resident.empty() && admit.empty() && !in_flight[prev];
      if (stop && idle) break;
      if (idle) {
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        continue;
      }
    }
    // uploads of the admitted requests on the side stream, beside the tick in
    // flight (add_run and upload_counts wait for the side stream only)
    const double t_host0 = now();
    for (size_t j = 0; j < admit.size(); ++j) {
      Request* q = admit[j];
      rdx_status st = eng.add_run(&q->run, up_stream);
      if (st == RDX_EBUDGET) {  // fragmentation: back to the head of the queue
        std::lock_guard<std::mutex> lk(mu);
        for (size_t x = admit.size(); x-- > j;) queue.push_front(admit[x]);
        break;
      }
      if (st == RDX_OK) st = eng.reset_run(&q->run, up_stream);
      if (st == RDX_OK) st = eng.upload_counts(&q->run, q->counts0.data(), false, up_stream);
      std::lock_guard<std::mutex> lk(mu);
      if (st != RDX_OK) {
        eng.remove_run(&q->run, up_stream);
        finish(q, RDX_REQ_FAILED, st, rdx_last_error());
        continue;
      }
      q->state = RDX_REQ_RUNNING;
      q->t_admit = now();
      resident.push_back(q);
    }
    // plan and enqueue the next tick: up to tick_windows windows of every
    // resident request; cancelled ones leave without windows
    std::vector<Run*> runs;
    std::vector<Request*> planned, keep;
    bool ok = true;
    for (Request* q : resident) {
      bool cancel;
      {
        std::lock_guard<std::mutex> lk(mu);
        cancel = q->cancel || stop;
      }
      if (cancel) {
        leaving[prev].push_back(q);  // its last launches are in the tick in flight
        continue;
      }
      if (Engine::plan_until(&q->run, q->t_end, tick_windows) != RDX_OK) ok = false;
      runs.push_back(&q->run);
      planned.push_back(q);
    }
    rdx_status st = RDX_OK;
    if (!planned.empty()) {
      st = hipEventRecord(tick_begin[cur], stream) == hipSuccess ? RDX_OK : RDX_EHIP;
      if (st == RDX_OK) st = ok ? eng.sequence(runs, stream) : RDX_EINVAL;
      if (st == RDX_OK && hipEventRecord(tick_end[cur], stream) != hipSuccess) st = RDX_EHIP;
    }
    const std::string tick_err = st == RDX_OK ? std::string() : std::string(rdx_last_error());
    if (st != RDX_OK) {
      // a failed tick may have enqueued part of its launches: retire its
      // requests once the stream has drained
      (void)hipStreamSynchronize(stream);
      for (Request* q : planned) {
        eng.remove_run(&q->run, stream);
        std::lock_guard<std::mutex> lk(mu);
        finish(q, RDX_REQ_FAILED, st, tick_err);
      }
      planned.clear();
    }
    for (Request* q : planned) {
      if (q->run.t >= q->t_end) leaving[cur].push_back(q);
      else keep.push_back(q);
    }
    resident.swap(keep);
    const bool launched = !planned.empty();
    {
      std::lock_guard<std::mutex> lk(mu);
      host_s += now() - t_host0;
    }
    // retire the previous tick's leavers (this waits for its end only)
    if (in_flight[prev] || !leaving[prev].empty()) {
      if (in_flight[prev]) {
        retire(leaving[prev], prev, RDX_OK, std::string());
        float ms = 0.f;
        if (hipEventSynchronize(tick_end[prev]) == hipSuccess &&
            hipEventElapsedTime(&ms, tick_begin[prev], tick_end[prev]) == hipSuccess) {
          std::lock_guard<std::mutex> lk(mu);
          gpu_busy_s += 1e-3 * (double)ms;
        }
      } else {  // cancelled while nothing was in flight
        (void)hipStreamSynchronize(stream);
        for (Request* q : leaving[prev]) {
          eng.remove_run(&q->run, stream);
          std::lock_guard<std::mutex> lk(mu);
          finish(q, RDX_REQ_CANCELLED, RDX_ECANCELLED, "cancelled");
        }
        leaving[prev].clear();
      }
      in_flight[prev] = false;
    }
    in_flight[cur] = launched;  // leaving[cur] is empty unless it launched
    if (launched) {
      std::lock_guard<std::mutex> lk(mu);
      ticks += 1;
    }
    cur ^= 1;
  }
}

extern "C" {

rdx_status rdx_server_create(const rdx_model* structure, const rdx_server_options* opts, rdx_server** out) {
  clear_error();
  if (!out || !structure || !opts) return set_error(RDX_EINVAL, "null argument");
  *out = nullptr;
  if (opts->hbm_budget_bytes < ((size_t)1 << 20) || opts->max_runs < 0 || opts->tick_windows < 0 ||
      opts->graph_windows < 0 || opts->graph_windows > 256)
    return set_error(RDX_EINVAL, "server options out of range");
  // the structure is validated as a model on a one-tet mesh
  const double verts[12] = {0, 0, 0, 1e-6, 0, 0, 0, 1e-6, 0, 0, 0, 1e-6};
  const int32_t tets[4] = {0, 1, 2, 3};
  rdx_mesh one{4, 1, verts, tets, nullptr};
  HostInstance proto;
  std::string err;
  rdx_status st = build_instance(&one, structure, 1.0, &proto, &err);
  if (st != RDX_OK) return set_error(st, err);

  std::unique_ptr<rdx_server> s(new (std::nothrow) rdx_server());
  if (!s) return set_error(RDX_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&s->device);
  // default: at most 1024 resident requests, and their padded worklist tiles
  // at most an eighth of the budget
  const size_t wl_tet0 = Engine::worklist_bytes_per_tet(proto.S);
  const int max_runs = opts->max_runs
                           ? opts->max_runs
                           : (int)std::max<size_t>(1, std::min<size_t>(1024, opts->hbm_budget_bytes / (512 * wl_tet0)));
  s->tick_windows = opts->tick_windows ? opts->tick_windows : 8;
  // the budget holds the worklist (per tet of capacity, plus a padded tile
  // per resident run) and the runs' state
  const size_t wl_tet = Engine::worklist_bytes_per_tet(proto.S);
  const size_t pad = 64 * (size_t)max_runs * wl_tet;
  if (opts->hbm_budget_bytes < 2 * pad) return set_error(RDX_EINVAL, "budget too small for max_runs");
  const size_t per_tet = wl_tet + 8 * (size_t)proto.S + 57;
  int64_t cap = (int64_t)((opts->hbm_budget_bytes - pad) / per_tet);
  cap = std::min<int64_t>(cap, INT32_MAX / 256);
  const size_t wl = (size_t)cap * wl_tet + pad;
  const size_t arena = opts->hbm_budget_bytes - wl;
  s->capacity_tets = cap;
  st = s->eng.init(proto, arena, max_runs, cap);
  if (st != RDX_OK) return st;
  const int gw = opts->graph_windows ? opts->graph_windows : s->tick_windows;
  s->eng.set_shape(ExecShape{1, gw, 4});
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->up_stream, hipStreamNonBlocking) != hipSuccess)
    return set_error(RDX_EHIP, "stream creation failed");
  for (int j = 0; j < 2; ++j)
    if (hipEventCreate(&s->tick_begin[j]) != hipSuccess || hipEventCreate(&s->tick_end[j]) != hipSuccess)
      return set_error(RDX_EHIP, "event creation failed");
  if (hipHostMalloc(reinterpret_cast<void**>(&s->readout), sizeof(Engine::Readout) * (size_t)max_runs) !=
      hipSuccess)
    return set_error(RDX_ENOMEM, "pinned host allocation failed");
  s->t0 = std::chrono::steady_clock::now();
  rdx_server* raw = s.get();
  s->worker = std::thread([raw] { raw->run_loop(); });
  *out = s.release();
  return RDX_OK;
}

void rdx_server_destroy(rdx_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  delete s;
}

rdx_status rdx_server_submit(rdx_server* s, const rdx_mesh* mesh, const rdx_model* model, uint64_t seed,
                             const int32_t* counts0, double t_end, double tau_override, int64_t* ticket) {
  clear_error();
  if (!s || !counts0 || !ticket) return set_error(RDX_EINVAL, "null argument");
  if (!std::isfinite(t_end) || t_end < 0.0) return set_error(RDX_EINVAL, "t_end must be finite and >= 0");
  std::unique_ptr<Request> q(new (std::nothrow) Request());
  if (!q) return set_error(RDX_ENOMEM, "host allocation failed");
  std::string err;
  rdx_status st = build_instance(mesh, model, tau_override, &q->run.host, &err);
  if (st != RDX_OK) return set_error(st, err);
  if (!s->eng.compatible(q->run.host))
    return set_error(RDX_EINVAL, "model does not share the server's species/reaction structure");
  const HostInstance& I = q->run.host;
  if (I.T > s->capacity_tets || Engine::run_bytes(I) > s->eng.arena().capacity())
    return set_error(RDX_EBUDGET, "request can never fit the server's device-memory budget");
  const size_t n = (size_t)I.S * (size_t)I.T;
  for (size_t x = 0; x < n; ++x)
    if (counts0[x] < 0 || counts0[x] > kCountCap) return set_error(RDX_EINVAL, "counts must lie in [0, 2^30]");
  // the schedule must stay inside the 32-bit window counter
  {
    Run probe;
    probe.host.tau = I.tau;
    st = Engine::plan_until(&probe, t_end, -1);
    if (st != RDX_OK) return st;
  }
  q->counts0.assign(counts0, counts0 + n);
  q->run.seed = seed;
  q->t_end = t_end;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(RDX_ESTATE, "server is shutting down");
    q->ticket = s->next_ticket++;
    q->t_submit = s->now();
    *ticket = q->ticket;
    s->queue.push_back(q.get());
    s->requests[q->ticket] = std::move(q);
    s->submitted += 1;
  }
  s->cv_work.notify_one();
  return RDX_OK;
}

static void fill_info(const Request& q, rdx_request_info* info) {
  info->state = q.state;
  info->status = q.status;
  info->n_tets = q.run.host.T;
  info->n_species = q.run.host.S;
  info->t_submit = q.t_submit;
  info->t_admit = q.t_admit;
  info->t_done = q.t_done;
  info->stats = q.stats;
}

rdx_status rdx_server_poll(rdx_server* s, int64_t ticket, rdx_request_info* info) {
  clear_error();
  if (!s || !info) return set_error(RDX_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return set_error(RDX_EINVAL, "unknown ticket");
  fill_info(*it->second, info);
  return RDX_OK;
}

rdx_status rdx_server_wait(rdx_server* s, int64_t ticket, double timeout_s, int32_t* counts_out,
                           rdx_request_info* info) {
  clear_error();
  if (!s) return set_error(RDX_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return set_error(RDX_EINVAL, "unknown ticket");
  Request* q = it->second.get();
  auto finished = [q] { return q->state >= RDX_REQ_DONE; };
  if (timeout_s < 0.0) {
    s->cv_done.wait(lk, finished);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
    if (info) fill_info(*q, info);
    return set_error(RDX_ESTATE, "request not finished within the timeout");
  }
  if (info) fill_info(*q, info);
  const rdx_status st = q->status;
  const std::string msg = q->error;
  if (q->state == RDX_REQ_DONE && counts_out)
    std::memcpy(counts_out, q->counts0.data(), sizeof(int32_t) * q->counts0.size());
  s->requests.erase(it);  // the record goes with the first completed wait
  if (st != RDX_OK) return set_error(st, msg);
  return RDX_OK;
}

rdx_status rdx_server_cancel(rdx_server* s, int64_t ticket) {
  clear_error();
  if (!s) return set_error(RDX_EINVAL, "null argument");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(RDX_EINVAL, "unknown ticket");
    it->second->cancel = true;
  }
  s->cv_work.notify_all();
  return RDX_OK;
}

rdx_status rdx_server_get_stats(rdx_server* s, rdx_server_stats* out) {
  clear_error();
  if (!s || !out) return set_error(RDX_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->cancelled = s->cancelled;
  out->queued = (int64_t)s->queue.size();
  int64_t running = 0;
  for (const auto& kv : s->requests) running += kv.second->state == RDX_REQ_RUNNING;
  out->running = running;
  out->ticks = s->ticks;
  out->voxel_steps = s->voxel_steps;
  out->ssa_events = s->ssa_events;
  out->moves = s->moves;
  out->busy_s = s->gpu_busy_s;
  out->worker_s = s->host_s;
  out->uptime_s = s->now();
  out->latency_p50_s = quantile(s->latencies, 0.50);
  out->latency_p99_s = quantile(s->latencies, 0.99);
  out->capacity_tets = s->capacity_tets;
  return RDX_OK;
}

}  // extern "C"
