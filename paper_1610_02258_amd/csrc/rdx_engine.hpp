// rdx_engine.hpp -- the host runtime that drives the window kernels.
//
// An Engine owns the device state of a set of independent runs (each one a
// complete simulation: mesh arrays, double-buffered counts, seed, rate
// constants, window schedule) that share the species/reaction structure, and
// advances any subset of them together: one window launch covers the tiles of
// every run taking part.  The single simulation, the batch and the server
// are all Engines; they differ only in how runs come and go.
//
// Device memory of the runs comes from one arena reserved up front (no
// allocation in the stepping loop); the per-window worklist is sized for the
// engine's tet capacity.  Sequences of windows are replayed from captured
// HIP graphs when that pays, and the launch shape can be tuned online
// (results do not depend on it).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "rdx.h"
#include "rdx_internal.hpp"
#include "rdx_kernels.hpp"

namespace rdx {

// First-fit sub-allocator over one device reservation (256-byte granules,
// neighbouring free blocks coalesced).
class DeviceArena {
 public:
  DeviceArena() = default;
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  ~DeviceArena();
  hipError_t reserve(size_t bytes);
  // Offset of a block of `bytes`, or SIZE_MAX when nothing fits.
  size_t alloc(size_t bytes);
  void release(size_t off);
  char* base() const { return base_; }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_bytes_; }
  size_t largest_free() const;

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_bytes_ = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  std::map<size_t, size_t> used_;  // offset -> size
};

// One run's host state.  The counts of the current window index live in
// cnt[window & 1]; the other buffer is all zero between windows.
struct Run {
  HostInstance host;
  uint64_t seed = 0;
  size_t arena_off = SIZE_MAX;
  int32_t* cnt[2] = {nullptr, nullptr};
  int32_t* nbr = nullptr;
  double* geo = nullptr;      // (G, cum0, cum1, cum2) per tet
  double* nav = nullptr;
  uint8_t* region = nullptr;  // only with more than one region
  double* kcst = nullptr;     // [8][32], then the listing coefficients
  double* lcoef = nullptr;    // [8][kLStride]
  unsigned long long* tally = nullptr;  // [kTallySlots][kTallyWords]
  int32_t* err = nullptr;
  double t = 0.0;
  int64_t window = 0;
  int64_t windows_run = 0;
  int64_t voxel_steps = 0;
  // the windows planned for the next sequence
  int64_t plan_steps = 0, plan_full = 0;
  double plan_tau_last = 0.0, plan_t_after = 0.0;
};

// Launch shape of a sequence.  fast_grid_div: the main kernel's grid is its
// resident grid divided by this (1, 2, 4); graph_windows: windows per
// captured graph (1 = plain launches).
struct ExecShape {
  int fast_grid_div = 1;
  int graph_windows = 1;
  int event_group = 4;  // most queued tiles packed into one event chunk
  int event_bins = 1;   // listed tets binned by expected events (heavy, light)
  int tile_claim = 0;   // diffusion tiles after the first claimed at run time
  bool operator<(const ExecShape& o) const {
    if (fast_grid_div != o.fast_grid_div) return fast_grid_div < o.fast_grid_div;
    if (graph_windows != o.graph_windows) return graph_windows < o.graph_windows;
    if (event_group != o.event_group) return event_group < o.event_group;
    if (event_bins != o.event_bins) return event_bins < o.event_bins;
    return tile_claim < o.tile_claim;
  }
};

class Engine {
 public:
  Engine() = default;
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  ~Engine();

  // Device bytes of one run's state (counts, mesh arrays, tables, tallies).
  static size_t run_bytes(const HostInstance& I);
  // Worklist bytes per tet of capacity (64 entries per tile, each tile
  // of a run padded to 64 tets).
  static size_t worklist_bytes_per_tet(int S);

  // `proto` fixes the shared species/reaction structure.  arena_bytes holds
  // the runs' state; max_runs and max_tets bound what may be resident.
  rdx_status init(const HostInstance& proto, size_t arena_bytes, int max_runs, int64_t max_tets);

  // Same S, R, stoichiometry as the engine's structure.
  bool compatible(const HostInstance& I) const;

  // Places the run in the arena and uploads its mesh arrays and tables;
  // counts start at zero at t = 0.  RDX_EBUDGET when the arena or the
  // capacity cannot take it now.
  rdx_status add_run(Run* r, hipStream_t stream);
  // Waits for `stream` (where every launch that touched the run went) and
  // returns the run's memory to the arena.
  void remove_run(Run* r, hipStream_t stream);

  // Counts for the run's current window index (host or device pointer).
  rdx_status upload_counts(Run* r, const int32_t* counts, bool device, hipStream_t stream);
  rdx_status reset_run(Run* r, hipStream_t stream);  // tallies, error flag, other buffer
  // Every run to t = 0 with counts copied from device pointers src[j], all in
  // one launch (the state the pair reset_run + upload_counts leaves).
  rdx_status reset_runs_device(Run* const* runs, size_t n, const int32_t* const* src, hipStream_t stream);
  rdx_status download_counts(const Run* r, int32_t* out, bool device, hipStream_t stream);
  // Time-varying forcing: new rate constants [n_regions*R] for the windows
  // enqueued after this call on `stream` (waits for the upload).
  rdx_status set_rates(Run* r, const double* kcst, hipStream_t stream);
  // Recording: per-region sums of the current counts into the device array
  // out [n_regions*S], enqueued on `stream`; scratch holds kRegionScratchBytes.
  // `mark` = false leaves `stream` out of the fences (no event is recorded,
  // for callers under graph capture).
  rdx_status region_counts(const Run* r, unsigned long long* scratch, unsigned long long* out,
                           hipStream_t stream, bool mark = true);
  // Recording inside a sequence: while set, sequence() launches plain
  // windows (no tuning, no graphs) and after every `every`-th window of
  // `run` writes its per-region sums to ring slot (records mod slots).
  struct RecordHook {
    const Run* run = nullptr;
    int64_t every = 0;
    unsigned long long* scratch = nullptr;
    unsigned long long* ring = nullptr;
    int64_t slots = 0;
    int64_t records = 0;  // written so far
  };
  void set_record_hook(const RecordHook* h) {
    rec_on_ = h != nullptr;
    if (h) rec_ = *h;
  }
  int64_t records_written() const { return rec_.records; }

  // Plans (Algorithm 1 schedule): windows up to t_end, at most max_windows
  // (< 0: no limit); or n full windows.
  static rdx_status plan_until(Run* r, double t_end, int64_t max_windows);
  static rdx_status plan_steps(Run* r, int64_t n);

  // Enqueues the planned windows of `runs` on `stream` and advances their
  // host state.  Runs with nothing planned are left out.
  rdx_status sequence(const std::vector<Run*>& runs, hipStream_t stream);

  // Launch shape: fixed, or tuned online over the first sequences.
  void set_shape(const ExecShape& s) { shape_ = s; tuning_ = false; }
  void set_autotune(bool on);
  ExecShape shape() const { return shape_; }
  bool tuning() const { return tuning_; }

  // Per-kernel timing (plain launches, three events per window).
  void set_timing(bool on) { timing_ = on; }
  rdx_status kernel_times(rdx_kernel_times* out, bool reset);

  // Device error flag of one run, and its tallies; synchronous, on the
  // engine's own stream, so the caller first waits for the stream that ran
  // the run's windows.
  rdx_status run_error(const Run* r) const;
  // SSA events, molecules moved, nonzero (tet, species, face) moves
  rdx_status run_tally(const Run* r, unsigned long long tal[3]) const;
  // The same two read back on `stream` into `out` (pinned host memory), so
  // that only that stream is waited for; `out` is valid once it has been
  // synchronised, and decode_readout then gives the error and the tallies.
  struct Readout {
    int32_t err;
    int32_t pad;
    unsigned long long slots[kTallyWords * kTallySlots];
  };
  rdx_status read_run_async(const Run* r, Readout* out, hipStream_t stream) const;
  static rdx_status decode_readout(const Readout& in, unsigned long long tal[3]);

  // The engine's own stream, for set-up work that has no caller stream.
  hipStream_t own_stream() const { return own_; }
  // Every method that enqueues on a stream marks it here; drain() waits for
  // the last enqueue on each marked stream.  The engine's memory can then be
  // released without a device-wide synchronisation, which fails while any
  // other thread holds a stream in graph capture.
  void fence(hipStream_t stream);
  void drain();

  int S() const { return S_; }
  int R() const { return R_; }
  int64_t resident_tets() const { return resident_tets_; }
  int resident_runs() const { return resident_runs_; }
  int64_t max_tets() const { return max_tets_; }
  int max_runs() const { return max_runs_; }
  const DeviceArena& arena() const { return arena_; }

 private:
  rdx_status upload_tables(const std::vector<Run*>& active, int64_t k0, hipStream_t stream,
                           int64_t* n_tiles_out);
  rdx_status launch_plain(const StepArgs& a, int64_t K, hipStream_t stream);
  rdx_status launch_graphs(const StepArgs& a, int64_t reps, hipStream_t stream);
  void grids_for(int64_t n_tiles, int div, int* detect, int* main) const;
  void free_graphs();

  int S_ = 0, R_ = 0;
  DevModel model_host_{};
  DevModel* model_ = nullptr;
  DeviceArena arena_;
  int max_runs_ = 0;
  int64_t max_tets_ = 0, max_tiles_ = 0;
  int resident_runs_ = 0;
  int64_t resident_tets_ = 0;

  RunDesc* d_runs_ = nullptr;
  int2* d_tile_map_ = nullptr;
  int32_t* d_n_tiles_ = nullptr;
  int32_t* d_base_ = nullptr;
  int32_t* wl_tile_count_ = nullptr;
  unsigned long long* wl_mask_ = nullptr;
  int32_t* evq_ = nullptr;
  unsigned long long* evq_count_ = nullptr;
  int32_t* wl_tet_ = nullptr;
  int32_t* tile_ctr_ = nullptr;  // [2][8][kCtrStride]

  // pinned staging of the run table and tile map; `staged_` marks the
  // completion of the last upload from them
  RunDesc* h_runs_ = nullptr;
  int2* h_tile_map_ = nullptr;
  int32_t* h_n_tiles_ = nullptr;
  hipEvent_t staged_ = nullptr;
  // batched reset: pinned chunk table, its device copy, and the event that
  // marks the pinned table free again
  ResetChunk* h_reset_ = nullptr;
  ResetChunk* d_reset_ = nullptr;
  size_t reset_cap_ = 0;
  hipEvent_t reset_staged_ = nullptr;
  std::vector<const Run*> tile_runs_;  // runs of the tile map on the device
  std::vector<int64_t> tile_run_T_;
  int64_t k_now_ = 0;                  // batch step index == *d_base_

  // graphs by (windows, grids); captured on a private stream
  hipStream_t capture_stream_ = nullptr;
  hipStream_t own_ = nullptr;
  std::vector<std::pair<hipStream_t, hipEvent_t>> fences_;
  RecordHook rec_{};
  bool rec_on_ = false;
  std::map<std::pair<int, long long>, hipGraphExec_t> graphs_;

  ExecShape shape_;
  bool tuning_ = false;
  std::vector<ExecShape> candidates_;
  size_t cand_next_ = 0;
  std::map<ExecShape, double> cand_ms_;  // per voxel-step cost measured per candidate
  hipEvent_t tune_ev_[2] = {nullptr, nullptr};

  bool timing_ = false;
  std::vector<hipEvent_t> marks_;
  size_t marks_used_ = 0;
  int64_t timed_windows_ = 0;
  double detect_ms_ = 0.0, main_ms_ = 0.0;
};

// DevModel of a validated instance (packed reaction entries, net changes,
// dependency masks).
DevModel make_dev_model(const HostInstance& I);

}  // namespace rdx
