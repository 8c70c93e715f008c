// rdx_kernels.hpp -- launch interface of the gfx950 kernels (host side).
//
// The kernels advance a batch of independent runs (one simulation is a batch
// of one).  Every run has its own mesh arrays, count buffers, seed, rate
// constants and window schedule; all runs share the species/reaction
// structure.  The tets of all runs are cut into tiles of 64 (a tile never
// spans two runs), and a persistent grid walks the tiles.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace rdx {

// Reaction tables shared by the runs of a batch (one device copy).  info[r]
// packs reaction r's order (bits 0-7) and reactant species r0, r1 (bits 8-15,
// 16-23; 0xff if absent; r0 == r1 for a homodimer) in one dword so that
// uniform reads are scalar loads.  delta[r][s] is the net change of species
// s, deps[r] the reactions whose propensity reads a species r changes.
struct alignas(16) DevModel {
  int32_t S, R, pad0, pad1;
  int32_t info[32];
  int8_t delta[32][16];
  unsigned long long deps[32];
};

// Listing coefficients of one region: a_0 regrouped as
//   N_A V alpha + sum_s beta_s N_s + (1 / N_A V) sum_p gamma_p x_p y_p
// with alpha the summed order-0 constants, beta_s the summed order-1
// constants of species s, and gamma_p the summed order-2 constants of
// reactant pair p (x y = N_a N_b, or N_a (N_a - 1) with the 1/2 folded into
// gamma_p for A + A).
constexpr int kLStride = 56;  // 1 + 16 + 32, rounded up
void listing_pairs(const DevModel& m, int32_t pairs[32], int32_t* n_pairs, int32_t pair_of[32]);
void listing_coefficients(const DevModel& m, const double* k, double* out);  // one region: k[R] -> out[kLStride]

// One run of the batch, as the kernels read it (device memory).
struct alignas(16) RunDesc {
  int32_t* cnt[2];             // [S][T] count buffers; window w reads cnt[w & 1], writes cnt[(w + 1) & 1]
  const int32_t* nbr;          // [T][4] neighbours (-1 = boundary)
  const double* geo;           // [T][4] (G, cum0, cum1, cum2)
  const double* nav;           // [T] N_A V[L]
  const uint8_t* region;       // [T] region labels, nullptr when the model has one region
  const double* kcst;          // [8][32] rate constants by region
  const double* lcoef;         // [8][kLStride] listing coefficients by region (alpha, beta[16], gamma[32])
  unsigned long long* tally;   // [kTallySlots][kTallyWords] SSA events, molecules moved, nonzero
                               // (tet, species, face) moves (summed on read)
  int32_t* err;                // error-flag bits
  int32_t T;
  int32_t n_steps;             // windows of the current sequence (steps 0 .. n_steps-1)
  int32_t n_full;              // steps < n_full last tau, step n_full (if < n_steps) tau_last
  uint32_t window0;            // run-local window index of step 0
  uint32_t key0, key1;         // Philox key = seed
  double tau, tau_last;
  double D[16];                // diffusion coefficients
};

// Arguments of one window of a batch (identical for every window of a
// sequence except k_rel).
struct StepArgs {
  const RunDesc* runs;
  const int2* tile_map;        // [n_tiles] (run, first tet of the tile within the run)
  const int32_t* n_tiles;      // device: number of tiles
  const int32_t* step_base;    // device: step index of k_rel = 0 (nullptr: 0)
  int32_t k_rel;
  int32_t S, R;
  int32_t detect_grid;         // persistent grid of the detect kernel
  int32_t main_grid;           // grid of the main kernel (event blocks + persistent diffusion blocks), >= 2
  int32_t ev_group_max;        // most queued tiles an event block takes as one group (1..64)
  double heavy_events;         // a listed tet with a0 tau_k above this goes to the heavy bin
  int32_t single_run;          // 1: one run, tile t is (run 0, first tet 64 t) without the tile map
  const DevModel* model;
  int32_t info[32];            // = model->info, in kernel arguments for scalar loads
  int32_t n_pairs;             // distinct reactant pairs of the second-order reactions
  int32_t pairs[32];           // a | b << 8 | (a == b) << 16
  // worklist of the tets whose first SSA event falls inside the window: the
  // entries of tile t are slots 64 t .. 64 t + wl_tile_count[t] - 1
  unsigned long long* wl_mask; // [tiles] listed tets of each tile (bit = lane)
  int32_t* wl_tile_count;      // [tiles], valid for the tiles in the queue
  // queues of the tiles with listed tets, one per bin (heavy: tets expected
  // to have more than heavy_events events; light: the others), each in
  // kQueues sub-queues (tile t goes to sub-queue t mod kQueues, slots
  // q * evq_cap ...) so that no counter is contended by every tile; a tile's
  // listed tets take its worklist slots heavy first, wl_tile_count[t] =
  // heavy | light << 8
  int32_t* evq;                // [kBins][kQueues][evq_cap]
  int32_t evq_cap;
  unsigned long long* evq_count;  // [2][kBins][kQueues][16] by step parity, one 128-byte line per
                                  // counter: queued tiles (low word), their listed tets (high word)
  int32_t* wl_tet;
  // diffusion tiles claimed at run time: after its first (static) tile, a
  // diffusion block takes the next unclaimed tile of its sub-range of its
  // XCD's range from tile_ctr[(k & 1)][xcd][sub] (one 128-byte line each);
  // 0: static ranges
  int32_t tile_claim;
  int32_t* tile_ctr;           // [2][8][kClaimSubs][kCtrStride] by step parity
};

constexpr int kCtrStride = 32;  // int32 per claim counter line
constexpr int kClaimSubs = 8;   // claim counters (sub-ranges) per XCD range

constexpr int kQueues = 64;
constexpr int kBins = 2;  // heavy, light
constexpr int kQueueStride = 16;  // u64 per counter line

// Tallies are spread over this many slots per run (block b adds to slot
// b mod kTallySlots), so that blocks finishing together do not queue on one
// address.
constexpr int kTallySlots = 64;
constexpr int kTallyWords = 4;  // SSA events, molecules moved, face moves, unused

// Blocks of the detect and of the main kernel for (S, R) the device holds at
// once (occupancy x compute units).
void grid_resident(int S, int R, int* detect, int* main);

// One window: the detect kernel, then the main kernel; the instance is picked
// by (S, R).  Both are enqueued on `stream`; when `marks` is given,
// marks[0..2] are recorded before, between and after.
hipError_t launch_window(const StepArgs& a, hipStream_t stream, hipEvent_t* marks = nullptr);

// *base += add (one thread): advances the step base at the end of a replayed
// sequence of windows.
hipError_t launch_advance_base(int32_t* base, int32_t add, hipStream_t stream);
// *base = value (one thread).
hipError_t launch_set_base(int32_t* base, int32_t value, hipStream_t stream);

// One chunk of a batched reset: elements [begin, end) of a run's counts are
// copied from src to dst and cleared in other; the chunk with begin == 0 also
// clears the run's tallies and error flag.
struct ResetChunk {
  const int32_t* src;
  int32_t* dst;
  int32_t* other;
  unsigned long long* tally;  // [kTallySlots][kTallyWords]
  int32_t* err;
  int64_t begin, end;
};
constexpr int64_t kResetChunk = 16384;  // elements per chunk
hipError_t launch_reset_chunks(const ResetChunk* chunks, int64_t n_chunks, hipStream_t stream);

// Recording (rdx_record.hip): out [n_regions * S] = per-region sums of the
// counts [S][T]; region may be null when n_regions == 1.  scratch is a device
// array of kRegionScratchBytes for per-block partial sums (calls sharing it
// must be ordered on one stream).
constexpr size_t kRegionScratchBytes = 4096 * 8 * 8;
hipError_t launch_region_counts(const int32_t* counts, const uint8_t* region, int32_t T, int32_t S,
                                int32_t n_regions, unsigned long long* scratch, unsigned long long* out,
                                hipStream_t stream);
// Scratch bytes launch_region_counts writes for T tets and S species (at most
// kRegionScratchBytes).
size_t region_scratch_bytes(int32_t T, int32_t S);
// Device address and size of the static partial-sum array on the current
// device, looked up once per device (hipGetSymbolAddress) and kept; no
// allocation.
hipError_t static_region_scratch(unsigned long long** ptr, size_t* bytes);

hipError_t launch_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_selftest_ln(const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_copy(const int4* src, int4* dst, int64_t n16, hipStream_t s);
hipError_t launch_selftest_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m,
                                 double p, int64_t n, long long* out, hipStream_t s);

}  // namespace rdx
