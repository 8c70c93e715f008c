// rdx_kernels.hpp -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace rdx {

// Model tables in the layout the window kernels read (one device copy per sim).
// info[r] packs reaction r's order (bits 0-7) and reactant species r0, r1
// (bits 8-15, 16-23; 0xff if absent; r0 == r1 for a homodimer) in one dword so
// that uniform reads are scalar loads.  delta[r][s] is the net change of
// species s, deps[r] the reactions whose propensity reads a species r changes.
struct alignas(16) DevModel {
  int32_t S, R, n_regions, pad;
  int32_t info[32];
  int8_t delta[32][16];
  unsigned long long deps[32];
  double kcst[8][32];              // [region][reaction]
};

// The reaction constants the all-tets kernel reads from its kernel arguments:
// packed reaction info and the rate constants of region 0 (models with several
// regions read DevModel::kcst per tet).
struct alignas(16) KModel {
  int32_t info[32];
  double kcst0[32];
};

// Arguments of one window over one simulation.
struct WindowArgs {
  int32_t* cnt_in;                 // [S][T] counts at the window start; zeroed as they are read
  int32_t* cnt_out;                // [S][T] all zero on entry; receives the counts after the window
  const int32_t* nbr;              // [T][4] int4 per tet
  const double* geo;               // [T][4] (G, cum0, cum1, cum2) double4 per tet
  const double* nav;               // [T]
  const uint8_t* region;           // [T] or nullptr
  const DevModel* model;
  unsigned long long* tally;       // [2] SSA events, molecules moved
  int* err;                        // error-flag bits
  int32_t T;
  int32_t S, R;
  uint32_t key0, key1;
  uint32_t window;
  double tau_k;
  double tauD[16];                 // tau_k * D_s, 0 for immobile species
  int32_t* wl_tet;                 // [T] tets with an SSA event in this window
  int32_t* wl_cnt;                 // [S][T] their counts at the window start (row stride T)
  double* wl_nav;                  // [T] their N_A V[L]
  int32_t* wl_nbr;                 // [T][4] their neighbours
  double* wl_geo;                  // [T][4] their (G, cum0, cum1, cum2)
  int32_t* wl_count;               // length of this window's list (zero on entry)
  int32_t* wl_reset;               // the other list length, zeroed for the next window
  int32_t event_blocks;            // grid of the event kernel
  KModel km;
};

// One window: the all-tets kernel, then the event kernel over the tets it
// listed; the instance is picked by (S, R).  Both are enqueued on `stream`;
// when `marks` is given, marks[0..2] are recorded before, between and after.
hipError_t launch_window(const WindowArgs& a, hipStream_t stream, hipEvent_t* marks = nullptr);

hipError_t launch_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_selftest_ln(const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_copy(const int4* src, int4* dst, int64_t n16, hipStream_t s);
hipError_t launch_selftest_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m,
                                 double p, int64_t n, long long* out, hipStream_t s);

}  // namespace rdx
