// rdx_kernels.hpp -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace rdx {

// Model tables in the layout the window kernel reads (one device copy per sim).
// For reaction r: its order, its reactant species (r0 <= r1, -1 if absent;
// r0 == r1 for a homodimer), the net change of each species, and the set of
// reactions whose propensity depends on a species r changes.
struct alignas(16) DevModel {
  int32_t S, R, n_regions, pad;
  int8_t order[32];
  int8_t r0[32];
  int8_t r1[32];
  int8_t delta[32][16];            // net stoichiometric change, [reaction][species]
  unsigned long long deps[32];     // bit j: reaction j must be recomputed after r fires
  double kcst[8][32];              // [region][reaction]
};

// Arguments of one window over one simulation.
struct WindowArgs {
  int32_t* cnt_in;                 // [S][T] counts at the window start; zeroed as they are read
  int32_t* cnt_out;                // [S][T] all zero on entry; receives the counts after the window
  const int32_t* nbr;              // [T][4] int4 per tet
  const double* geo;               // [T][4] (G, c0, c1, c2) double4 per tet
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
};

// Picks the kernel instance by (S, R) and launches it on `stream`.
hipError_t launch_window(const WindowArgs& a, hipStream_t stream);

hipError_t launch_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_selftest_ln(const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_selftest_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m,
                                 double p, int64_t n, long long* out, hipStream_t s);

}  // namespace rdx
