// rdx_internal.hpp -- host-side types shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "rdx.h"

namespace rdx {

// Compile-time limits of the window kernels (per-lane state lives in registers).
constexpr int kMaxSpecies = 16;
constexpr int kMaxReactions = 32;
constexpr int kMaxRegions = 8;
constexpr int kMaxChanges = 8;
constexpr int32_t kCountCap = 1 << 30;   // a count above this raises RDX_EOVERFLOW
constexpr int32_t kEventCap = 1 << 22;   // SSA events per tet per window before RDX_EEVENTS

// Device-error flag bits (set by kernels, read by rdx_sync / rdx_get_stats).
constexpr int kErrOverflow = 1;
constexpr int kErrEvents = 2;

// The set-up step of section 2.1, computed once on the host.
struct HostInstance {
  int32_t T = 0, S = 0, R = 0, n_regions = 1;
  std::vector<int32_t> nbr;      // [T*4] neighbour across face k (opposite local vertex k), -1 boundary
  std::vector<double> g;         // [T*4] A_k / (V h_k), 0 on boundary faces
  std::vector<double> G;         // [T]   g_0 + (g_1 + (g_2 + g_3))
  std::vector<double> cum;       // [T*4] (g_0 + ... + g_k) / G for k < 3, cum_3 = 1
  std::vector<double> nav;       // [T]   N_A * V[L]
  std::vector<uint8_t> region;   // [T]
  std::vector<double> D;         // [S]
  std::vector<int32_t> lhs, rhs; // [R*S]
  std::vector<double> kcst;      // [n_regions*R]
  double tau = 0.0;
};

// Validates the inputs and fills `out`.  Returns RDX_OK or an error status
// with a message in *err.
rdx_status build_instance(const rdx_mesh* mesh, const rdx_model* model, double tau_override,
                          HostInstance* out, std::string* err);

// Thread-local last-error helpers.
rdx_status set_error(rdx_status st, const std::string& msg);
void clear_error();

}  // namespace rdx
