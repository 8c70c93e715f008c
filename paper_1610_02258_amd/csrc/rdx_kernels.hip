// rdx_kernels.hip -- gfx950 kernels of the operator-splitting reaction-diffusion
// window ("Parallel STEPS", Algorithm 1), one lane per tetrahedron.
//
// Per window and tet, in the paper's order:
//   1. load the tet's counts (species-major SoA, coalesced over tets);
//   2. the reaction SSA operator: propensities of the tet's reactions, exact
//      SSA events until the next one would fall outside the window, reaction
//      selection by composition-rejection (Slepoy, Thompson & Plimpton 2008),
//      FP64 time, occupancy O_S += N_S (dt - t_S) for every species an event
//      changes, finalised at the window end;
//   3. the diffusion operator for each diffusive species: mean occupancy
//      Nbar = O_S / tau, leavers Bin(round(Nbar), tau D_S G) (stochastic
//      rounding, at most the post-reaction count), each leaver sent to a face
//      with probability g_k / G (per-molecule draws for small counts);
//   4. integer adds of the remainder and of the face moves into the next
//      count buffer -- the single-GPU form of the paper's local application
//      plus remote change buffers; integer addition makes the result
//      independent of order.
// Random numbers are Philox4x32-10 (Salmon et al., SC'11) with the counter
// (draw call, stream, tet, window); stream 0 is the tet's SSA, stream 1+s the
// diffusion of species s.  The logarithm and the binomial use only correctly
// rounded IEEE-754 binary64 operations in a fixed order (no fp contraction),
// so results are reproducible bit for bit on any IEEE implementation of the
// same operation sequence.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "rdx_internal.hpp"
#include "rdx_kernels.hpp"

#pragma clang fp contract(off)

namespace rdx {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- Philox ----
// a ^ b ^ k in one VALU instruction, k wave-uniform (an SGPR operand):
// gfx950's three-input bitwise op with truth table 0x96 (odd parity); the
// compiler would split the three-way xor into two v_xor_b32.
__device__ __forceinline__ uint32_t xor3_sk(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// The key (the run's seed) must be the same on every lane of the wave.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32x32->64 multiply each (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = xor3_sk((uint32_t)(p1 >> 32), x1, k0);
    const uint32_t y2 = xor3_sk((uint32_t)(p0 >> 32), x3, k1);
    x0 = y0;
    x1 = (uint32_t)p1;
    x2 = y2;
    x3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// SSA stream: 53-bit uniforms, two per Philox call (words 0-1, then 2-3).
struct Draw53 {
  uint32_t k0, k1, sid, tet, win, call;
  uint64_t spare;
  bool has_spare;
  __device__ Draw53(uint32_t key0, uint32_t key1, uint32_t stream, uint32_t t, uint32_t w)
      : k0(key0), k1(key1), sid(stream), tet(t), win(w), call(0), spare(0), has_spare(false) {}
  __device__ __forceinline__ uint64_t next() {
    if (has_spare) {
      has_spare = false;
      return spare;
    }
    uint32_t x0 = call, x1 = sid, x2 = tet, x3 = win;
    philox4x32_10(x0, x1, x2, x3, k0, k1);
    ++call;
    spare = ((uint64_t)x2 << 21) | (uint64_t)(x3 >> 11);
    has_spare = true;
    return ((uint64_t)x0 << 21) | (uint64_t)(x1 >> 11);
  }
  __device__ __forceinline__ double co() { return (double)next() * 0x1p-53; }        // [0, 1)
  __device__ __forceinline__ double oc() { return (double)(next() + 1u) * 0x1p-53; } // (0, 1]
};

// Species stream: 32-bit uniforms in [0, 1), four per Philox call.
struct Draw32 {
  uint32_t k0, k1, sid, tet, win, call;
  uint32_t w0, w1, w2, w3;
  int pos;
  __device__ Draw32(uint32_t key0, uint32_t key1, uint32_t stream, uint32_t t, uint32_t w)
      : k0(key0), k1(key1), sid(stream), tet(t), win(w), call(0), w0(0), w1(0), w2(0), w3(0),
        pos(4) {}
  // Computes the stream's first Philox call up front, so that every item of a
  // wave refills at the same program point (draw values are unchanged).
  __device__ __forceinline__ void prime() {
    w0 = call;
    w1 = sid;
    w2 = tet;
    w3 = win;
    philox4x32_10(w0, w1, w2, w3, k0, k1);
    ++call;
    pos = 0;
  }
  // The stream's next Philox call (all four words unused).
  __device__ __forceinline__ void refill() {
    w0 = call;
    w1 = sid;
    w2 = tet;
    w3 = win;
    philox4x32_10(w0, w1, w2, w3, k0, k1);
    ++call;
    pos = 0;
  }
  // The next 32-bit word of the stream, and the uniform w 2^-32 it stands for.
  __device__ __forceinline__ uint32_t word() {
    if (pos == 4) refill();
    const uint32_t w = pos == 0 ? w0 : (pos == 1 ? w1 : (pos == 2 ? w2 : w3));
    ++pos;
    return w;
  }
  __device__ __forceinline__ double u() { return (double)word() * 0x1p-32; }
};

// ------------------------------------------------------------------ ln ----
// x = m 2^e, m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s) with s = (m-1)/(m+1)
// summed to s^21; e ln 2 added through the Cody-Waite split of ln 2.
__device__ __forceinline__ double ln_basic(double x) {
  const long long bits = __double_as_longlong(x);
  int e = (int)((bits >> 52) & 0x7ff) - 1022;
  double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3fe0000000000000LL);
  if (m < 0.70710678118654752440) {
    m = m + m;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0;
  const double lnm = (s + s) * p;
  const double de = (double)e;
  const double ln2_hi = 6.93147180369123816490e-01;  // 0x3fe62e42fee00000
  const double ln2_lo = 1.90821492927058770002e-10;  // 0x3dea39ef35793c76
  return de * ln2_hi + (de * ln2_lo + lnm);
}

// ------------------------------------------------------------ binomial ----
// Sequential-search inversion, one uniform per chunk of <= 1000 trials
// (q^c >= 2^-1000 stays normal), complement for p > 1/2.
__device__ __forceinline__ double pow_int(double q, int c) {
  double result = 1.0, base = q;
  while (c > 0) {
    if (c & 1) result = result * base;
    base = base * base;
    c >>= 1;
  }
  return result;
}

// Reciprocals 1/(k + 1) for k < 1000 (every step of a chunk's search),
// rounded once, at compile time, as the division rounds them.  The search's
// step counter is the same on every lane of a wave (the lanes step together),
// so the table is read with scalar loads that do not depend on the running
// pmf value, instead of a double division on the search's dependent chain.
struct ReciprocalTable {
  double v[1000];
  constexpr ReciprocalTable() : v() {
    for (int k = 0; k < 1000; ++k) v[k] = 1.0 / (double)(k + 1);
  }
};
__constant__ constexpr ReciprocalTable kRecip{};

__device__ long long binom_core(long long m, double p, Draw32& st) {
  const double q = 1.0 - p;
  const double r = p / q;
  long long total = 0;
  while (m > 0) {
    const int c = m < 1000 ? (int)m : 1000;
    const double u = st.u();
    double f = pow_int(q, c);
    double F = f;
    int k = 0;
    while (u >= F && k < c) {
      f = ((f * r) * (double)(c - k)) * kRecip.v[k];
      k = k + 1;
      F = F + f;
    }
    total += k;
    m -= c;
  }
  return total;
}

// One code path for both sides of 1/2 (the complement is taken by flipping),
// so that lanes of a wave with different p do not run two copies.
__device__ __forceinline__ long long binom(long long m, double p, Draw32& st) {
  if (m <= 0 || !(p > 0.0)) return 0;
  if (p >= 1.0) return m;
  const bool flip = p > 0.5;
  const long long k = binom_core(m, flip ? 1.0 - p : p, st);
  return flip ? m - k : k;
}

// ---------------------------------------------------------- propensity ----
__device__ __forceinline__ int exp_field(double a) {
  return (int)((__double_as_longlong(a) >> 52) & 0x7ff);
}

// a_r = c_r h_r(N) with c = k N_A V[L] (order 0), k (order 1), k / (N_A V[L])
// (order 2) and h = 1, N_A, N_A N_B or N_A (N_A - 1) / 2, in a branch-free
// form whose products are those of the case-by-case definition: h = (x y) w
// with x = N_A (1 for order 0), y = N_B, N_A - 1 (A + A) or 1, w = 1/2 for
// A + A, and c = k f with f = N_A V, 1 or 1 / (N_A V).  Values below 2^-1000
// are taken as zero.  `info` is the packed reaction entry (uniform); `N`
// holds the counts as one vector value, so that the uniform species index
// selects a register.
template <int SMAX, typename NV>
__device__ __forceinline__ double propensity(int info, double k, const NV& N, double nav, double inv_nav) {
  const int order = info & 0xff;
  const int s0 = (info >> 8) & 0xff, s1 = (info >> 16) & 0xff;
  const bool same = order == 2 && s0 == s1;
  const int x = order == 0 ? 1 : (s0 < SMAX ? N[s0] : 0);
  const int y = order == 2 ? (s1 < SMAX ? N[s1] : 0) - (same ? 1 : 0) : 1;
  const double f = order == 0 ? nav : (order == 1 ? 1.0 : inv_nav);
  const double v = (k * f) * (((double)x * (double)y) * (same ? 0.5 : 1.0));
  return v >= 0x1p-1000 ? v : 0.0;
}

// Composition: groups of reactions with equal binary exponent, visited from
// the largest exponent down, picked with probability proportional to their
// totals; rejection: a uniform member is accepted with probability a / 2^g.
// Group totals are summed in reaction order.  The propensities are the
// lane's column of an LDS table (a_r at col[r * stride]); the scans are
// loops, so that one SSA step stays a short stretch of code.
__device__ int cr_select_col(const double* col, int stride, int R, double a0, Draw53& st) {
  double x = st.co() * a0;
  int gprev = 4096, chosen = -1;
  for (;;) {
    int gcur = -1;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
      const double v = col[r * stride];
      const int e = v > 0.0 ? exp_field(v) : -1;
      if (e < gprev && e > gcur) gcur = e;
    }
    if (gcur < 0) break;
    double sum = 0.0;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
      const double v = col[r * stride];
      if (v > 0.0 && exp_field(v) == gcur) sum = sum + v;
    }
    chosen = gcur;
    if (x < sum) break;
    x = x - sum;
    gprev = gcur;
  }
  int n = 0;
#pragma unroll 4
  for (int r = 0; r < R; ++r) {
    const double v = col[r * stride];
    n += (v > 0.0 && exp_field(v) == chosen) ? 1 : 0;
  }
  const double bound = __longlong_as_double((long long)(chosen + 1) << 52);
  for (;;) {
    const double u2 = st.co();
    int j = (int)(u2 * (double)n);
    if (j >= n) j = n - 1;
    const double u3 = st.co();
    double aj = 0.0;
    int rj = 0, seen = 0;
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
      const double v = col[r * stride];
      if (v > 0.0 && exp_field(v) == chosen) {
        if (seen == j) {
          aj = v;
          rj = r;
        }
        ++seen;
      }
    }
    if (u3 * bound < aj) return rj;
  }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ------------------------------------------------------- window kernels ----
// A window of a batch is two launches, one wave (64 lanes) per block, one lane
// per tet, 64 tets per tile (a tile belongs to one run).
//
// window_detect_kernel, over all tiles: a0 from regrouped coefficients and the
// tet's first SSA uniform.  A tet whose first event may fall inside the
// window is listed (its index goes to the tile's worklist slots, the tile to
// one of 64 sub-queues); a per-tile bit mask marks the listed tets.
//
// window_main_kernel: its first blocks take groups of queued tiles and run
// the full SSA window (composition-rejection, occupancy) and the diffusion of
// the listed tets; the other blocks walk all tiles and do the diffusion of
// every tet that is not listed (no count changes, the mean occupancy is the
// count itself).  The serial SSA chains of the few listed tets so run
// alongside the diffusion of the rest instead of after it.
//
// Diffusion items: every (tet, species) pair with something to sample becomes
// an item; ballots pack them into LDS (items of more than 16 molecules first,
// species-major), and they are sampled in rounds of 64 (item_round).  Moves
// into the tile's own tets accumulate in LDS and are flushed once, coalesced;
// the rest are integer atomics into the next count buffer.
constexpr int kWave = 64;

// Tables the window kernels only read -- the run table, the tile map, the
// reaction tables, the step base and tile count -- are read through the
// constant address space: nothing writes them while a kernel runs, and a
// uniform address can then be served by a scalar load, whose wait does not
// hold up the vector loads in flight.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}

// Element j of a read-only int4 / double2 array through the constant address
// space (the HIP vector types cannot be copied out of it directly).
typedef int int4_v __attribute__((ext_vector_type(4)));
typedef double double2_v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int4 ld_int4(const int4* p, size_t j) {
  const int4_v v = ((cptr<int4_v>)p)[j];
  return make_int4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double2 ld_double2(const double2* p, size_t j) {
  const double2_v v = ((cptr<double2_v>)p)[j];
  return make_double2(v.x, v.y);
}

// Every block of the window kernels is a single wave: its lanes execute in
// lockstep and its LDS operations complete in issue order, so handing LDS
// data from lane to lane only needs the compiler to keep the accesses in
// program order (a wavefront-scope fence), not a workgroup barrier, whose
// fence would also wait for every global load and atomic in flight.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_inclusive_scan(int v) {
  // v in [0, 31]: the sum over lanes <= this one, one bit plane at a time
  // (five ballots and bit counts; no LDS traffic)
  int acc = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const unsigned long long m = __ballot((v >> b) & 1);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    acc += (int)((below + (uint32_t)((v >> b) & 1)) << b);
  }
  return acc;
}

// Inclusive prefix sum over the 64 lanes for any int (six shuffle steps).
__device__ __forceinline__ int wave_scan_add(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int u = __shfl_up(v, d, kWave);
    if (lane >= d) v += u;
  }
  return v;
}

// Diffusion items.  An item is one (tet, species) pair of a window: m trials
// of leaving, m = nbar stochastically rounded (a draw only when nbar is
// fractional).  With m <= 16 every molecule draws one 32-bit uniform u and
// leaves when u < p, to the first face k before the last face present with
// u < p cum_k, else to the last face; once npost molecules have left the
// rest stay.  With m > 16 the faces in order take successive binomials of
// the molecules not yet placed (face k: Bin(rest, p s_k / (1 - p cum_{k-1})),
// s_k the face's share of the couplings) and the rest stay; should more than
// npost leave, npost leave instead, split afresh by the shares.  Both are
// exact samplers of binomial leavers split among the faces in proportion to
// the face couplings.
//
// The per-molecule draws of an item (m <= 16) are the words w0, w0 + 1, ...
// of its species stream, w0 the words the rounding used (0 or 1); word j is
// word j mod 4 of Philox call j / 4, so an item takes at most five calls,
// which its own lane makes, testing the words against the item's
// probabilities.  (With m > npost the cap can bind in the middle of the
// walk; such an item -- only a tet whose counts changed in the window can
// have one -- is walked word by word in stream order.)
constexpr int kSmallM = 16;

struct ItemMoves {
  int n, o0, o1, o2, o3;
};

// A draw w stands for the uniform w 2^-32, and w 2^-32 < t holds exactly
// when w < ceil(t 2^32) (t 2^32 is exact in binary64).  For t in [0, 1] the
// threshold is at most 2^32: returned as a 32-bit value, with `full` set when
// it is 2^32 (every draw passes).
__device__ __forceinline__ uint32_t draw_threshold(double t, bool& full) {
  const double c = ceil(t * 0x1p32);
  full = c >= 0x1p32;
  return full ? 0xffffffffu : (uint32_t)c;
}

__device__ __forceinline__ int last_face(int4 nb) {
  return nb.w >= 0 ? 3 : (nb.z >= 0 ? 2 : (nb.y >= 0 ? 1 : 0));
}

// Per-lane face counts of a round's split and walked items.
struct ItemLds {
  uint32_t face[4][kWave];  // leavers by face of the split and walked items, by lane
};

// The per-tet arrays a round reads, by tet lane (LDS of the tile or chunk).
struct ItemView {
  const int4* nbr;      // neighbours
  const double2* geo0;  // (G, cum0)
  const double2* geo1;  // (cum1, cum2)
  const double* tauD;   // tau_k D_s by species
  const int* tet;       // run-local tet of each tet lane, or null: base + lane
  int base;
  __device__ __forceinline__ uint32_t tet_of(int ln) const { return (uint32_t)(tet ? tet[ln] : base + ln); }
};

// What a lane brings to a round: its item, or valid == false.
struct ItemIn {
  bool valid;
  int sp;      // species
  int ln;      // tet lane
  double nbar; // mean occupancy (the count itself when nothing changed it)
  int npost;   // count after the reactions
};

// Face of a leaving draw w: the number of faces k < last whose threshold w
// reaches (the thresholds rise with k; faces at or after `last` carry the
// "never" bit), and whether w leaves at all.
__device__ __forceinline__ int draw_face(uint32_t w, uint32_t t0, uint32_t t1, uint32_t t2, uint32_t full) {
  return (int)(((full & 1u) == 0u && w >= t0)) + (int)(((full & 2u) == 0u && w >= t1)) +
         (int)(((full & 4u) == 0u && w >= t2));
}

__device__ __forceinline__ bool draw_leaves(uint32_t w, uint32_t ts, uint32_t full) {
  return (full & 8u) != 0u || w < ts;
}

// The item's leave probability: min(1, tau_k D_s G).
__device__ __forceinline__ double item_p(const ItemView& V, int sp, int ln) {
  const double pr = V.tauD[sp] * V.geo0[ln].x;
  return pr > 1.0 ? 1.0 : pr;
}

// Integer thresholds of an item's face draws (scale = p); `full` bit k:
// threshold k is never reached (k at or after the last face) or always
// (2^32), bit 3: every draw leaves.
__device__ __forceinline__ void item_thresholds(const ItemView& V, int ln, double scale, uint32_t th[4],
                                                uint32_t& full) {
  const int last = last_face(V.nbr[ln]);
  const double2 g0 = V.geo0[ln], g1 = V.geo1[ln];
  bool f0, f1, f2, fs;
  th[0] = draw_threshold(scale * g0.y, f0);
  th[1] = draw_threshold(scale * g1.x, f1);
  th[2] = draw_threshold(scale * g1.y, f2);
  th[3] = draw_threshold(scale, fs);
  full = (f0 || last <= 0 ? 1u : 0u) | (f1 || last <= 1 ? 2u : 0u) | (f2 || last <= 2 ? 4u : 0u) | (fs ? 8u : 0u);
}

__device__ ItemMoves item_round(uint32_t key0, uint32_t key1, uint32_t window, const ItemIn& it,
                                const ItemView& V, ItemLds& X) {
  const int lane = threadIdx.x;
  uint32_t own = 0;     // leavers by face drawn on this lane, a byte each
  bool walked = false;  // this lane's face counts are in X.face, by the walk
  bool split = false;   // this lane's face counts are in X.face, by the split
  if (it.valid) {
    const uint32_t tet = V.tet_of(it.ln);
    Draw32 st(key0, key1, 1u + (uint32_t)it.sp, tet, window);
    const double fl = floor(it.nbar);
    const double frac = it.nbar - fl;
    long long m = (long long)fl;
    uint32_t used = 0;  // words taken before the face draws
    if (frac > 0.0) {
      if (st.u() < frac) m += 1;
      used = 1;
    }
    const double p = item_p(V, it.sp, it.ln);
    long long trials = 0;
    if (m > 0 && p > 0.0) {
      if (m <= kSmallM) {
        trials = m;
        walked = m > (long long)it.npost;  // the cap may bind mid-walk
      } else {
        // the multinomial over the faces and staying, one binomial per stage
        // from one call site, in stream order on this lane: stage k <= last
        // gives face k Bin(rest, p s_k / (1 - p cum_{k-1})) of the molecules
        // not yet placed (s_k the face's share, the last face present taking
        // all that remains of p), the rest stay.  Should more leave than
        // the post-reaction count (only a listed tet's item can), stages
        // last + 1 .. 2 last split that count afresh by the shares (face k
        // Bin(rest, s_k / (1 - cum_{k-1})), the last face the rest).
        const int last = last_face(V.nbr[it.ln]);
        const double2 g0 = V.geo0[it.ln], g1 = V.geo1[it.ln];
        const long long npost = (long long)it.npost;
        long long rest = m, n = 0;
        double prev = 0.0;
        bool capped = false;
        int end = last;
#pragma unroll 1
        for (int stage = 0; stage <= end; ++stage) {
          const int f = capped ? stage - last - 1 : stage;
          const double cum = (!capped && f == last) ? 1.0 : (f == 0 ? g0.y : (f == 1 ? g1.x : g1.y));
          double qq;
          if (!capped) {
            // den is 0 only for p = 1 with the shares before face f summing to 1
            const double den = 1.0 - p * prev;
            qq = den > 0.0 ? (p * (cum - prev)) / den : (f == last ? 1.0 : 0.0);
          } else {
            qq = (cum - prev) / (1.0 - prev);
          }
          const long long k = binom(rest, qq, st);
          X.face[f][lane] = (uint32_t)k;
          rest -= k;
          prev = cum;
          if (!capped) {
            n += k;
            if (f == last && n > npost) {
              capped = true;
              end = last + last;
              rest = npost;
              prev = 0.0;
            }
          }
        }
        if (capped) X.face[last][lane] = (uint32_t)rest;
#pragma unroll
        for (int f = 0; f < 4; ++f)
          if (f > last) X.face[f][lane] = 0u;
        split = true;
      }
    }
    const uint32_t w0 = used, nw = (uint32_t)trials;
    if (nw > 0u && !walked) {
      // at most five Philox calls (16 draws after the rounding draw): this
      // lane makes them, comparing each uniform w 2^-32 with the item's
      // probabilities as they are (the face counts fit a byte each)
      const int last = last_face(V.nbr[it.ln]);
      const double2 g0 = V.geo0[it.ln], g1 = V.geo1[it.ln];
      // u = w 2^-32 < t exactly when w < t 2^32 (both scalings are exact), so
      // the words are compared, as doubles, with the thresholds scaled once
      const double ts = p * 0x1p32;
      const double t0 = (p * g0.y) * 0x1p32, t1 = (p * g1.x) * 0x1p32, t2 = (p * g1.y) * 0x1p32;
      for (uint32_t call = w0 >> 2; call <= (w0 + nw - 1u) >> 2; ++call) {
        uint32_t x0 = call, x1 = 1u + (uint32_t)it.sp, x2 = tet, x3 = window;
        philox4x32_10(x0, x1, x2, x3, key0, key1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t w = q == 0 ? x0 : (q == 1 ? x1 : (q == 2 ? x2 : x3));
          const uint32_t idx = 4u * call + (uint32_t)q;
          const double u = (double)w;
          if (idx >= w0 && idx - w0 < nw && u < ts) {
            const int f = (0 < last && u < t0) ? 0 : ((1 < last && u < t1) ? 1 : ((2 < last && u < t2) ? 2 : last));
            own += 1u << (8 * f);
          }
        }
      }
    }
    if (walked) {  // in stream order, after the rounding draw
      uint32_t th[4], full;
      item_thresholds(V, it.ln, p, th, full);
#pragma unroll
      for (int k = 0; k < 4; ++k) X.face[k][lane] = 0u;
      long long n = 0;
      for (long long j = 0; j < trials; ++j) {
        const uint32_t w = st.word();
        if (draw_leaves(w, th[3], full) && n < (long long)it.npost) {
          X.face[draw_face(w, th[0], th[1], th[2], full)][lane] += 1u;
          ++n;
        }
      }
    }
  }
  ItemMoves r{0, 0, 0, 0, 0};
  if (it.valid) {
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = ((own >> (8 * k)) & 0xffu) + (walked || split ? X.face[k][lane] : 0u);
    r.o0 = (int)o[0];
    r.o1 = (int)o[1];
    r.o2 = (int)o[2];
    r.o3 = (int)o[3];
    r.n = r.o0 + r.o1 + r.o2 + r.o3;
  }
  return r;
}

// item_round for a round in which every item is a diffusion-only tet's
// species with at most 16 molecules (mean occupancy = count = npost, so no
// rounding draw, no binomial, no cap, words 0 .. m-1 of the stream): the
// same draws and decisions as item_round's own-lane path, without its
// set-up for the other cases.
__device__ __forceinline__ ItemMoves item_round_small(uint32_t key0, uint32_t key1, uint32_t window,
                                                     const ItemIn& it, const ItemView& V) {
  uint32_t own = 0;  // leavers by face, a byte each
  if (it.valid) {
    const uint32_t tet = V.tet_of(it.ln);
    const double p = item_p(V, it.sp, it.ln);
    const uint32_t m = (uint32_t)it.npost;
    if (p > 0.0) {
      const int last = last_face(V.nbr[it.ln]);
      const double2 g0 = V.geo0[it.ln], g1 = V.geo1[it.ln];
      // the words against the thresholds scaled by 2^32 (exact, as above)
      const double ps = p * 0x1p32;
      const double t0 = (p * g0.y) * 0x1p32, t1 = (p * g1.x) * 0x1p32, t2 = (p * g1.y) * 0x1p32;
      const uint32_t calls = (m + 3u) >> 2;
      for (uint32_t call = 0; call < calls; ++call) {
        uint32_t x0 = call, x1 = 1u + (uint32_t)it.sp, x2 = tet, x3 = window;
        philox4x32_10(x0, x1, x2, x3, key0, key1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t w = q == 0 ? x0 : (q == 1 ? x1 : (q == 2 ? x2 : x3));
          const double u = (double)w;
          if (4u * call + (uint32_t)q < m && u < ps) {
            const int f = (0 < last && u < t0) ? 0 : ((1 < last && u < t1) ? 1 : ((2 < last && u < t2) ? 2 : last));
            own += 1u << (8 * f);
          }
        }
      }
    }
  }
  ItemMoves r;
  r.o0 = (int)(own & 0xffu);
  r.o1 = (int)((own >> 8) & 0xffu);
  r.o2 = (int)((own >> 16) & 0xffu);
  r.o3 = (int)(own >> 24);
  r.n = r.o0 + r.o1 + r.o2 + r.o3;
  return r;
}

// Tile schedule of a persistent block: the blocks are dispatched round-robin
// over the 8 XCDs, so XCD x (= block % 8) owns one contiguous range of tiles
// (its L2 then sees neighbouring tets), shared round-robin by its blocks.
// The schedule is static: per-tile work is balanced by the grid size (every
// block gets the same number of tiles, to within one).
struct TileRange {
  int first, end, stride;
};

__device__ __forceinline__ TileRange tile_range(int b, int G, int n_tiles) {
  if (G < 8 || n_tiles < 8) return TileRange{b, n_tiles, G};
  const int x = b & 7, j = b >> 3;
  const int Gx = (G - x + 7) >> 3;  // blocks with block % 8 == x
  const int lo = (int)(((long long)n_tiles * x) >> 3);
  const int hi = (int)(((long long)n_tiles * (x + 1)) >> 3);
  return TileRange{lo + j, hi, Gx};
}

// The run a tile belongs to and what this step is for that run.
struct TileCtx {
  cptr<RunDesc> rd;
  int run;
  int base;        // first tet of the tile, run-local
  int T;
  bool active;     // the run takes part in this step
  uint32_t window; // run-local window index
  double tau_k;
  int32_t* cin;
  int32_t* cout;
};

__device__ __forceinline__ TileCtx tile_ctx(const StepArgs& A, int tile, int k) {
  // with one run the tile map is (0, 64 t): no load on the chain to the counts
  const int run = A.single_run ? 0 : as_const(reinterpret_cast<const int*>(A.tile_map))[2 * tile];
  const int first = A.single_run ? tile * kWave : as_const(reinterpret_cast<const int*>(A.tile_map))[2 * tile + 1];
  const cptr<RunDesc> rd = as_const(A.runs) + run;
  TileCtx c;
  c.rd = rd;
  c.run = run;
  c.base = first;
  c.T = rd->T;
  c.active = k < rd->n_steps;
  c.window = rd->window0 + (uint32_t)k;
  c.tau_k = k < rd->n_full ? rd->tau : rd->tau_last;
  c.cin = rd->cnt[c.window & 1u];
  c.cout = rd->cnt[(c.window + 1u) & 1u];
  return c;
}

// Everything one lane reads from global memory for its tet.
template <int SMAX>
struct TetData {
  // counts as one vector value, so that a uniform (run-time) species index
  // selects a register rather than spilling the array to memory
  int __attribute__((ext_vector_type(SMAX))) N;
  double nav;
  int4 nb;
  double2 ga, gb;  // (G, cum0), (cum1, cum2)
  int reg;
};

template <int SMAX>
__device__ __forceinline__ void load_tet(const TileCtx& c, int S, int i, TetData<SMAX>& d) {
  const bool active = c.active && i < c.T;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) d.N[s] = (active && s < S) ? c.cin[(size_t)s * c.T + i] : 0;
  d.nav = 1.0;
  d.nb = make_int4(-1, -1, -1, -1);
  d.ga = make_double2(0.0, 0.0);
  d.gb = make_double2(0.0, 0.0);
  d.reg = 0;
  if (active) {
    d.nav = as_const(c.rd->nav)[i];
    d.nb = ld_int4(reinterpret_cast<const int4*>(c.rd->nbr), (size_t)i);
    d.ga = ld_double2(reinterpret_cast<const double2*>(c.rd->geo), 2 * (size_t)i);
    d.gb = ld_double2(reinterpret_cast<const double2*>(c.rd->geo), 2 * (size_t)i + 1);
    if (c.rd->region) d.reg = as_const(c.rd->region)[i];
  }
}

__device__ __forceinline__ unsigned long long* tally_slot(const StepArgs& A, int run) {
  return as_const(A.runs)[run].tally + kTallyWords * (blockIdx.x & (kTallySlots - 1));
}

__device__ __forceinline__ int step_index(const StepArgs& A) {
  return (A.step_base ? *as_const(A.step_base) : 0) + A.k_rel;
}

// What the detect kernel reads for one lane's tet.
template <int SMAX>
struct TetCounts {
  int __attribute__((ext_vector_type(SMAX))) N;  // a uniform species index selects a register
  double nav;
  int reg;
};

template <int SMAX>
__device__ __forceinline__ void load_counts(const TileCtx& c, int S, int i, TetCounts<SMAX>& d) {
  const bool active = c.active && i < c.T;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) d.N[s] = (active && s < S) ? c.cin[(size_t)s * c.T + i] : 0;
  d.nav = active ? as_const(c.rd->nav)[i] : 1.0;
  d.reg = (active && c.rd->region) ? (int)as_const(c.rd->region)[i] : 0;
}

// a_0 of one tet from the regrouped listing coefficients of its region (`lc`,
// a scalar pointer when the run has one region, a per-lane one otherwise).
// The terms are those of the reaction-by-reaction sum, so the result agrees
// with it to within a few roundings (relative 1e-14 at most; fused
// multiply-adds are fine here); it is only used with a margin far above that.
template <int SMAX, typename P, typename NV>
__device__ __forceinline__ double listing_rate(const StepArgs& A, P lc, const NV& N, double nav, double inv_nav) {
  // beta_s is zero for s >= S, and so are the counts there
  double lin = nav * lc[0];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) lin = __builtin_fma(lc[1 + s], (double)N[s], lin);
  double quad = 0.0;
#pragma unroll 1
  for (int p = 0; p < A.n_pairs; ++p) {
    const int pr = A.pairs[p];
    const int a = pr & 0xff, b = (pr >> 8) & 0xff;
    const int x = a < SMAX ? N[a] : 0;
    const int y = (b < SMAX ? N[b] : 0) - ((pr >> 16) & 1);
    quad = __builtin_fma(lc[17 + p], (double)x * (double)y, quad);
  }
  return __builtin_fma(inv_nav, quad, lin);
}

// One block per tile by default (the grid may also be smaller: a block then
// walks its tiles, the next tile's loads in flight while the current one is
// worked on).
template <int SMAX, int RMAX>
__global__ void __launch_bounds__(kWave) window_detect_kernel(const StepArgs A) {
  const int lane = threadIdx.x;
  const int S = A.S;
  const int k = step_index(A);
  const int n_tiles = *as_const(A.n_tiles);
  const TileRange tr = tile_range(blockIdx.x, gridDim.x, n_tiles);

  TileCtx cc, nc;
  TetCounts<SMAX> cur, nxt;
  if (tr.first < tr.end) {
    cc = tile_ctx(A, tr.first, k);
    load_counts<SMAX>(cc, S, cc.base + lane, cur);
  }
  nc = cc;

  for (int tile = tr.first; tile < tr.end; tile += tr.stride) {
    const bool has_next = tile + tr.stride < tr.end;
    const bool run_active = cc.active;
    const cptr<RunDesc> rd = cc.rd;
    const int i = cc.base + lane;
    const bool active = i < cc.T;

    // a_0 from the listing coefficients
    const double nav = cur.nav;
    const int reg = cur.reg;
    const auto Nc = cur.N;
    double a0 = 0.0;
    if (run_active) {
      const double inv_nav = 1.0 / nav;
      if (rd->region == nullptr) a0 = listing_rate<SMAX>(A, as_const(rd->lcoef), Nc, nav, inv_nav);
      else a0 = listing_rate<SMAX>(A, rd->lcoef + reg * kLStride, Nc, nav, inv_nav);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (has_next) {
      nc = tile_ctx(A, tile + tr.stride, k);
      load_counts<SMAX>(nc, S, nc.base + lane, nxt);
    }
    __builtin_amdgcn_sched_barrier(0);

    // listing: the window's first SSA event falls inside [0, tau_k] only if
    // t_reac = -ln(u) / a0 <= tau_k, and -ln(u) >= 1 - u; so a tet whose first
    // uniform u of the window has 1 - u above a0 tau_k (with a relative
    // margin of 1e-6, far above the rounding of a0, of ln and of the
    // division) has no event, and every other tet with a0 > 0 is listed.  A
    // listed tet without an event is harmless: its SSA ends at the first draw
    // and its items are those of an unlisted tet.
    bool event = false;
    if (run_active && active && a0 > 0.0) {
      Draw53 st(rd->key0, rd->key1, 0u, (uint32_t)i, cc.window);
      const double u = st.oc();
      event = !(1.0 - u > (cc.tau_k * a0) * 1.000001);
    }
    // binning by expected events: a listed tet with a0 tau_k above the
    // threshold goes to the heavy bin, the others to the light bin, so that
    // no event chunk runs light tets in lock-step with a long chain
    const bool heavy = event && cc.tau_k * a0 > A.heavy_events;
    const unsigned long long bh = __ballot(heavy), bl = __ballot(event && !heavy);
    const int nh = (int)__popcll(bh), nl = (int)__popcll(bl);
    if (lane == 0) {
      A.wl_mask[tile] = bh | bl;
      if (nh + nl) {
        A.wl_tile_count[tile] = nh | (nl << 8);
        // per bin, one atomic on the tile's sub-queue counts the queued tile
        // (low word) and its listed tets (high word); the old low word is
        // the tile's slot in that sub-queue
        const int qj = tile & (kQueues - 1);
#pragma unroll
        for (int bin = 0; bin < kBins; ++bin) {
          const int nb = bin == 0 ? nh : nl;
          if (nb) {
            const unsigned long long old = atomicAdd(
                A.evq_count + (((size_t)(k & 1) * kBins + bin) * kQueues + qj) * kQueueStride,
                ((unsigned long long)nb << 32) | 1ull);
            A.evq[((size_t)bin * kQueues + qj) * A.evq_cap + (size_t)(old & 0xffffffffull)] = tile;
          }
        }
      }
    }
    if (event) {  // the tile's listed tets take its own worklist slots, heavy first
      const unsigned long long below = (1ull << lane) - 1ull;
      const int pos = heavy ? (int)__popcll(bh & below) : nh + (int)__popcll(bl & below);
      A.wl_tet[(size_t)tile * kWave + (size_t)pos] = i;
    }
    cc = nc;
    cur = nxt;
  }
}

// LDS of the main kernel: a block is either a diffusion block or an event
// block, so the two layouts share the space.
template <int SMAX>
struct DiffusionLds {
  int acc[SMAX][kWave];         // counts, then next counts of own tets
  double tauD[SMAX];            // tau_k D_s of the current run
  uint32_t item[SMAX * kWave];  // packed items: count << 10 | lane << 4 | species
  int4 nbr[kWave];
  double2 geo[2][kWave];        // (G, cum0), (cum1, cum2)
  ItemLds x;                    // the current round of items
};

// Lanes of an event chunk: the propensity table takes RMAX doubles per lane,
// kept to 6 KiB.
template <int RMAX>
constexpr int chunk_width() {
  return RMAX * 8 * kWave <= 6144 ? kWave : (RMAX * 8 * 32 <= 6144 ? 32 : 16);
}

template <int SMAX, int RMAX>
struct EventLds {
  static constexpr int CW = chunk_width<RMAX>();
  // net changes and dependencies (copied whole from the device model) and
  // the rate constants of the tile's run by region
  uint32_t delta_w[32 * 16 / 4];        // int8 [32][16]
  uint32_t deps_w[32 * 2];              // uint64 [32]: reactions whose propensity a reaction changes
  uint32_t kc_w[kMaxRegions * 32 * 2];  // double [8][32]
  union {
    double a[RMAX][CW];                 // propensities of the chunk's tets, one column per lane
    ItemLds x;                          // then the rounds of their diffusion items
  };
  double td[SMAX];                      // tau_k D_s of the tile's run
  double nbar[kWave];                   // mean occupancy of the round's items
  int npost[kWave];                     // post-reaction count of the round's items
  uint16_t item[kWave];                 // the round's items: lane << 4 | species
  int4 nbr[kWave];
  double2 geo[2][kWave];                // (G, cum0), (cum1, cum2)
  int tet[kWave];
};

template <int SMAX, int RMAX>
union MainLds {
  DiffusionLds<SMAX> d;
  EventLds<SMAX, RMAX> e;
};

// Diffusion blocks (b of G): the tets not listed, tile by tile, persistent,
// the next tile's loads in flight while the current one is worked on.  With
// `claim_only` (an event block done with its groups, b its XCD) the block has
// no static tile and takes only claimed ones.
template <int SMAX, int RMAX>
__device__ __forceinline__ void diffusion_part(const StepArgs& A, int k, int b, int G, DiffusionLds<SMAX>& L,
                                               bool claim_only) {
  const int lane = threadIdx.x;
  const int S = A.S;
  const int n_tiles = *as_const(A.n_tiles);
  const TileRange tr = tile_range(b, G, n_tiles);
  // Run-time claiming (a launch-shape setting, for workloads whose tiles
  // differ in cost): the block's first tile is its static one, lo + j; the
  // tiles from lo + Gx on are cut into kClaimSubs sub-ranges (fewer if the
  // XCD has fewer blocks), each handed out in order by a counter of its own
  // to the blocks with j mod kClaimSubs equal to its index, each claim
  // issued one tile ahead so that its latency hides behind a tile's work.
  // Eight counters per XCD keep the claims at a window's start from queueing
  // on one address.  A block stops at its first claim past its sub-range,
  // so every block ends, and the slowest finishes within about one tile of
  // the others.
  const bool claim = A.tile_claim != 0 && G >= 8 && n_tiles >= 8;
  const int dyn0 = tr.first - (b >> 3) + tr.stride;  // lo + Gx
  const int nsub = tr.stride < kClaimSubs ? (tr.stride > 0 ? tr.stride : 1) : kClaimSubs;
  const int sub = (claim_only ? (int)(blockIdx.x >> 3) : (b >> 3)) % nsub;
  int32_t* const ctr =
      A.tile_ctr + ((size_t)(k & 1) * 8 * kClaimSubs + (size_t)(b & 7) * kClaimSubs + (size_t)sub) * kCtrStride;
  const int n_claim = tr.end > dyn0 ? tr.end - dyn0 : 0;
  const int sub_lo = dyn0 + (int)(((long long)n_claim * sub) / nsub);
  const int sub_hi = dyn0 + (int)(((long long)n_claim * (sub + 1)) / nsub);
  int first = tr.first;
  if (claim_only) {
    int r0 = 0;
    if (lane == 0) r0 = atomicAdd(ctr, 1);
    const int c0 = __builtin_amdgcn_readfirstlane(r0);
    first = sub_lo + c0 < sub_hi ? sub_lo + c0 : tr.end;
  }
  int raw = 0;  // lane 0: the counter value of the claim in flight
  if (claim && lane == 0) raw = atomicAdd(ctr, 1);
  int cache_run = -1;
  unsigned long long n_moved = 0, n_faces = 0;
  uint32_t key0 = 0, key1 = 0, dmask = 0;  // per-run constants (uniform)

  TileCtx cc, nc;
  TetData<SMAX> cur, nxt;
  unsigned long long cmask = 0, nmask = 0;  // listed tets of the tile
  if (first < tr.end) {
    cc = tile_ctx(A, first, k);
    load_tet<SMAX>(cc, S, cc.base + lane, cur);
    cmask = as_const(A.wl_mask)[first];
  }
  nc = cc;

  for (int tile = first, next = 0; tile < tr.end; tile = next) {
    if (claim) {
      const int c = __builtin_amdgcn_readfirstlane(raw);
      next = sub_lo + c < sub_hi ? sub_lo + c : tr.end;
    } else {
      next = tile + tr.stride;
    }
    const bool has_next = next < tr.end;
    const bool run_active = cc.active;  // else the tile only forwards the prefetch
    const cptr<RunDesc> rd = cc.rd;
    const int T = cc.T;
    const int i = cc.base + lane;
    const bool active = i < T;
    if (run_active && cc.run != cache_run) {
      if (cache_run >= 0) {  // tallies are kept per run
        const unsigned long long mv = wave_sum(n_moved), fm = wave_sum(n_faces);
        if (lane == 0 && mv) atomicAdd(tally_slot(A, cache_run) + 1, mv);
        if (lane == 0 && fm) atomicAdd(tally_slot(A, cache_run) + 2, fm);
        n_moved = 0;
        n_faces = 0;
      }
      key0 = rd->key0;
      key1 = rd->key1;
      const double d = lane < S ? rd->D[lane < SMAX ? lane : 0] : 0.0;
      if (lane < SMAX) L.tauD[lane] = lane < S ? cc.tau_k * d : 0.0;
      dmask = (uint32_t)__ballot(lane < S && d > 0.0);
      cache_run = cc.run;
    }
    // the tile's data moves from registers to LDS before the next tile's
    // loads are issued, so that waiting for this tile's loads never waits for
    // the next tile's (an inactive tile's data is all zero)
#pragma unroll
    for (int s = 0; s < SMAX; ++s) L.acc[s][lane] = cur.N[s];
    L.nbr[lane] = cur.nb;
    L.geo[0][lane] = cur.ga;
    L.geo[1][lane] = cur.gb;
    const bool event = (cmask >> lane) & 1ull;
    wave_sync();
    __builtin_amdgcn_sched_barrier(0);
    if (has_next) {
      nc = tile_ctx(A, next, k);
      load_tet<SMAX>(nc, S, nc.base + lane, nxt);
      nmask = as_const(A.wl_mask)[next];
      if (claim && lane == 0) raw = atomicAdd(ctr, 1);  // the tile after next
    }
    __builtin_amdgcn_sched_barrier(0);

    if (run_active) {
      int n_own[SMAX];
#pragma unroll
      for (int s = 0; s < SMAX; ++s) n_own[s] = L.acc[s][lane];
      const double Gl = L.geo[0][lane].x;

      // a listed tet is left to the event blocks; for the others Nbar = N
      uint32_t mask = 0;
      if (active && !event && Gl > 0.0) {
#pragma unroll
        for (int s = 0; s < SMAX; ++s)
          if (((dmask >> s) & 1u) && n_own[s] > 0) mask |= 1u << s;
      }
      // items in three classes, each species-major: more than 16 molecules
      // (binomial face counts), so that few rounds wait on a binomial; then
      // 5 to 16 (two to four Philox calls on the item's lane); then 1 to 4
      // (one call).  A round's lanes step through as many calls as its
      // longest item has, so grouping items by their number of calls keeps
      // the short ones from idling behind the long ones.
      int total = 0, errbits = 0;
      const unsigned long long below = (1ull << lane) - 1ull;
      uint32_t large = 0, multi = 0;  // species of this tet in the first two classes
#pragma unroll
      for (int s = 0; s < SMAX; ++s)
        if ((mask >> s) & 1u) {
          if (n_own[s] > kSmallM) large |= 1u << s;
          else if (n_own[s] > 4) multi |= 1u << s;
        }
      const bool any_large = __ballot(large != 0u) != 0ull;  // uniform
      const bool any_multi = __ballot(multi != 0u) != 0ull;
#pragma unroll 1
      for (int cls = 0; cls < 3; ++cls) {
        if ((cls == 0 && !any_large) || (cls == 1 && !any_multi)) continue;
        const uint32_t cm = cls == 0 ? large : (cls == 1 ? multi : mask & ~(large | multi));
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
          const bool has = (cm >> s) & 1u;
          const unsigned long long bs = __ballot(has);
          if (has) {  // a count of 2^22 or more does not fit the packed field (0 marks it)
            const int n = n_own[s];
            L.item[total + __popcll(bs & below)] =
                ((uint32_t)(n < (1 << 22) ? n : 0) << 10) | (uint32_t)(lane << 4) | (uint32_t)s;
          }
          total += (int)__popcll(bs);
        }
      }
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        const int n = n_own[s];
        if (n > kCountCap) errbits |= kErrOverflow;
        // the accumulator starts with what cannot leave
        L.acc[s][lane] = ((mask >> s) & 1u) || event || !active ? 0 : n;
      }
      wave_sync();

      const int base = cc.base;
      const ItemView view{L.nbr, L.geo[0], L.geo[1], L.tauD, nullptr, base};
      for (int r0 = 0; r0 < total; r0 += kWave) {
        ItemIn in;
        in.valid = lane < total - r0;
        int Ln = 0, sp = 0, m = 0;
        int4 tnb = make_int4(-1, -1, -1, -1);
        if (in.valid) {
          const uint32_t itw = L.item[r0 + lane];
          Ln = (int)((itw >> 4) & 63);
          sp = (int)(itw & 15);
          m = (int)(itw >> 10);
          tnb = L.nbr[Ln];
        }
        // A count of 2^22 or more does not fit the packed field (0 marks
        // it): its lane reads it from the count buffer, in a rare uniform
        // branch that hands the value on through LDS.  Any later use of a
        // register still awaiting a global load would otherwise make the
        // whole round wait on the vector-memory counter, i.e. for the next
        // tile's loads and this tile's atomics as well.
        if (__ballot(in.valid && m == 0) != 0ull) {
          if (in.valid && m == 0) L.item[r0 + lane] = (uint32_t)cc.cin[(size_t)sp * T + base + Ln];
          wave_sync();
          if (in.valid && m == 0) m = (int)L.item[r0 + lane];
        }
        in.sp = sp;
        in.ln = Ln;
        in.nbar = (double)m;
        in.npost = m;
        const bool big_round = __ballot(in.valid && m > kSmallM) != 0ull;  // uniform
        const ItemMoves mv = big_round ? item_round(key0, key1, cc.window, in, view, L.x)
                                       : item_round_small(key0, key1, cc.window, in, view);
        if (in.valid) {
          // own remainder and moves to the tile's own tets go to LDS, the
          // rest to the next count buffer
          int32_t* __restrict__ out_s = cc.cout + (size_t)sp * T;
          if (m != mv.n) atomicAdd(&L.acc[sp][Ln], m - mv.n);
#define RDX_DEPOSIT(t, v)                                               \
          if (v) {                                                      \
            const unsigned off = (unsigned)((t) - base);                 \
            if (off < (unsigned)kWave) atomicAdd(&L.acc[sp][off], (v));  \
            else atomicAdd(out_s + (t), (v));                            \
            ++n_faces;                                                   \
          }
          RDX_DEPOSIT(tnb.x, mv.o0)
          RDX_DEPOSIT(tnb.y, mv.o1)
          RDX_DEPOSIT(tnb.z, mv.o2)
          RDX_DEPOSIT(tnb.w, mv.o3)
#undef RDX_DEPOSIT
          n_moved += (unsigned long long)mv.n;
        }
      }
      wave_sync();
      // coalesced flush of the tile's own tets (other tiles add into them too)
      int v[SMAX];
#pragma unroll
      for (int s = 0; s < SMAX; ++s) v[s] = L.acc[s][lane];
      if (active) {
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
          if (s < S) {
            if (v[s] != 0) atomicAdd(cc.cout + (size_t)s * T + i, v[s]);
            // the target of the window after next (a listed tet's counts are
            // read and cleared by its event block)
            if (!event) cc.cin[(size_t)s * T + i] = 0;
          }
        }
      }
      if (errbits) atomicOr(rd->err, errbits);
    }
    wave_sync();  // LDS is rebuilt for the next tile
    cc = nc;
    cur = nxt;
    cmask = nmask;
  }

  const unsigned long long mv = wave_sum(n_moved), fm = wave_sum(n_faces);
  if (lane == 0 && cache_run >= 0 && mv) atomicAdd(tally_slot(A, cache_run) + 1, mv);
  if (lane == 0 && cache_run >= 0 && fm) atomicAdd(tally_slot(A, cache_run) + 2, fm);
}

// One event chunk: up to CW listed tets of one run (worklist slot `slot` on
// the lanes below `n_work`; `tile0` gives the run), one per lane: the SSA
// window, the occupancies, then the diffusion of their items.  `tables`,
// `cache_run` and `dmask` carry what is already in LDS from the previous
// chunk of the block.
template <int SMAX, int RMAX>
__device__ __forceinline__ void event_chunk(const StepArgs& A, int k, int tile0, int n_work, size_t slot,
                                            EventLds<SMAX, RMAX>& L, bool& tables, int& cache_run,
                                            uint32_t& dmask) {
  constexpr int CW = EventLds<SMAX, RMAX>::CW;
  const int lane = threadIdx.x;
  const int S = A.S, R = A.R;
  {
    const TileCtx cc = tile_ctx(A, tile0, k);
    const cptr<RunDesc> rd = cc.rd;
    const int T = cc.T;
    const double tau = cc.tau_k;

    // the worklist entry names the tet; its counts, N_A V, region,
    // neighbours and couplings are read in place (the diffusion blocks leave
    // a listed tet's counts alone), then its counts are cleared for the
    // window after next
    const bool active = lane < n_work;
    int N[SMAX];
    int i = 0;
    double nav = 1.0;
    int4 nb = make_int4(-1, -1, -1, -1);
    double2 ga = make_double2(0.0, 0.0), gb = make_double2(0.0, 0.0);
    if (active) i = A.wl_tet[slot];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) N[s] = (active && s < S) ? cc.cin[(size_t)s * T + i] : 0;
    if (active) {
      nav = as_const(rd->nav)[i];
      nb = ld_int4(reinterpret_cast<const int4*>(rd->nbr), (size_t)i);
      ga = ld_double2(reinterpret_cast<const double2*>(rd->geo), 2 * (size_t)i);
      gb = ld_double2(reinterpret_cast<const double2*>(rd->geo), 2 * (size_t)i + 1);
    }
    // tables and per-run constants: every load issued before any is used
    const bool need_tables = !tables, need_run = cc.run != cache_run;
    const bool regions = rd->region != nullptr;
    const cptr<uint32_t> mw = as_const(reinterpret_cast<const uint32_t*>(A.model));
    const cptr<uint32_t> kw = as_const(reinterpret_cast<const uint32_t*>(rd->kcst));
    uint32_t d0 = 0, d1 = 0, dp = 0, kv[kMaxRegions];
    double dv = 0.0;
    int reg = 0;
    if (need_tables) {
      d0 = mw[offsetof(DevModel, delta) / 4 + lane];
      d1 = mw[offsetof(DevModel, delta) / 4 + kWave + lane];
      dp = mw[offsetof(DevModel, deps) / 4 + lane];
    }
    if (need_run) {
#pragma unroll
      for (int q = 0; q < kMaxRegions; ++q) kv[q] = (q == 0 || regions) ? kw[q * kWave + lane] : 0u;
      if (lane < SMAX && lane < S) dv = rd->D[lane];
    }
    if (active && regions) reg = as_const(rd->region)[i];
    if (need_tables) {
      L.delta_w[lane] = d0;
      L.delta_w[kWave + lane] = d1;
      L.deps_w[lane] = dp;
      tables = true;
    }
    if (need_run) {
#pragma unroll
      for (int q = 0; q < kMaxRegions; ++q)
        if (q == 0 || regions) L.kc_w[q * kWave + lane] = kv[q];
      if (lane < SMAX) L.td[lane] = lane < S ? tau * dv : 0.0;
      dmask = (uint32_t)__ballot(lane < SMAX && lane < S && tau * dv > 0.0);
      cache_run = cc.run;
    }
    wave_sync();
    const double(*s_kc)[32] = reinterpret_cast<const double(*)[32]>(L.kc_w);

    // the tet's neighbours and couplings wait in LDS while the SSA runs
    L.tet[lane] = i;
    L.nbr[lane] = nb;
    L.geo[0][lane] = ga;
    L.geo[1][lane] = gb;

    unsigned long long n_ev = 0, n_mv = 0, n_fm = 0;
    int errbits = 0;
    uint32_t mask = 0;
    double nbv[SMAX];  // mean occupancies of the tet's items
    int npv[SMAX];     // post-reaction counts
    if (active) {
      // counts as one vector value (uniform species indices select
      // registers); rate constants of the tet's region from LDS
      int __attribute__((ext_vector_type(SMAX))) Nv;
#pragma unroll
      for (int s = 0; s < SMAX; ++s) Nv[s] = N[s];
      const double inv_nav = 1.0 / nav;
      const double* kreg = s_kc[reg];
      double* col = &L.a[0][lane];  // a_r at col[r * CW]
#pragma unroll 1
      for (int r = 0; r < R; ++r) col[r * CW] = propensity<SMAX>(A.info[r], kreg[r], Nv, nav, inv_nav);
      // the counts are in registers now; clear them for the window after next
#pragma unroll
      for (int s = 0; s < SMAX; ++s)
        if (s < S) cc.cin[(size_t)s * T + i] = 0;

      // ---- reaction SSA operator over [0, tau_k] ----
      double O[SMAX], tS[SMAX];
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        O[s] = 0.0;
        tS[s] = 0.0;
      }
      uint32_t touched = 0;
      Draw53 st(rd->key0, rd->key1, 0u, (uint32_t)i, cc.window);
      double dt = 0.0;
      unsigned int ev_tet = 0;
      for (;;) {
        double a0 = 0.0;
#pragma unroll 4
        for (int r = 0; r < R; ++r) a0 = a0 + col[r * CW];
        if (!(a0 > 0.0)) break;
        const double u = st.oc();
        const double t_reac = -ln_basic(u) / a0;
        if (dt + t_reac > tau) break;
        const int rn = cr_select_col(col, CW, R, a0, st);
        dt = dt + t_reac;
        // few lanes of a wave are in the loop at a time, so branches that
        // skip unchanged species and unaffected reactions are cheap
        const uint4 drow = reinterpret_cast<const uint4*>(L.delta_w)[rn];
        const unsigned long long dep = reinterpret_cast<const unsigned long long*>(L.deps_w)[rn];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
          if (s < S) {
            const uint32_t wd = (s >> 2) == 0 ? drow.x : ((s >> 2) == 1 ? drow.y : ((s >> 2) == 2 ? drow.z : drow.w));
            const int d = (int)(int8_t)((wd >> (8 * (s & 3))) & 0xffu);
            if (d != 0) {
              const int n = Nv[s];
              O[s] = O[s] + (double)n * (dt - tS[s]);
              tS[s] = dt;
              touched |= 1u << s;
              Nv[s] = n + d;
              if (n + d > kCountCap) errbits |= kErrOverflow;
            }
          }
        }
        // the propensities that read a changed species
#pragma unroll 1
        for (int r = 0; r < R; ++r)
          if ((dep >> r) & 1ull) col[r * CW] = propensity<SMAX>(A.info[r], kreg[r], Nv, nav, inv_nav);
        ++ev_tet;
        if (errbits) break;
        if (ev_tet >= (unsigned int)kEventCap) {
          errbits |= kErrEvents;
          break;
        }
      }
      n_ev = ev_tet;

      // ---- mean occupancies; items for the diffusion operator ----
      const bool coupled = L.geo[0][lane].x > 0.0;
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        nbv[s] = 0.0;
        npv[s] = 0;
        if (s >= S) continue;
        const int n = Nv[s];
        const double occ = (O[s] + (double)n * (tau - tS[s])) / tau;
        const double nbar = ((touched >> s) & 1u) ? occ : (double)n;
        if (((dmask >> s) & 1u) && coupled && nbar > 0.0) {
          mask |= 1u << s;
          nbv[s] = nbar;
          npv[s] = n;
        } else if (n != 0) {
          atomicAdd(cc.cout + (size_t)s * T + i, n);  // nothing can leave
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        nbv[s] = 0.0;
        npv[s] = 0;
      }
    }
    const int cnt = __popc(mask);
    const int incl = wave_inclusive_scan(cnt);
    const int total = __shfl(incl, kWave - 1);
    const int first = incl - cnt;
    const ItemView view{L.nbr, L.geo[0], L.geo[1], L.td, L.tet, 0};
    // items in rounds of 64: each lane parks the items of the round that
    // are its own, then every lane samples one
    for (int r0 = 0; r0 < total; r0 += kWave) {
      int pos = first;
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        if ((mask >> s) & 1u) {
          const unsigned slot = (unsigned)(pos - r0);
          if (slot < (unsigned)kWave) {
            L.item[slot] = (uint16_t)((lane << 4) | s);
            L.nbar[slot] = nbv[s];
            L.npost[slot] = npv[s];
          }
          ++pos;
        }
      }
      wave_sync();
      ItemIn in;
      in.valid = lane < total - r0;
      int sp = 0, ti = 0, npost = 0, Ln = 0;
      double nbar = 0.0;
      int4 tnb = make_int4(-1, -1, -1, -1);
      if (in.valid) {
        const int it = L.item[lane];
        Ln = it >> 4;
        sp = it & 15;
        ti = L.tet[Ln];
        npost = L.npost[lane];
        nbar = L.nbar[lane];
        tnb = L.nbr[Ln];
      }
      in.sp = sp;
      in.ln = Ln;
      in.nbar = nbar;
      in.npost = npost;
      const ItemMoves mv = item_round(rd->key0, rd->key1, cc.window, in, view, L.x);
      if (in.valid) {
        int32_t* out_s = cc.cout + (size_t)sp * T;
        if (npost != mv.n) atomicAdd(out_s + ti, npost - mv.n);
        if (mv.o0) atomicAdd(out_s + tnb.x, mv.o0);
        if (mv.o1) atomicAdd(out_s + tnb.y, mv.o1);
        if (mv.o2) atomicAdd(out_s + tnb.z, mv.o2);
        if (mv.o3) atomicAdd(out_s + tnb.w, mv.o3);
        n_mv += (unsigned long long)mv.n;
        n_fm += (unsigned long long)((mv.o0 != 0) + (mv.o1 != 0) + (mv.o2 != 0) + (mv.o3 != 0));
      }
      wave_sync();  // the round's LDS entries are rebuilt for the next
    }
    const unsigned long long ev_sum = wave_sum(n_ev), mv_sum = wave_sum(n_mv), fm_sum = wave_sum(n_fm);
    if (lane == 0) {
      if (ev_sum) atomicAdd(tally_slot(A, cc.run), ev_sum);
      if (mv_sum) atomicAdd(tally_slot(A, cc.run) + 1, mv_sum);
      if (fm_sum) atomicAdd(tally_slot(A, cc.run) + 2, fm_sum);
    }
    if (errbits) atomicOr(rd->err, errbits);
    wave_sync();  // LDS is rebuilt for the next chunk
  }
}

// The queue of one bin, as the main kernel reassembles it: lane j holds its
// sub-queue j's inclusive prefix of queued tiles.
struct BinQueue {
  int n_queued;  // queued tiles of the bin
  int K;         // queued tiles per group
  int n_groups;
  int q_incl;    // per lane
};

// Event blocks (b of E): groups of K consecutive queue entries of a bin,
// group b, b + E, ... over the heavy bin's groups and then the light bin's;
// the listed tets of a group's tiles are packed CW to a chunk (a chunk holds
// one run and one bin), so that tiles with one or two listed tets share one
// pass of the SSA, and tets expected to have several events share chunks
// with each other only.
template <int SMAX, int RMAX>
__device__ __forceinline__ void event_part(const StepArgs& A, int k, int b, int E, const BinQueue* Q,
                                           EventLds<SMAX, RMAX>& L) {
  constexpr int CW = EventLds<SMAX, RMAX>::CW;
  const int lane = threadIdx.x;
  bool tables = false;
  int cache_run = -1;
  uint32_t dmask = 0;  // species with tau_k D_s > 0 in the cached run
  const cptr<int> tile_run = as_const(reinterpret_cast<const int*>(A.tile_map));
  const int n_groups = Q[0].n_groups + Q[1].n_groups;

  for (int gg = b; gg < n_groups; gg += E) {
    const int bin = gg < Q[0].n_groups ? 0 : 1;
    const BinQueue& B = Q[bin];
    const int g = gg - (bin ? Q[0].n_groups : 0);
    const int* evq = A.evq + (size_t)bin * kQueues * A.evq_cap;
    // the group's tiles, listed counts and runs: lane j loads entry j (one
    // round of loads for the whole group)
    const int q0 = g * B.K;
    const int nq = B.n_queued - q0 < B.K ? B.n_queued - q0 : B.K;
    // entry q is slot q - (tiles of the sub-queues before j) of sub-queue j,
    // j the first sub-queue whose inclusive prefix exceeds q
    int g_tile = 0, g_n = 0, g_first = 0, g_run = -1;
    for (int l = 0; l < nq; ++l) {
      const int q = q0 + l;
      const int j = (int)__popcll(__ballot(B.q_incl <= q));
      const int before = j > 0 ? __builtin_amdgcn_readlane(B.q_incl, j - 1) : 0;
      if (lane == l) g_tile = evq[(size_t)j * A.evq_cap + (size_t)(q - before)];
    }
    if (lane < nq) {
      // the bin's listed tets of the tile and their first worklist slot
      // (heavy tets first)
      const int c = A.wl_tile_count[g_tile];
      g_n = bin == 0 ? (c & 0xff) : (c >> 8);
      g_first = bin == 0 ? 0 : (c & 0xff);
      g_run = A.single_run ? 0 : tile_run[2 * g_tile];
    }
    // walk the group's tiles and their listed tets in order; the chunk is
    // run from one place in the code
    int q = -1, tile = 0, n = 0, first = 0, run = -1, j0 = 0;
    int fill = 0, tile0 = 0, run0 = -1;
    size_t slot = 0;
    for (;;) {
      if (j0 >= n) {  // the next tile of the group with listed tets
        j0 = 0;
        n = 0;
        for (++q; q < nq; ++q) {
          n = __builtin_amdgcn_readlane(g_n, q);
          if (n > 0) break;
        }
        if (q < nq) {
          tile = __builtin_amdgcn_readlane(g_tile, q);
          first = __builtin_amdgcn_readlane(g_first, q);
          run = __builtin_amdgcn_readlane(g_run, q);
        }
      }
      const bool done = q >= nq;
      if (fill > 0 && (done || run != run0 || fill == CW)) {
        event_chunk<SMAX, RMAX>(A, k, tile0, fill, slot, L, tables, cache_run, dmask);
        fill = 0;
      }
      if (done) break;
      if (fill == 0) {
        tile0 = tile;
        run0 = run;
      }
      const int take = n - j0 < CW - fill ? n - j0 : CW - fill;
      if (lane >= fill && lane < fill + take) slot = (size_t)tile * kWave + (size_t)(first + j0 + lane - fill);
      fill += take;
      j0 += take;
    }
  }
}

// Three waves per SIMD: the diffusion blocks need the occupancy to hide
// their load latency, so the compiler keeps the event part (the larger
// register footprint) within that budget, spilling if it must.
template <int SMAX, int RMAX>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3)))
window_main_kernel(const StepArgs A) {
  __shared__ MainLds<SMAX, RMAX> lds;
  const int k = step_index(A);
  // the sub-queues of each bin: lane j holds sub-queue j's tiles and their
  // inclusive prefix sum over the sub-queues
  const int lane = threadIdx.x;
  const int G = gridDim.x;
  const int K_max = A.ev_group_max >= 1 ? A.ev_group_max : 1;
  BinQueue Q[kBins];
  int n_groups = 0;
#pragma unroll
  for (int bin = 0; bin < kBins; ++bin) {
    const size_t at = (((size_t)(k & 1) * kBins + bin) * kQueues + lane) * kQueueStride;
    const unsigned long long qc = A.evq_count[at];
    Q[bin].q_incl = wave_scan_add((int)(qc & 0xffffffffull));
    Q[bin].n_queued = __builtin_amdgcn_readlane(Q[bin].q_incl, kWave - 1);
    const int n_listed = __builtin_amdgcn_readlane(wave_scan_add((int)(qc >> 32)), kWave - 1);
    // one group of K queued tiles per event block, K chosen so that a group
    // lists about 64 tets, at most ev_group_max tiles (a launch-shape
    // setting: longer groups can make the event blocks the last to finish)
    int K = n_listed > 0 ? (int)((64ll * Q[bin].n_queued) / n_listed) : 1;
    K = K < 1 ? 1 : (K > K_max ? K_max : K);
    Q[bin].K = K;
    Q[bin].n_groups = (Q[bin].n_queued + K - 1) / K;
    n_groups += Q[bin].n_groups;
    if (blockIdx.x == 0)  // the next window's queue starts empty
      A.evq_count[(((size_t)((k + 1) & 1) * kBins + bin) * kQueues + lane) * kQueueStride] = 0;
  }
  if (blockIdx.x == 0 && lane < 8 * kClaimSubs)  // and so do its tile claim counters
    A.tile_ctr[((size_t)((k + 1) & 1) * 8 * kClaimSubs + (size_t)lane) * kCtrStride] = 0;
  // event blocks: one per group, a multiple of the 8 XCDs (so that the
  // diffusion blocks keep their XCD mapping), at most half the grid
  int E = 0;
  if (n_groups > 0) {
    const int cap = G / 2 >= 8 ? (G / 2) & ~7 : (G / 2 > 0 ? G / 2 : 1);
    E = (n_groups + 7) & ~7;
    if (E > cap) E = cap;
  }
  // with tiles claimed at run time an event block done with its groups
  // takes diffusion tiles of its XCD (E is a multiple of 8, so block b is on
  // the XCD of diffusion block b - E)
  const int GD = G - E;
  const bool join = A.tile_claim != 0 && GD >= 8 && *as_const(A.n_tiles) >= 8;
  const bool ev = (int)blockIdx.x < E;
  if (ev) {
    event_part<SMAX, RMAX>(A, k, blockIdx.x, E, Q, lds.e);
    if (!join) return;
    wave_sync();  // the event layout's last reads are done before the diffusion layout is written
  }
  diffusion_part<SMAX, RMAX>(A, k, ev ? (int)(blockIdx.x & 7u) : (int)blockIdx.x - E, GD, lds.d, ev);
}

__global__ void advance_base_kernel(int32_t* base, int32_t add) { *base += add; }

// Batched reset: one block per chunk.
__global__ void __launch_bounds__(kBlock) reset_chunks_kernel(const ResetChunk* chunks) {
  const ResetChunk c = chunks[blockIdx.x];
  for (int64_t j = c.begin + threadIdx.x; j < c.end; j += kBlock) {
    c.dst[j] = c.src[j];
    c.other[j] = 0;
  }
  if (c.begin == 0) {
    if (threadIdx.x < kTallyWords * kTallySlots) c.tally[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) *c.err = 0;
  }
}
__global__ void set_base_kernel(int32_t* base, int32_t value) { *base = value; }

// ----------------------------------------------------------- self-tests ----
// One vector per wave (block j of 64 lanes), so that its key is wave-uniform
// as in the window kernels; lane 0 writes.
__global__ void __launch_bounds__(kWave) selftest_philox_kernel(const uint32_t* in, uint32_t* out) {
  const int64_t j = blockIdx.x;
  const cptr<uint32_t> v = as_const(in) + 6 * j;
  uint32_t x0 = v[0], x1 = v[1], x2 = v[2], x3 = v[3];
  philox4x32_10(x0, x1, x2, x3, v[4], v[5]);
  if (threadIdx.x == 0) {
    out[4 * j] = x0;
    out[4 * j + 1] = x1;
    out[4 * j + 2] = x2;
    out[4 * j + 3] = x3;
  }
}

__global__ void selftest_ln_kernel(const double* x, double* y, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) y[j] = ln_basic(x[j]);
}

__global__ void selftest_binom_kernel(uint32_t key0, uint32_t key1, uint32_t stream_id,
                                      uint32_t window, long long m, double p, int64_t n,
                                      long long* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  Draw32 st(key0, key1, stream_id, (uint32_t)j, window);
  out[j] = binom(m, p, st);
}

__global__ void copy_kernel(const int4* __restrict__ src, int4* __restrict__ dst, int64_t n16) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n16;
       j += (int64_t)gridDim.x * blockDim.x)
    dst[j] = src[j];
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// Blocks of a window kernel the device holds at once (occupancy x CUs).
template <typename K>
int resident_blocks_of(K kernel) {
  int dev = 0, n_cu = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), kWave, 0);
  return n_cu > 0 && per_cu > 0 ? n_cu * per_cu : 2048;
}

template <int SMAX, int RMAX>
int main_resident() {
  static const int r = resident_blocks_of(&window_main_kernel<SMAX, RMAX>);
  return r;
}

template <int SMAX, int RMAX>
int detect_resident() {
  static const int r = resident_blocks_of(&window_detect_kernel<SMAX, RMAX>);
  return r;
}

template <int SMAX, int RMAX>
hipError_t launch_pair(const StepArgs& a, hipStream_t stream, hipEvent_t* marks) {
  if (marks) (void)hipEventRecord(marks[0], stream);
  hipLaunchKernelGGL((window_detect_kernel<SMAX, RMAX>), dim3((unsigned)a.detect_grid), dim3(kWave), 0,
                     stream, a);
  if (marks) (void)hipEventRecord(marks[1], stream);
  hipLaunchKernelGGL((window_main_kernel<SMAX, RMAX>), dim3((unsigned)a.main_grid), dim3(kWave), 0, stream, a);
  if (marks) (void)hipEventRecord(marks[2], stream);
  return hipGetLastError();
}

void grid_resident(int S, int R, int* detect, int* main) {
  if (S <= 4 && R <= 4) {
    *detect = detect_resident<4, 4>();
    *main = main_resident<4, 4>();
  } else if (S <= 8 && R <= 8) {
    *detect = detect_resident<8, 8>();
    *main = main_resident<8, 8>();
  } else if (S <= 12 && R <= 12) {
    *detect = detect_resident<12, 12>();
    *main = main_resident<12, 12>();
  } else if (S <= 16 && R <= 24) {
    *detect = detect_resident<16, 24>();
    *main = main_resident<16, 24>();
  } else {
    *detect = detect_resident<16, 32>();
    *main = main_resident<16, 32>();
  }
}

hipError_t launch_window(const StepArgs& a, hipStream_t stream, hipEvent_t* marks) {
  if (a.S <= 4 && a.R <= 4) return launch_pair<4, 4>(a, stream, marks);
  if (a.S <= 8 && a.R <= 8) return launch_pair<8, 8>(a, stream, marks);
  if (a.S <= 12 && a.R <= 12) return launch_pair<12, 12>(a, stream, marks);
  if (a.S <= 16 && a.R <= 24) return launch_pair<16, 24>(a, stream, marks);
  return launch_pair<16, 32>(a, stream, marks);
}

hipError_t launch_advance_base(int32_t* base, int32_t add, hipStream_t stream) {
  hipLaunchKernelGGL(advance_base_kernel, dim3(1), dim3(1), 0, stream, base, add);
  return hipGetLastError();
}

hipError_t launch_set_base(int32_t* base, int32_t value, hipStream_t stream) {
  hipLaunchKernelGGL(set_base_kernel, dim3(1), dim3(1), 0, stream, base, value);
  return hipGetLastError();
}

hipError_t launch_reset_chunks(const ResetChunk* chunks, int64_t n_chunks, hipStream_t stream) {
  if (n_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(reset_chunks_kernel, dim3((unsigned)n_chunks), dim3(kBlock), 0, stream, chunks);
  return hipGetLastError();
}

hipError_t launch_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(selftest_philox_kernel, dim3((unsigned)n), dim3(kWave), 0, s, in, out);
  return hipGetLastError();
}

hipError_t launch_selftest_ln(const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(selftest_ln_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_copy(const int4* src, int4* dst, int64_t n16, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(256 * 16), dim3(kBlock), 0, s, src, dst, n16);
  return hipGetLastError();
}

hipError_t launch_selftest_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m,
                                 double p, int64_t n, long long* out, hipStream_t s) {
  hipLaunchKernelGGL(selftest_binom_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), stream_id, window,
                     (long long)m, p, n, out);
  return hipGetLastError();
}

}  // namespace rdx
