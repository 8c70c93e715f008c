// rdx_kernels.hip -- gfx950 kernels of the operator-splitting reaction-diffusion
// window ("Parallel STEPS", Algorithm 1), one lane per tetrahedron.
//
// Per window and tet the kernel does, in the paper's order:
//   1. load the tet's counts (species-major SoA, coalesced over tets);
//   2. the reaction SSA operator: propensities of the tet's reactions, exact
//      SSA events until the next one would fall outside the window, reaction
//      selection by composition-rejection (Slepoy, Thompson & Plimpton 2008),
//      FP64 time, occupancy O_S += N_S (dt - t_S) for every species an event
//      changes, finalised at the window end;
//   3. the diffusion operator for each diffusive species: mean occupancy
//      Nbar = O_S / tau, leavers n = Bin(round(Nbar), tau D_S G) (stochastic
//      rounding, clamped to the post-reaction count), split over the faces by
//      sequential conditional binomials with probabilities g_k / sum_{j>=k} g_j;
//   4. integer atomic adds of the remainder into the tet's own slot and of the
//      face moves into the neighbours' slots of the next count buffer -- the
//      single-GPU form of the paper's local application plus remote change
//      buffers; integer addition makes the result independent of order.
// Random numbers are Philox4x32-10 (Salmon et al., SC'11) with the counter
// (draw call, stream, tet, window); stream 0 is the tet's SSA, stream 1+s the
// diffusion of species s.  The logarithm and the binomial use only correctly
// rounded IEEE-754 binary64 operations in a fixed order (no fp contraction),
// so results are reproducible bit for bit on any IEEE implementation of the
// same operation sequence.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rdx_internal.hpp"
#include "rdx_kernels.hpp"

#pragma clang fp contract(off)

namespace rdx {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- Philox ----
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo0 = 0xD2511F53u * x0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t lo1 = 0xCD9E8D57u * x2;
    const uint32_t y0 = hi1 ^ x1 ^ k0;
    const uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
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
  __device__ __forceinline__ double u() {
    if (pos == 4) {
      w0 = call;
      w1 = sid;
      w2 = tet;
      w3 = win;
      philox4x32_10(w0, w1, w2, w3, k0, k1);
      ++call;
      pos = 0;
    }
    const uint32_t w = pos == 0 ? w0 : (pos == 1 ? w1 : (pos == 2 ? w2 : w3));
    ++pos;
    return (double)w * 0x1p-32;
  }
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
      f = ((f * r) * (double)(c - k)) / (double)(k + 1);
      k = k + 1;
      F = F + f;
    }
    total += k;
    m -= c;
  }
  return total;
}

__device__ __forceinline__ long long binom(long long m, double p, Draw32& st) {
  if (m <= 0 || !(p > 0.0)) return 0;
  if (p >= 1.0) return m;
  if (p > 0.5) return m - binom_core(m, 1.0 - p, st);
  return binom_core(m, p, st);
}

// ---------------------------------------------------------- propensity ----
__device__ __forceinline__ int exp_field(double a) {
  return (int)((__double_as_longlong(a) >> 52) & 0x7ff);
}

template <int SMAX>
__device__ __forceinline__ int select_count(const int (&N)[SMAX], int s) {
  int v = 0;
#pragma unroll
  for (int j = 0; j < SMAX; ++j) v = (j == s) ? N[j] : v;
  return v;
}

// a_r = c_r h_r(N): c = k N_A V[L] (order 0), k (order 1), k / (N_A V[L])
// (order 2); h = 1, N_A, N_A N_B or N_A (N_A - 1) / 2.  Values below 2^-1000
// are taken as zero.
template <int SMAX>
__device__ __forceinline__ double propensity(const DevModel* __restrict__ M, int r, double k,
                                             const int (&N)[SMAX], double nav, double inv_nav) {
  const int order = M->order[r];
  double c, h;
  if (order == 0) {
    c = k * nav;
    h = 1.0;
  } else if (order == 1) {
    c = k;
    h = (double)select_count<SMAX>(N, M->r0[r]);
  } else {
    c = k * inv_nav;
    const int n0 = select_count<SMAX>(N, M->r0[r]);
    if (M->r0[r] == M->r1[r]) {
      h = n0 >= 2 ? ((double)n0 * (double)(n0 - 1)) * 0.5 : 0.0;
    } else {
      const int n1 = select_count<SMAX>(N, M->r1[r]);
      h = (double)n0 * (double)n1;
    }
  }
  const double a = c * h;
  return a >= 0x1p-1000 ? a : 0.0;
}

// Composition: groups of reactions with equal binary exponent, visited from
// the largest exponent down, picked with probability proportional to their
// totals; rejection: a uniform member is accepted with probability a / 2^g.
template <int RMAX>
__device__ int cr_select(const double (&a)[RMAX], int R, double a0, Draw53& st) {
  double x = st.co() * a0;
  int gprev = 4096, chosen = -1;
  for (;;) {
    int gcur = -1;
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
      if (r < R && a[r] > 0.0) {
        const int E = exp_field(a[r]);
        if (E < gprev && E > gcur) gcur = E;
      }
    if (gcur < 0) break;
    double sum = 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
      if (r < R && a[r] > 0.0 && exp_field(a[r]) == gcur) sum = sum + a[r];
    chosen = gcur;
    if (x < sum) break;
    x = x - sum;
    gprev = gcur;
  }
  int n = 0;
#pragma unroll
  for (int r = 0; r < RMAX; ++r)
    if (r < R && a[r] > 0.0 && exp_field(a[r]) == chosen) ++n;
  const double bound = __longlong_as_double((long long)(chosen + 1) << 52);
  for (;;) {
    const double u2 = st.co();
    int j = (int)(u2 * (double)n);
    if (j >= n) j = n - 1;
    const double u3 = st.co();
    double aj = 0.0;
    int rj = 0, seen = 0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
      if (r < R && a[r] > 0.0 && exp_field(a[r]) == chosen) {
        if (seen == j) {
          aj = a[r];
          rj = r;
        }
        ++seen;
      }
    if (u3 * bound < aj) return rj;
  }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD one
// contiguous range of tets so that neighbour updates stay in its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, xcd = b & 7, slot = b >> 3;
  return (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + slot;
}

// ------------------------------------------------------- window kernel ----
template <int SMAX, int RMAX>
__global__ void __launch_bounds__(kBlock) window_kernel(const WindowArgs A) {
  __shared__ double s_kc[kMaxRegions][RMAX];
  __shared__ int8_t s_delta[RMAX][SMAX];
  __shared__ unsigned long long s_deps[RMAX];
  const DevModel* __restrict__ M = A.model;
  for (int x = threadIdx.x; x < kMaxRegions * RMAX; x += kBlock)
    s_kc[x / RMAX][x % RMAX] = M->kcst[x / RMAX][x % RMAX];
  for (int x = threadIdx.x; x < RMAX * SMAX; x += kBlock)
    s_delta[x / SMAX][x % SMAX] = M->delta[x / SMAX][x % SMAX];
  for (int x = threadIdx.x; x < RMAX; x += kBlock) s_deps[x] = M->deps[x];
  __syncthreads();

  const int T = A.T, S = A.S, R = A.R;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  unsigned long long n_ev = 0, n_moved = 0;
  int errbits = 0;

  if (i < T) {
    int N[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      N[s] = 0;
      if (s < S) {
        int32_t* p = A.cnt_in + (size_t)s * T + i;
        const int v = *p;
        N[s] = v;
        if (v != 0) *p = 0;  // the buffer is the next window's (zeroed) target
      }
    }
    const int reg = A.region ? (int)A.region[i] : 0;
    const double nav = A.nav[i];
    const double inv_nav = 1.0 / nav;
    double a[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
      a[r] = r < R ? propensity<SMAX>(M, r, s_kc[reg][r], N, nav, inv_nav) : 0.0;

    // ---- reaction SSA operator over [0, tau_k] ----
    double O[SMAX], tS[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      O[s] = 0.0;
      tS[s] = 0.0;
    }
    uint32_t touched = 0;
    const double tau = A.tau_k;
    Draw53 st(A.key0, A.key1, 0u, (uint32_t)i, A.window);
    double dt = 0.0;
    for (;;) {
      double a0 = 0.0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r)
        if (r < R) a0 = a0 + a[r];
      if (!(a0 > 0.0)) break;
      const double u = st.oc();
      const double t_reac = -ln_basic(u) / a0;
      if (dt + t_reac > tau) break;
      const int rn = cr_select<RMAX>(a, R, a0, st);
      dt = dt + t_reac;
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        if (s < S) {
          const int d = s_delta[rn][s];
          if (d != 0) {
            O[s] = O[s] + (double)N[s] * (dt - tS[s]);
            tS[s] = dt;
            touched |= 1u << s;
            N[s] += d;
            if (N[s] > kCountCap) errbits |= kErrOverflow;
          }
        }
      }
      const unsigned long long dep = s_deps[rn];
#pragma unroll
      for (int r = 0; r < RMAX; ++r)
        if (r < R && ((dep >> r) & 1ull)) a[r] = propensity<SMAX>(M, r, s_kc[reg][r], N, nav, inv_nav);
      ++n_ev;
      if (errbits) break;
      if (n_ev >= (unsigned long long)kEventCap) {
        errbits |= kErrEvents;
        break;
      }
    }
#pragma unroll
    for (int s = 0; s < SMAX; ++s)
      if ((touched >> s) & 1u) O[s] = O[s] + (double)N[s] * (tau - tS[s]);

    // ---- diffusion operator ----
    const int4 nb = reinterpret_cast<const int4*>(A.nbr)[i];
    const double2* gp = reinterpret_cast<const double2*>(A.geo) + 2 * (size_t)i;
    const double2 ga = gp[0], gb = gp[1];
    const double G = ga.x;  // sum of the face couplings
    const int last = nb.w >= 0 ? 3 : (nb.z >= 0 ? 2 : (nb.y >= 0 ? 1 : (nb.x >= 0 ? 0 : -1)));
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s >= S) continue;
      long long n = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
      if (A.tauD[s] > 0.0 && G > 0.0) {
        Draw32 sp(A.key0, A.key1, 1u + (uint32_t)s, (uint32_t)i, A.window);
        const double Nbar = ((touched >> s) & 1u) ? O[s] / tau : (double)N[s];
        const double fl = floor(Nbar);
        const double frac = Nbar - fl;
        long long m = (long long)fl;
        if (frac > 0.0) {
          if (sp.u() < frac) m += 1;
        }
        double p = A.tauD[s] * G;
        if (p > 1.0) p = 1.0;
        n = binom(m, p, sp);
        if (n > N[s]) n = N[s];
        long long rem = n;
        if (rem > 0 && nb.x >= 0) {
          if (last == 0) { o0 = rem; rem = 0; }
          else { o0 = binom(rem, ga.y, sp); rem -= o0; }
        }
        if (rem > 0 && nb.y >= 0) {
          if (last == 1) { o1 = rem; rem = 0; }
          else { o1 = binom(rem, gb.x, sp); rem -= o1; }
        }
        if (rem > 0 && nb.z >= 0) {
          if (last == 2) { o2 = rem; rem = 0; }
          else { o2 = binom(rem, gb.y, sp); rem -= o2; }
        }
        if (rem > 0 && nb.w >= 0) { o3 = rem; rem = 0; }
      }
      int32_t* out = A.cnt_out + (size_t)s * T;
      const int keep = N[s] - (int)n;
      if (keep != 0) atomicAdd(out + i, keep);
      if (o0) atomicAdd(out + nb.x, (int)o0);
      if (o1) atomicAdd(out + nb.y, (int)o1);
      if (o2) atomicAdd(out + nb.z, (int)o2);
      if (o3) atomicAdd(out + nb.w, (int)o3);
      n_moved += (unsigned long long)(o0 + o1 + o2 + o3);
    }
  }

  const unsigned long long ev_sum = wave_sum(n_ev);
  const unsigned long long mv_sum = wave_sum(n_moved);
  if ((threadIdx.x & 63) == 0) {
    if (ev_sum) atomicAdd(A.tally + 0, ev_sum);
    if (mv_sum) atomicAdd(A.tally + 1, mv_sum);
  }
  if (errbits) atomicOr(A.err, errbits);
}

// ----------------------------------------------------------- self-tests ----
__global__ void selftest_philox_kernel(const uint32_t* in, uint32_t* out, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t x0 = in[6 * j], x1 = in[6 * j + 1], x2 = in[6 * j + 2], x3 = in[6 * j + 3];
  philox4x32_10(x0, x1, x2, x3, in[6 * j + 4], in[6 * j + 5]);
  out[4 * j] = x0;
  out[4 * j + 1] = x1;
  out[4 * j + 2] = x2;
  out[4 * j + 3] = x3;
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

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_window(const WindowArgs& a, hipStream_t stream) {
  const dim3 grid(grid_for(a.T)), block(kBlock);
  if (a.S <= 4 && a.R <= 4)
    hipLaunchKernelGGL((window_kernel<4, 4>), grid, block, 0, stream, a);
  else if (a.S <= 8 && a.R <= 8)
    hipLaunchKernelGGL((window_kernel<8, 8>), grid, block, 0, stream, a);
  else if (a.S <= 12 && a.R <= 12)
    hipLaunchKernelGGL((window_kernel<12, 12>), grid, block, 0, stream, a);
  else if (a.S <= 16 && a.R <= 24)
    hipLaunchKernelGGL((window_kernel<16, 24>), grid, block, 0, stream, a);
  else
    hipLaunchKernelGGL((window_kernel<16, 32>), grid, block, 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(selftest_philox_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_selftest_ln(const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(selftest_ln_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
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
