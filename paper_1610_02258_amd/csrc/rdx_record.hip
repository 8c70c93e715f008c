// rdx_record.hip -- recording of per-region counts (gfx950).
//
// Section 3.2 records, at a fixed simulated interval, how many molecules of
// each species sit in each region.  out[g * S + s] = sum over the tets t of
// region g of counts[s][t], as unsigned 64-bit sums (a region of 1e6 tets at
// 2^30 molecules per count would overflow 32 bits).
//
// The reduction is HBM-bound: it reads the S x T int32 counts once (4 S bytes
// per tet) and the region labels once per species (T bytes, from L2 after the
// first species).  A few thousand blocks share the species; each walks its
// species' tets with a grid stride, every lane keeping one register
// accumulator per region; the 64 lanes of a wave combine them by cross-lane
// exchange, the waves through LDS, and the block writes its sums to a slot of
// its own in a scratch array.  A second kernel, one block per species, adds
// the slots and writes out.  No atomics: device-scope atomics on one address
// from hundreds of blocks serialise (about 0.1 us each, measured), which made
// an atomic version 5-10x slower than the streaming read.  Integer sums are
// exact, so the order of the additions does not change the result.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rdx_kernels.hpp"

namespace rdx {
namespace {

constexpr int kRecThreads = 256;
constexpr int kRecUnroll = 4;
constexpr int kRecMaxBlocks = 4096;  // all species together
constexpr int kRecMaxRegions = 8;
constexpr int kRecMaxSpecies = 16;

__device__ inline unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// grid: x = blocks sharing one species (grid-stride over its tets), y =
// species.  NR >= n_regions keeps one accumulator per region (selected by
// compare, so that they stay in registers; labels are < n_regions); NR = 1
// ignores labels.
template <int NR>
__global__ __launch_bounds__(kRecThreads) void region_counts_kernel(
    const int32_t* __restrict__ counts, const uint8_t* __restrict__ region, int T, int S,
    int n_regions, unsigned long long* __restrict__ partial) {
  __shared__ unsigned long long part[kRecThreads / 64][NR];
  const int s = blockIdx.y;
  const int32_t* c = counts + (size_t)s * (size_t)T;
  unsigned long long acc[NR];
#pragma unroll
  for (int g = 0; g < NR; ++g) acc[g] = 0ull;
  const int64_t stride = (int64_t)gridDim.x * kRecThreads;
  int64_t t = (int64_t)blockIdx.x * kRecThreads + threadIdx.x;
  for (; t + (kRecUnroll - 1) * stride < T; t += kRecUnroll * stride) {
    unsigned v[kRecUnroll];
    int g[kRecUnroll];
#pragma unroll
    for (int k = 0; k < kRecUnroll; ++k) {
      v[k] = (unsigned)c[t + k * stride];  // counts are never negative
      g[k] = NR > 1 ? (int)region[t + k * stride] : 0;
    }
#pragma unroll
    for (int k = 0; k < kRecUnroll; ++k)
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] += (g[k] == q) ? (unsigned long long)v[k] : 0ull;
  }
  for (; t < T; t += stride) {
    const unsigned long long v = (unsigned)c[t];
    const int g = NR > 1 ? (int)region[t] : 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] += (g == q) ? v : 0ull;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < n_regions) {  // uniform: only the regions the model has
      const unsigned long long v = wave_sum(acc[q]);
      if (lane == 0) part[wave][q] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < n_regions) {
    unsigned long long v = 0ull;
#pragma unroll
    for (int w = 0; w < kRecThreads / 64; ++w) v += part[w][threadIdx.x];
    partial[((size_t)s * gridDim.x + blockIdx.x) * kRecMaxRegions + threadIdx.x] = v;
  }
}

// one block per species: out[g * S + s] = sum over the nb slots of species s
__global__ __launch_bounds__(kRecThreads) void region_sums_finish_kernel(
    const unsigned long long* __restrict__ partial, int nb, int S, int n_regions,
    unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[kRecThreads / 64];
  const int s = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int g = 0; g < n_regions; ++g) {
    unsigned long long v = 0ull;
    for (int b = threadIdx.x; b < nb; b += kRecThreads)
      v += partial[((size_t)s * nb + b) * kRecMaxRegions + g];
    v = wave_sum(v);
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long sum = 0ull;
#pragma unroll
      for (int w = 0; w < kRecThreads / 64; ++w) sum += part[w];
      out[g * S + s] = sum;
    }
    __syncthreads();
  }
}

// Partial sums of the allocation-free recording entry point: a file-scope
// device array, one copy on every device the library runs on, kept until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name stands for a host-side shadow, not a device address); it
// passes the device address that hipGetSymbolAddress returns for the current
// device.
static __device__ __align__(256) unsigned long long scratch[kRegionScratchBytes / sizeof(unsigned long long)];

// Slots the region-sum kernels write for (T, S): nb blocks per species, one
// slot of kRecMaxRegions sums per block.
int region_blocks(int32_t T, int32_t S) {
  const int64_t want = ((int64_t)T + kRecThreads * kRecUnroll - 1) / (kRecThreads * kRecUnroll);
  const int64_t cap = kRecMaxBlocks / S > 0 ? kRecMaxBlocks / S : 1;
  int nb = (int)(want < cap ? want : cap);
  // workgroups go to the 8 XCDs round-robin by linear id (x + s nb): with nb
  // a multiple of 8, block x sits on the same XCD for every species, so the
  // region labels of its tets come from that XCD's L2 after the first species
  if (nb >= 8) nb &= ~7;
  return nb;
}

}  // namespace

size_t region_scratch_bytes(int32_t T, int32_t S) {
  if (T <= 0 || S <= 0) return 0;
  return (size_t)S * (size_t)region_blocks(T, S) * kRecMaxRegions * sizeof(unsigned long long);
}

hipError_t static_region_scratch(unsigned long long** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static unsigned long long* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {  // first call on this device (it is the current one)
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<unsigned long long*>(p);
  }
  *ptr = addr[dev];
  *bytes = sizeof(scratch);
  return hipSuccess;
}

hipError_t launch_region_counts(const int32_t* counts, const uint8_t* region, int32_t T, int32_t S,
                                int32_t n_regions, unsigned long long* scratch, unsigned long long* out,
                                hipStream_t stream) {
  if (!counts || !scratch || !out || T <= 0 || S <= 0 || S > kRecMaxSpecies || n_regions <= 0 ||
      n_regions > kRecMaxRegions || (n_regions > 1 && !region))
    return hipErrorInvalidValue;
  // enough blocks to fill the chip, few enough that each thread sums several
  // tets; S * nb * kRecMaxRegions slots <= kRecMaxBlocks * kRecMaxRegions
  const int nb = region_blocks(T, S);
  static_assert((size_t)kRecMaxBlocks * kRecMaxRegions * sizeof(unsigned long long) <= kRegionScratchBytes,
                "region-sum scratch too small");
  const dim3 grid((unsigned)nb, (unsigned)S);
  // the fewest accumulators that hold every region: each costs a compare and
  // a 64-bit add per tet
  if (n_regions > 4)
    region_counts_kernel<8><<<grid, kRecThreads, 0, stream>>>(counts, region, T, S, n_regions, scratch);
  else if (n_regions > 2)
    region_counts_kernel<4><<<grid, kRecThreads, 0, stream>>>(counts, region, T, S, n_regions, scratch);
  else if (n_regions == 2)
    region_counts_kernel<2><<<grid, kRecThreads, 0, stream>>>(counts, region, T, S, n_regions, scratch);
  else
    region_counts_kernel<1><<<grid, kRecThreads, 0, stream>>>(counts, nullptr, T, S, 1, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  region_sums_finish_kernel<<<S, kRecThreads, 0, stream>>>(scratch, nb, S, n_regions, out);
  return hipGetLastError();
}

}  // namespace rdx
