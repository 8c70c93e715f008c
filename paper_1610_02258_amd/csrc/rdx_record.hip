// rdx_record.hip -- recording of per-region counts (gfx950).
//
// Section 3.2 records, at a fixed simulated interval, how many molecules of
// each species sit in each region.  out[g * S + s] = sum over the tets t of
// region g of counts[s][t], as unsigned 64-bit sums (a region of 1e6 tets at
// 2^30 molecules per count would overflow 32 bits).
//
// The reduction is HBM-bound: it reads the S x T int32 counts once (4 S bytes
// per tet) and the region labels once per species (T bytes, from L2 after the
// first species).  Each block sums 2048 tets of one species: every lane keeps
// one register accumulator per region, the 64 lanes of a wave combine them by
// cross-lane exchange, the waves through LDS, and one global integer atomic
// per (block, region) adds the block's sum.  Integer sums are exact, so the
// order of the atomics does not change the result.
#include <hip/hip_runtime.h>

#include "rdx_kernels.hpp"

namespace rdx {
namespace {

constexpr int kRecThreads = 256;
constexpr int kRecTetsPerThread = 8;
constexpr int kRecTetsPerBlock = kRecThreads * kRecTetsPerThread;
constexpr int kRecMaxRegions = 8;
constexpr int kRecMaxSpecies = 16;

__global__ void zero_sums_kernel(unsigned long long* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 0ull;
}

// grid: x = blocks of kRecTetsPerBlock tets, y = species
__global__ __launch_bounds__(kRecThreads) void region_counts_kernel(
    const int32_t* __restrict__ counts, const uint8_t* __restrict__ region, int T, int S,
    int n_regions, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[kRecThreads / 64][kRecMaxRegions];
  const int s = blockIdx.y;
  const int32_t* c = counts + (size_t)s * (size_t)T;
  const int64_t first = (int64_t)blockIdx.x * kRecTetsPerBlock + threadIdx.x;
  unsigned long long acc[kRecMaxRegions];
#pragma unroll
  for (int g = 0; g < kRecMaxRegions; ++g) acc[g] = 0ull;
#pragma unroll
  for (int k = 0; k < kRecTetsPerThread; ++k) {
    const int64_t t = first + (int64_t)k * kRecThreads;
    if (t < T) {
      const unsigned long long v = (unsigned)c[t];  // counts are never negative
      const int g = region ? (int)region[t] : 0;
#pragma unroll
      for (int q = 0; q < kRecMaxRegions; ++q) acc[q] += (g == q) ? v : 0ull;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kRecMaxRegions; ++q) {
    unsigned long long v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) part[wave][q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < n_regions) {
    unsigned long long v = 0ull;
#pragma unroll
    for (int w = 0; w < kRecThreads / 64; ++w) v += part[w][threadIdx.x];
    if (v) atomicAdd(&out[threadIdx.x * S + s], v);
  }
}

}  // namespace

hipError_t launch_region_counts(const int32_t* counts, const uint8_t* region, int32_t T, int32_t S,
                                int32_t n_regions, unsigned long long* out, hipStream_t stream) {
  if (!counts || !out || T <= 0 || S <= 0 || S > kRecMaxSpecies || n_regions <= 0 ||
      n_regions > kRecMaxRegions || (n_regions > 1 && !region))
    return hipErrorInvalidValue;
  const int n = n_regions * S;  // <= 128
  zero_sums_kernel<<<1, 128, 0, stream>>>(out, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((T + kRecTetsPerBlock - 1) / kRecTetsPerBlock), (unsigned)S);
  region_counts_kernel<<<grid, kRecThreads, 0, stream>>>(counts, n_regions > 1 ? region : nullptr, T, S,
                                                         n_regions, out);
  return hipGetLastError();
}

}  // namespace rdx
