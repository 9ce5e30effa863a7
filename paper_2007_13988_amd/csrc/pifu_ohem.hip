// Point-OHEM sampling for the surrogate's distillation (Sec. 3.3, Eq. 6 right): every
// training point keeps an inverse sampling probability w = 1 / (exp(-L / alpha) + beta)
// from its last BCE loss L, and batches are drawn with replacement with probability
// proportional to w.
//
// Weights are quantised to q = floor(w * 2^16) (w is capped at 2^20, so with at most
// 2^27 points the 64-bit prefix sums cannot overflow) and summed exactly in integers, so
// every draw is reproducible whatever the scan order.  Draw b takes
// r = SplitMix64 output number counter * batch + b of state seed, the target
// t = floor(r * S / 2^64) with S the total, and the first point whose inclusive prefix
// sum exceeds t.
#include "pifu_internal.h"

namespace pifu {

namespace {

constexpr int kScanTile = 4096;   // points per scan workgroup (256 threads x 16)
constexpr float kWMax = 1048576.f;

inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline uint64_t quantize(float w) {
  // w * 2^16 is exact in float32 (a power-of-two scale) and below 2^36
  return (uint64_t)floorf(w * 65536.f);
}

// Block-wide inclusive scan of 256 per-thread uint64 values (wave scans, then waves).
__device__ inline uint64_t block_scan_incl(uint64_t v, uint64_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  uint64_t add = 0;
  for (int w = 0; w < wave; ++w) add += wsum[w];
  __syncthreads();
  return v + add;
}

// Pass 1: total of each tile of quantised weights.
__global__ void __launch_bounds__(256) k_ohem_tile_sums(const float* __restrict__ w, uint32_t n,
                                                        uint64_t* __restrict__ tsum) {
  __shared__ uint64_t wsum[4];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * 16;
  uint64_t v = 0;
  for (int i = 0; i < 16; ++i)
    if (base + i < n) v += quantize(w[base + i]);
  v = block_scan_incl(v, wsum);
  if (threadIdx.x == 255) tsum[blockIdx.x] = v;
}

// Pass 2 (one workgroup): exclusive scan of the tile totals, in order.
__global__ void __launch_bounds__(256) k_ohem_scan_tiles(uint64_t* __restrict__ tsum, uint32_t nt) {
  __shared__ uint64_t wsum[4];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < nt; c0 += 256) {
    const uint32_t i = c0 + threadIdx.x;
    const uint64_t v = i < nt ? tsum[i] : 0;
    const uint64_t incl = block_scan_incl(v, wsum);
    const uint64_t base = carry;
    if (i < nt) tsum[i] = base + incl - v;
    __syncthreads();
    if (threadIdx.x == 255) carry = base + incl;
    __syncthreads();
  }
}

// Pass 3: inclusive prefix sums S[m] = q[0] + ... + q[m].
__global__ void __launch_bounds__(256) k_ohem_prefix(const float* __restrict__ w, uint32_t n,
                                                     const uint64_t* __restrict__ toff,
                                                     uint64_t* __restrict__ S) {
  __shared__ uint64_t wsum[4];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * 16;
  uint64_t q[16];
  uint64_t v = 0;
  for (int i = 0; i < 16; ++i) {
    q[i] = base + i < n ? quantize(w[base + i]) : 0;
    v += q[i];
  }
  uint64_t run = block_scan_incl(v, wsum) - v + toff[blockIdx.x];
  for (int i = 0; i < 16; ++i) {
    run += q[i];
    if (base + i < n) S[base + i] = run;
  }
}

// One thread per draw: the target in [0, S) and a binary search for the first prefix sum
// above it; the drawn point is copied into the batch.
__global__ void __launch_bounds__(256)
k_ohem_draw(const uint64_t* __restrict__ S, uint32_t n, uint32_t batch, uint64_t seed,
            uint64_t counter, const float4* __restrict__ pool, uint32_t* __restrict__ idx,
            float4* __restrict__ out) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const uint64_t total = S[n - 1];
  const uint64_t r = splitmix64(seed, counter * (uint64_t)batch + b);
  const uint64_t t = __umul64hi(r, total);
  uint32_t lo = 0, hi = n - 1;   // S[hi] = total > t
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (S[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  idx[b] = lo;
  if (out) out[b] = pool[lo];
}

// w[idx[b]] = min(1 / (exp(-L[b] / alpha) + beta), 2^20).  Points drawn twice in a batch
// have equal losses, so their stores agree.
__global__ void __launch_bounds__(256)
k_ohem_update(const float* __restrict__ L, const uint32_t* __restrict__ idx, uint32_t batch,
              float alpha, float beta, float* __restrict__ w) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const float v = 1.f / (expf(-L[b] / alpha) + beta);
  w[idx[b]] = fminf(v, kWMax);
}

}  // namespace

size_t ohem_workspace_bytes(uint32_t n) {
  const size_t nt = (n + kScanTile - 1) / kScanTile;
  return (nt + (size_t)n) * sizeof(uint64_t) + 256;
}

void launch_ohem_sample(const float* w, uint32_t n, const float4* pool, uint32_t batch,
                        uint64_t seed, uint64_t counter, uint32_t* idx, float4* out, void* ws,
                        hipStream_t s) {
  const uint32_t nt = (n + kScanTile - 1) / kScanTile;
  uint64_t* tsum = reinterpret_cast<uint64_t*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~(uintptr_t)255);
  uint64_t* S = tsum + nt;
  hipLaunchKernelGGL(k_ohem_tile_sums, dim3(nt), dim3(256), 0, s, w, n, tsum);
  hipLaunchKernelGGL(k_ohem_scan_tiles, dim3(1), dim3(256), 0, s, tsum, nt);
  hipLaunchKernelGGL(k_ohem_prefix, dim3(nt), dim3(256), 0, s, w, n, tsum, S);
  hipLaunchKernelGGL(k_ohem_draw, dim3(grid1d(batch, 256)), dim3(256), 0, s, S, n, batch, seed,
                     counter, pool, idx, out);
}

void launch_ohem_update(const float* L, const uint32_t* idx, uint32_t batch, float alpha,
                        float beta, float* w, hipStream_t s) {
  hipLaunchKernelGGL(k_ohem_update, dim3(grid1d(batch, 256)), dim3(256), 0, s, L, idx, batch,
                     alpha, beta, w);
}

}  // namespace pifu
