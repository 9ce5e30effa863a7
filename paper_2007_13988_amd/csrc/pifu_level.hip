// Level kernels of hierarchical surface localization (Sec. 3.2): level transition
// (binarize + trilinear x2), 1-ring dilation, stable stream compaction, conflict
// expansion, surface-cell extraction.  All are HBM/L2-bound byte-state passes.
#include <algorithm>

#include "pifu_internal.h"

namespace pifu {

static inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

__global__ void k_fill_u8(uint8_t* __restrict__ p, uint8_t v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_set_words(uint32_t* __restrict__ p, uint32_t v, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Fills n words with a kernel (not hipMemsetAsync: the calls that may be captured into a
// graph clear their counters this way).
void launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s, uint32_t n) {
  if (n) hipLaunchKernelGGL(k_set_words, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
}

// Bookkeeping of the device-driven calls: a few counter updates in order, one thread.
__global__ void k_book(BookOps b) {
  for (int i = 0; i < b.n; ++i) {
    const BookOp& o = b.op[i];
    const uint32_t a = o.src ? *o.src : 0u;
    const uint32_t c = o.src2 ? *o.src2 : 0u;
    const bool flag = o.aux ? *o.aux != 0u : true;
    switch (o.kind) {
      case BK_ADD: *o.dst += a; break;
      case BK_ADD_NZ: *o.dst += a != 0u; break;
      case BK_SET: *o.dst = a; break;
      case BK_SET_IMM: *o.dst = o.imm; break;
      case BK_FLAG_GT: if (a > o.imm) *o.dst |= o.bit; break;
      case BK_SEL: *o.dst = flag ? a : 0u; break;
      case BK_ADD_SEL: *o.dst += flag ? a : c; break;
      default: break;
    }
  }
}

void launch_book(const BookOps& b, hipStream_t s) {
  if (b.n) hipLaunchKernelGGL(k_book, dim3(1), dim3(1), 0, s, b);
}

void launch_fill_u8(uint8_t* p, uint8_t v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u8, dim3(grid1d(n, 256)), dim3(256), 0, s, p, v, n);
}

// Count read-back: words c[0 .. n) to host-mapped, fine-grained memory, then the
// sequence number the host waits for.  Every lane makes its stores visible at system
// scope before the barrier, so the release store of the sequence word is ordered
// after all of them.
__global__ void __launch_bounds__(256) k_publish(const uint32_t* __restrict__ c, int n,
                                                 uint32_t* host, uint32_t* seq_word, uint32_t seq) {
  for (int t = threadIdx.x; t < n; t += blockDim.x)
    __hip_atomic_store(host + t, c[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(seq_word, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish(const uint32_t* c, int n, uint32_t* host, uint32_t* seq_word, uint32_t seq,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, s, c, n, host, seq_word, seq);
}

__global__ void k_iota(uint32_t* __restrict__ list, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) list[i] = i;
}

void launch_iota(uint32_t* list, uint32_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_iota, dim3(grid1d(n, 256)), dim3(256), 0, s, list, n);
}

// Occupancy p = sigmoid(logit), in float32 with the expression the grid's apply kernels use.
__global__ void k_occupancy(const float* __restrict__ logit, uint32_t n, float* __restrict__ occ) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) occ[i] = 1.0f / (1.0f + expf(-logit[i]));
}

void launch_occupancy(const float* logit, uint32_t n, float* occ, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_occupancy, dim3(grid1d(n, 256)), dim3(256), 0, s, logit, n, occ);
}

// Level transition.  Coarse level nodes keep their label, evaluated flag and value;
// every other fine node gets the mean of the binarized labels of its 2/4/8 enclosing
// coarse corners (trilinear interpolation of the binary field).  Fractional means are
// boundary candidates (ST_B0); integral ones are the culled value.
__global__ void k_transition(const uint8_t* __restrict__ cst, const float* __restrict__ cocc,
                             Lat c, uint8_t* __restrict__ fst, float* __restrict__ focc, Lat f,
                             FrameOcc fo) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;   // one frame has < 2^32 nodes
  if (n >= (uint32_t)f.n()) return;
  // frame blockIdx.y of a multi-frame state array
  cst += (size_t)blockIdx.y * c.n();
  cocc += (size_t)blockIdx.y * c.n();
  fst += (size_t)blockIdx.y * f.n();
  focc = fo.p[blockIdx.y] ? fo.p[blockIdx.y] : focc + (size_t)blockIdx.y * f.n();
  const uint32_t nyz = (uint32_t)f.ny * f.nz;
  const uint32_t a = n / nyz;
  const uint32_t r = n - a * nyz;
  const uint32_t b = r / f.nz;
  const uint32_t k = r - b * f.nz;
  const uint32_t a0 = a >> 1, a1 = (a + 1) >> 1;
  const uint32_t b0 = b >> 1, b1 = (b + 1) >> 1;
  const uint32_t k0 = k >> 1, k1 = (k + 1) >> 1;
  const uint32_t cyz = (uint32_t)c.ny * c.nz;
  if (!((a | b | k) & 1)) {
    size_t cn = (size_t)a0 * cyz + (size_t)b0 * c.nz + k0;
    uint8_t s = cst[cn] & (ST_LABEL | ST_EVAL);
    fst[n] = s | ((s & ST_LABEL) ? ST_HI : 0);
    focc[n] = cocc[cn];
    return;
  }
  int sum = 0, cnt = 0;
  for (int da = 0; da < 2; ++da) {
    uint32_t ia = da ? a1 : a0;
    if (da && a1 == a0) continue;
    for (int db = 0; db < 2; ++db) {
      uint32_t ib = db ? b1 : b0;
      if (db && b1 == b0) continue;
      const uint8_t* row = cst + (size_t)ia * cyz + (size_t)ib * c.nz;
      sum += row[k0] & ST_LABEL;
      ++cnt;
      if (k1 != k0) {
        sum += row[k1] & ST_LABEL;
        ++cnt;
      }
    }
  }
  uint8_t s;
  float v;
  if (sum == 0) {
    s = 0;
    v = 0.f;
  } else if (sum == cnt) {
    s = ST_LABEL | ST_HI;
    v = 1.f;
  } else {
    const bool hi = 2 * sum > cnt;
    s = ST_B0 | (hi ? (ST_HI | ST_LABEL) : 0);
    v = (float)sum / (float)cnt;
  }
  fst[n] = s;
  focc[n] = v;
}

void launch_transition(const uint8_t* cst, const float* cocc, Lat c, uint8_t* fst, float* focc,
                       Lat f, hipStream_t s, int frames, const FrameOcc* fo) {
  FrameOcc t{};
  if (fo) t = *fo;
  hipLaunchKernelGGL(k_transition, dim3(grid1d(f.n(), 256), frames), dim3(256), 0, s, cst, cocc, c,
                     fst, focc, f, t);
}

// 1-ring dilation of the boundary candidates: a node not evaluated before is selected
// when any node of its 3x3x3 neighbourhood (clipped at the grid edge) is a candidate.
__global__ void k_select(uint8_t* __restrict__ st, Lat f) {
  // one frame has < 2^32 nodes: 32-bit index arithmetic
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (uint32_t)f.n()) return;
  st += (size_t)blockIdx.y * f.n();   // frame of a multi-frame state array
  uint8_t s = st[n];
  if (s & ST_EVAL) return;
  const uint32_t nyz = (uint32_t)f.ny * f.nz;
  const int a = (int)(n / nyz);
  const int r = (int)(n - (uint32_t)a * nyz);
  const int b = r / f.nz;
  const int k = r - b * f.nz;
  bool any = false;
  for (int da = -1; da <= 1 && !any; ++da) {
    int ia = a + da;
    if (ia < 0 || ia >= f.nx) continue;
    for (int db = -1; db <= 1 && !any; ++db) {
      int ib = b + db;
      if (ib < 0 || ib >= f.ny) continue;
      const uint8_t* row = st + (size_t)ia * nyz + (size_t)ib * f.nz;
      for (int dk = -1; dk <= 1; ++dk) {
        int ik = k + dk;
        if (ik < 0 || ik >= f.nz) continue;
        if (row[ik] & ST_B0) {
          any = true;
          break;
        }
      }
    }
  }
  if (any) st[n] = s | ST_PEND;
}

void launch_select(uint8_t* st, Lat f, hipStream_t s, int frames) {
  hipLaunchKernelGGL(k_select, dim3(grid1d(f.n(), 256), frames), dim3(256), 0, s, st, f);
}

// Boundary-candidate bit masks: word w of column c (c = a * ny + b) holds the ST_B0 bits
// of nodes [64 w, 64 w + 64) of that column, one thread per word.  The word's 64 state
// bytes start at an arbitrary byte address: five aligned 16-byte loads cover them (a load
// starting at or past the frame's end is skipped; the state arrays carry 16 bytes of
// padding), each 4 bytes give 4 bits, and an 80-bit funnel shift aligns the word.  The
// count of candidates goes to counts[frame * count_stride], one atomic per workgroup.
__device__ inline uint32_t b0_nibble(uint32_t x) {
  const uint32_t v = (x >> 2) & 0x01010101u;   // ST_B0 is bit 2 of each byte
  return (v | (v >> 7) | (v >> 14) | (v >> 21)) & 0xFu;
}

__global__ void __launch_bounds__(256)
k_b0_masks(const uint8_t* __restrict__ st, Lat f, uint64_t* __restrict__ masks,
           uint32_t* __restrict__ counts, int count_stride) {
  static_assert(ST_B0 == 0x04, "b0_nibble reads bit 2");
  __shared__ uint32_t wsum[4];
  const uint32_t nw = (uint32_t)(f.nz + 63) >> 6;
  const uint32_t units = (uint32_t)f.nx * f.ny * nw;
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  st += (size_t)blockIdx.y * f.n();
  masks += (size_t)blockIdx.y * units;
  uint32_t c = 0;
  if (u < units) {
    const uint32_t col = u / nw, w = u - col * nw;
    const uint8_t* p = st + (size_t)col * f.nz + 64 * w;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    const int sh = (int)(addr & 15u);
    const uint8_t* q = reinterpret_cast<const uint8_t*>(addr - (uintptr_t)sh);
    const uint8_t* end = st + f.n();
    uint64_t lo = 0ull, hi = 0ull;   // 80 bits: byte i of the window -> bit i
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      uint4 x = make_uint4(0u, 0u, 0u, 0u);
      if (q + 16 * i < end) x = *reinterpret_cast<const uint4*>(q + 16 * i);
      const uint32_t b16 = b0_nibble(x.x) | (b0_nibble(x.y) << 4) | (b0_nibble(x.z) << 8) |
                           (b0_nibble(x.w) << 12);
      if (i < 4) lo |= (uint64_t)b16 << (16 * i);
      else hi = b16;
    }
    uint64_t m = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
    const int valid = f.nz - 64 * (int)w;   // nodes of this word inside the column
    if (valid < 64) m &= (1ull << valid) - 1ull;
    masks[u] = m;
    c = (uint32_t)__popcll(m);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (t && counts) atomicAdd(counts + (size_t)blockIdx.y * count_stride, t);
  }
}

// Marks the nodes that are not evaluated yet and have a boundary candidate among their
// 26 neighbours (or are one) as pending: one thread per mask word; the OR of the 3 x 3
// neighbouring columns' words, each widened by one node along z, gives the word's
// selected nodes, and only those state bytes are read and written.
__global__ void __launch_bounds__(256)
k_select_masks(uint8_t* __restrict__ st, Lat f, const uint64_t* __restrict__ masks) {
  const uint32_t nw = (uint32_t)(f.nz + 63) >> 6;
  const uint32_t units = (uint32_t)f.nx * f.ny * nw;
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= units) return;
  st += (size_t)blockIdx.y * f.n();
  masks += (size_t)blockIdx.y * units;
  const uint32_t col = u / nw, w = u - col * nw;
  const int a = (int)(col / (uint32_t)f.ny), b = (int)(col - (uint32_t)a * f.ny);
  uint64_t d = 0;
  for (int da = -1; da <= 1; ++da) {
    const int ia = a + da;
    if (ia < 0 || ia >= f.nx) continue;
    for (int db = -1; db <= 1; ++db) {
      const int ib = b + db;
      if (ib < 0 || ib >= f.ny) continue;
      const uint64_t* m = masks + ((size_t)ia * f.ny + ib) * nw;
      const uint64_t m0 = m[w];
      const uint64_t lo = w > 0 ? m[w - 1] : 0ull;
      const uint64_t hi = w + 1 < nw ? m[w + 1] : 0ull;
      d |= m0 | (m0 << 1) | (lo >> 63) | (m0 >> 1) | (hi << 63);
    }
  }
  const int valid = f.nz - 64 * (int)w;   // nodes of this word inside the column
  if (valid < 64) d &= (1ull << valid) - 1ull;
  uint8_t* p = st + (size_t)col * f.nz + 64 * w;
  while (d) {
    const int bit = __ffsll((unsigned long long)d) - 1;
    d &= d - 1ull;
    const uint8_t sv = p[bit];
    if (!(sv & ST_EVAL)) p[bit] = sv | ST_PEND;
  }
}

size_t b0_mask_words(Lat f) { return (size_t)f.nx * f.ny * (size_t)((f.nz + 63) / 64); }

void launch_select_b0(uint8_t* st, Lat f, int frames, uint64_t* masks, uint32_t* counts,
                      int count_stride, hipStream_t s) {
  const size_t units = b0_mask_words(f);
  if (!units) return;
  const unsigned gb = (unsigned)((units + 255) / 256);
  hipLaunchKernelGGL(k_b0_masks, dim3(gb, frames), dim3(256), 0, s, st, f, masks, counts,
                     count_stride);
  hipLaunchKernelGGL(k_select_masks, dim3((unsigned)((units + 255) / 256), frames), dim3(256), 0, s,
                     st, f, masks);
}

// ------------------------------------------------------------------ compaction
// Three passes: per-tile counts, exclusive scan of the tile counts, ordered write.
// Thread t of tile b owns nodes [b*4096 + 16t, +16), so output order is node order.

__device__ inline uint32_t pred_mask16(const uint8_t* __restrict__ st, size_t base, size_t n,
                                       uint8_t mask, uint8_t val) {
  uint32_t m = 0;
  if (base + 16 <= n) {
    uint4 q = *reinterpret_cast<const uint4*>(st + base);
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      uint8_t s = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
      m |= (uint32_t)((s & mask) == val) << i;
    }
  } else {
    for (int i = 0; i < 16; ++i)
      if (base + i < n) m |= (uint32_t)((st[base + i] & mask) == val) << i;
  }
  return m;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__global__ void __launch_bounds__(COMPACT_BLOCK)
k_compact_count(const uint8_t* __restrict__ st, size_t n, uint8_t mask, uint8_t val,
                uint32_t* __restrict__ bcount, const uint32_t* __restrict__ gate) {
  __shared__ uint32_t wsum[COMPACT_BLOCK / 64];
  if (gate && *gate == 0) return;   // nothing can be selected: the scan writes total 0
  size_t base = (size_t)blockIdx.x * COMPACT_TILE + (size_t)threadIdx.x * COMPACT_PER_THREAD;
  uint32_t c = __popc(pred_mask16(st, base, n, mask, val));
  uint32_t inc = wave_incl_scan(c);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < COMPACT_BLOCK / 64; ++w) t += wsum[w];
    bcount[blockIdx.x] = t;
  }
}

// Exclusive scan of n words by one workgroup of 1024 threads; writes the total.
__global__ void __launch_bounds__(1024)
k_scan_small(const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ out,
             uint32_t* __restrict__ total, const uint32_t* __restrict__ n_dev = nullptr,
             const uint32_t* __restrict__ gate = nullptr) {
  __shared__ uint32_t wsum[16];
  if (gate && *gate == 0) {   // gated compaction: nothing selected
    if (threadIdx.x == 0 && total) *total = 0;
    return;
  }
  const uint32_t per = (n + 1023) / 1024;   // the capacity sets the split, the count the end
  if (n_dev) n = min(n, *n_dev);
  const uint32_t beg = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (beg + i < n) loc += in[beg + i];
  uint32_t inc = wave_incl_scan(loc);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < 16; ++w) {
      uint32_t t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    if (total) *total = run;
  }
  __syncthreads();
  uint32_t run = wsum[threadIdx.x >> 6] + inc - loc;
  for (uint32_t i = 0; i < per; ++i)
    if (beg + i < n) {
      uint32_t v = in[beg + i];
      out[beg + i] = run;
      run += v;
    }
}

__global__ void __launch_bounds__(COMPACT_BLOCK)
k_compact_write(const uint8_t* __restrict__ st, size_t n, uint8_t mask, uint8_t val,
                const uint32_t* __restrict__ boff, uint32_t* __restrict__ out, uint32_t cap,
                int mode, Lat f, uint32_t index_base, const uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[COMPACT_BLOCK / 64];
  if (total && *total == 0) return;   // gated compaction with nothing selected
  size_t base = (size_t)blockIdx.x * COMPACT_TILE + (size_t)threadIdx.x * COMPACT_PER_THREAD;
  uint32_t m = pred_mask16(st, base, n, mask, val);
  uint32_t c = __popc(m);
  uint32_t inc = wave_incl_scan(c);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) woff += wsum[w];
  uint32_t pos = boff[blockIdx.x] + woff + inc - c;
  const uint32_t nyz = (uint32_t)f.ny * f.nz;
  while (m) {
    int i = __ffs(m) - 1;
    m &= m - 1;
    if (pos < cap) {
      size_t node = base + i;
      uint32_t v = index_base + (uint32_t)node;
      if (mode == 1) {
        uint32_t a = (uint32_t)(node / nyz);
        uint32_t r = (uint32_t)(node - (size_t)a * nyz);
        uint32_t b = r / f.nz;
        uint32_t k = r - b * f.nz;
        v = (a * (uint32_t)(f.ny - 1) + b) * (uint32_t)(f.nz - 1) + k;
      }
      out[pos] = v;
    }
    ++pos;
  }
}

size_t scan_scratch_words(size_t n);
// tile counts + tile offsets (+ the multi-workgroup scan's scratch for long inputs)
size_t compact_scratch_words(size_t n) {
  const size_t nb = (n + COMPACT_TILE - 1) / COMPACT_TILE;
  return nb * 2 + scan_scratch_words(nb) + 64;
}

void launch_compact(const uint8_t* st, size_t n, uint8_t mask, uint8_t val, uint32_t* bcount,
                    uint32_t* total, uint32_t* out, uint32_t cap, int mode, Lat f, hipStream_t s,
                    uint32_t index_base, const uint32_t* gate) {
  uint32_t nb = (uint32_t)((n + COMPACT_TILE - 1) / COMPACT_TILE);
  if (nb == 0) {
    launch_set_u32(total, 0, s);
    return;
  }
  uint32_t* boff = bcount + nb;
  hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(COMPACT_BLOCK), 0, s, st, n, mask, val, bcount,
                     gate);
  // one workgroup scans up to a few thousand tile counts quickly; longer inputs (many
  // frames of a batch) take the multi-workgroup scan
  if (nb <= 8192)
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, bcount, nb, boff, total, nullptr,
                       gate);
  else
    launch_scan_u32(bcount, nb, boff, bcount + 2 * (size_t)nb, total, s, nullptr, gate);
  hipLaunchKernelGGL(k_compact_write, dim3(nb), dim3(COMPACT_BLOCK), 0, s, st, n, mask, val, boff,
                     out, cap, mode, f, index_base, gate ? total : nullptr);
}

// ------------------------------------------------------------------ generic scan (render)
__global__ void __launch_bounds__(1024)
k_scan_tiles(const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ tsum,
             const uint32_t* __restrict__ n_dev, const uint32_t* __restrict__ gate) {
  __shared__ uint32_t wsum[16];
  if (gate && *gate == 0) return;
  if (n_dev) n = min(n, *n_dev);
  uint32_t i = blockIdx.x * 1024 + threadIdx.x;
  uint32_t v = i < n ? in[i] : 0;
  uint32_t inc = wave_incl_scan(v);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < 16; ++w) t += wsum[w];
    tsum[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(1024)
k_scan_apply(const uint32_t* __restrict__ in, uint32_t n, const uint32_t* __restrict__ toff,
             uint32_t* __restrict__ out, const uint32_t* __restrict__ n_dev,
             const uint32_t* __restrict__ gate) {
  __shared__ uint32_t wsum[16];
  // gated: the gate word may be the total the middle pass rewrote; 0 means no output
  if (gate && *gate == 0) return;
  if (n_dev) n = min(n, *n_dev);
  uint32_t i = blockIdx.x * 1024 + threadIdx.x;
  uint32_t v = i < n ? in[i] : 0;
  uint32_t inc = wave_incl_scan(v);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) woff += wsum[w];
  if (i < n) out[i] = toff[blockIdx.x] + woff + inc - v;
}

size_t scan_scratch_words(size_t n) { return (n + 1023) / 1024 * 2 + 64; }

void launch_scan_u32(const uint32_t* in, uint32_t n, uint32_t* out_excl, uint32_t* scratch,
                     uint32_t* total, hipStream_t s, const uint32_t* n_dev, const uint32_t* gate) {
  uint32_t nt = (n + 1023) / 1024;
  if (nt == 0) {
    launch_set_u32(total, 0, s);
    return;
  }
  if (n <= 8192) {   // up to 8 words per thread: one workgroup, one launch
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, in, n, out_excl, total, n_dev,
                       gate);
    return;
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(1024), 0, s, in, n, scratch, n_dev, gate);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, scratch, nt, scratch + nt, total,
                     nullptr, gate);
  hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(1024), 0, s, in, n, scratch + nt, out_excl,
                     n_dev, gate);
}

// ------------------------------------------------------------------ evaluation results
// Writes the network's label and value into the level state; flags conflicts
// ([logit > 0] != [interp > 1/2]) among the nodes evaluated at this level.
__global__ void k_apply_grid(const uint32_t* __restrict__ list, uint32_t n,
                             const uint32_t* __restrict__ n_dev,
                             const float* __restrict__ logit, const uint8_t* __restrict__ lab,
                             uint8_t* __restrict__ st, float* __restrict__ occ,
                             uint32_t* __restrict__ conflicts, uint8_t* __restrict__ eval_level,
                             float* __restrict__ eval_logit, int level_id, Lat lvl, int stride,
                             Lat fin, int check_conflict, uint32_t frame_nodes, FrameOcc fo) {
  const uint32_t ne = n_dev ? min(n, *n_dev) : n;
  // the block's base index is uniform, so every lane of a wave runs the same iterations
  for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < ne; b0 += gridDim.x * blockDim.x) {
  const uint32_t m = b0 + threadIdx.x;
  bool conf = false;
  if (frame_nodes) {
    // multi-frame: one conflict counter per frame (no evaluation-level map)
    uint32_t frame = 0;
    if (m < ne) {
      const uint32_t node = list[m];
      const uint8_t s = st[node];
      const uint8_t l = lab[m] ? ST_LABEL : 0;
      frame = node / frame_nodes;
      const float p = 1.0f / (1.0f + expf(-logit[m]));
      if (fo.p[frame]) fo.p[frame][node - frame * frame_nodes] = p;
      else occ[node] = p;
      uint8_t ns = (uint8_t)((s & ~(ST_LABEL | ST_PEND | ST_CONF)) | ST_EVAL | ST_NOW | l);
      if (check_conflict && ((l != 0) != ((s & ST_HI) != 0))) {
        ns |= ST_CONF;
        conf = true;
      }
      st[node] = ns;
    }
    if (!conflicts) continue;
    // the list is sorted, so a wave's conflicts nearly always share one frame: one atomic
    // per wave then, one per conflict where a wave straddles frames
    const unsigned long long bal = __ballot(conf);
    if (!bal) continue;
    const int first = __ffsll((long long)bal) - 1;
    const uint32_t f0 = __shfl(frame, first, 64);
    if (__all(!conf || frame == f0)) {
      if ((int)(threadIdx.x & 63) == first) atomicAdd(conflicts + f0, (uint32_t)__popcll(bal));
    } else if (conf) {
      atomicAdd(conflicts + frame, 1u);
    }
    continue;
  }
  if (m < ne) {
    const uint32_t node = list[m];
    const uint8_t s = st[node];
    const uint8_t l = lab[m] ? ST_LABEL : 0;
    const float x = logit[m];
    const float p = 1.0f / (1.0f + expf(-x));
    uint8_t ns = (uint8_t)((s & ~(ST_LABEL | ST_PEND | ST_CONF)) | ST_EVAL | ST_NOW | l);
    if (check_conflict && ((l != 0) != ((s & ST_HI) != 0))) {
      ns |= ST_CONF;
      conf = true;
    }
    st[node] = ns;
    occ[node] = p;
    if (eval_level) {
      const uint32_t nyz = (uint32_t)lvl.ny * lvl.nz;
      uint32_t a = node / nyz;
      uint32_t r = node - a * nyz;
      uint32_t b = r / lvl.nz;
      uint32_t k = r - b * lvl.nz;
      size_t fn = ((size_t)(a * stride) * fin.ny + (size_t)(b * stride)) * fin.nz + (size_t)k * stride;
      eval_level[fn] = (uint8_t)level_id;
      if (eval_logit) eval_logit[fn] = x;
    }
  }
  if (conflicts) {
    unsigned long long bal = __ballot(conf);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(conflicts, (uint32_t)__popcll(bal));
  }
  }
}

void launch_apply_grid(const uint32_t* list, uint32_t n, const float* logit, const uint8_t* lab,
                       uint8_t* st, float* occ, uint32_t* conflicts, uint8_t* eval_level,
                       int level_id, Lat lvl, int stride, Lat fin, int check_conflict,
                       hipStream_t s, uint32_t frame_nodes, const FrameOcc* fo, float* eval_logit,
                       const uint32_t* n_dev) {
  if (!n) return;
  FrameOcc t{};
  if (fo) t = *fo;
  unsigned g = grid1d(n, 256);
  if (n_dev && g > kStrideBlocks) g = kStrideBlocks;
  hipLaunchKernelGGL(k_apply_grid, dim3(g), dim3(256), 0, s, list, n, n_dev, logit, lab, st, occ,
                     conflicts, eval_level, eval_logit, level_id, lvl, stride, fin, check_conflict,
                     frame_nodes, t);
}

// Conflict expansion: every not-yet-evaluated node of the 26-neighbourhood of a
// conflict node of the last wave is selected.  Concurrent read-modify-writes of one
// byte only ever add ST_PEND, so they agree.
__global__ void k_expand(const uint32_t* __restrict__ list, uint32_t n,
                         const uint32_t* __restrict__ n_dev, uint8_t* __restrict__ st0, Lat f,
                         uint32_t frame_nodes) {
  const uint32_t ne = n_dev ? min(n, *n_dev) : n;
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < ne; m += gridDim.x * blockDim.x) {
  uint8_t* st = st0;
  uint32_t node = list[m];
  if (!(st[node] & ST_CONF)) continue;
  if (frame_nodes) {   // neighbours stay inside the node's frame
    const uint32_t local = node % frame_nodes;
    st += (size_t)(node - local);
    node = local;
  }
  const uint32_t nyz = (uint32_t)f.ny * f.nz;
  const int a = (int)(node / nyz);
  const int r = (int)(node - (uint32_t)a * nyz);
  const int b = r / f.nz;
  const int k = r - b * f.nz;
  for (int da = -1; da <= 1; ++da) {
    int ia = a + da;
    if (ia < 0 || ia >= f.nx) continue;
    for (int db = -1; db <= 1; ++db) {
      int ib = b + db;
      if (ib < 0 || ib >= f.ny) continue;
      uint8_t* row = st + (size_t)ia * nyz + (size_t)ib * f.nz;
      for (int dk = -1; dk <= 1; ++dk) {
        int ik = k + dk;
        if (ik < 0 || ik >= f.nz) continue;
        uint8_t s = row[ik];
        if (!(s & (ST_EVAL | ST_PEND))) row[ik] = s | ST_PEND;
      }
    }
  }
  }
}

void launch_expand(const uint32_t* list, uint32_t n, uint8_t* st, Lat f, hipStream_t s,
                   uint32_t frame_nodes, const uint32_t* n_dev) {
  if (!n) return;
  unsigned g = grid1d(n, 256);
  if (n_dev && g > kStrideBlocks) g = kStrideBlocks;
  hipLaunchKernelGGL(k_expand, dim3(g), dim3(256), 0, s, list, n, n_dev, st, f, frame_nodes);
}

// bounds[f] = first position of the sorted list whose entry is >= f * frame_nodes.
__global__ void k_segment_bounds(const uint32_t* __restrict__ list, uint32_t n,
                                 uint32_t frame_nodes, int frames, uint32_t* __restrict__ bounds) {
  const int f = threadIdx.x;
  if (f > frames) return;
  const uint64_t key = (uint64_t)f * frame_nodes;
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if ((uint64_t)list[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  bounds[f] = lo;
}

void launch_segment_bounds(const uint32_t* list, uint32_t n, uint32_t frame_nodes, int frames,
                           uint32_t* bounds, hipStream_t s) {
  hipLaunchKernelGGL(k_segment_bounds, dim3(1), dim3(64), 0, s, list, n, frame_nodes, frames, bounds);
}

// ------------------------------------------------------------------ per-frame tallies
// tally[f] += entries m < min(n, *n_dev) whose node (list[pos[m]], or list[m] without
// pos) lies in frame f = node / frame_nodes: a block histogram in LDS, then one atomic
// per frame and block.
__global__ void __launch_bounds__(256)
k_frame_tally(const uint32_t* __restrict__ list, const uint32_t* __restrict__ pos, uint32_t n,
              const uint32_t* __restrict__ n_dev, uint32_t frame_nodes, uint32_t* __restrict__ tally) {
  __shared__ uint32_t h[kMaxBatch];
  if (threadIdx.x < kMaxBatch) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t ne = n_dev ? min(n, *n_dev) : n;
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < ne; m += gridDim.x * blockDim.x) {
    const uint32_t node = list[pos ? pos[m] : m];
    const uint32_t f = node / frame_nodes;
    if (f < kMaxBatch) atomicAdd(&h[f], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kMaxBatch && h[threadIdx.x]) atomicAdd(tally + threadIdx.x, h[threadIdx.x]);
}

void launch_frame_tally(const uint32_t* list, const uint32_t* pos, uint32_t n,
                        const uint32_t* n_dev, uint32_t frame_nodes, uint32_t* tally,
                        hipStream_t s) {
  if (!n) return;
  unsigned g = (unsigned)((n + 255) / 256);
  if (g > kStrideBlocks) g = kStrideBlocks;
  hipLaunchKernelGGL(k_frame_tally, dim3(g), dim3(256), 0, s, list, pos, n, n_dev, frame_nodes,
                     tally);
}

// For frame p < a.frames and op q < a.nops: *a.dst[q][p] += tally[p] (ADD), += (tally[p]
// != 0) (ADD_NZ) or = tally[p] (SET); then tally[0 .. kMaxBatch) = 0.  One block.
__global__ void k_frame_apply(uint32_t* __restrict__ tally, FrameApply a) {
  const int p = threadIdx.x;
  uint32_t v = 0;
  if (p < kMaxBatch) v = tally[p];
  __syncthreads();
  if (p < a.frames) {
    for (int q = 0; q < a.nops; ++q) {
      uint32_t* d = a.dst[q][p];
      if (!d) continue;
      if (a.kind[q] == BK_ADD) *d += v;
      else if (a.kind[q] == BK_ADD_NZ) *d += v != 0;
      else *d = v;
    }
  }
  if (p < kMaxBatch) tally[p] = 0;
}

void launch_frame_apply(uint32_t* tally, const FrameApply& a, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_apply, dim3(1), dim3(64), 0, s, tally, a);
}

// Final level: export the 0/1 labels and flag mixed cells (8 corner labels differ).
__global__ void k_cells(uint8_t* __restrict__ st, Lat f, uint8_t* __restrict__ labels) {
  size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= f.n()) return;
  const uint8_t s = st[n];
  const uint8_t l = s & ST_LABEL;
  labels[n] = l;
  const uint32_t nyz = (uint32_t)f.ny * f.nz;
  const uint32_t a = (uint32_t)(n / nyz);
  const uint32_t r = (uint32_t)(n - (size_t)a * nyz);
  const uint32_t b = r / f.nz;
  const uint32_t k = r - b * f.nz;
  if (a + 1 >= (uint32_t)f.nx || b + 1 >= (uint32_t)f.ny || k + 1 >= (uint32_t)f.nz) return;
  int sum = 0;
  for (int da = 0; da < 2; ++da)
    for (int db = 0; db < 2; ++db) {
      const uint8_t* row = st + (size_t)(a + da) * nyz + (size_t)(b + db) * f.nz + k;
      sum += (row[0] & ST_LABEL) + (row[1] & ST_LABEL);
    }
  if (sum != 0 && sum != 8) st[n] = s | ST_CELL;
}

void launch_cells(uint8_t* st, Lat f, uint8_t* labels, hipStream_t s) {
  hipLaunchKernelGGL(k_cells, dim3(grid1d(f.n(), 256)), dim3(256), 0, s, st, f, labels);
}

__global__ void k_count_bits(const uint8_t* __restrict__ st, size_t n, uint8_t bit,
                             uint32_t* __restrict__ out) {
  // 16 nodes per thread, one atomic per workgroup
  __shared__ uint32_t wsum[COMPACT_BLOCK / 64];
  size_t base = (size_t)blockIdx.x * COMPACT_TILE + (size_t)threadIdx.x * COMPACT_PER_THREAD;
  uint32_t c = __popc(pred_mask16(st, base, n, bit, bit));
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < COMPACT_BLOCK / 64; ++w) t += wsum[w];
    if (t) atomicAdd(out, t);
  }
}

void launch_count_bits(const uint8_t* st, size_t n, uint8_t bit, uint32_t* out, hipStream_t s) {
  if (n)
    hipLaunchKernelGGL(k_count_bits, dim3((unsigned)((n + COMPACT_TILE - 1) / COMPACT_TILE)),
                       dim3(COMPACT_BLOCK), 0, s, st, n, bit, out);
}

}  // namespace pifu
