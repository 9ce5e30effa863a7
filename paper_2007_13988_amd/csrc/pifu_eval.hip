// Point evaluation kernels: point projection (with the optional target->input view
// transform), bilinear feature gather (the sampler of Eq. 1), analytic stand-in
// fields, the MLP output head, the FP64 guard re-evaluation, and the per-ray
// kernels of mesh-free rendering (Sec. 3.2, Eq. 3).
#include "pifu_internal.h"

namespace pifu {

static inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Grid of a list kernel.  With the length known on the host the grid covers the list
// once; with a device-side count (n_dev) the list may be anything up to its capacity n,
// so the grid is bounded and the threads stride over the count.
static inline unsigned list_grid(size_t threads, int block, const uint32_t* n_dev) {
  const unsigned g = grid1d(threads, block);
  return n_dev && g > kStrideBlocks ? kStrideBlocks : g;
}
__device__ inline uint32_t eff_count(uint32_t n, const uint32_t* n_dev) {
  return n_dev ? min(n, *n_dev) : n;
}

// Node or explicit point -> input-view NDC.  Lattice coordinates are exact dyadic
// values; the view product is taken in float64 in a fixed order without fused
// multiply-add so the clip decision is reproducible.  Returns false when the point
// falls outside [-1,1]^3 after the view transform.
__device__ inline bool src_point(const PointSrc& s, const uint32_t* __restrict__ list, uint32_t m,
                                 double P[3], float* occ, int* frame = nullptr) {
  uint32_t idx = (list ? list[m] : m) - s.base_sub;
  if (s.frame_nodes) {
    const uint32_t f = idx / s.frame_nodes;
    idx -= f * s.frame_nodes;
    if (frame) *frame = (int)f;
  }
  if (s.mode == 1) {
    const float4 q = s.pts[idx];
    P[0] = q.x;
    P[1] = q.y;
    P[2] = q.z;
    if (occ) *occ = q.w;
    return true;
  }
  const uint32_t nyz = (uint32_t)s.ny * s.nz;
  const uint32_t a = idx / nyz;
  const uint32_t r = idx - a * nyz;
  const uint32_t b = r / s.nz;
  const uint32_t k = r - b * s.nz;
  double x = __dadd_rn(-1.0, __ddiv_rn(__dmul_rn(2.0, (double)a), (double)(s.nx - 1)));
  double y = __dadd_rn(-1.0, __ddiv_rn(__dmul_rn(2.0, (double)b), (double)(s.ny - 1)));
  double z = __dadd_rn(-1.0, __ddiv_rn(__dmul_rn(2.0, (double)k), (double)(s.nz - 1)));
  if (!s.has_view) {
    P[0] = x;
    P[1] = y;
    P[2] = z;
    return true;
  }
  bool in = true;
#pragma unroll
  for (int r3 = 0; r3 < 3; ++r3) {
    const double* v = s.view + 4 * r3;
    double t = __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn(v[0], x), __dmul_rn(v[1], y)),
                                   __dmul_rn(v[2], z)), v[3]);
    P[r3] = t;
    in = in && (t >= -1.0) && (t <= 1.0);
  }
  return in;
}

__device__ inline void bilinear_setup(double x, double y, int H, int W, int& u0, int& v0,
                                      double w[4]) {
  double u = __dmul_rn(__dmul_rn(__dadd_rn(x, 1.0), 0.5), (double)(W - 1));
  double v = __dmul_rn(__dmul_rn(__dadd_rn(y, 1.0), 0.5), (double)(H - 1));
  double fu0 = floor(u), fv0 = floor(v);
  double fu = u - fu0, fv = v - fv0;
  u0 = (int)fu0;
  v0 = (int)fv0;
  w[0] = (1.0 - fu) * (1.0 - fv);
  w[1] = fu * (1.0 - fv);
  w[2] = (1.0 - fu) * fv;
  w[3] = fu * fv;
}

// ------------------------------------------------------------------ analytic fields
__global__ void k_eval_analytic(PointSrc src, const uint32_t* __restrict__ list, uint32_t n,
                                const uint32_t* __restrict__ n_dev, int kind, Ellipsoids ell0,
                                float4 plane, float* __restrict__ logit, uint8_t* __restrict__ lab,
                                const Ellipsoids* __restrict__ ell_tab) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < ne; m += gridDim.x * blockDim.x) {
  double P[3];
  int frame = 0;
  bool in = src_point(src, list, m, P, nullptr, &frame);
  // multi-frame lists: each frame's shapes from the table
  const Ellipsoids& ell = ell_tab ? ell_tab[frame] : ell0;
  double lg;
  if (!in) {
    lg = -INFINITY;
  } else if (kind == PIFU_FIELD_PLANE) {
    lg = (double)plane.x * P[0] + (double)plane.y * P[1] + (double)plane.z * P[2] + (double)plane.w;
  } else {
    double qmin = INFINITY;
    for (int e = 0; e < ell.n; ++e) {
      const float* E = ell.e + 12 * e;
      double d0 = P[0] - E[0], d1 = P[1] - E[1], d2 = P[2] - E[2];
      double q = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        double t = (double)E[3 + 3 * r] * d0 + (double)E[4 + 3 * r] * d1 + (double)E[5 + 3 * r] * d2;
        q += t * t;
      }
      qmin = q < qmin ? q : qmin;
    }
    lg = (double)ell.k * (1.0 - qmin);
  }
  logit[m] = (float)lg;
  lab[m] = lg > 0.0;
  }
}

void launch_eval_analytic(const PointSrc& src, const uint32_t* list, uint32_t n, int kind,
                          const Ellipsoids& ell, const float plane[4], float* logit, uint8_t* lab,
                          hipStream_t s, const uint32_t* n_dev, const Ellipsoids* ell_tab) {
  if (!n) return;
  float4 pl = make_float4(plane[0], plane[1], plane[2], plane[3]);
  hipLaunchKernelGGL(k_eval_analytic, dim3(list_grid(n, 128, n_dev)), dim3(128), 0, s, src, list,
                     n, n_dev, kind, ell, pl, logit, lab, ell_tab);
}

__global__ void k_store_ellipsoids(Ellipsoids e, Ellipsoids* __restrict__ dst) {
  const int n = (int)(sizeof(Ellipsoids) / 4);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&e);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = src[i];
}

void launch_store_ellipsoids(Ellipsoids* dst, const Ellipsoids& e, hipStream_t s) {
  hipLaunchKernelGGL(k_store_ellipsoids, dim3(1), dim3(256), 0, s, e, dst);
}

// ------------------------------------------------------------------ bilinear gather
// A group of C/4 lanes handles one point; each lane blends 4 channels of the four
// texels (float4 loads from the HWC map) and writes them to row m of feat in format
// FMT (FMT_F16: a value outside the binary16 range sets *ovf).
template <int FMT>
__global__ void __launch_bounds__(256)
k_gather(PointSrc src, const uint32_t* __restrict__ list, uint32_t n,
         const uint32_t* __restrict__ n_dev, const float* __restrict__ F, int H, int W, int C,
         void* __restrict__ feat, float* __restrict__ ext, uint32_t* __restrict__ ovf) {
  const int lanes = C >> 2;
  const int per = lanes < 64 ? lanes : 64;   // lanes per point group (<= one wave)
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x; gid < ne * (uint32_t)per;
       gid += gridDim.x * blockDim.x) {
  const uint32_t m = gid / per;
  const int lane = gid % per;
  double P[3];
  float occ = 0.f;
  int frame = 0;
  const bool in = src_point(src, list, m, P, &occ, &frame);
  if (src.frame_nodes) F = src.feat_tab[frame];
  int u0, v0;
  double w[4];
  bilinear_setup(P[0], P[1], H, W, u0, v0, w);
  const float wf[4] = {(float)w[0], (float)w[1], (float)w[2], (float)w[3]};
  const int tu[4] = {u0, u0 + 1, u0, u0 + 1};
  const int tv[4] = {v0, v0, v0 + 1, v0 + 1};
  for (int c4 = lane; c4 < lanes; c4 += per) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (tu[t] < 0 || tu[t] > W - 1 || tv[t] < 0 || tv[t] > H - 1) continue;
      const float4 q = *reinterpret_cast<const float4*>(F + ((size_t)tv[t] * W + tu[t]) * C + 4 * c4);
      acc.x = fmaf(wf[t], q.x, acc.x);
      acc.y = fmaf(wf[t], q.y, acc.y);
      acc.z = fmaf(wf[t], q.z, acc.z);
      acc.w = fmaf(wf[t], q.w, acc.w);
    }
    if (FMT == FMT_BF16) {
      uint2 o;
      o.x = (uint32_t)f32_to_bf16_bits(acc.x) | ((uint32_t)f32_to_bf16_bits(acc.y) << 16);
      o.y = (uint32_t)f32_to_bf16_bits(acc.z) | ((uint32_t)f32_to_bf16_bits(acc.w) << 16);
      *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(feat) + (size_t)m * C + 4 * c4) = o;
    } else if (FMT == FMT_F16) {
      uint2 o;
      o.x = (uint32_t)f32_to_f16_bits(acc.x) | ((uint32_t)f32_to_f16_bits(acc.y) << 16);
      o.y = (uint32_t)f32_to_f16_bits(acc.z) | ((uint32_t)f32_to_f16_bits(acc.w) << 16);
      *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(feat) + (size_t)m * C + 4 * c4) = o;
      const float big = fmaxf(fmaxf(fabsf(acc.x), fabsf(acc.y)), fmaxf(fabsf(acc.z), fabsf(acc.w)));
      if (!(big <= kF16Max) && ovf) atomicOr(ovf, 1u);
    } else {
      *reinterpret_cast<float4*>(reinterpret_cast<float*>(feat) + (size_t)m * C + 4 * c4) = acc;
    }
  }
  if (lane == 0)
    *reinterpret_cast<float4*>(ext + 4 * (size_t)m) =
        make_float4((float)P[2], occ, in ? 0.f : 1.f, 0.f);
  }
}

void launch_gather(const PointSrc& src, const uint32_t* list, uint32_t n, const float* F, int H,
                   int W, int C, void* feat, int feat_fmt, float* ext, hipStream_t s,
                   const uint32_t* n_dev, uint32_t* ovf) {
  if (!n) return;
  const int lanes = C >> 2;
  const int per = lanes < 64 ? lanes : 64;
  size_t threads = (size_t)n * per;
  const unsigned g = list_grid(threads, 256, n_dev);
  if (feat_fmt == FMT_BF16)
    hipLaunchKernelGGL(k_gather<FMT_BF16>, dim3(g), dim3(256), 0, s, src, list, n, n_dev, F, H, W,
                       C, feat, ext, ovf);
  else if (feat_fmt == FMT_F16)
    hipLaunchKernelGGL(k_gather<FMT_F16>, dim3(g), dim3(256), 0, s, src, list, n, n_dev, F, H, W,
                       C, feat, ext, ovf);
  else
    hipLaunchKernelGGL(k_gather<FMT_F32>, dim3(g), dim3(256), 0, s, src, list, n, n_dev, F, H, W,
                       C, feat, ext, ovf);
}

// ------------------------------------------------------------------ output head
// Sixteen lanes per point (four points per wave): the last linear layer (<= 4 outputs)
// as a dot product over K (a multiple of 64; each lane takes float4 slices 64 apart),
// reduced across the 16 lanes, then the output rule.  n_out == 1: occupancy logit
// (-inf when clipped), label = [logit > 0].  n_out == 3: colour, tanh, written to
// rgb_out[pixel * 3 + c].
__global__ void __launch_bounds__(256)
k_head(const float* __restrict__ h, int K, const float* __restrict__ W, const float* __restrict__ b,
       int n_out, int out_act, uint32_t n, const uint32_t* __restrict__ n_dev,
       const float* __restrict__ ext, float* __restrict__ logit, uint8_t* __restrict__ lab,
       float* __restrict__ rgb_out, const uint32_t* __restrict__ rgb_index) {
  const int q = threadIdx.x & 15;
  const uint32_t ne = eff_count(n, n_dev);
  // whole 16-lane groups take the same points and leave together
  for (uint32_t m = (blockIdx.x * blockDim.x + threadIdx.x) >> 4; m < ne;
       m += (gridDim.x * blockDim.x) >> 4) {
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const float* hr = h + (size_t)m * K;
  for (int k = 4 * q; k < K; k += 64) {
    const float4 x = *reinterpret_cast<const float4*>(hr + k);
    for (int o = 0; o < n_out; ++o) {
      const float4 w = *reinterpret_cast<const float4*>(W + (size_t)o * K + k);
      float a = acc[o];
      a = fmaf(x.x, w.x, a);
      a = fmaf(x.y, w.y, a);
      a = fmaf(x.z, w.z, a);
      a = fmaf(x.w, w.w, a);
      acc[o] = a;
    }
  }
  for (int o = 0; o < n_out; ++o) {
    float v = acc[o];
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    acc[o] = v + b[o];
  }
  if (q != 0) continue;
  if (n_out == 1) {
    float v = acc[0];
    if (ext && ext[4 * (size_t)m + 2] != 0.f) v = -INFINITY;
    logit[m] = v;
    lab[m] = v > 0.f;
  } else {
    const uint32_t pix = rgb_index ? rgb_index[m] : m;
    for (int o = 0; o < n_out; ++o) {
      float v = acc[o];
      if (out_act == PIFU_ACT_TANH) v = tanhf(v);
      else if (out_act == PIFU_ACT_SIGMOID) v = 1.f / (1.f + expf(-v));
      rgb_out[(size_t)pix * n_out + o] = v;
    }
  }
  }
}

void launch_head(const float* h, int K, const float* W, const float* b, int n_out, int out_act,
                 uint32_t n, const float* ext, float* logit, uint8_t* lab, float* rgb_out,
                 const uint32_t* rgb_index, hipStream_t s, const uint32_t* n_dev) {
  if (!n) return;
  hipLaunchKernelGGL(k_head, dim3(list_grid((size_t)n * 16, 256, n_dev)), dim3(256), 0, s, h, K, W,
                     b, n_out, out_act, n, n_dev, ext, logit, lab, rgb_out, rgb_index);
}

// ------------------------------------------------------------------ FP64 guard band
// Appends the positions m < n with |logit[m]| < g (map[m] instead of m when map is
// given); one atomic per wave reserves the wave's slots.  The order of the appended
// positions across waves is unspecified; every consumer treats the points
// independently.
__global__ void k_guard_select(const float* __restrict__ logit, uint32_t n,
                               const uint32_t* __restrict__ n_dev, float g,
                               const uint32_t* __restrict__ map, uint32_t* __restrict__ glist,
                               uint32_t* __restrict__ gcount, uint32_t start) {
  const uint32_t ne = eff_count(n, n_dev);
  // the block's base index is uniform, so every lane of a wave runs the same iterations
  for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < ne; b0 += gridDim.x * blockDim.x) {
    const uint32_t m = b0 + threadIdx.x;
    const bool take = m < ne && fabsf(logit[m]) < g;
    const unsigned long long bal = __ballot(take);
    if (!bal) continue;
    const int lane = threadIdx.x & 63;
    const int first = __ffsll((long long)bal) - 1;
    uint32_t base = 0;
    if (lane == first) base = atomicAdd(gcount, (uint32_t)__popcll(bal));
    base = __shfl(base, first, 64) - start;   // the counter held `start` before this launch
    if (take) {
      const uint32_t slot = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
      glist[slot] = map ? map[m] : m;
    }
  }
}

void launch_guard_select(const float* logit, uint32_t n, float g, uint32_t* glist,
                         uint32_t* gcount, hipStream_t s, const uint32_t* map, uint32_t start,
                         const uint32_t* n_dev) {
  if (!n || !(g > 0.f)) return;
  hipLaunchKernelGGL(k_guard_select, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, logit, n,
                     n_dev, g, map, glist, gcount, start);
}


// ------------------------------------------------------------------ mesh-free rendering
// Level-L interpolation along a pixel column (u, v) of the target lattice, from the
// binarized labels of level L-1: S(kc) sums the labels of the 1/2/4 coarse columns
// around (u, v); even k use S(k/2), odd k the two neighbours.  A fine node is full
// (S = count) where every coarse label involved is 1 and fractional where some but not
// all are.  A workgroup takes a 16 x 16 tile of pixel columns and stages the labels of
// their 9 x 9 coarse columns into LDS as bit masks along z (one wave ballot per 64
// nodes); a ray then works on the AND and OR of its columns' masks:
//   full(2m) = A_m,           nonzero(2m) = O_m,
//   full(2m+1) = A_m A_m+1,   nonzero(2m+1) = O_m | O_m+1.
constexpr int kRayTile = 16;
constexpr int kRayCoarse = kRayTile / 2 + 1;
constexpr int kRayMaxWords = 9;   // coarse columns of up to 576 nodes (depth 2^10)

__host__ __device__ inline int ray_words(int nz) { return (nz + 63) >> 6; }

size_t ray_lds_bytes(Lat c) {
  return (size_t)kRayCoarse * kRayCoarse * ray_words(c.nz) * sizeof(uint64_t);
}

__device__ inline void stage_ray_bits(const uint8_t* __restrict__ stc, Lat c, int cu0, int cv0,
                                      uint64_t* bits) {
  // columns past the lattice edge are staged as 0 (no pixel column reads them)
  const int nw = ray_words(c.nz);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int idx = wave; idx < kRayCoarse * kRayCoarse; idx += nwaves) {
    const int cu = cu0 + idx / kRayCoarse, cv = cv0 + idx % kRayCoarse;
    const bool in = cu < c.nx && cv < c.ny;
    const uint8_t* src = stc + ((size_t)(in ? cu : 0) * c.ny + (in ? cv : 0)) * c.nz;
    for (int q = 0; q < nw; ++q) {
      const int k = 64 * q + lane;
      const bool l = in && k < c.nz && (src[k] & ST_LABEL);
      const uint64_t m = __ballot(l);
      if (lane == 0) bits[idx * nw + q] = m;
    }
  }
  __syncthreads();
}

// The ray of pixel column (u, v): its coarse columns (LDS word offsets) and the AND / OR
// of their label masks.
struct Ray {
  // the up to four coarse columns around the pixel column: (ua, va), (ua, vb), (ub, va),
  // (ub, vb); use[i] says whether column i is a distinct one (every loop below has a
  // fixed trip count, so these arrays and A / O stay in registers)
  int off[4];
  bool use[4];
  int ncol, nw, nzc;
  uint64_t A[kRayMaxWords], O[kRayMaxWords];

  __device__ inline void init(const uint64_t* bits, int nz, int u, int v, int cu0, int cv0) {
    nzc = nz;
    nw = ray_words(nz);
    const int ua = u >> 1, ub = (u + 1) >> 1, va = v >> 1, vb = (v + 1) >> 1;
    off[0] = ((ua - cu0) * kRayCoarse + (va - cv0)) * nw;
    off[1] = ((ua - cu0) * kRayCoarse + (vb - cv0)) * nw;
    off[2] = ((ub - cu0) * kRayCoarse + (va - cv0)) * nw;
    off[3] = ((ub - cu0) * kRayCoarse + (vb - cv0)) * nw;
    use[0] = true;
    use[1] = vb != va;
    use[2] = ub != ua;
    use[3] = ub != ua && vb != va;
    ncol = 1 + (int)use[1] + (int)use[2] + (int)use[3];
#pragma unroll
    for (int q = 0; q < kRayMaxWords; ++q) {
      uint64_t a = ~0ull, o = 0ull;
      if (q < nw) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (use[i]) {
            const uint64_t m = bits[off[i] + q];
            a &= m;
            o |= m;
          }
      } else {
        a = 0ull;
      }
      A[q] = a;
      O[q] = o;
    }
  }
  // bit m of word q of the mask shifted down by one node (m + 1 -> m); q is a constant
  // after unrolling
  __device__ static inline uint64_t next(const uint64_t* X, int q) {
    return (X[q] >> 1) | (q + 1 < kRayMaxWords ? X[q + 1] << 63 : 0ull);
  }
  // odd node 2m + 1 exists for m <= nzc - 2
  __device__ inline uint64_t odd_valid(int q) const {
    const int lim = nzc - 1 - 64 * q;   // bits [0, lim) of word q
    return lim >= 64 ? ~0ull : (lim <= 0 ? 0ull : ((1ull << lim) - 1ull));
  }
  // bits m >= m0 of word q
  __device__ static inline uint64_t from(int m0, int q) {
    const int r = m0 - 64 * q;
    return r <= 0 ? ~0ull : (r >= 64 ? 0ull : ~0ull << r);
  }
  // k* = the node nearest the observer (largest k) that is full, -1 if none
  __device__ inline int kstar() const {
    int ke = -1, ko = -1;
#pragma unroll
    for (int q = kRayMaxWords - 1; q >= 0; --q)
      if (q < nw && ke < 0 && A[q]) ke = 2 * (64 * q + 63 - __clzll(A[q]));
#pragma unroll
    for (int q = kRayMaxWords - 1; q >= 0; --q) {
      const uint64_t aa = A[q] & next(A, q) & odd_valid(q);
      if (q < nw && ko < 0 && aa) ko = 2 * (64 * q + 63 - __clzll(aa)) + 1;
    }
    return ke > ko ? ke : ko;
  }
  // candidates above k (the nodes the network evaluates): nonzero, not full
  __device__ inline uint64_t even_cand(int ks, int q) const {
    return O[q] & from(ks < 0 ? 0 : ks / 2 + 1, q);
  }
  __device__ inline uint64_t odd_cand(int ks, int q) const {
    return (O[q] | next(O, q)) & odd_valid(q) & from(ks < 0 ? 0 : (ks + 1) / 2, q);
  }
  // sum and count of the coarse labels behind fine node k
  __device__ inline void at(const uint64_t* bits, int k, int& sum, int& cnt) const {
    auto S = [&](int kc) {
      int s = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (use[i]) s += (int)((bits[off[i] + (kc >> 6)] >> (kc & 63)) & 1ull);
      return s;
    };
    if (k & 1) {
      sum = S(k >> 1) + S((k >> 1) + 1);
      cnt = 2 * ncol;
    } else {
      sum = S(k >> 1);
      cnt = ncol;
    }
  }
};

// Per column: k* = the node nearest the observer whose interpolated value is 1;
// nodes below it are shadow nodes.  Counts the non-shadow nodes with a fractional
// interpolated value (the ones the network evaluates).
__global__ void __launch_bounds__(256) k_ray_count(const uint8_t* __restrict__ stc, Lat c, int W,
                                                   int H, int D, uint32_t* __restrict__ cnt,
                                                   uint32_t* __restrict__ kstar,
                                                   uint32_t* __restrict__ shadow_total) {
  extern __shared__ uint64_t bits[];
  const int u0 = blockIdx.x * kRayTile, v0 = blockIdx.y * kRayTile;
  stage_ray_bits(stc, c, u0 >> 1, v0 >> 1, bits);
  const int u = u0 + (int)(threadIdx.x >> 4), v = v0 + (int)(threadIdx.x & 15);
  uint32_t shadow = 0;
  if (u < W && v < H) {
    Ray r;
    r.init(bits, c.nz, u, v, u0 >> 1, v0 >> 1);
    const int ks = r.kstar();
    uint32_t n = 0;
#pragma unroll
    for (int q = 0; q < kRayMaxWords; ++q)
      if (q < r.nw) n += (uint32_t)(__popcll(r.even_cand(ks, q)) + __popcll(r.odd_cand(ks, q)));
    const uint32_t col = (uint32_t)u * H + v;
    cnt[col] = n;
    kstar[col] = (uint32_t)ks;
    shadow = ks > 0 ? (uint32_t)ks : 0u;
  }
  for (int d = 32; d >= 1; d >>= 1) shadow += __shfl_xor(shadow, d, 64);
  if ((threadIdx.x & 63) == 0 && shadow) atomicAdd(shadow_total, shadow);
}

dim3 ray_grid(int W, int H) {
  return dim3((unsigned)((W + kRayTile - 1) / kRayTile), (unsigned)((H + kRayTile - 1) / kRayTile));
}

void launch_ray_count(const uint8_t* stc, Lat c, int W, int H, int D, uint32_t* cnt,
                      uint32_t* kstar, uint32_t* shadow_total, hipStream_t s) {
  hipLaunchKernelGGL(k_ray_count, ray_grid(W, H), dim3(kRayTile * kRayTile), ray_lds_bytes(c), s,
                     stc, c, W, H, D, cnt, kstar, shadow_total);
}

// Writes the level-L lattice indices of each column's candidates in increasing k.
__global__ void __launch_bounds__(256) k_ray_list(const uint8_t* __restrict__ stc, Lat c, int W,
                                                  int H, int D, const uint32_t* __restrict__ kstar,
                                                  const uint32_t* __restrict__ off,
                                                  uint32_t* __restrict__ list) {
  extern __shared__ uint64_t bits[];
  const int u0 = blockIdx.x * kRayTile, v0 = blockIdx.y * kRayTile;
  stage_ray_bits(stc, c, u0 >> 1, v0 >> 1, bits);
  const int u = u0 + (int)(threadIdx.x >> 4), v = v0 + (int)(threadIdx.x & 15);
  if (u >= W || v >= H) return;
  const uint32_t col = (uint32_t)u * H + v;
  Ray r;
  r.init(bits, c.nz, u, v, u0 >> 1, v0 >> 1);
  const int ks = (int)kstar[col];
  uint32_t pos = off[col];
  const size_t base = ((size_t)u * (H + 1) + v) * (size_t)(D + 1);
  // the candidate words first (fixed trip count: the Ray stays in registers), then the
  // bit walk over them
  uint64_t evw[kRayMaxWords], odw[kRayMaxWords];
#pragma unroll
  for (int q = 0; q < kRayMaxWords; ++q) {
    evw[q] = q < r.nw ? r.even_cand(ks, q) : 0ull;
    odw[q] = q < r.nw ? r.odd_cand(ks, q) : 0ull;
  }
#pragma unroll
  for (int q = 0; q < kRayMaxWords; ++q) {
    const uint64_t ev = evw[q], od = odw[q];
    uint64_t any = ev | od;
    while (any) {
      const int bit = __ffsll((unsigned long long)any) - 1;
      any &= any - 1ull;
      const int m = 64 * q + bit;
      if ((ev >> bit) & 1ull) list[pos++] = (uint32_t)(base + 2 * m);
      if ((od >> bit) & 1ull) list[pos++] = (uint32_t)(base + 2 * m + 1);
    }
  }
}

void launch_ray_list(const uint8_t* stc, Lat c, int W, int H, int D, const uint32_t* kstar,
                     const uint32_t* off, uint32_t* list, hipStream_t s) {
  hipLaunchKernelGGL(k_ray_list, ray_grid(W, H), dim3(kRayTile * kRayTile), ray_lds_bytes(c), s,
                     stc, c, W, H, D, kstar, off, list);
}

// Second argmax after evaluation: k1 = the node nearest the observer labelled inside,
// i.e. the highest evaluated candidate labelled inside, else k*; the surface point is
// the 0.5 crossing of the occupancy values of k1 and k1 + 1.
__global__ void __launch_bounds__(256) k_ray_hit(
    const uint8_t* __restrict__ stc, const float* __restrict__ occc, Lat c, int W, int H, int D,
    const uint32_t* __restrict__ off, const uint32_t* __restrict__ cnt,
    const uint32_t* __restrict__ list, const float* __restrict__ logit,
    const uint8_t* __restrict__ lab, float* __restrict__ depth, uint8_t* __restrict__ hit,
    float4* __restrict__ hitpts, double4 v0, double4 v1, double4 v2, int32_t* __restrict__ kstar_out,
    int32_t* __restrict__ k1_out) {
  extern __shared__ uint64_t bits[];
  const int u0 = blockIdx.x * kRayTile, vt0 = blockIdx.y * kRayTile;
  const int cu0 = u0 >> 1, cv0 = vt0 >> 1;
  stage_ray_bits(stc, c, cu0, cv0, bits);
  const int u = u0 + (int)(threadIdx.x >> 4), v = vt0 + (int)(threadIdx.x & 15);
  if (u >= W || v >= H) return;
  const uint32_t col = (uint32_t)u * H + v;
  Ray r;
  r.init(bits, c.nz, u, v, cu0, cv0);
  const bool even_col = !((u | v) & 1);
  const uint32_t base = ((uint32_t)u * (H + 1) + v) * (uint32_t)(D + 1);
  const int jmin = (int)off[col], jend = (int)off[col] + (int)cnt[col] - 1;
  int k1 = -1, j1 = -1;
  for (int j = jend; j >= jmin; --j)
    if (lab[j]) {
      k1 = (int)(list[j] - base);
      j1 = j;
      break;
    }
  const uint32_t pixel = (uint32_t)v * W + u;
  if (kstar_out) kstar_out[pixel] = r.kstar();
  if (k1 < 0) k1 = r.kstar();
  if (k1_out) k1_out[pixel] = k1;
  if (k1 < 0) return;
  // node k1 + 1, when evaluated, is the list entry after k1's (or the first entry)
  const int jn = j1 >= 0 ? j1 + 1 : jmin;
  const int jprev = (k1 < D && jn <= jend && list[jn] == base + (uint32_t)(k1 + 1)) ? jn : -1;
  // occupancy of node k of this column: a coarse node's stored value, an evaluated
  // node's sigmoid, else the interpolated fraction
  auto value = [&](int k, int jk) -> float {
    if (even_col && !(k & 1)) return occc[((size_t)(u >> 1) * c.ny + (v >> 1)) * c.nz + (k >> 1)];
    if (jk >= 0) return 1.0f / (1.0f + expf(-logit[jk]));
    int s, t;
    r.at(bits, k, s, t);
    return (float)s / (float)t;
  };
  const float ob = value(k1, j1);
  const float of = k1 < D ? value(k1 + 1, jprev) : 0.f;
  const uint32_t pix = pixel;
  double z;
  if (k1 == D) {
    z = 1.0;
  } else {
    const double t = (ob - of > 0.f) ? (0.5 - (double)of) / ((double)ob - (double)of) : 0.0;
    const double zf = -1.0 + 2.0 * (double)(k1 + 1) / D;
    const double zb = -1.0 + 2.0 * (double)k1 / D;
    z = zf + t * (zb - zf);
  }
  depth[pix] = (float)z;
  hit[pix] = 1;
  const double x = -1.0 + 2.0 * (double)u / W;
  const double y = -1.0 + 2.0 * (double)v / H;
  hitpts[pix] = make_float4((float)(v0.x * x + v0.y * y + v0.z * z + v0.w),
                            (float)(v1.x * x + v1.y * y + v1.z * z + v1.w),
                            (float)(v2.x * x + v2.y * y + v2.z * z + v2.w), ob);
}

void launch_ray_hit(const uint8_t* stc, const float* occc, Lat c, int W, int H, int D,
                    const uint32_t* off, const uint32_t* cnt, const uint32_t* list,
                    const float* logit, const uint8_t* lab, const double* view, float* depth,
                    uint8_t* hit, float4* hitpts, hipStream_t s, int32_t* kstar_out,
                    int32_t* k1_out) {
  double4 v0 = make_double4(view[0], view[1], view[2], view[3]);
  double4 v1 = make_double4(view[4], view[5], view[6], view[7]);
  double4 v2 = make_double4(view[8], view[9], view[10], view[11]);
  hipLaunchKernelGGL(k_ray_hit, ray_grid(W, H), dim3(kRayTile * kRayTile), ray_lds_bytes(c), s, stc,
                     occc, c, W, H, D, off, cnt, list, logit, lab, depth, hit, hitpts, v0, v1, v2,
                     kstar_out, k1_out);
}

__global__ void k_trace_scatter(const uint32_t* __restrict__ list, uint32_t n,
                                const uint32_t* __restrict__ n_dev, const float* __restrict__ logit,
                                int level_id, uint8_t* __restrict__ eval_level,
                                float* __restrict__ eval_logit) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < ne; m += gridDim.x * blockDim.x) {
    const uint32_t node = list[m];
    if (eval_level) eval_level[node] = (uint8_t)level_id;
    if (eval_logit) eval_logit[node] = logit[m];
  }
}

void launch_trace_scatter(const uint32_t* list, uint32_t n, const float* logit, int level_id,
                          uint8_t* eval_level, float* eval_logit, hipStream_t s,
                          const uint32_t* n_dev) {
  if (!n || (!eval_level && !eval_logit)) return;
  hipLaunchKernelGGL(k_trace_scatter, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, list, n,
                     n_dev, logit, level_id, eval_level, eval_logit);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

__global__ void k_fill_image(float* __restrict__ rgb, float* __restrict__ depth,
                             uint8_t* __restrict__ hit, uint32_t npix, float bg0, float bg1,
                             float bg2) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  rgb[3 * (size_t)p + 0] = bg0;
  rgb[3 * (size_t)p + 1] = bg1;
  rgb[3 * (size_t)p + 2] = bg2;
  depth[p] = __int_as_float(0x7fc00000);
  hit[p] = 0;
}

void launch_fill_image(float* rgb, float* depth, uint8_t* hit, uint32_t npix, float bg0, float bg1,
                       float bg2, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_image, dim3(grid1d(npix, 256)), dim3(256), 0, s, rgb, depth, hit, npix,
                     bg0, bg1, bg2);
}

}  // namespace pifu

namespace pifu {

__global__ void k_gather_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ pos,
                             uint32_t n, const uint32_t* __restrict__ n_dev,
                             uint32_t* __restrict__ out) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += gridDim.x * blockDim.x)
    out[i] = src[pos[i]];
}

void launch_gather_u32(const uint32_t* src, const uint32_t* pos, uint32_t n, uint32_t* out,
                       hipStream_t s, const uint32_t* n_dev) {
  if (n)
    hipLaunchKernelGGL(k_gather_u32, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, src, pos, n,
                       n_dev, out);
}

__global__ void k_scatter_results(const uint32_t* __restrict__ pos, uint32_t n,
                                  const uint32_t* __restrict__ n_dev,
                                  const float* __restrict__ tl, const uint8_t* __restrict__ tb,
                                  float* __restrict__ logit, uint8_t* __restrict__ lab) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += gridDim.x * blockDim.x) {
    const uint32_t p = pos[i];
    logit[p] = tl[i];
    lab[p] = tb[i];
  }
}

// ------------------------------------------------------------------ per-column hoisting
// In the input view the sampled feature depends only on the (x, y) column of a node,
// so the feature part of every layer (W_f f + b) is computed once per column run.
__global__ void k_col_flags(const uint32_t* __restrict__ list, uint32_t n,
                            const uint32_t* __restrict__ n_dev, uint32_t nz,
                            uint32_t* __restrict__ flags) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += gridDim.x * blockDim.x)
    flags[i] = (i == 0) || (list[i] / nz != list[i - 1] / nz);
}

void launch_col_flags(const uint32_t* list, uint32_t n, uint32_t nz, uint32_t* flags,
                      hipStream_t s, const uint32_t* n_dev) {
  if (n)
    hipLaunchKernelGGL(k_col_flags, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, list, n, n_dev,
                       nz, flags);
}

__global__ void k_col_ids(const uint32_t* __restrict__ list, const uint32_t* __restrict__ flags,
                          const uint32_t* __restrict__ excl, uint32_t n,
                          const uint32_t* __restrict__ n_dev, uint32_t* __restrict__ cid,
                          uint32_t* __restrict__ col_node) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += gridDim.x * blockDim.x) {
    const uint32_t c = excl[i] + flags[i] - 1;
    cid[i] = c;
    if (flags[i]) col_node[c] = list[i];
  }
}

void launch_col_ids(const uint32_t* list, const uint32_t* flags, const uint32_t* excl, uint32_t n,
                    uint32_t* cid, uint32_t* col_node, hipStream_t s, const uint32_t* n_dev) {
  if (n)
    hipLaunchKernelGGL(k_col_ids, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, list, flags,
                       excl, n, n_dev, cid, col_node);
}

__global__ void k_hoist_layer0(const float* __restrict__ P, int ldp, const uint32_t* __restrict__ cid,
                               const uint32_t* __restrict__ list, uint32_t n,
                               const uint32_t* __restrict__ n_dev, int nz,
                               const float* __restrict__ wz, int N, int act,
                               void* __restrict__ h, int h_fmt, uint32_t* __restrict__ ovf) {
  // four consecutive outputs per thread (N % 4 == 0, ldp % 4 == 0; n * N / 4 < 2^32)
  const uint32_t n4 = (uint32_t)N >> 2;
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < ne * n4;
       e += gridDim.x * blockDim.x) {
  const uint32_t i = e / n4;
  const uint32_t o = (e - i * n4) << 2;
  const uint32_t k = list[i] % (uint32_t)nz;
  const float z = (float)(-1.0 + 2.0 * (double)k / (double)(nz - 1));
  const float4 p = *reinterpret_cast<const float4*>(P + (size_t)cid[i] * ldp + o);
  const float4 w = *reinterpret_cast<const float4*>(wz + o);
  float v[4] = {fmaf(z, w.x, p.x), fmaf(z, w.y, p.y), fmaf(z, w.z, p.z), fmaf(z, w.w, p.w)};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (act == PIFU_ACT_RELU) v[q] = v[q] > 0.f ? v[q] : 0.f;
    else if (act == PIFU_ACT_LRELU) v[q] = v[q] > 0.f ? v[q] : 0.01f * v[q];
  }
  const size_t at = (size_t)i * N + o;
  if (h_fmt == FMT_BF16) {
    uint2 u;
    u.x = (uint32_t)f32_to_bf16_bits(v[0]) | ((uint32_t)f32_to_bf16_bits(v[1]) << 16);
    u.y = (uint32_t)f32_to_bf16_bits(v[2]) | ((uint32_t)f32_to_bf16_bits(v[3]) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(h) + at) = u;
  } else if (h_fmt == FMT_F16) {
    uint2 u;
    u.x = (uint32_t)f32_to_f16_bits(v[0]) | ((uint32_t)f32_to_f16_bits(v[1]) << 16);
    u.y = (uint32_t)f32_to_f16_bits(v[2]) | ((uint32_t)f32_to_f16_bits(v[3]) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(h) + at) = u;
    const float big = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
    if (!(big <= kF16Max) && ovf) atomicOr(ovf, 1u);
  } else {
    *reinterpret_cast<float4*>(reinterpret_cast<float*>(h) + at) = make_float4(v[0], v[1], v[2], v[3]);
  }
  }
}

void launch_hoist_layer0(const float* P, int ldp, const uint32_t* cid, const uint32_t* list,
                         uint32_t n, int nz, const float* wz, int N, int act, void* h, int h_fmt,
                         hipStream_t s, uint32_t* ovf, const uint32_t* n_dev) {
  const size_t tot = (size_t)n * (N >> 2);
  if (tot)
    hipLaunchKernelGGL(k_hoist_layer0, dim3(list_grid(tot, 256, n_dev)), dim3(256), 0, s, P, ldp,
                       cid, list, n, n_dev, nz, wz, N, act, h, h_fmt, ovf);
}

// ------------------------------------------------------------------ per-texel hoisting
// Every layer that reads the sampled feature f is linear in f before its activation, and
// f is the bilinear blend of four texels, so W_f f = sum_t w_t (W_f F[texel_t]): the
// products W_f F of all texels are computed once per call (a GEMM over the feature map)
// and each point blends four rows of them.  This holds for any point, in any view.
__global__ void k_taps(PointSrc src, const uint32_t* __restrict__ list, uint32_t n,
                       const uint32_t* __restrict__ n_dev, int H, int W, int4* __restrict__ tidx,
                       float4* __restrict__ tw, float* __restrict__ ext) {
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < ne; m += gridDim.x * blockDim.x) {
    double P[3];
    float occ = 0.f;
    const bool in = src_point(src, list, m, P, &occ);
    int u0, v0;
    double w[4];
    bilinear_setup(P[0], P[1], H, W, u0, v0, w);
    const int tu[4] = {u0, u0 + 1, u0, u0 + 1};
    const int tv[4] = {v0, v0, v0 + 1, v0 + 1};
    int id[4];
    float wf[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool ok = tu[t] >= 0 && tu[t] <= W - 1 && tv[t] >= 0 && tv[t] <= H - 1;
      id[t] = ok ? tv[t] * W + tu[t] : 0;
      wf[t] = ok ? (float)w[t] : 0.f;
    }
    tidx[m] = make_int4(id[0], id[1], id[2], id[3]);
    tw[m] = make_float4(wf[0], wf[1], wf[2], wf[3]);
    *reinterpret_cast<float4*>(ext + 4 * (size_t)m) = make_float4((float)P[2], occ, in ? 0.f : 1.f, 0.f);
  }
}

void launch_taps(const PointSrc& src, const uint32_t* list, uint32_t n, int H, int W, int4* tidx,
                 float4* tw, float* ext, hipStream_t s, const uint32_t* n_dev) {
  if (n)
    hipLaunchKernelGGL(k_taps, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, src, list, n,
                       n_dev, H, W, tidx, tw, ext);
}

__global__ void k_taps_layer0(const float* __restrict__ T, int ldt, const int4* __restrict__ tidx,
                              const float4* __restrict__ tw, const float* __restrict__ ext,
                              uint32_t n, const uint32_t* __restrict__ n_dev,
                              const float* __restrict__ bias, const float* __restrict__ wz, int N,
                              int act, float* __restrict__ h) {
  // four consecutive outputs per thread (N % 4 == 0, ldt % 4 == 0)
  const uint32_t n4 = (uint32_t)N >> 2;
  const uint32_t ne = eff_count(n, n_dev);
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < ne * n4;
       e += gridDim.x * blockDim.x) {
    const uint32_t i = e / n4;
    const uint32_t o = (e - i * n4) << 2;
    const int4 id = tidx[i];
    const float4 w = tw[i];
    const float z = ext[4 * (size_t)i];
    const int ids[4] = {id.x, id.y, id.z, id.w};
    const float ws[4] = {w.x, w.y, w.z, w.w};
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float4 p = *reinterpret_cast<const float4*>(T + (size_t)ids[t] * ldt + o);
      acc.x = fmaf(ws[t], p.x, acc.x);
      acc.y = fmaf(ws[t], p.y, acc.y);
      acc.z = fmaf(ws[t], p.z, acc.z);
      acc.w = fmaf(ws[t], p.w, acc.w);
    }
    const float4 b = *reinterpret_cast<const float4*>(bias + o);
    const float4 wzv = *reinterpret_cast<const float4*>(wz + o);
    float v[4] = {fmaf(z, wzv.x, acc.x + b.x), fmaf(z, wzv.y, acc.y + b.y),
                  fmaf(z, wzv.z, acc.z + b.z), fmaf(z, wzv.w, acc.w + b.w)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (act == PIFU_ACT_RELU) v[q] = v[q] > 0.f ? v[q] : 0.f;
      else if (act == PIFU_ACT_LRELU) v[q] = v[q] > 0.f ? v[q] : 0.01f * v[q];
    }
    *reinterpret_cast<float4*>(h + (size_t)i * N + o) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

void launch_taps_layer0(const float* T, int ldt, const int4* tidx, const float4* tw,
                        const float* ext, uint32_t n, const float* bias, const float* wz, int N,
                        int act, float* h, hipStream_t s, const uint32_t* n_dev) {
  const size_t tot = (size_t)n * (N >> 2);
  if (tot)
    hipLaunchKernelGGL(k_taps_layer0, dim3(list_grid(tot, 256, n_dev)), dim3(256), 0, s, T, ldt,
                       tidx, tw, ext, n, n_dev, bias, wz, N, act, h);
}

// The library's number-format conversions applied to an array (for checking them).
__global__ void k_convert(const float* __restrict__ in, uint32_t n, int fmt, void* __restrict__ out) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (fmt == PIFU_PREC_BF16) reinterpret_cast<uint16_t*>(out)[i] = f32_to_bf16_bits(in[i]);
  else if (fmt == PIFU_PREC_FP16) reinterpret_cast<uint16_t*>(out)[i] = f32_to_f16_bits(in[i]);
  else reinterpret_cast<uint8_t*>(out)[i] = f32_to_e4m3(in[i]);
}

void launch_convert(const float* in, uint32_t n, int fmt, void* out, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_convert, dim3(grid1d(n, 256)), dim3(256), 0, s, in, n, fmt, out);
}

void launch_scatter_results(const uint32_t* pos, uint32_t n, const float* tl, const uint8_t* tb,
                            float* logit, uint8_t* lab, hipStream_t s, const uint32_t* n_dev) {
  if (n)
    hipLaunchKernelGGL(k_scatter_results, dim3(list_grid(n, 256, n_dev)), dim3(256), 0, s, pos, n,
                       n_dev, tl, tb, logit, lab);
}

}  // namespace pifu
