// Float64 re-evaluation of the points whose FP32 logit lies in the guard band
// |logit| < g, so that the binary label [logit > 0] is decided in float64.  The
// guarded points are batched: float64 gather, float64 MFMA GEMMs per hidden layer,
// float64 head -- the same network as the FP32 path, evaluated in double precision.
#include <algorithm>

#include "pifu_internal.h"

namespace pifu {

typedef double f64x4 __attribute__((ext_vector_type(4)));

static inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

__device__ inline bool src_point64(const PointSrc& s, uint32_t idx, double P[3], double* occ,
                                   int* frame = nullptr) {
  idx -= s.base_sub;
  if (s.frame_nodes) {   // an index into frames of frame_nodes nodes stored back to back
    const uint32_t f = idx / s.frame_nodes;
    idx -= f * s.frame_nodes;
    if (frame) *frame = (int)f;
  }
  if (s.mode == 1) {
    const float4 q = s.pts[idx];
    P[0] = q.x;
    P[1] = q.y;
    P[2] = q.z;
    *occ = q.w;
    return true;
  }
  *occ = 0.0;
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

// Node list of the guarded points: gnode[i] = list[glist[i]].
__global__ void k_guard_nodes(const uint32_t* __restrict__ list, const uint32_t* __restrict__ glist,
                              uint32_t gn, const uint32_t* __restrict__ gn_dev,
                              uint32_t* __restrict__ gnode) {
  if (gn_dev) gn = min(gn, *gn_dev);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
    gnode[i] = list ? list[glist[i]] : glist[i];
}

// One wave per point: float64 bilinear blend of C channels; ext64 = (z', occ, clipped, 0).
__global__ void __launch_bounds__(256)
k_gather64(PointSrc src, const uint32_t* __restrict__ nodes, uint32_t n,
           const uint32_t* __restrict__ n_dev, const float* __restrict__ F, int H, int W, int C,
           double* __restrict__ feat, double* __restrict__ ext) {
  const int lane = threadIdx.x & 63;
  if (n_dev) n = min(n, *n_dev);
  const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t m = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; m < n; m += waves) {
  double P[3], occ;
  int frame = 0;
  const bool in = src_point64(src, nodes[m], P, &occ, &frame);
  const float* __restrict__ Fm = src.frame_nodes ? src.feat_tab[frame] : F;
  double u = __dmul_rn(__dmul_rn(__dadd_rn(P[0], 1.0), 0.5), (double)(W - 1));
  double v = __dmul_rn(__dmul_rn(__dadd_rn(P[1], 1.0), 0.5), (double)(H - 1));
  const double fu0 = floor(u), fv0 = floor(v);
  const double fu = u - fu0, fv = v - fv0;
  const int u0 = (int)fu0, v0 = (int)fv0;
  const double w[4] = {(1.0 - fu) * (1.0 - fv), fu * (1.0 - fv), (1.0 - fu) * fv, fu * fv};
  const int tu[4] = {u0, u0 + 1, u0, u0 + 1};
  const int tv[4] = {v0, v0, v0 + 1, v0 + 1};
  for (int c = lane; c < C; c += 64) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (tu[t] < 0 || tu[t] > W - 1 || tv[t] < 0 || tv[t] > H - 1) continue;
      acc += w[t] * (double)Fm[((size_t)tv[t] * W + tu[t]) * C + c];
    }
    feat[(size_t)m * C + c] = acc;
  }
  if (lane == 0) {
    double* e = ext + 4 * (size_t)m;
    e[0] = P[2];
    e[1] = occ;
    e[2] = in ? 0.0 : 1.0;
    e[3] = 0.0;
  }
  }
}

// Dense float64 operand copy of the first K columns of a [N][ldw_src] fp32 matrix.
__global__ void k_pack64(const float* __restrict__ W, int N, int ldw_src, int K,
                         double* __restrict__ dst) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)N * K) return;
  const int n = (int)(i / K), k = (int)(i - (size_t)n * K);
  dst[i] = (double)W[(size_t)n * ldw_src + k];
}

struct Gemm64Args {
  const double* A1;
  int K1, lda1;
  const double* A2;
  int K2, lda2;
  const double* W;   // [N][K1 + K2]
  const float* Wf;   // original fp32 weights (extras columns)
  int ldwf;
  const float* bias;
  const double* ext;
  int n_ext, ext_col;
  double* C;
  int M, N, act;
  const uint32_t* M_dev;   // device-side row count (nullable): rows = min(M, *M_dev)
};

// One 16 x 16 output tile per workgroup (v_mfma_f64_16x16x4f64).  The guard band
// holds few points, so the tile is small (many workgroups) and the kGuardWaves waves
// split the contraction: wave q sums the q-th share of the 16-wide k steps, and the
// partial tiles are added in wave order through LDS, so every output is the same
// fixed-order sum whatever the number of points.  A launch is a chain of dependent
// loads and MFMAs per wave; eight waves keep that chain short.  Lane group g = lane/16 feeds the
// k values {4g .. 4g+3} of each 16-wide step (s-th MFMA: k = 4g + s; same
// permutation for A and B).  Output layout (checked on gfx950 with a lane probe):
// lane l, register r holds row 4*r + l/16, column l%16.
constexpr int kGuardWaves = 8;

__global__ void __launch_bounds__(64 * kGuardWaves) k_gemm64(Gemm64Args a) {
  __shared__ double red[kGuardWaves - 1][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = blockIdx.y * 16;
  const int K = a.K1 + a.K2;
  const int M = a.M_dev ? min(a.M, (int)*a.M_dev) : a.M;
  const int g = lane >> 4, r16 = lane & 15;
  const double* wrow = a.W + (size_t)(n0 + r16) * K;
  const int nst = K >> 4;
  const int s0 = nst * wave / kGuardWaves, s1 = nst * (wave + 1) / kGuardWaves;
  // row tiles in turn (a fixed grid covers any device-side count)
  for (int m0 = blockIdx.x * 16; m0 < M; m0 += gridDim.x * 16) {
    const int arow = m0 + r16;
    const bool arow_ok = arow < M;
    f64x4 acc = (f64x4){0.0, 0.0, 0.0, 0.0};
    for (int st = s0; st < s1; ++st) {
      const int k = st * 16 + 4 * g;
      double2 a01 = make_double2(0.0, 0.0), a23 = make_double2(0.0, 0.0);
      if (arow_ok) {
        const double* ap = k < a.K1 ? a.A1 + (size_t)arow * a.lda1 + k
                                    : a.A2 + (size_t)arow * a.lda2 + (k - a.K1);
        a01 = *reinterpret_cast<const double2*>(ap);
        a23 = *reinterpret_cast<const double2*>(ap + 2);
      }
      const double2 b01 = *reinterpret_cast<const double2*>(wrow + k);
      const double2 b23 = *reinterpret_cast<const double2*>(wrow + k + 2);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.x, b01.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.y, b01.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.x, b23.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.y, b23.y, acc, 0, 0, 0);
    }
    if (wave) {
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave - 1][r][lane] = acc[r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < kGuardWaves - 1; ++q) acc[r] += red[q][r][lane];   // wave order
      const int col = n0 + r16;
      const double bias = a.bias[col];
      double we0 = 0.0, we1 = 0.0;
      if (a.n_ext > 0) we0 = a.Wf[(size_t)col * a.ldwf + a.ext_col];
      if (a.n_ext > 1) we1 = a.Wf[(size_t)col * a.ldwf + a.ext_col + 1];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + 4 * r + g;
        if (row >= M) continue;
        double v = acc[r] + bias;
        if (a.n_ext > 0) v += a.ext[4 * (size_t)row] * we0;
        if (a.n_ext > 1) v += a.ext[4 * (size_t)row + 1] * we1;
        if (a.act == PIFU_ACT_RELU) v = v > 0.0 ? v : 0.0;
        else if (a.act == PIFU_ACT_LRELU) v = v > 0.0 ? v : 0.01 * v;
        a.C[(size_t)row * a.N + col] = v;
      }
    }
    __syncthreads();   // red is reused by the next row tile
  }
}

// One wave per point: last layer in float64, then scatter to the guarded positions.
__global__ void __launch_bounds__(256)
k_head64(const double* __restrict__ h, int K, const float* __restrict__ W,
         const float* __restrict__ b, uint32_t n, const uint32_t* __restrict__ n_dev,
         const double* __restrict__ ext, const uint32_t* __restrict__ glist,
         float* __restrict__ logit, uint8_t* __restrict__ lab) {
  const int lane = threadIdx.x & 63;
  if (n_dev) n = min(n, *n_dev);
  const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t m = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; m < n; m += waves) {
    double acc = 0.0;
    for (int k = lane; k < K; k += 64) acc += h[(size_t)m * K + k] * (double)W[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) {
      double v = acc + (double)b[0];
      if (ext[4 * (size_t)m + 2] != 0.0) v = -INFINITY;
      const uint32_t pos = glist[m];
      logit[pos] = (float)v;
      lab[pos] = v > 0.0;
    }
  }
}

size_t guard64_ws_bytes(const MLPDesc& d, uint32_t chunk) {
  size_t w = 0;
  int maxw = 1;
  for (int l = 0; l + 1 < d.n_layers; ++l) {
    const int Kp = l == 0 ? d.feat_dim : d.in_w[l];
    w += (size_t)d.widths[l] * Kp;
    maxw = d.widths[l] > maxw ? d.widths[l] : maxw;
  }
  const size_t elems = w + (size_t)chunk * (d.feat_dim + 4 + 2 * maxw) + 64;
  return elems * sizeof(double) + (size_t)chunk * 4 + 4096;
}

// Re-evaluates the gn guarded points (positions glist into the evaluated list) in
// float64 and overwrites their logit and label.  ws holds guard64_ws_bytes(d, chunk).
void run_guard64(const PointSrc& src, const uint32_t* list, const uint32_t* glist, uint32_t gn,
                 const MLPDesc& d, const float* F, int H, int W, int C, float* logit, uint8_t* lab,
                 void* ws, uint32_t chunk, bool pack, hipStream_t s, const uint32_t* gn_dev) {
  if (!gn) return;
  // with a device-side count the list holds at most one chunk (gn is its capacity)
  if (gn_dev && gn > chunk) gn = chunk;
  const uint32_t max_waves = 2048;
  double* base = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  double* Wp[PIFU_MAX_LAYERS];
  int maxw = 1;
  for (int l = 0; l + 1 < d.n_layers; ++l) {
    const int Kp = l == 0 ? d.feat_dim : d.in_w[l];
    Wp[l] = base;
    base += (size_t)d.widths[l] * Kp;
    if (pack)   // the float64 weight copies persist in ws for the rest of the call
      hipLaunchKernelGGL(k_pack64, dim3(grid1d((size_t)d.widths[l] * Kp, 256)), dim3(256), 0, s,
                         d.W[l], d.widths[l], d.in_w[l], Kp, Wp[l]);
    maxw = d.widths[l] > maxw ? d.widths[l] : maxw;
  }
  double* feat = base;
  base += (size_t)chunk * C;
  double* ext = base;
  base += (size_t)chunk * 4;
  double* hA = base;
  base += (size_t)chunk * maxw;
  double* hB = base;
  base += (size_t)chunk * maxw;
  uint32_t* gnode = reinterpret_cast<uint32_t*>(base);
  for (uint32_t c0 = 0; c0 < gn; c0 += chunk) {
    const uint32_t m = gn - c0 < chunk ? gn - c0 : chunk;
    hipLaunchKernelGGL(k_guard_nodes, dim3(std::min(grid1d(m, 256), kStrideBlocks)), dim3(256), 0,
                       s, list, glist + c0, m, gn_dev, gnode);
    const uint32_t pw = std::min(m, max_waves);   // point-per-wave kernels: waves in the grid
    hipLaunchKernelGGL(k_gather64, dim3(grid1d((size_t)pw * 64, 256)), dim3(256), 0, s, src, gnode,
                       m, gn_dev, F, H, W, C, feat, ext);
    const double* prev = nullptr;
    double* out = hA;
    for (int l = 0; l + 1 < d.n_layers; ++l) {
      Gemm64Args g = {};
      if (l == 0) {
        g.A1 = feat;
        g.K1 = C;
        g.lda1 = C;
        g.n_ext = d.n_extra;
        g.ext_col = C;
      } else {
        g.A1 = prev;
        g.K1 = d.widths[l - 1];
        g.lda1 = d.widths[l - 1];
        if (d.skip[l]) {
          g.A2 = feat;
          g.K2 = C;
          g.lda2 = C;
        }
      }
      g.W = Wp[l];
      g.Wf = d.W[l];
      g.ldwf = d.in_w[l];
      g.bias = d.b[l];
      g.ext = ext;
      g.C = out;
      g.M = (int)m;
      g.N = d.widths[l];
      g.act = d.hidden_act;
      g.M_dev = gn_dev;
      hipLaunchKernelGGL(k_gemm64, dim3(std::min<uint32_t>((m + 15) / 16, 64), d.widths[l] / 16),
                         dim3(64 * kGuardWaves), 0, s, g);
      prev = out;
      out = out == hA ? hB : hA;
    }
    const int L = d.n_layers - 1;
    hipLaunchKernelGGL(k_head64, dim3(grid1d((size_t)pw * 64, 256)), dim3(256), 0, s, prev,
                       d.widths[L - 1], d.W[L], d.b[L], m, gn_dev, ext, glist + c0, logit, lab);
  }
}

// ------------------------------------------------------------------ CBN network guard
// One workgroup per guarded point evaluates the conditional-batch-norm network in float64
// (the FP32 path's arithmetic, in double): gamma / beta of every block from the point's
// float64 feature, the soft one-hot layer, the blocks and the head.
constexpr int kCbnThreads = 256;

__global__ void __launch_bounds__(kCbnThreads)
k_cbn64(CbnDesc d, const double* __restrict__ feat, const double* __restrict__ ext, uint32_t gn,
        const uint32_t* __restrict__ glist, float* __restrict__ logit, uint8_t* __restrict__ lab) {
  extern __shared__ double sh[];
  double* f = sh;                                  // C
  double* gb = f + d.C;                            // 2 nb width
  double* h = gb + 2 * (size_t)d.nb * d.width;     // width
  double* a = h + d.width;                         // width
  __shared__ double red[kCbnThreads];
  const uint32_t m = blockIdx.x;
  if (m >= gn) return;
  const int tid = threadIdx.x;
  for (int k = tid; k < d.C; k += kCbnThreads) f[k] = feat[(size_t)m * d.C + k];
  __syncthreads();
  const int rows = 2 * d.nb * d.width;
  for (int r = tid; r < rows; r += kCbnThreads) {
    const int blk = (r / d.width) % d.nb, c = r % d.width;
    const bool is_g = r < d.nb * d.width;
    const float* W = (is_g ? d.Wg[blk] : d.Wb[blk]) + (size_t)c * d.C;
    double acc = 0.0;
    for (int k = 0; k < d.C; ++k) acc += (double)W[k] * f[k];
    gb[r] = acc + (double)(is_g ? d.bg[blk][c] : d.bb[blk][c]);
  }
  const double z = fmin(fmax(ext[4 * (size_t)m], -1.0), 1.0);   // the code's interval
  const double s = (double)(d.n_z - 1) * 0.5 * (z + 1.0);
  double fj = floor(s);
  int j = (int)fj;
  if (j > d.n_z - 1) {
    j = d.n_z - 1;
    fj = (double)j;
  }
  const double frac = s - fj;
  for (int c = tid; c < d.width; c += kCbnThreads) {
    const float* wr = d.Wp + (size_t)c * d.n_z;
    double v = (1.0 - frac) * (double)wr[j] + (double)d.bp[c];
    if (j + 1 < d.n_z) v += frac * (double)wr[j + 1];
    h[c] = v;
  }
  __syncthreads();
  for (int blk = 0; blk < d.nb; ++blk) {
    if (blk > 0) {
      for (int c = tid; c < d.width; c += kCbnThreads) {
        const float* wr = d.W[blk - 1] + (size_t)c * d.width;
        double acc = 0.0;
        for (int k = 0; k < d.width; ++k) acc += (double)wr[k] * a[k];
        h[c] = acc + (double)d.b[blk - 1][c];
      }
      __syncthreads();
    }
    for (int c = tid; c < d.width; c += kCbnThreads) {
      const double hn = (h[c] - (double)d.mean[blk][c]) / sqrt((double)d.var[blk][c] + (double)d.eps);
      const double v = gb[(size_t)blk * d.width + c] * hn + gb[((size_t)d.nb + blk) * d.width + c];
      a[c] = v > 0.0 ? v : 0.0;
    }
    __syncthreads();
  }
  double part = 0.0;
  for (int k = tid; k < d.width; k += kCbnThreads) part += (double)d.Wo[k] * a[k];
  red[tid] = part;
  __syncthreads();
  for (int w = kCbnThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const double lg = red[0] + (double)d.bo[0];
    const uint32_t pos = glist[m];
    logit[pos] = (float)lg;
    lab[pos] = lg > 0.0;
  }
}

size_t guard_cbn64_ws_bytes(const CbnDesc& d, uint32_t chunk) {
  return ((size_t)chunk * (d.C + 4) + 64) * sizeof(double) + (size_t)chunk * 4 + 4096;
}

void run_guard_cbn64(const PointSrc& src, const uint32_t* list, const uint32_t* glist, uint32_t gn,
                     const CbnDesc& d, const float* F, int H, int W, float* logit, uint8_t* lab,
                     void* ws, uint32_t chunk, hipStream_t s) {
  if (!gn) return;
  double* feat = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  double* ext = feat + (size_t)chunk * d.C;
  uint32_t* gnode = reinterpret_cast<uint32_t*>(ext + (size_t)chunk * 4);
  const size_t shmem = ((size_t)d.C + 2 * (size_t)d.nb * d.width + 2 * (size_t)d.width) * sizeof(double);
  for (uint32_t c0 = 0; c0 < gn; c0 += chunk) {
    const uint32_t m = gn - c0 < chunk ? gn - c0 : chunk;
    hipLaunchKernelGGL(k_guard_nodes, dim3(std::min(grid1d(m, 256), kStrideBlocks)), dim3(256), 0,
                       s, list, glist + c0, m, nullptr, gnode);
    const uint32_t pw = std::min(m, 2048u);
    hipLaunchKernelGGL(k_gather64, dim3(grid1d((size_t)pw * 64, 256)), dim3(256), 0, s, src, gnode,
                       m, nullptr, F, H, W, d.C, feat, ext);
    hipLaunchKernelGGL(k_cbn64, dim3(m), dim3(kCbnThreads), shmem, s, d, feat, ext, m, glist + c0,
                       logit, lab);
  }
}

}  // namespace pifu
