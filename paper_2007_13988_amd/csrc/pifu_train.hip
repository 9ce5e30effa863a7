// Training kernels for the distilled surrogate occupancy network: soft-target binary
// cross entropy (the occupancy loss of Sec. 3.1) and its gradient, the backward pass
// of a fully connected ReLU network with feature skips, and RMSProp (the optimizer
// of the shape network, appendix A1.2).  Every reduction over the batch runs in a
// fixed order (split partials + ordered sums), so gradients are bit-reproducible.
#include "pifu_internal.h"

namespace pifu {

static inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

// g[m] = (sigmoid(s) - t) / n ; per-block partial sums of softplus(s) - t s.
__global__ void __launch_bounds__(256)
k_bce_grad(const float* __restrict__ s, const float4* __restrict__ pts, uint32_t n,
           float* __restrict__ g, float* __restrict__ loss_part, float* __restrict__ point_loss) {
  __shared__ float red[256];
  const uint32_t m = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (m < n) {
    const float x = s[m];
    const float t = pts[m].w;
    const float p = 1.f / (1.f + expf(-x));
    g[m] = (p - t) / (float)n;
    l = fmaxf(x, 0.f) - t * x + log1pf(expf(-fabsf(x)));
    if (point_loss) point_loss[m] = l;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Ordered sum of np partials, scaled: out[0] = scale * sum_i part[i].
__global__ void k_sum_ordered(const float* __restrict__ part, uint32_t np, float scale,
                              float* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (uint32_t i = 0; i < np; ++i) acc += part[i];
  *out = (float)(acc * scale);
}

// Split-K "TN" product: part[s][o][k] = sum over m in split s of G[m][o] * X[m][k],
// where X = [A1 (K1 cols) ; A2 (K2 cols) ; ext extras (n_ext cols)].  64 x 64 output
// tile per workgroup, 4 x 4 per thread, 16 batch rows per LDS stage.
struct TNArgs {
  const float* G;
  int N;            // columns of G (= outputs of the layer)
  const float* A1;
  int K1, lda1;
  const float* A2;
  int K2, lda2;
  const float* ext;
  int n_ext;
  int K;            // K1 + K2 + n_ext
  uint32_t M;       // batch rows
  uint32_t rows_per_split;
  float* part;      // [splits][N][K]
};

__device__ inline float tn_x(const TNArgs& a, uint32_t m, int k) {
  if (k < a.K1) return a.A1[(size_t)m * a.lda1 + k];
  k -= a.K1;
  if (k < a.K2) return a.A2[(size_t)m * a.lda2 + k];
  k -= a.K2;
  if (k < a.n_ext) return a.ext[4 * (size_t)m + k];
  return 0.f;
}

__global__ void __launch_bounds__(256) k_tn_partial(TNArgs a) {
  __shared__ float Gs[16][64 + 1];
  __shared__ float Xs[16][64 + 1];
  const int o0 = blockIdx.x * 64, k0 = blockIdx.y * 64, split = blockIdx.z;
  const uint32_t mb = (uint32_t)split * a.rows_per_split;
  const uint32_t me = min(a.M, mb + a.rows_per_split);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // 16 x 16 threads
  float acc[4][4] = {};
  for (uint32_t m0 = mb; m0 < me; m0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      const uint32_t m = m0 + r;
      const bool ok = m < me;
      Gs[r][c] = (ok && o0 + c < a.N) ? a.G[(size_t)m * a.N + o0 + c] : 0.f;
      Xs[r][c] = (ok && k0 + c < a.K) ? tn_x(a, m, k0 + c) : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
      float gv[4], xv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gv[i] = Gs[r][ty + 16 * i];
        xv[i] = Xs[r][tx + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(gv[i], xv[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* out = a.part + (size_t)split * a.N * a.K;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = o0 + ty + 16 * i, k = k0 + tx + 16 * j;
      if (o < a.N && k < a.K) out[(size_t)o * a.K + k] = acc[i][j];
    }
}

// out[i] = sum_s part[s][i] in split order.
__global__ void k_reduce_splits(const float* __restrict__ part, int splits, size_t len,
                                float* __restrict__ out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float acc = 0.f;
  for (int s = 0; s < splits; ++s) acc += part[(size_t)s * len + i];
  out[i] = acc;
}

// Column sums of G per split: part[s][o] = sum over m in split s of G[m][o].
__global__ void k_colsum_partial(const float* __restrict__ G, int N, uint32_t M,
                                 uint32_t rows_per_split, float* __restrict__ part) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int split = blockIdx.y;
  if (o >= N) return;
  const uint32_t mb = (uint32_t)split * rows_per_split;
  const uint32_t me = min(M, mb + rows_per_split);
  float acc = 0.f;
  for (uint32_t m = mb; m < me; ++m) acc += G[(size_t)m * N + o];
  part[(size_t)split * N + o] = acc;
}

// dH[m][k] = (sum_o G[m][o] W[o][k]) * [H[m][k] > 0] for k < Kh (ReLU backward;
// LeakyReLU uses slope 0.01 for non-positive H).  64 x 64 tile, 4 x 4 per thread.
__global__ void __launch_bounds__(256)
k_backprop_input(const float* __restrict__ G, int N, const float* __restrict__ W, int ldw,
                 const float* __restrict__ H, int Kh, uint32_t M, int act,
                 float* __restrict__ dH) {
  __shared__ float Gs[64][16 + 1];
  __shared__ float Ws[16][64 + 1];
  const uint32_t m0 = blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4] = {};
  for (int o0 = 0; o0 < N; o0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e >> 4, c = e & 15;
      const uint32_t m = m0 + r;
      Gs[r][c] = (m < M && o0 + c < N) ? G[(size_t)m * N + o0 + c] : 0.f;
      const int rr = e >> 6, cc = e & 63;
      Ws[rr][cc] = (o0 + rr < N && k0 + cc < Kh) ? W[(size_t)(o0 + rr) * ldw + k0 + cc] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < 16; ++c) {
      float gv[4], wv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gv[i] = Gs[ty + 16 * i][c];
        wv[i] = Ws[c][tx + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(gv[i], wv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t m = m0 + ty + 16 * i;
      const int k = k0 + tx + 16 * j;
      if (m >= M || k >= Kh) continue;
      const float h = H[(size_t)m * Kh + k];
      const float d = h > 0.f ? 1.f : (act == PIFU_ACT_LRELU ? 0.01f : 0.f);
      dH[(size_t)m * Kh + k] = acc[i][j] * d;
    }
}

__global__ void k_rmsprop(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ v,
                          size_t n, float lr, float alpha, float eps) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float vi = alpha * v[i] + (1.f - alpha) * gi * gi;
  v[i] = vi;
  w[i] = w[i] - lr * gi / (sqrtf(vi) + eps);
}

// ------------------------------------------------------------------ launchers
uint32_t bce_partials(uint32_t n) { return (n + 255) / 256; }

void launch_bce_grad(const float* s, const float4* pts, uint32_t n, float* g, float* loss_part,
                     float* loss, hipStream_t st, float* point_loss) {
  if (!n) return;
  const uint32_t nb = bce_partials(n);
  hipLaunchKernelGGL(k_bce_grad, dim3(nb), dim3(256), 0, st, s, pts, n, g, loss_part, point_loss);
  if (loss) hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(64), 0, st, loss_part, nb, 1.f / n, loss);
}

int tn_splits(uint32_t M) {
  int s = (int)((M + 2047) / 2048);
  return s < 1 ? 1 : (s > 64 ? 64 : s);
}

// dW = G^T X (N x K, row-major, ld K) and db = column sums of G, ordered reductions.
void launch_weight_grad(const float* G, int N, const float* A1, int K1, int lda1, const float* A2,
                        int K2, int lda2, const float* ext, int n_ext, uint32_t M, float* part,
                        float* dW, float* db, hipStream_t st) {
  const int splits = tn_splits(M);
  const uint32_t rps = (uint32_t)((M + splits - 1) / splits);
  TNArgs a;
  a.G = G;
  a.N = N;
  a.A1 = A1;
  a.K1 = K1;
  a.lda1 = lda1;
  a.A2 = A2;
  a.K2 = K2;
  a.lda2 = lda2;
  a.ext = ext;
  a.n_ext = n_ext;
  a.K = K1 + K2 + n_ext;
  a.M = M;
  a.rows_per_split = (rps + 15) / 16 * 16;
  a.part = part;
  const int sp = (int)((M + a.rows_per_split - 1) / a.rows_per_split);
  hipLaunchKernelGGL(k_tn_partial, dim3((N + 63) / 64, (a.K + 63) / 64, sp), dim3(256), 0, st, a);
  const size_t len = (size_t)N * a.K;
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid1d(len, 256)), dim3(256), 0, st, part, sp, len, dW);
  hipLaunchKernelGGL(k_colsum_partial, dim3((N + 63) / 64, sp), dim3(64), 0, st, G, N, M,
                     a.rows_per_split, part);
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid1d(N, 256)), dim3(256), 0, st, part, sp, (size_t)N, db);
}

size_t weight_grad_part_floats(int N, int K, uint32_t M) {
  return (size_t)tn_splits(M) * N * (K + 1) + 64;
}

void launch_backprop_input(const float* G, int N, const float* W, int ldw, const float* H, int Kh,
                           uint32_t M, int act, float* dH, hipStream_t st) {
  hipLaunchKernelGGL(k_backprop_input, dim3((M + 63) / 64, (Kh + 63) / 64), dim3(256), 0, st, G, N,
                     W, ldw, H, Kh, M, act, dH);
}

void launch_rmsprop(float* w, const float* g, float* v, size_t n, float lr, float alpha, float eps,
                    hipStream_t st) {
  if (n)
    hipLaunchKernelGGL(k_rmsprop, dim3(grid1d(n, 256)), dim3(256), 0, st, w, g, v, n, lr, alpha, eps);
}

}  // namespace pifu
