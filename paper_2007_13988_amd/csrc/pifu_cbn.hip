// The paper's final lifting network (appendix, "Depth Representation" and "Pixel-aligned
// 3D Lifting"; Tab. 2, HRNet-CBN-SoftZ): a soft one-hot depth code enters a chain of
// [linear layer, conditional batch norm, ReLU] blocks whose scale gamma(c) and shift
// beta(c) are linear maps of the pixel-aligned feature c.
//
// On the input-view grid c depends only on a node's (x, y) column, so every block's
// gamma and beta are computed once per column: one GEMM [columns x C] x [C x 2 nb width]
// (the "hoisted rows").  Per point there remain the soft one-hot layer (two non-zero
// inputs: a blend of two weight columns), nb - 1 width x width GEMMs whose epilogue applies
// the batch norm and the column's gamma / beta, and the head.
#include "pifu_internal.h"

namespace pifu {

namespace {

inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Packs the conditional maps and the batch-norm constants (one thread per output).
__global__ void k_cbn_pack(CbnDesc d, float* __restrict__ Wgb, float* __restrict__ bgb,
                           float* __restrict__ mu, float* __restrict__ rstd) {
  const size_t rows = 2 * (size_t)d.nb * d.width;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * d.C) {
    const size_t r = i / d.C, k = i - r * d.C;
    const int blk = (int)(r / d.width) % d.nb, c = (int)(r % d.width);
    const float* W = r < (size_t)d.nb * d.width ? d.Wg[blk] : d.Wb[blk];
    Wgb[i] = W[(size_t)c * d.C + k];
  }
  if (i < rows) {
    const int blk = (int)(i / d.width) % d.nb, c = (int)(i % d.width);
    bgb[i] = i < (size_t)d.nb * d.width ? d.bg[blk][c] : d.bb[blk][c];
  }
  if (i < (size_t)d.nb * d.width) {
    const int blk = (int)(i / d.width), c = (int)(i % d.width);
    mu[i] = d.mean[blk][c];
    rstd[i] = (float)(1.0 / sqrt((double)d.var[blk][c] + (double)d.eps));
  }
}

// z of point m: lattice node (mode 0, input view) or explicit point (mode 1, clamped to
// [-1, 1], the interval the depth code is defined on).
__device__ inline double point_z(const PointSrc& s, const uint32_t* list, uint32_t m) {
  const uint32_t idx = (list ? list[m] : m) - s.base_sub;
  if (s.mode == 1) return fmin(fmax((double)s.pts[idx].z, -1.0), 1.0);
  const uint32_t k = idx % (uint32_t)s.nz;
  return __dadd_rn(-1.0, __ddiv_rn(__dmul_rn(2.0, (double)k), (double)(s.nz - 1)));
}

// One thread per (point, channel): the soft one-hot layer, batch norm with the column's
// gamma_0 / beta_0, ReLU.
__global__ void __launch_bounds__(256)
k_cbn_first(PointSrc src, const uint32_t* __restrict__ list, uint32_t n, CbnDesc d,
            const float* __restrict__ P, const uint32_t* __restrict__ cid,
            const float* __restrict__ mu, const float* __restrict__ rstd, float* __restrict__ a) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * d.width) return;
  const uint32_t m = (uint32_t)(t / d.width);
  const int c = (int)(t - (size_t)m * d.width);
  const double s = (double)(d.n_z - 1) * 0.5 * (point_z(src, list, m) + 1.0);
  double fj = floor(s);
  int j = (int)fj;
  if (j > d.n_z - 1) {
    j = d.n_z - 1;
    fj = (double)j;
  }
  const double frac = s - fj;
  const float* wr = d.Wp + (size_t)c * d.n_z;
  double h = (1.0 - frac) * (double)wr[j] + (double)d.bp[c];
  if (j + 1 < d.n_z) h += frac * (double)wr[j + 1];
  const size_t ld = 2 * (size_t)d.nb * d.width;
  const float* row = P + (size_t)cid[m] * ld;
  const float g = row[c], bt = row[(size_t)d.nb * d.width + c];
  const float v = ((float)h - mu[c]) * rstd[c] * g + bt;
  a[t] = v > 0.f ? v : 0.f;
}

}  // namespace

void launch_cbn_pack(const CbnDesc& d, float* Wgb, float* bgb, float* mu, float* rstd,
                     hipStream_t s) {
  const size_t n = 2 * (size_t)d.nb * d.width * d.C;
  hipLaunchKernelGGL(k_cbn_pack, dim3(grid1d(n, 256)), dim3(256), 0, s, d, Wgb, bgb, mu, rstd);
}

void launch_cbn_first(const PointSrc& src, const uint32_t* list, uint32_t n, const CbnDesc& d,
                      const float* P, const uint32_t* cid, const float* mu, const float* rstd,
                      float* a, hipStream_t s) {
  if (n)
    hipLaunchKernelGGL(k_cbn_first, dim3(grid1d((size_t)n * d.width, 256)), dim3(256), 0, s, src,
                       list, n, d, P, cid, mu, rstd, a);
}

}  // namespace pifu
