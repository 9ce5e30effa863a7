// Level kernels of the two octree subdivisions that Sec. 3.2 ("Octree-based Robust
// Surface Localization") sets against its own localization, and that Fig. 3 compares
// by accuracy against evaluated points:
//   binarized: a coarse cell is subdivided when the binarized occupancy [p > 0.5] of its
//              8 corners is not all equal (the inside/outside interface);
//   threshold: a coarse cell is subdivided when the largest absolute deviation of its 8
//              corner occupancy values from their mean exceeds a threshold.
// Every node of a subdivided cell that was not evaluated before is evaluated at the
// finer level; there is no dilation and no conflict search.  Other nodes take the
// trilinear interpolation of the coarse values (binarized: of the corner labels).
//
// Both rules read the stored float32 occupancy values.  Means, deviations and
// interpolations are taken in float64 in a fixed order: the corner sum runs over
// (di, dj, dk) with dk fastest, and the interpolation is separable, first along x,
// then y, then z, each step 0.5 * (lo + hi).
#include "pifu_internal.h"

namespace pifu {

namespace {

inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

__device__ __forceinline__ uint32_t cell_index(uint32_t a, uint32_t b, uint32_t k, Lat c) {
  return (a * (uint32_t)(c.ny - 1) + b) * (uint32_t)(c.nz - 1) + k;
}

// One thread per coarse cell: the subdivision decision, and the count of subdivided cells.
__global__ void __launch_bounds__(256)
k_oct_flags(const uint8_t* __restrict__ cst, const float* __restrict__ cocc, Lat c, int mode,
            double thr, uint8_t* __restrict__ flags, uint32_t* __restrict__ count) {
  const uint32_t cy = (uint32_t)c.ny - 1, cz = (uint32_t)c.nz - 1;
  const uint32_t ncell = ((uint32_t)c.nx - 1) * cy * cz;
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  bool f = false;
  if (m < ncell) {
    const uint32_t a = m / (cy * cz);
    const uint32_t r = m - a * cy * cz;
    const uint32_t b = r / cz;
    const uint32_t k = r - b * cz;
    const uint32_t nyz = (uint32_t)c.ny * c.nz;
    const size_t base = (size_t)a * nyz + (size_t)b * c.nz + k;
    if (mode == PIFU_OCTREE_BINARIZED) {
      int sum = 0;
#pragma unroll
      for (int di = 0; di < 2; ++di)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj) {
          const uint8_t* row = cst + base + (size_t)di * nyz + (size_t)dj * c.nz;
          sum += (row[0] & ST_LABEL) + (row[1] & ST_LABEL);
        }
      f = sum != 0 && sum != 8;
    } else {
      double v[8];
      double s = 0.0;
#pragma unroll
      for (int di = 0; di < 2; ++di)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
          for (int dk = 0; dk < 2; ++dk) {
            const double x = (double)cocc[base + (size_t)di * nyz + (size_t)dj * c.nz + dk];
            v[di * 4 + dj * 2 + dk] = x;
            s = s + x;
          }
      const double mean = s / 8.0;
      double dev = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) dev = fmax(dev, fabs(v[q] - mean));
      f = dev > thr;
    }
    flags[m] = f ? 1 : 0;
  }
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0 && bal) atomicAdd(count, (uint32_t)__popcll(bal));
}

// x, y or z: the coarse cells containing fine index i (one for odd i, one or two for even).
__device__ __forceinline__ int cells_along(uint32_t i, uint32_t ncells, uint32_t out[2]) {
  if (i & 1) {
    out[0] = i >> 1;
    return 1;
  }
  int n = 0;
  const uint32_t h = i >> 1;
  if (h >= 1) out[n++] = h - 1;
  if (h < ncells) out[n++] = h;
  return n;
}

// One thread per fine node: the culled value and label, the evaluated flag of coarse
// nodes, and ST_PEND for every node of a subdivided cell not evaluated before.
__global__ void __launch_bounds__(256)
k_oct_transition(const uint8_t* __restrict__ cst, const float* __restrict__ cocc, Lat c,
                 const uint8_t* __restrict__ flags, uint8_t* __restrict__ fst,
                 float* __restrict__ focc, Lat f, int mode) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;   // a lattice has < 2^32 nodes
  if (n >= (uint32_t)f.n()) return;
  const uint32_t nyz = (uint32_t)f.ny * f.nz;
  const uint32_t a = n / nyz;
  const uint32_t r = n - a * nyz;
  const uint32_t b = r / f.nz;
  const uint32_t k = r - b * f.nz;
  // in a subdivided cell?
  uint32_t ca[2], cb[2], ck[2];
  const int na = cells_along(a, (uint32_t)c.nx - 1, ca);
  const int nb = cells_along(b, (uint32_t)c.ny - 1, cb);
  const int nk = cells_along(k, (uint32_t)c.nz - 1, ck);
  bool sub = false;
  for (int x = 0; x < na; ++x)
    for (int y = 0; y < nb; ++y)
      for (int z = 0; z < nk; ++z) sub |= flags[cell_index(ca[x], cb[y], ck[z], c)] != 0;
  const uint32_t cyz = (uint32_t)c.ny * c.nz;
  const uint32_t a0 = a >> 1, a1 = (a + 1) >> 1;
  const uint32_t b0 = b >> 1, b1 = (b + 1) >> 1;
  const uint32_t k0 = k >> 1, k1 = (k + 1) >> 1;
  if (!((a | b | k) & 1)) {
    const size_t cn = (size_t)a0 * cyz + (size_t)b0 * c.nz + k0;
    const uint8_t s = cst[cn] & (ST_LABEL | ST_EVAL);
    fst[n] = s | ((sub && !(s & ST_EVAL)) ? ST_PEND : 0);
    focc[n] = cocc[cn];
    return;
  }
  uint8_t s;
  float v;
  if (mode == PIFU_OCTREE_BINARIZED) {
    int sum = 0, cnt = 0;
    for (int da = 0; da < 2; ++da) {
      if (da && a1 == a0) continue;
      for (int db = 0; db < 2; ++db) {
        if (db && b1 == b0) continue;
        const uint8_t* row = cst + (size_t)(da ? a1 : a0) * cyz + (size_t)(db ? b1 : b0) * c.nz;
        sum += row[k0] & ST_LABEL;
        ++cnt;
        if (k1 != k0) {
          sum += row[k1] & ST_LABEL;
          ++cnt;
        }
      }
    }
    s = 2 * sum > cnt ? ST_LABEL : 0;
    v = (float)sum / (float)cnt;
  } else {
    // separable: x first, then y, then z
    double Y[2];
    for (int dk = 0; dk < 2; ++dk) {
      const uint32_t kk = dk ? k1 : k0;
      double X[2];
      for (int db = 0; db < 2; ++db) {
        const uint32_t bb = db ? b1 : b0;
        const double lo = (double)cocc[(size_t)a0 * cyz + (size_t)bb * c.nz + kk];
        if (a1 != a0) {
          const double hi = (double)cocc[(size_t)a1 * cyz + (size_t)bb * c.nz + kk];
          X[db] = 0.5 * (lo + hi);
        } else {
          X[db] = lo;
        }
      }
      Y[dk] = b1 != b0 ? 0.5 * (X[0] + X[1]) : X[0];
    }
    const double z = k1 != k0 ? 0.5 * (Y[0] + Y[1]) : Y[0];
    s = z > 0.5 ? ST_LABEL : 0;
    v = (float)z;
  }
  fst[n] = s | (sub ? ST_PEND : 0);
  focc[n] = v;
}

}  // namespace

void launch_oct_flags(const uint8_t* cst, const float* cocc, Lat c, int mode, double thr,
                      uint8_t* flags, uint32_t* count, hipStream_t s) {
  const size_t ncell = (size_t)(c.nx - 1) * (c.ny - 1) * (c.nz - 1);
  if (ncell)
    hipLaunchKernelGGL(k_oct_flags, dim3(grid1d(ncell, 256)), dim3(256), 0, s, cst, cocc, c, mode,
                       thr, flags, count);
}

void launch_oct_transition(const uint8_t* cst, const float* cocc, Lat c, const uint8_t* flags,
                           uint8_t* fst, float* focc, Lat f, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_oct_transition, dim3(grid1d(f.n(), 256)), dim3(256), 0, s, cst, cocc, c,
                     flags, fst, focc, f, mode);
}

}  // namespace pifu
