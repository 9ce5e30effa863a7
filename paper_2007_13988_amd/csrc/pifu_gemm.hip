// MLP layers as MFMA GEMMs over compacted point tiles (Eq. 1's f_O / Eq. 2's f_T).
//
// One workgroup computes a BM x BN tile of C = act(A W^T + b + extras) where A is
// the concatenation [A1 ; A2] of the previous activation and the sampled feature
// (the skip connection), both row-major with the contraction index contiguous.
// Tiles are staged through LDS with double buffering; each wave owns a
// (BM/WM) x (BN/WN) sub-tile built from 32x32 MFMA blocks.
//
// The contraction index is permuted inside each MFMA group: lane half h feeds the
// k values [c*h, c*h + c) of the group (c = elements per lane per MFMA) so that a
// lane's operand is one contiguous 16-byte LDS read.  A and B use the same
// permutation, so the sum over k is unchanged.
#include <hip/hip_ext.h>

#include <algorithm>

#include "pifu_internal.h"

namespace pifu {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
// Native vectors for the global->LDS staging registers (HIP's float4/uint4 structs are
// copied as memcpy, which keeps the staging array in scratch memory).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Tile of this workgroup.  Workgroups are dispatched in order x + gridDim.x * y and dealt
// round-robin to the 8 XCDs, each with its own L2.  The grid's row-tile count is a
// multiple of 8 (launches round it up; the extra tiles lie past M and exit at once).
// XCD k takes the row tiles k, k + 8, k + 16, ... in increasing order, with the column
// tiles of one row tile dispatched next to each other: a row tile of A is fetched from
// HBM once and its other column tiles read it from the same L2, and the rows a launch
// covers stay spread over all XCDs (launches whose device-side row count is below the
// grid's exit their last row tiles on every XCD alike).  The tile set is unchanged.
__device__ inline void tile_of_block(int& rt, int& ct) {
  const int nby = gridDim.y;
  const int id = blockIdx.x + gridDim.x * blockIdx.y;
  const int q = id >> 3;
  rt = (q / nby) * 8 + (id & 7);
  ct = q - (q / nby) * nby;
}

// Row tiles of a launch over M rows in tiles of bm, rounded up to a multiple of 8.
inline unsigned row_tiles(int M, int bm) { return (unsigned)(((M + bm - 1) / bm + 7) / 8 * 8); }

// The same order for a persistent launch: a 1-D grid (a multiple of 8 workgroups) whose
// workgroups take tile ids id, id + gridDim.x, ... of the tile set of the device-side
// row count; tile id maps to (rt, ct) as workgroup id does above, so a workgroup stays
// on one XCD's row tiles.
__device__ inline void tile_of_id(int id, int nby, int& rt, int& ct) {
  const int q = id >> 3;
  rt = (q / nby) * 8 + (id & 7);
  ct = q - (q / nby) * nby;
}
__device__ inline int tiles_of(int M, int bm, int nby) {
  return ((M + bm - 1) / bm + 7) / 8 * 8 * nby;
}
// Workgroups of a persistent GEMM launch.
constexpr unsigned kPersistBlocks = 512;

__device__ inline float act_apply(float v, int act) {
  if (act == PIFU_ACT_RELU) return v > 0.f ? v : 0.f;
  if (act == PIFU_ACT_LRELU) return v > 0.f ? v : 0.01f * v;
  return v;
}

// Epilogue: 32x32 accumulator block -> C in format OUT (FMT_*).  Output layout of a
// 32x32 MFMA block: lane l, register r holds row 8*(r/4) + 4*(l/32) + (r%4), column l%32.
// FMT_F16: a value outside the binary16 range sets *a.ovf.
template <int OUT, bool TAPS = false>
__device__ inline void store_block(const GemmArgs& a, const f32x16& acc, int row0, int col0,
                                   int lane, int M) {
  const int col = col0 + (lane & 31);
  const float bias = a.bias ? a.bias[col] : 0.f;
  const float we0 = a.n_ext > 0 ? a.Wf[(size_t)col * a.ldwf + a.ext_col] : 0.f;
  const float we1 = a.n_ext > 1 ? a.Wf[(size_t)col * a.ldwf + a.ext_col + 1] : 0.f;
  // loads use the row clamped into range (M >= 1 here), so all of them can be in
  // flight together; only the stores are predicated
  int rr[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) rr[r] = min(row0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), M - 1);
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = acc[r] * a.scale + bias;
  if constexpr (TAPS) {
    // per-texel hoisting: blend the four texel rows of each point
    // (four rows at a time: the scheduling barrier keeps the loads of only four rows in
    // flight, so the blend needs few registers beside the accumulators)
    const float* rb = a.rowadd + a.rowadd_off + col;
    const size_t ld = (size_t)a.rowadd_ld;
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += 4) {
#pragma unroll
      for (int r = r0; r < r0 + 4; ++r) {
        const int4 ti = a.tap_idx[rr[r]];
        const float4 tw = a.tap_w[rr[r]];
        float t = tw.x * rb[(size_t)ti.x * ld];
        t = fmaf(tw.y, rb[(size_t)ti.y * ld], t);
        t = fmaf(tw.z, rb[(size_t)ti.z * ld], t);
        t = fmaf(tw.w, rb[(size_t)ti.w * ld], t);
        v[r] += t;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if (a.rowadd) {
    uint32_t ix[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ix[r] = a.rowadd_idx[rr[r]];
    if (OUT == FMT_F32 && a.rowmul) {   // conditional batch norm: scale, then shift
      const float mu = a.cbn_mu[col], rs = a.cbn_rstd[col];
#pragma unroll
      for (int r = 0; r < 16; ++r)
        v[r] = (v[r] - mu) * rs * a.rowmul[(size_t)ix[r] * a.rowadd_ld + a.rowmul_off + col];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] += a.rowadd[(size_t)ix[r] * a.rowadd_ld + a.rowadd_off + col];
  }
  if (a.n_ext > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float* ex = a.ext + 4 * (size_t)rr[r];
      v[r] = fmaf(ex[0], we0, v[r]);
      if (a.n_ext > 1) v[r] = fmaf(ex[1], we1, v[r]);
    }
  }
  bool big = false;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = row0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row >= M) continue;
    const float x = act_apply(v[r], a.act);
    if (OUT == FMT_BF16) {
      reinterpret_cast<uint16_t*>(a.C)[(size_t)row * a.ldc + col] = f32_to_bf16_bits(x);
    } else if (OUT == FMT_F16) {
      big |= !(__builtin_fabsf(x) <= kF16Max);
      reinterpret_cast<uint16_t*>(a.C)[(size_t)row * a.ldc + col] = f32_to_f16_bits(x);
    } else {
      reinterpret_cast<float*>(a.C)[(size_t)row * a.ldc + col] = x;
    }
  }
  if (OUT == FMT_F16 && big && a.ovf) atomicOr(a.ovf, 1u);
}

// As store_block, for a 16-bit output staged in LDS: the block's converted values go to
// T[(lrow0 + row) * ldt + lcol0 + col] (tile-local rows and columns; rows past M are
// staged too and skipped when the tile is written out).  Returns whether a value left
// the binary16 range (FMT_F16).
template <int OUT>
__device__ inline bool stage_block(const GemmArgs& a, const f32x16& acc, int m0, int lrow0, int col0,
                                   int lcol0, int lane, int M, uint16_t* T, int ldt) {
  const int col = col0 + (lane & 31);
  const float bias = a.bias ? a.bias[col] : 0.f;
  const float we0 = a.n_ext > 0 ? a.Wf[(size_t)col * a.ldwf + a.ext_col] : 0.f;
  const float we1 = a.n_ext > 1 ? a.Wf[(size_t)col * a.ldwf + a.ext_col + 1] : 0.f;
  int rr[16];
#pragma unroll
  for (int r = 0; r < 16; ++r)
    rr[r] = min(m0 + lrow0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), M - 1);
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = acc[r] * a.scale + bias;
  if (a.rowadd) {
    uint32_t ix[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ix[r] = a.rowadd_idx[rr[r]];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] += a.rowadd[(size_t)ix[r] * a.rowadd_ld + a.rowadd_off + col];
  }
  if (a.n_ext > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float* ex = a.ext + 4 * (size_t)rr[r];
      v[r] = fmaf(ex[0], we0, v[r]);
      if (a.n_ext > 1) v[r] = fmaf(ex[1], we1, v[r]);
    }
  }
  bool big = false;
  uint16_t* t = T + (size_t)(lrow0 + 4 * (lane >> 5)) * ldt + lcol0 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float x = act_apply(v[r], a.act);
    uint16_t bits;
    if (OUT == FMT_F16) {
      big |= !(__builtin_fabsf(x) <= kF16Max);
      bits = f32_to_f16_bits(x);
    } else {
      bits = f32_to_bf16_bits(x);
    }
    t[(8 * (r >> 2) + (r & 3)) * ldt] = bits;
  }
  return big;
}

// FP32 epilogue of a whole tile staged in LDS (T: BM rows of ldt floats, tile-local):
// each thread finishes four consecutive columns of a row at a time, so the tile's bias,
// hoisted-row and texel-row loads and its stores are 16 bytes per lane.  Same arithmetic,
// in the same order, as store_block<FMT_F32, TAPS>.
template <int BM, int BN, int NT, bool TAPS>
__device__ inline void finish_tile(const GemmArgs& a, const float* T, int ldt, int m0, int n0,
                                   int M, int tid) {
  constexpr int CPR = BN / 4;     // four-column chunks per row
  constexpr int RPP = NT / CPR;   // rows per pass
  static_assert(NT % CPR == 0 && BM % RPP == 0, "tile and thread count do not match");
  const int c4 = tid % CPR, lr0 = tid / CPR;
  const int col = n0 + 4 * c4;
  const float4 b = a.bias ? *reinterpret_cast<const float4*>(a.bias + col) : make_float4(0.f, 0.f, 0.f, 0.f);
  const float bb[4] = {b.x, b.y, b.z, b.w};
  float we0[4], we1[4], mu[4], rs[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    we0[c] = a.n_ext > 0 ? a.Wf[(size_t)(col + c) * a.ldwf + a.ext_col] : 0.f;
    we1[c] = a.n_ext > 1 ? a.Wf[(size_t)(col + c) * a.ldwf + a.ext_col + 1] : 0.f;
    mu[c] = a.rowmul ? a.cbn_mu[col + c] : 0.f;
    rs[c] = a.rowmul ? a.cbn_rstd[col + c] : 0.f;
  }
#pragma unroll 4
  for (int q = 0; q < BM / RPP; ++q) {
    const int lr = lr0 + q * RPP;
    const int row = m0 + lr;
    if (row >= M) break;   // rows grow with q
    const float4 s = *reinterpret_cast<const float4*>(T + lr * ldt + 4 * c4);
    const float ss[4] = {s.x, s.y, s.z, s.w};
    float v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = ss[c] * a.scale + bb[c];
    if constexpr (TAPS) {
      // per-texel hoisting: blend the four texel rows of the point
      const int4 ti = a.tap_idx[row];
      const float4 tw = a.tap_w[row];
      const float* rb = a.rowadd + a.rowadd_off + col;
      const size_t ld = (size_t)a.rowadd_ld;
      const float4 p0 = *reinterpret_cast<const float4*>(rb + (size_t)ti.x * ld);
      const float4 p1 = *reinterpret_cast<const float4*>(rb + (size_t)ti.y * ld);
      const float4 p2 = *reinterpret_cast<const float4*>(rb + (size_t)ti.z * ld);
      const float4 p3 = *reinterpret_cast<const float4*>(rb + (size_t)ti.w * ld);
      const float q0[4] = {p0.x, p0.y, p0.z, p0.w}, q1[4] = {p1.x, p1.y, p1.z, p1.w};
      const float q2[4] = {p2.x, p2.y, p2.z, p2.w}, q3[4] = {p3.x, p3.y, p3.z, p3.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float t = tw.x * q0[c];
        t = fmaf(tw.y, q1[c], t);
        t = fmaf(tw.z, q2[c], t);
        t = fmaf(tw.w, q3[c], t);
        v[c] += t;
      }
    } else if (a.rowadd) {
      const size_t base = (size_t)a.rowadd_idx[row] * a.rowadd_ld;
      if (a.rowmul) {   // conditional batch norm: scale, then shift
        const float4 g = *reinterpret_cast<const float4*>(a.rowmul + base + a.rowmul_off + col);
        const float gg[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = (v[c] - mu[c]) * rs[c] * gg[c];
      }
      const float4 p = *reinterpret_cast<const float4*>(a.rowadd + base + a.rowadd_off + col);
      const float pp[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] += pp[c];
    }
    if (a.n_ext > 0) {
      const float* ex = a.ext + 4 * (size_t)row;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        v[c] = fmaf(ex[0], we0[c], v[c]);
        if (a.n_ext > 1) v[c] = fmaf(ex[1], we1[c], v[c]);
      }
    }
    *reinterpret_cast<float4*>(reinterpret_cast<float*>(a.C) + (size_t)row * a.ldc + col) =
        make_float4(act_apply(v[0], a.act), act_apply(v[1], a.act), act_apply(v[2], a.act),
                    act_apply(v[3], a.act));
  }
}

// ------------------------------------------------------------------ FP32 operands
// v_mfma_f32_32x32x2_f32: per lane one A and one B element per MFMA; 4 MFMAs consume
// a float4 of k from LDS (k-group of 8).
//
// Pipeline of one 32-deep k stage (two LDS buffers): first the LDS writes of stage k + 1,
// whose global loads were issued one stage earlier, then the LDS reads of group 0 and
// the global loads of stage k + 2, then the 64 MFMAs of the stage, each group's LDS reads
// issued during the previous group's MFMAs; one barrier per stage.  The body is one basic
// block (the last stages reload the last k tile and write it into the idle buffer, which
// nobody reads), so the scheduling groups below can spread the LDS writes, global loads
// and LDS reads between the MFMAs.  Rows past M load row M - 1 (their outputs are never
// stored).  Instruction order only: every accumulator sums k in the same order in every
// tile shape.
template <int BM, int BN, int WM, int WN, int MINB, int NT = 256, bool PERSIST = false,
          bool TAPS = false>
__global__ void __launch_bounds__(NT, MINB) k_gemm_f32(GemmArgs a) {
  // TAPS: the epilogue blends four texel rows per point (per-texel hoisting)
  // NT = 64 * WM * WN threads (the 32-point tile for tiny launches uses 2 waves)
  constexpr int BK = 32;
  constexpr int LD = BK + 4;
  constexpr int TI = BM / WM / 32, TJ = BN / WN / 32;
  // one LDS block: the double-buffered A and B stages during the k loop, the output tile
  // (row-major, LDT floats per row: the two row groups of a 32 x 32 block's store land
  // 32 banks apart) after it
  constexpr int LDT = BN + 8;
  constexpr int SM_OP = 2 * (BM + BN) * LD;
  // the output tile is staged EPR rows at a time, as many as the operand stages' LDS holds
  // (the 256 x 128 tile in two halves), so the epilogue adds no LDS to the workgroup
  constexpr int EPR = BM * LDT <= SM_OP ? BM : BM / 2;
  static_assert(EPR * LDT <= SM_OP && EPR % (BM / WM) == 0, "output staging");
  __shared__ __attribute__((aligned(16))) float smem[SM_OP];
  float (*const As)[BM * LD] = reinterpret_cast<float (*)[BM * LD]>(smem);              // As[stage]
  float (*const Bs)[BN * LD] = reinterpret_cast<float (*)[BN * LD]>(smem + 2 * BM * LD);  // Bs[stage]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int M = a.M_dev ? min(a.M, (int)*a.M_dev) : a.M;
  // persistent launches stride over the tiles of the device-side row count; others
  // take the one tile of their workgroup
  const int nby = a.N / BN;
  const int n_ids = PERSIST ? tiles_of(M, BM, nby) : 1;
  for (int id = PERSIST ? (int)blockIdx.x : 0; id < n_ids; id += PERSIST ? (int)gridDim.x : 1) {
  int rt, ct;
  if (PERSIST) tile_of_id(id, nby, rt, ct);
  else tile_of_block(rt, ct);
  const int m0 = rt * BM, n0 = ct * BN;
  if (m0 >= M) continue;
  const int K = a.K1 + a.K2;
  const int nk = K / BK;
  constexpr int A_LOADS = BM * (BK / 4) / NT;
  constexpr int B_LOADS = BN * (BK / 4) / NT;
  f32x4 ra[A_LOADS], rb[B_LOADS];
  // this thread's global rows (A rows clamped into [0, M)) and LDS slots, per load
  const float* pa1[A_LOADS];
  const float* pa2[A_LOADS];
  const float* pb[B_LOADS];
  int sa[A_LOADS], sb[B_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int e = tid + NT * i;
    const int gm = min(m0 + (e >> 3), M - 1);
    pa1[i] = reinterpret_cast<const float*>(a.A1) + (size_t)gm * a.lda1 + 4 * (e & 7);
    pa2[i] = a.A2 ? reinterpret_cast<const float*>(a.A2) + (size_t)gm * a.lda2 + 4 * (e & 7) : pa1[i];
    sa[i] = (e >> 3) * LD + 4 * (e & 7);
  }
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int e = tid + NT * i;
    pb[i] = reinterpret_cast<const float*>(a.W) + (size_t)(n0 + (e >> 3)) * a.ldw + 4 * (e & 7);
    sb[i] = (e >> 3) * LD + 4 * (e & 7);
  }
  auto gload = [&](int kt) {
    const int k0 = kt * BK;
    const bool first = k0 < a.K1;   // A = [A1 ; A2] along k
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i)
      ra[i] = *reinterpret_cast<const f32x4*>(first ? pa1[i] + k0 : pa2[i] + (k0 - a.K1));
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) rb[i] = *reinterpret_cast<const f32x4*>(pb[i] + k0);
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) *reinterpret_cast<f32x4*>(&As[buf][sa[i]]) = ra[i];
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) *reinterpret_cast<f32x4*>(&Bs[buf][sb[i]]) = rb[i];
  };

  f32x16 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int h = lane >> 5, l32 = lane & 31;
  const int wrow = wm * (BM / WM), wcol = wn * (BN / WN);
  gload(0);
  sstore(0);
  gload(min(1, nk - 1));
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    sstore(buf ^ 1);
    float4 av[2][TI], bv[2][TJ];
    auto lread = [&](int kk, int sl) {
#pragma unroll
      for (int i = 0; i < TI; ++i)
        av[sl][i] = *reinterpret_cast<const float4*>(&As[buf][(wrow + 32 * i + l32) * LD + kk + 4 * h]);
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        bv[sl][j] = *reinterpret_cast<const float4*>(&Bs[buf][(wcol + 32 * j + l32) * LD + kk + 4 * h]);
    };
    // k slot outermost: consecutive MFMAs write different accumulators
    auto mfma = [&](int sl) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[sl][i][c], bv[sl][j][c], acc[i][j], 0, 0, 0);
    };
    lread(0, 0);
    gload(min(kt + 2, nk - 1));
    lread(8, 1);
    mfma(0);
    lread(16, 0);
    mfma(1);
    lread(24, 1);
    mfma(0);
    mfma(1);
    // scheduling groups (mask 0x008 MFMA, 0x020 global load, 0x100 LDS read, 0x200 LDS
    // write): the writes and group 0's reads, then one global load or group 1 read after
    // each MFMA, then the reads of groups 2 and 3 spread over groups 1 and 2
    constexpr int NW = A_LOADS + B_LOADS, NR = TI + TJ, NM = TI * TJ * 4;
    __builtin_amdgcn_sched_group_barrier(0x200, NW, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, NR, 0);
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    if (NM > NW + NR) __builtin_amdgcn_sched_group_barrier(0x008, NM - NW - NR, 0);
#pragma unroll
    for (int g = 1; g < 3; ++g) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      if (NM > 2 * NR) __builtin_amdgcn_sched_group_barrier(0x008, NM - 2 * NR, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NM, 0);
    __syncthreads();
  }
  if (!PERSIST && a.ep_vec) {
    // the loop's last barrier has retired every read of the operand stages: stage the
    // tile in LDS, then finish it four columns per lane (persistent tiles keep the block
    // epilogue: their tap variant has no registers to spare for both)
#pragma unroll
    for (int q = 0; q < BM / EPR; ++q) {
      // rows [q EPR, (q + 1) EPR) of the tile: whole wave rows, so a wave stages in one
      // round only
      if (q > 0) __syncthreads();   // the previous round's rows have been read
      if (wrow / EPR == q) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            float* t = smem + (wrow - q * EPR + 32 * i + 4 * h) * LDT + wcol + 32 * j + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) t[(8 * (r >> 2) + (r & 3)) * LDT] = acc[i][j][r];
          }
      }
      __syncthreads();
      finish_tile<EPR, BN, NT, TAPS>(a, smem, LDT, m0 + q * EPR, n0, M, tid);
    }
  } else {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        store_block<FMT_F32, TAPS>(a, acc[i][j], m0 + wrow + 32 * i, n0 + wcol + 32 * j, lane, M);
  }
  if (PERSIST) __syncthreads();   // LDS is reused by the next tile
  }
}

// ------------------------------------------------------------------ 16-bit operands
// v_mfma_f32_32x32x16_bf16 (F16 = false) or v_mfma_f32_32x32x16_f16 (F16 = true): 8
// 16-bit values per lane per MFMA (one 16-byte LDS read); BK = 64 per stage.  A, W and
// (OUT16) C hold the same 16-bit format.
template <int BM, int BN, int WM, int WN, int MINB, bool OUT16, bool F16, int NT = 256,
          bool PERSIST = false>
__global__ void __launch_bounds__(NT, MINB) k_gemm_h16(GemmArgs a) {
  // NT = 64 * WM * WN threads; the 256 x 256 tile uses 512 threads (8 waves of 128 x 64)
  constexpr int BK = 64;
  constexpr int LD = BK + 8;   // in bf16 elements
  constexpr int TI = BM / WM / 32, TJ = BN / WN / 32;
  // one LDS block: the double-buffered A and B stages, and after the k loop the
  // converted output tile (OUT16)
  constexpr int SMEM = 2 * (BM + BN) * LD;
  __shared__ __attribute__((aligned(16))) __bf16 smem[SMEM];
  __bf16* const As = smem;                  // stage b of A at As + b * BM * LD
  __bf16* const Bs = smem + 2 * BM * LD;    // stage b of B at Bs + b * BN * LD
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int M = a.M_dev ? min(a.M, (int)*a.M_dev) : a.M;
  // persistent launches stride over the tiles of the device-side row count; others
  // take the one tile of their workgroup
  const int nby = a.N / BN;
  const int n_ids = PERSIST ? tiles_of(M, BM, nby) : 1;
  for (int id = PERSIST ? (int)blockIdx.x : 0; id < n_ids; id += PERSIST ? (int)gridDim.x : 1) {
  int rt, ct;
  if (PERSIST) tile_of_id(id, nby, rt, ct);
  else tile_of_block(rt, ct);
  const int m0 = rt * BM, n0 = ct * BN;
  if (m0 >= M) continue;
  const int K = a.K1 + a.K2;
  const int nk = K / BK;
  constexpr int A_LOADS = BM * (BK / 8) / NT;
  constexpr int B_LOADS = BN * (BK / 8) / NT;
  constexpr int S_LOADS = A_LOADS > B_LOADS ? A_LOADS : B_LOADS;
  // Large tiles: one staging set, used in turn for the next stage's A tile and then its
  // B tile (registers are scarce).  Tiles up to 128 x 128 give B a set of its own, so
  // that both loads of the next stage are in flight while this stage computes: their
  // short k loops are bound by load latency, not by MFMA time.
  constexpr bool kTwoSets = BM * BN <= 128 * 128;
  u32x4 rs[S_LOADS];
  u32x4 rb[kTwoSets ? B_LOADS : 1];
  const __bf16* A1 = reinterpret_cast<const __bf16*>(a.A1);
  const __bf16* A2 = reinterpret_cast<const __bf16*>(a.A2);
  const __bf16* Wp = reinterpret_cast<const __bf16*>(a.W);

  auto gload_a = [&](int kt) {
    const int k0 = kt * BK;
    const __bf16* src;
    int ld, kk0;
    if (k0 < a.K1) {
      src = A1;
      ld = a.lda1;
      kk0 = k0;
    } else {
      src = A2;
      ld = a.lda2;
      kk0 = k0 - a.K1;
    }
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int e = tid + NT * i;
      const int row = e >> 3, c8 = e & 7;
      const int gm = m0 + row;
      rs[i] = gm < M ? *reinterpret_cast<const u32x4*>(src + (size_t)gm * ld + kk0 + 8 * c8)
                     : (u32x4){0u, 0u, 0u, 0u};
    }
  };
  auto gload_b = [&](int kt, u32x4* dst) {
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int e = tid + NT * i;
      const int row = e >> 3, c8 = e & 7;
      dst[i] = *reinterpret_cast<const u32x4*>(Wp + (size_t)(n0 + row) * a.ldw + k0 + 8 * c8);
    }
  };
  auto sstore_a = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int e = tid + NT * i;
      *reinterpret_cast<u32x4*>(&As[buf * BM * LD + (e >> 3) * LD + 8 * (e & 7)]) = rs[i];
    }
  };
  auto sstore_b = [&](int buf, const u32x4* src) {
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int e = tid + NT * i;
      *reinterpret_cast<u32x4*>(&Bs[buf * BN * LD + (e >> 3) * LD + 8 * (e & 7)]) = src[i];
    }
  };

  f32x16 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int h = lane >> 5, l32 = lane & 31;
  const int wrow = wm * (BM / WM), wcol = wn * (BN / WN);
  // operand fragments of one 16-wide k step, double-buffered across the steps
  bf16x8 av[2][TI], bv[2][TJ];
  auto load_frags = [&](int buf, int kk, int q) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
      av[q][i] = *reinterpret_cast<const bf16x8*>(&As[buf * BM * LD + (wrow + 32 * i + l32) * LD + kk + 8 * h]);
#pragma unroll
    for (int j = 0; j < TJ; ++j)
      bv[q][j] = *reinterpret_cast<const bf16x8*>(&Bs[buf * BN * LD + (wcol + 32 * j + l32) * LD + kk + 8 * h]);
  };
  auto mfmas = [&](int q) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        if constexpr (F16)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[q][i]),
                                                              __builtin_bit_cast(f16x8, bv[q][j]),
                                                              acc[i][j], 0, 0, 0);
        else
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[q][i], bv[q][j], acc[i][j], 0, 0, 0);
  };

  gload_a(0);
  sstore_a(0);
  gload_b(0, rs);
  sstore_b(0, rs);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if constexpr (kTwoSets) {
      if (more) {
        gload_a(kt + 1);
        gload_b(kt + 1, rb);
      }
      load_frags(buf, 0, 0);
      load_frags(buf, 16, 1);
      mfmas(0);
      load_frags(buf, 32, 0);
      mfmas(1);
      load_frags(buf, 48, 1);
      mfmas(0);
      mfmas(1);
      // the other buffer was last read before the previous barrier
      if (more) {
        sstore_a(buf ^ 1);
        sstore_b(buf ^ 1, rb);
      }
    } else {
      if (more) gload_a(kt + 1);
      load_frags(buf, 0, 0);
      load_frags(buf, 16, 1);
      mfmas(0);
      load_frags(buf, 32, 0);
      mfmas(1);
      // the other buffer was last read before the previous barrier: stage A there, then
      // reuse the staging registers for B
      if (more) {
        sstore_a(buf ^ 1);
        gload_b(kt + 1, rs);
      }
      load_frags(buf, 48, 1);
      mfmas(0);
      mfmas(1);
      if (more) sstore_b(buf ^ 1, rs);
    }
    __syncthreads();
  }
  if constexpr (OUT16) {
    // the loop's last barrier has retired every read of the operand stages: stage the
    // converted tile there (row-major, LDT per row), then write whole rows with 16-byte
    // stores instead of one 2-byte store per element
    constexpr int LDT = BN + 8;
    static_assert(BM * LDT <= SMEM, "output tile exceeds the operand stages");
    uint16_t* T = reinterpret_cast<uint16_t*>(smem);
    bool big = false;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        big |= stage_block<F16 ? FMT_F16 : FMT_BF16>(a, acc[i][j], m0, wrow + 32 * i,
                                                     n0 + wcol + 32 * j, wcol + 32 * j, lane, M, T,
                                                     LDT);
    if (F16 && big && a.ovf) atomicOr(a.ovf, 1u);
    __syncthreads();
    constexpr int CPR = BN / 8;   // 16-byte chunks per tile row
    uint16_t* Cg = reinterpret_cast<uint16_t*>(a.C);
#pragma unroll 4
    for (int e = tid; e < BM * CPR; e += NT) {
      const int r = e / CPR, c8 = e - (e / CPR) * CPR;
      if (m0 + r < M)
        *reinterpret_cast<u32x4*>(Cg + (size_t)(m0 + r) * a.ldc + n0 + 8 * c8) =
            *reinterpret_cast<const u32x4*>(T + r * LDT + 8 * c8);
    }
  } else {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        store_block<FMT_F32>(a, acc[i][j], m0 + wrow + 32 * i, n0 + wcol + 32 * j, lane, M);
  }
  if (PERSIST) __syncthreads();   // LDS is reused by the next tile
  }
}

// ------------------------------------------------------------------ FP32 from FP16 x 3
// An FP32-accurate product on the FP16 MFMA (v_mfma_f32_32x32x16_f16): every operand x
// is split into x_hi = f16(x) and x_lo = f16((x - x_hi) * 2^11), and
//   sum_k a w = sum_k a_hi w_hi + 2^-11 sum_k (a_hi w_lo + a_lo w_hi)
// up to the dropped a_lo w_lo term (relative 2^-22), with the two sums in separate FP32
// accumulators.  A arrives as FP32 and is split while it is staged into LDS; W arrives as
// its hi / lo copies (W, Wlo).  Values must lie in the binary16 range: an A value outside
// it sets *a.ovf (the caller then re-runs in FP32).  BK = 32 or 64; every variant walks k
// in the same 16-wide steps in the same order.
template <int BM, int BN, int WM, int WN, int MINB, int NT = 256, int BK = 32, bool PERSIST = false>
__global__ void __launch_bounds__(NT, MINB) k_gemm_x3(GemmArgs a) {
  constexpr int LD = BK + 8;   // halves per LDS row
  constexpr int CA = BK / 4, CB = BK / 8;   // 16-byte chunks per staged A / W row
  constexpr int TI = BM / WM / 32, TJ = BN / WN / 32;
  // per stage: A hi, A lo, W hi, W lo
  __shared__ __attribute__((aligned(16))) _Float16 smem[2 * 2 * (BM + BN) * LD];
  auto Ah = [&](int b) { return smem + (size_t)b * 2 * (BM + BN) * LD; };
  auto Al = [&](int b) { return Ah(b) + BM * LD; };
  auto Bh = [&](int b) { return Ah(b) + 2 * BM * LD; };
  auto Bl = [&](int b) { return Ah(b) + 2 * BM * LD + BN * LD; };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int M = a.M_dev ? min(a.M, (int)*a.M_dev) : a.M;
  // persistent launches stride over the tiles of the device-side row count; others
  // take the one tile of their workgroup
  const int nby = a.N / BN;
  const int n_ids = PERSIST ? tiles_of(M, BM, nby) : 1;
  for (int id = PERSIST ? (int)blockIdx.x : 0; id < n_ids; id += PERSIST ? (int)gridDim.x : 1) {
  int rt, ct;
  if (PERSIST) tile_of_id(id, nby, rt, ct);
  else tile_of_block(rt, ct);
  const int m0 = rt * BM, n0 = ct * BN;
  if (m0 >= M) continue;
  const int K = a.K1 + a.K2;
  const int nk = K / BK;
  constexpr int A_LOADS = BM * (BK / 4) / NT;   // f32x4 per thread
  constexpr int B_LOADS = BN * (BK / 8) / NT;   // u32x4 (8 halves) per thread, each of hi / lo
  f32x4 ra[A_LOADS];
  u32x4 rbh[B_LOADS], rbl[B_LOADS];
  const float* A1 = reinterpret_cast<const float*>(a.A1);
  const float* A2 = reinterpret_cast<const float*>(a.A2);
  const uint16_t* Wh = reinterpret_cast<const uint16_t*>(a.W);
  const uint16_t* Wl = reinterpret_cast<const uint16_t*>(a.Wlo);

  auto gload = [&](int kt) {
    const int k0 = kt * BK;
    const float* src;
    int ld, kk0;
    if (k0 < a.K1) {
      src = A1;
      ld = a.lda1;
      kk0 = k0;
    } else {
      src = A2;
      ld = a.lda2;
      kk0 = k0 - a.K1;
    }
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int e = tid + NT * i;
      const int row = e / CA, c4 = e % CA;
      const int gm = m0 + row;
      ra[i] = gm < M ? *reinterpret_cast<const f32x4*>(src + (size_t)gm * ld + kk0 + 4 * c4)
                     : (f32x4){0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int e = tid + NT * i;
      const int row = e / CB, c8 = e % CB;
      const size_t o = (size_t)(n0 + row) * a.ldw + k0 + 8 * c8;
      rbh[i] = *reinterpret_cast<const u32x4*>(Wh + o);
      rbl[i] = *reinterpret_cast<const u32x4*>(Wl + o);
    }
  };
  bool big = false;   // an A operand outside the binary16 range (reported through a.ovf)
  auto sstore = [&](int b) {
    _Float16* ah = Ah(b);
    _Float16* al = Al(b);
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int e = tid + NT * i;
      const int at = (e / CA) * LD + 4 * (e % CA);
      typedef _Float16 h4 __attribute__((ext_vector_type(4)));
      h4 hi, lo;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const _Float16 x = (_Float16)ra[i][q];
        hi[q] = x;
        lo[q] = (_Float16)((ra[i][q] - (float)x) * 2048.f);
        big |= !(__builtin_fabsf(ra[i][q]) <= kF16Max);
      }
      *reinterpret_cast<h4*>(ah + at) = hi;
      *reinterpret_cast<h4*>(al + at) = lo;
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int e = tid + NT * i;
      const int at = (e / CB) * LD + 8 * (e % CB);
      *reinterpret_cast<u32x4*>(Bh(b) + at) = rbh[i];
      *reinterpret_cast<u32x4*>(Bl(b) + at) = rbl[i];
    }
  };

  f32x16 am[TI][TJ], ac[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) am[i][j][r] = ac[i][j][r] = 0.f;

  gload(0);
  sstore(0);
  __syncthreads();
  const int h = lane >> 5, l32 = lane & 31;
  const int wrow = wm * (BM / WM), wcol = wn * (BN / WN);
  for (int kt = 0; kt < nk; ++kt) {
    const int b = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) gload(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      f16x8 ahv[TI], alv[TI], bhv[TJ], blv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const int at = (wrow + 32 * i + l32) * LD + kk + 8 * h;
        ahv[i] = *reinterpret_cast<const f16x8*>(Ah(b) + at);
        alv[i] = *reinterpret_cast<const f16x8*>(Al(b) + at);
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int at = (wcol + 32 * j + l32) * LD + kk + 8 * h;
        bhv[j] = *reinterpret_cast<const f16x8*>(Bh(b) + at);
        blv[j] = *reinterpret_cast<const f16x8*>(Bl(b) + at);
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          am[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahv[i], bhv[j], am[i][j], 0, 0, 0);
          ac[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahv[i], blv[j], ac[i][j], 0, 0, 0);
          ac[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alv[i], bhv[j], ac[i][j], 0, 0, 0);
        }
    }
    if (more) sstore(b ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      f32x16 v;
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = am[i][j][r] + ac[i][j][r] * (1.f / 2048.f);
      store_block<FMT_F32>(a, v, m0 + wrow + 32 * i, n0 + wcol + 32 * j, lane, M);
    }
  if (big && a.ovf) atomicOr(a.ovf, 1u);
  if (PERSIST) __syncthreads();   // LDS is reused by the next tile
  }
}

// Copies the first K columns of a row-major [N][ldw_src] fp32 weight matrix into a
// dense [N][K] operand matrix of format fmt (FMT_*); FMT_F16 flags values outside the
// binary16 range in *ovf.  Element i of the dense matrix:
__device__ inline void pack_element(const float* __restrict__ W, int ldw_src, int K, size_t i,
                                    void* __restrict__ dst, int fmt, uint32_t* __restrict__ ovf) {
  const int n = (int)(i / K), k = (int)(i - (size_t)n * K);
  const float v = W[(size_t)n * ldw_src + k];
  if (fmt == FMT_BF16) {
    reinterpret_cast<uint16_t*>(dst)[i] = f32_to_bf16_bits(v);
  } else if (fmt == FMT_F16) {
    reinterpret_cast<uint16_t*>(dst)[i] = f32_to_f16_bits(v);
    if (!(__builtin_fabsf(v) <= kF16Max) && ovf) atomicOr(ovf, 1u);
  } else if (fmt == FMT_F16LO) {
    // the residual of the binary16 copy, scaled by 2^11 (FP16 x 3 products)
    const _Float16 hi = (_Float16)v;
    reinterpret_cast<uint16_t*>(dst)[i] = f32_to_f16_bits((v - (float)hi) * 2048.f);
  } else {
    reinterpret_cast<float*>(dst)[i] = v;
  }
}

__global__ void k_pack_weights(const float* __restrict__ W, int N, int ldw_src, int K,
                               void* __restrict__ dst, int fmt, uint32_t* __restrict__ ovf) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)N * K) return;
  pack_element(W, ldw_src, K, i, dst, fmt, ovf);
}

void launch_pack_weights(const float* W, int N, int ldw_src, int K, void* dst, int fmt,
                         hipStream_t s, uint32_t* ovf) {
  size_t n = (size_t)N * K;
  if (n)
    hipLaunchKernelGGL(k_pack_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, N,
                       ldw_src, K, dst, fmt, ovf);
}

// Every copy of a network's preparation in one launch: workgroup row y takes job y.
__global__ void k_pack_many(PackJobs jobs) {
  const PackJob& J = jobs.j[blockIdx.y];
  const size_t tot = (size_t)J.N * J.K;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (size_t)gridDim.x * blockDim.x)
    pack_element(J.W, J.ldw, J.K, i, J.dst, J.fmt, J.ovf);
}

void launch_pack_many(const PackJobs& jobs, hipStream_t s) {
  if (!jobs.n) return;
  size_t most = 0;
  for (int q = 0; q < jobs.n; ++q) most = std::max(most, (size_t)jobs.j[q].N * jobs.j[q].K);
  const unsigned gx = (unsigned)std::min<size_t>((most + 255) / 256, 256);
  hipLaunchKernelGGL(k_pack_many, dim3(gx, (unsigned)jobs.n), dim3(256), 0, s, jobs);
}

// ------------------------------------------------------------------ FP8 (OCP e4m3) operands
// v_mfma_scale_f32_32x32x64_f8f6f4 with both formats e4m3 and unit block scales
// (E8M0 127): 32 fp8 values per lane per MFMA (two 16-byte LDS reads).  A arrives
// as bf16 and is quantized while it is staged into LDS (e4m3(a / s_a), saturating);
// W is pre-quantized per layer; the epilogue multiplies by s_a * s_w.
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline uint32_t quant4(uint32_t lo2, uint32_t hi2, float inv) {
  // two uint32 holding 4 bf16 values -> 4 e4m3 bytes
  const uint32_t b0 = f32_to_e4m3(bf16_to_f32((uint16_t)(lo2 & 0xffff)) * inv);
  const uint32_t b1 = f32_to_e4m3(bf16_to_f32((uint16_t)(lo2 >> 16)) * inv);
  const uint32_t b2 = f32_to_e4m3(bf16_to_f32((uint16_t)(hi2 & 0xffff)) * inv);
  const uint32_t b3 = f32_to_e4m3(bf16_to_f32((uint16_t)(hi2 >> 16)) * inv);
  return b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
}

template <int BM, int BN, int WM, int WN, int MINB, bool OUT_BF16, int BK>
__global__ void __launch_bounds__(256, MINB) k_gemm_fp8(GemmArgs a) {
  // BK fp8 bytes (= elements) per stage: 128, or 64 when a K range is not a multiple of 128
  constexpr int LD = BK + 16;    // bytes
  constexpr int TI = BM / WM / 32, TJ = BN / WN / 32;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][BN * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int rt, ct;
  tile_of_block(rt, ct);
  const int m0 = rt * BM, n0 = ct * BN;
  const int M = a.M_dev ? min(a.M, (int)*a.M_dev) : a.M;
  if (m0 >= M) return;
  const int K = a.K1 + a.K2;
  const int nk = K / BK;
  // A: BM rows x BK bf16 = BK/8 uint4 per row; B: BN rows x BK bytes = BK/16 uint4 per row
  constexpr int AV = BK / 8, BV = BK / 16;
  constexpr int A_LOADS = BM * AV / 256;
  constexpr int B_LOADS = BN * BV / 256 > 0 ? BN * BV / 256 : 1;
  u32x4 ra[A_LOADS], rb[B_LOADS];
  const uint16_t* A1 = reinterpret_cast<const uint16_t*>(a.A1);
  const uint16_t* A2 = reinterpret_cast<const uint16_t*>(a.A2);
  const uint8_t* Wp = reinterpret_cast<const uint8_t*>(a.W);
  const float inv = a.a_inv_scale;

  auto gload = [&](int kt) {
    const int k0 = kt * BK;
    const uint16_t* src;
    int ld, kk0;
    if (k0 < a.K1) {
      src = A1;
      ld = a.lda1;
      kk0 = k0;
    } else {
      src = A2;
      ld = a.lda2;
      kk0 = k0 - a.K1;
    }
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int e = tid + 256 * i;
      const int row = e / AV, c8 = e % AV;
      const int gm = m0 + row;
      ra[i] = gm < M ? *reinterpret_cast<const u32x4*>(src + (size_t)gm * ld + kk0 + 8 * c8)
                       : (u32x4){0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int e = tid + 256 * i;
      const int row = e / BV, c16 = e % BV;
      if (row < BN)
        rb[i] = *reinterpret_cast<const u32x4*>(Wp + (size_t)(n0 + row) * a.ldw + k0 + 16 * c16);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int e = tid + 256 * i;
      const int row = e / AV, c8 = e % AV;
      uint2 q;
      q.x = quant4(ra[i].x, ra[i].y, inv);
      q.y = quant4(ra[i].z, ra[i].w, inv);
      *reinterpret_cast<uint2*>(&As[buf][row * LD + 8 * c8]) = q;
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int e = tid + 256 * i;
      if (e / BV < BN) *reinterpret_cast<u32x4*>(&Bs[buf][(e / BV) * LD + 16 * (e % BV)]) = rb[i];
    }
  };

  f32x16 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  gload(0);
  sstore(0);
  __syncthreads();
  const int h = lane >> 5, l32 = lane & 31;
  const int wrow = wm * (BM / WM), wcol = wn * (BN / WN);
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 64) {
      i32x8 av[TI], bv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const uint8_t* p = &As[buf][(wrow + 32 * i + l32) * LD + kk + 32 * h];
        const uint4 x0 = *reinterpret_cast<const uint4*>(p);
        const uint4 x1 = *reinterpret_cast<const uint4*>(p + 16);
        av[i] = (i32x8){(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w,
                        (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const uint8_t* p = &Bs[buf][(wcol + 32 * j + l32) * LD + kk + 32 * h];
        const uint4 x0 = *reinterpret_cast<const uint4*>(p);
        const uint4 x1 = *reinterpret_cast<const uint4*>(p + 16);
        bv[j] = (i32x8){(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w,
                        (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av[i], bv[j], acc[i][j], 0, 0,
                                                                      0, 127, 0, 127);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
      store_block<OUT_BF16 ? FMT_BF16 : FMT_F32>(a, acc[i][j], m0 + wrow + 32 * i, n0 + wcol + 32 * j,
                                                 lane, M);
}

// Per-layer weight quantization: dst = e4m3(W / s_w) for the first K columns, where
// s_w = amax / 448 comes from *amax_bits (an atomicMax over |W| as float bits).
__global__ void k_absmax(const float* __restrict__ W, int N, int ldw, int K,
                         uint32_t* __restrict__ amax_bits) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float v = 0.f;
  if (i < (size_t)N * K) {
    const int n = (int)(i / K), k = (int)(i - (size_t)n * K);
    v = fabsf(W[(size_t)n * ldw + k]);
  }
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(amax_bits, __float_as_uint(v));
}

void launch_absmax(const float* X, int rows, int ld, int K, uint32_t* amax_bits, hipStream_t s) {
  const size_t n = (size_t)rows * K;
  if (n)
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, rows, ld, K,
                       amax_bits);
}

__global__ void k_pack_fp8(const float* __restrict__ W, int N, int ldw, int K,
                           const uint32_t* __restrict__ amax_bits, uint8_t* __restrict__ dst) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)N * K) return;
  const float amax = __uint_as_float(*amax_bits);
  const float inv = amax > 0.f ? 448.f / amax : 1.f;
  const int n = (int)(i / K), k = (int)(i - (size_t)n * K);
  dst[i] = f32_to_e4m3(W[(size_t)n * ldw + k] * inv);
}

void launch_pack_fp8(const float* W, int N, int ldw, int K, uint32_t* amax_bits, uint8_t* dst,
                     hipStream_t s) {
  const size_t n = (size_t)N * K;
  if (!n) return;
  (void)hipMemsetAsync(amax_bits, 0, 4, s);
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, N, ldw, K,
                     amax_bits);
  hipLaunchKernelGGL(k_pack_fp8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, N, ldw, K,
                     amax_bits, dst);
}

// A GEMM launch, carrying the caller's event pair when it has one.
#define PIFU_GO(K, G, B, SH, ST, ...)                                                           \
  do {                                                                                           \
    if (ev0)                                                                                     \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, ev0, ev1, 0, __VA_ARGS__);                          \
    else                                                                                         \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                          \
  } while (0)

#define PIFU_H16(BM_, BN_, WM_, WN_, MB_, F16_)                                                  \
  do {                                                                                           \
    if (a.c_bf16)                                                                                \
      PIFU_GO((k_gemm_h16<BM_, BN_, WM_, WN_, MB_, true, F16_>),                      \
                         dim3(row_tiles(a.M, BM_), a.N / BN_), dim3(256), 0, s, a);             \
    else                                                                                         \
      PIFU_GO((k_gemm_h16<BM_, BN_, WM_, WN_, MB_, false, F16_>),                     \
                         dim3(row_tiles(a.M, BM_), a.N / BN_), dim3(256), 0, s, a);             \
  } while (0)

// FP32 tiles: 256: 256 x 128 (or 256 x 64) over eight waves; 128: 128 x 128 (or 128 x 64);
// 96: 128 x 64; 64: 64 x 64; 32: 32 x 64 tiles of two 32 x 32 waves (tiny launches spread
// over more CUs).  Every shape walks k in the same order.
template <bool TAPS>
void launch_f32(const GemmArgs& a, int bm, bool bn128, hipStream_t s, hipEvent_t ev0,
                hipEvent_t ev1) {
  if (bm == 32) {
    PIFU_GO((k_gemm_f32<32, 64, 1, 2, 2, 128, false, TAPS>), dim3(row_tiles(a.M, 32), a.N / 64),
            dim3(128), 0, s, a);
  } else if (bm == 256) {
    if (bn128)
      PIFU_GO((k_gemm_f32<256, 128, 4, 2, 1, 512, false, TAPS>), dim3(row_tiles(a.M, 256), a.N / 128),
              dim3(512), 0, s, a);
    else
      PIFU_GO((k_gemm_f32<256, 64, 4, 2, 1, 512, false, TAPS>), dim3(row_tiles(a.M, 256), a.N / 64),
              dim3(512), 0, s, a);
  } else if (bm == 128 && bn128) {
    PIFU_GO((k_gemm_f32<128, 128, 2, 2, 2, 256, false, TAPS>), dim3(row_tiles(a.M, 128), a.N / 128),
            dim3(256), 0, s, a);
  } else if (bm == 128 || bm == 96) {
    PIFU_GO((k_gemm_f32<128, 64, 2, 2, 2, 256, false, TAPS>), dim3(row_tiles(a.M, 128), a.N / 64),
            dim3(256), 0, s, a);
  } else {
    PIFU_GO((k_gemm_f32<64, 64, 2, 2, 2, 256, false, TAPS>), dim3(row_tiles(a.M, 64), a.N / 64),
            dim3(256), 0, s, a);
  }
}

template <bool F16>
void launch_h16(const GemmArgs& a, int bm, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const bool bn128 = (a.N % 128) == 0;
  // 64-point tiles (launches too small for the chip with 128-point ones) take 64 x 64
  // outputs: twice the workgroups of 64 x 128, measured faster at every such size
  // (e.g. layer 1, 2k / 5k / 12k points: 10.9 / 15.6 / 30.8 us against 14.4 / 18.8 / 37.6)
  if (bm == 64) {
    PIFU_H16(64, 64, 2, 2, 2, F16);
    return;
  }
  if (bn128) {
    if (bm == 128) PIFU_H16(128, 128, 2, 2, 2, F16);
    else if (a.N % 256 == 0) {
      // 256 x 256 tile, 8 waves: half the L2 traffic per FLOP of the 128-wide tiles
      if (a.c_bf16)
        PIFU_GO((k_gemm_h16<256, 256, 2, 4, 1, true, F16, 512>),
                           dim3(row_tiles(a.M, 256), a.N / 256), dim3(512), 0, s, a);
      else
        PIFU_GO((k_gemm_h16<256, 256, 2, 4, 1, false, F16, 512>),
                           dim3(row_tiles(a.M, 256), a.N / 256), dim3(512), 0, s, a);
    } else PIFU_H16(256, 128, 2, 2, 1, F16);
  } else {
    if (bm == 128) PIFU_H16(128, 64, 4, 1, 2, F16);
    else PIFU_H16(256, 64, 4, 1, 1, F16);
  }
}
#undef PIFU_H16

// Whether an FP32 tile is finished through LDS, four columns at a time (GemmArgs::ep_vec):
// where every array it reads or writes that way is 16-byte aligned, for the launches it
// speeds up (measured on the layer shapes: the tap blend 2-7% and the extra columns 0-7%
// faster; hoisted rows and plain bias within 1-4% either way, so they keep the block
// epilogue).
bool vec_epilogue_ok(const GemmArgs& a) {
  if (!a.tap_idx && a.n_ext <= 0) return false;
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if ((a.N % 4) || (a.ldc % 4) || !al(a.C) || (a.bias && !al(a.bias))) return false;
  if (a.rowadd && (!al(a.rowadd) || (a.rowadd_ld % 4) || (a.rowadd_off % 4))) return false;
  if (a.rowmul && (!al(a.rowmul) || (a.rowmul_off % 4))) return false;
  return true;
}

// Persistent launch for a device-side row count (a.M_dev; a.M is the capacity): one tile
// shape per precision, a 1-D grid of at most kPersistBlocks workgroups striding over the
// tiles.  Same k order as every other tile, so the same results.
int launch_gemm_persist(const GemmArgs& a, int precision, hipStream_t s) {
  if (a.M <= 0) return 0;
  const bool bn128 = (a.N % 128) == 0;
  if (!bn128 && (a.N % 64) != 0) return -1;
  auto grid = [&](int bm, int bn) {
    size_t t = (size_t)row_tiles(a.M, bm) * (a.N / bn);
    if (t > kPersistBlocks) t = kPersistBlocks;
    return dim3((unsigned)t);   // row_tiles is a multiple of 8, so is t
  };
  if (precision == PIFU_PREC_FP32) {
    if ((a.K1 % 32) || (a.K2 % 32)) return -1;
    if (bn128 && a.tap_idx)
      hipLaunchKernelGGL((k_gemm_f32<128, 128, 2, 2, 2, 256, true, true>), grid(128, 128), dim3(256), 0, s, a);
    else if (bn128)
      hipLaunchKernelGGL((k_gemm_f32<128, 128, 2, 2, 2, 256, true>), grid(128, 128), dim3(256), 0, s, a);
    else if (a.tap_idx)
      hipLaunchKernelGGL((k_gemm_f32<128, 64, 4, 1, 2, 256, true, true>), grid(128, 64), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_gemm_f32<128, 64, 4, 1, 2, 256, true>), grid(128, 64), dim3(256), 0, s, a);
    return 0;
  }
  if (precision == PREC_F32X3) {
    if ((a.K1 % 32) || (a.K2 % 32)) return -1;
    hipLaunchKernelGGL((k_gemm_x3<64, 64, 2, 2, 2, 256, 32, true>), grid(64, 64), dim3(256), 0, s, a);
    return 0;
  }
  if (precision == PIFU_PREC_BF16 || precision == PIFU_PREC_FP16) {
    if ((a.K1 % 64) || (a.K2 % 64)) return -1;
    const bool f16 = precision == PIFU_PREC_FP16;
#define PIFU_HP(BN_, WM_, WN_)                                                                    \
  do {                                                                                           \
    if (f16 && a.c_bf16)                                                                         \
      hipLaunchKernelGGL((k_gemm_h16<128, BN_, WM_, WN_, 2, true, true, 256, true>), grid(128, BN_), \
                         dim3(256), 0, s, a);                                                    \
    else if (f16)                                                                                \
      hipLaunchKernelGGL((k_gemm_h16<128, BN_, WM_, WN_, 2, false, true, 256, true>),           \
                         grid(128, BN_), dim3(256), 0, s, a);                                    \
    else if (a.c_bf16)                                                                           \
      hipLaunchKernelGGL((k_gemm_h16<128, BN_, WM_, WN_, 2, true, false, 256, true>),           \
                         grid(128, BN_), dim3(256), 0, s, a);                                    \
    else                                                                                         \
      hipLaunchKernelGGL((k_gemm_h16<128, BN_, WM_, WN_, 2, false, false, 256, true>),          \
                         grid(128, BN_), dim3(256), 0, s, a);                                    \
  } while (0)
    if (bn128) PIFU_HP(128, 2, 2);
    else PIFU_HP(64, 4, 1);
#undef PIFU_HP
    return 0;
  }
  return -1;   // FP8 runs read their weight scales back on the host: no persistent form
}

int launch_gemm(const GemmArgs& a_in, int precision, int tile_m, hipStream_t s, hipEvent_t ev0,
                hipEvent_t ev1) {
  GemmArgs a = a_in;
  a.ep_vec = precision == PIFU_PREC_FP32 && vec_epilogue_ok(a_in);
  if (a.M <= 0) return 0;
  const bool bn128 = (a.N % 128) == 0;
  if (!bn128 && (a.N % 64) != 0) return -1;
  int bm = tile_m == 64 ? 64 : (tile_m == 256 ? 256 : (tile_m == 32 ? 32 : (tile_m == 96 ? 96 : 128)));
  if (precision == PIFU_PREC_FP32) {
    if ((a.K1 % 32) || (a.K2 % 32)) return -1;
    if (a.tap_idx) launch_f32<true>(a, bm, bn128, s, ev0, ev1);
    else launch_f32<false>(a, bm, bn128, s, ev0, ev1);
    return 0;
  }
  if (precision == PREC_F32X3) {
    // one shape for every launch: 64 x 64 tiles of four 32 x 32 waves, at most 128
    // registers (four workgroups per CU) so that four waves fit per SIMD (with 140
    // registers and three waves the band launches ran 6-9% longer; a 128 x 128 tile holds
    // both accumulator sets in 369 registers, one wave per SIMD, and ran 1.3-1.7x slower
    // at every band size measured; 128 x 64 tiles ran as fast as 64 x 64)
    if ((a.K1 % 32) || (a.K2 % 32)) return -1;
    // a launch that fits one round at two workgroups per CU and has a deep contraction
    // takes 64-deep k stages (half the stages of its latency chain; e.g. layer 1 at 1k /
    // 3k points 24.4 / 33.5 -> 20.6 / 27.2 us); larger ones keep 32-deep stages, whose
    // smaller LDS footprint doubles the workgroups per CU (8k points: 42 vs 52 us)
    const unsigned rows = row_tiles(a.M, 64);
    if ((a.K1 % 64) == 0 && (a.K2 % 64) == 0 && a.K1 + a.K2 >= 512 &&
        (size_t)rows * (a.N / 64) <= 512)
      PIFU_GO((k_gemm_x3<64, 64, 2, 2, 2, 256, 64>), dim3(rows, a.N / 64), dim3(256), 0, s, a);
    else
      PIFU_GO((k_gemm_x3<64, 64, 2, 2, 4>), dim3(rows, a.N / 64), dim3(256), 0, s, a);
    return 0;
  }
  if (bm == 32) bm = 64;   // the 32-point tile exists for FP32 only
  if (bm == 96) bm = 128;  // so does the 128 x 64 choice
  if (precision == PIFU_PREC_BF16 || precision == PIFU_PREC_FP16) {
    if ((a.K1 % 64) || (a.K2 % 64)) return -1;
    if (precision == PIFU_PREC_FP16) launch_h16<true>(a, bm, s, ev0, ev1);
    else launch_h16<false>(a, bm, s, ev0, ev1);
    return 0;
  }
  if (precision == PIFU_PREC_FP8) {
    const bool k128 = (a.K1 % 128) == 0 && (a.K2 % 128) == 0;
    if ((a.K1 % 64) || (a.K2 % 64)) return -1;
#define PIFU_F8(BM_, BN_, WM_, WN_, MB_, BK_)                                                    \
  do {                                                                                           \
    if (a.c_bf16)                                                                                \
      PIFU_GO((k_gemm_fp8<BM_, BN_, WM_, WN_, MB_, true, BK_>),                       \
                         dim3(row_tiles(a.M, BM_), a.N / BN_), dim3(256), 0, s, a);             \
    else                                                                                         \
      PIFU_GO((k_gemm_fp8<BM_, BN_, WM_, WN_, MB_, false, BK_>),                      \
                         dim3(row_tiles(a.M, BM_), a.N / BN_), dim3(256), 0, s, a);             \
  } while (0)
    if (k128) {
      if (bn128) {
        if (bm == 64) PIFU_F8(64, 128, 1, 4, 2, 128);
        else if (bm == 128) PIFU_F8(128, 128, 2, 2, 2, 128);
        else PIFU_F8(256, 128, 2, 2, 1, 128);
      } else {
        if (bm == 64) PIFU_F8(64, 64, 2, 2, 2, 128);
        else if (bm == 128) PIFU_F8(128, 64, 4, 1, 2, 128);
        else PIFU_F8(256, 64, 4, 1, 1, 128);
      }
    } else {
      if (bn128) {
        if (bm == 64) PIFU_F8(64, 128, 1, 4, 2, 64);
        else if (bm == 128) PIFU_F8(128, 128, 2, 2, 2, 64);
        else PIFU_F8(256, 128, 2, 2, 1, 64);
      } else {
        if (bm == 64) PIFU_F8(64, 64, 2, 2, 2, 64);
        else if (bm == 128) PIFU_F8(128, 64, 4, 1, 2, 64);
        else PIFU_F8(256, 64, 4, 1, 1, 64);
      }
    }
#undef PIFU_F8
    return 0;
  }
  return -1;
}

}  // namespace pifu
