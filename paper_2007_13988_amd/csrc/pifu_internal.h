// Internal declarations shared by the libpifu translation units (kernels, GEMM, host).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pifu.h"

namespace pifu {

// Per-node state byte of a level lattice.
enum : uint8_t {
  ST_LABEL = 0x01,  // current binary label
  ST_EVAL = 0x02,   // evaluated by the network at this or a coarser level
  ST_B0 = 0x04,     // boundary candidate: interpolated value strictly between 0 and 1
  ST_HI = 0x08,     // interpolated value > 1/2 (the value the conflict test compares with)
  ST_PEND = 0x10,   // selected for evaluation, not evaluated yet
  ST_NOW = 0x20,    // evaluated at this level
  ST_CONF = 0x40,   // conflict: network label differs from the binarized interpolation
  ST_CELL = 0x80,   // final level: the cell with this node as lowest corner is mixed
};

struct Lat {
  int nx, ny, nz;
  __host__ __device__ size_t n() const { return (size_t)nx * ny * nz; }
};

// Where the points of an evaluation come from.
//   mode 0: lattice nodes; point m is node list[m] of lattice (nx, ny, nz),
//           optionally mapped by the 3x4 view (target NDC -> input NDC).
//   mode 1: explicit points pts[list ? list[m] : m] (x, y, z, occ), input NDC.
//   base_sub is subtracted from every list entry first (a frame's offset inside a
//   multi-frame state array).
//   frame_nodes > 0 (mode 0): entries index frames of frame_nodes nodes stored back to
//   back; frame f samples the feature map feat_tab[f].
constexpr int kMaxTabFrames = 16;
struct PointSrc {
  int mode;
  int nx, ny, nz;
  int has_view;
  double view[12];
  const float4* pts;
  uint32_t base_sub;
  uint32_t frame_nodes;
  const float* feat_tab[kMaxTabFrames];
};

struct MLPDesc {
  int n_layers, feat_dim, n_extra, hidden_act, out_act;
  int widths[PIFU_MAX_LAYERS];
  int skip[PIFU_MAX_LAYERS];
  int in_w[PIFU_MAX_LAYERS];
  const float* W[PIFU_MAX_LAYERS];
  const float* b[PIFU_MAX_LAYERS];
};

struct Ellipsoids {
  int n;
  float k;
  float e[PIFU_MAX_ELLIPSOIDS * 12];
};

// float32 -> bfloat16 bits, round to nearest even (NaN stays a quiet NaN).
__host__ __device__ inline uint16_t f32_to_bf16_bits(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// float32 -> IEEE binary16 bits, round to nearest even (overflow gives infinity).
__host__ __device__ inline uint16_t f32_to_f16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (_Float16)x);
}

// Largest finite binary16 magnitude: a value above it does not convert faithfully.
constexpr float kF16Max = 65504.f;

// Storage format of an MLP operand or activation array (FMT_F16LO: the binary16 residual
// x - f16(x), scaled by 2^11, of an FP16 x 3 operand).
enum { FMT_F32 = 0, FMT_BF16 = 1, FMT_F16 = 2, FMT_F16LO = 3 };
// Internal run precision: FP32-accurate GEMMs from three FP16 MFMA products per k step
// (operands split into binary16 hi and scaled lo parts); FP32 activations.
constexpr int PREC_F32X3 = 16;
// The 16-bit format a run precision stores activations in (FP8 stages bf16 values).
inline int h16_fmt(int precision) {
  return precision == PIFU_PREC_FP32 ? FMT_F32 : precision == PIFU_PREC_FP16 ? FMT_F16 : FMT_BF16;
}

// Blocks of a list kernel whose length lives on the device: the grid strides over it.
constexpr unsigned kStrideBlocks = 1024;

constexpr int COMPACT_BLOCK = 256;
constexpr int COMPACT_PER_THREAD = 16;
constexpr int COMPACT_TILE = COMPACT_BLOCK * COMPACT_PER_THREAD;

// ------------------------------------------------------------------ level kernels
void launch_fill_u8(uint8_t* p, uint8_t v, size_t n, hipStream_t s);
// Counter updates of the device-driven calls, applied in order by one thread:
//   ADD: *dst += *src;  ADD_NZ: *dst += (*src != 0);  SET: *dst = *src;  SET_IMM: *dst = imm;
//   FLAG_GT: *dst |= bit if *src > imm;  SEL: *dst = *aux ? *src : 0;
//   ADD_SEL: *dst += *aux ? *src : *src2  (a null src / src2 reads 0, a null aux is true)
enum { BK_ADD, BK_ADD_NZ, BK_SET, BK_SET_IMM, BK_FLAG_GT, BK_SEL, BK_ADD_SEL };
struct BookOp {
  uint32_t* dst;
  const uint32_t* src;
  const uint32_t* src2;
  const uint32_t* aux;
  uint32_t imm, bit;
  int kind;
};
constexpr int kMaxBookOps = 12;
struct BookOps {
  BookOp op[kMaxBookOps];
  int n = 0;
};
void launch_book(const BookOps& b, hipStream_t s);
// p[0 .. n) = v by a kernel (graph-capturable, unlike hipMemsetAsync)
void launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s, uint32_t n = 1);
// host[0 .. n) = c[0 .. n) (host: device view of mapped fine-grained host memory), then
// *seq_word = seq once those stores are visible to the host
void launch_publish(const uint32_t* c, int n, uint32_t* host, uint32_t* seq_word, uint32_t seq,
                    hipStream_t s);
void launch_iota(uint32_t* list, uint32_t n, hipStream_t s);
void launch_occupancy(const float* logit, uint32_t n, float* occ, hipStream_t s);
// frames > 1: `frames` lattices stored back to back (coarse and fine), one grid row each.
// Frames of one batched call; per frame, where its occupancy goes at a level (null:
// the combined array's slice of that frame).
constexpr int kMaxBatch = 16;
struct FrameOcc {
  float* p[kMaxBatch];
};

void launch_transition(const uint8_t* cst, const float* cocc, Lat c, uint8_t* fst, float* focc,
                       Lat f, hipStream_t s, int frames = 1, const FrameOcc* fo = nullptr);
void launch_select(uint8_t* st, Lat f, hipStream_t s, int frames = 1);
// The same selection from bit masks of the boundary candidates, and their count per frame
// (counts[p * count_stride] += candidates of frame p).  masks: b0_mask_words(f) words per
// frame, 8-byte aligned scratch that nothing reads afterwards.
size_t b0_mask_words(Lat f);
void launch_select_b0(uint8_t* st, Lat f, int frames, uint64_t* masks, uint32_t* counts,
                      int count_stride, hipStream_t s);
// bounds[f] (f = 0..frames) = first list position with entry >= f * frame_nodes.
void launch_segment_bounds(const uint32_t* list, uint32_t n, uint32_t frame_nodes, int frames,
                           uint32_t* bounds, hipStream_t s);
// Stable compaction of the nodes whose state byte satisfies (st & mask) == val.
// mode 0 writes node indices (plus index_base), mode 1 cell indices (i*(nx-1)+j)*(nz... of
// lattice f).  st must be 16-byte aligned.
// gate (device, nullable): when *gate is 0 at the start, nothing is selected and the
// passes exit at once (total = 0); the gate may be the total word itself.
void launch_compact(const uint8_t* st, size_t n, uint8_t mask, uint8_t val, uint32_t* bcount,
                    uint32_t* total, uint32_t* out, uint32_t cap, int mode, Lat f, hipStream_t s,
                    uint32_t index_base = 0, const uint32_t* gate = nullptr);
size_t compact_scratch_words(size_t n);
void launch_apply_grid(const uint32_t* list, uint32_t n, const float* logit, const uint8_t* lab,
                       uint8_t* st, float* occ, uint32_t* conflicts, uint8_t* eval_level,
                       int level_id, Lat lvl, int stride, Lat fin, int check_conflict,
                       hipStream_t s, uint32_t frame_nodes = 0, const FrameOcc* fo = nullptr,
                       float* eval_logit = nullptr, const uint32_t* n_dev = nullptr);
// eval_level[list[m]] = level_id and eval_logit[list[m]] = logit[m] for m < n (list holds
// indices of the lattice the two maps cover)
void launch_trace_scatter(const uint32_t* list, uint32_t n, const float* logit, int level_id,
                          uint8_t* eval_level, float* eval_logit, hipStream_t s,
                          const uint32_t* n_dev = nullptr);
void launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
// frame_nodes > 0: list entries index a multi-frame state array of frames of that size.
void launch_expand(const uint32_t* list, uint32_t n, uint8_t* st, Lat f, hipStream_t s,
                   uint32_t frame_nodes = 0, const uint32_t* n_dev = nullptr);
void launch_cells(uint8_t* st, Lat f, uint8_t* labels, hipStream_t s);
// Per-frame counts of a list over frames of frame_nodes nodes (tally[f] +=; pos: the
// list positions to count, null for the first min(n, *n_dev) entries), then the stats
// updates that read them (FrameApply; BK_ADD, BK_ADD_NZ or BK_SET per op), which also
// clear the tally.
void launch_frame_tally(const uint32_t* list, const uint32_t* pos, uint32_t n,
                        const uint32_t* n_dev, uint32_t frame_nodes, uint32_t* tally,
                        hipStream_t s);
constexpr int kMaxFrameOps = 4;
struct FrameApply {
  int frames, nops;
  int kind[kMaxFrameOps];
  uint32_t* dst[kMaxFrameOps][kMaxBatch];
};
void launch_frame_apply(uint32_t* tally, const FrameApply& a, hipStream_t s);
void launch_count_bits(const uint8_t* st, size_t n, uint8_t bit, uint32_t* out, hipStream_t s);
// Octree-subdivision baselines: per coarse cell of lattice c, flags[cell] = subdivide
// (mode PIFU_OCTREE_*, threshold thr), *count += subdivided cells; then the fine level's
// state and values with ST_PEND on every node of a subdivided cell not evaluated before.
void launch_oct_flags(const uint8_t* cst, const float* cocc, Lat c, int mode, double thr,
                      uint8_t* flags, uint32_t* count, hipStream_t s);
void launch_oct_transition(const uint8_t* cst, const float* cocc, Lat c, const uint8_t* flags,
                           uint8_t* fst, float* focc, Lat f, int mode, hipStream_t s);

// ------------------------------------------------------------------ evaluation kernels
// List kernels below take an optional device-side count n_dev: the list then holds
// min(n, *n_dev) entries (n is its capacity) and the grid strides over them.
// ell_tab (device, nullable): with a multi-frame source, frame f's shapes are ell_tab[f].
void launch_eval_analytic(const PointSrc& src, const uint32_t* list, uint32_t n, int kind,
                          const Ellipsoids& ell, const float plane[4], float* logit,
                          uint8_t* lab, hipStream_t s, const uint32_t* n_dev = nullptr,
                          const Ellipsoids* ell_tab = nullptr);
// *dst = e, by a kernel (graph-capturable)
void launch_store_ellipsoids(Ellipsoids* dst, const Ellipsoids& e, hipStream_t s);
// Bilinear gather of C channels (Eq. 1's sampler) for points m in [0, n); writes
// feat (n x C, in format feat_fmt: FMT_F32 / FMT_BF16 / FMT_F16) and ext (n x 4: z',
// occ, clipped, 0).  n_dev (nullable): device-side point count <= n; the grid covers
// n points.  ovf (FMT_F16): set to 1 when a feature exceeds the binary16 range.
void launch_gather(const PointSrc& src, const uint32_t* list, uint32_t n, const float* F, int H,
                   int W, int C, void* feat, int feat_fmt, float* ext, hipStream_t s,
                   const uint32_t* n_dev = nullptr, uint32_t* ovf = nullptr);
void launch_head(const float* h, int K, const float* W, const float* b, int n_out, int out_act,
                 uint32_t n, const float* ext, float* logit, uint8_t* lab, float* rgb_out,
                 const uint32_t* rgb_index, hipStream_t s, const uint32_t* n_dev = nullptr);
// Positions m < n with |logit[m]| < g (any order) into glist (map[m] with a map).
// *gcount is a running counter that holds `start` before the launch: the positions go to
// glist[0 ..) and the count is *gcount - start afterwards (no reset between launches).
void launch_guard_select(const float* logit, uint32_t n, float g, uint32_t* glist,
                         uint32_t* gcount, hipStream_t s, const uint32_t* map = nullptr,
                         uint32_t start = 0, const uint32_t* n_dev = nullptr);

// out[i] = src[pos[i]]
void launch_gather_u32(const uint32_t* src, const uint32_t* pos, uint32_t n, uint32_t* out,
                       hipStream_t s, const uint32_t* n_dev = nullptr);
void launch_convert(const float* in, uint32_t n, int fmt, void* out, hipStream_t s);
// logit[pos[i]] = tl[i], lab[pos[i]] = tb[i]
void launch_scatter_results(const uint32_t* pos, uint32_t n, const float* tl, const uint8_t* tb,
                            float* logit, uint8_t* lab, hipStream_t s,
                            const uint32_t* n_dev = nullptr);
size_t guard64_ws_bytes(const MLPDesc& d, uint32_t chunk);
// pack: write the float64 weight copies into ws (once per call; later calls reuse them).
void run_guard64(const PointSrc& src, const uint32_t* list, const uint32_t* glist, uint32_t gn,
                 const MLPDesc& d, const float* F, int H, int W, int C, float* logit, uint8_t* lab,
                 void* ws, uint32_t chunk, bool pack, hipStream_t s,
                 const uint32_t* gn_dev = nullptr);

// ------------------------------------------------------------------ render kernels
void launch_ray_count(const uint8_t* stc, Lat c, int W, int H, int D, uint32_t* cnt,
                      uint32_t* kstar, uint32_t* shadow_total, hipStream_t s);
void launch_scan_u32(const uint32_t* in, uint32_t n, uint32_t* out_excl, uint32_t* scratch,
                     uint32_t* total, hipStream_t s, const uint32_t* n_dev = nullptr,
                     const uint32_t* gate = nullptr);
size_t scan_scratch_words(size_t n);
void launch_ray_list(const uint8_t* stc, Lat c, int W, int H, int D, const uint32_t* kstar,
                     const uint32_t* off, uint32_t* list, hipStream_t s);
// kstar_out / k1_out (nullable, image layout): the two argmax indices of each pixel
// (-1 where there is none)
void launch_ray_hit(const uint8_t* stc, const float* occc, Lat c, int W, int H, int D,
                    const uint32_t* off, const uint32_t* cnt, const uint32_t* list,
                    const float* logit, const uint8_t* lab, const double* view, float* depth,
                    uint8_t* hit, float4* hitpts, hipStream_t s, int32_t* kstar_out = nullptr,
                    int32_t* k1_out = nullptr);
void launch_fill_image(float* rgb, float* depth, uint8_t* hit, uint32_t npix, float bg0, float bg1,
                       float bg2, hipStream_t s);

// ------------------------------------------------------------------ GEMM (MFMA)
// C[m][n] = act(sum_k A[m][k] W[n][k] + b[n] + sum_e ext[m][e] W[n][ext_col + e]) for m < M,
// A = [A1 (K1 columns, ld lda1) ; A2 (K2 columns, ld lda2)].  precision selects the MFMA
// operand type; for BF16/FP16 A1, A2 and C are in that 16-bit format (FP8: bf16) and W is
// the pre-converted copy.
struct GemmArgs {
  const void* A1;
  int K1, lda1;
  const void* A2;
  int K2, lda2;
  const void* W;     // [N][ldw] operand copy (fp32 or bf16 / fp8)
  int ldw;
  const float* Wf;   // fp32 original (for the extras columns)
  int ldwf;
  const float* bias;
  const float* ext;  // M x 4
  int n_ext, ext_col;
  void* C;
  int ldc;
  int M, N;
  int act;
  float scale;       // FP8: product of operand scales (dequantization), else 1
  int c_bf16;        // 16-bit/FP8 paths: write C in the run's 16-bit format, else fp32
  float a_inv_scale; // FP8: activations are quantized as e4m3(a * a_inv_scale)
  // per-row precomputed term (per-column hoisting): v += rowadd[rowadd_idx[row] *
  // rowadd_ld + rowadd_off + col]; bias may then be null.
  const float* rowadd;
  const uint32_t* rowadd_idx;
  int rowadd_ld, rowadd_off;
  // device-side row count (nullable): rows = min(M, *M_dev); the grid covers M rows and
  // workgroups past the count exit at once (no host read-back of the count)
  const uint32_t* M_dev;
  // FP16 (nullable): set to 1 when a value written as binary16 exceeds its range
  uint32_t* ovf;
  // PREC_F32X3: the lo copy of W (W holds the hi copy)
  const void* Wlo;
  // conditional batch norm (FP32 only): v = (v - cbn_mu[col]) * cbn_rstd[col] *
  // rowmul[rowadd_idx[row] * rowadd_ld + rowmul_off + col], before the rowadd term
  const float* rowmul;
  int rowmul_off;
  const float* cbn_mu;
  const float* cbn_rstd;
  // per-texel hoisting (FP32 output only): with rowadd, each row's term is the bilinear
  // blend sum_t tap_w[row].t * rowadd[tap_idx[row].t * rowadd_ld + rowadd_off + col] of
  // four texel rows (rowadd_idx unused); bias is added as usual
  const int4* tap_idx;
  const float4* tap_w;
  // FP32 kernels, set by the launch code (callers leave it 0): every array the epilogue
  // reads or writes four columns at a time is 16-byte aligned, so the tile is finished
  // through LDS with 16-byte accesses (else block by block, 4 bytes per lane)
  int ep_vec;
};

// The conditional-batch-norm lifting network (pifu_cbn) as kernels read it.
struct CbnDesc {
  int C, n_z, width, nb;
  float eps;
  const float* Wp;
  const float* bp;
  const float* W[PIFU_CBN_MAX_BLOCKS];
  const float* b[PIFU_CBN_MAX_BLOCKS];
  const float* Wg[PIFU_CBN_MAX_BLOCKS];
  const float* bg[PIFU_CBN_MAX_BLOCKS];
  const float* Wb[PIFU_CBN_MAX_BLOCKS];
  const float* bb[PIFU_CBN_MAX_BLOCKS];
  const float* mean[PIFU_CBN_MAX_BLOCKS];
  const float* var[PIFU_CBN_MAX_BLOCKS];
  const float* Wo;
  const float* bo;
};
// Packs [Wg_0 .. Wg_nb-1; Wb_0 .. Wb_nb-1] (2 nb width x C) and their biases, and the
// batch-norm constants mu[i][c], rstd[i][c] = 1 / sqrt(var[i][c] + eps).
void launch_cbn_pack(const CbnDesc& d, float* Wgb, float* bgb, float* mu, float* rstd,
                     hipStream_t s);
// First block for points m < n: the soft one-hot depth layer, then conditional batch norm
// with gamma_0 / beta_0 from the hoisted rows P[cid[m]] (ld 2 nb width), and ReLU; a is
// n x width.
void launch_cbn_first(const PointSrc& src, const uint32_t* list, uint32_t n, const CbnDesc& d,
                      const float* P, const uint32_t* cid, const float* mu, const float* rstd,
                      float* a, hipStream_t s);
// FP64 re-evaluation of the guarded points (positions glist into list): logit and label.
size_t guard_cbn64_ws_bytes(const CbnDesc& d, uint32_t chunk);
void run_guard_cbn64(const PointSrc& src, const uint32_t* list, const uint32_t* glist, uint32_t gn,
                     const CbnDesc& d, const float* F, int H, int W, float* logit, uint8_t* lab,
                     void* ws, uint32_t chunk, hipStream_t s);

// ------------------------------------------------------------------ per-column hoisting
// flags[i] = point i starts a new (x, y) column (list sorted or not: runs of one column)
void launch_col_flags(const uint32_t* list, uint32_t n, uint32_t nz, uint32_t* flags,
                      hipStream_t s, const uint32_t* n_dev = nullptr);
// cid[i] = index of point i's column run; col_node[cid] = a node of that column
void launch_col_ids(const uint32_t* list, const uint32_t* flags, const uint32_t* excl, uint32_t n,
                    uint32_t* cid, uint32_t* col_node, hipStream_t s,
                    const uint32_t* n_dev = nullptr);
// layer 0 with hoisting: h[i][o] = act(P[cid[i]][o] + wz[o] * z_i), z from the node index;
// h in format h_fmt (ovf as for launch_gather)
void launch_hoist_layer0(const float* P, int ldp, const uint32_t* cid, const uint32_t* list,
                         uint32_t n, int nz, const float* wz, int N, int act, void* h, int h_fmt,
                         hipStream_t s, uint32_t* ovf = nullptr, const uint32_t* n_dev = nullptr);
// Per-texel hoisting: the four bilinear taps (texel index, weight; texels outside the map
// get weight 0) of each point and its extras as launch_gather writes them.
void launch_taps(const PointSrc& src, const uint32_t* list, uint32_t n, int H, int W, int4* tidx,
                 float4* tw, float* ext, hipStream_t s, const uint32_t* n_dev = nullptr);
// Layer 0 from the texel table T (ldt per texel): h = act(sum_t w_t T[idx_t] + bias + wz z),
// N outputs (N % 4 == 0), float32 out.
void launch_taps_layer0(const float* T, int ldt, const int4* tidx, const float4* tw,
                        const float* ext, uint32_t n, const float* bias, const float* wz, int N,
                        int act, float* h, hipStream_t s, const uint32_t* n_dev = nullptr);

// float32 -> OCP FP8 E4M3FN code (bias 7, 3 mantissa bits, no infinities), round to
// nearest even, saturating at +-448; NaN -> 0x7f.
__host__ __device__ inline uint8_t f32_to_e4m3(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  float a = __builtin_fabsf(x);
  if (!(a == a)) return 0x7f;
  if (a >= 448.f) return sign | 0x7e;
  int e = (int)((u >> 23) & 0xffu) - 127;
  uint32_t code;
  if (e < -6) {
    code = (uint32_t)__builtin_rintf(a * 512.f);            // subnormal quantum 2^-9
  } else {
    const float q = __builtin_ldexpf(a, 3 - e);             // in [8, 16)
    code = (uint32_t)((e + 7) << 3) + ((uint32_t)__builtin_rintf(q) - 8u);
  }
  if (code > 0x7e) code = 0x7e;
  return sign | (uint8_t)code;
}
// ev0/ev1 (nullable): an event pair the launch carries (hipExtLaunchKernelGGL), stamped
// with the kernel's own start and end
int launch_gemm(const GemmArgs& a, int precision, int tile_m, hipStream_t s,
                hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// The same GEMM over a device-side row count (a.M_dev; a.M = capacity), as a persistent
// launch whose size does not depend on the count.  FP32, BF16, FP16 and split-FP16.
int launch_gemm_persist(const GemmArgs& a, int precision, hipStream_t s);
// FP8 operand copy: amax_bits <- max |W| (float bits), dst = e4m3(W * 448 / amax).
void launch_pack_fp8(const float* W, int N, int ldw, int K, uint32_t* amax_bits, uint8_t* dst,
                     hipStream_t s);
// *amax_bits = max(*amax_bits, max |X[r][k]|) over r < rows, k < K (float bits; X row
// stride ld)
void launch_absmax(const float* X, int rows, int ld, int K, uint32_t* amax_bits, hipStream_t s);
// dst = the first K columns of W in format fmt (ovf as for launch_gather)
void launch_pack_weights(const float* W, int N, int ldw_src, int K, void* dst, int fmt,
                         hipStream_t s, uint32_t* ovf = nullptr);
// Several such copies in one launch.
struct PackJob {
  const float* W;
  void* dst;
  uint32_t* ovf;
  int N, ldw, K, fmt;
};
constexpr int kMaxPackJobs = 40;
struct PackJobs {
  PackJob j[kMaxPackJobs];
  int n = 0;
};
void launch_pack_many(const PackJobs& jobs, hipStream_t s);

}  // namespace pifu

namespace pifu {
// ------------------------------------------------------------------ mesh hand-off
// Builds the Marching Cubes triangle table and copies it to the device's constant memory
// (the current device); called by pifu_create.
int mesh_table_upload();
void launch_mesh_edge_flags(const uint8_t* labels, int nn, uint8_t* flags, hipStream_t s);
void launch_mesh_front(const uint8_t* labels, int nn, int32_t* kf, hipStream_t s);
void launch_mesh_verts(const uint32_t* ids, uint32_t nv, const float* occ, int nn, const int32_t* kf,
                       float* verts, uint8_t* hidden, float4* pts, hipStream_t s);
void launch_mesh_tri_count(const uint32_t* cells, uint32_t nc, const uint8_t* labels, int nn,
                           uint32_t* cnt, hipStream_t s);
void launch_mesh_tri_write(const uint32_t* cells, uint32_t nc, const uint8_t* labels, int nn,
                           const uint32_t* off, const uint32_t* ids, uint32_t nv, uint32_t* tris,
                           uint32_t tri_cap, hipStream_t s);
void launch_mesh_pixel_colors(const float* verts, const uint8_t* hidden, uint32_t nv,
                              const float* img, int H, int W, float* colors, hipStream_t s);

// ------------------------------------------------------------------ handle helpers
// The device a handle is bound to.
int ctx_device(const pifu_ctx* c);
// Looks up this device's copy of the no-allocation scratch array (the device must be
// current); called by pifu_create.
int noalloc_setup(int device);

// ------------------------------------------------------------------ training kernels
uint32_t bce_partials(uint32_t n);
void launch_bce_grad(const float* s, const float4* pts, uint32_t n, float* g, float* loss_part,
                     float* loss, hipStream_t st, float* point_loss = nullptr);
// point-OHEM: weighted draws (quantised weights, exact 64-bit prefix sums, SplitMix64)
// and the weight update from per-point losses
size_t ohem_workspace_bytes(uint32_t n);
void launch_ohem_sample(const float* w, uint32_t n, const float4* pool, uint32_t batch,
                        uint64_t seed, uint64_t counter, uint32_t* idx, float4* out, void* ws,
                        hipStream_t s);
void launch_ohem_update(const float* L, const uint32_t* idx, uint32_t batch, float alpha,
                        float beta, float* w, hipStream_t s);
void launch_weight_grad(const float* G, int N, const float* A1, int K1, int lda1, const float* A2,
                        int K2, int lda2, const float* ext, int n_ext, uint32_t M, float* part,
                        float* dW, float* db, hipStream_t st);
size_t weight_grad_part_floats(int N, int K, uint32_t M);
void launch_backprop_input(const float* G, int N, const float* W, int ldw, const float* H, int Kh,
                           uint32_t M, int act, float* dH, hipStream_t st);
void launch_rmsprop(float* w, const float* g, float* v, size_t n, float lr, float alpha, float eps,
                    hipStream_t st);
}  // namespace pifu
