// Host side of libpifu: argument validation, workspace carving, the level loop of
// hierarchical surface localization (Sec. 3.2), mesh-free rendering (Sec. 3.2,
// Eq. 3) and the C ABI declared in include/pifu.h.
#include <hip/hip_runtime.h>

#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <thread>
#include <vector>

#include "pifu_internal.h"

using namespace pifu;

struct ProfRecord {
  int kind;
  int ev;            // index of the start event; stop is ev + 1
  double flops, bytes;
  int slot = -1;     // pinned slot holding a device-side unit count (-1: none)
  double flops_per = 0.0, bytes_per = 0.0;   // added per counted unit
};

constexpr int kProfSlots = 16384;   // device-side counts per call that the profiler can hold

struct pifu_ctx {
  int device;
  // read-back words: mapped, fine-grained pinned memory (kHostWords words, then the
  // sequence word that the publish kernel sets last); host_counters_dev is its device view
  uint32_t* host_counters;
  uint32_t* host_counters_dev = nullptr;
  uint32_t seq = 0;          // sequence number of the last read-back
  // autotuned point tile per (precision, N, K, batch bucket); filled by pifu_autotune_mlp
  std::map<uint64_t, int> tile_cache;
  bool prof_on = false;
  std::vector<hipEvent_t> events;
  std::vector<ProfRecord> pending;
  uint32_t* prof_slots = nullptr;   // pinned, kProfSlots words (allocated when profiling starts)
  int prof_used = 0;
  pifu_kernel_profile prof[PIFU_KERN_COUNT];
  // companion state for the second host thread of pifu_grid_and_render (null in a companion)
  pifu_ctx* peer = nullptr;
};

namespace {

// Event pair around one launch when profiling is on.
struct ProfScope {
  pifu_ctx* c;
  hipStream_t s;
  int idx = -1;
  bool carry = false;
  // flops/bytes: fixed part; with dev_count, flops_per/bytes_per per unit counted on
  // the device (copied asynchronously to a pinned slot, read when the call resolves).
  // carry: the launch itself records the event pair (start(), stop() passed to a
  // hipExtLaunchKernelGGL, which stamps the kernel's own dispatch: no marker packets
  // around it); else markers are recorded around the scope.
  ProfScope(pifu_ctx* ctx, hipStream_t st, int kind, double flops, double bytes,
            const uint32_t* dev_count = nullptr, double flops_per = 0.0, double bytes_per = 0.0,
            bool carried = false)
      : c(ctx), s(st), carry(carried) {
    if (!c || !c->prof_on) return;
    const size_t need = 2 * (c->pending.size() + 1);
    while (c->events.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->events.push_back(e);
    }
    idx = (int)(2 * c->pending.size());
    ProfRecord rec{kind, idx, flops, bytes};
    if (dev_count && c->prof_slots && c->prof_used < kProfSlots &&
        hipMemcpyAsync(c->prof_slots + c->prof_used, dev_count, sizeof(uint32_t),
                       hipMemcpyDeviceToHost, s) == hipSuccess) {
      rec.slot = c->prof_used++;
      rec.flops_per = flops_per;
      rec.bytes_per = bytes_per;
    }
    c->pending.push_back(rec);
    if (!carry) (void)hipEventRecord(c->events[idx], s);
  }
  hipEvent_t start() const { return idx >= 0 && carry ? c->events[idx] : nullptr; }
  hipEvent_t stop() const { return idx >= 0 && carry ? c->events[idx + 1] : nullptr; }
  ~ProfScope() {
    if (idx >= 0 && !carry) (void)hipEventRecord(c->events[idx + 1], s);
  }
};

// Folds the recorded launches into the accumulators; the stream must be idle.
void prof_resolve(pifu_ctx* c) {
  if (!c) return;
  for (const ProfRecord& r : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->events[r.ev], c->events[r.ev + 1]) != hipSuccess) continue;
    pifu_kernel_profile& p = c->prof[r.kind];
    const double units = r.slot >= 0 ? (double)c->prof_slots[r.slot] : 0.0;
    p.launches += 1;
    p.total_ms += ms;
    p.flops += r.flops + r.flops_per * units;
    p.bytes += r.bytes + r.bytes_per * units;
  }
  c->pending.clear();
  c->prof_used = 0;
}

constexpr size_t kAlign = 256;
constexpr int kCounters = 64;
constexpr int AW_COUNT_WORDS = 16;   // count words of a device-driven call
constexpr int kHostWords = 256;   // pinned read-back buffer (>= every device counter block)
constexpr uint32_t kDefaultChunk = 65536;

// Device-side counters (words of the counters array).
// C_OVF: set when a value converted to binary16 leaves its range (FP16 runs: any such
// value; BF16 runs: the binary16 weight copies and the split-FP16 band's operands).  It
// is cleared once per call (before the weights are packed) and kept by the per-level
// counter clears, so that an overflow sends every later evaluation of the call (FP16) or
// every later band (BF16) to FP32 as well.
enum { C_TOTAL = 0, C_CONFLICTS = 1, C_B0 = 2, C_GUARD = 3, C_SHADOW = 4, C_OVF = 15 };

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

#define HIP_TRY(x)                        \
  do {                                    \
    if ((x) != hipSuccess) return PIFU_ERR_HIP; \
  } while (0)

inline int check_launch() { return hipGetLastError() == hipSuccess ? PIFU_OK : PIFU_ERR_HIP; }

// ------------------------------------------------------------------ validation
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int validate_mlp(const pifu_mlp* m, int C, int n_extra_expected, int n_out_expected) {
  if (!m) return PIFU_ERR_INVALID_ARGUMENT;
  if (m->n_layers < 2 || m->n_layers > PIFU_MAX_LAYERS) return PIFU_ERR_INVALID_ARGUMENT;
  if (m->feat_dim != C || C % 32 != 0 || C > 512) return PIFU_ERR_INVALID_ARGUMENT;
  if (m->n_extra != n_extra_expected) return PIFU_ERR_INVALID_ARGUMENT;
  if (m->hidden_act != PIFU_ACT_RELU && m->hidden_act != PIFU_ACT_LRELU)
    return PIFU_ERR_INVALID_ARGUMENT;
  for (int l = 0; l < m->n_layers; ++l) {
    if (!m->W[l] || !m->b[l]) return PIFU_ERR_INVALID_ARGUMENT;
    if (reinterpret_cast<uintptr_t>(m->W[l]) % 16 != 0) return PIFU_ERR_INVALID_ARGUMENT;
    const bool last = l == m->n_layers - 1;
    if (last) {
      if (m->widths[l] != n_out_expected) return PIFU_ERR_INVALID_ARGUMENT;
    } else if (m->widths[l] <= 0 || m->widths[l] % 64 != 0 || m->widths[l] > 1024) {
      return PIFU_ERR_INVALID_ARGUMENT;
    }
    if (l > 0 && m->skip[l] && last) return PIFU_ERR_INVALID_ARGUMENT;
  }
  return PIFU_OK;
}

int validate_cbn(const pifu_field* f);

int validate_field(const pifu_field* f, int n_extra, int n_out) {
  if (!f) return PIFU_ERR_INVALID_ARGUMENT;
  if (f->kind == PIFU_FIELD_MLP) {
    if (!f->feat || f->H < 2 || f->W < 2 || f->C <= 0) return PIFU_ERR_INVALID_ARGUMENT;
    if (!aligned(f->feat, 16)) return PIFU_ERR_INVALID_ARGUMENT;
    int r = validate_mlp(f->mlp, f->C, n_extra, n_out);
    if (r) return r;
    if (f->surrogate) {
      r = validate_mlp(f->surrogate, f->C, n_extra, n_out);
      if (r) return r;
    }
    return PIFU_OK;
  }
  if (n_out != 1) return PIFU_ERR_INVALID_ARGUMENT;
  if (f->kind == PIFU_FIELD_CBN) {
    if (n_extra != 1) return PIFU_ERR_INVALID_ARGUMENT;
    if (!f->feat || f->H < 2 || f->W < 2 || !aligned(f->feat, 16)) return PIFU_ERR_INVALID_ARGUMENT;
    return validate_cbn(f);
  }
  if (f->kind == PIFU_FIELD_ELLIPSOIDS) {
    if (!f->ell || f->n_ell < 1 || f->n_ell > PIFU_MAX_ELLIPSOIDS) return PIFU_ERR_INVALID_ARGUMENT;
    return PIFU_OK;
  }
  if (f->kind == PIFU_FIELD_PLANE) return PIFU_OK;
  return PIFU_ERR_INVALID_ARGUMENT;
}

int validate_precision(int p) {
  if (p == PIFU_PREC_FP32 || p == PIFU_PREC_BF16 || p == PIFU_PREC_FP8 || p == PIFU_PREC_FP16)
    return PIFU_OK;
  return PIFU_ERR_INVALID_ARGUMENT;
}

// ------------------------------------------------------------------ MLP preparation
struct MlpPrep {
  MLPDesc d;
  float* Wp32[PIFU_MAX_LAYERS];      // FP32 operand copies [N][Kp]
  uint16_t* Wp16[PIFU_MAX_LAYERS];   // 16-bit operand copies (BF16 or FP16 runs, that format)
  // split-FP16 band operands (FP16 and BF16 runs): binary16 hi copies (an FP16 run's are
  // Wp16) and scaled binary16 residuals
  uint16_t* Wh16[PIFU_MAX_LAYERS] = {};
  uint16_t* Wlo16[PIFU_MAX_LAYERS] = {};
  uint8_t* Wp8[PIFU_MAX_LAYERS];     // FP8 e4m3 operand copies (FP8 runs), scaled by 1/w_scale
  uint32_t* amax;                    // device: per-layer max |W| (float bits), FP8 runs
  float w_scale[PIFU_MAX_LAYERS];    // FP8 weight scale amax/448 (host, after pack)
  float a_scale[PIFU_MAX_LAYERS];    // FP8 activation scale (calibrated amax)/448
  int Kp[PIFU_MAX_LAYERS];
  int max_hidden;
  int prec;
  // per-column hoisting: the feature columns of every layer that reads f, stacked
  int NP = 0;                        // total outputs of those layers (0: no hoisting)
  int hoist_off[PIFU_MAX_LAYERS];    // offset of layer l in the stacked outputs, -1 if none
  float* Wf32 = nullptr;             // [NP][C]
  uint16_t* Wf16 = nullptr;          // [NP][C] (BF16 or FP16 runs)
  uint16_t* Wfh16 = nullptr;         // [NP][C] binary16 hi copies (BF16 runs)
  uint16_t* Wflo16 = nullptr;        // [NP][C] residuals (FP16 and BF16 runs)
  float* bf = nullptr;               // [NP] biases of those layers
  float* wz = nullptr;               // [widths[0]] layer 0's weights of z, contiguous
};

void describe_mlp(const pifu_mlp* m, MLPDesc& d) {
  std::memset(&d, 0, sizeof(d));
  d.n_layers = m->n_layers;
  d.feat_dim = m->feat_dim;
  d.n_extra = m->n_extra;
  d.hidden_act = m->hidden_act;
  d.out_act = m->out_act;
  for (int l = 0; l < m->n_layers; ++l) {
    d.widths[l] = m->widths[l];
    d.skip[l] = l > 0 ? (m->skip[l] != 0) : 0;
    d.in_w[l] = l == 0 ? m->feat_dim + m->n_extra
                       : m->widths[l - 1] + (d.skip[l] ? m->feat_dim : 0);
    d.W[l] = m->W[l];
    d.b[l] = m->b[l];
  }
}

// Carves the packed operand copies of the hidden layers: one in the run precision, an
// FP32 copy, and for BF16/FP16 runs the binary16 hi / lo copies of the split-FP16 band.
void carve_mlp(Carver& cv, const pifu_mlp* m, int precision, MlpPrep& p) {
  describe_mlp(m, p.d);
  const bool split = precision == PIFU_PREC_FP16 || precision == PIFU_PREC_BF16;
  p.max_hidden = 0;
  p.prec = precision;
  p.amax = precision == PIFU_PREC_FP8 ? cv.take<uint32_t>(PIFU_MAX_LAYERS) : nullptr;
  for (int l = 0; l + 1 < m->n_layers; ++l) {
    p.Kp[l] = l == 0 ? m->feat_dim : p.d.in_w[l];
    const size_t n = (size_t)m->widths[l] * p.Kp[l];
    p.Wp32[l] = cv.take<float>(n);
    p.Wp16[l] = precision == PIFU_PREC_BF16 || precision == PIFU_PREC_FP16 ? cv.take<uint16_t>(n)
                                                                           : nullptr;
    p.Wh16[l] = precision == PIFU_PREC_BF16 ? cv.take<uint16_t>(n) : nullptr;
    p.Wlo16[l] = split ? cv.take<uint16_t>(n) : nullptr;
    p.Wp8[l] = precision == PIFU_PREC_FP8 ? cv.take<uint8_t>(n) : nullptr;
    p.max_hidden = std::max(p.max_hidden, m->widths[l]);
    const float amax_a = m->fp8_amax[l] > 0.f ? m->fp8_amax[l] : 16.f;
    p.a_scale[l] = amax_a / 448.f;
    p.w_scale[l] = 1.f;
  }
  // hoisting applies to occupancy networks whose layer 0 reads [f; z]
  p.NP = 0;
  for (int l = 0; l < PIFU_MAX_LAYERS; ++l) p.hoist_off[l] = -1;
  if (m->n_extra == 1 && precision != PIFU_PREC_FP8) {
    for (int l = 0; l + 1 < m->n_layers; ++l)
      if (l == 0 || p.d.skip[l]) {
        p.hoist_off[l] = p.NP;
        p.NP += m->widths[l];
      }
    const size_t n = (size_t)p.NP * m->feat_dim;
    p.Wf32 = cv.take<float>(n);
    p.Wf16 = precision == PIFU_PREC_BF16 || precision == PIFU_PREC_FP16 ? cv.take<uint16_t>(n)
                                                                        : nullptr;
    p.Wfh16 = precision == PIFU_PREC_BF16 ? cv.take<uint16_t>(n) : nullptr;
    p.Wflo16 = split ? cv.take<uint16_t>(n) : nullptr;
    p.bf = cv.take<float>(p.NP);
    p.wz = cv.take<float>(m->widths[0]);
  }
}

int pack_mlp(MlpPrep& p, pifu_ctx* ctx, hipStream_t s, uint32_t* ovf) {
  const int f16 = h16_fmt(p.prec);
  // the copies go out in batches of one launch each
  PackJobs jobs;
  auto add = [&](const float* W, int N, int ldw, int K, void* dst, int fmt, uint32_t* ov) {
    if (jobs.n == kMaxPackJobs) {
      launch_pack_many(jobs, s);
      jobs.n = 0;
    }
    jobs.j[jobs.n++] = PackJob{W, dst, ov, N, ldw, K, fmt};
  };
  for (int l = 0; l + 1 < p.d.n_layers; ++l) {
    add(p.d.W[l], p.d.widths[l], p.d.in_w[l], p.Kp[l], p.Wp32[l], FMT_F32, nullptr);
    if (p.Wp16[l])
      add(p.d.W[l], p.d.widths[l], p.d.in_w[l], p.Kp[l], p.Wp16[l], f16,
          f16 == FMT_F16 ? ovf : nullptr);
    if (p.Wh16[l]) add(p.d.W[l], p.d.widths[l], p.d.in_w[l], p.Kp[l], p.Wh16[l], FMT_F16, ovf);
    if (p.Wlo16[l]) add(p.d.W[l], p.d.widths[l], p.d.in_w[l], p.Kp[l], p.Wlo16[l], FMT_F16LO, nullptr);
    if (p.Wp8[l])
      launch_pack_fp8(p.d.W[l], p.d.widths[l], p.d.in_w[l], p.Kp[l], p.amax + l, p.Wp8[l], s);
    if (p.hoist_off[l] >= 0) {
      const int C = p.d.feat_dim;
      const int fcol = l == 0 ? 0 : p.d.widths[l - 1];   // where f starts in layer l's input
      const size_t off = (size_t)p.hoist_off[l];
      add(p.d.W[l] + fcol, p.d.widths[l], p.d.in_w[l], C, p.Wf32 + off * C, FMT_F32, nullptr);
      if (p.Wf16)
        add(p.d.W[l] + fcol, p.d.widths[l], p.d.in_w[l], C, p.Wf16 + off * C, f16,
            f16 == FMT_F16 ? ovf : nullptr);
      if (p.Wfh16)
        add(p.d.W[l] + fcol, p.d.widths[l], p.d.in_w[l], C, p.Wfh16 + off * C, FMT_F16, ovf);
      if (p.Wflo16)
        add(p.d.W[l] + fcol, p.d.widths[l], p.d.in_w[l], C, p.Wflo16 + off * C, FMT_F16LO, nullptr);
      // the layer's biases, as a one-row copy
      add(p.d.b[l], 1, p.d.widths[l], p.d.widths[l], p.bf + off, FMT_F32, nullptr);
      if (l == 0)   // the z column of layer 0 (input [f; z])
        add(p.d.W[0] + C, p.d.widths[0], p.d.in_w[0], 1, p.wz, FMT_F32, nullptr);
    }
  }
  launch_pack_many(jobs, s);
  if (!p.amax) return check_launch();
  // the FP8 weight scales enter the GEMM epilogue: read them back once per call
  const int nl = p.d.n_layers - 1;
  HIP_TRY(hipMemcpyAsync(ctx->host_counters + 32, p.amax, sizeof(uint32_t) * nl,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int l = 0; l < nl; ++l) {
    float a;
    std::memcpy(&a, ctx->host_counters + 32 + l, 4);
    p.w_scale[l] = a > 0.f ? a / 448.f : 1.f;
  }
  return check_launch();
}

// ------------------------------------------------------------------ evaluator
struct EvalWs {
  uint32_t chunk = 0;
  void* feat = nullptr;
  float* ext = nullptr;
  void* hA = nullptr;
  void* hB = nullptr;
  uint32_t* glist = nullptr;
  void* g64 = nullptr;       // float64 guard-band evaluation scratch
  uint32_t chunk64 = 0;
  // re-evaluation of a subset (band: FP32 re-run; sur: surrogate fallback)
  uint32_t *band_pos = nullptr, *band_nodes = nullptr;
  float* band_logit = nullptr;
  uint8_t* band_lab = nullptr;
  uint32_t *sur_pos = nullptr, *sur_nodes = nullptr;
  float* sur_logit = nullptr;
  uint8_t* sur_lab = nullptr;
  // per-column hoisting (input view)
  uint32_t *cflags = nullptr, *cexcl = nullptr, *cid = nullptr, *cnode = nullptr, *cscan = nullptr;
  float* Pcol = nullptr;     // col_rows x NP
  uint32_t col_rows = 0;
  // per-texel hoisting (points in any view, FP32 runs of the network ttex_mlp): the
  // feature terms of every texel (H W x NP, no biases) and each point's four taps
  float* Ttex = nullptr;
  const MlpPrep* ttex_mlp = nullptr;
  int4* tidx = nullptr;
  float4* tw = nullptr;
};

struct FieldPrep {
  const pifu_field* f = nullptr;
  MlpPrep mlp, sur;
  bool has_mlp = false, has_sur = false;
  Ellipsoids ell;
  // PIFU_FIELD_CBN: the network, its stacked conditional maps [gamma_i; beta_i] (NPc rows)
  // and biases, and the batch-norm constants
  bool has_cbn = false;
  CbnDesc cd;
  int NPc = 0;
  float *Wgb = nullptr, *bgb = nullptr, *mu = nullptr, *rstd = nullptr;
};

CbnDesc cbn_desc(const pifu_field* f) {
  CbnDesc d;
  std::memset(&d, 0, sizeof(d));
  const pifu_cbn* n = f->cbn;
  d.C = n->feat_dim;
  d.n_z = n->n_z;
  d.width = n->width;
  d.nb = n->n_blocks;
  d.eps = n->eps;
  d.Wp = n->Wp;
  d.bp = n->bp;
  for (int i = 0; i < PIFU_CBN_MAX_BLOCKS; ++i) {
    d.W[i] = n->W[i];
    d.b[i] = n->b[i];
    d.Wg[i] = n->Wg[i];
    d.bg[i] = n->bg[i];
    d.Wb[i] = n->Wb[i];
    d.bb[i] = n->bb[i];
    d.mean[i] = n->mean[i];
    d.var[i] = n->var[i];
  }
  d.Wo = n->Wo;
  d.bo = n->bo;
  return d;
}

int validate_cbn(const pifu_field* f) {
  const pifu_cbn* n = f->cbn;
  if (!n) return PIFU_ERR_INVALID_ARGUMENT;
  if (n->feat_dim != f->C || f->C % 32 != 0 || f->C > 512) return PIFU_ERR_INVALID_ARGUMENT;
  if (n->width <= 0 || n->width % 64 != 0 || n->width > 512) return PIFU_ERR_INVALID_ARGUMENT;
  if (n->n_z < 2 || n->n_z > 256 || n->n_blocks < 1 || n->n_blocks > PIFU_CBN_MAX_BLOCKS)
    return PIFU_ERR_INVALID_ARGUMENT;
  if (!(n->eps > 0.f)) return PIFU_ERR_INVALID_ARGUMENT;
  // the float64 guard keeps one point's feature, maps and activations in LDS
  if (((size_t)f->C + 2 * (size_t)n->n_blocks * n->width + 2 * (size_t)n->width) * 8 > 60 * 1024)
    return PIFU_ERR_UNSUPPORTED;
  if (!n->Wp || !n->bp || !n->Wo || !n->bo || !aligned(n->Wp, 16) || !aligned(n->Wo, 16))
    return PIFU_ERR_INVALID_ARGUMENT;
  for (int i = 0; i < n->n_blocks; ++i) {
    if (!n->Wg[i] || !n->bg[i] || !n->Wb[i] || !n->bb[i] || !n->mean[i] || !n->var[i])
      return PIFU_ERR_INVALID_ARGUMENT;
    if (i > 0 && (!n->W[i - 1] || !n->b[i - 1] || !aligned(n->W[i - 1], 16)))
      return PIFU_ERR_INVALID_ARGUMENT;
  }
  return PIFU_OK;
}

void carve_field(Carver& cv, const pifu_field* f, int precision, FieldPrep& fp) {
  fp.f = f;
  fp.has_mlp = f->kind == PIFU_FIELD_MLP;
  fp.has_sur = fp.has_mlp && f->surrogate != nullptr;
  fp.has_cbn = f->kind == PIFU_FIELD_CBN;
  std::memset(&fp.ell, 0, sizeof(fp.ell));
  if (fp.has_cbn) {
    fp.cd = cbn_desc(f);
    fp.NPc = 2 * fp.cd.nb * fp.cd.width;
    fp.Wgb = cv.take<float>((size_t)fp.NPc * fp.cd.C);
    fp.bgb = cv.take<float>(fp.NPc);
    fp.mu = cv.take<float>((size_t)fp.cd.nb * fp.cd.width);
    fp.rstd = cv.take<float>((size_t)fp.cd.nb * fp.cd.width);
  }
  if (fp.has_mlp) {
    carve_mlp(cv, f->mlp, precision, fp.mlp);
    if (fp.has_sur) carve_mlp(cv, f->surrogate, PIFU_PREC_BF16, fp.sur);
  } else if (f->kind == PIFU_FIELD_ELLIPSOIDS) {
    fp.ell.n = f->n_ell;
    fp.ell.k = f->sharpness;
    if (f->ell) std::memcpy(fp.ell.e, f->ell, sizeof(float) * 12 * f->n_ell);
  }
}

// The field's occupancy network holds split-FP16 operand copies (FP16 and BF16 runs):
// its precision band runs on split-FP16 products.
bool split_band(const FieldPrep& fp) {
  return fp.has_mlp && (fp.mlp.prec == PIFU_PREC_FP16 || fp.mlp.prec == PIFU_PREC_BF16);
}

// Packs the operand copies of the field's networks.  The binary16 copies of an FP16 or
// BF16 network report values outside the binary16 range into the call's overflow flag
// (counters[C_OVF]), which `clear` resets first (once per call).
int pack_field(FieldPrep& fp, pifu_ctx* ctx, hipStream_t s, uint32_t* counters,
               bool clear = true) {
  int r = PIFU_OK;
  uint32_t* ovf = nullptr;
  if (split_band(fp)) {
    ovf = counters + C_OVF;
    if (clear) launch_set_u32(ovf, 0, s);   // a kernel: the call may be captured
  }
  if (fp.has_mlp) r = pack_mlp(fp.mlp, ctx, s, ovf);
  if (!r && fp.has_sur) r = pack_mlp(fp.sur, ctx, s, nullptr);
  if (!r && fp.has_cbn) {
    launch_cbn_pack(fp.cd, fp.Wgb, fp.bgb, fp.mu, fp.rstd, s);
    r = check_launch();
  }
  return r;
}

void carve_guard(Carver& cv, const FieldPrep& fp, uint32_t max_points, EvalWs& ew) {
  if (fp.has_cbn) {
    ew.chunk64 = std::max<uint32_t>(64, std::min<uint32_t>(16384, max_points));
    ew.g64 = cv.take<char>(guard_cbn64_ws_bytes(fp.cd, ew.chunk64));
    return;
  }
  if (!fp.has_mlp) return;
  ew.chunk64 = std::max<uint32_t>(64, std::min<uint32_t>(16384, max_points));
  ew.g64 = cv.take<char>(guard64_ws_bytes(fp.mlp.d, ew.chunk64));
  const size_t n = std::max<uint32_t>(max_points, 1);
  ew.band_pos = cv.take<uint32_t>(n);
  ew.band_nodes = cv.take<uint32_t>(n);
  ew.band_logit = cv.take<float>(n);
  ew.band_lab = cv.take<uint8_t>(n);
  if (fp.has_sur) {
    ew.sur_pos = cv.take<uint32_t>(n);
    ew.sur_nodes = cv.take<uint32_t>(n);
    ew.sur_logit = cv.take<float>(n);
    ew.sur_lab = cv.take<uint8_t>(n);
  }
}

// whole: one chunk holds max_points (device-driven calls, whose lists have device-side
// lengths); else chunks of at most kDefaultChunk points.
void carve_eval(Carver& cv, uint32_t max_points, int C, int max_hidden, EvalWs& ew,
                bool whole = false) {
  ew.chunk = whole ? std::max<uint32_t>(128, (max_points + 127) / 128 * 128)
                   : std::max<uint32_t>(128, std::min<uint32_t>(kDefaultChunk,
                                                                 (max_points + 127) / 128 * 128));
  const size_t ch = ew.chunk;
  ew.feat = cv.take<float>(ch * std::max(C, 1));
  ew.ext = cv.take<float>(ch * 4);
  ew.hA = cv.take<float>(ch * std::max(max_hidden, 1));
  ew.hB = cv.take<float>(ch * std::max(max_hidden, 1));
  ew.glist = cv.take<uint32_t>(std::max<uint32_t>(max_points, 1));
}

// Buffers of per-column hoisting for a network with NP stacked feature outputs.
// col_cap (non-zero): at most this many columns per evaluation (the lattice's x-y
// columns), so the hoisted rows need no more than that.
void carve_hoist(Carver& cv, int NP, EvalWs& ew, uint32_t col_cap = 0) {
  if (NP <= 0) return;
  const size_t ch = ew.chunk;
  ew.col_rows = col_cap ? std::min<uint32_t>(ew.chunk, col_cap) : ew.chunk;
  ew.cflags = cv.take<uint32_t>(ch);
  ew.cexcl = cv.take<uint32_t>(ch);
  ew.cid = cv.take<uint32_t>(ch);
  ew.cnode = cv.take<uint32_t>(ch);
  ew.cscan = cv.take<uint32_t>(scan_scratch_words(ch));
  ew.Pcol = cv.take<float>((size_t)ew.col_rows * NP);
}

// Buffers of per-texel hoisting for the occupancy network of an MLP field (whose layer 0
// reads [f; z]): the texel table and the taps of one chunk.
void carve_texel(Carver& cv, const FieldPrep& fp, EvalWs& ew) {
  if (!fp.has_mlp) return;
  const MlpPrep& mp = fp.mlp;
  if (mp.NP <= 0 || mp.NP % 4 || mp.d.widths[0] % 4 || mp.hoist_off[0] != 0) return;
  ew.Ttex = cv.take<float>((size_t)fp.f->H * fp.f->W * mp.NP);
  ew.tidx = cv.take<int4>(ew.chunk);
  ew.tw = cv.take<float4>(ew.chunk);
  ew.ttex_mlp = &fp.mlp;
}

// Feature channels and widest hidden layer of a network field (0 for analytic fields).
int net_channels(const FieldPrep& fp) { return fp.has_mlp || fp.has_cbn ? fp.f->C : 0; }
int net_hidden(const FieldPrep& fp) {
  return fp.has_mlp ? fp.mlp.max_hidden : (fp.has_cbn ? fp.cd.width : 0);
}

int hoist_np(const FieldPrep& fp) {
  if (fp.has_cbn) return fp.NPc;
  if (!fp.has_mlp) return 0;
  return std::max(fp.mlp.NP, fp.has_sur ? fp.sur.NP : 0);
}

struct FrameCount;

struct EvalCtx {
  pifu_ctx* ctx;
  hipStream_t s;
  uint32_t* counters;     // device
  int precision;
  float guard;            // |logit| below which FP32 results are re-run in FP64
  float band = 0.f;       // |logit| below which BF16/FP16/FP8 results are re-run in FP32
  float sur_band = 0.f;   // |logit| below which surrogate results go to the full MLP
  int tile_m = 0;         // forced point tile (32/64/128/256), 0 = chosen per launch
  bool g64_packed = false;  // float64 guard weights already written into the workspace
  // value of counters[C_GUARD], a running selection counter: known after every read-back,
  // 0 after every clear of the counters
  uint32_t sel_base = 0;
  // FP8 calibration (FP32 plain path only): amax[0] <- max |feature|, amax[1 + l] <-
  // max |output of hidden layer l| (float bits, atomicMax)
  uint32_t* amax = nullptr;
  // device-driven calls: their count words (AW_*) and the device stats record of the
  // level being evaluated
  uint32_t* aw = nullptr;
  pifu_level_stats* st_dev = nullptr;
  // multi-frame device-driven calls: per-frame attribution of the evaluation counters
  // (null: every count goes to st_dev)
  const FrameCount* fc = nullptr;
};

int batch_bucket(uint32_t m) { return m <= 8192 ? 0 : (m <= 32768 ? 1 : 2); }

uint64_t tile_key(int prec, int N, int K, uint32_t m) {
  return ((uint64_t)prec << 48) | ((uint64_t)N << 32) | ((uint64_t)K << 8) | (uint64_t)batch_bucket(m);
}

// Point tile without an autotuned entry: the largest tile that still gives the launch
// at least 256 workgroups (one per CU).  16-bit 256-point tiles pay off on long
// contractions (K >= 512) or wide layers (N a multiple of 256, >= 512), but not on
// short contractions into at most 1024 outputs (layer 0 over the feature, K = 256: its
// four k stages leave each tile bound by load and store latency, which many 64 x 64
// tiles overlap best; BF16, 65k / 20k points: 127 / 42 us against 144 / 71 us with
// 256 x 256 tiles) or on 128-wide layers (128 x 128 tiles: 23 against 29 us at 65k).
int default_tile(int prec, int N, int K, uint32_t m) {
  auto blocks = [&](int bm, int bn) { return ((m + bm - 1) / bm) * (uint64_t)((N + bn - 1) / bn); };
  const int bn128 = N % 128 == 0 ? 128 : 64;
  const bool h16 = prec == PIFU_PREC_BF16 || prec == PIFU_PREC_FP16;
  if (h16 && K <= 256 && N <= 1024) return 64;
  if (h16 && N > 128 && (K >= 512 || (N % 256 == 0 && N >= 512)) &&
      blocks(256, N % 256 == 0 ? 256 : bn128) >= 256)
    return 256;
  if (blocks(128, bn128) >= 256) return 128;
  return 64;
}

// FP32 tile without an autotuned entry (measured on gfx950 over the MLP's layer shapes):
// launches of 48k+ points take 256 x 128 tiles over eight waves (one workgroup per CU,
// 0.63-0.72 of the FP32 MFMA peak on 64k points); wide layers from 20k points, and the
// 1024+-wide column and texel GEMMs, take 128 x 64 tiles while they give 512+
// workgroups (two per CU); everything else takes 64 x 64 tiles, which beat 32 x 64 ones
// even where they leave CUs idle (layer 1 at 2k points: 28 against 43 us; the 128-wide
// last layer at 5k: 10 against 14 us) and 128 x 64 ones up to ~16k points (layer 1 at
// 9k: 109 against 131 us).  (The tile code 96 names the 128 x 64 shape.)
int fp32_tile(int N, uint32_t m) {
  auto tiles = [&](int bm, int bn) { return ((m + bm - 1) / bm) * (uint64_t)(N / bn); };
  if (N % 64 != 0) return 128;
  if (m >= 49152) return 256;
  if (tiles(128, 64) >= 512 && (N >= 1024 || (N > 128 && m >= 20480))) return 96;
  return 64;
}

int pick_tile(const EvalCtx& e, int prec, int N, int K, uint32_t m) {
  if (e.tile_m) return e.tile_m;
  if (prec == PIFU_PREC_FP32) {
    auto it = e.ctx->tile_cache.find(tile_key(prec, N, K, m));
    return it == e.ctx->tile_cache.end() ? fp32_tile(N, m) : it->second;
  }
  auto it = e.ctx->tile_cache.find(tile_key(prec, N, K, m));
  return it == e.ctx->tile_cache.end() ? default_tile(prec, N, K, m) : it->second;
}

// Brings counters [0, nwords) back to host_counters.  A one-workgroup kernel writes them
// into mapped host memory and then a sequence number; it runs after all earlier work on
// the stream, so the counts are final.  The host spins on the sequence word (a round
// trip about 4 us shorter than a copy plus a stream synchronization), and after 2 ms
// falls back to blocking on the stream, so the wait always ends.
int read_counters(EvalCtx& e, int nwords) {
  pifu_ctx* c = e.ctx;
  if (nwords < 1 || nwords > kHostWords) return PIFU_ERR_INVALID_ARGUMENT;
  const uint32_t seq = ++c->seq;
  launch_publish(e.counters, nwords, c->host_counters_dev, c->host_counters_dev + kHostWords, seq,
                 e.s);
  HIP_TRY(hipGetLastError());
  uint32_t* word = c->host_counters + kHostWords;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t i = 1;; ++i) {
    if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == seq) return PIFU_OK;
    if ((i & 1023) == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000))
      break;
    _mm_pause();
  }
  HIP_TRY(hipStreamSynchronize(e.s));
  return __atomic_load_n(word, __ATOMIC_ACQUIRE) == seq ? PIFU_OK : PIFU_ERR_HIP;
}

// |p - 0.5| < delta  <=>  |logit| < log((0.5 + delta) / (0.5 - delta)).
float logit_band(float delta) {
  if (!(delta > 0.f)) return 0.f;
  if (delta >= 0.5f) return INFINITY;
  return (float)std::log((0.5 + (double)delta) / (0.5 - (double)delta));
}

// A run of list entries whose points sample one frame's feature map.
struct Seg {
  uint32_t begin, count;
  const float* F;
  uint32_t base_sub;
};

// Algorithmic HBM bytes of one GEMM launch: each operand read once, the output written
// once (A and C in the launch's activation types, W in its operand type).
double gemm_bytes(const GemmArgs& g, int prec) {
  const bool f32a = prec == PIFU_PREC_FP32 || prec == PREC_F32X3;   // FP32 activations
  const double ea = f32a ? 4.0 : 2.0;
  const double ew = f32a ? 4.0 : prec == PIFU_PREC_FP8 ? 1.0 : 2.0;   // X3: hi + lo copies
  const double K = (double)g.K1 + g.K2, M = g.M, N = g.N;
  double b = M * K * ea + N * K * ew + M * N * (g.c_bf16 ? 2.0 : 4.0);
  if (g.rowadd) b += g.tap_idx ? M * (N * 16.0 + 32.0) : M * N * 4.0;   // taps: four rows
  if (g.n_ext) b += M * 16.0;
  return b;
}

// Profiler family of a hidden-layer GEMM of the given run precision.
int gemm_kind(int prec) {
  return prec == PIFU_PREC_FP32   ? PIFU_KERN_GEMM_F32
         : prec == PIFU_PREC_BF16 ? PIFU_KERN_GEMM_BF16
         : prec == PIFU_PREC_FP16 ? PIFU_KERN_GEMM_F16
         : prec == PREC_F32X3     ? PIFU_KERN_GEMM_F16X3
                                  : PIFU_KERN_GEMM_FP8;
}

// Operand copy of hidden layer l for a run precision (16-bit copies hold the format the
// network was prepared for).
const void* layer_weights(const MlpPrep& mp, int prec, int l) {
  if (prec == PREC_F32X3)   // the binary16 hi copy
    return mp.prec == PIFU_PREC_FP16 ? (const void*)mp.Wp16[l] : (const void*)mp.Wh16[l];
  return prec == PIFU_PREC_FP8    ? (const void*)mp.Wp8[l]
         : prec == PIFU_PREC_FP32 ? (const void*)mp.Wp32[l]
                                  : (const void*)mp.Wp16[l];
}

// The texel table of per-texel hoisting: the feature terms of every layer that reads f,
// for every texel of the feature map (one FP32 GEMM [H W x C] x [C x NP], no biases).
// Run once per call, after the network is packed.
int fill_texel(EvalCtx& e, const FieldPrep& fp, const EvalWs& ew) {
  if (!ew.Ttex) return PIFU_OK;
  const MlpPrep& mp = *ew.ttex_mlp;
  const pifu_field* f = fp.f;
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A1 = f->feat;
  g.K1 = g.lda1 = f->C;
  g.W = mp.Wf32;
  g.ldw = f->C;
  g.C = ew.Ttex;
  g.ldc = g.N = mp.NP;
  g.M = f->H * f->W;
  g.scale = 1.f;
  ProfScope ps(e.ctx, e.s, PIFU_KERN_GEMM_F32, 2.0 * g.M * g.N * g.K1,
               gemm_bytes(g, PIFU_PREC_FP32), nullptr, 0.0, 0.0, true);
  if (launch_gemm(g, PIFU_PREC_FP32, pick_tile(e, PIFU_PREC_FP32, g.N, g.K1, (uint32_t)g.M), e.s,
                  ps.start(), ps.stop()))
    return PIFU_ERR_UNSUPPORTED;
  return PIFU_OK;
}

// Runs an MLP over n points (chunked): gather -> hidden GEMMs -> head.  prec selects
// the MFMA operand type of the hidden layers.  segs (nullable) splits the list into
// frames that share the network but not the feature map; the GEMMs span all frames.
int run_mlp(EvalCtx& e, const FieldPrep& fp, const MlpPrep& mp, int prec, const PointSrc& src,
            const uint32_t* list, uint32_t n, const EvalWs& ew, float* logit, uint8_t* lab,
            float* rgb, const Seg* segs = nullptr, int nseg = 0) {
  const pifu_field* f = fp.f;
  const MLPDesc& d = mp.d;
  const int C = f->C;
  const bool x3 = prec == PREC_F32X3;   // FP32 activations, split-FP16 products
  const bool b16 = prec != PIFU_PREC_FP32 && !x3;
  const int hf = x3 ? FMT_F32 : h16_fmt(prec);
  // a 16-bit run needs the operand copies of its own format; X3 the FP16 hi / lo copies
  if ((prec == PIFU_PREC_BF16 || prec == PIFU_PREC_FP16) && mp.prec != prec)
    return PIFU_ERR_UNSUPPORTED;
  if (x3 && !mp.Wlo16[0]) return PIFU_ERR_UNSUPPORTED;
  // FP16 conversions and split-FP16 operands report values outside the binary16 range
  uint32_t* ovf = prec == PIFU_PREC_FP16 || x3 ? e.counters + C_OVF : nullptr;
  Seg one{0, n, f->feat, src.base_sub};
  if (!segs) {
    segs = &one;
    nseg = 1;
  }
  // input-view lattice points of one frame: hoist the feature terms per column
  // (the layer-0 kernel handles four outputs per thread: widths and NP multiples of 4)
  const bool hoist = src.mode == 0 && !src.has_view && prec != PIFU_PREC_FP8 && mp.NP > 0 &&
                     mp.NP % 4 == 0 && d.widths[0] % 4 == 0 && ew.Pcol != nullptr &&
                     (nseg == 1 || src.frame_nodes);
  for (uint32_t c0 = 0; c0 < n && hoist; c0 += ew.chunk) {
    const uint32_t m = std::min(ew.chunk, n - c0);
    const uint32_t* lst = list + c0;
    // the number of column runs (<= m) stays on the device: the column gather and
    // GEMM cover m rows and skip the rows past the count
    const uint32_t* ncol_dev = e.counters + C_TOTAL;
    launch_col_flags(lst, m, (uint32_t)src.nz, ew.cflags, e.s);
    launch_scan_u32(ew.cflags, m, ew.cexcl, ew.cscan, e.counters + C_TOTAL, e.s);
    launch_col_ids(lst, ew.cflags, ew.cexcl, m, ew.cid, ew.cnode, e.s);
    {
      ProfScope ps(e.ctx, e.s, PIFU_KERN_GATHER, 0.0, 0.0, ncol_dev, 0.0,
                   16.0 * C + (b16 ? 2 : 4) * C + 20.0);
      PointSrc sq = src;
      if (!src.frame_nodes) sq.base_sub = segs[0].base_sub;   // else the frame table decodes
      launch_gather(sq, ew.cnode, m, segs[0].F, f->H, f->W, C, ew.feat, hf, ew.ext, e.s, ncol_dev,
                    ovf);
    }
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.A1 = ew.feat;
    g.K1 = g.lda1 = C;
    g.W = x3 ? (mp.prec == PIFU_PREC_FP16 ? (const void*)mp.Wf16 : (const void*)mp.Wfh16)
          : b16 ? (const void*)mp.Wf16 : (const void*)mp.Wf32;
    g.Wlo = x3 ? (const void*)mp.Wflo16 : nullptr;
    g.ovf = ovf;
    g.ldw = C;
    g.bias = mp.bf;
    g.C = ew.Pcol;
    g.ldc = g.N = mp.NP;
    g.M = (int)m;
    g.M_dev = ncol_dev;
    g.act = 0;
    g.scale = 1.f;
    {
      const double ea = b16 ? 2.0 : 4.0;
      ProfScope ps(e.ctx, e.s, gemm_kind(prec), 0.0,
                   (double)mp.NP * C * ea, ncol_dev, 2.0 * mp.NP * C, C * ea + mp.NP * 4.0, true);
      if (launch_gemm(g, prec, pick_tile(e, prec, g.N, C, m), e.s, ps.start(), ps.stop()))
        return PIFU_ERR_UNSUPPORTED;
    }
    launch_hoist_layer0(ew.Pcol, mp.NP, ew.cid, lst, m, src.nz, mp.wz, d.widths[0], d.hidden_act,
                        ew.hA, d.n_layers > 2 ? hf : FMT_F32, e.s, ovf);
    const void* prev = ew.hA;
    void* out = ew.hB;
    for (int l = 1; l + 1 < d.n_layers; ++l) {
      std::memset(&g, 0, sizeof(g));
      g.A1 = prev;
      g.K1 = g.lda1 = d.widths[l - 1];
      g.W = layer_weights(mp, prec, l);
      g.Wlo = x3 ? (const void*)mp.Wlo16[l] : nullptr;
      g.ldw = mp.Kp[l];
      g.Wf = d.W[l];
      g.ldwf = d.in_w[l];
      if (mp.hoist_off[l] >= 0) {
        g.rowadd = ew.Pcol;
        g.rowadd_idx = ew.cid;
        g.rowadd_ld = mp.NP;
        g.rowadd_off = mp.hoist_off[l];
      } else {
        g.bias = d.b[l];
      }
      g.C = out;
      g.ldc = g.N = d.widths[l];
      g.M = (int)m;
      g.act = d.hidden_act;
      g.scale = 1.f;
      g.c_bf16 = b16 && (l + 2 < d.n_layers);
      g.ovf = ovf;
      {
        ProfScope ps(e.ctx, e.s, gemm_kind(prec), 2.0 * m * g.N * g.K1, gemm_bytes(g, prec), nullptr,
                     0.0, 0.0, true);
        if (launch_gemm(g, prec, pick_tile(e, prec, g.N, g.K1, m), e.s, ps.start(), ps.stop()))
          return PIFU_ERR_UNSUPPORTED;
      }
      prev = out;
      out = (out == ew.hA) ? ew.hB : ew.hA;
    }
    const int L = d.n_layers - 1;
    ProfScope ps(e.ctx, e.s, PIFU_KERN_HEAD, 2.0 * m * d.widths[L - 1] * d.widths[L], 0.0);
    launch_head(reinterpret_cast<const float*>(prev), d.widths[L - 1], d.W[L], d.b[L], d.widths[L],
                d.out_act, m, nullptr, logit ? logit + c0 : nullptr, lab ? lab + c0 : nullptr, rgb,
                rgb ? lst : nullptr, e.s);
  }
  if (hoist) return check_launch();
  // other points of one frame in an FP32 run of the network the texel table was built for:
  // blend four texel rows per point instead of gathering the feature
  const bool texel = ew.Ttex && &mp == ew.ttex_mlp && prec == PIFU_PREC_FP32 && nseg == 1 &&
                     !src.frame_nodes && segs[0].F == f->feat && !e.amax;
  for (uint32_t c0 = 0; c0 < n && texel; c0 += ew.chunk) {
    const uint32_t m = std::min(ew.chunk, n - c0);
    const uint32_t* lst = list + c0;
    {
      ProfScope ps(e.ctx, e.s, PIFU_KERN_GATHER, 0.0, (double)m * 52.0);
      PointSrc sq = src;
      sq.base_sub = segs[0].base_sub;
      launch_taps(sq, lst, m, f->H, f->W, ew.tidx, ew.tw, ew.ext, e.s);
    }
    launch_taps_layer0(ew.Ttex, mp.NP, ew.tidx, ew.tw, ew.ext, m, mp.bf, mp.wz, d.widths[0],
                       d.hidden_act, reinterpret_cast<float*>(ew.hA), e.s);
    const void* prev = ew.hA;
    void* out = ew.hB;
    for (int l = 1; l + 1 < d.n_layers; ++l) {
      GemmArgs g;
      std::memset(&g, 0, sizeof(g));
      g.A1 = prev;
      g.K1 = g.lda1 = d.widths[l - 1];
      g.W = mp.Wp32[l];
      g.ldw = mp.Kp[l];
      g.Wf = d.W[l];
      g.ldwf = d.in_w[l];
      g.bias = d.b[l];
      if (mp.hoist_off[l] >= 0) {
        g.rowadd = ew.Ttex;
        g.rowadd_ld = mp.NP;
        g.rowadd_off = mp.hoist_off[l];
        g.tap_idx = ew.tidx;
        g.tap_w = ew.tw;
      }
      g.C = out;
      g.ldc = g.N = d.widths[l];
      g.M = (int)m;
      g.act = d.hidden_act;
      g.scale = 1.f;
      {
        ProfScope ps(e.ctx, e.s, PIFU_KERN_GEMM_F32, 2.0 * m * g.N * g.K1,
                     gemm_bytes(g, PIFU_PREC_FP32), nullptr, 0.0, 0.0, true);
        if (launch_gemm(g, PIFU_PREC_FP32, pick_tile(e, PIFU_PREC_FP32, g.N, g.K1, m), e.s,
                        ps.start(), ps.stop()))
          return PIFU_ERR_UNSUPPORTED;
      }
      prev = out;
      out = (out == ew.hA) ? ew.hB : ew.hA;
    }
    const int L = d.n_layers - 1;
    ProfScope ps(e.ctx, e.s, PIFU_KERN_HEAD, 2.0 * m * d.widths[L - 1] * d.widths[L], 0.0);
    launch_head(reinterpret_cast<const float*>(prev), d.widths[L - 1], d.W[L], d.b[L], d.widths[L],
                d.out_act, m, ew.ext, logit ? logit + c0 : nullptr, lab ? lab + c0 : nullptr, rgb,
                rgb ? lst : nullptr, e.s);
  }
  if (texel) return check_launch();
  for (uint32_t c0 = 0; c0 < n; c0 += ew.chunk) {
    const uint32_t m = std::min(ew.chunk, n - c0);
    const uint32_t* lst = list + c0;
    {
      ProfScope ps(e.ctx, e.s, PIFU_KERN_GATHER, 0.0, (double)m * (16.0 * C + (b16 ? 2 : 4) * C + 20.0));
      if (src.frame_nodes)
        launch_gather(src, lst, m, segs[0].F, f->H, f->W, C, ew.feat, hf, ew.ext, e.s, nullptr, ovf);
      for (int q = 0; q < nseg && !src.frame_nodes; ++q) {
        const uint32_t lo = std::max(c0, segs[q].begin);
        const uint32_t hi = std::min(c0 + m, segs[q].begin + segs[q].count);
        if (lo >= hi) continue;
        PointSrc sq = src;
        sq.base_sub = segs[q].base_sub;
        char* fb = reinterpret_cast<char*>(ew.feat) + (size_t)(lo - c0) * C * (b16 ? 2 : 4);
        launch_gather(sq, list + lo, hi - lo, segs[q].F, f->H, f->W, C, fb, hf,
                      ew.ext + 4 * (size_t)(lo - c0), e.s, nullptr, ovf);
      }
    }
    if (e.amax && prec == PIFU_PREC_FP32)
      launch_absmax(reinterpret_cast<const float*>(ew.feat), (int)m, C, C, e.amax, e.s);
    const void* prev = nullptr;
    void* out = ew.hA;
    for (int l = 0; l + 1 < d.n_layers; ++l) {
      GemmArgs g;
      std::memset(&g, 0, sizeof(g));
      if (l == 0) {
        g.A1 = ew.feat;
        g.K1 = C;
        g.lda1 = C;
        g.n_ext = d.n_extra;
        g.ext_col = C;
      } else {
        g.A1 = prev;
        g.K1 = d.widths[l - 1];
        g.lda1 = d.widths[l - 1];
        if (d.skip[l]) {
          g.A2 = ew.feat;
          g.K2 = C;
          g.lda2 = C;
        }
      }
      g.W = layer_weights(mp, prec, l);
      g.Wlo = x3 ? (const void*)mp.Wlo16[l] : nullptr;
      g.a_inv_scale = prec == PIFU_PREC_FP8 ? 1.f / mp.a_scale[l] : 1.f;
      g.ldw = mp.Kp[l];
      g.Wf = d.W[l];
      g.ldwf = d.in_w[l];
      g.bias = d.b[l];
      g.ext = ew.ext;
      g.C = out;
      g.ldc = d.widths[l];
      g.M = (int)m;
      g.N = d.widths[l];
      g.act = d.hidden_act;
      g.scale = prec == PIFU_PREC_FP8 ? mp.a_scale[l] * mp.w_scale[l] : 1.f;
      g.c_bf16 = b16 && (l + 2 < d.n_layers);   // the head reads FP32
      g.ovf = ovf;
      {
        ProfScope ps(e.ctx, e.s, gemm_kind(prec), 2.0 * m * g.N * (g.K1 + g.K2 + g.n_ext),
                     gemm_bytes(g, prec), nullptr, 0.0, 0.0, true);
        if (launch_gemm(g, prec, pick_tile(e, prec, g.N, g.K1 + g.K2, m), e.s, ps.start(),
                        ps.stop()))
          return PIFU_ERR_UNSUPPORTED;
      }
      if (e.amax && prec == PIFU_PREC_FP32)
        launch_absmax(reinterpret_cast<const float*>(out), (int)m, g.ldc, g.N, e.amax + 1 + l, e.s);
      prev = out;
      out = (out == ew.hA) ? ew.hB : ew.hA;
    }
    const int L = d.n_layers - 1;
    ProfScope ps(e.ctx, e.s, PIFU_KERN_HEAD, 2.0 * m * d.widths[L - 1] * d.widths[L], 0.0);
    launch_head(reinterpret_cast<const float*>(prev), d.widths[L - 1], d.W[L], d.b[L], d.widths[L],
                d.out_act, m, ew.ext, logit ? logit + c0 : nullptr, lab ? lab + c0 : nullptr, rgb,
                rgb ? lst : nullptr, e.s);
  }
  return check_launch();
}

// Positions m < n with |logit[m]| < bound (any order) and their count.
int select_near(EvalCtx& e, const float* logit, uint32_t n, float bound, uint32_t* pos,
                uint32_t* count, const uint32_t* map = nullptr) {
  *count = 0;
  if (!(bound > 0.f) || !n) return PIFU_OK;
  launch_guard_select(logit, n, bound, pos, e.counters + C_GUARD, e.s, map, e.sel_base);
  int r = check_launch();
  if (r) return r;
  r = read_counters(e, C_OVF + 1);   // the overflow flag comes back with the count
  if (r) return r;
  const uint32_t now = e.ctx->host_counters[C_GUARD];
  *count = now - e.sel_base;
  e.sel_base = now;
  return PIFU_OK;
}

// After the run-precision pass: the FP32-accurate band (BF16/FP16/FP8 runs), then the FP64
// guard.  F is the feature map of the points' frame.  FP16 and BF16 runs re-run their band
// on split-FP16 products, FP8 runs on FP32 MFMA.  An FP16 run whose call has seen a value
// outside the binary16 range is re-run whole in FP32 instead of the band; so is one whose
// split-FP16 band reports such a value (read back with the guard's count).  A BF16 run's
// own pass does not depend on that range: there only the band's points go to FP32.
int post_full(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const float* F,
              const uint32_t* list, uint32_t n, const EvalWs& ew, float* logit, uint8_t* lab,
              pifu_level_stats* st) {
  const pifu_field* f = fp.f;
  int r = PIFU_OK;
  const Seg one{0, n, F, src.base_sub};
  uint32_t nb_run = 0;   // points re-run by the band
  bool over = false;     // FP16 overflow: all n points re-run in FP32
  const bool f16 = e.precision == PIFU_PREC_FP16;
  bool bx3 = false;      // a BF16 run's band on split-FP16 products
  auto rerun_fp32 = [&]() {
    int q = run_mlp(e, fp, fp.mlp, PIFU_PREC_FP32, src, list, n, ew, logit, lab, nullptr, &one, 1);
    if (!q && st) st->band_fp32 += n - nb_run;
    nb_run = 0;
    return q;
  };
  auto rerun_band_fp32 = [&]() {
    const Seg bseg{0, nb_run, F, src.base_sub};
    int q = run_mlp(e, fp, fp.mlp, PIFU_PREC_FP32, src, ew.band_nodes, nb_run, ew, ew.band_logit,
                    ew.band_lab, nullptr, &bseg, 1);
    if (!q) launch_scatter_results(ew.band_pos, nb_run, ew.band_logit, ew.band_lab, logit, lab, e.s);
    return q;
  };
  // after split-FP16 products: a value outside the binary16 range sends an FP16 run's
  // points, or a BF16 run's band, to FP32
  auto overflow_rerun = [&]() { return f16 ? rerun_fp32() : rerun_band_fp32(); };
  if (e.precision != PIFU_PREC_FP32 && e.band > 0.f) {
    uint32_t nb = 0;
    r = select_near(e, logit, n, e.band, ew.band_pos, &nb);
    if (r) return r;
    over = f16 && e.ctx->host_counters[C_OVF] != 0;
    if (nb && !over) {
      nb_run = nb;
      launch_gather_u32(list, ew.band_pos, nb, ew.band_nodes, e.s);
      const Seg bseg{0, nb, F, src.base_sub};
      // an FP16 run's band: FP32-accurate split-FP16 products (operands inside the
      // binary16 range, which the FP16 pass checked; the band reports its own); a BF16
      // run's too, unless a value of this call already left that range (its binary16
      // weight copies report theirs when packed)
      bx3 = e.precision == PIFU_PREC_BF16 && split_band(fp) && e.ctx->host_counters[C_OVF] == 0;
      const int bprec = f16 || bx3 ? PREC_F32X3 : PIFU_PREC_FP32;
      r = run_mlp(e, fp, fp.mlp, bprec, src, ew.band_nodes, nb, ew, ew.band_logit, ew.band_lab,
                  nullptr, &bseg, 1);
      if (r) return r;
      launch_scatter_results(ew.band_pos, nb, ew.band_logit, ew.band_lab, logit, lab, e.s);
      if (st) st->band_fp32 += nb;
    }
  } else if (f16) {
    r = read_counters(e, C_OVF + 1);
    if (r) return r;
    over = e.ctx->host_counters[C_OVF] != 0;
  }
  if (over) {
    r = rerun_fp32();
    if (r) return r;
  }
  if (!(e.guard > 0.f)) {
    if ((f16 || bx3) && nb_run) {   // no guard read-back to carry the band's overflow report
      r = read_counters(e, C_OVF + 1);
      if (!r && e.ctx->host_counters[C_OVF]) r = overflow_rerun();
    }
    return r;
  }
  uint32_t gn = 0;
  if (e.precision != PIFU_PREC_FP32 && e.band > e.guard && !over) {
    // every point with |logit| < guard lies inside the band and now holds its FP32
    // result: the guard picks from the band's results only
    if (nb_run) r = select_near(e, ew.band_logit, nb_run, e.guard, ew.glist, &gn, ew.band_pos);
    if (!r && (f16 || bx3) && nb_run && e.ctx->host_counters[C_OVF]) {
      r = overflow_rerun();
      if (!r && f16) r = select_near(e, logit, n, e.guard, ew.glist, &gn);
      else if (!r) r = select_near(e, ew.band_logit, nb_run, e.guard, ew.glist, &gn, ew.band_pos);
    }
  } else {
    r = select_near(e, logit, n, e.guard, ew.glist, &gn);
  }
  if (r) return r;
  run_guard64(src, list, ew.glist, gn, fp.mlp.d, F, f->H, f->W, f->C, logit, lab, ew.g64,
              ew.chunk64, !e.g64_packed, e.s);
  if (gn) e.g64_packed = true;
  if (st) st->guard_fp64 += gn;
  return check_launch();
}

// Full-network evaluation: run precision, then the FP32 band, then the FP64 guard.
int eval_full(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const uint32_t* list,
              uint32_t n, const EvalWs& ew, float* logit, uint8_t* lab, pifu_level_stats* st,
              const float* F = nullptr) {
  if (!F) F = fp.f->feat;
  const Seg one{0, n, F, src.base_sub};
  int r = run_mlp(e, fp, fp.mlp, e.precision, src, list, n, ew, logit, lab, nullptr, &one, 1);
  if (r) return r;
  if (st) st->mlp_points += n;
  return post_full(e, fp, src, F, list, n, ew, logit, lab, st);
}

// Evaluates the occupancy field at n points; fills logit and label per point.  With
// use_surrogate, the surrogate network (BF16) runs first and the points whose
// surrogate occupancy lies within the fallback band of 0.5 go to the full network.
// The conditional-batch-norm network (PIFU_FIELD_CBN) on n points, FP32, then the FP64
// guard.  Input-view lattice points share their column's gamma / beta rows (computed once
// per column); other points take one row each.
int eval_cbn(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const uint32_t* list,
             uint32_t n, const EvalWs& ew, float* logit, uint8_t* lab, pifu_level_stats* st) {
  const pifu_field* f = fp.f;
  const CbnDesc& d = fp.cd;
  const int C = f->C;
  if (!ew.Pcol || ew.col_rows < ew.chunk) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  const bool columns = src.mode == 0 && !src.has_view && !src.frame_nodes;
  for (uint32_t c0 = 0; c0 < n; c0 += ew.chunk) {
    const uint32_t m = std::min(ew.chunk, n - c0);
    const uint32_t* lst = list + c0;
    const uint32_t* rows_dev = nullptr;   // rows of the conditional GEMM (device count)
    const uint32_t* rows_src = lst;       // the point whose feature each row samples
    if (columns) {
      launch_col_flags(lst, m, (uint32_t)src.nz, ew.cflags, e.s);
      launch_scan_u32(ew.cflags, m, ew.cexcl, ew.cscan, e.counters + C_TOTAL, e.s);
      launch_col_ids(lst, ew.cflags, ew.cexcl, m, ew.cid, ew.cnode, e.s);
      rows_dev = e.counters + C_TOTAL;
      rows_src = ew.cnode;
    } else {
      launch_iota(ew.cid, m, e.s);
    }
    {
      ProfScope ps(e.ctx, e.s, PIFU_KERN_GATHER, 0.0, 0.0, rows_dev ? rows_dev : nullptr,
                   0.0, 20.0 * C + 20.0);
      launch_gather(src, rows_src, m, f->feat, f->H, f->W, C, ew.feat, FMT_F32, ew.ext, e.s,
                    rows_dev, nullptr);
    }
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.A1 = ew.feat;
    g.K1 = g.lda1 = C;
    g.W = fp.Wgb;
    g.ldw = C;
    g.bias = fp.bgb;
    g.C = ew.Pcol;
    g.ldc = g.N = fp.NPc;
    g.M = (int)m;
    g.M_dev = rows_dev;
    g.scale = 1.f;
    {
      ProfScope ps(e.ctx, e.s, PIFU_KERN_GEMM_F32, rows_dev ? 0.0 : 2.0 * m * g.N * C,
                   rows_dev ? (double)g.N * C * 4.0 : 0.0, rows_dev, 2.0 * g.N * C,
                   C * 4.0 + g.N * 4.0, true);
      if (launch_gemm(g, PIFU_PREC_FP32, pick_tile(e, PIFU_PREC_FP32, g.N, C, m), e.s, ps.start(),
                      ps.stop()))
        return PIFU_ERR_UNSUPPORTED;
    }
    launch_cbn_first(src, lst, m, d, ew.Pcol, ew.cid, fp.mu, fp.rstd,
                     reinterpret_cast<float*>(ew.hA), e.s);
    const void* prev = ew.hA;
    void* out = ew.hB;
    for (int i = 1; i < d.nb; ++i) {
      std::memset(&g, 0, sizeof(g));
      g.A1 = prev;
      g.K1 = g.lda1 = d.width;
      g.W = d.W[i - 1];
      g.ldw = d.width;
      g.bias = d.b[i - 1];
      g.rowadd = ew.Pcol;
      g.rowadd_idx = ew.cid;
      g.rowadd_ld = fp.NPc;
      g.rowadd_off = (d.nb + i) * d.width;   // beta_i
      g.rowmul = ew.Pcol;
      g.rowmul_off = i * d.width;            // gamma_i
      g.cbn_mu = fp.mu + (size_t)i * d.width;
      g.cbn_rstd = fp.rstd + (size_t)i * d.width;
      g.C = out;
      g.ldc = g.N = d.width;
      g.M = (int)m;
      g.act = PIFU_ACT_RELU;
      g.scale = 1.f;
      {
        ProfScope ps(e.ctx, e.s, PIFU_KERN_GEMM_F32, 2.0 * m * g.N * g.K1,
                     4.0 * ((double)m * (g.K1 + 3.0 * g.N) + (double)g.N * g.K1), nullptr, 0.0, 0.0,
                     true);
        if (launch_gemm(g, PIFU_PREC_FP32, pick_tile(e, PIFU_PREC_FP32, g.N, g.K1, m), e.s,
                        ps.start(), ps.stop()))
          return PIFU_ERR_UNSUPPORTED;
      }
      prev = out;
      out = (out == ew.hA) ? ew.hB : ew.hA;
    }
    ProfScope ps(e.ctx, e.s, PIFU_KERN_HEAD, 2.0 * m * d.width, 0.0);
    launch_head(reinterpret_cast<const float*>(prev), d.width, d.Wo, d.bo, 1, PIFU_ACT_SIGMOID, m,
                nullptr, logit + c0, lab + c0, nullptr, nullptr, e.s);
  }
  int r = check_launch();
  if (r) return r;
  if (st) st->mlp_points += n;
  if (!(e.guard > 0.f)) return PIFU_OK;
  uint32_t gn = 0;
  r = select_near(e, logit, n, e.guard, ew.glist, &gn);
  if (r) return r;
  run_guard_cbn64(src, list, ew.glist, gn, d, f->feat, f->H, f->W, logit, lab, ew.g64, ew.chunk64,
                  e.s);
  if (st) st->guard_fp64 += gn;
  return check_launch();
}

int eval_occupancy(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const uint32_t* list,
                   uint32_t n, const EvalWs& ew, float* logit, uint8_t* lab, pifu_level_stats* st,
                   bool use_surrogate = false) {
  if (!n) return PIFU_OK;
  if (fp.has_cbn) return eval_cbn(e, fp, src, list, n, ew, logit, lab, st);
  if (!fp.has_mlp) {
    launch_eval_analytic(src, list, n, fp.f->kind, fp.ell, fp.f->plane, logit, lab, e.s);
    return check_launch();
  }
  if (!(use_surrogate && fp.has_sur)) return eval_full(e, fp, src, list, n, ew, logit, lab, st);
  int r = run_mlp(e, fp, fp.sur, PIFU_PREC_BF16, src, list, n, ew, logit, lab, nullptr);
  if (r) return r;
  uint32_t ns = 0;
  r = select_near(e, logit, n, e.sur_band, ew.sur_pos, &ns);
  if (r) return r;
  if (ns) {
    launch_gather_u32(list, ew.sur_pos, ns, ew.sur_nodes, e.s);
    r = eval_full(e, fp, src, ew.sur_nodes, ns, ew, ew.sur_logit, ew.sur_lab, st);
    if (r) return r;
    launch_scatter_results(ew.sur_pos, ns, ew.sur_logit, ew.sur_lab, logit, lab, e.s);
  }
  if (st) st->surrogate_fallback += ns;
  return check_launch();
}

// ------------------------------------------------------------------ localization
struct LevelBuf {
  Lat lat;
  uint8_t* st;
  float* occ;
  int level_id;
};

struct LocalizeWs {
  uint32_t* list;
  uint32_t* cscratch;
  float* logit;
  uint8_t* lab;
};

Lat level_lattice(const int log2_cells[3], int T, int t) {
  Lat l;
  l.nx = (1 << (log2_cells[0] - (T - t))) + 1;
  l.ny = (1 << (log2_cells[1] - (T - t))) + 1;
  l.nz = (1 << (log2_cells[2] - (T - t))) + 1;
  return l;
}

int compact_count(EvalCtx& e, const uint8_t* st, size_t n, uint8_t mask, uint8_t val,
                  uint32_t* scratch, uint32_t* out, uint32_t cap, int mode, Lat f, uint32_t* count) {
  launch_compact(st, n, mask, val, scratch, e.counters + C_TOTAL, out, cap, mode, f, e.s);
  int r = check_launch();
  if (r) return r;
  r = read_counters(e, C_OVF + 1);   // the level's other counters come back with the count
  if (r) return r;
  *count = e.ctx->host_counters[C_TOTAL];
  return PIFU_OK;
}

// Levels 0..last of the hierarchy (level T is the finest lattice of `fin_log2`).
int localize(EvalCtx& e, const FieldPrep& fp, const EvalWs& ew, const double* view,
             const int fin_log2[3], int T, int last, LevelBuf* lv, const LocalizeWs& w,
             uint8_t* eval_level, Lat eval_lat, int max_waves, int sur_max_log2,
             pifu_level_stats* stats, float* eval_logit = nullptr) {
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  if (view) {
    src.has_view = 1;
    for (int i = 0; i < 12; ++i) src.view[i] = view[i];
  }
  for (int t = 0; t <= last; ++t) {
    LevelBuf& L = lv[t];
    pifu_level_stats st;
    std::memset(&st, 0, sizeof(st));
    st.level = L.level_id;
    st.nodes = (uint32_t)L.lat.n();
    src.nx = L.lat.nx;
    src.ny = L.lat.ny;
    src.nz = L.lat.nz;
    // spacing of this level's nodes on the lattice of the evaluation-level map
    const int stride = (eval_lat.nx - 1) / (L.lat.nx - 1);
    const uint32_t n_nodes = (uint32_t)L.lat.n();
    HIP_TRY(hipMemsetAsync(e.counters, 0, sizeof(uint32_t) * C_OVF, e.s));   // keeps C_OVF
    e.sel_base = 0;
    bool fresh = false;   // the host copy holds every counter of this level
    if (t == 0) {
      // coarsest level: every node is evaluated
      launch_fill_u8(L.st, 0, n_nodes, e.s);
      launch_iota(w.list, n_nodes, e.s);
      int r = eval_occupancy(e, fp, src, w.list, n_nodes, ew, w.logit, w.lab, &st,
                             L.level_id <= sur_max_log2);
      if (r) return r;
      launch_apply_grid(w.list, n_nodes, w.logit, w.lab, L.st, L.occ, nullptr, eval_level,
                        L.level_id, L.lat, stride, eval_lat, 0, e.s, 0, nullptr, eval_logit);
      st.dilated = n_nodes;
      st.evaluated = n_nodes;
    } else {
      LevelBuf& Cc = lv[t - 1];
      launch_transition(Cc.st, Cc.occ, Cc.lat, L.st, L.occ, L.lat, e.s);
      // the candidate list is consumed: its buffer (n_nodes words) holds the candidate
      // bit masks until this level's compaction rewrites it
      if (2 * b0_mask_words(L.lat) <= n_nodes) {
        launch_select_b0(L.st, L.lat, 1, reinterpret_cast<uint64_t*>(w.list), e.counters + C_B0, 0,
                         e.s);
      } else {
        launch_count_bits(L.st, n_nodes, ST_B0, e.counters + C_B0, e.s);
        launch_select(L.st, L.lat, e.s);
      }
      uint32_t n = 0;
      int r = compact_count(e, L.st, n_nodes, ST_PEND, ST_PEND, w.cscratch, w.list, n_nodes, 0,
                            L.lat, &n);
      if (r) return r;
      fresh = true;
      st.dilated = n;
      int waves = 0;
      while (n) {
        r = eval_occupancy(e, fp, src, w.list, n, ew, w.logit, w.lab, &st,
                           L.level_id <= sur_max_log2);
        if (r) return r;
        launch_apply_grid(w.list, n, w.logit, w.lab, L.st, L.occ, e.counters + C_CONFLICTS,
                          eval_level, L.level_id, L.lat, stride, eval_lat, 1, e.s, 0, nullptr,
                          eval_logit);
        fresh = false;
        st.evaluated += n;
        if (max_waves > 0 && waves >= max_waves) break;
        launch_expand(w.list, n, L.st, L.lat, e.s);
        r = compact_count(e, L.st, n_nodes, ST_PEND, ST_PEND, w.cscratch, w.list, n_nodes, 0,
                          L.lat, &n);
        if (r) return r;
        fresh = true;
        if (n) ++waves;
      }
      st.waves = (uint32_t)waves;
    }
    int r = check_launch();
    if (r) return r;
    // a level that ended on an empty wave has its counters from that wave's read-back
    if (!fresh) r = read_counters(e, C_SHADOW + 1);
    if (r) return r;
    st.conflicts = e.ctx->host_counters[C_CONFLICTS];
    st.b0 = e.ctx->host_counters[C_B0];
    if (stats) stats[t] = st;
  }
  return PIFU_OK;
}

// Octree subdivision (the baselines of Sec. 3.2 / Fig. 3): levels 0..T of the input-view
// grid.  Level 0 is evaluated densely; level t evaluates every node of the level-(t-1)
// cells that `mode` subdivides and that was not evaluated before.  The cell flags live in
// w.lab until the level's evaluation rewrites it.
int octree_levels(EvalCtx& e, const FieldPrep& fp, const EvalWs& ew, int T, LevelBuf* lv,
                  const LocalizeWs& w, uint8_t* eval_level, Lat eval_lat, int mode, double thr,
                  pifu_level_stats* stats) {
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  for (int t = 0; t <= T; ++t) {
    LevelBuf& L = lv[t];
    pifu_level_stats st;
    std::memset(&st, 0, sizeof(st));
    st.level = L.level_id;
    st.nodes = (uint32_t)L.lat.n();
    src.nx = L.lat.nx;
    src.ny = L.lat.ny;
    src.nz = L.lat.nz;
    const int stride = (eval_lat.nx - 1) / (L.lat.nx - 1);
    const uint32_t n_nodes = (uint32_t)L.lat.n();
    HIP_TRY(hipMemsetAsync(e.counters, 0, sizeof(uint32_t) * C_OVF, e.s));   // keeps C_OVF
    e.sel_base = 0;
    uint32_t n = n_nodes;
    if (t == 0) {
      launch_fill_u8(L.st, 0, n_nodes, e.s);
      launch_iota(w.list, n_nodes, e.s);
    } else {
      LevelBuf& Cc = lv[t - 1];
      launch_oct_flags(Cc.st, Cc.occ, Cc.lat, mode, thr, w.lab, e.counters + C_B0, e.s);
      launch_oct_transition(Cc.st, Cc.occ, Cc.lat, w.lab, L.st, L.occ, L.lat, mode, e.s);
      int r = compact_count(e, L.st, n_nodes, ST_PEND, ST_PEND, w.cscratch, w.list, n_nodes, 0,
                            L.lat, &n);
      if (r) return r;
      st.b0 = e.ctx->host_counters[C_B0];
    }
    int r = eval_occupancy(e, fp, src, w.list, n, ew, w.logit, w.lab, &st);
    if (r) return r;
    launch_apply_grid(w.list, n, w.logit, w.lab, L.st, L.occ, nullptr, eval_level, L.level_id,
                      L.lat, stride, eval_lat, 0, e.s);
    r = check_launch();
    if (r) return r;
    st.dilated = n;
    st.evaluated = n;
    if (stats) stats[t] = st;
  }
  return PIFU_OK;
}

// ------------------------------------------------------------------ occupancy grid layout
struct GridWs {
  LevelBuf lv[11];
  LocalizeWs w;
  EvalWs ew;
  FieldPrep fp;
  uint32_t* counters;
  uint32_t* aw = nullptr;    // device-driven calls: count words
  int T;
  int log2[3];
  size_t bytes;
};

// async_cap > 0: the layout of the device-driven call, whose evaluations hold up to
// async_cap points in one pass.
int plan_grid(const pifu_field* field, const pifu_grid_opts* o, void* base, float* occ_out,
              GridWs& g, uint32_t async_cap = 0) {
  const int L = o->log2_final;
  const int l0 = o->dense ? L : o->log2_coarse;
  g.T = L - l0;
  g.log2[0] = g.log2[1] = g.log2[2] = L;
  Carver cv(base);
  g.counters = cv.take<uint32_t>(kCounters);
  size_t max_n = 0;
  for (int t = 0; t <= g.T; ++t) {
    LevelBuf& b = g.lv[t];
    b.lat = level_lattice(g.log2, g.T, t);
    b.level_id = L - (g.T - t);
    b.st = cv.take<uint8_t>(b.lat.n() + 16);
    b.occ = (t == g.T) ? occ_out : cv.take<float>(b.lat.n());
    max_n = std::max(max_n, b.lat.n());
  }
  g.w.list = cv.take<uint32_t>(max_n);
  g.w.cscratch = cv.take<uint32_t>(compact_scratch_words(max_n));
  g.w.logit = cv.take<float>(max_n);
  g.w.lab = cv.take<uint8_t>(max_n);
  carve_field(cv, field, o->precision, g.fp);
  const int C = net_channels(g.fp);
  const int mh = net_hidden(g.fp);
  if (async_cap) {
    g.aw = cv.take<uint32_t>(AW_COUNT_WORDS);
    const uint32_t cap = (uint32_t)std::min<size_t>(async_cap, max_n);
    if (g.fp.has_mlp) {
      carve_eval(cv, cap, C, mh, g.ew, true);
      carve_guard(cv, g.fp, cap, g.ew);
      const Lat fin = g.lv[g.T].lat;
      carve_hoist(cv, hoist_np(g.fp), g.ew, (uint32_t)fin.nx * fin.ny);
    }
  } else {
    carve_eval(cv, (uint32_t)max_n, C, mh, g.ew);
    carve_guard(cv, g.fp, (uint32_t)max_n, g.ew);
    carve_hoist(cv, hoist_np(g.fp), g.ew);
  }
  g.bytes = cv.off + kAlign;
  return PIFU_OK;
}

int validate_grid_opts(const pifu_field* field, const pifu_grid_opts* o) {
  if (!o) return PIFU_ERR_INVALID_ARGUMENT;
  if (o->log2_final < 1 || o->log2_final > 9) return PIFU_ERR_INVALID_ARGUMENT;
  if (!o->dense && (o->log2_coarse < 1 || o->log2_coarse > o->log2_final))
    return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_precision(o->precision);
  if (r) return r;
  r = validate_field(field, 1, 1);
  if (r) return r;
  // the lifting network runs in FP32 (with the FP64 guard), without a surrogate
  if (field->kind == PIFU_FIELD_CBN && o->precision != PIFU_PREC_FP32) return PIFU_ERR_UNSUPPORTED;
  return PIFU_OK;
}

// ------------------------------------------------------------------ render layout
struct RenderWs {
  LevelBuf lv[11];
  LocalizeWs w;
  EvalWs ew;
  FieldPrep fp, cp;
  uint32_t* counters;
  uint32_t* aw = nullptr;    // device-driven calls: count words
  uint32_t *cnt, *kstar, *off, *scan_scratch, *hitlist;
  float4* hitpts;
  int T;
  int log2[3];
  size_t bytes;
};

int validate_render_opts(const pifu_field* occ, const pifu_field* col, const pifu_render_opts* o) {
  if (!o) return PIFU_ERR_INVALID_ARGUMENT;
  if (o->log2_w < 2 || o->log2_w > 10 || o->log2_d < 2 || o->log2_d > 10)
    return PIFU_ERR_INVALID_ARGUMENT;
  const int T = o->log2_w - o->log2_coarse_w;
  if (T < 1 || o->log2_coarse_w < 1 || o->log2_d - T < 1) return PIFU_ERR_INVALID_ARGUMENT;
  const double nodes = std::ldexp(1.0, o->log2_w) * std::ldexp(1.0, o->log2_w) *
                       (std::ldexp(1.0, o->log2_d) + 1.0);
  if (nodes >= 4294967295.0) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_precision(o->precision);
  if (r) return r;
  r = validate_field(occ, 1, 1);
  if (r) return r;
  if (occ->kind == PIFU_FIELD_CBN) return PIFU_ERR_UNSUPPORTED;
  if (!col || col->kind != PIFU_FIELD_MLP) return PIFU_ERR_INVALID_ARGUMENT;
  return validate_field(col, 2, 3);
}

int plan_render(const pifu_field* occ, const pifu_field* col, const pifu_render_opts* o, void* base,
                RenderWs& g, uint32_t async_cap = 0) {
  g.T = o->log2_w - o->log2_coarse_w;
  g.log2[0] = g.log2[1] = o->log2_w;
  g.log2[2] = o->log2_d;
  Carver cv(base);
  g.counters = cv.take<uint32_t>(kCounters);
  size_t max_n = 0;
  for (int t = 0; t < g.T; ++t) {
    LevelBuf& b = g.lv[t];
    b.lat = level_lattice(g.log2, g.T, t);
    b.level_id = o->log2_w - (g.T - t);
    b.st = cv.take<uint8_t>(b.lat.n() + 16);
    b.occ = cv.take<float>(b.lat.n());
    max_n = std::max(max_n, b.lat.n());
  }
  const size_t W = (size_t)1 << o->log2_w, D = (size_t)1 << o->log2_d;
  const size_t ncol = W * W;
  const size_t last_n = ncol * (D + 1);
  max_n = std::max(max_n, last_n);
  g.w.list = cv.take<uint32_t>(max_n);
  g.w.cscratch = cv.take<uint32_t>(std::max(compact_scratch_words(max_n), scan_scratch_words(ncol)));
  g.w.logit = cv.take<float>(max_n);
  g.w.lab = cv.take<uint8_t>(max_n);
  g.cnt = cv.take<uint32_t>(ncol);
  g.kstar = cv.take<uint32_t>(ncol);
  g.off = cv.take<uint32_t>(ncol);
  g.scan_scratch = cv.take<uint32_t>(scan_scratch_words(ncol));
  g.hitlist = cv.take<uint32_t>(ncol);
  g.hitpts = cv.take<float4>(ncol);
  carve_field(cv, occ, o->precision, g.fp);
  // 16-bit runs colour the hits with FP32-accurate split-FP16 products (binary16 hi / lo
  // copies of the colour network; a value outside the binary16 range re-runs them in
  // FP32); FP32 and FP8 runs in FP32
  const bool col16 = o->precision == PIFU_PREC_FP16 || o->precision == PIFU_PREC_BF16;
  carve_field(cv, col, col16 ? PIFU_PREC_FP16 : PIFU_PREC_FP32, g.cp);
  int C = 0, mh = 0;
  if (g.fp.has_mlp) {
    C = occ->C;
    mh = g.fp.mlp.max_hidden;
  }
  C = std::max(C, col->C);
  mh = std::max(mh, g.cp.mlp.max_hidden);
  if (async_cap) {
    // every evaluation, the colour of all W x W pixels included, fits one pass
    g.aw = cv.take<uint32_t>(AW_COUNT_WORDS);
    const uint32_t cap = (uint32_t)std::min<size_t>(std::max<size_t>(async_cap, ncol), max_n);
    carve_eval(cv, cap, C, mh, g.ew, true);
    carve_guard(cv, g.fp, cap, g.ew);
  } else {
    carve_eval(cv, (uint32_t)max_n, C, mh, g.ew);
    carve_guard(cv, g.fp, (uint32_t)max_n, g.ew);
  }
  // the texel table serves the plain FP32 render (the bands of BF16 and FP16 renders run on
  // split-FP16 products and do not read it; FP8 renders keep the plain path throughout)
  if (o->precision == PIFU_PREC_FP32) carve_texel(cv, g.fp, g.ew);
  g.bytes = cv.off + kAlign;
  return PIFU_OK;
}

hipStream_t as_stream(pifu_stream s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// ================================================================== C ABI
extern "C" {

}  // extern "C"

namespace {

pifu_ctx* ctx_new(int dev) {
  pifu_ctx* c = new (std::nothrow) pifu_ctx;
  if (!c) return nullptr;
  c->device = dev;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_counters),
                    sizeof(uint32_t) * (kHostWords + 64),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete c;
    return nullptr;
  }
  std::memset(c->host_counters, 0, sizeof(uint32_t) * (kHostWords + 64));
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&c->host_counters_dev), c->host_counters,
                              0) != hipSuccess) {
    (void)hipHostFree(c->host_counters);
    delete c;
    return nullptr;
  }
  return c;
}

}  // namespace

int pifu::ctx_device(const pifu_ctx* c) { return c ? c->device : -1; }

namespace {

void ctx_free(pifu_ctx* c) {
  if (!c) return;
  if (c->host_counters) (void)hipHostFree(c->host_counters);
  if (c->prof_slots) (void)hipHostFree(c->prof_slots);
  for (hipEvent_t ev : c->events) (void)hipEventDestroy(ev);
  delete c;
}

void prof_enable_one(pifu_ctx* c, bool on) {
  c->prof_on = on;
  if (on && !c->prof_slots &&
      hipHostMalloc(reinterpret_cast<void**>(&c->prof_slots), sizeof(uint32_t) * kProfSlots,
                    hipHostMallocDefault) != hipSuccess) {
    c->prof_slots = nullptr;   // counted launches then report their fixed part only
  }
  c->pending.clear();
  c->prof_used = 0;
  std::memset(c->prof, 0, sizeof(c->prof));
}

}  // namespace

extern "C" {

int32_t pifu_create(pifu_ctx** out) {
  if (!out) return PIFU_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PIFU_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return PIFU_ERR_HIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PIFU_ERR_UNSUPPORTED;
  if (int r = pifu::noalloc_setup(dev)) return r;
  if (int r = pifu::mesh_table_upload()) return r;
  pifu_ctx* c = ctx_new(dev);
  if (!c) return PIFU_ERR_HIP;
  c->peer = ctx_new(dev);
  if (!c->peer) {
    ctx_free(c);
    return PIFU_ERR_HIP;
  }
  *out = c;
  return PIFU_OK;
}

void pifu_destroy(pifu_ctx* ctx) {
  if (!ctx) return;
  ctx_free(ctx->peer);
  ctx_free(ctx);
}

const char* pifu_status_string(int32_t s) {
  switch (s) {
    case PIFU_OK: return "ok";
    case PIFU_ERR_INVALID_ARGUMENT: return "invalid argument";
    case PIFU_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case PIFU_ERR_UNSUPPORTED: return "unsupported";
    case PIFU_ERR_HIP: return "HIP runtime error";
    case PIFU_ERR_SCRATCH_TOO_SMALL:
      return "the options need more workspace than the no-allocation entry point's fixed scratch";
    default: return "unknown status";
  }
}

int32_t pifu_occupancy_grid_workspace_size(const pifu_field* field, const pifu_grid_opts* opts,
                                           size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_grid_opts(field, opts);
  if (r) return r;
  GridWs* g = new (std::nothrow) GridWs;
  if (!g) return PIFU_ERR_HIP;
  plan_grid(field, opts, nullptr, nullptr, *g);
  *bytes = g->bytes;
  delete g;
  return PIFU_OK;
}

int32_t pifu_occupancy_grid(pifu_ctx* ctx, const pifu_field* field, const pifu_grid_opts* opts,
                            float* occ, uint8_t* labels, uint8_t* eval_level, uint32_t* cells,
                            uint32_t cells_cap, uint32_t* n_cells, pifu_level_stats* stats,
                            void* workspace, size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !occ || !labels || !n_cells || !workspace) return PIFU_ERR_INVALID_ARGUMENT;
  if (cells_cap && !cells) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_grid_opts(field, opts);
  if (r) return r;
  GridWs* gp = new (std::nothrow) GridWs;
  if (!gp) return PIFU_ERR_HIP;
  GridWs& g = *gp;
  plan_grid(field, opts, nullptr, nullptr, g);
  if (workspace_bytes < g.bytes) {
    delete gp;
    return PIFU_ERR_WORKSPACE_TOO_SMALL;
  }
  void* base = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(workspace) + kAlign - 1) /
                                       kAlign * kAlign);
  plan_grid(field, opts, base, occ, g);
  hipStream_t s = as_stream(stream);
  EvalCtx e{ctx, s, g.counters, opts->precision, opts->guard_logit};
  e.band = logit_band(opts->band_delta);
  e.sur_band = logit_band(opts->surrogate_delta);
  e.tile_m = opts->tile_m;
  if (int pr = pack_field(g.fp, ctx, s, g.counters)) {
    delete gp;
    return pr;
  }
  const Lat fin = g.lv[g.T].lat;
  if (eval_level) launch_fill_u8(eval_level, 255, fin.n(), s);
  r = localize(e, g.fp, g.ew, nullptr, g.log2, g.T, g.T, g.lv, g.w, eval_level, fin,
               opts->max_waves, opts->surrogate_max_log2, stats);
  if (!r) {
    launch_cells(g.lv[g.T].st, fin, labels, s);
    uint32_t nc = 0;
    r = compact_count(e, g.lv[g.T].st, fin.n(), ST_CELL, ST_CELL, g.w.cscratch, cells, cells_cap,
                      1, fin, &nc);
    *n_cells = nc;
  }
  if (!r) r = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  prof_resolve(ctx);
  delete gp;
  return r;
}

int32_t pifu_octree_grid(pifu_ctx* ctx, const pifu_field* field, const pifu_grid_opts* opts,
                         int32_t mode, double threshold, float* occ, uint8_t* labels,
                         uint8_t* eval_level, uint32_t* cells, uint32_t cells_cap,
                         uint32_t* n_cells, pifu_level_stats* stats, void* workspace,
                         size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !occ || !labels || !n_cells || !workspace) return PIFU_ERR_INVALID_ARGUMENT;
  if (cells_cap && !cells) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  if (mode != PIFU_OCTREE_BINARIZED && mode != PIFU_OCTREE_THRESHOLD)
    return PIFU_ERR_INVALID_ARGUMENT;
  if (mode == PIFU_OCTREE_THRESHOLD && !(threshold >= 0.0)) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_grid_opts(field, opts);
  if (r) return r;
  if (opts->dense) return PIFU_ERR_INVALID_ARGUMENT;
  GridWs* gp = new (std::nothrow) GridWs;
  if (!gp) return PIFU_ERR_HIP;
  GridWs& g = *gp;
  plan_grid(field, opts, nullptr, nullptr, g);
  if (workspace_bytes < g.bytes) {
    delete gp;
    return PIFU_ERR_WORKSPACE_TOO_SMALL;
  }
  plan_grid(field, opts, workspace, occ, g);
  hipStream_t s = as_stream(stream);
  EvalCtx e{ctx, s, g.counters, opts->precision, opts->guard_logit};
  e.band = logit_band(opts->band_delta);
  e.tile_m = opts->tile_m;
  if (int pr = pack_field(g.fp, ctx, s, g.counters)) {
    delete gp;
    return pr;
  }
  const Lat fin = g.lv[g.T].lat;
  if (eval_level) launch_fill_u8(eval_level, 255, fin.n(), s);
  r = octree_levels(e, g.fp, g.ew, g.T, g.lv, g.w, eval_level, fin, mode, threshold, stats);
  if (!r) {
    launch_cells(g.lv[g.T].st, fin, labels, s);
    uint32_t nc = 0;
    r = compact_count(e, g.lv[g.T].st, fin.n(), ST_CELL, ST_CELL, g.w.cscratch, cells, cells_cap,
                      1, fin, &nc);
    *n_cells = nc;
  }
  if (!r) r = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  prof_resolve(ctx);
  delete gp;
  return r;
}

int32_t pifu_render_view_workspace_size(const pifu_field* occ_field, const pifu_field* color_field,
                                        const pifu_render_opts* opts, size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_render_opts(occ_field, color_field, opts);
  if (r) return r;
  RenderWs* g = new (std::nothrow) RenderWs;
  if (!g) return PIFU_ERR_HIP;
  plan_render(occ_field, color_field, opts, nullptr, *g);
  *bytes = g->bytes;
  delete g;
  return PIFU_OK;
}

}  // extern "C"

namespace {

int32_t render_impl(pifu_ctx* ctx, const pifu_field* occ_field, const pifu_field* color_field,
                    const float* view, const pifu_render_opts* opts, const float* bg, float* rgb,
                    float* depth, uint8_t* hit, pifu_level_stats* stats, void* workspace,
                    size_t workspace_bytes, pifu_stream stream, const pifu_render_trace* trace) {
  if (!ctx || !view || !bg || !rgb || !depth || !hit || !workspace) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_render_opts(occ_field, color_field, opts);
  if (r) return r;
  RenderWs* gp = new (std::nothrow) RenderWs;
  if (!gp) return PIFU_ERR_HIP;
  RenderWs& g = *gp;
  plan_render(occ_field, color_field, opts, nullptr, g);
  if (workspace_bytes < g.bytes) {
    delete gp;
    return PIFU_ERR_WORKSPACE_TOO_SMALL;
  }
  void* base = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(workspace) + kAlign - 1) /
                                       kAlign * kAlign);
  plan_render(occ_field, color_field, opts, base, g);
  hipStream_t s = as_stream(stream);
  EvalCtx e{ctx, s, g.counters, opts->precision, opts->guard_logit};
  e.band = logit_band(opts->band_delta);
  e.sur_band = logit_band(opts->surrogate_delta);
  e.tile_m = opts->tile_m;
  if (int pr = pack_field(g.fp, ctx, s, g.counters)) {
    delete gp;
    return pr;
  }
  // one clear of the overflow flag per call: by the occupancy network's pack when it has
  // binary16 copies (FP16, BF16)
  if (int pr = pack_field(g.cp, ctx, s, g.counters, !split_band(g.fp))) {
    delete gp;
    return pr;
  }
  if (int pr = fill_texel(e, g.fp, g.ew)) {
    delete gp;
    return pr;
  }
  double vd[12];
  for (int i = 0; i < 12; ++i) vd[i] = view[i];
  const int T = g.T;
  const int W = 1 << opts->log2_w, H = W, D = 1 << opts->log2_d;
  const Lat finL = level_lattice(g.log2, T, T);
  uint8_t* tr_level = trace ? trace->eval_level : nullptr;
  float* tr_logit = trace ? trace->logit : nullptr;
  if (tr_level) launch_fill_u8(tr_level, 255, finL.n(), s);
  if (trace && trace->kstar) launch_fill_i32(trace->kstar, -1, (size_t)W * H, s);
  if (trace && trace->k1) launch_fill_i32(trace->k1, -1, (size_t)W * H, s);
  r = localize(e, g.fp, g.ew, vd, g.log2, T, T - 1, g.lv, g.w, tr_level, finL, opts->max_waves,
               opts->surrogate_max_log2, stats, tr_logit);
  if (r) {
    delete gp;
    return r;
  }
  // last level: interpolate, argmax along z from the observer, shadow nodes
  pifu_level_stats st;
  std::memset(&st, 0, sizeof(st));
  st.level = opts->log2_w;
  st.nodes = (uint32_t)((size_t)W * H * (D + 1));
  const LevelBuf& C = g.lv[T - 1];
  HIP_TRY(hipMemsetAsync(g.counters, 0, sizeof(uint32_t) * C_OVF, s));   // keeps C_OVF
  e.sel_base = 0;
  launch_fill_image(rgb, depth, hit, (uint32_t)(W * H), bg[0], bg[1], bg[2], s);
  launch_ray_count(C.st, C.lat, W, H, D, g.cnt, g.kstar, g.counters + C_SHADOW, s);
  launch_scan_u32(g.cnt, (uint32_t)(W * H), g.off, g.scan_scratch, g.counters + C_TOTAL, s);
  r = check_launch();
  if (!r) r = read_counters(e, C_SHADOW + 1);
  uint32_t nT = 0;
  if (!r) {
    nT = ctx->host_counters[C_TOTAL];
    st.shadow = ctx->host_counters[C_SHADOW];
    launch_ray_list(C.st, C.lat, W, H, D, g.kstar, g.off, g.w.list, s);
    PointSrc src;
    std::memset(&src, 0, sizeof(src));
    src.mode = 0;
    src.nx = finL.nx;
    src.ny = finL.ny;
    src.nz = finL.nz;
    src.has_view = 1;
    for (int i = 0; i < 12; ++i) src.view[i] = vd[i];
    r = eval_occupancy(e, g.fp, src, g.w.list, nT, g.ew, g.w.logit, g.w.lab, &st,
                       opts->log2_w <= opts->surrogate_max_log2);
    st.dilated = nT;
    st.evaluated = nT;
    if (!r) launch_trace_scatter(g.w.list, nT, g.w.logit, opts->log2_w, tr_level, tr_logit, s);
  }
  if (!r) {
    launch_ray_hit(C.st, C.occ, C.lat, W, H, D, g.off, g.cnt, g.w.list, g.w.logit, g.w.lab, vd,
                   depth, hit, g.hitpts, s, trace ? trace->kstar : nullptr,
                   trace ? trace->k1 : nullptr);
    uint32_t nh = 0;
    Lat img{1, 1, W * H};
    r = compact_count(e, hit, (size_t)W * H, 1, 1, g.w.cscratch, g.hitlist, (uint32_t)(W * H), 0,
                      img, &nh);
    st.hits = nh;
    if (!r && nh) {
      PointSrc ps;
      std::memset(&ps, 0, sizeof(ps));
      ps.mode = 1;
      ps.pts = g.hitpts;
      EvalCtx ec{ctx, s, g.counters, PIFU_PREC_FP32, 0.f};
      // split-FP16 colour unless a value of this call already left the binary16 range;
      // the split kernels report their own operands, and an overflow re-runs in FP32
      const bool x3 = g.cp.mlp.prec == PIFU_PREC_FP16 && ctx->host_counters[C_OVF] == 0;
      r = run_mlp(ec, g.cp, g.cp.mlp, x3 ? PREC_F32X3 : PIFU_PREC_FP32, ps, g.hitlist, nh, g.ew,
                  nullptr, nullptr, rgb);
      if (!r && x3) r = read_counters(e, C_OVF + 1);
      if (!r && x3 && ctx->host_counters[C_OVF])
        r = run_mlp(ec, g.cp, g.cp.mlp, PIFU_PREC_FP32, ps, g.hitlist, nh, g.ew, nullptr, nullptr,
                    rgb);
    }
  }
  if (!r) r = check_launch();
  if (!r) r = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  if (stats) stats[T] = st;
  prof_resolve(ctx);
  delete gp;
  return r;
}

}  // namespace

extern "C" {

int32_t pifu_render_view(pifu_ctx* ctx, const pifu_field* occ_field, const pifu_field* color_field,
                         const float* view, const pifu_render_opts* opts, const float* bg,
                         float* rgb, float* depth, uint8_t* hit, pifu_level_stats* stats,
                         void* workspace, size_t workspace_bytes, pifu_stream stream) {
  return render_impl(ctx, occ_field, color_field, view, opts, bg, rgb, depth, hit, stats,
                     workspace, workspace_bytes, stream, nullptr);
}

int32_t pifu_render_view_traced(pifu_ctx* ctx, const pifu_field* occ_field,
                                const pifu_field* color_field, const float* view,
                                const pifu_render_opts* opts, const float* bg, float* rgb,
                                float* depth, uint8_t* hit, pifu_level_stats* stats,
                                void* workspace, size_t workspace_bytes, pifu_stream stream,
                                const pifu_render_trace* trace) {
  if (!trace) return PIFU_ERR_INVALID_ARGUMENT;
  return render_impl(ctx, occ_field, color_field, view, opts, bg, rgb, depth, hit, stats,
                     workspace, workspace_bytes, stream, trace);
}

// One frame: the grid on the calling thread, the render on a second host thread with
// the companion state (its own pinned read-back words, events and profile records).
// Both argument sets are checked before either call starts, so a rejected frame
// launches nothing.
int32_t pifu_grid_and_render(pifu_ctx* ctx, const pifu_grid_call* gc, const pifu_render_call* rc) {
  if (!ctx || !gc || !rc) return PIFU_ERR_INVALID_ARGUMENT;
  if (!gc->occ || !gc->labels || !gc->n_cells || !gc->workspace || (gc->cells_cap && !gc->cells) ||
      !aligned(gc->workspace, kAlign))
    return PIFU_ERR_INVALID_ARGUMENT;
  if (!rc->view || !rc->bg || !rc->rgb || !rc->depth || !rc->hit || !rc->workspace ||
      !aligned(rc->workspace, kAlign))
    return PIFU_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  if (int r = pifu_occupancy_grid_workspace_size(gc->field, gc->opts, &need)) return r;
  if (gc->workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  if (int r = pifu_render_view_workspace_size(rc->occ_field, rc->color_field, rc->opts, &need))
    return r;
  if (rc->workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;

  auto grid = [gc](pifu_ctx* c) -> int32_t {
    return pifu_occupancy_grid(c, gc->field, gc->opts, gc->occ, gc->labels, gc->eval_level,
                               gc->cells, gc->cells_cap, gc->n_cells, gc->stats, gc->workspace,
                               gc->workspace_bytes, gc->stream);
  };
  auto render = [rc](pifu_ctx* c) -> int32_t {
    return pifu_render_view(c, rc->occ_field, rc->color_field, rc->view, rc->opts, rc->bg,
                            rc->rgb, rc->depth, rc->hit, rc->stats, rc->workspace,
                            rc->workspace_bytes, rc->stream);
  };
  pifu_ctx* p = ctx->peer;
  std::thread t;
  int32_t r_render = PIFU_OK;
  if (p && gc->stream != rc->stream) {
    try {
      p->tile_cache = ctx->tile_cache;   // the render picks the same autotuned tiles
      t = std::thread([p, &render, &r_render] {
        r_render = hipSetDevice(p->device) == hipSuccess ? render(p) : PIFU_ERR_HIP;
      });
    } catch (...) {
      // no second thread: the render runs after the grid on this thread
    }
  }
  const int32_t r_grid = grid(ctx);
  if (t.joinable()) t.join();
  else r_render = render(ctx);
  return r_grid ? r_grid : r_render;
}

int32_t pifu_eval_points_workspace_size(const pifu_field* field, int32_t precision, uint32_t n,
                                        size_t* bytes) {
  if (!bytes || !field) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_precision(precision);
  if (r) return r;
  r = validate_field(field, 1, 1);
  if (r) return r;
  if (field->kind == PIFU_FIELD_CBN && precision != PIFU_PREC_FP32) return PIFU_ERR_UNSUPPORTED;
  Carver cv(nullptr);
  cv.take<uint32_t>(kCounters);
  cv.take<uint32_t>(std::max<uint32_t>(n, 1));
  FieldPrep fp;
  carve_field(cv, field, precision, fp);
  EvalWs ew;
  carve_eval(cv, std::max<uint32_t>(n, 1), net_channels(fp), net_hidden(fp), ew);
  carve_guard(cv, fp, std::max<uint32_t>(n, 1), ew);
  if (fp.has_cbn) carve_hoist(cv, hoist_np(fp), ew);
  *bytes = cv.off + kAlign;
  return PIFU_OK;
}

int32_t pifu_eval_points(pifu_ctx* ctx, const pifu_field* field, int32_t precision,
                         float band_delta, float guard_logit, const float* pts, uint32_t n,
                         float* logit, uint8_t* labels, float* occ, void* workspace,
                         size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !pts || !logit || !workspace) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(pts, 16) || !aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  int r = pifu_eval_points_workspace_size(field, precision, n, &need);
  if (r) return r;
  if (workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  if (!n) return PIFU_OK;
  Carver cv(workspace);
  uint32_t* counters = cv.take<uint32_t>(kCounters);
  uint32_t* iota = cv.take<uint32_t>(n);
  FieldPrep fp;
  carve_field(cv, field, precision, fp);
  EvalWs ew;
  carve_eval(cv, n, net_channels(fp), net_hidden(fp), ew);
  carve_guard(cv, fp, n, ew);
  if (fp.has_cbn) carve_hoist(cv, hoist_np(fp), ew);
  hipStream_t s = as_stream(stream);
  uint8_t* lab = labels;
  if (!lab) lab = reinterpret_cast<uint8_t*>(ew.glist);   // scratch when labels are not wanted
  EvalCtx e{ctx, s, counters, precision, guard_logit};
  e.band = logit_band(band_delta);
  HIP_TRY(hipMemsetAsync(counters, 0, sizeof(uint32_t) * C_OVF, s));   // selection counter = 0
  if (int pr = pack_field(fp, ctx, s, counters)) return pr;
  launch_iota(iota, n, s);
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 1;
  src.pts = reinterpret_cast<const float4*>(pts);
  if (!labels && (fp.has_mlp || fp.has_cbn) && guard_logit > 0.f) return PIFU_ERR_INVALID_ARGUMENT;
  r = eval_occupancy(e, fp, src, iota, n, ew, logit, lab, nullptr);
  if (!r && occ) launch_occupancy(logit, n, occ, s);
  if (!r) r = check_launch();
  if (!r) r = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  prof_resolve(ctx);
  return r;
}

int32_t pifu_fp8_calibrate(pifu_ctx* ctx, const pifu_field* field, const float* pts, uint32_t n,
                           float* amax, void* workspace, size_t workspace_bytes,
                           pifu_stream stream) {
  if (!ctx || !pts || !amax || !workspace || !n) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(pts, 16) || !aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  if (!field || field->kind != PIFU_FIELD_MLP) return PIFU_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  int r = pifu_eval_points_workspace_size(field, PIFU_PREC_FP32, n, &need);
  if (r) return r;
  if (workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  Carver cv(workspace);
  uint32_t* counters = cv.take<uint32_t>(kCounters);
  uint32_t* iota = cv.take<uint32_t>(n);
  FieldPrep fp;
  carve_field(cv, field, PIFU_PREC_FP32, fp);
  fp.has_sur = false;
  EvalWs ew;
  carve_eval(cv, n, field->C, fp.mlp.max_hidden, ew);
  carve_guard(cv, fp, n, ew);
  hipStream_t s = as_stream(stream);
  EvalCtx e{ctx, s, counters, PIFU_PREC_FP32, 0.f};
  e.amax = counters + 16;
  HIP_TRY(hipMemsetAsync(counters, 0, sizeof(uint32_t) * kCounters, s));
  if (int pr = pack_field(fp, ctx, s, counters)) return pr;
  launch_iota(iota, n, s);
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 1;
  src.pts = reinterpret_cast<const float4*>(pts);
  r = run_mlp(e, fp, fp.mlp, PIFU_PREC_FP32, src, iota, n, ew, ew.band_logit, ew.band_lab, nullptr);
  if (r) return r;
  const int nh = fp.mlp.d.n_layers - 1;
  uint32_t bits[PIFU_MAX_LAYERS + 1];
  HIP_TRY(hipMemcpyAsync(bits, e.amax, sizeof(uint32_t) * (nh + 1), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float a[PIFU_MAX_LAYERS + 1];
  std::memcpy(a, bits, sizeof(float) * (nh + 1));
  for (int l = 0; l < nh; ++l) {
    // layer 0 reads [f; z] (z enters the epilogue in FP32), layer l reads [h_{l-1}; f?]
    float v = l == 0 ? a[0] : a[l];
    if (l > 0 && fp.mlp.d.skip[l]) v = std::max(v, a[0]);
    amax[l] = v;
  }
  return PIFU_OK;
}

int32_t pifu_profile_enable(pifu_ctx* ctx, int32_t on) {
  if (!ctx) return PIFU_ERR_INVALID_ARGUMENT;
  prof_enable_one(ctx, on != 0);
  if (ctx->peer) prof_enable_one(ctx->peer, on != 0);
  return PIFU_OK;
}

// Autotuner: times every hidden layer of the field's network (and of its surrogate)
// with point tiles 64, 128 and 256 on m gathered lattice points, and caches the
// fastest per (precision, layer shape, batch bucket).  A tile within 3% of the
// fastest loses to 128 (then to the smaller tile), so ties break deterministically.
// All tiles give bit-identical results (same k order), so tuning never changes output.
int32_t pifu_autotune_mlp(pifu_ctx* ctx, const pifu_field* field, int32_t precision, uint32_t m,
                          int32_t* chosen, void* workspace, size_t workspace_bytes,
                          pifu_stream stream) {
  if (!ctx || !workspace || m == 0 || !field || field->kind != PIFU_FIELD_MLP)
    return PIFU_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  int r = pifu_eval_points_workspace_size(field, precision, m, &need);
  if (r) return r;
  if (workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  Carver cv(workspace);
  uint32_t* counters = cv.take<uint32_t>(kCounters);
  uint32_t* iota = cv.take<uint32_t>(m);
  FieldPrep fp;
  carve_field(cv, field, precision, fp);
  EvalWs ew;
  carve_eval(cv, m, field->C, fp.mlp.max_hidden, ew);
  (void)counters;
  hipStream_t s = as_stream(stream);
  if (int pr = pack_field(fp, ctx, s, counters)) return pr;
  launch_iota(iota, m, s);
  // points: the first m nodes of a 129^3 lattice (z fastest), i.e. whole columns
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  src.nx = src.ny = src.nz = 129;
  const uint32_t mm = std::min<uint32_t>(m, ew.chunk);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PIFU_ERR_HIP;
  int out_i = 0;
  for (int net = 0; net < 2; ++net) {
    if (net == 1 && !fp.has_sur) break;
    const MlpPrep& mp = net ? fp.sur : fp.mlp;
    const int prec = net ? PIFU_PREC_BF16 : precision;
    const bool b16 = prec != PIFU_PREC_FP32;
    launch_gather(src, iota, mm, field->feat, field->H, field->W, field->C, ew.feat, h16_fmt(prec),
                  ew.ext, s);
    const MLPDesc& d = mp.d;
    const void* prev = nullptr;
    void* out = ew.hA;
    for (int l = 0; l + 1 < d.n_layers; ++l) {
      GemmArgs g;
      std::memset(&g, 0, sizeof(g));
      if (l == 0) {
        g.A1 = ew.feat;
        g.K1 = field->C;
        g.lda1 = field->C;
        g.n_ext = d.n_extra;
        g.ext_col = field->C;
      } else {
        g.A1 = prev;
        g.K1 = g.lda1 = d.widths[l - 1];
        if (d.skip[l]) {
          g.A2 = ew.feat;
          g.K2 = g.lda2 = field->C;
        }
      }
      g.W = layer_weights(mp, prec, l);
      g.a_inv_scale = prec == PIFU_PREC_FP8 ? 1.f / mp.a_scale[l] : 1.f;
      g.ldw = mp.Kp[l];
      g.Wf = d.W[l];
      g.ldwf = d.in_w[l];
      g.bias = d.b[l];
      g.ext = ew.ext;
      g.C = out;
      g.ldc = g.N = d.widths[l];
      g.M = (int)mm;
      g.act = d.hidden_act;
      g.scale = prec == PIFU_PREC_FP8 ? mp.a_scale[l] * mp.w_scale[l] : 1.f;
      g.c_bf16 = b16 && (l + 2 < d.n_layers);
      const int tiles[3] = {64, 128, 256};
      float best[3];
      for (int t = 0; t < 3; ++t) {
        launch_gemm(g, prec, tiles[t], s);   // warm-up
        float tot = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
          (void)hipEventRecord(e0, s);
          launch_gemm(g, prec, tiles[t], s);
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) return PIFU_ERR_HIP;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          tot += ms;
        }
        best[t] = tot;
      }
      const float fastest = std::min(best[0], std::min(best[1], best[2]));
      const int pref[3] = {1, 0, 2};   // 128, then 64, then 256
      int pick = 128;
      for (int q = 0; q < 3; ++q)
        if (best[pref[q]] <= 1.03f * fastest) {
          pick = tiles[pref[q]];
          break;
        }
      ctx->tile_cache[tile_key(prec, g.N, g.K1 + g.K2, m)] = pick;
      if (chosen && out_i < 2 * PIFU_MAX_LAYERS) chosen[out_i] = pick;
      ++out_i;
      prev = out;
      out = out == ew.hA ? ew.hB : ew.hA;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return check_launch();
}

int32_t pifu_convert_f32(pifu_ctx* ctx, const float* in, uint32_t n, int32_t precision, void* out,
                         pifu_stream stream) {
  if (!ctx || !in || !out) return PIFU_ERR_INVALID_ARGUMENT;
  if (precision != PIFU_PREC_BF16 && precision != PIFU_PREC_FP8 && precision != PIFU_PREC_FP16)
    return PIFU_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(stream);
  launch_convert(in, n, precision, out, s);
  int r = check_launch();
  if (!r) r = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  return r;
}

int32_t pifu_autotune_clear(pifu_ctx* ctx) {
  if (!ctx) return PIFU_ERR_INVALID_ARGUMENT;
  ctx->tile_cache.clear();
  return PIFU_OK;
}

int32_t pifu_profile_read(pifu_ctx* ctx, pifu_kernel_profile* out) {
  if (!ctx || !out) return PIFU_ERR_INVALID_ARGUMENT;
  std::memcpy(out, ctx->prof, sizeof(ctx->prof));
  if (const pifu_ctx* p = ctx->peer) {   // launches made by pifu_grid_and_render's second thread
    for (int k = 0; k < PIFU_KERN_COUNT; ++k) {
      out[k].launches += p->prof[k].launches;
      out[k].total_ms += p->prof[k].total_ms;
      out[k].flops += p->prof[k].flops;
      out[k].bytes += p->prof[k].bytes;
    }
  }
  return PIFU_OK;
}

}  // extern "C"

// ================================================================== surrogate training
namespace {

struct TrainWs {
  MlpPrep mp;
  float* feat;
  float* ext;
  float* H[PIFU_MAX_LAYERS];
  float* s;
  uint8_t* lab;
  float* g;
  float* dA;
  float* dB;
  float* part;
  float* loss_part;
  size_t bytes;
};

void plan_train(const pifu_field* f, uint32_t n, void* base, TrainWs& t) {
  Carver cv(base);
  carve_mlp(cv, f->mlp, PIFU_PREC_FP32, t.mp);
  const MLPDesc& d = t.mp.d;
  const size_t N = std::max<uint32_t>(n, 1);
  t.feat = cv.take<float>(N * f->C);
  t.ext = cv.take<float>(N * 4);
  size_t maxpart = 0;
  int maxw = 1;
  for (int l = 0; l < d.n_layers; ++l) {
    t.H[l] = l + 1 < d.n_layers ? cv.take<float>(N * d.widths[l]) : nullptr;
    maxpart = std::max(maxpart, weight_grad_part_floats(d.widths[l], d.in_w[l], (uint32_t)N));
    if (l + 1 < d.n_layers) maxw = std::max(maxw, d.widths[l]);
  }
  t.s = cv.take<float>(N);
  t.lab = cv.take<uint8_t>(N);
  t.g = cv.take<float>(N);
  t.dA = cv.take<float>(N * maxw);
  t.dB = cv.take<float>(N * maxw);
  t.part = cv.take<float>(maxpart);
  t.loss_part = cv.take<float>(bce_partials((uint32_t)N) + 1);
  t.bytes = cv.off + kAlign;
}

int validate_train_field(const pifu_field* f) {
  if (!f || f->kind != PIFU_FIELD_MLP) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_field(f, 1, 1);
  if (r) return r;
  const pifu_mlp* m = f->mlp;
  for (int l = 0; l + 1 < m->n_layers; ++l)
    if (m->hidden_act != PIFU_ACT_RELU && m->hidden_act != PIFU_ACT_LRELU) return PIFU_ERR_INVALID_ARGUMENT;
  return PIFU_OK;
}

}  // namespace

extern "C" {

int32_t pifu_mlp_train_workspace_size(const pifu_field* field, uint32_t max_batch, size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_train_field(field);
  if (r) return r;
  TrainWs t;
  plan_train(field, max_batch, nullptr, t);
  *bytes = t.bytes;
  return PIFU_OK;
}

int32_t pifu_mlp_grad(pifu_ctx* ctx, const pifu_field* field, const float* pts, uint32_t n,
                      float* const* dW, float* const* db, float* loss, void* workspace,
                      size_t workspace_bytes, pifu_stream stream) {
  return pifu_mlp_grad_ex(ctx, field, pts, n, dW, db, loss, nullptr, workspace, workspace_bytes,
                          stream);
}

int32_t pifu_mlp_grad_ex(pifu_ctx* ctx, const pifu_field* field, const float* pts, uint32_t n,
                         float* const* dW, float* const* db, float* loss, float* point_loss,
                         void* workspace, size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !pts || !dW || !db || !workspace || n == 0) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(pts, 16) || !aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_train_field(field);
  if (r) return r;
  TrainWs t;
  plan_train(field, n, nullptr, t);
  if (workspace_bytes < t.bytes) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  plan_train(field, n, workspace, t);
  const MLPDesc& d = t.mp.d;
  for (int l = 0; l < d.n_layers; ++l)
    if (!dW[l] || !db[l]) return PIFU_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(stream);
  if (int pr = pack_mlp(t.mp, ctx, s, nullptr)) return pr;
  const int C = field->C;
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 1;
  src.pts = reinterpret_cast<const float4*>(pts);
  // forward, keeping every hidden activation
  launch_gather(src, nullptr, n, field->feat, field->H, field->W, C, t.feat, 0, t.ext, s);
  for (int l = 0; l + 1 < d.n_layers; ++l) {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    if (l == 0) {
      g.A1 = t.feat;
      g.K1 = C;
      g.lda1 = C;
      g.n_ext = d.n_extra;
      g.ext_col = C;
    } else {
      g.A1 = t.H[l - 1];
      g.K1 = d.widths[l - 1];
      g.lda1 = d.widths[l - 1];
      if (d.skip[l]) {
        g.A2 = t.feat;
        g.K2 = C;
        g.lda2 = C;
      }
    }
    g.W = t.mp.Wp32[l];
    g.ldw = t.mp.Kp[l];
    g.Wf = d.W[l];
    g.ldwf = d.in_w[l];
    g.bias = d.b[l];
    g.ext = t.ext;
    g.C = t.H[l];
    g.ldc = d.widths[l];
    g.M = (int)n;
    g.N = d.widths[l];
    g.act = d.hidden_act;
    g.scale = 1.f;
    if (launch_gemm(g, PIFU_PREC_FP32, 0, s)) return PIFU_ERR_UNSUPPORTED;
  }
  const int L = d.n_layers - 1;
  launch_head(t.H[L - 1], d.widths[L - 1], d.W[L], d.b[L], 1, d.out_act, n, t.ext, t.s, t.lab,
              nullptr, nullptr, s);
  // loss and dloss/dlogit
  launch_bce_grad(t.s, src.pts, n, t.g, t.loss_part, loss, s, point_loss);
  // backward
  const float* G = t.g;
  int Ng = 1;
  float* bufs[2] = {t.dA, t.dB};
  int which = 0;
  for (int l = L; l >= 0; --l) {
    if (l == 0) {
      launch_weight_grad(G, Ng, t.feat, C, C, nullptr, 0, 0, t.ext, d.n_extra, n, t.part, dW[l],
                         db[l], s);
    } else {
      launch_weight_grad(G, Ng, t.H[l - 1], d.widths[l - 1], d.widths[l - 1],
                         d.skip[l] ? t.feat : nullptr, d.skip[l] ? C : 0, C, nullptr, 0, n,
                         t.part, dW[l], db[l], s);
      float* dH = bufs[which];
      which ^= 1;
      launch_backprop_input(G, Ng, d.W[l], d.in_w[l], t.H[l - 1], d.widths[l - 1], n,
                            d.hidden_act, dH, s);
      G = dH;
      Ng = d.widths[l - 1];
    }
  }
  r = check_launch();
  return r;
}

int32_t pifu_ohem_sample_workspace_size(uint32_t n, size_t* bytes) {
  if (!bytes || n == 0 || n > (1u << 27)) return PIFU_ERR_INVALID_ARGUMENT;
  *bytes = ohem_workspace_bytes(n);
  return PIFU_OK;
}

int32_t pifu_ohem_sample(pifu_ctx* ctx, const float* weights, uint32_t n, const float* pool,
                         uint32_t batch, uint64_t seed, uint64_t counter, uint32_t* idx,
                         float* batch_pts, void* workspace, size_t workspace_bytes,
                         pifu_stream stream) {
  if (!ctx || !weights || !idx || !workspace || batch == 0 || n == 0 || n > (1u << 27))
    return PIFU_ERR_INVALID_ARGUMENT;
  if (batch_pts && (!pool || !aligned(pool, 16) || !aligned(batch_pts, 16)))
    return PIFU_ERR_INVALID_ARGUMENT;
  if (workspace_bytes < ohem_workspace_bytes(n)) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  launch_ohem_sample(weights, n, reinterpret_cast<const float4*>(pool), batch, seed, counter, idx,
                     reinterpret_cast<float4*>(batch_pts), workspace, as_stream(stream));
  return check_launch();
}

int32_t pifu_ohem_update(pifu_ctx* ctx, const float* point_loss, const uint32_t* idx,
                         uint32_t batch, float alpha, float beta, float* weights,
                         pifu_stream stream) {
  if (!ctx || !point_loss || !idx || !weights || batch == 0) return PIFU_ERR_INVALID_ARGUMENT;
  if (!(alpha > 0.f) || !(beta >= 0.f)) return PIFU_ERR_INVALID_ARGUMENT;
  launch_ohem_update(point_loss, idx, batch, alpha, beta, weights, as_stream(stream));
  return check_launch();
}

int32_t pifu_rmsprop_step(pifu_ctx* ctx, const pifu_mlp* net, const float* const* dW,
                          const float* const* db, float* const* vW, float* const* vb, float lr,
                          float alpha, float eps, pifu_stream stream) {
  if (!ctx || !net || !dW || !db || !vW || !vb) return PIFU_ERR_INVALID_ARGUMENT;
  if (net->n_layers < 1 || net->n_layers > PIFU_MAX_LAYERS) return PIFU_ERR_INVALID_ARGUMENT;
  MLPDesc d;
  describe_mlp(net, d);
  hipStream_t s = as_stream(stream);
  for (int l = 0; l < d.n_layers; ++l) {
    if (!dW[l] || !db[l] || !vW[l] || !vb[l] || !d.W[l] || !d.b[l]) return PIFU_ERR_INVALID_ARGUMENT;
    // the network's parameters are updated in place
    launch_rmsprop(const_cast<float*>(d.W[l]), dW[l], vW[l], (size_t)d.widths[l] * d.in_w[l], lr,
                   alpha, eps, s);
    launch_rmsprop(const_cast<float*>(d.b[l]), db[l], vb[l], (size_t)d.widths[l], lr, alpha, eps, s);
  }
  return check_launch();
}

}  // extern "C"

// ================================================================== multi-frame batching
namespace {

constexpr int kMaxFrames = kMaxBatch;
constexpr uint32_t kBatchListCap = 1u << 28;
enum { C_SEG = 16, C_CONF_F = 40, C_B0_F = 56 };   // counter words (per frame blocks of 16)

struct BatchPlan {
  int n = 0;
  int order[kMaxFrames];       // frames sorted by number of refinements, descending
  int pos[kMaxFrames];         // position of frame f in the combined arrays
  int T[kMaxFrames];
  int Tmax = 0, l0 = 0;
  Lat lat[11];
  int active[11];
  uint8_t* st[11];
  float* occ[11];
  uint32_t* counters = nullptr;
  LocalizeWs w;
  uint32_t list_cap = 0;
  size_t list_words = 0;   // words of w.list: >= list_cap and >= every level's candidate masks
  FieldPrep fps[kMaxFrames];
  EvalWs ew;
  uint32_t* aw = nullptr;             // device-driven calls: count words
  Ellipsoids* ell_tab = nullptr;      // device-driven calls: each frame position's shapes
  size_t bytes = 0;
};

int validate_batch(int n, const pifu_field* const* fields, const pifu_grid_opts* const* opts) {
  if (n < 1 || n > kMaxFrames || !fields || !opts) return PIFU_ERR_INVALID_ARGUMENT;
  for (int f = 0; f < n; ++f) {
    int r = validate_grid_opts(fields[f], opts[f]);
    if (r) return r;
    const pifu_grid_opts& a = *opts[0];
    const pifu_grid_opts& b = *opts[f];
    if (b.dense || b.log2_coarse != a.log2_coarse || b.precision != a.precision ||
        b.band_delta != a.band_delta || b.guard_logit != a.guard_logit ||
        b.surrogate_max_log2 != a.surrogate_max_log2 || b.surrogate_delta != a.surrogate_delta ||
        b.max_waves != a.max_waves || b.tile_m != a.tile_m)
      return PIFU_ERR_INVALID_ARGUMENT;
    const pifu_field* A = fields[0];
    const pifu_field* B = fields[f];
    if (A->kind != B->kind) return PIFU_ERR_INVALID_ARGUMENT;
    if (A->kind == PIFU_FIELD_CBN) return PIFU_ERR_UNSUPPORTED;
    if (A->kind == PIFU_FIELD_MLP) {
      // frames share one network; only the feature maps differ
      if (B->H != A->H || B->W != A->W || B->C != A->C) return PIFU_ERR_INVALID_ARGUMENT;
      if (std::memcmp(A->mlp, B->mlp, sizeof(pifu_mlp)) != 0) return PIFU_ERR_INVALID_ARGUMENT;
      if ((A->surrogate == nullptr) != (B->surrogate == nullptr)) return PIFU_ERR_INVALID_ARGUMENT;
      if (A->surrogate && std::memcmp(A->surrogate, B->surrogate, sizeof(pifu_mlp)) != 0)
        return PIFU_ERR_INVALID_ARGUMENT;
    }
  }
  return PIFU_OK;
}

// async_cap > 0: the layout of the device-driven call, whose evaluations hold up to
// async_cap points of the combined list in one pass.
void plan_batch(int n, const pifu_field* const* fields, const pifu_grid_opts* const* opts, void* base,
                BatchPlan& b, uint32_t async_cap = 0) {
  b.n = n;
  b.l0 = opts[0]->log2_coarse;
  b.Tmax = 0;
  for (int f = 0; f < n; ++f) {
    b.T[f] = opts[f]->log2_final - b.l0;
    b.order[f] = f;
    b.Tmax = std::max(b.Tmax, b.T[f]);
  }
  std::stable_sort(b.order, b.order + n, [&](int x, int y) { return b.T[x] > b.T[y]; });
  for (int p = 0; p < n; ++p) b.pos[b.order[p]] = p;
  Carver cv(base);
  b.counters = cv.take<uint32_t>(kCounters + 2 * kMaxFrames + 64);
  size_t max_n = 0;
  for (int r = 0; r <= b.Tmax; ++r) {
    const int lg = b.l0 + r;
    b.lat[r] = Lat{(1 << lg) + 1, (1 << lg) + 1, (1 << lg) + 1};
    int a = 0;
    for (int f = 0; f < n; ++f) a += b.T[f] >= r;
    b.active[r] = a;
    const size_t tot = b.lat[r].n() * a;
    b.st[r] = cv.take<uint8_t>(tot + 16);
    b.occ[r] = cv.take<float>(tot);
    max_n = std::max(max_n, tot);
  }
  b.list_cap = (uint32_t)std::min<size_t>(max_n, async_cap ? async_cap : kBatchListCap);
  // the list buffer also holds a level's candidate bit masks before its compaction
  b.list_words = b.list_cap;
  for (int r = 1; r <= b.Tmax; ++r)
    b.list_words = std::max(b.list_words, 2 * b0_mask_words(b.lat[r]) * (size_t)b.active[r]);
  b.w.list = cv.take<uint32_t>(b.list_words);
  b.w.cscratch = cv.take<uint32_t>(compact_scratch_words(max_n));
  b.w.logit = cv.take<float>(b.list_cap);
  b.w.lab = cv.take<uint8_t>(b.list_cap);
  // one network for every frame: carve its operand copies once
  carve_field(cv, fields[0], opts[0]->precision, b.fps[0]);
  for (int f = 1; f < n; ++f) {
    b.fps[f] = b.fps[0];
    b.fps[f].f = fields[f];
    if (fields[f]->kind == PIFU_FIELD_ELLIPSOIDS) {
      std::memset(&b.fps[f].ell, 0, sizeof(b.fps[f].ell));
      b.fps[f].ell.n = fields[f]->n_ell;
      b.fps[f].ell.k = fields[f]->sharpness;
      if (fields[f]->ell) std::memcpy(b.fps[f].ell.e, fields[f]->ell, sizeof(float) * 12 * fields[f]->n_ell);
    }
  }
  const int C = fields[0]->kind == PIFU_FIELD_MLP ? fields[0]->C : 0;
  int mh = b.fps[0].has_mlp ? b.fps[0].mlp.max_hidden : 0;
  if (b.fps[0].has_sur) mh = std::max(mh, b.fps[0].sur.max_hidden);
  if (async_cap) {
    b.aw = cv.take<uint32_t>(AW_COUNT_WORDS);
    b.ell_tab = cv.take<Ellipsoids>(kMaxFrames);
    if (b.fps[0].has_mlp) {
      carve_eval(cv, b.list_cap, C, mh, b.ew, true);
      carve_guard(cv, b.fps[0], b.list_cap, b.ew);
      // an evaluation covers at most every x-y column of every active frame
      size_t cols = 0;
      for (int r = 0; r <= b.Tmax; ++r)
        cols = std::max(cols, (size_t)b.active[r] * b.lat[r].nx * b.lat[r].ny);
      carve_hoist(cv, hoist_np(b.fps[0]), b.ew, (uint32_t)std::min<size_t>(cols, UINT32_MAX));
    }
  } else {
    carve_eval(cv, b.list_cap, C, mh, b.ew);
    carve_guard(cv, b.fps[0], b.list_cap, b.ew);
    carve_hoist(cv, hoist_np(b.fps[0]), b.ew);
  }
  b.bytes = cv.off + kAlign;
}

// Stable compaction over the combined array, then the per-frame bounds of the list;
// one read-back carries the total and the bounds.
// Compacts the pending nodes of frames [p_lo, p_hi) of the combined level-r state (the
// other frames have none); the list holds combined indices p * n_nodes + node.
int compact_frames(EvalCtx& e, BatchPlan& b, int r, uint32_t* n_out, uint32_t* bounds, int p_lo,
                   int p_hi) {
  const Lat L = b.lat[r];
  const int A = b.active[r];
  const size_t start = (L.n() * (size_t)p_lo) & ~(size_t)15;   // keeps 16-byte state loads aligned
  const size_t end = L.n() * (size_t)p_hi;
  launch_compact(b.st[r] + start, end - start, ST_PEND, ST_PEND, b.w.cscratch,
                 e.counters + C_TOTAL, b.w.list, b.list_cap, 0, L, e.s, (uint32_t)start);
  int rc = check_launch();
  if (rc) return rc;
  rc = read_counters(e, 1);
  if (rc) return rc;
  const uint32_t n = e.ctx->host_counters[C_TOTAL];
  if (n > b.list_cap) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  launch_segment_bounds(b.w.list, n, (uint32_t)L.n(), A, e.counters + C_SEG, e.s);
  rc = read_counters(e, C_SEG + A + 1);
  if (rc) return rc;
  for (int p = 0; p <= A; ++p) bounds[p] = e.ctx->host_counters[C_SEG + p];
  *n_out = n;
  return PIFU_OK;
}

// Evaluates the combined list: the network's GEMMs span every frame, the gathers and
// the band / guard / surrogate-fallback re-runs stay per frame.
int eval_frames(EvalCtx& e, BatchPlan& b, int r, const uint32_t* bounds, uint32_t n,
                pifu_level_stats* st, bool use_sur) {
  const int A = b.active[r];
  const Lat L = b.lat[r];
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  src.nx = L.nx;
  src.ny = L.ny;
  src.nz = L.nz;
  Seg segs[kMaxFrames];
  int ns = 0;
  for (int p = 0; p < A; ++p) {
    const int f = b.order[p];
    segs[ns++] = Seg{bounds[p], bounds[p + 1] - bounds[p], b.fps[f].f->feat,
                     (uint32_t)(L.n() * p)};
  }
  const FieldPrep& fp0 = b.fps[0];
  if (!fp0.has_mlp) {
    for (int q = 0; q < ns; ++q) {
      const int f = b.order[q];
      if (!segs[q].count) continue;
      PointSrc sq = src;
      sq.base_sub = segs[q].base_sub;
      launch_eval_analytic(sq, b.w.list + segs[q].begin, segs[q].count, b.fps[f].f->kind,
                           b.fps[f].ell, b.fps[f].f->plane, b.w.logit + segs[q].begin,
                           b.w.lab + segs[q].begin, e.s);
    }
    return check_launch();
  }
  const bool sur = use_sur && fp0.has_sur;
  // one pass over every frame's points: the gathers pick each frame's feature map
  PointSrc sall = src;
  sall.frame_nodes = (uint32_t)L.n();
  for (int p = 0; p < A; ++p) sall.feat_tab[p] = b.fps[b.order[p]].f->feat;
  int rc = run_mlp(e, fp0, sur ? fp0.sur : fp0.mlp, sur ? PIFU_PREC_BF16 : e.precision, sall,
                   b.w.list, n, b.ew, b.w.logit, b.w.lab, nullptr);
  if (rc) return rc;
  for (int q = 0; q < ns; ++q) {
    const int f = b.order[q];
    if (!segs[q].count) continue;
    PointSrc sq = src;
    sq.frame_nodes = 0;
    sq.base_sub = segs[q].base_sub;
    const uint32_t* lst = b.w.list + segs[q].begin;
    float* lg = b.w.logit + segs[q].begin;
    uint8_t* lb = b.w.lab + segs[q].begin;
    pifu_level_stats* sf = st ? &st[f] : nullptr;
    if (!sur) {
      if (sf) sf->mlp_points += segs[q].count;
      rc = post_full(e, b.fps[f], sq, segs[q].F, lst, segs[q].count, b.ew, lg, lb, sf);
      if (rc) return rc;
      continue;
    }
    uint32_t nsur = 0;
    rc = select_near(e, lg, segs[q].count, e.sur_band, b.ew.sur_pos, &nsur);
    if (rc) return rc;
    if (nsur) {
      launch_gather_u32(lst, b.ew.sur_pos, nsur, b.ew.sur_nodes, e.s);
      rc = eval_full(e, b.fps[f], sq, b.ew.sur_nodes, nsur, b.ew, b.ew.sur_logit, b.ew.sur_lab, sf,
                     segs[q].F);
      if (rc) return rc;
      launch_scatter_results(b.ew.sur_pos, nsur, b.ew.sur_logit, b.ew.sur_lab, lg, lb, e.s);
    }
    if (sf) sf->surrogate_fallback += nsur;
  }
  return check_launch();
}

}  // namespace

extern "C" {

int32_t pifu_occupancy_grid_batched_workspace_size(int32_t n, const pifu_field* const* fields,
                                                   const pifu_grid_opts* const* opts,
                                                   size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_batch(n, fields, opts);
  if (r) return r;
  BatchPlan* b = new (std::nothrow) BatchPlan;
  if (!b) return PIFU_ERR_HIP;
  plan_batch(n, fields, opts, nullptr, *b);
  *bytes = b->bytes;
  delete b;
  return PIFU_OK;
}

int32_t pifu_occupancy_grid_batched(pifu_ctx* ctx, int32_t n, const pifu_field* const* fields,
                                    const pifu_grid_opts* const* opts, pifu_grid_out* outs,
                                    void* workspace, size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !outs || !workspace || !aligned(workspace, kAlign)) return PIFU_ERR_INVALID_ARGUMENT;
  int rc = validate_batch(n, fields, opts);
  if (rc) return rc;
  for (int f = 0; f < n; ++f)
    if (!outs[f].occ || !outs[f].labels || (outs[f].cells_cap && !outs[f].cells))
      return PIFU_ERR_INVALID_ARGUMENT;
  BatchPlan* bp = new (std::nothrow) BatchPlan;
  if (!bp) return PIFU_ERR_HIP;
  BatchPlan& b = *bp;
  plan_batch(n, fields, opts, nullptr, b);
  if (workspace_bytes < b.bytes) {
    delete bp;
    return PIFU_ERR_WORKSPACE_TOO_SMALL;
  }
  plan_batch(n, fields, opts, workspace, b);
  hipStream_t s = as_stream(stream);
  const pifu_grid_opts& o = *opts[0];
  EvalCtx e{ctx, s, b.counters, o.precision, o.guard_logit};
  e.band = logit_band(o.band_delta);
  e.sur_band = logit_band(o.surrogate_delta);
  e.tile_m = o.tile_m;
  if (int pr = pack_field(b.fps[0], ctx, s, b.counters)) {
    delete bp;
    return pr;
  }
  for (int f = 1; f < n; ++f) {   // frames share the packed network and its scales
    b.fps[f].mlp = b.fps[0].mlp;
    b.fps[f].sur = b.fps[0].sur;
  }
  pifu_level_stats st[kMaxFrames];
  uint32_t bounds[kMaxFrames + 1];
  for (int r = 0; r <= b.Tmax && !rc; ++r) {
    const Lat L = b.lat[r];
    const int A = b.active[r];
    const uint32_t nl = (uint32_t)L.n();
    const int level_id = b.l0 + r;
    std::memset(st, 0, sizeof(st));
    for (int f = 0; f < n; ++f) {
      st[f].level = level_id;
      st[f].nodes = nl;
    }
    // every word but C_OVF
    if (hipMemsetAsync(b.counters, 0, sizeof(uint32_t) * C_OVF, s) != hipSuccess ||
        hipMemsetAsync(b.counters + C_OVF + 1, 0,
                       sizeof(uint32_t) * (kCounters + 2 * kMaxFrames + 64 - C_OVF - 1),
                       s) != hipSuccess) {
      rc = PIFU_ERR_HIP;
      break;
    }
    e.sel_base = 0;
    const bool use_sur = level_id <= o.surrogate_max_log2;
    // frames whose final level this is write their occupancy straight into their output
    FrameOcc fo{};
    for (int p = 0; p < A; ++p)
      if (b.T[b.order[p]] == r) fo.p[p] = outs[b.order[p]].occ;
    uint32_t cnt = 0;
    if (r == 0) {
      const uint32_t tot = nl * (uint32_t)A;
      launch_fill_u8(b.st[0], 0, tot, s);
      launch_iota(b.w.list, tot, s);
      for (int p = 0; p <= A; ++p) bounds[p] = nl * (uint32_t)p;
      rc = eval_frames(e, b, 0, bounds, tot, st, use_sur);
      if (rc) break;
      launch_apply_grid(b.w.list, tot, b.w.logit, b.w.lab, b.st[0], b.occ[0], nullptr, nullptr,
                        level_id, L, 1, L, 0, s, nl, &fo);
      for (int p = 0; p < A; ++p) {
        st[b.order[p]].dilated = nl;
        st[b.order[p]].evaluated = nl;
      }
    } else {
      launch_transition(b.st[r - 1], b.occ[r - 1], b.lat[r - 1], b.st[r], b.occ[r], L, s, A, &fo);
      if (2 * b0_mask_words(L) * (size_t)A <= b.list_words) {
        // the candidate list is consumed until compact_frames rewrites it
        launch_select_b0(b.st[r], L, A, reinterpret_cast<uint64_t*>(b.w.list), b.counters + C_B0_F,
                         1, s);
      } else {
        for (int p = 0; p < A; ++p)
          launch_count_bits(b.st[r] + (size_t)p * nl, nl, ST_B0, b.counters + C_B0_F + p, s);
        launch_select(b.st[r], L, s, A);
      }
      rc = compact_frames(e, b, r, &cnt, bounds, 0, A);
      if (rc) break;
      for (int p = 0; p < A; ++p) st[b.order[p]].dilated = bounds[p + 1] - bounds[p];
      int waves = 0;
      while (cnt) {
        rc = eval_frames(e, b, r, bounds, cnt, st, use_sur);
        if (rc) break;
        launch_apply_grid(b.w.list, cnt, b.w.logit, b.w.lab, b.st[r], b.occ[r],
                          b.counters + C_CONF_F, nullptr, level_id, L, 1, L, 1, s, nl, &fo);
        for (int p = 0; p < A; ++p) {
          const uint32_t c = bounds[p + 1] - bounds[p];
          st[b.order[p]].evaluated += c;
          if (waves > 0 && c) st[b.order[p]].waves += 1;
        }
        if (o.max_waves > 0 && waves >= o.max_waves) break;
        launch_expand(b.w.list, cnt, b.st[r], L, s, nl);
        // only frames with nodes in this wave can gain pending nodes (expansion stays
        // inside a frame): compact the range of those frames
        int p_lo = A, p_hi = 0;
        for (int p = 0; p < A; ++p)
          if (bounds[p + 1] > bounds[p]) {
            p_lo = std::min(p_lo, p);
            p_hi = p + 1;
          }
        rc = compact_frames(e, b, r, &cnt, bounds, p_lo, p_hi);
        if (rc) break;
        if (cnt) ++waves;
      }
      if (rc) break;
    }
    rc = check_launch();
    if (!rc) rc = read_counters(e, C_B0_F + kMaxFrames);
    if (rc) break;
    for (int p = 0; p < A; ++p) {
      const int f = b.order[p];
      st[f].conflicts = ctx->host_counters[C_CONF_F + p];
      st[f].b0 = r ? ctx->host_counters[C_B0_F + p] : 0;
      if (outs[f].stats) outs[f].stats[r] = st[f];
    }
    // frames whose final level this is: labels, cells and occupancy out
    for (int p = 0; p < A && !rc; ++p) {
      const int f = b.order[p];
      if (b.T[f] != r) continue;
      uint8_t* sf = b.st[r] + (size_t)p * nl;
      launch_cells(sf, L, outs[f].labels, s);
      uint32_t nc = 0;
      rc = compact_count(e, sf, nl, ST_CELL, ST_CELL, b.w.cscratch, outs[f].cells, outs[f].cells_cap,
                         1, L, &nc);
      outs[f].n_cells = nc;
    }
  }
  if (!rc) rc = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  prof_resolve(ctx);
  delete bp;
  return rc;
}

}  // extern "C"

// ================================================================== device-driven calls
// Asynchronous forms of pifu_occupancy_grid and pifu_render_view: every count stays in
// device memory, every launch is sized from host-known capacities, and the level loop
// runs a fixed ladder of conflict waves whose kernels find an empty list once the
// waves have converged.  Nothing is read back and nothing is allocated, so a call can
// be captured into a HIP graph and replayed.  The kernels and their arithmetic are the
// blocking calls' own (persistent GEMM launches walk k in the same order), so results
// are identical.
namespace {

// count words of a device-driven call (AW_*), after the level counters
enum {
  AW_NCOL = 0,   // columns of the hoisted evaluation
  AW_NB,         // points of the precision band
  AW_NS,         // surrogate points sent to the full network
  AW_GN,         // points of the FP64 guard
  AW_RR,         // points re-run in FP32 after a binary16 range overflow (0, or all / the band)
  AW_N0,         // a host-known count, stored for kernels that read counts from memory
  AW_NH,         // render hits
  AW_STATUS,     // status bits (kStatus*)
  AW_NBSEL,      // multi-frame FP16 runs: band points counted (0 after an overflow)
  AW_COUNT = 16
};
// bits of the status word
constexpr uint32_t kStatusListOver = 1;    // a list exceeded max_points (results invalid)
constexpr uint32_t kStatusWavesLeft = 2;   // conflicts remained after the wave budget
constexpr uint32_t kStatusGuardOver = 4;   // more guard points than the FP64 chunk holds
constexpr uint32_t kStatusCellsOver = 8;   // more surface cells than cells_cap
constexpr int kDefaultWaveBudget = 12;

struct Book {
  BookOps ops;
  hipStream_t s;
  explicit Book(hipStream_t st) : s(st) {}
  void add(int kind, uint32_t* dst, const uint32_t* src = nullptr, uint32_t imm = 0,
           uint32_t bit = 0, const uint32_t* aux = nullptr, const uint32_t* src2 = nullptr) {
    if (ops.n == kMaxBookOps) flush();
    ops.op[ops.n++] = BookOp{dst, src, src2, aux, imm, bit, kind};
  }
  void flush() {
    launch_book(ops, s);
    ops.n = 0;
  }
  ~Book() { flush(); }
};

uint32_t* stat_word(pifu_level_stats* st, uint32_t pifu_level_stats::*f) {
  return reinterpret_cast<uint32_t*>(&(st->*f));
}

// Per-frame statistics of a multi-frame device-driven evaluation: list entries are
// combined indices frame * frame_nodes + node; st[p] is frame position p's record of the
// level being evaluated.
struct FrameCount {
  int frames = 0;
  uint32_t frame_nodes = 0;
  uint32_t* tally = nullptr;   // kMaxBatch device words, zero between uses
  pifu_level_stats* st[kMaxBatch] = {};
};

// field of every frame's record op= (entries of the list, or of its positions pos, per
// frame), for the first min(cap, *n_dev) entries.
void count_frames(EvalCtx& e, const uint32_t* list, const uint32_t* pos, uint32_t cap,
                  const uint32_t* n_dev, uint32_t pifu_level_stats::*field, int op = BK_ADD,
                  uint32_t pifu_level_stats::*field2 = nullptr, int op2 = BK_ADD) {
  const FrameCount& fc = *e.fc;
  launch_frame_tally(list, pos, cap, n_dev, fc.frame_nodes, fc.tally, e.s);
  FrameApply a{};
  a.frames = fc.frames;
  a.nops = field2 ? 2 : 1;
  a.kind[0] = op;
  a.kind[1] = op2;
  for (int p = 0; p < fc.frames; ++p) {
    a.dst[0][p] = stat_word(fc.st[p], field);
    if (field2) a.dst[1][p] = stat_word(fc.st[p], field2);
  }
  launch_frame_apply(fc.tally, a, e.s);
}

// run_mlp over a list whose length lives on the device (at most cap <= ew.chunk
// points): one pass, persistent GEMMs, list kernels striding over the count.
int run_mlp_dev(EvalCtx& e, const FieldPrep& fp, const MlpPrep& mp, int prec, const PointSrc& src,
                const uint32_t* list, uint32_t cap, const uint32_t* n_dev, const EvalWs& ew,
                float* logit, uint8_t* lab, float* rgb, const float* F = nullptr) {
  const pifu_field* f = fp.f;
  const MLPDesc& d = mp.d;
  const int C = f->C;
  if (!cap) return PIFU_OK;
  if (cap > ew.chunk) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  const bool x3 = prec == PREC_F32X3;
  const bool b16 = prec != PIFU_PREC_FP32 && !x3;
  const int hf = x3 ? FMT_F32 : h16_fmt(prec);
  if ((prec == PIFU_PREC_BF16 || prec == PIFU_PREC_FP16) && mp.prec != prec)
    return PIFU_ERR_UNSUPPORTED;
  if (x3 && !mp.Wlo16[0]) return PIFU_ERR_UNSUPPORTED;
  if (prec == PIFU_PREC_FP8) return PIFU_ERR_UNSUPPORTED;
  if (!F) F = f->feat;
  uint32_t* ovf = prec == PIFU_PREC_FP16 || x3 ? e.counters + C_OVF : nullptr;
  const bool hoist = src.mode == 0 && !src.has_view && mp.NP > 0 && mp.NP % 4 == 0 &&
                     d.widths[0] % 4 == 0 && ew.Pcol != nullptr;
  // per-texel hoisting, as in run_mlp
  const bool texel = !hoist && ew.Ttex && &mp == ew.ttex_mlp && prec == PIFU_PREC_FP32 &&
                     !src.frame_nodes && F == f->feat;
  const void* prev = nullptr;
  void* out = ew.hA;
  int l0 = 0;
  GemmArgs g;
  if (hoist) {
    uint32_t* ncol = e.aw + AW_NCOL;
    const uint32_t ccap = std::min(cap, ew.col_rows);
    launch_col_flags(list, cap, (uint32_t)src.nz, ew.cflags, e.s, n_dev);
    launch_scan_u32(ew.cflags, cap, ew.cexcl, ew.cscan, ncol, e.s, n_dev);
    launch_col_ids(list, ew.cflags, ew.cexcl, cap, ew.cid, ew.cnode, e.s, n_dev);
    launch_gather(src, ew.cnode, ccap, F, f->H, f->W, C, ew.feat, hf, ew.ext, e.s, ncol, ovf);
    std::memset(&g, 0, sizeof(g));
    g.A1 = ew.feat;
    g.K1 = g.lda1 = C;
    g.W = x3 ? (mp.prec == PIFU_PREC_FP16 ? (const void*)mp.Wf16 : (const void*)mp.Wfh16)
          : b16 ? (const void*)mp.Wf16 : (const void*)mp.Wf32;
    g.Wlo = x3 ? (const void*)mp.Wflo16 : nullptr;
    g.ovf = ovf;
    g.ldw = C;
    g.bias = mp.bf;
    g.C = ew.Pcol;
    g.ldc = g.N = mp.NP;
    g.M = (int)ccap;
    g.M_dev = ncol;
    g.scale = 1.f;
    if (launch_gemm_persist(g, prec, e.s)) return PIFU_ERR_UNSUPPORTED;
    launch_hoist_layer0(ew.Pcol, mp.NP, ew.cid, list, cap, src.nz, mp.wz, d.widths[0],
                        d.hidden_act, ew.hA, d.n_layers > 2 ? hf : FMT_F32, e.s, ovf, n_dev);
    prev = ew.hA;
    out = ew.hB;
    l0 = 1;
  } else if (texel) {
    launch_taps(src, list, cap, f->H, f->W, ew.tidx, ew.tw, ew.ext, e.s, n_dev);
    launch_taps_layer0(ew.Ttex, mp.NP, ew.tidx, ew.tw, ew.ext, cap, mp.bf, mp.wz, d.widths[0],
                       d.hidden_act, reinterpret_cast<float*>(ew.hA), e.s, n_dev);
    prev = ew.hA;
    out = ew.hB;
    l0 = 1;
  } else {
    launch_gather(src, list, cap, F, f->H, f->W, C, ew.feat, hf, ew.ext, e.s, n_dev, ovf);
  }
  for (int l = l0; l + 1 < d.n_layers; ++l) {
    std::memset(&g, 0, sizeof(g));
    if (l == 0) {
      g.A1 = ew.feat;
      g.K1 = g.lda1 = C;
      g.n_ext = d.n_extra;
      g.ext_col = C;
      g.bias = d.b[l];
    } else {
      g.A1 = prev;
      g.K1 = g.lda1 = d.widths[l - 1];
      if (hoist && mp.hoist_off[l] >= 0) {
        g.rowadd = ew.Pcol;
        g.rowadd_idx = ew.cid;
        g.rowadd_ld = mp.NP;
        g.rowadd_off = mp.hoist_off[l];
      } else if (texel && mp.hoist_off[l] >= 0) {
        g.bias = d.b[l];
        g.rowadd = ew.Ttex;
        g.rowadd_ld = mp.NP;
        g.rowadd_off = mp.hoist_off[l];
        g.tap_idx = ew.tidx;
        g.tap_w = ew.tw;
      } else {
        g.bias = d.b[l];
        if (d.skip[l]) {
          g.A2 = ew.feat;
          g.K2 = g.lda2 = C;
        }
      }
    }
    g.W = layer_weights(mp, prec, l);
    g.Wlo = x3 ? (const void*)mp.Wlo16[l] : nullptr;
    g.ldw = mp.Kp[l];
    g.Wf = d.W[l];
    g.ldwf = d.in_w[l];
    g.ext = ew.ext;
    g.C = out;
    g.ldc = g.N = d.widths[l];
    g.M = (int)cap;
    g.M_dev = n_dev;
    g.act = d.hidden_act;
    g.scale = 1.f;
    g.c_bf16 = b16 && (l + 2 < d.n_layers);
    g.ovf = ovf;
    if (launch_gemm_persist(g, prec, e.s)) return PIFU_ERR_UNSUPPORTED;
    prev = out;
    out = (out == ew.hA) ? ew.hB : ew.hA;
  }
  const int L = d.n_layers - 1;
  launch_head(reinterpret_cast<const float*>(prev), d.widths[L - 1], d.W[L], d.b[L], d.widths[L],
              d.out_act, cap, hoist ? nullptr : ew.ext, logit, lab, rgb, rgb ? list : nullptr, e.s,
              n_dev);
  return check_launch();
}

// Positions m < *n_dev with |logit[m]| < bound into pos; their count into *cnt.
void select_dev(EvalCtx& e, const float* logit, uint32_t cap, const uint32_t* n_dev, float bound,
                uint32_t* pos, uint32_t* cnt) {
  launch_set_u32(cnt, 0, e.s);
  launch_guard_select(logit, cap, bound, pos, cnt, e.s, nullptr, 0, n_dev);
}

// post_full for a device-side count: the precision band (with the FP32 re-run of an FP16
// call whose values left the binary16 range, or of a BF16 call's band), then the FP64 guard.
int post_full_dev(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const float* F,
                  const uint32_t* list, uint32_t cap, const uint32_t* n_dev, const EvalWs& ew,
                  float* logit, uint8_t* lab) {
  const pifu_field* f = fp.f;
  int r = PIFU_OK;
  const bool f16 = e.precision == PIFU_PREC_FP16;
  const bool band = e.precision != PIFU_PREC_FP32 && e.band > 0.f;
  const bool bx3 = band && e.precision == PIFU_PREC_BF16 && split_band(fp);
  uint32_t* nb = e.aw + AW_NB;
  if (band) {
    select_dev(e, logit, cap, n_dev, e.band, ew.band_pos, nb);
    launch_gather_u32(list, ew.band_pos, cap, ew.band_nodes, e.s, nb);
    r = run_mlp_dev(e, fp, fp.mlp, f16 || bx3 ? PREC_F32X3 : PIFU_PREC_FP32, src, ew.band_nodes,
                    cap, nb, ew, ew.band_logit, ew.band_lab, nullptr, F);
    if (r) return r;
    launch_scatter_results(ew.band_pos, cap, ew.band_logit, ew.band_lab, logit, lab, e.s, nb);
  }
  if (bx3) {
    // a BF16 call with a value outside the binary16 range so far: the band's points in FP32
    uint32_t* rr = e.aw + AW_RR;
    {
      Book b(e.s);
      b.add(BK_SEL, rr, nb, 0, 0, e.counters + C_OVF);
    }
    r = run_mlp_dev(e, fp, fp.mlp, PIFU_PREC_FP32, src, ew.band_nodes, cap, rr, ew, ew.band_logit,
                    ew.band_lab, nullptr, F);
    if (r) return r;
    launch_scatter_results(ew.band_pos, cap, ew.band_logit, ew.band_lab, logit, lab, e.s, rr);
  }
  Book b(e.s);
  uint32_t* band_stat = e.fc ? nullptr : stat_word(e.st_dev, &pifu_level_stats::band_fp32);
  if (f16) {
    // a value outside the binary16 range so far in this call: all points in FP32
    uint32_t* rr = e.aw + AW_RR;
    b.add(BK_SEL, rr, n_dev, 0, 0, e.counters + C_OVF);
    if (e.fc) {
      // per frame: every point after an overflow, else the band's points
      uint32_t* nb_sel = e.aw + AW_NBSEL;
      b.add(BK_SET_IMM, nb_sel, nullptr, 0);
      b.add(BK_ADD_SEL, nb_sel, nullptr, 0, 0, e.counters + C_OVF, band ? nb : nullptr);
      b.flush();
      count_frames(e, list, nullptr, cap, rr, &pifu_level_stats::band_fp32);
      if (band) count_frames(e, list, ew.band_pos, cap, nb_sel, &pifu_level_stats::band_fp32);
    } else {
      b.add(BK_ADD_SEL, band_stat, n_dev, 0, 0, e.counters + C_OVF, band ? nb : nullptr);
      b.flush();
    }
    r = run_mlp_dev(e, fp, fp.mlp, PIFU_PREC_FP32, src, list, cap, rr, ew, logit, lab, nullptr, F);
    if (r) return r;
  } else if (band) {
    if (e.fc) count_frames(e, list, ew.band_pos, cap, nb, &pifu_level_stats::band_fp32);
    else b.add(BK_ADD, band_stat, nb);
  }
  if (!(e.guard > 0.f)) return PIFU_OK;
  uint32_t* gn = e.aw + AW_GN;
  select_dev(e, logit, cap, n_dev, e.guard, ew.glist, gn);
  run_guard64(src, list, ew.glist, std::min(cap, ew.chunk64), fp.mlp.d, F, f->H, f->W, f->C, logit,
              lab, ew.g64, ew.chunk64, !e.g64_packed, e.s, gn);
  e.g64_packed = true;
  if (e.fc) count_frames(e, list, ew.glist, std::min(cap, ew.chunk64), gn,
                         &pifu_level_stats::guard_fp64);
  else b.add(BK_ADD, stat_word(e.st_dev, &pifu_level_stats::guard_fp64), gn);
  b.add(BK_FLAG_GT, e.aw + AW_STATUS, gn, ew.chunk64, kStatusGuardOver);
  return check_launch();
}

int eval_full_dev(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const uint32_t* list,
                  uint32_t cap, const uint32_t* n_dev, const EvalWs& ew, float* logit,
                  uint8_t* lab) {
  int r = run_mlp_dev(e, fp, fp.mlp, e.precision, src, list, cap, n_dev, ew, logit, lab, nullptr);
  if (r) return r;
  if (e.fc) {
    count_frames(e, list, nullptr, cap, n_dev, &pifu_level_stats::mlp_points);
  } else {
    Book b(e.s);
    b.add(BK_ADD, stat_word(e.st_dev, &pifu_level_stats::mlp_points), n_dev);
  }
  return post_full_dev(e, fp, src, fp.f->feat, list, cap, n_dev, ew, logit, lab);
}

// eval_occupancy for a device-side count.
int eval_occupancy_dev(EvalCtx& e, const FieldPrep& fp, const PointSrc& src, const uint32_t* list,
                       uint32_t cap, const uint32_t* n_dev, const EvalWs& ew, float* logit,
                       uint8_t* lab, bool use_surrogate) {
  if (!cap) return PIFU_OK;
  if (!fp.has_mlp) {
    launch_eval_analytic(src, list, cap, fp.f->kind, fp.ell, fp.f->plane, logit, lab, e.s, n_dev);
    return check_launch();
  }
  if (!(use_surrogate && fp.has_sur)) return eval_full_dev(e, fp, src, list, cap, n_dev, ew, logit, lab);
  int r = run_mlp_dev(e, fp, fp.sur, PIFU_PREC_BF16, src, list, cap, n_dev, ew, logit, lab, nullptr);
  if (r) return r;
  uint32_t* ns = e.aw + AW_NS;
  select_dev(e, logit, cap, n_dev, e.sur_band, ew.sur_pos, ns);
  launch_gather_u32(list, ew.sur_pos, cap, ew.sur_nodes, e.s, ns);
  r = eval_full_dev(e, fp, src, ew.sur_nodes, cap, ns, ew, ew.sur_logit, ew.sur_lab);
  if (r) return r;
  launch_scatter_results(ew.sur_pos, cap, ew.sur_logit, ew.sur_lab, logit, lab, e.s, ns);
  Book b(e.s);
  b.add(BK_ADD, stat_word(e.st_dev, &pifu_level_stats::surrogate_fallback), ns);
  return check_launch();
}

// localize with device-side counts and a fixed ladder of waves per level: rung 0
// evaluates the candidates, rungs 1 .. budget the conflict waves.  max_waves > 0 is the
// caller's own cap (as in the blocking call); with max_waves == 0 the ladder has
// kDefaultWaveBudget waves and a level with conflicts left after it sets
// kStatusWavesLeft.  stats_dev: one device record per level.
int localize_dev(EvalCtx& e, const FieldPrep& fp, const EvalWs& ew, const double* view,
                 int T, int last, LevelBuf* lv, const LocalizeWs& w, uint8_t* eval_level,
                 Lat eval_lat, int max_waves, int sur_max_log2, pifu_level_stats* stats_dev,
                 uint32_t cap, float* eval_logit = nullptr) {
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  if (view) {
    src.has_view = 1;
    for (int i = 0; i < 12; ++i) src.view[i] = view[i];
  }
  const bool bounded = max_waves > 0;
  const int budget = bounded ? max_waves : kDefaultWaveBudget;
  uint32_t* n_dev = e.counters + C_TOTAL;
  for (int t = 0; t <= last; ++t) {
    LevelBuf& L = lv[t];
    pifu_level_stats* sd = stats_dev + t;
    e.st_dev = sd;
    src.nx = L.lat.nx;
    src.ny = L.lat.ny;
    src.nz = L.lat.nz;
    const int stride = (eval_lat.nx - 1) / (L.lat.nx - 1);
    const uint32_t n_nodes = (uint32_t)L.lat.n();
    const bool sur = L.level_id <= sur_max_log2;
    launch_set_u32(e.counters, 0, e.s, C_OVF);   // keeps C_OVF
    {
      Book b(e.s);
      b.add(BK_SET_IMM, reinterpret_cast<uint32_t*>(&sd->level), nullptr, (uint32_t)L.level_id);
      b.add(BK_SET_IMM, stat_word(sd, &pifu_level_stats::nodes), nullptr, n_nodes);
    }
    if (t == 0) {
      if (n_nodes > cap) return PIFU_ERR_WORKSPACE_TOO_SMALL;
      launch_fill_u8(L.st, 0, n_nodes, e.s);
      launch_iota(w.list, n_nodes, e.s);
      {
        Book b(e.s);
        b.add(BK_SET_IMM, e.aw + AW_N0, nullptr, n_nodes);
      }
      int r = eval_occupancy_dev(e, fp, src, w.list, n_nodes, e.aw + AW_N0, ew, w.logit, w.lab, sur);
      if (r) return r;
      launch_apply_grid(w.list, n_nodes, w.logit, w.lab, L.st, L.occ, nullptr, eval_level,
                        L.level_id, L.lat, stride, eval_lat, 0, e.s, 0, nullptr, eval_logit);
      Book b(e.s);
      b.add(BK_SET_IMM, stat_word(sd, &pifu_level_stats::dilated), nullptr, n_nodes);
      b.add(BK_SET_IMM, stat_word(sd, &pifu_level_stats::evaluated), nullptr, n_nodes);
      continue;
    }
    LevelBuf& Cc = lv[t - 1];
    launch_transition(Cc.st, Cc.occ, Cc.lat, L.st, L.occ, L.lat, e.s);
    if (2 * b0_mask_words(L.lat) <= n_nodes) {
      launch_select_b0(L.st, L.lat, 1, reinterpret_cast<uint64_t*>(w.list), e.counters + C_B0, 0,
                       e.s);
    } else {
      launch_count_bits(L.st, n_nodes, ST_B0, e.counters + C_B0, e.s);
      launch_select(L.st, L.lat, e.s);
    }
    launch_compact(L.st, n_nodes, ST_PEND, ST_PEND, w.cscratch, n_dev, w.list, n_nodes, 0, L.lat,
                   e.s);
    const uint32_t ecap = std::min(n_nodes, cap);
    {
      Book b(e.s);
      b.add(BK_SET, stat_word(sd, &pifu_level_stats::dilated), n_dev);
      b.add(BK_FLAG_GT, e.aw + AW_STATUS, n_dev, cap, kStatusListOver);
    }
    for (int rung = 0; rung <= budget; ++rung) {
      int r = eval_occupancy_dev(e, fp, src, w.list, ecap, n_dev, ew, w.logit, w.lab, sur);
      if (r) return r;
      launch_apply_grid(w.list, ecap, w.logit, w.lab, L.st, L.occ, e.counters + C_CONFLICTS,
                        eval_level, L.level_id, L.lat, stride, eval_lat, 1, e.s, 0, nullptr,
                        eval_logit, n_dev);
      {
        Book b(e.s);
        b.add(BK_ADD, stat_word(sd, &pifu_level_stats::evaluated), n_dev);
      }
      if (rung == budget && bounded) break;
      launch_expand(w.list, ecap, L.st, L.lat, e.s, 0, n_dev);
      // an empty wave selects nothing: the compaction is gated on its count
      launch_compact(L.st, n_nodes, ST_PEND, ST_PEND, w.cscratch, n_dev, w.list, n_nodes, 0, L.lat,
                     e.s, 0, n_dev);
      Book b(e.s);
      if (rung < budget) {
        b.add(BK_ADD_NZ, stat_word(sd, &pifu_level_stats::waves), n_dev);
        b.add(BK_FLAG_GT, e.aw + AW_STATUS, n_dev, cap, kStatusListOver);
      } else {
        b.add(BK_FLAG_GT, e.aw + AW_STATUS, n_dev, 0, kStatusWavesLeft);
      }
    }
    Book b(e.s);
    b.add(BK_SET, stat_word(sd, &pifu_level_stats::conflicts), e.counters + C_CONFLICTS);
    b.add(BK_SET, stat_word(sd, &pifu_level_stats::b0), e.counters + C_B0);
  }
  return check_launch();
}

}  // namespace

namespace {

uint32_t default_async_cap(size_t max_n) {
  return (uint32_t)std::min<size_t>(max_n, (size_t)1 << 20);
}

}  // namespace

extern "C" {

int32_t pifu_occupancy_grid_async_workspace_size(const pifu_field* field,
                                                 const pifu_grid_opts* opts, uint32_t max_points,
                                                 size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_grid_opts(field, opts);
  if (r) return r;
  if (opts->precision == PIFU_PREC_FP8 || field->kind == PIFU_FIELD_CBN) return PIFU_ERR_UNSUPPORTED;
  GridWs* g = new (std::nothrow) GridWs;
  if (!g) return PIFU_ERR_HIP;
  plan_grid(field, opts, nullptr, nullptr, *g, 1);
  size_t max_n = 0;
  for (int t = 0; t <= g->T; ++t) max_n = std::max(max_n, g->lv[t].lat.n());
  const uint32_t cap = max_points ? max_points : default_async_cap(max_n);
  plan_grid(field, opts, nullptr, nullptr, *g, cap);
  *bytes = g->bytes;
  delete g;
  return PIFU_OK;
}

int32_t pifu_occupancy_grid_async(pifu_ctx* ctx, const pifu_field* field,
                                  const pifu_grid_opts* opts, uint32_t max_points, float* occ,
                                  uint8_t* labels, uint8_t* eval_level, uint32_t* cells,
                                  uint32_t cells_cap, uint32_t* n_cells_dev,
                                  pifu_level_stats* stats_dev, uint32_t* status_dev,
                                  void* workspace, size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !occ || !labels || !n_cells_dev || !stats_dev || !status_dev || !workspace)
    return PIFU_ERR_INVALID_ARGUMENT;
  if (cells_cap && !cells) return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(workspace, kAlign) || !aligned(stats_dev, 4) || !aligned(n_cells_dev, 4) ||
      !aligned(status_dev, 4))
    return PIFU_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  int r = pifu_occupancy_grid_async_workspace_size(field, opts, max_points, &need);
  if (r) return r;
  if (workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  GridWs* gp = new (std::nothrow) GridWs;
  if (!gp) return PIFU_ERR_HIP;
  GridWs& g = *gp;
  plan_grid(field, opts, nullptr, nullptr, g, 1);
  size_t max_n = 0;
  for (int t = 0; t <= g.T; ++t) max_n = std::max(max_n, g.lv[t].lat.n());
  const uint32_t cap = (uint32_t)std::min<size_t>(max_points ? max_points : default_async_cap(max_n),
                                                  max_n);
  plan_grid(field, opts, workspace, occ, g, cap);
  hipStream_t s = as_stream(stream);
  EvalCtx e{ctx, s, g.counters, opts->precision, opts->guard_logit};
  e.band = logit_band(opts->band_delta);
  e.sur_band = logit_band(opts->surrogate_delta);
  e.aw = g.aw;
  const int n_levels = g.T + 1;
  launch_set_u32(g.aw, 0, s, AW_COUNT_WORDS);
  launch_set_u32(reinterpret_cast<uint32_t*>(stats_dev), 0, s,
                 (uint32_t)(n_levels * sizeof(pifu_level_stats) / 4));
  r = pack_field(g.fp, ctx, s, g.counters);
  const Lat fin = g.lv[g.T].lat;
  if (!r && eval_level) launch_fill_u8(eval_level, 255, fin.n(), s);
  if (!r)
    r = localize_dev(e, g.fp, g.ew, nullptr, g.T, g.T, g.lv, g.w, eval_level, fin, opts->max_waves,
                     opts->surrogate_max_log2, stats_dev, cap);
  if (!r) {
    launch_cells(g.lv[g.T].st, fin, labels, s);
    launch_compact(g.lv[g.T].st, fin.n(), ST_CELL, ST_CELL, g.w.cscratch, g.counters + C_TOTAL,
                   cells, cells_cap, 1, fin, s);
    Book b(s);
    b.add(BK_SET, n_cells_dev, g.counters + C_TOTAL);
    b.add(BK_FLAG_GT, g.aw + AW_STATUS, g.counters + C_TOTAL, cells_cap, kStatusCellsOver);
    b.add(BK_SET, status_dev, g.aw + AW_STATUS);
  }
  if (!r) r = check_launch();
  delete gp;
  return r;
}

int32_t pifu_render_view_async_workspace_size(const pifu_field* occ_field,
                                              const pifu_field* color_field,
                                              const pifu_render_opts* opts, uint32_t max_points,
                                              size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_render_opts(occ_field, color_field, opts);
  if (r) return r;
  if (opts->precision == PIFU_PREC_FP8) return PIFU_ERR_UNSUPPORTED;
  RenderWs* g = new (std::nothrow) RenderWs;
  if (!g) return PIFU_ERR_HIP;
  const size_t W = (size_t)1 << opts->log2_w, D = (size_t)1 << opts->log2_d;
  const uint32_t cap = max_points ? max_points : default_async_cap(W * W * (D + 1));
  plan_render(occ_field, color_field, opts, nullptr, *g, cap);
  *bytes = g->bytes;
  delete g;
  return PIFU_OK;
}

int32_t pifu_render_view_async(pifu_ctx* ctx, const pifu_field* occ_field,
                               const pifu_field* color_field, const float* view,
                               const pifu_render_opts* opts, uint32_t max_points, const float* bg,
                               float* rgb, float* depth, uint8_t* hit, pifu_level_stats* stats_dev,
                               uint32_t* status_dev, void* workspace, size_t workspace_bytes,
                               pifu_stream stream) {
  if (!ctx || !view || !bg || !rgb || !depth || !hit || !stats_dev || !status_dev || !workspace)
    return PIFU_ERR_INVALID_ARGUMENT;
  if (!aligned(workspace, kAlign) || !aligned(stats_dev, 4) || !aligned(status_dev, 4))
    return PIFU_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  int r = pifu_render_view_async_workspace_size(occ_field, color_field, opts, max_points, &need);
  if (r) return r;
  if (workspace_bytes < need) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  RenderWs* gp = new (std::nothrow) RenderWs;
  if (!gp) return PIFU_ERR_HIP;
  RenderWs& g = *gp;
  const int T = opts->log2_w - opts->log2_coarse_w;
  const int W = 1 << opts->log2_w, H = W, D = 1 << opts->log2_d;
  const size_t ncol = (size_t)W * H, last_n = ncol * (D + 1);
  const uint32_t cap0 = max_points ? max_points : default_async_cap(last_n);
  plan_render(occ_field, color_field, opts, workspace, g, cap0);
  const uint32_t cap = g.ew.chunk ? g.ew.chunk : cap0;   // what one pass holds
  hipStream_t s = as_stream(stream);
  EvalCtx e{ctx, s, g.counters, opts->precision, opts->guard_logit};
  e.band = logit_band(opts->band_delta);
  e.sur_band = logit_band(opts->surrogate_delta);
  e.aw = g.aw;
  launch_set_u32(g.aw, 0, s, AW_COUNT_WORDS);
  launch_set_u32(reinterpret_cast<uint32_t*>(stats_dev), 0, s,
                 (uint32_t)((T + 1) * sizeof(pifu_level_stats) / 4));
  r = pack_field(g.fp, ctx, s, g.counters);
  if (!r)
    r = pack_field(g.cp, ctx, s, g.counters, !split_band(g.fp));
  if (!r) r = fill_texel(e, g.fp, g.ew);
  double vd[12];
  for (int i = 0; i < 12; ++i) vd[i] = view[i];
  const Lat finL = level_lattice(g.log2, T, T);
  if (!r)
    r = localize_dev(e, g.fp, g.ew, vd, T, T - 1, g.lv, g.w, nullptr, finL, opts->max_waves,
                     opts->surrogate_max_log2, stats_dev, cap);
  if (r) {
    delete gp;
    return r;
  }
  // last level: interpolate, argmax along z from the observer, shadow nodes
  pifu_level_stats* sd = stats_dev + T;
  e.st_dev = sd;
  const LevelBuf& C = g.lv[T - 1];
  uint32_t* n_dev = g.counters + C_TOTAL;
  launch_set_u32(g.counters, 0, s, C_OVF);   // keeps C_OVF
  launch_fill_image(rgb, depth, hit, (uint32_t)(W * H), bg[0], bg[1], bg[2], s);
  launch_ray_count(C.st, C.lat, W, H, D, g.cnt, g.kstar, g.counters + C_SHADOW, s);
  launch_scan_u32(g.cnt, (uint32_t)(W * H), g.off, g.scan_scratch, n_dev, s);
  launch_ray_list(C.st, C.lat, W, H, D, g.kstar, g.off, g.w.list, s);
  {
    Book b(s);
    b.add(BK_SET_IMM, reinterpret_cast<uint32_t*>(&sd->level), nullptr, (uint32_t)opts->log2_w);
    b.add(BK_SET_IMM, stat_word(sd, &pifu_level_stats::nodes), nullptr, (uint32_t)last_n);
    b.add(BK_SET, stat_word(sd, &pifu_level_stats::shadow), g.counters + C_SHADOW);
    b.add(BK_SET, stat_word(sd, &pifu_level_stats::dilated), n_dev);
    b.add(BK_SET, stat_word(sd, &pifu_level_stats::evaluated), n_dev);
    b.add(BK_FLAG_GT, g.aw + AW_STATUS, n_dev, cap, kStatusListOver);
  }
  PointSrc src;
  std::memset(&src, 0, sizeof(src));
  src.mode = 0;
  src.nx = finL.nx;
  src.ny = finL.ny;
  src.nz = finL.nz;
  src.has_view = 1;
  for (int i = 0; i < 12; ++i) src.view[i] = vd[i];
  const uint32_t ecap = (uint32_t)std::min<size_t>(last_n, cap);
  r = eval_occupancy_dev(e, g.fp, src, g.w.list, ecap, n_dev, g.ew, g.w.logit, g.w.lab,
                         opts->log2_w <= opts->surrogate_max_log2);
  if (!r) {
    launch_ray_hit(C.st, C.occ, C.lat, W, H, D, g.off, g.cnt, g.w.list, g.w.logit, g.w.lab, vd,
                   depth, hit, g.hitpts, s);
    Lat img{1, 1, W * H};
    uint32_t* nh = g.aw + AW_NH;
    launch_compact(hit, (size_t)W * H, 1, 1, g.w.cscratch, nh, g.hitlist, (uint32_t)(W * H), 0, img,
                   s);
    {
      Book b(s);
      b.add(BK_SET, stat_word(sd, &pifu_level_stats::hits), nh);
    }
    PointSrc ps;
    std::memset(&ps, 0, sizeof(ps));
    ps.mode = 1;
    ps.pts = g.hitpts;
    EvalCtx ec{ctx, s, g.counters, PIFU_PREC_FP32, 0.f};
    ec.aw = g.aw;
    ec.st_dev = sd;
    // 16-bit renders colour with split-FP16 products; a value of this call outside the
    // binary16 range (an FP16 occupancy pass's or these products') re-runs them in FP32
    const bool x3 = g.cp.mlp.prec == PIFU_PREC_FP16;
    r = run_mlp_dev(ec, g.cp, g.cp.mlp, x3 ? PREC_F32X3 : PIFU_PREC_FP32, ps, g.hitlist,
                    (uint32_t)(W * H), nh, g.ew, nullptr, nullptr, rgb);
    if (!r && x3) {
      uint32_t* rr = g.aw + AW_RR;
      {
        Book b(s);
        b.add(BK_SEL, rr, nh, 0, 0, g.counters + C_OVF);
      }
      r = run_mlp_dev(ec, g.cp, g.cp.mlp, PIFU_PREC_FP32, ps, g.hitlist, (uint32_t)(W * H), rr,
                      g.ew, nullptr, nullptr, rgb);
    }
  }
  if (!r) {
    Book b(s);
    b.add(BK_SET, status_dev, g.aw + AW_STATUS);
  }
  if (!r) r = check_launch();
  delete gp;
  return r;
}

}  // extern "C"

// ================================================================== device-driven batch
// Several frames' levels in lockstep, as pifu_occupancy_grid_batched, with every count in
// device memory and a fixed ladder of conflict waves per level (as
// pifu_occupancy_grid_async): one set of launches per level and wave covers every
// frame's work list, nothing is read back, and the whole call can be captured into one
// HIP graph.  Per-frame statistics are tallied from the combined lists on the device.
namespace {

constexpr int C_TALLY = 72;   // kMaxBatch counter words for per-frame tallies
constexpr uint32_t kDefaultBatchCap = 1u << 21;

// Evaluates min(cap, *n_dev) entries of the combined list (indices p * frame_nodes +
// node): one pass of the network over every frame (the gathers pick each frame's feature
// map), the precision band and the FP64 guard over the combined list; analytic frames
// read their shapes from the device table.
int eval_frames_dev(EvalCtx& e, BatchPlan& b, const PointSrc& sall, uint32_t cap,
                    const uint32_t* n_dev) {
  const FieldPrep& fp0 = b.fps[0];
  if (!fp0.has_mlp) {
    launch_eval_analytic(sall, b.w.list, cap, fp0.f->kind, fp0.ell, fp0.f->plane, b.w.logit,
                         b.w.lab, e.s, n_dev, b.ell_tab);
    return check_launch();
  }
  return eval_full_dev(e, fp0, sall, b.w.list, cap, n_dev, b.ew, b.w.logit, b.w.lab);
}

int validate_batch_async(int n, const pifu_field* const* fields, const pifu_grid_opts* const* opts) {
  int r = validate_batch(n, fields, opts);
  if (r) return r;
  const pifu_grid_opts& o = *opts[0];
  if (o.precision == PIFU_PREC_FP8) return PIFU_ERR_UNSUPPORTED;
  if (fields[0]->kind == PIFU_FIELD_PLANE) return PIFU_ERR_UNSUPPORTED;
  if (fields[0]->kind == PIFU_FIELD_MLP && fields[0]->surrogate &&
      o.surrogate_max_log2 >= o.log2_coarse)
    return PIFU_ERR_UNSUPPORTED;
  return PIFU_OK;
}

// The combined capacity of one evaluation pass.
uint32_t batch_async_cap(int n, const pifu_field* const* fields, const pifu_grid_opts* const* opts,
                         uint32_t max_points, size_t* max_n_out) {
  BatchPlan* bp = new (std::nothrow) BatchPlan;
  if (!bp) return 0;
  plan_batch(n, fields, opts, nullptr, *bp, 1);
  size_t max_n = 0;
  for (int r = 0; r <= bp->Tmax; ++r) max_n = std::max(max_n, bp->lat[r].n() * bp->active[r]);
  delete bp;
  if (max_n_out) *max_n_out = max_n;
  const size_t want = max_points ? max_points : std::min<size_t>(max_n, kDefaultBatchCap);
  return (uint32_t)std::min<size_t>(want, max_n);
}

}  // namespace

extern "C" {

int32_t pifu_occupancy_grid_batched_async_workspace_size(int32_t n, const pifu_field* const* fields,
                                                         const pifu_grid_opts* const* opts,
                                                         uint32_t max_points, size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  int r = validate_batch_async(n, fields, opts);
  if (r) return r;
  const uint32_t cap = batch_async_cap(n, fields, opts, max_points, nullptr);
  if (!cap) return PIFU_ERR_HIP;
  BatchPlan* bp = new (std::nothrow) BatchPlan;
  if (!bp) return PIFU_ERR_HIP;
  plan_batch(n, fields, opts, nullptr, *bp, cap);
  *bytes = bp->bytes;
  delete bp;
  return PIFU_OK;
}

int32_t pifu_occupancy_grid_batched_async(pifu_ctx* ctx, int32_t n, const pifu_field* const* fields,
                                          const pifu_grid_opts* const* opts, uint32_t max_points,
                                          const pifu_grid_out_dev* outs, uint32_t* status_dev,
                                          void* workspace, size_t workspace_bytes,
                                          pifu_stream stream) {
  if (!ctx || !outs || !status_dev || !workspace || !aligned(workspace, kAlign) ||
      !aligned(status_dev, 4))
    return PIFU_ERR_INVALID_ARGUMENT;
  int rc = validate_batch_async(n, fields, opts);
  if (rc) return rc;
  for (int f = 0; f < n; ++f) {
    const pifu_grid_out_dev& o = outs[f];
    if (!o.occ || !o.labels || !o.n_cells_dev || !o.stats_dev || (o.cells_cap && !o.cells) ||
        !aligned(o.n_cells_dev, 4) || !aligned(o.stats_dev, 4))
      return PIFU_ERR_INVALID_ARGUMENT;
  }
  const uint32_t cap = batch_async_cap(n, fields, opts, max_points, nullptr);
  if (!cap) return PIFU_ERR_HIP;
  BatchPlan* bp = new (std::nothrow) BatchPlan;
  if (!bp) return PIFU_ERR_HIP;
  BatchPlan& b = *bp;
  plan_batch(n, fields, opts, nullptr, b, cap);
  if (workspace_bytes < b.bytes) {
    delete bp;
    return PIFU_ERR_WORKSPACE_TOO_SMALL;
  }
  plan_batch(n, fields, opts, workspace, b, cap);
  // the first level evaluates every node of every frame in one pass
  if ((size_t)b.lat[0].n() * b.active[0] > cap) {
    delete bp;
    return PIFU_ERR_WORKSPACE_TOO_SMALL;
  }
  hipStream_t s = as_stream(stream);
  const pifu_grid_opts& o = *opts[0];
  EvalCtx e{ctx, s, b.counters, o.precision, o.guard_logit};
  e.band = logit_band(o.band_delta);
  e.aw = b.aw;
  FrameCount fc;
  fc.tally = b.counters + C_TALLY;
  e.fc = &fc;
  launch_set_u32(b.aw, 0, s, AW_COUNT_WORDS);
  launch_set_u32(b.counters, 0, s, kCounters + 2 * kMaxFrames + 64);
  for (int f = 0; f < n; ++f)
    launch_set_u32(reinterpret_cast<uint32_t*>(outs[f].stats_dev), 0, s,
                   (uint32_t)((b.T[f] + 1) * sizeof(pifu_level_stats) / 4));
  rc = pack_field(b.fps[0], ctx, s, b.counters);
  if (rc) {
    delete bp;
    return rc;
  }
  for (int f = 1; f < n; ++f) {   // frames share the packed network
    b.fps[f].mlp = b.fps[0].mlp;
    b.fps[f].sur = b.fps[0].sur;
  }
  if (!b.fps[0].has_mlp)
    for (int p = 0; p < n; ++p) launch_store_ellipsoids(b.ell_tab + p, b.fps[b.order[p]].ell, s);
  const bool bounded = o.max_waves > 0;
  const int budget = bounded ? o.max_waves : kDefaultWaveBudget;
  uint32_t* n_dev = b.counters + C_TOTAL;
  for (int r = 0; r <= b.Tmax && !rc; ++r) {
    const Lat L = b.lat[r];
    const int A = b.active[r];
    const uint32_t nl = (uint32_t)L.n();
    const uint32_t tot = nl * (uint32_t)A;
    const int level_id = b.l0 + r;
    fc.frames = A;
    fc.frame_nodes = nl;
    for (int p = 0; p < A; ++p) fc.st[p] = outs[b.order[p]].stats_dev + r;
    launch_set_u32(b.counters, 0, s, C_OVF);   // keeps C_OVF
    launch_set_u32(b.counters + C_SEG, 0, s, C_TALLY + kMaxFrames - C_SEG);
    {
      Book bk(s);
      for (int p = 0; p < A; ++p) {
        bk.add(BK_SET_IMM, reinterpret_cast<uint32_t*>(&fc.st[p]->level), nullptr,
               (uint32_t)level_id);
        bk.add(BK_SET_IMM, stat_word(fc.st[p], &pifu_level_stats::nodes), nullptr, nl);
      }
    }
    FrameOcc fo{};
    for (int p = 0; p < A; ++p)
      if (b.T[b.order[p]] == r) fo.p[p] = outs[b.order[p]].occ;
    PointSrc sall;
    std::memset(&sall, 0, sizeof(sall));
    sall.mode = 0;
    sall.nx = L.nx;
    sall.ny = L.ny;
    sall.nz = L.nz;
    sall.frame_nodes = nl;
    for (int p = 0; p < A; ++p) sall.feat_tab[p] = b.fps[b.order[p]].f->feat;
    if (r == 0) {
      launch_fill_u8(b.st[0], 0, tot, s);
      launch_iota(b.w.list, tot, s);
      {
        Book bk(s);
        bk.add(BK_SET_IMM, b.aw + AW_N0, nullptr, tot);
      }
      rc = eval_frames_dev(e, b, sall, tot, b.aw + AW_N0);
      if (rc) break;
      launch_apply_grid(b.w.list, tot, b.w.logit, b.w.lab, b.st[0], b.occ[0], nullptr, nullptr,
                        level_id, L, 1, L, 0, s, nl, &fo, nullptr, b.aw + AW_N0);
      Book bk(s);
      for (int p = 0; p < A; ++p) {
        bk.add(BK_SET_IMM, stat_word(fc.st[p], &pifu_level_stats::dilated), nullptr, nl);
        bk.add(BK_SET_IMM, stat_word(fc.st[p], &pifu_level_stats::evaluated), nullptr, nl);
      }
    } else {
      launch_transition(b.st[r - 1], b.occ[r - 1], b.lat[r - 1], b.st[r], b.occ[r], L, s, A, &fo);
      if (2 * b0_mask_words(L) * (size_t)A <= b.list_words) {
        launch_select_b0(b.st[r], L, A, reinterpret_cast<uint64_t*>(b.w.list), b.counters + C_B0_F,
                         1, s);
      } else {
        for (int p = 0; p < A; ++p)
          launch_count_bits(b.st[r] + (size_t)p * nl, nl, ST_B0, b.counters + C_B0_F + p, s);
        launch_select(b.st[r], L, s, A);
      }
      const uint32_t ecap = std::min(tot, cap);
      launch_compact(b.st[r], tot, ST_PEND, ST_PEND, b.w.cscratch, n_dev, b.w.list, b.list_cap, 0,
                     L, s);
      count_frames(e, b.w.list, nullptr, ecap, n_dev, &pifu_level_stats::dilated, BK_SET);
      {
        Book bk(s);
        bk.add(BK_FLAG_GT, b.aw + AW_STATUS, n_dev, cap, kStatusListOver);
      }
      for (int rung = 0; rung <= budget; ++rung) {
        rc = eval_frames_dev(e, b, sall, ecap, n_dev);
        if (rc) break;
        launch_apply_grid(b.w.list, ecap, b.w.logit, b.w.lab, b.st[r], b.occ[r],
                          b.counters + C_CONF_F, nullptr, level_id, L, 1, L, 1, s, nl, &fo, nullptr,
                          n_dev);
        count_frames(e, b.w.list, nullptr, ecap, n_dev, &pifu_level_stats::evaluated, BK_ADD,
                     rung > 0 ? &pifu_level_stats::waves : nullptr, BK_ADD_NZ);
        if (rung == budget && bounded) break;
        launch_expand(b.w.list, ecap, b.st[r], L, s, nl, n_dev);
        launch_compact(b.st[r], tot, ST_PEND, ST_PEND, b.w.cscratch, n_dev, b.w.list, b.list_cap,
                       0, L, s, 0, n_dev);
        Book bk(s);
        if (rung < budget) bk.add(BK_FLAG_GT, b.aw + AW_STATUS, n_dev, cap, kStatusListOver);
        else bk.add(BK_FLAG_GT, b.aw + AW_STATUS, n_dev, 0, kStatusWavesLeft);
      }
      if (rc) break;
      Book bk(s);
      for (int p = 0; p < A; ++p) {
        bk.add(BK_SET, stat_word(fc.st[p], &pifu_level_stats::conflicts), b.counters + C_CONF_F + p);
        bk.add(BK_SET, stat_word(fc.st[p], &pifu_level_stats::b0), b.counters + C_B0_F + p);
      }
    }
    // frames whose final level this is: labels, cells and their count out
    for (int p = 0; p < A; ++p) {
      const int f = b.order[p];
      if (b.T[f] != r) continue;
      uint8_t* sf = b.st[r] + (size_t)p * nl;
      launch_cells(sf, L, outs[f].labels, s);
      launch_compact(sf, nl, ST_CELL, ST_CELL, b.w.cscratch, n_dev, outs[f].cells, outs[f].cells_cap,
                     1, L, s);
      Book bk(s);
      bk.add(BK_SET, outs[f].n_cells_dev, n_dev);
      bk.add(BK_FLAG_GT, b.aw + AW_STATUS, n_dev, outs[f].cells_cap, kStatusCellsOver);
    }
    if (!rc) rc = check_launch();
  }
  if (!rc) {
    Book bk(s);
    bk.add(BK_SET, status_dev, b.aw + AW_STATUS);
  }
  if (!rc) rc = check_launch();
  delete bp;
  return rc;
}

}  // extern "C"

// ================================================================== mesh hand-off
namespace {

struct MeshWs {
  uint32_t* counters = nullptr;
  uint8_t* flags = nullptr;      // 3 per node: the lattice edge from the node crosses
  uint32_t* ids = nullptr;       // crossed edge ids, sorted (one vertex each)
  uint32_t* cscratch = nullptr;
  int32_t* kf = nullptr;         // front node per input-view column
  uint32_t *tcnt = nullptr, *toff = nullptr, *tscan = nullptr;
  uint8_t* hidden = nullptr;     // per vertex: not visible from the input camera
  uint32_t* hlist = nullptr;     // vertices coloured by the network
  float4* pts = nullptr;         // per vertex (x, y, z, 0.5): the colour network's input
  FieldPrep cp;
  EvalWs ew;
  size_t bytes = 0;
};

void plan_mesh(int L, uint32_t n_cells, uint32_t vert_cap, const pifu_field* col, void* base,
               MeshWs& m) {
  const size_t nn = ((size_t)1 << L) + 1, N = nn * nn * nn;
  Carver cv(base);
  m.counters = cv.take<uint32_t>(kCounters);
  m.flags = cv.take<uint8_t>(3 * N + 16);
  m.ids = cv.take<uint32_t>(std::max<uint32_t>(vert_cap, 1));
  m.cscratch = cv.take<uint32_t>(std::max(compact_scratch_words(3 * N),
                                          std::max(compact_scratch_words(vert_cap),
                                                   scan_scratch_words(n_cells))));
  m.kf = cv.take<int32_t>(nn * nn);
  m.tcnt = cv.take<uint32_t>(std::max<uint32_t>(n_cells, 1));
  m.toff = cv.take<uint32_t>(std::max<uint32_t>(n_cells, 1));
  m.tscan = cv.take<uint32_t>(scan_scratch_words(std::max<uint32_t>(n_cells, 1)));
  m.hidden = cv.take<uint8_t>((size_t)vert_cap + 16);
  m.hlist = cv.take<uint32_t>(std::max<uint32_t>(vert_cap, 1));
  m.pts = cv.take<float4>(std::max<uint32_t>(vert_cap, 1));
  if (col) {
    carve_field(cv, col, PIFU_PREC_FP32, m.cp);
    carve_eval(cv, std::max<uint32_t>(vert_cap, 1), col->C, m.cp.mlp.max_hidden, m.ew);
  }
  m.bytes = cv.off + kAlign;
}

int validate_mesh(int L, uint32_t n_cells, const uint32_t* cells, const pifu_field* col,
                  const float* image, int img_h, int img_w) {
  if (L < 1 || L > 9) return PIFU_ERR_INVALID_ARGUMENT;
  if (n_cells && !cells) return PIFU_ERR_INVALID_ARGUMENT;
  if ((uint64_t)n_cells > ((uint64_t)1 << (3 * L))) return PIFU_ERR_INVALID_ARGUMENT;
  if (col) {
    if (col->kind != PIFU_FIELD_MLP) return PIFU_ERR_INVALID_ARGUMENT;
    if (int r = validate_field(col, 2, 3)) return r;
  }
  if (image && (img_h < 2 || img_w < 2)) return PIFU_ERR_INVALID_ARGUMENT;
  return PIFU_OK;
}

}  // namespace

extern "C" {

int32_t pifu_mesh_workspace_size(int32_t log2_final, uint32_t n_cells, uint32_t vert_cap,
                                 const pifu_field* color_field, size_t* bytes) {
  if (!bytes) return PIFU_ERR_INVALID_ARGUMENT;
  static const uint32_t kNoCells = 0;   // the cell pointer is not needed for the size
  if (int r = validate_mesh(log2_final, n_cells, &kNoCells, color_field, nullptr, 0, 0)) return r;
  MeshWs m;
  plan_mesh(log2_final, n_cells, vert_cap, color_field, nullptr, m);
  *bytes = m.bytes;
  return PIFU_OK;
}

int32_t pifu_mesh(pifu_ctx* ctx, int32_t log2_final, const float* occ, const uint8_t* labels,
                  const uint32_t* cells, uint32_t n_cells, const pifu_field* color_field,
                  const float* image, int32_t img_h, int32_t img_w, float* verts, float* colors,
                  uint32_t vert_cap, uint32_t* n_verts, uint32_t* tris, uint32_t tri_cap,
                  uint32_t* n_tris, void* workspace, size_t workspace_bytes, pifu_stream stream) {
  if (!ctx || !occ || !labels || !n_verts || !n_tris || !workspace || !aligned(workspace, kAlign))
    return PIFU_ERR_INVALID_ARGUMENT;
  if ((vert_cap && !verts) || (tri_cap && !tris)) return PIFU_ERR_INVALID_ARGUMENT;
  if (colors && !color_field) return PIFU_ERR_INVALID_ARGUMENT;
  if (int r = validate_mesh(log2_final, n_cells, cells, color_field, image, img_h, img_w)) return r;
  MeshWs m;
  plan_mesh(log2_final, n_cells, vert_cap, colors ? color_field : nullptr, nullptr, m);
  if (workspace_bytes < m.bytes) return PIFU_ERR_WORKSPACE_TOO_SMALL;
  plan_mesh(log2_final, n_cells, vert_cap, colors ? color_field : nullptr, workspace, m);
  hipStream_t s = as_stream(stream);
  const int nn = (1 << log2_final) + 1;
  const size_t N = (size_t)nn * nn * nn;
  EvalCtx e{ctx, s, m.counters, PIFU_PREC_FP32, 0.f};
  HIP_TRY(hipMemsetAsync(m.counters, 0, sizeof(uint32_t) * kCounters, s));
  // vertices: the crossed lattice edges, in edge-id order
  launch_mesh_edge_flags(labels, nn, m.flags, s);
  uint32_t nv_all = 0;
  Lat flat{1, 1, (int)std::min<size_t>(3 * N, INT32_MAX)};
  int r = compact_count(e, m.flags, 3 * N, 1, 1, m.cscratch, m.ids, vert_cap, 0, flat, &nv_all);
  if (r) return r;
  const uint32_t nv = std::min(nv_all, vert_cap);
  launch_mesh_front(labels, nn, m.kf, s);
  launch_mesh_verts(m.ids, nv, occ, nn, m.kf, verts, colors ? m.hidden : nullptr,
                    colors ? m.pts : nullptr, s);
  // triangles: per-cell counts, offsets, then each cell's triangles
  uint32_t nt_all = 0;
  if (n_cells) {
    launch_mesh_tri_count(cells, n_cells, labels, nn, m.tcnt, s);
    launch_scan_u32(m.tcnt, n_cells, m.toff, m.tscan, m.counters + C_GUARD, s);
    r = read_counters(e, C_GUARD + 1);
    if (r) return r;
    nt_all = ctx->host_counters[C_GUARD];
    launch_mesh_tri_write(cells, n_cells, labels, nn, m.toff, m.ids, nv, tris, tri_cap, s);
  }
  // colours: the input pixel where visible, the colour network elsewhere
  if (colors && nv) {
    if (image) {
      launch_mesh_pixel_colors(verts, m.hidden, nv, image, img_h, img_w, colors, s);
    } else {
      launch_fill_u8(m.hidden, 1, nv, s);
    }
    uint32_t nh = 0;
    Lat vl{1, 1, (int)nv};
    r = compact_count(e, m.hidden, nv, 1, 1, m.cscratch, m.hlist, nv, 0, vl, &nh);
    if (r) return r;
    if (nh) {
      r = pack_field(m.cp, ctx, s, m.counters);
      if (r) return r;
      PointSrc ps;
      std::memset(&ps, 0, sizeof(ps));
      ps.mode = 1;
      ps.pts = m.pts;
      EvalCtx ec{ctx, s, m.counters, PIFU_PREC_FP32, 0.f};
      r = run_mlp(ec, m.cp, m.cp.mlp, PIFU_PREC_FP32, ps, m.hlist, nh, m.ew, nullptr, nullptr,
                  colors);
      if (r) return r;
    }
  }
  r = check_launch();
  if (!r) r = hipStreamSynchronize(s) == hipSuccess ? PIFU_OK : PIFU_ERR_HIP;
  *n_verts = nv_all;
  *n_tris = nt_all;
  prof_resolve(ctx);
  return r;
}

}  // extern "C"
