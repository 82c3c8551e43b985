// Host side of the C ABI: configuration checks, weight segments, workspace
// layout, the stage sequence of etx_run, HIP-graph capture and replay.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "seg.hpp"
#include "tile.hpp"

namespace etx {

int embed_attributes(size_t max_lds);
int gnn_attributes(size_t max_lds);
int graph_attributes(size_t max_lds);
int radius_attributes(size_t max_lds);
int prefilter_attributes(size_t max_lds);
int train_attributes(size_t max_lds);
int triplet_attributes(size_t max_lds);

bool GraphKey::operator<(const GraphKey& o) const {
  for (int i = 0; i < 16; ++i)
    if (p[i] != o.p[i]) return p[i] < o.p[i];
  for (int i = 0; i < 4; ++i)
    if (n[i] != o.n[i]) return n[i] < o.n[i];
  return false;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

WsLayout ws_layout(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_cap) {
  const etx_config& c = ctx->cfg;
  const int64_t H = c.gnn_hidden;
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(std::max<size_t>(bytes, 1));
    return at;
  };
  L.n_scan_blocks = (n_hits + kScanBlock - 1) / kScanBlock;
  L.bucket = take(sizeof(int32_t) * n_hits);
  L.plane_off = take(sizeof(int32_t) * n_events * (c.n_planes + 1));
  L.emb = take(sizeof(float) * n_hits * kDpad);
  L.cnt = take(sizeof(int32_t) * n_hits);
  L.slots = take(sizeof(int32_t) * n_hits * c.k_max);
  L.row_ptr = take(sizeof(int64_t) * (n_hits + 1));
  L.scan_tmp = take(sizeof(int64_t) * (L.n_scan_blocks + 1));
  L.col_ptr = take(sizeof(int64_t) * (n_hits + 1));
  L.csc = take(sizeof(int32_t) * edge_cap);
  L.h = take(sizeof(float) * n_hits * H);
  L.ps = take(sizeof(float) * n_hits * H);
  L.pd = take(sizeof(float) * n_hits * H);
  L.msg = take(sizeof(float) * n_hits * 2 * H);
  L.e = take(sizeof(float) * edge_cap * H);
  L.opart = take(sizeof(float) * 2 * ((edge_cap + kEdgeTile - 1) / kEdgeTile) * H);
  L.kept = take(sizeof(int32_t) * edge_cap);
  L.kept_cnt = take(sizeof(int32_t) * n_events);
  L.calib = take(sizeof(float) * ETX_N_CALIB);
  L.pf_keep = take(sizeof(uint8_t) * edge_cap);
  L.pf_tmp = take(sizeof(int64_t) * (n_hits + 1));
  L.cand_src = take(sizeof(int32_t) * edge_cap);
  L.cand_dst = take(sizeof(int32_t) * edge_cap);
  L.pf_prob = take(sizeof(float) * edge_cap);
  L.pf_part = take(sizeof(float) * (size_t)kPfMaxWaves * kPfGradStride);
  L.pf_grad = take(sizeof(float) * kPfGradStride);
  L.pf_polar = take(sizeof(float) * 2 * n_hits);
  L.pf_feat = take(ctx->pf_features ? sizeof(float) * 8 * edge_cap : 0);
  L.pf_fallback = take(sizeof(int32_t) * n_events);
  L.total = o;
  return L;
}

// ---------------------------------------------------------------------------
// host-side number formats
// ---------------------------------------------------------------------------

static uint16_t host_bf16(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);   // quiet NaN
  b += 0x7fffu + ((b >> 16) & 1u);                                          // round to nearest even
  return (uint16_t)(b >> 16);
}

// OCP E4M3: round to nearest even, saturate to +-448.
static uint8_t host_e4m3(double x) {
  uint8_t sign = std::signbit(x) ? 0x80 : 0;
  double a = std::fabs(x);
  if (!(a == a)) return 0;
  if (a > 448.0) a = 448.0;
  int e;
  std::frexp(a, &e);                     // a = f 2^e, f in [0.5, 1)
  int lead = std::max(e - 1, -6);        // subnormal spacing below 2^-6
  double q = std::nearbyint(a / std::ldexp(1.0, lead - 3));   // ties to even
  double v = q * std::ldexp(1.0, lead - 3);
  if (v > 448.0) v = 448.0;
  if (v == 0.0) return sign;
  int ve;
  double vf = std::frexp(v, &ve);        // v = vf 2^ve
  int E = ve - 1 + 7;                    // biased exponent
  uint8_t code;
  if (E <= 0) code = (uint8_t)std::lround(v / std::ldexp(1.0, -9));      // subnormal
  else code = (uint8_t)((E << 3) | (int)std::lround((vf * 2.0 - 1.0) * 8.0));
  return sign | code;
}

// Power of two at or above amax / 448 (1 when amax is 0).
static float pow2_scale(double amax) {
  if (!(amax > 0.0)) return 1.0f;
  int e;
  double f = std::frexp(amax / 448.0, &e);
  return (float)std::ldexp(1.0, f == 0.5 ? e - 1 : e);
}

// Write a row-major [K][M] weight (M padded to Mpad) permuted for the column
// layout of tile.hpp in segment format `prec`; FP8 and INT8 store codes of W / scale.
static float bf16_float(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static void put_perm(char* out, const float* W, int K, int M, int Mpad, int prec, double scale) {
  for (int mb = 0; mb < Mpad / 16; ++mb)
    for (int lane = 0; lane < 64; ++lane) {
      const int col = 16 * mb + lane % 16, g = lane / 16;
      if (prec == ETX_FP32) {
        for (int t = 0; t < K / 4; ++t) {
          const int row = phi(t, g);
          float v = col < M ? W[(size_t)row * M + col] : 0.f;
          std::memcpy(out + (((size_t)mb * (K / 4) + t) * 64 + lane) * 4, &v, 4);
        }
      } else {
        for (int t = 0; t < K / 32; ++t)
          for (int q = 0; q < 8; ++q) {
            const int row = phi(8 * t + q, g);
            const float v = col < M ? W[(size_t)row * M + col] : 0.f;
            const size_t at = (((size_t)mb * (K / 32) + t) * 64 + lane) * 8 + q;
            if (prec == kF32Split) {
              // three BF16 planes: hi, mid, lo with v = hi + mid + lo to 24 bits
              const size_t plane = (size_t)Mpad * K;
              const uint16_t h = host_bf16(v);
              const float r = v - bf16_float(h);
              const uint16_t m = host_bf16(r);
              const uint16_t l = host_bf16(r - bf16_float(m));
              std::memcpy(out + at * 2, &h, 2);
              std::memcpy(out + (plane + at) * 2, &m, 2);
              std::memcpy(out + (2 * plane + at) * 2, &l, 2);
            } else if (prec == ETX_BF16) {
              uint16_t b = host_bf16(v);
              std::memcpy(out + at * 2, &b, 2);
            } else if (prec == kI8Seg) {
              // symmetric INT8: clip(round(W / S), -127, 127), ties to even
              const double q = std::nearbyint((double)v / scale);
              out[at] = (char)(int8_t)std::max(-127.0, std::min(127.0, q));
            } else {
              out[at] = (char)host_e4m3((double)v / scale);
            }
          }
      }
    }
}

static float layer_amax(const float* W, size_t n) {
  float m = 0.f;
  for (size_t i = 0; i < n; ++i) m = std::max(m, std::fabs(W[i]));
  return m;
}

namespace {

struct BlobLayer {
  const float* W;
  const float* b;
  int K, M;
};

bool parse_blob(const etx_config& c, const void* blob, size_t nbytes, std::vector<float>& payload,
                std::vector<BlobLayer>& layers) {
  if (nbytes < 32) return false;
  int32_t hd[8];
  std::memcpy(hd, blob, 32);
  if (hd[0] != 0x57585445 || hd[1] != 1 || hd[2] != 3 || hd[3] != c.emb_hidden || hd[4] != c.emb_layers ||
      hd[5] != c.emb_dim || hd[6] != c.gnn_hidden || hd[7] != c.gnn_steps)
    return false;
  size_t need = 0;
  std::vector<std::pair<int, int>> dims;
  const int W = c.emb_hidden, H = c.gnn_hidden;
  dims.push_back({3, W});
  for (int l = 1; l < c.emb_layers; ++l) dims.push_back({W, W});
  dims.push_back({W, c.emb_dim});
  dims.push_back({3, H});
  dims.push_back({H, H});
  dims.push_back({2 * H, H});
  dims.push_back({H, H});
  for (int k = 0; k < c.gnn_steps; ++k) {
    dims.push_back({3 * H, H});
    dims.push_back({H, H});
    dims.push_back({3 * H, H});
    dims.push_back({H, H});
  }
  dims.push_back({H, H});
  dims.push_back({H, 1});
  for (auto& d : dims) need += (size_t)d.first * d.second + d.second;
  if (nbytes != 32 + need * sizeof(float)) return false;
  payload.resize(need);
  std::memcpy(payload.data(), static_cast<const char*>(blob) + 32, need * sizeof(float));
  for (float v : payload)
    if (!std::isfinite(v)) return false;
  size_t o = 0;
  for (auto& d : dims) {
    BlobLayer L{payload.data() + o, payload.data() + o + (size_t)d.first * d.second, d.first, d.second};
    o += (size_t)d.first * d.second + d.second;
    layers.push_back(L);
  }
  return true;
}

size_t blob_floats(const etx_config& c) {
  const size_t W = c.emb_hidden, H = c.gnn_hidden;
  size_t n = 3 * W + W + (c.emb_layers - 1) * (W * W + W) + W * c.emb_dim + c.emb_dim;
  n += 3 * H + H + H * H + H + 2 * H * H + H + H * H + H;
  n += (size_t)c.gnn_steps * 2 * (3 * H * H + H + H * H + H);
  n += H * H + H + H + 1;
  return n;
}

etx_status check_config(const etx_config* c) {
  if (!c) return ETX_ERR_INVALID_ARG;
  if (c->n_planes < 1 || c->n_planes > ETX_MAX_PLANES) return ETX_ERR_INVALID_ARG;
  if (!(c->r_scale_mm > 0) || !(c->z_scale_mm > 0) || !std::isfinite(c->r_scale_mm) || !std::isfinite(c->z_scale_mm))
    return ETX_ERR_INVALID_ARG;
  if (c->emb_hidden != 32 && c->emb_hidden != 64 && c->emb_hidden != 128) return ETX_ERR_UNSUPPORTED;
  if (c->emb_layers < 1 || c->emb_layers > 4) return ETX_ERR_UNSUPPORTED;
  if (c->emb_dim < 1 || c->emb_dim > kDpad) return ETX_ERR_UNSUPPORTED;
  if (!(c->radius >= 0) || !std::isfinite(c->radius)) return ETX_ERR_INVALID_ARG;
  if (c->k_max < 1 || c->k_max > 64) return ETX_ERR_UNSUPPORTED;
  if (c->plane_window < 1 || c->plane_window > 4) return ETX_ERR_UNSUPPORTED;
  if (c->gnn_hidden != 32 && c->gnn_hidden != 64) return ETX_ERR_UNSUPPORTED;
  if (c->gnn_steps < 1 || c->gnn_steps > 16) return ETX_ERR_UNSUPPORTED;
  if (!std::isfinite(c->edge_threshold)) return ETX_ERR_INVALID_ARG;
  if (c->precision < ETX_FP32 || c->precision > ETX_INT8) return ETX_ERR_INVALID_ARG;
  if (c->prefilter != 0 && c->prefilter != 1) return ETX_ERR_INVALID_ARG;
  if (!std::isfinite(c->prefilter_tau)) return ETX_ERR_INVALID_ARG;
  return ETX_OK;
}

void clear_graphs(etx_ctx* ctx) {
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs.clear();
}

}  // namespace

// Build the weight segments of one operand precision on the host and upload them.
static etx_status build_segments(etx_ctx* ctx, const std::vector<BlobLayer>& Ls, int prec) {
  const etx_config& c = ctx->cfg;
  const int W = c.emb_hidden, H = c.gnn_hidden, S = c.gnn_steps, LE = c.emb_layers;
  const int ES = kSegBytes[prec];
  WeightMap& m = ctx->wmap[prec];
  std::vector<char> buf;
  auto reserve = [&](int n) {
    int64_t at = (int64_t)buf.size();
    buf.resize(buf.size() + ((n + 15) & ~15), 0);
    return at;
  };
  auto put_vec = [&](int64_t at, const float* v, int n) { std::memcpy(buf.data() + at, v, sizeof(float) * n); };
  // weight scales of this set (INT8: the exact max|W| / 127 the codes divide by)
  double sc[N_SCALES] = {};
  for (int i = 0; i < 256; ++i) sc[i] = prec == kI8Seg ? ctx->i8_wscale[i] : (double)ctx->host_scales[i];
  size_t li = 0;
  {
    SegEmb s{W, LE, ES};
    m.emb = reserve(s.size());
    const BlobLayer& l1 = Ls[li++];
    put_vec(m.emb + s.w1(), l1.W, 3 * W);
    put_vec(m.emb + s.b1(), l1.b, W);
    for (int l = 1; l < LE; ++l) {
      const BlobLayer& L = Ls[li++];
      put_perm(buf.data() + m.emb + s.wh(l), L.W, W, W, W, prec, sc[SW_EMB + l]);
      put_vec(m.emb + s.bh(l), L.b, W);
    }
    const BlobLayer& lo = Ls[li++];
    put_perm(buf.data() + m.emb + s.wo(), lo.W, W, c.emb_dim, 16, prec, sc[SW_EMB + LE]);
    put_vec(m.emb + s.bo(), lo.b, c.emb_dim);
  }
  const BlobLayer ne1 = Ls[li++], ne2 = Ls[li++], ee1 = Ls[li++], ee2 = Ls[li++];
  std::vector<BlobLayer> nn1(S), nn2(S), en1(S), en2(S);
  for (int k = 0; k < S; ++k) {
    nn1[k] = Ls[li++];
    nn2[k] = Ls[li++];
    en1[k] = Ls[li++];
    en2[k] = Ls[li++];
  }
  const BlobLayer c1 = Ls[li++], c2 = Ls[li++];
  const size_t HH = (size_t)H * H;
  {
    SegNodeEnc s{H, ES};
    m.node_enc = reserve(s.size());
    put_vec(m.node_enc + s.w1(), ne1.W, 3 * H);
    put_vec(m.node_enc + s.b1(), ne1.b, H);
    put_perm(buf.data() + m.node_enc + s.w2(), ne2.W, H, H, H, prec, sc[SW_NE2]);
    put_vec(m.node_enc + s.b2(), ne2.b, H);
    put_perm(buf.data() + m.node_enc + s.ws(), ee1.W, H, H, H, prec, sc[SW_EE1]);        // rows 0..H-1: h_src
    put_perm(buf.data() + m.node_enc + s.wd(), ee1.W + HH, H, H, H, prec, sc[SW_EE1]);   // rows H..2H-1: h_dst
  }
  {
    SegEdgeEnc s{H, ES};
    m.edge_enc = reserve(s.size());
    put_vec(m.edge_enc + s.b1(), ee1.b, H);
    put_perm(buf.data() + m.edge_enc + s.w2(), ee2.W, H, H, H, prec, sc[SW_EE2]);
    put_vec(m.edge_enc + s.b2(), ee2.b, H);
  }
  for (int k = 0; k < S; ++k) {
    SegNode s{H, ES};
    m.node[k] = reserve(s.size());
    put_perm(buf.data() + m.node[k] + s.w1(), nn1[k].W, 3 * H, H, H, prec, sc[SW_STEP + 4 * k]);
    put_vec(m.node[k] + s.b1(), nn1[k].b, H);
    put_perm(buf.data() + m.node[k] + s.w2(), nn2[k].W, H, H, H, prec, sc[SW_STEP + 4 * k + 1]);
    put_vec(m.node[k] + s.b2(), nn2[k].b, H);
    put_perm(buf.data() + m.node[k] + s.ws(), en1[k].W + HH, H, H, H, prec, sc[SW_STEP + 4 * k + 2]);      // h_src rows
    put_perm(buf.data() + m.node[k] + s.wd(), en1[k].W + 2 * HH, H, H, H, prec, sc[SW_STEP + 4 * k + 2]);  // h_dst rows
    SegEdge se{H, ES};
    m.edge[k] = reserve(se.size());
    put_perm(buf.data() + m.edge[k] + se.we(), en1[k].W, H, H, H, prec, sc[SW_STEP + 4 * k + 2]);          // e rows
    put_vec(m.edge[k] + se.b1(), en1[k].b, H);
    put_perm(buf.data() + m.edge[k] + se.w2(), en2[k].W, H, H, H, prec, sc[SW_STEP + 4 * k + 3]);
    put_vec(m.edge[k] + se.b2(), en2[k].b, H);
  }
  {
    SegCls s{H, ES};
    m.cls = reserve(s.size());
    put_perm(buf.data() + m.cls + s.w1(), c1.W, H, H, H, prec, sc[SW_CLS1]);
    put_vec(m.cls + s.b1(), c1.b, H);
    put_vec(m.cls + s.w2(), c2.W, H);
    put_vec(m.cls + s.b2(), c2.b, 1);
  }
  m.total = (int64_t)buf.size();
  if (hipMalloc(&ctx->seg_base[prec], buf.size()) != hipSuccess) return ETX_ERR_HIP;
  if (hipMemcpy(ctx->seg_base[prec], buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess) return ETX_ERR_HIP;
  return ETX_OK;
}

// Per-layer weight scales into host_scales: FP8 powers of two at 64.., INT8
// max|W| / 127 at SC_I8 + 64.. (and exactly in i8_wscale).
static void weight_scales(etx_ctx* ctx, const std::vector<BlobLayer>& Ls) {
  const etx_config& c = ctx->cfg;
  const int S = c.gnn_steps, LE = c.emb_layers;
  float* sc = ctx->host_scales;
  for (int i = 0; i < N_SCALES; ++i) sc[i] = 1.0f;
  auto amax = [&](const BlobLayer& L) { return layer_amax(L.W, (size_t)L.K * L.M); };
  size_t li = 0;
  for (int l = 0; l <= LE; ++l) {
    const BlobLayer& L = Ls[li++];
    if (l >= 1) sc[SW_EMB + l] = pow2_scale(amax(L));
  }
  li++;                                           // node encoder layer 1 (FP32)
  sc[SW_NE2] = pow2_scale(amax(Ls[li++]));
  sc[SW_EE1] = pow2_scale(amax(Ls[li++]));
  sc[SW_EE2] = pow2_scale(amax(Ls[li++]));
  for (int k = 0; k < S; ++k)
    for (int j = 0; j < 4; ++j) sc[SW_STEP + 4 * k + j] = pow2_scale(amax(Ls[li++]));
  sc[SW_CLS1] = pow2_scale(amax(Ls[li++]));
  // the INT8 set: max|W| / 127 for the same layers (1 for an all-zero layer)
  for (int i = 0; i < 256; ++i) ctx->i8_wscale[i] = 1.0;
  li = 0;
  auto i8 = [&](int slot, const BlobLayer& L) {
    const double m = amax(L);
    ctx->i8_wscale[slot] = m > 0.0 ? m / 127.0 : 1.0;
  };
  for (int l = 0; l <= LE; ++l) {
    const BlobLayer& L = Ls[li++];
    if (l >= 1) i8(SW_EMB + l, L);
  }
  li++;
  i8(SW_NE2, Ls[li++]);
  i8(SW_EE1, Ls[li++]);
  i8(SW_EE2, Ls[li++]);
  for (int k = 0; k < S; ++k)
    for (int j = 0; j < 4; ++j) i8(SW_STEP + 4 * k + j, Ls[li++]);
  i8(SW_CLS1, Ls[li++]);
  for (int i = 0; i < 256; ++i) sc[SC_I8 + i] = (float)ctx->i8_wscale[i];
}

thread_local std::string g_last_error;

void note_error(const char* what, hipError_t e) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

int set_kernel_attributes() {
  static int done = -1;
  if (done >= 0) return done;
  // dynamic LDS limit for every kernel that stages weights or candidates; kept
  // below the 160 KiB per workgroup so that static LDS still fits beside it
  size_t max_lds = 150 * 1024;
  done = embed_attributes(max_lds) | gnn_attributes(max_lds) | graph_attributes(max_lds) |
         radius_attributes(max_lds) | prefilter_attributes(max_lds) | train_attributes(max_lds) |
         triplet_attributes(max_lds);
  return done;
}

static const char* kStageNames[] = {"init",      "validate",   "bucket",      "embed",       "radius_count",
                                     "scan",      "radius_emit", "prefilter",  "csc",         "node_encode",
                                     "edge_encode", "segsum",    "node_step",   "edge_step",   "edge_step_final",
                                     "compact",   "union_find", "triplets",    "triplet_score", "tracks"};
constexpr int kNumStages = sizeof(kStageNames) / sizeof(kStageNames[0]);

// Record a pair of HIP events around one stage on the stage's stream.
struct StageTimer {
  etx_ctx* ctx;
  hipStream_t s;
  int idx = -1;
  StageTimer(const RunArgs& a, int stage) : ctx(const_cast<etx_ctx*>(a.ctx)), s(a.stream) {
    if (!ctx->profile || a.untimed || !((ctx->profile_mask >> stage) & 1)) return;
    if (ctx->n_marks == ctx->marks.size()) {
      etx_ctx::Mark m{stage, nullptr, nullptr};
      if (hipEventCreate(&m.start) != hipSuccess) return;
      if (hipEventCreate(&m.end) != hipSuccess) {
        (void)hipEventDestroy(m.start);
        return;
      }
      ctx->marks.push_back(m);
    }
    idx = (int)ctx->n_marks++;
    ctx->marks[idx].stage = stage;
    (void)hipEventRecord(ctx->marks[idx].start, s);   // a failed record shows up when the marks are read
  }
  ~StageTimer() {
    if (idx >= 0) (void)hipEventRecord(ctx->marks[idx].end, s);
  }
};

// The stage sequence of one batch.
static hipError_t enqueue_pipeline(const RunArgs& a) {
  hipError_t err;
#define STEP(stage, x)                         \
  do {                                         \
    StageTimer timer_(a, stage);               \
    if ((err = (x)) != hipSuccess) return err; \
  } while (0)
  const etx_config& c = a.ctx->cfg;
  STEP(0, launch_init_status(a));
  STEP(1, launch_validate(a));
  STEP(2, launch_bucket(a));
  STEP(3, launch_embed(a));
  const bool pf = c.prefilter != 0;
  if (a.ctx->radius_single) {
    STEP(4, launch_radius(a, 2, pf));
    STEP(5, launch_scan_counts(a, pf));
    STEP(6, launch_slots_copy(a, pf));
  } else {
    STEP(4, launch_radius(a, 0, pf));
    STEP(5, launch_scan_counts(a, pf));
    STEP(6, launch_radius(a, 1, pf));
  }
  if (pf) {
    // learned prefilter: keep flags on the candidates, then the surviving
    // edges become the graph of the rest of the path
    STEP(7, launch_prefilter_infer(a));
    STEP(7, launch_prefilter_band(a));
    STEP(7, launch_prefilter_count(a));
    STEP(7, launch_scan_counts(a, false));
    STEP(7, launch_prefilter_compact(a));
  }
  STEP(8, launch_csc(a));
  STEP(9, launch_node_encode(a));
  STEP(10, launch_edge_encode(a));
  for (int k = 0; k < c.gnn_steps; ++k) {
    STEP(11, launch_segsum(a, k));
    STEP(12, launch_node_step(a, k));
    STEP(k + 1 == c.gnn_steps ? 14 : 13, launch_edge_step(a, k, k + 1 == c.gnn_steps));
  }
  STEP(15, launch_compact(a));
  STEP(16, launch_union_find(a));
#undef STEP
  return hipSuccess;
}

static etx_status check_run_args(const etx_ctx* ctx, const etx_hits* hits, const etx_out* out, void* ws,
                                 size_t ws_bytes, WsLayout* L) {
  if (!ctx || !hits || !out) return ETX_ERR_INVALID_ARG;
  if (hits->n_events < 0 || hits->n_hits < 0 || hits->n_hits >= 0x7fffffffLL) return ETX_ERR_INVALID_ARG;
  if (!hits->hit_off) return ETX_ERR_INVALID_ARG;
  if (hits->n_hits > 0 && (!hits->x || !hits->y || !hits->z || !hits->plane)) return ETX_ERR_INVALID_ARG;
  if (out->edge_capacity < 0 || !out->edge_off || !out->status) return ETX_ERR_INVALID_ARG;
  if (hits->n_hits > 0 && !out->labels) return ETX_ERR_INVALID_ARG;
  if (out->edge_capacity > 0 && (!out->src || !out->dst || !out->score)) return ETX_ERR_INVALID_ARG;
  if (out->edge_capacity >= 0x7fffffffLL) return ETX_ERR_UNSUPPORTED;
  *L = ws_layout(ctx, hits->n_events, hits->n_hits, out->edge_capacity);
  if (!ws || ws_bytes < L->total || (reinterpret_cast<uintptr_t>(ws) & 255)) return ETX_ERR_INVALID_ARG;
  return ETX_OK;
}

// Device scratch of the no-allocation entry point: one array per device (each
// GPU the library runs on holds its own copy until the process ends), used as
// the workspace of etx_run_noalloc.  Host code never passes `scratch` itself
// (in host code it names a host-side stand-in); it passes the device address
// that hipGetSymbolAddress returned for the device, resolved once per device
// at context creation with that device current.
static __device__ __align__(256) char scratch[ETX_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static etx_status scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return ETX_ERR_UNSUPPORTED;
  if (g_scratch_ptr[device]) return ETX_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    note_error("hipGetSymbolAddress(scratch)", e);
    return ETX_ERR_HIP;
  }
  g_scratch_ptr[device] = ptr;
  return ETX_OK;
}

static void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

size_t blob_floats_of(const etx_config& c) { return blob_floats(c); }

etx_status check_run(const etx_ctx* ctx, const etx_hits* hits, const etx_out* out, void* ws, size_t ws_bytes,
                     WsLayout* L) {
  return check_run_args(ctx, hits, out, ws, ws_bytes, L);
}

// Replace the context's weights by a new payload (the blob's floats after its
// header): every segment set and the weight scales are rebuilt, calibrated
// activation scales are dropped (they belong to the old weights).
etx_status rebuild_weights(etx_ctx* ctx, const float* payload) {
  std::vector<char> blob = ctx->blob;
  std::memcpy(blob.data() + 32, payload, sizeof(float) * blob_floats(ctx->cfg));
  std::vector<float> pl;
  std::vector<BlobLayer> layers;
  if (!parse_blob(ctx->cfg, blob.data(), blob.size(), pl, layers)) return ETX_ERR_WEIGHTS;
  clear_graphs(ctx);
  for (int p = 0; p < kNumSegs; ++p)
    if (ctx->seg_base[p]) {
      (void)hipFree(ctx->seg_base[p]);
      ctx->seg_base[p] = nullptr;
    }
  weight_scales(ctx, layers);
  etx_status st = ETX_OK;
  for (int p = 0; p < kNumSegs && st == ETX_OK; ++p) st = build_segments(ctx, layers, p);
  if (st != ETX_OK) return st;
  if (hipMemcpy(ctx->dev_scales, ctx->host_scales, sizeof(float) * N_SCALES, hipMemcpyHostToDevice) != hipSuccess)
    return ETX_ERR_HIP;
  ctx->blob = blob;
  ctx->calibrated = false;
  return ETX_OK;
}

}  // namespace etx

using namespace etx;

extern "C" {

const char* etx_last_error(void) { return g_last_error.c_str(); }

const char* etx_status_str(etx_status s) {
  switch (s) {
    case ETX_OK: return "ok";
    case ETX_ERR_INVALID_ARG: return "invalid argument";
    case ETX_ERR_CAPACITY: return "edge capacity exceeded";
    case ETX_ERR_INPUT: return "invalid input hits";
    case ETX_ERR_WEIGHTS: return "weight blob does not match the configuration";
    case ETX_ERR_UNSUPPORTED: return "unsupported size or configuration";
    case ETX_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

etx_status etx_weight_blob_size(const etx_config* cfg, size_t* nbytes) {
  etx_status st = check_config(cfg);
  if (st != ETX_OK) return st;
  if (!nbytes) return ETX_ERR_INVALID_ARG;
  *nbytes = 32 + sizeof(float) * blob_floats(*cfg);
  return ETX_OK;
}

etx_status etx_create(const etx_config* cfg, const void* weights, size_t nbytes, int device, etx_ctx** out) {
  if (!out) return ETX_ERR_INVALID_ARG;
  *out = nullptr;
  etx_status st = check_config(cfg);
  if (st != ETX_OK) return st;
  if (!weights) return ETX_ERR_INVALID_ARG;
  std::vector<float> payload;
  std::vector<BlobLayer> layers;
  if (!parse_blob(*cfg, weights, nbytes, payload, layers)) return ETX_ERR_WEIGHTS;
  int ndev = 0;
  hipError_t he = hipGetDeviceCount(&ndev);
  if (he != hipSuccess) {
    note_error("hipGetDeviceCount", he);
    return ETX_ERR_HIP;
  }
  if (device < 0 || device >= ndev) return ETX_ERR_INVALID_ARG;
  if ((he = hipSetDevice(device)) != hipSuccess) {
    note_error("hipSetDevice", he);
    return ETX_ERR_HIP;
  }
  if (set_kernel_attributes() != 0) {
    g_last_error = "hipFuncSetAttribute(MaxDynamicSharedMemorySize) failed";
    return ETX_ERR_HIP;
  }
  if ((st = scratch_init(device)) != ETX_OK) return st;
  etx_ctx* ctx = new etx_ctx();
  ctx->cfg = *cfg;
  ctx->device = device;
  ctx->blob.assign(static_cast<const char*>(weights), static_cast<const char*>(weights) + nbytes);
  if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    delete ctx;
    return ETX_ERR_HIP;
  }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
      delete ctx;
      return ETX_ERR_HIP;
    }
    ctx->arch = prop.gcnArchName;
    const size_t colon = ctx->arch.find(':');
    if (colon != std::string::npos) ctx->arch.resize(colon);
  }
  weight_scales(ctx, layers);
  st = ETX_OK;
  for (int p = 0; p < kNumSegs && st == ETX_OK; ++p) st = build_segments(ctx, layers, p);
  if (st == ETX_OK && hipMalloc(&ctx->dev_scales, sizeof(float) * N_SCALES) != hipSuccess) st = ETX_ERR_HIP;
  if (st == ETX_OK && hipMemcpy(ctx->dev_scales, ctx->host_scales, sizeof(float) * N_SCALES, hipMemcpyHostToDevice) != hipSuccess)
    st = ETX_ERR_HIP;
  if (st == ETX_OK && hipMalloc(&ctx->dev_pf, sizeof(float) * 3 * ETX_PF_NPARAM) != hipSuccess) st = ETX_ERR_HIP;
  if (st == ETX_OK && hipMemset(ctx->dev_pf, 0, sizeof(float) * 3 * ETX_PF_NPARAM) != hipSuccess) st = ETX_ERR_HIP;
  if (st != ETX_OK) {
    etx_destroy(ctx);
    return st;
  }
  // a tuning table named by the environment (a missing or unreadable file is no error: no entries)
  if (const char* table = std::getenv("ETX_TUNING_TABLE")) (void)etx_tuning_load(ctx, table);
  *out = ctx;
  return ETX_OK;
}

etx_status etx_destroy(etx_ctx* ctx) {
  if (!ctx) return ETX_ERR_INVALID_ARG;
  // teardown is best effort: a failing release cannot be acted on here
  (void)hipSetDevice(ctx->device);
  clear_graphs(ctx);
  for (auto& m : ctx->marks) {
    (void)hipEventDestroy(m.start);
    (void)hipEventDestroy(m.end);
  }
  for (int p = 0; p < kNumSegs; ++p)
    if (ctx->seg_base[p]) (void)hipFree(ctx->seg_base[p]);
  if (ctx->dev_scales) (void)hipFree(ctx->dev_scales);
  if (ctx->dev_pf) (void)hipFree(ctx->dev_pf);
  if (ctx->dev_train) (void)hipFree(ctx->dev_train);
  if (ctx->dev_tri) (void)hipFree(ctx->dev_tri);
  if (ctx->dev_tri_train) (void)hipFree(ctx->dev_tri_train);
  delete ctx;
  return ETX_OK;
}

etx_status etx_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                              size_t* bytes) {
  if (!ctx || !bytes || n_events < 0 || n_hits < 0 || edge_capacity < 0) return ETX_ERR_INVALID_ARG;
  *bytes = ws_layout(ctx, n_events, n_hits, edge_capacity).total;
  return ETX_OK;
}

etx_status etx_workspace_view(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                              int32_t which, size_t* offset, size_t* bytes) {
  if (!ctx || !offset || !bytes || n_events < 0 || n_hits < 0 || edge_capacity < 0) return ETX_ERR_INVALID_ARG;
  WsLayout L = ws_layout(ctx, n_events, n_hits, edge_capacity);
  const int64_t H = ctx->cfg.gnn_hidden;
  switch (which) {
    case ETX_VIEW_EMBEDDING: *offset = L.emb; *bytes = sizeof(float) * n_hits * kDpad; break;
    case ETX_VIEW_BUCKET: *offset = L.bucket; *bytes = sizeof(int32_t) * n_hits; break;
    case ETX_VIEW_PLANE_OFF: *offset = L.plane_off; *bytes = sizeof(int32_t) * n_events * (ctx->cfg.n_planes + 1); break;
    case ETX_VIEW_ROW_PTR: *offset = L.row_ptr; *bytes = sizeof(int64_t) * (n_hits + 1); break;
    case ETX_VIEW_COL_PTR: *offset = L.col_ptr; *bytes = sizeof(int64_t) * (n_hits + 1); break;
    case ETX_VIEW_CSC_EDGE: *offset = L.csc; *bytes = sizeof(int32_t) * edge_capacity; break;
    case ETX_VIEW_NODE_H: *offset = L.h; *bytes = sizeof(float) * n_hits * H; break;
    case ETX_VIEW_KEPT_EDGE: *offset = L.kept; *bytes = sizeof(int32_t) * edge_capacity; break;
    case ETX_VIEW_KEPT_COUNT: *offset = L.kept_cnt; *bytes = sizeof(int32_t) * n_events; break;
    case ETX_VIEW_CALIB: *offset = L.calib; *bytes = sizeof(float) * ETX_N_CALIB; break;
    case ETX_VIEW_PF_KEEP: *offset = L.pf_keep; *bytes = edge_capacity; break;
    case ETX_VIEW_PF_GRAD: *offset = L.pf_grad; *bytes = sizeof(float) * (ETX_PF_NPARAM + 1); break;
    case ETX_VIEW_PF_PROB: *offset = L.pf_prob; *bytes = sizeof(float) * edge_capacity; break;
    case ETX_VIEW_PF_FALLBACK: *offset = L.pf_fallback; *bytes = sizeof(int32_t) * n_events; break;
    case ETX_VIEW_PF_FEAT:
      if (!ctx->pf_features) return ETX_ERR_INVALID_ARG;
      *offset = L.pf_feat;
      *bytes = sizeof(float) * 8 * edge_capacity;
      break;
    default: return ETX_ERR_INVALID_ARG;
  }
  return ETX_OK;
}

etx_status etx_set_option(etx_ctx* ctx, int32_t key, int64_t value) {
  if (!ctx) return ETX_ERR_INVALID_ARG;
  switch (key) {
    case ETX_OPT_USE_GRAPH:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->use_graph = (int)value;
      break;
    case ETX_OPT_EDGE_WG_PER_CU:
      if (value < 1 || value > 8) return ETX_ERR_INVALID_ARG;
      ctx->edge_wg_per_cu = (int)value;
      break;
    case ETX_OPT_NODE_WG_PER_CU:
      if (value < 1 || value > 8) return ETX_ERR_INVALID_ARG;
      ctx->node_wg_per_cu = (int)value;
      break;
    case ETX_OPT_RADIUS_LDS:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->radius_lds = (int)value;
      break;
    case ETX_OPT_SEGSUM_UNROLL:
      if (value != 1 && value != 2 && value != 4 && value != 8) return ETX_ERR_INVALID_ARG;
      ctx->segsum_unroll = (int)value;
      break;
    case ETX_OPT_PROFILE:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->profile = (int)value;
      return ETX_OK;
    case ETX_OPT_EDGE_PIPELINE:
      if (value < 0 || value > 2) return ETX_ERR_INVALID_ARG;
      ctx->edge_pipeline = (int)value;
      break;
    case ETX_OPT_EDGE_WG_SIZE:
      if (value != 256 && value != 512) return ETX_ERR_INVALID_ARG;
      ctx->edge_threads = (int)value;
      break;
    case ETX_OPT_EDGE_WREG:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->edge_wreg = (int)value;
      break;
    case ETX_OPT_EMBED_PRECISION:
      if (value < -1 || value > ETX_INT8) return ETX_ERR_INVALID_ARG;
      ctx->emb_precision = (int)value;
      break;
    case ETX_OPT_OUTSUM_LDS:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->outsum_lds = (int)value;
      break;
    case ETX_OPT_F32_SPLIT:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->f32_split = (int)value;
      break;
    case ETX_OPT_RADIUS_SINGLE_PASS:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->radius_single = (int)value;
      break;
    case ETX_OPT_RADIUS_SORT_MIN:
      if (value < 0 || value > ETX_MAX_EVENT_HITS) return ETX_ERR_INVALID_ARG;
      ctx->radius_sort_min = (int)value;
      break;
    case ETX_OPT_FUSE_MESSAGES:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->fuse_messages = (int)value;
      break;
    case ETX_OPT_RADIUS_FAST:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->radius_fast = (int)value;
      break;
    case ETX_OPT_RADIUS_SPLIT:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->radius_split = (int)value;
      break;
    case ETX_OPT_XCD_MAP:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->xcd_map = (int)value;
      break;
    case ETX_OPT_EDGE_PRODUCTS:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->edge_products = (int)value;
      break;
    case ETX_OPT_CSC_PLACE:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->csc_place = (int)value;
      break;
    case ETX_OPT_COMPACT_STATE:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->compact_state = (int)value;
      break;
    case ETX_OPT_PF_FEATURES:
      if (value != 0 && value != 1) return ETX_ERR_INVALID_ARG;
      ctx->pf_features = (int)value;
      break;
    case ETX_OPT_PROFILE_STAGES:
      if (value <= 0 || value >= (int64_t(1) << kNumStages)) return ETX_ERR_INVALID_ARG;
      ctx->profile_mask = value;
      return ETX_OK;
    default: return ETX_ERR_INVALID_ARG;
  }
  if (key != ETX_OPT_USE_GRAPH) clear_graphs(ctx);
  return ETX_OK;
}

const char* etx_stage_name(int32_t stage) {
  return (stage >= 0 && stage < kNumStages) ? kStageNames[stage] : "";
}

etx_status etx_profile_read(etx_ctx* ctx, int32_t n_stages, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches || n_stages < 0) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  for (size_t i = 0; i < ctx->n_marks; ++i) {
    const etx_ctx::Mark& m = ctx->marks[i];
    if (hipEventSynchronize(m.end) != hipSuccess) return ETX_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.start, m.end) != hipSuccess) return ETX_ERR_HIP;
    ctx->stage_ms[m.stage] += ms;
    ctx->stage_launches[m.stage] += 1;
  }
  ctx->n_marks = 0;
  for (int i = 0; i < n_stages; ++i) {
    total_ms[i] = i < kNumStages ? ctx->stage_ms[i] : 0.0;
    launches[i] = i < kNumStages ? ctx->stage_launches[i] : 0;
  }
  return ETX_OK;
}

etx_status etx_profile_reset(etx_ctx* ctx) {
  if (!ctx) return ETX_ERR_INVALID_ARG;
  ctx->n_marks = 0;
  for (int i = 0; i < 32; ++i) {
    ctx->stage_ms[i] = 0;
    ctx->stage_launches[i] = 0;
  }
  return ETX_OK;
}

etx_status etx_get_option(const etx_ctx* ctx, int32_t key, int64_t* value) {
  if (!ctx || !value) return ETX_ERR_INVALID_ARG;
  switch (key) {
    case ETX_OPT_USE_GRAPH: *value = ctx->use_graph; break;
    case ETX_OPT_EDGE_WG_PER_CU: *value = ctx->edge_wg_per_cu; break;
    case ETX_OPT_NODE_WG_PER_CU: *value = ctx->node_wg_per_cu; break;
    case ETX_OPT_RADIUS_LDS: *value = ctx->radius_lds; break;
    case ETX_OPT_SEGSUM_UNROLL: *value = ctx->segsum_unroll; break;
    case ETX_OPT_EDGE_PIPELINE: *value = ctx->edge_pipeline; break;
    case ETX_OPT_EDGE_WG_SIZE: *value = ctx->edge_threads; break;
    case ETX_OPT_EDGE_WREG: *value = ctx->edge_wreg; break;
    case ETX_OPT_EMBED_PRECISION: *value = ctx->emb_precision; break;
    case ETX_OPT_OUTSUM_LDS: *value = ctx->outsum_lds; break;
    case ETX_OPT_F32_SPLIT: *value = ctx->f32_split; break;
    case ETX_OPT_RADIUS_SINGLE_PASS: *value = ctx->radius_single; break;
    case ETX_OPT_RADIUS_SORT_MIN: *value = ctx->radius_sort_min; break;
    case ETX_OPT_FUSE_MESSAGES: *value = ctx->fuse_messages; break;
    case ETX_OPT_RADIUS_FAST: *value = ctx->radius_fast; break;
    case ETX_OPT_RADIUS_SPLIT: *value = ctx->radius_split; break;
    case ETX_OPT_XCD_MAP: *value = ctx->xcd_map; break;
    case ETX_OPT_EDGE_PRODUCTS: *value = ctx->edge_products; break;
    case ETX_OPT_CSC_PLACE: *value = ctx->csc_place; break;
    case ETX_OPT_COMPACT_STATE: *value = ctx->compact_state; break;
    case ETX_OPT_PROFILE: *value = ctx->profile; break;
    case ETX_OPT_PROFILE_STAGES: *value = ctx->profile_mask; break;
    case ETX_OPT_PF_FEATURES: *value = ctx->pf_features; break;
    default: return ETX_ERR_INVALID_ARG;
  }
  return ETX_OK;
}

// Kernel precision of a run: the low-precision GEMM modes keep node and edge
// state in FP32 unless the compact form is asked for.
static int kernel_precision(const etx_ctx* ctx) {
  const int p = ctx->cfg.precision;
  if (p == ETX_INT8) return kI8Master;          // INT8 keeps the state in FP32 only
  if (p == ETX_FP32 || ctx->compact_state) return p;
  return p == ETX_BF16 ? kBf16Master : kFp8Master;
}

etx_status etx_run(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes, etx_stream stream) {
  WsLayout L;
  etx_status st = check_run_args(ctx, hits, out, ws, ws_bytes, &L);
  if (st != ETX_OK) return st;
  auto scaled = [](int p) { return p == ETX_FP8_E4M3 || p == ETX_INT8; };
  if ((scaled(ctx->cfg.precision) || scaled(ctx->emb_precision)) && !ctx->calibrated) return ETX_ERR_INVALID_ARG;
  if (ctx->cfg.prefilter && !ctx->pf_set) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  if (!ctx->tuning.empty()) {
    // the tuning table's schedule for this batch's shape bucket, when it has one
    const std::string key = tuning_key(ctx, hits->n_events, hits->n_hits);
    if (key != ctx->tuning_applied) {
      auto it = ctx->tuning.find(key);
      if (it != ctx->tuning.end()) {
        for (const auto& kv : it->second)
          if ((st = etx_set_option(ctx, kv.first, kv.second)) != ETX_OK) return st;
        ctx->tuning_applied = key;
      }
    }
  }
  RunArgs a{ctx, *hits, *out, L, static_cast<char*>(ws), static_cast<hipStream_t>(stream), false,
            kernel_precision(ctx)};
  if (!ctx->use_graph || stream == nullptr) {
    hipError_t e = enqueue_pipeline(a);
    if (e != hipSuccess) {
      note_error("etx_run launch", e);
      return ETX_ERR_HIP;
    }
    return ETX_OK;
  }
  GraphKey key{};
  const void* ps[16] = {hits->hit_off, hits->x, hits->y, hits->z, hits->plane, out->src, out->dst, out->score,
                        out->edge_off, out->labels, out->status, ws, nullptr, nullptr, nullptr, nullptr};
  std::memcpy(key.p, ps, sizeof(ps));
  key.n[0] = hits->n_events;
  key.n[1] = hits->n_hits;
  key.n[2] = out->edge_capacity;
  key.n[3] = ((int64_t)ctx->cfg.precision << 1) | ctx->cfg.prefilter;
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    hipStream_t s = a.stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return ETX_ERR_HIP;
    const int prof = ctx->profile;
    ctx->profile = 0;
    hipError_t e1 = enqueue_pipeline(a);
    ctx->profile = prof;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e1 != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return ETX_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);   // the executable graph keeps what it needs
    if (e3 != hipSuccess) return ETX_ERR_HIP;
    it = ctx->graphs.emplace(key, ex).first;
  }
  return hipGraphLaunch(it->second, a.stream) == hipSuccess ? ETX_OK : ETX_ERR_HIP;
}

etx_status etx_run_noalloc(etx_ctx* ctx, const etx_hits* hits, etx_out* out, etx_stream stream) {
  if (!ctx || !hits || !out) return ETX_ERR_INVALID_ARG;
  if (hits->n_events < 0 || hits->n_hits < 0 || out->edge_capacity < 0) return ETX_ERR_INVALID_ARG;
  void* ptr = scratch_ptr(ctx->device);
  if (!ptr) return ETX_ERR_HIP;
  if (ws_layout(ctx, hits->n_events, hits->n_hits, out->edge_capacity).total > (size_t)ETX_SCRATCH_BYTES) {
    g_last_error = "etx_run_noalloc: the batch needs more workspace than the static scratch holds";
    return ETX_ERR_UNSUPPORTED;
  }
  WsLayout L;
  etx_status st = check_run_args(ctx, hits, out, ptr, (size_t)ETX_SCRATCH_BYTES, &L);
  if (st != ETX_OK) return st;
  auto scaled = [](int p) { return p == ETX_FP8_E4M3 || p == ETX_INT8; };
  if ((scaled(ctx->cfg.precision) || scaled(ctx->emb_precision)) && !ctx->calibrated) return ETX_ERR_INVALID_ARG;
  if (ctx->cfg.prefilter && !ctx->pf_set) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  RunArgs a{ctx, *hits, *out, L, static_cast<char*>(ptr), static_cast<hipStream_t>(stream), false,
            kernel_precision(ctx)};
  a.untimed = true;
  const hipError_t e = enqueue_pipeline(a);
  if (e != hipSuccess) {
    note_error("etx_run_noalloc launch", e);
    return ETX_ERR_HIP;
  }
  return ETX_OK;
}

etx_status etx_calibrate(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes,
                         etx_stream stream) {
  WsLayout L;
  etx_status st = check_run_args(ctx, hits, out, ws, ws_bytes, &L);
  if (st != ETX_OK) return st;
  if (ctx->cfg.prefilter) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  RunArgs a{ctx, *hits, *out, L, static_cast<char*>(ws), static_cast<hipStream_t>(stream), true, ETX_FP32};
  hipError_t e = enqueue_pipeline(a);
  if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
  int64_t status[2] = {0, 0};
  float amax[ETX_N_CALIB];
  if (e == hipSuccess) e = hipMemcpy(status, out->status, sizeof(status), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(amax, a.ws + L.calib, sizeof(amax), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    note_error("etx_calibrate", e);
    return ETX_ERR_HIP;
  }
  if (status[0] != ETX_OK) return (etx_status)status[0];
  for (int i = 0; i < ETX_N_CALIB; ++i) {
    ctx->host_scales[i] = pow2_scale(amax[i]);
    ctx->host_scales[SC_I8 + i] = amax[i] > 0.f ? (float)((double)amax[i] / 127.0) : 1.0f;
  }
  if ((e = hipMemcpy(ctx->dev_scales, ctx->host_scales, sizeof(float) * N_SCALES, hipMemcpyHostToDevice)) !=
      hipSuccess) {
    note_error("etx_calibrate upload", e);
    return ETX_ERR_HIP;
  }
  ctx->calibrated = true;
  clear_graphs(ctx);
  return ETX_OK;
}

etx_status etx_set_precision(etx_ctx* ctx, int32_t precision) {
  if (!ctx || precision < ETX_FP32 || precision > ETX_INT8) return ETX_ERR_INVALID_ARG;
  ctx->cfg.precision = precision;
  clear_graphs(ctx);
  return ETX_OK;
}

etx_status etx_get_scales(const etx_ctx* ctx, float* scales, int32_t n) {
  if (!ctx || !scales || n < 0 || n > N_SCALES) return ETX_ERR_INVALID_ARG;
  std::memcpy(scales, ctx->host_scales, sizeof(float) * n);
  return ETX_OK;
}

etx_status etx_quantize(int32_t precision, const float* in, float* out, int64_t n, float scale, etx_stream stream) {
  if (precision < ETX_FP32 || precision > ETX_INT8 || n < 0 || (n > 0 && (!in || !out)) || !(scale > 0))
    return ETX_ERR_INVALID_ARG;
  if (n == 0) return ETX_OK;
  hipError_t e = launch_quantize(precision, in, out, n, scale, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    note_error("etx_quantize", e);
    return ETX_ERR_HIP;
  }
  return ETX_OK;
}

// ---------------------------------------------------------------------------
// triplet stage
// ---------------------------------------------------------------------------

etx_status etx_triplet_set(etx_ctx* ctx, const float* params, int64_t n) {
  if (!ctx || !params) return ETX_ERR_INVALID_ARG;
  const int H = ctx->cfg.gnn_hidden;
  if (n != ETX_TRIPLET_NPARAM(H)) return ETX_ERR_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return ETX_ERR_WEIGHTS;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  const int hf = tri_head_floats(H);
  std::vector<float> dev(2 * (size_t)hf);
  const int64_t per = ETX_TRIPLET_NPARAM(H) / 2;
  tri_prepare_head(params, H, dev.data());
  tri_prepare_head(params + per, H, dev.data() + hf);
  hipError_t e = hipSuccess;
  if (!ctx->dev_tri) e = hipMalloc(&ctx->dev_tri, sizeof(float) * dev.size());
  if (e == hipSuccess) e = hipMemcpy(ctx->dev_tri, dev.data(), sizeof(float) * dev.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    note_error("etx_triplet_set", e);
    return ETX_ERR_HIP;
  }
  ctx->tri_host.assign(params, params + n);
  return ETX_OK;
}

etx_status etx_triplet_get(const etx_ctx* ctx, float* params, int64_t n) {
  if (!ctx || !params || ctx->tri_host.empty() || n != (int64_t)ctx->tri_host.size()) return ETX_ERR_INVALID_ARG;
  std::memcpy(params, ctx->tri_host.data(), sizeof(float) * n);
  return ETX_OK;
}

etx_status etx_tracks_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                                     int64_t triplet_capacity, int64_t track_capacity, size_t* bytes) {
  if (!ctx || !bytes || n_events < 0 || n_hits < 0 || edge_capacity < 0 || triplet_capacity < 0 ||
      track_capacity < 0)
    return ETX_ERR_INVALID_ARG;
  *bytes = ws_layout(ctx, n_events, n_hits, edge_capacity).total +
           tri_layout(n_events, n_hits, edge_capacity, triplet_capacity, track_capacity).total;
  return ETX_OK;
}

etx_status etx_run_tracks(etx_ctx* ctx, const etx_hits* hits, etx_out* out, etx_tracks* tracks, void* ws,
                          size_t ws_bytes, etx_stream stream) {
  if (!tracks) return ETX_ERR_INVALID_ARG;
  WsLayout L;
  etx_status st = check_run_args(ctx, hits, out, ws, ws_bytes, &L);
  if (st != ETX_OK) return st;
  const etx_tracks& T = *tracks;
  if (T.triplet_capacity < 0 || T.track_capacity < 0 || T.hit_capacity < 0 || !T.status || !T.art_off ||
      !T.elb_off || !T.event_track_off || !T.track_off)
    return ETX_ERR_INVALID_ARG;
  if (T.triplet_capacity > 0 && (!T.tri_a || !T.tri_b || !T.tri_score || !T.tri_kind)) return ETX_ERR_INVALID_ARG;
  if (T.hit_capacity > 0 && !T.track_hits) return ETX_ERR_INVALID_ARG;
  if (T.triplet_capacity >= 0x7fffffffLL || T.track_capacity >= 0x7fffffffLL) return ETX_ERR_UNSUPPORTED;
  const TriLayout TL = tri_layout(hits->n_events, hits->n_hits, out->edge_capacity, T.triplet_capacity,
                                  T.track_capacity);
  if (ws_bytes < L.total + TL.total) return ETX_ERR_INVALID_ARG;
  if (ctx->tri_host.empty()) return ETX_ERR_INVALID_ARG;
  const int prec = kernel_precision(ctx);
  if (prec == ETX_FP8_E4M3) return ETX_ERR_UNSUPPORTED;   // compact FP8 state: e_S as FP8 codes
  auto scaled = [](int p) { return p == ETX_FP8_E4M3 || p == ETX_INT8; };
  if ((scaled(ctx->cfg.precision) || scaled(ctx->emb_precision)) && !ctx->calibrated) return ETX_ERR_INVALID_ARG;
  if (ctx->cfg.prefilter && !ctx->pf_set) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  RunArgs a{ctx, *hits, *out, L, static_cast<char*>(ws), static_cast<hipStream_t>(stream), false, prec};
  a.keep_final_e = true;
  char* tws = static_cast<char*>(ws) + L.total;
  hipError_t e = enqueue_pipeline(a);
  for (int part = 0; part < 3 && e == hipSuccess; ++part) {
    StageTimer timer_(a, 17 + part);
    e = launch_triplet_stage(a, T, tws, TL, part);
  }
  if (e != hipSuccess) {
    note_error("etx_run_tracks launch", e);
    return ETX_ERR_HIP;
  }
  return ETX_OK;
}

etx_status etx_prefilter_set(etx_ctx* ctx, const float* params, int64_t n) {
  if (!ctx || !params || n != ETX_PF_NPARAM) return ETX_ERR_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return ETX_ERR_WEIGHTS;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  std::vector<float> st(3 * ETX_PF_NPARAM, 0.f);
  std::memcpy(st.data(), params, sizeof(float) * ETX_PF_NPARAM);
  hipError_t e = hipMemcpy(ctx->dev_pf, st.data(), sizeof(float) * st.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    note_error("etx_prefilter_set", e);
    return ETX_ERR_HIP;
  }
  ctx->pf_set = true;
  clear_graphs(ctx);
  return ETX_OK;
}

etx_status etx_prefilter_get(const etx_ctx* ctx, float* params, int64_t n) {
  if (!ctx || !params || n != ETX_PF_NPARAM) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  hipError_t e = hipMemcpy(params, ctx->dev_pf, sizeof(float) * ETX_PF_NPARAM, hipMemcpyDeviceToHost);
  return e == hipSuccess ? ETX_OK : ETX_ERR_HIP;
}

etx_status etx_prefilter_state(etx_ctx* ctx, float* host_state, int64_t n, int32_t set) {
  if (!ctx || !host_state || n != 3 * ETX_PF_NPARAM || (set != 0 && set != 1)) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  hipError_t e = set ? hipMemcpy(ctx->dev_pf, host_state, sizeof(float) * n, hipMemcpyHostToDevice)
                     : hipMemcpy(host_state, ctx->dev_pf, sizeof(float) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    note_error("etx_prefilter_state", e);
    return ETX_ERR_HIP;
  }
  if (set) {
    ctx->pf_set = true;
    clear_graphs(ctx);
  }
  return ETX_OK;
}

// ---------------------------------------------------------------------------
// checkpoints: everything a context holds beyond its buffers
// ---------------------------------------------------------------------------

namespace {

struct SaveHeader {
  uint32_t magic, version, config_bytes, n_scales, n_pf, n_options;
  uint64_t blob_bytes;
  int32_t calibrated, pf_set;
  uint32_t n_tri;               // triplet classifier floats (0: none set)
  float pf_band_lo, pf_band_hi; // prefilter fallback band
  uint32_t reserved;
};
constexpr uint32_t kSaveMagic = 0x53585445;   // "ETXS"
constexpr uint32_t kSaveVersion = 2;
constexpr int kSavedOptions = 20;             // etx_option keys 0 .. 19

size_t save_bytes(const etx_ctx* ctx) {
  return sizeof(SaveHeader) + sizeof(etx_config) + sizeof(float) * (N_SCALES + 3 * ETX_PF_NPARAM) +
         sizeof(int64_t) * kSavedOptions + ctx->blob.size() + sizeof(float) * ctx->tri_host.size();
}

}  // namespace

etx_status etx_save(const etx_ctx* ctx, void* buf, size_t* nbytes) {
  if (!ctx || !nbytes) return ETX_ERR_INVALID_ARG;
  const size_t need = save_bytes(ctx);
  if (!buf) {
    *nbytes = need;
    return ETX_OK;
  }
  if (*nbytes < need) {
    *nbytes = need;
    return ETX_ERR_INVALID_ARG;
  }
  char* o = static_cast<char*>(buf);
  SaveHeader h{kSaveMagic, kSaveVersion, (uint32_t)sizeof(etx_config), (uint32_t)N_SCALES,
               (uint32_t)(3 * ETX_PF_NPARAM), (uint32_t)kSavedOptions, (uint64_t)ctx->blob.size(),
               ctx->calibrated ? 1 : 0, ctx->pf_set ? 1 : 0, (uint32_t)ctx->tri_host.size(), ctx->pf_band_lo,
               ctx->pf_band_hi, 0u};
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  std::memcpy(o, &ctx->cfg, sizeof(etx_config));
  o += sizeof(etx_config);
  std::memcpy(o, ctx->host_scales, sizeof(float) * N_SCALES);
  o += sizeof(float) * N_SCALES;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  hipError_t e = hipMemcpy(o, ctx->dev_pf, sizeof(float) * 3 * ETX_PF_NPARAM, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    note_error("etx_save", e);
    return ETX_ERR_HIP;
  }
  o += sizeof(float) * 3 * ETX_PF_NPARAM;
  for (int k = 0; k < kSavedOptions; ++k) {
    int64_t v = 0;
    etx_get_option(ctx, k, &v);
    std::memcpy(o, &v, sizeof v);
    o += sizeof v;
  }
  std::memcpy(o, ctx->blob.data(), ctx->blob.size());
  o += ctx->blob.size();
  if (!ctx->tri_host.empty()) std::memcpy(o, ctx->tri_host.data(), sizeof(float) * ctx->tri_host.size());
  *nbytes = need;
  return ETX_OK;
}

etx_status etx_load(const void* buf, size_t nbytes, int device, etx_ctx** out) {
  if (!buf || !out) return ETX_ERR_INVALID_ARG;
  *out = nullptr;
  SaveHeader h;
  if (nbytes < sizeof h) return ETX_ERR_INVALID_ARG;
  std::memcpy(&h, buf, sizeof h);
  if (h.magic != kSaveMagic || h.version != kSaveVersion || h.config_bytes != sizeof(etx_config) ||
      h.n_scales != N_SCALES || h.n_pf != 3 * ETX_PF_NPARAM || h.n_options != kSavedOptions)
    return ETX_ERR_INVALID_ARG;
  const size_t need = sizeof h + sizeof(etx_config) + sizeof(float) * (N_SCALES + 3 * ETX_PF_NPARAM) +
                      sizeof(int64_t) * kSavedOptions + h.blob_bytes + sizeof(float) * (size_t)h.n_tri;
  if (nbytes != need) return ETX_ERR_INVALID_ARG;
  const char* p = static_cast<const char*>(buf) + sizeof h;
  etx_config cfg;
  std::memcpy(&cfg, p, sizeof cfg);
  p += sizeof cfg;
  const char* scales = p;
  p += sizeof(float) * N_SCALES;
  const char* pf = p;
  p += sizeof(float) * 3 * ETX_PF_NPARAM;
  const char* opts = p;
  p += sizeof(int64_t) * kSavedOptions;
  const char* tri = p + h.blob_bytes;
  if (h.n_tri != 0 && h.n_tri != (uint32_t)ETX_TRIPLET_NPARAM(cfg.gnn_hidden)) return ETX_ERR_INVALID_ARG;
  etx_ctx* ctx = nullptr;
  etx_status st = etx_create(&cfg, p, (size_t)h.blob_bytes, device, &ctx);
  if (st != ETX_OK) return st;
  if (h.n_tri) {
    std::vector<float> tp(h.n_tri);
    std::memcpy(tp.data(), tri, sizeof(float) * h.n_tri);
    if ((st = etx_triplet_set(ctx, tp.data(), (int64_t)h.n_tri)) != ETX_OK) {
      etx_destroy(ctx);
      return st;
    }
  }
  if ((st = etx_prefilter_band(ctx, h.pf_band_lo, h.pf_band_hi)) != ETX_OK) {
    etx_destroy(ctx);
    return st;
  }
  std::memcpy(ctx->host_scales, scales, sizeof(float) * N_SCALES);
  ctx->calibrated = h.calibrated != 0;
  hipError_t e = hipMemcpy(ctx->dev_scales, ctx->host_scales, sizeof(float) * N_SCALES, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->dev_pf, pf, sizeof(float) * 3 * ETX_PF_NPARAM, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    note_error("etx_load", e);
    etx_destroy(ctx);
    return ETX_ERR_HIP;
  }
  ctx->pf_set = h.pf_set != 0;
  for (int k = 0; k < kSavedOptions; ++k) {
    int64_t v;
    std::memcpy(&v, opts + sizeof(int64_t) * k, sizeof v);
    if (k != ETX_OPT_PROFILE && (st = etx_set_option(ctx, k, v)) != ETX_OK) {
      etx_destroy(ctx);
      return st;
    }
  }
  *out = ctx;
  return ETX_OK;
}

etx_status etx_prefilter_train_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const uint8_t* edge_labels,
                                    float lr, float pos_weight, int64_t step, float* loss_dev, void* ws,
                                    size_t ws_bytes, etx_stream stream) {
  WsLayout L;
  etx_status st = check_run_args(ctx, hits, out, ws, ws_bytes, &L);
  if (st != ETX_OK) return st;
  if (!edge_labels || !(lr > 0) || !(pos_weight > 0) || step < 1 || !ctx->pf_set) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  RunArgs a{ctx, *hits, *out, L, static_cast<char*>(ws), static_cast<hipStream_t>(stream), false, ETX_FP32};
  hipError_t e;
#define STEP(x)                                   \
  do {                                            \
    if ((e = (x)) != hipSuccess) {                \
      note_error("etx_prefilter_train_step", e);  \
      return ETX_ERR_HIP;                         \
    }                                             \
  } while (0)
  // the candidate graph (unpruned) of the batch, then one optimiser step
  STEP(launch_init_status(a));
  STEP(launch_validate(a));
  STEP(launch_bucket(a));
  STEP(launch_embed(a));
  if (ctx->radius_single) {
    STEP(launch_radius(a, 2, false));
    STEP(launch_scan_counts(a, false));
    STEP(launch_slots_copy(a, false));
  } else {
    STEP(launch_radius(a, 0, false));
    STEP(launch_scan_counts(a, false));
    STEP(launch_radius(a, 1, false));
  }
  STEP(launch_prefilter_train(a, edge_labels, lr, pos_weight, step, loss_dev));
#undef STEP
  return ETX_OK;
}

etx_status etx_prefilter_config(etx_ctx* ctx, int32_t enabled, float tau) {
  if (!ctx || (enabled != 0 && enabled != 1) || !std::isfinite(tau)) return ETX_ERR_INVALID_ARG;
  ctx->cfg.prefilter = enabled;
  ctx->cfg.prefilter_tau = tau;
  clear_graphs(ctx);
  return ETX_OK;
}

etx_status etx_prefilter_band(etx_ctx* ctx, float lo, float hi) {
  if (!ctx || !(lo >= 0.f) || !(hi <= 1.f) || !(lo <= hi)) return ETX_ERR_INVALID_ARG;
  ctx->pf_band_lo = lo;
  ctx->pf_band_hi = hi;
  clear_graphs(ctx);
  return ETX_OK;
}

}  // extern "C"
