// Host side of in-library training: the training parameters in the context,
// the workspace layout of a training step, and the step sequences.
//
// The graph of a step is built by the inference stages (bucketing, radius
// graph, CSC permutation); the embedding step builds it in its own training
// embedding at the training radius (hard negatives, thesis ch. 8), the
// network step with the context's inference embedding (the rough graph).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <vector>

#include "internal.hpp"
#include "train.hpp"

namespace etx {

size_t blob_floats_of(const etx_config& c);
etx_status check_run(const etx_ctx* ctx, const etx_hits* hits, const etx_out* out, void* ws, size_t ws_bytes,
                     WsLayout* L);
etx_status rebuild_weights(etx_ctx* ctx, const float* payload);

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct TrainLayout {
  // embedding
  size_t cyl, emb_a[8], emb_yh[8], de, edz, edx[2], g_gen, g_rnd, g_edge, counts, counts2, hparts;
  // network
  size_t cart, y1n, hst, mo, mi, t1n, yh_n, rs_n, t1ee, est, t1e, cls, yh_e, rs_e, lab, dlogit, de_e, dz_e, da_e,
      dxs, dxd, dh, dz_n, da_n, dmo, dmi;
  // shared
  size_t part, grad, lpart, loss;
  size_t total;
};

TrainLayout train_layout(const etx_ctx* ctx, const WsLayout& L, int64_t n, int64_t E) {
  const etx_config& c = ctx->cfg;
  const int64_t H = c.gnn_hidden, S = c.gnn_steps, W = c.emb_hidden, D = c.emb_dim;
  TrainLayout T{};
  size_t o = L.total;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += a256(std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t f = sizeof(float);
  T.cyl = take(f * n * 3);
  for (int l = 0; l < c.emb_layers + 1 && l < 8; ++l) {
    const int64_t M = l < c.emb_layers ? W : D;
    T.emb_a[l] = take(f * n * M);
    T.emb_yh[l] = take(f * n * M);
  }
  T.de = take(f * n * kDpad);
  T.edz = take(f * n * std::max<int64_t>(W, H));
  T.edx[0] = take(f * n * std::max<int64_t>(W, 3 * H));
  T.edx[1] = take(f * n * std::max<int64_t>(W, 3 * H));
  T.g_gen = take(f * n * D);
  T.g_rnd = take(f * n * D);
  T.g_edge = take(f * E * D);
  T.counts = take(f * 2);
  T.counts2 = take(f * 2);
  T.hparts = take(f * 3 * kTrainLossBlocks);
  T.cart = take(f * n * 3);
  T.y1n = take(f * n * H);
  T.hst = take(f * (S + 1) * n * H);
  T.mo = take(f * S * n * H);
  T.mi = take(f * S * n * H);
  T.t1n = take(f * S * n * H);
  T.yh_n = take(f * (2 + 2 * S) * n * H);
  T.rs_n = take(f * (2 + 2 * S) * n);
  T.t1ee = take(f * E * H);
  T.est = take(f * (S + 1) * E * H);
  T.t1e = take(f * S * E * H);
  T.cls = take(f * E * H);
  T.yh_e = take(f * (3 + 2 * S) * E * H);
  T.rs_e = take(f * (3 + 2 * S) * E);
  T.lab = take(E);
  T.dlogit = take(f * E);
  T.de_e = take(f * E * H);
  T.dz_e = take(f * E * H);
  T.da_e = take(f * E * H);
  T.dxs = take(f * E * H);
  T.dxd = take(f * E * H);
  T.dh = take(f * n * H);
  T.dz_n = take(f * n * std::max<int64_t>(H, W));
  T.da_n = take(f * n * H);
  T.dmo = take(f * n * H);
  T.dmi = take(f * n * H);
  T.part = take(f * kTrainChunks * (std::max<int64_t>(3 * H, W) * std::max<int64_t>(H, W) + std::max<int64_t>(H, W)));
  T.grad = take(f * blob_floats_of(c));
  T.lpart = take(f * kTrainLossBlocks);
  T.loss = take(f * 4);
  T.total = o;
  return T;
}

// The triplet part of a network step's workspace (after the TrainLayout).
struct TripLayout {
  size_t ta, tb, kind, tscore, art_off, elb_off, tstatus, tri, lab, yh1, y1, rs1, yh2, y2, rs2, dlogit, dc, dz, da,
      dxa, dxb, tgrad, total;
  TriLayout TL;
};

TripLayout trip_layout(const etx_ctx* ctx, size_t base, int64_t n_events, int64_t n, int64_t E, int64_t tcap) {
  const int64_t H = ctx->cfg.gnn_hidden;
  TripLayout X{};
  size_t o = base;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += a256(std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t f = sizeof(float), T = (size_t)tcap;
  X.ta = take(4 * T);
  X.tb = take(4 * T);
  X.kind = take(T);
  X.tscore = take(f * T);
  X.art_off = take(8 * (size_t)(n_events + 1));
  X.elb_off = take(8 * (size_t)(n_events + 1));
  X.tstatus = take(8 * 4);
  X.TL = tri_layout(n_events, n, E, tcap, 0);
  X.tri = take(X.TL.total);
  X.lab = take(T);
  X.yh1 = take(f * T * H);
  X.y1 = take(f * T * H);
  X.rs1 = take(f * T);
  X.yh2 = take(f * T * H);
  X.y2 = take(f * T * H);
  X.rs2 = take(f * T);
  X.dlogit = take(f * T);
  X.dc = take(f * T * H);
  X.dz = take(f * T * H);
  X.da = take(f * T * H);
  X.dxa = take(f * T * H);
  X.dxb = take(f * T * H);
  X.tgrad = take(f * ETX_TRIPLET_NPARAM(H));
  X.total = o;
  return X;
}

// offsets (floats) of the parameter blocks in the blob payload
struct ParamMap {
  int64_t emb[8];           // embedding layer l
  int64_t ne1, ne2, ee1, ee2, nn1[16], nn2[16], en1[16], en2[16], cls1, cls2, gnn_begin, total;
};

ParamMap param_map(const etx_config& c) {
  ParamMap P{};
  int64_t o = 0;
  const int64_t W = c.emb_hidden, D = c.emb_dim, H = c.gnn_hidden;
  for (int l = 0; l <= c.emb_layers && l < 8; ++l) {
    const int64_t K = l == 0 ? 3 : W, M = l < c.emb_layers ? W : D;
    P.emb[l] = o;
    o += K * M + M;
  }
  P.gnn_begin = o;
  auto take = [&](int64_t K, int64_t M) {
    int64_t at = o;
    o += K * M + M;
    return at;
  };
  P.ne1 = take(3, H);
  P.ne2 = take(H, H);
  P.ee1 = take(2 * H, H);
  P.ee2 = take(H, H);
  for (int k = 0; k < c.gnn_steps; ++k) {
    P.nn1[k] = take(3 * H, H);
    P.nn2[k] = take(H, H);
    P.en1[k] = take(3 * H, H);
    P.en2[k] = take(H, H);
  }
  P.cls1 = take(H, H);
  P.cls2 = take(H, 1);
  P.total = o;
  return P;
}

TrainSeg seg(const float* base, const int32_t* idx, int width, int ld) { return TrainSeg{base, idx, width, ld}; }
TrainOut tout(float* base, int width, int ld, int add) { return TrainOut{base, width, ld, add}; }

}  // namespace
}  // namespace etx

using namespace etx;

#define F(off) reinterpret_cast<float*>(ws + (off))
#define HIPCHK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) {                    \
      note_error(what, e_);                    \
      return ETX_ERR_HIP;                      \
    }                                          \
  } while (0)

namespace etx {
void note_error(const char* what, hipError_t e);
}

extern "C" {

etx_status etx_train_begin(etx_ctx* ctx) {
  if (!ctx) return ETX_ERR_INVALID_ARG;
  const char* what = "etx_train_begin";
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  const size_t n = blob_floats_of(ctx->cfg);
  if (!ctx->dev_train) HIPCHK(hipMalloc(&ctx->dev_train, sizeof(float) * 3 * n));
  HIPCHK(hipMemcpy(ctx->dev_train, ctx->blob.data() + 32, sizeof(float) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(ctx->dev_train + n, 0, sizeof(float) * 2 * n));
  ctx->tri_train_fresh = true;
  return ETX_OK;
}

}  // extern "C"

namespace {

// the triplet classifiers' training state, (re)started from the context's
// triplet parameters after etx_train_begin
etx_status tri_train_state(etx_ctx* ctx) {
  const char* what = "triplet training state";
  if (!ctx->dev_train || ctx->tri_host.empty()) return ETX_ERR_INVALID_ARG;
  const size_t np = ctx->tri_host.size();
  if (!ctx->dev_tri_train) HIPCHK(hipMalloc(&ctx->dev_tri_train, sizeof(float) * 3 * np));
  if (ctx->tri_train_fresh) {
    HIPCHK(hipMemcpy(ctx->dev_tri_train, ctx->tri_host.data(), sizeof(float) * np, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(ctx->dev_tri_train + np, 0, sizeof(float) * 2 * np));
    ctx->tri_train_fresh = false;
  }
  return ETX_OK;
}

}  // namespace

extern "C" {

etx_status etx_train_triplet_params(etx_ctx* ctx, float* host, int64_t n, int32_t set) {
  if (!ctx || !host || (set != 0 && set != 1)) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  etx_status st = tri_train_state(ctx);
  if (st != ETX_OK) return st;
  const int64_t np = (int64_t)ctx->tri_host.size();
  if (n < 1 || n > 3 * np) return ETX_ERR_INVALID_ARG;
  const char* what = "etx_train_triplet_params";
  HIPCHK(set ? hipMemcpy(ctx->dev_tri_train, host, sizeof(float) * n, hipMemcpyHostToDevice)
             : hipMemcpy(host, ctx->dev_tri_train, sizeof(float) * n, hipMemcpyDeviceToHost));
  return ETX_OK;
}

etx_status etx_train_params(etx_ctx* ctx, float* host, int64_t n, int32_t set) {
  if (!ctx || !host || !ctx->dev_train) return ETX_ERR_INVALID_ARG;
  const int64_t nb = (int64_t)blob_floats_of(ctx->cfg);
  if (n < 1 || n > 3 * nb) return ETX_ERR_INVALID_ARG;
  const char* what = "etx_train_params";
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  HIPCHK(set ? hipMemcpy(ctx->dev_train, host, sizeof(float) * n, hipMemcpyHostToDevice)
             : hipMemcpy(host, ctx->dev_train, sizeof(float) * n, hipMemcpyDeviceToHost));
  return ETX_OK;
}

etx_status etx_train_apply(etx_ctx* ctx) {
  if (!ctx || !ctx->dev_train) return ETX_ERR_INVALID_ARG;
  const char* what = "etx_train_apply";
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  std::vector<float> p(blob_floats_of(ctx->cfg));
  HIPCHK(hipMemcpy(p.data(), ctx->dev_train, sizeof(float) * p.size(), hipMemcpyDeviceToHost));
  etx_status st = rebuild_weights(ctx, p.data());
  if (st != ETX_OK || !ctx->dev_tri_train || ctx->tri_train_fresh) return st;
  std::vector<float> q(ctx->tri_host.size());
  HIPCHK(hipMemcpy(q.data(), ctx->dev_tri_train, sizeof(float) * q.size(), hipMemcpyDeviceToHost));
  return etx_triplet_set(ctx, q.data(), (int64_t)q.size());
}

etx_status etx_train_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                                    size_t* bytes) {
  if (!ctx || !bytes || n_events < 0 || n_hits < 0 || edge_capacity < 0) return ETX_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(ctx, n_events, n_hits, edge_capacity);
  *bytes = train_layout(ctx, L, n_hits, edge_capacity).total;
  return ETX_OK;
}

etx_status etx_train_triplet_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits,
                                            int64_t edge_capacity, int64_t triplet_capacity, size_t* bytes) {
  if (!ctx || !bytes || n_events < 0 || n_hits < 0 || edge_capacity < 0 || triplet_capacity < 0)
    return ETX_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(ctx, n_events, n_hits, edge_capacity);
  const TrainLayout T = train_layout(ctx, L, n_hits, edge_capacity);
  *bytes = trip_layout(ctx, T.total, n_events, n_hits, edge_capacity, triplet_capacity).total;
  return ETX_OK;
}

etx_status etx_train_triplet_view(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                                  int64_t triplet_capacity, int32_t which, size_t* offset, size_t* bytes) {
  if (!ctx || !offset || !bytes || triplet_capacity < 0) return ETX_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(ctx, n_events, n_hits, edge_capacity);
  const TrainLayout T = train_layout(ctx, L, n_hits, edge_capacity);
  const TripLayout X = trip_layout(ctx, T.total, n_events, n_hits, edge_capacity, triplet_capacity);
  const size_t tc = (size_t)triplet_capacity;
  switch (which) {
    case 0: *offset = X.tgrad; *bytes = sizeof(float) * ETX_TRIPLET_NPARAM(ctx->cfg.gnn_hidden); break;
    case 1: *offset = X.lab; *bytes = tc; break;
    case 2: *offset = X.ta; *bytes = 4 * tc; break;
    case 3: *offset = X.tb; *bytes = 4 * tc; break;
    case 4: *offset = X.kind; *bytes = tc; break;
    case 5: *offset = X.art_off; *bytes = 8 * (size_t)(n_events + 1); break;
    case 6: *offset = X.elb_off; *bytes = 8 * (size_t)(n_events + 1); break;
    default: return ETX_ERR_INVALID_ARG;
  }
  return ETX_OK;
}

etx_status etx_train_view(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity, int32_t which,
                          size_t* offset, size_t* bytes) {
  if (!ctx || !offset || !bytes) return ETX_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(ctx, n_events, n_hits, edge_capacity);
  const TrainLayout T = train_layout(ctx, L, n_hits, edge_capacity);
  switch (which) {
    case 0: *offset = T.grad; *bytes = sizeof(float) * blob_floats_of(ctx->cfg); break;
    case 1: *offset = T.loss; *bytes = sizeof(float) * 4; break;
    case 2: *offset = T.lab; *bytes = edge_capacity; break;
    default: return ETX_ERR_INVALID_ARG;
  }
  return ETX_OK;
}

}  // extern "C"

namespace {

// the inference stages that build a batch's graph: bucketing, (embedding), radius graph, CSC permutation
hipError_t build_graph(const RunArgs& a, bool inference_embedding) {
  hipError_t e;
  if ((e = launch_init_status(a)) != hipSuccess) return e;
  if ((e = launch_validate(a)) != hipSuccess) return e;
  if ((e = launch_bucket(a)) != hipSuccess) return e;
  if (inference_embedding && (e = launch_embed(a)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t radius_and_csc(const RunArgs& a) {
  hipError_t e;
  if (a.ctx->radius_single) {
    if ((e = launch_radius(a, 2, false)) != hipSuccess) return e;
    if ((e = launch_scan_counts(a, false)) != hipSuccess) return e;
    if ((e = launch_slots_copy(a, false)) != hipSuccess) return e;
  } else {
    if ((e = launch_radius(a, 0, false)) != hipSuccess) return e;
    if ((e = launch_scan_counts(a, false)) != hipSuccess) return e;
    if ((e = launch_radius(a, 1, false)) != hipSuccess) return e;
  }
  return launch_csc(a);
}

}  // namespace

extern "C" {

etx_status etx_train_embed_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth,
                                float margin, float w_gen, float r_train, float lr, int64_t step, float* loss_dev,
                                void* ws_, size_t ws_bytes, etx_stream stream) {
  const char* what = "etx_train_embed_step";
  if (!ctx || !hits || !out || !truth || !ctx->dev_train) return ETX_ERR_INVALID_ARG;
  if (!truth->particle || !truth->succ || !truth->pred || !truth->query || !truth->rnd || !truth->rnd_ptr ||
      (!truth->rnd_src && hits->n_hits > 0))
    return ETX_ERR_INVALID_ARG;
  if (!(margin > 0) || !(w_gen > 0) || !(r_train > 0) || !(lr >= 0) || step < 1) return ETX_ERR_INVALID_ARG;
  const etx_config& c = ctx->cfg;
  if (c.emb_dim != 4 && c.emb_dim != 8 && c.emb_dim != 12 && c.emb_dim != 16) return ETX_ERR_UNSUPPORTED;
  WsLayout L;
  etx_status st = check_run(ctx, hits, out, ws_, ws_bytes, &L);
  if (st != ETX_OK) return st;
  const int64_t n = hits->n_hits, cap = out->edge_capacity;
  const TrainLayout T = train_layout(ctx, L, n, cap);
  if (ws_bytes < T.total) return ETX_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  char* ws = static_cast<char*>(ws_);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RunArgs a{ctx, *hits, *out, L, ws, s, false, ETX_FP32};
  const ParamMap P = param_map(c);
  float* prm = ctx->dev_train;
  float* grad = F(T.grad);
  const int64_t* status = out->status;
  const int W = c.emb_hidden, D = c.emb_dim, NL = c.emb_layers + 1;
  HIPCHK(build_graph(a, false));
  // training embedding: forward, keeping every layer's z and output; the output goes to the embedding buffer
  HIPCHK(launch_inputs(n, hits->x, hits->y, hits->z, 1.0f / c.r_scale_mm, 1.0f / c.z_scale_mm, nullptr, F(T.cyl),
                       status, s, ctx));
  for (int l = 0; l < NL; ++l) {
    const int K = l == 0 ? 3 : W, M = l + 1 < NL ? W : D;
    BlkFwd A{};
    A.rows = n;
    A.seg[0] = seg(l == 0 ? F(T.cyl) : F(T.emb_a[l - 1]), nullptr, K, K);
    A.nseg = 1;
    A.K = K;
    A.W = prm + P.emb[l];
    A.yhat = F(T.emb_yh[l]);
    const bool last = l + 1 == NL;
    A.y = last ? F(L.emb) : F(T.emb_a[l]);
    A.ldy = last ? kDpad : M;
    A.pad_zero = last ? 1 : 0;
    A.status = status;
    HIPCHK(launch_blk_fwd(A, M, last ? 0 : 1, s, ctx));
  }
  // hard negatives: the radius graph of the training embedding at the training radius
  RunArgs ar = a;
  ar.radius_override = r_train;
  HIPCHK(radius_and_csc(ar));
  HingeArgs Hg{};
  Hg.n = n;
  Hg.emb = F(L.emb);
  Hg.lde = kDpad;
  Hg.query = truth->query;
  Hg.succ = truth->succ;
  Hg.pred = truth->pred;
  Hg.particle = truth->particle;
  Hg.rnd = truth->rnd;
  Hg.rnd_ptr = truth->rnd_ptr;
  Hg.rnd_src = truth->rnd_src;
  Hg.row_ptr = reinterpret_cast<const int64_t*>(ws + L.row_ptr);
  Hg.dst = out->dst;
  Hg.col_ptr = reinterpret_cast<const int64_t*>(ws + L.col_ptr);
  Hg.csc = reinterpret_cast<const int32_t*>(ws + L.csc);
  Hg.margin = margin;
  Hg.w_gen = w_gen;
  Hg.counts = F(T.counts);
  Hg.counts_scratch = F(T.counts2);
  Hg.block_part = F(T.hparts);
  Hg.g_gen = F(T.g_gen);
  Hg.g_rnd = F(T.g_rnd);
  Hg.g_edge = F(T.g_edge);
  Hg.de = F(T.de);
  Hg.ldde = kDpad;
  Hg.status = status;
  HIPCHK(launch_hinge(Hg, D, F(T.loss), s));
  // backward through the layers
  for (int l = NL - 1; l >= 0; --l) {
    const int K = l == 0 ? 3 : W, M = l + 1 < NL ? W : D;
    BlkBwd B{};
    B.rows = n;
    B.dy = l + 1 == NL ? F(T.de) : F(T.edx[l % 2]);
    B.lddy = l + 1 == NL ? kDpad : M;
    B.yhat = F(T.emb_yh[l]);
    B.W = prm + P.emb[l];
    B.K = K;
    B.dz = F(T.edz);
    B.out[0] = tout(l > 0 ? F(T.edx[(l + 1) % 2]) : nullptr, K, K, 0);
    B.nseg = 1;
    B.status = status;
    HIPCHK(launch_blk_bwd(B, M, l + 1 == NL ? 0 : 1, s, ctx));
    Wgrad G{};
    G.rows = n;
    G.seg[0] = seg(l == 0 ? F(T.cyl) : F(T.emb_a[l - 1]), nullptr, K, K);
    G.nseg = 1;
    G.K = K;
    G.dz = F(T.edz);
    G.partial = F(T.part);
    G.status = status;
    HIPCHK(launch_wgrad(G, M, grad + P.emb[l], s));
  }
  const int64_t np = P.gnn_begin;
  const int64_t nb = (int64_t)blob_floats_of(c);
  if (lr > 0) HIPCHK(launch_adam(np, prm, prm + nb, prm + 2 * nb, grad, lr, step, status, s, ctx));
  if (loss_dev) HIPCHK(hipMemcpyAsync(loss_dev, F(T.loss), sizeof(float), hipMemcpyDeviceToDevice, s));
  return ETX_OK;
}

}  // extern "C"

namespace {

// One network step; tcap >= 0 adds the triplet term of eq. gnn-loss.
etx_status gnn_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth, float alpha,
                    float gamma, float lr, int64_t step, int64_t tcap, int64_t* needed, float* loss_dev, void* ws_,
                    size_t ws_bytes, etx_stream stream) {
  const char* what = tcap >= 0 ? "etx_train_triplet_step" : "etx_train_gnn_step";
  if (!ctx || !hits || !out || !truth || !truth->succ || !ctx->dev_train) return ETX_ERR_INVALID_ARG;
  if (!(alpha >= 0 && alpha <= 1) || !(gamma >= 0) || !(lr >= 0) || step < 1) return ETX_ERR_INVALID_ARG;
  const bool trip = tcap >= 0;
  if (trip && (!truth->particle || tcap >= 0x7fffffffLL)) return ETX_ERR_INVALID_ARG;
  const etx_config& c = ctx->cfg;
  WsLayout L;
  etx_status st = check_run(ctx, hits, out, ws_, ws_bytes, &L);
  if (st != ETX_OK) return st;
  const int64_t n = hits->n_hits, cap = out->edge_capacity;
  const TrainLayout T = train_layout(ctx, L, n, cap);
  if (ws_bytes < T.total) return ETX_ERR_INVALID_ARG;
  TripLayout X{};
  if (trip) {
    X = trip_layout(ctx, T.total, hits->n_events, n, cap, tcap);
    if (ws_bytes < X.total) return ETX_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
    if ((st = tri_train_state(ctx)) != ETX_OK) return st;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return ETX_ERR_HIP;
  char* ws = static_cast<char*>(ws_);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RunArgs a{ctx, *hits, *out, L, ws, s, false, ETX_FP32};
  const ParamMap P = param_map(c);
  float* prm = ctx->dev_train;
  float* grad = F(T.grad);
  const int64_t* status = out->status;
  const int H = c.gnn_hidden, S = c.gnn_steps;
  HIPCHK(build_graph(a, true));
  HIPCHK(radius_and_csc(a));
  // the number of edges (this step synchronises the stream once)
  int64_t dev_status[2];
  int64_t E = 0;
  HIPCHK(hipMemcpyAsync(&E, ws + L.row_ptr + sizeof(int64_t) * n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(dev_status, out->status, sizeof(dev_status), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (dev_status[0] != ETX_OK) return static_cast<etx_status>(dev_status[0]);
  const int32_t* src = out->src;
  const int32_t* dst = out->dst;
  const int64_t* row_ptr = reinterpret_cast<const int64_t*>(ws + L.row_ptr);
  const int64_t* col_ptr = reinterpret_cast<const int64_t*>(ws + L.col_ptr);
  const int32_t* csc = reinterpret_cast<const int32_t*>(ws + L.csc);
  const int64_t nH = n * H, eH = E * H;
  auto hst = [&](int k) { return F(T.hst) + k * nH; };
  auto est = [&](int k) { return F(T.est) + k * eH; };
  auto yhn = [&](int j) { return F(T.yh_n) + j * nH; };
  auto rsn = [&](int j) { return F(T.rs_n) + j * n; };
  auto yhe = [&](int j) { return F(T.yh_e) + j * eH; };
  auto rse = [&](int j) { return F(T.rs_e) + j * E; };
  // node-row block j: 0 ne1, 1 ne2, 2 + 2k nn1_k, 3 + 2k nn2_k; edge-row block j: 0 ee1, 1 ee2, 2 + 2k en1_k,
  // 3 + 2k en2_k, 2 + 2S cls
  auto fwd = [&](int64_t rows, std::initializer_list<TrainSeg> segs, const float* Wp, float* yh, float* rs, float* y,
                 const float* resid) {
    BlkFwd A{};
    A.rows = rows;
    int i = 0, K = 0;
    for (const TrainSeg& g : segs) {
      A.seg[i++] = g;
      K += g.width;
    }
    A.nseg = i;
    A.K = K;
    A.W = Wp;
    A.yhat = yh;
    A.rstd = rs;
    A.y = y;
    A.ldy = H;
    A.resid = resid;
    A.status = status;
    return launch_blk_fwd(A, H, 2, s, ctx);
  };
  auto bwd = [&](int64_t rows, const float* dy, const float* dy2, const float* yh, const float* rs, const float* Wp,
                 int K, float* dz, std::initializer_list<TrainOut> outs) {
    BlkBwd B{};
    B.rows = rows;
    B.dy = dy;
    B.dy2 = dy2;
    B.lddy = H;
    B.yhat = yh;
    B.rstd = rs;
    B.W = Wp;
    B.K = K;
    B.dz = dz;
    int i = 0;
    for (const TrainOut& o : outs) B.out[i++] = o;
    B.nseg = i;
    B.status = status;
    return launch_blk_bwd(B, H, 2, s, ctx);
  };
  auto wg = [&](int64_t rows, std::initializer_list<TrainSeg> segs, const float* dz, int M, int64_t goff) {
    Wgrad G{};
    G.rows = rows;
    int i = 0, K = 0;
    for (const TrainSeg& g : segs) {
      G.seg[i++] = g;
      K += g.width;
    }
    G.nseg = i;
    G.K = K;
    G.dz = dz;
    G.partial = F(T.part);
    G.status = status;
    return launch_wgrad(G, M, grad + goff, s);
  };
  // ---- forward
  HIPCHK(launch_edge_labels(E, src, dst, truth->succ, truth->succ2, reinterpret_cast<uint8_t*>(ws + T.lab), status, s,
                            ctx));
  HIPCHK(launch_inputs(n, hits->x, hits->y, hits->z, 1.0f / c.r_scale_mm, 1.0f / c.z_scale_mm, F(T.cart), nullptr,
                       status, s, ctx));
  HIPCHK(fwd(n, {seg(F(T.cart), nullptr, 3, 3)}, prm + P.ne1, yhn(0), rsn(0), F(T.y1n), nullptr));
  HIPCHK(fwd(n, {seg(F(T.y1n), nullptr, H, H)}, prm + P.ne2, yhn(1), rsn(1), hst(0), nullptr));
  HIPCHK(fwd(E, {seg(hst(0), src, H, H), seg(hst(0), dst, H, H)}, prm + P.ee1, yhe(0), rse(0), F(T.t1ee), nullptr));
  HIPCHK(fwd(E, {seg(F(T.t1ee), nullptr, H, H)}, prm + P.ee2, yhe(1), rse(1), est(0), nullptr));
  for (int k = 0; k < S; ++k) {
    float* mo = F(T.mo) + k * nH;
    float* mi = F(T.mi) + k * nH;
    HIPCHK(launch_node_sum(n, H, row_ptr, est(k), col_ptr, csc, nullptr, mo, 0, status, s, ctx));
    HIPCHK(launch_node_sum(n, H, row_ptr, nullptr, col_ptr, csc, est(k), mi, 0, status, s, ctx));
    float* t1n = F(T.t1n) + k * nH;
    HIPCHK(fwd(n, {seg(hst(k), nullptr, H, H), seg(mo, nullptr, H, H), seg(mi, nullptr, H, H)}, prm + P.nn1[k],
               yhn(2 + 2 * k), rsn(2 + 2 * k), t1n, nullptr));
    HIPCHK(fwd(n, {seg(t1n, nullptr, H, H)}, prm + P.nn2[k], yhn(3 + 2 * k), rsn(3 + 2 * k), hst(k + 1), hst(k)));
    float* t1e = F(T.t1e) + k * eH;
    HIPCHK(fwd(E, {seg(est(k), nullptr, H, H), seg(hst(k + 1), src, H, H), seg(hst(k + 1), dst, H, H)},
               prm + P.en1[k], yhe(2 + 2 * k), rse(2 + 2 * k), t1e, nullptr));
    HIPCHK(fwd(E, {seg(t1e, nullptr, H, H)}, prm + P.en2[k], yhe(3 + 2 * k), rse(3 + 2 * k), est(k + 1), est(k)));
  }
  const int jc = 2 + 2 * S;
  HIPCHK(fwd(E, {seg(est(S), nullptr, H, H)}, prm + P.cls1, yhe(jc), rse(jc), F(T.cls), nullptr));
  HIPCHK(launch_focal(E, H, F(T.cls), prm + P.cls2, reinterpret_cast<const uint8_t*>(ws + T.lab), alpha, gamma,
                      F(T.dlogit), F(T.da_e), F(T.lpart), F(T.loss), 0, status, s, trip ? out->score : nullptr));
  // ---- triplets of the purified graph of this step's scores, and the two classifiers on them
  etx_tracks TS{};
  int64_t nrow[2] = {0, 0};
  const int64_t hsz = 3 * (int64_t)H * H + 3 * H + 1;
  float* tprm = ctx->dev_tri_train;
  auto I32 = [&](size_t off) { return reinterpret_cast<int32_t*>(ws + off); };
  if (trip) {
    TS.triplet_capacity = tcap;
    TS.tri_a = I32(X.ta);
    TS.tri_b = I32(X.tb);
    TS.tri_score = F(X.tscore);
    TS.tri_kind = reinterpret_cast<uint8_t*>(ws + X.kind);
    TS.art_off = reinterpret_cast<int64_t*>(ws + X.art_off);
    TS.elb_off = reinterpret_cast<int64_t*>(ws + X.elb_off);
    TS.status = reinterpret_cast<int64_t*>(ws + X.tstatus);
    HIPCHK(launch_triplet_stage(a, TS, ws + X.tri, X.TL, 0));
    int64_t cnt[2];
    HIPCHK(hipMemcpyAsync(&cnt[0], ws + X.tri + X.TL.art_pos + sizeof(int64_t) * n, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&cnt[1], ws + X.tri + X.TL.elb_pos + sizeof(int64_t) * n, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (needed) *needed = cnt[0] + cnt[1];
    if (cnt[0] + cnt[1] > tcap) return ETX_ERR_CAPACITY;
    nrow[0] = cnt[0];
    nrow[1] = cnt[1];
    uint8_t* tlab = reinterpret_cast<uint8_t*>(ws + X.lab);
    HIPCHK(launch_tri_labels(a, ws + X.tri, X.TL, TS, *truth, tlab));
    HIPCHK(hipMemsetAsync(F(X.tgrad), 0, sizeof(float) * 2 * hsz, s));
    HIPCHK(hipMemsetAsync(F(T.loss) + 1, 0, sizeof(float) * 2, s));
    for (int hd = 0; hd < 2; ++hd) {
      const int64_t nh = nrow[hd], r0 = hd ? nrow[0] : 0;
      if (nh == 0) continue;
      const float* hp = tprm + hd * hsz;
      HIPCHK(fwd(nh, {seg(est(S), TS.tri_a + r0, H, H), seg(est(S), TS.tri_b + r0, H, H)}, hp, F(X.yh1) + r0 * H,
                 F(X.rs1) + r0, F(X.y1) + r0 * H, nullptr));
      HIPCHK(fwd(nh, {seg(F(X.y1) + r0 * H, nullptr, H, H)}, hp + 2 * H * H + H, F(X.yh2) + r0 * H, F(X.rs2) + r0,
                 F(X.y2) + r0 * H, nullptr));
      HIPCHK(launch_focal(nh, H, F(X.y2) + r0 * H, hp + 3 * H * H + 2 * H, tlab + r0, alpha, gamma, F(X.dlogit) + r0,
                          F(X.dc) + r0 * H, F(T.lpart), F(T.loss), 1 + hd, status, s));
    }
  }
  // ---- backward
  HIPCHK(wg(E, {seg(F(T.cls), nullptr, H, H)}, F(T.dlogit), 1, P.cls2));
  HIPCHK(bwd(E, F(T.da_e), nullptr, yhe(jc), rse(jc), prm + P.cls1, H, F(T.dz_e), {tout(F(T.de_e), H, H, 0)}));
  HIPCHK(wg(E, {seg(est(S), nullptr, H, H)}, F(T.dz_e), H, P.cls1));
  if (trip) {
    auto wgt = [&](int64_t rows, std::initializer_list<TrainSeg> segs, const float* dz, int M, float* gp) {
      Wgrad G{};
      G.rows = rows;
      int i = 0, K = 0;
      for (const TrainSeg& g : segs) {
        G.seg[i++] = g;
        K += g.width;
      }
      G.nseg = i;
      G.K = K;
      G.dz = dz;
      G.partial = F(T.part);
      G.status = status;
      return launch_wgrad(G, M, gp, s);
    };
    for (int hd = 0; hd < 2; ++hd) {
      const int64_t nh = nrow[hd], r0 = hd ? nrow[0] : 0;
      if (nh == 0) continue;
      const float* hp = tprm + hd * hsz;
      float* hg = F(X.tgrad) + hd * hsz;
      HIPCHK(wgt(nh, {seg(F(X.y2) + r0 * H, nullptr, H, H)}, F(X.dlogit) + r0, 1, hg + 3 * H * H + 2 * H));
      HIPCHK(bwd(nh, F(X.dc) + r0 * H, nullptr, F(X.yh2) + r0 * H, F(X.rs2) + r0, hp + 2 * H * H + H, H, F(X.dz),
                 {tout(F(X.da), H, H, 0)}));
      HIPCHK(wgt(nh, {seg(F(X.y1) + r0 * H, nullptr, H, H)}, F(X.dz), H, hg + 2 * H * H + H));
      HIPCHK(bwd(nh, F(X.da), nullptr, F(X.yh1) + r0 * H, F(X.rs1) + r0, hp, 2 * H, F(X.dz),
                 {tout(F(X.dxa) + r0 * H, H, H, 0), tout(F(X.dxb) + r0 * H, H, H, 0)}));
      HIPCHK(wgt(nh, {seg(est(S), TS.tri_a + r0, H, H), seg(est(S), TS.tri_b + r0, H, H)}, F(X.dz), H, hg));
    }
    HIPCHK(launch_tri_edge_grad(a, ws + X.tri, X.TL, TS, F(X.dxa), F(X.dxb), F(T.de_e)));
  }
  for (int k = S - 1; k >= 0; --k) {
    float* t1e = F(T.t1e) + k * eH;
    // edge update k
    HIPCHK(bwd(E, F(T.de_e), nullptr, yhe(3 + 2 * k), rse(3 + 2 * k), prm + P.en2[k], H, F(T.dz_e),
               {tout(F(T.da_e), H, H, 0)}));
    HIPCHK(wg(E, {seg(t1e, nullptr, H, H)}, F(T.dz_e), H, P.en2[k]));
    HIPCHK(bwd(E, F(T.da_e), nullptr, yhe(2 + 2 * k), rse(2 + 2 * k), prm + P.en1[k], 3 * H, F(T.dz_e),
               {tout(F(T.de_e), H, H, 1), tout(F(T.dxs), H, H, 0), tout(F(T.dxd), H, H, 0)}));
    HIPCHK(wg(E, {seg(est(k), nullptr, H, H), seg(hst(k + 1), src, H, H), seg(hst(k + 1), dst, H, H)}, F(T.dz_e),
              H, P.en1[k]));
    HIPCHK(launch_node_sum(n, H, row_ptr, F(T.dxs), col_ptr, csc, F(T.dxd), F(T.dh), k == S - 1 ? 0 : 1, status, s,
                           ctx));
    // node update k
    float* t1n = F(T.t1n) + k * nH;
    HIPCHK(bwd(n, F(T.dh), nullptr, yhn(3 + 2 * k), rsn(3 + 2 * k), prm + P.nn2[k], H, F(T.dz_n),
               {tout(F(T.da_n), H, H, 0)}));
    HIPCHK(wg(n, {seg(t1n, nullptr, H, H)}, F(T.dz_n), H, P.nn2[k]));
    HIPCHK(bwd(n, F(T.da_n), nullptr, yhn(2 + 2 * k), rsn(2 + 2 * k), prm + P.nn1[k], 3 * H, F(T.dz_n),
               {tout(F(T.dh), H, H, 1), tout(F(T.dmo), H, H, 0), tout(F(T.dmi), H, H, 0)}));
    HIPCHK(wg(n, {seg(hst(k), nullptr, H, H), seg(F(T.mo) + k * nH, nullptr, H, H), seg(F(T.mi) + k * nH, nullptr, H, H)},
              F(T.dz_n), H, P.nn1[k]));
    HIPCHK(launch_edge_gather_add(E, H, src, dst, F(T.dmo), F(T.dmi), F(T.de_e), status, s, ctx));
  }
  // edge encoder, node encoder
  HIPCHK(bwd(E, F(T.de_e), nullptr, yhe(1), rse(1), prm + P.ee2, H, F(T.dz_e), {tout(F(T.da_e), H, H, 0)}));
  HIPCHK(wg(E, {seg(F(T.t1ee), nullptr, H, H)}, F(T.dz_e), H, P.ee2));
  HIPCHK(bwd(E, F(T.da_e), nullptr, yhe(0), rse(0), prm + P.ee1, 2 * H, F(T.dz_e),
             {tout(F(T.dxs), H, H, 0), tout(F(T.dxd), H, H, 0)}));
  HIPCHK(wg(E, {seg(hst(0), src, H, H), seg(hst(0), dst, H, H)}, F(T.dz_e), H, P.ee1));
  HIPCHK(launch_node_sum(n, H, row_ptr, F(T.dxs), col_ptr, csc, F(T.dxd), F(T.dh), S > 0 ? 1 : 0, status, s, ctx));
  HIPCHK(bwd(n, F(T.dh), nullptr, yhn(1), rsn(1), prm + P.ne2, H, F(T.dz_n), {tout(F(T.da_n), H, H, 0)}));
  HIPCHK(wg(n, {seg(F(T.y1n), nullptr, H, H)}, F(T.dz_n), H, P.ne2));
  HIPCHK(bwd(n, F(T.da_n), nullptr, yhn(0), rsn(0), prm + P.ne1, 3, F(T.dz_n), {tout(nullptr, 3, 3, 0)}));
  HIPCHK(wg(n, {seg(F(T.cart), nullptr, 3, 3)}, F(T.dz_n), H, P.ne1));
  const int64_t nb = (int64_t)blob_floats_of(c);
  const int64_t g0 = P.gnn_begin, ng = P.total - P.gnn_begin;
  if (lr > 0) HIPCHK(launch_adam(ng, prm + g0, prm + nb + g0, prm + 2 * nb + g0, grad + g0, lr, step, status, s, ctx));
  if (trip && lr > 0)
    HIPCHK(launch_adam(2 * hsz, tprm, tprm + 2 * hsz, tprm + 4 * hsz, F(X.tgrad), lr, step, status, s, ctx));
  if (loss_dev)
    HIPCHK(hipMemcpyAsync(loss_dev, F(T.loss), sizeof(float) * (trip ? 3 : 1), hipMemcpyDeviceToDevice, s));
  return ETX_OK;
}

}  // namespace

extern "C" {

etx_status etx_train_gnn_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth, float alpha,
                              float gamma, float lr, int64_t step, float* loss_dev, void* ws, size_t ws_bytes,
                              etx_stream stream) {
  return gnn_step(ctx, hits, out, truth, alpha, gamma, lr, step, -1, nullptr, loss_dev, ws, ws_bytes, stream);
}

etx_status etx_train_triplet_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth,
                                  float alpha, float gamma, float lr, int64_t step, int64_t triplet_capacity,
                                  int64_t* triplets_needed, float* loss_dev, void* ws, size_t ws_bytes,
                                  etx_stream stream) {
  if (triplet_capacity < 0) return ETX_ERR_INVALID_ARG;
  return gnn_step(ctx, hits, out, truth, alpha, gamma, lr, step, triplet_capacity, triplets_needed, loss_dev, ws,
                  ws_bytes, stream);
}

}  // extern "C"
