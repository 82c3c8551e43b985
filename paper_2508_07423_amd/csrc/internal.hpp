// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/etx.h"

namespace etx {

constexpr int kEdgeTile = 16;      // edges per wave tile of the MLP kernels (the MFMA column count)
constexpr int kDpad = 16;          // padded embedding width in HBM
constexpr int kScanBlock = 8192;   // elements per block of the device-wide scan

// Kernel precisions (tile.hpp's Prec): FP32, BF16, FP8, FP32 as three BF16
// parts, BF16 / FP8 / INT8 operands with FP32 node and edge state.
// weight bytes per element
constexpr int kPrecBytes[7] = {4, 2, 1, 6, 2, 1, 1};
// the weight segment set a precision uses (the FP32-state forms share BF16's and FP8's)
constexpr int kSegPrec[7] = {0, 1, 2, 3, 1, 2, 4};
// the etx_precision of a kernel precision's operands
constexpr int kEtxPrec[7] = {ETX_FP32, ETX_BF16, ETX_FP8_E4M3, ETX_FP32, ETX_BF16, ETX_FP8_E4M3, ETX_INT8};
constexpr int kF32Split = 3;                  // segment set of the split-FP32 edge kernels
constexpr int kBf16Master = 4;                // BF16 operands, FP32 node and edge state
constexpr int kFp8Master = 5;                 // FP8 operands, FP32 node and edge state
constexpr int kI8Master = 6;                  // INT8 operands, FP32 node and edge state
constexpr int kI8Seg = 4;                     // segment set of the INT8 weights
constexpr int kNumSegs = 5;
constexpr int kSegBytes[kNumSegs] = {4, 2, 1, 6, 1};   // weight bytes per element of each segment set

// Offsets (in bytes) of the per-kernel weight segments in a precision's device buffer.
struct WeightMap {
  int64_t emb = 0;                 // embedding segment
  int64_t node_enc = 0;            // node encoder + edge-encoder source/target products
  int64_t edge_enc = 0;            // edge encoder second layer
  int64_t node[16] = {};           // node net k + edge net k source/target products
  int64_t edge[16] = {};           // edge net k (edge part) + second layer
  int64_t cls = 0;                 // classifier
  int64_t total = 0;
};

// Byte offsets of the workspace buffers.
struct WsLayout {
  size_t bucket, plane_off, emb, cnt, slots, row_ptr, scan_tmp, col_ptr, csc, h, ps, pd, msg, e, opart, kept, kept_cnt,
      calib, pf_keep, pf_tmp, cand_src, cand_dst, pf_prob, pf_part, pf_grad, pf_polar, pf_feat, pf_fallback, total;
  int64_t n_scan_blocks;
};

struct GraphKey {
  const void* p[16];
  int64_t n[4];
  bool operator<(const GraphKey& o) const;
};

}  // namespace etx

struct etx_ctx {
  etx_config cfg;
  int device = 0;
  int n_cu = 256;
  void* seg_base[etx::kNumSegs] = {};   // weight segments per set (FP32, BF16, FP8, split FP32, INT8)
  etx::WeightMap wmap[etx::kNumSegs];
  float* dev_scales = nullptr;     // [512] per-tensor scales: FP8 set 0..255, INT8 set 256..511
  float host_scales[512] = {};
  double i8_wscale[256] = {};      // INT8 weight scales max|W| / 127 (slots 64..), exact, for the codes
  bool calibrated = false;
  // prefilter (params, Adam m, v) in FP32 on the device
  float* dev_pf = nullptr;
  // in-library training: the weight blob's parameters, Adam m, v (FP32, device; etx_train_begin)
  float* dev_train = nullptr;
  // triplet classifiers: both heads permuted for the column tiles (device), and as given (host)
  float* dev_tri = nullptr;
  std::vector<float> tri_host;
  // triplet classifiers in training: params, Adam m, v (FP32, device), allocated at the first triplet step
  float* dev_tri_train = nullptr;
  bool tri_train_fresh = false;    // etx_train_begin ran since the classifiers' training state was set
  bool pf_set = false;
  float pf_band_lo = 0.f, pf_band_hi = 1.f;   // validated band of an event's kept fraction
  // tuning
  int edge_wg_per_cu = 8;
  int node_wg_per_cu = 1;
  int radius_lds = 1;
  int segsum_unroll = 4;
  int edge_pipeline = 1;
  int edge_threads = 256;
  int edge_wreg = 0;
  int emb_precision = -1;          // -1: cfg.precision
  int outsum_lds = 1;
  int f32_split = 0;               // FP32 runs: edge-kernel GEMMs as split BF16 products
  int radius_single = 1;           // radius graph: one selection pass + slot copy (0: count and emit passes)
  int fuse_messages = 0;           // message sums gathered inside the node-update kernel
  int radius_sort_min = 512;       // staged windows from this size on are sorted along their widest axis
  int radius_fast = 0;             // select pass: 16-lane path for sources with few candidates
  int radius_split = 0;            // radius search: small windows in a launch of its own with less LDS
  int xcd_map = 0;                 // tile and node kernels: contiguous work per XCD
  int edge_products = 0;           // 1: edge kernels form the node-product terms from gathered h rows
  int csc_place = 1;               // short-row CSC placed by the whole block, then columns sorted
  int pf_features = 0;             // 1: prefilter inference also stores each candidate's features
  int compact_state = 0;           // BF16/FP8 runs: 1 keeps h, e in the operand format, 0 in FP32 (residual masters)
  std::vector<char> blob;          // the weight blob as given (for etx_save)
  int use_graph = 0;
  std::map<etx::GraphKey, hipGraphExec_t> graphs;
  // stage timing with HIP events (ETX_OPT_PROFILE)
  int profile = 0;
  int64_t profile_mask = 0x7fffffff;   // stages timed when profiling (bit i: stage i)
  struct Mark { int stage; hipEvent_t start, end; };
  std::vector<Mark> marks;
  size_t n_marks = 0;
  double stage_ms[32] = {};
  int64_t stage_launches[32] = {};
  // tuning table: "signature bucket" -> tuned option values (etx_autotune, etx_tuning_load)
  std::string arch;                // device architecture name, e.g. "gfx950"
  std::map<std::string, std::vector<std::pair<int32_t, int64_t>>> tuning;
  std::string tuning_applied;      // key of the entry whose options are in effect
};

namespace etx {

WsLayout ws_layout(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_cap);

struct RunArgs {
  const etx_ctx* ctx;
  etx_hits hits;
  etx_out out;
  WsLayout L;
  char* ws;
  hipStream_t stream;
  bool calibrate;                  // record amax observers (FP32 run)
  int prec;                        // kernel precision: etx_precision, or kBf16Master / kFp8Master
  bool untimed = false;            // no stage timing even when profiling is on (the no-allocation entry point)
  float radius_override = 0.f;     // > 0: the radius graph at this radius instead of the configuration's (training)
  bool keep_final_e = false;       // the final edge step also stores e_S (the triplet classifiers' input)
};

// Byte offsets (from the start of the triplet area) of the triplet stage's buffers.
struct TriLayout {
  size_t deg_in, deg_out, cnt_art, cnt_elb, art_pos, elb_pos, part, lstate, dup, touched, par, comp, ccount, cstart,
      cedge, ntr, c1, c2, tev, tlen, total;
};
TriLayout tri_layout(int64_t n_events, int64_t n_hits, int64_t edge_cap, int64_t triplet_cap, int64_t track_cap);
// Floats of one triplet classifier in its device form.
int tri_head_floats(int H);
// Permute one classifier (host parameters W1 b1 W2 b2 W3 b3) into its device form.
void tri_prepare_head(const float* p, int H, float* out);
// The triplet stage in three parts (0: triplets of the purified graph, 1: classifier scores, 2: tracks).
hipError_t launch_triplet_stage(const RunArgs& a, const etx_tracks& T, char* tws, const TriLayout& TL, int part);
// training: labels of the triplets of part 0, and the triplet rows' input gradients added into dL/de_S
hipError_t launch_tri_labels(const RunArgs& a, char* tws, const TriLayout& TL, const etx_tracks& T,
                             const etx_truth& truth, uint8_t* lab);
hipError_t launch_tri_edge_grad(const RunArgs& a, char* tws, const TriLayout& TL, const etx_tracks& T,
                                const float* dxa, const float* dxb, float* de);

// launchers (graph.hip)
hipError_t launch_init_status(const RunArgs& a);
hipError_t launch_validate(const RunArgs& a);
hipError_t launch_bucket(const RunArgs& a);
// radius graph passes (mode: 0 count, 1 emit CSR rows, 2 select into slots)
hipError_t launch_radius(const RunArgs& a, int mode, bool candidates);
hipError_t launch_slots_copy(const RunArgs& a, bool candidates);
hipError_t launch_scan_counts(const RunArgs& a, bool candidates);
hipError_t launch_csc(const RunArgs& a);
hipError_t launch_compact(const RunArgs& a);
hipError_t launch_union_find(const RunArgs& a);
// launchers (embed.hip)
hipError_t launch_embed(const RunArgs& a);
// launchers (gnn.hip)
hipError_t launch_node_encode(const RunArgs& a);
hipError_t launch_edge_encode(const RunArgs& a);
hipError_t launch_segsum(const RunArgs& a, int k);
hipError_t launch_node_step(const RunArgs& a, int k);
hipError_t launch_edge_step(const RunArgs& a, int k, bool final_step);
// launchers (prefilter.hip)
hipError_t launch_prefilter_infer(const RunArgs& a);        // candidates -> keep flags -> compacted edges
hipError_t launch_prefilter_band(const RunArgs& a);           // events outside the band keep every candidate
hipError_t launch_prefilter_count(const RunArgs& a);
hipError_t launch_prefilter_compact(const RunArgs& a);
hipError_t launch_prefilter_train(const RunArgs& a, const uint8_t* labels, float lr, float pos_weight, int64_t step,
                                  float* loss_dev);
constexpr int kPfGradStride = 1320;                         // floats per wave partial of the prefilter gradient
constexpr int kPfMaxWaves = 256 * 2 * 8;                    // partial slots (CUs x workgroups x waves)
hipError_t launch_quantize(int prec, const float* in, float* out, int64_t n, float scale, hipStream_t s);

int set_kernel_attributes();

// Tuning-table key of a batch for this context: the configuration and run
// modes that change the best schedule, then the shape bucket.
std::string tuning_key(const etx_ctx* ctx, int64_t n_events, int64_t n_hits);
// Options the autotuner sets (saved in the tuning table).
extern const int32_t kTunedOptions[];
extern const int kNumTunedOptions;

}  // namespace etx
