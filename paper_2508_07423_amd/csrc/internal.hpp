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

constexpr int kTile = 32;          // columns (hits or edges) per wave tile
constexpr int kDpad = 16;          // padded embedding width in HBM
constexpr int kScanBlock = 1024;   // elements per block of the device-wide scan

// Calibration observer slots (absolute maxima of quantised activations).
enum CalibSlot {
  CAL_EMB_IN = 0,                  // + layer (embedding GEMM inputs, layers >= 1), 4 slots
  CAL_NE_L2 = 4,                   // node encoder layer-2 input
  CAL_H0 = 5,                      // node encodings (inputs of Ws/Wd products), per step: CAL_H0 + k
  CAL_EE_L2 = 22,                  // edge encoder layer-2 input
  CAL_E = 23,                      // stored edge encodings: CAL_E + k (k = 0..S)
  CAL_NN_IN = 40,                  // node net k layer-1 input [h, mo, mi] (one scale): + k
  // the remaining slots hold layer-2 inputs and classifier inputs
  CAL_NN_L2 = 56,                  // node net layer-2 inputs (shared over steps)
  CAL_EN_L2 = 57,                  // edge net layer-2 inputs (shared over steps)
  CAL_CLS_IN = 58,                 // classifier layer-1 input
  CAL_CLS_L2 = 59,                 // classifier hidden
};

// Offsets (in floats) of the per-kernel weight segments in the device buffer.
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
  size_t bucket, plane_off, emb, cnt, row_ptr, scan_tmp, col_ptr, csc, h, ps, pd, msg, e, kept, kept_cnt,
      calib, pf_keep, pf_tmp, pf_grad, total;
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
  float* dev_w = nullptr;          // FP32 weight segments
  etx::WeightMap wmap;
  void* dev_wq = nullptr;          // low-precision (BF16/FP8) weight copies
  int64_t wq_bytes = 0;
  std::vector<int64_t> wq_off;     // per-layer offsets into dev_wq (bytes)
  float* dev_scales = nullptr;     // [ETX_N_CALIB] activation scales + weight scales
  bool calibrated = false;
  std::vector<float> host_blob;    // the weight payload (for etx_set_precision rebuilds)
  // prefilter (params, Adam m, v) in FP32 on the device
  float* dev_pf = nullptr;
  bool pf_set = false;
  // tuning
  int edge_wg_per_cu = 2;
  int node_wg_per_cu = 1;
  int radius_lds = 1;
  int segsum_unroll = 4;
  int use_graph = 0;
  std::map<etx::GraphKey, hipGraphExec_t> graphs;
  // stage timing with HIP events (ETX_OPT_PROFILE)
  int profile = 0;
  struct Mark { int stage; hipEvent_t start, end; };
  std::vector<Mark> marks;
  size_t n_marks = 0;
  double stage_ms[32] = {};
  int64_t stage_launches[32] = {};
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
  bool calibrate;                  // record amax observers
};

// launchers (graph.hip)
hipError_t launch_init_status(const RunArgs& a);
hipError_t launch_validate(const RunArgs& a);
hipError_t launch_bucket(const RunArgs& a);
hipError_t launch_radius(const RunArgs& a, bool emit);
hipError_t launch_scan_counts(const RunArgs& a);
hipError_t launch_csc(const RunArgs& a);
hipError_t launch_compact(const RunArgs& a);
hipError_t launch_union_find(const RunArgs& a);
// launchers (embed.hip)
hipError_t launch_embed(const RunArgs& a);
// launchers (gnn.hip)
hipError_t launch_node_encode(const RunArgs& a);
hipError_t launch_edge_encode(const RunArgs& a);
hipError_t launch_segsum(const RunArgs& a);
hipError_t launch_node_step(const RunArgs& a, int k);
hipError_t launch_edge_step(const RunArgs& a, int k, bool final_step);
// launchers (prefilter.hip)
hipError_t launch_prefilter_infer(const RunArgs& a);
hipError_t launch_prefilter_train(const RunArgs& a, const uint8_t* labels, float lr, float pos_weight, int64_t step,
                                  float* loss_dev);

int set_kernel_attributes();

}  // namespace etx
