// Row-wise training kernels (train.hip) and their argument blocks.
#pragma once
#include "internal.hpp"

namespace etx {

constexpr int kTrainChunks = 256;       // row chunks of a weight-gradient reduction
constexpr int kTrainLossBlocks = 512;   // blocks of the loss kernels (partials summed in block order)

// One input segment of a row: `width` features at base[row * ld], row = idx ? idx[r] : r.
struct TrainSeg {
  const float* base;
  const int32_t* idx;
  int width;
  int ld;
};

// Gradient output of one input segment: dx[r * ld + k] (= or +=), or skipped when base is null.
struct TrainOut {
  float* base;
  int width;
  int ld;
  int add;
};

struct BlkFwd {
  int64_t rows;
  TrainSeg seg[3];
  int nseg;
  int K;                 // total input width
  const float* W;        // [K][M] then b[M] (FP32 parameters on the device)
  float* yhat;           // [rows][M]: z (no activation, ReLU) or the normalised value (LayerNorm); may be null
  float* rstd;           // [rows] (LayerNorm)
  float* y;              // output rows, stride ldy
  int ldy;
  int pad_zero;          // 1: columns M..ldy-1 of y are written as zeros
  const float* resid;    // optional residual added to the output (stride ldy)
  const int64_t* status;
};

struct BlkBwd {
  int64_t rows;
  const float* dy;       // dL/dy rows (stride lddy)
  const float* dy2;      // optional second term added to dy
  int lddy;
  const float* yhat;
  const float* rstd;
  const float* W;        // [K][M]
  int K;
  float* dz;             // [rows][M]: dL/dz
  TrainOut out[3];       // dL/dx per input segment
  int nseg;
  const int64_t* status;
};

struct Wgrad {
  int64_t rows;
  TrainSeg seg[3];
  int nseg;
  int K;
  const float* dz;       // [rows][M]
  float* partial;        // [kTrainChunks][K * M + M]
  const int64_t* status;
};

struct HingeArgs {
  int64_t n;                 // hits
  const float* emb;          // [n][lde]
  int lde;
  const uint8_t* query;      // 1: the hit belongs to a particle with at least three hits
  const int32_t* succ;       // successor hit on the hit's particle (-1: none)
  const int32_t* pred;       // predecessor hit (-1: none)
  const int32_t* particle;   // -1: noise
  const int32_t* rnd;        // random partner of each query (-1: none)
  const int64_t* rnd_ptr;    // [n + 1] random pairs grouped by target: rnd_src[rnd_ptr[b] .. rnd_ptr[b+1]]
  const int32_t* rnd_src;
  const int64_t* row_ptr;    // training radius graph (CSR by source)
  const int32_t* dst;
  const int64_t* col_ptr;    // its CSC
  const int32_t* csc;
  float margin, w_gen;
  float* counts;             // [2]: genuine and fake pair counts (written by the counting pass)
  float* counts_scratch;     // [2]
  float* block_part;         // [kTrainLossBlocks][3]
  float* g_gen;              // [n][D]
  float* g_rnd;              // [n][D]
  float* g_edge;             // [E][D]
  float* de;                 // [n][ldde]: dL/de per hit
  int ldde;
  const int64_t* status;
};

hipError_t launch_blk_fwd(const BlkFwd& A, int M, int act, hipStream_t s, const etx_ctx* c);
hipError_t launch_blk_bwd(const BlkBwd& A, int M, int act, hipStream_t s, const etx_ctx* c);
hipError_t launch_wgrad(const Wgrad& A, int M, float* grad, hipStream_t s);
hipError_t launch_node_sum(int64_t n, int H, const int64_t* row_ptr, const float* a, const int64_t* col_ptr,
                           const int32_t* csc, const float* b, float* out, int add, const int64_t* status,
                           hipStream_t s, const etx_ctx* c);
hipError_t launch_edge_gather_add(int64_t E, int H, const int32_t* src, const int32_t* dst, const float* A,
                                  const float* B, float* out, const int64_t* status, hipStream_t s, const etx_ctx* c);
hipError_t launch_inputs(int64_t n, const float* x, const float* y, const float* z, float inv_r, float inv_z,
                         float* cart, float* cyl, const int64_t* status, hipStream_t s, const etx_ctx* c);
hipError_t launch_edge_labels(int64_t E, const int32_t* src, const int32_t* dst, const int32_t* succ,
                              const int32_t* succ2, uint8_t* lab, const int64_t* status, hipStream_t s,
                              const etx_ctx* c);
// score (may be null) receives sigmoid(z) of every row
hipError_t launch_focal(int64_t E, int H, const float* cls_out, const float* w2, const uint8_t* lab, float alpha,
                        float gamma, float* dlogit, float* dc, float* loss_part, float* loss_out, int slot,
                        const int64_t* status, hipStream_t s, float* score = nullptr);
hipError_t launch_adam(int64_t n, float* p, float* m, float* v, const float* g, float lr, int64_t step,
                       const int64_t* status, hipStream_t s, const etx_ctx* c);
hipError_t launch_hinge(const HingeArgs& A, int D, float* loss_out, hipStream_t s);

}  // namespace etx
