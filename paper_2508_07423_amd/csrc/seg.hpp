// Layout (in bytes) of the per-kernel weight segments.  The host builds each
// segment once per context and precision; a kernel copies its segment into LDS
// with one linear pass.  "perm(K, M)" is a K x M Linear weight permuted for
// the column layout of tile.hpp in the GEMM operand format (K*M*ES bytes,
// ES = 4 FP32, 2 BF16, 1 FP8; M padded to a multiple of 16); "nat(K, M)" is the
// plain row-major FP32 matrix; vectors are FP32 biases.  Every block starts on
// a 16-byte boundary.
#pragma once
#include <stdint.h>

namespace etx {

// embedding: nat(3,W) b1[W] | per extra hidden layer: perm(W,W) b[W] | perm(W,16) bo[16]
struct SegEmb {
  int W, L, ES;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return 12 * W; }
  __host__ __device__ constexpr int wh(int l) const { return 16 * W + (l - 1) * (W * W * ES + 4 * W); }  // l = 1..L-1
  __host__ __device__ constexpr int bh(int l) const { return wh(l) + W * W * ES; }
  __host__ __device__ constexpr int wo() const { return 16 * W + (L - 1) * (W * W * ES + 4 * W); }
  __host__ __device__ constexpr int bo() const { return wo() + 16 * W * ES; }
  __host__ __device__ constexpr int size() const { return bo() + 64; }
};

// node encoder: nat(3,H) b1[H] perm(H,H) b2[H] | edge-encoder products perm(H,H) (source) perm(H,H) (target)
struct SegNodeEnc {
  int H, ES;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return 12 * H; }
  __host__ __device__ constexpr int w2() const { return 16 * H; }
  __host__ __device__ constexpr int b2() const { return 16 * H + H * H * ES; }
  __host__ __device__ constexpr int ws() const { return 20 * H + H * H * ES; }
  __host__ __device__ constexpr int wd() const { return 20 * H + 2 * H * H * ES; }
  __host__ __device__ constexpr int size() const { return 20 * H + 3 * H * H * ES; }
};

// edge encoder: b1[H] perm(H,H) b2[H]
struct SegEdgeEnc {
  int H, ES;
  __host__ __device__ constexpr int b1() const { return 0; }
  __host__ __device__ constexpr int w2() const { return 4 * H; }
  __host__ __device__ constexpr int b2() const { return 4 * H + H * H * ES; }
  __host__ __device__ constexpr int size() const { return 8 * H + H * H * ES; }
};

// node net k: perm(3H,H) b1[H] perm(H,H) b2[H] | edge net k products perm(H,H) (source) perm(H,H) (target)
struct SegNode {
  int H, ES;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return 3 * H * H * ES; }
  __host__ __device__ constexpr int w2() const { return 3 * H * H * ES + 4 * H; }
  __host__ __device__ constexpr int b2() const { return 4 * H * H * ES + 4 * H; }
  __host__ __device__ constexpr int ws() const { return 4 * H * H * ES + 8 * H; }
  __host__ __device__ constexpr int wd() const { return 5 * H * H * ES + 8 * H; }
  __host__ __device__ constexpr int size() const { return 6 * H * H * ES + 8 * H; }
};

// edge net k: perm(H,H) (edge part of layer 1) b1[H] perm(H,H) b2[H]
struct SegEdge {
  int H, ES;
  __host__ __device__ constexpr int we() const { return 0; }
  __host__ __device__ constexpr int b1() const { return H * H * ES; }
  __host__ __device__ constexpr int w2() const { return H * H * ES + 4 * H; }
  __host__ __device__ constexpr int b2() const { return 2 * H * H * ES + 4 * H; }
  __host__ __device__ constexpr int size() const { return 2 * H * H * ES + 8 * H; }
};

// classifier: perm(H,H) b1[H] w2[H] (FP32) b2 (padded to 16 bytes)
struct SegCls {
  int H, ES;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return H * H * ES; }
  __host__ __device__ constexpr int w2() const { return H * H * ES + 4 * H; }
  __host__ __device__ constexpr int b2() const { return H * H * ES + 8 * H; }
  __host__ __device__ constexpr int size() const { return H * H * ES + 8 * H + 16; }
};

// Slots of the per-tensor scales (ctx->dev_scales): activations 0..63,
// weights 64..255; the same slots again from SC_I8 for the INT8 scales.
// Activation slots follow the oracle's numbering.
enum ScaleSlot {
  SC_EMB = 0,          // + l: input of embedding layer l (l >= 1)
  SC_GNN = 8,          // + Q_* below
  Q_NE2 = 0, Q_H = 1, Q_MO = 2, Q_MI = 3, Q_EE2 = 4, Q_NN2 = 5, Q_EN2 = 6, Q_E = 7,   // Q_E + k, k = 0..S
  SW = 64,             // weight scales
  SW_EMB = 64,         // + l
  SW_NE2 = 72, SW_EE1 = 73, SW_EE2 = 74, SW_CLS1 = 75,
  SW_STEP = 80,        // + 4k + {0: node L1, 1: node L2, 2: edge L1, 3: edge L2}
  SC_I8 = 256,         // INT8 scale set
  N_SCALES = 512
};

}  // namespace etx
