// Layout (in floats) of the per-kernel weight segments.  The host builds each
// segment once per context; a kernel copies its segment into LDS with one
// linear pass.  "perm(K, M)" is a K x M Linear weight permuted for the column
// layout of tile.hpp (K*M floats, M padded to a multiple of 32); "nat(K, M)"
// is the plain row-major [K][M] matrix; vectors are biases.
#pragma once
#include <stdint.h>

namespace etx {

// embedding: nat(3,W) b1[W] | per extra hidden layer: perm(W,W) b[W] | perm(W,16) bo[16]
struct SegEmb {
  int W, L;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return 3 * W; }
  __host__ __device__ constexpr int wh(int l) const { return 4 * W + (l - 1) * (W * W + W); }   // l = 1..L-1
  __host__ __device__ constexpr int bh(int l) const { return wh(l) + W * W; }
  __host__ __device__ constexpr int wo() const { return 4 * W + (L - 1) * (W * W + W); }
  __host__ __device__ constexpr int bo() const { return wo() + 16 * W; }
  __host__ __device__ constexpr int size() const { return bo() + 16; }
};

// node encoder: nat(3,H) b1[H] perm(H,H) b2[H] | edge-encoder products perm(H,H) (source) perm(H,H) (target)
struct SegNodeEnc {
  int H;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return 3 * H; }
  __host__ __device__ constexpr int w2() const { return 4 * H; }
  __host__ __device__ constexpr int b2() const { return 4 * H + H * H; }
  __host__ __device__ constexpr int ws() const { return 5 * H + H * H; }
  __host__ __device__ constexpr int wd() const { return 5 * H + 2 * H * H; }
  __host__ __device__ constexpr int size() const { return 5 * H + 3 * H * H; }
};

// edge encoder: b1[H] perm(H,H) b2[H]
struct SegEdgeEnc {
  int H;
  __host__ __device__ constexpr int b1() const { return 0; }
  __host__ __device__ constexpr int w2() const { return H; }
  __host__ __device__ constexpr int b2() const { return H + H * H; }
  __host__ __device__ constexpr int size() const { return 2 * H + H * H; }
};

// node net k: perm(3H,H) b1[H] perm(H,H) b2[H] | edge net k products perm(H,H) (source) perm(H,H) (target)
struct SegNode {
  int H;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return 3 * H * H; }
  __host__ __device__ constexpr int w2() const { return 3 * H * H + H; }
  __host__ __device__ constexpr int b2() const { return 4 * H * H + H; }
  __host__ __device__ constexpr int ws() const { return 4 * H * H + 2 * H; }
  __host__ __device__ constexpr int wd() const { return 5 * H * H + 2 * H; }
  __host__ __device__ constexpr int size() const { return 6 * H * H + 2 * H; }
};

// edge net k: perm(H,H) (edge part of layer 1) b1[H] perm(H,H) b2[H]
struct SegEdge {
  int H;
  __host__ __device__ constexpr int we() const { return 0; }
  __host__ __device__ constexpr int b1() const { return H * H; }
  __host__ __device__ constexpr int w2() const { return H * H + H; }
  __host__ __device__ constexpr int b2() const { return 2 * H * H + H; }
  __host__ __device__ constexpr int size() const { return 2 * H * H + 2 * H; }
};

// classifier: perm(H,H) b1[H] w2[H] b2 (padded to 4)
struct SegCls {
  int H;
  __host__ __device__ constexpr int w1() const { return 0; }
  __host__ __device__ constexpr int b1() const { return H * H; }
  __host__ __device__ constexpr int w2() const { return H * H + H; }
  __host__ __device__ constexpr int b2() const { return H * H + 2 * H; }
  __host__ __device__ constexpr int size() const { return H * H + 2 * H + 4; }
};

}  // namespace etx
