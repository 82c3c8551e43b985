// Column-tile MLP building blocks for CDNA4 (gfx950) MFMA.
//
// A wave evaluates a small MLP on a tile of 32 "columns" (hits or edges).  The
// product of one Linear layer is computed transposed, Y^T = W^T X^T, so that
// the 32x32 MFMA output block has one column per lane pair:
//   lane l (0..63), half h = l / 32, column j = l % 32
//   accumulator register v of output block mb holds output feature
//       32*mb + 8*(v/4) + 4*h + (v%4)
// of column j.  We call this the column layout: register r = 16*mb + v of a
// lane holds feature phi(r, h) of its column.  The same registers are directly
// the B operand of the next layer's MFMA (B[k][j] with k = phi(t, h) at K-step
// t), because the order of the K-sum is free: the A operand (weights) is
// stored pre-permuted by the host with the same phi, so layers chain without
// any data movement.  LayerNorm over a column is an in-register sum plus one
// exchange with lane l ^ 32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace etx {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__host__ __device__ constexpr int phi(int r, int h) {
  return 32 * (r / 16) + 8 * ((r % 16) / 4) + 4 * h + (r % 4);
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

// Load F features of a row-major [col][F] array into column layout (F/2 registers).
template <int F>
__device__ inline void load_cols(float* a, const float* __restrict__ row, bool valid) {
  const int h = lane_id() >> 5;
#pragma unroll
  for (int g = 0; g < F / 8; ++g) {
    float4 v = valid ? *reinterpret_cast<const float4*>(row + 8 * g + 4 * h) : make_float4(0.f, 0.f, 0.f, 0.f);
    a[4 * g + 0] = v.x;
    a[4 * g + 1] = v.y;
    a[4 * g + 2] = v.z;
    a[4 * g + 3] = v.w;
  }
}

// Same, adding into the registers.
template <int F>
__device__ inline void add_cols(float* a, const float* __restrict__ row, bool valid) {
  const int h = lane_id() >> 5;
  if (!valid) return;
#pragma unroll
  for (int g = 0; g < F / 8; ++g) {
    float4 v = *reinterpret_cast<const float4*>(row + 8 * g + 4 * h);
    a[4 * g + 0] += v.x;
    a[4 * g + 1] += v.y;
    a[4 * g + 2] += v.z;
    a[4 * g + 3] += v.w;
  }
}

template <int F>
__device__ inline void store_cols(float* __restrict__ row, const float* a, bool valid) {
  const int h = lane_id() >> 5;
  if (!valid) return;
#pragma unroll
  for (int g = 0; g < F / 8; ++g)
    *reinterpret_cast<float4*>(row + 8 * g + 4 * h) = make_float4(a[4 * g], a[4 * g + 1], a[4 * g + 2], a[4 * g + 3]);
}

// Bias (row-major [F]) into column layout.
template <int F>
__device__ inline void bias_cols(float* a, const float* __restrict__ b) {
  const int h = lane_id() >> 5;
#pragma unroll
  for (int r = 0; r < F / 2; ++r) a[r] = b[phi(r, h)];
}

// acc (column layout, M = 32*MB outputs) += W^T x for x in column layout with K
// inputs.  w holds the permuted weights: w[(mb*(K/2) + t)*64 + lane] =
// W[phi(t, lane/32)][32*mb + lane%32].
template <int K, int MB>
__device__ inline void mfma_f32(float* acc, const float* x, const float* __restrict__ w) {
  const int lane = lane_id();
  floatx16 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) c[mb][v] = acc[16 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 2; ++t) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[(mb * (K / 2) + t) * 64 + lane], x[t], c[mb], 0, 0, 0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[16 * mb + v] = c[mb][v];
}

// BF16 operands: w holds 8 bf16 per lane per K-step of 16:
// w[((mb*(K/16) + t)*64 + lane)] = W[phi(8t+q, lane/32)][32*mb + lane%32], q = 0..7.
template <int K, int MB>
__device__ inline void mfma_bf16(float* acc, const float* x, const bf16x8* __restrict__ w) {
  const int lane = lane_id();
  floatx16 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) c[mb][v] = acc[16 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 16; ++t) {
    bf16x8 b;
#pragma unroll
    for (int q = 0; q < 8; ++q) b[q] = (__bf16)x[8 * t + q];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[(mb * (K / 16) + t) * 64 + lane], b, c[mb], 0, 0, 0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[16 * mb + v] = c[mb][v];
}

// LayerNorm over the F features of each column (biased variance, eps 1e-5,
// no affine), then ReLU.  Two passes (mean, then squared deviations).
template <int F>
__device__ inline void ln_relu(float* a) {
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < F / 2; ++r) s += a[r];
  s += __shfl_xor(s, 32);
  const float mean = s * (1.0f / F);
  float q = 0.f;
#pragma unroll
  for (int r = 0; r < F / 2; ++r) {
    const float d = a[r] - mean;
    q = fmaf(d, d, q);
  }
  q += __shfl_xor(q, 32);
  const float rstd = 1.0f / sqrtf(q * (1.0f / F) + 1e-5f);
#pragma unroll
  for (int r = 0; r < F / 2; ++r) a[r] = fmaxf((a[r] - mean) * rstd, 0.f);
}

template <int F>
__device__ inline void relu(float* a) {
#pragma unroll
  for (int r = 0; r < F / 2; ++r) a[r] = fmaxf(a[r], 0.f);
}

// Copy n floats global -> LDS with 16-byte accesses (n multiple of 4, both aligned).
__device__ inline void stage(float* __restrict__ dst, const float* __restrict__ src, int n) {
  for (int i = threadIdx.x * 4; i < n; i += blockDim.x * 4)
    *reinterpret_cast<float4*>(dst + i) = *reinterpret_cast<const float4*>(src + i);
}

}  // namespace etx
