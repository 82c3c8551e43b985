// Column-tile MLP building blocks for CDNA4 (gfx950) MFMA.
//
// A wave evaluates a small MLP on a tile of 16 "columns" (hits or edges).
// Each Linear layer is computed transposed, Y^T = W^T X^T, with 16x16 MFMA
// output blocks so that every column is owned by four lanes:
//   lane l (0..63), lane group g = l / 16, column j = l % 16
//   accumulator register v (0..3) of output block mb holds output feature
//       16*mb + 4*g + v
// of column j.  We call this the column layout: register r = 4*mb + v of a
// lane holds feature phi(r, g) = 16*(r/4) + 4*g + r%4 of its column.  The same
// registers are directly the B operand of the next layer's MFMA (B[k][j] with
// k = phi(t, g) at K-step t), because the order of the K-sum is free: the A
// operand (weights) is stored pre-permuted by the host with the same phi, so
// layers chain without data movement.  A LayerNorm over a column is an
// in-register sum plus two exchanges (lanes l ^ 16 and l ^ 32).  A column of F
// features costs F/4 registers per lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace etx {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kCols = 16;  // columns per wave tile of the MLP kernels

__host__ __device__ constexpr int phi(int r, int g) { return 16 * (r / 4) + 4 * g + (r % 4); }

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int lane_group() { return (threadIdx.x & 63) >> 4; }
// The wave's index in its workgroup, as a wave-uniform (scalar) value: tile
// indices derived from it stay in scalar registers.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Load F features of a row-major [col][F] array into column layout (F/4 registers).
template <int F>
__device__ inline void load_cols(float* a, const float* __restrict__ row, bool valid) {
  const int g = lane_group();
#pragma unroll
  for (int c = 0; c < F / 16; ++c) {
    float4 v = valid ? *reinterpret_cast<const float4*>(row + 16 * c + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
    a[4 * c + 0] = v.x;
    a[4 * c + 1] = v.y;
    a[4 * c + 2] = v.z;
    a[4 * c + 3] = v.w;
  }
}

// Same, adding into the registers.
template <int F>
__device__ inline void add_cols(float* a, const float* __restrict__ row, bool valid) {
  const int g = lane_group();
  if (!valid) return;
#pragma unroll
  for (int c = 0; c < F / 16; ++c) {
    float4 v = *reinterpret_cast<const float4*>(row + 16 * c + 4 * g);
    a[4 * c + 0] += v.x;
    a[4 * c + 1] += v.y;
    a[4 * c + 2] += v.z;
    a[4 * c + 3] += v.w;
  }
}

template <int F>
__device__ inline void store_cols(float* __restrict__ row, const float* a, bool valid) {
  const int g = lane_group();
  if (!valid) return;
#pragma unroll
  for (int c = 0; c < F / 16; ++c)
    *reinterpret_cast<float4*>(row + 16 * c + 4 * g) = make_float4(a[4 * c], a[4 * c + 1], a[4 * c + 2], a[4 * c + 3]);
}

// Bias (row-major [F]) into column layout.
template <int F>
__device__ inline void bias_cols(float* a, const float* __restrict__ b) {
  const int g = lane_group();
#pragma unroll
  for (int c = 0; c < F / 16; ++c) {
    float4 v = *reinterpret_cast<const float4*>(b + 16 * c + 4 * g);
    a[4 * c + 0] = v.x;
    a[4 * c + 1] = v.y;
    a[4 * c + 2] = v.z;
    a[4 * c + 3] = v.w;
  }
}

// acc (column layout, M = 16*MB outputs) += W^T x for x in column layout with
// K inputs.  w holds the permuted weights:
//   w[(mb*(K/4) + t)*64 + lane] = W[phi(t, lane/16)][16*mb + lane%16].
template <int K, int MB>
__device__ inline void mfma_f32(float* acc, const float* x, const float* __restrict__ w) {
  const int lane = lane_id();
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mb][v] = acc[4 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 4; ++t) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[(mb * (K / 4) + t) * 64 + lane], x[t], c[mb], 0, 0, 0);
    // bound how far the scheduler hoists the LDS weight loads (register pressure)
    if (t % 4 == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = c[mb][v];
}

// The same product with the layer's weights held in registers for the
// whole kernel (wr[i] = w[i*64 + lane], i = mb*(K/4) + t): no LDS traffic
// and no waits inside the MFMA chain.
template <int K, int MB>
__device__ inline void load_wreg(float* wr, const float* __restrict__ w) {
  const int lane = lane_id();
#pragma unroll
  for (int i = 0; i < MB * (K / 4); ++i) wr[i] = w[i * 64 + lane];
}

template <int K, int MB>
__device__ inline void mfma_f32_reg(float* acc, const float* x, const float* wr) {
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mb][v] = acc[4 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 4; ++t)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[mb * (K / 4) + t], x[t], c[mb], 0, 0, 0);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = c[mb][v];
}

// BF16 operands, K-steps of 32: lane group g supplies registers 8t..8t+7.
//   w[(mb*(K/32) + t)*64 + lane][q] = W[phi(8t+q, lane/16)][16*mb + lane%16], q = 0..7.
template <int K, int MB>
__device__ inline void mfma_bf16(float* acc, const float* x, const bf16x8* __restrict__ w) {
  const int lane = lane_id();
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mb][v] = acc[4 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 32; ++t) {
    bf16x8 b;
#pragma unroll
    for (int q = 0; q < 8; ++q) b[q] = (__bf16)x[8 * t + q];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[(mb * (K / 32) + t) * 64 + lane], b, c[mb], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = c[mb][v];
}

// Same with the operand already in BF16: chunk t holds registers 8t .. 8t+7
// (low half first), the K-step's operand as it is.
template <int K, int MB>
__device__ inline void mfma_bf16_chunks(float* acc, const uint4* xr, const bf16x8* __restrict__ w) {
  const int lane = lane_id();
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mb][v] = acc[4 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 32; ++t) {
    const bf16x8 b = __builtin_bit_cast(bf16x8, xr[t]);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[(mb * (K / 32) + t) * 64 + lane], b, c[mb], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = c[mb][v];
}

// ---------------------------------------------------------------------------
// low-precision formats
// ---------------------------------------------------------------------------

// P_F32X: FP32 operands on the BF16 matrix cores, each operand split into
// three BF16 parts (below); FP32 everywhere else.  P_BF16M / P_FP8M: BF16 /
// FP8 GEMM operands with the node and edge state kept in FP32 between kernels
// (residual masters); P_BF16 / P_FP8 keep that state in the operand format.
// P_I8M: symmetric INT8 operands (real per-tensor scales), FP32 state.
enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2, P_F32X = 3, P_BF16M = 4, P_FP8M = 5, P_I8M = 6 };
// bytes per weight element of a GEMM in precision P (P_F32X: three BF16 planes)
template <int P>
struct PrecBytes {
  static constexpr int value = P == P_F32 ? 4 : (P == P_BF16 || P == P_BF16M) ? 2
                             : (P == P_FP8 || P == P_FP8M || P == P_I8M) ? 1 : 6;
};
// storage format of the state (edge encodings) in precision P
template <int P>
struct StorePrec { static constexpr int value = (P == P_BF16 || P == P_FP8) ? P : P_F32; };
// operand formats
template <int P>
constexpr bool kBf16Ops = P == P_BF16 || P == P_BF16M;
template <int P>
constexpr bool kFp8Ops = P == P_FP8 || P == P_FP8M;
template <int P>
constexpr bool kI8Ops = P == P_I8M;

// OCP FP8 E4M3 (bias 7, 3 mantissa bits, subnormals, max 448, no infinity),
// converted by the gfx950 instructions v_cvt_pk_fp8_f32 (round to nearest
// even) and v_cvt_f32_fp8.  The clamp keeps values beyond the largest finite
// code at +-448 (saturation).
__device__ inline float e4m3_clamp(float x) { return fminf(fmaxf(x, -448.f), 448.f); }

// four values -> four codes, value q in byte q
__device__ inline uint32_t e4m3_encode4(float a, float b, float c, float d) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(a), e4m3_clamp(b), 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(c), e4m3_clamp(d), lo, true);
}

__device__ inline uint32_t e4m3_encode(float x) { return e4m3_encode4(x, 0.f, 0.f, 0.f) & 0xffu; }

// byte Q of a word of codes -> value
template <int Q>
__device__ inline float e4m3_byte(uint32_t w) { return __builtin_amdgcn_cvt_f32_fp8((int)w, Q); }

__device__ inline float e4m3_decode(uint32_t c) { return e4m3_byte<0>(c); }

// Symmetric INT8 (thesis ch. 4 "Quantization"): code = clip(round(x / S),
// -127, 127) with round to nearest even (v_rndne_f32), value = S * code.  The
// caller passes x / S (as x * (1 / S)).
__device__ inline uint32_t i8_byte(float v) {
  return (uint32_t)(int)__builtin_rintf(fminf(fmaxf(v, -127.f), 127.f)) & 0xffu;
}
__device__ inline uint32_t i8_encode4(float a, float b, float c, float d) {
  return i8_byte(a) | (i8_byte(b) << 8) | (i8_byte(c) << 16) | (i8_byte(d) << 24);
}

__device__ inline uint32_t bf16_bits(float x) { return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// Node rows stored as BF16 (the low-precision runs keep node encodings so):
// lane group g holds features 16c + 4g .. 16c + 4g + 3, eight bytes per block.
template <int F>
__device__ inline void load_cols_bf16(float* a, const uint16_t* __restrict__ row, bool valid) {
  const int g = lane_group();
#pragma unroll
  for (int c = 0; c < F / 16; ++c) {
    const uint2 v = valid ? *reinterpret_cast<const uint2*>(row + 16 * c + 4 * g) : make_uint2(0u, 0u);
    a[4 * c + 0] = bf16_value(v.x & 0xffffu);
    a[4 * c + 1] = bf16_value(v.x >> 16);
    a[4 * c + 2] = bf16_value(v.y & 0xffffu);
    a[4 * c + 3] = bf16_value(v.y >> 16);
  }
}

template <int F>
__device__ inline void store_cols_bf16(uint16_t* __restrict__ row, const float* a, bool valid) {
  const int g = lane_group();
  if (!valid) return;
#pragma unroll
  for (int c = 0; c < F / 16; ++c)
    *reinterpret_cast<uint2*>(row + 16 * c + 4 * g) =
        make_uint2(bf16_bits(a[4 * c]) | (bf16_bits(a[4 * c + 1]) << 16), bf16_bits(a[4 * c + 2]) | (bf16_bits(a[4 * c + 3]) << 16));
}

// The values a BF16 store keeps (round to nearest even).
template <int F>
__device__ inline void round_bf16_cols(float* a) {
#pragma unroll
  for (int r = 0; r < F / 4; ++r) a[r] = bf16_value(bf16_bits(a[r]));
}

// FP8 operands, K-steps of 32: lane group g supplies registers 8t..8t+7 as
// codes of x * inv_s; w holds 8 codes per lane per step (same order as BF16).
// acc += out_scale * (W_q^T x_q).
// T0..T1 restricts the K-steps (one input block of a concatenated operand).
template <int K, int MB, int T0 = 0, int T1 = K / 32>
__device__ inline void mfma_fp8(float* acc, const float* x, const uint64_t* __restrict__ w, float inv_s,
                                float out_scale) {
  const int lane = lane_id();
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = T0; t < T1; ++t) {
    const float* xs = x + 8 * t;
    const uint64_t b = (uint64_t)e4m3_encode4(xs[0] * inv_s, xs[1] * inv_s, xs[2] * inv_s, xs[3] * inv_s) |
                       ((uint64_t)e4m3_encode4(xs[4] * inv_s, xs[5] * inv_s, xs[6] * inv_s, xs[7] * inv_s) << 32);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)w[(mb * (K / 32) + t) * 64 + lane], (long)b, c[mb], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = fmaf(out_scale, c[mb][v], acc[4 * mb + v]);
}

// Same with the operand already as FP8 codes: word c of a lane holds the codes
// of registers 4c .. 4c+3 (the stored edge encodings).
template <int K, int MB>
__device__ inline void mfma_fp8_codes(float* acc, const uint32_t* xw, const uint64_t* __restrict__ w, float out_scale) {
  const int lane = lane_id();
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < K / 32; ++t) {
    const uint64_t b = (uint64_t)xw[2 * t] | ((uint64_t)xw[2 * t + 1] << 32);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)w[(mb * (K / 32) + t) * 64 + lane], (long)b, c[mb], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = fmaf(out_scale, c[mb][v], acc[4 * mb + v]);
}

// INT8 operands, K-steps of 32 (the FP8 form's lane layout, 8 codes per lane
// per step): acc += out_scale * (W_q^T x_q), the integer products summed
// exactly in INT32 (|sum| <= K * 127^2 < 2^24, so the conversion is exact).
template <int K, int MB, int T0 = 0, int T1 = K / 32>
__device__ inline void mfma_i8(float* acc, const float* x, const uint64_t* __restrict__ w, float inv_s,
                               float out_scale) {
  static_assert(K * 127 * 127 < (1 << 24), "INT32 sums must convert to FP32 exactly");
  const int lane = lane_id();
  intx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = intx4{0, 0, 0, 0};
#pragma unroll
  for (int t = T0; t < T1; ++t) {
    const float* xs = x + 8 * t;
    const uint64_t b = (uint64_t)i8_encode4(xs[0] * inv_s, xs[1] * inv_s, xs[2] * inv_s, xs[3] * inv_s) |
                       ((uint64_t)i8_encode4(xs[4] * inv_s, xs[5] * inv_s, xs[6] * inv_s, xs[7] * inv_s) << 32);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)w[(mb * (K / 32) + t) * 64 + lane], (long)b, c[mb], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = fmaf(out_scale, (float)c[mb][v], acc[4 * mb + v]);
}

// FP32 product on the BF16 matrix cores.  Each FP32 value is split exactly
// into three BF16 parts, x = hi + mid + lo (hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid); both differences are exact in FP32, and lo is
// within 2^-25 |x| of the remainder); w holds the same parts of W as three
// consecutive BF16 planes in the BF16 layout.  The six products down to
// 2^-16 relative (lo*hi, hi*lo, mid*mid, mid*hi, hi*mid, hi*hi: BF16 x BF16
// products are exact in FP32) accumulate in FP32; the terms left out
// (mid*lo, lo*mid, lo*lo) are below 2^-23 relative together, the size of
// FP32 rounding.
__device__ inline void split3(const float* x, bf16x8& h, bf16x8& m, bf16x8& l) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const __bf16 bh = (__bf16)x[q];
    const float r = x[q] - (float)bh;
    const __bf16 bm = (__bf16)r;
    h[q] = bh;
    m[q] = bm;
    l[q] = (__bf16)(r - (float)bm);
  }
}

template <int K, int MB>
__device__ inline void mfma_split(float* acc, const float* x, const bf16x8* __restrict__ w) {
  constexpr int PLANE = MB * (K / 32) * 64;
  const int lane = lane_id();
  floatx4 c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mb][v] = acc[4 * mb + v];
#pragma unroll
  for (int t = 0; t < K / 32; ++t) {
    bf16x8 xh, xm, xl;
    split3(x + 8 * t, xh, xm, xl);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int i = (mb * (K / 32) + t) * 64 + lane;
      const bf16x8 wh = w[i], wm = w[PLANE + i], wl = w[2 * PLANE + i];
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, c[mb], 0, 0, 0);
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, c[mb], 0, 0, 0);
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm, xm, c[mb], 0, 0, 0);
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm, xh, c[mb], 0, 0, 0);
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xm, c[mb], 0, 0, 0);
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, c[mb], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[4 * mb + v] = c[mb][v];
}

// One Linear layer in precision P: acc += W^T x with weights w (permuted for
// P); FP8 and INT8 quantise x with inv_s and rescale the product by out_scale.
template <int P, int K, int MB>
__device__ inline void gemm(float* acc, const float* x, const void* w, float inv_s, float out_scale) {
  if constexpr (P == P_F32) {
    mfma_f32<K, MB>(acc, x, static_cast<const float*>(w));
  } else if constexpr (kBf16Ops<P>) {
    mfma_bf16<K, MB>(acc, x, static_cast<const bf16x8*>(w));
  } else if constexpr (P == P_F32X) {
    mfma_split<K, MB>(acc, x, static_cast<const bf16x8*>(w));
  } else if constexpr (kI8Ops<P>) {
    mfma_i8<K, MB>(acc, x, static_cast<const uint64_t*>(w), inv_s, out_scale);
  } else {
    mfma_fp8<K, MB>(acc, x, static_cast<const uint64_t*>(w), inv_s, out_scale);
  }
}

// Sum over the four lanes of a column (lanes l, l^16, l^32, l^48) with the
// gfx950 row swaps: permlane16_swap of a register with itself leaves each lane
// its own value in one result and its l^16 partner's in the other (which is
// which depends on the row), so their sum is s + s(l^16) in every lane;
// permlane32_swap does the same across the halves.  The additions are those
// of a butterfly through LDS permutes, in the same order and with the same
// bits, without the LDS round trip.  Called by the whole wave.
__device__ inline float col_sum(float s) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(s), __float_as_uint(s), false, false);
  s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// LayerNorm over the F features of each column (biased variance, eps 1e-5,
// no affine), then ReLU.  Two passes (mean, then squared deviations); the
// reciprocal square root is the hardware's (1 ulp; its argument is at least
// the epsilon, never subnormal) rather than a correctly rounded square root
// and division, which cost some thirty vector instructions per column.
template <int F>
__device__ inline void ln_relu(float* a) {
  float s = a[0];
#pragma unroll
  for (int r = 1; r < F / 4; ++r) s += a[r];
  const float mean = col_sum(s) * (1.0f / F);
  float q = 0.f;
#pragma unroll
  for (int r = 0; r < F / 4; ++r) {
    const float d = a[r] - mean;
    q = fmaf(d, d, q);
  }
  const float rstd = __builtin_amdgcn_rsqf(col_sum(q) * (1.0f / F) + 1e-5f);
#pragma unroll
  for (int r = 0; r < F / 4; ++r) a[r] = fmaxf((a[r] - mean) * rstd, 0.f);
}

// Copy n floats global -> LDS with 16-byte accesses (n multiple of 4, both aligned).
__device__ inline void stage(float* __restrict__ dst, const float* __restrict__ src, int n) {
  for (int i = threadIdx.x * 4; i < n; i += blockDim.x * 4)
    *reinterpret_cast<float4*>(dst + i) = *reinterpret_cast<const float4*>(src + i);
}

}  // namespace etx
