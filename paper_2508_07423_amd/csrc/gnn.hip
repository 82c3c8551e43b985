// Interaction network (thesis ch. 8 "Graph Neural Network and Classifiers").
//
//   h0   = MLP(x/R_s, y/R_s, z/Z_s)                         node encoder
//   e0   = MLP([h0_src, h0_dst])                            edge encoder
//   step k:  mo_l = sum_{l->j} e_lj,  mi_l = sum_{i->l} e_il   (message)
//            h <- h + MLP_node_k([h, mo, mi])
//            e <- e + MLP_edge_k([e, h_src, h_dst])           (updated h)
//   logit = Linear(H->1)(Block(H->H)(e)),  score = sigmoid(logit)
// with MLP = Block(.->H) then Block(H->H), Block(x) = ReLU(LayerNorm(x W + b)).
//
// The first layer of every edge-side MLP is split by input block: [a, b, c] W
// = a W_a + b W_b + c W_c.  The node-side products (h W_src, h W_dst) are
// computed once per node in the node kernels and gathered per edge, so the
// per-edge work is one H x H product per layer.  Messages are atomic-free
// segmented sums: the out-sums (runs of the source-major edge list) are
// reduced in registers by the kernels that write the edge encodings, the
// in-sums gathered through the (dst, src)-ordered CSC permutation.
//
// Every MLP kernel is instantiated for the GEMM operand precision P (FP32,
// BF16, FP8-E4M3 with per-tensor power-of-two scales).  Accumulation,
// LayerNorm, residual node encodings, the message sums and the scores stay
// FP32.  The edge encodings, the largest tensor, are stored in the operand
// format (FP8 with the per-step scale of the stored tensor), which is also
// the operand the next edge-net product reads.
#include <type_traits>

#include "internal.hpp"
#include "seg.hpp"
#include "tile.hpp"

namespace etx {

namespace {

__device__ inline void atomic_amax(float* slot, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(slot), __float_as_uint(fabsf(v)));
}

template <int N>
__device__ inline void observe(float* calib, int slot, const float* a, bool valid) {
  if (!calib) return;
  float m = 0.f;
#pragma unroll
  for (int r = 0; r < N; ++r) m = fmaxf(m, fabsf(a[r]));
  if (valid) atomic_amax(calib + slot, m);
}

struct GnnArgs {
  int64_t n_hits;
  const float* x;
  const float* y;
  const float* z;
  float inv_r, inv_z;
  const int64_t* row_ptr;   // [n_hits+1]; row_ptr[n_hits] = edge count
  const int64_t* col_ptr;
  const int32_t* csc;
  const int32_t* src;
  const int32_t* dst;
  const char* seg;          // weight segment of the kernel
  const char* seg2;         // classifier segment (final edge step)
  const char* seg3;         // edge-side products: W_src then W_dst of edge net k, layer 1
  int seg_bytes, seg2_bytes, seg3_bytes;
  float* h;                 // [n_hits][H] node encodings (BF16 bits in BF16 and FP8 runs)
  float* ps;                // [n_hits][H] h W_src (source product)
  float* pd;                // [n_hits][H] h W_dst (target product)
  float* msg;               // [n_hits][2H] (out-sum, in-sum)
  void* e;                  // [edges][H] edge encodings in the operand format
  float* opart;             // [2 x edge tiles][H] out-sum partials of source rows that cross a tile
  float* score;             // [edges]
  float* calib;             // amax observers (calibration runs, FP32 only)
  const float* sc;          // per-tensor scales (seg.hpp ScaleSlot)
  int step;
  int xcd_map;              // 1: logical workgroup ids contiguous per XCD
  int keep_final;           // 1: the final edge step also stores e_S (the triplet classifiers' input)
  const int64_t* status;
};

// Workgroups of a launch are dispatched to the eight XCDs in turn (b -> b % 8).
// With the remap the workgroups of one XCD hold a contiguous range of logical
// ids, so at any time an XCD works on neighbouring tiles of one region of the
// batch and its own L2 holds the node rows those tiles gather; without it every
// XCD sees every region in flight.  The map is a bijection on [0, grid), so
// which tiles run is unchanged.
constexpr int kXcds = 8;
__device__ inline int64_t logical_block(const GnnArgs& A) {
  const int64_t G = gridDim.x, b = blockIdx.x;
  if (!A.xcd_map || G % kXcds != 0) return b;
  return (b % kXcds) * (G / kXcds) + b / kXcds;
}

__device__ inline void stage_bytes(char* dst, const char* src, int n) {
  stage(reinterpret_cast<float*>(dst), reinterpret_cast<const float*>(src), n / 4);
}

// scale of an activation slot and of a weight slot
__device__ inline float asc(const GnnArgs& A, int q) { return A.sc[SC_GNN + q]; }
__device__ inline float wsc(const GnnArgs& A, int s) { return A.sc[s]; }

// Node encodings h: FP32 rows, except in the compact-state BF16 and FP8 runs
// (P_BF16, P_FP8), which keep node state like edge state in low precision:
// BF16 rows (round to nearest even).  A store rounds the registers first, so
// that what a kernel goes on computing with is what the next kernel reads.
template <int P>
constexpr bool kHalfH = P == P_BF16 || P == P_FP8;

template <int H, int P>
__device__ inline void load_h(float* x, const GnnArgs& A, int64_t col, bool valid) {
  if constexpr (kHalfH<P>)
    load_cols_bf16<H>(x, reinterpret_cast<const uint16_t*>(A.h) + col * H, valid);
  else
    load_cols<H>(x, A.h + col * H, valid);
}

template <int H, int P>
__device__ inline void store_h(const GnnArgs& A, int64_t col, float* o, bool valid) {
  if constexpr (kHalfH<P>) {
    round_bf16_cols<H>(o);
    store_cols_bf16<H>(reinterpret_cast<uint16_t*>(A.h) + col * H, o, valid);
  } else {
    store_cols<H>(A.h + col * H, o, valid);
  }
}

// --------------------------------------------------------------------------
// edge-encoding rows in the operand format
// --------------------------------------------------------------------------

// Stored edge-row layout.  Lane group g of a column holds registers
// r = 0 .. H/4-1 (features phi(r, g)); in the operand format these are
// LB = H/4 * ES bytes, kept in the row as contiguous 16-byte chunks: chunk q
// of group g at byte 64 q + 16 g (rows of FP8 at H = 32 have 8 bytes per
// group, at byte 8 g).  Every load or store instruction of a wave then moves
// 64 contiguous bytes per column, and a chunk of BF16 or FP8 codes is
// directly the MFMA operand of one 32-wide K-step.  FP32 rows are the plain
// feature order.
template <int P, int H>
struct ELayout {
  static constexpr int ES = PrecBytes<StorePrec<P>::value>::value;
  static constexpr int LB = H / 4 * ES;                 // bytes per lane group
  static constexpr int NQ = LB >= 16 ? LB / 16 : 1;     // 16-byte chunks per lane group
  static constexpr int ROW = H * ES;                    // bytes per row
  // feature stored at byte b of a row
  __host__ __device__ static constexpr int feature(int b) {
    return LB >= 16 ? phi((b / 64) * (16 / ES) + (b % 16) / ES, (b % 64) / 16) : phi((b % LB) / ES, b / LB);
  }
};

template <int P, int H>
struct RawE { uint4 v[ELayout<P, H>::NQ]; };

// Non-temporal stores of edge rows (the edge encoder's: its writes then do
// not push the gathered node-product rows out of L2; measured 17.8 -> 16.1 ms
// at c2.  In the edge updates, non-temporal loads and stores of the rows cut
// the read traffic but raised the write traffic and did not pay.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline void store_stream4(char* p, uint4 v) {
  __builtin_nontemporal_store(u32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<u32x4*>(p));
}
__device__ inline void store_stream2(char* p, uint2 v) {
  __builtin_nontemporal_store(u32x2{v.x, v.y}, reinterpret_cast<u32x2*>(p));
}

// col must address a stored row (callers clamp the tail of the last tile).
template <int P, int H>
__device__ inline void fetch_e(RawE<P, H>& r, const void* e, int64_t col) {
  using L = ELayout<P, H>;
  const int g = lane_group();
  const char* row = static_cast<const char*>(e) + col * L::ROW;
  if constexpr (L::LB >= 16) {
#pragma unroll
    for (int q = 0; q < L::NQ; ++q) r.v[q] = *reinterpret_cast<const uint4*>(row + 64 * q + 16 * g);
  } else {
    const uint2 h = *reinterpret_cast<const uint2*>(row + L::LB * g);
    r.v[0] = make_uint4(h.x, h.y, 0u, 0u);
  }
}

// 32-bit word i of a lane group's bytes
template <int P, int H>
__device__ inline uint32_t raw_word(const RawE<P, H>& r, int i) {
  const uint4 c = r.v[i / 4];
  return (i % 4) == 0 ? c.x : (i % 4) == 1 ? c.y : (i % 4) == 2 ? c.z : c.w;
}

// Register values of the row (FP8: decoded times `scale`).
template <int P, int H>
__device__ inline void decode_e(float* ef, const RawE<P, H>& r, float scale) {
#pragma unroll
  for (int x = 0; x < H / 4; ++x) {
    if constexpr (StorePrec<P>::value == P_F32) {
      ef[x] = __uint_as_float(raw_word<P, H>(r, x));
    } else if constexpr (P == P_BF16) {
      const uint32_t w = raw_word<P, H>(r, x / 2);
      ef[x] = bf16_value((x % 2) ? (w >> 16) : (w & 0xffffu));
    } else {
      const uint32_t w = raw_word<P, H>(r, x / 4);
      const float v = (x % 4) == 0 ? e4m3_byte<0>(w) : (x % 4) == 1 ? e4m3_byte<1>(w)
                    : (x % 4) == 2 ? e4m3_byte<2>(w) : e4m3_byte<3>(w);
      ef[x] = v * scale;
    }
  }
}

// The source and target rows of an edge, gathered ahead: FP32 node-product
// rows, or (HB) the BF16 node encodings as stored, four features (8 bytes)
// per lane group and 16-feature block.
template <int H, bool HB = false>
struct NodeRows { float4 s[H / 16], d[H / 16]; };
template <int H>
struct NodeRows<H, true> { uint2 s[H / 16], d[H / 16]; };

template <int H, bool HB = false>
__device__ inline void fetch_rows(NodeRows<H, HB>& n, const float* ps, const float* pd, int src, int dst) {
  const int g = lane_group();
  if constexpr (HB) {
    const uint2* rs = reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(ps) + (int64_t)src * H);
    const uint2* rd = reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(pd) + (int64_t)dst * H);
#pragma unroll
    for (int c = 0; c < H / 16; ++c) {
      n.s[c] = rs[4 * c + g];
      n.d[c] = rd[4 * c + g];
    }
  } else {
    const float4* rs = reinterpret_cast<const float4*>(ps + (int64_t)src * H);
    const float4* rd = reinterpret_cast<const float4*>(pd + (int64_t)dst * H);
#pragma unroll
    for (int c = 0; c < H / 16; ++c) {
      n.s[c] = rs[4 * c + g];
      n.d[c] = rd[4 * c + g];
    }
  }
}

// a += source row, then a += target row (a fixed order for every pipeline depth)
template <int H>
__device__ inline void add_rows(float* a, const NodeRows<H>& n) {
#pragma unroll
  for (int c = 0; c < H / 16; ++c) {
    a[4 * c + 0] += n.s[c].x; a[4 * c + 1] += n.s[c].y; a[4 * c + 2] += n.s[c].z; a[4 * c + 3] += n.s[c].w;
  }
#pragma unroll
  for (int c = 0; c < H / 16; ++c) {
    a[4 * c + 0] += n.d[c].x; a[4 * c + 1] += n.d[c].y; a[4 * c + 2] += n.d[c].z; a[4 * c + 3] += n.d[c].w;
  }
}

// a gathered row in column layout (the B operand of the next product)
template <int H>
__device__ inline void rows_cols(float* x, const float4 (&r)[H / 16]) {
#pragma unroll
  for (int c = 0; c < H / 16; ++c) {
    x[4 * c + 0] = r[c].x; x[4 * c + 1] = r[c].y; x[4 * c + 2] = r[c].z; x[4 * c + 3] = r[c].w;
  }
}
template <int H>
__device__ inline void rows_cols(float* x, const uint2 (&r)[H / 16]) {
#pragma unroll
  for (int c = 0; c < H / 16; ++c) {
    x[4 * c + 0] = bf16_value(r[c].x & 0xffffu); x[4 * c + 1] = bf16_value(r[c].x >> 16);
    x[4 * c + 2] = bf16_value(r[c].y & 0xffffu); x[4 * c + 3] = bf16_value(r[c].y >> 16);
  }
}

// One gathered row's product with a BF16 weight block (a zero start): the
// stored BF16 features of 32-feature step t are the MFMA operand as they are
// (blocks 2t and 2t+1 in register order), the bits mfma_bf16 would pack.
template <int H>
__device__ inline void row_product_bf16(float* q, const uint2 (&r)[H / 16], const bf16x8* __restrict__ w) {
  uint4 xr[H / 32];
#pragma unroll
  for (int t = 0; t < H / 32; ++t) xr[t] = make_uint4(r[2 * t].x, r[2 * t].y, r[2 * t + 1].x, r[2 * t + 1].y);
#pragma unroll
  for (int i = 0; i < H / 4; ++i) q[i] = 0.f;
  mfma_bf16_chunks<H, H / 16>(q, xr, w);
}

// Software pipeline over a wave's tiles (tile, tile + stride, ...): with
// depth 0 every tile loads its own operands; depth 1 issues the next tile's
// edge indices and edge row before the current tile's arithmetic; depth 2
// keeps the indices two tiles ahead and also issues the next tile's
// node-product gathers early.  The arithmetic is the same at every depth.
// Columns past the last edge (the tail of the last tile, tiles beyond the
// end) read the last edge instead, so every load is unconditional; their
// results are never stored.
// Tile indices: the column's source and target, and the sources of the edges
// just before and just after the tile (-1 past either end of the list).
struct TileIdx {
  int s, d, before, after;
};

// HB: the gathered node rows are BF16 node encodings (edge-side products in
// the low-precision runs), else FP32 product rows.
template <int P, int H, int PIPE, bool HB = false>
struct EdgeFeed {
  const int32_t* src;
  const int32_t* dst;
  const void* e;
  const float* ps;
  const float* pd;
  int64_t E, stride;
  int lane16;
  TileIdx i1{0, 0, -1, -1};     // indices of the next tile (depth 2)
  TileIdx i0{0, 0, -1, -1};     // indices of the fetched tile
  RawE<P, H> raw;
  using Rows = NodeRows<H, HB>;
  Rows rows;
  bool want_e;

  __device__ int64_t col(int64_t t) const { return t * kCols + lane16; }
  __device__ int64_t clamped(int64_t t) const { return min(col(t), E - 1); }
  __device__ void idx(int64_t t, TileIdx& x) const {
    const int64_t c = clamped(t), c0 = t * kCols;
    x.s = src[c];
    x.d = dst[c];
    const int b = src[max(min(c0 - 1, E - 1), (int64_t)0)], a = src[min(c0 + kCols, E - 1)];
    x.before = c0 > 0 ? b : -1;
    x.after = c0 + kCols < E ? a : -1;
  }
  // operands of tile t into the feed registers
  __device__ void fetch(int64_t t) {
    if constexpr (PIPE == 2) {
      i0 = i1;
      idx(t + stride, i1);
    } else {
      idx(t, i0);
    }
    if (want_e) fetch_e<P, H>(raw, e, clamped(t));
    if constexpr (PIPE == 2) fetch_rows<H, HB>(rows, ps, pd, i0.s, i0.d);
  }
  __device__ void start(int64_t t) {
    if constexpr (PIPE == 2) idx(t, i1);
    if constexpr (PIPE >= 1) fetch(t);
  }
  // hand out tile t's operands and indices (key: the column's source node,
  // -1 past the last edge) and issue tile t + stride's
  __device__ void next(int64_t t, RawE<P, H>& r, Rows& n, TileIdx& x, int& key) {
    const bool v = col(t) < E;
    if constexpr (PIPE == 0) {
      fetch(t);
      r = raw;
      fetch_rows<H, HB>(n, ps, pd, i0.s, i0.d);
      x = i0;
    } else if constexpr (PIPE == 1) {
      r = raw;
      fetch_rows<H, HB>(n, ps, pd, i0.s, i0.d);
      x = i0;
      fetch(t + stride);
    } else {
      r = raw;
      n = rows;
      x = i0;
      fetch(t + stride);
    }
    key = v ? x.s : -1;
  }
};

// Store an edge row in the operand format.  q (if not null) receives the
// values as stored (FP8: decoded times `scale`), the terms of the message sums.
template <int P, int H, bool NT = false>
__device__ inline void store_e(void* e, int64_t col, const float* o, bool valid, float inv_scale, float scale = 1.f,
                               float* q = nullptr) {
  using L = ELayout<P, H>;
  const int g = lane_group();
  char* row = static_cast<char*>(e) + col * L::ROW;
  uint32_t w[L::NQ * 4];
  if constexpr (StorePrec<P>::value == P_F32) {
#pragma unroll
    for (int x = 0; x < H / 4; ++x) w[x] = __float_as_uint(o[x]);
    if (q) {
#pragma unroll
      for (int x = 0; x < H / 4; ++x) q[x] = o[x];
    }
  } else if constexpr (P == P_BF16) {
#pragma unroll
    for (int x = 0; x < H / 8; ++x) {
      const uint32_t b0 = bf16_bits(o[2 * x]), b1 = bf16_bits(o[2 * x + 1]);
      w[x] = b0 | (b1 << 16);
      if (q) {
        q[2 * x] = bf16_value(b0);
        q[2 * x + 1] = bf16_value(b1);
      }
    }
  } else {
#pragma unroll
    for (int x = 0; x < H / 16; ++x) {
      w[x] = e4m3_encode4(o[4 * x] * inv_scale, o[4 * x + 1] * inv_scale, o[4 * x + 2] * inv_scale,
                          o[4 * x + 3] * inv_scale);
      if (q) {
        q[4 * x + 0] = e4m3_byte<0>(w[x]) * scale;
        q[4 * x + 1] = e4m3_byte<1>(w[x]) * scale;
        q[4 * x + 2] = e4m3_byte<2>(w[x]) * scale;
        q[4 * x + 3] = e4m3_byte<3>(w[x]) * scale;
      }
    }
  }
  if (!valid) return;
  if constexpr (L::LB >= 16) {
#pragma unroll
    for (int c = 0; c < L::NQ; ++c) {
      const uint4 v = make_uint4(w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]);
      if constexpr (NT) store_stream4(row + 64 * c + 16 * g, v);
      else *reinterpret_cast<uint4*>(row + 64 * c + 16 * g) = v;
    }
  } else {
    const uint2 v = make_uint2(w[0], w[1]);
    if constexpr (NT) store_stream2(row + L::LB * g, v);
    else *reinterpret_cast<uint2*>(row + L::LB * g) = v;
  }
}

// --------------------------------------------------------------------------
// out-sums fused into the edge kernels
// --------------------------------------------------------------------------
// Edges are source-major, so the out-sum of a node is the sum over one
// contiguous run of edge columns.  A wave tile (16 consecutive edges, one per
// lane of each 16-lane DPP row) reduces its runs with a segmented scan along
// the row; the last column of each run then holds the run's sum.  A run that
// lies inside the tile is the node's whole row and is written straight to the
// message buffer; a run cut by a tile boundary goes to the tile's partial
// slots (0: the run that began before the tile, 1: the run that continues
// past it), which the message kernel adds up in tile order.

// Row shifts within the 16-lane DPP rows.  Lanes whose source is outside
// the row read -2 (keys; 0 for the values of the scan below); the shifts run
// with the whole wave active, never under a lane-dependent branch, since a
// lane whose source lane is inactive would read the fallback value too.
template <int N>
__device__ inline int row_shr_i(int v) {
  return __builtin_amdgcn_update_dpp(-2, v, 0x110 + N, 0xf, 0xf, false);
}
__device__ inline int row_shl1_i(int v) { return __builtin_amdgcn_update_dpp(-2, v, 0x101, 0xf, 0xf, false); }

// Inclusive segmented sums along the 16 columns of a tile, N registers per
// lane; key is non-decreasing in the column.  Level i adds, to each column,
// the value 2^i columns to its left when both belong to the same run:
// v = fma(v[column - 2^i], m_i, v) with m_i = 1 or 0, one v_fmac_f32 whose
// first source is read through a DPP row shift (lanes whose source lies
// outside the 16-lane row read 0).  The compiler keeps a DPP move apart from
// a multiply-add, two instructions, and copies registers at the joins of
// per-level branches, so the four levels are written out as one block.  A
// level whose mask is zero in every lane (no run of the wave's tiles that
// long) would add exact zeros to finite values: it is skipped on its ballot
// (wave-uniform scalar branches inside the block).  A DPP read needs two
// wait states after a vector write of its source and five after a vector
// write of EXEC: the leading s_nop 4 covers both; inside the block a
// register is read at least N instructions after it was written.
#define ETX_FMAC_SHR(i, D, M) \
  "v_fmac_f32_dpp %" #i ", %" #i ", %" #M " row_shr:" #D " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
#define ETX_LEVEL8(D, M)                                                                                     \
  ETX_FMAC_SHR(0, D, M) ETX_FMAC_SHR(1, D, M) ETX_FMAC_SHR(2, D, M) ETX_FMAC_SHR(3, D, M) ETX_FMAC_SHR(4, D, M) \
  ETX_FMAC_SHR(5, D, M) ETX_FMAC_SHR(6, D, M) ETX_FMAC_SHR(7, D, M)
#define ETX_LEVEL16(D, M)                                                                                      \
  ETX_LEVEL8(D, M) ETX_FMAC_SHR(8, D, M) ETX_FMAC_SHR(9, D, M) ETX_FMAC_SHR(10, D, M) ETX_FMAC_SHR(11, D, M)     \
  ETX_FMAC_SHR(12, D, M) ETX_FMAC_SHR(13, D, M) ETX_FMAC_SHR(14, D, M) ETX_FMAC_SHR(15, D, M)
#define ETX_SKIP(B, L) "s_cmp_eq_u64 %" #B ", 0\n\ts_cbranch_scc1 " L "%=\n\t"
#define ETX_SCAN(LEVEL, M1, M2, M4, M8, B1, B2, B4, B8)                                                      \
  "s_nop 4\n\t" ETX_SKIP(B1, ".Lscan2_") LEVEL(1, M1) ".Lscan2_%=:\n\t" ETX_SKIP(B2, ".Lscan4_") LEVEL(2, M2)   \
  ".Lscan4_%=:\n\t" ETX_SKIP(B4, ".Lscan8_") LEVEL(4, M4) ".Lscan8_%=:\n\t" ETX_SKIP(B8, ".Lscan_end_")        \
  LEVEL(8, M8) ".Lscan_end_%=:\n\t"

template <int N>
__device__ inline void seg_scan_cols(float* v, int key) {
  static_assert(N == 8 || N == 16, "hidden size 32 or 64");
  const int j = lane_id() & 15;
  const int k1 = row_shr_i<1>(key), k2 = row_shr_i<2>(key), k4 = row_shr_i<4>(key), k8 = row_shr_i<8>(key);
  const float m1 = ((j >= 1) & (k1 == key)) ? 1.f : 0.f, m2 = ((j >= 2) & (k2 == key)) ? 1.f : 0.f;
  const float m4 = ((j >= 4) & (k4 == key)) ? 1.f : 0.f, m8 = ((j >= 8) & (k8 == key)) ? 1.f : 0.f;
  const uint64_t b1 = __ballot(m1 != 0.f), b2 = __ballot(m2 != 0.f), b4 = __ballot(m4 != 0.f),
                 b8 = __ballot(m8 != 0.f);
  if constexpr (N == 8) {
    asm volatile(ETX_SCAN(ETX_LEVEL8, 8, 9, 10, 11, 12, 13, 14, 15)
                 : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
                 : "v"(m1), "v"(m2), "v"(m4), "v"(m8), "s"(b1), "s"(b2), "s"(b4), "s"(b8)
                 : "scc");
  } else {
    asm volatile(ETX_SCAN(ETX_LEVEL16, 16, 17, 18, 19, 20, 21, 22, 23)
                 : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
                   "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]),
                   "+v"(v[15])
                 : "v"(m1), "v"(m2), "v"(m4), "v"(m8), "s"(b1), "s"(b2), "s"(b4), "s"(b8)
                 : "scc");
  }
}
#undef ETX_SCAN
#undef ETX_SKIP
#undef ETX_LEVEL16
#undef ETX_LEVEL8
#undef ETX_FMAC_SHR

// q: stored values of this lane's column; key: its source node (-1 past the
// last edge); x.before / x.after: sources of the neighbouring edges of the
// tile.  Called by the whole wave.
template <int H>
__device__ inline void out_sums(const GnnArgs& A, int64_t tile, const TileIdx& x, int key, float* q) {
  const int key0 = __builtin_amdgcn_readlane(key, 0), key15 = __builtin_amdgcn_readlane(key, 15);
  seg_scan_cols<H / 4>(q, key);
  const int knext = row_shl1_i(key);
  const bool last = ((lane_id() & 15) == 15) | (knext != key);
  if (key >= 0 && last) {
    const bool before = key == key0 && x.before == key, after = key == key15 && x.after == key;
    float* dst = (!before && !after) ? A.msg + (int64_t)key * 2 * H : A.opart + (tile * 2 + (before ? 0 : 1)) * H;
    store_cols<H>(dst, q, true);
  }
}

// The same out-sums through LDS (H = 64: one lane per feature).  The tile is
// transposed into the wave's buffer (row f holds feature f of the 16 columns,
// rows padded to 20 floats so that the writes of a half-wave hit distinct
// banks); lane f then adds its row along the columns, closing a run wherever
// the (wave-uniform) source changes, and writes each run's sum as one
// coalesced 256-byte row.  Both orders are fixed.  (With hidden size 32 and
// the short rows of trained networks, many runs per tile, the DPP scan is the
// faster form.)
constexpr int kOutRow = 20;                     // floats per transposed feature row
constexpr int kOutBufFloats = 64 * kOutRow;     // per wave

template <int H>
__device__ inline void out_sums_lds(const GnnArgs& A, int64_t tile, const TileIdx& x, int key, const float* q,
                                    float* buf) {
  static_assert(H == 64, "one lane per feature");
  const int lane = lane_id(), j = lane & 15, g = lane_group();
#pragma unroll
  for (int r = 0; r < H / 4; ++r) buf[phi(r, g) * kOutRow + j] = q[r];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  float v[16];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float4 t = *reinterpret_cast<const float4*>(buf + lane * kOutRow + 4 * c);
    v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
  }
  int k[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) k[c] = __builtin_amdgcn_readlane(key, c);
  const int before = __builtin_amdgcn_readfirstlane(x.before), after = __builtin_amdgcn_readfirstlane(x.after);
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    acc += v[c];
    if (c == 15 || k[c + 1 < 16 ? c + 1 : 15] != k[c]) {
      if (k[c] >= 0) {
        const bool b = k[c] == k[0] && before == k[c], a = c == 15 && after == k[c];
        float* dst = (!b && !a) ? A.msg + (int64_t)k[c] * 2 * H : A.opart + (tile * 2 + (b ? 0 : 1)) * H;
        dst[lane] = acc;
      }
      acc = 0.f;
    }
  }
  // the next tile's writes must not overtake this tile's reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// --------------------------------------------------------------------------
// node encoder (+ edge-encoder source/target products)
// --------------------------------------------------------------------------
// FP32 node kernels hold up to 98 KiB of weights in LDS: one 16-wave workgroup
// per CU; the low-precision segments are 2-4x smaller and run 8-wave groups.
template <int P>
struct NodeThreads { static constexpr int value = P == P_F32 ? 1024 : 512; };

// NP: also write the edge encoder's node products (else the edge encoder forms
// them from the gathered rows of h).
template <int H, int P, bool NP>
__global__ __launch_bounds__(NodeThreads<P>::value) void k_node_encode(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float lds[];
  char* w = reinterpret_cast<char*>(lds);
  stage_bytes(w, A.seg, A.seg_bytes);
  __syncthreads();
  constexpr SegNodeEnc S{H, PrecBytes<P>::value};
  const int lane = lane_id(), g = lane_group(), wave = wave_id(), nw = blockDim.x >> 6;
  const float s_ne2 = asc(A, Q_NE2), s_h = asc(A, Q_H);
  const float o_ne2 = s_ne2 * wsc(A, SW_NE2), o_h = s_h * wsc(A, SW_EE1);
  const int64_t ntiles = (A.n_hits + kCols - 1) / kCols;
  for (int64_t tile = logical_block(A) * nw + wave; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < A.n_hits;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
    if (valid) {
      v0 = A.x[col] * A.inv_r;
      v1 = A.y[col] * A.inv_r;
      v2 = A.z[col] * A.inv_z;
    }
    float a[H / 4];
    const float* w1 = reinterpret_cast<const float*>(w + S.w1());
    const float* b1 = reinterpret_cast<const float*>(w + S.b1());
#pragma unroll
    for (int r = 0; r < H / 4; ++r) {
      const int f = phi(r, g);
      float acc = v0 * w1[f];
      acc = fmaf(v1, w1[H + f], acc);
      acc = fmaf(v2, w1[2 * H + f], acc);
      a[r] = acc + b1[f];
    }
    ln_relu<H>(a);
    observe<H / 4>(A.calib, SC_GNN + Q_NE2, a, valid);
    float hh[H / 4];
    bias_cols<H>(hh, reinterpret_cast<const float*>(w + S.b2()));
    gemm<P, H, H / 16>(hh, a, w + S.w2(), 1.0f / s_ne2, o_ne2);
    ln_relu<H>(hh);
    store_h<H, P>(A, col, hh, valid);
    observe<H / 4>(A.calib, SC_GNN + Q_H, hh, valid);
    if constexpr (NP) {
      float q[H / 4];
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<P, H, H / 16>(q, hh, w + S.ws(), 1.0f / s_h, o_h);
      store_cols<H>(A.ps + col * H, q, valid);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<P, H, H / 16>(q, hh, w + S.wd(), 1.0f / s_h, o_h);
      store_cols<H>(A.pd + col * H, q, valid);
    }
  }
}

// --------------------------------------------------------------------------
// edge encoder
// --------------------------------------------------------------------------
// OL (H = 64): out-sums through an LDS transpose instead of the DPP scan; the
// wave buffers follow the weight segment in LDS.
// GH: the node products of layer 1 are formed here from the gathered rows of
// h (the node encoder's weights, precision and order: the same bits), and the
// node encoder writes none.
template <int H, int P, int PIPE, bool OL, bool GH>
__global__ __launch_bounds__(512) void k_edge_encode(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float lds[];
  char* w = reinterpret_cast<char*>(lds);
  stage_bytes(w, A.seg, A.seg_bytes);
  const char* wp = w + A.seg_bytes;                    // W_src, W_dst (GH)
  const int off = A.seg_bytes + (GH ? A.seg3_bytes : 0);
  if (GH) stage_bytes(w + A.seg_bytes, A.seg3, A.seg3_bytes);
  __syncthreads();
  constexpr SegEdgeEnc S{H, PrecBytes<P>::value};
  const int lane = lane_id(), wave = wave_id(), nw = blockDim.x >> 6;
  const float s_ee2 = asc(A, Q_EE2), o_ee2 = s_ee2 * wsc(A, SW_EE2);
  const float s_e0 = asc(A, Q_E + 0), inv_e0 = 1.0f / s_e0;
  const int64_t E = A.row_ptr[A.n_hits];
  const int64_t ntiles = (E + kCols - 1) / kCols;
  const int64_t stride = (int64_t)gridDim.x * nw;
  EdgeFeed<P, H, PIPE, GH && kHalfH<P>> feed{A.src, A.dst, nullptr, GH ? A.h : A.ps, GH ? A.h : A.pd, E, stride, lane & 15};
  feed.want_e = false;
  int64_t tile = logical_block(A) * nw + wave;
  if (tile < ntiles) feed.start(tile);
  for (; tile < ntiles; tile += stride) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < E;
    RawE<P, H> unused;
    typename decltype(feed)::Rows rows;
    TileIdx ti;
    int key;
    feed.next(tile, unused, rows, ti, key);
    float a[H / 4];
    bias_cols<H>(a, reinterpret_cast<const float*>(w + S.b1()));
    if constexpr (GH && P == P_BF16) {
      float q[H / 4];
      row_product_bf16<H>(q, rows.s, reinterpret_cast<const bf16x8*>(wp));
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
      row_product_bf16<H>(q, rows.d, reinterpret_cast<const bf16x8*>(wp + H * H * 2));
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
    } else if constexpr (GH) {
      constexpr int PP = P == P_F32X ? P_F32 : P;
      const float s_h = asc(A, Q_H), o_h = s_h * wsc(A, SW_EE1);
      float x[H / 4], q[H / 4];
      rows_cols<H>(x, rows.s);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<PP, H, H / 16>(q, x, wp, 1.0f / s_h, o_h);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
      rows_cols<H>(x, rows.d);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<PP, H, H / 16>(q, x, wp + H * H * PrecBytes<PP>::value, 1.0f / s_h, o_h);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
    } else {
      add_rows<H>(a, rows);
    }
    ln_relu<H>(a);
    observe<H / 4>(A.calib, SC_GNN + Q_EE2, a, valid);
    float o[H / 4];
    bias_cols<H>(o, reinterpret_cast<const float*>(w + S.b2()));
    gemm<P, H, H / 16>(o, a, w + S.w2(), 1.0f / s_ee2, o_ee2);
    ln_relu<H>(o);
    observe<H / 4>(A.calib, SC_GNN + Q_E, o, valid);
    store_e<P, H, true>(A.e, col, o, valid, inv_e0, s_e0, o);
    if constexpr (OL)
      out_sums_lds<H>(A, tile, ti, key, o, reinterpret_cast<float*>(w + off) + wave * kOutBufFloats);
    else
      out_sums<H>(A, tile, ti, key, o);
  }
}

// --------------------------------------------------------------------------
// messages: the out-sum from the edge kernels' tile partials, the in-sum
// through the CSC permutation.  A node is handled by one lane group as wide
// as a stored edge row (each lane reads 16 bytes of it), so a wave serves
// several nodes at once and needs no cross-lane reduction; the additions run
// in CSC order.
// --------------------------------------------------------------------------
template <int P>
__device__ inline void add_chunk(float* acc, uint4 v) {
  constexpr int FPL = 16 / PrecBytes<P>::value;
  if constexpr (P == P_F32) {
    acc[0] += __uint_as_float(v.x); acc[1] += __uint_as_float(v.y);
    acc[2] += __uint_as_float(v.z); acc[3] += __uint_as_float(v.w);
  } else if constexpr (P == P_BF16) {
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[2 * i] += bf16_value(u[i] & 0xffffu);
      acc[2 * i + 1] += bf16_value(u[i] >> 16);
    }
  } else {
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[4 * i + 0] += e4m3_byte<0>(u[i]);
      acc[4 * i + 1] += e4m3_byte<1>(u[i]);
      acc[4 * i + 2] += e4m3_byte<2>(u[i]);
      acc[4 * i + 3] += e4m3_byte<3>(u[i]);
    }
  }
  (void)FPL;
}

template <int H, int P, int U>
__global__ __launch_bounds__(256) void k_segsum(GnnArgs A) {
  if (A.status[0] != 0) return;
  constexpr int ES = PrecBytes<P>::value;
  constexpr int FPL = 16 / ES;         // features per lane of a stored edge row (16-byte chunks)
  constexpr int LPR = H / FPL;         // lanes per node: one lane group reads a whole row
  constexpr int NPW = 64 / LPR;        // nodes per wave
  constexpr int OPL = H / LPR;         // out-sum features per lane
  const int lane = lane_id(), fl = lane % LPR, sg = lane / LPR, wave = threadIdx.x >> 6;
  const char* eb = static_cast<const char*>(A.e);
  const float scale = P == P_FP8 ? asc(A, Q_E + A.step) : 1.0f;
  const int64_t stride = (int64_t)gridDim.x * 4 * NPW;
  for (int64_t node = (logical_block(A) * 4 + wave) * NPW + sg; node - sg < A.n_hits; node += stride) {
    const bool live = node < A.n_hits;
    float* out = A.msg + node * 2 * H;
    // out-sum: a source row inside one edge tile was written whole by the edge
    // kernel; a longer row is its tile partials, first tile's slot 1 then
    // slot 0 of each later tile
    const int64_t rb = live ? A.row_ptr[node] : 0, re = live ? A.row_ptr[node + 1] : 0;
    const int64_t cb = live ? A.col_ptr[node] : 0, ce = live ? A.col_ptr[node + 1] : 0;   // issued with rb, re
    // the first in-edge ids load with the out-sum's partials
    int id[U];
#pragma unroll
    for (int u = 0; u < U; ++u) id[u] = cb + u < ce ? A.csc[cb + u] : -1;
    const int64_t t0 = rb / kCols, t1 = re > rb ? (re - 1) / kCols : t0;
    if (live && (re == rb || t1 > t0)) {
      float mo[OPL];
#pragma unroll
      for (int x = 0; x < OPL; ++x) mo[x] = 0.f;
      for (int64_t i = 0; re > rb && i <= t1 - t0; ++i) {
        const float* prow = A.opart + ((t0 + i) * 2 + (i == 0 ? 1 : 0)) * H + fl * OPL;
#pragma unroll
        for (int x = 0; x < OPL; x += 4) {
          const float4 v = *reinterpret_cast<const float4*>(prow + x);
          mo[x] += v.x; mo[x + 1] += v.y; mo[x + 2] += v.z; mo[x + 3] += v.w;
        }
      }
#pragma unroll
      for (int x = 0; x < OPL; x += 4)
        *reinterpret_cast<float4*>(out + fl * OPL + x) = make_float4(mo[x], mo[x + 1], mo[x + 2], mo[x + 3]);
    }
    // in-sum through the CSC permutation, U rows in flight per node
    float mi[FPL];
#pragma unroll
    for (int x = 0; x < FPL; ++x) mi[x] = 0.f;
    for (int64_t t = cb; t < ce; t += U) {
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        v[u] = id[u] >= 0 ? *reinterpret_cast<const uint4*>(eb + ((int64_t)id[u] * H + fl * FPL) * ES)
                          : make_uint4(0u, 0u, 0u, 0u);
      // the next ids load while these rows are in flight
#pragma unroll
      for (int u = 0; u < U; ++u) id[u] = t + U + u < ce ? A.csc[t + U + u] : -1;
#pragma unroll
      for (int u = 0; u < U; ++u) add_chunk<P>(mi, v[u]);
    }
    if (live) {
      // value x of chunk fl is the feature stored at byte 16 fl + x ES; runs of
      // four values are four consecutive features
#pragma unroll
      for (int x = 0; x < FPL; x += 4)
        *reinterpret_cast<float4*>(out + H + ELayout<P, H>::feature(16 * fl + x * ES)) =
            make_float4(mi[x] * scale, mi[x + 1] * scale, mi[x + 2] * scale, mi[x + 3] * scale);
    }
  }
}

// The messages of the node tile's columns, gathered in the node kernel
// itself (the fused form of k_segsum, same sums in the same order): lane
// group g of a column holds features phi(r, g), which are exactly its chunks
// of every stored edge row, so the in-sum needs no rearrangement; the out-sum
// comes from the edge kernel's whole-row write or its tile partials.
// Rows of in-edges in flight per node (register budget).
template <int H, int P>
constexpr int kGatherU = (StorePrec<P>::value == P_F32 && H == 64) ? 1 : 4;

// A node's message indices: its CSR and CSC ranges and its first in-edge ids.
template <int H, int P>
struct MsgIdx {
  int64_t rb = 0, re = 0, cb = 0, ce = 0;
  int id0[kGatherU<H, P>];
};

// All index loads of a node at once (nothing here depends on another load
// but the ids on the CSC range), so that they can be issued a tile ahead.
template <int H, int P>
__device__ inline void fetch_msg_idx(const GnnArgs& A, int64_t node, bool valid, MsgIdx<H, P>& m) {
  constexpr int U = kGatherU<H, P>;
  m.rb = m.re = m.cb = m.ce = 0;
  if (valid) {
    m.rb = A.row_ptr[node];
    m.re = A.row_ptr[node + 1];
    m.cb = A.col_ptr[node];
    m.ce = A.col_ptr[node + 1];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) m.id0[u] = m.cb + u < m.ce ? A.csc[m.cb + u] : -1;
}

// Messages of a node gathered in the node kernel: the out-sum from the edge
// kernels' tile partials (as k_segsum), the in-sum over the CSC rows in CSC
// order, so the sums are bit-identical to k_segsum's.
template <int H, int P>
__device__ inline void gather_messages(const GnnArgs& A, int64_t node, bool valid, const MsgIdx<H, P>& m, float* mo,
                                       float* mi) {
  constexpr int U = kGatherU<H, P>;
#pragma unroll
  for (int r = 0; r < H / 4; ++r) mo[r] = mi[r] = 0.f;
  if (!valid) return;
  const int64_t rb = m.rb, re = m.re, cb = m.cb, ce = m.ce;
  if (re > rb) {
    const int64_t t0 = rb / kCols, t1 = (re - 1) / kCols;
    if (t0 == t1) {
      load_cols<H>(mo, A.msg + node * 2 * H, true);
    } else {
      for (int64_t i = 0; i <= t1 - t0; ++i) add_cols<H>(mo, A.opart + ((t0 + i) * 2 + (i == 0 ? 1 : 0)) * H, true);
    }
  }
  int id[U];
#pragma unroll
  for (int u = 0; u < U; ++u) id[u] = m.id0[u];
  for (int64_t t = cb; t < ce; t += U) {
    RawE<P, H> raw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (id[u] >= 0) fetch_e<P, H>(raw[u], A.e, id[u]);
      else
#pragma unroll
        for (int q = 0; q < ELayout<P, H>::NQ; ++q) raw[u].v[q] = make_uint4(0u, 0u, 0u, 0u);
    }
    // the next ids load while these rows are in flight
#pragma unroll
    for (int u = 0; u < U; ++u) id[u] = t + U + u < ce ? A.csc[t + U + u] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float v[H / 4];
      decode_e<P, H>(v, raw[u], 1.0f);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) mi[r] += v[r];
    }
  }
  if constexpr (P == P_FP8) {
    const float scale = asc(A, Q_E + A.step);
#pragma unroll
    for (int r = 0; r < H / 4; ++r) mi[r] *= scale;
  }
}

// --------------------------------------------------------------------------
// node update k (+ edge net k source/target products)
// --------------------------------------------------------------------------
// FUSE: the messages are gathered here (k_segsum is not launched).
// NP: also write the node products h W_src and h W_dst of edge net k (else
// the edge kernel forms them from the gathered rows of h).
template <int H, int P, bool FUSE, bool NP>
__global__ __launch_bounds__(NodeThreads<P>::value) void k_node_step(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float lds[];
  char* w = reinterpret_cast<char*>(lds);
  stage_bytes(w, A.seg, A.seg_bytes);
  __syncthreads();
  constexpr SegNode S{H, PrecBytes<P>::value};
  const int lane = lane_id(), wave = wave_id(), nw = blockDim.x >> 6;
  const int k = A.step;
  const float s_h = asc(A, Q_H), s_mo = asc(A, Q_MO), s_mi = asc(A, Q_MI), s_nn2 = asc(A, Q_NN2);
  const float w1s = wsc(A, SW_STEP + 4 * k), w2s = wsc(A, SW_STEP + 4 * k + 1), wes = wsc(A, SW_STEP + 4 * k + 2);
  const int64_t ntiles = (A.n_hits + kCols - 1) / kCols;
  const int64_t stride = (int64_t)gridDim.x * nw;
  // with fused messages the next tile's message indices load a tile ahead
  MsgIdx<H, P> mnext;
  int64_t tile = logical_block(A) * nw + wave;
  if constexpr (FUSE) {
    const int64_t c0 = tile * kCols + (lane & 15);
    fetch_msg_idx<H, P>(A, c0, tile < ntiles && c0 < A.n_hits, mnext);
  }
  for (; tile < ntiles; tile += stride) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < A.n_hits;
    float x[3 * H / 4];
    load_h<H, P>(x, A, col, valid);
    if constexpr (FUSE) {
      const MsgIdx<H, P> m = mnext;
      const int64_t cn = (tile + stride) * kCols + (lane & 15);
      fetch_msg_idx<H, P>(A, cn, tile + stride < ntiles && cn < A.n_hits, mnext);
      gather_messages<H, P>(A, col, valid, m, x + H / 4, x + H / 2);
    } else {
      load_cols<H>(x + H / 4, A.msg + col * 2 * H, valid);
      load_cols<H>(x + H / 2, A.msg + col * 2 * H + H, valid);
    }
    observe<H / 4>(A.calib, SC_GNN + Q_H, x, valid);
    observe<H / 4>(A.calib, SC_GNN + Q_MO, x + H / 4, valid);
    observe<H / 4>(A.calib, SC_GNN + Q_MI, x + H / 2, valid);
    float a[H / 4];
    bias_cols<H>(a, reinterpret_cast<const float*>(w + S.b1()));
    if constexpr (kFp8Ops<P>) {
      // the three input blocks carry their own activation scales
      const uint64_t* w1 = reinterpret_cast<const uint64_t*>(w + S.w1());
      mfma_fp8<3 * H, H / 16, 0, H / 32>(a, x, w1, 1.0f / s_h, s_h * w1s);
      mfma_fp8<3 * H, H / 16, H / 32, 2 * H / 32>(a, x, w1, 1.0f / s_mo, s_mo * w1s);
      mfma_fp8<3 * H, H / 16, 2 * H / 32, 3 * H / 32>(a, x, w1, 1.0f / s_mi, s_mi * w1s);
    } else if constexpr (kI8Ops<P>) {
      const uint64_t* w1 = reinterpret_cast<const uint64_t*>(w + S.w1());
      mfma_i8<3 * H, H / 16, 0, H / 32>(a, x, w1, 1.0f / s_h, s_h * w1s);
      mfma_i8<3 * H, H / 16, H / 32, 2 * H / 32>(a, x, w1, 1.0f / s_mo, s_mo * w1s);
      mfma_i8<3 * H, H / 16, 2 * H / 32, 3 * H / 32>(a, x, w1, 1.0f / s_mi, s_mi * w1s);
    } else {
      gemm<P, 3 * H, H / 16>(a, x, w + S.w1(), 1.f, 1.f);
    }
    ln_relu<H>(a);
    observe<H / 4>(A.calib, SC_GNN + Q_NN2, a, valid);
    float o[H / 4];
    bias_cols<H>(o, reinterpret_cast<const float*>(w + S.b2()));
    gemm<P, H, H / 16>(o, a, w + S.w2(), 1.0f / s_nn2, s_nn2 * w2s);
    ln_relu<H>(o);
#pragma unroll
    for (int r = 0; r < H / 4; ++r) o[r] += x[r];
    store_h<H, P>(A, col, o, valid);
    observe<H / 4>(A.calib, SC_GNN + Q_H, o, valid);
    if constexpr (NP) {
      float q[H / 4];
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<P, H, H / 16>(q, o, w + S.ws(), 1.0f / s_h, s_h * wes);
      store_cols<H>(A.ps + col * H, q, valid);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<P, H, H / 16>(q, o, w + S.wd(), 1.0f / s_h, s_h * wes);
      store_cols<H>(A.pd + col * H, q, valid);
    }
  }
}

// --------------------------------------------------------------------------
// edge update k; the last step also runs the classifier and writes scores
// --------------------------------------------------------------------------
// WR (FP32 only): both H x H weight matrices stay in registers for the whole
// persistent loop instead of being read from LDS by every MFMA.  OL as in the
// edge encoder (steps before the last).  GH: the node-product terms of layer 1
// are formed here, W_src h_src and W_dst h_dst on the gathered rows of h, and
// the node kernel writes no products; it trades 2H^2 multiply-adds per edge for
// the node kernel's product rows (written once, gathered per edge), which pays
// when edges per node are few and the matrix cores are fast (BF16, FP8).
template <int H, bool FINAL, int P, int PIPE, bool WR, bool OL, bool GH>
__global__ __launch_bounds__(512) void k_edge_step(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float lds[];
  char* w = reinterpret_cast<char*>(lds);
  constexpr int ES = PrecBytes<P>::value;
  constexpr SegEdge S{H, ES};
  constexpr SegCls C{H, ES};
  static_assert(!(GH && WR), "edge-side products use the LDS weights");
  stage_bytes(w, A.seg, A.seg_bytes);
  const char* wp = w + A.seg_bytes;                    // W_src, W_dst (GH)
  const int off = A.seg_bytes + (GH ? A.seg3_bytes : 0);
  if (GH) stage_bytes(w + A.seg_bytes, A.seg3, A.seg3_bytes);
  if (FINAL) stage_bytes(w + off, A.seg2, A.seg2_bytes);
  __syncthreads();
  const char* wc = w + off;
  const int lane = lane_id(), g = lane_group(), wave = wave_id(), nw = blockDim.x >> 6;
  const int k = A.step;
  const float s_e = asc(A, Q_E + k), s_en2 = asc(A, Q_EN2), s_next = asc(A, Q_E + k + 1);
  const float w1s = wsc(A, SW_STEP + 4 * k + 2), w2s = wsc(A, SW_STEP + 4 * k + 3), wcs = wsc(A, SW_CLS1);
  const int64_t E = A.row_ptr[A.n_hits];
  const int64_t ntiles = (E + kCols - 1) / kCols;
  const int64_t stride = (int64_t)gridDim.x * nw;
  EdgeFeed<P, H, PIPE, GH && kHalfH<P>> feed{A.src, A.dst, A.e, GH ? A.h : A.ps, GH ? A.h : A.pd, E, stride, lane & 15};
  feed.want_e = true;
  static_assert(!WR || P == P_F32, "register-resident weights are FP32 only");
  float wr_e[WR ? H * H / 64 : 1], wr_2[WR ? H * H / 64 : 1];
  if constexpr (WR) {
    load_wreg<H, H / 16>(wr_e, reinterpret_cast<const float*>(w + S.we()));
    load_wreg<H, H / 16>(wr_2, reinterpret_cast<const float*>(w + S.w2()));
  }
  int64_t tile = logical_block(A) * nw + wave;
  if (tile < ntiles) feed.start(tile);
  for (; tile < ntiles; tile += stride) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < E;
    RawE<P, H> raw;
    typename decltype(feed)::Rows rows;
    TileIdx ti;
    int key;
    feed.next(tile, raw, rows, ti, key);
    // layer 1: b1 + W_e e (the stored operand as it is), then the gathered
    // h W_src and h W_dst rows
    float a[H / 4];
    bias_cols<H>(a, reinterpret_cast<const float*>(w + S.b1()));
    if constexpr (P == P_FP8) {
      mfma_fp8_codes<H, H / 16>(a, reinterpret_cast<const uint32_t*>(raw.v), reinterpret_cast<const uint64_t*>(w + S.we()),
                                s_e * w1s);
    } else if constexpr (P == P_BF16) {
      mfma_bf16_chunks<H, H / 16>(a, raw.v, reinterpret_cast<const bf16x8*>(w + S.we()));
    } else {
      float ef[H / 4];
      decode_e<P, H>(ef, raw, s_e);
      if constexpr (WR)
        mfma_f32_reg<H, H / 16>(a, ef, wr_e);
      else
        gemm<P, H, H / 16>(a, ef, w + S.we(), 1.0f / s_e, s_e * w1s);   // scales: FP8 operands only
    }
    if constexpr (GH && P == P_BF16) {
      // BF16: the stored rows of h are the MFMA operands as they are
      float q[H / 4];
      row_product_bf16<H>(q, rows.s, reinterpret_cast<const bf16x8*>(wp));
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
      row_product_bf16<H>(q, rows.d, reinterpret_cast<const bf16x8*>(wp + H * H * 2));
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
    } else if constexpr (GH) {
      // the node kernel's products, formed the same way (its precision, its
      // weights, a zero start) from the rows of h and added in the same order:
      // the same bits as gathering them
      constexpr int PP = P == P_F32X ? P_F32 : P;
      const float s_h = asc(A, Q_H);
      float x[H / 4], q[H / 4];
      rows_cols<H>(x, rows.s);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<PP, H, H / 16>(q, x, wp, 1.0f / s_h, s_h * w1s);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
      rows_cols<H>(x, rows.d);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
      gemm<PP, H, H / 16>(q, x, wp + H * H * PrecBytes<PP>::value, 1.0f / s_h, s_h * w1s);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) a[r] += q[r];
    } else {
      add_rows<H>(a, rows);
    }
    ln_relu<H>(a);
    observe<H / 4>(A.calib, SC_GNN + Q_EN2, a, valid);
    float o[H / 4];
    bias_cols<H>(o, reinterpret_cast<const float*>(w + S.b2()));
    if constexpr (WR)
      mfma_f32_reg<H, H / 16>(o, a, wr_2);
    else
      gemm<P, H, H / 16>(o, a, w + S.w2(), 1.0f / s_en2, s_en2 * w2s);
    ln_relu<H>(o);
    {
      float e[H / 4];
      decode_e<P, H>(e, raw, s_e);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) o[r] += e[r];
    }
    observe<H / 4>(A.calib, SC_GNN + Q_E + k + 1, o, valid);
    if (!FINAL) {
      store_e<P, H>(A.e, col, o, valid, 1.0f / s_next, s_next, o);
      if constexpr (OL)
        out_sums_lds<H>(A, tile, ti, key, o, reinterpret_cast<float*>(w + off) + wave * kOutBufFloats);
      else
        out_sums<H>(A, tile, ti, key, o);
    } else {
      if (A.keep_final) store_e<P, H>(A.e, col, o, valid, 1.0f / s_next, s_next);
      // classifier on the final edge encodings (quantised like a stored e_S)
      float c[H / 4];
      bias_cols<H>(c, reinterpret_cast<const float*>(wc + C.b1()));
      gemm<P, H, H / 16>(c, o, wc + C.w1(), 1.0f / s_next, s_next * wcs);
      ln_relu<H>(c);
      const float* w2 = reinterpret_cast<const float*>(wc + C.w2());
      float dot = 0.f;
#pragma unroll
      for (int r = 0; r < H / 4; ++r) dot = fmaf(c[r], w2[phi(r, g)], dot);
      dot = col_sum(dot);
      const float logit = dot + reinterpret_cast<const float*>(wc + C.b2())[0];
      if (valid && g == 0) A.score[col] = 1.0f / (1.0f + expf(-logit));
    }
  }
}

}  // namespace

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

static GnnArgs gnn_args(const RunArgs& a) {
  const etx_ctx* c = a.ctx;
  GnnArgs A{};
  A.n_hits = a.hits.n_hits;
  A.x = a.hits.x;
  A.y = a.hits.y;
  A.z = a.hits.z;
  A.inv_r = 1.0f / c->cfg.r_scale_mm;
  A.inv_z = 1.0f / c->cfg.z_scale_mm;
  A.row_ptr = reinterpret_cast<const int64_t*>(a.ws + a.L.row_ptr);
  A.col_ptr = reinterpret_cast<const int64_t*>(a.ws + a.L.col_ptr);
  A.csc = reinterpret_cast<const int32_t*>(a.ws + a.L.csc);
  A.src = a.out.src;
  A.dst = a.out.dst;
  A.h = reinterpret_cast<float*>(a.ws + a.L.h);
  A.ps = reinterpret_cast<float*>(a.ws + a.L.ps);
  A.pd = reinterpret_cast<float*>(a.ws + a.L.pd);
  A.msg = reinterpret_cast<float*>(a.ws + a.L.msg);
  A.e = a.ws + a.L.e;
  A.opart = reinterpret_cast<float*>(a.ws + a.L.opart);
  A.score = a.out.score;
  A.calib = a.calibrate ? reinterpret_cast<float*>(a.ws + a.L.calib) : nullptr;
  A.sc = c->dev_scales + (a.prec == P_I8M ? SC_I8 : 0);   // the INT8 scale set
  A.xcd_map = a.ctx->xcd_map;
  A.keep_final = a.keep_final_e ? 1 : 0;
  A.status = a.out.status;
  return A;
}

static int node_threads(int prec) { return prec == P_F32 ? 1024 : 512; }

static unsigned node_grid(const RunArgs& a, int per_cu) {
  int64_t tiles = (a.hits.n_hits + kCols - 1) / kCols;
  int64_t waves = node_threads(a.prec) / 64;
  // low-precision node kernels run two 8-wave groups per CU for each FP32 group
  if (a.prec != P_F32) per_cu *= 2;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + waves - 1) / waves, (int64_t)a.ctx->n_cu * per_cu));
}

static const char* seg_ptr(const RunArgs& a, int64_t off) {
  return static_cast<const char*>(a.ctx->seg_base[kSegPrec[a.prec]]) + off;
}

#define DISPATCH_HP(H_, P_, ...)                                            \
  switch ((H_) * 8 + (P_)) {                                                \
    case 32 * 8 + 0: { constexpr int H = 32, P = 0; __VA_ARGS__; } break;  \
    case 32 * 8 + 1: { constexpr int H = 32, P = 1; __VA_ARGS__; } break;  \
    case 32 * 8 + 2: { constexpr int H = 32, P = 2; __VA_ARGS__; } break;  \
    case 32 * 8 + 4: { constexpr int H = 32, P = 4; __VA_ARGS__; } break;  \
    case 32 * 8 + 5: { constexpr int H = 32, P = 5; __VA_ARGS__; } break;  \
    case 32 * 8 + 6: { constexpr int H = 32, P = 6; __VA_ARGS__; } break;  \
    case 64 * 8 + 0: { constexpr int H = 64, P = 0; __VA_ARGS__; } break;  \
    case 64 * 8 + 1: { constexpr int H = 64, P = 1; __VA_ARGS__; } break;  \
    case 64 * 8 + 2: { constexpr int H = 64, P = 2; __VA_ARGS__; } break;  \
    case 64 * 8 + 4: { constexpr int H = 64, P = 4; __VA_ARGS__; } break;  \
    case 64 * 8 + 5: { constexpr int H = 64, P = 5; __VA_ARGS__; } break;  \
    case 64 * 8 + 6: { constexpr int H = 64, P = 6; __VA_ARGS__; } break;  \
    default: return hipErrorInvalidValue;                                   \
  }

hipError_t launch_node_encode(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  const WeightMap& m = a.ctx->wmap[kSegPrec[a.prec]];
  A.seg = seg_ptr(a, m.node_enc);
  A.seg_bytes = SegNodeEnc{Hh, kPrecBytes[a.prec]}.size();
  unsigned grid = node_grid(a, a.ctx->node_wg_per_cu);
  if (a.ctx->edge_products) {
    DISPATCH_HP(Hh, a.prec, hipLaunchKernelGGL((k_node_encode<H, P, false>), dim3(grid), dim3(node_threads(P)), A.seg_bytes, a.stream, A));
  } else {
    DISPATCH_HP(Hh, a.prec, hipLaunchKernelGGL((k_node_encode<H, P, true>), dim3(grid), dim3(node_threads(P)), A.seg_bytes, a.stream, A));
  }
  return hipGetLastError();
}

// The edge-kernel instantiation for a run-time launch schedule (also used to
// set the LDS attribute of every instantiation once).
template <int H, int P>
static const void* edge_encode_kernel(int pipe, bool ol, bool gh) {
  auto pick = [&](auto PI) -> const void* {
    constexpr int pi = decltype(PI)::value;
    if constexpr (H == 64) {
      if (ol) return gh ? reinterpret_cast<const void*>(k_edge_encode<H, P, pi, true, true>)
                        : reinterpret_cast<const void*>(k_edge_encode<H, P, pi, true, false>);
    }
    return gh ? reinterpret_cast<const void*>(k_edge_encode<H, P, pi, false, true>)
              : reinterpret_cast<const void*>(k_edge_encode<H, P, pi, false, false>);
  };
  switch (pipe) {
    case 0: return pick(std::integral_constant<int, 0>{});
    case 2: return pick(std::integral_constant<int, 2>{});
    default: return pick(std::integral_constant<int, 1>{});
  }
}

template <int H, int P>
static const void* edge_step_kernel(bool fin, int pipe, bool wr, bool ol, bool gh) {
  auto pick_o = [&](auto F, auto PI, auto WRC) -> const void* {
    constexpr bool f = decltype(F)::value, wv = decltype(WRC)::value;
    constexpr int pi = decltype(PI)::value;
    if constexpr (!wv) {
      if (gh) {
        if constexpr (H == 64 && !f) {
          if (ol) return reinterpret_cast<const void*>(k_edge_step<H, f, P, pi, false, true, true>);
        }
        return reinterpret_cast<const void*>(k_edge_step<H, f, P, pi, false, false, true>);
      }
    }
    if constexpr (H == 64 && !f) {
      if (ol) return reinterpret_cast<const void*>(k_edge_step<H, f, P, pi, wv, true, false>);
    }
    return reinterpret_cast<const void*>(k_edge_step<H, f, P, pi, wv, false, false>);
  };
  // edge-side products take the LDS-weight form
  auto pick_w = [&](auto F, auto PI) -> const void* {
    if constexpr (P == P_F32) {
      if (wr && !gh) return pick_o(F, PI, std::true_type{});
    }
    return pick_o(F, PI, std::false_type{});
  };
  auto pick_p = [&](auto F) -> const void* {
    switch (pipe) {
      case 0: return pick_w(F, std::integral_constant<int, 0>{});
      case 2: return pick_w(F, std::integral_constant<int, 2>{});
      default: return pick_w(F, std::integral_constant<int, 1>{});
    }
  };
  return fin ? pick_p(std::true_type{}) : pick_p(std::false_type{});
}

static bool outsum_lds(const RunArgs& a) { return a.ctx->outsum_lds && a.ctx->cfg.gnn_hidden == 64; }

static size_t outsum_lds_bytes(const RunArgs& a) {
  return outsum_lds(a) ? (size_t)(a.ctx->edge_threads / 64) * kOutBufFloats * sizeof(float) : 0;
}

// precision of the edge kernels' GEMMs (FP32 runs may use the split form)
static int edge_prec(const RunArgs& a) { return (a.prec == P_F32 && a.ctx->f32_split) ? kF32Split : a.prec; }

hipError_t launch_edge_encode(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  const int kp = edge_prec(a);
  const WeightMap& m = a.ctx->wmap[kSegPrec[kp]];
  A.seg = static_cast<const char*>(a.ctx->seg_base[kSegPrec[kp]]) + m.edge_enc;
  A.seg_bytes = SegEdgeEnc{Hh, kPrecBytes[kp]}.size();
  const bool gh = a.ctx->edge_products != 0;
  // the node encoder's W_src and W_dst (its segment, its precision)
  A.seg3 = seg_ptr(a, a.ctx->wmap[kSegPrec[a.prec]].node_enc + SegNodeEnc{Hh, kPrecBytes[a.prec]}.ws());
  A.seg3_bytes = gh ? 2 * Hh * Hh * kPrecBytes[a.prec] : 0;
  const unsigned grid = (unsigned)(a.ctx->n_cu * a.ctx->edge_wg_per_cu);
  const size_t lds = A.seg_bytes + A.seg3_bytes + outsum_lds_bytes(a);
  const int pipe = a.ctx->edge_pipeline;
  const bool ol = outsum_lds(a);
  const void* fn = nullptr;
#define ENC_K(H_, P_) edge_encode_kernel<H_, P_>(pipe, ol, gh)
  switch (Hh * 8 + kp) {
    case 32 * 8 + 0: fn = ENC_K(32, 0); break;
    case 32 * 8 + 1: fn = ENC_K(32, 1); break;
    case 32 * 8 + 2: fn = ENC_K(32, 2); break;
    case 32 * 8 + 3: fn = ENC_K(32, 3); break;
    case 32 * 8 + 4: fn = ENC_K(32, 4); break;
    case 32 * 8 + 5: fn = ENC_K(32, 5); break;
    case 32 * 8 + 6: fn = ENC_K(32, 6); break;
    case 64 * 8 + 0: fn = ENC_K(64, 0); break;
    case 64 * 8 + 1: fn = ENC_K(64, 1); break;
    case 64 * 8 + 2: fn = ENC_K(64, 2); break;
    case 64 * 8 + 3: fn = ENC_K(64, 3); break;
    case 64 * 8 + 4: fn = ENC_K(64, 4); break;
    case 64 * 8 + 5: fn = ENC_K(64, 5); break;
    case 64 * 8 + 6: fn = ENC_K(64, 6); break;
    default: return hipErrorInvalidValue;
  }
#undef ENC_K
  void* args[] = {&A};
  return hipLaunchKernel(fn, dim3(grid), dim3(a.ctx->edge_threads), args, lds, a.stream);
}

hipError_t launch_segsum(const RunArgs& a, int k) {
  if (a.hits.n_hits == 0 || a.ctx->fuse_messages) return hipSuccess;
  GnnArgs A = gnn_args(a);
  A.step = k;
  const int Hh = a.ctx->cfg.gnn_hidden;
  unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.hits.n_hits + 3) / 4, (int64_t)a.ctx->n_cu * 32));
  const int U = a.ctx->segsum_unroll;
  // the sums read the stored edge rows: FP32 whenever the state is kept in FP32
  const int sp = (a.prec == P_BF16 || a.prec == P_FP8) ? a.prec : P_F32;
#define SEG_U(U_) DISPATCH_HP(Hh, sp, hipLaunchKernelGGL((k_segsum<H, P, U_>), dim3(grid), dim3(256), 0, a.stream, A))
  switch (U) {
    case 1: SEG_U(1); break;
    case 2: SEG_U(2); break;
    case 8: SEG_U(8); break;
    default: SEG_U(4); break;
  }
#undef SEG_U
  return hipGetLastError();
}

hipError_t launch_node_step(const RunArgs& a, int k) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  const WeightMap& m = a.ctx->wmap[kSegPrec[a.prec]];
  A.seg = seg_ptr(a, m.node[k]);
  A.seg_bytes = SegNode{Hh, kPrecBytes[a.prec]}.size();
  A.step = k;
  unsigned grid = node_grid(a, a.ctx->node_wg_per_cu);
  const bool np = !a.ctx->edge_products;
#define NODE_K(F_, N_) \
  DISPATCH_HP(Hh, a.prec, hipLaunchKernelGGL((k_node_step<H, P, F_, N_>), dim3(grid), dim3(node_threads(P)), A.seg_bytes, a.stream, A))
  if (a.ctx->fuse_messages && np) {
    NODE_K(true, true);
  } else if (a.ctx->fuse_messages) {
    NODE_K(true, false);
  } else if (np) {
    NODE_K(false, true);
  } else {
    NODE_K(false, false);
  }
#undef NODE_K
  return hipGetLastError();
}

hipError_t launch_edge_step(const RunArgs& a, int k, bool final_step) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  const int kp = edge_prec(a);
  const WeightMap& m = a.ctx->wmap[kSegPrec[kp]];
  const char* base = static_cast<const char*>(a.ctx->seg_base[kSegPrec[kp]]);
  A.seg = base + m.edge[k];
  A.seg_bytes = SegEdge{Hh, kPrecBytes[kp]}.size();
  A.seg2 = base + m.cls;
  A.seg2_bytes = SegCls{Hh, kPrecBytes[kp]}.size();
  const bool gh = a.ctx->edge_products != 0;
  // W_src and W_dst of edge net k as the node kernel holds them (node net k's
  // segment, the node kernels' precision), so the products are the same bits
  A.seg3 = seg_ptr(a, a.ctx->wmap[kSegPrec[a.prec]].node[k] + SegNode{Hh, kPrecBytes[a.prec]}.ws());
  A.seg3_bytes = gh ? 2 * Hh * Hh * kPrecBytes[a.prec] : 0;
  A.step = k;
  const bool ol = !final_step && outsum_lds(a);
  const size_t lds = A.seg_bytes + A.seg3_bytes + (final_step ? A.seg2_bytes : 0) + (ol ? outsum_lds_bytes(a) : 0);
  const unsigned grid = (unsigned)(a.ctx->n_cu * a.ctx->edge_wg_per_cu);
  const int pipe = a.ctx->edge_pipeline;
  const bool wr = a.ctx->edge_wreg != 0;
  const void* fn = nullptr;
#define STEP_K(H_, P_) edge_step_kernel<H_, P_>(final_step, pipe, wr, ol, gh)
  switch (Hh * 8 + kp) {
    case 32 * 8 + 0: fn = STEP_K(32, 0); break;
    case 32 * 8 + 1: fn = STEP_K(32, 1); break;
    case 32 * 8 + 2: fn = STEP_K(32, 2); break;
    case 32 * 8 + 3: fn = STEP_K(32, 3); break;
    case 32 * 8 + 4: fn = STEP_K(32, 4); break;
    case 32 * 8 + 5: fn = STEP_K(32, 5); break;
    case 32 * 8 + 6: fn = STEP_K(32, 6); break;
    case 64 * 8 + 0: fn = STEP_K(64, 0); break;
    case 64 * 8 + 1: fn = STEP_K(64, 1); break;
    case 64 * 8 + 2: fn = STEP_K(64, 2); break;
    case 64 * 8 + 3: fn = STEP_K(64, 3); break;
    case 64 * 8 + 4: fn = STEP_K(64, 4); break;
    case 64 * 8 + 5: fn = STEP_K(64, 5); break;
    case 64 * 8 + 6: fn = STEP_K(64, 6); break;
    default: return hipErrorInvalidValue;
  }
#undef STEP_K
  void* args[] = {&A};
  return hipLaunchKernel(fn, dim3(grid), dim3(a.ctx->edge_threads), args, lds, a.stream);
}

__global__ void k_quantize(int prec, const float* __restrict__ in, float* __restrict__ out, int64_t n, float scale) {
  const float inv = 1.0f / scale;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = in[i];
    float v = x;
    if (prec == ETX_BF16) v = bf16_value(bf16_bits(x));
    else if (prec == ETX_FP8_E4M3) v = e4m3_decode(e4m3_encode(x * inv)) * scale;
    else if (prec == ETX_INT8) v = (float)(int8_t)i8_byte(x * inv) * scale;
    out[i] = v;
  }
}

hipError_t launch_quantize(int prec, const float* in, float* out, int64_t n, float scale, hipStream_t s) {
  unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_quantize, dim3(grid), dim3(256), 0, s, prec, in, out, n, scale);
  return hipGetLastError();
}

template <int H, int P>
static void set_gnn_attr(int& bad, size_t max_lds) {
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  set(reinterpret_cast<const void*>(k_node_encode<H, P, false>));
  set(reinterpret_cast<const void*>(k_node_encode<H, P, true>));
  set(reinterpret_cast<const void*>(k_node_step<H, P, false, false>));
  set(reinterpret_cast<const void*>(k_node_step<H, P, true, false>));
  set(reinterpret_cast<const void*>(k_node_step<H, P, false, true>));
  set(reinterpret_cast<const void*>(k_node_step<H, P, true, true>));
  for (int fin = 0; fin < 2; ++fin)
    for (int pipe = 0; pipe < 3; ++pipe)
      for (int wr = 0; wr < 2; ++wr)
        for (int ol = 0; ol < 2; ++ol)
          for (int gh = 0; gh < 2; ++gh) set(edge_step_kernel<H, P>(fin, pipe, wr, ol, gh));
  for (int pipe = 0; pipe < 3; ++pipe)
    for (int ol = 0; ol < 2; ++ol)
      for (int gh = 0; gh < 2; ++gh) set(edge_encode_kernel<H, P>(pipe, ol, gh));
}

template <int H>
static void set_split_attr(int& bad, size_t max_lds) {
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  for (int fin = 0; fin < 2; ++fin)
    for (int pipe = 0; pipe < 3; ++pipe)
      for (int ol = 0; ol < 2; ++ol)
        for (int gh = 0; gh < 2; ++gh) set(edge_step_kernel<H, P_F32X>(fin, pipe, false, ol, gh));
  for (int pipe = 0; pipe < 3; ++pipe)
    for (int ol = 0; ol < 2; ++ol)
      for (int gh = 0; gh < 2; ++gh) set(edge_encode_kernel<H, P_F32X>(pipe, ol, gh));
}

int gnn_attributes(size_t max_lds) {
  int bad = 0;
  set_split_attr<32>(bad, max_lds);
  set_split_attr<64>(bad, max_lds);
  set_gnn_attr<32, 0>(bad, max_lds);
  set_gnn_attr<32, 1>(bad, max_lds);
  set_gnn_attr<32, 2>(bad, max_lds);
  set_gnn_attr<32, 4>(bad, max_lds);
  set_gnn_attr<32, 5>(bad, max_lds);
  set_gnn_attr<32, 6>(bad, max_lds);
  set_gnn_attr<64, 0>(bad, max_lds);
  set_gnn_attr<64, 1>(bad, max_lds);
  set_gnn_attr<64, 2>(bad, max_lds);
  set_gnn_attr<64, 4>(bad, max_lds);
  set_gnn_attr<64, 5>(bad, max_lds);
  set_gnn_attr<64, 6>(bad, max_lds);
  return bad;
}

}  // namespace etx
