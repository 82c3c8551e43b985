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
// segmented sums: out-sums over the source-major edge list (CSR rows),
// in-sums through the (dst, src)-ordered CSC permutation.
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
  const float* seg;         // weight segment of the kernel
  const float* seg2;        // classifier segment (final edge step)
  int seg_floats, seg2_floats;
  float* h;                 // [n_hits][H]
  float* ps;                // [n_hits][H] h W_src (source product)
  float* pd;                // [n_hits][H] h W_dst (target product)
  float* msg;               // [n_hits][2H] (out-sum, in-sum)
  float* e;                 // [edges][H]
  float* score;             // [edges]
  float* calib;
  int step;
  int unroll;
  const int64_t* status;
};

// --------------------------------------------------------------------------
// node encoder (+ edge-encoder source/target products)
// --------------------------------------------------------------------------
template <int H>
__global__ __launch_bounds__(1024) void k_node_encode(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float w[];
  stage(w, A.seg, A.seg_floats);
  __syncthreads();
  constexpr SegNodeEnc S{H};
  const int lane = lane_id(), g = lane_group(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t ntiles = (A.n_hits + kCols - 1) / kCols;
  for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < A.n_hits;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
    if (valid) {
      v0 = A.x[col] * A.inv_r;
      v1 = A.y[col] * A.inv_r;
      v2 = A.z[col] * A.inv_z;
    }
    float a[H / 4];
    const float* w1 = w + S.w1();
    const float* b1 = w + S.b1();
#pragma unroll
    for (int r = 0; r < H / 4; ++r) {
      const int f = phi(r, g);
      float acc = v0 * w1[f];
      acc = fmaf(v1, w1[H + f], acc);
      acc = fmaf(v2, w1[2 * H + f], acc);
      a[r] = acc + b1[f];
    }
    ln_relu<H>(a);
    observe<H / 4>(A.calib, CAL_NE_L2, a, valid);
    float hh[H / 4];
    bias_cols<H>(hh, w + S.b2());
    mfma_f32<H, H / 16>(hh, a, w + S.w2());
    ln_relu<H>(hh);
    store_cols<H>(A.h + col * H, hh, valid);
    observe<H / 4>(A.calib, CAL_H0, hh, valid);
    float q[H / 4];
#pragma unroll
    for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
    mfma_f32<H, H / 16>(q, hh, w + S.ws());
    store_cols<H>(A.ps + col * H, q, valid);
#pragma unroll
    for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
    mfma_f32<H, H / 16>(q, hh, w + S.wd());
    store_cols<H>(A.pd + col * H, q, valid);
  }
}

// --------------------------------------------------------------------------
// edge encoder
// --------------------------------------------------------------------------
template <int H>
__global__ __launch_bounds__(512) void k_edge_encode(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float w[];
  stage(w, A.seg, A.seg_floats);
  __syncthreads();
  constexpr SegEdgeEnc S{H};
  const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t E = A.row_ptr[A.n_hits];
  const int64_t ntiles = (E + kCols - 1) / kCols;
  for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < E;
    const int s = valid ? A.src[col] : 0, d = valid ? A.dst[col] : 0;
    float a[H / 4];
    bias_cols<H>(a, w + S.b1());
    add_cols<H>(a, A.ps + (int64_t)s * H, valid);
    add_cols<H>(a, A.pd + (int64_t)d * H, valid);
    ln_relu<H>(a);
    observe<H / 4>(A.calib, CAL_EE_L2, a, valid);
    float o[H / 4];
    bias_cols<H>(o, w + S.b2());
    mfma_f32<H, H / 16>(o, a, w + S.w2());
    ln_relu<H>(o);
    observe<H / 4>(A.calib, CAL_E, o, valid);
    store_cols<H>(A.e + col * H, o, valid);
  }
}

// --------------------------------------------------------------------------
// messages: segmented out-sums (CSR rows) and in-sums (CSC), one wave per node
// --------------------------------------------------------------------------
template <int H, int U>
__global__ __launch_bounds__(256) void k_segsum(GnnArgs A) {
  if (A.status[0] != 0) return;
  constexpr int NS = 64 / H;          // edge streams per wave (1 for H=64, 2 for H=32)
  const int lane = lane_id(), f = lane % H, sub = lane / H, wave = threadIdx.x >> 6;
  for (int64_t node = (int64_t)blockIdx.x * 4 + wave; node < A.n_hits; node += (int64_t)gridDim.x * 4) {
    // out-sum over the contiguous row
    const int64_t rb = A.row_ptr[node], re = A.row_ptr[node + 1];
    float mo = 0.f;
    for (int64_t t = rb + sub; t < re; t += NS * U) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t q = t + (int64_t)u * NS;
        v[u] = q < re ? A.e[q * H + f] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) mo += v[u];
    }
    // in-sum through the CSC permutation
    const int64_t cb = A.col_ptr[node], ce = A.col_ptr[node + 1];
    float mi = 0.f;
    for (int64_t t = cb + sub; t < ce; t += NS * U) {
      int id[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t q = t + (int64_t)u * NS;
        id[u] = q < ce ? A.csc[q] : -1;
      }
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = id[u] >= 0 ? A.e[(int64_t)id[u] * H + f] : 0.f;
#pragma unroll
      for (int u = 0; u < U; ++u) mi += v[u];
    }
    if (NS == 2) {
      mo += __shfl_xor(mo, 32);
      mi += __shfl_xor(mi, 32);
    }
    if (sub == 0) {
      A.msg[node * 2 * H + f] = mo;
      A.msg[node * 2 * H + H + f] = mi;
    }
  }
}

// --------------------------------------------------------------------------
// node update k (+ edge net k source/target products)
// --------------------------------------------------------------------------
template <int H>
__global__ __launch_bounds__(1024) void k_node_step(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float w[];
  stage(w, A.seg, A.seg_floats);
  __syncthreads();
  constexpr SegNode S{H};
  const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t ntiles = (A.n_hits + kCols - 1) / kCols;
  for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < A.n_hits;
    float x[3 * H / 4];
    load_cols<H>(x, A.h + col * H, valid);
    load_cols<H>(x + H / 4, A.msg + col * 2 * H, valid);
    load_cols<H>(x + H / 2, A.msg + col * 2 * H + H, valid);
    observe<3 * H / 4>(A.calib, CAL_NN_IN + A.step, x, valid);
    float a[H / 4];
    bias_cols<H>(a, w + S.b1());
    mfma_f32<3 * H, H / 16>(a, x, w + S.w1());
    ln_relu<H>(a);
    observe<H / 4>(A.calib, CAL_NN_L2, a, valid);
    float o[H / 4];
    bias_cols<H>(o, w + S.b2());
    mfma_f32<H, H / 16>(o, a, w + S.w2());
    ln_relu<H>(o);
#pragma unroll
    for (int r = 0; r < H / 4; ++r) o[r] += x[r];
    store_cols<H>(A.h + col * H, o, valid);
    observe<H / 4>(A.calib, CAL_H0 + 1 + A.step, o, valid);
    float q[H / 4];
#pragma unroll
    for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
    mfma_f32<H, H / 16>(q, o, w + S.ws());
    store_cols<H>(A.ps + col * H, q, valid);
#pragma unroll
    for (int r = 0; r < H / 4; ++r) q[r] = 0.f;
    mfma_f32<H, H / 16>(q, o, w + S.wd());
    store_cols<H>(A.pd + col * H, q, valid);
  }
}

// --------------------------------------------------------------------------
// edge update k; the last step also runs the classifier and writes scores
// --------------------------------------------------------------------------
template <int H, bool FINAL>
__global__ __launch_bounds__(512) void k_edge_step(GnnArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float w[];
  constexpr SegEdge S{H};
  constexpr SegCls C{H};
  stage(w, A.seg, A.seg_floats);
  if (FINAL) stage(w + S.size(), A.seg2, A.seg2_floats);
  __syncthreads();
  const float* wc = w + S.size();
  const int lane = lane_id(), g = lane_group(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t E = A.row_ptr[A.n_hits];
  const int64_t ntiles = (E + kCols - 1) / kCols;
  for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < E;
    const int s = valid ? A.src[col] : 0, d = valid ? A.dst[col] : 0;
    float e[H / 4];
    load_cols<H>(e, A.e + col * H, valid);
    float a[H / 4];
    bias_cols<H>(a, w + S.b1());
    add_cols<H>(a, A.ps + (int64_t)s * H, valid);
    add_cols<H>(a, A.pd + (int64_t)d * H, valid);
    mfma_f32<H, H / 16>(a, e, w + S.we());
    ln_relu<H>(a);
    observe<H / 4>(A.calib, CAL_EN_L2, a, valid);
    float o[H / 4];
    bias_cols<H>(o, w + S.b2());
    mfma_f32<H, H / 16>(o, a, w + S.w2());
    ln_relu<H>(o);
#pragma unroll
    for (int r = 0; r < H / 4; ++r) o[r] += e[r];
    observe<H / 4>(A.calib, CAL_E + 1 + A.step, o, valid);
    if (!FINAL) {
      store_cols<H>(A.e + col * H, o, valid);
    } else {
      observe<H / 4>(A.calib, CAL_CLS_IN, o, valid);
      float c[H / 4];
      bias_cols<H>(c, wc + C.b1());
      mfma_f32<H, H / 16>(c, o, wc + C.w1());
      ln_relu<H>(c);
      observe<H / 4>(A.calib, CAL_CLS_L2, c, valid);
      float dot = 0.f;
#pragma unroll
      for (int r = 0; r < H / 4; ++r) dot = fmaf(c[r], wc[C.w2() + phi(r, g)], dot);
      dot = col_sum(dot);
      const float logit = dot + wc[C.b2()];
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
  A.e = reinterpret_cast<float*>(a.ws + a.L.e);
  A.score = a.out.score;
  A.calib = a.calibrate ? reinterpret_cast<float*>(a.ws + a.L.calib) : nullptr;
  A.status = a.out.status;
  A.unroll = c->segsum_unroll;
  return A;
}

constexpr int kNodeThreads = 1024;   // 16 waves: the node kernels hold up to 98 KiB of weights in LDS
constexpr int kEdgeThreads = 512;

static unsigned node_grid(const RunArgs& a, int per_cu) {
  int64_t tiles = (a.hits.n_hits + kCols - 1) / kCols;
  int64_t waves = kNodeThreads / 64;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + waves - 1) / waves, (int64_t)a.ctx->n_cu * per_cu));
}

#define DISPATCH_H(H_, ...)                    \
  switch (H_) {                                \
    case 32: { constexpr int H = 32; __VA_ARGS__; } break; \
    case 64: { constexpr int H = 64; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;      \
  }

hipError_t launch_node_encode(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  A.seg = a.ctx->dev_w + a.ctx->wmap.node_enc;
  A.seg_floats = SegNodeEnc{Hh}.size();
  size_t lds = sizeof(float) * A.seg_floats;
  unsigned grid = node_grid(a, a.ctx->node_wg_per_cu);
  DISPATCH_H(Hh, hipLaunchKernelGGL(k_node_encode<H>, dim3(grid), dim3(kNodeThreads), lds, a.stream, A));
  return hipGetLastError();
}

hipError_t launch_edge_encode(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  A.seg = a.ctx->dev_w + a.ctx->wmap.edge_enc;
  A.seg_floats = SegEdgeEnc{Hh}.size();
  size_t lds = sizeof(float) * A.seg_floats;
  unsigned grid = (unsigned)(a.ctx->n_cu * a.ctx->edge_wg_per_cu);
  DISPATCH_H(Hh, hipLaunchKernelGGL(k_edge_encode<H>, dim3(grid), dim3(kEdgeThreads), lds, a.stream, A));
  return hipGetLastError();
}

hipError_t launch_segsum(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.hits.n_hits + 3) / 4, (int64_t)a.ctx->n_cu * 32));
  const int U = a.ctx->segsum_unroll;
#define SEG_U(U_) DISPATCH_H(Hh, hipLaunchKernelGGL((k_segsum<H, U_>), dim3(grid), dim3(256), 0, a.stream, A))
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
  A.seg = a.ctx->dev_w + a.ctx->wmap.node[k];
  A.seg_floats = SegNode{Hh}.size();
  A.step = k;
  size_t lds = sizeof(float) * A.seg_floats;
  unsigned grid = node_grid(a, a.ctx->node_wg_per_cu);
  DISPATCH_H(Hh, hipLaunchKernelGGL(k_node_step<H>, dim3(grid), dim3(kNodeThreads), lds, a.stream, A));
  return hipGetLastError();
}

hipError_t launch_edge_step(const RunArgs& a, int k, bool final_step) {
  if (a.hits.n_hits == 0) return hipSuccess;
  GnnArgs A = gnn_args(a);
  const int Hh = a.ctx->cfg.gnn_hidden;
  A.seg = a.ctx->dev_w + a.ctx->wmap.edge[k];
  A.seg_floats = SegEdge{Hh}.size();
  A.seg2 = a.ctx->dev_w + a.ctx->wmap.cls;
  A.seg2_floats = SegCls{Hh}.size();
  A.step = k;
  size_t lds = sizeof(float) * (A.seg_floats + (final_step ? A.seg2_floats : 0));
  unsigned grid = (unsigned)(a.ctx->n_cu * a.ctx->edge_wg_per_cu);
  if (final_step) {
    DISPATCH_H(Hh, hipLaunchKernelGGL((k_edge_step<H, true>), dim3(grid), dim3(kEdgeThreads), lds, a.stream, A));
  } else {
    DISPATCH_H(Hh, hipLaunchKernelGGL((k_edge_step<H, false>), dim3(grid), dim3(kEdgeThreads), lds, a.stream, A));
  }
  return hipGetLastError();
}

int gnn_attributes(size_t max_lds) {
  int bad = 0;
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  set(reinterpret_cast<const void*>(k_node_encode<32>));
  set(reinterpret_cast<const void*>(k_node_encode<64>));
  set(reinterpret_cast<const void*>(k_node_step<32>));
  set(reinterpret_cast<const void*>(k_node_step<64>));
  set(reinterpret_cast<const void*>(k_edge_step<32, true>));
  set(reinterpret_cast<const void*>(k_edge_step<64, true>));
  set(reinterpret_cast<const void*>(k_edge_step<32, false>));
  set(reinterpret_cast<const void*>(k_edge_step<64, false>));
  set(reinterpret_cast<const void*>(k_edge_encode<32>));
  set(reinterpret_cast<const void*>(k_edge_encode<64>));
  return bad;
}

}  // namespace etx
