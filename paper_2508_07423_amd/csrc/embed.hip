// Embedding MLP (thesis ch. 8 "Hit Embedding and Rough Graph Construction"):
// normalised cylindrical coordinates (r/R_s, phi/pi, z/Z_s) -> Linear -> ReLU
// -> ... -> Linear, fused with the feature computation.  The 3-wide first layer
// runs on the vector ALU in FP32; the W x W hidden layers and the output layer
// run on MFMA in the column layout of tile.hpp with operands in precision P.
// Output: [n_hits][16] FP32 (padded).
#include "internal.hpp"
#include "seg.hpp"
#include "tile.hpp"

namespace etx {

namespace {

struct EmbedArgs {
  const float* x;
  const float* y;
  const float* z;
  int64_t n_hits;
  float inv_r, inv_z;
  const char* seg;
  int seg_bytes;
  int layers;
  float* emb;
  float* calib;
  const float* sc;
  const int64_t* status;
};

__device__ inline void atomic_amax(float* slot, float v) {
  // non-negative floats order like their bit patterns
  atomicMax(reinterpret_cast<unsigned int*>(slot), __float_as_uint(fabsf(v)));
}

template <int W, int P>
__global__ __launch_bounds__(256) void k_embed(EmbedArgs A) {
  if (A.status[0] != 0) return;
  extern __shared__ float lds[];
  char* w = reinterpret_cast<char*>(lds);
  stage(lds, reinterpret_cast<const float*>(A.seg), A.seg_bytes / 4);
  __syncthreads();
  const SegEmb S{W, A.layers, PrecBytes<P>::value};
  const int lane = lane_id(), g = lane_group(), wave = threadIdx.x >> 6;
  const int64_t ntiles = (A.n_hits + kCols - 1) / kCols;
  const int64_t tstride = (int64_t)gridDim.x * 4;
  // the next tile's coordinates are loaded one tile ahead
  float xn = 0.f, yn = 0.f, zn = 0.f;
  auto fetch = [&](int64_t t) {
    const int64_t c = t * kCols + (lane & 15);
    if (t < ntiles && c < A.n_hits) {
      xn = A.x[c];
      yn = A.y[c];
      zn = A.z[c];
    }
  };
  int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  fetch(tile);
  for (; tile < ntiles; tile += tstride) {
    const int64_t col = tile * kCols + (lane & 15);
    const bool valid = col < A.n_hits;
    const float xx = xn, yy = yn, zz = zn;
    fetch(tile + tstride);
    float u0 = 0.f, u1 = 0.f, u2 = 0.f;
    if (valid) {
      u0 = hypotf(xx, yy) * A.inv_r;
      u1 = atan2f(yy, xx) * 0.318309886183790672f;   // 1/pi
      u2 = zz * A.inv_z;
    }
    float a[W / 4];
    const float* w1 = reinterpret_cast<const float*>(w + S.w1());
    const float* b1 = reinterpret_cast<const float*>(w + S.b1());
#pragma unroll
    for (int r = 0; r < W / 4; ++r) {
      const int f = phi(r, g);
      float acc = u0 * w1[f];
      acc = fmaf(u1, w1[W + f], acc);
      acc = fmaf(u2, w1[2 * W + f], acc);
      a[r] = fmaxf(acc + b1[f], 0.f);
    }
    auto observe = [&](int l) {
      if (!A.calib) return;
      float m = 0.f;
#pragma unroll
      for (int r = 0; r < W / 4; ++r) m = fmaxf(m, fabsf(a[r]));
      if (valid) atomic_amax(A.calib + SC_EMB + l, m);
    };
    for (int l = 1; l < A.layers; ++l) {
      float acc[W / 4];
      bias_cols<W>(acc, reinterpret_cast<const float*>(w + S.bh(l)));
      observe(l);
      const float s = A.sc[SC_EMB + l];
      gemm<P, W, W / 16>(acc, a, w + S.wh(l), 1.0f / s, s * A.sc[SW_EMB + l]);
#pragma unroll
      for (int r = 0; r < W / 4; ++r) a[r] = fmaxf(acc[r], 0.f);
    }
    float o[4];
    bias_cols<16>(o, reinterpret_cast<const float*>(w + S.bo()));
    observe(A.layers);
    const float so = A.sc[SC_EMB + A.layers];
    gemm<P, W, 1>(o, a, w + S.wo(), 1.0f / so, so * A.sc[SW_EMB + A.layers]);
    // features 4g .. 4g+3 of the 16 padded outputs
    if (valid) *reinterpret_cast<float4*>(A.emb + col * kDpad + 4 * g) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

}  // namespace

hipError_t launch_embed(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  const etx_ctx* c = a.ctx;
  // the embedding may run at its own operand precision (calibration runs stay FP32)
  const int ep = (!a.calibrate && c->emb_precision >= 0) ? c->emb_precision : kEtxPrec[a.prec];
  const int prec = ep == ETX_INT8 ? kI8Seg : ep;                       // weight segment set
  const int kp = ep == ETX_INT8 ? (int)P_I8M : ep;                     // kernel precision
  EmbedArgs A;
  A.x = a.hits.x;
  A.y = a.hits.y;
  A.z = a.hits.z;
  A.n_hits = a.hits.n_hits;
  A.inv_r = 1.0f / c->cfg.r_scale_mm;
  A.inv_z = 1.0f / c->cfg.z_scale_mm;
  A.seg = static_cast<const char*>(c->seg_base[prec]) + c->wmap[prec].emb;
  A.layers = c->cfg.emb_layers;
  A.sc = c->dev_scales + (ep == ETX_INT8 ? SC_I8 : 0);
  A.emb = reinterpret_cast<float*>(a.ws + a.L.emb);
  A.calib = a.calibrate ? reinterpret_cast<float*>(a.ws + a.L.calib) : nullptr;
  A.status = a.out.status;
  const int W = c->cfg.emb_hidden;
  A.seg_bytes = SegEmb{W, A.layers, kSegBytes[prec]}.size();
  size_t lds = A.seg_bytes;
  int64_t tiles = (A.n_hits + kCols - 1) / kCols;
  // as many workgroups as are resident at once (registers or LDS decide)
  auto resident = [&](const void* f) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 256, lds) != hipSuccess || nb < 1) nb = 2;
    return (unsigned)std::min<int64_t>((tiles + 3) / 4, (int64_t)c->n_cu * nb);
  };
#define EMB(W_, P_)                                                                          \
  hipLaunchKernelGGL((k_embed<W_, P_>), dim3(resident(reinterpret_cast<const void*>(k_embed<W_, P_>))), dim3(256), \
                     lds, a.stream, A)
  switch (W * 8 + kp) {
    case 32 * 8 + 0: EMB(32, 0); break;
    case 32 * 8 + 1: EMB(32, 1); break;
    case 32 * 8 + 2: EMB(32, 2); break;
    case 32 * 8 + 6: EMB(32, 6); break;
    case 64 * 8 + 0: EMB(64, 0); break;
    case 64 * 8 + 1: EMB(64, 1); break;
    case 64 * 8 + 2: EMB(64, 2); break;
    case 64 * 8 + 6: EMB(64, 6); break;
    case 128 * 8 + 0: EMB(128, 0); break;
    case 128 * 8 + 1: EMB(128, 1); break;
    case 128 * 8 + 2: EMB(128, 2); break;
    case 128 * 8 + 6: EMB(128, 6); break;
    default: return hipErrorInvalidValue;
  }
#undef EMB
  return hipGetLastError();
}

int embed_attributes(size_t max_lds) {
  int bad = 0;
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  set(reinterpret_cast<const void*>(k_embed<32, 0>));
  set(reinterpret_cast<const void*>(k_embed<32, 1>));
  set(reinterpret_cast<const void*>(k_embed<32, 2>));
  set(reinterpret_cast<const void*>(k_embed<32, 6>));
  set(reinterpret_cast<const void*>(k_embed<64, 0>));
  set(reinterpret_cast<const void*>(k_embed<64, 1>));
  set(reinterpret_cast<const void*>(k_embed<64, 2>));
  set(reinterpret_cast<const void*>(k_embed<64, 6>));
  set(reinterpret_cast<const void*>(k_embed<128, 0>));
  set(reinterpret_cast<const void*>(k_embed<128, 1>));
  set(reinterpret_cast<const void*>(k_embed<128, 2>));
  set(reinterpret_cast<const void*>(k_embed<128, 6>));
  return bad;
}

}  // namespace etx
