// Learned edge prefilter: a small MLP on candidate-edge features that prunes
// the radius graph before the interaction network, trained on the device by
// the kernels below (forward, backward, deterministic gradient reduction,
// Adam).  The thesis's own pipeline has no such stage; its closest relative
// is the filter step of Exa.TrkX that the thesis removed (ch. 9 "Development").
//
// Features of candidate i -> j (normalised by R_s, R_s, Z_s, R_s, pi, 1):
//   (x_j - x_i, y_j - y_i, z_j - z_i, r_j - r_i, wrap(phi_j - phi_i), |e_j - e_i|)
// MLP 6 -> 32 -> 32 -> 1 with ReLU; keep the edge when sigmoid(logit) >= tau.
// The 32 x 32 product runs on BF16 MFMA (forward, and the backward product
// W2 delta2); the 6-wide input layer, the output layer and every weight
// gradient accumulate in FP32.  Loss: class-weighted binary cross-entropy
// averaged over the candidate edges; optimiser: Adam (thesis ch. 4, "Gradient
// Descent"), FP32 master weights and moments.
#include "internal.hpp"
#include "tile.hpp"

namespace etx {

namespace {

constexpr int PF = ETX_PF_HIDDEN;
constexpr int O_W1 = 0, O_B1 = 6 * PF, O_W2 = O_B1 + PF, O_B2 = O_W2 + PF * PF, O_W3 = O_B2 + PF, O_B3 = O_W3 + PF;
constexpr int N_P = O_B3 + 1;
static_assert(N_P == ETX_PF_NPARAM, "prefilter parameter layout");
static_assert(kPfGradStride >= N_P + 1, "gradient partial stride");

constexpr int kPfThreads = 512;
constexpr int kPfWaves = kPfThreads / 64;

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct PfArgs {
  int64_t n_hits;
  const float* x;
  const float* y;
  const float* z;
  const float* emb;          // [n_hits][16]
  const float2* polar;       // [n_hits] (r, phi) of every hit
  const int64_t* row_ptr;    // candidate CSR; row_ptr[n_hits] = candidate count
  const int32_t* src;
  const int32_t* dst;
  const float* params;       // FP32 parameters (device)
  float inv_r, inv_z, tau;
  uint8_t* keep;             // inference output [candidates]
  float* prob;               // inference output: probability per candidate
  float* feat;               // inference output when requested: features per candidate [8] (else null)
  const uint8_t* label;      // training labels [candidates]
  float pos_weight;
  float* partial;            // [waves][kPfGradStride]
  const int64_t* status;
};

// LDS: small FP32 parameter vectors + the BF16 W2 and W2^T, permuted for tile.hpp
struct PfLds {
  float w1[6 * PF], b1[PF], b2[PF], w3[PF], b3[4];
  bf16x8 w2p[2 * 64], w2tp[2 * 64];
};

__device__ inline void stage_params(PfLds& L, const float* __restrict__ p) {
  for (int i = threadIdx.x; i < 6 * PF; i += blockDim.x) L.w1[i] = p[O_W1 + i];
  for (int i = threadIdx.x; i < PF; i += blockDim.x) {
    L.b1[i] = p[O_B1 + i];
    L.b2[i] = p[O_B2 + i];
    L.w3[i] = p[O_W3 + i];
  }
  if (threadIdx.x == 0) L.b3[0] = p[O_B3];
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) {
    const int mb = i / 64, lane = i % 64, g = lane / 16, col = 16 * mb + lane % 16;
    bf16x8 a, b;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int row = phi(q, g);
      a[q] = (__bf16)p[O_W2 + row * PF + col];     // W2[k][m] for the forward product
      b[q] = (__bf16)p[O_W2 + col * PF + row];     // W2^T for the backward product
    }
    L.w2p[i] = a;
    L.w2tp[i] = b;
  }
}

// (r, phi) of every hit, once per batch, so that the per-edge features are
// differences (the same FP32 values as evaluating them per edge).
__global__ void k_hit_polar(int64_t n, const float* __restrict__ x, const float* __restrict__ y,
                            float2* __restrict__ polar, const int64_t* status) {
  if (status[0] != 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    polar[i] = make_float2(hypotf(x[i], y[i]), atan2f(y[i], x[i]));
}

// Features of a candidate edge.  DP: the embedding width rounded up to 8 or
// 16; the padding of a row up to 16 floats is zero and would add exact zeros
// to the squared distance, so it is not read.
template <int DP>
__device__ inline void edge_features(const PfArgs& A, int s, int d, float (&f)[6]) {
  const float xi = A.x[s], yi = A.y[s], zi = A.z[s], xj = A.x[d], yj = A.y[d], zj = A.z[d];
  const float2 pi_ = A.polar[s], pj = A.polar[d];
  float dphi = pj.y - pi_.y;
  const float pi = 3.14159265358979f;
  if (dphi > pi) dphi -= 2.f * pi;
  if (dphi <= -pi) dphi += 2.f * pi;
  float d2 = 0.f;
  const float* ei = A.emb + (int64_t)s * kDpad;
  const float* ej = A.emb + (int64_t)d * kDpad;
#pragma unroll
  for (int k = 0; k < DP; k += 4) {
    const float4 u = *reinterpret_cast<const float4*>(ei + k), v = *reinterpret_cast<const float4*>(ej + k);
    const float t0 = v.x - u.x, t1 = v.y - u.y, t2 = v.z - u.z, t3 = v.w - u.w;
    d2 = fmaf(t0, t0, d2);
    d2 = fmaf(t1, t1, d2);
    d2 = fmaf(t2, t2, d2);
    d2 = fmaf(t3, t3, d2);
  }
  f[0] = (xj - xi) * A.inv_r;
  f[1] = (yj - yi) * A.inv_r;
  f[2] = (zj - zi) * A.inv_z;
  f[3] = (pj.x - pi_.x) * A.inv_r;
  f[4] = dphi * (1.0f / pi);
  f[5] = sqrtf(d2);
}

template <bool TRAIN, int DP>
__global__ __launch_bounds__(kPfThreads) void k_pf(PfArgs A) {
  static_assert(DP == 8 || DP == 16, "embedding width rounded up to 8 or 16");
  if (A.status[0] != 0) return;
  __shared__ PfLds L;
  __shared__ float tr[kPfWaves][16 * 32 * 3 + 16 * 16];   // per-wave transposes (training)
  stage_params(L, A.params);
  __syncthreads();
  const int lane = lane_id(), g = lane_group(), j = lane & 15, wave = threadIdx.x >> 6;
  const int64_t E = A.row_ptr[A.n_hits];
  const float inv_n = E > 0 ? 1.0f / (float)E : 0.f;
  float* a1t = tr[wave];                 // [16 edges][32]
  float* d2t = a1t + 16 * 32;            // [16][32]
  float* d1t = d2t + 16 * 32;            // [16][32]
  float* ft = d1t + 16 * 32;             // [16][16] (6 used)
  floatx4 gw2[2][2], gw1[2];
  float gb1[8], gb2[8], gw3[8], gb3 = 0.f, loss = 0.f;
  if (TRAIN) {
    for (int m = 0; m < 2; ++m) {
      gw1[m] = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int n = 0; n < 2; ++n) gw2[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int r = 0; r < 8; ++r) gb1[r] = gb2[r] = gw3[r] = 0.f;
    for (int i = lane; i < 16 * 16; i += 64) ft[i] = 0.f;
    wave_sync();
  }
  const int64_t ntiles = (E + kCols - 1) / kCols;
  const int64_t tstride = (int64_t)gridDim.x * kPfWaves;
  // The wave's tiles are t0, t0 + tstride, ...; per round lane group g
  // gathers the features of tile t0 + g * tstride (four tiles' loads in
  // flight), then the four tiles run through the network in order, each
  // taking its features from its group.  Edge ends are loaded a round ahead.
  int s_next = 0, d_next = 0;
  auto fetch_ends = [&](int64_t t0) {
    const int64_t t = t0 + g * tstride, c = t * kCols + j;
    if (t < ntiles && c < E) {
      s_next = A.src[c];
      d_next = A.dst[c];
    }
  };
  const int64_t first = (int64_t)blockIdx.x * kPfWaves + wave;
  fetch_ends(first);
  for (int64_t t0 = first; t0 < ntiles; t0 += 4 * tstride) {
    const int64_t tg = t0 + g * tstride;
    const bool vg = tg < ntiles && tg * kCols + j < E;
    const int s_cur = s_next, d_cur = d_next;
    fetch_ends(t0 + 4 * tstride);
    float fg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (vg) edge_features<DP>(A, s_cur, d_cur, fg);
    for (int u = 0; u < 4; ++u) {
      const int64_t tile = t0 + u * tstride;
      if (tile >= ntiles) break;   // wave-uniform
      const int64_t col = tile * kCols + j;
      const bool valid = col < E;
      float f[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) f[k] = __shfl(fg[k], j + 16 * u);
      float z1[8], a1[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int c = phi(r, g);
        float acc = L.b1[c];
#pragma unroll
        for (int k = 0; k < 6; ++k) acc = fmaf(f[k], L.w1[k * PF + c], acc);
        z1[r] = acc;
        a1[r] = fmaxf(acc, 0.f);
      }
      float z2[8];
      bias_cols<PF>(z2, L.b2);
      mfma_bf16<PF, 2>(z2, a1, L.w2p);
      float a2[8];
      float dot = 0.f;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        a2[r] = fmaxf(z2[r], 0.f);
        dot = fmaf(a2[r], L.w3[phi(r, g)], dot);
      }
      const float z3 = col_sum(dot) + L.b3[0];
      const float prob = 1.0f / (1.0f + expf(-z3));
      if (!TRAIN) {
        if (valid && g == 0) {
          A.keep[col] = prob >= A.tau ? 1 : 0;
          A.prob[col] = prob;
          if (A.feat) {
            float4* fo = reinterpret_cast<float4*>(A.feat + col * 8);
            fo[0] = make_float4(f[0], f[1], f[2], f[3]);
            fo[1] = make_float4(f[4], f[5], 0.f, 0.f);
          }
        }
        continue;
      }
      const bool y = valid && A.label[col] != 0;
      const float wt = y ? A.pos_weight : 1.f;
      const float dz = valid ? wt * (prob - (y ? 1.f : 0.f)) * inv_n : 0.f;
      if (valid && g == 0) {
        const float v = y ? -z3 : z3;       // softplus(v) = max(v, 0) + log1p(exp(-|v|))
        loss += wt * (fmaxf(v, 0.f) + log1pf(expf(-fabsf(v))));
        gb3 += dz;
      }
      float d2[8], t1[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        d2[r] = z2[r] > 0.f ? L.w3[phi(r, g)] * dz : 0.f;
        t1[r] = 0.f;
      }
      mfma_bf16<PF, 2>(t1, d2, L.w2tp);     // W2 delta2
      float d1[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        d1[r] = z1[r] > 0.f ? t1[r] : 0.f;
        gw3[r] = fmaf(a2[r], dz, gw3[r]);
        gb2[r] += d2[r];
        gb1[r] += d1[r];
        const int c = phi(r, g);
        a1t[j * 32 + c] = a1[r];
        d2t[j * 32 + c] = d2[r];
        d1t[j * 32 + c] = d1[r];
      }
      if (g == 0)
#pragma unroll
        for (int k = 0; k < 6; ++k) ft[j * 16 + k] = f[k];
      wave_sync();
      // weight gradients: sums over the tile's 16 edges as FP32 MFMA with K = edges
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int e = 4 * t + (lane >> 4);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const float b2v = d2t[e * 32 + 16 * nb + (lane & 15)];
          const float b1v = d1t[e * 32 + 16 * nb + (lane & 15)];
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
            gw2[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1t[e * 32 + 16 * mb + (lane & 15)], b2v, gw2[mb][nb], 0, 0, 0);
          gw1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ft[e * 16 + (lane & 15)], b1v, gw1[nb], 0, 0, 0);
        }
      }
      wave_sync();
    }
  }
  if (!TRAIN) return;
  float* out = A.partial + ((int64_t)blockIdx.x * kPfWaves + wave) * kPfGradStride;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[O_W2 + (16 * mb + 4 * g + v) * PF + 16 * nb + (lane & 15)] = gw2[mb][nb][v];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * g + v < 6) out[O_W1 + (4 * g + v) * PF + 16 * nb + (lane & 15)] = gw1[nb][v];
  // column sums of the per-lane vectors: reduce over the 16 columns of each lane group
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
      gw3[r] += __shfl_xor(gw3[r], m);
      gb2[r] += __shfl_xor(gb2[r], m);
      gb1[r] += __shfl_xor(gb1[r], m);
    }
  if (j == 0)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int c = phi(r, g);
      out[O_W3 + c] = gw3[r];
      out[O_B2 + c] = gb2[r];
      out[O_B1 + c] = gb1[r];
    }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    gb3 += __shfl_xor(gb3, m);
    loss += __shfl_xor(loss, m);
  }
  if (lane == 0) {
    out[O_B3] = gb3;
    out[N_P] = loss * inv_n;
  }
}

// Gradient = sum of the per-wave partials in a fixed order (deterministic):
// the waves are cut into kPfChunks chunks of consecutive waves, each summed
// in wave order by its own thread per parameter (the result replaces the
// chunk's first row, which only that thread reads), then the chunk sums are
// added in chunk order.
constexpr int kPfChunks = 64;

__global__ void k_pf_reduce_chunks(float* __restrict__ partial, int n_waves, const int64_t* status) {
  if (status[0] != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = (n_waves + kPfChunks - 1) / kPfChunks;
  const int w0 = blockIdx.y * per, w1 = min(w0 + per, n_waves);
  if (i > N_P || w0 >= w1) return;
  float s = 0.f;
  int w = w0;
  for (; w + 8 <= w1; w += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(w + u) * kPfGradStride + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; w < w1; ++w) s += partial[(int64_t)w * kPfGradStride + i];
  partial[(int64_t)w0 * kPfGradStride + i] = s;
}

__global__ void k_pf_reduce(const float* __restrict__ partial, int n_waves, float* __restrict__ grad, float* loss,
                            const int64_t* status) {
  if (status[0] != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > N_P) return;
  const int per = (n_waves + kPfChunks - 1) / kPfChunks;
  float s = 0.f;
  for (int w0 = 0; w0 < n_waves; w0 += per) s += partial[(int64_t)w0 * kPfGradStride + i];
  grad[i] = s;
  if (i == N_P && loss) *loss = s;
}

__global__ void k_pf_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                          const float* __restrict__ grad, float lr, float b1, float b2, float eps, float c1, float c2,
                          const int64_t* status) {
  if (status[0] != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N_P) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Fallback to the unpruned graph: an event whose kept fraction of candidates
// lies outside [lo, hi] (the band validated when tau was chosen) keeps every
// candidate.  One workgroup per event: a block sum of its keep flags, then, if
// the event falls back, every flag of its candidate range set.
__global__ __launch_bounds__(256) void k_pf_band(int64_t n_events, const int64_t* __restrict__ hit_off,
                                                 const int64_t* __restrict__ cand_ptr, uint8_t* __restrict__ keep,
                                                 float lo, float hi, int32_t* __restrict__ fallback,
                                                 const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int part[4];
  for (int64_t e = blockIdx.x; e < n_events; e += gridDim.x) {
    const int64_t c0 = cand_ptr[hit_off[e]], c1 = cand_ptr[hit_off[e + 1]];
    int cnt = 0;
    for (int64_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) cnt += keep[q];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) cnt += __shfl_xor(cnt, m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    const int64_t total = (int64_t)part[0] + part[1] + part[2] + part[3];
    const int64_t n = c1 - c0;
    const double frac = n > 0 ? (double)total / (double)n : 1.0;
    const bool fb = n > 0 && (frac < (double)lo || frac > (double)hi);
    if (fb)
      for (int64_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) keep[q] = 1;
    if (threadIdx.x == 0) fallback[e] = fb ? 1 : 0;
    __syncthreads();     // part[] is reused by the next event
  }
}

// Surviving candidates per source (!WRITE) and their compaction into the
// output edge list (WRITE).  A workgroup takes 256 sources at a time; their
// candidate rows are one contiguous range, read 256 candidates per round
// (coalesced).  Counting adds each kept candidate to its source's LDS
// counter; compaction gives a kept candidate the rank of its keep flag in
// the range (wave ballots, then the waves' sums in order) past the output
// offset of the first source, which is where the per-source walk put it.
constexpr int kPfRowHits = 256;

template <bool WRITE>
__global__ __launch_bounds__(kPfRowHits) void k_pf_rows(int64_t n_hits, const int64_t* __restrict__ cand_ptr,
                                                        const uint8_t* __restrict__ keep, int32_t* __restrict__ cnt,
                                                        const int64_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ csrc, const int32_t* __restrict__ cdst,
                                                        int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                        const int64_t* status) {
  if (status[0] != 0) return;
  constexpr int kWaves = kPfRowHits / 64;
  __shared__ int lc[kPfRowHits];
  __shared__ int wsum[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t h0 = (int64_t)blockIdx.x * kPfRowHits; h0 < n_hits; h0 += (int64_t)gridDim.x * kPfRowHits) {
    const int64_t h1 = min(h0 + kPfRowHits, n_hits);
    const int64_t q0 = cand_ptr[h0], q1 = cand_ptr[h1];
    if (!WRITE) {
      lc[threadIdx.x] = 0;
      __syncthreads();
    }
    int64_t out = WRITE ? row_ptr[h0] : 0;
    for (int64_t b = q0; b < q1; b += kPfRowHits) {
      const int64_t q = b + threadIdx.x;
      const bool k = q < q1 && keep[q] != 0;
      if (!WRITE) {
        // the candidate's source is its row's hit, one of this block's
        const int r = k ? csrc[q] - (int)h0 : -1;
        if (r >= 0 && r < kPfRowHits) atomicAdd(&lc[r], 1);
      } else {
        const uint64_t m = __ballot(k);
        if (lane == 0) wsum[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          before += w < wave ? wsum[w] : 0;
          total += wsum[w];
        }
        if (k) {
          const int64_t pos = out + before + __popcll(m & ((1ull << lane) - 1ull));
          src[pos] = csrc[q];
          dst[pos] = cdst[q];
        }
        out += total;
        __syncthreads();   // wsum is reused by the next round
      }
    }
    if (!WRITE) {
      __syncthreads();
      if (h0 + threadIdx.x < h1) cnt[h0 + threadIdx.x] = lc[threadIdx.x];
      __syncthreads();     // lc is cleared for the next block of sources
    }
  }
}

PfArgs pf_args(const RunArgs& a, bool candidates) {
  PfArgs A{};
  A.n_hits = a.hits.n_hits;
  A.x = a.hits.x;
  A.y = a.hits.y;
  A.z = a.hits.z;
  A.emb = reinterpret_cast<const float*>(a.ws + a.L.emb);
  A.polar = reinterpret_cast<const float2*>(a.ws + a.L.pf_polar);
  A.row_ptr = reinterpret_cast<const int64_t*>(a.ws + (candidates ? a.L.pf_tmp : a.L.row_ptr));
  A.src = candidates ? reinterpret_cast<const int32_t*>(a.ws + a.L.cand_src) : a.out.src;
  A.dst = candidates ? reinterpret_cast<const int32_t*>(a.ws + a.L.cand_dst) : a.out.dst;
  A.params = a.ctx->dev_pf;
  A.inv_r = 1.0f / a.ctx->cfg.r_scale_mm;
  A.inv_z = 1.0f / a.ctx->cfg.z_scale_mm;
  A.tau = a.ctx->cfg.prefilter_tau;
  A.keep = reinterpret_cast<uint8_t*>(a.ws + a.L.pf_keep);
  A.prob = reinterpret_cast<float*>(a.ws + a.L.pf_prob);
  A.feat = a.ctx->pf_features ? reinterpret_cast<float*>(a.ws + a.L.pf_feat) : nullptr;
  A.partial = reinterpret_cast<float*>(a.ws + a.L.pf_part);
  A.status = a.out.status;
  return A;
}

unsigned pf_grid(const etx_ctx* c) { return (unsigned)std::min(c->n_cu * 2, kPfMaxWaves / kPfWaves); }

}  // namespace

static void launch_polar(const RunArgs& a) {
  if (a.hits.n_hits == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((a.hits.n_hits + 255) / 256, (int64_t)a.ctx->n_cu * 16);
  hipLaunchKernelGGL(k_hit_polar, dim3(grid), dim3(256), 0, a.stream, a.hits.n_hits, a.hits.x, a.hits.y,
                     reinterpret_cast<float2*>(a.ws + a.L.pf_polar), a.out.status);
}

hipError_t launch_prefilter_infer(const RunArgs& a) {
  PfArgs A = pf_args(a, true);
  launch_polar(a);
  // inference keeps no per-wave partials: a full grid of persistent waves
  if (a.ctx->cfg.emb_dim <= 8)
    hipLaunchKernelGGL((k_pf<false, 8>), dim3((unsigned)(a.ctx->n_cu * 4)), dim3(kPfThreads), 0, a.stream, A);
  else
    hipLaunchKernelGGL((k_pf<false, 16>), dim3((unsigned)(a.ctx->n_cu * 4)), dim3(kPfThreads), 0, a.stream, A);
  return hipGetLastError();
}

hipError_t launch_prefilter_band(const RunArgs& a) {
  if (a.hits.n_events == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(a.hits.n_events, (int64_t)a.ctx->n_cu * 8);
  hipLaunchKernelGGL(k_pf_band, dim3(grid), dim3(256), 0, a.stream, a.hits.n_events, a.hits.hit_off,
                     reinterpret_cast<const int64_t*>(a.ws + a.L.pf_tmp), reinterpret_cast<uint8_t*>(a.ws + a.L.pf_keep),
                     a.ctx->pf_band_lo, a.ctx->pf_band_hi, reinterpret_cast<int32_t*>(a.ws + a.L.pf_fallback),
                     a.out.status);
  return hipGetLastError();
}

hipError_t launch_prefilter_count(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((a.hits.n_hits + kPfRowHits - 1) / kPfRowHits, (int64_t)a.ctx->n_cu * 16);
  hipLaunchKernelGGL(k_pf_rows<false>, dim3(grid), dim3(kPfRowHits), 0, a.stream, a.hits.n_hits,
                     reinterpret_cast<const int64_t*>(a.ws + a.L.pf_tmp),
                     reinterpret_cast<const uint8_t*>(a.ws + a.L.pf_keep), reinterpret_cast<int32_t*>(a.ws + a.L.cnt),
                     nullptr, reinterpret_cast<const int32_t*>(a.ws + a.L.cand_src), nullptr, nullptr, nullptr,
                     a.out.status);
  return hipGetLastError();
}

hipError_t launch_prefilter_compact(const RunArgs& a) {
  if (a.hits.n_hits == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((a.hits.n_hits + kPfRowHits - 1) / kPfRowHits, (int64_t)a.ctx->n_cu * 16);
  hipLaunchKernelGGL(k_pf_rows<true>, dim3(grid), dim3(kPfRowHits), 0, a.stream, a.hits.n_hits,
                     reinterpret_cast<const int64_t*>(a.ws + a.L.pf_tmp),
                     reinterpret_cast<const uint8_t*>(a.ws + a.L.pf_keep), nullptr,
                     reinterpret_cast<const int64_t*>(a.ws + a.L.row_ptr),
                     reinterpret_cast<const int32_t*>(a.ws + a.L.cand_src),
                     reinterpret_cast<const int32_t*>(a.ws + a.L.cand_dst), a.out.src, a.out.dst, a.out.status);
  return hipGetLastError();
}

hipError_t launch_prefilter_train(const RunArgs& a, const uint8_t* labels, float lr, float pos_weight, int64_t step,
                                  float* loss_dev) {
  PfArgs A = pf_args(a, false);
  A.label = labels;
  A.pos_weight = pos_weight;
  launch_polar(a);
  const unsigned grid = pf_grid(a.ctx);
  if (a.ctx->cfg.emb_dim <= 8)
    hipLaunchKernelGGL((k_pf<true, 8>), dim3(grid), dim3(kPfThreads), 0, a.stream, A);
  else
    hipLaunchKernelGGL((k_pf<true, 16>), dim3(grid), dim3(kPfThreads), 0, a.stream, A);
  float* grad = reinterpret_cast<float*>(a.ws + a.L.pf_grad);
  hipLaunchKernelGGL(k_pf_reduce_chunks, dim3((N_P + 1 + 255) / 256, kPfChunks), dim3(256), 0, a.stream, A.partial,
                     (int)(grid * kPfWaves), a.out.status);
  hipLaunchKernelGGL(k_pf_reduce, dim3((N_P + 1 + 255) / 256), dim3(256), 0, a.stream, A.partial,
                     (int)(grid * kPfWaves), grad, loss_dev, a.out.status);
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, (double)step)), c2 = (float)(1.0 - std::pow(b2, (double)step));
  float* p = a.ctx->dev_pf;
  hipLaunchKernelGGL(k_pf_adam, dim3((N_P + 255) / 256), dim3(256), 0, a.stream, p, p + N_P, p + 2 * N_P, grad, lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2, a.out.status);
  return hipGetLastError();
}

int prefilter_attributes(size_t) { return 0; }

}  // namespace etx
