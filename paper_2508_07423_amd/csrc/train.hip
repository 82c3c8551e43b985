// In-library training of the embedding MLP and the interaction network
// (thesis ch. 8 "Hit Embedding and Rough Graph Construction", eqs. loss1-loss3,
// and "Graph Neural Network and Classifiers", eq. gnn-loss without the triplet
// term): forward passes that keep what the backward needs, reverse-mode
// gradients layer by layer, and Adam on FP32 master parameters.
//
// Every layer is a row-wise kernel: one thread per row (a hit or an edge)
// holds the row's outputs in registers, reads its input from up to three
// segments (each a row of a node or edge buffer, directly or through a
// source / target index), and takes the layer's weights from LDS.  The weight
// gradients are sums over rows: every chunk of rows adds its rows in order
// into a partial, and the partials are added in chunk order, so a training
// step is bitwise reproducible.  The transpose of a gather by source (target)
// is a sum over the node's out-edges (in-edges), taken through the CSR rows
// (the CSC permutation); the transpose of the out-/in-sums is a gather.
#include <cmath>

#include "internal.hpp"
#include "train.hpp"

namespace etx {

namespace {

constexpr int kRowThreads = 128;
constexpr int kWgradThreads = 256;

__device__ inline float seg_x(const TrainSeg& s, int64_t r, int k) {
  const int64_t row = s.idx ? (int64_t)s.idx[r] : r;
  return s.base[row * s.ld + k];
}

// y = act(x W + b) per row; ACT 0 none, 1 ReLU, 2 LayerNorm (no affine,
// biased variance, eps 1e-5) then ReLU.  yhat keeps z (ACT 0, 1) or the
// normalised value before the ReLU (ACT 2); rstd its reciprocal standard
// deviation (ACT 2).  resid (optional): y = resid + act(...).
template <int M, int ACT>
__global__ __launch_bounds__(kRowThreads) void k_blk_fwd(BlkFwd A) {
  if (A.status[0] != 0) return;
  extern __shared__ float w[];
  const int K = A.K;
  for (int i = threadIdx.x; i < K * M + M; i += blockDim.x) w[i] = A.W[i];
  __syncthreads();
  const float* b = w + K * M;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < A.rows; r += (int64_t)gridDim.x * blockDim.x) {
    float z[M];
#pragma unroll
    for (int m = 0; m < M; ++m) z[m] = b[m];
    int ko = 0;
    for (int s = 0; s < A.nseg; ++s) {
      const TrainSeg& g = A.seg[s];
      const int64_t row = g.idx ? (int64_t)g.idx[r] : r;
      const float* x = g.base + row * g.ld;
      for (int k = 0; k < g.width; ++k) {
        const float xv = x[k];
        const float* wk = w + (ko + k) * M;
#pragma unroll
        for (int m = 0; m < M; ++m) z[m] = fmaf(xv, wk[m], z[m]);
      }
      ko += g.width;
    }
    float* yh = A.yhat ? A.yhat + r * M : nullptr;
    float* y = A.y + r * A.ldy;
    const float* res = A.resid ? A.resid + r * A.ldy : nullptr;
    if (ACT == 2) {
      float mean = 0.f;
#pragma unroll
      for (int m = 0; m < M; ++m) mean += z[m];
      mean *= 1.0f / M;
      float var = 0.f;
#pragma unroll
      for (int m = 0; m < M; ++m) var = fmaf(z[m] - mean, z[m] - mean, var);
      const float rs = 1.0f / sqrtf(var * (1.0f / M) + 1e-5f);
      A.rstd[r] = rs;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const float t = (z[m] - mean) * rs;
        if (yh) yh[m] = t;
        const float v = fmaxf(t, 0.f);
        y[m] = res ? res[m] + v : v;
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (yh) yh[m] = z[m];
        const float v = ACT == 1 ? fmaxf(z[m], 0.f) : z[m];
        y[m] = res ? res[m] + v : v;
      }
    }
    for (int m = M; m < A.ldy && A.pad_zero; ++m) y[m] = 0.f;
  }
}

// dz = d(act)/dz applied to dy (+ dy2); dx = W dz into the input segments'
// gradient buffers (written, or added to, per segment).
template <int M, int ACT>
__global__ __launch_bounds__(kRowThreads) void k_blk_bwd(BlkBwd A) {
  if (A.status[0] != 0) return;
  extern __shared__ float w[];
  const int K = A.K;
  for (int i = threadIdx.x; i < K * M; i += blockDim.x) w[i] = A.W[i];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < A.rows; r += (int64_t)gridDim.x * blockDim.x) {
    float dz[M];
    const float* dy = A.dy + r * A.lddy;
    const float* dy2 = A.dy2 ? A.dy2 + r * A.lddy : nullptr;
    const float* yh = A.yhat + r * M;
#pragma unroll
    for (int m = 0; m < M; ++m) dz[m] = dy2 ? dy[m] + dy2[m] : dy[m];
    if (ACT == 2) {
      float mg = 0.f, mgy = 0.f;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        dz[m] = yh[m] > 0.f ? dz[m] : 0.f;
        mg += dz[m];
        mgy = fmaf(dz[m], yh[m], mgy);
      }
      mg *= 1.0f / M;
      mgy *= 1.0f / M;
      const float rs = A.rstd[r];
#pragma unroll
      for (int m = 0; m < M; ++m) dz[m] = rs * (dz[m] - mg - yh[m] * mgy);
    } else if (ACT == 1) {
#pragma unroll
      for (int m = 0; m < M; ++m) dz[m] = yh[m] > 0.f ? dz[m] : 0.f;
    }
    float* dzo = A.dz + r * M;
#pragma unroll
    for (int m = 0; m < M; ++m) dzo[m] = dz[m];
    int ko = 0;
    for (int s = 0; s < A.nseg; ++s) {
      const TrainOut& o = A.out[s];
      if (o.base) {
        float* dx = o.base + r * o.ld;
        for (int k = 0; k < o.width; ++k) {
          const float* wk = w + (ko + k) * M;
          float v = 0.f;
#pragma unroll
          for (int m = 0; m < M; ++m) v = fmaf(wk[m], dz[m], v);
          dx[k] = o.add ? dx[k] + v : v;
        }
      }
      ko += o.width;
    }
  }
}

// weight gradient partials: chunk c adds, row by row in order, x_r[k] dz_r[m]
// (and dz_r[m] for the bias) over its rows; one thread per output
template <int M>
__global__ __launch_bounds__(kWgradThreads) void k_wgrad(Wgrad A) {
  if (A.status[0] != 0) return;
  const int K = A.K;
  const int n_out = K * M + M;
  const int o = blockIdx.y * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  const int64_t per = (A.rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < A.rows ? r0 + per : A.rows;
  float acc = 0.f;
  if (o < K * M) {
    const int k = o / M, m = o % M;
    // the segment holding input feature k
    int s = 0, kk = k;
    while (kk >= A.seg[s].width) kk -= A.seg[s++].width;
    const TrainSeg g = A.seg[s];
    for (int64_t r = r0; r < r1; ++r) acc = fmaf(seg_x(g, r, kk), A.dz[r * M + m], acc);
  } else {
    const int m = o - K * M;
    for (int64_t r = r0; r < r1; ++r) acc += A.dz[r * M + m];
  }
  A.partial[(int64_t)blockIdx.x * n_out + o] = acc;
}

// grad[o] (+)= sum of the chunk partials in chunk order
__global__ void k_reduce_partials(const float* __restrict__ partial, int n_chunks, int n_out, float* __restrict__ grad,
                                  const int64_t* status) {
  if (status[0] != 0) return;
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  float s = 0.f;
  for (int c = 0; c < n_chunks; ++c) s += partial[(int64_t)c * n_out + o];
  grad[o] = s;
}

// out[l] (+)= sum over l's out-edges (CSR rows, in edge order) of a[t], plus
// the sum over its in-edges (CSC permutation, in CSC order) of b[t]
__global__ void k_node_sum(int64_t n, int H, const int64_t* __restrict__ row_ptr, const float* __restrict__ a,
                           const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ csc,
                           const float* __restrict__ b, float* __restrict__ out, int add, const int64_t* status) {
  if (status[0] != 0) return;
  const int64_t total = n * H;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / H;
    const int f = (int)(i % H);
    float s = add ? out[i] : 0.f;
    if (a)
      for (int64_t t = row_ptr[l]; t < row_ptr[l + 1]; ++t) s += a[t * H + f];
    if (b)
      for (int64_t q = col_ptr[l]; q < col_ptr[l + 1]; ++q) s += b[(int64_t)csc[q] * H + f];
    out[i] = s;
  }
}

// out[t] += A[src[t]] + B[dst[t]]
__global__ void k_edge_gather_add(int64_t E, int H, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                  const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ out,
                                  const int64_t* status) {
  if (status[0] != 0) return;
  const int64_t total = E * H;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = i / H;
    const int f = (int)(i % H);
    out[i] += A[(int64_t)src[t] * H + f] + B[(int64_t)dst[t] * H + f];
  }
}

// the network's inputs: normalised Cartesian (x/R, y/R, z/Z) per hit
__global__ void k_cart(int64_t n, const float* x, const float* y, const float* z, float inv_r, float inv_z,
                       float* __restrict__ cart, const int64_t* status) {
  if (status[0] != 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    cart[3 * i] = x[i] * inv_r;
    cart[3 * i + 1] = y[i] * inv_r;
    cart[3 * i + 2] = z[i] * inv_z;
  }
}

// the embedding's inputs: (r/R, phi/pi, z/Z) per hit
__global__ void k_cyl(int64_t n, const float* x, const float* y, const float* z, float inv_r, float inv_z,
                      float* __restrict__ cyl, const int64_t* status) {
  if (status[0] != 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    cyl[3 * i] = hypotf(x[i], y[i]) * inv_r;
    cyl[3 * i + 1] = atan2f(y[i], x[i]) * (1.0f / 3.14159265358979f);
    cyl[3 * i + 2] = z[i] * inv_z;
  }
}

// an edge is genuine when its target is the source's successor on one of its particles
__global__ void k_edge_labels(int64_t E, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                              const int32_t* __restrict__ succ, const int32_t* __restrict__ succ2,
                              uint8_t* __restrict__ lab, const int64_t* status) {
  if (status[0] != 0) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < E; t += (int64_t)gridDim.x * blockDim.x)
    lab[t] = (succ[src[t]] == dst[t] || (succ2 && succ2[src[t]] == dst[t])) ? 1 : 0;
}

// Sigmoid focal loss of every edge (Lin et al.): logit z = c w2 + b2; per-edge
// dL/dz / E into dlogit, dL/dc = w2 dlogit into dc, and the loss per block.
__global__ __launch_bounds__(256) void k_focal(int64_t E, int H, const float* __restrict__ c,
                                               const float* __restrict__ w2, const uint8_t* __restrict__ lab,
                                               float alpha, float gamma, float* __restrict__ dlogit,
                                               float* __restrict__ dc, float* __restrict__ loss_part,
                                               float* __restrict__ score, const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ float part[256];
  float acc = 0.f;
  const float inv_e = E > 0 ? 1.0f / (float)E : 0.f;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < E; t += (int64_t)gridDim.x * blockDim.x) {
    float z = w2[H];
    for (int q = 0; q < H; ++q) z = fmaf(c[t * H + q], w2[q], z);
    const float p = 1.0f / (1.0f + expf(-z));
    if (score) score[t] = p;
    const float lp = -(z < 0.f ? -z + log1pf(expf(z)) : log1pf(expf(-z)));     // log p
    const float l1p = -(z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z)));     // log (1 - p)
    float l, d;
    if (lab[t]) {
      const float wt = powf(1.f - p, gamma);
      l = -alpha * wt * lp;
      d = alpha * wt * (gamma * p * lp - (1.f - p));
    } else {
      const float wt = powf(p, gamma);
      l = -(1.f - alpha) * wt * l1p;
      d = (1.f - alpha) * wt * (p - gamma * (1.f - p) * l1p);
    }
    acc += l;
    d *= inv_e;
    dlogit[t] = d;
    for (int q = 0; q < H; ++q) dc[t * H + q] = w2[q] * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = part[0] * inv_e;
}

// loss = sum of the block partials in block order
__global__ void k_sum(const float* __restrict__ part, int n, float* __restrict__ out, int slot, const int64_t* status) {
  if (status[0] != 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += part[i];
    out[slot] = s;
  }
}

__global__ void k_adam(int64_t n, float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2,
                       const int64_t* status) {
  if (status[0] != 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------------------
// pairwise hinge loss of the embedding
// ---------------------------------------------------------------------------

// Pairs of query q (a hit of a particle with at least three hits): its
// genuine pair (q, succ[q]); fake pairs: its hard negatives (the targets of
// the training radius graph that belong to a particle and are not succ[q])
// and its random pair (q, rnd[q]) unless that is succ[q].  Pass 0 counts them
// per block; pass 1 writes, per pair, g = dL/de_q (its negative is dL/de_b)
// and adds the loss.
template <int D>
__global__ __launch_bounds__(256) void k_hinge(HingeArgs A, int pass) {
  if (A.status[0] != 0) return;
  __shared__ float part[3][256];
  float n_gen = 0.f, n_fake = 0.f, loss = 0.f;
  float inv_g = 0.f, inv_f = 0.f;
  if (pass == 1) {
    inv_g = A.counts[0] > 0.f ? 1.0f / A.counts[0] : 0.f;
    inv_f = A.counts[1] > 0.f ? 1.0f / A.counts[1] : 0.f;
  }
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < A.n; q += (int64_t)gridDim.x * blockDim.x) {
    float eq[D], gq[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      eq[k] = A.emb[q * A.lde + k];
      gq[k] = 0.f;
    }
    const bool query = A.query[q] != 0;
    const int sq = A.succ[q];
    auto pair = [&](int b, bool genuine, float* gout) {
      float d2 = 0.f, diff[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        diff[k] = eq[k] - A.emb[(int64_t)b * A.lde + k];
        d2 = fmaf(diff[k], diff[k], d2);
      }
      float c = 0.f;
      if (genuine) {
        loss += A.w_gen * d2 * inv_g;
        c = 2.f * A.w_gen * inv_g;
      } else if (A.margin - d2 > 0.f) {
        loss += (A.margin - d2) * inv_f;
        c = -2.f * inv_f;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float v = c * diff[k];
        gq[k] += v;
        if (gout) gout[k] = v;
      }
    };
    // genuine
    if (query && sq >= 0) {
      n_gen += 1.f;
      if (pass == 1) pair(sq, true, A.g_gen + q * D);
    } else if (pass == 1) {
#pragma unroll
      for (int k = 0; k < D; ++k) A.g_gen[q * D + k] = 0.f;
    }
    // hard negatives: the training radius graph's row of q
    for (int64_t t = A.row_ptr[q]; t < A.row_ptr[q + 1]; ++t) {
      const int b = A.dst[t];
      const bool fake = query && A.particle[b] >= 0 && b != sq;
      if (fake) n_fake += 1.f;
      if (pass == 1) {
        if (fake) {
          pair(b, false, A.g_edge + t * D);
        } else {
#pragma unroll
          for (int k = 0; k < D; ++k) A.g_edge[t * D + k] = 0.f;
        }
      }
    }
    // random pair
    const int rb = A.rnd[q];
    const bool rfake = query && rb >= 0 && rb != sq;
    if (rfake) n_fake += 1.f;
    if (pass == 1) {
      if (rfake) {
        pair(rb, false, A.g_rnd + q * D);
      } else {
#pragma unroll
        for (int k = 0; k < D; ++k) A.g_rnd[q * D + k] = 0.f;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) A.de[q * A.ldde + k] = gq[k];
    }
  }
  part[0][threadIdx.x] = n_gen;
  part[1][threadIdx.x] = n_fake;
  part[2][threadIdx.x] = loss;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int j = 0; j < 3; ++j) part[j][threadIdx.x] += part[j][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) A.block_part[(int64_t)blockIdx.x * 3 + j] = part[j][0];
}

__global__ void k_hinge_counts(const float* __restrict__ block_part, int n_blocks, float* __restrict__ counts,
                               float* loss_out, const int64_t* status) {
  if (status[0] != 0) return;
  if (blockIdx.x == 0 && threadIdx.x < 3) {
    float s = 0.f;
    for (int i = 0; i < n_blocks; ++i) s += block_part[(int64_t)i * 3 + threadIdx.x];
    if (threadIdx.x < 2) counts[threadIdx.x] = s;
    else if (loss_out) *loss_out = s;
  }
}

// the other end of every pair: de[b] -= the pair's g, over b's in-edges of the
// training graph (CSC order), its predecessor's genuine pair and the random
// pairs that picked b (given grouped by target, in order)
template <int D>
__global__ void k_hinge_bside(HingeArgs A) {
  if (A.status[0] != 0) return;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < A.n; b += (int64_t)gridDim.x * blockDim.x) {
    float s[D];
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] = 0.f;
    for (int64_t q = A.col_ptr[b]; q < A.col_ptr[b + 1]; ++q) {
      const int64_t t = A.csc[q];
#pragma unroll
      for (int k = 0; k < D; ++k) s[k] += A.g_edge[t * D + k];
    }
    const int p = A.pred[b];
    if (p >= 0)
#pragma unroll
      for (int k = 0; k < D; ++k) s[k] += A.g_gen[(int64_t)p * D + k];
    for (int64_t i = A.rnd_ptr[b]; i < A.rnd_ptr[b + 1]; ++i) {
      const int q = A.rnd_src[i];
#pragma unroll
      for (int k = 0; k < D; ++k) s[k] += A.g_rnd[(int64_t)q * D + k];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) A.de[b * A.ldde + k] -= s[k];
  }
}

unsigned row_grid(int64_t rows, const etx_ctx* c) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + kRowThreads - 1) / kRowThreads, (int64_t)c->n_cu * 8));
}

unsigned flat_grid(int64_t n, const etx_ctx* c) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, (int64_t)c->n_cu * 16));
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define BY_M(M_, FN) \
  case M_: FN(M_); break;

hipError_t launch_blk_fwd(const BlkFwd& A, int M, int act, hipStream_t s, const etx_ctx* c) {
  if (A.rows == 0) return hipSuccess;
  const size_t lds = sizeof(float) * ((size_t)A.K * M + M);
  const unsigned g = row_grid(A.rows, c);
#define L(M_)                                                                                        \
  if (act == 2) hipLaunchKernelGGL((k_blk_fwd<M_, 2>), dim3(g), dim3(kRowThreads), lds, s, A);       \
  else if (act == 1) hipLaunchKernelGGL((k_blk_fwd<M_, 1>), dim3(g), dim3(kRowThreads), lds, s, A); \
  else hipLaunchKernelGGL((k_blk_fwd<M_, 0>), dim3(g), dim3(kRowThreads), lds, s, A);
  switch (M) {
    BY_M(1, L) BY_M(4, L) BY_M(8, L) BY_M(12, L) BY_M(16, L) BY_M(32, L) BY_M(64, L) BY_M(128, L)
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

hipError_t launch_blk_bwd(const BlkBwd& A, int M, int act, hipStream_t s, const etx_ctx* c) {
  if (A.rows == 0) return hipSuccess;
  const size_t lds = sizeof(float) * (size_t)A.K * M;
  const unsigned g = row_grid(A.rows, c);
#define L(M_)                                                                                        \
  if (act == 2) hipLaunchKernelGGL((k_blk_bwd<M_, 2>), dim3(g), dim3(kRowThreads), lds, s, A);       \
  else if (act == 1) hipLaunchKernelGGL((k_blk_bwd<M_, 1>), dim3(g), dim3(kRowThreads), lds, s, A); \
  else hipLaunchKernelGGL((k_blk_bwd<M_, 0>), dim3(g), dim3(kRowThreads), lds, s, A);
  switch (M) {
    BY_M(1, L) BY_M(4, L) BY_M(8, L) BY_M(12, L) BY_M(16, L) BY_M(32, L) BY_M(64, L) BY_M(128, L)
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

hipError_t launch_wgrad(const Wgrad& A, int M, float* grad, hipStream_t s) {
  const int n_out = A.K * M + M;
  const int chunks = kTrainChunks;
  dim3 grid(chunks, (n_out + kWgradThreads - 1) / kWgradThreads);
#define L(M_) hipLaunchKernelGGL((k_wgrad<M_>), grid, dim3(kWgradThreads), 0, s, A);
  switch (M) {
    BY_M(1, L) BY_M(4, L) BY_M(8, L) BY_M(12, L) BY_M(16, L) BY_M(32, L) BY_M(64, L) BY_M(128, L)
    default: return hipErrorInvalidValue;
  }
#undef L
  hipLaunchKernelGGL(k_reduce_partials, dim3((n_out + 255) / 256), dim3(256), 0, s, A.partial, chunks, n_out, grad,
                     A.status);
  return hipGetLastError();
}
#undef BY_M

hipError_t launch_node_sum(int64_t n, int H, const int64_t* row_ptr, const float* a, const int64_t* col_ptr,
                           const int32_t* csc, const float* b, float* out, int add, const int64_t* status,
                           hipStream_t s, const etx_ctx* c) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_sum, dim3(flat_grid(n * H, c)), dim3(256), 0, s, n, H, row_ptr, a, col_ptr, csc, b, out,
                     add, status);
  return hipGetLastError();
}

hipError_t launch_edge_gather_add(int64_t E, int H, const int32_t* src, const int32_t* dst, const float* A,
                                  const float* B, float* out, const int64_t* status, hipStream_t s, const etx_ctx* c) {
  if (E == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_gather_add, dim3(flat_grid(E * H, c)), dim3(256), 0, s, E, H, src, dst, A, B, out, status);
  return hipGetLastError();
}

hipError_t launch_inputs(int64_t n, const float* x, const float* y, const float* z, float inv_r, float inv_z,
                         float* cart, float* cyl, const int64_t* status, hipStream_t s, const etx_ctx* c) {
  if (n == 0) return hipSuccess;
  if (cart) hipLaunchKernelGGL(k_cart, dim3(flat_grid(n, c)), dim3(256), 0, s, n, x, y, z, inv_r, inv_z, cart, status);
  if (cyl) hipLaunchKernelGGL(k_cyl, dim3(flat_grid(n, c)), dim3(256), 0, s, n, x, y, z, inv_r, inv_z, cyl, status);
  return hipGetLastError();
}

hipError_t launch_edge_labels(int64_t E, const int32_t* src, const int32_t* dst, const int32_t* succ,
                              const int32_t* succ2, uint8_t* lab, const int64_t* status, hipStream_t s,
                              const etx_ctx* c) {
  if (E == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_labels, dim3(flat_grid(E, c)), dim3(256), 0, s, E, src, dst, succ, succ2, lab, status);
  return hipGetLastError();
}

hipError_t launch_focal(int64_t E, int H, const float* cls_out, const float* w2, const uint8_t* lab, float alpha,
                        float gamma, float* dlogit, float* dc, float* loss_part, float* loss_out, int slot,
                        const int64_t* status, hipStream_t s, float* score) {
  hipLaunchKernelGGL(k_focal, dim3(kTrainLossBlocks), dim3(256), 0, s, E, H, cls_out, w2, lab, alpha, gamma, dlogit,
                     dc, loss_part, score, status);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, loss_part, kTrainLossBlocks, loss_out, slot, status);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* p, float* m, float* v, const float* g, float lr, int64_t step,
                       const int64_t* status, hipStream_t s, const etx_ctx* c) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, (double)step)), c2 = (float)(1.0 - std::pow(b2, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(flat_grid(n, c)), dim3(256), 0, s, n, p, m, v, g, lr, (float)b1, (float)b2, 1e-8f,
                     c1, c2, status);
  return hipGetLastError();
}

hipError_t launch_hinge(const HingeArgs& A, int D, float* loss_out, hipStream_t s) {
#define L(D_)                                                                                   \
  hipLaunchKernelGGL((k_hinge<D_>), dim3(kTrainLossBlocks), dim3(256), 0, s, A, 0);             \
  hipLaunchKernelGGL(k_hinge_counts, dim3(1), dim3(64), 0, s, A.block_part, kTrainLossBlocks,   \
                     const_cast<float*>(A.counts), nullptr, A.status);                           \
  hipLaunchKernelGGL((k_hinge<D_>), dim3(kTrainLossBlocks), dim3(256), 0, s, A, 1);             \
  hipLaunchKernelGGL(k_hinge_counts, dim3(1), dim3(64), 0, s, A.block_part, kTrainLossBlocks,   \
                     A.counts_scratch, loss_out, A.status);                                      \
  hipLaunchKernelGGL((k_hinge_bside<D_>), dim3(256), dim3(256), 0, s, A);
  switch (D) {
    case 4: L(4); break;
    case 8: L(8); break;
    case 12: L(12); break;
    case 16: L(16); break;
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

int train_attributes(size_t max_lds) {
  int bad = 0;
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  // the widest layers (embedding hidden size 128) stage 66 KB of weights
  set(reinterpret_cast<const void*>(k_blk_fwd<128, 0>));
  set(reinterpret_cast<const void*>(k_blk_fwd<128, 1>));
  set(reinterpret_cast<const void*>(k_blk_fwd<128, 2>));
  set(reinterpret_cast<const void*>(k_blk_bwd<128, 0>));
  set(reinterpret_cast<const void*>(k_blk_bwd<128, 1>));
  set(reinterpret_cast<const void*>(k_blk_bwd<128, 2>));
  return bad;
}

}  // namespace etx
