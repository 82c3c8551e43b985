// Triplet stage (thesis ch. 8 "The ETX4VELO Pipeline", "Triplet Building" and
// "Track Building"): triplets of the purified hit graph, the two triplet
// classifiers, and track building from the purified edge graph.
//
// Layout.  Around every hit C with kept in-edges I (CSC order, by source) and
// kept out-edges O (CSR order, by target), a = |I|, b = |O|:
//   articulation (I[i], O[o])          at art_pos[C] + i*b + o
//   left elbow   (O[p], O[q]), p < q   at n_art + elb_pos[C] + tri(p, q, b)
//   right elbow  (I[p], I[q]), p < q   at n_art + elb_pos[C] + b(b-1)/2 + tri(p, q, a)
// with tri(p, q, m) = p*m - p(p+1)/2 + q - p - 1 (the row-major upper
// triangle), art_pos / elb_pos the exclusive scans of the per-hit counts and
// n_art the batch's articulation count.  Every triplet of an edge is thus found
// from the edge's rank in its source's out-list and in its target's in-list,
// without a search: the duplicate test and the link-sharing test read the
// triplet scores at computed positions and need no atomics.  The kept flag of
// an edge is its score against the threshold, read where it is needed.
//
// Track building runs on global edge ids: a lock-free union-find over the
// kept, non-duplicate edges of the batch (events never link to each other),
// per-event ballot compaction of the tracks, per-component edge lists, and the
// hits of each track gathered by one wave into an LDS bitmap of its event's
// hits (at most ETX_MAX_EVENT_HITS bits), read back in ascending order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "tile.hpp"

namespace etx {
namespace {

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bool halted(const int64_t* status, const int64_t* tstatus) { return status[0] != 0 || tstatus[0] != 0; }

__device__ inline int64_t tri_idx(int64_t p, int64_t q, int64_t m) { return p * m - p * (p + 1) / 2 + (q - p - 1); }

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// 64-bit wave scan from two 32-bit shuffles
__device__ inline int64_t shfl_up64(int64_t v, int d) {
  const int lo = __shfl_up((int)(v & 0xffffffff), d);
  const int hi = __shfl_up((int)(v >> 32), d);
  return ((int64_t)hi << 32) | (uint32_t)lo;
}

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t t = shfl_up64(v, d);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan over a 256-thread block; *total receives the block's sum.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[4];
  const int64_t inc = wave_incl_scan(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int64_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off += k < w ? wsum[k] : 0;
    tot += wsum[k];
  }
  __syncthreads();   // wsum is reused by the next call
  *total = tot;
  return off + inc - v;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan (counts -> offsets, out[n] = total)
// ---------------------------------------------------------------------------

constexpr int kScanTile = 1024;   // 256 threads x 4 consecutive elements

template <typename T>
__global__ __launch_bounds__(256) void k_scan_sum(const T* __restrict__ in, int64_t n, int64_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += base + k < n ? (int64_t)in[base + k] : 0;
  int64_t tot;
  (void)block_excl_scan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__device__ inline void k_scan_part_body(int64_t* __restrict__ part, int64_t nb, int64_t* __restrict__ total) {
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanTile) {
    const int64_t i0 = c0 + 4 * threadIdx.x;
    int64_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = i0 + k < nb ? part[i0 + k] : 0;
      s += v[k];
    }
    int64_t tot;
    int64_t run = carry + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < nb) part[i0 + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void k_scan_part(int64_t* __restrict__ part, int64_t nb, int64_t* __restrict__ total) {
  k_scan_part_body(part, nb, total);
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(const T* __restrict__ in, int64_t n, const int64_t* __restrict__ part,
                                                    int64_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  int64_t v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = base + k < n ? (int64_t)in[base + k] : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t run = part[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// The same scan over a length known on the device only, clamped to [0, n_max]
// (n_max the buffers' capacity): a fixed grid walks the tiles, so no block is
// launched for the unused tail of a capacity.  Skipped, like every kernel of
// the stage, once a status word holds an error: the length may then never
// have been written.
__device__ inline int64_t dscan_len(const int64_t* n_ptr, int64_t n_max) { return max((int64_t)0, min(*n_ptr, n_max)); }

template <typename T>
__global__ __launch_bounds__(256) void k_dscan_sum(const T* __restrict__ in, const int64_t* __restrict__ n_ptr,
                                                   int64_t n_max, int64_t* __restrict__ part, const int64_t* status,
                                                   const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n = dscan_len(n_ptr, n_max), tiles = (n + kScanTile - 1) / kScanTile;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t base = tile * kScanTile + 4 * threadIdx.x;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) s += base + k < n ? (int64_t)in[base + k] : 0;
    int64_t tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) part[tile] = tot;
  }
}

__global__ __launch_bounds__(256) void k_dscan_part(int64_t* __restrict__ part, const int64_t* __restrict__ n_ptr,
                                                    int64_t n_max, int64_t* __restrict__ out, const int64_t* status,
                                                    const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n = dscan_len(n_ptr, n_max);
  k_scan_part_body(part, (n + kScanTile - 1) / kScanTile, out + n);
}

template <typename T>
__global__ __launch_bounds__(256) void k_dscan_apply(const T* __restrict__ in, const int64_t* __restrict__ n_ptr,
                                                     int64_t n_max, const int64_t* __restrict__ part,
                                                     int64_t* __restrict__ out, const int64_t* status,
                                                     const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n = dscan_len(n_ptr, n_max), tiles = (n + kScanTile - 1) / kScanTile;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t base = tile * kScanTile + 4 * threadIdx.x;
    int64_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = base + k < n ? (int64_t)in[base + k] : 0;
      s += v[k];
    }
    int64_t tot;
    int64_t run = part[tile] + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (base + k < n) out[base + k] = run;
      run += v[k];
    }
  }
}

template <typename T>
hipError_t dscan(const T* in, const int64_t* n_ptr, int64_t n_max, int64_t* out, int64_t* part, int grid,
                 const int64_t* status, const int64_t* tstatus, hipStream_t s) {
  hipLaunchKernelGGL(k_dscan_sum<T>, dim3(grid), dim3(256), 0, s, in, n_ptr, n_max, part, status, tstatus);
  hipLaunchKernelGGL(k_dscan_part, dim3(1), dim3(256), 0, s, part, n_ptr, n_max, out, status, tstatus);
  hipLaunchKernelGGL(k_dscan_apply<T>, dim3(grid), dim3(256), 0, s, in, n_ptr, n_max, part, out, status, tstatus);
  return hipGetLastError();
}

template <typename T>
hipError_t scan(const T* in, int64_t n, int64_t* out, int64_t* part, hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb > 0) hipLaunchKernelGGL(k_scan_sum<T>, dim3((unsigned)nb), dim3(256), 0, s, in, n, part);
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(256), 0, s, part, nb, out + n);
  if (nb > 0) hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(256), 0, s, in, n, part, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// triplets of the purified graph
// ---------------------------------------------------------------------------

__global__ void k_tri_init(int64_t* tstatus) {
  if (threadIdx.x < 4) tstatus[threadIdx.x] = 0;
}

// kept in- and out-degree of every hit, and its triplet counts
__global__ __launch_bounds__(256) void k_tri_degrees(int64_t n, const int64_t* __restrict__ row_ptr,
                                                     const int64_t* __restrict__ col_ptr,
                                                     const int32_t* __restrict__ csc, const float* __restrict__ score,
                                                     float thr, int32_t* __restrict__ deg_in,
                                                     int32_t* __restrict__ deg_out, int64_t* __restrict__ cnt_art,
                                                     int64_t* __restrict__ cnt_elb, const int64_t* status,
                                                     const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    int64_t b = 0, a = 0;
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) b += score[q] >= thr ? 1 : 0;
    for (int64_t q = col_ptr[i]; q < col_ptr[i + 1]; ++q) a += score[csc[q]] >= thr ? 1 : 0;
    deg_in[i] = (int32_t)a;
    deg_out[i] = (int32_t)b;
    cnt_art[i] = a * b;
    cnt_elb[i] = b * (b - 1) / 2 + a * (a - 1) / 2;
  }
}

// per-event offsets of the two lists, and the capacity check
__global__ __launch_bounds__(256) void k_tri_offsets(int64_t n_events, int64_t n, const int64_t* __restrict__ hit_off,
                                                     const int64_t* __restrict__ art_pos,
                                                     const int64_t* __restrict__ elb_pos, int64_t cap,
                                                     int64_t* __restrict__ art_off, int64_t* __restrict__ elb_off,
                                                     const int64_t* status, int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n_art = art_pos[n], n_elb = elb_pos[n];
  if (gtid() == 0 && n_art + n_elb > cap) {
    tstatus[1] = n_art + n_elb;
    tstatus[0] = ETX_ERR_CAPACITY;
  }
  for (int64_t e = gtid(); e <= n_events; e += gstride()) {
    const int64_t h = hit_off[e];
    art_off[e] = art_pos[h];
    elb_off[e] = n_art + elb_pos[h];
  }
}

__global__ __launch_bounds__(256) void k_tri_fill(int64_t n, const int64_t* __restrict__ row_ptr,
                                                  const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ csc,
                                                  const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                  const int32_t* __restrict__ plane, const float* __restrict__ score,
                                                  float thr, const int32_t* __restrict__ deg_in,
                                                  const int32_t* __restrict__ deg_out,
                                                  const int64_t* __restrict__ art_pos,
                                                  const int64_t* __restrict__ elb_pos, int32_t* __restrict__ ta,
                                                  int32_t* __restrict__ tb, uint8_t* __restrict__ kind,
                                                  const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n_art = art_pos[n];
  for (int64_t c = gtid(); c < n; c += gstride()) {
    const int64_t a = deg_in[c], b = deg_out[c];
    const int64_t r0 = row_ptr[c], r1 = row_ptr[c + 1], c0 = col_ptr[c], c1 = col_ptr[c + 1];
    if (a > 0 && b > 0) {
      int64_t t = art_pos[c];
      for (int64_t q = c0; q < c1; ++q) {
        const int32_t ein = csc[q];
        if (!(score[ein] >= thr)) continue;
        for (int64_t r = r0; r < r1; ++r) {
          if (!(score[r] >= thr)) continue;
          ta[t] = ein;
          tb[t] = (int32_t)r;
          kind[t] = 0;
          ++t;
        }
      }
    }
    const int64_t eb = n_art + elb_pos[c];
    if (b >= 2) {
      int64_t p = 0;
      for (int64_t r = r0; r < r1; ++r) {
        if (!(score[r] >= thr)) continue;
        int64_t q = p + 1;
        for (int64_t r2 = r + 1; r2 < r1; ++r2) {
          if (!(score[r2] >= thr)) continue;
          const int64_t t = eb + tri_idx(p, q, b);
          const bool swap = plane[dst[r2]] < plane[dst[r]];   // the shorter edge first
          ta[t] = swap ? (int32_t)r2 : (int32_t)r;
          tb[t] = swap ? (int32_t)r : (int32_t)r2;
          kind[t] = 1;
          ++q;
        }
        ++p;
      }
    }
    if (a >= 2) {
      const int64_t base = eb + b * (b - 1) / 2;
      int64_t p = 0;
      for (int64_t q0 = c0; q0 < c1; ++q0) {
        const int32_t e1 = csc[q0];
        if (!(score[e1] >= thr)) continue;
        int64_t q = p + 1;
        for (int64_t q2 = q0 + 1; q2 < c1; ++q2) {
          const int32_t e2 = csc[q2];
          if (!(score[e2] >= thr)) continue;
          const int64_t t = base + tri_idx(p, q, a);
          const bool swap = plane[src[e2]] > plane[src[e1]];  // the source on the nearer plane first
          ta[t] = swap ? e2 : e1;
          tb[t] = swap ? e1 : e2;
          kind[t] = 2;
          ++q;
        }
        ++p;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// triplet classifiers: column tiles of 16 triplets per wave (tile.hpp)
// ---------------------------------------------------------------------------

// device form of one classifier (floats): W1 permuted (K = 2H), b1, W2
// permuted (K = H), b2, w3 (plain), b3 and three zeros
template <int H>
struct TriHead {
  static constexpr int W1 = 0;
  static constexpr int B1 = 2 * H * H;
  static constexpr int W2 = B1 + H;
  static constexpr int B2 = W2 + H * H;
  static constexpr int W3 = B2 + H;
  static constexpr int B3 = W3 + H;
  static constexpr int SIZE = B3 + 4;
};

// A stored edge row in BF16 (the compact state) into column layout: lane
// group g's 16-byte chunk c of the row (at byte 64c + 16g) holds its registers
// 8c .. 8c+7, features phi(r, g) (the edge kernels' row layout).
template <int H>
__device__ inline void load_cols_bf16_row(float* x, const char* __restrict__ row, bool valid) {
  const int g = lane_group();
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    const uint4 v = valid ? *reinterpret_cast<const uint4*>(row + 64 * c + 16 * g) : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[8 * c + 2 * i] = bf16_value(u[i] & 0xffffu);
      x[8 * c + 2 * i + 1] = bf16_value(u[i] >> 16);
    }
  }
}

// BF: the final edge encodings are stored as BF16 (compact state), else FP32.
template <int H, bool BF>
__global__ __launch_bounds__(256) void k_tri_score(const void* __restrict__ e_, const int32_t* __restrict__ ta,
                                                   const int32_t* __restrict__ tb, const int64_t* __restrict__ art_pos,
                                                   const int64_t* __restrict__ elb_pos, int64_t n, int head,
                                                   const float* __restrict__ wt, float* __restrict__ ts,
                                                   const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  using Hd = TriHead<H>;
  extern __shared__ float4 lds4[];
  float* w = reinterpret_cast<float*>(lds4);
  stage(w, wt + head * Hd::SIZE, Hd::SIZE);
  __syncthreads();
  const int64_t n_art = art_pos[n];
  const int64_t r0 = head ? n_art : 0;
  const int64_t r1 = head ? n_art + elb_pos[n] : n_art;
  const int g = lane_group(), j = lane_id() & 15;
  const int64_t tiles = (r1 - r0 + kCols - 1) / kCols;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave_id(); tile < tiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t r = r0 + tile * kCols + j;
    const bool valid = r < r1;
    const int64_t ea = valid ? ta[r] : 0, eb = valid ? tb[r] : 0;
    float x[H / 2];
    if constexpr (BF) {
      const char* e = static_cast<const char*>(e_);
      load_cols_bf16_row<H>(x, e + ea * H * 2, valid);
      load_cols_bf16_row<H>(x + H / 4, e + eb * H * 2, valid);
    } else {
      const float* e = static_cast<const float*>(e_);
      load_cols<H>(x, e + ea * H, valid);
      load_cols<H>(x + H / 4, e + eb * H, valid);
    }
    float a1[H / 4];
    bias_cols<H>(a1, w + Hd::B1);
    mfma_f32<2 * H, H / 16>(a1, x, w + Hd::W1);
    ln_relu<H>(a1);
    float a2[H / 4];
    bias_cols<H>(a2, w + Hd::B2);
    mfma_f32<H, H / 16>(a2, a1, w + Hd::W2);
    ln_relu<H>(a2);
    float dot = 0.f;
#pragma unroll
    for (int q = 0; q < H / 4; ++q) dot = fmaf(a2[q], w[Hd::W3 + phi(q, g)], dot);
    dot = col_sum(dot);
    const float logit = dot + w[Hd::B3];
    if (valid && g == 0) ts[r] = 1.0f / (1.0f + expf(-logit));
  }
}

// ---------------------------------------------------------------------------
// track building
// ---------------------------------------------------------------------------

// step 1: duplicates (the longer edge of a kept left elbow at its source and of
// a kept right elbow at its target)
__global__ __launch_bounds__(256) void k_tri_dup(int64_t n, const int64_t* __restrict__ row_ptr,
                                                 const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ csc,
                                                 const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                 const int32_t* __restrict__ plane, const float* __restrict__ score,
                                                 float thr, const int32_t* __restrict__ deg_in,
                                                 const int32_t* __restrict__ deg_out,
                                                 const int64_t* __restrict__ art_pos,
                                                 const int64_t* __restrict__ elb_pos, const float* __restrict__ ts,
                                                 uint8_t* __restrict__ dup, int32_t* __restrict__ par,
                                                 uint8_t* __restrict__ touched, int32_t* __restrict__ ccount,
                                                 const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t E = row_ptr[n], n_art = art_pos[n];
  for (int64_t d = gtid(); d < E; d += gstride()) {
    par[d] = (int32_t)d;                 // the union-find starts from singletons
    touched[d] = 0;
    ccount[d] = 0;
    bool left = false, right = false;
    if (score[d] >= thr) {
      const int32_t X = src[d], Y = dst[d];
      const int64_t b = deg_out[X];
      if (b >= 2) {
        const int64_t r0 = row_ptr[X], r1 = row_ptr[X + 1];
        int64_t od = 0;
        for (int64_t r = r0; r < d; ++r) od += score[r] >= thr ? 1 : 0;
        const int64_t base = n_art + elb_pos[X];
        int64_t o = 0;
        for (int64_t r = r0; r < r1; ++r) {
          if (!(score[r] >= thr)) continue;
          if (r != d) {
            const int64_t t = base + tri_idx(min(o, od), max(o, od), b);
            if (ts[t] >= thr && plane[Y] > plane[dst[r]]) left = true;
          }
          ++o;
        }
      }
      const int64_t a = deg_in[Y];
      if (left && a >= 2) {
        const int64_t c0 = col_ptr[Y], c1 = col_ptr[Y + 1];
        int64_t id = 0;
        for (int64_t q = c0; q < c1; ++q) {
          if (csc[q] == d) break;
          id += score[csc[q]] >= thr ? 1 : 0;
        }
        const int64_t bY = deg_out[Y];
        const int64_t base = n_art + elb_pos[Y] + bY * (bY - 1) / 2;
        int64_t i = 0;
        for (int64_t q = c0; q < c1; ++q) {
          const int32_t e2 = csc[q];
          if (!(score[e2] >= thr)) continue;
          if (e2 != d) {
            const int64_t t = base + tri_idx(min(i, id), max(i, id), a);
            if (ts[t] >= thr && plane[X] < plane[src[e2]]) right = true;
          }
          ++i;
        }
      }
    }
    dup[d] = (left && right) ? 1 : 0;
  }
}

// step 2a: links (kept articulations of two non-duplicate edges) and which of
// them are shared: 0 none, 1 link, 2 shared link
__global__ __launch_bounds__(256) void k_tri_links(int64_t n, const int32_t* __restrict__ deg_in,
                                                   const int32_t* __restrict__ deg_out,
                                                   const int64_t* __restrict__ art_pos, const int32_t* __restrict__ ta,
                                                   const int32_t* __restrict__ tb, const float* __restrict__ ts,
                                                   float thr, const uint8_t* __restrict__ dup,
                                                   uint8_t* __restrict__ lstate, const int64_t* status,
                                                   const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  for (int64_t c = gtid(); c < n; c += gstride()) {
    const int64_t a = deg_in[c], b = deg_out[c];
    if (a == 0 || b == 0) continue;
    const int64_t base = art_pos[c];
    auto live = [&](int64_t i, int64_t o) {
      const int64_t t = base + i * b + o;
      return ts[t] >= thr && !dup[ta[t]] && !dup[tb[t]];
    };
    for (int64_t i = 0; i < a; ++i)
      for (int64_t o = 0; o < b; ++o) {
        uint8_t st = 0;
        if (live(i, o)) {
          int nr = 0, nc = 0;
          for (int64_t o2 = 0; o2 < b && nr < 2; ++o2) nr += live(i, o2) ? 1 : 0;
          for (int64_t i2 = 0; i2 < a && nc < 2; ++i2) nc += live(i2, o) ? 1 : 0;
          st = (nr > 1 || nc > 1) ? 2 : 1;
        }
        lstate[base + i * b + o] = st;
      }
  }
}

// lock-free union-find on global memory; every root is its tree's smallest index
__device__ inline int32_t ld(const int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ inline int32_t g_find(int32_t* par, int32_t x) {
  int32_t p = ld(par + x);
  while (p != x) {
    const int32_t gp = ld(par + p);
    if (gp != p) __hip_atomic_store(par + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // path halving
    x = p;
    p = gp;
  }
  return x;
}

__device__ inline void g_unite(int32_t* par, int32_t u, int32_t v) {
  while (true) {
    u = g_find(par, u);
    v = g_find(par, v);
    if (u == v) return;
    if (u > v) {
      const int32_t t = u;
      u = v;
      v = t;
    }
    const int32_t old = atomicCAS(par + v, v, u);
    if (old == v) return;
    v = old;
  }
}

__global__ __launch_bounds__(256) void k_uf_unite(int64_t n, const int64_t* __restrict__ art_pos,
                                                  const int32_t* __restrict__ ta, const int32_t* __restrict__ tb,
                                                  const uint8_t* __restrict__ lstate, int32_t* par,
                                                  const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n_art = art_pos[n];
  for (int64_t t = gtid(); t < n_art; t += gstride())
    if (lstate[t] == 1) g_unite(par, ta[t], tb[t]);
}

// component names (the roots are final once every link is united), and the
// edge count of every component
__global__ __launch_bounds__(256) void k_uf_find(int64_t n, const int64_t* __restrict__ row_ptr,
                                                 const float* __restrict__ score, float thr,
                                                 const uint8_t* __restrict__ dup, int32_t* par,
                                                 int32_t* __restrict__ comp, int32_t* __restrict__ ccount,
                                                 const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t E = row_ptr[n];
  for (int64_t e = gtid(); e < E; e += gstride()) {
    int32_t c = -1;
    if (score[e] >= thr && !dup[e]) {
      c = g_find(par, (int32_t)e);
      atomicAdd(ccount + c, 1);
    }
    comp[e] = c;
  }
}

// step 3a: components that a shared link touches
__global__ __launch_bounds__(256) void k_touch(int64_t n, const int64_t* __restrict__ art_pos,
                                               const int32_t* __restrict__ ta, const int32_t* __restrict__ tb,
                                               const uint8_t* __restrict__ lstate, const int32_t* __restrict__ comp,
                                               uint8_t* __restrict__ touched, const int64_t* status,
                                               const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t n_art = art_pos[n];
  for (int64_t t = gtid(); t < n_art; t += gstride())
    if (lstate[t] == 2) {
      touched[comp[ta[t]]] = 1;
      touched[comp[tb[t]]] = 1;
    }
}

// per-event track count: untouched component names, then shared links
__global__ __launch_bounds__(256) void k_track_count(const int64_t* __restrict__ hit_off,
                                                     const int64_t* __restrict__ row_ptr,
                                                     const int64_t* __restrict__ art_off,
                                                     const int32_t* __restrict__ comp,
                                                     const uint8_t* __restrict__ touched,
                                                     const uint8_t* __restrict__ lstate, int64_t* __restrict__ ntr,
                                                     const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int ev = blockIdx.x;
  const int64_t eb = row_ptr[hit_off[ev]], ee = row_ptr[hit_off[ev + 1]];
  int64_t s = 0;
  for (int64_t e = eb + threadIdx.x; e < ee; e += 256) s += (comp[e] == e && !touched[e]) ? 1 : 0;
  for (int64_t t = art_off[ev] + threadIdx.x; t < art_off[ev + 1]; t += 256) s += lstate[t] == 2 ? 1 : 0;
  int64_t tot;
  (void)block_excl_scan(s, &tot);
  if (threadIdx.x == 0) ntr[ev] = tot;
}

// Ballot compaction over [b, e) of the items whose predicate holds, in
// order, by a 256-thread block: `emit(item, rank)` for each.
template <class Pred, class Emit>
__device__ inline int64_t block_compact(int64_t b, int64_t e, Pred pred, Emit emit) {
  __shared__ int wtot[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  int64_t cnt = 0;
  int slot = 0;
  for (int64_t q0 = b; q0 < e; q0 += 256) {
    const int64_t q = q0 + threadIdx.x;
    const uint64_t m = __ballot(q < e && pred(q));
    if (lane == 0) wtot[slot][wave] = __popcll(m);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      base += w < wave ? wtot[slot][w] : 0;
      total += wtot[slot][w];
    }
    if ((m >> lane) & 1) emit(q, cnt + base + __popcll(m & below));
    cnt += total;
    slot ^= 1;
  }
  return cnt;
}

__global__ __launch_bounds__(256) void k_track_fill(int64_t n_events, const int64_t* __restrict__ hit_off,
                                                    const int64_t* __restrict__ row_ptr,
                                                    const int64_t* __restrict__ art_off,
                                                    const int32_t* __restrict__ ta, const int32_t* __restrict__ tb,
                                                    const int32_t* __restrict__ comp,
                                                    const uint8_t* __restrict__ touched,
                                                    const uint8_t* __restrict__ lstate,
                                                    const int64_t* __restrict__ ev_off, int64_t cap,
                                                    int32_t* __restrict__ c1, int32_t* __restrict__ c2,
                                                    int32_t* __restrict__ tev, const int64_t* status,
                                                    int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int ev = blockIdx.x;
  if (ev_off[n_events] > cap) {
    if (ev == 0 && threadIdx.x == 0) {
      tstatus[2] = ev_off[n_events];
      tstatus[0] = ETX_ERR_CAPACITY;
    }
    return;
  }
  const int64_t p0 = ev_off[ev];
  const int64_t eb = row_ptr[hit_off[ev]], ee = row_ptr[hit_off[ev + 1]];
  const int64_t n1 = block_compact(
      eb, ee, [&](int64_t e) { return comp[e] == e && !touched[e]; },
      [&](int64_t e, int64_t r) {
        c1[p0 + r] = (int32_t)e;
        c2[p0 + r] = -1;
        tev[p0 + r] = ev;
      });
  block_compact(
      art_off[ev], art_off[ev + 1], [&](int64_t t) { return lstate[t] == 2; },
      [&](int64_t t, int64_t r) {
        c1[p0 + n1 + r] = comp[ta[t]];
        c2[p0 + n1 + r] = comp[tb[t]];
        tev[p0 + n1 + r] = ev;
      });
}

// component edge lists: placement after the counts of k_uf_find (the order inside
// a list is free: a track's hits are sorted afterwards)
__global__ __launch_bounds__(256) void k_comp_place(int64_t n, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ comp, int32_t* __restrict__ ccount,
                                                    const int64_t* __restrict__ cstart, int32_t* __restrict__ cedge,
                                                    const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t E = row_ptr[n];
  for (int64_t e = gtid(); e < E; e += gstride()) {
    const int32_t c = comp[e];
    if (c >= 0) cedge[cstart[c] + atomicSub(ccount + c, 1) - 1] = (int32_t)e;
  }
}

// step 4: the hits of each track, 16 lanes per track (four tracks per wave)
// through an LDS bitmap of its event's hits.  WRITE = false: hit counts;
// true: the hits, ascending, at track_off.
constexpr int kBitmapWords = ETX_MAX_EVENT_HITS / 32;
constexpr int kTrackLanes = 16;

template <bool WRITE>
__global__ __launch_bounds__(256) void k_track_hits(int64_t n_events, int64_t cap, const int64_t* __restrict__ hit_off,
                                                    const int64_t* __restrict__ ev_off,
                                                    const int32_t* __restrict__ c1, const int32_t* __restrict__ c2,
                                                    const int32_t* __restrict__ tev,
                                                    const int64_t* __restrict__ cstart,
                                                    const int32_t* __restrict__ cedge, const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dst, int32_t* __restrict__ tlen,
                                                    const int64_t* __restrict__ track_off, int64_t hit_cap,
                                                    int32_t* __restrict__ hits, const int64_t* status,
                                                    int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t nt = ev_off[n_events];
  if (nt < 0 || nt > cap) return;
  if (WRITE && track_off[nt] > hit_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      tstatus[3] = track_off[nt];
      tstatus[0] = ETX_ERR_CAPACITY;
    }
    return;
  }
  constexpr int G = kTrackLanes, PER_WAVE = 64 / G;
  __shared__ uint32_t bitmap[4 * PER_WAVE][kBitmapWords];
  const int lane = lane_id(), wave = wave_id();
  const int sub = lane / G, l = lane % G;
  uint32_t* bm = bitmap[wave * PER_WAVE + sub];
  const int64_t stride = (int64_t)gridDim.x * 4 * PER_WAVE;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * PER_WAVE; base < nt; base += stride) {
    const int64_t t = base + sub;
    const bool valid = t < nt;
    int ev = 0, words = 0;
    int64_t a = 0;
    if (valid) {
      ev = tev[t];
      a = hit_off[ev];
      words = (int)((hit_off[ev + 1] - a + 31) / 32);
      for (int w = l; w < words; w += G) bm[w] = 0;
    }
    wave_sync();
    if (valid) {
      const int32_t cs[2] = {c1[t], c2[t]};
      for (int k = 0; k < 2; ++k) {
        const int32_t c = cs[k];
        if (c < 0 || (k == 1 && c == cs[0])) continue;
        for (int64_t q = cstart[c] + l; q < cstart[c + 1]; q += G) {
          const int32_t e = cedge[q];
          const int s = (int)(src[e] - a), d = (int)(dst[e] - a);
          atomicOr(bm + (s >> 5), 1u << (s & 31));
          atomicOr(bm + (d >> 5), 1u << (d & 31));
        }
      }
    }
    wave_sync();
    if (valid) {
      if (!WRITE) {
        int cnt = 0;
        for (int w = l; w < words; w += G) cnt += __popc(bm[w]);
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, G);
        if (l == 0) tlen[t] = cnt;
      } else {
        int64_t run = track_off[t];
        for (int w0 = 0; w0 < words; w0 += G) {
          const int w = w0 + l;
          uint32_t m = w < words ? bm[w] : 0u;
          const int pc = __popc(m);
          int inc = pc;
#pragma unroll
          for (int d = 1; d < G; d <<= 1) {
            const int u = __shfl_up(inc, d, G);
            if (l >= d) inc += u;
          }
          int64_t at = run + inc - pc;
          while (m) {
            const int bit = __ffs(m) - 1;
            hits[at++] = (int32_t)(a + 32 * w + bit);
            m &= m - 1;
          }
          run += __shfl(inc, G - 1, G);   // a round adds at most G x 32 hits
        }
      }
    }
    wave_sync();   // every lane is done with the bitmap before the next track clears it
  }
}

// ---------------------------------------------------------------------------
// training: triplet labels and the triplet classifiers' gradient into the edges
// ---------------------------------------------------------------------------

struct Truth {
  const int32_t* particle;
  const int32_t* particle2;   // may be null
  const int32_t* succ;
  const int32_t* succ2;       // may be null
  __device__ int32_t part(int32_t h, int j) const { return j == 0 ? particle[h] : (particle2 ? particle2[h] : -1); }
  __device__ bool owns(int32_t h, int32_t p) const { return particle[h] == p || (particle2 && particle2[h] == p); }
  // the next hit of particle p after hit h (-1: none, or h is not p's)
  __device__ int32_t next(int32_t h, int32_t p) const {
    if (particle[h] == p) return succ[h];
    if (particle2 && particle2[h] == p) return succ2 ? succ2[h] : -1;
    return -1;
  }
};

// genuine: one particle runs A -> C -> B along its successor chain
// (articulation), or owns all three hits (elbow)
__global__ __launch_bounds__(256) void k_tri_labels(int64_t n, const int64_t* __restrict__ art_pos,
                                                    const int64_t* __restrict__ elb_pos,
                                                    const int32_t* __restrict__ ta, const int32_t* __restrict__ tb,
                                                    const uint8_t* __restrict__ kind, const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dst, Truth tr,
                                                    uint8_t* __restrict__ lab, const int64_t* status,
                                                    const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  const int64_t T = art_pos[n] + elb_pos[n];
  for (int64_t t = gtid(); t < T; t += gstride()) {
    const int32_t a = ta[t], b = tb[t];
    bool g = false;
    if (kind[t] == 0) {
      const int32_t A = src[a], C = dst[a], B = dst[b];
      for (int j = 0; j < 2; ++j) {
        const int32_t p = tr.part(A, j);
        if (p >= 0 && tr.next(A, p) == C && tr.next(C, p) == B) g = true;
      }
    } else {
      const bool left = kind[t] == 1;
      const int32_t C = left ? src[a] : dst[a];
      const int32_t A = left ? dst[a] : src[a];
      const int32_t B = left ? dst[b] : src[b];
      for (int j = 0; j < 2; ++j) {
        const int32_t p = tr.part(C, j);
        if (p >= 0 && tr.owns(A, p) && tr.owns(B, p)) g = true;
      }
    }
    lab[t] = g ? 1 : 0;
  }
}

// de[d] += the input gradients of every triplet row that reads edge d (dxa
// where d is the first edge, dxb where it is the second), gathered at the
// computed positions in a fixed order; H/4 threads per edge, four features each
template <int H>
__global__ __launch_bounds__(256) void k_tri_edge_grad(int64_t n, const int64_t* __restrict__ row_ptr,
                                                       const int64_t* __restrict__ col_ptr,
                                                       const int32_t* __restrict__ csc,
                                                       const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ dst,
                                                       const float* __restrict__ score, float thr,
                                                       const int32_t* __restrict__ deg_in,
                                                       const int32_t* __restrict__ deg_out,
                                                       const int64_t* __restrict__ art_pos,
                                                       const int64_t* __restrict__ elb_pos,
                                                       const int32_t* __restrict__ ta, const float* __restrict__ dxa,
                                                       const float* __restrict__ dxb, float* __restrict__ de,
                                                       const int64_t* status, const int64_t* tstatus) {
  if (halted(status, tstatus)) return;
  constexpr int Q = H / 4;
  const int64_t E = row_ptr[n], n_art = art_pos[n];
  for (int64_t u = gtid(); u < E * Q; u += gstride()) {
    const int64_t d = u / Q;
    const int c4 = (int)(u % Q) * 4;
    if (!(score[d] >= thr)) continue;
    const int32_t X = src[d], Y = dst[d];
    const int64_t bX = deg_out[X], aX = deg_in[X], aY = deg_in[Y], bY = deg_out[Y];
    int64_t od = 0, id = 0;
    for (int64_t r = row_ptr[X]; r < d; ++r) od += score[r] >= thr ? 1 : 0;
    for (int64_t q = col_ptr[Y]; q < col_ptr[Y + 1]; ++q) {
      if (csc[q] == d) break;
      id += score[csc[q]] >= thr ? 1 : 0;
    }
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    auto add = [&](const float* g, int64_t row) {
      const float4 v = *reinterpret_cast<const float4*>(g + row * H + c4);
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    };
    for (int64_t o = 0; o < bY; ++o) add(dxa, art_pos[Y] + id * bY + o);          // first edge at C = Y
    for (int64_t i = 0; i < aX; ++i) add(dxb, art_pos[X] + i * bX + od);          // second edge at C = X
    if (bX >= 2) {
      const int64_t base = n_art + elb_pos[X];
      for (int64_t o = 0; o < bX; ++o) {
        if (o == od) continue;
        const int64_t row = base + tri_idx(min(o, od), max(o, od), bX);
        add(ta[row] == d ? dxa : dxb, row);
      }
    }
    if (aY >= 2) {
      const int64_t base = n_art + elb_pos[Y] + bY * (bY - 1) / 2;
      for (int64_t i = 0; i < aY; ++i) {
        if (i == id) continue;
        const int64_t row = base + tri_idx(min(i, id), max(i, id), aY);
        add(ta[row] == d ? dxa : dxb, row);
      }
    }
    float4* out = reinterpret_cast<float4*>(de + d * H + c4);
    float4 v = *out;
    v.x += acc.x;
    v.y += acc.y;
    v.z += acc.z;
    v.w += acc.w;
    *out = v;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

TriLayout tri_layout(int64_t n_events, int64_t n_hits, int64_t edge_cap, int64_t triplet_cap, int64_t track_cap) {
  TriLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += a256(bytes);
    return at;
  };
  const size_t n = (size_t)n_hits, E = (size_t)edge_cap, T = (size_t)triplet_cap, K = (size_t)track_cap;
  const size_t longest = std::max({n, E, K, (size_t)n_events, (size_t)1});
  L.deg_in = take(4 * n);
  L.deg_out = take(4 * n);
  L.cnt_art = take(8 * n);
  L.cnt_elb = take(8 * n);
  L.art_pos = take(8 * (n + 1));
  L.elb_pos = take(8 * (n + 1));
  L.part = take(8 * ((longest + kScanTile - 1) / kScanTile + 1));
  L.lstate = take(T);
  L.dup = take(E);
  L.touched = take(E);
  L.par = take(4 * E);
  L.comp = take(4 * E);
  L.ccount = take(4 * E);
  L.cstart = take(8 * (E + 1));
  L.cedge = take(4 * E);
  L.ntr = take(8 * (size_t)n_events);
  L.c1 = take(4 * K);
  L.c2 = take(4 * K);
  L.tev = take(4 * K);
  L.tlen = take(4 * K);
  L.total = o;
  return L;
}

int tri_head_floats(int H) { return 3 * H * H + 3 * H + 4; }

// W[K][M] row-major -> the A-operand order of mfma_f32 (tile.hpp):
// out[(mb*(K/4) + t)*64 + lane] = W[phi(t, lane/16)][16*mb + lane%16]
static void permute(const float* W, int K, int M, float* out) {
  for (int mb = 0; mb < M / 16; ++mb)
    for (int t = 0; t < K / 4; ++t)
      for (int lane = 0; lane < 64; ++lane)
        out[((size_t)mb * (K / 4) + t) * 64 + lane] = W[(size_t)phi(t, lane / 16) * M + 16 * mb + lane % 16];
}

void tri_prepare_head(const float* p, int H, float* out) {
  const float* W1 = p;
  const float* b1 = W1 + 2 * H * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* w3 = b2 + H;
  const float* b3 = w3 + H;
  float* o = out;
  permute(W1, 2 * H, H, o);
  o += 2 * H * H;
  std::memcpy(o, b1, sizeof(float) * H);
  o += H;
  permute(W2, H, H, o);
  o += H * H;
  std::memcpy(o, b2, sizeof(float) * H);
  o += H;
  std::memcpy(o, w3, sizeof(float) * H);
  o += H;
  o[0] = b3[0];
  o[1] = o[2] = o[3] = 0.f;
}

int triplet_attributes(size_t max_lds) {
  int bad = 0;
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  set(reinterpret_cast<const void*>(k_tri_score<32, false>));
  set(reinterpret_cast<const void*>(k_tri_score<64, false>));
  set(reinterpret_cast<const void*>(k_tri_score<32, true>));
  set(reinterpret_cast<const void*>(k_tri_score<64, true>));
  return bad;
}

static int grid_for(int64_t work, int n_cu) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, (int64_t)n_cu * 8));
}

hipError_t launch_triplet_stage(const RunArgs& a, const etx_tracks& T, char* tws, const TriLayout& TL, int part) {
  const etx_ctx* ctx = a.ctx;
  hipStream_t s = a.stream;
  const int64_t n = a.hits.n_hits, ne = a.hits.n_events, cap = a.out.edge_capacity;
  const float thr = ctx->cfg.edge_threshold;
  const int64_t* status = a.out.status;
  int64_t* tstatus = T.status;
  const int64_t* row_ptr = reinterpret_cast<const int64_t*>(a.ws + a.L.row_ptr);
  const int64_t* col_ptr = reinterpret_cast<const int64_t*>(a.ws + a.L.col_ptr);
  const int32_t* csc = reinterpret_cast<const int32_t*>(a.ws + a.L.csc);
  const float* score = a.out.score;
  const int32_t* src = a.out.src;
  const int32_t* dst = a.out.dst;
  const int32_t* plane = a.hits.plane;
#define TW(off, Ty) reinterpret_cast<Ty*>(tws + TL.off)
  int32_t* deg_in = TW(deg_in, int32_t);
  int32_t* deg_out = TW(deg_out, int32_t);
  int64_t* art_pos = TW(art_pos, int64_t);
  int64_t* elb_pos = TW(elb_pos, int64_t);
  int64_t* part_buf = TW(part, int64_t);
  const int gn = grid_for(n, ctx->n_cu);
  const int ge = grid_for(cap, ctx->n_cu);
  hipError_t err;
  if (part == 0) {
    hipLaunchKernelGGL(k_tri_init, dim3(1), dim3(64), 0, s, tstatus);
    hipLaunchKernelGGL(k_tri_degrees, dim3(gn), dim3(256), 0, s, n, row_ptr, col_ptr, csc, score, thr, deg_in, deg_out,
                       TW(cnt_art, int64_t), TW(cnt_elb, int64_t), status, tstatus);
    if ((err = scan<int64_t>(TW(cnt_art, int64_t), n, art_pos, part_buf, s)) != hipSuccess) return err;
    if ((err = scan<int64_t>(TW(cnt_elb, int64_t), n, elb_pos, part_buf, s)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_tri_offsets, dim3(grid_for(ne + 1, ctx->n_cu)), dim3(256), 0, s, ne, n, a.hits.hit_off,
                       art_pos, elb_pos, T.triplet_capacity, T.art_off, T.elb_off, status, tstatus);
    hipLaunchKernelGGL(k_tri_fill, dim3(gn), dim3(256), 0, s, n, row_ptr, col_ptr, csc, src, dst, plane, score, thr,
                       deg_in, deg_out, art_pos, elb_pos, T.tri_a, T.tri_b, T.tri_kind, status, tstatus);
    return hipGetLastError();
  }
  if (part == 1) {
    const void* e = a.ws + a.L.e;
    const int H = ctx->cfg.gnn_hidden;
    const bool bf = a.prec == ETX_BF16;   // compact BF16 state
    // enough waves per SIMD to hide the row gathers: 8 workgroups per CU at hidden size 32
    // (12.7 KiB of weights each), 3 at 64 (50 KiB)
    const int grid = ctx->n_cu * (H == 32 ? 8 : 3);
    for (int head = 0; head < 2; ++head) {
#define SCORE(H_, BF_)                                                                                      \
  hipLaunchKernelGGL((k_tri_score<H_, BF_>), dim3(grid), dim3(256), sizeof(float) * TriHead<H_>::SIZE, s, e, \
                     T.tri_a, T.tri_b, art_pos, elb_pos, n, head, ctx->dev_tri, T.tri_score, status, tstatus)
      if (H == 32) {
        if (bf) SCORE(32, true); else SCORE(32, false);
      } else {
        if (bf) SCORE(64, true); else SCORE(64, false);
      }
#undef SCORE
    }
    return hipGetLastError();
  }
  uint8_t* dup = TW(dup, uint8_t);
  uint8_t* lstate = TW(lstate, uint8_t);
  uint8_t* touched = TW(touched, uint8_t);
  int32_t* par = TW(par, int32_t);
  int32_t* comp = TW(comp, int32_t);
  int32_t* ccount = TW(ccount, int32_t);
  int64_t* cstart = TW(cstart, int64_t);
  int32_t* cedge = TW(cedge, int32_t);
  int64_t* ntr = TW(ntr, int64_t);
  int32_t* c1 = TW(c1, int32_t);
  int32_t* c2 = TW(c2, int32_t);
  int32_t* tev = TW(tev, int32_t);
  int32_t* tlen = TW(tlen, int32_t);
  const int64_t tcap = T.track_capacity;
  hipLaunchKernelGGL(k_tri_dup, dim3(ge), dim3(256), 0, s, n, row_ptr, col_ptr, csc, src, dst, plane, score, thr,
                     deg_in, deg_out, art_pos, elb_pos, T.tri_score, dup, par, touched, ccount, status, tstatus);
  hipLaunchKernelGGL(k_tri_links, dim3(gn), dim3(256), 0, s, n, deg_in, deg_out, art_pos, T.tri_a, T.tri_b,
                     T.tri_score, thr, dup, lstate, status, tstatus);
  hipLaunchKernelGGL(k_uf_unite, dim3(ge), dim3(256), 0, s, n, art_pos, T.tri_a, T.tri_b, lstate, par, status,
                     tstatus);
  hipLaunchKernelGGL(k_uf_find, dim3(ge), dim3(256), 0, s, n, row_ptr, score, thr, dup, par, comp, ccount, status,
                     tstatus);
  hipLaunchKernelGGL(k_touch, dim3(ge), dim3(256), 0, s, n, art_pos, T.tri_a, T.tri_b, lstate, comp, touched, status,
                     tstatus);
  if (ne > 0)
    hipLaunchKernelGGL(k_track_count, dim3((unsigned)ne), dim3(256), 0, s, a.hits.hit_off, row_ptr, T.art_off, comp,
                       touched, lstate, ntr, status, tstatus);
  if ((err = scan<int64_t>(ntr, ne, T.event_track_off, part_buf, s)) != hipSuccess) return err;
  if (ne > 0)
    hipLaunchKernelGGL(k_track_fill, dim3((unsigned)ne), dim3(256), 0, s, ne, a.hits.hit_off, row_ptr, T.art_off,
                       T.tri_a, T.tri_b, comp, touched, lstate, T.event_track_off, tcap, c1, c2, tev, status, tstatus);
  const int gs = ctx->n_cu * 4;
  if ((err = dscan<int32_t>(ccount, row_ptr + n, cap, cstart, part_buf, gs, status, tstatus, s)) != hipSuccess) return err;
  hipLaunchKernelGGL(k_comp_place, dim3(ge), dim3(256), 0, s, n, row_ptr, comp, ccount, cstart, cedge, status, tstatus);
  const int gt = grid_for(tcap * kTrackLanes / 4, ctx->n_cu);   // 16 lanes per track
  hipLaunchKernelGGL(k_track_hits<false>, dim3(gt), dim3(256), 0, s, ne, tcap, a.hits.hit_off, T.event_track_off, c1,
                     c2, tev, cstart, cedge, src, dst, tlen, T.track_off, T.hit_capacity, T.track_hits, status,
                     tstatus);
  if ((err = dscan<int32_t>(tlen, T.event_track_off + ne, tcap, T.track_off, part_buf, gs, status, tstatus, s)) != hipSuccess) return err;
  hipLaunchKernelGGL(k_track_hits<true>, dim3(gt), dim3(256), 0, s, ne, tcap, a.hits.hit_off, T.event_track_off, c1,
                     c2, tev, cstart, cedge, src, dst, tlen, T.track_off, T.hit_capacity, T.track_hits, status,
                     tstatus);
#undef TW
  return hipGetLastError();
}

hipError_t launch_tri_labels(const RunArgs& a, char* tws, const TriLayout& TL, const etx_tracks& T,
                             const etx_truth& truth, uint8_t* lab) {
  const int64_t n = a.hits.n_hits;
  const Truth tr{truth.particle, truth.particle2, truth.succ, truth.succ2};
  hipLaunchKernelGGL(k_tri_labels, dim3(grid_for(T.triplet_capacity, a.ctx->n_cu)), dim3(256), 0, a.stream, n,
                     reinterpret_cast<const int64_t*>(tws + TL.art_pos), reinterpret_cast<const int64_t*>(tws + TL.elb_pos),
                     T.tri_a, T.tri_b, T.tri_kind, a.out.src, a.out.dst, tr, lab, a.out.status, T.status);
  return hipGetLastError();
}

hipError_t launch_tri_edge_grad(const RunArgs& a, char* tws, const TriLayout& TL, const etx_tracks& T,
                                const float* dxa, const float* dxb, float* de) {
  const etx_ctx* ctx = a.ctx;
  const int64_t n = a.hits.n_hits;
  const int H = ctx->cfg.gnn_hidden;
  const int grid = grid_for(a.out.edge_capacity * (H / 4), ctx->n_cu);
#define ARGS                                                                                                       \
  n, reinterpret_cast<const int64_t*>(a.ws + a.L.row_ptr), reinterpret_cast<const int64_t*>(a.ws + a.L.col_ptr),   \
      reinterpret_cast<const int32_t*>(a.ws + a.L.csc), a.out.src, a.out.dst, a.out.score, ctx->cfg.edge_threshold, \
      reinterpret_cast<const int32_t*>(tws + TL.deg_in), reinterpret_cast<const int32_t*>(tws + TL.deg_out),        \
      reinterpret_cast<const int64_t*>(tws + TL.art_pos), reinterpret_cast<const int64_t*>(tws + TL.elb_pos),       \
      T.tri_a, dxa, dxb, de, a.out.status, T.status
  if (H == 32)
    hipLaunchKernelGGL(k_tri_edge_grad<32>, dim3(grid), dim3(256), 0, a.stream, ARGS);
  else
    hipLaunchKernelGGL(k_tri_edge_grad<64>, dim3(grid), dim3(256), 0, a.stream, ARGS);
#undef ARGS
  return hipGetLastError();
}

}  // namespace etx
