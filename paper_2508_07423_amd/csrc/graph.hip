// Integer and graph kernels of the hot path: input validation, plane
// bucketing, edge offsets, the CSC permutation, edge compaction after the
// score cut, and union-find components.
#include "internal.hpp"

namespace etx {

namespace {

__device__ inline void set_status(int64_t* status, int64_t code) {
  atomicCAS(reinterpret_cast<unsigned long long*>(status), 0ull, static_cast<unsigned long long>(code));
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan over a 256-thread block; returns the exclusive prefix and the
// block total.  `tmp` holds 4 ints of LDS.
__device__ inline int block_exclusive_scan(int v, int* tmp, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = wave_inclusive_scan(v);
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  int base = 0;
  total = 0;
  for (int w = 0; w < 4; ++w) {
    int s = tmp[w];
    if (w < wave) base += s;
    total += s;
  }
  __syncthreads();
  return base + inc - v;
}

// --------------------------------------------------------------------------
// status / validation
// --------------------------------------------------------------------------

__global__ void k_init_status(int64_t* status, float* calib, int n_calib) {
  int t = threadIdx.x;
  if (t < 2) status[t] = 0;
  if (calib && t < n_calib) calib[t] = 0.f;
}

__global__ void k_validate(int64_t n_events, int64_t n_hits, const int64_t* __restrict__ hit_off,
                           const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
                           const int32_t* __restrict__ plane, int n_planes, int64_t* status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_hits + n_events + 1; i += stride) {
    if (i < n_hits) {
      int p = plane[i];
      if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]) || p < 0 || p >= n_planes) set_status(status, ETX_ERR_INPUT);
    } else {
      int64_t e = i - n_hits;
      if (e == n_events) {
        if (hit_off[n_events] != n_hits || hit_off[0] != 0) set_status(status, ETX_ERR_INPUT);
      } else {
        int64_t cnt = hit_off[e + 1] - hit_off[e];
        if (cnt < 0) set_status(status, ETX_ERR_INPUT);
        else if (cnt > ETX_MAX_EVENT_HITS) set_status(status, ETX_ERR_UNSUPPORTED);
      }
    }
  }
}

// --------------------------------------------------------------------------
// plane bucketing: per event, a stable counting sort of hits by plane
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bucket(const int64_t* __restrict__ hit_off, const int32_t* __restrict__ plane,
                                                int n_planes, int32_t* __restrict__ bucket,
                                                int32_t* __restrict__ plane_off, const int64_t* status) {
  if (status[0] != 0) return;
  extern __shared__ int cnt[];            // [n_planes][256]
  __shared__ int tmp[4];
  const int ev = blockIdx.x, t = threadIdx.x;
  const int64_t a = hit_off[ev];
  const int n = (int)(hit_off[ev + 1] - a);
  const int chunk = (n + 255) / 256;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  for (int p = 0; p < n_planes; ++p) cnt[p * 256 + t] = 0;
  for (int i = lo; i < hi; ++i) cnt[plane[a + i] * 256 + t] += 1;
  __syncthreads();
  int base = 0;
  int32_t* po = plane_off + (int64_t)ev * (n_planes + 1);
  for (int p = 0; p < n_planes; ++p) {
    int total;
    int ex = block_exclusive_scan(cnt[p * 256 + t], tmp, total);
    cnt[p * 256 + t] = base + ex;
    if (t == 0) po[p] = base;
    base += total;
  }
  if (t == 0) po[n_planes] = n;
  __syncthreads();
  for (int i = lo; i < hi; ++i) {
    int p = plane[a + i];
    int pos = cnt[p * 256 + t]++;
    bucket[a + pos] = (int32_t)(a + i);
  }
}

// --------------------------------------------------------------------------
// device-wide exclusive scan of per-hit edge counts -> row_ptr
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ part,
                                                     const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int64_t red[256];
  int64_t b = blockIdx.x;
  int64_t s = 0;
  for (int q = 0; q < kScanBlock / 256; ++q) {
    int64_t i = b * kScanBlock + q * 256 + threadIdx.x;
    if (i < n) s += cnt[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b] = red[0];
}

__global__ __launch_bounds__(256) void k_scan_top(int64_t* __restrict__ part, int64_t nb, int64_t* __restrict__ row_ptr,
                                                  int64_t n, int64_t capacity, int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int64_t sh[256];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 256) {
    int64_t b = b0 + threadIdx.x;
    int64_t v = b < nb ? part[b] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      int64_t t = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nb) part[b] = carry + sh[threadIdx.x] - v;
    int64_t tot = sh[255];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) {
    row_ptr[n] = carry;
    if (carry > capacity) {
      status[1] = carry;
      set_status(status, ETX_ERR_CAPACITY);
    } else if (carry >= 0x7fffffffLL) {
      status[1] = carry;
      set_status(status, ETX_ERR_UNSUPPORTED);
    }
  }
}

__global__ __launch_bounds__(256) void k_scan_down(const int32_t* __restrict__ cnt, int64_t n, const int64_t* __restrict__ part,
                                                   int64_t* __restrict__ row_ptr, const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int tmp[4];
  int64_t base = part[blockIdx.x];
  for (int q = 0; q < kScanBlock / 256; ++q) {
    int64_t i = (int64_t)blockIdx.x * kScanBlock + q * 256 + threadIdx.x;
    int v = i < n ? cnt[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, tmp, total);
    if (i < n) row_ptr[i] = base + ex;
    base += total;
  }
}

__global__ void k_edge_off(const int64_t* __restrict__ hit_off, int64_t n_events, const int64_t* __restrict__ row_ptr,
                           int64_t* __restrict__ edge_off, const int64_t* status) {
  if (status[0] != 0) return;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e <= n_events) edge_off[e] = row_ptr[hit_off[e]];
}

// --------------------------------------------------------------------------
// CSC: edge ids ordered by (dst, src), per event
// --------------------------------------------------------------------------

// Long rows (at least kCscRowWalk edges per source on average) are placed a
// row per step by one wave; short rows by the whole block through LDS cursors
// with a sort of every column afterwards (place = 1), or 64 edges per step by
// one wave (place = 0).  All keep (dst, src) order.
constexpr int kCscRowWalk = 16;

// The per-event kernels that keep one LDS word per hit of the event run as
// two launches: events of up to kSmallEventHits hits in workgroups with 16 KiB
// of LDS (six to eight to a CU, registers deciding, so that their chains of
// loads and barriers overlap),
// the larger ones with room for ETX_MAX_EVENT_HITS; each launch skips the
// other's events.
constexpr int kSmallEventHits = 4096;

template <int CAP>
__device__ inline bool event_in_launch(int n) {
  return CAP == kSmallEventHits ? n <= kSmallEventHits : n > kSmallEventHits;
}

template <int CAP>
__global__ __launch_bounds__(256) void k_csc(const int64_t* __restrict__ hit_off, const int64_t* __restrict__ row_ptr,
                                             const int32_t* __restrict__ dst, int64_t* __restrict__ col_ptr,
                                             int32_t* __restrict__ csc, int place, const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int cur[CAP];
  __shared__ int tmp[4];
  const int ev = blockIdx.x, t = threadIdx.x, lane = t & 63;
  const int64_t a = hit_off[ev];
  const int n = (int)(hit_off[ev + 1] - a);
  if (!event_in_launch<CAP>(n)) return;
  const int64_t eb = row_ptr[a], ee = row_ptr[a + n];
  for (int i = t; i < n; i += 256) cur[i] = 0;
  __syncthreads();
  for (int64_t q = eb + t; q < ee; q += 256) atomicAdd(&cur[dst[q] - a], 1);
  __syncthreads();
  int base = 0;
  for (int i0 = 0; i0 < n; i0 += 256) {
    int i = i0 + t;
    int v = i < n ? cur[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, tmp, total);
    if (i < n) {
      cur[i] = base + ex;
      col_ptr[a + i] = eb + base + ex;
    }
    base += total;
  }
  if (t == 0) col_ptr[a + n] = ee;
  __syncthreads();
  if (place && ee - eb < (int64_t)kCscRowWalk * n) {
    // short rows, whole block: every thread drops its edges into their columns
    // through the LDS cursors (any order within a column), then every column
    // is sorted by edge index, which is source order (insertion sort: fewer
    // than kCscRowWalk edges per column on average).
    for (int64_t q = eb + t; q < ee; q += 256) {
      const int pos = atomicAdd(&cur[dst[q] - (int)a], 1);
      csc[eb + pos] = (int32_t)q;
    }
    __syncthreads();
    for (int i = t; i < n; i += 256) {
      const int64_t c0 = col_ptr[a + i], c1 = col_ptr[a + i + 1];
      for (int64_t j = c0 + 1; j < c1; ++j) {
        const int32_t v = csc[j];
        int64_t k = j - 1;
        for (; k >= c0; --k) {
          const int32_t u = csc[k];
          if (u < v) break;
          csc[k + 1] = u;
        }
        csc[k + 1] = v;
      }
    }
    return;
  }
  if (t >= 64) return;
  if (ee - eb >= (int64_t)kCscRowWalk * n) {
    // one wave walks the rows in source order; the targets of one row are
    // distinct, so its lanes never share a cursor.  Row bounds and targets are
    // loaded kRow rows ahead so that HBM latency overlaps the LDS updates.
    constexpr int kRow = 8;
    int64_t rb[kRow + 1];
    int dd[kRow];
    auto load_block = [&](int i0, int64_t (&b)[kRow + 1], int (&d)[kRow]) {
#pragma unroll
      for (int q = 0; q <= kRow; ++q) b[q] = row_ptr[a + min(i0 + q, n)];
#pragma unroll
      for (int q = 0; q < kRow; ++q) d[q] = (b[q] + lane < b[q + 1]) ? dst[b[q] + lane] : 0;
    };
    if (n > 0) load_block(0, rb, dd);
    for (int i0 = 0; i0 < n; i0 += kRow) {
      int64_t nb[kRow + 1];
      int nd[kRow];
      if (i0 + kRow < n) load_block(i0 + kRow, nb, nd);
#pragma unroll
      for (int q = 0; q < kRow; ++q) {
        if (rb[q] + lane < rb[q + 1]) {
          const int dl = dd[q] - (int)a;
          const int pos = cur[dl];
          cur[dl] = pos + 1;
          csc[eb + pos] = (int32_t)(rb[q] + lane);
        }
        wave_sync();
      }
      if (i0 + kRow < n) {
#pragma unroll
        for (int q = 0; q <= kRow; ++q) rb[q] = nb[q];
#pragma unroll
        for (int q = 0; q < kRow; ++q) dd[q] = nd[q];
      }
    }
    return;
  }
  // one wave scatters the edges in source-major order, 64 at a time: a lane's
  // rank among the lanes of the chunk with the same target (lower lanes are
  // earlier edges) gives its slot after the target's cursor, and the last of
  // them advances the cursor, so every column keeps source order.  The next
  // chunk's targets load while this one is placed.
  int dn = eb + lane < ee ? dst[eb + lane] - (int)a : -1;
  for (int64_t q0 = eb; q0 < ee; q0 += 64) {
    const int64_t q = q0 + lane;
    const int d = dn;
    dn = q + 64 < ee ? dst[q + 64] - (int)a : -1;
    int rank = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const int o = __builtin_amdgcn_readlane(d, k);
      cnt += o == d ? 1 : 0;
      rank += (o == d && k < lane) ? 1 : 0;
    }
    const int pos = d >= 0 ? cur[d] + rank : 0;
    wave_sync();
    if (d >= 0) {
      csc[eb + pos] = (int32_t)q;
      if (rank == cnt - 1) cur[d] = pos + 1;
    }
    wave_sync();
  }
}

// --------------------------------------------------------------------------
// score cut + compaction (wave ballot + block prefix scan), per event
// --------------------------------------------------------------------------

// One 1024-thread workgroup per event; every wave takes 256 consecutive scores
// per round (four ballots of 64), so a round covers 4096 edges with one
// barrier: the wave totals go to LDS (two slots, alternating between rounds,
// so that no wave overwrites a slot another wave still reads), each wave adds
// the totals of the waves before it, and every kept edge is written at its
// rank.  The kept list is in edge order.
constexpr int kCompactThreads = 1024;
constexpr int kCompactWaves = kCompactThreads / 64;
constexpr int kCompactBallots = 4;                   // 64-score ballots per wave per round

__global__ __launch_bounds__(kCompactThreads) void k_compact(const int64_t* __restrict__ hit_off,
                                                             const int64_t* __restrict__ row_ptr,
                                                             const float* __restrict__ score, float thr,
                                                             int32_t* __restrict__ kept,
                                                             int32_t* __restrict__ kept_cnt, const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int tot[2][kCompactWaves];
  const int ev = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t eb = row_ptr[hit_off[ev]], ee = row_ptr[hit_off[ev + 1]];
  const uint64_t below = (uint64_t(1) << lane) - 1;    // lanes before this one
  int64_t cnt = 0;
  int slot = 0;
  // the next round's scores are loaded before this round's barrier
  constexpr int64_t kRound = (int64_t)kCompactBallots * kCompactThreads;
  float sc[kCompactBallots];
  auto load = [&](int64_t q0) {
#pragma unroll
    for (int j = 0; j < kCompactBallots; ++j) {
      const int64_t q = q0 + (int64_t)wave * 64 * kCompactBallots + 64 * j + lane;
      sc[j] = q < ee ? score[q] : 0.f;
    }
  };
  if (eb < ee) load(eb);
  for (int64_t q0 = eb; q0 < ee; q0 += kRound) {
    const int64_t w0 = q0 + (int64_t)wave * 64 * kCompactBallots;
    uint64_t m[kCompactBallots];
    int n = 0;
#pragma unroll
    for (int j = 0; j < kCompactBallots; ++j) {
      const int64_t q = w0 + 64 * j + lane;
      m[j] = __ballot(q < ee && sc[j] >= thr);
      n += __popcll(m[j]);
    }
    if (q0 + kRound < ee) load(q0 + kRound);
    if (lane == 0) tot[slot][wave] = n;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kCompactWaves; ++w) {
      const int t = tot[slot][w];
      base += w < wave ? t : 0;
      total += t;
    }
#pragma unroll
    for (int j = 0; j < kCompactBallots; ++j) {
      const int64_t q = w0 + 64 * j + lane;
      if ((m[j] >> lane) & 1) kept[eb + cnt + base + __popcll(m[j] & below)] = (int32_t)q;
      base += __popcll(m[j]);
    }
    cnt += total;
    slot ^= 1;
  }
  if (threadIdx.x == 0) kept_cnt[ev] = (int32_t)cnt;
}

// --------------------------------------------------------------------------
// components: lock-free union-find in LDS, per event
// --------------------------------------------------------------------------

__device__ inline int uf_find(volatile int* par, int x) {
  int p = par[x];
  while (p != x) {
    int gp = par[p];
    if (gp != p) par[x] = gp;   // path halving: gp is an ancestor of x
    x = p;
    p = gp;
  }
  return x;
}

__device__ inline void uf_unite(volatile int* par, int u, int v) {
  while (true) {
    u = uf_find(par, u);
    v = uf_find(par, v);
    if (u == v) return;
    if (u > v) { int t = u; u = v; v = t; }
    // hook the larger root under the smaller one, so every root is its tree's minimum
    int old = atomicCAS(const_cast<int*>(reinterpret_cast<volatile int*>(par + v)), v, u);
    if (old == v) return;
    v = old;
  }
}

template <int CAP>
__global__ __launch_bounds__(256) void k_union_find(const int64_t* __restrict__ hit_off, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                    const int32_t* __restrict__ kept, const int32_t* __restrict__ kept_cnt,
                                                    int32_t* __restrict__ labels, const int64_t* status) {
  if (status[0] != 0) return;
  __shared__ int par[CAP];
  const int ev = blockIdx.x;
  const int64_t a = hit_off[ev];
  const int n = (int)(hit_off[ev + 1] - a);
  if (!event_in_launch<CAP>(n)) return;
  const int64_t eb = row_ptr[a];
  const int nk = kept_cnt[ev];
  for (int i = threadIdx.x; i < n; i += 256) par[i] = i;
  __syncthreads();
  for (int q = threadIdx.x; q < nk; q += 256) {
    int e = kept[eb + q];
    uf_unite(par, src[e] - (int)a, dst[e] - (int)a);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) labels[a + i] = (int32_t)(a + uf_find(par, i));
}

}  // namespace

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

#define WS(a, off, T) reinterpret_cast<T*>((a).ws + (a).L.off)

hipError_t launch_init_status(const RunArgs& a) {
  hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, a.stream, a.out.status,
                     a.calibrate ? WS(a, calib, float) : nullptr, ETX_N_CALIB);
  return hipGetLastError();
}

hipError_t launch_validate(const RunArgs& a) {
  int64_t work = a.hits.n_hits + a.hits.n_events + 1;
  int grid = (int)std::min<int64_t>((work + 255) / 256, 4096);
  hipLaunchKernelGGL(k_validate, dim3(grid), dim3(256), 0, a.stream, a.hits.n_events, a.hits.n_hits, a.hits.hit_off,
                     a.hits.x, a.hits.y, a.hits.z, a.hits.plane, a.ctx->cfg.n_planes, a.out.status);
  return hipGetLastError();
}

hipError_t launch_bucket(const RunArgs& a) {
  if (a.hits.n_events == 0) return hipSuccess;
  size_t lds = sizeof(int) * 256 * a.ctx->cfg.n_planes;
  hipLaunchKernelGGL(k_bucket, dim3((unsigned)a.hits.n_events), dim3(256), lds, a.stream, a.hits.hit_off,
                     a.hits.plane, a.ctx->cfg.n_planes, WS(a, bucket, int32_t), WS(a, plane_off, int32_t),
                     a.out.status);
  return hipGetLastError();
}

hipError_t launch_scan_counts(const RunArgs& a, bool candidates) {
  // counts (ws.cnt) -> CSR offsets: the candidate offsets of the prefilter
  // path, or the main row_ptr (+ per-event edge offsets)
  const int64_t n = a.hits.n_hits;
  const int64_t nb = a.L.n_scan_blocks;
  int64_t* part = WS(a, scan_tmp, int64_t);
  int64_t* row_ptr = candidates ? WS(a, pf_tmp, int64_t) : WS(a, row_ptr, int64_t);
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, a.stream, WS(a, cnt, int32_t), n, part,
                       a.out.status);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, a.stream, part, nb, row_ptr, n, a.out.edge_capacity,
                     a.out.status);
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(256), 0, a.stream, WS(a, cnt, int32_t), n, part, row_ptr,
                       a.out.status);
  if (!candidates) {
    int64_t ne = a.hits.n_events + 1;
    hipLaunchKernelGGL(k_edge_off, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, a.stream, a.hits.hit_off,
                       a.hits.n_events, row_ptr, a.out.edge_off, a.out.status);
  }
  return hipGetLastError();
}

hipError_t launch_csc(const RunArgs& a) {
  if (a.hits.n_events == 0) return hipSuccess;
#define CSC(C_)                                                                                           \
  hipLaunchKernelGGL(k_csc<C_>, dim3((unsigned)a.hits.n_events), dim3(256), 0, a.stream, a.hits.hit_off,  \
                     WS(a, row_ptr, int64_t), a.out.dst, WS(a, col_ptr, int64_t), WS(a, csc, int32_t),     \
                     a.ctx->csc_place, a.out.status)
  CSC(kSmallEventHits);
  CSC(ETX_MAX_EVENT_HITS);
#undef CSC
  return hipGetLastError();
}

hipError_t launch_compact(const RunArgs& a) {
  if (a.hits.n_events == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)a.hits.n_events), dim3(kCompactThreads), 0, a.stream, a.hits.hit_off,
                     WS(a, row_ptr, int64_t), a.out.score, a.ctx->cfg.edge_threshold, WS(a, kept, int32_t),
                     WS(a, kept_cnt, int32_t), a.out.status);
  return hipGetLastError();
}

hipError_t launch_union_find(const RunArgs& a) {
  if (a.hits.n_events == 0) return hipSuccess;
#define UF(C_)                                                                                                   \
  hipLaunchKernelGGL(k_union_find<C_>, dim3((unsigned)a.hits.n_events), dim3(256), 0, a.stream, a.hits.hit_off,  \
                     WS(a, row_ptr, int64_t), a.out.src, a.out.dst, WS(a, kept, int32_t), WS(a, kept_cnt, int32_t), \
                     a.out.labels, a.out.status)
  UF(kSmallEventHits);
  UF(ETX_MAX_EVENT_HITS);
#undef UF
  return hipGetLastError();
}

int graph_attributes(size_t max_lds) {
  int bad = 0;
  bad |= hipFuncSetAttribute(reinterpret_cast<const void*>(k_bucket), hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  return bad;
}

}  // namespace etx
