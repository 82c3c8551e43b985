// Fixed-radius graph in embedding space (thesis ch. 8, squared-distance
// equation; ch. 9 "k-NN Implementation"): a hit on plane p connects to hits on
// planes p+1 .. p+window whose squared embedding distance is below r^2,
// keeping at most k_max per source: the k_max smallest by (d^2, target index).
//
// One workgroup per (event, source plane).  The candidate window (hits of the
// next planes) is staged in LDS and binned along its widest embedding axis into
// cells about r wide (a counting sort), a one-dimensional cell list: a source
// only scans the cells its coordinate on that axis reaches within r, which is
// exact because a distance below r bounds every coordinate difference.  Sources
// with few candidates are handled four to a wave; otherwise each wave handles one source
// at a time: in-radius candidates are compacted into an LDS list with a wave
// ballot and prefix count, the k_max boundary is found by a radix select on
// the float bits of d^2 (ties at the boundary resolved by the target index), and
// the kept targets are ranked by index and written as one CSR row.  Windows
// larger than the LDS capacity are read from HBM without the cell list.
#include "internal.hpp"

namespace etx {

namespace {

constexpr int kRadiusThreads = 512;     // 8 waves
constexpr int kRadiusWaves = kRadiusThreads / 64;
constexpr int kList = 256;              // per-wave list of in-radius candidates
constexpr int kCells = 256;             // most cells of a window's cell list

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct RadiusArgs {
  const int64_t* hit_off;
  const int32_t* bucket;
  const int32_t* plane_off;
  const float* emb;        // [n_hits][kDpad]
  int n_planes, window, k_max, dim;
  int stage_window;        // 0: always read the window from HBM
  int sort_min;            // staged windows of at least this many hits are sorted (cell list)
  int fast;                // select pass: sources with at most 16 in-radius candidates take the 16-lane path
  int split;               // 1: windows up to the small capacity go to the small-LDS launch, the rest to the other
  float r2, r;
  int32_t* cnt;            // count pass output (and the select pass's)
  const int64_t* row_ptr;  // emit pass input
  int32_t* slots;          // select pass output: kept targets, ascending (slot_index)
  int64_t n_hits;
  int32_t* src;
  int32_t* dst;
  const int64_t* status;
};

template <int DP>
__device__ inline float dist2(const float (&s)[DP], const float* c) {
  float d2 = 0.f;
#pragma unroll
  for (int k = 0; k < DP; k += 4) {
    float4 v = *reinterpret_cast<const float4*>(c + k);
    float t0 = s[k] - v.x, t1 = s[k + 1] - v.y, t2 = s[k + 2] - v.z, t3 = s[k + 3] - v.w;
    d2 = fmaf(t0, t0, d2);
    d2 = fmaf(t1, t1, d2);
    d2 = fmaf(t2, t2, d2);
    d2 = fmaf(t3, t3, d2);
  }
  return d2;
}

// LDS capacity of the staged window for a padded embedding width DP.  The
// SMALL form stages half as many hits: 48 KiB instead of 72 KiB at width 8,
// so that three workgroups share a CU instead of two (at width 16 the
// registers still allow only two).  A workgroup's few hundred distance
// evaluations on a trained embedding wait mostly on memory latency (one
// workgroup per CU instead of two nearly doubles the search time), so the
// small windows gain from the third workgroup in flight.
template <int DP, bool SMALL = false>
struct RadiusLds {
  static constexpr int cap = (DP <= 8 ? 1024 : 512) / (SMALL ? 2 : 1);
  static constexpr size_t bytes = (size_t)cap * (DP * 4 + 12) + kRadiusWaves * (kList * 8 + 64 * 4 + 256 * 4) + 64;
};

// MODE: 0 counts the kept neighbours of every source; 1 writes them as CSR rows
// at the offsets the count pass produced; 2 does the whole selection once,
// writing each source's kept targets (ascending) to its k_max slots and its
// count, so that the CSR rows are a copy after the scan.
enum RadiusMode { R_COUNT = 0, R_EMIT = 1, R_SELECT = 2 };

// Slot of rank r of hit i in the select pass's output: the first kSlotHead
// ranks of every hit side by side ([n_hits][kSlotHead]), the others after
// them ([n_hits][k_max - kSlotHead]).  Rows of a trained embedding hold a few
// targets, so the copy into CSR rows reads the dense head instead of a
// k_max-wide row per hit; long rows stay contiguous in both parts.
constexpr int kSlotHead = 4;

__device__ inline int64_t slot_index(int64_t i, int r, int64_t n_hits, int k_max) {
  const int head = min(kSlotHead, k_max);
  return r < head ? i * head + r : n_hits * head + i * (k_max - head) + (r - head);
}

// Window size of an (event, plane) unit: hits on the planes after p within
// the plane window (0 on the last plane).
__device__ inline int window_hits(const int32_t* po, int p, int P, int window) {
  return p + 1 < P ? po[min(p + window, P - 1) + 1] - po[p + 1] : 0;
}

// One (event, plane) unit: its sources against their candidate window.
// Entered by the whole workgroup; every early return is workgroup-uniform.
template <int MODE, int DP, bool SMALL>
__device__ inline void radius_unit(const RadiusArgs& A, float* lds, int ev, int p) {
  constexpr bool EMIT = MODE != R_COUNT;
  constexpr int CAP = RadiusLds<DP, SMALL>::cap;
  float* cemb = lds;                                              // [CAP][DP]
  int* cj = reinterpret_cast<int*>(cemb + CAP * DP);              // [CAP] target hit index
  float* skey = reinterpret_cast<float*>(cj + CAP);               // [CAP] cell ends, then hard sources
  int* sidx = reinterpret_cast<int*>(skey + CAP);                 // [CAP] slots in cell order
  float* ld2 = reinterpret_cast<float*>(sidx + CAP);              // [waves][kList]
  int* lj = reinterpret_cast<int*>(ld2 + kRadiusWaves * kList);   // [waves][kList]
  int* sel = lj + kRadiusWaves * kList;                           // [waves][64]
  int* hist = sel + kRadiusWaves * 64;                            // [waves][256] radix-select histogram
  int* misc = hist + kRadiusWaves * 256;                          // [16]

  const int P = A.n_planes;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the status word is read together with the unit's offsets (all in bounds
  // whatever their contents); nothing read here is used before the check
  const int64_t status = A.status[0];
  const int64_t a = A.hit_off[ev];
  const int32_t* po = A.plane_off + (int64_t)ev * (P + 1);
  const int s0 = po[p], s1 = po[p + 1];
  const int nwin = window_hits(po, p, P, A.window);
  if (status != 0) return;
  const int nsrc = s1 - s0;
  if (nsrc == 0) return;
  const int w0 = s1;
  // split launches: each unit goes to exactly one of the two
  if (A.split && (SMALL ? nwin > CAP : nwin <= RadiusLds<DP, true>::cap)) return;
  const int32_t* wb = A.bucket + a + w0;
  const bool staged = A.stage_window && nwin <= CAP;
  // windows of at least sort_min hits get a cell list along their widest axis
  // and each source scans only the cells within reach; smaller ones are
  // scanned whole
  const bool sorted = staged && nwin >= A.sort_min;
  // Fast path of the select pass over a staged window (below): four sources
  // per wave.  Each row's first source index is loaded now, beside the
  // window's, and its embedding row once the window is staged, so that both
  // arrive while the cell list is built; later sources are fetched one
  // iteration ahead.
  const bool fast = MODE == R_SELECT && A.fast && staged && nsrc <= (sorted ? CAP - kCells : CAP);
  const int sub = lane >> 4, l16 = lane & 15;
  int32_t i_pf = 0;
  float4 e_pf[DP / 4];
  if (fast && wave * 4 + sub < nsrc) i_pf = A.bucket[a + s0 + wave * 4 + sub];
  bool pf_done = false;
  auto prefetch_row = [&](bool live) {
#pragma unroll
    for (int q = 0; q < DP / 4; ++q)
      e_pf[q] = live ? *reinterpret_cast<const float4*>(A.emb + (int64_t)i_pf * kDpad + 4 * q)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
    pf_done = true;
  };
  // cell list of a sorted window (in the key array's place): cend[k] ends up
  // as the end of cell k in the slot order sidx
  int* cend = reinterpret_cast<int*>(skey);
  float cell_lo = 0.f, cell_inv = 0.f;
  int ncell = 1;
  auto cell_of = [&](float key) {
    return min(ncell - 1, max(0, (int)((key - cell_lo) * cell_inv)));
  };
  if (staged && !sorted) {
    for (int c = threadIdx.x; c < nwin; c += kRadiusThreads) {
      const int j = wb[c];
      cj[c] = j;
#pragma unroll
      for (int q = 0; q < DP; q += 4)
        *reinterpret_cast<float4*>(cemb + c * DP + q) = *reinterpret_cast<const float4*>(A.emb + (int64_t)j * kDpad + q);
    }
    if (fast) prefetch_row(wave * 4 + sub < nsrc);
    __syncthreads();
  }
  if (sorted && nwin > 0) {
    // stage the window and find its widest axis
    float lo[DP], hi[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) {
      lo[k] = INFINITY;
      hi[k] = -INFINITY;
    }
    for (int c = threadIdx.x; c < nwin; c += kRadiusThreads) {
      int j = wb[c];
      cj[c] = j;
#pragma unroll
      for (int q = 0; q < DP; q += 4) {
        float4 v = *reinterpret_cast<const float4*>(A.emb + (int64_t)j * kDpad + q);
        *reinterpret_cast<float4*>(cemb + c * DP + q) = v;
        lo[q] = fminf(lo[q], v.x); hi[q] = fmaxf(hi[q], v.x);
        lo[q + 1] = fminf(lo[q + 1], v.y); hi[q + 1] = fmaxf(hi[q + 1], v.y);
        lo[q + 2] = fminf(lo[q + 2], v.z); hi[q + 2] = fmaxf(hi[q + 2], v.z);
        lo[q + 3] = fminf(lo[q + 3], v.w); hi[q + 3] = fmaxf(hi[q + 3], v.w);
      }
    }
    if (fast) prefetch_row(wave * 4 + sub < nsrc);
    // block max of each axis range through the per-wave lists (reused as scratch)
#pragma unroll
    for (int k = 0; k < DP; ++k) {
      float l = lo[k], h = hi[k];
      for (int d = 32; d > 0; d >>= 1) {
        l = fminf(l, __shfl_xor(l, d));
        h = fmaxf(h, __shfl_xor(h, d));
      }
      if (lane == 0) {
        ld2[wave * DP + k] = l;
        ld2[kRadiusWaves * DP + wave * DP + k] = h;
      }
    }
    __syncthreads();
    if (wave == 0) {
      // one lane per axis: its range over the waves (in wave order), then the
      // widest axis, the first one among equal widths (an axis whose width is
      // not above -1, or NaN, is never chosen; none: axis 0)
      float l = INFINITY, h = -INFINITY;
      if (lane < A.dim) {
        for (int w = 0; w < kRadiusWaves; ++w) {
          l = fminf(l, ld2[w * DP + lane]);
          h = fmaxf(h, ld2[kRadiusWaves * DP + w * DP + lane]);
        }
      }
      const float wd = h - l;
      const bool valid = lane < A.dim && wd > -1.f;
      float m = valid ? wd : -INFINITY;
      for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
      const uint64_t at = __ballot(valid && wd == m);
      const int best = at ? __ffsll((unsigned long long)at) - 1 : 0;
      if (lane == best) {
        misc[0] = best;
        misc[2] = __float_as_int(l);
        misc[3] = __float_as_int(h);
      }
    }
    __syncthreads();
    // cell list along that axis: cells about r wide over the window's extent
    // (at most kCells), counted, scanned and filled through LDS cursors.  The
    // order inside a cell is arbitrary: what is kept below does not depend on
    // the order in which candidates are visited.
    const int axis = misc[0];
    cell_lo = __int_as_float(misc[2]);
    const float width = __int_as_float(misc[3]) - cell_lo;
    ncell = width > 0.f ? (int)fminf((float)kCells, width / A.r + 1.0f) : 1;
    cell_inv = width > 0.f ? (float)ncell / width : 0.f;
    for (int k = threadIdx.x; k < ncell; k += kRadiusThreads) hist[k] = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < nwin; c += kRadiusThreads) atomicAdd(&hist[cell_of(cemb[c * DP + axis])], 1);
    __syncthreads();
    if (wave == 0) {
      // exclusive scan of the counts, four cells per lane
      int v[kCells / 64], sum = 0;
#pragma unroll
      for (int i = 0; i < kCells / 64; ++i) {
        const int k = lane * (kCells / 64) + i;
        v[i] = k < ncell ? hist[k] : 0;
        sum += v[i];
      }
      int incl = sum;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
      }
      int run = incl - sum;
#pragma unroll
      for (int i = 0; i < kCells / 64; ++i) {
        const int k = lane * (kCells / 64) + i;
        if (k < ncell) cend[k] = run;
        run += v[i];
      }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nwin; c += kRadiusThreads) sidx[atomicAdd(&cend[cell_of(cemb[c * DP + axis])], 1)] = c;
    __syncthreads();
  }
  const int axis = (sorted && nwin > 0) ? misc[0] : 0;
  // candidate range [cb, ce) of a source on a sorted window: the cells that
  // its axis coordinate +- reach falls in (reach covers the rounding of the
  // coordinates and of d^2, so no candidate within r is missed)
  auto range = [&](const float (&se)[DP], int& cb, int& ce) {
    cb = 0;
    ce = nwin;
    if (sorted && nwin > 0) {
      float sa = 0.f;
#pragma unroll
      for (int k = 0; k < DP; ++k)
        if (k == axis) sa = se[k];
      const float reach = A.r * (1.0f + 1.0f / 65536.0f) + fabsf(sa) * (1.0f / 1048576.0f) + 1e-30f;
      const int clo = cell_of(sa - reach), chi = cell_of(sa + reach);
      cb = clo > 0 ? cend[clo - 1] : 0;
      ce = cend[chi];
    }
  };
  float* wl2 = ld2 + wave * kList;
  int* wlj = lj + wave * kList;
  int* sl = sel + wave * 64;
  int* hw = hist + wave * 256;

  // Fast path of the select pass over a staged window: four sources per wave,
  // one per 16-lane row, each over its own candidate range.  A source with at
  // most 16 in-radius candidates (and no k_max cut) is finished here: its
  // targets, ranked by index, are exactly what the full path keeps.  Other
  // sources go to a list (the slot array of a scanned window, the key array
  // past the cell ends of a sorted one) for the one-wave-per-source path.
  int* hard = sorted ? cend + kCells : sidx;
  int nwork = nsrc;
  if (fast) {
    if (!pf_done) prefetch_row(wave * 4 + sub < nsrc);
    if (threadIdx.x == 0) misc[1] = 0;
    __syncthreads();
    int* sb = sl + 16 * sub;
    for (int s4 = wave * 4; s4 < nsrc; s4 += kRadiusWaves * 4) {
      const int s = s4 + sub;
      const bool live = s < nsrc;
      const int32_t i = i_pf;
      float se[DP];
#pragma unroll
      for (int q = 0; q < DP / 4; ++q) {
        se[4 * q] = e_pf[q].x; se[4 * q + 1] = e_pf[q].y; se[4 * q + 2] = e_pf[q].z; se[4 * q + 3] = e_pf[q].w;
      }
      const bool live_next = s + kRadiusWaves * 4 < nsrc;
      i_pf = live_next ? A.bucket[a + s0 + s + kRadiusWaves * 4] : 0;
      int cb, ce;
      range(se, cb, ce);
      // the longest of the four ranges (rows hold one value each)
      int len = live ? ce - cb : 0;
      len = max(len, __shfl_xor(len, 16));
      len = max(len, __shfl_xor(len, 32));
      int n = 0;
      for (int c0 = 0; c0 < len; c0 += 16) {
        const int c = cb + c0 + l16;
        bool in = false;
        int j = 0;
        if (live && c < ce) {
          const int slot = sorted ? sidx[c] : c;
          j = cj[slot];
          in = dist2<DP>(se, cemb + slot * DP) < A.r2;
        }
        const uint32_t m = (uint32_t)(__ballot(in) >> (16 * sub)) & 0xffffu;
        if (in) {
          const int pos = n + __popc(m & ((1u << l16) - 1u));
          if (pos < 16) sb[pos] = j;
        }
        n += __popc(m);
      }
      prefetch_row(live_next);
      wave_sync();
      const bool done = live && n <= 16 && n <= A.k_max;
      if (done) {
        if (l16 < n) {
          const int my = sb[l16];
          int rank = 0;
          for (int q = 0; q < n; ++q) rank += sb[q] < my;
          A.slots[slot_index(i, rank, A.n_hits, A.k_max)] = my;
        }
        if (l16 == 0) A.cnt[i] = n;
      } else if (live && l16 == 0) {
        hard[atomicAdd(&misc[1], 1)] = s;
      }
      wave_sync();
    }
    __syncthreads();
    nwork = misc[1];
  }
  auto source_of = [&](int h) { return fast ? hard[h] : h; };

  // the next source's index and embedding load while this one is processed
  int32_t i_next = wave < nwork ? A.bucket[a + s0 + source_of(wave)] : 0;
  float4 e_next[DP / 4];
#pragma unroll
  for (int q = 0; q < DP / 4; ++q)
    e_next[q] = wave < nwork ? *reinterpret_cast<const float4*>(A.emb + (int64_t)i_next * kDpad + 4 * q)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int h = wave; h < nwork; h += kRadiusWaves) {
    const int32_t i = i_next;
    float se[DP];
#pragma unroll
    for (int q = 0; q < DP / 4; ++q) {
      se[4 * q] = e_next[q].x; se[4 * q + 1] = e_next[q].y; se[4 * q + 2] = e_next[q].z; se[4 * q + 3] = e_next[q].w;
    }
    if (h + kRadiusWaves < nwork) {
      i_next = A.bucket[a + s0 + source_of(h + kRadiusWaves)];
#pragma unroll
      for (int q = 0; q < DP / 4; ++q)
        e_next[q] = *reinterpret_cast<const float4*>(A.emb + (int64_t)i_next * kDpad + 4 * q);
    }
    int cb, ce;
    range(se, cb, ce);
    auto cand = [&](int c, int& j) -> float {
      if (staged) {
        const int slot = sorted ? sidx[c] : c;
        j = cj[slot];
        return dist2<DP>(se, cemb + slot * DP);
      }
      j = wb[c];
      return dist2<DP>(se, A.emb + (int64_t)j * kDpad);
    };
    // pass 1: in-radius candidates, compacted into the wave's list
    int n = 0;
    for (int c0 = cb; c0 < ce; c0 += 64) {
      const int c = c0 + lane;
      bool in = false;
      float d2 = 0.f;
      int j = 0;
      if (c < ce) {
        d2 = cand(c, j);
        in = d2 < A.r2;
      }
      const uint64_t m = __ballot(in);
      if (EMIT && in) {
        const int pos = n + __popcll(m & ((1ull << lane) - 1ull));
        if (pos < kList) {
          wl2[pos] = d2;
          wlj[pos] = j;
        }
      }
      n += __popcll(m);
    }
    if (!EMIT) {
      if (lane == 0) A.cnt[i] = min(n, A.k_max);
      continue;
    }
    if (n == 0) {
      if (MODE == R_SELECT && lane == 0) A.cnt[i] = 0;
      continue;
    }
    wave_sync();
    const bool listed = n <= kList;
    // wave-uniform count of in-radius candidates satisfying pred(d2, j)
    auto count_if = [&](auto pred) -> int {
      int m = 0;
      if (listed) {
        for (int q0 = 0; q0 < n; q0 += 64) {
          const int q = q0 + lane;
          const bool b = q < n && pred(wl2[q], wlj[q]);
          m += __popcll(__ballot(b));
        }
      } else {
        for (int c0 = cb; c0 < ce; c0 += 64) {
          const int c = c0 + lane;
          bool b = false;
          if (c < ce) {
            int j;
            const float d2 = cand(c, j);
            b = d2 < A.r2 && pred(d2, j);
          }
          m += __popcll(__ballot(b));
        }
      }
      return m;
    };
    const bool capped = n > A.k_max;
    float T = A.r2;
    int Jt = 0x7fffffff;
    if (capped) {
      // radix select of the k-th smallest d2: four 8-bit digits of its float
      // bits (non-negative floats order like their bits), over the list, or
      // with more than kList in-radius candidates over the candidate range
      // again (four scans)
      unsigned prefix = 0;
      int need = A.k_max, eq = 0;
      for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int b = lane; b < 256; b += 64) hw[b] = 0;
        wave_sync();
        auto bump = [&](float d2) {
          const unsigned key = __float_as_uint(d2);
          if (pass == 0 || (key >> (shift + 8)) == (prefix >> (shift + 8))) atomicAdd(&hw[(key >> shift) & 255u], 1);
        };
        if (listed) {
          for (int q = lane; q < n; q += 64) bump(wl2[q]);
        } else {
          for (int c0 = cb; c0 < ce; c0 += 64) {
            const int c = c0 + lane;
            if (c < ce) {
              int j;
              const float d2 = cand(c, j);
              if (d2 < A.r2) bump(d2);
            }
          }
        }
        wave_sync();
        int c[4], sum = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          c[i] = hw[4 * lane + i];
          sum += c[i];
        }
        int incl = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int t = __shfl_up(incl, d);
          if (lane >= d) incl += t;
        }
        int run = incl - sum, bin = -1, before = 0, cnt = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (bin < 0 && run < need && need <= run + c[i]) {
            bin = 4 * lane + i;
            before = run;
            cnt = c[i];
          }
          run += c[i];
        }
        const uint64_t m = __ballot(bin >= 0);
        const int src_lane = __ffsll((unsigned long long)m) - 1;
        bin = __shfl(bin, src_lane);
        before = __shfl(before, src_lane);
        cnt = __shfl(cnt, src_lane);
        prefix |= (unsigned)bin << shift;
        need -= before;
        eq = cnt;
        wave_sync();
      }
      T = __uint_as_float(prefix);
      if (eq > need) {
        // ties at the boundary distance: keep the `need` smallest hit indices
        int jlo = (int)a, jhi = (int)(A.hit_off[ev + 1] - 1);
        while (jlo < jhi) {
          const int mid = jlo + (jhi - jlo) / 2;
          const int m = count_if([&](float d2, int j) { return d2 == T && j <= mid; });
          if (m >= need) jhi = mid; else jlo = mid + 1;
        }
        Jt = jlo;
      }
    }
    // compact the kept targets (at most k_max <= 64) into the wave's row buffer
    int ns = 0;
    auto keep = [&](float d2, int j) { return d2 < A.r2 && (!capped || d2 < T || (d2 == T && j <= Jt)); };
    if (listed) {
      for (int q0 = 0; q0 < n; q0 += 64) {
        const int q = q0 + lane;
        const bool b = q < n && keep(wl2[q], wlj[q]);
        const uint64_t m = __ballot(b);
        if (b) {
          const int pos = ns + __popcll(m & ((1ull << lane) - 1ull));
          if (pos < 64) sl[pos] = wlj[q];
        }
        ns += __popcll(m);
      }
    } else {
      for (int c0 = cb; c0 < ce; c0 += 64) {
        const int c = c0 + lane;
        bool b = false;
        int j = 0;
        if (c < ce) {
          const float d2 = cand(c, j);
          b = keep(d2, j);
        }
        const uint64_t m = __ballot(b);
        if (b) {
          const int pos = ns + __popcll(m & ((1ull << lane) - 1ull));
          if (pos < 64) sl[pos] = j;
        }
        ns += __popcll(m);
      }
    }
    if (MODE == R_SELECT) {
      ns = min(ns, A.k_max);
      if (lane == 0) A.cnt[i] = ns;
    } else {
      // never write past the row the count pass reserved
      ns = min(ns, (int)(A.row_ptr[i + 1] - A.row_ptr[i]));
    }
    wave_sync();
    if (lane < ns) {
      const int my = sl[lane];
      int rank = 0;
      for (int q = 0; q < ns; ++q) rank += sl[q] < my;
      if (MODE == R_SELECT) {
        A.slots[slot_index(i, rank, A.n_hits, A.k_max)] = my;
      } else {
        const int64_t pos = A.row_ptr[i] + rank;
        A.src[pos] = i;
        A.dst[pos] = my;
      }
    }
    wave_sync();
  }
}

// One workgroup per (event, plane) unit.
template <int MODE, int DP, bool SMALL>
__global__ __launch_bounds__(kRadiusThreads) void k_radius(RadiusArgs A) {
  extern __shared__ float lds[];
  radius_unit<MODE, DP, SMALL>(A, lds, blockIdx.x / A.n_planes, blockIdx.x % A.n_planes);
}

// CSR rows from the select pass's slots: thread (source i, rank r) copies
// slot r of source i when r is below its count.
// One wave per chunk of 64 hits.  The chunk's CSR rows are one contiguous
// range of the output, so lane l writes positions l, l + 64, ... of it (every
// store coalesced, no idle lanes whatever the row lengths); the row of a
// position is found by a binary search over the chunk's row starts, one per
// lane, read with lane shuffles.
__global__ __launch_bounds__(256) void k_slots_to_csr(const int32_t* __restrict__ slots, const int64_t* __restrict__ row_ptr,
                                                      int64_t n_hits, int k_max, int32_t* __restrict__ src,
                                                      int32_t* __restrict__ dst, const int64_t* status) {
  if (status[0] != 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t nchunks = (n_hits + 63) / 64;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t ch = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; ch < nchunks; ch += stride) {
    const int64_t h0 = ch * 64;
    const int64_t base = row_ptr[h0];
    const int64_t end = row_ptr[min(h0 + 64, n_hits)];
    // row start of this lane's hit relative to the chunk (past the last hit:
    // the chunk's end, so that no position maps there)
    const int rel = (int)((h0 + lane < n_hits ? row_ptr[h0 + lane] : end) - base);
    const int total = (int)(end - base);
    // the whole wave runs every round (the shuffles read every lane's rel)
    for (int q0 = 0; q0 < total; q0 += 64) {
      const int q = q0 + lane;
      int lo = 0, hi = 63;                       // largest l with rel_l <= q
#pragma unroll
      for (int step = 0; step < 6; ++step) {
        const int mid = (lo + hi + 1) >> 1;
        if (__shfl(rel, mid) <= q) lo = mid; else hi = mid - 1;
      }
      const int r0 = __shfl(rel, lo);
      if (q < total) {
        const int64_t i = h0 + lo;
        src[base + q] = (int32_t)i;
        dst[base + q] = slots[slot_index(i, q - r0, n_hits, k_max)];
      }
    }
  }
}

}  // namespace

hipError_t launch_slots_copy(const RunArgs& a, bool candidates) {
  const int64_t n = a.hits.n_hits;
  if (n == 0) return hipSuccess;
  const int k = a.ctx->cfg.k_max;
  const int64_t chunks = (n + 63) / 64;
  const unsigned grid = (unsigned)std::min<int64_t>((chunks + 3) / 4, (int64_t)a.ctx->n_cu * 32);
  const int32_t* slots = reinterpret_cast<const int32_t*>(a.ws + a.L.slots);
  const int64_t* rp = reinterpret_cast<const int64_t*>(a.ws + (candidates ? a.L.pf_tmp : a.L.row_ptr));
  int32_t* s = candidates ? reinterpret_cast<int32_t*>(a.ws + a.L.cand_src) : a.out.src;
  int32_t* d = candidates ? reinterpret_cast<int32_t*>(a.ws + a.L.cand_dst) : a.out.dst;
  hipLaunchKernelGGL(k_slots_to_csr, dim3(grid), dim3(256), 0, a.stream, slots, rp, n, k, s, d, a.out.status);
  return hipGetLastError();
}

hipError_t launch_radius(const RunArgs& a, int mode, bool candidates) {
  if (a.hits.n_events == 0) return hipSuccess;
  const etx_config& c = a.ctx->cfg;
  RadiusArgs A;
  A.hit_off = a.hits.hit_off;
  A.bucket = reinterpret_cast<const int32_t*>(a.ws + a.L.bucket);
  A.plane_off = reinterpret_cast<const int32_t*>(a.ws + a.L.plane_off);
  A.emb = reinterpret_cast<const float*>(a.ws + a.L.emb);
  A.n_planes = c.n_planes;
  A.window = c.plane_window;
  A.k_max = c.k_max;
  A.dim = c.emb_dim;
  A.r = a.radius_override > 0.f ? a.radius_override : c.radius;
  A.r2 = A.r * A.r;
  A.cnt = reinterpret_cast<int32_t*>(a.ws + a.L.cnt);
  // with the prefilter the candidate graph goes to workspace buffers first
  A.row_ptr = reinterpret_cast<const int64_t*>(a.ws + (candidates ? a.L.pf_tmp : a.L.row_ptr));
  A.src = candidates ? reinterpret_cast<int32_t*>(a.ws + a.L.cand_src) : a.out.src;
  A.dst = candidates ? reinterpret_cast<int32_t*>(a.ws + a.L.cand_dst) : a.out.dst;
  A.slots = reinterpret_cast<int32_t*>(a.ws + a.L.slots);
  A.n_hits = a.hits.n_hits;
  A.status = a.out.status;
  dim3 grid((unsigned)(a.hits.n_events * c.n_planes));
  const bool small = c.emb_dim <= 8;
  A.stage_window = a.ctx->radius_lds;
  A.sort_min = a.ctx->radius_sort_min;
  A.fast = a.ctx->radius_fast;
  // the split needs staged windows (it exists for the occupancy of staging)
  A.split = a.ctx->radius_split && A.stage_window ? 1 : 0;
#define LAUNCH_R(M_, D_, S_) \
  hipLaunchKernelGGL((k_radius<M_, D_, S_>), grid, dim3(kRadiusThreads), (RadiusLds<D_, S_>::bytes), a.stream, A)
#define BY_MODE(D_, S_)                                  \
  switch (mode) {                                        \
    case R_COUNT: LAUNCH_R(R_COUNT, D_, S_); break;      \
    case R_EMIT: LAUNCH_R(R_EMIT, D_, S_); break;        \
    default: LAUNCH_R(R_SELECT, D_, S_); break;          \
  }
  if (small) {
    if (A.split) BY_MODE(8, true)
    BY_MODE(8, false)
  } else {
    if (A.split) BY_MODE(16, true)
    BY_MODE(16, false)
  }
#undef BY_MODE
#undef LAUNCH_R
  return hipGetLastError();
}

int radius_attributes(size_t max_lds) {
  int bad = 0;
  auto set = [&](const void* f) {
    bad |= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds) != hipSuccess;
  };
  for (const void* f : {reinterpret_cast<const void*>(k_radius<R_COUNT, 8, false>),
                        reinterpret_cast<const void*>(k_radius<R_EMIT, 8, false>),
                        reinterpret_cast<const void*>(k_radius<R_SELECT, 8, false>),
                        reinterpret_cast<const void*>(k_radius<R_COUNT, 16, false>),
                        reinterpret_cast<const void*>(k_radius<R_EMIT, 16, false>),
                        reinterpret_cast<const void*>(k_radius<R_SELECT, 16, false>),
                        reinterpret_cast<const void*>(k_radius<R_COUNT, 8, true>),
                        reinterpret_cast<const void*>(k_radius<R_EMIT, 8, true>),
                        reinterpret_cast<const void*>(k_radius<R_SELECT, 8, true>),
                        reinterpret_cast<const void*>(k_radius<R_COUNT, 16, true>),
                        reinterpret_cast<const void*>(k_radius<R_EMIT, 16, true>),
                        reinterpret_cast<const void*>(k_radius<R_SELECT, 16, true>)})
    set(f);
  return bad;
}

}  // namespace etx
