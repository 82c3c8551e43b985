/*
 * FP64 CPU oracle of the triplet stage (thesis ch. 8 "The ETX4VELO Pipeline",
 * "Triplet Building" and "Track Building").
 *
 * TEST INFRASTRUCTURE ONLY, like etx_oracle.c (same library): only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code with the HIP path.  One event at a time, hits 0..n-1,
 * edges as the radius graph lists them (sorted by (src, dst)), `keep` the
 * score cut of the edge classifier (the purified hit graph).
 *
 * Readings of the thesis (it describes these steps in words only):
 *  - Triplets are formed around every hit C from its kept in-edges (in edge
 *    order, i.e. by source) and kept out-edges (by target): articulations
 *    (A->C, C->B) for every in/out pair, left elbows (C->A, C->B) for every
 *    pair of out-edges, right elbows (A->C, B->C) for every pair of in-edges.
 *    The batch lists all articulations first (hit by hit, in-edge major),
 *    then all elbows (hit by hit, left before right, pairs in list order).
 *  - A triplet classifier sees the concatenation [e_a, e_b] of the final edge
 *    encodings; for an articulation a is the in-edge, for an elbow a is the
 *    shorter edge (the one whose other hit lies on the plane nearer to C;
 *    equal planes: list order).  Two classifiers, one for articulations and
 *    one for both kinds of elbow, each Linear(H->1)(Block(H->H)(Block(2H->H)))
 *    with Block(x) = ReLU(LN(x W + b)), score = sigmoid; a triplet is kept
 *    when its score reaches the edge threshold.
 *  - Track building, step 1: a kept edge is a duplicate when it is the longer
 *    edge of a kept left elbow at its source and the longer edge of a kept
 *    right elbow at its target (the two elbows connect around the shorter
 *    path through the middle hit); duplicates leave the edge graph.
 *    Step 2: the links of the edge graph are the kept articulations of two
 *    non-duplicate edges; a link (p, q) is shared when p is the first edge of
 *    another link or q the second edge of another link.  Weakly connected
 *    components over the non-shared links; a component is named by its
 *    smallest edge index.  Step 3: every component that no shared link
 *    touches is a track; every shared link (p, q) is a track made of the
 *    components of p and q.  Step 4: a track's hits are the endpoints of its
 *    edges (ascending, without repeats).  Track order: the untouched
 *    components by name, then the shared links in triplet order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <math.h>

/* kept in- and out-edge lists of every hit */
typedef struct {
  int64_t *in_ptr, *out_ptr;
  int32_t *in_e, *out_e;
} adj_t;

static void adj_build(int64_t n, int64_t E, const int32_t* src, const int32_t* dst, const uint8_t* keep, adj_t* A) {
  A->in_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  A->out_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t nk = 0;
  for (int64_t e = 0; e < E; ++e)
    if (keep[e]) { A->out_ptr[src[e] + 1]++; A->in_ptr[dst[e] + 1]++; ++nk; }
  for (int64_t i = 0; i < n; ++i) { A->out_ptr[i + 1] += A->out_ptr[i]; A->in_ptr[i + 1] += A->in_ptr[i]; }
  A->in_e = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nk + 1));
  A->out_e = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nk + 1));
  int64_t* fi = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* fo = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  memcpy(fi, A->in_ptr, sizeof(int64_t) * (size_t)(n + 1));
  memcpy(fo, A->out_ptr, sizeof(int64_t) * (size_t)(n + 1));
  /* visiting edges in increasing index keeps both lists in edge order */
  for (int64_t e = 0; e < E; ++e)
    if (keep[e]) { A->out_e[fo[src[e]]++] = (int32_t)e; A->in_e[fi[dst[e]]++] = (int32_t)e; }
  free(fi); free(fo);
}

static void adj_free(adj_t* A) { free(A->in_ptr); free(A->out_ptr); free(A->in_e); free(A->out_e); }

/* Triplets of the purified graph.  kind: 0 articulation, 1 left elbow,
 * 2 right elbow; (ta[t], tb[t]) in classifier input order.  Returns the
 * number of triplets (entries beyond cap are counted, not written). */
int64_t oracle_triplets(int64_t n, int64_t E, const int32_t* src, const int32_t* dst, const int32_t* plane,
                        const uint8_t* keep, int32_t* ta, int32_t* tb, uint8_t* kind, int64_t cap) {
  adj_t A;
  adj_build(n, E, src, dst, keep, &A);
  int64_t t = 0;
#define PUT(a, b, k) do { if (t < cap) { ta[t] = (a); tb[t] = (b); kind[t] = (uint8_t)(k); } ++t; } while (0)
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = A.in_ptr[c]; i < A.in_ptr[c + 1]; ++i)
      for (int64_t o = A.out_ptr[c]; o < A.out_ptr[c + 1]; ++o) PUT(A.in_e[i], A.out_e[o], 0);
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t o1 = A.out_ptr[c]; o1 < A.out_ptr[c + 1]; ++o1)
      for (int64_t o2 = o1 + 1; o2 < A.out_ptr[c + 1]; ++o2) {
        const int32_t a = A.out_e[o1], b = A.out_e[o2];
        /* shorter first: the target on the nearer plane */
        if (plane[dst[b]] < plane[dst[a]]) PUT(b, a, 1); else PUT(a, b, 1);
      }
    for (int64_t i1 = A.in_ptr[c]; i1 < A.in_ptr[c + 1]; ++i1)
      for (int64_t i2 = i1 + 1; i2 < A.in_ptr[c + 1]; ++i2) {
        const int32_t a = A.in_e[i1], b = A.in_e[i2];
        /* shorter first: the source on the nearer (higher) plane */
        if (plane[src[b]] > plane[src[a]]) PUT(b, a, 2); else PUT(a, b, 2);
      }
  }
#undef PUT
  adj_free(&A);
  return t;
}

/* LayerNorm over n features (biased variance, eps 1e-5, unit gain, zero
 * shift), then ReLU. */
static void ln_relu(double* v, int n) {
  double mean = 0.0, var = 0.0;
  for (int i = 0; i < n; ++i) mean += v[i];
  mean /= n;
  for (int i = 0; i < n; ++i) var += (v[i] - mean) * (v[i] - mean);
  var /= n;
  const double rs = 1.0 / sqrt(var + 1e-5);
  for (int i = 0; i < n; ++i) {
    const double y = (v[i] - mean) * rs;
    v[i] = y > 0.0 ? y : 0.0;
  }
}

/* y[m] = b[m] + sum_k x[k] W[k][m] */
static void lin(const double* x, int K, const double* W, const double* b, int M, double* y) {
  for (int m = 0; m < M; ++m) {
    double s = b[m];
    for (int k = 0; k < K; ++k) s += x[k] * W[(int64_t)k * M + m];
    y[m] = s;
  }
}

/* Floats of one triplet classifier of width H. */
int64_t oracle_triplet_head_size(int H) { return 2LL * H * H + H + (int64_t)H * H + H + H + 1; }

/* Logits of the triplets.  e: final edge encodings [E][H]; params: the
 * articulation classifier, then the elbow classifier, each W1[2H][H] b1[H]
 * W2[H][H] b2[H] w3[H] b3[1]. */
void oracle_triplet_logits(int64_t T, const int32_t* ta, const int32_t* tb, const uint8_t* kind, const double* e,
                           int H, const double* params, double* logit) {
  const int64_t hs = oracle_triplet_head_size(H);
  double* x = (double*)malloc(sizeof(double) * 2 * H);
  double* y1 = (double*)malloc(sizeof(double) * H);
  double* y2 = (double*)malloc(sizeof(double) * H);
  for (int64_t t = 0; t < T; ++t) {
    const double* p = params + (kind[t] == 0 ? 0 : hs);
    const double *W1 = p, *b1 = W1 + 2 * H * H, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H, *b3 = w3 + H;
    memcpy(x, e + (int64_t)ta[t] * H, sizeof(double) * H);
    memcpy(x + H, e + (int64_t)tb[t] * H, sizeof(double) * H);
    lin(x, 2 * H, W1, b1, H, y1);
    ln_relu(y1, H);
    lin(y1, H, W2, b2, H, y2);
    ln_relu(y2, H);
    double s = b3[0];
    for (int m = 0; m < H; ++m) s += y2[m] * w3[m];
    logit[t] = s;
  }
  free(x); free(y1); free(y2);
}

static int cmp_i32(const void* A, const void* B) {
  const int32_t a = *(const int32_t*)A, b = *(const int32_t*)B;
  return (a > b) - (a < b);
}

/* Tracks of the purified edge graph (the four steps above).  tkeep[t]: the
 * triplet's score cut.  Writes dup[E] (1: duplicate edge), comp[E] (component
 * name of a kept non-duplicate edge, else -1), the track list as
 * track_off[0..n_tracks] into track_hits, and, per track, its components
 * (track_c1, track_c2; c2 = -1 for an untouched component).  Returns the
 * number of tracks; entries beyond track_cap / hit_cap are counted only
 * (*n_track_hits receives the hits needed). */
int64_t oracle_build_tracks(int64_t n, int64_t E, const int32_t* src, const int32_t* dst, const int32_t* plane,
                            const uint8_t* keep, int64_t T, const int32_t* ta, const int32_t* tb,
                            const uint8_t* kind, const uint8_t* tkeep, uint8_t* dup, int32_t* comp,
                            int64_t* track_off, int32_t* track_hits, int32_t* track_c1, int32_t* track_c2,
                            int64_t track_cap, int64_t hit_cap, int64_t* n_track_hits) {
  /* step 1: duplicates (longer edge of a kept left elbow and of a kept right elbow) */
  uint8_t* far_left = (uint8_t*)calloc((size_t)E + 1, 1);
  uint8_t* far_right = (uint8_t*)calloc((size_t)E + 1, 1);
  for (int64_t t = 0; t < T; ++t) {
    if (!tkeep[t] || kind[t] == 0) continue;
    const int32_t a = ta[t], b = tb[t];
    if (kind[t] == 1 && plane[dst[b]] > plane[dst[a]]) far_left[b] = 1;
    if (kind[t] == 2 && plane[src[b]] < plane[src[a]]) far_right[b] = 1;
  }
  for (int64_t e = 0; e < E; ++e) dup[e] = (uint8_t)(keep[e] && far_left[e] && far_right[e]);
  free(far_left); free(far_right);
  /* step 2: links, shared links, components over the non-shared links */
  int32_t* n_first = (int32_t*)calloc((size_t)E + 1, sizeof(int32_t));
  int32_t* n_second = (int32_t*)calloc((size_t)E + 1, sizeof(int32_t));
  uint8_t* live = (uint8_t*)calloc((size_t)T + 1, 1);
  for (int64_t t = 0; t < T; ++t)
    if (kind[t] == 0 && tkeep[t] && !dup[ta[t]] && !dup[tb[t]]) {
      live[t] = 1;
      n_first[ta[t]]++;
      n_second[tb[t]]++;
    }
  uint8_t* shared = (uint8_t*)calloc((size_t)T + 1, 1);
  for (int64_t t = 0; t < T; ++t) shared[t] = (uint8_t)(live[t] && (n_first[ta[t]] > 1 || n_second[tb[t]] > 1));
  /* undirected adjacency of the edge graph over the non-shared links */
  int64_t* deg = (int64_t*)calloc((size_t)E + 1, sizeof(int64_t));
  for (int64_t t = 0; t < T; ++t)
    if (live[t] && !shared[t]) { deg[ta[t] + 1]++; deg[tb[t] + 1]++; }
  for (int64_t e = 0; e < E; ++e) deg[e + 1] += deg[e];
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(deg[E] + 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(E + 1));
  memcpy(fill, deg, sizeof(int64_t) * (size_t)(E + 1));
  for (int64_t t = 0; t < T; ++t)
    if (live[t] && !shared[t]) { nb[fill[ta[t]]++] = tb[t]; nb[fill[tb[t]]++] = ta[t]; }
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(E + 1));
  for (int64_t e = 0; e < E; ++e) comp[e] = -1;
  for (int64_t r = 0; r < E; ++r) {
    if (!keep[r] || dup[r] || comp[r] >= 0) continue;
    /* roots in increasing index: each component is named by its smallest edge */
    int64_t qh = 0, qt = 0;
    queue[qt++] = (int32_t)r;
    comp[r] = (int32_t)r;
    while (qh < qt) {
      const int32_t u = queue[qh++];
      for (int64_t k = deg[u]; k < deg[u + 1]; ++k)
        if (comp[nb[k]] < 0) { comp[nb[k]] = (int32_t)r; queue[qt++] = nb[k]; }
    }
  }
  /* step 3: tracks */
  uint8_t* touched = (uint8_t*)calloc((size_t)E + 1, 1);
  for (int64_t t = 0; t < T; ++t)
    if (shared[t]) { touched[comp[ta[t]]] = 1; touched[comp[tb[t]]] = 1; }
  int64_t nt = 0;
  for (int64_t e = 0; e < E; ++e)
    if (keep[e] && !dup[e] && comp[e] == e && !touched[e]) {
      if (nt < track_cap) { track_c1[nt] = (int32_t)e; track_c2[nt] = -1; }
      ++nt;
    }
  for (int64_t t = 0; t < T; ++t)
    if (shared[t]) {
      if (nt < track_cap) { track_c1[nt] = comp[ta[t]]; track_c2[nt] = comp[tb[t]]; }
      ++nt;
    }
  /* step 4: hits of every track (endpoints of its components' edges) */
  int64_t* cptr = (int64_t*)calloc((size_t)E + 1, sizeof(int64_t));
  for (int64_t e = 0; e < E; ++e)
    if (comp[e] >= 0) cptr[comp[e] + 1]++;
  for (int64_t e = 0; e < E; ++e) cptr[e + 1] += cptr[e];
  int32_t* cedge = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cptr[E] + 1));
  memcpy(fill, cptr, sizeof(int64_t) * (size_t)(E + 1));
  for (int64_t e = 0; e < E; ++e)
    if (comp[e] >= 0) cedge[fill[comp[e]]++] = (int32_t)e;
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * cptr[E] + 2));
  int64_t nh = 0;
  const int64_t ntw = nt < track_cap ? nt : track_cap;
  if (track_cap > 0) track_off[0] = 0;
  for (int64_t k = 0; k < ntw; ++k) {
    int64_t m = 0;
    const int32_t cs[2] = {track_c1[k], track_c2[k]};
    for (int j = 0; j < 2; ++j) {
      if (cs[j] < 0 || (j == 1 && cs[1] == cs[0])) continue;
      for (int64_t q = cptr[cs[j]]; q < cptr[cs[j] + 1]; ++q) {
        buf[m++] = src[cedge[q]];
        buf[m++] = dst[cedge[q]];
      }
    }
    qsort(buf, (size_t)m, sizeof(int32_t), cmp_i32);
    for (int64_t q = 0; q < m; ++q)
      if (q == 0 || buf[q] != buf[q - 1]) {
        if (nh < hit_cap) track_hits[nh] = buf[q];
        ++nh;
      }
    track_off[k + 1] = nh;
  }
  *n_track_hits = nh;
  free(n_first); free(n_second); free(live); free(shared); free(deg); free(nb); free(fill); free(queue);
  free(touched); free(cptr); free(cedge); free(buf);
  return nt;
}
