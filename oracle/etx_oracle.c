/*
 * FP64 CPU oracle of the GNN track-finding hot path (ETX4VELO, thesis ch. 8-9).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with the
 * HIP path: every step below is written from its definition in the thesis,
 * in double precision, with plain loops, one event at a time.
 *
 * Steps (one event, hits indexed 0..n-1 in the caller's order):
 *   features    ch. 8 "Hit Embedding and Rough Graph Construction" (normalised
 *               cylindrical input of the embedding) and ch. 8 "Graph Neural
 *               Network and Classifiers" (normalised Cartesian node input)
 *   embedding   the embedding MLP (Linear, ReLU between layers, linear output)
 *   radius      the squared-distance equation of ch. 8 and the k-NN algorithm of
 *               ch. 9 "k-NN Implementation": brute force over the next
 *               `window` planes, d^2 < r^2, keep the k_max smallest by (d^2, j)
 *   gnn         ch. 8 "Graph Neural Network": node/edge encoders, the message
 *               equation (concatenated out-sum and in-sum), residual node and
 *               edge updates with distinct networks per step, edge classifier
 *   components  ch. 9 "WCC Implementation" (DFS/BFS weakly connected
 *               components); the label is the smallest hit index in the
 *               component
 *
 * Optional quantisation (thesis ch. 4 "Quantization", symmetric scale
 * x = S x_q with a per-tensor scale): every GEMM operand is replaced by its
 * exactly rounded BF16 (qmode 1), FP8-E4M3 (qmode 2, value / S rounded, then
 * times S) or INT8 (qmode 3, value / S rounded to an integer in [-127, 127],
 * then times S) value before the FP64 product.  FP8 scales are powers of two
 * chosen from the tensor's absolute maximum, INT8 scales are that maximum over
 * 127 (static calibration: the maxima come from an unquantised run of this
 * oracle).  qmode 0 disables it.  The node
 * and edge state between layers stays full precision unless the network is
 * asked to store it compactly (see oracle_gnn).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* quantisers written from the number formats' definitions                   */
/* ------------------------------------------------------------------------ */

/* Round x to the nearest value with `mbits` fraction bits and minimum normal
 * exponent emin (subnormals below it), ties to even; saturate at +-maxv. */
static double round_format(double x, int mbits, int emin, double maxv) {
  if (x != x) return x;
  double a = fabs(x);
  if (a == 0.0) return x;
  int e;
  frexp(a, &e);            /* a = f * 2^e, f in [0.5, 1) -> leading bit is 2^(e-1) */
  int lead = e - 1;
  if (lead < emin) lead = emin;            /* subnormal spacing */
  double ulp = ldexp(1.0, lead - mbits);
  double q = a / ulp;                       /* exact: power-of-two scaling */
  double r = nearbyint(q);                  /* default rounding mode: ties to even */
  double v = r * ulp;
  if (v > maxv) v = maxv;
  return x < 0 ? -v : v;
}

double oracle_round_bf16(double x) { return round_format(x, 7, -126, 3.3895313892515355e38); }
double oracle_round_e4m3(double x) { return round_format(x, 3, -6, 448.0); }

/* symmetric INT8 code of v (= x / S): round to nearest, ties to even, clipped to +-127 */
double oracle_round_int8(double v) {
  double q = nearbyint(v);
  return q > 127.0 ? 127.0 : (q < -127.0 ? -127.0 : q);
}

/* quantise a GEMM operand: value -> S * round(value / S) (S = 1 for BF16) */
static double qv(int mode, double x, double scale) {
  if (mode == 1) return oracle_round_bf16(x);
  if (mode == 2) return scale * oracle_round_e4m3(x / scale);
  if (mode == 3) return scale * oracle_round_int8(x / scale);
  return x;
}

/* Per-tensor scale from an absolute maximum: the power of two at or above
 * amax / 448, so that amax maps inside the E4M3 range (1 when amax is 0). */
double oracle_pow2_scale(double amax) {
  if (!(amax > 0.0)) return 1.0;
  int e;
  double f = frexp(amax / 448.0, &e);   /* amax/448 = f 2^e, f in [0.5, 1) */
  return ldexp(1.0, f == 0.5 ? e - 1 : e);
}

/* weight scale of a K x M layer: FP8 the power of two at or above max|W| / 448,
 * INT8 (qmode 3) max|W| / 127, the thesis's symmetric range [-max, max]
 * mapped onto [-127, 127] */
static double wscale(int qmode, const double* W, int64_t n) {
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i) m = fabs(W[i]) > m ? fabs(W[i]) : m;
  if (qmode == 3) return m > 0.0 ? m / 127.0 : 1.0;
  return oracle_pow2_scale(m);
}

static void observe(double* amax, int slot, const double* v, int n) {
  if (!amax) return;
  for (int i = 0; i < n; ++i)
    if (fabs(v[i]) > amax[slot]) amax[slot] = fabs(v[i]);
}

/* ------------------------------------------------------------------------ */
/* features                                                                  */
/* ------------------------------------------------------------------------ */

void oracle_features(int64_t n, const float* x, const float* y, const float* z,
                     double r_scale, double z_scale, double* cyl, double* cart) {
  for (int64_t i = 0; i < n; ++i) {
    double xi = x[i], yi = y[i], zi = z[i];
    double r = hypot(xi, yi);
    double phi = atan2(yi, xi);
    cyl[3 * i + 0] = r / r_scale;
    cyl[3 * i + 1] = phi / M_PI;
    cyl[3 * i + 2] = zi / z_scale;
    cart[3 * i + 0] = xi / r_scale;
    cart[3 * i + 1] = yi / r_scale;
    cart[3 * i + 2] = zi / z_scale;
  }
}

/* ------------------------------------------------------------------------ */
/* dense layers                                                              */
/* ------------------------------------------------------------------------ */

/* FP32 evaluation (f32 set): every arithmetic result is rounded to FP32, as
 * an FP32 implementation of the same network would round it.  Used only to
 * measure how far two FP32 evaluations of one (quantised) network fall apart,
 * which sets the low-precision parity tolerances; f32 = 0 is the oracle. */
#define RF(f32, x) ((f32) ? (double)(float)(x) : (x))

/* the quantised copy of a weight matrix (each element rounded once) */
static double* qcopy(int qmode, const double* W, int64_t n, double scale) {
  double* q = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) q[i] = qv(qmode, W[i], scale);
  return q;
}

/* a GEMM input operand: its quantised value; in FP32 evaluation an INT8 code
 * is taken from x times the FP32 reciprocal of the scale */
static double qin(int qmode, double x, double scale, int f32) {
  if (f32 && qmode == 3) return scale * oracle_round_int8(RF(1, x * RF(1, 1.0 / scale)));
  return qv(qmode, x, scale);
}

/* out[m] = b[m] + sum_k q[k] Wq[k][m]: every output's sum runs over k in
 * order (the outputs are independent; they advance together, row by row of Wq) */
static void dot_rows(const double* q, int K, const double* Wq, const double* b, int M, double* out, int f32) {
  double accs[512];
  float accf[512];
  double* acc = M <= 512 ? accs : (double*)malloc(sizeof(double) * M);
  float* af = M <= 512 ? accf : (float*)malloc(sizeof(float) * M);
  if (!f32) {
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    for (int k = 0; k < K; ++k) {
      const double qk = q[k];
      const double* w = Wq + (int64_t)k * M;
      for (int m = 0; m < M; ++m) acc[m] += qk * w[m];
    }
    for (int m = 0; m < M; ++m) out[m] = acc[m] + b[m];
  } else {
    for (int m = 0; m < M; ++m) af[m] = 0.f;
    for (int k = 0; k < K; ++k) {
      const double qk = q[k];
      const double* w = Wq + (int64_t)k * M;
      for (int m = 0; m < M; ++m) af[m] = (float)((double)af[m] + qk * w[m]);
    }
    for (int m = 0; m < M; ++m) out[m] = (float)((double)af[m] + b[m]);
  }
  if (acc != accs) free(acc);
  if (af != accf) free(af);
}

/* out[m] = b[m] + sum_k q(in[k]) Wq[k][m]; Wq row-major [K][M], already
 * quantised; the sum runs over k in order */
static void linear(const double* in, int K, const double* Wq, const double* b, int M,
                   double* out, int qmode, double s_in, int f32) {
  double qs[512];
  double* q = K <= 512 ? qs : (double*)malloc(sizeof(double) * K);
  for (int k = 0; k < K; ++k) q[k] = qin(qmode, in[k], s_in, f32);
  dot_rows(q, K, Wq, b, M, out, f32);
  if (q != qs) free(q);
}

/* Same for an input made of `nb` consecutive blocks of `bk` features, block b
 * quantised with its own scale s_in[b] (one weight scale for the matrix). */
static void linear_blocks(const double* in, int nb, int bk, const double* Wq, const double* b, int M, double* out,
                          int qmode, const double* s_in, int f32) {
  double qs[512];
  double* q = nb * bk <= 512 ? qs : (double*)malloc(sizeof(double) * nb * bk);
  for (int k = 0; k < nb * bk; ++k) q[k] = qin(qmode, in[k], s_in ? s_in[k / bk] : 1.0, f32);
  dot_rows(q, nb * bk, Wq, b, M, out, f32);
  if (q != qs) free(q);
}

/* LayerNorm over the feature axis (biased variance, eps 1e-5, no affine), then ReLU */
static void layernorm_relu(double* v, int n, int f32) {
  double mean = 0.0;
  for (int i = 0; i < n; ++i) mean = RF(f32, mean + v[i]);
  mean = RF(f32, mean / n);
  double var = 0.0;
  for (int i = 0; i < n; ++i) var = RF(f32, var + RF(f32, (v[i] - mean) * (v[i] - mean)));
  var = RF(f32, var / n);
  double inv = RF(f32, 1.0 / sqrt(RF(f32, var + 1e-5)));
  for (int i = 0; i < n; ++i) {
    double t = RF(f32, RF(f32, v[i] - mean) * inv);
    v[i] = t > 0.0 ? t : 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* embedding MLP                                                             */
/* ------------------------------------------------------------------------ */

/* dims[0..n_layers]: widths (dims[0] = 3); params: W0 b0 W1 b1 ...;
 * hidden layers use ReLU, the output layer is linear.  With qmode the GEMM
 * operands of layers l >= 1 are quantised: input with act_scale[l] (FP8),
 * weights with their per-layer power-of-two scale; the 3-wide first layer is
 * not.  amax (may be NULL): running max |input| of layer l in amax[l].
 * f32: FP32 evaluation (see RF). */
void oracle_embed(int64_t n, const double* cyl, int n_layers, const int* dims, const double* params, double* emb,
                  int qmode, const double* act_scale, double* amax, int f32) {
  int maxw = 0;
  for (int l = 0; l <= n_layers; ++l) if (dims[l] > maxw) maxw = dims[l];
  double* a = (double*)malloc(sizeof(double) * maxw);
  double* b = (double*)malloc(sizeof(double) * maxw);
  double* wq[16];
  const double* bias[16];
  {
    const double* p = params;
    for (int l = 0; l < n_layers && l < 16; ++l) {
      int64_t nw = (int64_t)dims[l] * dims[l + 1];
      wq[l] = qcopy(l == 0 ? 0 : qmode, p, nw, wscale(qmode, p, nw));
      bias[l] = p + nw;
      p += nw + dims[l + 1];
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < dims[0]; ++k) a[k] = RF(f32, cyl[3 * i + k]);
    for (int l = 0; l < n_layers; ++l) {
      int K = dims[l], M = dims[l + 1];
      if (l > 0) observe(amax, l, a, K);
      double si = (act_scale && l > 0) ? act_scale[l] : 1.0;
      linear(a, K, wq[l], bias[l], M, b, l == 0 ? 0 : qmode, si, f32);
      if (l + 1 < n_layers)
        for (int m = 0; m < M; ++m) b[m] = b[m] > 0.0 ? b[m] : 0.0;
      memcpy(a, b, sizeof(double) * M);
    }
    for (int m = 0; m < dims[n_layers]; ++m) emb[i * dims[n_layers] + m] = a[m];
  }
  for (int l = 0; l < n_layers && l < 16; ++l) free(wq[l]);
  free(a);
  free(b);
}

/* ------------------------------------------------------------------------ */
/* radius graph (brute force, the definition)                                */
/* ------------------------------------------------------------------------ */

typedef struct { double d2; int32_t j; } cand_t;

static int cand_cmp(const void* A, const void* B) {
  const cand_t* a = (const cand_t*)A;
  const cand_t* b = (const cand_t*)B;
  if (a->d2 < b->d2) return -1;
  if (a->d2 > b->d2) return 1;
  return (a->j > b->j) - (a->j < b->j);
}

static int int_cmp(const void* A, const void* B) {
  int32_t a = *(const int32_t*)A, b = *(const int32_t*)B;
  return (a > b) - (a < b);
}

/* Edges i -> j with 1 <= plane_j - plane_i <= window and d^2(e_i, e_j) < r^2,
 * at most k_max per source (smallest (d^2, j)), sorted by (i, j).
 * Writes at most cap edges; returns the number of edges the graph has. */
int64_t oracle_radius(int64_t n, const int32_t* plane, const double* emb, int D,
                      double radius, int k_max, int window,
                      int32_t* src, int32_t* dst, int64_t cap) {
  double r2 = radius * radius;
  cand_t* c = (cand_t*)malloc(sizeof(cand_t) * (n > 0 ? n : 1));
  int32_t* sel = (int32_t*)malloc(sizeof(int32_t) * (k_max > 0 ? k_max : 1));
  int64_t E = 0;
  for (int64_t i = 0; i < n; ++i) {
    int nc = 0;
    for (int64_t j = 0; j < n; ++j) {
      int dp = plane[j] - plane[i];
      if (dp < 1 || dp > window) continue;
      double d2 = 0.0;
      for (int k = 0; k < D; ++k) {
        double t = emb[i * D + k] - emb[j * D + k];
        d2 += t * t;
      }
      if (d2 < r2) { c[nc].d2 = d2; c[nc].j = (int32_t)j; ++nc; }
    }
    qsort(c, nc, sizeof(cand_t), cand_cmp);
    int keep = nc < k_max ? nc : k_max;
    for (int t = 0; t < keep; ++t) sel[t] = c[t].j;
    qsort(sel, keep, sizeof(int32_t), int_cmp);
    for (int t = 0; t < keep; ++t) {
      if (E < cap) { src[E] = (int32_t)i; dst[E] = sel[t]; }
      ++E;
    }
  }
  free(c);
  free(sel);
  return E;
}

/* Per-source candidate statistics used by the decidability rule of the parity
 * protocol: for source i, the distance gap at the k boundary and the closest
 * |d - r| over its candidate window.  dist_gap[i] = +inf when fewer than
 * k_max+1 candidates lie inside r. */
void oracle_radius_margins(int64_t n, const int32_t* plane, const double* emb, int D,
                           double radius, int k_max, int window,
                           double* r_margin, double* k_gap) {
  cand_t* c = (cand_t*)malloc(sizeof(cand_t) * (n > 0 ? n : 1));
  double r2 = radius * radius;
  for (int64_t i = 0; i < n; ++i) {
    int nc = 0;
    double rm = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      int dp = plane[j] - plane[i];
      if (dp < 1 || dp > window) continue;
      double d2 = 0.0;
      for (int k = 0; k < D; ++k) {
        double t = emb[i * D + k] - emb[j * D + k];
        d2 += t * t;
      }
      double dm = fabs(sqrt(d2) - radius);
      if (dm < rm) rm = dm;
      if (d2 < r2) { c[nc].d2 = d2; c[nc].j = (int32_t)j; ++nc; }
    }
    r_margin[i] = rm;
    if (nc > k_max && k_max > 0) {
      qsort(c, nc, sizeof(cand_t), cand_cmp);
      k_gap[i] = sqrt(c[k_max].d2) - sqrt(c[k_max - 1].d2);
    } else {
      k_gap[i] = INFINITY;
    }
  }
  free(c);
}

/* ------------------------------------------------------------------------ */
/* interaction network                                                       */
/* ------------------------------------------------------------------------ */

/* Activation-scale slots of the quantised interaction network (qmode 2, 3) and
 * of the amax observers; the same tensors are quantised in qmode 1 (BF16,
 * no scale):
 *   0 node-encoder layer-2 input      1 node encodings h (every GEMM use)
 *   2 out-sums mo                     3 in-sums mi
 *   4 edge-encoder layer-2 input      5 node-net layer-2 inputs
 *   6 edge-net layer-2 inputs         7 + k: edge encodings e_k, k = 0..S
 * Every GEMM operand is quantised where it enters the GEMM; LayerNorm, the
 * residual additions, the message sums and the classifier's last layer stay
 * in full precision, and the node and edge encodings between layers are the
 * full-precision (master) values.  With `compact` set, the state itself is
 * stored in low precision instead: the edge encodings e_k <- q(e_k) after the
 * encoder and after every update (the message sums then run over the stored
 * values), and the node encodings h rounded to BF16 after the encoder and
 * after every residual update. */
enum { Q_NE2 = 0, Q_H = 1, Q_MO = 2, Q_MI = 3, Q_EE2 = 4, Q_NN2 = 5, Q_EN2 = 6, Q_E = 7 };

/* Parameter block order: node encoder (3->H->H), edge encoder (2H->H->H),
 * then per step k: node net k (3H->H->H), edge net k (3H->H->H), then the
 * classifier Block(H->H) and Linear(H->1).  Block(x) = ReLU(LN(x W + b)).
 * qmode 0: plain FP64.  act_scale: [8 + S] slots above (qmode 2, 3).  amax
 * (may be NULL, [8 + S]): running max |x| of every quantised tensor.
 * compact (qmode 1, 2): store h and e in low precision (above).
 * f32: FP32 evaluation (see RF).  e_out (may be NULL, [E][H]): the final edge
 * encodings e_S. */
void oracle_gnn(int64_t n, const double* cart, int64_t E, const int32_t* src, const int32_t* dst,
                int H, int S, const double* params, double* logit, int qmode, const double* act_scale,
                double* amax, int compact, int f32, double* e_out) {
  const int qs = qmode && compact;   /* state rounding */
  double* h = (double*)calloc((size_t)n * H + 1, sizeof(double));
  double* e = (double*)calloc((size_t)E * H + 1, sizeof(double));
  double* mo = (double*)calloc((size_t)n * H + 1, sizeof(double));
  double* mi = (double*)calloc((size_t)n * H + 1, sizeof(double));
  double* in = (double*)malloc(sizeof(double) * 3 * H);
  double* tmp = (double*)malloc(sizeof(double) * H);
  double* out = (double*)malloc(sizeof(double) * H);
  double x3[3];
  const double one[3] = {1.0, 1.0, 1.0};
#define SC(slot) (act_scale ? act_scale[slot] : 1.0)
  const int64_t HH = (int64_t)H * H;
  const double* p = params;

  /* node encoder: h0 = Block(Block(x/R, y/R, z/Z)); the 3-wide layer is not quantised */
  {
    const double *W1 = p, *b1 = p + 3 * H, *W2 = b1 + H, *b2 = W2 + HH;
    double* W1q = qcopy(0, W1, 3 * H, 1.0);
    double* W2q = qcopy(qmode, W2, HH, wscale(qmode, W2, HH));
    for (int64_t l = 0; l < n; ++l) {
      for (int c = 0; c < 3; ++c) x3[c] = RF(f32, cart[3 * l + c]);
      linear(x3, 3, W1q, b1, H, tmp, 0, 1.0, f32);
      layernorm_relu(tmp, H, f32);
      observe(amax, Q_NE2, tmp, H);
      linear(tmp, H, W2q, b2, H, h + l * H, qmode, SC(Q_NE2), f32);
      layernorm_relu(h + l * H, H, f32);
      if (qs) for (int c = 0; c < H; ++c) h[l * H + c] = qv(1, h[l * H + c], 1.0);
    }
    free(W1q); free(W2q);
    p = b2 + H;
  }
  /* edge encoder: e0_ij = Block(Block([h_i, h_j])) */
  {
    const double *W1 = p, *b1 = p + 2 * HH, *W2 = b1 + H, *b2 = W2 + HH;
    double* W1q = qcopy(qmode, W1, 2 * HH, wscale(qmode, W1, 2 * HH));
    double* W2q = qcopy(qmode, W2, HH, wscale(qmode, W2, HH));
    double sh[2] = {SC(Q_H), SC(Q_H)};
    for (int64_t l = 0; l < n; ++l) observe(amax, Q_H, h + l * H, H);
    for (int64_t t = 0; t < E; ++t) {
      memcpy(in, h + (int64_t)src[t] * H, sizeof(double) * H);
      memcpy(in + H, h + (int64_t)dst[t] * H, sizeof(double) * H);
      linear_blocks(in, 2, H, W1q, b1, H, tmp, qmode, qmode >= 2 ? sh : NULL, f32);
      layernorm_relu(tmp, H, f32);
      observe(amax, Q_EE2, tmp, H);
      linear(tmp, H, W2q, b2, H, e + t * H, qmode, SC(Q_EE2), f32);
      layernorm_relu(e + t * H, H, f32);
      observe(amax, Q_E + 0, e + t * H, H);
      if (qs) for (int c = 0; c < H; ++c) e[t * H + c] = qv(qmode, e[t * H + c], SC(Q_E + 0));
    }
    free(W1q); free(W2q);
    p = b2 + H;
  }

  for (int k = 0; k < S; ++k) {
    /* messages: m_l = [sum_{l->j} e_lj, sum_{i->l} e_il] in edge order */
    memset(mo, 0, sizeof(double) * n * H);
    memset(mi, 0, sizeof(double) * n * H);
    for (int64_t t = 0; t < E; ++t)
      for (int c = 0; c < H; ++c) {
        mo[(int64_t)src[t] * H + c] = RF(f32, mo[(int64_t)src[t] * H + c] + e[t * H + c]);
        mi[(int64_t)dst[t] * H + c] = RF(f32, mi[(int64_t)dst[t] * H + c] + e[t * H + c]);
      }
    /* node update with residual: h <- h + Block(Block([h, mo, mi])) */
    {
      const double *W1 = p, *b1 = p + 3 * HH, *W2 = b1 + H, *b2 = W2 + HH;
      double* W1q = qcopy(qmode, W1, 3 * HH, wscale(qmode, W1, 3 * HH));
      double* W2q = qcopy(qmode, W2, HH, wscale(qmode, W2, HH));
      double sb[3] = {SC(Q_H), SC(Q_MO), SC(Q_MI)};
      for (int64_t l = 0; l < n; ++l) {
        memcpy(in, h + l * H, sizeof(double) * H);
        memcpy(in + H, mo + l * H, sizeof(double) * H);
        memcpy(in + 2 * H, mi + l * H, sizeof(double) * H);
        observe(amax, Q_H, in, H);
        observe(amax, Q_MO, in + H, H);
        observe(amax, Q_MI, in + 2 * H, H);
        linear_blocks(in, 3, H, W1q, b1, H, tmp, qmode, qmode >= 2 ? sb : (qmode ? one : NULL), f32);
        layernorm_relu(tmp, H, f32);
        observe(amax, Q_NN2, tmp, H);
        linear(tmp, H, W2q, b2, H, out, qmode, SC(Q_NN2), f32);
        layernorm_relu(out, H, f32);
        for (int c = 0; c < H; ++c)
          h[l * H + c] = qs ? qv(1, RF(f32, h[l * H + c] + out[c]), 1.0) : RF(f32, h[l * H + c] + out[c]);
      }
      free(W1q); free(W2q);
      p = b2 + H;
    }
    /* edge update with residual, using the updated h */
    {
      const double *W1 = p, *b1 = p + 3 * HH, *W2 = b1 + H, *b2 = W2 + HH;
      double* W1q = qcopy(qmode, W1, 3 * HH, wscale(qmode, W1, 3 * HH));
      double* W2q = qcopy(qmode, W2, HH, wscale(qmode, W2, HH));
      double sb[3] = {SC(Q_E + k), SC(Q_H), SC(Q_H)};
      for (int64_t l = 0; l < n; ++l) observe(amax, Q_H, h + l * H, H);
      for (int64_t t = 0; t < E; ++t) {
        memcpy(in, e + t * H, sizeof(double) * H);
        memcpy(in + H, h + (int64_t)src[t] * H, sizeof(double) * H);
        memcpy(in + 2 * H, h + (int64_t)dst[t] * H, sizeof(double) * H);
        linear_blocks(in, 3, H, W1q, b1, H, tmp, qmode, qmode >= 2 ? sb : (qmode ? one : NULL), f32);
        layernorm_relu(tmp, H, f32);
        observe(amax, Q_EN2, tmp, H);
        linear(tmp, H, W2q, b2, H, out, qmode, SC(Q_EN2), f32);
        layernorm_relu(out, H, f32);
        for (int c = 0; c < H; ++c) out[c] = RF(f32, out[c] + e[t * H + c]);
        observe(amax, Q_E + k + 1, out, H);
        for (int c = 0; c < H; ++c) e[t * H + c] = qs ? qv(qmode, out[c], SC(Q_E + k + 1)) : out[c];
      }
      free(W1q); free(W2q);
      p = b2 + H;
    }
  }

  /* the final edge encodings e_S (the triplet classifiers' input) */
  if (e_out) memcpy(e_out, e, sizeof(double) * (size_t)E * H);
  /* classifier: Linear(H->1)(Block(H->H)(e)); the input is the stored e_S */
  {
    const double *W1 = p, *b1 = p + HH, *w2 = b1 + H, *b2 = w2 + H;
    double* W1q = qcopy(qmode, W1, HH, wscale(qmode, W1, HH));
    for (int64_t t = 0; t < E; ++t) {
      linear(e + t * H, H, W1q, b1, H, tmp, qmode, SC(Q_E + S), f32);
      layernorm_relu(tmp, H, f32);
      double acc = 0.0;
      for (int c = 0; c < H; ++c) acc = RF(f32, acc + tmp[c] * w2[c]);
      logit[t] = RF(f32, acc + b2[0]);
    }
    free(W1q);
  }
#undef SC
  free(h); free(e); free(mo); free(mi); free(in); free(tmp); free(out);
}

/* ------------------------------------------------------------------------ */
/* connected components (BFS)                                                */
/* ------------------------------------------------------------------------ */

/* Undirected graph of the kept edges; label = smallest hit index of the
 * component (singletons label themselves). */
void oracle_components(int64_t n, int64_t E, const int32_t* src, const int32_t* dst,
                       const uint8_t* keep, int32_t* label) {
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t t = 0; t < E; ++t)
    if (keep[t]) { deg[src[t] + 1]++; deg[dst[t] + 1]++; }
  for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (deg[n] + 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  memcpy(fill, deg, sizeof(int64_t) * (n + 1));
  for (int64_t t = 0; t < E; ++t)
    if (keep[t]) { adj[fill[src[t]]++] = dst[t]; adj[fill[dst[t]]++] = src[t]; }
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  for (int64_t i = 0; i < n; ++i) label[i] = -1;
  /* visiting roots in increasing index order makes each root its component's minimum */
  for (int64_t r = 0; r < n; ++r) {
    if (label[r] >= 0) continue;
    int64_t qh = 0, qt = 0;
    queue[qt++] = (int32_t)r;
    label[r] = (int32_t)r;
    while (qh < qt) {
      int32_t u = queue[qh++];
      for (int64_t a = deg[u]; a < deg[u + 1]; ++a) {
        int32_t v = adj[a];
        if (label[v] < 0) { label[v] = (int32_t)r; queue[qt++] = v; }
      }
    }
  }
  free(deg); free(adj); free(fill); free(queue);
}

/* ------------------------------------------------------------------------ */
/* prefilter features and MLP (forward, loss, backward) for the learned part */
/* ------------------------------------------------------------------------ */

/* f = (dx, dy, dz, dr, dphi, d_emb) of candidate edge i -> j, normalised by
 * (R_s, R_s, Z_s, R_s, pi, 1); dphi wrapped to (-pi, pi]. */
void oracle_prefilter_features(int64_t E, const int32_t* src, const int32_t* dst,
                               const float* x, const float* y, const float* z,
                               const double* emb, int D, double r_scale, double z_scale, double* f) {
  for (int64_t t = 0; t < E; ++t) {
    int32_t i = src[t], j = dst[t];
    double xi = x[i], yi = y[i], zi = z[i], xj = x[j], yj = y[j], zj = z[j];
    double dphi = atan2(yj, xj) - atan2(yi, xi);
    while (dphi > M_PI) dphi -= 2.0 * M_PI;
    while (dphi <= -M_PI) dphi += 2.0 * M_PI;
    double d2 = 0.0;
    for (int k = 0; k < D; ++k) {
      double u = emb[(int64_t)j * D + k] - emb[(int64_t)i * D + k];
      d2 += u * u;
    }
    f[6 * t + 0] = (xj - xi) / r_scale;
    f[6 * t + 1] = (yj - yi) / r_scale;
    f[6 * t + 2] = (zj - zi) / z_scale;
    f[6 * t + 3] = (hypot(xj, yj) - hypot(xi, yi)) / r_scale;
    f[6 * t + 4] = dphi / M_PI;
    f[6 * t + 5] = sqrt(d2);
  }
}

/* Prefilter MLP 6 -> P -> P -> 1 with ReLU; params W1 b1 W2 b2 W3 b3.
 * Forward logits for E edges.  With qmode 1 the operands of the P x P product
 * (hidden activations and W2) are rounded to BF16; the 6-wide input layer
 * and the P -> 1 output layer stay in full precision. */
void oracle_prefilter_forward(int64_t E, const double* f, int P, const double* params,
                              double* logit, int qmode) {
  const double* W1 = params;
  const double* b1 = W1 + 6 * P;
  const double* W2 = b1 + P;
  const double* b2 = W2 + P * P;
  const double* W3 = b2 + P;
  const double* b3 = W3 + P;
  double* a1 = (double*)malloc(sizeof(double) * P);
  double* a2 = (double*)malloc(sizeof(double) * P);
  double* W2q = qcopy(qmode, W2, (int64_t)P * P, 1.0);
  for (int64_t t = 0; t < E; ++t) {
    linear(f + 6 * t, 6, W1, b1, P, a1, 0, 1.0, 0);
    for (int c = 0; c < P; ++c) a1[c] = a1[c] > 0 ? a1[c] : 0;
    linear(a1, P, W2q, b2, P, a2, qmode, 1.0, 0);
    for (int c = 0; c < P; ++c) a2[c] = a2[c] > 0 ? a2[c] : 0;
    double o;
    linear(a2, P, W3, b3, 1, &o, 0, 1.0, 0);
    logit[t] = o;
  }
  free(a1); free(a2); free(W2q);
}

/* Mean class-weighted binary cross-entropy over E edges and its gradient
 * with respect to every parameter (reverse-mode chain rule, thesis ch. 4
 * "Backpropagation"), written out layer by layer.
 * loss = (1/E) sum_t w_t * [softplus(-z) if y=1 else softplus(z)], w_t = pos_w for y=1.
 * With qmode 1 the two P x P products (forward a1 W2 and backward W2 delta2)
 * take BF16-rounded operands; the weight gradients are full precision.
 * grad has the layout of params.  Returns the loss. */
double oracle_prefilter_loss_grad(int64_t E, const double* f, const uint8_t* label, int P,
                                  const double* params, double pos_w, double* grad, int qmode) {
  const double* W1 = params;
  const double* b1 = W1 + 6 * P;
  const double* W2 = b1 + P;
  const double* b2 = W2 + P * P;
  const double* W3 = b2 + P;
  const double* b3 = W3 + P;
  int64_t np = 6 * P + P + P * P + P + P + 1;
  double* gW1 = grad;
  double* gb1 = gW1 + 6 * P;
  double* gW2 = gb1 + P;
  double* gb2 = gW2 + P * P;
  double* gW3 = gb2 + P;
  double* gb3 = gW3 + P;
  memset(grad, 0, sizeof(double) * np);
  double* a1 = (double*)malloc(sizeof(double) * P);
  double* a2 = (double*)malloc(sizeof(double) * P);
  double* d1 = (double*)malloc(sizeof(double) * P);
  double* d2 = (double*)malloc(sizeof(double) * P);
  double* W2q = qcopy(qmode, W2, (int64_t)P * P, 1.0);
  double loss = 0.0;
  for (int64_t t = 0; t < E; ++t) {
    const double* in = f + 6 * t;
    linear(in, 6, W1, b1, P, a1, 0, 1.0, 0);
    for (int c = 0; c < P; ++c) a1[c] = a1[c] > 0 ? a1[c] : 0;
    linear(a1, P, W2q, b2, P, a2, qmode, 1.0, 0);
    for (int c = 0; c < P; ++c) a2[c] = a2[c] > 0 ? a2[c] : 0;
    double z;
    linear(a2, P, W3, b3, 1, &z, 0, 1.0, 0);
    double y = label[t] ? 1.0 : 0.0;
    double w = label[t] ? pos_w : 1.0;
    /* softplus(v) = log(1 + exp(v)), evaluated stably */
    double v = y > 0.5 ? -z : z;
    double sp = v > 0 ? v + log1p(exp(-v)) : log1p(exp(v));
    loss += w * sp;
    double sig = 1.0 / (1.0 + exp(-z));
    double dz = w * (sig - y) / (double)E;
    /* output layer */
    for (int c = 0; c < P; ++c) gW3[c] += a2[c] * dz;
    gb3[0] += dz;
    for (int c = 0; c < P; ++c) d2[c] = (a2[c] > 0 ? 1.0 : 0.0) * W3[c] * dz;
    /* hidden layer 2 */
    for (int k = 0; k < P; ++k)
      for (int c = 0; c < P; ++c) gW2[k * P + c] += a1[k] * d2[c];
    for (int c = 0; c < P; ++c) gb2[c] += d2[c];
    for (int k = 0; k < P; ++k) {
      double s = 0.0;
      for (int c = 0; c < P; ++c) s += W2q[k * P + c] * qv(qmode, d2[c], 1.0);
      d1[k] = (a1[k] > 0 ? 1.0 : 0.0) * s;
    }
    /* hidden layer 1 */
    for (int k = 0; k < 6; ++k)
      for (int c = 0; c < P; ++c) gW1[k * P + c] += in[k] * d1[c];
    for (int c = 0; c < P; ++c) gb1[c] += d1[c];
  }
  free(a1); free(a2); free(d1); free(d2); free(W2q);
  return E > 0 ? loss / (double)E : 0.0;
}

/* One Adam step (Kingma & Ba, cited in thesis ch. 4 "Gradient Descent"):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; mhat = m/(1-b1^t); vhat = v/(1-b2^t);
 * p -= lr mhat / (sqrt(vhat) + eps).  t is the 1-based step number. */
void oracle_adam(int64_t np, double* p, double* m, double* v, const double* g,
                 double lr, double b1, double b2, double eps, int64_t t) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < np; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* training losses and their gradients (embedding and interaction network)   */
/* ------------------------------------------------------------------------ */

/* Pairwise hinge embedding loss of thesis ch. 8 (eqs. loss1-loss3) over the
 * given pairs, with the embedding MLP of oracle_embed (FP64, unquantised):
 *   L = L_fake + w_gen L_gen,
 *   L_gen  = (1/|T_gen|)  sum over genuine pairs (q, a) of d^2(q, a),
 *   L_fake = (1/|T_fake|) sum over fake pairs (q, b) of max(0, m - d^2(q, b)).
 * grad (layout of params) receives dL/dparams by the chain rule through
 * every layer (thesis ch. 4 "Backpropagation").  Returns L. */
double oracle_embed_hinge_loss_grad(int64_t n, const double* cyl, int n_layers, const int* dims,
                                    const double* params, int64_t n_gen, const int32_t* gsrc, const int32_t* gdst,
                                    int64_t n_fake, const int32_t* fsrc, const int32_t* fdst, double margin,
                                    double w_gen, double* grad) {
  int64_t np = 0, tot = 0;
  for (int l = 0; l < n_layers; ++l) np += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
  for (int l = 0; l <= n_layers; ++l) tot += dims[l];
  const int D = dims[n_layers];
  memset(grad, 0, sizeof(double) * np);
  /* forward: the input of every layer and the output, per hit */
  double* act = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * tot);
  int64_t* aoff = (int64_t*)malloc(sizeof(int64_t) * (n_layers + 1));
  aoff[0] = 0;
  for (int l = 0; l < n_layers; ++l) aoff[l + 1] = aoff[l] + dims[l];
  for (int64_t i = 0; i < n; ++i) {
    double* a = act + i * tot;
    for (int k = 0; k < dims[0]; ++k) a[k] = cyl[3 * i + k];
    const double* p = params;
    for (int l = 0; l < n_layers; ++l) {
      const int K = dims[l], M = dims[l + 1];
      const double* in = a + aoff[l];
      double* out = a + aoff[l + 1];
      for (int m = 0; m < M; ++m) {
        double s = p[(int64_t)K * M + m];
        for (int k = 0; k < K; ++k) s += in[k] * p[(int64_t)k * M + m];
        out[m] = (l + 1 < n_layers && s < 0.0) ? 0.0 : s;
      }
      p += (int64_t)K * M + M;
    }
  }
  /* loss and dL/de per hit */
  double* de = (double*)calloc((size_t)(n > 0 ? n : 1) * D, sizeof(double));
  double lg = 0.0, lf = 0.0;
  for (int64_t t = 0; t < n_gen; ++t) {
    const double* eq = act + (int64_t)gsrc[t] * tot + aoff[n_layers];
    const double* ea = act + (int64_t)gdst[t] * tot + aoff[n_layers];
    double d2 = 0.0;
    for (int k = 0; k < D; ++k) d2 += (eq[k] - ea[k]) * (eq[k] - ea[k]);
    lg += d2;
    const double c = w_gen * 2.0 / (double)n_gen;
    for (int k = 0; k < D; ++k) {
      de[(int64_t)gsrc[t] * D + k] += c * (eq[k] - ea[k]);
      de[(int64_t)gdst[t] * D + k] -= c * (eq[k] - ea[k]);
    }
  }
  for (int64_t t = 0; t < n_fake; ++t) {
    const double* eq = act + (int64_t)fsrc[t] * tot + aoff[n_layers];
    const double* eb = act + (int64_t)fdst[t] * tot + aoff[n_layers];
    double d2 = 0.0;
    for (int k = 0; k < D; ++k) d2 += (eq[k] - eb[k]) * (eq[k] - eb[k]);
    if (margin - d2 > 0.0) {
      lf += margin - d2;
      const double c = -2.0 / (double)n_fake;
      for (int k = 0; k < D; ++k) {
        de[(int64_t)fsrc[t] * D + k] += c * (eq[k] - eb[k]);
        de[(int64_t)fdst[t] * D + k] -= c * (eq[k] - eb[k]);
      }
    }
  }
  const double loss = (n_fake > 0 ? lf / (double)n_fake : 0.0) + w_gen * (n_gen > 0 ? lg / (double)n_gen : 0.0);
  /* backward through the layers, hit by hit */
  int maxw = 0;
  for (int l = 0; l <= n_layers; ++l) maxw = dims[l] > maxw ? dims[l] : maxw;
  double* dcur = (double*)malloc(sizeof(double) * maxw);
  double* dprev = (double*)malloc(sizeof(double) * maxw);
  int64_t* poff = (int64_t*)malloc(sizeof(int64_t) * (n_layers + 1));
  poff[0] = 0;
  for (int l = 0; l < n_layers; ++l) poff[l + 1] = poff[l] + (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
  for (int64_t i = 0; i < n; ++i) {
    const double* a = act + i * tot;
    for (int k = 0; k < D; ++k) dcur[k] = de[i * D + k];
    for (int l = n_layers - 1; l >= 0; --l) {
      const int K = dims[l], M = dims[l + 1];
      const double* in = a + aoff[l];
      const double* W = params + poff[l];
      double* gW = grad + poff[l];
      double* gb = gW + (int64_t)K * M;
      for (int k = 0; k < K; ++k)
        for (int m = 0; m < M; ++m) gW[(int64_t)k * M + m] += in[k] * dcur[m];
      for (int m = 0; m < M; ++m) gb[m] += dcur[m];
      if (l > 0) {
        /* the input of layer l is ReLU(z) of layer l - 1: its derivative is 1 where the value is positive */
        for (int k = 0; k < K; ++k) {
          double s = 0.0;
          for (int m = 0; m < M; ++m) s += W[(int64_t)k * M + m] * dcur[m];
          dprev[k] = in[k] > 0.0 ? s : 0.0;
        }
        for (int k = 0; k < K; ++k) dcur[k] = dprev[k];
      }
    }
  }
  free(act); free(aoff); free(de); free(dcur); free(dprev); free(poff);
  return loss;
}

/* One Block(x) = ReLU(LN(x W + b)) over `rows` rows, saving what its
 * backward needs: the input rows, the normalised values (before the ReLU) and
 * the reciprocal standard deviations. */
typedef struct {
  int K, M;
  int64_t rows;
  const double* W;
  const double* b;
  double* x;      /* [rows][K] */
  double* yhat;   /* [rows][M] */
  double* rstd;   /* [rows] */
} blk_t;

static void blk_init(blk_t* B, int K, int M, int64_t rows, const double* W) {
  B->K = K; B->M = M; B->rows = rows; B->W = W; B->b = W + (int64_t)K * M;
  B->x = (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1) * K);
  B->yhat = (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1) * M);
  B->rstd = (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
}

static void blk_free(blk_t* B) { free(B->x); free(B->yhat); free(B->rstd); }

/* forward of row r: B->x[r] must hold the input; writes the ReLU output to y */
static void blk_fwd(blk_t* B, int64_t r, double* y) {
  const int K = B->K, M = B->M;
  const double* x = B->x + r * K;
  double* yh = B->yhat + r * M;
  for (int m = 0; m < M; ++m) {
    double s = B->b[m];
    for (int k = 0; k < K; ++k) s += x[k] * B->W[(int64_t)k * M + m];
    yh[m] = s;
  }
  double mean = 0.0, var = 0.0;
  for (int m = 0; m < M; ++m) mean += yh[m];
  mean /= M;
  for (int m = 0; m < M; ++m) var += (yh[m] - mean) * (yh[m] - mean);
  var /= M;
  const double rs = 1.0 / sqrt(var + 1e-5);
  B->rstd[r] = rs;
  for (int m = 0; m < M; ++m) {
    yh[m] = (yh[m] - mean) * rs;
    y[m] = yh[m] > 0.0 ? yh[m] : 0.0;
  }
}

/* backward of row r: dy (dL/d output) -> gW, gb accumulated, dx written */
static void blk_bwd(const blk_t* B, int64_t r, const double* dy, double* gW, double* dx) {
  const int K = B->K, M = B->M;
  const double* yh = B->yhat + r * M;
  const double rs = B->rstd[r];
  double g[256], dz[256];
  double mg = 0.0, mgy = 0.0;
  for (int m = 0; m < M; ++m) {
    g[m] = yh[m] > 0.0 ? dy[m] : 0.0;             /* through the ReLU */
    mg += g[m];
    mgy += g[m] * yh[m];
  }
  mg /= M;
  mgy /= M;
  /* LayerNorm: z -> (z - mean) rstd; dz = rstd (g - mean(g) - yhat mean(g yhat)) */
  for (int m = 0; m < M; ++m) dz[m] = rs * (g[m] - mg - yh[m] * mgy);
  const double* x = B->x + r * K;
  double* gb = gW + (int64_t)K * M;
  for (int k = 0; k < K; ++k)
    for (int m = 0; m < M; ++m) gW[(int64_t)k * M + m] += x[k] * dz[m];
  for (int m = 0; m < M; ++m) gb[m] += dz[m];
  if (dx)
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int m = 0; m < M; ++m) s += B->W[(int64_t)k * M + m] * dz[m];
      dx[k] = s;
    }
}

/* Sigmoid focal loss (Lin et al., cited for eq. gnn-loss in thesis ch. 8) of
 * one edge with logit z and label y: -alpha_t (1 - p_t)^gamma log p_t with
 * p = sigmoid(z), p_t = p for y = 1 and 1 - p for y = 0, alpha_t = alpha for
 * y = 1 and 1 - alpha for y = 0.  *dz receives its derivative in z. */
static double focal(double z, int y, double alpha, double gamma, double* dz) {
  const double p = 1.0 / (1.0 + exp(-z));
  /* log p = -softplus(-z), log(1 - p) = -softplus(z), evaluated stably */
  const double lp = -(z < 0 ? -z + log1p(exp(z)) : log1p(exp(-z)));
  const double l1p = -(z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)));
  if (y) {
    const double w = pow(1.0 - p, gamma);
    *dz = alpha * w * (gamma * p * lp - (1.0 - p));
    return -alpha * w * lp;
  }
  const double w = pow(p, gamma);
  *dz = (1.0 - alpha) * w * (p - gamma * (1.0 - p) * l1p);
  return -(1.0 - alpha) * w * l1p;
}

/* Mean sigmoid focal loss of the edge classifier (eq. gnn-loss without the
 * triplet term) over the E edges with labels y, through the interaction
 * network of oracle_gnn (FP64, unquantised), and its gradient with respect
 * to every network parameter (layout of params) by reverse-mode chain rule:
 * the classifier, then the message-passing steps from the last to the first
 * (the transpose of a gather by source or target is a sum over that node's
 * edges, and the transpose of the out-/in-sums a gather), then the encoders.
 * Returns the loss. */
static double gnn_loss_grad(int64_t n, const double* cart, int64_t E, const int32_t* src, const int32_t* dst, int H,
                            int S, const double* params, const uint8_t* label, int64_t T, const int32_t* ta,
                            const int32_t* tb, const uint8_t* kind, const uint8_t* tlabel, const double* tparams,
                            double alpha, double gamma, double* grad, double* tgrad);

double oracle_gnn_focal_loss_grad(int64_t n, const double* cart, int64_t E, const int32_t* src,
                                  const int32_t* dst, int H, int S, const double* params, const uint8_t* label,
                                  double alpha, double gamma, double* grad) {
  return gnn_loss_grad(n, cart, E, src, dst, H, S, params, label, 0, NULL, NULL, NULL, NULL, NULL, alpha, gamma,
                       grad, NULL);
}

/* The loss of eq. gnn-loss with its triplet term: the edge classifier's mean
 * focal loss plus, for each of the two triplet classifiers (articulations,
 * kind 0; elbows, kinds 1 and 2), the mean focal loss over its triplets
 * (ta[t], tb[t]) with labels tlabel; the classifier of a triplet reads
 * [e_S(ta), e_S(tb)] (the final edge encodings), so its gradient flows back
 * into the interaction network.  tparams: both classifiers, each W1[2H][H]
 * b1 W2[H][H] b2 w3[H] b3; tgrad: their gradient in that layout. */
double oracle_gnn_triplet_loss_grad(int64_t n, const double* cart, int64_t E, const int32_t* src,
                                    const int32_t* dst, int H, int S, const double* params, const uint8_t* label,
                                    int64_t T, const int32_t* ta, const int32_t* tb, const uint8_t* kind,
                                    const uint8_t* tlabel, const double* tparams, double alpha, double gamma,
                                    double* grad, double* tgrad) {
  return gnn_loss_grad(n, cart, E, src, dst, H, S, params, label, T, ta, tb, kind, tlabel, tparams, alpha, gamma,
                       grad, tgrad);
}

static double gnn_loss_grad(int64_t n, const double* cart, int64_t E, const int32_t* src, const int32_t* dst, int H,
                            int S, const double* params, const uint8_t* label, int64_t T, const int32_t* ta,
                            const int32_t* tb, const uint8_t* kind, const uint8_t* tlabel, const double* tparams,
                            double alpha, double gamma, double* grad, double* tgrad) {
  const int64_t HH = (int64_t)H * H;
  /* parameter offsets in the layout of oracle_gnn */
  const int64_t o_ne1 = 0, o_ne2 = o_ne1 + 3 * H + H, o_ee1 = o_ne2 + HH + H, o_ee2 = o_ee1 + 2 * HH + H;
  const int64_t o_step = o_ee2 + HH + H, step_sz = 2 * (3 * HH + H + HH + H);
  const int64_t o_cls = o_step + S * step_sz;
  const int64_t np = o_cls + HH + H + H + 1;
  memset(grad, 0, sizeof(double) * np);
  blk_t ne1, ne2, ee1, ee2, cb;
  blk_t* nn1 = (blk_t*)malloc(sizeof(blk_t) * (S > 0 ? S : 1));
  blk_t* nn2 = (blk_t*)malloc(sizeof(blk_t) * (S > 0 ? S : 1));
  blk_t* en1 = (blk_t*)malloc(sizeof(blk_t) * (S > 0 ? S : 1));
  blk_t* en2 = (blk_t*)malloc(sizeof(blk_t) * (S > 0 ? S : 1));
  blk_init(&ne1, 3, H, n, params + o_ne1);
  blk_init(&ne2, H, H, n, params + o_ne2);
  blk_init(&ee1, 2 * H, H, E, params + o_ee1);
  blk_init(&ee2, H, H, E, params + o_ee2);
  for (int k = 0; k < S; ++k) {
    const int64_t o = o_step + k * step_sz;
    blk_init(&nn1[k], 3 * H, H, n, params + o);
    blk_init(&nn2[k], H, H, n, params + o + 3 * HH + H);
    blk_init(&en1[k], 3 * H, H, E, params + o + 4 * HH + 2 * H);
    blk_init(&en2[k], H, H, E, params + o + 7 * HH + 3 * H);
  }
  blk_init(&cb, H, H, E, params + o_cls);
  const double* w2 = params + o_cls + HH + H;
  const double b2 = w2[H];
  /* node and edge state per step: h[k] (k = 0..S), e[k] (k = 0..S) */
  double* h = (double*)calloc((size_t)(S + 1) * (n > 0 ? n : 1) * H, sizeof(double));
  double* e = (double*)calloc((size_t)(S + 1) * (E > 0 ? E : 1) * H, sizeof(double));
  double* mo = (double*)calloc((size_t)(n > 0 ? n : 1) * H, sizeof(double));
  double* mi = (double*)calloc((size_t)(n > 0 ? n : 1) * H, sizeof(double));
  double* c = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1) * H);
  double* tmp = (double*)malloc(sizeof(double) * 3 * H);
#define HK(k, l) (h + ((int64_t)(k) * n + (l)) * H)
#define EK(k, t) (e + ((int64_t)(k) * E + (t)) * H)
  /* forward */
  for (int64_t l = 0; l < n; ++l) {
    memcpy(ne1.x + l * 3, cart + 3 * l, sizeof(double) * 3);
    blk_fwd(&ne1, l, ne2.x + l * H);
    blk_fwd(&ne2, l, HK(0, l));
  }
  for (int64_t t = 0; t < E; ++t) {
    memcpy(ee1.x + t * 2 * H, HK(0, src[t]), sizeof(double) * H);
    memcpy(ee1.x + t * 2 * H + H, HK(0, dst[t]), sizeof(double) * H);
    blk_fwd(&ee1, t, ee2.x + t * H);
    blk_fwd(&ee2, t, EK(0, t));
  }
  for (int k = 0; k < S; ++k) {
    memset(mo, 0, sizeof(double) * n * H);
    memset(mi, 0, sizeof(double) * n * H);
    for (int64_t t = 0; t < E; ++t)
      for (int q = 0; q < H; ++q) {
        mo[(int64_t)src[t] * H + q] += EK(k, t)[q];
        mi[(int64_t)dst[t] * H + q] += EK(k, t)[q];
      }
    for (int64_t l = 0; l < n; ++l) {
      double* x = nn1[k].x + l * 3 * H;
      memcpy(x, HK(k, l), sizeof(double) * H);
      memcpy(x + H, mo + l * H, sizeof(double) * H);
      memcpy(x + 2 * H, mi + l * H, sizeof(double) * H);
      blk_fwd(&nn1[k], l, nn2[k].x + l * H);
      blk_fwd(&nn2[k], l, tmp);
      for (int q = 0; q < H; ++q) HK(k + 1, l)[q] = HK(k, l)[q] + tmp[q];
    }
    for (int64_t t = 0; t < E; ++t) {
      double* x = en1[k].x + t * 3 * H;
      memcpy(x, EK(k, t), sizeof(double) * H);
      memcpy(x + H, HK(k + 1, src[t]), sizeof(double) * H);
      memcpy(x + 2 * H, HK(k + 1, dst[t]), sizeof(double) * H);
      blk_fwd(&en1[k], t, en2[k].x + t * H);
      blk_fwd(&en2[k], t, tmp);
      for (int q = 0; q < H; ++q) EK(k + 1, t)[q] = EK(k, t)[q] + tmp[q];
    }
  }
  double loss = 0.0;
  double* dlog = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
  for (int64_t t = 0; t < E; ++t) {
    memcpy(cb.x + t * H, EK(S, t), sizeof(double) * H);
    blk_fwd(&cb, t, c + t * H);
    double z = b2;
    for (int q = 0; q < H; ++q) z += c[t * H + q] * w2[q];
    double dz;
    loss += focal(z, label[t] != 0, alpha, gamma, &dz);
    dlog[t] = dz / (double)E;
  }
  loss = E > 0 ? loss / (double)E : 0.0;
  /* backward */
  double* de = (double*)calloc((size_t)(E > 0 ? E : 1) * H, sizeof(double));
  double* dh = (double*)calloc((size_t)(n > 0 ? n : 1) * H, sizeof(double));
  double* dx = (double*)malloc(sizeof(double) * 3 * H);
  double* dy = (double*)malloc(sizeof(double) * H);
  double* gw2 = grad + o_cls + HH + H;
  for (int64_t t = 0; t < E; ++t) {
    for (int q = 0; q < H; ++q) {
      gw2[q] += c[t * H + q] * dlog[t];
      dy[q] = w2[q] * dlog[t];
    }
    gw2[H] += dlog[t];
    blk_bwd(&cb, t, dy, grad + o_cls, de + t * H);
  }
  /* triplet classifiers on [e_S(ta), e_S(tb)]: forward, focal loss, backward into de */
  if (tparams) {
    const int64_t hs = 3 * HH + 3 * H + 1;
    memset(tgrad, 0, sizeof(double) * 2 * hs);
    int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
    double* y2 = (double*)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * H);
    double* dl = (double*)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
    double* dy1 = (double*)malloc(sizeof(double) * H);
    double* dx2 = (double*)malloc(sizeof(double) * 2 * H);
    for (int head = 0; head < 2; ++head) {
      int64_t nh = 0;
      for (int64_t t = 0; t < T; ++t)
        if ((kind[t] == 0) == (head == 0)) rows[nh++] = t;
      if (nh == 0) continue;
      const double* hp = tparams + head * hs;
      double* hg = tgrad + head * hs;
      const double* w3 = hp + 3 * HH + 2 * H;
      double* gw3 = hg + 3 * HH + 2 * H;
      blk_t b1, b2;
      blk_init(&b1, 2 * H, H, nh, hp);
      blk_init(&b2, H, H, nh, hp + 2 * HH + H);
      double lh = 0.0;
      for (int64_t r = 0; r < nh; ++r) {
        const int64_t t = rows[r];
        memcpy(b1.x + r * 2 * H, EK(S, ta[t]), sizeof(double) * H);
        memcpy(b1.x + r * 2 * H + H, EK(S, tb[t]), sizeof(double) * H);
        blk_fwd(&b1, r, b2.x + r * H);
        blk_fwd(&b2, r, y2 + r * H);
        double z = w3[H];
        for (int q = 0; q < H; ++q) z += y2[r * H + q] * w3[q];
        double dz;
        lh += focal(z, tlabel[t] != 0, alpha, gamma, &dz);
        dl[r] = dz / (double)nh;
      }
      loss += lh / (double)nh;
      for (int64_t r = 0; r < nh; ++r) {
        const int64_t t = rows[r];
        for (int q = 0; q < H; ++q) {
          gw3[q] += y2[r * H + q] * dl[r];
          dy[q] = w3[q] * dl[r];
        }
        gw3[H] += dl[r];
        blk_bwd(&b2, r, dy, hg + 2 * HH + H, dy1);
        blk_bwd(&b1, r, dy1, hg, dx2);
        for (int q = 0; q < H; ++q) {
          de[(int64_t)ta[t] * H + q] += dx2[q];
          de[(int64_t)tb[t] * H + q] += dx2[H + q];
        }
      }
      blk_free(&b1); blk_free(&b2);
    }
    free(rows); free(y2); free(dl); free(dy1); free(dx2);
  }
  double* dmo = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * H);
  double* dmi = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * H);
  for (int k = S - 1; k >= 0; --k) {
    const int64_t o = o_step + k * step_sz;
    /* edge update k: e_{k+1} = e_k + Block2(Block1([e_k, h_{k+1}[src], h_{k+1}[dst]])) */
    for (int64_t t = 0; t < E; ++t) {
      blk_bwd(&en2[k], t, de + t * H, grad + o + 7 * HH + 3 * H, dy);
      blk_bwd(&en1[k], t, dy, grad + o + 4 * HH + 2 * H, dx);
      for (int q = 0; q < H; ++q) {
        de[t * H + q] += dx[q];                      /* residual: de_k = de_{k+1} + the e block of dx */
        dh[(int64_t)src[t] * H + q] += dx[H + q];
        dh[(int64_t)dst[t] * H + q] += dx[2 * H + q];
      }
    }
    /* node update k: h_{k+1} = h_k + Block2(Block1([h_k, mo_k, mi_k])) */
    for (int64_t l = 0; l < n; ++l) {
      blk_bwd(&nn2[k], l, dh + l * H, grad + o + 3 * HH + H, dy);
      blk_bwd(&nn1[k], l, dy, grad + o, dx);
      for (int q = 0; q < H; ++q) {
        dh[l * H + q] += dx[q];
        dmo[l * H + q] = dx[H + q];
        dmi[l * H + q] = dx[2 * H + q];
      }
    }
    /* the out-sum of a node is the sum of its outgoing edges' e_k, the in-sum of its incoming ones */
    for (int64_t t = 0; t < E; ++t)
      for (int q = 0; q < H; ++q) de[t * H + q] += dmo[(int64_t)src[t] * H + q] + dmi[(int64_t)dst[t] * H + q];
  }
  /* edge encoder: e_0 = Block2(Block1([h_0[src], h_0[dst]])) */
  for (int64_t t = 0; t < E; ++t) {
    blk_bwd(&ee2, t, de + t * H, grad + o_ee2, dy);
    blk_bwd(&ee1, t, dy, grad + o_ee1, dx);
    for (int q = 0; q < H; ++q) {
      dh[(int64_t)src[t] * H + q] += dx[q];
      dh[(int64_t)dst[t] * H + q] += dx[H + q];
    }
  }
  /* node encoder: h_0 = Block2(Block1(x / R, y / R, z / Z)) */
  for (int64_t l = 0; l < n; ++l) {
    blk_bwd(&ne2, l, dh + l * H, grad + o_ne2, dy);
    blk_bwd(&ne1, l, dy, grad + o_ne1, NULL);
  }
#undef HK
#undef EK
  blk_free(&ne1); blk_free(&ne2); blk_free(&ee1); blk_free(&ee2); blk_free(&cb);
  for (int k = 0; k < S; ++k) {
    blk_free(&nn1[k]); blk_free(&nn2[k]); blk_free(&en1[k]); blk_free(&en2[k]);
  }
  free(nn1); free(nn2); free(en1); free(en2);
  free(h); free(e); free(mo); free(mi); free(c); free(tmp); free(dlog); free(de); free(dh); free(dx); free(dy);
  free(dmo); free(dmi);
  return loss;
}
