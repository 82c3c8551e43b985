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
 * f32: FP32 evaluation (see RF). */
void oracle_gnn(int64_t n, const double* cart, int64_t E, const int32_t* src, const int32_t* dst,
                int H, int S, const double* params, double* logit, int qmode, const double* act_scale,
                double* amax, int compact, int f32) {
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
