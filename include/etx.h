/*
 * etx.h -- C ABI of the MI355X GNN track-finding hot path.
 *
 * The problem (thesis ch. 7 "Track reconstruction" and ch. 8 "The ETX4VELO
 * Pipeline"): the input is the point cloud of each event's detector hits, the
 * output is a grouping of the hits into tracks, together with the edge scores
 * behind it.  One call runs, for a packed batch of independent events:
 *
 *   embedding MLP on normalised (r, phi, z)           ch. 8 "Hit Embedding ..."
 *   fixed-radius graph: hit on plane p -> hits on planes p+1..p+window with
 *     squared embedding distance below radius^2, at most k_max per source
 *     (the k_max nearest, ties broken by the smaller hit index)
 *                                                     ch. 8 (d^2 equation), ch. 9 "k-NN Implementation"
 *   interaction network: node and edge encoders, `gnn_steps` message-passing
 *     steps with concatenated out/in sums and residual node then edge updates,
 *     edge classifier with a sigmoid score           ch. 8 "Graph Neural Network and Classifiers"
 *   score cut: an edge is kept when score >= edge_threshold
 *   connected components of the kept graph; the label of a hit is the
 *     smallest global hit index in its component     ch. 9 "WCC Implementation"
 *
 * etx_run_tracks adds the triplet stage of the full method (triplets of the
 * kept graph, triplet classifiers, tracks that may share hits; ch. 8
 * "Triplet Building" and "Track Building"), documented at its declaration.
 *
 * Conventions
 *  - Every entry point returns an etx_status; nothing throws across the ABI.
 *  - "device" pointers are HIP device memory on the context's device; the
 *    caller owns every input, output and workspace buffer.  The context owns
 *    its device copy of the weights, scales and cached HIP graphs.
 *  - etx_stream is a hipStream_t (NULL = the default stream).  Calls that take
 *    a stream are asynchronous: they only enqueue work and never synchronise.
 *    Errors found on the device (bad input, edge capacity) are written to
 *    out->status, which the caller reads after synchronising the stream.
 *  - Hit indices are global indices into the packed batch (int32); offsets
 *    are int64.  Hits may come in any order within an event.
 */
#ifndef ETX_H
#define ETX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ETX_OK = 0,
  ETX_ERR_INVALID_ARG = 1,   /* bad pointer, size or configuration value */
  ETX_ERR_CAPACITY = 2,      /* device: more edges than out->edge_capacity; status[1] = edges needed */
  ETX_ERR_INPUT = 3,         /* device: NaN/inf coordinate, plane outside [0, n_planes), bad hit_off */
  ETX_ERR_WEIGHTS = 4,       /* weight blob does not match the configuration */
  ETX_ERR_UNSUPPORTED = 5,   /* a size the library does not handle (e.g. an event above ETX_MAX_EVENT_HITS) */
  ETX_ERR_HIP = 6            /* a HIP runtime call failed */
} etx_status;

typedef enum { ETX_FP32 = 0, ETX_BF16 = 1, ETX_FP8_E4M3 = 2, ETX_INT8 = 3 } etx_precision;

/* Largest event (hits) the per-event kernels accept. */
#define ETX_MAX_EVENT_HITS 16384
/* Largest number of planes. */
#define ETX_MAX_PLANES 64

typedef void* etx_stream; /* hipStream_t */

typedef struct {
  int32_t n_planes;          /* planes are numbered 0..n_planes-1 along the beam */
  float r_scale_mm;          /* R_s: r, x, y are divided by it */
  float z_scale_mm;          /* Z_s: z is divided by it */
  int32_t emb_hidden;        /* embedding hidden width: 32, 64 or 128 */
  int32_t emb_layers;        /* hidden layers of the embedding MLP: 1..4 */
  int32_t emb_dim;           /* embedding dimension: 1..16 */
  float radius;              /* edge if squared distance < radius^2 */
  int32_t k_max;             /* 1..64 neighbours per source hit */
  int32_t plane_window;      /* 1..4: targets on planes p+1..p+plane_window */
  int32_t gnn_hidden;        /* node and edge encoding width: 32 or 64 */
  int32_t gnn_steps;         /* message-passing steps: 1..16 */
  float edge_threshold;      /* keep edge when score >= threshold (0.5) */
  int32_t precision;         /* etx_precision of the MLP GEMM operands; node and edge encodings stay FP32
                                between kernels unless ETX_OPT_COMPACT_STATE is set */
  int32_t prefilter;         /* 1: prune candidate edges with the learned prefilter before the GNN */
  float prefilter_tau;       /* prune when prefilter probability < tau */
} etx_config;

typedef struct etx_ctx etx_ctx;

typedef struct {             /* device pointers, caller-owned, read-only */
  int64_t n_events;
  int64_t n_hits;            /* == hit_off[n_events] (host copy of the total) */
  const int64_t* hit_off;    /* [n_events+1] event e owns hits hit_off[e] .. hit_off[e+1]-1 */
  const float* x;            /* [n_hits] mm */
  const float* y;            /* [n_hits] mm */
  const float* z;            /* [n_hits] mm */
  const int32_t* plane;      /* [n_hits] plane index */
} etx_hits;

typedef struct {             /* device pointers, caller-owned, written by etx_run */
  int64_t edge_capacity;     /* length of src, dst, score */
  int32_t* src;              /* [edge_capacity] global hit index; sorted by (src, dst) within each event */
  int32_t* dst;              /* [edge_capacity] global hit index on a later plane */
  float* score;              /* [edge_capacity] classifier score in (0, 1) */
  int64_t* edge_off;         /* [n_events+1] event e owns edges edge_off[e] .. edge_off[e+1]-1 */
  int32_t* labels;           /* [n_hits] smallest global hit index of the hit's component */
  int64_t* status;           /* [2] status[0] = etx_status of the device work, status[1] = edges needed */
} etx_out;

/* Create a context on `device`.  `weights` is a host blob (see etx_weight_blob_size):
 * int32 header {0x57585445, 1, 3, emb_hidden, emb_layers, emb_dim, gnn_hidden, gnn_steps}
 * followed by float32 Linear layers (W row-major [fan_in][fan_out], then b) in the
 * order: embedding layers; node encoder (3->H, H->H); edge encoder (2H->H, H->H);
 * per step k: node net k (3H->H, H->H) then edge net k (3H->H, H->H); classifier
 * (H->H, H->1).  Node-net input is [h, out-sum, in-sum]; edge-net input is
 * [e, h_src, h_dst]; edge-encoder input is [h_src, h_dst].  The blob is copied. */
etx_status etx_create(const etx_config* cfg, const void* weights, size_t nbytes, int device, etx_ctx** out);
etx_status etx_destroy(etx_ctx* ctx);

/* Bytes a weight blob for `cfg` must have. */
etx_status etx_weight_blob_size(const etx_config* cfg, size_t* nbytes);

/* Workspace bytes etx_run needs for a batch of this size. */
etx_status etx_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                              size_t* bytes);

/* Run the whole hot path on one batch (see the top of this file).  `ws` is
 * device memory of at least etx_workspace_size bytes, 256-byte aligned. */
etx_status etx_run(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes, etx_stream stream);

/* etx_run without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same stages and kernels as etx_run, with the library's
 * static device scratch of ETX_SCRATCH_BYTES as the workspace.  The caller
 * still owns `hits` and `out`.  A batch whose workspace (etx_workspace_size)
 * exceeds ETX_SCRATCH_BYTES is rejected with ETX_ERR_UNSUPPORTED before
 * anything is enqueued.  Each device holds one scratch array for the life of
 * the process, shared by every call on that device: calls that overlap on one
 * device (other streams, other threads, other contexts) race and must be
 * ordered by the caller.  The scratch keeps the last call's contents; no stage
 * relies on it starting zeroed.  Runs eagerly on `stream` (ETX_OPT_USE_GRAPH,
 * stage timing and the tuning table are not applied: the options in effect
 * are used), allocates nothing and never synchronises. */
#define ETX_SCRATCH_BYTES (128u << 20)
etx_status etx_run_noalloc(etx_ctx* ctx, const etx_hits* hits, etx_out* out, etx_stream stream);

/* Internal buffers of the workspace, for inspection after etx_run. */
typedef enum {
  ETX_VIEW_EMBEDDING = 0,    /* float [n_hits][16]: embedding, zero-padded to 16 */
  ETX_VIEW_BUCKET = 1,       /* int32 [n_hits]: hits of each event ordered by plane (global indices) */
  ETX_VIEW_PLANE_OFF = 2,    /* int32 [n_events][n_planes+1]: per-event plane offsets into the bucket */
  ETX_VIEW_ROW_PTR = 3,      /* int64 [n_hits+1]: CSR by source hit (global edge positions) */
  ETX_VIEW_COL_PTR = 4,      /* int64 [n_hits+1]: CSC by target hit */
  ETX_VIEW_CSC_EDGE = 5,     /* int32 [edge_capacity]: edge ids sorted by (dst, src) */
  ETX_VIEW_NODE_H = 6,       /* [n_hits][H] node encodings after the last step: float, or BF16 bits (uint16)
                                in BF16 and FP8 runs with ETX_OPT_COMPACT_STATE set */
  ETX_VIEW_KEPT_EDGE = 7,    /* int32 [edge_capacity]: kept edge ids, per event from edge_off[e] */
  ETX_VIEW_KEPT_COUNT = 8,   /* int32 [n_events]: kept edges per event */
  ETX_VIEW_CALIB = 9,        /* float [ETX_N_CALIB]: per-tensor amax (calibration observers) */
  ETX_VIEW_PF_KEEP = 10,     /* uint8 [edge_capacity]: prefilter decision per candidate edge */
  ETX_VIEW_PF_GRAD = 11,     /* float [ETX_PF_NPARAM + 1]: last prefilter gradient, then the loss */
  ETX_VIEW_PF_PROB = 12,     /* float [edge_capacity]: prefilter probability per candidate edge */
  ETX_VIEW_PF_FEAT = 13,     /* float [edge_capacity][8]: the six prefilter features of every candidate edge (then two
                                zeros), written only with ETX_OPT_PF_FEATURES set (otherwise ETX_ERR_INVALID_ARG) */
  ETX_VIEW_PF_FALLBACK = 14  /* int32 [n_events]: 1 where the event fell back to the unpruned graph (its kept fraction
                                left the prefilter band), else 0; written by prefiltered runs */
} etx_view;
#define ETX_N_CALIB 64
etx_status etx_workspace_view(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                              int32_t which, size_t* offset, size_t* bytes);

/* Tuning knobs (also set by etx_autotune). */
typedef enum {
  ETX_OPT_USE_GRAPH = 0,     /* 1: etx_run captures the batch into a HIP graph and replays it */
  ETX_OPT_EDGE_WG_PER_CU = 1,/* persistent workgroups per CU of the edge kernels (1..8) */
  ETX_OPT_NODE_WG_PER_CU = 2,/* persistent workgroups per CU of the node kernels (1..8) */
  ETX_OPT_RADIUS_LDS = 3,    /* 1: stage and sort candidate windows in LDS when they fit; 0: always read HBM */
  ETX_OPT_SEGSUM_UNROLL = 4, /* edge rows in flight per wave in the segmented sums: 1, 2, 4 or 8 */
  ETX_OPT_PROFILE = 5,       /* 1: time every stage of eager runs with HIP events on the run's stream */
  ETX_OPT_EDGE_PIPELINE = 6, /* software pipeline of the per-edge kernels: 0 none, 1 prefetch the next
                                tile's indices and edge rows, 2 also its node-product gathers */
  ETX_OPT_EDGE_WG_SIZE = 7,  /* threads per workgroup of the per-edge kernels: 256 or 512 */
  ETX_OPT_EDGE_WREG = 8,     /* 1: FP32 edge-update kernels keep their weights in registers (0: read LDS) */
  ETX_OPT_EMBED_PRECISION = 9, /* GEMM operand precision of the embedding MLP (etx_precision), or -1 (default):
                                  the same as the configuration's precision */
  ETX_OPT_OUTSUM_LDS = 10,    /* 1 (default): hidden size 64 reduces the out-sums through an LDS transpose; 0: DPP scan
                                 (the two forms add in different orders: results agree to FP32 rounding, not bitwise) */
  ETX_OPT_F32_SPLIT = 11,     /* 1: in FP32 runs the edge kernels compute their GEMMs on the BF16 matrix cores with
                                 every FP32 operand split exactly into three BF16 parts (six partial products,
                                 FP32 accumulation; error at FP32 rounding level); 0: FP32 matrix cores */
  ETX_OPT_RADIUS_SINGLE_PASS = 12, /* 1 (default): the radius search selects each source's neighbours once into
                                      k_max workspace slots per hit and the CSR rows are copied after the scan;
                                      0: a count pass and an emit pass */
  ETX_OPT_RADIUS_SORT_MIN = 13, /* staged candidate windows with at least this many hits are binned along their
                                   widest axis into cells about r wide and searched as a cell list; smaller ones
                                   are scanned whole (default 512; 0: always bin) */
  ETX_OPT_FUSE_MESSAGES = 14,  /* 1: the node-update kernel gathers its messages itself (no separate message-sum
                                  kernel, no message buffer round trip); same sums, same order, same bits */
  ETX_OPT_RADIUS_FAST = 15,    /* 1: in staged windows, sources with at most 16 in-radius candidates are handled four
                                  to a wave; the others by the one-wave-per-source path; same bits */
  ETX_OPT_XCD_MAP = 16,        /* 1: the edge, message-sum and node kernels give each of the chip's eight XCDs a
                                  contiguous range of tiles, so that the node rows a region of the batch gathers stay
                                  in that XCD's L2; which tiles run is unchanged, same bits */
  ETX_OPT_EDGE_PRODUCTS = 17,  /* 0 (default): the node encoder and the node update also write h W_src and h W_dst per
                                  node (layer 1 of the edge encoder / edge net split by input block) and the edge
                                  kernels gather them; 1: the edge kernels gather the rows of h and form the same
                                  products themselves, and the node kernels write none (less HBM traffic, 2H^2 more
                                  multiply-adds per edge; same bits) */
  ETX_OPT_CSC_PLACE = 18,      /* 1 (default): for events with short rows (< 16 edges per hit) the whole block drops
                                  the edges into their CSC columns through LDS cursors and then sorts every column by
                                  edge index (source order); 0: one wave ranks 64 edges at a time; same permutation */
  ETX_OPT_COMPACT_STATE = 19,  /* BF16 and FP8 runs only (FP32 and INT8 runs ignore it).  0 (default): the node encodings h and edge encodings e
                                  are kept in FP32 between kernels (residual master copies) and quantised only where
                                  they enter a GEMM.  1: both are stored in low precision (h as BF16; e in the
                                  operand format, FP8 with the e_k scale), which halves or quarters their HBM
                                  traffic; the residual sums are then rounded at every step (different results) */
  ETX_OPT_PROFILE_STAGES = 20, /* bit mask of the stages (etx_stage_name indices) that ETX_OPT_PROFILE times; default
                                  every stage.  Timing one kernel alone leaves the rest of a pass uninstrumented */
  ETX_OPT_PF_FEATURES = 21,    /* 1: the prefilter's inference pass also stores the features of every candidate edge
                                  (ETX_VIEW_PF_FEAT; the workspace grows by 32 bytes per edge of capacity: set it
                                  before sizing the workspace); 0 (default): features are formed in registers only */
  ETX_OPT_RADIUS_SPLIT = 22    /* 1: the radius search runs as two launches over the (event, plane) units: candidate
                                  windows of up to 512 hits (256 above embedding width 8) in workgroups with half the
                                  staging LDS (three to a CU at embedding width up to 8), the larger ones as before;
                                  each launch skips the other's units; the same bits (needs ETX_OPT_RADIUS_LDS = 1).
                                  0 (default): one launch */
} etx_option;
etx_status etx_set_option(etx_ctx* ctx, int32_t key, int64_t value);
etx_status etx_get_option(const etx_ctx* ctx, int32_t key, int64_t* value);

/* Stage timing: with ETX_OPT_PROFILE set, every eager etx_run records a pair of
 * HIP events around each stage on its stream.  etx_profile_read waits for the
 * recorded events, adds their durations to running totals per stage (indices
 * 0..n_stages-1, names from etx_stage_name) and returns the totals and launch
 * counts; etx_profile_reset clears them. */
etx_status etx_profile_read(etx_ctx* ctx, int32_t n_stages, double* total_ms, int64_t* launches);
etx_status etx_profile_reset(etx_ctx* ctx);
const char* etx_stage_name(int32_t stage);   /* "" for an unknown stage */

/* Try each candidate launch schedule on this batch (one knob at a time, each
 * judged by the HIP-event time of the stages it drives; no knob changes a
 * result bit), keep the fastest, and record it in the context's tuning table
 * under the batch's key: the configuration and run modes (precision, embedding
 * precision, compact state, prefilter) plus the shape bucket (hits per event
 * and events per batch, each rounded to the nearest power of two).  Appends the
 * trials to `json_path` (JSON lines; may be NULL).  Synchronises the stream.
 * The device status of the first trial is read back: an error there (edge
 * capacity, bad input) is returned, and the options in effect before the call
 * are restored, as after any failure. */
etx_status etx_autotune(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes,
                        etx_stream stream, const char* json_path);
/* Tuning table.  etx_run applies the entry of its batch's key when the table
 * has one (the options stay until a batch of another key with an entry comes,
 * or etx_set_option changes them).  etx_tuning_save merges the context's
 * entries into the text file at `path` (entries of other architectures,
 * configurations or buckets are kept); etx_tuning_load adds the file's entries
 * for this device's architecture (ETX_ERR_INVALID_ARG if it cannot be read).
 * etx_create loads the file named by the environment variable
 * ETX_TUNING_TABLE, if set and readable. */
etx_status etx_tuning_save(const etx_ctx* ctx, const char* path);
etx_status etx_tuning_load(etx_ctx* ctx, const char* path);

/* Static calibration for the low-precision modes (thesis ch. 4 "Quantization",
 * static post-training quantisation): runs the FP32 path on `hits`, records
 * the per-tensor absolute maximum of every quantised activation, and sets the
 * per-tensor scales of both 8-bit formats: FP8-E4M3 the power of two at or
 * above amax / 448, INT8 S = amax / 127 (symmetric, thesis ch. 4
 * "Quantization").  Synchronises the stream.  Needed before FP8 or INT8 runs. */
etx_status etx_calibrate(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes,
                         etx_stream stream);
/* Switch the GEMM operand precision (etx_precision) of an existing context
 * (every weight format is built at etx_create). */
etx_status etx_set_precision(etx_ctx* ctx, int32_t precision);
/* Copy the first n (<= 512) per-tensor scales: activation slots 0..63 (0..7
 * embedding layer inputs; 8 + {0 node-encoder layer-2 input, 1 node
 * encodings, 2 out-sums, 3 in-sums, 4 edge-encoder layer-2 input, 5 node-net
 * layer-2 inputs, 6 edge-net layer-2 inputs, 7 + k stored edge encodings e_k}),
 * weight slots 64..255: the FP8 scales, each a power of two >= amax / 448;
 * slots 256 + i: the INT8 scales of the same tensors, amax / 127. */
etx_status etx_get_scales(const etx_ctx* ctx, float* scales, int32_t n);
/* Round n device floats through the library's operand format: out = in
 * rounded to BF16 (nearest even), scale * E4M3(in / scale) (nearest even,
 * saturating at +-448), or scale * clip(round(in * (1 / scale)), -127, 127)
 * (INT8, nearest even; the product with the FP32 reciprocal is what the GEMMs
 * quantise); FP32 copies.  Asynchronous on `stream`. */
etx_status etx_quantize(int32_t precision, const float* in, float* out, int64_t n, float scale, etx_stream stream);

/* Learned edge prefilter: MLP 6 -> 32 -> 32 -> 1 (ReLU) on the candidate-edge
 * features (dx, dy, dz, dr, dphi, embedding distance), normalised by
 * (R_s, R_s, Z_s, R_s, pi, 1), dphi wrapped to (-pi, pi].  Parameters are
 * float32 W1[6][32] b1[32] W2[32][32] b2[32] W3[32][1] b3[1] (1281 floats). */
#define ETX_PF_HIDDEN 32
#define ETX_PF_NPARAM (6 * 32 + 32 + 32 * 32 + 32 + 32 + 1)
etx_status etx_prefilter_set(etx_ctx* ctx, const float* params, int64_t n);            /* host params */
etx_status etx_prefilter_get(const etx_ctx* ctx, float* params, int64_t n);            /* host params */
/* One training step on the candidate edges of `hits` (the radius graph is built
 * first): BF16 forward/backward kernels, mean class-weighted BCE loss with
 * positive weight `pos_weight`, FP32 Adam (beta1 0.9, beta2 0.999, eps 1e-8)
 * with learning rate `lr`, step number `step` (1-based).  edge_labels[e] is 1
 * when candidate edge e (in the radius-graph order of out->src/out->dst) is kept
 * by the full pipeline.  *loss_dev (device float) receives the loss. */
etx_status etx_prefilter_train_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const uint8_t* edge_labels,
                                    float lr, float pos_weight, int64_t step, float* loss_dev, void* ws,
                                    size_t ws_bytes, etx_stream stream);
/* Turn the prefilter on or off and set its threshold (keep when p >= tau). */
etx_status etx_prefilter_config(etx_ctx* ctx, int32_t enabled, float tau);
/* Fallback band: an event whose fraction of kept candidate edges lies outside
 * [lo, hi] (0 <= lo <= hi <= 1) is run unpruned: every candidate of the event
 * is kept, so its edges, scores and labels are those of the pipeline without
 * the prefilter.  The band is the range validated with tau (the prefilter's
 * efficiency loss was measured there); outside it the pruning is not trusted.
 * Default [0, 1]: no fallback.  Which events fell back: ETX_VIEW_PF_FALLBACK. */
etx_status etx_prefilter_band(etx_ctx* ctx, float lo, float hi);
/* Optimiser state for checkpointing: params, Adam m, Adam v (3 * ETX_PF_NPARAM floats). */
etx_status etx_prefilter_state(etx_ctx* ctx, float* host_state, int64_t n, int32_t set);

/* In-library training of the embedding MLP and the interaction network
 * (thesis ch. 8 "Hit Embedding and Rough Graph Construction", eqs. loss1-loss3,
 * and "Graph Neural Network and Classifiers", eq. gnn-loss without the triplet
 * term).  The context keeps FP32 master copies of every parameter of the
 * weight blob with their Adam moments (beta1 0.9, beta2 0.999, eps 1e-8);
 * forward and backward run in FP32 on the device, the weight gradients are
 * summed over rows in a fixed order (reproducible to the bit).
 *
 * Generator truth of a batch, device pointers, caller-owned: */
typedef struct {
  const int32_t* particle;   /* [n_hits] particle of each hit, -1 for noise */
  const int32_t* succ;       /* [n_hits] the next hit of the same particle along the beam (global index), -1: none */
  const int32_t* pred;       /* [n_hits] the previous hit, -1: none (pred[succ[i]] == i) */
  const uint8_t* query;      /* [n_hits] 1: the hit's particle has hits on at least three planes (a training query) */
  const int32_t* rnd;        /* [n_hits] one random hit of a particle on the next two planes per query, -1: none */
  const int64_t* rnd_ptr;    /* [n_hits + 1] the random pairs grouped by their second hit: */
  const int32_t* rnd_src;    /*   rnd_src[rnd_ptr[b] .. rnd_ptr[b+1]-1] are the queries q with rnd[q] == b, ascending */
  const int32_t* particle2;  /* [n_hits] or NULL: the second particle of a hit that two particles share, -1: none */
  const int32_t* succ2;      /* [n_hits] or NULL: the next hit of that second particle, -1: none */
} etx_truth;
/* Copy the context's current weights into the training parameters and clear the moments (allocates them once). */
etx_status etx_train_begin(etx_ctx* ctx);
/* Host copy of the training state (set = 0) or its replacement (set = 1): the first n floats of
 * [params (blob payload order), Adam m, Adam v], n <= 3 x the payload's float count. */
etx_status etx_train_params(etx_ctx* ctx, float* host, int64_t n, int32_t set);
/* Rebuild the context's inference weights from the training parameters (every precision's segments and the
 * weight scales; FP8 / INT8 activation scales must be calibrated again). */
etx_status etx_train_apply(etx_ctx* ctx);
/* Workspace bytes of a training step (the etx_run workspace plus the saved activations and gradients). */
etx_status etx_train_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                                    size_t* bytes);
/* Training buffers of the workspace: 0 = float gradient in blob payload order, 1 = float[4] loss (slot 0),
 * 2 = uint8 [edge_capacity] edge labels of the last network step. */
etx_status etx_train_view(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity, int32_t which,
                          size_t* offset, size_t* bytes);
/* One embedding step: the embedding of the training parameters, its radius graph at r_train (at most k_max
 * targets per hit: the hard negatives), the training set of thesis ch. 8 (genuine pairs (q, succ[q]); fake
 * pairs: hard negatives of particles other than succ[q], and the random pair), the loss
 * L_fake + w_gen L_gen with L_gen the mean squared distance of the genuine pairs and L_fake the mean
 * max(0, margin - d^2) of the fake ones, its gradient, and an Adam step with learning rate lr (lr = 0: the
 * gradient only) on the embedding parameters.  *loss_dev (device float, may be NULL) receives the loss.
 * The graph is left in out->src/dst (CSR of the training radius). */
etx_status etx_train_embed_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth,
                                float margin, float w_gen, float r_train, float lr, int64_t step, float* loss_dev,
                                void* ws, size_t ws_bytes, etx_stream stream);
/* One network step on the rough graph of the context's inference embedding (radius, k_max): an edge is
 * genuine when its target is succ[source]; mean sigmoid focal loss (alpha, gamma) of the edge scores, its
 * gradient through the classifier, the message-passing steps and the encoders, and an Adam step (lr = 0: the
 * gradient only) on the network parameters.  Synchronises the stream once (the edge count sizes the step);
 * a device error of the graph building is returned. */
etx_status etx_train_gnn_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth, float alpha,
                              float gamma, float lr, int64_t step, float* loss_dev, void* ws, size_t ws_bytes,
                              etx_stream stream);

/* Triplet stage (thesis ch. 8 "The ETX4VELO Pipeline", "Triplet Building" and
 * "Track Building"): after the score cut, the purified hit graph is turned
 * into a graph of edges whose links are triplets, two triplet classifiers
 * purify it, and tracks are built from it; tracks may share hits (the
 * thesis's reason for the stage: particles that leave the same first hits).
 *
 * Triplets around every hit C, from its kept in-edges (by source) and kept
 * out-edges (by target):
 *   articulation (A->C, C->B)  every in/out pair            kind 0
 *   left elbow   (C->A, C->B)  every pair of out-edges      kind 1
 *   right elbow  (A->C, B->C)  every pair of in-edges       kind 2
 * The batch lists all its articulations (event by event, hit by hit, in-edge
 * major) and then all its elbows (same order, a hit's left elbows before its
 * right ones).  (tri_a, tri_b) is the classifier's input order: the in-edge
 * first for an articulation, the shorter edge first for an elbow (its other
 * hit on the plane nearer to C; equal planes: the earlier edge).
 *
 * Classifiers: one for articulations, one for both kinds of elbow, each
 * Linear(H->1)(Block(H->H)(Block(2H->H)([e_a, e_b]))) on the final edge
 * encodings, Block(x) = ReLU(LN(x W + b)), score = sigmoid; FP32 arithmetic in
 * every precision mode.  A triplet is kept when its score >= edge_threshold.
 *
 * Track building (four steps): (1) a kept edge that is the longer edge of a
 * kept left elbow at its source and of a kept right elbow at its target
 * duplicates the path through the middle hit and leaves the edge graph;
 * (2) the links are the kept articulations of two remaining edges; a link
 * (p, q) is shared when another link starts at p or another link ends at q;
 * weakly connected components over the non-shared links, each named by its
 * smallest edge index; (3) every component that no shared link touches is a
 * track, and every shared link (p, q) is a track made of the components of p
 * and q; (4) a track's hits are the endpoints of its edges, ascending.  Per
 * event the tracks are the untouched components by name, then the shared
 * links in triplet order.
 *
 * Parameters: float32, the articulation classifier then the elbow classifier,
 * each W1[2H][H] b1[H] W2[H][H] b2[H] W3[H][1] b3[1]. */
#define ETX_TRIPLET_NPARAM(H) (2 * (3 * (H) * (H) + 3 * (H) + 1))
etx_status etx_triplet_set(etx_ctx* ctx, const float* params, int64_t n);   /* host params */
etx_status etx_triplet_get(const etx_ctx* ctx, float* params, int64_t n);   /* host params */

typedef struct {             /* device pointers, caller-owned, written by etx_run_tracks */
  int64_t triplet_capacity;  /* length of tri_a, tri_b, tri_score, tri_kind */
  int32_t* tri_a;            /* first edge of the triplet (global edge index into out->src / out->dst) */
  int32_t* tri_b;            /* second edge */
  float* tri_score;          /* triplet classifier score */
  uint8_t* tri_kind;         /* 0 articulation, 1 left elbow, 2 right elbow */
  int64_t* art_off;          /* [n_events+1] event e's articulations: art_off[e] .. art_off[e+1]-1 */
  int64_t* elb_off;          /* [n_events+1] its elbows: elb_off[e] .. elb_off[e+1]-1 (after all articulations) */
  int64_t track_capacity;    /* tracks */
  int64_t* event_track_off;  /* [n_events+1] event e's tracks: event_track_off[e] .. event_track_off[e+1]-1 */
  int64_t* track_off;        /* [track_capacity+1] track t's hits: track_hits[track_off[t] .. track_off[t+1]-1]
                                (entries 0 .. n_tracks are written, n_tracks = event_track_off[n_events]) */
  int64_t hit_capacity;      /* length of track_hits */
  int32_t* track_hits;       /* global hit indices, ascending within a track */
  int64_t* status;           /* [4] status[0] = etx_status of the stage (ETX_ERR_CAPACITY when a capacity is too
                                small), status[1] = triplets needed, status[2] = tracks needed, status[3] = track
                                hits needed (each set when its capacity was the one exceeded) */
} etx_tracks;

/* Workspace bytes of etx_run_tracks: the etx_run workspace of the batch plus
 * the triplet stage's buffers for these capacities. */
etx_status etx_tracks_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                                     int64_t triplet_capacity, int64_t track_capacity, size_t* bytes);
/* The whole hot path of etx_run (same outputs in `out`), then the triplet
 * stage into `tracks`.  Needs the triplet parameters (etx_triplet_set); the
 * classifiers read the final edge encodings as the network stores them (FP32,
 * or BF16 with ETX_OPT_COMPACT_STATE in BF16 runs); FP8 runs with the compact
 * state are not supported (ETX_ERR_UNSUPPORTED).  Runs
 * eagerly on `stream` (ETX_OPT_USE_GRAPH is not applied); asynchronous.  A
 * device error of etx_run's stages (out->status) skips the triplet stage. */
etx_status etx_run_tracks(etx_ctx* ctx, const etx_hits* hits, etx_out* out, etx_tracks* tracks, void* ws,
                          size_t ws_bytes, etx_stream stream);

/* One network step with the triplet term of eq. gnn-loss (thesis ch. 8 "Graph
 * Neural Network and Classifiers"): the step of etx_train_gnn_step, then the
 * triplets of the purified graph of the step's own edge scores (score >=
 * edge_threshold, as in etx_run_tracks), the two triplet classifiers of the
 * training state on them, and the loss L_edges + L_art + L_elb, each the mean
 * sigmoid focal loss (alpha, gamma) of its classifier over its items.  A
 * triplet is genuine when one particle runs through all three hits along its
 * successor chain (articulation: C = next(A), B = next(C)) or, for an elbow,
 * when one particle owns all three hits; an edge is genuine when its target
 * is succ or succ2 of its source.  The triplet classifiers' gradient flows
 * back through the final edge encodings into the whole network; Adam (lr = 0:
 * the gradient only) updates the network and both classifiers.  The training
 * state of the classifiers starts from the context's triplet parameters
 * (etx_triplet_set) at the first such step after etx_train_begin.
 * `triplet_capacity` sizes the step's triplet buffers (workspace:
 * etx_train_triplet_workspace_size); more triplets than that return
 * ETX_ERR_CAPACITY with *triplets_needed (host, may be NULL) set.  *loss_dev
 * (device, may be NULL) receives float[3]: L_edges, L_art, L_elb.
 * Synchronises the stream twice (edge and triplet counts). */
etx_status etx_train_triplet_workspace_size(const etx_ctx* ctx, int64_t n_events, int64_t n_hits,
                                            int64_t edge_capacity, int64_t triplet_capacity, size_t* bytes);
etx_status etx_train_triplet_step(etx_ctx* ctx, const etx_hits* hits, etx_out* out, const etx_truth* truth,
                                  float alpha, float gamma, float lr, int64_t step, int64_t triplet_capacity,
                                  int64_t* triplets_needed, float* loss_dev, void* ws, size_t ws_bytes,
                                  etx_stream stream);
/* Triplet buffers of that workspace: 0 = float [ETX_TRIPLET_NPARAM(H)] classifier gradient, 1 = uint8 labels,
 * 2 = int32 first edges, 3 = int32 second edges, 4 = uint8 kinds (the step's triplets, in etx_run_tracks'
 * order), 5 = int64 [n_events+1] articulation offsets, 6 = int64 [n_events+1] elbow offsets (as in etx_tracks). */
etx_status etx_train_triplet_view(const etx_ctx* ctx, int64_t n_events, int64_t n_hits, int64_t edge_capacity,
                                  int64_t triplet_capacity, int32_t which, size_t* offset, size_t* bytes);
/* Host copy of the triplet classifiers' training state (set = 0) or its replacement (set = 1): the first n
 * floats of [params, Adam m, Adam v], n <= 3 x ETX_TRIPLET_NPARAM(H).  etx_train_apply also makes the trained
 * classifiers the context's triplet parameters. */
etx_status etx_train_triplet_params(etx_ctx* ctx, float* host, int64_t n, int32_t set);

/* Checkpoint of a context: configuration, weight blob, per-tensor scales and
 * calibration flag, prefilter parameters with their Adam moments and fallback
 * band, the triplet classifiers (when set), and the launch options (the state
 * that training, calibration and tuning build up).
 * etx_save with buf == NULL stores the byte count in *nbytes; with a buffer of
 * *nbytes bytes it writes the checkpoint (ETX_ERR_INVALID_ARG and the needed
 * size if it is too small).  The prefilter moments are read from the device,
 * so the call waits for the device.  etx_load creates a context on `device`
 * from such a buffer (ETX_ERR_INVALID_ARG for a buffer that is not one, of
 * this library's layout and size), exactly as etx_create would with the saved
 * configuration and weights, then restores the rest.  Plain host memory; the
 * format is this library's own (native byte order). */
etx_status etx_save(const etx_ctx* ctx, void* buf, size_t* nbytes);
etx_status etx_load(const void* buf, size_t nbytes, int device, etx_ctx** out);

const char* etx_status_str(etx_status s);
/* Text of the last HIP failure seen by this thread ("" if none). */
const char* etx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ETX_H */
