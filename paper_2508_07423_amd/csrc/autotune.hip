// Launch-schedule autotuner: times the batch with each candidate setting of
// the launch knobs (workgroup size and persistent workgroups per CU of the
// edge kernels, their software-pipeline depth, workgroups per CU of the node
// kernels, whether the node kernel gathers its own messages, rows in flight
// of the segmented sums, the window size from which the radius search sorts)
// and keeps the fastest, one knob at a time, judging
// each knob by the HIP-event time of the stages it drives.  None of the knobs
// changes a result bit.
#include <chrono>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.hpp"

extern "C" etx_status etx_profile_read(etx_ctx* ctx, int32_t n_stages, double* total_ms, int64_t* launches);
extern "C" etx_status etx_profile_reset(etx_ctx* ctx);

namespace {

// A knob sets one or more options together; each candidate gives one value per key.
struct Knob {
  std::vector<int32_t> keys;
  const char* name;
  std::vector<std::vector<int64_t>> values;
  std::vector<int> stages;   // stage indices whose time the knob drives
};

std::string join(const std::vector<int64_t>& v) {
  std::string s;
  for (size_t i = 0; i < v.size(); ++i) s += (i ? "x" : "") + std::to_string(v[i]);
  return s;
}

// stage indices as listed by etx_stage_name
constexpr int ST_RADIUS_COUNT = 4, ST_RADIUS_EMIT = 6, ST_CSC = 8, ST_NODE_ENC = 9, ST_EDGE_ENC = 10, ST_SEGSUM = 11,
              ST_NODE_STEP = 12, ST_EDGE_STEP = 13, ST_EDGE_FINAL = 14;

double timed_run(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes, etx_stream stream,
                 const std::vector<int>& stages, etx_status* st) {
  double best = 1e30;
  for (int rep = 0; rep < 3; ++rep) {
    etx_profile_reset(ctx);
    *st = etx_run(ctx, hits, out, ws, ws_bytes, stream);
    if (*st != ETX_OK) return 1e30;
    double ms[32];
    int64_t n[32];
    *st = etx_profile_read(ctx, 17, ms, n);
    if (*st != ETX_OK) return 1e30;
    double t = 0;
    for (int s : stages) t += ms[s];
    if (rep > 0) best = std::min(best, t);   // the first run warms caches and code objects
  }
  return best;
}

}  // namespace

extern "C" etx_status etx_autotune(etx_ctx* ctx, const etx_hits* hits, etx_out* out, void* ws, size_t ws_bytes,
                                   etx_stream stream, const char* json_path) {
  if (!ctx || !hits || !out) return ETX_ERR_INVALID_ARG;
  const std::vector<int> edge_stages = {ST_EDGE_ENC, ST_EDGE_STEP, ST_EDGE_FINAL};
  std::vector<Knob> knobs = {
      {{ETX_OPT_EDGE_WG_SIZE, ETX_OPT_EDGE_WG_PER_CU}, "edge_threads_x_wg_per_cu",
       {{512, 1}, {512, 2}, {512, 3}, {512, 4}, {256, 2}, {256, 3}, {256, 4}, {256, 5}, {256, 6}, {256, 8}},
       edge_stages},
      {{ETX_OPT_EDGE_PRODUCTS}, "edge_products", {{0}, {1}},
       {ST_NODE_ENC, ST_EDGE_ENC, ST_EDGE_STEP, ST_EDGE_FINAL, ST_NODE_STEP}},
      {{ETX_OPT_EDGE_PIPELINE}, "edge_pipeline", {{0}, {1}, {2}}, edge_stages},
      {{ETX_OPT_XCD_MAP}, "xcd_map", {{0}, {1}}, {ST_EDGE_ENC, ST_EDGE_STEP, ST_EDGE_FINAL, ST_SEGSUM, ST_NODE_STEP}},
      {{ETX_OPT_NODE_WG_PER_CU}, "node_wg_per_cu", {{1}, {2}, {3}, {4}}, {ST_NODE_ENC, ST_NODE_STEP}},
      {{ETX_OPT_FUSE_MESSAGES}, "fuse_messages", {{0}, {1}}, {ST_SEGSUM, ST_NODE_STEP}},
      {{ETX_OPT_SEGSUM_UNROLL}, "segsum_unroll", {{1}, {2}, {4}, {8}}, {ST_SEGSUM}},
      {{ETX_OPT_RADIUS_SORT_MIN}, "radius_sort_min", {{64}, {128}, {256}, {512}, {1024}}, {ST_RADIUS_COUNT, ST_RADIUS_EMIT}},
      {{ETX_OPT_RADIUS_FAST}, "radius_fast", {{0}, {1}}, {ST_RADIUS_COUNT, ST_RADIUS_EMIT}},
      {{ETX_OPT_CSC_PLACE}, "csc_place", {{0}, {1}}, {ST_CSC}},
  };
  const int prev_profile = ctx->profile, prev_graph = ctx->use_graph;
  ctx->profile = 1;
  ctx->use_graph = 0;
  etx_status st = ETX_OK;
  std::string record = "{\"arch\": \"gfx950\", \"n_events\": " + std::to_string(hits->n_events) +
                       ", \"n_hits\": " + std::to_string(hits->n_hits) +
                       ", \"gnn_hidden\": " + std::to_string(ctx->cfg.gnn_hidden) +
                       ", \"precision\": " + std::to_string(ctx->cfg.precision) + ", \"choice\": {";
  for (size_t ki = 0; ki < knobs.size() && st == ETX_OK; ++ki) {
    const Knob& k = knobs[ki];
    std::vector<int64_t> best_v;
    double best_t = 1e30;
    std::string trials;
    for (const std::vector<int64_t>& v : k.values) {
      for (size_t j = 0; j < k.keys.size() && st == ETX_OK; ++j) st = etx_set_option(ctx, k.keys[j], v[j]);
      if (st != ETX_OK) break;
      double t = timed_run(ctx, hits, out, ws, ws_bytes, stream, k.stages, &st);
      if (st != ETX_OK) break;
      char buf[96];
      std::snprintf(buf, sizeof(buf), "%s\"%s\": %.3f", trials.empty() ? "" : ", ", join(v).c_str(), t);
      trials += buf;
      if (t < best_t) {
        best_t = t;
        best_v = v;
      }
    }
    if (st != ETX_OK) break;
    for (size_t j = 0; j < k.keys.size(); ++j) etx_set_option(ctx, k.keys[j], best_v[j]);
    record += std::string(ki ? ", " : "") + "\"" + k.name + "\": \"" + join(best_v) + "\"";
    record += std::string(", \"") + k.name + "_ms\": {" + trials + "}";
  }
  ctx->profile = prev_profile;
  ctx->use_graph = prev_graph;
  etx_profile_reset(ctx);
  if (st != ETX_OK) return st;
  record += "}}\n";
  if (json_path) {
    FILE* f = std::fopen(json_path, "a");
    if (!f) return ETX_ERR_INVALID_ARG;
    std::fputs(record.c_str(), f);
    std::fclose(f);
  }
  return ETX_OK;
}
