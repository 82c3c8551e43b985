// Launch-schedule autotuner and its tuning table.
//
// The tuner times the batch with each candidate setting of the launch knobs
// (workgroup size and persistent workgroups per CU of the edge kernels, their
// software-pipeline depth, workgroups per CU of the node kernels, whether the
// node kernel gathers its own messages, rows in flight of the segmented sums,
// the window size from which the radius search sorts, ...) and keeps the
// fastest, one knob at a time, judging each knob by the HIP-event time of the
// stages it drives.  None of the knobs changes a result bit.
//
// The choice is kept in the context's tuning table under the key
// (configuration and run modes, shape bucket of the batch); etx_run applies the
// entry of a batch's bucket.  The table is saved to and loaded from a text
// file, one entry per line: "<arch> <signature> <bucket> <option>=<value> ...".
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

extern "C" etx_status etx_profile_read(etx_ctx* ctx, int32_t n_stages, double* total_ms, int64_t* launches);
extern "C" etx_status etx_profile_reset(etx_ctx* ctx);

namespace etx {

const int32_t kTunedOptions[] = {ETX_OPT_EDGE_WG_SIZE,  ETX_OPT_EDGE_WG_PER_CU,    ETX_OPT_EDGE_PRODUCTS,
                                 ETX_OPT_EDGE_PIPELINE, ETX_OPT_XCD_MAP,           ETX_OPT_NODE_WG_PER_CU,
                                 ETX_OPT_FUSE_MESSAGES, ETX_OPT_SEGSUM_UNROLL,     ETX_OPT_RADIUS_SORT_MIN,
                                 ETX_OPT_RADIUS_FAST,   ETX_OPT_CSC_PLACE,         ETX_OPT_RADIUS_SPLIT};
const int kNumTunedOptions = sizeof(kTunedOptions) / sizeof(kTunedOptions[0]);

// Shape bucket: hits per event and events per batch, each rounded to the
// nearest power of two (the schedules that win change with both: how many
// persistent workgroups the batch fills, how long the edge rows are).
std::string tuning_key(const etx_ctx* ctx, int64_t n_events, int64_t n_hits) {
  const etx_config& c = ctx->cfg;
  const double per_event = n_events > 0 ? double(n_hits) / double(n_events) : 0.0;
  const int hb = per_event >= 1.0 ? (int)std::lround(std::log2(per_event)) : 0;
  const int nb = n_events >= 1 ? (int)std::lround(std::log2(double(n_events))) : 0;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "P%d.e%dx%d-%d.r%.6g.k%d.w%d.H%d.S%d.p%d.ep%d.cs%d.pf%d h%d.n%d", c.n_planes,
                c.emb_hidden, c.emb_layers, c.emb_dim, (double)c.radius, c.k_max, c.plane_window, c.gnn_hidden,
                c.gnn_steps, c.precision, ctx->emb_precision, ctx->compact_state, c.prefilter, hb, nb);
  return buf;
}

}  // namespace etx

using namespace etx;

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

// Best of two timed runs after a warm-up run.  The device status of the first
// run is read back: a batch that overflows its edge capacity or fails input
// validation makes every kernel exit early, and timing such runs would tune on
// nothing.
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
    if (rep == 0) {
      int64_t dev_status[2] = {0, 0};
      if (hipMemcpyAsync(dev_status, out->status, sizeof(dev_status), hipMemcpyDeviceToHost,
                         static_cast<hipStream_t>(stream)) != hipSuccess ||
          hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) {
        *st = ETX_ERR_HIP;
        return 1e30;
      }
      if (dev_status[0] != ETX_OK) {
        *st = static_cast<etx_status>(dev_status[0]);
        return 1e30;
      }
    }
    double t = 0;
    for (int s : stages) t += ms[s];
    if (rep > 0) best = std::min(best, t);   // the first run warms caches and code objects
  }
  return best;
}

bool split_line(const std::string& line, std::string* arch, std::string* sig, std::string* bucket,
                std::vector<std::pair<int32_t, int64_t>>* opts) {
  if (line.empty() || line[0] == '#') return false;
  std::istringstream is(line);
  if (!(is >> *arch >> *sig >> *bucket)) return false;
  opts->clear();
  std::string kv;
  while (is >> kv) {
    const size_t eq = kv.find('=');
    if (eq == std::string::npos) return false;
    char* end = nullptr;
    const long k = std::strtol(kv.c_str(), &end, 10);
    if (end != kv.c_str() + eq) return false;
    const long long v = std::strtoll(kv.c_str() + eq + 1, &end, 10);
    if (*end != '\0') return false;
    opts->emplace_back((int32_t)k, (int64_t)v);
  }
  return true;
}

}  // namespace

extern "C" etx_status etx_tuning_load(etx_ctx* ctx, const char* path) {
  if (!ctx || !path) return ETX_ERR_INVALID_ARG;
  std::ifstream f(path);
  if (!f) return ETX_ERR_INVALID_ARG;
  std::string line, arch, sig, bucket;
  std::vector<std::pair<int32_t, int64_t>> opts;
  while (std::getline(f, line)) {
    if (!split_line(line, &arch, &sig, &bucket, &opts)) continue;
    if (arch != ctx->arch) continue;
    bool ok = true;
    for (const auto& kv : opts) {
      int64_t cur;
      bool tuned = false;
      for (int i = 0; i < kNumTunedOptions; ++i) tuned |= kv.first == kTunedOptions[i];
      if (!tuned || etx_get_option(ctx, kv.first, &cur) != ETX_OK) ok = false;
    }
    if (ok) ctx->tuning[sig + " " + bucket] = opts;
  }
  ctx->tuning_applied.clear();
  return ETX_OK;
}

extern "C" etx_status etx_tuning_save(const etx_ctx* ctx, const char* path) {
  if (!ctx || !path) return ETX_ERR_INVALID_ARG;
  // keep the file's other entries (other architectures, configurations, buckets)
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line, arch, sig, bucket;
    std::vector<std::pair<int32_t, int64_t>> opts;
    while (f && std::getline(f, line)) {
      if (!split_line(line, &arch, &sig, &bucket, &opts)) continue;
      if (arch == ctx->arch && ctx->tuning.count(sig + " " + bucket)) continue;
      keep.push_back(line);
    }
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* out = std::fopen(tmp.c_str(), "w");
  if (!out) return ETX_ERR_INVALID_ARG;
  std::fputs("# etx tuning table: <arch> <configuration signature> <shape bucket> <option>=<value> ...\n", out);
  for (const std::string& l : keep) std::fprintf(out, "%s\n", l.c_str());
  for (const auto& e : ctx->tuning) {
    std::fprintf(out, "%s %s", ctx->arch.c_str(), e.first.c_str());
    for (const auto& kv : e.second) std::fprintf(out, " %d=%lld", kv.first, (long long)kv.second);
    std::fputc('\n', out);
  }
  const bool ok = std::fclose(out) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) return ETX_ERR_INVALID_ARG;
  return ETX_OK;
}

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
      {{ETX_OPT_RADIUS_SPLIT}, "radius_split", {{0}, {1}}, {ST_RADIUS_COUNT, ST_RADIUS_EMIT}},
      {{ETX_OPT_CSC_PLACE}, "csc_place", {{0}, {1}}, {ST_CSC}},
  };
  // the options in effect before tuning come back if tuning fails
  int64_t before[kNumTunedOptions];
  for (int i = 0; i < kNumTunedOptions; ++i) etx_get_option(ctx, kTunedOptions[i], &before[i]);
  const std::string key = tuning_key(ctx, hits->n_events, hits->n_hits);
  // etx_run must not switch to a stored entry while the knobs are tried
  auto stored = ctx->tuning.find(key);
  std::vector<std::pair<int32_t, int64_t>> stored_opts;
  const bool had_entry = stored != ctx->tuning.end();
  if (had_entry) {
    stored_opts = stored->second;
    ctx->tuning.erase(stored);
  }
  const int prev_profile = ctx->profile, prev_graph = ctx->use_graph;
  const int64_t prev_mask = ctx->profile_mask;
  ctx->profile = 1;
  ctx->profile_mask = 0x7fffffff;
  ctx->use_graph = 0;
  etx_status st = ETX_OK;
  std::string record = "{\"arch\": \"" + ctx->arch + "\", \"key\": \"" + key +
                       "\", \"n_events\": " + std::to_string(hits->n_events) +
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
  ctx->profile_mask = prev_mask;
  ctx->use_graph = prev_graph;
  etx_profile_reset(ctx);
  if (st != ETX_OK) {
    for (int i = 0; i < kNumTunedOptions; ++i) etx_set_option(ctx, kTunedOptions[i], before[i]);
    if (had_entry) ctx->tuning[key] = stored_opts;
    return st;
  }
  std::vector<std::pair<int32_t, int64_t>> chosen;
  for (int i = 0; i < kNumTunedOptions; ++i) {
    int64_t v;
    etx_get_option(ctx, kTunedOptions[i], &v);
    chosen.emplace_back(kTunedOptions[i], v);
  }
  ctx->tuning[key] = chosen;
  ctx->tuning_applied = key;
  record += "}}\n";
  if (json_path) {
    FILE* f = std::fopen(json_path, "a");
    if (!f) return ETX_ERR_INVALID_ARG;
    std::fputs(record.c_str(), f);
    std::fclose(f);
  }
  return ETX_OK;
}
