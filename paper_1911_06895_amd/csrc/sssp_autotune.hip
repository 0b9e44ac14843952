// Schedule autotuner: the method has one knob, delta (the bucket width, which
// also decides which edges are light, Sec. III-A/IV-A); the library adds its
// own: the number of sources solved concurrently and the tile schedule (the
// workgroup size, the hub threshold, the chunk size, the largest step run by
// one workgroup alone). sssp_autotune times solves of a sample of sources:
// first over (delta, concurrent groups), then, on the fastest handle, over
// each tile parameter and the chaining of the leader's light steps in turn
// (coordinate search, keeping a value only when it is at least 2 % faster
// than the current choice), and returns that handle.
// Host code only, over the public entry points.
#include <cmath>
#include <cstring>
#include <vector>

#include "sssp.h"
#include "sssp_internal.h"

namespace {

// Candidate deltas from the weights: powers of two around the mean weight (an
// integer >= 1 for integer weights). Small deltas mean many buckets with
// small phases; large ones mean light edges relaxed again and again.
sssp_status derive_deltas(const sssp_graph* g, hipStream_t s, std::vector<double>* out) {
  uint32_t* scratch = nullptr;  // [0] status, [2..3] max weight bits, [4..5] fp64 weight total
  if (hipMalloc(reinterpret_cast<void**>(&scratch), 6 * sizeof(uint32_t)) != hipSuccess) return SSSP_ERR_OUT_OF_MEMORY;
  hipError_t e = hipMemsetAsync(scratch, 0, 6 * sizeof(uint32_t), s);
  if (e == hipSuccess)
    e = sssp::launch_validate(g->row_ptr, g->col_idx, g->weights, g->wtype, g->n, g->m, scratch,
                              reinterpret_cast<unsigned long long*>(scratch + 2), reinterpret_cast<double*>(scratch + 4),
                              s);
  uint32_t res[6] = {0, 0, 0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(res, scratch, sizeof(res), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (e != hipSuccess) return SSSP_ERR_DEVICE;
  if (res[0] & (sssp::kBadRowPtr | sssp::kBadCol)) return SSSP_ERR_INVALID_ARGUMENT;
  if (res[0] & sssp::kBadWeight) return SSSP_ERR_INVALID_WEIGHT;
  double wsum;
  std::memcpy(&wsum, res + 4, sizeof(double));
  const double mean = g->m > 0 ? wsum / static_cast<double>(g->m) : 1.0;
  const int c = static_cast<int>(std::floor(std::log2(mean)));
  out->clear();
  if (g->wtype == SSSP_WEIGHT_U32) {
    uint64_t wmax_bits;
    std::memcpy(&wmax_bits, res + 2, sizeof(wmax_bits));
    const double wmax = static_cast<double>(wmax_bits);
    for (int j = c - 4; j <= c + 1; ++j) {
      const double d = std::ldexp(1.0, j);
      if (d >= 1.0 && (d <= wmax || out->empty())) out->push_back(d);
    }
  } else {
    for (int j = c - 4; j <= c + 2; ++j) out->push_back(std::ldexp(1.0, j));
  }
  if (out->empty()) out->push_back(1.0);
  return SSSP_OK;
}

// Device time of one solve of the sample (after a warm-up solve), or a status;
// with reps = 2 the faster of two timed solves.
sssp_status time_solve(sssp_handle* h, const int32_t* src_dev, int32_t k, int32_t mode, void* dist, hipStream_t s,
                       float* ms, int reps = 1) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SSSP_ERR_DEVICE;
  }
  auto enqueue = [&] {
    return mode == 0 ? sssp_solve_async(h, src_dev, k, dist, s) : sssp_solve_multi_async(h, src_dev, k, dist, s);
  };
  sssp_status st = enqueue();
  if (st == SSSP_OK) st = sssp_solve_status(h, s);
  *ms = INFINITY;
  for (int r = 0; r < reps && st == SSSP_OK; ++r) {
    float t = 0;
    if (hipEventRecord(e0, s) != hipSuccess) st = SSSP_ERR_DEVICE;
    if (st == SSSP_OK) st = enqueue();
    if (st == SSSP_OK && hipEventRecord(e1, s) != hipSuccess) st = SSSP_ERR_DEVICE;
    if (st == SSSP_OK) st = sssp_solve_status(h, s);
    if (st == SSSP_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = SSSP_ERR_DEVICE;
    if (st == SSSP_OK && t < *ms) *ms = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // namespace

extern "C" {

sssp_status sssp_autotune(const sssp_graph* g, const int32_t* sources, int32_t k, int32_t mode, const double* deltas,
                          int32_t n_deltas, void* dist, void* stream, sssp_handle** out,
                          sssp_autotune_result* result) {
  if (!out) return SSSP_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!g || !sources || k < 1 || !dist || (mode != 0 && mode != 1) || n_deltas < 0 || (n_deltas > 0 && !deltas))
    return SSSP_ERR_INVALID_ARGUMENT;
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= g->n) return SSSP_ERR_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<double> cand;
  if (n_deltas > 0) {
    cand.assign(deltas, deltas + n_deltas);
  } else {
    const sssp_status st = derive_deltas(g, s, &cand);
    if (st != SSSP_OK) return st;
  }
  int32_t* src_dev = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&src_dev), sizeof(int32_t) * k) != hipSuccess) return SSSP_ERR_OUT_OF_MEMORY;
  if (hipMemcpy(src_dev, sources, sizeof(int32_t) * k, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(src_dev);
    return SSSP_ERR_DEVICE;
  }
  // concurrent groups: powers of two up to the sample size (one group for multi-source solves)
  std::vector<int32_t> groups = {1};
  if (mode == 0)
    for (int32_t gcount = 8; gcount <= sssp::kMaxGroups && gcount <= k; gcount *= 2) groups.push_back(gcount);

  sssp_handle* best = nullptr;
  sssp_autotune_result res{};
  res.ms = INFINITY;
  sssp_status last_error = SSSP_OK;
  for (double delta : cand) {
    sssp_handle* h = nullptr;
    sssp_status st = sssp_create(g, delta, stream, &h);
    if (st != SSSP_OK) {  // e.g. an fp32 delta too small for the bucket range
      last_error = st;
      continue;
    }
    int32_t h_groups = 1;
    float h_ms = INFINITY;
    for (int32_t gcount : groups) {
      sssp_tuning t{};
      t.concurrent_sources = gcount;
      if (sssp_set_tuning(h, &t) != SSSP_OK) break;  // group count or memory exhausted
      float ms = 0;
      st = time_solve(h, src_dev, k, mode, dist, s, &ms);
      ++res.trials;
      if (st != SSSP_OK) {
        last_error = st;
        break;
      }
      if (ms < h_ms) {
        h_ms = ms;
        h_groups = gcount;
      } else if (ms > 1.05f * h_ms) {
        break;  // past the best group count for this delta
      }
    }
    if (h_ms < res.ms) {
      sssp_tuning t{};
      t.concurrent_sources = h_groups;
      if (sssp_set_tuning(h, &t) == SSSP_OK) {
        if (best) sssp_destroy(best);
        best = h;
        res.delta = delta;
        res.concurrent_sources = h_groups;
        res.ms = h_ms;
        continue;
      }
    }
    sssp_destroy(h);
  }
  if (!best) {
    (void)hipFree(src_dev);
    return last_error != SSSP_OK ? last_error : SSSP_ERR_UNSUPPORTED;
  }
  // the tile schedule, one parameter at a time on the chosen (delta, groups)
  sssp_tuning cur{};
  cur.concurrent_sources = res.concurrent_sources;
  float cur_ms = INFINITY;
  if (time_solve(best, src_dev, k, mode, dist, s, &cur_ms, 2) == SSSP_OK) {
    ++res.trials;
    struct Knob {
      int32_t sssp_tuning::*field;
      std::vector<int32_t> values;
    };
    std::vector<Knob> knobs = {{&sssp_tuning::hub_edges, {512, 2048, 4096}},
                               {&sssp_tuning::chunk_entries, {64, 128, 256, 512}},
                               {&sssp_tuning::inline_edges, {1024, 16384}},
                               {&sssp_tuning::inline_entries, {64, 128}},
                               {&sssp_tuning::leader_chain, {1, 2}}};
    if (res.concurrent_sources == 1) knobs.insert(knobs.begin(), Knob{&sssp_tuning::workgroups_per_cu, {1}});
    for (const Knob& kb : knobs) {
      int32_t keep = cur.*kb.field;
      for (int32_t v : kb.values) {
        sssp_tuning t = cur;
        t.*kb.field = v;
        if (sssp_set_tuning(best, &t) != SSSP_OK) continue;
        float ms = 0;
        if (time_solve(best, src_dev, k, mode, dist, s, &ms, 2) != SSSP_OK) continue;
        ++res.trials;
        if (ms < 0.98f * cur_ms) {
          cur_ms = ms;
          keep = v;
        }
      }
      cur.*kb.field = keep;
    }
    if (sssp_set_tuning(best, &cur) == SSSP_OK) res.ms = cur_ms;
  }
  (void)hipFree(src_dev);
  (void)sssp_get_tuning(best, &res.tuning);
  *out = best;
  if (result) *result = res;
  return SSSP_OK;
}

}  // extern "C"
