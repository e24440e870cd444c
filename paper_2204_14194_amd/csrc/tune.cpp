// Autotuner for the batched path: times the candidate workgroup shapes of the
// iteration loop (every shape with the same padded row length, so tables
// stay valid) and the two tile sizes of the projection GEMM on the caller's
// own batch, and records the fastest per (K, area pixels, batch-size
// bucket).  For rows on demand it times the row products' tile and split of
// a plan, per (dense atoms, area pixels, batch-size bucket).  The batched calls consult the record; without one they use the
// default shape and the tile heuristic.  Records can be exported as text and
// imported again (one line per entry).
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "se_internal.h"

namespace sefase {

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, TuneChoice> g_tune;

static int bucket(int n_blk) {
  int b = 0;
  while ((1 << b) < n_blk && b < 30) ++b;
  return b;
}

TuneChoice tune_lookup(int K, int P, int n_blk) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({K, P, bucket(n_blk)});
  return it == g_tune.end() ? TuneChoice{} : it->second;
}

static void tune_store(int K, int P, int n_blk, const TuneChoice& c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[{K, P, bucket(n_blk)}] = c;
}

// rows on demand: (dense atoms, pixels, bucket) -> row-product shape
static std::map<std::tuple<int, int, int>, RowTune> g_tune_rows;

RowTune tune_lookup_rows(int Kd, int P, int n_blk) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_rows.find({Kd, P, bucket(n_blk)});
  return it == g_tune_rows.end() ? RowTune{} : it->second;
}

static bool row_tune_valid(int tile, int split) {
  return (tile == 0 || tile == 64 || tile == 128 || tile == kTile128x64) &&
         (split == -1 || split == 1 || split == 2 || split == 4 || split == 8) &&
         !(tile == 128 && split > 1);
}

}  // namespace sefase

using namespace sefase;

extern "C" {

se_status se_autotune_batch(const se_tables* t, uint8_t* images, int32_t n_img, int32_t H,
                            int32_t W, const se_block* dev_blocks, int32_t n_blk, se_params prm,
                            float* R, int32_t ldR, void* ws, size_t ws_bytes, int32_t reps,
                            void* stream, se_tune_result* out) {
  if (!out || reps < 1 || n_blk < 1) return fail(SE_EINVAL, "bad autotune arguments");
  if (t && t->phi_im) return fail(SE_EINVAL, "the autotuner takes tables of real dictionaries");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SE_EHIP, "event creation failed");
  se_status st = SE_OK;
  TuneChoice best;
  float best_proj = 1e30f, best_loop = 1e30f;
  const int P = t ? area_samples(t) : 0;
  // projection: both tiles (FP32 tables only; the split path has one tile rule)
  const int tiles[2] = {64, 128};
  for (int ti = 0; ti < 2 && st == SE_OK; ++ti) {
    if (t && t->precision != SE_FP32 && ti > 0) break;
    tune_store(t ? t->K : 0, P, n_blk, TuneChoice{0, 0, tiles[ti]});
    float ms = 0.0f;
    for (int r = 0; r <= reps && st == SE_OK; ++r) {   // first run warms up
      hipEventRecord(e0, s);
      st = se_project(t, images, n_img, H, W, dev_blocks, n_blk, R, ldR, ws, ws_bytes, stream);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float v = 0.0f;
      hipEventElapsedTime(&v, e0, e1);
      if (r > 0) ms += v / reps;
    }
    if (st == SE_OK && ms < best_proj) {
      best_proj = ms;
      best.proj_tile = tiles[ti];
    }
  }
  // loop: every shape with the same row length
  int wv[8], vp[8];
  const int ns = st == SE_OK ? greedy_shapes_for(t->K, wv, vp, 8) : 0;
  for (int i = 0; i < ns && st == SE_OK; ++i) {
    tune_store(t->K, P, n_blk, TuneChoice{wv[i], vp[i], best.proj_tile});
    float ms = 0.0f;
    for (int r = 0; r <= reps && st == SE_OK; ++r) {
      hipEventRecord(e0, s);
      st = se_iterate(t, R, ldR, images, n_img, H, W, dev_blocks, n_blk, prm, nullptr, nullptr,
                      nullptr, 0, stream);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float v = 0.0f;
      hipEventElapsedTime(&v, e0, e1);
      if (r > 0) ms += v / reps;
    }
    if (st == SE_OK && ms < best_loop) {
      best_loop = ms;
      best.loop_waves = wv[i];
      best.loop_vpl = vp[i];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SE_OK) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.erase({t ? t->K : 0, P, bucket(n_blk)});
    return st;
  }
  tune_store(t->K, P, n_blk, best);
  out->loop_waves = best.loop_waves;
  out->loop_vpl = best.loop_vpl;
  out->proj_tile = best.proj_tile;
  out->loop_ms = best_loop;
  out->proj_ms = best_proj;
  return SE_OK;
}

se_status se_autotune_ondemand(se_od_plan* p, const float* w, uint8_t* images, int32_t reps,
                               void* stream, se_tune_rows_result* out) {
  if (!p || !out || reps < 1) return fail(SE_EINVAL, "bad autotune arguments");
  const int nd = ondemand_plan_dense(p, nullptr, nullptr);
  const int n = ondemand_plan_blocks(p);
  if (nd == 0 || n == 0) return fail(SE_EINVAL, "the plan has no dense row products to tune");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SE_EHIP, "event creation failed");
  static const RowTune cand[] = {{64, 1},          {64, 2},          {64, 4},
                                 {64, 8},          {128, 1},         {kTile128x64, 1},
                                 {kTile128x64, 2}, {kTile128x64, 4}, {0, -1}};
  se_status st = SE_OK;
  RowTune best;
  float best_ms = 1e30f;
  for (const RowTune& c : cand) {
    ondemand_plan_set_rows(p, c.tile, c.split);
    float ms = 0.0f;
    for (int r = 0; r <= reps && st == SE_OK; ++r) {   // first run warms up
      hipEventRecord(e0, s);
      st = se_ondemand_run(p, w, images, nullptr, nullptr, nullptr, 0, stream);
      if (st == SE_ENUMERIC) st = SE_OK;   // blocks without support: a result, not an error
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float v = 0.0f;
      hipEventElapsedTime(&v, e0, e1);
      if (r > 0) ms += v / reps;
    }
    if (st != SE_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SE_OK) {
    ondemand_plan_set_rows(p, 0, -1);
    return st;
  }
  ondemand_plan_set_rows(p, best.tile, best.split);
  int kd[3], P = 0;
  const int nr = ondemand_plan_dense(p, kd, &P);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int r = 0; r < nr; ++r) g_tune_rows[{kd[r], P, bucket(n)}] = best;
  }
  out->row_tile = best.tile;
  out->row_split = best.split;
  out->run_ms = best_ms;
  return SE_OK;
}

int32_t se_tune_export(char* buf, int32_t cap) {
  std::string s;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    char line[128];
    for (auto& kv : g_tune) {
      snprintf(line, sizeof(line), "%d %d %d %d %d %d\n", std::get<0>(kv.first),
               std::get<1>(kv.first), std::get<2>(kv.first), kv.second.loop_waves,
               kv.second.loop_vpl, kv.second.proj_tile);
      s += line;
    }
    for (auto& kv : g_tune_rows) {
      snprintf(line, sizeof(line), "rows %d %d %d %d %d\n", std::get<0>(kv.first),
               std::get<1>(kv.first), std::get<2>(kv.first), kv.second.tile, kv.second.split);
      s += line;
    }
  }
  if (buf && cap > 0) {
    const size_t n = s.size() < (size_t)cap - 1 ? s.size() : (size_t)cap - 1;
    memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return (int32_t)s.size();
}

se_status se_tune_import(const char* text) {
  if (!text) return fail(SE_EINVAL, "NULL text");
  const char* p = text;
  while (*p) {
    if (strncmp(p, "rows ", 5) == 0) {
      int Kd, P, b, tile, split, used = 0;
      if (sscanf(p + 5, "%d %d %d %d %d%n", &Kd, &P, &b, &tile, &split, &used) != 5)
        return fail(SE_EINVAL, "malformed tuning line");
      if (Kd < 1 || Kd > 32768 || P < 1 || b < 0 || b > 30 || !row_tune_valid(tile, split))
        return fail(SE_EINVAL, "tuning entry out of range");
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_rows[{Kd, P, b}] = RowTune{tile, split};
      }
      p += 5 + used;
      while (*p == '\n' || *p == ' ' || *p == '\r' || *p == '\t') ++p;
      continue;
    }
    int K, P, b, w, v, tile, used = 0;
    if (sscanf(p, "%d %d %d %d %d %d%n", &K, &P, &b, &w, &v, &tile, &used) != 6)
      return fail(SE_EINVAL, "malformed tuning line");
    int wv[8], vp[8];
    const int ns = (K >= 1 && K <= 32768) ? greedy_shapes_for(K, wv, vp, 8) : 0;
    bool ok = (w == 0 && v == 0);
    for (int i = 0; i < ns; ++i) ok = ok || (wv[i] == w && vp[i] == v);
    if (!ok || (tile != 0 && tile != 64 && tile != 128) || b < 0 || b > 30 || P < 1)
      return fail(SE_EINVAL, "tuning entry out of range");
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[{K, P, b}] = TuneChoice{w, v, tile};
    }
    p += used;
    while (*p == '\n' || *p == ' ' || *p == '\r' || *p == '\t') ++p;
  }
  return SE_OK;
}

void se_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_rows.clear();
}

}  // extern "C"
