// Serving loop of the C ABI (se_serve_*): frame slots, a device cache of the
// tables of isolated weight patterns (Algorithm 2 computed once per pattern
// and kept, as the paper suggests for recurring patterns), and continuous
// batching of requests over a pool of streams.
//
// One worker thread owns every device call.  Each cycle it
//   1. admits queued requests while frame slots are free;
//   2. launches all admitted, not yet launched requests as one batch on the
//      next stream: frames are copied into their slots, the lost-pixel masks
//      built, blocks grouped by weight pattern (isolated blocks, per
//      (dictionary, loss rectangle, gamma, I)) or by dictionary (blocks with
//      their own weights), each group concealed by one batched call, and
//      the frames copied back;
//   3. retires finished batches (event query), releasing slots and cache
//      references.
// A batch launched while earlier ones still run goes to another stream, so
// their kernels overlap on the device.  Every block's arithmetic depends
// only on its own frame, so results do not depend on the batch a request
// lands in.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "se_internal.h"

namespace sefase {

static uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// weight pattern of an isolated block: dictionary + loss rectangle in the area
struct PatternKey {
  int basis, ly, lx, lh, lw;
  bool operator<(const PatternKey& o) const {
    return std::tie(basis, ly, lx, lh, lw) < std::tie(o.basis, o.ly, o.lx, o.lh, o.lw);
  }
};

struct CachedTables {
  se_tables t{};
  void* mem = nullptr;
  size_t bytes = 0;
  uint64_t last_use = 0;
  int refs = 0;
};

struct Req {
  uint64_t ticket = 0;
  uint8_t* frame = nullptr;
  std::vector<se_loss> losses;
  se_params prm{};
  int slot = -1;
  int state = 0;   // 0 queued, 1 admitted, 2 launched, 3 done
  int n_degenerate = 0;   // blocks with no available sample in their area
  se_result res{};
};

struct Batch {
  hipEvent_t done = nullptr;
  std::vector<Req*> reqs;
  std::vector<PatternKey> refs;
  se_status status = SE_OK;
};

struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace sefase

struct se_server {
  se_serve_config cfg{};
  std::vector<se_basis> sets;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<sefase::Req*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<sefase::Req>> reqs;
  std::vector<int> free_slots;
  uint64_t next_ticket = 1;
  bool stopping = false;
  // device state (worker thread only)
  uint8_t* slot_frames = nullptr;
  uint8_t* slot_lost = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<sefase::Scratch> scratch;   // one per stream
  int next_stream = 0;
  std::map<sefase::PatternKey, sefase::CachedTables> cache;
  std::deque<sefase::Batch> inflight;
  size_t bytes_slots = 0, bytes_tables = 0, bytes_scratch = 0;
  // dictionaries prepared for rows on demand, per basis set (on first use;
  // counted with the tables, never evicted)
  std::vector<se_od_dict*> dicts;
  std::vector<bool> dict_tried;
  se_serve_stats stats{};    // published under mu
  se_serve_stats wstats{};   // worker-side counters
  std::thread worker;
};

namespace sefase {

using Server = se_server;

// Whether a basis set can have parity-class tables (the weight pattern's
// symmetry is decided when its tables are built): two transform parts
// covering the dictionary of an even-sided area, K a multiple of 1024 equal
// to the loop's row length.
static bool class_capable(const se_basis& b) {
  if (b.n_parts != 2 || (b.M & 1) || (b.N & 1) || b.K % 1024 || b.K != greedy_row_len(b.K))
    return false;
  int lo[3], hi[3];
  return dense_ranges(b.K, b.M * b.N, b.n_parts, b.parts, lo, hi) == 0;
}

static size_t tables_bytes(const se_basis& b) {
  const int K = b.K, P = b.M * b.N;
  const size_t ld = (size_t)greedy_row_len(K);
  const size_t cls = class_capable(b)
                         ? align_up((size_t)K * (K / 4) * 4, 256) + align_up((size_t)K * 8, 256)
                         : 0;
  return align_up((size_t)K * ld * 4, 256) + align_up((size_t)K * 4, 256) +
         align_up((size_t)K * P * 4, 256) + align_up((size_t)P * 4, 256) +
         align_up(tx_const_bytes(b.M, b.N, b.n_parts), 256) + cls + 256;
}

static void evict_for(Server* s, size_t need);

// The basis set prepared for rows on demand (parts verified and phi squared
// formed once: the one synchronisation of `st` for this basis), or nullptr
// when the budget cannot hold it beside `reserve` bytes of scratch for the
// stream's batch (the batch then takes the one-call form).  Prepared
// dictionaries stay until the server ends and count with the tables.
static se_od_dict* ondemand_dict(Server* s, int bs, int si, hipStream_t st, size_t reserve) {
  if (s->dicts[(size_t)bs]) return s->dicts[(size_t)bs];
  if (s->dict_tried[(size_t)bs]) return nullptr;
  const se_basis& b = s->sets[(size_t)bs];
  const size_t bytes = align_up((size_t)b.K * b.M * b.N * 4, 256) +
                       align_up(tx_const_bytes(b.M, b.N, b.n_parts), 256) + 512;
  const size_t mine = s->scratch[(size_t)si].bytes;
  const size_t scratch = s->bytes_scratch - mine + std::max(mine, reserve);
  if (s->bytes_tables + s->bytes_slots + scratch + bytes > s->cfg.hbm_budget_bytes)
    return nullptr;   // not now (the budget may hold it later)
  se_od_dict* d = nullptr;
  if (se_ondemand_prepare(&b, 0, &d, st) != SE_OK) {
    s->dict_tried[(size_t)bs] = true;   // not preparable: the one-call form from now on
    return nullptr;
  }
  s->dicts[(size_t)bs] = d;
  s->bytes_tables += bytes;
  return d;
}

static void evict_for(Server* s, size_t need) {
  while (s->bytes_tables + s->bytes_slots + s->bytes_scratch + need > s->cfg.hbm_budget_bytes) {
    auto victim = s->cache.end();
    for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
      if (it->second.refs == 0 && (victim == s->cache.end() ||
                                   it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == s->cache.end()) return;
    hipFree(victim->second.mem);
    s->bytes_tables -= victim->second.bytes;
    s->cache.erase(victim);
    s->wstats.table_evictions++;
  }
}

// Scratch of stream i grown to `need` bytes (the stream is drained first).
static se_status ensure_scratch(Server* s, int i, size_t need) {
  Scratch& sc = s->scratch[(size_t)i];
  if (sc.bytes >= need) return SE_OK;
  hipStreamSynchronize(s->streams[(size_t)i]);
  const size_t grow = need - sc.bytes;
  evict_for(s, grow);
  if (s->bytes_tables + s->bytes_slots + s->bytes_scratch + grow > s->cfg.hbm_budget_bytes)
    return fail(SE_ENOMEM, "scratch of %zu bytes exceeds the HBM budget", need);
  if (sc.p) hipFree(sc.p);
  s->bytes_scratch -= sc.bytes;
  sc.p = nullptr;
  sc.bytes = 0;
  if (hipMalloc(&sc.p, need) != hipSuccess) return fail(SE_ENOMEM, "hipMalloc of scratch failed");
  sc.bytes = need;
  s->bytes_scratch += need;
  return SE_OK;
}

// Tables of an isolated pattern: from the cache, or built on stream `st`
// (scratch must hold the small build workspace).  nullptr when the budget
// cannot hold them.
static CachedTables* get_tables(Server* s, const PatternKey& key, hipStream_t st, char* scratch,
                                size_t scratch_bytes) {
  auto it = s->cache.find(key);
  if (it != s->cache.end()) {
    s->wstats.table_hits++;
    it->second.last_use = now_ns();
    return &it->second;
  }
  const se_basis& b = s->sets[(size_t)key.basis];
  const int K = b.K, P = b.M * b.N, ld = greedy_row_len(K);
  const size_t bytes = tables_bytes(b);
  evict_for(s, bytes);
  if (s->bytes_tables + s->bytes_slots + s->bytes_scratch + bytes > s->cfg.hbm_budget_bytes)
    return nullptr;
  void* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) return nullptr;
  char* m = static_cast<char*>(mem);
  CachedTables ct;
  ct.mem = mem;
  ct.bytes = bytes;
  se_tables& t = ct.t;
  t.M = b.M;
  t.N = b.N;
  t.K = K;
  t.ldG = ld;
  size_t off = 0;
  auto take = [&](size_t n) {
    char* p = m + off;
    off += align_up(n, 256);
    return p;
  };
  t.G = reinterpret_cast<float*>(take((size_t)K * ld * 4));
  t.D = reinterpret_cast<float*>(take((size_t)K * 4));
  t.Y = reinterpret_cast<float*>(take((size_t)K * P * 4));
  t.sqrtw = reinterpret_cast<float*>(take((size_t)P * 4));
  t.phi = b.phi;
  t.info = nullptr;
  t.precision = SE_FP32;
  t.Yhi = t.Ylo = nullptr;
  t.tx = b.n_parts > 0 ? reinterpret_cast<float*>(take(tx_const_bytes(b.M, b.N, b.n_parts)))
                       : nullptr;
  if (class_capable(b)) {   // used when the pattern turns out mirror-symmetric
    t.Gc = reinterpret_cast<float*>(take((size_t)K * (K / 4) * 4));
    t.cls = reinterpret_cast<int32_t*>(take((size_t)K * 8));
  }
  // the pattern's weights: an M x N mask with the loss marked, one block at 0,0
  Carver cv(scratch);
  uint8_t* mask = cv.take<uint8_t>((size_t)P);
  float* w = cv.take<float>((size_t)P);
  int4* rect = cv.take<int4>(1);
  char* ws = cv.take<char>(0);
  const size_t ws_left = scratch_bytes > cv.off ? scratch_bytes - cv.off : 0;
  const int4 r = make_int4(key.ly, key.lx, key.lh, key.lw);
  bool ok = hipMemcpyAsync(rect, &r, sizeof(r), hipMemcpyHostToDevice, st) == hipSuccess;
  if (ok) {
    launch_lost_mask(mask, b.M, b.N, rect, 1, st);
    DevBlock blk{0, 0, 0, key.ly, key.lx, key.lh, key.lw, 0, 0, 1};
    DevBlock* dblk = reinterpret_cast<DevBlock*>(ws);
    ok = hipMemcpyAsync(dblk, &blk, sizeof(blk), hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok) {
      launch_area_weights(1, b.M, b.N, s->cfg.rho_hat, mask, b.M, b.N, dblk, 1, w, st);
      ok = se_weighted_gram(&b, w, SE_FP32, SE_DIAG_AUTO, &t, ws + 256, ws_left - 256, st) ==
           SE_OK;
    }
  }
  // the small host sources above must stay valid until the copies ran
  hipStreamSynchronize(st);
  if (!ok) {
    hipFree(mem);
    return nullptr;
  }
  ct.last_use = now_ns();
  s->bytes_tables += bytes;
  s->wstats.table_builds++;
  return &(s->cache[key] = ct);
}

struct Grouped {
  // isolated: pattern + gamma + iters -> blocks
  std::map<std::tuple<PatternKey, float, int>, std::vector<se_block>> iso;
  // own weights: dictionary + gamma -> blocks, per-block iterations
  std::map<std::pair<int, float>, std::pair<std::vector<se_block>, std::vector<int32_t>>> own;
};

// Classify every loss of a request and append its block to a group.
static void group_request(Server* s, Req* r, Grouped& g) {
  const int H = s->cfg.frame_H, W = s->cfg.frame_W;
  const std::vector<se_loss>& L = r->losses;
  // bucket losses by 64-pixel cells for the overlap test
  const int cs = 64, gw = (W + cs - 1) / cs, gh = (H + cs - 1) / cs;
  std::vector<std::vector<int>> cell((size_t)gw * gh);
  for (int i = 0; i < (int)L.size(); ++i)
    for (int cy = L[i].y / cs; cy <= (L[i].y + L[i].h - 1) / cs; ++cy)
      for (int cx = L[i].x / cs; cx <= (L[i].x + L[i].w - 1) / cs; ++cx)
        cell[(size_t)cy * gw + cx].push_back(i);
  int n_iso = 0, n_own = 0;
  for (int i = 0; i < (int)L.size(); ++i) {
    const se_loss& l = L[i];
    const se_basis& b = s->sets[(size_t)l.basis];
    const int ly = (b.M - l.h) / 2, lx = (b.N - l.w) / 2;
    se_block blk{r->slot, l.y - ly, l.x - lx, ly, lx, l.h, l.w, l.basis, 0, 1};
    bool iso = blk.y0 >= 0 && blk.x0 >= 0 && blk.y0 + b.M <= H && blk.x0 + b.N <= W;
    if (iso) {
      const int y1 = blk.y0 + b.M, x1 = blk.x0 + b.N;
      for (int cy = std::max(0, blk.y0 / cs); iso && cy <= std::min(gh - 1, (y1 - 1) / cs); ++cy)
        for (int cx = std::max(0, blk.x0 / cs); iso && cx <= std::min(gw - 1, (x1 - 1) / cs); ++cx)
          for (int j : cell[(size_t)cy * gw + cx]) {
            if (j == i) continue;
            const se_loss& o = L[j];
            if (o.y < y1 && o.y + o.h > blk.y0 && o.x < x1 && o.x + o.w > blk.x0) {
              iso = false;
              break;
            }
          }
    }
    // no available sample: the losses (disjoint) cover every in-frame
    // sample of the area; such a block reports sel = -1, keeps its loss, and
    // the request ends with SE_ENUMERIC
    {
      const int y0 = std::max(blk.y0, 0), y1 = std::min(blk.y0 + b.M, H);
      const int x0 = std::max(blk.x0, 0), x1 = std::min(blk.x0 + b.N, W);
      long long covered = 0;
      std::vector<int> seen;
      for (int cy = y0 / cs; cy <= (y1 - 1) / cs; ++cy)
        for (int cx = x0 / cs; cx <= (x1 - 1) / cs; ++cx)
          for (int j : cell[(size_t)cy * gw + cx]) seen.push_back(j);
      std::sort(seen.begin(), seen.end());
      seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
      for (int j : seen) {
        const se_loss& o = L[j];
        const int h = std::min(o.y + o.h, y1) - std::max(o.y, y0);
        const int w = std::min(o.x + o.w, x1) - std::max(o.x, x0);
        if (h > 0 && w > 0) covered += (long long)h * w;
      }
      if (covered >= (long long)(y1 - y0) * (x1 - x0)) r->n_degenerate++;
    }
    if (iso) {
      g.iso[{PatternKey{l.basis, ly, lx, l.h, l.w}, r->prm.gamma, r->prm.iters}].push_back(blk);
      ++n_iso;
    } else {
      auto& e = g.own[{l.basis, r->prm.gamma}];
      e.first.push_back(blk);
      e.second.push_back(r->prm.iters);
      ++n_own;
    }
  }
  r->res.n_blocks = (int32_t)L.size();
  r->res.n_isolated = n_iso;
  r->res.n_ondemand = n_own;
}

static se_status launch_batch(Server* s, std::vector<Req*>& reqs, Batch& bt) {
  const int si = s->next_stream;
  s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
  hipStream_t st = s->streams[(size_t)si];
  const int H = s->cfg.frame_H, W = s->cfg.frame_W, nslot = s->cfg.max_slots;
  const size_t fb = (size_t)H * W;
  Grouped g;
  size_t n_rects = 0;
  for (Req* r : reqs) {
    group_request(s, r, g);
    n_rects += r->losses.size();
  }
  // scratch: rectangles, then the largest call's workspace (+ weights)
  size_t need = align_up(n_rects * sizeof(int4), 256) + 256;
  size_t call_max = 1 << 20;
  // any isolated group may fall back to the on-demand path (budget), so size
  // the on-demand workspace for every block of a dictionary
  std::map<int, std::pair<int, int>> per_basis;   // basis -> (blocks, max loss)
  std::map<int, int> iters_of;                      // basis -> largest iteration count
  for (auto& e : g.iso) {
    const int bs = std::get<0>(e.first).basis;
    iters_of[bs] = std::max(iters_of[bs], std::get<2>(e.first));
    const se_basis& b = s->sets[(size_t)bs];
    se_tables t{};
    t.M = b.M;
    t.N = b.N;
    t.K = b.K;
    t.precision = SE_FP32;
    t.n_parts = b.n_parts;
    for (int q = 0; q < b.n_parts && q < 2; ++q) t.parts[q] = b.parts[q];
    call_max = std::max(call_max, se_extrapolate_batch_ws_bytes(&t, (int)e.second.size()));
    se_basis bb = b;
    call_max = std::max(call_max, se_weighted_gram_ws_bytes(&bb, SE_FP32) + 4096 +
                                      (size_t)b.M * b.N * 8);
    auto& pb = per_basis[bs];
    pb.first += (int)e.second.size();
    for (auto& bl : e.second) pb.second = std::max(pb.second, bl.lh * bl.lw);
  }
  for (auto& e : g.own) {
    auto& pb = per_basis[e.first.first];
    pb.first += (int)e.second.first.size();
    for (auto& bl : e.second.first) pb.second = std::max(pb.second, bl.lh * bl.lw);
    for (int v : e.second.second) iters_of[e.first.first] = std::max(iters_of[e.first.first], v);
  }
  // with the prepared dictionary, room for every table row a block forms
  // (each formed once: rows on demand with a row cache)
  for (auto& kv : per_basis) {
    const se_basis& b = s->sets[(size_t)kv.first];
    const int n = kv.second.first, ml = std::max(1, kv.second.second);
    const size_t extra = align_up((size_t)n * b.M * b.N * 4, 256) + se_area_weights_ws_bytes(n) + 512;
    call_max = std::max(call_max, se_extrapolate_ondemand_ws_bytes(&b, n, ml) + extra);
  }
  size_t call_cache = call_max;
  for (auto& kv : per_basis) {
    const se_basis& b = s->sets[(size_t)kv.first];
    const int n = kv.second.first, ml = std::max(1, kv.second.second);
    const size_t extra = align_up((size_t)n * b.M * b.N * 4, 256) + se_area_weights_ws_bytes(n) + 512;
    if (se_od_dict* dd = ondemand_dict(s, kv.first, si, st, need + call_max))
      call_cache = std::max(call_cache,
                            se_ondemand_plan_ws_bytes(dd, n, ml, iters_of[kv.first]) + extra);
  }
  // the row cache when the budget holds it, else every row formed on use
  se_status rc = ensure_scratch(s, si, need + call_cache);
  if (rc != SE_OK && call_cache > call_max) rc = ensure_scratch(s, si, need + call_max);
  need += call_max;
  if (rc) return rc;
  char* base = static_cast<char*>(s->scratch[(size_t)si].p);
  int4* rects = reinterpret_cast<int4*>(base);
  char* work = base + align_up(n_rects * sizeof(int4), 256) + 256;
  const size_t work_bytes = s->scratch[(size_t)si].bytes - (size_t)(work - base);

  std::vector<int4> hrect;
  hrect.reserve(n_rects);
  for (Req* r : reqs)
    for (const se_loss& l : r->losses) hrect.push_back(make_int4(l.y, l.x, l.h, l.w));
  if (!hrect.empty() &&
      hipMemcpyAsync(rects, hrect.data(), hrect.size() * sizeof(int4), hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return fail(SE_EHIP, "rectangle upload failed");
  size_t ro = 0;
  for (Req* r : reqs) {
    uint8_t* fr = s->slot_frames + (size_t)r->slot * fb;
    if (hipMemcpyAsync(fr, r->frame, fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(SE_EHIP, "frame copy failed");
    launch_lost_mask(s->slot_lost + (size_t)r->slot * fb, H, W, rects + ro,
                     (int)r->losses.size(), st);
    ro += r->losses.size();
  }
  // isolated blocks: cached tables of their pattern, one batched call each
  for (auto& e : g.iso) {
    const PatternKey& key = std::get<0>(e.first);
    // SE_INVARIANT: a batch mixes requests, and each request's result must
    // not depend on which others share it
    const se_params prm{std::get<1>(e.first), std::get<2>(e.first), SE_INVARIANT};
    CachedTables* ct = get_tables(s, key, st, work, work_bytes);
    std::vector<se_block>& blocks = e.second;
    if (!ct) {   // the budget cannot hold the tables: take the on-demand path
      auto& o = g.own[{key.basis, prm.gamma}];
      o.first.insert(o.first.end(), blocks.begin(), blocks.end());
      o.second.insert(o.second.end(), blocks.size(), prm.iters);
      s->wstats.degraded_blocks += blocks.size();
      continue;
    }
    ct->refs++;
    bt.refs.push_back(key);
    rc = se_extrapolate_batch(&ct->t, s->slot_frames, nslot, H, W, blocks.data(),
                              (int)blocks.size(), prm, nullptr, nullptr, nullptr, 0, work,
                              work_bytes, st);
    if (rc && rc != SE_ENUMERIC) return rc;   // blocks without support: per request below
  }
  // blocks with their own weights: per-block weights, then on-demand rows
  for (auto& e : g.own) {
    const se_basis& b = s->sets[(size_t)e.first.first];
    std::vector<se_block>& blocks = e.second.first;
    const int n = (int)blocks.size();
    Carver cv(work);
    float* w = cv.take<float>((size_t)n * b.M * b.N);
    char* aws = cv.take<char>(se_area_weights_ws_bytes(n));
    char* ows = cv.take<char>(0);
    const size_t ows_bytes = work_bytes - cv.off;
    rc = se_area_weights(b.M, b.N, s->cfg.rho_hat, s->slot_lost, nslot, H, W, blocks.data(), n,
                         w, aws, se_area_weights_ws_bytes(n), st);
    if (rc) return rc;
    const se_params prm{e.first.second, 0, SE_INVARIANT};
    int ml = 1;
    for (auto& bl : blocks) ml = std::max(ml, bl.lh * bl.lw);
    int itmax = 0;
    for (int v : e.second.second) itmax = std::max(itmax, v);
    se_od_dict* dd = s->dicts[(size_t)e.first.first];   // prepared while sizing, if at all
    // every table row cached if the scratch holds it (see the sizing above)
    const int slots = dd && se_ondemand_plan_ws_bytes(dd, n, ml, itmax) <= ows_bytes ? itmax : 0;
    if (dd && se_ondemand_plan_ws_bytes(dd, n, ml, slots) <= ows_bytes)   // no synchronisation
      rc = se_ondemand_extrapolate(dd, w, s->slot_frames, nslot, H, W, blocks.data(), n, prm,
                                   e.second.second.data(), nullptr, nullptr, nullptr, 0, slots,
                                   ows, ows_bytes, st);
    else
      rc = se_extrapolate_ondemand(&b, w, s->slot_frames, nslot, H, W, blocks.data(), n, prm,
                                   e.second.second.data(), nullptr, nullptr, nullptr, 0, ows,
                                   ows_bytes, st);
    if (rc && rc != SE_ENUMERIC) return rc;
  }
  for (Req* r : reqs) {
    if (hipMemcpyAsync(r->frame, s->slot_frames + (size_t)r->slot * fb, fb,
                       hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(SE_EHIP, "frame copy back failed");
  }
  // the host vectors read by pageable copies above were staged during the
  // calls; the event marks the end of the batch
  if (hipEventCreateWithFlags(&bt.done, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(bt.done, st) != hipSuccess)
    return fail(SE_EHIP, "event record failed");
  return SE_OK;
}

static void finish_batch(Server* s, Batch& bt) {
  const uint64_t t = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  for (Req* r : bt.reqs) {
    r->res.status = bt.status != SE_OK ? bt.status : r->n_degenerate ? SE_ENUMERIC : SE_OK;
    r->res.t_done_ns = t;
    r->state = 3;
    s->free_slots.push_back(r->slot);
    s->stats.completed++;
  }
  for (const PatternKey& k : bt.refs) {
    auto it = s->cache.find(k);
    if (it != s->cache.end()) it->second.refs--;
  }
  if (bt.done) hipEventDestroy(bt.done);
  s->cv_done.notify_all();
}

static void worker_main(Server* s) {
  hipSetDevice(s->cfg.device);
  for (;;) {
    std::vector<Req*> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(100), [&] {
        return s->stopping || !s->inflight.empty() ||
               (!s->queue.empty() && !s->free_slots.empty());
      });
      while (!s->queue.empty() && !s->free_slots.empty()) {
        Req* r = s->queue.front();
        s->queue.pop_front();
        r->slot = s->free_slots.back();
        s->free_slots.pop_back();
        r->state = 1;
        r->res.t_admit_ns = now_ns();
        batch.push_back(r);
      }
      if (s->stopping && s->queue.empty() && s->inflight.empty() && batch.empty()) break;
    }
    if (!batch.empty()) {
      Batch bt;
      bt.reqs = batch;
      for (Req* r : batch) r->state = 2;
      const se_status rc = launch_batch(s, batch, bt);
      s->wstats.batches++;
      if (rc != SE_OK) {
        bt.status = rc;
        // whatever was launched must finish before the slots are reused
        for (hipStream_t st : s->streams) hipStreamSynchronize(st);
        if (bt.done) hipEventDestroy(bt.done);
        bt.done = nullptr;
        finish_batch(s, bt);
      } else {
        s->inflight.push_back(bt);
      }
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stats.batches = s->wstats.batches;
      s->stats.table_hits = s->wstats.table_hits;
      s->stats.table_builds = s->wstats.table_builds;
      s->stats.table_evictions = s->wstats.table_evictions;
      s->stats.degraded_blocks = s->wstats.degraded_blocks;
      s->stats.bytes_tables = s->bytes_tables;
      s->stats.bytes_slots = s->bytes_slots;
      s->stats.bytes_scratch = s->bytes_scratch;
    }
    // retire finished batches (query every one)
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
      if (hipEventQuery(it->done) == hipSuccess) {
        finish_batch(s, *it);
        it = s->inflight.erase(it);
      } else {
        ++it;
      }
    }
  }
}

static se_status validate_request(Server* s, const se_request* r) {
  if (!r || !r->frame) return fail(SE_EINVAL, "NULL request or frame");
  if (r->H != s->cfg.frame_H || r->W != s->cfg.frame_W)
    return fail(SE_EINVAL, "frame %dx%d differs from the served %dx%d", r->H, r->W,
                s->cfg.frame_H, s->cfg.frame_W);
  if (r->n_losses < 0 || (r->n_losses > 0 && !r->losses)) return fail(SE_EINVAL, "bad loss list");
  if (!(r->prm.gamma > 0.0f && r->prm.gamma <= 1.0f) || r->prm.iters < 0 || r->prm.flags)
    return fail(SE_EINVAL, "bad parameters");
  for (int i = 0; i < r->n_losses; ++i) {
    const se_loss& l = r->losses[i];
    if (l.basis < 0 || l.basis >= (int)s->sets.size()) return fail(SE_EINVAL, "loss %d: unknown basis", i);
    const se_basis& b = s->sets[(size_t)l.basis];
    if (l.h < 1 || l.w < 1 || l.h > b.M || l.w > b.N)
      return fail(SE_EINVAL, "loss %d: %dx%d does not fit the %dx%d area", i, l.h, l.w, b.M, b.N);
    if (l.h * l.w > 256 * greedy_waves_for(b.K))
      return fail(SE_EINVAL, "loss %d: too many pixels", i);
    if (l.y < 0 || l.x < 0 || l.y + l.h > r->H || l.x + l.w > r->W)
      return fail(SE_EINVAL, "loss %d outside the frame", i);
  }
  // losses must not overlap (each lost pixel belongs to one block)
  std::vector<int> idx((size_t)r->n_losses);
  for (int i = 0; i < r->n_losses; ++i) idx[(size_t)i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return r->losses[a].y < r->losses[b].y; });
  for (size_t a = 0; a < idx.size(); ++a) {
    const se_loss& p = r->losses[idx[a]];
    for (size_t c = a + 1; c < idx.size(); ++c) {
      const se_loss& q = r->losses[idx[c]];
      if (q.y >= p.y + p.h) break;
      if (q.x < p.x + p.w && q.x + q.w > p.x) return fail(SE_EINVAL, "losses overlap");
    }
  }
  return SE_OK;
}

}  // namespace sefase

using namespace sefase;

extern "C" {

se_status se_serve_create(const se_serve_config* cfg, const se_basis* sets, int32_t n_sets,
                          se_server** out) {
  if (!cfg || !out || !sets || n_sets < 1) return fail(SE_EINVAL, "NULL argument");
  if (cfg->frame_H < 1 || cfg->frame_W < 1 || cfg->max_slots < 1 || cfg->max_queue < 1 ||
      cfg->n_streams < 1 || cfg->n_streams > 8 || !(cfg->rho_hat > 0.0f && cfg->rho_hat <= 1.0f))
    return fail(SE_EINVAL, "bad server configuration");
  for (int i = 0; i < n_sets; ++i)
    if (!sets[i].phi || sets[i].M < 1 || sets[i].N < 1 || sets[i].K < 1 ||
        greedy_waves_for(sets[i].K) == 0)
      return fail(SE_EINVAL, "basis set %d invalid", i);
  for (int i = 0; i < n_sets; ++i) {
    if (se_status st = check_basis_parts(&sets[i])) return st;
    if (sets[i].phi_im) return fail(SE_EINVAL, "basis set %d: the server takes real dictionaries", i);
    if (sets[i].T > 1)
      return fail(SE_EINVAL, "basis set %d: the server takes two-dimensional areas", i);
  }
  if (hipSetDevice(cfg->device) != hipSuccess) return fail(SE_EHIP, "hipSetDevice failed");
  std::unique_ptr<se_server> s(new se_server());
  s->cfg = *cfg;
  s->sets.assign(sets, sets + n_sets);
  s->dicts.assign((size_t)n_sets, nullptr);
  s->dict_tried.assign((size_t)n_sets, false);
  const size_t fb = (size_t)cfg->frame_H * cfg->frame_W;
  s->bytes_slots = 2 * fb * (size_t)cfg->max_slots;
  if (s->bytes_slots > cfg->hbm_budget_bytes) return fail(SE_ENOMEM, "slots exceed the budget");
  if (hipMalloc(reinterpret_cast<void**>(&s->slot_frames), fb * cfg->max_slots) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->slot_lost), fb * cfg->max_slots) != hipSuccess)
    return fail(SE_ENOMEM, "slot allocation failed");
  s->streams.resize((size_t)cfg->n_streams);
  s->scratch.resize((size_t)cfg->n_streams);
  for (auto& st : s->streams)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return fail(SE_EHIP, "stream creation failed");
  for (int i = cfg->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->worker = std::thread(worker_main, s.get());
  *out = s.release();
  return SE_OK;
}

se_status se_serve_submit(se_server* s, const se_request* r, uint64_t* ticket) {
  if (!s || !ticket) return fail(SE_EINVAL, "NULL argument");
  se_status rc = validate_request(s, r);
  if (rc) return rc;
  std::unique_ptr<Req> q(new Req());
  q->frame = r->frame;
  q->losses.assign(r->losses, r->losses + r->n_losses);
  q->prm = r->prm;
  q->res.t_submit_ns = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail(SE_ECANCELED, "server is shutting down");
  if ((int)s->queue.size() >= s->cfg.max_queue) return fail(SE_EBUSY, "queue full");
  q->ticket = s->next_ticket++;
  *ticket = q->ticket;
  s->queue.push_back(q.get());
  s->reqs[q->ticket] = std::move(q);
  s->stats.submitted++;
  s->cv_work.notify_one();
  return SE_OK;
}

static se_status take_result(se_server* s, uint64_t ticket, se_result* out, bool wait) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(SE_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Req* q = it->second.get();   // map iterators do not survive concurrent submits
  if (wait) s->cv_done.wait(lk, [&] { return q->state == 3; });
  if (q->state != 3) return SE_EAGAIN;
  if (out) *out = q->res;
  s->reqs.erase(ticket);
  return SE_OK;
}

se_status se_serve_poll(se_server* s, uint64_t ticket, se_result* out) {
  if (!s) return fail(SE_EINVAL, "NULL server");
  return take_result(s, ticket, out, false);
}

se_status se_serve_wait(se_server* s, uint64_t ticket, se_result* out) {
  if (!s) return fail(SE_EINVAL, "NULL server");
  return take_result(s, ticket, out, true);
}

se_status se_serve_stats_get(se_server* s, se_serve_stats* out) {
  if (!s || !out) return fail(SE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return SE_OK;
}

se_status se_serve_destroy(se_server* s) {
  if (!s) return fail(SE_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (hipStream_t st : s->streams) hipStreamSynchronize(st);
  for (auto& kv : s->cache) hipFree(kv.second.mem);
  for (se_od_dict* d : s->dicts) se_ondemand_release(d);
  for (auto& sc : s->scratch)
    if (sc.p) hipFree(sc.p);
  for (hipStream_t st : s->streams) hipStreamDestroy(st);
  hipFree(s->slot_frames);
  hipFree(s->slot_lost);
  delete s;
  return SE_OK;
}

}  // extern "C"
