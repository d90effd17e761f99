// Stream table: batched generation of many streams of mixed kinds and uneven
// lengths (include/prng.h, prng_table_*).  Planning, jump-ahead segmentation,
// workspace layout, graph capture and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <vector>

#include "host.h"
#include "jump.h"

using namespace prng;

// ================================================================ stream table
// Batched generation (not in the paper, whose instances are independent and
// launched together): rows of (generator object, stream, count, dtype,
// output buffer) are planned into wave-sized tasks and run by two persistent
// kernels (lane-per-stream kinds; MT19937), optionally captured into a graph.
// Long rows are cut into segments that start from jumped-ahead states, so that
// no single lane (or, for MT19937, workgroup) carries a whole long stream.
namespace {


// relative cost of one draw, used only to order tasks longest first
double draw_cost(int kind, uint32_t p) {
  switch (kind) {
    case RANMAR:
      return 1.1;
    case RANLUX:
      return 1.5 + (p > 24 ? (p - 24) / 24.0 * 0.35 : 0.0);
    case MT19937:
      return 1.3;
    default:
      return 1.0;
  }
}

constexpr uint32_t kSegAlign = 384;             // multiple of 24 (luxury blocks) and of 128 (chunks)
constexpr uint32_t kSegAuto = 0, kSegNever = 0xFFFFFFFFu;
constexpr uint64_t kMaxSegments = 4096;         // per row

std::mutex g_tune_mu;
std::map<std::tuple<uint64_t, uint64_t, uint64_t, uint64_t>, TableConfig> g_tune_cache;

struct RowRef {
  prng_gen* g;
  uint64_t stream;
  void* out;
  uint32_t draws;
  int dtype;
};

}  // namespace

int prng::make_plan(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows, const SegSpec& seg,
                    const JumpSource* js, Plan& P) {
  if (!gens || n_gens <= 0) return fail(PRNG_EINVAL, "no generator objects");
  if (!rows && n_rows) return fail(PRNG_EINVAL, "rows is NULL");
  for (int i = 0; i < n_gens; ++i)
    if (!gens[i]) return fail(PRNG_EINVAL, "generator %d is NULL", i);
  std::vector<RowRef> all;
  all.reserve(n_rows);
  std::set<std::pair<const uint32_t*, uint64_t>> seen;
  uint64_t lane_draws = 0;
  for (uint64_t i = 0; i < n_rows; ++i) {
    const prng_table_row& r = rows[i];
    if (r.gen >= (uint32_t)n_gens) return fail(PRNG_EINVAL, "row %llu: generator index out of range", (unsigned long long)i);
    prng_gen* g = gens[r.gen];
    if (r.dtype < U32 || r.dtype > F64) return fail(PRNG_EINVAL, "row %llu: unknown dtype", (unsigned long long)i);
    if (r.stream >= g->n) return fail(PRNG_EINVAL, "row %llu: stream out of range", (unsigned long long)i);
    if (r.count == 0) continue;
    const uint64_t per = r.dtype == F64 ? 2 : 1;
    if (r.count > kMaxDrawsPerLaunch / per)
      return fail(PRNG_EINVAL, "row %llu: count too large for one run", (unsigned long long)i);
    if (!r.d_out || (reinterpret_cast<uintptr_t>(r.d_out) % elem_bytes(r.dtype)))
      return fail(PRNG_EINVAL, "row %llu: output pointer NULL or misaligned", (unsigned long long)i);
    if (!seen.insert({g->d_state, r.stream}).second)
      return fail(PRNG_EINVAL, "row %llu: stream listed twice", (unsigned long long)i);
    const uint32_t d = (uint32_t)(r.count * per);
    all.push_back(RowRef{g, r.stream, r.d_out, d, (int)r.dtype});
    if (std::find(P.gens.begin(), P.gens.end(), g) == P.gens.end()) P.gens.push_back(g);
    P.total_draws += d;
    P.max_draws = std::max<uint64_t>(P.max_draws, d);
    if (g->kind != MT19937) lane_draws += d;
  }
  // ---- segment length per kind
  auto roundup = [](uint64_t v, uint64_t a) { return (v + a - 1) / a * a; };
  const uint64_t lane_auto = roundup(std::max<uint64_t>(lane_draws / 524288, 1536), kSegAlign);
  // MT19937 segments run on a workgroup and a jump costs about as much as 2^18
  // draws of one CU, so only rows far longer than the table's average share
  // of a workgroup are cut: at about 1/3200 of the table's draws
  const uint64_t mt_auto = roundup(std::min<uint64_t>(std::max<uint64_t>(P.total_draws / 3200, 1u << 18), 1u << 22),
                                   624);
  auto resolve = [&](uint32_t v, uint64_t automatic, uint64_t lo, uint64_t align) -> uint64_t {
    if (v == kSegNever) return 0;
    if (v == kSegAuto) return automatic;
    return roundup(std::max<uint64_t>(v, lo), align);
  };
  // RANMAR's jump costs ~20k operations: automatically four lane lengths
  const uint64_t L_lane = resolve(seg.lane, lane_auto, kSegAlign, kSegAlign);
  const uint64_t L_ranmar = resolve(seg.ranmar, 4 * lane_auto, kSegAlign, kSegAlign);
  const uint64_t L_mt = resolve(seg.mt, mt_auto, 1248, 624);
  P.resolved = SegSpec{(uint32_t)std::min<uint64_t>(L_lane, 0xFFFFFFFEu),
                       (uint32_t)std::min<uint64_t>(L_ranmar, 0xFFFFFFFEu), (uint32_t)std::min<uint64_t>(L_mt, 0xFFFFFFFEu)};
  // RANLUX shares the lane length scaled by its cost per draw (at least one
  // 384-position unit), so that its tasks take about as long as the others'
  auto seg_for = [&](int kind, uint32_t p) -> uint64_t {
    if (js) return js->seg_len(kind);
    if (kind == MT19937) return L_mt;
    if (kind == RANMAR) return L_ranmar;
    if (kind == RANLUX && L_lane)
      return std::max<uint64_t>(roundup((uint64_t)((double)L_lane / draw_cost(RANLUX, p)), kSegAlign), kSegAlign);
    return L_lane;
  };
  // ---- rows longer than one segment are cut; a cut row reads a snapshot
  std::vector<uint64_t> Lrow(all.size(), 0);
  std::vector<uint32_t> Krow(all.size(), 1);
  std::vector<int64_t> snap_of(all.size(), -1);
  std::map<std::tuple<int, uint32_t, uint64_t>, uint64_t> jump_base;  // (kind, p, L) -> word offset of j = 1
  std::map<std::tuple<int, uint32_t, uint64_t>, uint32_t> jump_count;
  uint64_t n_lane_snaps = 0, n_mt_snaps = 0;
  for (uint64_t i = 0; i < all.size(); ++i) {
    const int k = all[i].g->kind;
    uint64_t L = seg_for(k, all[i].g->p);
    const uint64_t D = all[i].draws;
    // (with resident jump tables the limit is theirs: checked at the lookup below)
    if (L && !js && (D + L - 1) / L > kMaxSegments)
      L = roundup((D + kMaxSegments - 1) / kMaxSegments, k == MT19937 ? 624 : kSegAlign);
    const uint64_t K = L ? (D + L - 1) / L : 1;  // (K - 1) L < D: the last segment is never empty
    if (K < 2) continue;
    Lrow[i] = L;
    Krow[i] = (uint32_t)K;
    if (k == MT19937) {
      snap_of[i] = (int64_t)n_mt_snaps++;
      P.snaps.push_back(SnapRow{all[i].g->d_state, 0, all[i].stream, nullptr, 0, (uint64_t)snap_of[i],
                                (uint32_t)kStateWords[k], 1u});
    } else {
      snap_of[i] = (int64_t)n_lane_snaps++;
      P.snaps.push_back(SnapRow{all[i].g->d_state, all[i].g->n, all[i].stream, nullptr, 0, (uint64_t)snap_of[i],
                                (uint32_t)kStateWords[k], 0u});
    }
    const auto key = std::make_tuple(k, all[i].g->p, L);
    jump_count[key] = std::max<uint32_t>(jump_count[key], (uint32_t)K - 1);
  }
  // jump data for every (kind, p, L): segment j starts J_j positions ahead
  for (auto& kc : jump_count) {
    if (js) break;
    const int k = std::get<0>(kc.first);
    const uint32_t p = std::get<1>(kc.first);
    const uint64_t L = std::get<2>(kc.first);
    const uint32_t nj = kc.second, stride = jump_slot_words(k);
    jump_base[kc.first] = P.jump.size();
    P.jump.resize(P.jump.size() + (size_t)nj * stride, 0u);
    if (!fill_jumps(k, p, L, nj, P.jump.data() + jump_base[kc.first]))
      return fail(PRNG_EINVAL, "no jump data for kind %d at segment length %llu", k, (unsigned long long)L);
  }
  bool need_aux = false;
  for (auto& kc : jump_count)
    if (std::get<0>(kc.first) == RANLUX) need_aux = true;
  if (need_aux && js) P.ext_aux = js->aux();
  if (need_aux && !js) {
    P.aux.resize(kRanluxAuxWords);
    fill_ranlux_aux(P.aux.data());
  }
  // ---- one descriptor per row, grouped by (kind, p, dtype), longest first;
  // the segments of a group are numbered through its rows in that order
  std::vector<uint64_t> order(all.size());
  for (uint64_t i = 0; i < order.size(); ++i) order[i] = i;
  auto gkey = [&](uint64_t i) { return std::make_tuple(all[i].g->kind, all[i].g->p, all[i].dtype); };
  std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
    if (gkey(a) != gkey(b)) return gkey(a) < gkey(b);
    if (all[a].draws != all[b].draws) return all[a].draws > all[b].draws;
    return a < b;
  });
  struct TP {
    double cost;
    TableTask task;
  };
  std::vector<TP> lane_plan[kLaneClasses], mt_plan;
  uint64_t gi = 0;
  while (gi < order.size()) {
    uint64_t ge = gi;
    while (ge < order.size() && gkey(order[ge]) == gkey(order[gi])) ++ge;
    const int k = all[order[gi]].g->kind;
    const uint32_t lux = all[order[gi]].g->p;
    const uint32_t dt = (uint32_t)all[order[gi]].dtype;
    const uint32_t r0 = (uint32_t)P.rows.size();
    uint64_t gcount = 0;
    for (uint64_t q = gi; q < ge; ++q) {
      const uint64_t i = order[q];
      const RowRef& rr = all[i];
      const bool split = Krow[i] > 1;
      TableRow tr{};
      if (split) {
        tr.state = nullptr;  // patched: snapshot area
        tr.sn = k == MT19937 ? 0 : n_lane_snaps;
        tr.si = (uint64_t)snap_of[i];
      } else {
        tr.state = rr.g->d_state;
        tr.sn = rr.g->n;
        tr.si = rr.stream;
      }
      tr.wstate = rr.g->d_state;
      tr.wsn = rr.g->n;
      tr.wsi = rr.stream;
      tr.out = rr.out;
      tr.draws = rr.draws;
      tr.seg_len = (uint32_t)Lrow[i];
      tr.first = gcount;  // full segments: cut rows come first (longest first, one L per kind)
      tr.nseg = Krow[i];
      tr.jstride = jump_slot_words(k);
      tr.jump = nullptr;
      tr.jstate = nullptr;
      int64_t jo = -1, slot = -1;
      if (split) {
        if (js) {
          tr.jump = js->lookup(k, rr.g->p, 1);
          if (!tr.jump || !js->lookup(k, rr.g->p, Krow[i] - 1))
            return fail(PRNG_EINVAL, "no jump data for %u segments", Krow[i]);
        } else {
          jo = (int64_t)jump_base[std::make_tuple(k, rr.g->p, Lrow[i])];
        }
        if (k == MT19937) {
          slot = (int64_t)P.n_jslots;
          P.n_jslots += Krow[i] - 1;
          for (uint32_t j = 1; j < Krow[i]; ++j) {
            P.mt_jump_list.push_back((uint32_t)P.rows.size());
            P.mt_jump_list.push_back(j);
          }
        }
      }
      P.rows.push_back(tr);
      P.row_snap.push_back(split ? (k == MT19937 ? 2 : 1) : 0);
      P.row_jump.push_back(jo);
      P.row_jslot.push_back(slot);
      gcount += Krow[i] - 1;
      P.n_segments += Krow[i];
    }
    // tasks of this group
    if (k == MT19937) {
      for (uint32_t r = r0; r < (uint32_t)P.rows.size(); ++r) {
        const TableRow& tr = P.rows[r];
        for (uint32_t j = 0; j < tr.nseg; ++j) {
          const uint64_t len = tr.nseg > 1 ? std::min<uint64_t>(tr.seg_len, tr.draws) : tr.draws;
          mt_plan.push_back(TP{len * draw_cost(k, lux) + (j ? 3000.0 : 0.0),
                               TableTask{(uint32_t)k, lux, dt, 1u, j, r, r, 0u, 0u}});
          P.max_task_draws = std::max<uint64_t>(P.max_task_draws, len);
        }
      }
    } else {
      // full segments (all of length L up to a draw): 64 per task, row by row
      uint32_t r = r0;
      for (uint64_t g0 = 0; g0 < gcount; g0 += 64) {
        const uint64_t g1 = std::min<uint64_t>(g0 + 64, gcount) - 1;  // last segment of the task
        while (P.rows[r].first + P.rows[r].nseg - 1 <= g0) ++r;
        uint32_t re = r;
        while (P.rows[re].first + P.rows[re].nseg - 1 <= g1) ++re;
        const uint64_t len = P.rows[r].seg_len;
        lane_plan[lane_class(k)].push_back(TP{len * draw_cost(k, lux) + 3000.0,
                                              TableTask{(uint32_t)k, lux, dt, (uint32_t)(g1 - g0 + 1), g0, r, re,
                                                        0u, 0u}});
        P.max_task_draws = std::max<uint64_t>(P.max_task_draws, len);
      }
      // the group's tail: every row's last segment, longest first, 64 per task
      std::vector<std::pair<uint64_t, uint32_t>> tail;  // (length, row)
      for (uint32_t q = r0; q < (uint32_t)P.rows.size(); ++q) {
        const TableRow& tr = P.rows[q];
        tail.push_back({tr.draws - (uint64_t)(tr.nseg - 1) * tr.seg_len, q});
      }
      std::stable_sort(tail.begin(), tail.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      for (size_t t0 = 0; t0 < tail.size(); t0 += 64) {
        const size_t t1 = std::min(t0 + 64, tail.size());
        const uint64_t at = P.tails.size();
        for (size_t q = t0; q < t1; ++q) P.tails.push_back(tail[q].second);
        lane_plan[lane_class(k)].push_back(TP{tail[t0].first * draw_cost(k, lux),
                                              TableTask{(uint32_t)k, lux, dt, (uint32_t)(t1 - t0), at, 0u, 0u, 1u,
                                                        0u}});
        P.max_task_draws = std::max<uint64_t>(P.max_task_draws, tail[t0].first);
      }
    }
    gi = ge;
  }
  auto by_cost = [](const TP& x, const TP& y) { return x.cost > y.cost; };
  for (int c = 0; c < kLaneClasses; ++c) {
    std::stable_sort(lane_plan[c].begin(), lane_plan[c].end(), by_cost);
    for (auto& t : lane_plan[c]) P.lane_tasks[c].push_back(t.task);
  }
  std::stable_sort(mt_plan.begin(), mt_plan.end(), by_cost);
  for (auto& t : mt_plan) P.mt_tasks.push_back(t.task);
  // ---- workspace layout
  size_t off = 256;  // task counters: the lane classes, then MT
  for (int c = 0; c < kLaneClasses; ++c) {
    P.o_lane[c] = off;
    off += align256(P.lane_tasks[c].size() * sizeof(TableTask));
  }
  P.o_mt = off;
  off += align256(P.mt_tasks.size() * sizeof(TableTask));
  P.o_rows = off;
  off += align256(P.rows.size() * sizeof(TableRow));
  P.o_snaprows = off;
  off += align256(P.snaps.size() * sizeof(SnapRow));
  P.o_snap = off;
  off += align256(n_lane_snaps * 98ull * 4ull);
  P.o_snap_mt = off;
  off += align256(n_mt_snaps * (uint64_t)kMtStride * 4ull);
  P.o_jstate = off;
  off += align256(P.n_jslots * (uint64_t)kMtStride * 4ull);
  P.o_mtj = off;
  off += align256(P.mt_jump_list.size() * 4ull);
  P.o_tails = off;
  off += align256(P.tails.size() * 4ull);
  P.o_jump = off;
  off += align256(P.jump.size() * 4ull);
  P.o_aux = off;
  off += align256(P.aux.size() * 4ull);
  P.total = off;
  return PRNG_OK;
}

namespace {

void drop_graph(prng_table* t) {
  if (t->exec) (void)hipGraphExecDestroy(t->exec);
  if (t->graph) (void)hipGraphDestroy(t->graph);
  t->exec = nullptr;
  t->graph = nullptr;
}

}  // namespace

// Enqueue one run: reset counters, copy the starting states of split streams,
// build the jumped MT19937 windows, then the persistent kernels.  cfg.concurrent
// 0: all of them one after the other; 1: the lane classes one after the
// other, MT19937 beside them on a forked stream; 2: MT19937 and every lane
// class on a stream of its own, so that a class with few tasks (RANMAR, one
// wavefront per SIMD) leaves the rest of the chip to the others; 3: as 2, but
// the lane classes start before the MT19937 jumps, which run on MT19937's
// stream (a few 1024-thread blocks with 88 KB of LDS each that otherwise hold
// the chip alone).  Forked streams join `s` at the end.
hipError_t prng::enqueue_run(prng_table* t, hipStream_t s) {
  hipError_t e = launch_table_prepare(t->d_counters, kLaneClasses + 1, t->d_snaps, t->n_snaps, t->snap_words, s);
  if (e != hipSuccess) return e;
  int used = 0;  // kernels to launch
  for (int c = 0; c < kLaneClasses; ++c) used += t->n_class_tasks[c] ? 1 : 0;
  used += t->n_mt_tasks ? 1 : 0;
  const int mode = used > 1 ? t->cfg.concurrent : 0;
  // Modes 2 and 3: a persistent kernel fills whatever CUs are free, so the one
  // dispatched first holds most of the chip until its list runs dry.  RANMAR's
  // class (few wavefronts, long tasks) goes first, on `s` itself, where it
  // does not wait for the fork event; the other kernels fill the rest.
  const int primary = mode >= 2 && t->n_class_tasks[1] ? 1 : 0;
  // kernel k: lane class k < kLaneClasses, MT19937 for k == kLaneClasses;
  // side slot of a lane class other than the primary one (-1: on `s`)
  auto slot_of = [&](int k) -> int {
    if (k == kLaneClasses || mode < 2 || k == primary) return -1;
    const int slot = k < primary ? k : k - 1;
    return t->lane_side[slot] ? slot : -1;
  };
  auto stream_of = [&](int k) -> hipStream_t {
    if (k == kLaneClasses) return mode >= 1 && t->side ? t->side : s;
    const int slot = slot_of(k);
    return slot < 0 ? s : t->lane_side[slot];
  };
  auto ran = [&](int k) { return k == kLaneClasses ? t->n_mt_tasks != 0 : t->n_class_tasks[k] != 0; };
  // every forked stream waits for one event recorded on `s` before any of the
  // persistent kernels is enqueued there
  bool forked = false;
  auto fork_all = [&]() -> hipError_t {
    for (int k = 0; k <= kLaneClasses; ++k) {
      const hipStream_t x = stream_of(k);
      if (!ran(k) || x == s) continue;
      if (!forked) {
        hipError_t r = hipEventRecord(t->fork, s);
        if (r != hipSuccess) return r;
        forked = true;
      }
      hipError_t r = hipStreamWaitEvent(x, t->fork, 0);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  // cfg.lane_grid: blocks of the one-per-CU class; 256 fill the chip
  auto lane_grid_of = [&](int c) {
    const int full = kClassFullGrid[c] * t->cfg.lane_grid / 256;
    return std::max(1, std::min<int>(full, (int)((t->n_class_tasks[c] + 3) / 4)));
  };
  // Modes 2 and 3: the other kernels leave room for the primary class's
  // blocks (one per CU at most), whatever order the dispatchers start them
  // in; otherwise persistent blocks that arrived first would keep it waiting
  // until their lists ran dry.
  const int reserved = mode >= 2 ? std::min(192, lane_grid_of(primary) * 256 / kClassFullGrid[primary]) : 0;
  auto launch_lane = [&](int c) -> hipError_t {
    const uint32_t n = t->n_class_tasks[c];
    if (!n) return hipSuccess;
    int g = lane_grid_of(c);
    if (mode >= 2 && c != primary) g = std::max(1, g * (256 - reserved) / 256);
    return launch_table_lane(c, t->d_class_tasks[c], n, t->d_rows, t->d_tails, t->d_counters + c, t->d_aux, g,
                             stream_of(c));
  };
  // mode 3: the lane classes do not wait for the MT19937 jumps, which run on
  // MT19937's stream; otherwise the jumps come first, over the whole chip
  if (mode == 3 && (e = fork_all()) != hipSuccess) return e;
  const hipStream_t xj = mode == 3 && t->n_mt_tasks ? stream_of(kLaneClasses) : s;
  if ((e = launch_table_mt_jump(t->d_mt_jumps, t->n_mt_jumps, t->d_rows, xj)) != hipSuccess) return e;
  if (mode != 3 && (e = fork_all()) != hipSuccess) return e;
  if (mode >= 2 && (e = launch_lane(primary)) != hipSuccess) return e;
  if (t->n_mt_tasks) {  // beside the lane kernels (5 KB of LDS per block)
    int g = std::min<int>(t->cfg.mt_grid, (int)t->n_mt_tasks);  // one task per workgroup
    if (mode >= 2) g = std::max(1, g * (256 - reserved) / 256);
    if ((e = launch_table_mt(t->d_mt_tasks, t->n_mt_tasks, t->d_rows, t->d_counters + kLaneClasses, g,
                             stream_of(kLaneClasses))) != hipSuccess)
      return e;
  }
  for (int c = 0; c < kLaneClasses; ++c)
    if (!(mode >= 2 && c == primary) && (e = launch_lane(c)) != hipSuccess) return e;
  // join: each forked stream records its own event, `s` waits for all
  for (int k = 0; forked && k <= kLaneClasses; ++k) {
    const hipStream_t x = stream_of(k);
    if (!ran(k) || x == s) continue;
    hipEvent_t j = k == kLaneClasses ? t->join : t->lane_join[slot_of(k)];
    if ((e = hipEventRecord(j, x)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, j, 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {
SegSpec spec_of(const prng_seg_lengths* seg) {
  return seg ? SegSpec{seg->lane, seg->ranmar, seg->mt} : SegSpec{};
}

size_t work_bytes_for(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows,
                      const SegSpec& seg) {
  try {
    Plan P;
    if (make_plan(gens, n_gens, rows, n_rows, seg, nullptr, P) != PRNG_OK) return 0;
    return P.total;
  } catch (const std::bad_alloc&) {
    fail(PRNG_ENOMEM, "out of host memory");
    return 0;
  }
}

// Lengths halved (a class that is not cut stays so); halving stops at the
// rounding minimum.
SegSpec halved(const SegSpec& a) {
  auto h = [](uint32_t v, uint32_t lo) { return v == 0 ? 0u : std::max(v / 2, lo); };
  return SegSpec{h(a.lane, kSegAlign), h(a.ranmar, kSegAlign), h(a.mt, 1248)};
}
// explicit lengths for make_plan: 0 (not cut) becomes PRNG_SEG_NEVER
SegSpec explicit_spec(const SegSpec& a) {
  auto e = [](uint32_t v) { return v == 0 ? kSegNever : v; };
  return SegSpec{e(a.lane), e(a.ranmar), e(a.mt)};
}
}  // namespace

PRNG_API size_t prng_table_work_bytes(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows,
                                      uint32_t seg_len) {
  return work_bytes_for(gens, n_gens, rows, n_rows, seg_spec_of(seg_len));
}

PRNG_API size_t prng_table_work_bytes_ex(prng_gen* const* gens, int n_gens, const prng_table_row* rows,
                                         uint64_t n_rows, const prng_seg_lengths* seg) {
  return work_bytes_for(gens, n_gens, rows, n_rows, spec_of(seg));
}

PRNG_API size_t prng_table_tune_work_bytes(prng_gen* const* gens, int n_gens, const prng_table_row* rows,
                                           uint64_t n_rows) {
  try {
    Plan P;
    if (make_plan(gens, n_gens, rows, n_rows, SegSpec{}, nullptr, P) != PRNG_OK) return 0;
    // the shortest candidates cut most: their plan needs the most workspace
    return std::max(P.total, work_bytes_for(gens, n_gens, rows, n_rows, explicit_spec(halved(P.resolved))));
  } catch (const std::bad_alloc&) {
    fail(PRNG_ENOMEM, "out of host memory");
    return 0;
  }
}

int prng::table_from_plan(Plan& P, void* d_work, hipStream_t s, bool sync, bool graph_streams, prng_table** out) {
  std::unique_ptr<prng_table> t(new prng_table());
  t->seg = P.resolved;
  char* w = static_cast<char*>(d_work);
  uint32_t* snap = reinterpret_cast<uint32_t*>(w + P.o_snap);
  uint32_t* snap_mt = reinterpret_cast<uint32_t*>(w + P.o_snap_mt);
  uint32_t* jstate = reinterpret_cast<uint32_t*>(w + P.o_jstate);
  const uint32_t* jump = reinterpret_cast<const uint32_t*>(w + P.o_jump);
  const uint64_t ns = P.snaps.size();
  uint64_t n_lane_snaps = 0;
  for (const SnapRow& r : P.snaps) n_lane_snaps += r.aos ? 0 : 1;
  bool mt_snaps = false;
  for (uint64_t i = 0; i < ns; ++i) {
    if (P.snaps[i].aos) {
      P.snaps[i].dst = snap_mt;  // di = MT snapshot index (set by the plan)
      mt_snaps = true;
    } else {
      P.snaps[i].dst = snap;
      P.snaps[i].dn = n_lane_snaps;
    }
  }
  for (uint64_t i = 0; i < P.rows.size(); ++i) {
    if (P.row_snap[i] == 1) P.rows[i].state = snap;     // sn = lane snapshots, si = index (set by the plan)
    if (P.row_snap[i] == 2) P.rows[i].state = snap_mt;  // si = MT snapshot index
    if (P.row_jump[i] >= 0) P.rows[i].jump = jump + P.row_jump[i];
    if (P.row_jslot[i] >= 0) P.rows[i].jstate = jstate + (uint64_t)P.row_jslot[i] * kMtStride;
  }
  t->gens = P.gens;
  for (int c = 0; c < kLaneClasses; ++c) {
    t->n_class_tasks[c] = (uint32_t)P.lane_tasks[c].size();
    t->d_class_tasks[c] = reinterpret_cast<TableTask*>(w + P.o_lane[c]);
    t->n_lane_tasks += t->n_class_tasks[c];
  }
  t->n_mt_tasks = (uint32_t)P.mt_tasks.size();
  t->n_snaps = (uint32_t)ns;
  t->snap_words = mt_snaps ? (uint32_t)kStateWords[MT19937] : 98u;
  t->n_mt_jumps = (uint32_t)(P.mt_jump_list.size() / 2);
  t->d_mt_jumps = reinterpret_cast<const uint32_t*>(w + P.o_mtj);
  t->total_draws = P.total_draws;
  t->max_draws = P.max_draws;
  t->max_task_draws = P.max_task_draws;
  t->n_segments = P.n_segments;
  t->d_counters = reinterpret_cast<uint32_t*>(w);

  t->d_mt_tasks = reinterpret_cast<TableTask*>(w + P.o_mt);
  t->d_rows = reinterpret_cast<TableRow*>(w + P.o_rows);
  t->d_snaps = reinterpret_cast<SnapRow*>(w + P.o_snaprows);
  t->d_aux = P.ext_aux ? P.ext_aux : (P.aux.empty() ? nullptr : reinterpret_cast<const uint32_t*>(w + P.o_aux));
  HIP_TRY(hipGetDevice(&t->device));
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  for (int c = 0; c < kLaneClasses; ++c)
    HIP_TRY(up(P.o_lane[c], P.lane_tasks[c].data(), P.lane_tasks[c].size() * sizeof(TableTask)));
  HIP_TRY(up(P.o_mt, P.mt_tasks.data(), P.mt_tasks.size() * sizeof(TableTask)));
  HIP_TRY(up(P.o_rows, P.rows.data(), P.rows.size() * sizeof(TableRow)));
  HIP_TRY(up(P.o_snaprows, P.snaps.data(), P.snaps.size() * sizeof(SnapRow)));
  HIP_TRY(up(P.o_jump, P.jump.data(), P.jump.size() * 4));
  HIP_TRY(up(P.o_aux, P.aux.data(), P.aux.size() * 4));
  HIP_TRY(up(P.o_mtj, P.mt_jump_list.data(), P.mt_jump_list.size() * 4));
  HIP_TRY(up(P.o_tails, P.tails.data(), P.tails.size() * 4));
  t->d_tails = reinterpret_cast<const uint32_t*>(w + P.o_tails);
  if (sync) HIP_TRY(hipStreamSynchronize(s));
  if (graph_streams) {
    HIP_TRY(hipStreamCreateWithFlags(&t->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&t->fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&t->join, hipEventDisableTiming));
    for (int c = 0; c < kLaneClasses - 1; ++c) {
      HIP_TRY(hipStreamCreateWithFlags(&t->lane_side[c], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&t->lane_join[c], hipEventDisableTiming));
    }
  } else {
    t->cfg.concurrent = 0;
  }
  *out = t.release();
  return PRNG_OK;
}

namespace {
int create_table(prng_table** out, prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows,
                 const SegSpec& seg, void* d_work, size_t work_bytes, void* stream) {
  if (!out) return fail(PRNG_EINVAL, "t is NULL");
  *out = nullptr;
  try {
    Plan P;
    const int rc = make_plan(gens, n_gens, rows, n_rows, seg, nullptr, P);
    if (rc != PRNG_OK) return rc;
    if (!d_work || work_bytes < P.total)
      return fail(PRNG_EINVAL, "workspace holds %zu bytes, %zu needed", work_bytes, P.total);
    if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(PRNG_EINVAL, "workspace must be 256-byte aligned");
    prng_table* t = nullptr;
    const int rc2 = table_from_plan(P, d_work, static_cast<hipStream_t>(stream), true, true, &t);
    if (rc2 != PRNG_OK) return rc2;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find({t->n_lane_tasks, t->n_mt_tasks, t->total_draws, t->max_task_draws});
      if (it != g_tune_cache.end()) t->cfg = it->second;
    }
    *out = t;
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  return PRNG_OK;
}
}  // namespace

PRNG_API int prng_table_create(prng_table** out, prng_gen* const* gens, int n_gens, const prng_table_row* rows,
                               uint64_t n_rows, uint32_t seg_len, void* d_work, size_t work_bytes, void* stream) {
  return create_table(out, gens, n_gens, rows, n_rows, seg_spec_of(seg_len), d_work, work_bytes, stream);
}

PRNG_API int prng_table_create_ex(prng_table** out, prng_gen* const* gens, int n_gens, const prng_table_row* rows,
                                  uint64_t n_rows, const prng_seg_lengths* seg, void* d_work, size_t work_bytes,
                                  void* stream) {
  return create_table(out, gens, n_gens, rows, n_rows, spec_of(seg), d_work, work_bytes, stream);
}

PRNG_API int prng_table_seg_lengths(const prng_table* t, prng_seg_lengths* out) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (!out) return fail(PRNG_EINVAL, "out is NULL");
  *out = prng_seg_lengths{t->seg.lane, t->seg.ranmar, t->seg.mt};
  return PRNG_OK;
}

PRNG_API void prng_table_destroy(prng_table* t) {
  if (!t) return;
  drop_graph(t);
  if (t->fork) (void)hipEventDestroy(t->fork);
  if (t->join) (void)hipEventDestroy(t->join);
  if (t->cap) (void)hipStreamDestroy(t->cap);
  if (t->side) (void)hipStreamDestroy(t->side);
  for (int c = 0; c < kLaneClasses - 1; ++c) {
    if (t->lane_join[c]) (void)hipEventDestroy(t->lane_join[c]);
    if (t->lane_side[c]) (void)hipStreamDestroy(t->lane_side[c]);
  }
  delete t;
}

PRNG_API int prng_table_get_config(const prng_table* t, int* lane_grid, int* mt_grid, int* concurrent) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (lane_grid) *lane_grid = t->cfg.lane_grid;
  if (mt_grid) *mt_grid = t->cfg.mt_grid;
  if (concurrent) *concurrent = t->cfg.concurrent;
  return PRNG_OK;
}

PRNG_API int prng_table_set_config(prng_table* t, int lane_grid, int mt_grid, int concurrent) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (lane_grid < 1 || lane_grid > 65536 || mt_grid < 1 || mt_grid > 65536)
    return fail(PRNG_EINVAL, "grid sizes must be in [1, 65536]");
  if (concurrent < 0 || concurrent > 3)
    return fail(PRNG_EINVAL, "concurrent must be 0, 1, 2 or 3 (got %d)", concurrent);
  t->cfg = TableConfig{lane_grid, mt_grid, concurrent};
  drop_graph(t);
  return PRNG_OK;
}

namespace {
// Captures the run into a graph unless one is held for the current setting.
int ensure_graph(prng_table* t) {
  if (t->exec) return PRNG_OK;
  if (!t->cap) return fail(PRNG_EUNSUPPORTED, "this table has no capture stream");
  HIP_TRY(hipStreamBeginCapture(t->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_run(t, t->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(t->cap, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "enqueue_run (capture)");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  t->graph = g;
  HIP_TRY(hipGraphInstantiate(&t->exec, t->graph, nullptr, nullptr, 0));
  return PRNG_OK;
}
}  // namespace

PRNG_API int prng_table_run(prng_table* t, int use_graph, void* stream) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  DeviceGuard dg(t->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!use_graph) {
    HIP_TRY(enqueue_run(t, s));
    return PRNG_OK;
  }
  if (int rc = ensure_graph(t)) return rc;
  HIP_TRY(hipGraphLaunch(t->exec, s));
  return PRNG_OK;
}

// Autotuner: times candidate (lane grid, MT grid, concurrency) settings on
// the real rows, restoring every referenced stream state after each trial so
// that tuning leaves the streams where they were (the output buffers are
// overwritten by the trials).  The best setting is cached per table shape.
namespace {
int autotune_table(prng_table* t, int repeats, hipStream_t s, float* best_time);
}

PRNG_API int prng_table_autotune(prng_table* t, int repeats, void* stream) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  DeviceGuard dg(t->device);
  return autotune_table(t, repeats, static_cast<hipStream_t>(stream), nullptr);
}

// Segment-length tuner (numbers per lane): a coordinate search from the
// automatic lengths A, trying A / 2 and 2 A for the lane kinds, then RANMAR,
// then MT19937, each candidate planned into d_work, autotuned and timed; a
// candidate whose plan does not fit work_bytes is skipped.
PRNG_API int prng_table_tune_segments(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows,
                                      int repeats, void* d_work, size_t work_bytes, void* stream,
                                      prng_seg_lengths* best, float* best_ms) {
  if (!best) return fail(PRNG_EINVAL, "best is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SegSpec A;
  try {
    Plan P;
    const int rc = make_plan(gens, n_gens, rows, n_rows, SegSpec{}, nullptr, P);
    if (rc != PRNG_OK) return rc;
    A = P.resolved;
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  // time of the tuned table for lengths L (resolved into *got); < 0: skipped
  auto measure = [&](const SegSpec& L, SegSpec* got, float* ms) -> int {
    *ms = -1.0f;
    if (work_bytes < work_bytes_for(gens, n_gens, rows, n_rows, explicit_spec(L))) return PRNG_OK;
    prng_table* t = nullptr;
    int rc = create_table(&t, gens, n_gens, rows, n_rows, explicit_spec(L), d_work, work_bytes, stream);
    if (rc != PRNG_OK) return rc;
    *got = t->seg;
    {
      DeviceGuard dg(t->device);
      rc = autotune_table(t, repeats, s, ms);
    }
    prng_table_destroy(t);
    return rc;
  };
  SegSpec cur{}, got{};
  float cur_ms = 0;
  if (int rc = measure(A, &cur, &cur_ms)) return rc;
  if (cur_ms < 0) return fail(PRNG_EINVAL, "workspace holds %zu bytes, %zu needed", work_bytes,
                              work_bytes_for(gens, n_gens, rows, n_rows, explicit_spec(A)));
  uint32_t SegSpec::*cls[3] = {&SegSpec::lane, &SegSpec::ranmar, &SegSpec::mt};
  for (auto c : cls) {
    if (A.*c == 0) continue;  // a class that is never cut
    const SegSpec base = cur;
    for (int f = 0; f < 2; ++f) {
      SegSpec L = base;
      L.*c = f == 0 ? halved(base).*c : base.*c * 2u;
      if (L.*c == base.*c) continue;
      float ms = 0;
      if (int rc = measure(L, &got, &ms)) return rc;
      if (ms >= 0 && ms < cur_ms) {
        cur = got;
        cur_ms = ms;
      }
    }
  }
  *best = prng_seg_lengths{cur.lane, cur.ranmar, cur.mt};
  if (best_ms) *best_ms = cur_ms;
  return PRNG_OK;
}

namespace {
int autotune_table(prng_table* t, int repeats, hipStream_t s, float* best_time) {
  if (repeats < 1) repeats = 1;
  std::vector<std::vector<char>> saved(t->gens.size());
  try {
    for (size_t i = 0; i < t->gens.size(); ++i) saved[i].resize(state_region_bytes(t->gens[i]->kind, t->gens[i]->n));
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t i = 0; i < t->gens.size(); ++i)
    HIP_TRY(hipMemcpy(saved[i].data(), t->gens[i]->d_state, saved[i].size(), hipMemcpyDeviceToHost));
  auto restore = [&]() -> hipError_t {
    for (size_t i = 0; i < t->gens.size(); ++i) {
      hipError_t e = hipMemcpy(t->gens[i]->d_state, saved[i].data(), saved[i].size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  const TableConfig keep = t->cfg;
  TableConfig best = keep;
  float best_ms = 1e30f;
  const int lane_opts[] = {128, 192, 256};  // lane classes on 1/2, 3/4 or all of the chip
  const int mt_opts[] = {128, 256, 512, 1024, 2048};
  hipError_t err = hipSuccess;
  int graph_rc = PRNG_OK;
  for (int conc = 0; conc < 4 && err == hipSuccess && graph_rc == PRNG_OK; ++conc)
    for (int lg : lane_opts)
      for (int mgi = 0; mgi < 5; ++mgi) {
        const int mg = mt_opts[mgi];
        if (err != hipSuccess || graph_rc != PRNG_OK) break;
        if (!t->n_lane_tasks && lg != lane_opts[0]) continue;
        if (!t->n_mt_tasks && mgi != 0) continue;
        t->cfg = TableConfig{lg, mg, conc};
        // timed as it is used: a replay of the run captured for this setting
        drop_graph(t);
        if (int rc = ensure_graph(t)) {
          graph_rc = rc;
          break;
        }
        // the median of the trials: concurrent kernels share the chip in an
        // order the dispatchers pick, so single replays can be lucky.  The
        // trials follow one untimed replay back to back, as the run is used
        // (the streams advance; they are restored once per setting): trials
        // with the chip idle in between, while the states were copied back,
        // ran faster than the same setting's replays in a row
        std::vector<float> times;
        err = hipGraphLaunch(t->exec, s);
        for (int r = 0; r < repeats && err == hipSuccess; ++r) {
          if ((err = hipEventRecord(a, s)) != hipSuccess) break;
          if ((err = hipGraphLaunch(t->exec, s)) != hipSuccess) break;
          if ((err = hipEventRecord(b, s)) != hipSuccess) break;
          if ((err = hipEventSynchronize(b)) != hipSuccess) break;
          float ms = 0;
          if ((err = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
          times.push_back(ms);
        }
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err == hipSuccess) err = restore();
        if (err == hipSuccess && !times.empty()) {
          std::sort(times.begin(), times.end());
          const float med = times[times.size() / 2];
          if (med < best_ms) {
            best_ms = med;
            best = t->cfg;
          }
        }
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (err != hipSuccess || graph_rc != PRNG_OK) {
    t->cfg = keep;
    drop_graph(t);
    (void)restore();
    return graph_rc != PRNG_OK ? graph_rc : hip_fail(err, "autotune trial");
  }
  t->cfg = best;
  drop_graph(t);
  if (best_time) *best_time = best_ms;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[{t->n_lane_tasks, t->n_mt_tasks, t->total_draws, t->max_task_draws}] = best;
  return PRNG_OK;
}
}  // namespace

PRNG_API int prng_table_info(const prng_table* t, uint32_t* n_lane_tasks, uint32_t* n_mt_tasks, uint64_t* total_draws,
                             uint64_t* max_draws, uint64_t* n_segments) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (n_lane_tasks) *n_lane_tasks = t->n_lane_tasks;
  if (n_mt_tasks) *n_mt_tasks = t->n_mt_tasks;
  if (total_draws) *total_draws = t->total_draws;
  if (max_draws) *max_draws = t->max_draws;
  if (n_segments) *n_segments = t->n_segments;
  return PRNG_OK;
}
