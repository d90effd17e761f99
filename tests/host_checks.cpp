// Host-side checks of libprng's C++ runtime, built for the CPU only under
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_host_sanitize.py):
// seeding, the stream-table planner, the jump-ahead data of every kind, the
// serving loop's bookkeeping (arena, request states, size checks), and the
// CPU oracle.  Nothing here touches a GPU: the device launchers are stubs
// that report "no device", and the planner works on generator objects whose
// device pointers are never dereferenced.
//
// Prints one "<check> ok" line per passed check; exits non-zero on the first
// failure (the sanitizers abort on the first error they find).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <vector>

#include "host.h"
#include "jump.h"
#include "server_book.h"
#include "bigint576.h"

extern "C" {
uint32_t orc_next(int kind, uint32_t p, uint32_t r, uint32_t* st);
int orc_init(int kind, const uint64_t* seed, uint32_t* st);
int orc_state_words(int kind);
void orc_generate(int kind, uint32_t p, uint32_t r, uint64_t n, uint32_t* states, uint64_t count, int dtype,
                  void* out);
void orc_fused(int kind, uint32_t p, uint32_t r, uint64_t n, uint32_t* states, uint64_t draws, uint64_t* sum,
               uint32_t* hist);
}

// ---------------------------------------------------------------- launcher stubs
namespace prng {
hipError_t static_scratch(int, void**) { return hipErrorNoDevice; }
hipError_t launch_init(int, uint32_t*, uint64_t, const uint64_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_generate(int, uint32_t, uint32_t*, uint64_t, uint64_t, int, void*, uint64_t, uint64_t,
                           hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_lux_plain(uint32_t, uint32_t*, const uint32_t*, uint64_t, uint64_t, int, uint32_t, uint32_t,
                            const uint32_t*, const uint32_t*, void*, uint64_t, uint64_t, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_lux_fused_split(uint32_t, uint32_t*, const uint32_t*, uint64_t, uint64_t, uint32_t, uint32_t,
                                  const uint32_t*, const uint32_t*, uint64_t*, uint32_t*, bool, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_generate_packed(int, uint32_t, uint32_t*, uint64_t, uint64_t, int, void*, uint64_t, uint64_t,
                                  hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_xor128_split(uint32_t*, const uint32_t*, uint64_t, uint64_t, int, uint32_t, uint32_t,
                               const uint32_t*, void*, uint64_t, uint64_t, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_ranlux_variant(int, uint32_t, uint32_t*, uint64_t, uint64_t, int, void*, uint64_t, uint64_t,
                                 hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_fused(int, uint32_t, uint32_t*, uint64_t, uint64_t, uint64_t*, uint32_t*, bool, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_table_prepare(uint32_t*, int, const SnapRow*, uint32_t, uint32_t, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_table_lane(int, const TableTask*, uint32_t, const TableRow*, const uint32_t*, uint32_t*,
                             const uint32_t*, int, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_table_mt_jump(const uint32_t*, uint32_t, const TableRow*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_table_mt(const TableTask*, uint32_t, const TableRow*, uint32_t*, int, hipStream_t) {
  return hipErrorNoDevice;
}
}  // namespace prng

using namespace prng;

static int g_failed = 0;
#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      exit(1);                                                           \
    }                                                                    \
  } while (0)

static void ok(const char* name) { printf("%s ok\n", name); }

// ---------------------------------------------------------------- seeding
static void check_seeding() {
  for (int k = GGL; k < kKinds; ++k) {
    const int W = prng_seed_tuple_words(k);
    CHECK(W == kSeedWords[k]);
    const uint64_t n = 3000;
    std::vector<uint64_t> w(n * W);
    CHECK(prng_seed_words(k, 42, n, w.data()) == PRNG_OK);
    std::set<std::vector<uint64_t>> seen;
    for (uint64_t s = 0; s < n; ++s) {
      std::vector<uint32_t> st(orc_state_words(k) + 8);
      CHECK(orc_init(k, w.data() + s * W, st.data()) == 0);  // in the generator's valid range
      CHECK(seen.insert(std::vector<uint64_t>(w.begin() + s * W, w.begin() + (s + 1) * W)).second);
    }
  }
  CHECK(prng_seed_words(99, 1, 1, nullptr) == PRNG_EINVAL);
  CHECK(prng_seed_words(GGL, 1, 5, nullptr) == PRNG_EINVAL);
  ok("seeding");
}

// ---------------------------------------------------------------- planner
struct FakeGens {
  std::vector<prng_gen> objs;
  std::vector<prng_gen*> ptrs;
  FakeGens(const std::vector<std::pair<int, uint32_t>>& kinds, uint64_t n) {
    objs.reserve(kinds.size());
    uintptr_t base = 0x10000000u;
    for (auto& kp : kinds) {
      prng_gen g{};
      g.kind = kp.first;
      g.p = kp.first == RANLUX ? kp.second : 0;
      g.n = n;
      g.d_state = reinterpret_cast<uint32_t*>(base);  // never dereferenced on the host
      base += 0x1000000u;
      objs.push_back(g);
    }
    for (auto& g : objs) ptrs.push_back(&g);
  }
};

static void check_plan_invariants(const Plan& P, const std::vector<prng_table_row>& rows) {
  uint64_t want_draws = 0;
  for (auto& r : rows) want_draws += r.count * (r.dtype == F64 ? 2 : 1);
  CHECK(P.total_draws == want_draws);
  CHECK(P.rows.size() == rows.size() - (size_t)std::count_if(rows.begin(), rows.end(),
                                                             [](const prng_table_row& r) { return r.count == 0; }));
  uint64_t segs = 0;
  for (const TableRow& tr : P.rows) {
    CHECK(tr.nseg >= 1 && tr.nseg <= 4096);
    if (tr.nseg > 1) {
      CHECK(tr.seg_len > 0);
      CHECK((uint64_t)(tr.nseg - 1) * tr.seg_len < tr.draws);  // the last segment is never empty
      CHECK((uint64_t)tr.nseg * tr.seg_len >= tr.draws);
    }
    segs += tr.nseg;
  }
  CHECK(segs == P.n_segments);
  for (int c = 0; c < kLaneClasses; ++c)
    for (const TableTask& t : P.lane_tasks[c]) {
      CHECK(t.nseg >= 1 && t.nseg <= 64);
      CHECK(lane_class((int)t.kind) == c);
      if (t.tail) {
        CHECK(t.g0 + t.nseg <= P.tails.size());
      } else {
        CHECK(t.row0 <= t.row1 && t.row1 < P.rows.size());
      }
    }
  for (const TableTask& t : P.mt_tasks) {
    CHECK(t.kind == MT19937 && t.nseg == 1 && t.row0 < P.rows.size());
    CHECK(t.g0 < P.rows[t.row0].nseg);
  }
  for (uint32_t r : P.tails) CHECK(r < P.rows.size());
  CHECK(P.mt_jump_list.size() % 2 == 0);
  for (size_t i = 0; i < P.mt_jump_list.size(); i += 2) {
    CHECK(P.mt_jump_list[i] < P.rows.size());
    CHECK(P.mt_jump_list[i + 1] >= 1 && P.mt_jump_list[i + 1] < P.rows[P.mt_jump_list[i]].nseg);
  }
  const size_t offs[] = {P.o_tails, P.o_lane[0], P.o_lane[1], P.o_mt, P.o_rows, P.o_snaprows,
                         P.o_snap, P.o_snap_mt, P.o_jstate, P.o_mtj, P.o_jump, P.o_aux};
  for (size_t o : offs) {
    CHECK(o % 256 == 0);
    CHECK(o <= P.total);
  }
  CHECK(P.o_rows + P.rows.size() * sizeof(TableRow) <= P.total);
  CHECK(P.o_jump + P.jump.size() * 4 <= P.total);
}

static void check_planner() {
  const std::vector<std::pair<int, uint32_t>> kinds = {{GGL, 0},     {XOR128, 0},  {RANECU, 0},  {RANMAR, 0},
                                                       {RANLUX, 223}, {RANLUX, 24}, {MT19937, 0}, {DRAND48, 0},
                                                       {RANNYU, 0}};
  FakeGens G(kinds, 500);
  std::mt19937_64 rng(7);
  const uint32_t seg_choices[] = {PRNG_SEG_AUTO, PRNG_SEG_NEVER, 384, 1152, 5000};
  int planned = 0;
  for (int trial = 0; trial < 24; ++trial) {
    std::vector<prng_table_row> rows;
    uintptr_t out = 0x700000000ull;
    std::set<std::pair<uint32_t, uint64_t>> used;
    const int nrows = 1 + (int)(rng() % 400);
    for (int i = 0; i < nrows; ++i) {
      const uint32_t gi = (uint32_t)(rng() % kinds.size());
      const uint64_t s = rng() % 500;
      if (!used.insert({gi, s}).second) continue;
      const int dt = 1 + (int)(rng() % 3);
      uint64_t count;
      switch (rng() % 4) {
        case 0: count = rng() % 5; break;                          // empty and tiny rows
        case 1: count = 1 + rng() % 3000; break;
        case 2: count = 1 + rng() % 300000; break;
        default: count = (1ull << (6 + rng() % 15)) + rng() % 97;  // up to 2^20
      }
      rows.push_back(prng_table_row{gi, (uint32_t)dt, s, count, reinterpret_cast<void*>(out)});
      out += ((count * 8 + 255) / 256 + 1) * 256;
    }
    SegSpec spec{seg_choices[rng() % 5], seg_choices[rng() % 5], seg_choices[rng() % 5]};
    if (spec.mt != PRNG_SEG_AUTO && spec.mt != PRNG_SEG_NEVER && spec.mt < 1248) spec.mt = 1248;
    Plan P;
    const int rc = make_plan(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), spec, nullptr, P);
    CHECK(rc == PRNG_OK);
    check_plan_invariants(P, rows);
    ++planned;
  }
  // rejections: a stream listed twice, a bad dtype, an out-of-range stream, a misaligned f64 output
  {
    std::vector<prng_table_row> rows = {{0, 1, 3, 10, reinterpret_cast<void*>(0x7000)},
                                        {0, 2, 3, 10, reinterpret_cast<void*>(0x8000)}};
    Plan P;
    CHECK(make_plan(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), SegSpec{}, nullptr, P) ==
          PRNG_EINVAL);
    rows = {{0, 9, 3, 10, reinterpret_cast<void*>(0x7000)}};
    Plan P2;
    CHECK(make_plan(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), SegSpec{}, nullptr, P2) ==
          PRNG_EINVAL);
    rows = {{0, 1, 500, 10, reinterpret_cast<void*>(0x7000)}};
    Plan P3;
    CHECK(make_plan(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), SegSpec{}, nullptr, P3) ==
          PRNG_EINVAL);
    rows = {{0, 3, 1, 10, reinterpret_cast<void*>(0x7004)}};
    Plan P4;
    CHECK(make_plan(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), SegSpec{}, nullptr, P4) ==
          PRNG_EINVAL);
  }
  // the public sizing calls run the same planner
  {
    std::vector<prng_table_row> rows;
    for (uint32_t gi = 0; gi < kinds.size(); ++gi)
      rows.push_back(prng_table_row{gi, 2u, gi, 70000u + gi, reinterpret_cast<void*>(0x800000000ull + gi * 0x100000)});
    CHECK(prng_table_work_bytes(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), 384) > 0);
    prng_seg_lengths sl{1152, PRNG_SEG_NEVER, 0};
    CHECK(prng_table_work_bytes_ex(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size(), &sl) > 0);
    CHECK(prng_table_tune_work_bytes(G.ptrs.data(), (int)G.ptrs.size(), rows.data(), rows.size()) > 0);
  }
  printf("planner ok (%d plans)\n", planned);
}

// ---------------------------------------------------------------- jump data
static void check_jumps() {
  const uint64_t Ls[] = {384, 1152, 2304, 9216};
  for (int k = GGL; k < kKinds; ++k) {
    for (uint64_t L : Ls) {
      if (k == MT19937 && L != Ls[0]) continue;  // x^J mod a degree-19937 polynomial is slow under the sanitizers
      const uint64_t Lk = k == MT19937 ? (L * 2 + 623) / 624 * 624 : L;
      const uint32_t nj = k == MT19937 ? 2 : 9;
      const uint32_t stride = jump_slot_words(k);
      std::vector<uint32_t> d((size_t)nj * stride + 16, 0xA5A5A5A5u);
      CHECK(fill_jumps(k, k == RANLUX ? 223 : 0, Lk, nj, d.data()));
      for (size_t i = (size_t)nj * stride; i < d.size(); ++i) CHECK(d[i] == 0xA5A5A5A5u);  // no overrun
      if (k == GGL)
        for (uint32_t j = 1; j <= nj; ++j) CHECK(d[(j - 1) * stride] == powmod31(16807, j * Lk, 2147483647u));
      if (k == RANECU)
        for (uint32_t j = 1; j <= nj; ++j) {
          CHECK(d[(j - 1) * stride] == powmod31(40014, j * Lk, 2147483563u));
          CHECK(d[(j - 1) * stride + 1] == powmod31(40692, j * Lk, 2147483399u));
        }
    }
  }
  // composition laws of the matrix and polynomial powers
  std::vector<uint32_t> a(512), b(512), c(512), ab(512);
  xor128_power(1000, a.data());
  xor128_power(2345, b.data());
  xor128_power(3345, c.data());
  xor128_compose(a.data(), b.data(), ab.data());
  CHECK(memcmp(ab.data(), c.data(), 512 * 4) == 0);
  std::vector<uint32_t> pa(97), pb(97), pc(97), pab(97);
  ranmar_power(777, pa.data());
  ranmar_power(5000, pb.data());
  ranmar_power(5777, pc.data());
  ranmar_polymul(pa.data(), pb.data(), pab.data());
  CHECK(memcmp(pab.data(), pc.data(), 97 * 4) == 0);
  CHECK(ranmar_c_shift(16777213) == 0);
  // the power-of-two table of split XOR128 generation: matrix k is T^(2^k)
  {
    std::vector<uint32_t> p2(kXorPow2Words), want(512);
    fill_xor128_pow2(p2.data());
    for (int k : {0, 1, 5, 12, 31}) {
      xor128_power(1ull << k, want.data());
      CHECK(memcmp(p2.data() + 512 * k, want.data(), 512 * 4) == 0);
    }
  }
  CHECK(ranlux_selfcheck());
  // the block-jump table: entry (d, v) is b^-(p v 256^d), and a jump of E blocks is the product of its digits' entries
  for (uint32_t p : {24u, 223u, 389u}) {
    std::vector<uint32_t> dig(kLuxDigitWords), want(18), prod(18, 0);
    fill_ranlux_digits(p, dig.data());
    for (int d = 0; d < kLuxDigits; ++d)
      for (uint32_t v : {0u, 1u, 2u, 77u, 255u}) {
        ranlux_power((uint64_t)p * v << (8 * d), want.data());
        CHECK(memcmp(dig.data() + (d * 256 + v) * 18, want.data(), 72) == 0);
      }
    const uint32_t E = 0x02A4FF13u;
    prod[0] = 1;
    for (int d = 0; d < kLuxDigits; ++d)
      mulmod576(prod.data(), dig.data() + (d * 256 + ((E >> (8 * d)) & 255u)) * 18, prod.data());
    ranlux_power((uint64_t)E * p, want.data());
    CHECK(prod == want);
  }
  std::vector<uint32_t> aux(kRanluxAuxWords);
  fill_ranlux_aux(aux.data());
  uint64_t A = 0, C = 0;
  lcg48_power(25214903917ull, 11, 0, &A, &C);
  CHECK(A == 1 && C == 0);
  std::vector<uint32_t> poly(624);
  CHECK(mt_jump_poly(624 * 3, poly.data()));
  ok("jumps");
}

// ---------------------------------------------------------------- serving bookkeeping
static void check_book() {
  RequestBook B;
  const size_t base = 4096, room = 1 << 20;
  B.arena.init(base, room);
  auto add = [&](uint32_t gen, uint64_t stream, uint64_t count, int dtype, int keep) {
    Req r;
    r.gen = gen;
    r.stream = stream;
    r.count = count;
    r.dtype = dtype;
    r.keep = keep;
    r.out_bytes = count * (dtype == F64 ? 8 : 4);
    CHECK(B.arena.alloc(r.out_bytes, &r.out_off));
    r.state = INFLIGHT;
    B.busy.insert({gen, stream});
    B.reqs.push_back(r);
    return (uint64_t)B.reqs.size() - 1;
  };
  // a batch that succeeds: kept outputs stay until released, the others go back at once
  const uint64_t t0 = add(0, 1, 1000, F32, 1), t1 = add(0, 2, 333, F64, 0), t2 = add(1, 1, 5, U32, 1);
  B.finish({t0, t1, t2}, true, 100);
  CHECK(B.reqs[t0].state == DONE && B.reqs[t1].state == RELEASED && B.reqs[t2].state == DONE);
  CHECK(B.status(t0, 0) == 1 && B.settled(t0, 0));
  CHECK(B.busy.empty() && B.n_completed == 3);
  // a batch whose completion event reports a device error: its requests fail,
  // their memory goes back, and their result is an error code, never an output
  const uint64_t t3 = add(2, 7, 4096, F32, 1), t4 = add(2, 8, 100, U32, 0);
  const size_t held = B.arena.used();
  B.finish({t3, t4}, false, 200);
  CHECK(B.reqs[t3].state == FAILED && B.reqs[t4].state == FAILED);
  CHECK(B.status(t3, PRNG_EHIP) == PRNG_EHIP && B.status(t4, 0) == PRNG_EHIP);
  CHECK(B.settled(t3, 0));
  CHECK(B.arena.used() < held && B.n_failed == 2 && B.n_completed == 3);
  CHECK(B.release(t3));        // retires the ticket, no memory to give back
  CHECK(!B.release(t3));       // already released
  CHECK(B.release(t0) && B.release(t2));
  CHECK(B.arena.used() == 0 && B.arena.fragments() == 1);
  // a pending request is not settled until the server stops
  const uint64_t t5 = add(3, 1, 10, U32, 1);
  B.reqs[t5].state = WAITING;
  CHECK(!B.settled(t5, 0) && B.status(t5, 0) == 0 && B.settled(t5, PRNG_EHIP) && B.status(t5, PRNG_EHIP) < 0);
  // size checks never overflow: 2^63 fp64 elements, 2^62 8-byte elements
  CHECK(check_request_size(1ull << 63, 2, 8, 1ull << 30, room) != nullptr);
  CHECK(check_request_size(~0ull, 1, 4, ~0ull, room) != nullptr);
  CHECK(check_request_size(1ull << 62, 1, 8, ~0ull, room) != nullptr);
  CHECK(check_request_size(0, 1, 4, 1u << 30, room) != nullptr);
  CHECK(check_request_size(1u << 20, 1, 4, 1u << 30, room) != nullptr);  // 4 MiB > 1 MiB room
  CHECK(check_request_size(1000, 2, 8, 1u << 30, room) == nullptr);
  CHECK(check_request_size(1u << 29, 2, 8, 1u << 30, ~size_t(0)) == nullptr);
  CHECK(check_request_size((1u << 29) + 1, 2, 8, 1u << 30, ~size_t(0)) != nullptr);
  ok("server_book");
}

static void check_arena_fuzz() {
  Arena A;
  const size_t base = 256 * 10, size = 256 * 5000;
  A.init(base, size);
  std::mt19937_64 rng(3);
  std::vector<std::pair<size_t, size_t>> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 2) {
      const size_t bytes = 1 + rng() % 9000;
      size_t off;
      if (A.alloc(bytes, &off)) {
        CHECK(off >= base && off + book_align256(bytes) <= base + size && off % 256 == 0);
        for (auto& l : live) CHECK(off + book_align256(bytes) <= l.first || l.first + book_align256(l.second) <= off);
        live.push_back({off, bytes});
      }
    } else {
      const size_t i = rng() % live.size();
      A.release(live[i].first, live[i].second);
      live.erase(live.begin() + (long)i);
    }
    size_t used = 0;
    for (auto& l : live) used += book_align256(l.second);
    CHECK(A.used() == used);
  }
  for (auto& l : live) A.release(l.first, l.second);
  CHECK(A.used() == 0 && A.fragments() == 1);
  ok("arena");
}

// ---------------------------------------------------------------- oracle
static void check_oracle() {
  for (int k = GGL; k < kKinds; ++k) {
    const int W = orc_state_words(k);
    const uint64_t n = 5;
    std::vector<uint64_t> seeds(n * 4);
    CHECK(prng_seed_words(k, 9, n, seeds.data()) == PRNG_OK);
    std::vector<uint32_t> st(n * W), st2;
    for (uint64_t s = 0; s < n; ++s) CHECK(orc_init(k, seeds.data() + s * kSeedWords[k], st.data() + s * W) == 0);
    st2 = st;
    for (int dt = 1; dt <= 4; ++dt) {
      if (dt == 4 && (k == DRAND48 || k == RANNYU)) continue;
      const uint64_t count = 1000 + 7 * dt;
      std::vector<uint64_t> out(n * count);
      orc_generate(k, 223, 24, n, st.data(), count, dt, out.data());
    }
    std::vector<uint64_t> sum(n);
    std::vector<uint32_t> hist(n * 64);
    orc_fused(k, 97, 24, n, st2.data(), 5000, sum.data(), hist.data());
    for (uint64_t s = 0; s < n; ++s) {
      uint64_t tot = 0;
      for (int b = 0; b < 64; ++b) tot += hist[s * 64 + b];
      CHECK(tot == 5000);
    }
  }
  ok("oracle");
}

int main() {
  check_seeding();
  check_planner();
  check_jumps();
  check_book();
  check_arena_fuzz();
  check_oracle();
  printf("all ok\n");
  return g_failed;
}
