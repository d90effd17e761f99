// Host bookkeeping of the serving loop (server.cpp): the output arena inside
// the caller's pool, the requests and their states, per-stream ordering and
// the completion of batches.  Plain C++ with no device calls, so that its
// rules are checked on the CPU (tests/host_checks.cpp).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <set>
#include <utility>
#include <vector>

#include "prng.h"

namespace prng {

inline size_t book_align256(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit allocator of byte ranges inside the pool (256-byte granules).
class Arena {
 public:
  void init(size_t base, size_t size) {
    free_.clear();
    if (size) free_[base] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = book_align256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = book_align256(std::max<size_t>(bytes, 1));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  // number of free ranges (1 when everything is free again)
  size_t fragments() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

// A request's life: waiting for admission, in flight in a batch, then done
// (output valid) or failed (its batch reported a device error; no output).
// Released: a done request whose output went back to the pool.
enum ReqState { WAITING = 0, INFLIGHT = 1, FAILED = 2, DONE = 3, RELEASED = 4 };

struct Req {
  uint32_t gen = 0;
  uint64_t stream = 0;
  uint64_t count = 0;
  int dtype = 0;
  int keep = 0;
  int64_t t_arrive = 0, t_admit = -1, t_done = -1;
  size_t out_off = 0, out_bytes = 0;
  int state = WAITING;
};

// Checks one request's size before any product is formed (count * draws per
// element and count * element bytes can exceed 64 bits).  draws_per_elem: 2
// for fp64, else 1; elem: element bytes.  Returns nullptr when the request
// fits, else the reason.
inline const char* check_request_size(uint64_t count, uint64_t draws_per_elem, uint64_t elem, uint64_t max_draws,
                                      size_t room) {
  if (count == 0 || count > max_draws / draws_per_elem) return "count must be in [1, max_request_draws]";
  if (count > room / elem || book_align256(count * elem) > room) return "larger than the pool";
  return nullptr;
}

struct RequestBook {
  std::vector<Req> reqs;
  Arena arena;
  std::set<std::pair<uint32_t, uint64_t>> busy;  // (generator, stream) with a request in flight
  uint64_t n_completed = 0, n_failed = 0;

  // The batch holding `tickets` has finished; ok: its completion event
  // reported success.  Done requests free their output unless kept; failed
  // ones always give it back (nothing valid was written) and stay FAILED.
  void finish(const std::vector<uint64_t>& tickets, bool ok, int64_t now) {
    for (uint64_t tk : tickets) {
      Req& r = reqs[tk];
      r.t_done = now;
      busy.erase({r.gen, r.stream});
      if (!ok) {
        arena.release(r.out_off, r.out_bytes);
        r.state = FAILED;
        ++n_failed;
        continue;
      }
      r.state = DONE;
      if (!r.keep) {
        arena.release(r.out_off, r.out_bytes);
        r.state = RELEASED;
      }
      ++n_completed;
    }
  }

  // Whether waiting on `ticket` can stop: it finished either way, or the
  // server stopped (err_code != 0) and it will never run.
  bool settled(uint64_t ticket, int err_code) const { return reqs[ticket].state >= FAILED || err_code != 0; }

  // Result of a ticket that is not released: 1 done (output valid), 0
  // pending, a negative code when it failed or the server stopped before
  // running it (err_code, PRNG_EHIP if none was recorded).
  int status(uint64_t ticket, int err_code) const {
    const Req& r = reqs[ticket];
    if (r.state == DONE) return 1;
    if (r.state == FAILED) return err_code ? err_code : PRNG_EHIP;
    return err_code ? err_code : 0;
  }

  // Give a kept request's output back: false when it is not done (pending or
  // already released).  A failed request holds no memory: releasing it only
  // retires the ticket.
  bool release(uint64_t ticket) {
    Req& r = reqs[ticket];
    if (r.state == FAILED) {
      r.state = RELEASED;
      return true;
    }
    if (r.state != DONE) return false;
    arena.release(r.out_off, r.out_bytes);
    r.state = RELEASED;
    return true;
  }
};

}  // namespace prng
