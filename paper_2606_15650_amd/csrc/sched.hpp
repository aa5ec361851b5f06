// Scheduler of the serving loop: host code only (no HIP), so the same state
// machine runs on the GPU server and, with a scripted executor on a fake
// clock, in CPU tests under the address/undefined-behaviour sanitizers.
//
// Requests are admitted in arrival order.  A free slot takes the longest run
// of queued requests that fits the micro-batch limits (tokens, records, text
// bytes) and whose device footprint fits the largest free block of the
// activation arena; the footprint is carved from the arena for exactly that
// micro-batch and returned when its results are back on the host.  A slot
// moves FREE -> RUNNING (kernels and the small result copies enqueued, first
// event) -> DRAINING (variable-size result copies enqueued, second event) ->
// FREE; the scheduler only ever queries events, it never waits on a stream.
//
// Executor interface (a template parameter E):
//   int64_t footprint(int B, int T, int64_t n_bytes) const   device bytes of a micro-batch
//   anon_status launch(int slot, std::vector<Request*>&, int64_t arena_off)
//   int query(int slot)            0 pending, 1 done, < 0 an anon_status error
//   anon_status drain(int slot)    after the first event: check the small results, enqueue the rest
//   void finish(int slot, std::vector<Request*>&, anon_status)   fill the requests' results
//   double now()
#pragma once

#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/anon.h"

namespace anon {
namespace sched {

struct Request {
  uint64_t ticket = 0;
  int n_records = 0, n_tokens = 0;
  int64_t n_bytes = 0;
  int64_t footprint = 0;  // device bytes of this request alone in a micro-batch
  std::vector<int32_t> ids, cu, tok_off;
  std::vector<uint8_t> text;
  std::vector<int64_t> cu_bytes;
  // results
  int status = ANON_PENDING;
  std::vector<uint8_t> out, labels;
  std::vector<int64_t> cu_out;
  std::vector<anon_span> spans;
  double t_submit = 0, t_start = 0, t_done = 0;
};

// Checks a request against the model and the server limits before it is
// copied.  Token byte ranges must lie inside their record, in order and
// without overlap (0 <= begin <= end <= next begin, last end <= record
// bytes): spans are unions of token ranges, so this keeps every span that
// decoding can form inside its record and disjoint from the others.
inline anon_status validate_request(const anon_request& q, int vocab, int max_pos, int max_request_tokens,
                                    int64_t max_bytes, std::string* why) {
  auto fail = [&](const char* m) {
    *why = m;
    return ANON_EINVAL;
  };
  const int B = q.n_records;
  if (B < 1 || !q.cu_seqlens || !q.cu_bytes) return fail("request has no records");
  if (q.cu_seqlens[0] != 0 || q.cu_bytes[0] != 0) return fail("cu arrays must start at 0");
  for (int b = 0; b < B; ++b) {
    const int64_t n = (int64_t)q.cu_seqlens[b + 1] - q.cu_seqlens[b];
    if (n < 1 || n > max_pos) return fail("record lengths must be in [1, max_pos]");
    if (q.cu_bytes[b + 1] < q.cu_bytes[b]) return fail("cu_bytes must be non-decreasing");
    if ((int64_t)q.cu_seqlens[b + 1] > (int64_t)max_request_tokens) return fail("request larger than a micro-batch");
  }
  const int T = q.cu_seqlens[B];
  const int64_t nb = q.cu_bytes[B];
  if (T > max_request_tokens || nb > max_bytes) return fail("request larger than a micro-batch");
  if (!q.ids || !q.tok_off) return fail("ids/tok_off NULL");
  if (nb > 0 && !q.text) return fail("text NULL");
  for (int t = 0; t < T; ++t)
    if (q.ids[t] < 0 || q.ids[t] >= vocab) return fail("token id out of range");
  for (int b = 0; b < B; ++b) {
    const int64_t rbytes = q.cu_bytes[b + 1] - q.cu_bytes[b];
    int64_t prev_end = 0;
    for (int t = q.cu_seqlens[b]; t < q.cu_seqlens[b + 1]; ++t) {
      const int64_t beg = q.tok_off[2 * (size_t)t], end = q.tok_off[2 * (size_t)t + 1];
      if (beg < prev_end || end < beg || end > rbytes)
        return fail("tok_off: token byte ranges must be ordered, disjoint and inside their record");
      prev_end = end;
    }
  }
  return ANON_OK;
}

// First-fit allocator over [0, capacity) in 256-byte granules; frees coalesce
// with their neighbours.  Offsets only: the memory itself is the executor's.
class Arena {
 public:
  explicit Arena(int64_t capacity) : cap_(capacity / 256 * 256) {
    if (cap_ > 0) free_[0] = cap_;
  }
  static int64_t granule(int64_t bytes) { return (bytes + 255) / 256 * 256; }
  int64_t capacity() const { return cap_; }
  int64_t in_use() const { return used_bytes_; }
  int64_t largest_free() const {
    int64_t m = 0;
    for (auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  // Offset of a block of at least `bytes`, or -1.
  int64_t alloc(int64_t bytes) {
    const int64_t n = granule(bytes < 1 ? 1 : bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const int64_t off = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest > 0) free_[off + n] = rest;
      used_[off] = n;
      used_bytes_ += n;
      return off;
    }
    return -1;
  }
  // Returns false for an offset that is not allocated.
  bool release(int64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    int64_t beg = off, len = u->second;
    used_bytes_ -= len;
    used_.erase(u);
    auto nxt = free_.lower_bound(beg);
    if (nxt != free_.end() && nxt->first == beg + len) {
      len += nxt->second;
      nxt = free_.erase(nxt);
    }
    if (nxt != free_.begin()) {
      auto prv = std::prev(nxt);
      if (prv->first + prv->second == beg) {
        beg = prv->first;
        len += prv->second;
        free_.erase(prv);
      }
    }
    free_[beg] = len;
    return true;
  }

 private:
  int64_t cap_;
  int64_t used_bytes_ = 0;
  std::map<int64_t, int64_t> free_, used_;
};

struct Limits {
  int max_batch_tokens = 0;  // tokens per micro-batch
  int max_records = 0;       // records per micro-batch
  int64_t max_bytes = 0;     // text bytes per micro-batch
  int max_queue = 0;         // queued requests before submit returns EBUSY
};

template <class E>
class Scheduler {
 public:
  Scheduler(E& ex, int n_slots, const Limits& lim, int64_t arena_bytes)
      : ex_(ex), lim_(lim), arena_(arena_bytes), slots_(n_slots) {}
  ~Scheduler() {
    for (auto& kv : reqs_) delete kv.second;
  }

  // Queues a validated request; takes ownership.  ANON_ECAPACITY when its
  // footprint alone exceeds the arena, ANON_EBUSY when the queue is full or
  // the scheduler is stopping.
  anon_status submit(Request* r, uint64_t* ticket, std::string* why) {
    std::unique_ptr<Request> own(r);
    r->footprint = ex_.footprint(r->n_records, r->n_tokens, r->n_bytes);
    if (Arena::granule(r->footprint) > arena_.capacity()) {
      *why = "request needs " + std::to_string(r->footprint) + " device bytes, over the activation budget of " +
             std::to_string(arena_.capacity());
      return ANON_ECAPACITY;
    }
    r->t_submit = ex_.now();
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_) {
      *why = "server is stopping";
      return ANON_EBUSY;
    }
    if ((int)queue_.size() >= lim_.max_queue) {
      *why = "queue full";
      return ANON_EBUSY;
    }
    r->ticket = next_ticket_++;
    reqs_[r->ticket] = own.release();
    queue_.push_back(r);
    *ticket = r->ticket;
    cv_.notify_all();
    return ANON_OK;
  }

  // ANON_ENOTFOUND, ANON_PENDING, or ANON_OK with *out pointing at the
  // finished request (valid until release).
  anon_status poll(uint64_t ticket, const Request** out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return ANON_ENOTFOUND;
    if (it->second->status == ANON_PENDING) return ANON_PENDING;
    *out = it->second;
    return ANON_OK;
  }

  anon_status release(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return ANON_ENOTFOUND;
    if (it->second->status == ANON_PENDING) return ANON_EBUSY;
    delete it->second;
    reqs_.erase(it);
    return ANON_OK;
  }

  // One pass: retire or advance busy slots, then admit queued requests into
  // free slots.  Called by one thread.  Returns true while any slot is busy.
  bool tick() {
    bool busy = false;
    for (int i = 0; i < (int)slots_.size(); ++i) {
      Slot& s = slots_[i];
      if (s.st == FREE) continue;
      const int q = ex_.query(i);
      if (q == 0) {
        busy = true;
        continue;
      }
      if (q < 0) {
        retire(i, (anon_status)q);
        continue;
      }
      if (s.st == RUNNING) {
        const anon_status rc = ex_.drain(i);
        if (rc != ANON_OK) {
          retire(i, rc);
          continue;
        }
        s.st = DRAINING;
        busy = true;
      } else {
        retire(i, ANON_OK);
      }
    }
    for (int i = 0; i < (int)slots_.size(); ++i) {
      Slot& s = slots_[i];
      if (s.st != FREE) continue;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (stopping_ || queue_.empty()) break;
        int B = 0, T = 0;
        int64_t nb = 0;
        const int64_t room = arena_.largest_free();
        while (!queue_.empty()) {
          Request* r = queue_.front();
          if (T + r->n_tokens > lim_.max_batch_tokens || B + r->n_records > lim_.max_records ||
              nb + r->n_bytes > lim_.max_bytes ||
              Arena::granule(ex_.footprint(B + r->n_records, T + r->n_tokens, nb + r->n_bytes)) > room)
            break;
          queue_.pop_front();
          s.reqs.push_back(r);
          B += r->n_records;
          T += r->n_tokens;
          nb += r->n_bytes;
        }
        if (s.reqs.empty()) break;  // the head waits for memory (arrival order is kept)
        s.off = arena_.alloc(ex_.footprint(B, T, nb));
        peak_in_use_ = arena_.in_use() > peak_in_use_ ? arena_.in_use() : peak_in_use_;
        ++micro_batches_;
        const double t = ex_.now();
        for (Request* r : s.reqs) r->t_start = t;
      }
      s.st = RUNNING;
      busy = true;
      {
        int n = 0;
        for (auto& o : slots_) n += o.st != FREE;
        max_concurrent_ = n > max_concurrent_ ? n : max_concurrent_;
      }
      const anon_status rc = ex_.launch(i, s.reqs, s.off);
      if (rc != ANON_OK) retire(i, rc);
    }
    return busy;
  }

  // The scheduler thread: ticks until stopped with no slot busy, sleeping on
  // the condition variable while nothing runs and polling events briefly
  // while something does; then fails whatever is still queued.
  void run(int poll_us = 50) {
    for (;;) {
      const bool busy = tick();
      std::unique_lock<std::mutex> lk(mu_);
      if (stopping_ && !busy) break;
      // (a system_clock deadline: for a short poll a clock step is harmless,
      // and the wait maps onto pthread_cond_timedwait, which thread
      // sanitizers understand; steady-clock waits use a call they may not)
      if (busy) cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(poll_us));
      else cv_.wait(lk, [&] { return stopping_ || !queue_.empty(); });
    }
    fail_queued();
  }

  void stop() {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = true;
    cv_.notify_all();
  }

  // Fails queued requests with ANON_EBUSY (after stop, once nothing runs).
  void fail_queued() {
    std::lock_guard<std::mutex> lk(mu_);
    for (Request* r : queue_) {
      r->status = ANON_EBUSY;
      r->t_done = ex_.now();
    }
    queue_.clear();
  }

  // counters since start: peak arena bytes in use, micro-batches launched,
  // most slots busy at once
  void stats(int64_t* peak, int64_t* batches, int* concurrent) {
    std::lock_guard<std::mutex> lk(mu_);
    *peak = peak_in_use_;
    *batches = micro_batches_;
    *concurrent = max_concurrent_;
  }

  // introspection (tests)
  int64_t arena_in_use() const { return arena_.in_use(); }
  int64_t arena_capacity() const { return arena_.capacity(); }
  int busy_slots() const {
    int n = 0;
    for (auto& s : slots_) n += s.st != FREE;
    return n;
  }
  size_t queued() {
    std::lock_guard<std::mutex> lk(mu_);
    return queue_.size();
  }

 private:
  enum State { FREE, RUNNING, DRAINING };
  struct Slot {
    State st = FREE;
    std::vector<Request*> reqs;
    int64_t off = -1;
  };

  void retire(int i, anon_status st) {
    Slot& s = slots_[i];
    ex_.finish(i, s.reqs, st);
    const double t = ex_.now();
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (Request* r : s.reqs) {
        r->status = st;
        r->t_done = t;
      }
      arena_.release(s.off);
      cv_.notify_all();
    }
    s.reqs.clear();
    s.off = -1;
    s.st = FREE;
  }

  E& ex_;
  Limits lim_;
  Arena arena_;
  std::vector<Slot> slots_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Request*> queue_;
  std::unordered_map<uint64_t, Request*> reqs_;
  uint64_t next_ticket_ = 1;
  bool stopping_ = false;
  int64_t peak_in_use_ = 0, micro_batches_ = 0;
  int max_concurrent_ = 0;
};

}  // namespace sched
}  // namespace anon
