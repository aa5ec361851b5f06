// The serving loop's scheduler (paper_2606_15650_amd/csrc/sched.hpp) driven
// by a scripted executor on a fake clock: no GPU, built with the address and
// undefined-behaviour sanitizers (and, for the threaded case, the thread
// sanitizer) by tests/test_sched_host.py.
//
// The fake executor "computes" each record as a pure function of its own
// token ids (label = id mod 7, output = the text reversed), takes a scripted
// number of ticks per micro-batch, and can be told to fail a launch or to
// report a device-data error for a micro-batch.  The checks: arrival order,
// every result equal to the request computed alone, the arena never over
// its capacity and every block returned, one micro-batch per slot at a time,
// admission limited by the footprint budget, over-budget and malformed
// requests rejected, unknown tickets, launch and data errors confined to
// their micro-batch, stop with work in flight, and a threaded run with
// concurrent submitters.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <thread>

#include "sched.hpp"

using anon::sched::Arena;
using anon::sched::Limits;
using anon::sched::Request;
using anon::sched::Scheduler;

static int g_fail = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                      \
    }                                                                \
  } while (0)

struct FakeExec {
  std::atomic<long> clock{0};
  struct Sim {
    bool active = false;
    int phase = 0;
    long done_at = 0;
    bool data_error = false;
    std::vector<Request*> reqs;
  };
  std::vector<Sim> slots;
  std::mutex mu;  // the threaded test reads the counters below
  int launches = 0, max_busy = 0, busy = 0;
  int64_t max_in_use = 0;
  std::vector<uint64_t> launch_order;   // tickets in launch order
  std::vector<int> fail_launch;         // launch indices that fail (EDEVICE)
  std::vector<int> data_error_launch;   // launch indices that report a data error
  long ticks_per_token_k = 1;           // duration = 1 + T / 1000 ticks

  explicit FakeExec(int n) : slots(n) {}

  int64_t footprint(int B, int T, int64_t nb) const { return 4096 + 100 * (int64_t)T + 16 * (int64_t)B + nb; }

  anon_status launch(int i, std::vector<Request*>& reqs, int64_t off) {
    std::lock_guard<std::mutex> lk(mu);
    Sim& s = slots[i];
    CHECK(!s.active);  // one micro-batch per slot at a time
    CHECK(off >= 0 && off % 256 == 0);
    const int idx = launches++;
    int T = 0;
    for (Request* r : reqs) {
      launch_order.push_back(r->ticket);
      T += r->n_tokens;
    }
    if (std::find(fail_launch.begin(), fail_launch.end(), idx) != fail_launch.end()) return ANON_EDEVICE;
    s.active = true;
    s.phase = 0;
    s.done_at = clock + 1 + T / 1000 * ticks_per_token_k;
    s.data_error = std::find(data_error_launch.begin(), data_error_launch.end(), idx) != data_error_launch.end();
    s.reqs = reqs;
    busy++;
    max_busy = std::max(max_busy, busy);
    return ANON_OK;
  }
  int query(int i) {
    std::lock_guard<std::mutex> lk(mu);
    return clock >= slots[i].done_at ? 1 : 0;
  }
  anon_status drain(int i) {
    std::lock_guard<std::mutex> lk(mu);
    Sim& s = slots[i];
    if (s.data_error) return ANON_EDATA;
    s.phase = 1;
    s.done_at = clock + 1;
    return ANON_OK;
  }
  void finish(int i, std::vector<Request*>& reqs, anon_status st) {
    std::lock_guard<std::mutex> lk(mu);
    Sim& s = slots[i];
    if (s.active) busy--;
    s.active = false;
    CHECK(st != ANON_OK || s.phase == 1);  // results only after the second phase
    if (st != ANON_OK) return;
    for (Request* r : reqs) {
      r->labels.resize(r->n_tokens);
      for (int t = 0; t < r->n_tokens; ++t) r->labels[t] = (uint8_t)(r->ids[t] % 7);
      r->out.assign(r->text.rbegin(), r->text.rend());
      r->cu_out = r->cu_bytes;
    }
  }
  double now() const { return (double)clock; }
};

static anon_request make_req(int n_records, int tok_per_rec, std::vector<int32_t>& ids, std::vector<int32_t>& cu,
                             std::vector<int32_t>& off, std::vector<uint8_t>& text, std::vector<int64_t>& cub,
                             int seed) {
  ids.clear(), cu.assign(1, 0), off.clear(), text.clear(), cub.assign(1, 0);
  for (int b = 0; b < n_records; ++b) {
    for (int t = 0; t < tok_per_rec; ++t) {
      ids.push_back((seed * 131 + b * 17 + t * 7) % 1000);
      const int64_t rb = (int64_t)(text.size() - cub.back());
      off.push_back((int32_t)rb);
      off.push_back((int32_t)rb + 3);
      for (int c = 0; c < 4; ++c) text.push_back((uint8_t)('a' + (seed + t + c) % 26));
    }
    cu.push_back((int32_t)ids.size());
    cub.push_back((int64_t)text.size());
  }
  anon_request q;
  q.n_records = n_records;
  q.ids = ids.data();
  q.cu_seqlens = cu.data();
  q.tok_off = off.data();
  q.text = text.data();
  q.cu_bytes = cub.data();
  return q;
}

static Request* copy_req(const anon_request& q) {
  Request* r = new Request();
  const int B = q.n_records, T = q.cu_seqlens[B];
  r->n_records = B;
  r->n_tokens = T;
  r->n_bytes = q.cu_bytes[B];
  r->ids.assign(q.ids, q.ids + T);
  r->cu.assign(q.cu_seqlens, q.cu_seqlens + B + 1);
  r->tok_off.assign(q.tok_off, q.tok_off + 2 * (size_t)T);
  r->text.assign(q.text, q.text + r->n_bytes);
  r->cu_bytes.assign(q.cu_bytes, q.cu_bytes + B + 1);
  return r;
}

static void expect_result(const Request* r) {
  CHECK(r->status == ANON_OK);
  CHECK((int)r->labels.size() == r->n_tokens);
  for (int t = 0; t < r->n_tokens; ++t) CHECK(r->labels[t] == (uint8_t)(r->ids[t] % 7));
  std::vector<uint8_t> rev(r->text.rbegin(), r->text.rend());
  CHECK(r->out == rev);
}

template <class S>
static void run_until_idle(S& sch, FakeExec& ex, int max_ticks = 100000) {
  for (int k = 0; k < max_ticks; ++k) {
    const bool busy = sch.tick();
    {
      std::lock_guard<std::mutex> lk(ex.mu);
      ex.max_in_use = std::max(ex.max_in_use, sch.arena_in_use());
    }
    CHECK(sch.arena_in_use() <= sch.arena_capacity());
    if (!busy && sch.queued() == 0) return;
    ex.clock++;
  }
  CHECK(!"scheduler did not go idle");
}

static Limits limits(int tokens, int qmax) {
  Limits l;
  l.max_batch_tokens = tokens;
  l.max_records = tokens;
  l.max_bytes = (int64_t)tokens * 64;
  l.max_queue = qmax;
  return l;
}

static void test_fifo_results_and_arena() {
  FakeExec ex(3);
  Scheduler<FakeExec> sch(ex, 3, limits(4000, 1000), 1 << 24);
  std::vector<uint64_t> tickets;
  std::vector<int32_t> ids, cu, off;
  std::vector<uint8_t> text;
  std::vector<int64_t> cub;
  for (int i = 0; i < 60; ++i) {
    anon_request q = make_req(1 + i % 5, 10 + 7 * (i % 9), ids, cu, off, text, cub, i);
    std::string why;
    CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 4000 * 64, &why) == ANON_OK);
    uint64_t t = 0;
    CHECK(sch.submit(copy_req(q), &t, &why) == ANON_OK);
    tickets.push_back(t);
  }
  run_until_idle(sch, ex);
  CHECK(ex.launch_order == tickets);  // arrival order
  for (uint64_t t : tickets) {
    const Request* r = nullptr;
    CHECK(sch.poll(t, &r) == ANON_OK);
    if (r) expect_result(r);
    CHECK(sch.release(t) == ANON_OK);
  }
  CHECK(sch.arena_in_use() == 0);
  CHECK(ex.max_busy <= 3);
  printf("PASS fifo_results_and_arena (launches %d, max busy slots %d)\n", ex.launches, ex.max_busy);
}

static void test_budget_limits_concurrency() {
  FakeExec ex(4);
  // one 200-token request needs 4096 + 100*200 + 16 + 800 = 24912 -> 25088
  // bytes; a budget of 2.5 such blocks keeps at most two in flight even with
  // four slots, and a micro-batch never packs two of them together
  const int64_t one = Arena::granule(ex.footprint(1, 200, 800));
  Scheduler<FakeExec> sch(ex, 4, limits(200, 100), one * 5 / 2);
  std::vector<int32_t> ids, cu, off;
  std::vector<uint8_t> text;
  std::vector<int64_t> cub;
  std::vector<uint64_t> tickets;
  for (int i = 0; i < 12; ++i) {
    anon_request q = make_req(1, 200, ids, cu, off, text, cub, i);
    uint64_t t = 0;
    std::string why;
    CHECK(sch.submit(copy_req(q), &t, &why) == ANON_OK);
    tickets.push_back(t);
  }
  run_until_idle(sch, ex);
  CHECK(ex.max_busy == 2);
  CHECK(ex.max_in_use <= one * 5 / 2);
  for (uint64_t t : tickets) {
    const Request* r = nullptr;
    CHECK(sch.poll(t, &r) == ANON_OK);
    if (r) expect_result(r);
  }
  // a request whose footprint alone exceeds the budget is refused at submit
  Scheduler<FakeExec> small(ex, 1, limits(4000, 100), 8192);
  anon_request q = make_req(2, 100, ids, cu, off, text, cub, 1);
  uint64_t t = 0;
  std::string why;
  CHECK(small.submit(copy_req(q), &t, &why) == ANON_ECAPACITY);
  printf("PASS budget_limits_concurrency (max busy %d of 4 slots)\n", ex.max_busy);
}

static void test_validation_rejects_malformed_requests() {
  std::vector<int32_t> ids, cu, off;
  std::vector<uint8_t> text;
  std::vector<int64_t> cub;
  std::string why;
  anon_request q = make_req(2, 5, ids, cu, off, text, cub, 3);
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_OK);
  off[2 * 3] = off[2 * 2];  // token 3 starts inside token 2
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(2, 5, ids, cu, off, text, cub, 3);
  off[2 * 4 + 1] = 1000;  // past the record
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(2, 5, ids, cu, off, text, cub, 3);
  off[0] = -1;
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(2, 5, ids, cu, off, text, cub, 3);
  off[2 * 1] = off[2 * 1 + 1] + 1;  // begin after end
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(2, 5, ids, cu, off, text, cub, 3);
  ids[4] = 1000;  // outside the vocabulary
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(2, 5, ids, cu, off, text, cub, 3);
  cu[1] = 0;  // empty record
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(3, 600, ids, cu, off, text, cub, 3);  // records over max_pos
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  q = make_req(9, 500, ids, cu, off, text, cub, 3);  // more tokens than a micro-batch
  CHECK(anon::sched::validate_request(q, 1000, 512, 4000, 1 << 20, &why) == ANON_EINVAL);
  printf("PASS validation_rejects_malformed_requests\n");
}

static void test_tickets_and_errors() {
  FakeExec ex(2);
  ex.fail_launch = {1};
  ex.data_error_launch = {2};
  Scheduler<FakeExec> sch(ex, 2, limits(100, 100), 1 << 22);
  const Request* r = nullptr;
  CHECK(sch.poll(12345, &r) == ANON_ENOTFOUND);
  CHECK(sch.release(12345) == ANON_ENOTFOUND);
  std::vector<int32_t> ids, cu, off;
  std::vector<uint8_t> text;
  std::vector<int64_t> cub;
  std::vector<uint64_t> tk;
  // 90-token requests: one per micro-batch, so launch k holds request k
  for (int i = 0; i < 5; ++i) {
    anon_request q = make_req(1, 90, ids, cu, off, text, cub, i);
    uint64_t t = 0;
    std::string why;
    CHECK(sch.submit(copy_req(q), &t, &why) == ANON_OK);
    tk.push_back(t);
  }
  CHECK(sch.poll(tk[4], &r) == ANON_PENDING);
  CHECK(sch.release(tk[4]) == ANON_EBUSY);
  run_until_idle(sch, ex);
  int st[5];
  for (int i = 0; i < 5; ++i) {
    CHECK(sch.poll(tk[i], &r) == ANON_OK);
    st[i] = r ? r->status : 99;
  }
  CHECK(st[0] == ANON_OK && st[1] == ANON_EDEVICE && st[2] == ANON_EDATA && st[3] == ANON_OK && st[4] == ANON_OK);
  CHECK(sch.arena_in_use() == 0);
  CHECK(sch.release(tk[1]) == ANON_OK);
  CHECK(sch.release(tk[1]) == ANON_ENOTFOUND);
  printf("PASS tickets_and_errors\n");
}

static void test_stop_with_work_in_flight() {
  FakeExec ex(1);
  ex.ticks_per_token_k = 20;
  Scheduler<FakeExec> sch(ex, 1, limits(100, 100), 1 << 22);
  std::vector<int32_t> ids, cu, off;
  std::vector<uint8_t> text;
  std::vector<int64_t> cub;
  std::vector<uint64_t> tk;
  for (int i = 0; i < 4; ++i) {
    anon_request q = make_req(1, 90, ids, cu, off, text, cub, i);
    uint64_t t = 0;
    std::string why;
    CHECK(sch.submit(copy_req(q), &t, &why) == ANON_OK);
    tk.push_back(t);
  }
  sch.tick();  // the first request is now on the slot
  CHECK(sch.busy_slots() == 1);
  sch.stop();
  std::string why;
  uint64_t t = 0;
  anon_request q = make_req(1, 5, ids, cu, off, text, cub, 9);
  CHECK(sch.submit(copy_req(q), &t, &why) == ANON_EBUSY);
  for (int k = 0; k < 1000 && sch.tick(); ++k) ex.clock++;
  sch.fail_queued();
  const Request* r = nullptr;
  CHECK(sch.poll(tk[0], &r) == ANON_OK && r && r->status == ANON_OK);
  for (int i = 1; i < 4; ++i) CHECK(sch.poll(tk[i], &r) == ANON_OK && r && r->status == ANON_EBUSY);
  CHECK(sch.arena_in_use() == 0);
  printf("PASS stop_with_work_in_flight\n");
}

static void test_threaded_submitters() {
  FakeExec ex(3);
  Scheduler<FakeExec> sch(ex, 3, limits(2000, 100000), 1 << 22);
  std::atomic<bool> run_clock{true};
  std::thread clk([&] {
    while (run_clock) {
      ex.clock++;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  });
  std::thread loop([&] { sch.run(10); });
  std::vector<std::thread> subs;
  std::vector<std::vector<uint64_t>> got(4);
  for (int w = 0; w < 4; ++w)
    subs.emplace_back([&, w] {
      std::vector<int32_t> ids, cu, off;
      std::vector<uint8_t> text;
      std::vector<int64_t> cub;
      for (int i = 0; i < 50; ++i) {
        anon_request q = make_req(1 + i % 3, 8 + i % 40, ids, cu, off, text, cub, w * 100 + i);
        uint64_t t = 0;
        std::string why;
        if (sch.submit(copy_req(q), &t, &why) == ANON_OK) got[w].push_back(t);
      }
    });
  for (auto& s : subs) s.join();
  size_t done = 0, total = 0;
  for (auto& g : got) total += g.size();
  for (int k = 0; k < 200000 && done < total; ++k) {
    done = 0;
    for (auto& g : got)
      for (uint64_t t : g) {
        const Request* r = nullptr;
        done += sch.poll(t, &r) == ANON_OK;
      }
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  CHECK(done == total && total == 200);
  for (auto& g : got)
    for (uint64_t t : g) {
      const Request* r = nullptr;
      if (sch.poll(t, &r) == ANON_OK && r) expect_result(r);
      CHECK(sch.release(t) == ANON_OK);
    }
  sch.stop();
  loop.join();
  run_clock = false;
  clk.join();
  CHECK(sch.arena_in_use() == 0);
  printf("PASS threaded_submitters (%zu requests)\n", total);
}

int main(int argc, char** argv) {
  const bool threaded_only = argc > 1 && std::string(argv[1]) == "threaded";
  if (!threaded_only) {
    test_fifo_results_and_arena();
    test_budget_limits_concurrency();
    test_validation_rejects_malformed_requests();
    test_tickets_and_errors();
    test_stop_with_work_in_flight();
  }
  test_threaded_submitters();
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("ALL PASSED\n");
  return 0;
}
