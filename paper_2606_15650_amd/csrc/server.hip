// Serving loop: continuous batching of record batches on one GPU.
//
// anon_submit validates a request, copies it into host memory and queues it
// with the scheduler (sched.hpp).  A scheduler thread packs queued requests
// (arrival order) into micro-batches and runs each on a slot: one HIP stream,
// two events and pinned host staging.  Device memory comes from one arena
// whose size is the HBM activation budget (capped at what all slots can use
// at once); each micro-batch takes exactly its own footprint -- inputs,
// outputs, error word and the three stages' workspaces -- so a slot admits
// work only while it fits the budget left.  The path per micro-batch is
// NER -> span decoding -> substitution on the slot's stream, then the labels,
// span/output offsets and the micro-batch's own error word come back (first
// event); once they have, the spans and bytes are copied back (second event)
// and split per request.  The thread only queries events.  Every kernel
// computes each record independently of its batch-mates, so a request's
// result is the same alone or mixed with others.
//
// With graph buckets on, each slot also owns fixed forward buffers (ids,
// boundaries, token count, labels, error word, NER workspace) sized for the
// largest micro-batch, and one instantiated HIP graph of the NER forward per
// token bucket (max_batch_tokens, half of it, a quarter, ...), captured on
// those buffers at start.  A micro-batch is uploaded into the slot's
// buffers (its boundaries padded with empty records to the bucket) and runs
// the forward as one graph launch of the smallest bucket that holds it; the
// kernels read its token count from device memory.  Decoding and
// substitution follow on the same stream as before.  The fixed buffers are
// taken from the HBM budget before the arena.
#include <string.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "sched.hpp"

using namespace anon;
using anon::sched::Request;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device buffers of one micro-batch, carved from its arena block.
struct BatchBufs {
  int32_t *ids, *cu, *tok_off, *cu_spans;
  uint8_t *text, *labels, *out;
  int64_t *cu_bytes, *cu_out;
  anon_span* spans;
  uint32_t* err;
  void *ws_ner, *ws_dec, *ws_ps;
  size_t ws_ner_b, ws_dec_b, ws_ps_b;
};

struct HipExecutor {
  anon_model* model = nullptr;
  anon_pcache* cache = nullptr;
  int n_types = 1;
  char* arena = nullptr;  // device
  bool graphs = false;    // NER forward as bucket graph replays
  std::vector<int> buckets;  // token capacities, largest first
  std::atomic<int64_t> graph_launches{0};

  // a slot's fixed forward buffers (graph mode), for T tokens at most
  struct GraphBufs {
    int32_t *ids, *cu, *n_tok;
    uint8_t* labels;
    uint32_t* err;
    void* ws;
    size_t ws_b;
  };
  void plan_fixed(Carver& k, int T, GraphBufs& g) const {
    g.ids = k.take<int32_t>(T);
    g.cu = k.take<int32_t>((size_t)T + 1);
    g.n_tok = k.take<int32_t>(1);
    g.labels = k.take<uint8_t>(T);
    g.err = k.take<uint32_t>(64);
    g.ws_b = 0;
    anon_ner_workspace_size(model, T, T, &g.ws_b);
    g.ws = k.take<uint8_t>(g.ws_b);
  }

  struct SlotRes {
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int phase = 0;  // event being waited on
    int B = 0, T = 0, span_cap = 0;
    int64_t nbytes = 0, out_cap = 0;
    BatchBufs d{};
    GraphBufs g{};
    std::vector<anon_graph*> graph;  // per bucket
    // pinned host staging, sized for the largest micro-batch
    void* hmem = nullptr;
    int32_t *h_ids, *h_cu, *h_tok_off, *h_cu_spans, *h_ntok;
    uint8_t *h_text, *h_labels, *h_out;
    int64_t *h_cu_bytes, *h_cu_out;
    anon_span* h_spans;
    uint32_t* h_err;
  };
  std::vector<SlotRes> slots;

  static int span_cap_for(int T) { return T; }  // at most one span per token
  // "[" + type (<= 32) + "_" + slug (<= 64) + "]" per span, besides the text
  static int64_t out_cap_for(int T, int64_t nb) { return nb + (int64_t)T * 99; }

  // A micro-batch's arena block.  In graph mode its ids, boundaries,
  // labels, error word and NER workspace are the slot's fixed buffers.
  void plan(Carver& k, int B, int T, int64_t nb, BatchBufs& b) const {
    const int sc = span_cap_for(T);
    b.ids = graphs ? nullptr : k.take<int32_t>(T);
    b.cu = graphs ? nullptr : k.take<int32_t>(B + 1);
    b.tok_off = k.take<int32_t>(2 * (size_t)T);
    b.text = k.take<uint8_t>(nb);
    b.cu_bytes = k.take<int64_t>(B + 1);
    b.labels = graphs ? nullptr : k.take<uint8_t>(T);
    b.spans = k.take<anon_span>(sc);
    b.cu_spans = k.take<int32_t>(B + 1);
    b.out = k.take<uint8_t>(out_cap_for(T, nb));
    b.cu_out = k.take<int64_t>(B + 1);
    b.err = graphs ? nullptr : k.take<uint32_t>(64);
    b.ws_ner_b = b.ws_dec_b = b.ws_ps_b = 0;
    if (!graphs) anon_ner_workspace_size(model, T, B, &b.ws_ner_b);
    anon_decode_workspace_size(T, B, &b.ws_dec_b);
    anon_pseudonymize_workspace_size(B, sc, &b.ws_ps_b);
    b.ws_ner = graphs ? nullptr : k.take<uint8_t>(b.ws_ner_b);
    b.ws_dec = k.take<uint8_t>(b.ws_dec_b);
    b.ws_ps = k.take<uint8_t>(b.ws_ps_b);
  }

  int64_t footprint(int B, int T, int64_t nb) const {
    Carver k(nullptr, SIZE_MAX);
    BatchBufs b;
    plan(k, B, T, nb, b);
    return (int64_t)k.used + 256;
  }

  static void carve_host(SlotRes& s, Carver& h, int T, int B, int64_t nb) {
    s.h_ids = h.take<int32_t>(T);
    s.h_cu = h.take<int32_t>(B + 1);
    s.h_tok_off = h.take<int32_t>(2 * (size_t)T);
    s.h_text = h.take<uint8_t>(nb);
    s.h_cu_bytes = h.take<int64_t>(B + 1);
    s.h_labels = h.take<uint8_t>(T);
    s.h_spans = h.take<anon_span>(span_cap_for(T));
    s.h_cu_spans = h.take<int32_t>(B + 1);
    s.h_out = h.take<uint8_t>(out_cap_for(T, nb));
    s.h_cu_out = h.take<int64_t>(B + 1);
    s.h_err = h.take<uint32_t>(64);
    s.h_ntok = h.take<int32_t>(1);
  }

  // smallest bucket that holds T tokens (buckets run largest first)
  int bucket_for(int T) const {
    int b = 0;
    while (b + 1 < (int)buckets.size() && buckets[b + 1] >= T) ++b;
    return b;
  }

  anon_status enqueue(int i, std::vector<Request*>& reqs, int64_t off) {
    SlotRes& s = slots[i];
    int B = 0, T = 0;
    int64_t nb = 0;
    s.h_cu[0] = 0;
    s.h_cu_bytes[0] = 0;
    for (Request* r : reqs) {
      memcpy(s.h_ids + T, r->ids.data(), r->ids.size() * 4);
      memcpy(s.h_tok_off + 2 * (size_t)T, r->tok_off.data(), r->tok_off.size() * 4);
      memcpy(s.h_text + nb, r->text.data(), r->text.size());
      for (int b = 0; b < r->n_records; ++b) {
        s.h_cu[B + b + 1] = T + r->cu[b + 1];
        s.h_cu_bytes[B + b + 1] = nb + r->cu_bytes[b + 1];
      }
      B += r->n_records;
      T += r->n_tokens;
      nb += r->n_bytes;
    }
    s.B = B;
    s.T = T;
    s.nbytes = nb;
    s.span_cap = span_cap_for(T);
    s.out_cap = out_cap_for(T, nb);
    const int64_t fp = footprint(B, T, nb);
    Carver k(arena + off, (size_t)fp);
    plan(k, B, T, nb, s.d);
    if (!k.ok()) return set_error(ANON_EINVAL, "micro-batch carve exceeds its arena block");
    const BatchBufs& d = s.d;
    hipStream_t st = s.stream;
    // graph mode: the forward's inputs and outputs are the slot's fixed buffers
    int32_t* ids = graphs ? s.g.ids : d.ids;
    int32_t* cu = graphs ? s.g.cu : d.cu;
    uint8_t* labels = graphs ? s.g.labels : d.labels;
    uint32_t* err = graphs ? s.g.err : d.err;
    const int bk = graphs ? bucket_for(T) : 0;
    int n_cu = B + 1;
    if (graphs) {  // empty records up to the bucket's record capacity
      n_cu = buckets[bk] + 1;
      for (int b = B + 1; b < n_cu; ++b) s.h_cu[b] = T;
      *s.h_ntok = T;
      ANON_HIP_CHECK(hipMemcpyAsync(s.g.n_tok, s.h_ntok, 4, hipMemcpyHostToDevice, st));
    }
    ANON_HIP_CHECK(hipMemcpyAsync(ids, s.h_ids, (size_t)T * 4, hipMemcpyHostToDevice, st));
    ANON_HIP_CHECK(hipMemcpyAsync(cu, s.h_cu, (size_t)n_cu * 4, hipMemcpyHostToDevice, st));
    ANON_HIP_CHECK(hipMemcpyAsync(d.tok_off, s.h_tok_off, (size_t)T * 8, hipMemcpyHostToDevice, st));
    if (nb > 0) ANON_HIP_CHECK(hipMemcpyAsync(d.text, s.h_text, nb, hipMemcpyHostToDevice, st));
    ANON_HIP_CHECK(hipMemcpyAsync(d.cu_bytes, s.h_cu_bytes, (size_t)(B + 1) * 8, hipMemcpyHostToDevice, st));
    launch_fill_u8((uint8_t*)err, 0, 4, st);
    ANON_HIP_CHECK(hipGetLastError());
    // this micro-batch's device-data errors go to its own word (graph mode:
    // the slot's, which the slot's graphs were captured with)
    set_thread_error_word(err);
    anon_status rc;
    if (graphs) {
      rc = anon_graph_launch(s.graph[bk], st);
      if (rc == ANON_OK) ++graph_launches;
    } else {
      rc = ner_forward(model, ids, cu, B, T, labels, nullptr, nullptr, d.ws_ner, d.ws_ner_b, st);
    }
    if (rc == ANON_OK)
      rc = decode_spans(labels, d.tok_off, cu, B, T, n_types, d.spans, s.span_cap, d.cu_spans, d.ws_dec,
                        d.ws_dec_b, st);
    if (rc == ANON_OK)
      rc = pseudonymize(cache, d.text, d.cu_bytes, B, d.spans, d.cu_spans, s.span_cap, d.out, s.out_cap, d.cu_out,
                        d.ws_ps, d.ws_ps_b, st);
    set_thread_error_word(nullptr);
    if (rc != ANON_OK) return rc;
    ANON_HIP_CHECK(hipMemcpyAsync(s.h_labels, labels, (size_t)T, hipMemcpyDeviceToHost, st));
    ANON_HIP_CHECK(hipMemcpyAsync(s.h_cu_spans, d.cu_spans, (size_t)(B + 1) * 4, hipMemcpyDeviceToHost, st));
    ANON_HIP_CHECK(hipMemcpyAsync(s.h_cu_out, d.cu_out, (size_t)(B + 1) * 8, hipMemcpyDeviceToHost, st));
    ANON_HIP_CHECK(hipMemcpyAsync(s.h_err, err, 4, hipMemcpyDeviceToHost, st));
    ANON_HIP_CHECK(hipEventRecord(s.ev[0], st));
    s.phase = 0;
    return ANON_OK;
  }

  // --- executor interface ---------------------------------------------------
  anon_status launch(int i, std::vector<Request*>& reqs, int64_t off) {
    (void)hipSetDevice(device);
    const anon_status rc = enqueue(i, reqs, off);
    // nothing may still use the block when the scheduler takes it back
    if (rc != ANON_OK) (void)hipStreamSynchronize(slots[i].stream);
    return rc;
  }
  int query(int i) {
    const hipError_t q = hipEventQuery(slots[i].ev[slots[i].phase]);
    if (q == hipErrorNotReady) return 0;
    return q == hipSuccess ? 1 : (int)ANON_EDEVICE;
  }
  anon_status drain(int i) {
    SlotRes& s = slots[i];
    if (*s.h_err) return set_error(ANON_EDATA, "malformed data in the micro-batch (error bits " +
                                                   std::to_string(*s.h_err) + ")");
    const int nsp = s.h_cu_spans[s.B];
    const int64_t nout = s.h_cu_out[s.B];
    if (nsp > s.span_cap || nout > s.out_cap) return set_error(ANON_ECAPACITY, "micro-batch output overflow");
    if (nsp > 0)
      ANON_HIP_CHECK(hipMemcpyAsync(s.h_spans, s.d.spans, (size_t)nsp * sizeof(anon_span), hipMemcpyDeviceToHost,
                                    s.stream));
    if (nout > 0) ANON_HIP_CHECK(hipMemcpyAsync(s.h_out, s.d.out, nout, hipMemcpyDeviceToHost, s.stream));
    ANON_HIP_CHECK(hipEventRecord(s.ev[1], s.stream));
    s.phase = 1;
    return ANON_OK;
  }
  void finish(int i, std::vector<Request*>& reqs, anon_status st) {
    SlotRes& s = slots[i];
    if (st != ANON_OK) {
      // the block goes back to the arena: let the stream drain first
      (void)hipStreamSynchronize(s.stream);
      return;
    }
    int rb = 0, rt = 0;
    for (Request* r : reqs) {
      r->labels.assign(s.h_labels + rt, s.h_labels + rt + r->n_tokens);
      const int s0 = s.h_cu_spans[rb], s1 = s.h_cu_spans[rb + r->n_records];
      r->spans.assign(s.h_spans + s0, s.h_spans + s1);
      for (auto& sp : r->spans) sp.record -= rb;
      const int64_t o0 = s.h_cu_out[rb], o1 = s.h_cu_out[rb + r->n_records];
      r->out.assign(s.h_out + o0, s.h_out + o1);
      r->cu_out.resize(r->n_records + 1);
      for (int b = 0; b <= r->n_records; ++b) r->cu_out[b] = s.h_cu_out[rb + b] - o0;
      rb += r->n_records;
      rt += r->n_tokens;
    }
  }
  double now() const { return now_s(); }

  int device = 0;
};

}  // namespace

struct anon_server {
  HipExecutor ex;
  std::unique_ptr<anon::sched::Scheduler<HipExecutor>> sch;
  anon_server_config cfg;
  int vocab = 0, max_pos = 0;
  int64_t max_bytes = 0;
  void* arena_mem = nullptr;
  void* fixed_mem = nullptr;  // the slots' forward buffers (graph mode)
  std::thread th;
};

static void free_server(anon_server* sv) {
  sv->sch.reset();
  for (auto& s : sv->ex.slots) {
    for (anon_graph* g : s.graph) anon_graph_free(g);
    for (auto& e : s.ev)
      if (e) (void)hipEventDestroy(e);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.hmem) (void)hipHostFree(s.hmem);
  }
  if (sv->arena_mem) (void)hipFree(sv->arena_mem);
  if (sv->fixed_mem) (void)hipFree(sv->fixed_mem);
  delete sv;
}

extern "C" {

anon_status anon_server_start(anon_model* model, anon_pcache* cache, const anon_server_config* cfg,
                              anon_server** out) {
  clear_error();
  if (!out || !model || !cache || !cfg) return set_error(ANON_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->max_batch_tokens < 1 || cfg->n_streams < 1 || cfg->n_streams > 8 || cfg->max_queue < 1 ||
      cfg->hbm_budget_bytes <= 0 || cfg->graph_buckets < 0 || cfg->graph_buckets > 16)
    return set_error(ANON_EINVAL, "bad server config");
  anon_server* sv = new anon_server();
  sv->cfg = *cfg;
  if (sv->cfg.max_request_tokens <= 0 || sv->cfg.max_request_tokens > cfg->max_batch_tokens)
    sv->cfg.max_request_tokens = cfg->max_batch_tokens;
  const anon_model_config* mc = model_config(model);
  sv->vocab = mc->vocab;
  sv->max_pos = mc->max_pos;
  HipExecutor& ex = sv->ex;
  ex.model = model;
  ex.cache = cache;
  ex.n_types = std::max(1, (mc->n_labels - 1) / 2);
  (void)hipGetDevice(&ex.device);
  const int T = cfg->max_batch_tokens;
  sv->max_bytes = (int64_t)T * 64;  // text bytes per micro-batch (64 per token)
  anon::sched::Limits lim;
  lim.max_batch_tokens = T;
  lim.max_records = T;  // every record holds at least one token
  lim.max_bytes = sv->max_bytes;
  lim.max_queue = cfg->max_queue;
  // the arena: the budget, but no more than all slots can fill at once; it
  // must hold the largest request that submit accepts
  // graph buckets: max_batch_tokens, then halving, at least 1 token each
  ex.graphs = cfg->graph_buckets > 0;
  for (int b = 0, cap = T; b < cfg->graph_buckets && cap >= 1; ++b, cap /= 2) ex.buckets.push_back(cap);
  int64_t fixed_slot = 0;
  if (ex.graphs) {
    Carver fk(nullptr, SIZE_MAX);
    HipExecutor::GraphBufs g;
    ex.plan_fixed(fk, T, g);
    fixed_slot = (int64_t)align_up(fk.used, 256);
  }
  const int64_t fixed = fixed_slot * cfg->n_streams;
  const int Rq = sv->cfg.max_request_tokens;
  const int64_t fp_slot = ex.footprint(T, T, sv->max_bytes);
  const int64_t fp_req = ex.footprint(Rq, Rq, (int64_t)Rq * 64);
  const int64_t arena =
      std::max<int64_t>(0, std::min<int64_t>(cfg->hbm_budget_bytes - fixed, fp_slot * cfg->n_streams)) / 256 * 256;
  if (arena < anon::sched::Arena::granule(fp_req)) {
    free_server(sv);
    return set_error(ANON_ENOMEM, "the largest admissible request needs " + std::to_string(fp_req) +
                                      " device bytes besides " + std::to_string(fixed) +
                                      " bytes of slot buffers, over the HBM budget of " +
                                      std::to_string(cfg->hbm_budget_bytes));
  }
  if (hipMalloc(&sv->arena_mem, arena) != hipSuccess) {
    free_server(sv);
    return set_error(ANON_ENOMEM, "cannot allocate the " + std::to_string(arena) + "-byte activation arena");
  }
  if (fixed > 0 && hipMalloc(&sv->fixed_mem, fixed) != hipSuccess) {
    free_server(sv);
    return set_error(ANON_ENOMEM, "cannot allocate " + std::to_string(fixed) + " bytes of slot buffers");
  }
  ex.arena = (char*)sv->arena_mem;
  ex.slots.resize(cfg->n_streams);
  Carver hl(nullptr, SIZE_MAX);
  HipExecutor::carve_host(ex.slots[0], hl, T, T, sv->max_bytes);
  const size_t hbytes = hl.used + 256;
  for (auto& s : ex.slots) {
    if (hipHostMalloc(&s.hmem, hbytes, 0) != hipSuccess ||
        hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s.ev[1], hipEventDisableTiming) != hipSuccess) {
      free_server(sv);
      return set_error(ANON_ENOMEM, "cannot allocate server slots");
    }
    Carver h(s.hmem, hbytes);
    HipExecutor::carve_host(s, h, T, T, sv->max_bytes);
  }
  // one forward graph per bucket and slot, captured on the slot's buffers
  // with the slot's error word (the model's tile choices are fixed now)
  for (int i = 0; ex.graphs && i < cfg->n_streams; ++i) {
    HipExecutor::SlotRes& s = ex.slots[i];
    Carver fk((char*)sv->fixed_mem + fixed_slot * i, (size_t)fixed_slot);
    ex.plan_fixed(fk, T, s.g);
    for (int cap : ex.buckets) {
      anon_graph* g = nullptr;
      set_thread_error_word(s.g.err);
      const anon_status rc = ner_forward_capture_bucket(model, s.g.ids, s.g.cu, s.g.n_tok, cap, cap, s.g.labels,
                                                        nullptr, nullptr, s.g.ws, s.g.ws_b, &g);
      set_thread_error_word(nullptr);
      if (rc != ANON_OK) {
        const std::string why = anon_last_error();
        free_server(sv);
        return set_error(rc, "capturing the forward of the " + std::to_string(cap) + "-token bucket: " + why);
      }
      s.graph.push_back(g);
    }
  }
  sv->sch.reset(new anon::sched::Scheduler<HipExecutor>(ex, cfg->n_streams, lim, arena));
  sv->th = std::thread([sv] {
    (void)hipSetDevice(sv->ex.device);
    sv->sch->run();
  });
  *out = sv;
  return ANON_OK;
}

anon_status anon_submit(anon_server* sv, const anon_request* req, uint64_t* ticket) {
  clear_error();
  if (!sv || !req || !ticket) return set_error(ANON_EINVAL, "NULL argument");
  std::string why;
  anon_status st = anon::sched::validate_request(*req, sv->vocab, sv->max_pos, sv->cfg.max_request_tokens,
                                                 sv->max_bytes, &why);
  if (st != ANON_OK) return set_error(st, why);
  const int B = req->n_records, T = req->cu_seqlens[B];
  const int64_t nb = req->cu_bytes[B];
  Request* r = new Request();
  r->n_records = B;
  r->n_tokens = T;
  r->n_bytes = nb;
  r->ids.assign(req->ids, req->ids + T);
  r->cu.assign(req->cu_seqlens, req->cu_seqlens + B + 1);
  r->tok_off.assign(req->tok_off, req->tok_off + 2 * (size_t)T);
  r->text.assign(req->text, req->text + nb);
  r->cu_bytes.assign(req->cu_bytes, req->cu_bytes + B + 1);
  st = sv->sch->submit(r, ticket, &why);
  if (st != ANON_OK) return set_error(st, why);
  return ANON_OK;
}

anon_status anon_poll(anon_server* sv, uint64_t ticket, anon_result* out) {
  if (!sv || !out) return set_error(ANON_EINVAL, "NULL argument");
  const Request* r = nullptr;
  const anon_status st = sv->sch->poll(ticket, &r);
  if (st == ANON_ENOTFOUND) return set_error(ANON_ENOTFOUND, "unknown ticket");
  if (st != ANON_OK) return st;
  out->status = r->status;
  out->n_records = r->n_records;
  out->n_tokens = r->n_tokens;
  out->n_spans = (int32_t)r->spans.size();
  out->out = r->out.data();
  out->cu_out = r->cu_out.data();
  out->labels = r->labels.data();
  out->spans = r->spans.data();
  out->t_submit = r->t_submit;
  out->t_start = r->t_start;
  out->t_done = r->t_done;
  return ANON_OK;
}

anon_status anon_release(anon_server* sv, uint64_t ticket) {
  if (!sv) return set_error(ANON_EINVAL, "NULL argument");
  const anon_status st = sv->sch->release(ticket);
  if (st == ANON_ENOTFOUND) return set_error(st, "unknown ticket");
  if (st == ANON_EBUSY) return set_error(st, "request still running");
  return st;
}

anon_status anon_server_stats(anon_server* sv, anon_server_counters* out) {
  if (!sv || !out) return set_error(ANON_EINVAL, "NULL argument");
  out->arena_bytes = sv->sch->arena_capacity();
  int conc = 0;
  sv->sch->stats(&out->peak_arena_bytes, &out->micro_batches, &conc);
  out->max_concurrent = conc;
  out->graph_launches = sv->ex.graph_launches.load();
  return ANON_OK;
}

anon_status anon_server_stop(anon_server* sv) {
  if (!sv) return set_error(ANON_EINVAL, "NULL argument");
  sv->sch->stop();
  if (sv->th.joinable()) sv->th.join();
  free_server(sv);
  return ANON_OK;
}

}  // extern "C"
