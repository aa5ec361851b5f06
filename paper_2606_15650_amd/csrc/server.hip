// Serving loop: continuous batching of record batches on one GPU.
//
// anon_submit copies a request into host memory and queues it.  A scheduler
// thread owns `n_streams` slots; each slot has its own HIP stream, pinned
// host staging and device buffers sized for `max_batch_tokens` tokens, so the
// device memory of all slots is allocated once, at start, and must fit the
// HBM budget.  Whenever a slot is free and requests wait, the thread packs
// queued requests (FIFO) into one micro-batch up to the slot's token, record
// and byte limits and launches NER -> span decoding -> substitution on the
// slot's stream; other slots keep running meanwhile.  When a slot's event
// completes, its outputs are copied back and split per request, and the slot
// takes the next micro-batch.  Every kernel computes each record
// independently of its batch-mates, so a request's result is the same alone
// or mixed with others.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"

using namespace anon;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket;
  int n_records = 0, n_tokens = 0;
  int64_t n_bytes = 0;
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

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<Req*> reqs;
  int B = 0, T = 0;
  int64_t nbytes = 0;
  // device
  void* dmem = nullptr;
  int32_t *d_ids, *d_cu, *d_tok_off, *d_cu_spans;
  uint8_t *d_text, *d_labels, *d_out;
  int64_t *d_cu_bytes, *d_cu_out;
  anon_span* d_spans;
  void *ws_ner, *ws_dec, *ws_ps;
  size_t ws_ner_b, ws_dec_b, ws_ps_b;
  // pinned host staging
  void* hmem = nullptr;
  int32_t *h_ids, *h_cu, *h_tok_off, *h_cu_spans;
  uint8_t *h_text, *h_labels, *h_out;
  int64_t *h_cu_bytes, *h_cu_out;
  anon_span* h_spans;
};

}  // namespace

struct anon_server {
  anon_model* model;
  anon_pcache* cache;
  anon_server_config cfg;
  int device;
  int max_records;
  int64_t max_bytes, out_cap;
  int span_cap;
  int n_types;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread th;
};

static void carve_slot(anon_server* sv, Slot& s, Carver& d, Carver& h) {
  const int T = sv->cfg.max_batch_tokens, B = sv->max_records;
  s.d_ids = d.take<int32_t>(T);
  s.d_cu = d.take<int32_t>(B + 1);
  s.d_tok_off = d.take<int32_t>(2 * (size_t)T);
  s.d_text = d.take<uint8_t>(sv->max_bytes);
  s.d_cu_bytes = d.take<int64_t>(B + 1);
  s.d_labels = d.take<uint8_t>(T);
  s.d_spans = d.take<anon_span>(sv->span_cap);
  s.d_cu_spans = d.take<int32_t>(B + 1);
  s.d_out = d.take<uint8_t>(sv->out_cap);
  s.d_cu_out = d.take<int64_t>(B + 1);
  s.ws_ner = d.take<uint8_t>(s.ws_ner_b);
  s.ws_dec = d.take<uint8_t>(s.ws_dec_b);
  s.ws_ps = d.take<uint8_t>(s.ws_ps_b);
  s.h_ids = h.take<int32_t>(T);
  s.h_cu = h.take<int32_t>(B + 1);
  s.h_tok_off = h.take<int32_t>(2 * (size_t)T);
  s.h_text = h.take<uint8_t>(sv->max_bytes);
  s.h_cu_bytes = h.take<int64_t>(B + 1);
  s.h_labels = h.take<uint8_t>(T);
  s.h_spans = h.take<anon_span>(sv->span_cap);
  s.h_cu_spans = h.take<int32_t>(B + 1);
  s.h_out = h.take<uint8_t>(sv->out_cap);
  s.h_cu_out = h.take<int64_t>(B + 1);
}

// Packs the requests of s.reqs and enqueues the whole path on the slot stream.
static anon_status launch_slot(anon_server* sv, Slot& s) {
  int B = 0, T = 0;
  int64_t nb = 0;
  s.h_cu[0] = 0;
  s.h_cu_bytes[0] = 0;
  for (Req* r : s.reqs) {
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
  hipStream_t st = s.stream;
  ANON_HIP_CHECK(hipMemcpyAsync(s.d_ids, s.h_ids, (size_t)T * 4, hipMemcpyHostToDevice, st));
  ANON_HIP_CHECK(hipMemcpyAsync(s.d_cu, s.h_cu, (size_t)(B + 1) * 4, hipMemcpyHostToDevice, st));
  ANON_HIP_CHECK(hipMemcpyAsync(s.d_tok_off, s.h_tok_off, (size_t)T * 8, hipMemcpyHostToDevice, st));
  if (nb > 0) ANON_HIP_CHECK(hipMemcpyAsync(s.d_text, s.h_text, nb, hipMemcpyHostToDevice, st));
  ANON_HIP_CHECK(hipMemcpyAsync(s.d_cu_bytes, s.h_cu_bytes, (size_t)(B + 1) * 8, hipMemcpyHostToDevice, st));
  anon_status rc = ner_forward(sv->model, s.d_ids, s.d_cu, B, T, s.d_labels, nullptr, nullptr, s.ws_ner,
                               s.ws_ner_b, st);
  if (rc != ANON_OK) return rc;
  rc = decode_spans(s.d_labels, s.d_tok_off, s.d_cu, B, T, sv->n_types, s.d_spans, sv->span_cap, s.d_cu_spans,
                    s.ws_dec, s.ws_dec_b, st);
  if (rc != ANON_OK) return rc;
  rc = pseudonymize(sv->cache, s.d_text, s.d_cu_bytes, B, s.d_spans, s.d_cu_spans, sv->span_cap, s.d_out,
                    sv->out_cap, s.d_cu_out, s.ws_ps, s.ws_ps_b, st);
  if (rc != ANON_OK) return rc;
  ANON_HIP_CHECK(hipMemcpyAsync(s.h_labels, s.d_labels, (size_t)T, hipMemcpyDeviceToHost, st));
  ANON_HIP_CHECK(hipMemcpyAsync(s.h_cu_spans, s.d_cu_spans, (size_t)(B + 1) * 4, hipMemcpyDeviceToHost, st));
  ANON_HIP_CHECK(hipMemcpyAsync(s.h_cu_out, s.d_cu_out, (size_t)(B + 1) * 8, hipMemcpyDeviceToHost, st));
  ANON_HIP_CHECK(hipEventRecord(s.done, st));
  return ANON_OK;
}

// Copies the variable-size outputs back and splits them per request.
static void finish_slot(anon_server* sv, Slot& s, int status) {
  const double t = now_s();
  int nsp = 0;
  int64_t nout = 0;
  if (status == ANON_OK) {
    nsp = s.h_cu_spans[s.B];
    nout = s.h_cu_out[s.B];
    if (nsp > sv->span_cap || nout > sv->out_cap) status = ANON_ECAPACITY;
  }
  if (status == ANON_OK) {
    hipError_t e = hipSuccess;
    if (nsp > 0) e = hipMemcpyAsync(s.h_spans, s.d_spans, (size_t)nsp * sizeof(anon_span), hipMemcpyDeviceToHost,
                                    s.stream);
    if (e == hipSuccess && nout > 0) e = hipMemcpyAsync(s.h_out, s.d_out, nout, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) status = ANON_EDEVICE;
  }
  int rb = 0, rt = 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  for (Req* r : s.reqs) {
    r->status = status;
    r->t_done = t;
    if (status == ANON_OK) {
      r->labels.assign(s.h_labels + rt, s.h_labels + rt + r->n_tokens);
      const int s0 = s.h_cu_spans[rb], s1 = s.h_cu_spans[rb + r->n_records];
      r->spans.assign(s.h_spans + s0, s.h_spans + s1);
      for (auto& sp : r->spans) sp.record -= rb;
      const int64_t o0 = s.h_cu_out[rb], o1 = s.h_cu_out[rb + r->n_records];
      r->out.assign(s.h_out + o0, s.h_out + o1);
      r->cu_out.resize(r->n_records + 1);
      for (int b = 0; b <= r->n_records; ++b) r->cu_out[b] = s.h_cu_out[rb + b] - o0;
    }
    rb += r->n_records;
    rt += r->n_tokens;
  }
  s.reqs.clear();
  s.busy = false;
  sv->cv.notify_all();
}

static void server_loop(anon_server* sv) {
  hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // retire finished slots
    bool any_busy = false;
    for (Slot& s : sv->slots) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      lk.unlock();
      finish_slot(sv, s, q == hipSuccess ? ANON_OK : ANON_EDEVICE);
      lk.lock();
    }
    if (sv->stopping && !any_busy) break;
    // admit queued requests into free slots
    if (!sv->stopping) {
      for (Slot& s : sv->slots) {
        if (s.busy || sv->queue.empty()) continue;
        int B = 0, T = 0;
        int64_t nb = 0;
        while (!sv->queue.empty()) {
          Req* r = sv->queue.front();
          if (T + r->n_tokens > sv->cfg.max_batch_tokens || B + r->n_records > sv->max_records ||
              nb + r->n_bytes > sv->max_bytes)
            break;
          sv->queue.pop_front();
          s.reqs.push_back(r);
          B += r->n_records;
          T += r->n_tokens;
          nb += r->n_bytes;
        }
        if (s.reqs.empty()) continue;
        const double t = now_s();
        for (Req* r : s.reqs) r->t_start = t;
        s.busy = true;
        any_busy = true;
        lk.unlock();
        const anon_status rc = launch_slot(sv, s);
        if (rc != ANON_OK) finish_slot(sv, s, rc);
        lk.lock();
      }
    }
    if (any_busy) sv->cv.wait_for(lk, std::chrono::microseconds(50));
    else sv->cv.wait(lk, [&] { return sv->stopping || !sv->queue.empty(); });
  }
  // fail what is still queued
  for (Req* r : sv->queue) {
    r->status = ANON_EBUSY;
    r->t_done = now_s();
  }
  sv->queue.clear();
}

static void free_server(anon_server* sv) {
  for (Slot& s : sv->slots) {
    if (s.done) hipEventDestroy(s.done);
    if (s.stream) hipStreamDestroy(s.stream);
    if (s.dmem) hipFree(s.dmem);
    if (s.hmem) hipHostFree(s.hmem);
  }
  for (auto& kv : sv->reqs) delete kv.second;
  delete sv;
}

extern "C" {

anon_status anon_server_start(anon_model* model, anon_pcache* cache, const anon_server_config* cfg,
                              anon_server** out) {
  clear_error();
  if (!out || !model || !cache || !cfg) return set_error(ANON_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->max_batch_tokens < 1 || cfg->n_streams < 1 || cfg->n_streams > 8 || cfg->max_queue < 1 ||
      cfg->hbm_budget_bytes <= 0)
    return set_error(ANON_EINVAL, "bad server config");
  anon_server* sv = new anon_server();
  sv->model = model;
  sv->cache = cache;
  sv->cfg = *cfg;
  if (sv->cfg.max_request_tokens <= 0 || sv->cfg.max_request_tokens > cfg->max_batch_tokens)
    sv->cfg.max_request_tokens = cfg->max_batch_tokens;
  int dev = 0;
  hipGetDevice(&dev);
  sv->device = dev;
  const int T = cfg->max_batch_tokens;
  sv->max_records = T;  // every record holds at least one token
  sv->max_bytes = (int64_t)T * 64;
  sv->span_cap = T;
  sv->out_cap = sv->max_bytes + (int64_t)T * 99;  // "[" + 32-char type + "_" + 64 hex + "]"
  sv->n_types = (model_config(model)->n_labels - 1) / 2;
  if (sv->n_types < 1) sv->n_types = 1;
  size_t ws_ner = 0, ws_dec = 0, ws_ps = 0;
  anon_ner_workspace_size(model, T, sv->max_records, &ws_ner);
  anon_decode_workspace_size(T, sv->max_records, &ws_dec);
  anon_pseudonymize_workspace_size(sv->max_records, sv->span_cap, &ws_ps);
  sv->slots.resize(cfg->n_streams);
  for (Slot& s : sv->slots) {
    s.ws_ner_b = ws_ner;
    s.ws_dec_b = ws_dec;
    s.ws_ps_b = ws_ps;
  }
  Carver dl(nullptr, SIZE_MAX), hl(nullptr, SIZE_MAX);
  carve_slot(sv, sv->slots[0], dl, hl);
  const size_t dbytes = dl.used + 256, hbytes = hl.used + 256;
  if ((int64_t)dbytes * cfg->n_streams > cfg->hbm_budget_bytes) {
    delete sv;
    return set_error(ANON_ENOMEM, "n_streams slots of max_batch_tokens need " +
                                      std::to_string(dbytes * cfg->n_streams) + " bytes, over the HBM budget");
  }
  for (Slot& s : sv->slots) {
    if (hipMalloc(&s.dmem, dbytes) != hipSuccess || hipHostMalloc(&s.hmem, hbytes, 0) != hipSuccess ||
        hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      free_server(sv);
      return set_error(ANON_ENOMEM, "cannot allocate server slots");
    }
    Carver d(s.dmem, dbytes), h(s.hmem, hbytes);
    carve_slot(sv, s, d, h);
  }
  sv->th = std::thread(server_loop, sv);
  *out = sv;
  return ANON_OK;
}

anon_status anon_submit(anon_server* sv, const anon_request* req, uint64_t* ticket) {
  clear_error();
  if (!sv || !req || !ticket) return set_error(ANON_EINVAL, "NULL argument");
  const int B = req->n_records;
  if (B < 1 || !req->cu_seqlens || !req->cu_bytes) return set_error(ANON_EINVAL, "request has no records");
  const int T = req->cu_seqlens[B];
  if (req->cu_seqlens[0] != 0 || req->cu_bytes[0] != 0) return set_error(ANON_EINVAL, "cu arrays must start at 0");
  for (int b = 0; b < B; ++b) {
    const int n = req->cu_seqlens[b + 1] - req->cu_seqlens[b];
    if (n < 1 || n > model_config(sv->model)->max_pos)
      return set_error(ANON_EINVAL, "record lengths must be in [1, max_pos]");
    if (req->cu_bytes[b + 1] < req->cu_bytes[b]) return set_error(ANON_EINVAL, "cu_bytes must be non-decreasing");
  }
  const int64_t nb = req->cu_bytes[B];
  if (T > sv->cfg.max_request_tokens || nb > sv->max_bytes)
    return set_error(ANON_EINVAL, "request larger than a micro-batch");
  if (T > 0 && (!req->ids || !req->tok_off)) return set_error(ANON_EINVAL, "ids/tok_off NULL");
  if (nb > 0 && !req->text) return set_error(ANON_EINVAL, "text NULL");
  for (int t = 0; t < T; ++t)
    if (req->ids[t] < 0 || req->ids[t] >= model_config(sv->model)->vocab)
      return set_error(ANON_EINVAL, "token id out of range");
  Req* r = new Req();
  r->n_records = B;
  r->n_tokens = T;
  r->n_bytes = nb;
  r->ids.assign(req->ids, req->ids + T);
  r->cu.assign(req->cu_seqlens, req->cu_seqlens + B + 1);
  r->tok_off.assign(req->tok_off, req->tok_off + 2 * (size_t)T);
  r->text.assign(req->text, req->text + nb);
  r->cu_bytes.assign(req->cu_bytes, req->cu_bytes + B + 1);
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stopping) {
    delete r;
    return set_error(ANON_EBUSY, "server is stopping");
  }
  if ((int)sv->queue.size() >= sv->cfg.max_queue) {
    delete r;
    return set_error(ANON_EBUSY, "queue full");
  }
  r->ticket = sv->next_ticket++;
  sv->reqs[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv.notify_all();
  return ANON_OK;
}

anon_status anon_poll(anon_server* sv, uint64_t ticket, anon_result* out) {
  if (!sv || !out) return set_error(ANON_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(ANON_ENOTFOUND, "unknown ticket");
  Req* r = it->second;
  if (r->status == ANON_PENDING) return ANON_PENDING;
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
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(ANON_ENOTFOUND, "unknown ticket");
  if (it->second->status == ANON_PENDING) return set_error(ANON_EBUSY, "request still running");
  delete it->second;
  sv->reqs.erase(it);
  return ANON_OK;
}

anon_status anon_server_stop(anon_server* sv) {
  if (!sv) return set_error(ANON_EINVAL, "NULL argument");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  free_server(sv);
  return ANON_OK;
}

}  // extern "C"
