// pq_serve.cpp -- the scan server: a request loop over resident files that
// admits scan requests against a device-memory budget, batches every
// admitted request that fits into one batched scan (continuous batching:
// requests that arrive while earlier batches run join the next batch, which
// starts as soon as a slot -- a stream -- and memory are free, so batches
// overlap on the device), keeps results resident until their client
// releases them (identical requests share a resident result), and reports
// per-request latency.  Built on the public batch calls of pq.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pq.h"

namespace {

using Clock = std::chrono::steady_clock;

thread_local char t_msg[256];
pq_status sfail(pq_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_msg, sizeof(t_msg), fmt, ap);
  va_end(ap);
  return s;
}

constexpr uint64_t ALIGN = 256;
inline uint64_t up(uint64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over one device arena: free ranges by offset,
// neighbours merged on release.
struct Arena {
  uint8_t* base = nullptr;
  uint64_t size = 0, used = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  void init(uint8_t* b, uint64_t n) { base = b; size = n; free_.clear(); free_[0] = n; used = 0; }
  bool alloc(uint64_t n, uint64_t& off) {
    n = up(std::max<uint64_t>(n, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      off = it->first;
      const uint64_t rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      used += n;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = up(std::max<uint64_t>(n, 1));
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
};

struct Key {
  int32_t file, rg_b, rg_e;
  uint64_t mask;
  bool operator==(const Key& o) const { return file == o.file && rg_b == o.rg_b && rg_e == o.rg_e && mask == o.mask; }
};

struct Result {  // one decoded request, resident in the arena
  Key key{};
  std::vector<uint64_t> waiters;  // requests sharing it before it is decoded
  std::vector<std::pair<uint64_t, uint64_t>> blocks;  // (offset, bytes) it holds
  std::vector<pq_column_out> outs;
  int64_t rows = 0;
  uint64_t bytes = 0;        // decoded bytes (values, validity, offsets, chars)
  int refs = 0;              // requests holding it
  bool done = false;
  pq_status status = PQ_OK;
  uint64_t last_use = 0;     // for eviction of unreferenced results
};

struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = k.mask * 0x9E3779B97F4A7C15ull;
    h ^= ((uint64_t)(uint32_t)k.file << 32 | (uint32_t)k.rg_b) + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.rg_e + 0x85EBCA77C2B2AE63ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

struct Req {
  uint64_t id;
  Key key;
  Clock::time_point submit, start, finish;
  std::shared_ptr<Result> res;
  bool hit = false;  // served by a resident result
  bool done = false;
};

struct Batch {
  std::vector<uint64_t> ids;
  std::vector<std::shared_ptr<Result>> results;  // being decoded by this batch
  uint64_t ws_off = 0, ws_bytes = 0;
  int slot = -1;
  // set by the stream callback, which takes no lock (a callback blocked on
  // the server's lock while the scheduler waits on a stream could deadlock)
  std::atomic<bool> finished{false};
  std::atomic<int64_t> finish_ns{0};
  struct pq_server_s* srv = nullptr;
};

}  // namespace

struct pq_server_s {
  std::vector<pq_file> files;
  std::vector<std::vector<int32_t>> types;       // per file, per column: physical type
  std::vector<std::vector<int64_t>> rg_rows;     // per file, per row group
  Arena arena;
  uint8_t* d_arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<Batch*> slot_batch;                // in flight per slot
  int max_batch = 64;
  pq_tuning tuning{};
  std::mutex mu;
  std::condition_variable cv;        // scheduler wake-up
  std::condition_variable done_cv;   // request completions
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Req> reqs;
  std::unordered_map<Key, std::shared_ptr<Result>, KeyHash> resident;
  uint64_t next_id = 1, tick = 0;
  bool stop = false;
  std::thread worker;
  pq_server_stats stats{};
};

namespace {

// Output bytes of one column of a request (values or offsets + chars, and
// the validity words).
void column_sizes(int32_t type, int64_t rows, int64_t chars, uint64_t& a, uint64_t& b, uint64_t& c) {
  c = (uint64_t)((rows + 31) / 32 * 4);
  if (type == PQ_BYTE_ARRAY) { a = 8ull * (uint64_t)(rows + 1); b = (uint64_t)std::max<int64_t>(chars, 1); }
  else { a = (uint64_t)std::max<int64_t>(rows, 1) * (type == PQ_INT32 ? 4u : 8u); b = 0; }
}

void on_batch_done(void* p) {
  Batch* b = static_cast<Batch*>(p);
  b->finish_ns.store(Clock::now().time_since_epoch().count(), std::memory_order_relaxed);
  b->finished.store(true, std::memory_order_release);
  b->srv->cv.notify_all();
}

void ids_done(pq_server_s* s, uint64_t id, Clock::time_point fin) {
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return;
  Req& r = it->second;
  r.finish = fin;
  r.done = true;
  if (r.res && r.res->status == PQ_OK) {
    s->stats.completed++;
    s->stats.decoded_bytes += r.res->bytes;
  } else {
    s->stats.failed++;
  }
}

// Frees unreferenced resident results, least recently used first, until
// `need` bytes could be allocated (true) or nothing is left to free.
bool make_room(pq_server_s* s, uint64_t need) {
  for (;;) {
    uint64_t off;
    if (s->arena.alloc(need, off)) { s->arena.release(off, need); return true; }
    std::shared_ptr<Result> victim;
    Key vkey{};
    for (auto& kv : s->resident)
      if (kv.second->refs == 0 && kv.second->done && (!victim || kv.second->last_use < victim->last_use)) {
        victim = kv.second;
        vkey = kv.first;
      }
    if (!victim) return false;
    for (auto& bl : victim->blocks) s->arena.release(bl.first, bl.second);
    victim->blocks.clear();
    s->resident.erase(vkey);
    s->stats.evictions++;
  }
}

// Arena bytes the outputs of a request take.
uint64_t result_bytes(pq_server_s* s, const Key& k, const std::vector<int64_t>& chars) {
  int64_t rows = 0;
  for (int g = k.rg_b; g < k.rg_e; ++g) rows += s->rg_rows[(size_t)k.file][(size_t)g];
  uint64_t total = 0;
  size_t j = 0;
  for (int c = 0; c < 64; ++c) {
    if (!((k.mask >> c) & 1)) continue;
    uint64_t a, b, v;
    column_sizes(s->types[(size_t)k.file][(size_t)c], rows, chars[j++], a, b, v);
    total += (a ? up(a) : 0) + (b ? up(b) : 0) + (v ? up(v) : 0);
  }
  return total;
}

// Allocates the outputs of a request's result; false when the budget has no
// room even after evictions.
bool alloc_result(pq_server_s* s, const Key& k, const std::vector<int64_t>& chars, Result& r) {
  const pq_file f = s->files[(size_t)k.file];
  (void)f;
  int64_t rows = 0;
  for (int g = k.rg_b; g < k.rg_e; ++g) rows += s->rg_rows[(size_t)k.file][(size_t)g];
  r.rows = rows;
  std::vector<uint64_t> sizes;
  size_t j = 0;
  for (int c = 0; c < 64; ++c) {
    if (!((k.mask >> c) & 1)) continue;
    uint64_t a, b, v;
    column_sizes(s->types[(size_t)k.file][(size_t)c], rows, chars[j++], a, b, v);
    sizes.push_back(a);
    sizes.push_back(b);
    sizes.push_back(v);
  }
  uint64_t total = 0;
  for (uint64_t z : sizes) total += z ? up(z) : 0;
  if (!make_room(s, total)) return false;
  uint64_t off = 0;
  if (!s->arena.alloc(total, off)) return false;
  r.blocks.push_back({off, total});
  uint64_t at = off;
  j = 0;
  r.bytes = 0;
  for (int c = 0; c < 64; ++c) {
    if (!((k.mask >> c) & 1)) continue;
    pq_column_out o;
    memset(&o, 0, sizeof(o));
    const uint64_t a = sizes[3 * j], b = sizes[3 * j + 1], v = sizes[3 * j + 2];
    const int32_t type = s->types[(size_t)k.file][(size_t)c];
    if (type == PQ_BYTE_ARRAY) {
      o.offsets = reinterpret_cast<int64_t*>(s->d_arena + at);
      at += up(a);
      o.chars = s->d_arena + at;
      o.chars_capacity = (uint64_t)chars[j];
      at += up(b);
      r.bytes += 8ull * (uint64_t)(rows + 1) + (uint64_t)chars[j];
    } else {
      o.values = s->d_arena + at;
      at += up(a);
      r.bytes += (uint64_t)rows * (type == PQ_INT32 ? 4u : 8u);
    }
    o.validity = s->d_arena + at;
    at += up(v);
    r.bytes += (uint64_t)(rows + 7) / 8;
    r.outs.push_back(o);
    ++j;
  }
  return true;
}

// Takes a result that never ran out of the resident set and the arena.
void drop_result(pq_server_s* s, const std::shared_ptr<Result>& res) {
  for (auto& bl : res->blocks) s->arena.release(bl.first, bl.second);
  res->blocks.clear();
  s->resident.erase(res->key);
}

void fail_request(pq_server_s* s, uint64_t id, pq_status st) {
  Req& r = s->reqs[id];
  auto res = std::make_shared<Result>();
  res->status = st;
  res->done = true;
  r.res = res;
  r.done = true;
  r.start = r.finish = Clock::now();
  s->stats.failed++;
  s->done_cv.notify_all();
}

// Starts one batch on a free slot from the pending queue, in arrival order.
// A request is admitted when its outputs, and the batch workspace with it,
// fit the arena (after evicting unreferenced resident results); the first
// that does not fit waits (with its successors) until memory is freed.  A
// request identical to a resident or in-flight result shares it instead.
// Called with the lock held; true when a request was consumed.
bool launch_batch(pq_server_s* s, int slot) {
  bool consumed = false;
  auto* b = new Batch();
  b->srv = s;
  b->slot = slot;
  std::vector<pq_request> rq;
  std::vector<uint64_t> taken;  // ids in admission order, hits on this batch's results included
  uint64_t ws_need = 0;
  while (!s->pending.empty() && (int)rq.size() < s->max_batch) {
    const uint64_t id = s->pending.front();
    Req& r = s->reqs[id];
    auto hit = s->resident.find(r.key);
    if (hit != s->resident.end()) {
      r.res = hit->second;
      r.res->refs++;
      r.res->last_use = ++s->tick;
      r.hit = true;
      r.start = Clock::now();
      s->stats.cache_hits++;
      if (r.res->done) {
        r.finish = r.start;
        r.done = true;
        s->stats.completed++;
        s->done_cv.notify_all();
      } else {
        r.res->waiters.push_back(id);  // completes with the batch decoding it
      }
      s->pending.pop_front();
      consumed = true;
      continue;
    }
    // plan the request alone: its chars sizes and its workspace share
    pq_request one{s->files[(size_t)r.key.file], r.key.mask, r.key.rg_b, r.key.rg_e, nullptr};
    uint64_t wsb = 0;
    std::vector<int64_t> chars((size_t)__builtin_popcountll(r.key.mask) + 1, 0);
    pq_status st = pq_plan_batch(&one, 1, &wsb, chars.data(), (int32_t)chars.size());
    if (st != PQ_OK) {
      s->pending.pop_front();
      fail_request(s, id, st);
      consumed = true;
      continue;
    }
    if (result_bytes(s, r.key, chars) + up(wsb) > s->arena.size) {
      // larger than the whole budget: it can never run
      s->pending.pop_front();
      fail_request(s, id, sfail(PQ_ECAPACITY, "request %llu needs more than the budget", (unsigned long long)id));
      consumed = true;
      continue;
    }
    auto res = std::make_shared<Result>();
    res->key = r.key;
    bool fits = alloc_result(s, r.key, chars, *res);
    if (fits && !make_room(s, ws_need + wsb)) {
      drop_result(s, res);
      fits = false;
    }
    if (!fits) break;  // waits for memory: batches finishing, results released
    ws_need += wsb;
    res->refs = 1;
    res->last_use = ++s->tick;
    r.res = res;
    r.start = Clock::now();
    s->resident[r.key] = res;
    b->results.push_back(res);
    b->ids.push_back(id);
    rq.push_back(pq_request{s->files[(size_t)r.key.file], r.key.mask, r.key.rg_b, r.key.rg_e, nullptr});
    s->pending.pop_front();
    consumed = true;
  }
  if (rq.empty()) { delete b; return consumed; }
  for (size_t i = 0; i < rq.size(); ++i) rq[i].outs = b->results[i]->outs.data();
  uint64_t wsb = 0;
  pq_status st = pq_plan_batch(rq.data(), (int32_t)rq.size(), &wsb, nullptr, 0);
  bool have_ws = false;
  if (st == PQ_OK) have_ws = make_room(s, wsb) && s->arena.alloc(wsb, b->ws_off);
  if (st == PQ_OK && !have_ws) {
    // the arena is too fragmented for the workspace: the batch's requests go
    // back to the front of the queue and wait for memory
    std::vector<uint64_t> back;
    for (size_t i = 0; i < b->results.size(); ++i) {
      auto& res = b->results[i];
      back.push_back(b->ids[i]);
      for (uint64_t w : res->waiters) back.push_back(w);
      res->waiters.clear();
      drop_result(s, res);
    }
    for (auto it = back.rbegin(); it != back.rend(); ++it) {
      Req& r = s->reqs[*it];
      if (r.res) { r.res->refs--; r.res.reset(); }
      r.hit = false;
      s->pending.push_front(*it);
    }
    delete b;
    return false;
  }
  b->ws_bytes = wsb;
  if (st == PQ_OK) st = pq_scan_batch(rq.data(), (int32_t)rq.size(), &s->tuning, s->d_arena + b->ws_off, wsb, s->streams[(size_t)slot]);
  if (st == PQ_OK && hipLaunchHostFunc(s->streams[(size_t)slot], on_batch_done, b) != hipSuccess) st = PQ_EHIP;
  if (st != PQ_OK) {
    // the batch never ran: its requests (and those sharing their results)
    // fail; the results leave the resident set and their memory is freed
    if (have_ws) s->arena.release(b->ws_off, b->ws_bytes);
    const auto now = Clock::now();
    for (auto& res : b->results) {
      res->status = st;
      res->done = true;
      drop_result(s, res);
      for (uint64_t w : res->waiters) { s->reqs[w].done = true; s->reqs[w].finish = now; s->stats.failed++; }
      res->waiters.clear();
    }
    for (uint64_t id : b->ids) { s->reqs[id].done = true; s->reqs[id].finish = now; s->stats.failed++; }
    s->done_cv.notify_all();
    delete b;
    return true;
  }
  s->stats.batches++;
  s->slot_batch[(size_t)slot] = b;
  return true;
}

// Retires finished batches: their workspace goes back to the arena, their
// results become resident, their requests (and those that joined a result
// while it was decoded) complete.  Lock held.
void retire(pq_server_s* s) {
  bool any = false;
  for (size_t k = 0; k < s->slot_batch.size(); ++k) {
    Batch* b = s->slot_batch[k];
    if (!b || !b->finished.load(std::memory_order_acquire)) continue;
    any = true;
    const Clock::time_point fin{Clock::duration(b->finish_ns.load(std::memory_order_relaxed))};
    const pq_status st = pq_scan_check(nullptr, s->d_arena + b->ws_off, s->streams[k]);
    s->arena.release(b->ws_off, b->ws_bytes);
    for (auto& res : b->results) {
      res->status = st;
      res->done = true;
      if (st != PQ_OK) s->resident.erase(res->key);
      for (uint64_t w : res->waiters) ids_done(s, w, fin);
      res->waiters.clear();
    }
    for (uint64_t id : b->ids) ids_done(s, id, fin);
    s->slot_batch[k] = nullptr;
    delete b;
  }
  if (any) s->done_cv.notify_all();
}

void serve_loop(pq_server_s* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    retire(s);
    bool launched = false;
    for (size_t k = 0; k < s->slot_batch.size() && !s->pending.empty(); ++k)
      if (!s->slot_batch[k] && launch_batch(s, (int)k)) launched = true;
    bool busy = false;
    for (Batch* b : s->slot_batch) busy = busy || b != nullptr;
    if (s->stop && !busy) break;
    if (launched) continue;
    s->cv.wait_for(lk, std::chrono::milliseconds(busy ? 1 : 50));
  }
}

}  // namespace

extern "C" pq_status pq_server_create(const pq_file* files, int32_t n_files, uint64_t budget_bytes, int32_t slots,
                                      int32_t max_batch, const pq_tuning* tuning, pq_server* out) {
  if (!out || (n_files > 0 && !files) || n_files <= 0) return sfail(PQ_EINVAL, "bad arguments");
  *out = nullptr;
  if (slots < 1 || slots > 16) return sfail(PQ_EINVAL, "slots must be 1..16");
  auto* s = new pq_server_s();
  s->max_batch = max_batch > 0 ? max_batch : 64;
  if (tuning) s->tuning = *tuning; else pq_tuning_default(&s->tuning);
  for (int32_t i = 0; i < n_files; ++i) {
    int32_t nc = 0, nrg = 0;
    if (!files[i] || pq_num_columns(files[i], &nc) != PQ_OK || pq_num_row_groups(files[i], &nrg) != PQ_OK) {
      delete s;
      return sfail(PQ_EINVAL, "file %d is not an open handle", i);
    }
    // batched scans need device-resident files: a one-request plan refuses
    // a host-resident handle
    pq_request probe{files[i], 0, 0, 0, nullptr};
    uint64_t probe_ws = 0;
    if (pq_plan_batch(&probe, 1, &probe_ws, nullptr, 0) != PQ_OK) {
      delete s;
      return sfail(PQ_EINVAL, "file %d cannot be served: %s", i, pq_last_error());
    }
    s->files.push_back(files[i]);
    std::vector<int32_t> t((size_t)nc);
    for (int32_t c = 0; c < nc; ++c) { pq_column_info ci; pq_column_info_get(files[i], c, &ci); t[(size_t)c] = ci.type; }
    s->types.push_back(t);
    std::vector<int64_t> r((size_t)nrg);
    for (int32_t g = 0; g < nrg; ++g) pq_row_group_rows(files[i], g, &r[(size_t)g]);
    s->rg_rows.push_back(r);
  }
  if (hipMalloc(&s->d_arena, budget_bytes) != hipSuccess) { delete s; return sfail(PQ_ENOMEM, "no device memory for the budget"); }
  s->arena.init(s->d_arena, budget_bytes);
  for (int32_t k = 0; k < slots; ++k) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      (void)hipFree(s->d_arena);
      delete s;
      return sfail(PQ_EHIP, "stream creation failed");
    }
    s->streams.push_back(st);
  }
  s->slot_batch.assign((size_t)slots, nullptr);
  s->stats.budget_bytes = budget_bytes;
  s->worker = std::thread(serve_loop, s);
  *out = s;
  return PQ_OK;
}

extern "C" pq_status pq_server_submit(pq_server s, int32_t file, uint64_t col_mask, int32_t rg_begin, int32_t rg_end,
                                      uint64_t* id) {
  if (!s || !id) return sfail(PQ_EINVAL, "NULL argument");
  if (file < 0 || file >= (int32_t)s->files.size()) return sfail(PQ_EINVAL, "bad file index %d", file);
  const int32_t nrg = (int32_t)s->rg_rows[(size_t)file].size(), nc = (int32_t)s->types[(size_t)file].size();
  if (rg_begin < 0 || rg_end > nrg || rg_begin > rg_end) return sfail(PQ_EINVAL, "bad row-group range");
  if (!col_mask || (nc < 64 && (col_mask >> nc))) return sfail(PQ_EINVAL, "bad column mask");
  std::lock_guard<std::mutex> lk(s->mu);
  Req r;
  r.id = s->next_id++;
  r.key = Key{file, rg_begin, rg_end, col_mask};
  r.submit = Clock::now();
  s->reqs[r.id] = r;
  s->pending.push_back(r.id);
  s->stats.submitted++;
  *id = r.id;
  s->cv.notify_all();
  return PQ_OK;
}

extern "C" pq_status pq_server_wait(pq_server s, uint64_t id, int32_t timeout_ms, pq_served* out) {
  if (!s || !out) return sfail(PQ_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(PQ_EINVAL, "unknown request %llu", (unsigned long long)id);
  const auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 3600000 : timeout_ms);
  while (!it->second.done) {
    if (s->done_cv.wait_until(lk, deadline) == std::cv_status::timeout && !it->second.done)
      return sfail(PQ_EBUSY, "request %llu not finished", (unsigned long long)id);
    it = s->reqs.find(id);
  }
  const Req& r = it->second;
  memset(out, 0, sizeof(*out));
  out->status = r.res ? r.res->status : PQ_EINVAL;
  out->rows = r.res ? r.res->rows : 0;
  out->decoded_bytes = r.res ? r.res->bytes : 0;
  out->queue_ms = std::chrono::duration<double, std::milli>(r.start - r.submit).count();
  out->latency_ms = std::chrono::duration<double, std::milli>(r.finish - r.submit).count();
  out->shared = r.hit ? 1 : 0;
  out->n_outs = r.res ? (int32_t)r.res->outs.size() : 0;
  for (int32_t k = 0; k < out->n_outs && k < 64; ++k) out->outs[k] = r.res->outs[(size_t)k];
  return (pq_status)out->status;
}

extern "C" pq_status pq_server_release(pq_server s, uint64_t id) {
  if (!s) return sfail(PQ_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end() || !it->second.done) return sfail(PQ_EINVAL, "request %llu unknown or not finished", (unsigned long long)id);
  if (it->second.res) {
    auto& res = it->second.res;
    if (--res->refs == 0 && res->status != PQ_OK) drop_result(s, res);
    res->last_use = ++s->tick;
  }
  s->reqs.erase(it);
  s->cv.notify_all();
  return PQ_OK;
}

extern "C" pq_status pq_server_stats_get(pq_server s, pq_server_stats* out) {
  if (!s || !out) return sfail(PQ_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->used_bytes = s->arena.used;
  out->resident_results = (uint64_t)s->resident.size();
  return PQ_OK;
}

extern "C" void pq_server_destroy(pq_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto x : s->streams) { (void)hipStreamSynchronize(x); (void)hipStreamDestroy(x); }
  (void)hipFree(s->d_arena);
  delete s;
}

extern "C" const char* pq_server_last_error(void) { return t_msg; }
