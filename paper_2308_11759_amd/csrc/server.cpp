// server.cpp -- a progressive-retrieval server over compressed stores.
//
// The paper's retrieval needs no decoder state: refining x~_k to x~_k' only
// adds components k+1..k' (Sec. 4.2, last paragraph), and components may be
// kept anywhere in the memory hierarchy, GPU memory included (Sec. 6.2).  The
// server builds on both: decoded partial sums stay resident on the device in
// a (field, k) cache, so a query for tolerance tau (k = smallest component
// count with tau_k <= tau, Sec. 6.2) is served by copying a cached x~_k, by
// refining the nearest cached x~_j with j < k, or by decoding from scratch.
//
// A host thread runs the request loop with continuous batching: at every step
// it admits waiting queries (first come, first served) while batch slots and
// the HBM budget allow, and launches one batched decode per element type for
// all of them; steps are enqueued while earlier ones still run, and a query
// completes when the event recorded after its step has fired.  Results are
// bit-identical whether a query runs alone or in a mix (the same left-to-right
// sums are formed either way).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

using namespace pmc;
using namespace pmc_host;

namespace {

using clk = std::chrono::steady_clock;

struct Span {
  uint64_t off, bytes;
};

// first-fit allocator over the caller's arena (256-byte granules)
struct Arena {
  uint64_t size = 0;
  std::vector<Span> free_list;  // sorted by offset, coalesced
  uint64_t used = 0, peak = 0;
  void init(uint64_t base, uint64_t n) {
    size = n;
    free_list.clear();
    if (n > 0) free_list.push_back(Span{base, n});
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = align256(bytes);
    for (size_t i = 0; i < free_list.size(); ++i) {
      if (free_list[i].bytes >= bytes) {
        *off = free_list[i].off;
        free_list[i].off += bytes;
        free_list[i].bytes -= bytes;
        if (free_list[i].bytes == 0) free_list.erase(free_list.begin() + i);
        used += bytes;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = align256(bytes);
    used -= bytes;
    auto it = std::lower_bound(free_list.begin(), free_list.end(), off,
                               [](const Span& s, uint64_t o) { return s.off < o; });
    it = free_list.insert(it, Span{off, bytes});
    size_t i = it - free_list.begin();
    if (i + 1 < free_list.size() && free_list[i].off + free_list[i].bytes == free_list[i + 1].off) {
      free_list[i].bytes += free_list[i + 1].bytes;
      free_list.erase(free_list.begin() + i + 1);
    }
    if (i > 0 && free_list[i - 1].off + free_list[i - 1].bytes == free_list[i].off) {
      free_list[i - 1].bytes += free_list[i].bytes;
      free_list.erase(free_list.begin() + i);
    }
  }
};

struct CacheEntry {
  int field, k;
  uint64_t off, bytes;
  uint64_t last_use;    // step counter
  uint64_t busy_step;   // last step that reads or writes the entry
  uint64_t made_step;   // the step whose tail copy fills the entry
};

enum QState { Q_PENDING = 0, Q_RUNNING = 1, Q_DONE = 2, Q_RELEASED = 3 };

struct Query {
  int field, k;
  void* out;            // caller memory, or NULL: a result slot in the arena
  uint64_t slot_off = 0, slot_bytes = 0;
  bool own_slot = false;
  int state = Q_PENDING;
  pmc_status status = PMC_OK;
  clk::time_point arrival, done;
  uint64_t step = 0;
  int source = 0;       // 0 miss, 1 partial, 2 hit
  bool cancel = false;  // cancelled while running: the result is dropped when its step ends
};

struct Step {
  uint64_t id;
  hipEvent_t ev;
  std::vector<uint64_t> queries;
  uint64_t budget_bytes;  // caller outputs of this step counted against the budget
  int table_slot;
};

constexpr int kMaxInflight = 4;
// (float32, float64) x (block transform, prediction), and float32 block
// transform queries whose residual components all take the decoder's
// high-half route (launched as their own instantiation)
constexpr int kGroups = 5;

}  // namespace

struct pmc_server {
  pmc_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  uint8_t* arena_base = nullptr;
  uint64_t arena_bytes = 0, budget = 0;
  int max_batch = 64;
  // device tables: kMaxInflight slots of [kGroups x max_batch QueryDev | kGroups x (max_batch+1) prefixes |
  // status]; a group per (element type, codec), each decoded by one launch
  uint64_t table_slot_bytes = 0;
  void* host_tables = nullptr;  // pinned staging, same layout
  bool slot_busy[kMaxInflight] = {false, false, false, false};
  Arena arena;
  std::vector<const pmc_store*> fields;
  std::vector<CacheEntry> cache;
  std::vector<Query> queries;
  std::deque<uint64_t> pending;
  std::deque<Step> inflight;
  uint64_t step_counter = 0, completed_steps = 0;
  uint64_t outputs_inflight = 0;  // caller-output bytes of running queries
  pmc_server_stats stats{};
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::thread worker;
  pmc_status worker_error = PMC_OK;
};

namespace {

uint64_t field_bytes(const pmc_store* s) { return s->g.nx * s->g.ny * s->g.nz * elem_size(&s->f); }

uint64_t cache_bytes_total(const pmc_server* sv) {
  uint64_t b = 0;
  for (const CacheEntry& e : sv->cache) b += align256(e.bytes);
  return b;
}

// arena bytes in use plus caller outputs of running queries
uint64_t budget_used(const pmc_server* sv) { return sv->arena.used + sv->outputs_inflight; }

// evict least-recently-used cache entries no running step touches until
// `need` more bytes fit in both the arena and the budget
bool make_room(pmc_server* sv, uint64_t need) {
  need = align256(need);
  for (;;) {
    uint64_t off;
    if (budget_used(sv) + need <= sv->budget && sv->arena.alloc(need, &off)) {
      sv->arena.release(off, need);  // only probing
      return true;
    }
    int victim = -1;
    for (size_t i = 0; i < sv->cache.size(); ++i) {
      const CacheEntry& e = sv->cache[i];
      if (e.busy_step > sv->completed_steps) continue;
      if (victim < 0 || e.last_use < sv->cache[victim].last_use) victim = (int)i;
    }
    if (victim < 0) return false;
    sv->arena.release(sv->cache[victim].off, sv->cache[victim].bytes);
    sv->cache.erase(sv->cache.begin() + victim);
  }
}

// best source for (field, k): the cached partial sum with the largest j <= k,
// among entries filled by an earlier step (stream order makes them ready)
int find_cache(const pmc_server* sv, int field, int kmax, uint64_t step) {
  int best = -1;
  for (size_t i = 0; i < sv->cache.size(); ++i) {
    const CacheEntry& e = sv->cache[i];
    if (e.field == field && e.k <= kmax && e.made_step < step && (best < 0 || e.k > sv->cache[best].k))
      best = (int)i;
  }
  return best;
}

void retire(pmc_server* sv) {
  while (!sv->inflight.empty()) {
    Step& st = sv->inflight.front();
    if (hipEventQuery(st.ev) != hipSuccess) break;
    const clk::time_point now = clk::now();
    unsigned int* status = (unsigned int*)((uint8_t*)sv->host_tables + st.table_slot * sv->table_slot_bytes +
                                           sv->table_slot_bytes - 256);
    const bool bad = *status != 0;
    for (uint64_t qi : st.queries) {
      Query& q = sv->queries[qi];
      q.state = Q_DONE;
      q.done = now;
      q.status = bad ? PMC_E_CORRUPT : PMC_OK;
      sv->stats.completed++;
      if (q.cancel) {  // its step has ended: nothing reads or writes the slot any more
        if (q.own_slot) sv->arena.release(q.slot_off, q.slot_bytes);
        q.own_slot = false;
        q.status = PMC_E_CANCELLED;
        q.state = Q_RELEASED;
      }
    }
    sv->outputs_inflight -= st.budget_bytes;
    sv->slot_busy[st.table_slot] = false;
    (void)hipEventDestroy(st.ev);
    sv->completed_steps = st.id;
    sv->inflight.pop_front();
  }
}

// build and launch one step from the pending queue; false if nothing admitted
bool launch_step(pmc_server* sv) {
  int slot = -1;
  for (int i = 0; i < kMaxInflight; ++i)
    if (!sv->slot_busy[i]) {
      slot = i;
      break;
    }
  if (slot < 0 || sv->pending.empty()) return false;
  const uint64_t step_id = ++sv->step_counter;
  uint8_t* htab = (uint8_t*)sv->host_tables + slot * sv->table_slot_bytes;
  uint8_t* dtab = sv->arena_base + slot * sv->table_slot_bytes;
  QueryDev* hq[kGroups];
  uint32_t* hpre[kGroups];
  uint32_t nq[kGroups], nw[kGroups];
  uint64_t span[kGroups];  // largest decode-wave span of the step's streams, per group
  uint32_t* const pre0 = (uint32_t*)(htab + kGroups * sv->max_batch * sizeof(QueryDev));
  for (int t = 0; t < kGroups; ++t) {
    hq[t] = (QueryDev*)htab + t * sv->max_batch;
    hpre[t] = pre0 + t * (sv->max_batch + 1);
    hpre[t][0] = 0;
    nq[t] = nw[t] = 0;
    span[t] = 0;
  }
  uint32_t admitted = 0;
  Step st{};
  st.id = step_id;
  st.table_slot = slot;
  struct CopyJob {
    void* dst;
    const void* src;
    uint64_t bytes;
  };
  std::vector<CopyJob> copies;
  while (!sv->pending.empty() && admitted < (uint32_t)sv->max_batch) {
    const uint64_t qi = sv->pending.front();
    Query& q = sv->queries[qi];
    const pmc_store* s = sv->fields[q.field];
    const uint64_t fb = field_bytes(s);
    // admission: the result's memory must fit the budget now
    if (!q.out) {
      if (!make_room(sv, fb)) break;
      if (!sv->arena.alloc(fb, &q.slot_off)) break;
      q.slot_bytes = fb;
      q.own_slot = true;
    } else {
      if (budget_used(sv) + fb > sv->budget) {
        if (!make_room(sv, fb)) break;
      }
      sv->outputs_inflight += fb;
      st.budget_bytes += fb;
    }
    sv->pending.pop_front();
    void* out = q.out ? q.out : (void*)(sv->arena_base + q.slot_off);
    const int ci = find_cache(sv, q.field, q.k, step_id);
    const int k0 = ci >= 0 ? sv->cache[ci].k : 0;
    bool hires = s->f.dtype == PMC_F32 && s->codec == 0;
    for (int c = k0; c < q.k; ++c)
      if (c > 0 && s->full[c] != 0) hires = false;
    const int t = hires ? 4 : (s->f.dtype == PMC_F32 ? 0 : 1) + 2 * s->codec;
    QueryDev& d = hq[t][nq[t]];
    std::memset(&d, 0, sizeof(d));
    d.in = nullptr;
    if (ci >= 0) {
      CacheEntry& e = sv->cache[ci];
      d.in = sv->arena_base + e.off;
      e.last_use = step_id;
      e.busy_step = step_id;
    }
    q.source = ci < 0 ? 0 : (k0 == q.k ? 2 : 1);
    (q.source == 2 ? sv->stats.hits : q.source == 1 ? sv->stats.partial : sv->stats.misses)++;
    d.ncomp = q.k - k0;
    for (int i = 0; i < d.ncomp; ++i) {
      const int c = k0 + i;
      d.s[i] = s->d_base + s->offset[c];
      d.aux[i] = (const uint32_t*)(s->d_base + s->aux_offset[c]);
      d.words[i] = s->words[c];
      d.minexp[i] = s->minexp[c];
      d.step[i] = 2.0 * s->tau[c];
      if (c > 0) d.relmask |= 1u << i;  // residual components
      span[t] = std::max(span[t], s->max_span[c]);
    }
    d.dtype = s->f.dtype;
    d.out = out;
    d.g = s->g;
    const uint32_t waves = (uint32_t)((s->g.nblocks + 63) / 64);
    hpre[t][nq[t] + 1] = hpre[t][nq[t]] + waves;
    nw[t] += waves;
    nq[t]++;
    admitted++;
    // keep the new partial sum if it is not cached yet and there is room
    if (q.source != 2) {
      bool have = false;
      for (const CacheEntry& e : sv->cache)
        if (e.field == q.field && e.k == q.k) have = true;
      uint64_t off;
      if (!have && make_room(sv, fb) && sv->arena.alloc(fb, &off)) {
        sv->cache.push_back(CacheEntry{q.field, q.k, off, fb, step_id, step_id, step_id});
        copies.push_back(CopyJob{sv->arena_base + off, out, fb});
      }
    }
    q.state = Q_RUNNING;
    q.step = step_id;
    st.queries.push_back(qi);
  }
  if (st.queries.empty()) {
    --sv->step_counter;
    return false;
  }
  unsigned int* hstatus = (unsigned int*)(htab + sv->table_slot_bytes - 256);
  *hstatus = 0;
  hipError_t e = hipMemcpyAsync(dtab, htab, sv->table_slot_bytes, hipMemcpyHostToDevice, sv->stream);
  for (int t = 0; t < kGroups && e == hipSuccess; ++t) {
    if (!nq[t]) continue;
    ServeArgs a{};
    a.q = (const QueryDev*)dtab + t * sv->max_batch;
    a.wave_prefix = (const uint32_t*)(dtab + kGroups * sv->max_batch * sizeof(QueryDev)) + t * (sv->max_batch + 1);
    a.nq = nq[t];
    a.nwaves = nw[t];
    a.status = (unsigned int*)(dtab + sv->table_slot_bytes - 256);
    if (t == 4) {
      e = launch_decode_queries<float>(a, span[t], 0, true, sv->stream);
    } else {
      const int codec = t / 2;
      e = t % 2 == 0 ? launch_decode_queries<float>(a, span[t], codec, false, sv->stream)
                     : launch_decode_queries<double>(a, span[t], codec, false, sv->stream);
    }
  }
  for (const CopyJob& c : copies)
    if (e == hipSuccess) e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, sv->stream);
  // the status word travels back into the pinned slot for retire()
  if (e == hipSuccess)
    e = hipMemcpyAsync(hstatus, dtab + sv->table_slot_bytes - 256, 4, hipMemcpyDeviceToHost, sv->stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&st.ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(st.ev, sv->stream);
  if (e != hipSuccess) {
    sv->worker_error = PMC_E_DEVICE;
    for (uint64_t qi : st.queries) {
      sv->queries[qi].state = Q_DONE;
      sv->queries[qi].status = PMC_E_DEVICE;
      sv->queries[qi].done = clk::now();
    }
    sv->outputs_inflight -= st.budget_bytes;
    return false;
  }
  sv->slot_busy[slot] = true;
  sv->stats.steps++;
  sv->stats.batched_queries += st.queries.size();
  sv->inflight.push_back(std::move(st));
  return true;
}

void worker_main(pmc_server* sv) {
  (void)hipSetDevice(sv->ctx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    retire(sv);
    if (sv->stop && sv->pending.empty() && sv->inflight.empty()) break;
    bool launched = false;
    while (!sv->pending.empty() && (int)sv->inflight.size() < kMaxInflight && launch_step(sv)) launched = true;
    if (sv->stop && !launched && sv->inflight.empty()) {
      // shutting down with queries that can no longer be admitted
      for (uint64_t qi : sv->pending) {
        sv->queries[qi].state = Q_DONE;
        sv->queries[qi].status = PMC_E_NOMEM;
        sv->queries[qi].done = clk::now();
      }
      sv->pending.clear();
      break;
    }
    sv->stats.max_queue = std::max<uint64_t>(sv->stats.max_queue, sv->pending.size());
    if (!launched) {
      // wait for a submission, or poll the running steps
      if (sv->inflight.empty()) sv->cv.wait_for(lk, std::chrono::milliseconds(2));
      else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
  }
}

}  // namespace

extern "C" {

pmc_status pmc_server_create(pmc_ctx* ctx, size_t hbm_budget, void* d_arena, size_t arena_bytes, int max_batch,
                             pmc_server** out) {
  if (!ctx) return PMC_E_ARG;
  if (!out || !d_arena || max_batch < 1 || max_batch > 1024) return fail(ctx, PMC_E_ARG, "bad server arguments");
  *out = nullptr;
  pmc_server* sv = new pmc_server();
  sv->ctx = ctx;
  sv->max_batch = max_batch;
  sv->table_slot_bytes = align256(kGroups * max_batch * sizeof(QueryDev) + kGroups * (max_batch + 1) * 4 + 256) + 256;
  const uint64_t tables = kMaxInflight * sv->table_slot_bytes;
  if (arena_bytes < tables + 256) {
    delete sv;
    return fail(ctx, PMC_E_NOMEM, "arena too small: need more than %llu bytes", (unsigned long long)tables);
  }
  sv->arena_base = (uint8_t*)d_arena;
  sv->arena_bytes = arena_bytes;
  sv->budget = hbm_budget;
  sv->arena.init(tables, (arena_bytes - tables) & ~255ull);
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc(&sv->host_tables, tables, hipHostMallocDefault) != hipSuccess) {
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
    return fail(ctx, PMC_E_DEVICE, "server stream or pinned staging failed");
  }
  std::memset(sv->host_tables, 0, tables);
  sv->worker = std::thread(worker_main, sv);
  *out = sv;
  return PMC_OK;
}

pmc_status pmc_server_add(pmc_server* sv, const pmc_store* s, int* field_id) {
  if (!sv || !s || !field_id) return PMC_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->fields.push_back(s);
  *field_id = (int)sv->fields.size() - 1;
  return PMC_OK;
}

double pmc_clock(void) { return std::chrono::duration<double>(clk::now().time_since_epoch()).count(); }

pmc_status pmc_server_submit(pmc_server* sv, int field_id, double tol, void* d_out, uint64_t* ticket) {
  return pmc_server_submit_at(sv, field_id, tol, d_out, 0.0, ticket);
}

pmc_status pmc_server_submit_at(pmc_server* sv, int field_id, double tol, void* d_out, double arrival,
                                uint64_t* ticket) {
  if (!sv || !ticket) return PMC_E_ARG;
  const clk::time_point now = clk::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (field_id < 0 || field_id >= (int)sv->fields.size()) return fail(sv->ctx, PMC_E_ARG, "unknown field");
  if (d_out && !aligned16(d_out)) return fail(sv->ctx, PMC_E_ARG, "d_out must be 16-byte aligned");
  int k = 0;
  if (pmc_select_k(sv->fields[field_id], tol, 0, &k) != PMC_OK)
    return fail(sv->ctx, PMC_E_UNREACHABLE, "tolerance below the last component's");
  if (field_bytes(sv->fields[field_id]) > sv->budget)
    return fail(sv->ctx, PMC_E_NOMEM, "a result of this field can never fit the budget");
  Query q;
  q.field = field_id;
  q.k = k;
  q.out = d_out;
  // the arrival the latency counts from: the caller's (e.g. the scheduled
  // time of a trace), never later than now; else the submission itself
  q.arrival = now;
  if (arrival > 0.0) {
    const clk::time_point a =
        clk::time_point(std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(arrival)));
    if (a < now) q.arrival = a;
  }
  sv->queries.push_back(q);
  *ticket = sv->queries.size() - 1;
  sv->pending.push_back(*ticket);
  sv->stats.submitted++;
  sv->cv.notify_one();
  return PMC_OK;
}

pmc_status pmc_server_poll(pmc_server* sv, uint64_t ticket, int* done, pmc_status* st, double* latency_s) {
  if (!sv) return PMC_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket >= sv->queries.size()) return PMC_E_ARG;
  const Query& q = sv->queries[ticket];
  const bool d = q.state >= Q_DONE;
  if (done) *done = d ? 1 : 0;
  if (st) *st = d ? q.status : PMC_OK;
  if (latency_s) *latency_s = d ? std::chrono::duration<double>(q.done - q.arrival).count() : -1.0;
  return PMC_OK;
}

pmc_status pmc_server_result(pmc_server* sv, uint64_t ticket, const void** d_result, int* k, int* source) {
  if (!sv) return PMC_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket >= sv->queries.size()) return PMC_E_ARG;
  const Query& q = sv->queries[ticket];
  if (q.state != Q_DONE) return PMC_E_ARG;
  if (d_result) *d_result = q.out ? q.out : (const void*)(sv->arena_base + q.slot_off);
  if (k) *k = q.k;
  if (source) *source = q.source;
  return PMC_OK;
}

pmc_status pmc_server_cancel(pmc_server* sv, uint64_t ticket) {
  if (!sv) return PMC_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket >= sv->queries.size()) return PMC_E_ARG;
  Query& q = sv->queries[ticket];
  if (q.state == Q_PENDING) {
    // not admitted yet: it holds no memory and no step refers to it
    const auto it = std::find(sv->pending.begin(), sv->pending.end(), ticket);
    if (it != sv->pending.end()) sv->pending.erase(it);
    q.state = Q_RELEASED;
    q.status = PMC_E_CANCELLED;
    q.done = clk::now();
    sv->stats.cancelled++;
    return PMC_OK;
  }
  if (q.state == Q_RUNNING) {
    if (!q.cancel) sv->stats.cancelled++;
    q.cancel = true;
    return PMC_OK;
  }
  if (q.status == PMC_E_CANCELLED) return PMC_OK;  // cancelled before
  return fail(sv->ctx, PMC_E_ARG, "the query has finished: release it instead");
}

pmc_status pmc_server_release(pmc_server* sv, uint64_t ticket) {
  if (!sv) return PMC_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket >= sv->queries.size()) return PMC_E_ARG;
  Query& q = sv->queries[ticket];
  if (q.state == Q_RELEASED && q.status == PMC_E_CANCELLED) return PMC_OK;  // nothing left to release
  if (q.state != Q_DONE) return PMC_E_ARG;
  if (q.own_slot) sv->arena.release(q.slot_off, q.slot_bytes);
  q.own_slot = false;
  q.state = Q_RELEASED;
  return PMC_OK;
}

pmc_status pmc_server_get_stats(pmc_server* sv, pmc_server_stats* out) {
  if (!sv || !out) return PMC_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  out->cache_entries = sv->cache.size();
  out->cache_bytes = cache_bytes_total(sv);
  out->arena_peak = sv->arena.peak;
  out->pending = sv->pending.size();
  out->running = 0;
  for (const Step& s : sv->inflight) out->running += s.queries.size();
  return sv->worker_error;
}

void pmc_server_destroy(pmc_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_one();
  }
  if (sv->worker.joinable()) sv->worker.join();
  if (sv->stream) {
    (void)hipStreamSynchronize(sv->stream);
    (void)hipStreamDestroy(sv->stream);
  }
  if (sv->host_tables) (void)hipHostFree(sv->host_tables);
  delete sv;
}

}  // extern "C"
