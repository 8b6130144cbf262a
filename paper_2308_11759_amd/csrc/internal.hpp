// internal.hpp -- host-side objects shared by the C-ABI translation units
// (capi.cpp: single fields and stores; batch.cpp: batches of fields).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pmc.h"
#include "launch.hpp"

struct ProfRec {
  int kernel;
  hipEvent_t start, stop;
};

// device fields are read and written with 16-byte row accesses
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

struct pmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int fused_decode = 1;
  int sync_check = 0;
  int profile = 0;
  int codec = 0;  // the codec pmc_compress uses: 0 block transform, 1 prediction
  std::vector<std::string> prof_names;
  std::vector<uint64_t> prof_launches;
  std::vector<double> prof_ms;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  // pinned host memory for the small device-to-host reads of the calls that
  // synchronise (range, compressed sizes, decode status): a direct copy
  // instead of one staged through pageable memory; null if it could not be
  // allocated (the calls then read into pageable memory)
  void* pin = nullptr;
};
constexpr size_t kPinBytes = 8192;  // >= kMaxComps * sizeof(CompMeta)

struct pmc_store {
  pmc_field f{};
  pmc::Geo g{};
  int n = 0;
  int codec = 0;  // 0 block transform, 1 prediction (every component of a store)
  std::vector<double> tau, linf;
  std::vector<int> minexp;
  std::vector<uint64_t> bytes, offset, aux_offset, words, nempty, ncoded, nraw, nesc, nmiss;
  std::vector<uint64_t> max_span;  // largest payload words of a decode wave's four chunks
  std::vector<uint64_t> full;      // nonzero: a coded block is outside the float32 high-half decode route
  const uint8_t* d_base = nullptr;  // caller-owned device memory holding the streams
};

namespace pmc_host {

pmc_status fail(pmc_ctx* ctx, pmc_status st, const char* fmt, ...);
pmc_status hipfail(pmc_ctx* ctx, hipError_t e, const char* what);
uint64_t elem_size(const pmc_field* f);
uint64_t stream_cap_one(const pmc::Geo& g, int dtype);
// a store from per-component device results (offsets relative to d_base)
pmc_store* store_from_meta(const pmc_field* f, const pmc::Geo& g, int n, const double* tau, const int* minexp,
                           const pmc::CompMeta* hm, const uint8_t* d_base, int codec);
// the decode arguments of components [i0, i1) of a store
template <class A> void fill_decode_args(const pmc_store* s, int i0, int i1, A& a) {
  for (int i = i0; i < i1; ++i) {
    a.s[i - i0] = s->d_base + s->offset[i];
    a.aux[i - i0] = (const uint32_t*)(s->d_base + s->aux_offset[i]);
    a.words[i - i0] = s->words[i];
    a.minexp[i - i0] = s->minexp[i];
    a.step[i - i0] = 2.0 * s->tau[i];
    if (i > 0) a.relmask |= 1u << (i - i0);  // residual components
  }
  a.ncomp = i1 - i0;
}

inline hipEvent_t prof_event(pmc_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  // timing only: pmc_prof_read synchronises the stream before it reads
  // them, so the events need no system-scope fence (whose cache writeback
  // and invalidation would also land between the kernels they bracket)
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

inline int prof_kernel_id(pmc_ctx* c, const char* name) {
  for (size_t i = 0; i < c->prof_names.size(); ++i)
    if (c->prof_names[i] == name) return (int)i;
  c->prof_names.push_back(name);
  c->prof_launches.push_back(0);
  c->prof_ms.push_back(0.0);
  return (int)c->prof_names.size() - 1;
}

// brackets one kernel launch (or graph launch) with events on the context
// stream when profiling is enabled
struct ProfScope {
  pmc_ctx* c;
  ProfRec r{};
  bool on;
  ProfScope(pmc_ctx* ctx, const char* name) : c(ctx), on(ctx->profile != 0) {
    if (!on) return;
    r.kernel = prof_kernel_id(c, name);
    r.start = prof_event(c);
    r.stop = prof_event(c);
    if (!r.start || !r.stop) {
      on = false;
      return;
    }
    (void)hipEventRecord(r.start, c->stream);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(r.stop, c->stream);
    c->prof_pending.push_back(r);
  }
};

}  // namespace pmc_host
