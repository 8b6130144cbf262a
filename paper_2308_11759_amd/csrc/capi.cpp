// capi.cpp -- C-ABI of the progressive multi-component codec (see include/pmc.h).
// Host code only: argument checks, workspace layout, kernel sequencing, and
// the per-component metadata of the store.  Every arithmetic step of the path
// runs in the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace pmc;
using namespace pmc_host;

namespace pmc_host {

pmc_status fail(pmc_ctx* ctx, pmc_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

pmc_status hipfail(pmc_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, PMC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

uint64_t elem_size(const pmc_field* f) { return f->dtype == PMC_F32 ? 4 : 8; }

struct WsLayout {
  uint64_t xt[2], staging, chunk_words, offsets, tile_sums, meta, berr, total;
};

// x~ is double-buffered: component i reads x~_{i-1} from xt[(i-1) & 1] and
// writes x~_i to xt[i & 1] (the first reads nothing, the last writes nothing),
// each in the encoder's tiled layout: 64 * 64 values per wave of 64 blocks
WsLayout ws_layout(const pmc_field* f, const Geo& g, int n) {
  WsLayout w{};
  uint64_t o = 0;
  const uint64_t field = align256((g.nblocks + 63) / 64 * 4096 * elem_size(f));
  w.xt[0] = o;
  if (n > 1) o += field;
  w.xt[1] = o;
  if (n > 2) o += field;
  w.staging = o;
  o += align256(g.nchunks * chunk_cap_words_host(f->dtype) * 4);
  w.chunk_words = o;
  o += align256(g.nchunks * 4);
  w.offsets = o;
  o += align256(g.nchunks * 4);
  w.tile_sums = o;
  o += align256((g.nchunks + kScanTile - 1) / kScanTile * 8);
  w.meta = o;
  o += align256((uint64_t)n * sizeof(CompMeta));
  w.berr = o;  // per-block error carried from one component to the next
  if (n > 1) o += align256(g.nblocks * 8);
  w.total = o;
  return w;
}

uint64_t stream_cap_one(const Geo& g, int dtype) {
  return kStreamHeader + 4 * g.nchunks + 4 * g.nchunks * chunk_cap_words_host(dtype);
}

pmc_store* store_from_meta(const pmc_field* f, const Geo& g, int n, const double* tau, const int* minexp,
                           const CompMeta* hm, const uint8_t* d_base, int codec) {
  pmc_store* s = new pmc_store();
  s->f = *f;
  s->g = g;
  s->n = n;
  s->codec = codec;
  s->d_base = d_base;
  const uint64_t auxb = aux_bytes(g);
  for (int i = 0; i < n; ++i) {
    double l;
    std::memcpy(&l, &hm[i].linf_bits, 8);
    s->tau.push_back(tau[i]);
    s->linf.push_back(l);
    s->minexp.push_back(minexp[i]);
    s->bytes.push_back(hm[i].stream_bytes);
    s->offset.push_back(hm[i].stream_offset);
    s->aux_offset.push_back(i * auxb);
    s->words.push_back(hm[i].payload_words);
    s->nempty.push_back(hm[i].nempty);
    s->ncoded.push_back(g.nblocks - hm[i].nempty - hm[i].nraw);  // the encoder counts the others only
    s->nraw.push_back(hm[i].nraw);
    s->nesc.push_back(hm[i].nesc);
    s->nmiss.push_back(hm[i].nmiss);
    s->max_span.push_back(hm[i].max_span);
    s->full.push_back(hm[i].full);
  }
  return s;
}

}  // namespace pmc_host

// ---- the static workspace of pmc_compress_static --------------------------
// One buffer per GPU, held until the process ends.  Host code never uses the
// array's name as an address (on the host it names a stand-in, not device
// memory): pmc_ctx_create looks up its device address once per device with
// hipGetSymbolAddress, and only that address is passed on.
static_assert(PMC_STATIC_WS_BYTES % 256 == 0, "static workspace size");
static_assert(kPinBytes >= kMaxComps * sizeof(CompMeta), "the pinned buffer holds every component's metadata");
static __device__ __align__(256) uint8_t scratch[PMC_STATIC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `device`, looked up on the first call for
// that device (with the device current; the caller's current device is
// restored afterwards)
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if ((e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  const hipError_t r = hipSetDevice(prev);
  if (e != hipSuccess) return e;
  if (r != hipSuccess) return r;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

extern "C" {

pmc_status pmc_ctx_create(int device, void* hip_stream, pmc_ctx** out) {
  if (!out) return PMC_E_ARG;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || device < 0 || device >= count) return PMC_E_DEVICE;
  if (scratch_setup(device) != hipSuccess) return PMC_E_DEVICE;
  pmc_ctx* c = new pmc_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  // the pinned readback buffer, allocated with the context's device current
  // (the caller's current device is restored afterwards)
  int prev = 0;
  if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(device) == hipSuccess) {
    if (hipHostMalloc(&c->pin, kPinBytes, hipHostMallocDefault) != hipSuccess) c->pin = nullptr;
    (void)hipSetDevice(prev);
  }
  *out = c;
  return PMC_OK;
}

// copy `bytes` of device memory to host `dst` on the context stream and wait
// for it, through the context's pinned buffer when it holds them
static hipError_t read_back(pmc_ctx* ctx, void* dst, const void* src, size_t bytes) {
  void* via = ctx->pin && bytes <= kPinBytes ? ctx->pin : dst;
  hipError_t e = hipMemcpyAsync(via, src, bytes, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess && via != dst) std::memcpy(dst, via, bytes);
  return e;
}

void pmc_ctx_destroy(pmc_ctx* ctx) {
  if (!ctx) return;
  if (!ctx->prof_pending.empty()) (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->prof_pending) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->pin) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipHostFree(ctx->pin);
  }
  delete ctx;
}

pmc_status pmc_prof_read(pmc_ctx* ctx, pmc_prof_entry* out, int cap, int* n, int reset) {
  if (!ctx) return PMC_E_ARG;
  if (!ctx->prof_pending.empty()) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "sync");
    for (auto& r : ctx->prof_pending) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
        ctx->prof_ms[r.kernel] += ms;
        ctx->prof_launches[r.kernel] += 1;
      }
      ctx->prof_pool.push_back(r.start);
      ctx->prof_pool.push_back(r.stop);
    }
    ctx->prof_pending.clear();
  }
  const int k = (int)ctx->prof_names.size();
  if (n) *n = k;
  for (int i = 0; i < k && i < cap && out; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::snprintf(out[i].name, sizeof(out[i].name), "%s", ctx->prof_names[i].c_str());
    out[i].launches = ctx->prof_launches[i];
    out[i].ms = ctx->prof_ms[i];
  }
  if (reset) {
    for (int i = 0; i < k; ++i) {
      ctx->prof_launches[i] = 0;
      ctx->prof_ms[i] = 0.0;
    }
  }
  return PMC_OK;
}

const char* pmc_last_error(const pmc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

pmc_status pmc_ctx_set_option(pmc_ctx* ctx, int option, int value) {
  if (!ctx) return PMC_E_ARG;
  if (option == PMC_OPT_FUSED_DECODE) ctx->fused_decode = value ? 1 : 0;
  else if (option == PMC_OPT_SYNC_CHECK) ctx->sync_check = value ? 1 : 0;
  else if (option == PMC_OPT_PROFILE) ctx->profile = value ? 1 : 0;
  else if (option == PMC_OPT_CODEC) {
    if (value != 0 && value != 1) return fail(ctx, PMC_E_ARG, "codec must be 0 or 1");
    ctx->codec = value;
  }
  else return fail(ctx, PMC_E_ARG, "unknown option %d", option);
  return PMC_OK;
}

pmc_status pmc_range(pmc_ctx* ctx, const pmc_field* f, const void* d_x, void* d_ws, size_t ws_bytes,
                     double* vmin, double* vmax, uint64_t* nonfinite) {
  if (!ctx) return PMC_E_ARG;
  Geo g;
  if (!make_geo(f, &g) || !d_x) return fail(ctx, PMC_E_ARG, "bad field");
  if (!d_ws || ws_bytes < 256) return fail(ctx, PMC_E_NOMEM, "range needs 256 bytes of workspace");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  unsigned long long* w = (unsigned long long*)d_ws;
  const uint64_t n = g.nx * g.ny * g.nz;
  // min key all ones; max key and non-finite count zero
  if ((e = launch_fill64_one(w, 3, 0ull, 0, ~0ull, ctx->stream)) != hipSuccess) return hipfail(ctx, e, "fill");
  if (f->dtype == PMC_F32) e = launch_range<float>((const float*)d_x, n, w, ctx->stream);
  else e = launch_range<double>((const double*)d_x, n, w, ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "range kernel");
  unsigned long long h[3];
  if ((e = read_back(ctx, h, w, sizeof(h))) != hipSuccess) return hipfail(ctx, e, "range read");
  auto unorder = [](unsigned long long o) {
    uint64_t b = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
    double v;
    std::memcpy(&v, &b, 8);
    return v;
  };
  if (nonfinite) *nonfinite = h[2];
  if (h[2] == n) {  // nothing finite
    if (vmin) *vmin = NAN;
    if (vmax) *vmax = NAN;
  } else {
    if (vmin) *vmin = unorder(h[0]);
    if (vmax) *vmax = unorder(h[1]);
  }
  return PMC_OK;
}

size_t pmc_stats_ws_bytes(void) { return (size_t)sum_sq_ws_bytes() + 256; }

pmc_status pmc_accuracy_gain(pmc_ctx* ctx, const pmc_field* f, const void* d_x, const void* d_xt, double rate,
                             void* d_ws, size_t ws_bytes, double out[3]) {
  if (!ctx) return PMC_E_ARG;
  Geo g;
  if (!make_geo(f, &g) || !d_x || !d_xt || !out) return fail(ctx, PMC_E_ARG, "bad field or null pointer");
  if (!d_ws || ws_bytes < pmc_stats_ws_bytes())
    return fail(ctx, PMC_E_NOMEM, "accuracy gain needs %llu bytes of workspace",
                (unsigned long long)pmc_stats_ws_bytes());
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  const uint64_t n = g.nx * g.ny * g.nz;
  double* ws = (double*)d_ws;
  double* res = (double*)((uint8_t*)d_ws + sum_sq_ws_bytes());
  // one sum pass: (shift, with xt?) -> host pair
  auto pass = [&](const void* b, double shift, double h[2]) -> pmc_status {
    hipError_t r;
    if (f->dtype == PMC_F32)
      r = launch_sum_sq<float>((const float*)d_x, (const float*)b, shift, n, ws, res, ctx->stream);
    else
      r = launch_sum_sq<double>((const double*)d_x, (const double*)b, shift, n, ws, res, ctx->stream);
    if (r != hipSuccess) return hipfail(ctx, r, "sum kernel");
    if ((r = hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
      return hipfail(ctx, r, "copy");
    if ((r = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hipfail(ctx, r, "sync");
    return PMC_OK;
  };
  double h[2];
  pmc_status st;
  if ((st = pass(nullptr, 0.0, h)) != PMC_OK) return st;
  const double mean = h[0] / (double)n;
  if ((st = pass(nullptr, mean, h)) != PMC_OK) return st;  // second pass about the mean
  const double sigma = std::sqrt(h[1] / (double)n);
  if ((st = pass(d_xt, 0.0, h)) != PMC_OK) return st;
  const double rmse = std::sqrt(h[1] / (double)n);
  out[0] = sigma;
  out[1] = rmse;
  out[2] = std::log2(sigma / rmse) - rate;
  return PMC_OK;
}

pmc_status pmc_cast_compress(pmc_ctx* ctx, const pmc_field* f, const void* d_x, int n, float* d_comps, void* d_ws,
                             size_t ws_bytes, double* linf) {
  if (!ctx) return PMC_E_ARG;
  Geo g;
  if (!make_geo(f, &g) || !d_x || !d_comps) return fail(ctx, PMC_E_ARG, "bad field or null pointer");
  if (n < 1 || n > kMaxComps) return fail(ctx, PMC_E_ARG, "n must be in [1, %d]", kMaxComps);
  if (!d_ws || ws_bytes < 8 * (size_t)kMaxComps)
    return fail(ctx, PMC_E_NOMEM, "cast compression needs %d bytes of workspace", 8 * kMaxComps);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  const uint64_t N = g.nx * g.ny * g.nz;
  unsigned long long* lb = (unsigned long long*)d_ws;
  if ((e = launch_fill64(lb, (uint64_t)n, 0ull, ctx->stream)) != hipSuccess) return hipfail(ctx, e, "fill");
  if (f->dtype == PMC_F32) e = launch_cast_encode<float>((const float*)d_x, N, n, d_comps, lb, ctx->stream);
  else e = launch_cast_encode<double>((const double*)d_x, N, n, d_comps, lb, ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "cast encode");
  if (linf) {
    std::vector<unsigned long long> h(n);
    if ((e = hipMemcpyAsync(h.data(), lb, 8 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
      return hipfail(ctx, e, "copy");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hipfail(ctx, e, "sync");
    for (int i = 0; i < n; ++i) std::memcpy(&linf[i], &h[i], 8);
  }
  return PMC_OK;
}

pmc_status pmc_cast_retrieve(pmc_ctx* ctx, const pmc_field* f, const float* d_comps, int k, void* d_out) {
  if (!ctx) return PMC_E_ARG;
  Geo g;
  if (!make_geo(f, &g) || !d_comps || !d_out) return fail(ctx, PMC_E_ARG, "bad field or null pointer");
  if (k < 0 || k > kMaxComps) return fail(ctx, PMC_E_ARG, "k must be in [0, %d]", kMaxComps);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  const uint64_t N = g.nx * g.ny * g.nz;
  if (f->dtype == PMC_F32) e = launch_cast_decode<float>(d_comps, N, k, (float*)d_out, ctx->stream);
  else e = launch_cast_decode<double>(d_comps, N, k, (double*)d_out, ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "cast decode");
  return PMC_OK;
}

pmc_status pmc_compress_sizes(const pmc_field* f, int n, size_t* ws_bytes, size_t* stream_cap_per_comp) {
  Geo g;
  if (!make_geo(f, &g) || n < 1 || n > kMaxComps) return PMC_E_ARG;
  WsLayout w = ws_layout(f, g, n);
  if (ws_bytes) *ws_bytes = w.total;
  if (stream_cap_per_comp) *stream_cap_per_comp = aux_bytes(g) + align256(stream_cap_one(g, f->dtype));
  return PMC_OK;
}

pmc_status pmc_compress(pmc_ctx* ctx, const pmc_field* f, const void* d_x, int n, const double* tau, void* d_ws,
                        size_t ws_bytes, void* d_streams, size_t streams_cap, pmc_store** out) {
  if (!ctx) return PMC_E_ARG;
  if (out) *out = nullptr;
  Geo g;
  if (!make_geo(f, &g)) return fail(ctx, PMC_E_ARG, "bad field");
  if (!d_x || !tau || !out || !d_streams) return fail(ctx, PMC_E_ARG, "null argument");
  if (!aligned16(d_x)) return fail(ctx, PMC_E_ARG, "d_x must be 16-byte aligned");
  if (n < 1 || n > kMaxComps) return fail(ctx, PMC_E_ARG, "n must be in [1, %d]", kMaxComps);
  const int codec = ctx->codec;
  for (int i = 0; i < n; ++i) {
    if (!(tau[i] > 0.0) || !std::isfinite(tau[i])) return fail(ctx, PMC_E_ARG, "tau[%d] must be > 0 and finite", i);
    if (i > 0 && !(tau[i] < tau[i - 1])) return fail(ctx, PMC_E_ARG, "tau must be strictly decreasing");
    // the prediction codec keeps every bin 2 tau 2^-d normal and 1 / (2 tau) finite
    if (codec == 1 && !(tau[i] >= std::ldexp(1.0, -960) && tau[i] <= std::ldexp(1.0, 1000)))
      return fail(ctx, PMC_E_ARG, "tau[%d] outside [2^-960, 2^1000], the prediction codec's range", i);
  }
  WsLayout w = ws_layout(f, g, n);
  if (!d_ws || ws_bytes < w.total)
    return fail(ctx, PMC_E_NOMEM, "workspace too small: need %llu bytes", (unsigned long long)w.total);
  // the per-block indexes sit at the front of d_streams and are written by
  // the encoder directly; the streams themselves are capacity-checked on the
  // device before they are packed
  const uint64_t min_cap = (uint64_t)n * aux_bytes(g) + (uint64_t)n * align256(kStreamHeader + 4 * g.nchunks);
  if (streams_cap < min_cap)
    return fail(ctx, PMC_E_NOMEM, "stream capacity too small: need at least %llu bytes",
                (unsigned long long)min_cap);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  uint8_t* ws = (uint8_t*)d_ws;
  CompMeta* meta = (CompMeta*)(ws + w.meta);
  // every counter zero; component 0's stream starts after the n block indexes
  const uint64_t auxb = aux_bytes(g);
  if ((e = launch_fill64_one((unsigned long long*)meta, (uint64_t)n * sizeof(CompMeta) / 8, 0ull,
                             offsetof(CompMeta, stream_offset) / 8, (unsigned long long)(n * auxb), ctx->stream)) !=
      hipSuccess)
    return hipfail(ctx, e, "meta init");

  std::vector<int> minexp(n);
  for (int i = 0; i < n; ++i) {
    minexp[i] = floor_log2(tau[i]);
    ScanArgs sa{};
    sa.chunk_words = (const uint32_t*)(ws + w.chunk_words);
    sa.offsets = (uint32_t*)(ws + w.offsets);
    sa.tile_sums = (unsigned long long*)(ws + w.tile_sums);
    sa.aux_bytes = auxb;
    sa.nchunks = g.nchunks;
    sa.meta = meta;
    sa.comp = i;
    sa.ncomp = n;
    sa.streams_cap = streams_cap;
    PackArgs pa{};
    pa.staging = (const uint32_t*)(ws + w.staging);
    pa.chunk_words = sa.chunk_words;
    pa.offsets = sa.offsets;
    pa.nchunks = g.nchunks;
    pa.meta = meta;
    pa.comp = i;
    pa.minexp = minexp[i];
    pa.streams = (uint8_t*)d_streams;
    pa.g = g;
    pa.tau = tau[i];
    pa.codec = codec;
    if (f->dtype == PMC_F32) {
      EncArgs<float> a{};
      a.x = (const float*)d_x;
      a.xt_in = i > 0 ? (const float*)(ws + w.xt[(i - 1) & 1]) : nullptr;
      a.xt_out = (float*)(ws + w.xt[i & 1]);
      a.g = g;
      a.tau = tau[i];
      a.minexp = minexp[i];
      a.first = i == 0;
      a.last = i == n - 1;
      a.staging = (uint32_t*)(ws + w.staging);
      a.chunk_words = (uint32_t*)(ws + w.chunk_words);
      a.aux = (uint32_t*)((uint8_t*)d_streams + i * auxb);
      a.meta = meta + i;
      a.berr = (double*)(ws + w.berr);
      a.h0 = 2.0 * tau[i];
      a.inv0 = 1.0 / a.h0;
      {
        ProfScope ps(ctx, codec == 0 ? "k_encode_f32" : "k_encode_pq_f32");
        e = launch_encode<float>(a, codec, ctx->stream);
      }
      if (e != hipSuccess) return hipfail(ctx, e, "encode");
      {
        ProfScope ps(ctx, "k_scan");
        e = launch_scan(sa, ctx->stream);
      }
      if (e != hipSuccess) return hipfail(ctx, e, "scan");
      {
        ProfScope ps(ctx, "k_pack_f32");
        e = launch_pack<float>(pa, ctx->stream);
      }
      if (e != hipSuccess) return hipfail(ctx, e, "pack");
    } else {
      EncArgs<double> a{};
      a.x = (const double*)d_x;
      a.xt_in = i > 0 ? (const double*)(ws + w.xt[(i - 1) & 1]) : nullptr;
      a.xt_out = (double*)(ws + w.xt[i & 1]);
      a.g = g;
      a.tau = tau[i];
      a.minexp = minexp[i];
      a.first = i == 0;
      a.last = i == n - 1;
      a.staging = (uint32_t*)(ws + w.staging);
      a.chunk_words = (uint32_t*)(ws + w.chunk_words);
      a.aux = (uint32_t*)((uint8_t*)d_streams + i * auxb);
      a.meta = meta + i;
      a.berr = (double*)(ws + w.berr);
      a.h0 = 2.0 * tau[i];
      a.inv0 = 1.0 / a.h0;
      {
        ProfScope ps(ctx, codec == 0 ? "k_encode_f64" : "k_encode_pq_f64");
        e = launch_encode<double>(a, codec, ctx->stream);
      }
      if (e != hipSuccess) return hipfail(ctx, e, "encode");
      {
        ProfScope ps(ctx, "k_scan");
        e = launch_scan(sa, ctx->stream);
      }
      if (e != hipSuccess) return hipfail(ctx, e, "scan");
      {
        ProfScope ps(ctx, "k_pack_f64");
        e = launch_pack<double>(pa, ctx->stream);
      }
      if (e != hipSuccess) return hipfail(ctx, e, "pack");
    }
  }
  std::vector<CompMeta> hm(n);
  if ((e = read_back(ctx, hm.data(), meta, n * sizeof(CompMeta))) != hipSuccess) return hipfail(ctx, e, "meta read");

  unsigned int flags = 0;
  unsigned long long misses = 0;
  for (int i = 0; i < n; ++i) {
    flags |= hm[i].flags;
    misses += hm[i].nmiss;
  }
  if (flags & FLAG_NONFINITE) return fail(ctx, PMC_E_NONFINITE, "input holds NaN or Inf");
  if (flags & FLAG_INDEX) return fail(ctx, PMC_E_NOMEM, "a stream exceeds 2^32 payload words");
  if (flags & FLAG_OVERFLOW) {
    unsigned long long need = n * auxb;
    for (int i = 0; i < n; ++i) need = align256(need) + hm[i].stream_bytes;
    return fail(ctx, PMC_E_NOMEM, "stream capacity too small: need %llu bytes", need);
  }
  pmc_store* s = store_from_meta(f, g, n, tau, minexp.data(), hm.data(), (const uint8_t*)d_streams, codec);
  *out = s;
  if (misses) return fail(ctx, PMC_E_BOUND, "%llu blocks missed their tolerance", misses);
  return PMC_OK;
}

pmc_status pmc_compress_static(pmc_ctx* ctx, const pmc_field* f, const void* d_x, int n, const double* tau,
                               void* d_streams, size_t streams_cap, pmc_store** out) {
  if (!ctx) return PMC_E_ARG;
  if (out) *out = nullptr;
  Geo g;
  if (!make_geo(f, &g)) return fail(ctx, PMC_E_ARG, "bad field");
  if (n < 1 || n > kMaxComps) return fail(ctx, PMC_E_ARG, "n must be in [1, %d]", kMaxComps);
  const uint64_t need = ws_layout(f, g, n).total;
  if (need > PMC_STATIC_WS_BYTES)
    return fail(ctx, PMC_E_NOMEM,
                "field needs %llu bytes of workspace; the static workspace holds %llu (use pmc_compress "
                "with a caller workspace)",
                (unsigned long long)need, (unsigned long long)PMC_STATIC_WS_BYTES);
  void* ws = scratch_ptr(ctx->device);
  if (!ws) return fail(ctx, PMC_E_DEVICE, "static workspace not set up on device %d", ctx->device);
  // the same kernels as pmc_compress; every workspace word they read is
  // written first in the same call (the per-component counters are cleared
  // by a fill kernel), so nothing of an earlier call carries over
  return pmc_compress(ctx, f, d_x, n, tau, ws, PMC_STATIC_WS_BYTES, d_streams, streams_cap, out);
}

pmc_status pmc_store_info(const pmc_store* s, int* n, double* tau, double* linf, uint64_t* bytes, uint64_t* nraw,
                          uint64_t* nesc) {
  if (!s) return PMC_E_ARG;
  if (n) *n = s->n;
  for (int i = 0; i < s->n; ++i) {
    if (tau) tau[i] = s->tau[i];
    if (linf) linf[i] = s->linf[i];
    if (bytes) bytes[i] = s->bytes[i];
    if (nraw) nraw[i] = s->nraw[i];
    if (nesc) nesc[i] = s->nesc[i];
  }
  return PMC_OK;
}

pmc_status pmc_store_codec(const pmc_store* s, int* codec) {
  if (!s || !codec) return PMC_E_ARG;
  *codec = s->codec;
  return PMC_OK;
}

pmc_status pmc_store_counts(const pmc_store* s, int i, uint64_t counts[5]) {
  if (!s || !counts || i < 0 || i >= s->n) return PMC_E_ARG;
  counts[0] = s->nempty[i];
  counts[1] = s->ncoded[i];
  counts[2] = s->nraw[i];
  counts[3] = s->nesc[i];
  counts[4] = s->nmiss[i];
  return PMC_OK;
}

pmc_status pmc_store_span(const pmc_store* s, int i, uint64_t* max_span_words, int* staged) {
  if (!s || i < 0 || i >= s->n) return PMC_E_ARG;
  if (max_span_words) *max_span_words = s->max_span[i];
  if (staged) *staged = s->max_span[i] <= stage_words() ? 1 : 0;
  return PMC_OK;
}

pmc_status pmc_store_decode_route(const pmc_store* s, int i, int* high_half) {
  if (!s || !high_half || i < 0 || i >= s->n) return PMC_E_ARG;
  *high_half = s->f.dtype == PMC_F32 && s->codec == 0 && s->full[i] == 0 ? 1 : 0;
  return PMC_OK;
}

pmc_status pmc_store_field(const pmc_store* s, pmc_field* f) {
  if (!s || !f) return PMC_E_ARG;
  *f = s->f;
  return PMC_OK;
}

pmc_status pmc_store_stream(const pmc_store* s, int i, const void** d_stream, uint64_t* bytes) {
  if (!s || i < 0 || i >= s->n) return PMC_E_ARG;
  if (d_stream) *d_stream = s->d_base + s->offset[i];
  if (bytes) *bytes = s->bytes[i];
  return PMC_OK;
}

pmc_status pmc_select_k(const pmc_store* s, double tol, int use_measured, int* k) {
  if (!s || !k) return PMC_E_ARG;
  for (int i = 0; i < s->n; ++i) {
    const double v = use_measured ? s->linf[i] : s->tau[i];
    if (v <= tol) {
      *k = i + 1;
      return PMC_OK;
    }
  }
  *k = 0;
  return PMC_E_UNREACHABLE;
}

size_t pmc_decode_ws_bytes(void) { return 256; }

static pmc_status decode_range(pmc_ctx* ctx, const pmc_store* s, int k0, int k1, const void* d_in, void* d_out,
                               void* d_ws, size_t ws_bytes) {
  if (!d_ws || ws_bytes < pmc_decode_ws_bytes()) return fail(ctx, PMC_E_NOMEM, "decode needs 256 bytes of workspace");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  unsigned int* status = (unsigned int*)d_ws;
  // the kernels only ever set the status word; it is cleared, and read,
  // when the call checks it
  if (ctx->sync_check && (e = launch_fill64((unsigned long long*)status, 1, 0ull, ctx->stream)) != hipSuccess)
    return hipfail(ctx, e, "status init");
  const int group = ctx->fused_decode ? kMaxDecode : 1;
  const void* in = d_in;
  for (int i0 = k0; i0 < k1; i0 += group) {
    const int i1 = i0 + group < k1 ? i0 + group : k1;
    uint64_t span = 0;
    bool hires = true;  // every residual component's blocks on the high-half route
    for (int i = i0; i < i1; ++i) {
      span = std::max(span, s->max_span[i]);
      if (i > 0 && s->full[i] != 0) hires = false;
    }
    if (s->f.dtype == PMC_F32) {
      DecArgs<float> a{};
      fill_decode_args(s, i0, i1, a);
      a.in = (const float*)in;
      a.out = (float*)d_out;
      a.g = s->g;
      a.status = status;
      ProfScope ps(ctx, s->codec == 0 ? "k_decode_f32" : "k_decode_pq_f32");
      e = launch_decode<float>(a, span, s->codec, hires, ctx->stream);
    } else {
      DecArgs<double> a{};
      fill_decode_args(s, i0, i1, a);
      a.in = (const double*)in;
      a.out = (double*)d_out;
      a.g = s->g;
      a.status = status;
      ProfScope ps(ctx, s->codec == 0 ? "k_decode_f64" : "k_decode_pq_f64");
      e = launch_decode<double>(a, span, s->codec, false, ctx->stream);
    }
    if (e != hipSuccess) return hipfail(ctx, e, "decode");
    in = d_out;
  }
  if (ctx->sync_check) {
    unsigned int h = 0;
    if ((e = read_back(ctx, &h, status, 4)) != hipSuccess) return hipfail(ctx, e, "status read");
    if (h) return fail(ctx, PMC_E_CORRUPT, "malformed stream");
  }
  return PMC_OK;
}

pmc_status pmc_retrieve_box(pmc_ctx* ctx, const pmc_store* s, int k, const uint64_t lo[3], const uint64_t hi[3],
                            void* d_out, void* d_ws, size_t ws_bytes) {
  if (!ctx) return PMC_E_ARG;
  if (!s || !d_out || !lo || !hi) return fail(ctx, PMC_E_ARG, "null argument");
  if (k < 1 || k > s->n) return fail(ctx, PMC_E_ARG, "k must be in [1, %d]", s->n);
  const uint64_t dims[3] = {s->g.nx, s->g.ny, s->g.nz};
  for (int a = 0; a < 3; ++a)
    if (!(lo[a] < hi[a] && hi[a] <= dims[a])) return fail(ctx, PMC_E_ARG, "box axis %d outside the field", a);
  if (!d_ws || ws_bytes < pmc_decode_ws_bytes()) return fail(ctx, PMC_E_NOMEM, "decode needs 256 bytes of workspace");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  unsigned int* status = (unsigned int*)d_ws;
  // the kernels only ever set the status word; it is cleared, and read,
  // when the call checks it
  if (ctx->sync_check && (e = launch_fill64((unsigned long long*)status, 1, 0ull, ctx->stream)) != hipSuccess)
    return hipfail(ctx, e, "status init");
  BoxArgs b{};
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = lo[a];
    b.hi[a] = hi[a];
    b.blo[a] = lo[a] / 4;
    b.bhi[a] = (hi[a] + 3) / 4;
  }
  b.waves_per_row = (uint32_t)((b.bhi[0] - b.blo[0] + 63) / 64 + 1);  // a row of blocks meets at most this many waves
  const void* in = nullptr;
  for (int i0 = 0; i0 < k; i0 += kMaxDecode) {
    const int i1 = i0 + kMaxDecode < k ? i0 + kMaxDecode : k;
    uint64_t span = 0;
    for (int i = i0; i < i1; ++i) span = std::max(span, s->max_span[i]);
    if (s->f.dtype == PMC_F32) {
      DecArgs<float> a{};
      fill_decode_args(s, i0, i1, a);
      a.in = (const float*)in;
      a.out = (float*)d_out;
      a.g = s->g;
      a.status = status;
      e = launch_decode_box<float>(a, b, span, s->codec, ctx->stream);
    } else {
      DecArgs<double> a{};
      fill_decode_args(s, i0, i1, a);
      a.in = (const double*)in;
      a.out = (double*)d_out;
      a.g = s->g;
      a.status = status;
      e = launch_decode_box<double>(a, b, span, s->codec, ctx->stream);
    }
    if (e != hipSuccess) return hipfail(ctx, e, "decode");
    in = d_out;
  }
  if (ctx->sync_check) {
    unsigned int h = 0;
    if ((e = read_back(ctx, &h, status, 4)) != hipSuccess) return hipfail(ctx, e, "status read");
    if (h) return fail(ctx, PMC_E_CORRUPT, "malformed stream");
  }
  return PMC_OK;
}

pmc_status pmc_retrieve(pmc_ctx* ctx, const pmc_store* s, int k, void* d_out, void* d_ws, size_t ws_bytes) {
  if (!ctx) return PMC_E_ARG;
  if (!s || !d_out) return fail(ctx, PMC_E_ARG, "null argument");
  if (!aligned16(d_out)) return fail(ctx, PMC_E_ARG, "d_out must be 16-byte aligned");
  if (k < 1 || k > s->n) return fail(ctx, PMC_E_ARG, "k must be in [1, %d]", s->n);
  return decode_range(ctx, s, 0, k, nullptr, d_out, d_ws, ws_bytes);
}

pmc_status pmc_refine(pmc_ctx* ctx, const pmc_store* s, int k_from, int k_to, void* d_inout, void* d_ws,
                      size_t ws_bytes) {
  if (!ctx) return PMC_E_ARG;
  if (!s || !d_inout) return fail(ctx, PMC_E_ARG, "null argument");
  if (!aligned16(d_inout)) return fail(ctx, PMC_E_ARG, "d_inout must be 16-byte aligned");
  if (k_from < 0 || k_to > s->n || k_from > k_to) return fail(ctx, PMC_E_ARG, "bad component range");
  if (k_from == k_to) return PMC_OK;
  return decode_range(ctx, s, k_from, k_to, k_from == 0 ? nullptr : d_inout, d_inout, d_ws, ws_bytes);
}

// ---- persistence -----------------------------------------------------------
pmc_status pmc_store_serialize(pmc_ctx* ctx, const pmc_store* s, void* host_buf, size_t cap, size_t* used) {
  if (!ctx) return PMC_E_ARG;
  if (!s || !used) return fail(ctx, PMC_E_ARG, "null argument");
  uint64_t region = 0;
  for (int i = 0; i < s->n; ++i) region = align256(region) + s->bytes[i];
  const uint64_t total = blob_header_bytes(s->n) + align256(region);
  *used = total;
  if (!host_buf) return PMC_OK;
  if (cap < total) return fail(ctx, PMC_E_NOMEM, "need %llu bytes", (unsigned long long)total);
  uint8_t* b = (uint8_t*)host_buf;
  std::memset(b, 0, total);
  uint32_t h32[4] = {kBlobMagic, 1u, (uint32_t)s->n, (uint32_t)s->codec};
  std::memcpy(b, h32, 16);
  uint64_t dims[3] = {s->f.nx, s->f.ny, s->f.nz};
  std::memcpy(b + 16, dims, 24);
  int32_t dt[2] = {s->f.dtype, 0};
  std::memcpy(b + 40, dt, 8);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  uint64_t off = 0;
  for (int i = 0; i < s->n; ++i) {
    uint8_t* c = b + 48 + 64ull * i;
    uint64_t v[8];
    std::memcpy(&v[0], &s->tau[i], 8);
    std::memcpy(&v[1], &s->linf[i], 8);
    v[2] = s->bytes[i];
    v[3] = s->nempty[i];
    v[4] = s->ncoded[i];
    v[5] = s->nraw[i];
    v[6] = s->nesc[i];
    v[7] = s->nmiss[i];
    std::memcpy(c, v, 64);
    off = align256(off);
    e = hipMemcpyAsync(b + blob_header_bytes(s->n) + off, s->d_base + s->offset[i], s->bytes[i],
                       hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "stream copy");
    off += s->bytes[i];
  }
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hipfail(ctx, e, "sync");
  return PMC_OK;
}

pmc_status pmc_store_deserialize(pmc_ctx* ctx, const void* host_buf, size_t size, void* d_streams, size_t cap,
                                 pmc_store** out) {
  if (!ctx) return PMC_E_ARG;
  if (!out || !d_streams) return fail(ctx, PMC_E_ARG, "null argument");
  *out = nullptr;
  BlobView v;
  if (!parse_blob(host_buf, size, &v)) return fail(ctx, PMC_E_CORRUPT, "malformed store blob");
  Geo g;
  if (!make_geo(&v.f, &g)) return fail(ctx, PMC_E_CORRUPT, "bad field in blob");
  const uint64_t auxb = aux_bytes(g);
  const uint64_t need = blob_device_bytes(v, g);
  if (cap < need) return fail(ctx, PMC_E_NOMEM, "need %llu bytes", (unsigned long long)need);
  const uint8_t* region = (const uint8_t*)host_buf + v.region_off;
  std::vector<uint64_t> words, spans;
  if (!check_blob_streams(v, g, region, &words, &spans)) return fail(ctx, PMC_E_CORRUPT, "malformed stream");
  pmc_store* s = new pmc_store();
  s->f = v.f;
  s->g = g;
  s->n = v.n;
  s->codec = v.codec;
  s->d_base = (const uint8_t*)d_streams;
  uint64_t off = 0;
  for (int i = 0; i < v.n; ++i) {
    const uint64_t* r = &v.rec[8 * i];
    double tau, linf;
    std::memcpy(&tau, &r[0], 8);
    std::memcpy(&linf, &r[1], 8);
    off = align256(off);
    s->tau.push_back(tau);
    s->linf.push_back(linf);
    s->minexp.push_back(floor_log2(tau));
    s->bytes.push_back(r[2]);
    s->offset.push_back(v.n * auxb + off);
    s->aux_offset.push_back(i * auxb);
    s->words.push_back(words[i]);
    s->nempty.push_back(r[3]);
    s->ncoded.push_back(r[4]);
    s->nraw.push_back(r[5]);
    s->nesc.push_back(r[6]);
    s->nmiss.push_back(r[7]);
    s->max_span.push_back(spans[i]);
    off += r[2];
  }
  hipError_t e = hipSetDevice(ctx->device);
  uint8_t* base = (uint8_t*)d_streams;
  // after the streams: a status word, set by the index rebuild when a
  // chunk's payload does not parse, then one flag per component, set when a
  // coded block is outside the float32 high-half decode route
  unsigned int* status = (unsigned int*)(base + need - kBlobTrailerBytes);
  unsigned long long* full = (unsigned long long*)(base + need - kBlobTrailerBytes) + 1;
  if (e == hipSuccess) e = launch_fill64((unsigned long long*)status, 1 + (uint64_t)v.n, 0ull, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + v.n * auxb, region, v.region_bytes, hipMemcpyHostToDevice, ctx->stream);
  // rebuild the per-block index of every stream
  for (int i = 0; i < v.n && e == hipSuccess; ++i) {
    AuxArgs a{};
    a.s = base + s->offset[i];
    a.aux = (uint32_t*)(base + s->aux_offset[i]);
    a.words = s->words[i];
    a.minexp = s->minexp[i];
    a.g = g;
    a.status = status;
    a.full = full + i;
    e = s->f.dtype == PMC_F32 ? launch_aux<float>(a, s->codec, ctx->stream)
                              : launch_aux<double>(a, s->codec, ctx->stream);
  }
  unsigned long long trailer[1 + kMaxComps] = {};
  if (e == hipSuccess)
    e = hipMemcpyAsync(trailer, status, 8 * (1 + (size_t)v.n), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  const unsigned int h = (unsigned int)(trailer[0] & 0xFFFFFFFFull);
  for (int i = 0; i < v.n; ++i) s->full.push_back(trailer[1 + i]);
  if (e != hipSuccess) {
    delete s;
    return hipfail(ctx, e, "stream upload");
  }
  if (h) {
    delete s;
    return fail(ctx, PMC_E_CORRUPT, "a chunk's payload does not parse");
  }
  *out = s;
  return PMC_OK;
}

void pmc_store_free(pmc_store* s) { delete s; }

}  // extern "C"
