// batch.cpp -- many fields of uneven sizes and mixed types compressed together
// (Alg. 1, Sec. 4.1, for every field).  All components of all fields run as
// one captured HIP graph: per component, a persistent encode kernel per
// element type over a list of (field, 64-block wave) items, a segmented chunk
// scan and a batched pack.  The schedule (persistent grid size, item order)
// is picked by a small autotuner; every schedule yields identical bytes since
// each wave's output depends only on its own blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace pmc;
using namespace pmc_host;

struct pmc_batch {
  pmc_ctx* ctx = nullptr;
  int nf = 0, maxn = 0;
  std::vector<pmc_field> f;
  std::vector<Geo> g;
  std::vector<int> n;
  std::vector<std::vector<double>> tau;
  std::vector<std::vector<int>> minexp;
  // workspace layout (byte offsets into d_ws)
  std::vector<uint64_t> off_xt0, off_xt1, off_staging, off_cw, off_offs, off_tiles, off_berr;
  std::vector<uint64_t> meta_first;  // index of the field's first CompMeta
  uint64_t off_table = 0, off_items = 0, off_meta = 0, ws_total = 0;
  // stream regions (byte offsets into d_streams)
  std::vector<uint64_t> region_off, region_cap;
  uint64_t streams_total = 0;
  // items: [encode f32 | encode f64 | scan tiles | chunk quads]
  std::vector<Item> items;
  uint32_t n32 = 0, n64 = 0, ntiles = 0, nquads = 0;
  uint64_t items_cap = 0;
  // schedule
  int grid_mult = 4, order = 0;
  int cus = 256;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_ws = nullptr;
  const void* g_streams = nullptr;
  int g_grid = -1, g_order = -1;
  bool items_uploaded = false;
  std::vector<int> uploaded_order;
};

namespace {

const char* kOrderName[3] = {"field-major", "interleaved", "largest-first"};

// wave items of one element type in the requested order
void build_items(pmc_batch* b) {
  b->items.clear();
  for (int dt = 1; dt <= 2; ++dt) {
    std::vector<int> fl;
    for (int i = 0; i < b->nf; ++i)
      if (b->f[i].dtype == dt) fl.push_back(i);
    if (b->order == 2)
      std::stable_sort(fl.begin(), fl.end(), [&](int a, int c) { return b->g[a].nblocks > b->g[c].nblocks; });
    size_t before = b->items.size();
    if (b->order == 1) {
      uint64_t maxw = 0;
      for (int i : fl) maxw = std::max<uint64_t>(maxw, (b->g[i].nblocks + 63) / 64);
      for (uint64_t w = 0; w < maxw; ++w)
        for (int i : fl)
          if (w < (b->g[i].nblocks + 63) / 64) b->items.push_back(Item{(uint32_t)i, (uint32_t)w});
    } else {
      for (int i : fl)
        for (uint64_t w = 0; w < (b->g[i].nblocks + 63) / 64; ++w) b->items.push_back(Item{(uint32_t)i, (uint32_t)w});
    }
    (dt == 1 ? b->n32 : b->n64) = (uint32_t)(b->items.size() - before);
  }
  b->ntiles = 0;
  for (int i = 0; i < b->nf; ++i) {
    const uint64_t t = (b->g[i].nchunks + kScanTile - 1) / kScanTile;
    for (uint64_t j = 0; j < t; ++j) b->items.push_back(Item{(uint32_t)i, (uint32_t)j});
    b->ntiles += (uint32_t)t;
  }
  b->nquads = 0;
  for (int i = 0; i < b->nf; ++i) {
    const uint64_t q = (b->g[i].nchunks + 3) / 4;
    for (uint64_t j = 0; j < q; ++j) b->items.push_back(Item{(uint32_t)i, (uint32_t)j});
    b->nquads += (uint32_t)q;
  }
}

void drop_graph(pmc_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->g_ws = b->g_streams = nullptr;
  b->g_grid = b->g_order = -1;
}

std::string tune_key(const pmc_batch* b) {
  uint64_t total = 0;
  int c32 = 0, c64 = 0;
  for (int i = 0; i < b->nf; ++i) {
    total += b->g[i].nblocks;
    (b->f[i].dtype == PMC_F32 ? c32 : c64)++;
  }
  int cls = 0;
  while ((1ull << (cls + 1)) <= total) ++cls;
  char k[128];
  std::snprintf(k, sizeof(k), "gfx950 f32=%d f64=%d blocks=2^%d maxn=%d", c32, c64, cls, b->maxn);
  return k;
}

bool tune_lookup(const pmc_batch* b, int* grid, int* order) {
  const char* path = std::getenv("PMC_TUNE_CACHE");
  if (!path) return false;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  const std::string key = tune_key(b);
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof(line), fp)) {
    char* bar = std::strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    if (key == line) {
      int gm = 0, od = 0;
      if (std::sscanf(bar + 1, "%d %d", &gm, &od) == 2 && gm >= 1 && gm <= 64 && od >= 0 && od <= 2) {
        *grid = gm;
        *order = od;
        found = true;
      }
    }
  }
  std::fclose(fp);
  return found;
}

void tune_store(const pmc_batch* b, float ms) {
  const char* path = std::getenv("PMC_TUNE_CACHE");
  if (!path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "%s|%d %d %.4f\n", tune_key(b).c_str(), b->grid_mult, b->order, ms);
  std::fclose(fp);
}

}  // namespace

extern "C" {

pmc_status pmc_batch_plan(pmc_ctx* ctx, int nf, const pmc_field* fields, const int* n, const double* const* tau,
                          pmc_batch** out) {
  if (!ctx) return PMC_E_ARG;
  if (!out || !fields || !n || !tau || nf < 1) return fail(ctx, PMC_E_ARG, "bad batch arguments");
  *out = nullptr;
  if (ctx->codec != 0) return fail(ctx, PMC_E_ARG, "batches use the block-transform codec (PMC_OPT_CODEC 0)");
  pmc_batch* b = new pmc_batch();
  b->ctx = ctx;
  b->nf = nf;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
    b->cus = prop.multiProcessorCount;
  uint64_t ws = 0, nmeta = 0, reg = 0;
  for (int i = 0; i < nf; ++i) {
    Geo g;
    if (!make_geo(&fields[i], &g) || n[i] < 1 || n[i] > kMaxComps || !tau[i]) {
      delete b;
      return fail(ctx, PMC_E_ARG, "field %d: bad field or component count", i);
    }
    std::vector<double> t(tau[i], tau[i] + n[i]);
    std::vector<int> me;
    for (int c = 0; c < n[i]; ++c) {
      if (!(t[c] > 0.0) || !std::isfinite(t[c]) || (c > 0 && !(t[c] < t[c - 1]))) {
        delete b;
        return fail(ctx, PMC_E_ARG, "field %d: tau must be positive and strictly decreasing", i);
      }
      me.push_back(floor_log2(t[c]));
    }
    b->f.push_back(fields[i]);
    b->g.push_back(g);
    b->n.push_back(n[i]);
    b->tau.push_back(t);
    b->minexp.push_back(me);
    b->maxn = std::max(b->maxn, n[i]);
    // x~ ping-pong buffers (component i reads buffer (i-1)&1, writes i&1),
    // in the encoder's tiled layout: 64 * 64 values per wave of 64 blocks
    const uint64_t tile = align256((g.nblocks + 63) / 64 * 4096 * elem_size(&fields[i]));
    b->off_xt0.push_back(ws);
    if (n[i] > 1) ws += tile;
    b->off_xt1.push_back(ws);
    if (n[i] > 2) ws += tile;
    b->off_staging.push_back(ws);
    ws += align256(g.nchunks * chunk_cap_words_host(fields[i].dtype) * 4);
    b->off_cw.push_back(ws);
    ws += align256(g.nchunks * 4);
    b->off_offs.push_back(ws);
    ws += align256(g.nchunks * 4);
    b->off_tiles.push_back(ws);
    ws += align256((g.nchunks + kScanTile - 1) / kScanTile * 8);
    b->off_berr.push_back(ws);  // per-block error carried between components
    if (n[i] > 1) ws += align256(g.nblocks * 8);
    b->meta_first.push_back(nmeta);
    nmeta += n[i];
    b->region_off.push_back(reg);
    const uint64_t cap = n[i] * aux_bytes(g) + n[i] * align256(stream_cap_one(g, fields[i].dtype));
    b->region_cap.push_back(cap);
    reg += align256(cap);
  }
  b->off_table = ws;
  ws += align256((uint64_t)nf * sizeof(FieldDev));
  b->off_meta = ws;
  ws += align256(nmeta * sizeof(CompMeta));
  b->off_items = ws;
  int gm = 4, od = 0;
  if (tune_lookup(b, &gm, &od)) {
    b->grid_mult = gm;
    b->order = od;
  }
  build_items(b);
  b->items_cap = b->items.size();
  ws += align256(b->items_cap * sizeof(Item));
  b->ws_total = ws;
  b->streams_total = reg;
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(ctx, PMC_E_DEVICE, "stream creation failed");
  }
  *out = b;
  return PMC_OK;
}

pmc_status pmc_batch_sizes(const pmc_batch* b, size_t* ws_bytes, size_t* streams_bytes) {
  if (!b) return PMC_E_ARG;
  if (ws_bytes) *ws_bytes = b->ws_total;
  if (streams_bytes) *streams_bytes = b->streams_total;
  return PMC_OK;
}

pmc_status pmc_batch_schedule(pmc_batch* b, int grid_mult, int order) {
  if (!b || grid_mult < 1 || grid_mult > 64 || order < 0 || order > 2) return PMC_E_ARG;
  if (b->grid_mult != grid_mult || b->order != order) {
    b->grid_mult = grid_mult;
    b->order = order;
    build_items(b);
    b->items_uploaded = false;
  }
  return PMC_OK;
}

pmc_status pmc_batch_get_schedule(const pmc_batch* b, int* grid_mult, int* order) {
  if (!b) return PMC_E_ARG;
  if (grid_mult) *grid_mult = b->grid_mult;
  if (order) *order = b->order;
  return PMC_OK;
}

static pmc_status batch_capture(pmc_batch* b, uint8_t* ws, uint8_t* streams) {
  pmc_ctx* ctx = b->ctx;
  drop_graph(b);
  const FieldDev* table = (const FieldDev*)(ws + b->off_table);
  const Item* items = (const Item*)(ws + b->off_items);
  hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hipfail(ctx, e, "begin capture");
  hipError_t le = launch_batch_init(table, (uint32_t)b->nf, b->cap_stream);
  const uint32_t grid = (uint32_t)(b->grid_mult * b->cus);
  for (int c = 0; c < b->maxn && le == hipSuccess; ++c) {
    BatchArgs a{table, (uint32_t)b->nf, items, b->n32, c};
    if (b->n32) le = launch_encode_batch<float>(a, std::min<uint32_t>(grid, b->n32), b->cap_stream);
    a.items = items + b->n32;
    a.nitems = b->n64;
    if (le == hipSuccess && b->n64)
      le = launch_encode_batch<double>(a, std::min<uint32_t>(grid, b->n64), b->cap_stream);
    a.items = items + b->n32 + b->n64;
    a.nitems = b->ntiles;
    if (le == hipSuccess) le = launch_batch_scan(a, (uint32_t)b->nf, b->cap_stream);
    a.items = items + b->n32 + b->n64 + b->ntiles;
    a.nitems = b->nquads;
    if (le == hipSuccess) le = launch_batch_pack(a, b->cap_stream);
  }
  e = hipStreamEndCapture(b->cap_stream, &b->graph);
  if (le != hipSuccess) return hipfail(ctx, le, "capture launch");
  if (e != hipSuccess) return hipfail(ctx, e, "end capture");
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hipfail(ctx, e, "instantiate");
  b->g_ws = ws;
  b->g_streams = streams;
  b->g_grid = b->grid_mult;
  b->g_order = b->order;
  return PMC_OK;
}

// upload the field table (current input pointers) and items, then replay
static pmc_status batch_launch(pmc_batch* b, const void* const* d_x, uint8_t* ws, uint8_t* streams) {
  pmc_ctx* ctx = b->ctx;
  std::vector<FieldDev> tab(b->nf);
  for (int i = 0; i < b->nf; ++i) {
    FieldDev& d = tab[i];
    std::memset(&d, 0, sizeof(d));
    d.x = d_x[i];
    d.xt[0] = ws + b->off_xt0[i];
    d.xt[1] = ws + b->off_xt1[i];
    d.g = b->g[i];
    d.staging = (uint32_t*)(ws + b->off_staging[i]);
    d.chunk_words = (uint32_t*)(ws + b->off_cw[i]);
    d.offsets = (uint32_t*)(ws + b->off_offs[i]);
    d.tile_sums = (unsigned long long*)(ws + b->off_tiles[i]);
    d.berr = (double*)(ws + b->off_berr[i]);
    d.region = streams + b->region_off[i];
    d.aux0 = (uint32_t*)d.region;
    d.aux_stride = aux_bytes(b->g[i]) / 4;
    d.meta0 = (CompMeta*)(ws + b->off_meta) + b->meta_first[i];
    d.region_cap = b->region_cap[i];
    d.ncomp = b->n[i];
    d.dtype = b->f[i].dtype;
    d.ntiles = (uint32_t)((b->g[i].nchunks + kScanTile - 1) / kScanTile);
    for (int c = 0; c < b->n[i]; ++c) {
      d.tau[c] = b->tau[i][c];
      d.minexp[c] = b->minexp[i][c];
    }
  }
  hipError_t e = hipMemcpyAsync(ws + b->off_table, tab.data(), tab.size() * sizeof(FieldDev),
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !b->items_uploaded) {
    e = hipMemcpyAsync(ws + b->off_items, b->items.data(), b->items.size() * sizeof(Item), hipMemcpyHostToDevice,
                       ctx->stream);
  }
  if (e != hipSuccess) return hipfail(ctx, e, "table upload");
  // the host vectors above are pageable: wait for the copies before they go
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hipfail(ctx, e, "sync");
  b->items_uploaded = true;
  if (!b->exec || b->g_ws != ws || b->g_streams != streams || b->g_grid != b->grid_mult || b->g_order != b->order) {
    pmc_status st = batch_capture(b, ws, streams);
    if (st != PMC_OK) return st;
  }
  {
    ProfScope ps(ctx, "batch_graph");
    e = hipGraphLaunch(b->exec, ctx->stream);
  }
  if (e != hipSuccess) return hipfail(ctx, e, "graph launch");
  return PMC_OK;
}

pmc_status pmc_batch_compress(pmc_batch* b, const void* const* d_x, void* d_ws, size_t ws_bytes, void* d_streams,
                              size_t streams_cap, pmc_store** out) {
  if (!b) return PMC_E_ARG;
  pmc_ctx* ctx = b->ctx;
  if (!d_x || !d_ws || !d_streams || !out) return fail(ctx, PMC_E_ARG, "null argument");
  for (int i = 0; i < b->nf; ++i) {
    out[i] = nullptr;
    if (!d_x[i]) return fail(ctx, PMC_E_ARG, "field %d: null input", i);
    if (!aligned16(d_x[i])) return fail(ctx, PMC_E_ARG, "field %d: input not 16-byte aligned", i);
  }
  if (ws_bytes < b->ws_total)
    return fail(ctx, PMC_E_NOMEM, "workspace too small: need %llu bytes", (unsigned long long)b->ws_total);
  if (streams_cap < b->streams_total)
    return fail(ctx, PMC_E_NOMEM, "stream capacity too small: need %llu bytes", (unsigned long long)b->streams_total);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  uint8_t* ws = (uint8_t*)d_ws;
  uint8_t* streams = (uint8_t*)d_streams;
  pmc_status st = batch_launch(b, d_x, ws, streams);
  if (st != PMC_OK) return st;
  const uint64_t nmeta = b->meta_first.back() + b->n.back();
  std::vector<CompMeta> hm(nmeta);
  e = hipMemcpyAsync(hm.data(), ws + b->off_meta, nmeta * sizeof(CompMeta), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "meta copy");
  unsigned int flags = 0;
  unsigned long long misses = 0;
  for (const CompMeta& m : hm) {
    flags |= m.flags;
    misses += m.nmiss;
  }
  if (flags & FLAG_NONFINITE) return fail(ctx, PMC_E_NONFINITE, "input holds NaN or Inf");
  if (flags & (FLAG_INDEX | FLAG_OVERFLOW)) return fail(ctx, PMC_E_NOMEM, "a stream exceeds its capacity");
  for (int i = 0; i < b->nf; ++i)
    out[i] = store_from_meta(&b->f[i], b->g[i], b->n[i], b->tau[i].data(), b->minexp[i].data(),
                             hm.data() + b->meta_first[i], streams + b->region_off[i], 0);
  if (misses) return fail(ctx, PMC_E_BOUND, "%llu blocks missed their tolerance", misses);
  return PMC_OK;
}

pmc_status pmc_batch_tune(pmc_batch* b, const void* const* d_x, void* d_ws, size_t ws_bytes, void* d_streams,
                          size_t streams_cap, float* best_ms) {
  if (!b) return PMC_E_ARG;
  pmc_ctx* ctx = b->ctx;
  if (!d_x || !d_ws || !d_streams) return fail(ctx, PMC_E_ARG, "null argument");
  if (ws_bytes < b->ws_total || streams_cap < b->streams_total) return fail(ctx, PMC_E_NOMEM, "buffers too small");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
    return fail(ctx, PMC_E_DEVICE, "event creation failed");
  const int grids[4] = {1, 2, 4, 8};
  float best = 1e30f;
  int bg = b->grid_mult, bo = b->order;
  pmc_status st = PMC_OK;
  for (int gi = 0; gi < 4 && st == PMC_OK; ++gi) {
    for (int od = 0; od < 3 && st == PMC_OK; ++od) {
      pmc_batch_schedule(b, grids[gi], od);
      st = batch_launch(b, d_x, (uint8_t*)d_ws, (uint8_t*)d_streams);  // warm-up (and capture)
      float ms = 1e30f;
      for (int rep = 0; rep < 2 && st == PMC_OK; ++rep) {
        (void)hipEventRecord(t0, ctx->stream);
        e = hipGraphLaunch(b->exec, ctx->stream);
        (void)hipEventRecord(t1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float m = 0.0f;
        if (e == hipSuccess && hipEventElapsedTime(&m, t0, t1) == hipSuccess) ms = std::min(ms, m);
        if (e != hipSuccess) st = hipfail(ctx, e, "tune launch");
      }
      if (ms < best) {
        best = ms;
        bg = grids[gi];
        bo = od;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != PMC_OK) return st;
  pmc_batch_schedule(b, bg, bo);
  tune_store(b, best);
  if (best_ms) *best_ms = best;
  return PMC_OK;
}

const char* pmc_batch_order_name(int order) { return order >= 0 && order < 3 ? kOrderName[order] : "?"; }

void pmc_batch_free(pmc_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
