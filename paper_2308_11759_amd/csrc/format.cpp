// format.cpp -- the block grid of a field and the host-side validation of
// component streams and store blobs (untrusted bytes).  No HIP here: the
// sanitizer builds of the CPU tests compile this file on its own.
#include "format.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

using namespace pmc;

namespace pmc_host {

bool make_geo(const pmc_field* f, pmc::Geo* g) {
  if (!f || f->nx < 1 || f->ny < 1 || f->nz < 1) return false;
  if (f->dtype != PMC_F32 && f->dtype != PMC_F64) return false;
  if (f->nx > (1ull << 40) || f->ny > (1ull << 40) || f->nz > (1ull << 40)) return false;
  // at most 2^36 values and 2^32 blocks (so every size below fits 64 bits and
  // every grid fits the launch limits), checked without wrapping
  uint64_t nxy = 0, n = 0, bxy = 0, nb = 0;
  if (__builtin_mul_overflow(f->nx, f->ny, &nxy) || __builtin_mul_overflow(nxy, f->nz, &n) || n > (1ull << 36))
    return false;
  g->nx = f->nx;
  g->ny = f->ny;
  g->nz = f->nz;
  g->nbx = (f->nx + 3) / 4;
  g->nby = (f->ny + 3) / 4;
  g->nbz = (f->nz + 3) / 4;
  if (__builtin_mul_overflow(g->nbx, g->nby, &bxy) || __builtin_mul_overflow(bxy, g->nbz, &nb) || nb > (1ull << 32))
    return false;
  g->nblocks = nb;
  g->nchunks = (g->nblocks + 15) / 16;
  g->rows_aligned = (f->nx % 4) == 0;
  g->pad = 0;
  return true;
}

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

int floor_log2(double tau) {
  uint64_t b;
  std::memcpy(&b, &tau, 8);
  int biased = (int)((b >> 52) & 0x7ff);
  uint64_t mant = b & ((1ull << 52) - 1);
  if (biased == 0) {  // subnormal: position of the leading mantissa bit
    int lead = 63 - __builtin_clzll(mant);
    return lead - 1074;
  }
  return biased - 1023;
}

uint64_t aux_bytes(const pmc::Geo& g) { return align256(4 * g.nblocks); }

uint64_t blob_header_bytes(int n) { return align256(48 + 64ull * n); }

bool parse_blob(const void* host_buf, size_t size, BlobView* v) {
  const uint8_t* b = (const uint8_t*)host_buf;
  if (!b || size < 48) return false;
  uint32_t h32[4];
  std::memcpy(h32, b, 16);
  if (h32[0] != kBlobMagic || h32[1] != 1u) return false;
  int n = (int)h32[2];
  if (n < 1 || n > kMaxComps) return false;
  if (h32[3] > 1u) return false;
  v->codec = (int)h32[3];
  if (size < blob_header_bytes(n)) return false;
  v->n = n;
  uint64_t dims[3];
  std::memcpy(dims, b + 16, 24);
  int32_t dt[2];
  std::memcpy(dt, b + 40, 8);
  v->f.nx = dims[0];
  v->f.ny = dims[1];
  v->f.nz = dims[2];
  v->f.dtype = dt[0];
  v->f.reserved = 0;
  v->rec.resize(8ull * n);
  std::memcpy(v->rec.data(), b + 48, 64ull * n);
  // the streams follow the header, each on a 256-byte boundary; every running
  // sum is checked against the blob size before it is formed, so no sum wraps
  v->region_off = blob_header_bytes(n);
  const uint64_t avail = size - v->region_off;
  uint64_t region = 0;
  for (int i = 0; i < n; ++i) {
    const uint64_t bytes = v->rec[8 * i + 2];
    region = align256(region);
    if (region > avail || bytes > avail - region) return false;
    region += bytes;
  }
  v->region_bytes = region;
  return true;
}

bool check_stream(const uint8_t* p, uint64_t bytes, const pmc_field* f, const pmc::Geo& g, double tau, int codec,
                         uint64_t* words, uint64_t* max_span) {
  if (bytes < 64) return false;
  uint32_t h[16];
  std::memcpy(h, p, 64);
  if (h[0] != kStreamMagic) return false;
  if ((h[1] & 0xFF) != kStreamVersion || ((h[1] >> 8) & 0xFF) != (uint32_t)codec ||
      ((h[1] >> 16) & 0xFF) != (uint32_t)f->dtype || (h[1] >> 24) != 3u)
    return false;
  uint64_t nx = h[2] | ((uint64_t)h[3] << 32), ny = h[4] | ((uint64_t)h[5] << 32), nz = h[6] | ((uint64_t)h[7] << 32);
  if (nx != f->nx || ny != f->ny || nz != f->nz) return false;
  uint64_t tb = h[8] | ((uint64_t)h[9] << 32);
  double t;
  std::memcpy(&t, &tb, 8);
  if (!(t == tau) || (int32_t)h[10] != floor_log2(tau) || h[11] != 16u) return false;
  uint64_t nch = h[12] | ((uint64_t)h[13] << 32), w = h[14] | ((uint64_t)h[15] << 32);
  if (nch != g.nchunks) return false;
  // bytes = 64 + 4 nch + 4 w, compared without forming a sum that could wrap
  if (bytes < 64 || nch > (bytes - 64) / 4) return false;
  const uint64_t rest = bytes - 64 - 4 * nch;
  if (rest % 4 != 0 || w != rest / 4 || w > 0xFFFFFFFFull) return false;
  // the index is read with memcpy: a caller's blob need not be 4-byte aligned
  auto idx = [p](uint64_t c) {
    uint32_t v;
    std::memcpy(&v, p + 64 + 4 * c, 4);
    return (uint64_t)v;
  };
  uint64_t prev = 0;
  for (uint64_t c = 0; c < nch; ++c) {
    if (idx(c) < prev || idx(c) > w) return false;
    prev = idx(c);
  }
  // largest span of four consecutive chunks (the chunks of one decode wave)
  uint64_t span = 0;
  for (uint64_t c = 0; c < nch; c += 4) {
    const uint64_t stop = c + 4 < nch ? idx(c + 4) : w;
    span = std::max<uint64_t>(span, stop - idx(c));
  }
  *words = w;
  *max_span = span;
  return true;
}

bool check_blob_streams(const BlobView& v, const pmc::Geo& g, const uint8_t* region, std::vector<uint64_t>* words,
                               std::vector<uint64_t>* spans) {
  uint64_t off = 0;
  double prev = 0.0;
  for (int i = 0; i < v.n; ++i) {
    const uint64_t* r = &v.rec[8 * i];
    double tau;
    std::memcpy(&tau, &r[0], 8);
    off = align256(off);
    uint64_t w = 0, span = 0;
    if (!(tau > 0.0) || !std::isfinite(tau) || (i > 0 && !(tau < prev)) ||
        !check_stream(region + off, r[2], &v.f, g, tau, v.codec, &w, &span))
      return false;
    if (words) words->push_back(w);
    if (spans) spans->push_back(span);
    prev = tau;
    off += r[2];
  }
  return true;
}

uint64_t blob_device_bytes(const BlobView& v, const pmc::Geo& g) {
  return v.n * aux_bytes(g) + align256(v.region_bytes) + kBlobTrailerBytes;
}

}  // namespace pmc_host

extern "C" {

pmc_status pmc_store_device_bytes(const void* host_buf, size_t size, size_t* need) {
  pmc_host::BlobView v;
  Geo g;
  if (!need || !pmc_host::parse_blob(host_buf, size, &v) || !pmc_host::make_geo(&v.f, &g)) return PMC_E_CORRUPT;
  if (!pmc_host::check_blob_streams(v, g, (const uint8_t*)host_buf + v.region_off, nullptr, nullptr))
    return PMC_E_CORRUPT;
  *need = pmc_host::blob_device_bytes(v, g);
  return PMC_OK;
}

}  // extern "C"
