// launch.hpp -- kernel argument blocks and host launchers shared by the HIP
// kernels (kernels.hip) and the C-ABI (capi.cpp).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "format.hpp"  // the block grid and the stream constants

namespace pmc {

constexpr int kMaxDecode = 16;  // components decoded by one k_decode launch

enum : unsigned int {
  FLAG_NONFINITE = 1u,  // NaN / Inf in the input field
  FLAG_OVERFLOW = 2u,   // stream capacity exceeded
  FLAG_INDEX = 4u       // payload too large for 32-bit word offsets
};

// per-component results kept on the device during compression
struct CompMeta {
  unsigned long long linf_bits;  // max measured error, float64 bits (>= 0)
  unsigned long long nempty, ncoded, nraw, nesc, nmiss;  // ncoded: not counted on the device
  unsigned long long payload_words;
  unsigned long long stream_offset;  // byte offset of the stream in the output
  unsigned long long stream_bytes;
  unsigned int flags;
  unsigned int pad;
  unsigned long long max_span;  // largest payload words of four consecutive chunks (one decode wave)
  unsigned long long full;      // nonzero: some coded block is outside the float32 high-half decode route
  unsigned long long reserved[4];
};
static_assert(sizeof(CompMeta) == 128, "CompMeta layout");

template <class T> struct EncArgs {
  const T* x;
  const T* xt_in;  // x~_{i-1} (not read for the first component)
  T* xt_out;       // x~_i (not written for the last component); never xt_in
  Geo g;
  double tau;
  int minexp;
  int first;  // x~_{i-1} = 0: not read
  int last;   // x~_i not written
  uint32_t* staging;
  uint32_t* chunk_words;
  uint32_t* aux;   // per block: bit offset of the block inside its chunk
  CompMeta* meta;  // this component's entry
  double* berr;    // per block: max error before this component (read unless first), after it (written unless last)
  double h0, inv0;  // codec 1: the bin 2 tau and its reciprocal (computed on the host)
};

// chunk offsets are an exclusive scan of chunk word counts, done in tiles of
// kScanTile chunks: tile sums, a scan of the tile sums, then per-tile scans
constexpr int kScanTile = 1024;

struct ScanArgs {
  const uint32_t* chunk_words;
  uint32_t* offsets;
  unsigned long long* tile_sums;  // ceil(nchunks / kScanTile) entries
  uint64_t nchunks;
  uint64_t aux_bytes;  // device bytes of one component's block index (256-aligned)
  CompMeta* meta;      // all components
  int comp, ncomp;
  unsigned long long streams_cap;
};

struct PackArgs {
  const uint32_t* staging;
  const uint32_t* chunk_words;
  const uint32_t* offsets;
  uint64_t nchunks;
  CompMeta* meta;  // the pack records each component's largest decode-wave span
  int comp;
  int minexp;
  uint8_t* streams;
  Geo g;
  double tau;
  int codec;  // written into the stream header
};

template <class T> struct DecArgs {
  const uint8_t* s[kMaxDecode];    // stream starts
  const uint32_t* aux[kMaxDecode];  // per-block bit offsets inside the chunk
  uint64_t words[kMaxDecode];      // payload words of each stream
  int minexp[kMaxDecode];
  double step[kMaxDecode];  // codec 1: the bin 2 tau of each component
  int ncomp;
  uint32_t relmask;  // bit i: component i is a residual (not a store's first), planes counted from its first non-empty one
  const T* in;  // x~ to continue from; NULL = +0
  T* out;
  Geo g;
  unsigned int* status;  // bit 0: malformed stream
};

// a box [lo, hi) of the field (value coordinates x, y, z) for region
// retrieval: blo/bhi are its block ranges; the output is the box alone, dense,
// x fastest.  Work: one workgroup per (block row of the box, wave of that row)
struct BoxArgs {
  uint64_t lo[3], hi[3];
  uint64_t blo[3], bhi[3];
  uint32_t waves_per_row;
  uint32_t pad;
  uint64_t row_first, row_last;  // set per workgroup: the blocks of its row inside the box
};

// one retrieval query of a server step: out = in (or +0) + components
// [0, ncomp) of the listed streams
struct QueryDev {
  const uint8_t* s[kMaxComps];
  const uint32_t* aux[kMaxComps];
  uint64_t words[kMaxComps];
  int minexp[kMaxComps];
  double step[kMaxComps];  // codec 1: the bin 2 tau of each component
  int ncomp;
  uint32_t relmask;  // as DecArgs::relmask
  int dtype;
  const void* in;
  void* out;
  Geo g;
};

struct ServeArgs {
  const QueryDev* q;
  const uint32_t* wave_prefix;  // nq + 1 entries
  uint32_t nq;
  uint32_t nwaves;
  unsigned int* status;
};

// rebuild the per-block bit offsets of one stream (one lane per chunk)
struct AuxArgs {
  const uint8_t* s;
  uint32_t* aux;
  uint64_t words;
  int minexp;
  Geo g;
  unsigned int* status;  // optional (NULL): set when a chunk fails to parse
  unsigned long long* full;  // optional (NULL): set when a coded block is outside the float32 high-half route
};

// ---- batches of fields (one table entry per field) -----------------------
struct FieldDev {
  const void* x;
  void* xt[2];  // x~ ping-pong: component i reads xt[(i-1)&1], writes xt[i&1]
  Geo g;
  uint32_t* staging;
  uint32_t* chunk_words;
  uint32_t* offsets;
  unsigned long long* tile_sums;
  uint32_t* aux0;           // block index of component 0; component i at aux0 + i * aux_stride
  uint64_t aux_stride;      // in 32-bit words
  CompMeta* meta0;          // meta of component 0; component i at meta0 + i
  double* berr;             // per-block error carried between components
  uint8_t* region;          // the field's stream region: block indexes, then streams
  unsigned long long region_cap;
  int ncomp;
  int dtype;                // 1 = f32, 2 = f64
  uint32_t ntiles;          // scan tiles of the field
  uint32_t pad;
  double tau[kMaxComps];
  int minexp[kMaxComps];
};

struct Item {  // (field, group) : a wave of 64 blocks, a scan tile, or 4 chunks
  uint32_t field, index;
};

struct BatchArgs {
  const FieldDev* fields;
  uint32_t nfields;
  const Item* items;  // encode waves of one dtype, scan tiles or chunk quads
  uint32_t nitems;
  int comp;
};

template <class T> hipError_t launch_encode_batch(const BatchArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_batch_scan(const BatchArgs& tiles, uint32_t nfields, hipStream_t s);
hipError_t launch_batch_pack(const BatchArgs& quads, hipStream_t s);
hipError_t launch_batch_init(const FieldDev* fields, uint32_t nfields, hipStream_t s);

// codec: 0 the block-transform codec, 1 prediction and quantisation
template <class T> hipError_t launch_encode(const EncArgs<T>& a, int codec, hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, hipStream_t s);
template <class T> hipError_t launch_aux(const AuxArgs& a, int codec, hipStream_t s);
// max_span: the largest word span of a wave's four chunks over the decoded
// streams; spans up to the LDS staging capacity use the staged kernel
// hires: as launch_decode's, for every query of the launch
template <class T>
hipError_t launch_decode_queries(const ServeArgs& a, uint64_t max_span, int codec, bool hires, hipStream_t s);
template <class T> hipError_t launch_pack(const PackArgs& a, hipStream_t s);
// hires: every residual component of the launch (store index > 0) has no
// block outside the float32 high-half route (CompMeta.full == 0), so the
// decoder may run them on that route alone
template <class T>
hipError_t launch_decode(const DecArgs<T>& a, uint64_t max_span, int codec, bool hires, hipStream_t s);
// components [0, a.ncomp) of the blocks meeting the box, written to a.out as the box alone
template <class T>
hipError_t launch_decode_box(const DecArgs<T>& a, const BoxArgs& b, uint64_t max_span, int codec, hipStream_t s);
uint64_t stage_words();  // capacity of the decoder's LDS staging buffer, in words
template <class T> hipError_t launch_range(const T* x, uint64_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_fill64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);
// the same with p[j] = vj instead (one launch)
hipError_t launch_fill64_one(unsigned long long* p, uint64_t n, unsigned long long v, uint64_t j,
                             unsigned long long vj, hipStream_t s);
// out[0] = sum of d, out[1] = sum of d^2 in float64, d = a - b - shift (b NULL: 0);
// ws holds sum_sq_ws_bytes() bytes of partials; out may lie inside ws past them
template <class T>
hipError_t launch_sum_sq(const T* a, const T* b, double shift, uint64_t n, double* ws, double* out, hipStream_t s);
uint64_t sum_sq_ws_bytes();
// the float32-cast compressor: comps holds n components of N values each;
// linf: n zeroed bit patterns of the measured errors (raised with atomics)
template <class T>
hipError_t launch_cast_encode(const T* x, uint64_t N, int n, float* comps, unsigned long long* linf, hipStream_t s);
template <class T> hipError_t launch_cast_decode(const float* comps, uint64_t N, int k, T* out, hipStream_t s);

// capacity of one chunk's staging slot in 32-bit words
inline uint64_t chunk_cap_words_host(int dtype) {
  const uint64_t raw = dtype == 1 ? 2 + 64 * 32 : 2 + 64 * 64;
  return (16 * raw + 31) / 32;
}

}  // namespace pmc
