// format.hpp -- the block grid of a field and the layouts of a component
// stream and of a serialised store, with their host-side validation.  Plain
// C++ with no HIP dependency, so that the parsers of untrusted bytes can also
// be built and exercised on their own (address and undefined-behaviour
// sanitizers in the CPU tests).  Internal to the library.
#pragma once
#include <stdint.h>

#include <vector>

#include "../../include/pmc.h"

namespace pmc {

constexpr int kMaxComps = 32;  // components per store
constexpr uint64_t kStreamHeader = 64;
constexpr uint32_t kStreamMagic = 0x31434D50u;  // "PMC1"
constexpr uint32_t kStreamVersion = 1;

// block grid of a field: 4x4x4 blocks, x fastest; chunks of 16 blocks
// (the block decomposition of Sec. 6.1 applied to a 3-D field)
struct Geo {
  uint64_t nx, ny, nz;
  uint64_t nbx, nby, nbz;
  uint64_t nblocks, nchunks;
  int rows_aligned;  // nx % 4 == 0: block rows can use 16-byte vector access
  int pad;
};

}  // namespace pmc

namespace pmc_host {

// the grid of a field; false for a bad dtype, an empty axis, or a field
// beyond 2^36 values / 2^32 blocks
bool make_geo(const pmc_field* f, pmc::Geo* g);
uint64_t align256(uint64_t v);
// floor(log2(tau)) of a positive finite double, from its bits
int floor_log2(double tau);
// the device buffer of a store holds, first, one per-block index (bit offset
// of each block inside its chunk, 4 bytes per block) per component, then the
// streams, each on a 256-byte boundary
uint64_t aux_bytes(const pmc::Geo& g);

// store blob: u32 "PMCS", u32 version, u32 n, u32 codec | u64 nx ny nz,
//             i32 dtype, i32 0 |
//             n x {f64 tau, f64 linf, u64 bytes, nempty, ncoded, nraw, nesc, nmiss} |
//             (256-aligned) streams, each on a 256-byte boundary of the region
constexpr uint32_t kBlobMagic = 0x53434D50u;
uint64_t blob_header_bytes(int n);

struct BlobView {
  int n;
  int codec;
  pmc_field f;
  std::vector<uint64_t> rec;  // 8 words per component
  uint64_t region_off, region_bytes;
};

// the blob's header and component records; every size is checked against
// the blob's length without forming a sum that could wrap
bool parse_blob(const void* host_buf, size_t size, BlobView* v);
// one stream's header fields and chunk index (its payload is checked on the
// device, block by block, when the per-block index is rebuilt)
bool check_stream(const uint8_t* p, uint64_t bytes, const pmc_field* f, const pmc::Geo& g, double tau, int codec,
                  uint64_t* words, uint64_t* max_span);
// every stream of a parsed blob: strictly decreasing positive tolerances and
// a valid header and chunk index; words / spans per component on success
bool check_blob_streams(const BlobView& v, const pmc::Geo& g, const uint8_t* region, std::vector<uint64_t>* words,
                        std::vector<uint64_t>* spans);
// device bytes of a store rebuilt from a blob: the block indexes, the
// streams, and a trailer (a status word and one 64-bit flag per component)
// at the end
constexpr uint64_t kBlobTrailerBytes = 512;
uint64_t blob_device_bytes(const BlobView& v, const pmc::Geo& g);

}  // namespace pmc_host
