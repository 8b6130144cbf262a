// Sanitizer driver for the library's host-side parser of store blobs and
// stream headers (paper_2308_11759_amd/csrc/format.cpp), test infrastructure,
// CPU only.  Built with that file alone under -fsanitize=address,undefined by
// tests/test_sanitizers.py.  For each blob file given (a valid store written
// around oracle streams) it checks that the blob is accepted, then calls
// pmc_store_device_bytes on many mutated copies: flipped bits, truncations,
// size and count fields set to extreme values (sums that would wrap 64 bits),
// and copies at an odd address.  Each copy is allocated at its exact length,
// so any read past it is reported.  Exit status 0 means no check failed and
// no sanitizer fired.
//
// usage: blob_fuzz SEED MUTATIONS BLOB...
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <vector>

#include "pmc.h"

static uint64_t rs;
static uint64_t rnd() {  // xorshift64* (Vigna)
  rs ^= rs >> 12;
  rs ^= rs << 25;
  rs ^= rs >> 27;
  return rs * 0x2545F4914F6CDD1Dull;
}

static int failures = 0;
static void check(bool c, const char* what) {
  if (!c) {
    std::fprintf(stderr, "%s\n", what);
    ++failures;
  }
}

// the blob copied into an allocation that ends at its last byte (at an odd
// address when `odd`), so that any read past it is reported
static pmc_status probe(const std::vector<uint8_t>& b, size_t len, bool odd, size_t* need) {
  const size_t shift = odd ? 1 : 0;
  uint8_t* raw = (uint8_t*)std::malloc(len + shift ? len + shift : 1);
  uint8_t* p = raw + shift;
  if (len) std::memcpy(p, b.data(), len);
  const pmc_status st = pmc_store_device_bytes(p, len, need);
  std::free(raw);
  return st;
}

static void put64(std::vector<uint8_t>& b, size_t off, uint64_t v) {
  if (off + 8 <= b.size()) std::memcpy(b.data() + off, &v, 8);
}

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  rs = std::strtoull(argv[1], nullptr, 10) * 0x9E3779B97F4A7C15ull + 1;
  const int mutations = std::atoi(argv[2]);
  const uint64_t extremes[] = {0, 1, 255, 256, 0xFFFFFFFFull, 0x100000000ull, 1ull << 62, 1ull << 63,
                               ~0ull - 255, ~0ull - 63, ~0ull};
  uint64_t accepted = 0, rejected = 0;
  for (int a = 3; a < argc; ++a) {
    std::ifstream in(argv[a], std::ios::binary);
    std::vector<uint8_t> blob((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    size_t need = 0;
    check(probe(blob, blob.size(), false, &need) == PMC_OK, "a valid blob was refused");
    check(probe(blob, blob.size(), true, &need) == PMC_OK, "a valid blob at an odd address was refused");
    uint32_t n = 0;
    std::memcpy(&n, blob.data() + 8, 4);
    const size_t head = (48 + 64 * (size_t)n + 255) / 256 * 256;
    // where the streams start: the component records give their sizes
    std::vector<size_t> starts;
    size_t off = 0;
    for (uint32_t i = 0; i < n; ++i) {
      uint64_t bytes;
      std::memcpy(&bytes, blob.data() + 48 + 64 * i + 16, 8);
      off = (off + 255) / 256 * 256;
      starts.push_back(head + off);
      off += bytes;
    }
    const size_t used = head + off;  // the last stream's end
    for (int m = 0; m < mutations; ++m) {
      std::vector<uint8_t> c = blob;
      size_t len = c.size();
      bool cut = false;
      switch (rnd() % 5) {
        case 0: {  // flips anywhere in the headers, records and stream headers
          const int k = 1 + (int)(rnd() % 4);
          for (int j = 0; j < k; ++j) {
            size_t b;
            if (rnd() % 2) b = rnd() % std::min<size_t>(head, c.size());
            else b = starts[rnd() % n] + rnd() % 128;
            if (b < c.size()) c[b] ^= (uint8_t)(1u << (rnd() % 8));
          }
          break;
        }
        case 1:  // truncated inside the streams
          len = used ? (size_t)(rnd() % used) : 0;
          cut = true;
          break;
        case 2: {  // a record's byte count set to an extreme value
          const uint32_t i = (uint32_t)(rnd() % n);
          put64(c, 48 + 64 * i + 16, extremes[rnd() % (sizeof(extremes) / 8)]);
          break;
        }
        case 3: {  // a stream's chunk count or payload word count extreme
          const size_t s = starts[rnd() % n];
          put64(c, s + (rnd() % 2 ? 48 : 56), extremes[rnd() % (sizeof(extremes) / 8)]);
          break;
        }
        default: {  // a stream's chunk index entry changed
          const size_t s = starts[rnd() % n];
          uint64_t nch = 0;
          std::memcpy(&nch, c.data() + s + 48, 8);
          const size_t at = s + 64 + 4 * (size_t)(rnd() % (nch ? nch : 1));
          const uint32_t v = (uint32_t)extremes[rnd() % (sizeof(extremes) / 8)];
          if (at + 4 <= c.size()) std::memcpy(c.data() + at, &v, 4);
          break;
        }
      }
      const pmc_status st = probe(c, len, rnd() % 2, &need);
      check(st == PMC_OK || st == PMC_E_CORRUPT, "unexpected status");
      if (cut) check(st == PMC_E_CORRUPT, "a blob cut inside its streams was accepted");
      (st == PMC_OK ? accepted : rejected)++;
    }
  }
  std::printf("blob_fuzz: %llu accepted, %llu rejected, %d failures\n", (unsigned long long)accepted,
              (unsigned long long)rejected, failures);
  return failures ? 1 : 0;
}
