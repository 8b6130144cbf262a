// codec_device.hpp -- device-side pieces of the zfp-style fixed-accuracy block
// codec for CDNA4 (gfx950).  One lane owns one 4x4x4 block: the 64 values, the
// quantised integers and the negabinary coefficients all live in registers
// (fully unrolled loops with compile-time indices), so the coefficient
// reordering is free register renaming.  Bit planes are produced 16 at a time
// by an in-register 32x32 bit-matrix transpose instead of 64 bit extractions
// per plane.
//
// The codec realises, for d = 3, the compressor the paper plugs into its
// multi-component loop (Sec. 4, Alg. 1 and Alg. 2): one common exponent per
// block and component (Sec. 4.4), a decorrelating block transform with bit-plane
// coding (Sec. 5, compressor list), group tests over bit planes (Sec. 2), and
// blocks of 4^d values that decode independently (Sec. 6.1).  Format version 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pmc {

constexpr int kVals = 64;         // values per block
constexpr int kChunkBlocks = 16;  // blocks per chunk (unit of the stream index)
constexpr int kGuard = 8;         // guard planes 2(d+1) for d = 3
constexpr int kHeaderBytes = 64;  // stream header
constexpr uint32_t kMagic = 0x31434D50u;
constexpr int kVersion = 1;
constexpr int kMaxComponents = 32;

template <class T> struct FT;
template <> struct FT<float> {
  typedef uint32_t U;  // P-bit unsigned word
  typedef int32_t S;   // P-bit signed word
  static constexpr int P = 32, EBITS = 8, BIAS = 127, MANT = 23, CODE = 1;
  static constexpr uint32_t NB = 0xAAAAAAAAu;
  static constexpr int RAW_BITS = 2 + kVals * 32;
};
template <> struct FT<double> {
  typedef uint64_t U;
  typedef int64_t S;
  static constexpr int P = 64, EBITS = 11, BIAS = 1023, MANT = 52, CODE = 2;
  static constexpr uint64_t NB = 0xAAAAAAAAAAAAAAAAull;
  static constexpr int RAW_BITS = 2 + kVals * 64;
};

// capacity of one chunk in 32-bit words: 16 raw blocks (coded blocks are never
// larger than raw ones, the acceptance rule falls back to raw first)
template <class T> constexpr int chunk_cap_words() {
  return (kChunkBlocks * FT<T>::RAW_BITS + 31) / 32;
}

// ---------------------------------------------------------------------------
// coefficient order: total sequency lx+ly+lz ascending, ties by local index.
// Generated at compile time level by level.
struct Order {
  int8_t at[64];
};
constexpr Order make_order() {
  Order o{};
  int r = 0;
  for (int level = 0; level <= 9; ++level)
    for (int l = 0; l < 64; ++l)
      if ((l & 3) + ((l >> 2) & 3) + ((l >> 4) & 3) == level) o.at[r++] = (int8_t)l;
  return o;
}
constexpr Order kOrder = make_order();
// its inverse: the coded position of block index l
constexpr Order make_inv_order() {
  Order o{};
  for (int r = 0; r < 64; ++r) o.at[kOrder.at[r]] = (int8_t)r;
  return o;
}
constexpr Order kInvOrder = make_inv_order();

// a copy the compiler cannot prove equal to the original: recomputing the
// residual from such copies stops common-subexpression elimination from
// keeping a 64-value array alive across the whole kernel, and a value used
// inside a loop through such a copy is not hoisted out of it
template <class T> __device__ __forceinline__ T opaque(T v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}
template <class T> __device__ __forceinline__ T* opaque(T* p) {
  __asm__ volatile("" : "+v"(p));
  return p;
}

// ---------------------------------------------------------------------------
// wrapping integer helpers (two's complement P-bit words)
template <class S> __device__ __forceinline__ S wadd(S a, S b) {
  typedef typename std::make_unsigned<S>::type W;
  return (S)((W)a + (W)b);
}
template <class S> __device__ __forceinline__ S wsub(S a, S b) {
  typedef typename std::make_unsigned<S>::type W;
  return (S)((W)a - (W)b);
}
template <class S> __device__ __forceinline__ S wdbl(S a) {
  typedef typename std::make_unsigned<S>::type W;
  return (S)((W)a << 1);
}
template <class S> __device__ __forceinline__ S half(S a) { return a >> 1; }  // floor(a/2)
// the same on two 16-bit values per 32-bit register (packed 16-bit
// operations), for the float32 decoder's high-half route
typedef short v2s __attribute__((ext_vector_type(2)));
typedef unsigned short v2u __attribute__((ext_vector_type(2)));
__device__ __forceinline__ v2s wadd(v2s a, v2s b) { return (v2s)((v2u)a + (v2u)b); }
__device__ __forceinline__ v2s wsub(v2s a, v2s b) { return (v2s)((v2u)a - (v2u)b); }
__device__ __forceinline__ v2s wdbl(v2s a) { return (v2s)((v2u)a << (v2u)1); }
__device__ __forceinline__ v2s half(v2s a) { return a >> (v2s)1; }

// 4-point lifting realisation of the basis (1/16)[[4,4,4,4],[5,1,-1,-5],
// [-4,4,4,-4],[-2,6,-6,2]]: the sums of the outer and inner pairs give the
// DC and second-order terms; the two half-differences are mixed by one
// halving step and two lifting steps into the first- and third-order terms.
template <class S> __device__ __forceinline__ void lift_fwd(S& a, S& b, S& c, S& d) {
  S s0 = half(wadd(a, d)), t0 = wsub(a, s0);
  S s1 = half(wadd(b, c)), t1 = wsub(b, s1);
  S dc = half(wadd(s0, s1)), q2 = wsub(s1, dc);
  S w = half(wadd(t0, t1));
  S q3 = wsub(t1, half(w));
  S q1 = wsub(w, half(q3));
  a = dc; b = q1; c = q2; d = q3;
}
template <class S> __device__ __forceinline__ void lift_inv(S& a, S& b, S& c, S& d) {
  S dc = a, q1 = b, q2 = c, q3 = d;
  S w = wadd(q1, half(q3));
  S t1 = wadd(q3, half(w));
  S t0 = wsub(wdbl(w), t1);
  S s1 = wadd(q2, dc);
  S s0 = wsub(dc, q2);
  a = wadd(t0, s0);
  d = wsub(s0, t0);
  b = wadd(t1, s1);
  c = wsub(s1, t1);
}

// separable forward transform on local index l = lx + 4 ly + 16 lz
template <class S> __device__ __forceinline__ void xform_fwd(S q[64]) {
#pragma unroll
  for (int l = 0; l < 16; ++l) {  // x lines: base 4*l
    const int b = 4 * l;
    lift_fwd(q[b], q[b + 1], q[b + 2], q[b + 3]);
  }
#pragma unroll
  for (int l = 0; l < 16; ++l) {  // y lines: base 16*z + x
    const int b = 16 * (l >> 2) + (l & 3);
    lift_fwd(q[b], q[b + 4], q[b + 8], q[b + 12]);
  }
#pragma unroll
  for (int l = 0; l < 16; ++l) {  // z lines: base 4*y + x
    const int b = l;
    lift_fwd(q[b], q[b + 16], q[b + 32], q[b + 48]);
  }
}

// ---------------------------------------------------------------------------
// 32x32 bit-matrix transpose in registers: afterwards A[r] bit c equals the
// old A[c] bit r.  Recursive block swap with strides 16, 8, 4, 2, 1.
// one butterfly stage: for each pair (a, b) = (A[k], A[k+J]) with bit J of k
// clear, b takes the M-bits of a >> J and a the (M << J)-bits of b << J.
// The 16- and 8-bit stages move whole bytes (one v_perm each); the others
// exchange the masked bits through one xor-difference.
template <int J, uint32_t M> __device__ __forceinline__ void tstage(uint32_t A[32]) {
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    if (k & J) continue;
    const uint32_t a = A[k], b = A[k + J];
    if constexpr (J == 16) {
      A[k] = __builtin_amdgcn_perm(b, a, 0x05040100u);      // a.lo16 | b.lo16 << 16
      A[k + J] = __builtin_amdgcn_perm(b, a, 0x07060302u);  // a.hi16 | b.hi16 << 16
    } else if constexpr (J == 8) {
      A[k] = __builtin_amdgcn_perm(b, a, 0x06020400u);      // a0 b0 a2 b2
      A[k + J] = __builtin_amdgcn_perm(b, a, 0x07030501u);  // a1 b1 a3 b3
    } else {
      const uint32_t t = ((a >> J) ^ b) & M;
      A[k + J] = b ^ t;
      A[k] = a ^ (t << J);
    }
  }
}
__device__ __forceinline__ void transpose32(uint32_t A[32]) {
  tstage<16, 0x0000FFFFu>(A);
  tstage<8, 0x00FF00FFu>(A);
  tstage<4, 0x0F0F0F0Fu>(A);
  tstage<2, 0x33333333u>(A);
  tstage<1, 0x55555555u>(A);
}

// 16 bits [base, base+16) of coefficients j and j+32 packed as one word
__device__ __forceinline__ uint32_t slice16(uint32_t v, int base) { return (v >> base) & 0xFFFFu; }
__device__ __forceinline__ uint32_t slice16(uint64_t v, int base) {
  return (uint32_t)(v >> base) & 0xFFFFu;
}

// planes [base, base+16) of the 64 coefficients as 32 words T:
//   plane base+r has coefficients 0..31 in T[r] and 32..63 in T[16+r]
template <class U> __device__ __forceinline__ void plane_group(const U u[64], int base, uint32_t T[32]) {
#pragma unroll
  for (int j = 0; j < 32; ++j) T[j] = slice16(u[j], base) | (slice16(u[j + 32], base) << 16);
  transpose32(T);
}

// bits one plane costs with the group-testing coder, given the significant
// prefix n (updated); closed form of the coder's emissions
__device__ __forceinline__ uint32_t plane_cost(uint64_t wd, uint32_t& n) {
  uint32_t c = n;
  if (n < 64) {
    uint64_t rest = wd >> n;
    if (rest == 0) {
      c += 1;
    } else {
      uint32_t m = (uint32_t)__popcll(rest);
      uint32_t h = 63u - (uint32_t)__clzll(rest) + n;
      c += m + (h - n + 1) + (h < 63 ? 1u : 0u) - (h == 63 ? 1u : 0u);
      n = h + 1;
    }
  }
  return c;
}

// ---------------------------------------------------------------------------
// LDS bit writer: bits LSB-first at an arbitrary start bit of a zeroed word
// buffer; words shared with neighbouring lanes are merged with ds_or.  Only
// words inside the window [w0, w0 + nw) are stored (buf points at word w0),
// so a chunk larger than the LDS window is emitted in several passes.
struct LdsBits {
  uint32_t* buf;
  uint32_t word;  // absolute word index of the word being filled
  uint32_t nacc;
  uint32_t w0, nw;
  uint64_t acc;
  __device__ __forceinline__ void init(uint32_t* b, uint32_t bitpos, uint32_t win0, uint32_t nwin) {
    buf = b;
    word = bitpos >> 5;
    nacc = bitpos & 31u;
    acc = 0;
    w0 = win0;
    nw = nwin;
  }
  __device__ __forceinline__ void emit_word(uint32_t v) {
    const uint32_t k = word - w0;  // wraps to a large value below the window
    if (k < nw && v != 0u) atomicOr(&buf[k], v);
  }
  // count <= 32, value holds only its low `count` bits
  __device__ __forceinline__ void put(uint64_t value, uint32_t count) {
    acc |= value << nacc;
    nacc += count;
    if (nacc >= 32) {
      emit_word((uint32_t)acc);
      ++word;
      acc >>= 32;
      nacc -= 32;
    }
  }
  // count <= 64
  __device__ __forceinline__ void put64(uint64_t value, uint32_t count) {
    if (count > 32) {
      put(value & 0xFFFFFFFFull, 32);
      put(value >> 32, count - 32);
    } else {
      put(value, count);
    }
  }
  __device__ __forceinline__ void flush() {
    if (nacc > 0) emit_word((uint32_t)acc);
  }
};

// unsqueeze, the inverse of squeeze: every set bit of m, at position k and
// i-th from the bottom (i >= 1), moves to k + i (128-bit result lo | hi<<64).
// Applied to the newly significant coefficients of a plane this gives the
// positions of the run terminators in its group-test section.  The table
// holds each byte's own unsqueeze (16 bits); the bytes are joined with
// shifts given by the number of set bits below them.
__device__ __forceinline__ uint32_t unsqueeze_byte(uint32_t b) {
  uint32_t r = 0, i = 0;
  for (uint32_t k = 0; k < 8; ++k)
    if ((b >> k) & 1u) r |= 1u << (k + ++i);
  return r;
}
__device__ __forceinline__ void unsqueeze_table(uint16_t* tab) {
  for (uint32_t b = threadIdx.x; b < 256; b += blockDim.x) tab[b] = (uint16_t)unsqueeze_byte(b);
  __syncthreads();
}
__device__ __forceinline__ void unsqueeze64(uint64_t m, const uint16_t* tab, uint64_t& lo, uint64_t& hi) {
  lo = 0;
  hi = 0;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t b = (uint32_t)(m >> (8 * k)) & 0xFFu;
    const uint64_t v = tab[b];
    const uint32_t sh = 8u * (uint32_t)k + c;  // < 120
    lo |= sh < 64u ? v << sh : 0ull;
    hi |= sh >= 64u ? v << (sh - 64u) : (sh > 48u ? v >> (64u - sh) : 0ull);
    c += (uint32_t)__builtin_popcount(b);
  }
}

// emit one plane with the group-testing coder, n = significant prefix: the
// n verbatim bits, then the whole group-test section at once.  In the section
// the i-th newly significant coefficient, at k past the prefix, puts its
// terminator at bit k + i (unsqueeze); every terminator but the last is
// followed by a positive test, bit 0 is the first test, and a negative test
// ends the section.  When the last significant coefficient is coefficient 63
// its terminator is implied and the section ends just before it.
__device__ __forceinline__ void plane_emit(LdsBits& w, uint64_t wd, uint32_t& n, const uint16_t* tab) {
  if (n > 0) w.put64(n == 64 ? wd : (wd & ((1ull << n) - 1ull)), n);
  if (n >= 64) return;
  const uint64_t rest = wd >> n;
  if (rest == 0) {  // a single negative test
    w.put(0, 1);
    return;
  }
  const uint32_t top = 63u - (uint32_t)__builtin_clzll(rest);  // last new coefficient, past the prefix
  const uint32_t lastt = top + (uint32_t)__builtin_popcountll(rest);  // its terminator's bit
  uint64_t tlo, thi;
  unsqueeze64(rest, tab, tlo, thi);
  // positive tests: bit 0 and the bit after every terminator but the last
  uint64_t slo = tlo | (tlo << 1) | 1ull, shi = thi | (thi << 1) | (tlo >> 63);
  const bool implied = n + top == 63u;
  // no positive test follows the last terminator (a negative test does,
  // unless the terminator is implied: then it is dropped as well)
  const uint32_t a = lastt + 1u;
  if (a < 64u) slo &= ~(1ull << a);
  else shi &= ~(1ull << (a - 64u));
  if (implied) {
    if (lastt < 64u) slo &= ~(1ull << lastt);
    else shi &= ~(1ull << (lastt - 64u));
  }
  const uint32_t len = implied ? lastt : lastt + 2u;
  w.put64(slo, len < 64u ? len : 64u);
  if (len > 64u) w.put64(shi, len - 64u);
  n += top + 1u;
}

// ---------------------------------------------------------------------------
// global-memory bit reader over the words [first, end) of a payload.  Word
// indices are 32-bit (the stream index limits a payload to 2^32 words) and the
// payload base is usually wave-uniform, which keeps the reader in few vector
// registers.  The word after the buffered ones is loaded one refill ahead
// (from the last word of the range once the range is exhausted, so every load
// stays inside it and its latency overlaps the decoding of the bits already
// buffered).  Bits past `end` are therefore unspecified; bad() reports any
// use of them.  A reader is refilled only when first < end.
struct GBits {
  const uint32_t* base;
  uint32_t p;  // index of the next word to load
  uint32_t end;
  uint64_t buf;
  uint32_t nbuf;
  uint32_t nxt;  // word p - 1, loaded ahead
  __device__ __forceinline__ void init(const uint32_t* b, uint32_t first, uint32_t e) {
    base = b;
    end = e;
    buf = 0;
    nbuf = 0;
    nxt = first < e ? b[first] : 0u;
    p = first + 1;
  }
  // afterwards at least 32 bits are buffered
  __device__ __forceinline__ void refill() {
    if (nbuf <= 32) {
      buf |= (uint64_t)nxt << nbuf;
      nbuf += 32;
      nxt = base[p < end ? p : end - 1];
      ++p;
    }
  }
  __device__ __forceinline__ void drop(uint32_t count) {  // count <= buffered bits
    buf >>= count;
    nbuf -= count;
  }
  __device__ __forceinline__ uint32_t get(uint32_t count) {  // count <= 32
    refill();
    uint32_t lo = (uint32_t)buf;
    uint32_t v = count >= 32 ? lo : (lo & ((1u << count) - 1u));
    drop(count);
    return v;
  }
  __device__ __forceinline__ uint64_t get64(uint32_t count) {  // count <= 64
    if (count > 32) {
      uint64_t lo = get(32);
      return lo | ((uint64_t)get(count - 32) << 32);
    }
    return get(count);
  }
  __device__ __forceinline__ uint64_t get64nz(uint32_t count) { return get64(count); }  // 1 <= count <= 64
  __device__ __forceinline__ void skip(uint32_t count) {  // count <= 32
    refill();
    drop(count);
  }
  __device__ __forceinline__ uint32_t peek32() {  // the next 32 bits
    refill();
    return (uint32_t)buf;
  }
  // bits consumed since word `from`: words moved into the buffer minus those held
  __device__ __forceinline__ uint64_t consumed(uint32_t from) const {
    return (uint64_t)(p - 1 - from) * 32 - nbuf;
  }
  // bits consumed past `end` (zero words fetched beyond it and not used are fine)
  __device__ __forceinline__ bool bad() const {
    return (int64_t)((int64_t)p - 1 - (int64_t)end) * 32 > (int64_t)nbuf;
  }
};

// LDS bit reader over words staged in LDS (a wave's chunks): three words and
// a bit offset; peeks are funnel shifts and every skip reloads the three
// words at the new position, so there is no refill branch.  Words
// [0, capw + 3) exist (the data fill at most capw); bits past `end` are
// unspecified and bad() reports any use of them.
struct LBits {
  const uint32_t* s;
  uint32_t p, o, end;  // word of the next bit, its bit offset, end word
  uint32_t capw;       // reads are clamped to words [0, capw + 3)
  uint32_t w0, w1, w2;
  __device__ __forceinline__ void load() {
    const uint32_t q = p < capw ? p : capw;  // only a malformed stream runs past the data
    w0 = s[q];
    w1 = s[q + 1];
    w2 = s[q + 2];
  }
  __device__ __forceinline__ void init(const uint32_t* st, uint32_t first, uint32_t e, uint32_t cap) {
    s = st;
    p = first;
    o = 0;
    end = e;
    capw = cap;
    load();
  }
  __device__ __forceinline__ uint32_t peek32() const { return __builtin_amdgcn_alignbit(w1, w0, o); }
  __device__ __forceinline__ uint64_t peek64() const {
    return (uint64_t)__builtin_amdgcn_alignbit(w1, w0, o) | ((uint64_t)__builtin_amdgcn_alignbit(w2, w1, o) << 32);
  }
  __device__ __forceinline__ void skip(uint32_t count) {  // count <= 64
    const uint32_t t = o + count;
    p += t >> 5;
    o = t & 31u;
    load();
  }
  __device__ __forceinline__ uint32_t get(uint32_t count) {  // count <= 32
    const uint32_t v = peek32();
    skip(count);
    return count >= 32 ? v : v & ((1u << count) - 1u);
  }
  __device__ __forceinline__ uint64_t get64(uint32_t count) {  // count <= 64
    const uint64_t v = peek64();
    skip(count);
    return count >= 64 ? v : v & ((1ull << count) - 1ull);
  }
  __device__ __forceinline__ uint64_t get64nz(uint32_t count) {  // 1 <= count <= 64: a shift pair masks
    const uint64_t v = peek64();
    skip(count);
    return (v << (64u - count)) >> (64u - count);
  }
  __device__ __forceinline__ uint64_t consumed(uint32_t from) const { return (uint64_t)(p - from) * 32 + o; }
  __device__ __forceinline__ bool bad() const { return (uint64_t)p * 32 + o > (uint64_t)end * 32; }
};

// The run terminators of a group-test section that starts with a positive
// test at bit 0: the ones with an even number of ones at or below them.
// Inside a section a test is always followed by its
// run and terminator, and a terminator by the next test, so apart from bit 0
// every maximal run of ones starts with a terminator and alternates
// terminator, test, ...: the terminators are the bits at even offsets from
// their run's first bit.  Runs that start at an even position are found by
// adding their first bits (the carry clears the run); the rest start at odd
// positions.  Past the section's end (garbage bits of what follows) the two
// forms may differ; the plane reader never takes a terminator from there.
__device__ __forceinline__ uint32_t terminators(uint32_t s) {
  const uint32_t x = s & ~1u;
  const uint32_t first = x & ~(x << 1);                        // first bit of each run
  const uint32_t even = ((x + (first & 0x55555555u)) ^ x) & x;  // runs starting at even positions
  return x & (even ^ 0xAAAAAAAAu);                             // even offsets within each run
}

// squeeze: every set bit of m, at position t and i-th from the bottom
// (i >= 1), moves to t - i.  Applied to the run terminators of a group-test
// section (which are at least two bits apart and never at bit 0) this drops
// the positive tests and leaves the plane bits.  The table holds, for each
// byte, its own squeeze shifted up by one (a byte's lowest set bit may sit at
// its bit 0); the bytes are joined with shifts given by the number of set
// bits below them.
__device__ __forceinline__ uint32_t squeeze_byte(uint32_t b) {
  uint32_t r = 0, i = 0;
  for (uint32_t t = 0; t < 8; ++t)
    if ((b >> t) & 1u) r |= 1u << (t + 1 - ++i);
  return r;
}
// fill the 256-entry table at tab (LDS) with all threads of the block
__device__ __forceinline__ void squeeze_table(uint8_t* tab) {
  for (uint32_t b = threadIdx.x; b < 256; b += blockDim.x) tab[b] = (uint8_t)squeeze_byte(b);
  __syncthreads();
}
__device__ __forceinline__ uint32_t squeeze32(uint32_t m, const uint8_t* tab) {
  const uint32_t b0 = m & 0xFFu, b1 = (m >> 8) & 0xFFu, b2 = (m >> 16) & 0xFFu, b3 = m >> 24;
  const uint32_t c1 = (uint32_t)__builtin_popcount(b0);
  const uint32_t c2 = c1 + (uint32_t)__builtin_popcount(b1);
  const uint32_t c3 = c2 + (uint32_t)__builtin_popcount(b2);
  return ((uint32_t)tab[b0] >> 1) | ((uint32_t)tab[b1] << (7 - c1)) | ((uint32_t)tab[b2] << (15 - c2)) |
         ((uint32_t)tab[b3] << (23 - c3));
}

// read one plane: n verbatim bits, then the group tests, 32 bits at a time.
// In the section "1 0^r1 1  1 0^r2 1 ... 0" the ones alternate between
// positive tests and run terminators, so within a window that starts at a
// test the terminators are the ones with an even inclusive prefix count; the
// i-th terminator at bit t marks coefficient n + t - i (squeeze32).  The
// section ends at the first terminator followed by a 0 (a negative test), or
// where a run reaches the last coefficient, whose one is implied (no
// terminator, no test after it).  A window that ends inside a run lets the
// next window start inside it: a virtual positive test (vg = 1) is put in
// front.  Each window is decoded without branches; the loop runs once per
// window.
template <class R>
__device__ __forceinline__ uint64_t plane_read(R& r, uint32_t& n, const uint8_t* sq) {
  uint64_t wd = 0;
  if (n > 0) wd = r.get64nz(n);  // the n verbatim bits
  uint32_t vg = 0;
  while (n < 64) {
    const uint32_t s = (r.peek32() << vg) | vg;
    const bool neg = (s & 1u) == 0u;  // negative first test: the plane ends here
    const uint32_t term = terminators(s);
    const uint32_t ends = term & ~(s >> 1) & 0x7FFFFFFFu;
    const uint32_t last = (uint32_t)__builtin_ctz(ends | 0x80000000u);
    const uint32_t tm = neg ? 0u : term & ((2u << last) - 1u);
    // terminators whose coefficient stays below 63; one beyond marks a run
    // that reaches coefficient 63 instead
    const uint32_t rel = squeeze32(tm, sq);
    // coefficients n..62 may carry a terminator; rel < 2^31 (a squeezed bit
    // moves down at least one place), so 31 low bits cover room >= 31
    const uint32_t room = 63u - n;
    const uint32_t vrel = __builtin_amdgcn_ubfe(rel, 0u, room < 31u ? room : 31u);
    const bool tokens = vrel == rel && tm != 0u;
    // bit length of vrel (0 for 0): vrel < 2^31, so (vrel << 1) | 1 is nonzero
    const uint32_t nn = 31u - (uint32_t)__builtin_clz((vrel << 1) | 1u);
    const uint32_t g = nn + (uint32_t)__builtin_popcount(vrel);  // the bit after the last one taken
    wd |= (uint64_t)vrel << n;
    n += nn;
    // otherwise a positive test at bit g starts a run from coefficient n:
    // it reaches coefficient 63 inside the window (implied one), or runs on
    const uint32_t z = 63u - n;
    const bool run = !neg && !tokens;
    const bool implied = run && z <= 31u - g;
    const bool done = neg || implied || (tokens && ends != 0u);
    const uint32_t c_tok = g + (ends != 0u ? 1u : 0u);
    const uint32_t c_run = implied ? g + 1u + z : 32u;
    const uint32_t c_any = tokens ? c_tok : c_run;
    const uint32_t c = neg ? 1u : c_any;
    r.skip(c - vg);
    wd |= implied ? (1ull << 63) : 0ull;
    n = implied ? 64u : run ? n + 31u - g : n;
    vg = run ? 1u : 0u;
    if (done) break;
  }
  return wd;
}

// ---------------------------------------------------------------------------
// block-floating-point quantisation and its inverse
__device__ __forceinline__ int32_t quantize(float e, int emax) {
  return (int32_t)__builtin_ldexpf(e, 30 - emax);  // exact scaling, truncation
}
__device__ __forceinline__ int64_t quantize(double e, int emax) {
  return (int64_t)__builtin_ldexp(e, 62 - emax);
}
// q * 2^(emax-30) with one rounding: exact in double, then the cast rounds
__device__ __forceinline__ float dequantize(int32_t q, int emax) {
  return (float)__builtin_ldexp((double)q, emax - 30);
}
// q * 2^(emax-62) with one rounding to double.  The int64 -> double
// conversion rounds once and the scaling is exact while the result is normal;
// when it would be subnormal the rounding is done on the integer instead.
__device__ __forceinline__ double dequantize(int64_t q, int emax) {
  if (q == 0) return 0.0;
  uint64_t a = q < 0 ? (uint64_t)0 - (uint64_t)q : (uint64_t)q;
  int lead = 63 - __clzll(a);  // leading bit position
  int s = emax - 62;
  if (lead + s >= -1022) return __builtin_ldexp((double)q, s);
  // subnormal: units of 2^-1074, shift right by r with round-half-even
  int r = -(s + 1074);
  uint64_t m;
  if (r <= 0) {
    m = a << (-r);
  } else if (r >= 64) {
    m = 0;  // a < 2^63 so a * 2^-64 < 1/2
  } else {
    m = a >> r;
    uint64_t rem = a & ((1ull << r) - 1ull);
    uint64_t halfw = 1ull << (r - 1);
    if (rem > halfw || (rem == halfw && (m & 1ull))) ++m;
  }
  uint64_t bits = m | (q < 0 ? 0x8000000000000000ull : 0ull);
  return __longlong_as_double((long long)bits);
}

__device__ __forceinline__ uint32_t abs_bits(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }
__device__ __forceinline__ uint64_t abs_bits(double v) {
  return (uint64_t)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
}
__device__ __forceinline__ uint32_t raw_bits_lo(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint64_t raw_bits_lo(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ float from_raw(uint32_t b, float) { return __uint_as_float(b); }
__device__ __forceinline__ double from_raw(uint64_t b, double) {
  return __longlong_as_double((long long)b);
}

// max biased exponent -> emax (frexp convention, zero/subnormal -> 2-bias)
template <class T> __device__ __forceinline__ int block_emax(typename FT<T>::U maxabs) {
  int biased = (int)(maxabs >> FT<T>::MANT);
  if (biased < 1) biased = 1;
  return biased - FT<T>::BIAS + 1;
}

template <class T> __device__ __forceinline__ typename FT<T>::U to_nb(typename FT<T>::S q) {
  typedef typename FT<T>::U U;
  return ((U)q + FT<T>::NB) ^ FT<T>::NB;
}
template <class T> __device__ __forceinline__ typename FT<T>::S from_nb(typename FT<T>::U u) {
  typedef typename FT<T>::S S;
  return (S)((u ^ FT<T>::NB) - FT<T>::NB);
}

// residual block -> negabinary coefficients in coded order (u[r])
template <class T>
__device__ __forceinline__ void forward_coeffs(const T e[64], int emax, typename FT<T>::U u[64]) {
  typedef typename FT<T>::S S;
  S q[64];
#pragma unroll
  for (int l = 0; l < 64; ++l) q[l] = (S)quantize(e[l], emax);
  xform_fwd(q);
#pragma unroll
  for (int r = 0; r < 64; ++r) u[r] = to_nb<T>(q[kOrder.at[r]]);
}

// the inverse transform: coded-order integers c (already out of negabinary)
// -> block order, then the z and y passes ...
template <class T>
__device__ __forceinline__ void inverse_zy_ints(const typename FT<T>::S c[64], typename FT<T>::S q[64]) {
#pragma unroll
  for (int r = 0; r < 64; ++r) q[kOrder.at[r]] = c[r];
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    const int b = l;
    lift_inv(q[b], q[b + 16], q[b + 32], q[b + 48]);
  }
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    const int b = 16 * (l >> 2) + (l & 3);
    lift_inv(q[b], q[b + 4], q[b + 8], q[b + 12]);
  }
}
// ... then the x pass of every row
template <class T> __device__ __forceinline__ void inverse_x(typename FT<T>::S q[64]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) lift_inv(q[4 * r], q[4 * r + 1], q[4 * r + 2], q[4 * r + 3]);
}
// While every nonzero q * 2^(emax-30) is a normal float (emax >= -96) and no
// product overflows (emax <= 126), the int -> float conversion performs the
// one rounding and the power-of-two scale is exact, so the product equals
// dequantize() without double precision, and acc + product equals one fused
// multiply-add of the converted integer (the product being exact).
__device__ __forceinline__ bool fast_dequant(int emax) { return emax >= -96 && emax <= 126; }
__device__ __forceinline__ float dequant_scale(int emax) {
  return __uint_as_float((uint32_t)(emax - 30 + 127) << 23);
}
// dv[l] * scale is the dequantised value, exactly (scale = 1 on the double route)
__device__ __forceinline__ float dequantize_block(const int32_t q[64], int emax, float dv[64]) {
  if (fast_dequant(emax)) {
#pragma unroll
    for (int l = 0; l < 64; ++l) dv[l] = (float)q[l];
    return dequant_scale(emax);
  }
#pragma unroll
  for (int l = 0; l < 64; ++l) dv[l] = dequantize(q[l], emax);
  return 1.0f;
}
__device__ __forceinline__ double dequantize_block(const int64_t q[64], int emax, double dv[64]) {
#pragma unroll
  for (int l = 0; l < 64; ++l) dv[l] = dequantize(q[l], emax);
  return 1.0;
}
__device__ __forceinline__ void dequant_add(const int32_t q[64], int emax, float acc[64]) {
  if (fast_dequant(emax)) {
    const float scale = dequant_scale(emax);
#pragma unroll
    for (int l = 0; l < 64; ++l) acc[l] = __builtin_fmaf((float)q[l], scale, acc[l]);
  } else {
#pragma unroll
    for (int l = 0; l < 64; ++l) acc[l] = acc[l] + dequantize(q[l], emax);
  }
}
__device__ __forceinline__ void dequant_add(const int64_t q[64], int emax, double acc[64]) {
#pragma unroll
  for (int l = 0; l < 64; ++l) acc[l] = acc[l] + dequantize(q[l], emax);
}

// The float32 high-half route: a block whose coded planes all lie in the top
// ten bit positions (p <= 10) has coefficients that are multiples of 2^22.
// Every word the inverse lifting then forms is a multiple of 2^16: sums,
// differences and doublings of such words act on their high halves modulo
// 2^16 exactly as on the words modulo 2^32, and each halving meets an even
// high half (the inputs are multiples of 2^16 * 2^6 and a value passes at most
// six halvings, two per pass), so the word's arithmetic shift is its high
// half's.  The lifting therefore runs on the high halves alone, two block
// values per register with packed 16-bit operations, and yields the same
// words q = h * 2^16: pairs of adjacent x for the z and y passes, pairs of
// adjacent rows for the x pass (one byte permute per register between).
// Then h * 2^(emax-14) equals q * 2^(emax-30) exactly while fast_dequant(emax)
// holds, so the fused multiply-add is the one of dequant_add.
// Float64 has the same property at the top of its 64-bit words: with p <= 10
// the coefficients are multiples of 2^54, the words the lifting forms are
// multiples of 2^48, and their top 16 bits h follow the same packed lifting;
// q = h * 2^48 is exact in double, so q * 2^(emax-62) = h * 2^(emax-14),
// computed exactly while it is normal (emax >= -1008), is what dequantize()
// gives, and the fused multiply-add of that exact product is acc + it.
template <class T> __device__ __forceinline__ T hi16_scale(int emax);
template <> __device__ __forceinline__ float hi16_scale<float>(int emax) {
  return __uint_as_float((uint32_t)(emax - 14 + 127) << 23);
}
template <> __device__ __forceinline__ double hi16_scale<double>(int emax) {
  return __longlong_as_double((long long)((uint64_t)(emax - 14 + 1023) << 52));
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <class T> __device__ __forceinline__ void lift_dequant_add_hi16(v2s R[32], int emax, T acc[64]) {
#pragma unroll
  for (int m = 0; m < 8; ++m) lift_inv(R[m], R[m + 8], R[m + 16], R[m + 24]);  // z: l, l+16, l+32, l+48
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // y: l, l+4, l+8, l+12 for l = 16 lz + lx
    const int m = 8 * (k >> 1) + (k & 1);
    lift_inv(R[m], R[m + 2], R[m + 4], R[m + 6]);
  }
  const T scale = hi16_scale<T>(emax);
#pragma unroll
  for (int s = 0; s < 8; ++s) {  // rows 2s and 2s+1: X[x] = (q[8s + x], q[8s + 4 + x])
    const uint32_t a0 = __builtin_bit_cast(uint32_t, R[4 * s]), a1 = __builtin_bit_cast(uint32_t, R[4 * s + 1]);
    const uint32_t b0 = __builtin_bit_cast(uint32_t, R[4 * s + 2]), b1 = __builtin_bit_cast(uint32_t, R[4 * s + 3]);
    v2s X0 = __builtin_bit_cast(v2s, __builtin_amdgcn_perm(b0, a0, 0x05040100u));
    v2s X1 = __builtin_bit_cast(v2s, __builtin_amdgcn_perm(b0, a0, 0x07060302u));
    v2s X2 = __builtin_bit_cast(v2s, __builtin_amdgcn_perm(b1, a1, 0x05040100u));
    v2s X3 = __builtin_bit_cast(v2s, __builtin_amdgcn_perm(b1, a1, 0x07060302u));
    lift_inv(X0, X1, X2, X3);
    const v2s X[4] = {X0, X1, X2, X3};
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      acc[8 * s + x] = fma_t((T)X[x].x, scale, acc[8 * s + x]);
      acc[8 * s + 4 + x] = fma_t((T)X[x].y, scale, acc[8 * s + 4 + x]);
    }
  }
}
// R[m] = (q[2m], q[2m+1]) in block order: high halves of the coded-order words c
__device__ __forceinline__ void pack_hi16(const int32_t c[64], v2s R[32]) {
#pragma unroll
  for (int m = 0; m < 32; ++m)
    R[m] = __builtin_bit_cast(v2s, __builtin_amdgcn_perm((uint32_t)c[kInvOrder.at[2 * m + 1]],
                                                         (uint32_t)c[kInvOrder.at[2 * m]], 0x07060302u));
}

template <class U> __device__ __forceinline__ U plane_mask(int P, int p) {
  return p >= P ? ~(U)0 : ~(((U)1 << (P - p)) - (U)1);
}

// Plane words of one 16-plane group are kept in LDS, one column per lane:
// word r of the calling lane at pw[r * 64] (plane base+r of coefficients
// 0..31 in r, of 32..63 in 16+r), so the plane loops below run as ordinary
// loops instead of 16 unrolled copies.
template <class U> __device__ __forceinline__ void group_to_lds(const U u[64], int base, uint32_t* pw) {
  uint32_t Tw[32];
  plane_group(u, base, Tw);
#pragma unroll
  for (int r = 0; r < 32; ++r) pw[r * 64] = Tw[r];
}
// t-th plane from the top of the group
__device__ __forceinline__ uint64_t lds_plane(const uint32_t* pw, int t) {
  return (uint64_t)pw[(15 - t) * 64] | ((uint64_t)pw[(31 - t) * 64] << 32);
}

// bits of p planes from the top, plane words in registers (the closed-form
// cost is short, so the 16-plane loop can be unrolled)
template <class T> __device__ __forceinline__ uint32_t planes_cost_reg(const typename FT<T>::U u[64], int p) {
  constexpr int P = FT<T>::P;
  uint32_t n = 0, bits = 0;
  for (int g = 0; 16 * g < p; ++g) {
    uint32_t Tw[32];
    plane_group(u, P - 16 * (g + 1), Tw);
    const int tmax = p - 16 * g;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      if (t < tmax) bits += plane_cost((uint64_t)Tw[15 - t] | ((uint64_t)Tw[31 - t] << 32), n);
    }
  }
  return bits;
}

template <class T>
__device__ __forceinline__ void planes_emit(LdsBits& w, const typename FT<T>::U u[64], int p, uint32_t* pw,
                                            const uint16_t* tab) {
  typedef typename FT<T>::U U;
  constexpr int P = FT<T>::P;
  // leading empty planes (no coefficient significant yet) are one 0 bit each:
  // the writer only advances over them, and groups made of them are skipped
  U any = 0;
#pragma unroll
  for (int l = 0; l < 64; ++l) any |= u[l];
  int zl = any ? (sizeof(U) == 4 ? __builtin_clz((uint32_t)any) : __builtin_clzll((uint64_t)any)) : P;
  zl = zl < p ? zl : p;
  w.put64(0, (uint32_t)zl);
  uint32_t n = 0;
  // each lane starts at its own first non-empty plane, so the wave's loop
  // runs max(p - zl) times rather than max(p) - min(zl)
  for (int g = zl / 16; 16 * g < p; ++g) {
    group_to_lds(u, P - 16 * (g + 1), pw);
    const int tmax = p - 16 * g < 16 ? p - 16 * g : 16;
    for (int t = 16 * g >= zl ? 0 : zl - 16 * g; t < tmax; ++t) plane_emit(w, lds_plane(pw, t), n, tab);
  }
}

// Transpose of the plane words of W slots (W = 4, 8 or 16) into W-bit
// slices, one per coefficient.  In: A[W-1-t'] holds slot t' of coefficients
// 0..31 (bit j: coefficient j), A[2W-1-t'] of coefficients 32..63.  Out: in
// word i of each half, the W-bit group g is the slice of coefficient W g + i
// of that half, slot t' at bit W-1-t'.  Each half is a row of independent
// W x W bit-matrix transposes, one per group, done by the recursive swap of
// off-diagonal blocks (strides W/2, ..., 1): stage J swaps, in each word pair
// (k, k+J) with bit J of k clear, the bits of a selected by M << J with the
// bits of b selected by M (M: the low J bits of every 2J-bit field).  The
// byte stage is one v_perm per word; the others exchange the masked bits
// through one xor-difference.
template <int J, uint32_t M, int N> __device__ __forceinline__ void gstage(uint32_t A[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k & J) continue;
    const uint32_t a = A[k], b = A[k + J];
    if constexpr (J == 8) {
      A[k] = __builtin_amdgcn_perm(b, a, 0x06020400u);      // a0 b0 a2 b2
      A[k + J] = __builtin_amdgcn_perm(b, a, 0x07030501u);  // a1 b1 a3 b3
    } else {
      const uint32_t t = ((a >> J) ^ b) & M;
      A[k + J] = b ^ t;
      A[k] = a ^ (t << J);
    }
  }
}
template <int W> __device__ __forceinline__ void transpose_groups(uint32_t A[2 * W]) {
  if constexpr (W >= 16) gstage<8, 0x00FF00FFu, 2 * W>(A);
  if constexpr (W >= 8) gstage<4, 0x0F0F0F0Fu, 2 * W>(A);
  gstage<2, 0x33333333u, 2 * W>(A);
  gstage<1, 0x55555555u, 2 * W>(A);
}

// the block's planes in [zlead, p) that fall in W slots (slot t' = plane
// base + t', base <= zlead), transposed into W-bit slices (transpose_groups);
// any deeper planes are left to the caller
template <int W, class R>
__device__ __forceinline__ void read_slots_at(R& r, uint32_t A[2 * W], int base, int p, int zlead, const uint8_t* sq,
                                              uint32_t& n) {
  n = 0;
#pragma unroll
  for (int tp = 0; tp < W; ++tp) {
    const int t = base + tp;
    uint64_t wd = 0;
    if (t >= zlead && t < p) wd = plane_read(r, n, sq);
    A[W - 1 - tp] = (uint32_t)wd;
    A[2 * W - 1 - tp] = (uint32_t)(wd >> 32);
  }
  transpose_groups<W>(A);
}

// the same with the slot base of the block's component (below); returns base
template <class T, int W, class R>
__device__ __forceinline__ int read_slots(R& r, uint32_t A[2 * W], int p, int zlead, const uint8_t* sq, bool rel,
                                          uint32_t& n) {
  constexpr int P = FT<T>::P;
  n = 0;
  // Which planes share a slot across the wave matters: a slot costs the wave
  // as many group-test windows as its slowest lane needs.  Residual
  // components are noise-like, and the planes where most coefficients become
  // significant follow each block's first non-empty plane, so slots count
  // from that plane.  In a store's first component those planes lie at a
  // similar absolute bit level in every block (the data's fine-scale
  // content), i.e. at a fixed distance above the last coded plane, so slots
  // count back from the last plane (base may be negative: leading slots then
  // hold no plane).  Planes above base are empty in either case (base <=
  // zlead).
  const int base = rel ? (zlead < P - W ? zlead : P - W) : (p - W < zlead ? p - W : zlead);
  read_slots_at<W>(r, A, base, p, zlead, sq, n);
  return base;
}

// the coded planes into coded-order two's complement integers; planes at or
// beyond base + W only exist for W = 16 and are added one at a time.
template <class T, int W, class R>
__device__ __forceinline__ void planes_slots(R& r, typename FT<T>::S c[64], int p, int zlead, const uint8_t* sq,
                                             bool rel) {
  typedef typename FT<T>::U U;
  typedef typename FT<T>::S S;
  constexpr int P = FT<T>::P;
  uint32_t A[2 * W], n;
  const int base = read_slots<T, W>(r, A, p, zlead, sq, rel, n);
  // A slice X stands for the coefficient X << sh (sh = P - W - base; the
  // planes above are empty), whose value is ((X ^ M) - M) << sh with M the
  // negabinary mask's bits at the slice's positions (1010... for even sh,
  // 0101... for odd): the mask's lower bits cancel.  One xor serves a whole
  // word of slices.  With base < 0 the slice's top -base bits are zero digits
  // and sh + W - 1 >= P: what the shift drops is the mask alone, dropped from
  // the offset alike (all modulo 2^P).
  const int sh = P - W - base;
  const uint32_t MM = (sh & 1) ? 0x55555555u : 0xAAAAAAAAu;
  constexpr uint32_t kSlice = (1u << W) - 1u;
  // -(M << sh), modulo 2^P, kept opaque so that each coefficient is one
  // shift-and-add of its slice rather than a shift and a subtraction
  const U off = opaque((U)0 - ((U)(MM & kSlice) << sh));
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const uint32_t xl = A[i] ^ MM, xh = A[W + i] ^ MM;
#pragma unroll
    for (int g = 0; g < 32 / W; ++g) {
      c[W * g + i] = (S)(((U)((xl >> (W * g)) & kSlice) << sh) + off);
      c[32 + W * g + i] = (S)(((U)((xh >> (W * g)) & kSlice) << sh) + off);
    }
  }
  if constexpr (W == 16) {
    // deeper planes (rare): a plane bit at an even position b adds 2^b to the
    // two's complement value, one at an odd position subtracts it (the
    // negabinary weight of bit b is (-2)^b)
    for (int t = base + 16 > zlead ? base + 16 : zlead; t < p; ++t) {
      const uint64_t wd = plane_read(r, n, sq);
      const uint32_t lo = (uint32_t)wd, hi = (uint32_t)(wd >> 32);
      const int b = P - 1 - t;
      const U m = (b & 1) ? ~(U)0 : (U)0;  // negate odd positions: (v ^ m) - m
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        c[j] = (S)((U)c[j] + ((((U)((lo >> j) & 1u) << b) ^ m) - m));
        c[j + 32] = (S)((U)c[j + 32] + ((((U)((hi >> j) & 1u) << b) ^ m) - m));
      }
    }
  }
}

// read planes [zlead, p) (the leading empty planes already skipped) and
// return the coefficients in coded order as two's complement integers
// (negabinary decoded; planes below p are zero).  The planes go through W
// register slots and one W x W bit transpose per group of W coefficients; W
// is the smallest of 4, 8 and 16 that holds every active lane's coded planes
// (a wave-uniform choice: residual components typically code 3 to 5 planes
// per block, a store's first one about 10).
template <class T, class R>
__device__ __forceinline__ void planes_read(R& r, typename FT<T>::S c[64], int p, int zlead, const uint8_t* sq,
                                            bool rel) {
  const int np = p - zlead;
  if (__all(np <= 4)) planes_slots<T, 4>(r, c, p, zlead, sq, rel);
  else if (__all(np <= 8)) planes_slots<T, 8>(r, c, p, zlead, sq, rel);
  else planes_slots<T, 16>(r, c, p, zlead, sq, rel);
}

// The float64 high-word route: a block whose coded planes all lie in the top
// 26 bit positions (p <= 26) has coefficients that are multiples of 2^38.
// Every word the inverse lifting then forms is a multiple of 2^32: sums,
// differences and doublings of such words act on their high 32-bit words
// modulo 2^32 exactly as on the words modulo 2^64, and each halving meets an
// even high word (the inputs are multiples of 2^32 * 2^6 and a value passes
// at most six halvings, two per pass), so the word's arithmetic shift is its
// high word's.  The lifting therefore runs on the high words alone, in 32-bit
// integers (half the registers and operations), giving the same words
// q = h * 2^32.
// The high word of a coefficient is (X << (sh - 32)) - (M << (sh - 32))
// modulo 2^32 (sh >= 38 here); deeper planes add their digits' weights to
// it.  Then q * 2^(emax-62) = h * 2^(emax-30), computed exactly by a
// conversion and a power-of-two scale while the result is normal (the caller
// checks emax >= -992), which is the value dequantize() gives.
template <int W, class R>
__device__ __forceinline__ void decode_hi32(R& r, int p, int zlead, int emax, double acc[64], const uint8_t* sq,
                                            bool rel) {
  uint32_t A[2 * W], n;
  const int base = read_slots<double, W>(r, A, p, zlead, sq, rel, n);
  const int sh32 = 32 - W - base;  // sh - 32
  const uint32_t MM = (sh32 & 1) ? 0x55555555u : 0xAAAAAAAAu;
  constexpr uint32_t kSlice = (1u << W) - 1u;
  const uint32_t off = opaque(0u - ((MM & kSlice) << sh32));
  int32_t c[64];
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const uint32_t xl = A[i] ^ MM, xh = A[W + i] ^ MM;
#pragma unroll
    for (int g = 0; g < 32 / W; ++g) {
      c[W * g + i] = (int32_t)((((xl >> (W * g)) & kSlice) << sh32) + off);
      c[32 + W * g + i] = (int32_t)((((xh >> (W * g)) & kSlice) << sh32) + off);
    }
  }
  if constexpr (W == 16) {
    // deeper planes: digit weights (-2)^b at b = 63 - t >= 38, in the high word
    for (int t = base + 16 > zlead ? base + 16 : zlead; t < p; ++t) {
      const uint64_t wd = plane_read(r, n, sq);
      const uint32_t lo = (uint32_t)wd, hi = (uint32_t)(wd >> 32);
      const int b = 31 - t;  // (63 - t) - 32
      const uint32_t m = (b & 1) ? ~0u : 0u;
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        c[j] = (int32_t)((uint32_t)c[j] + ((((lo >> j) & 1u) << b ^ m) - m));
        c[j + 32] = (int32_t)((uint32_t)c[j + 32] + ((((hi >> j) & 1u) << b ^ m) - m));
      }
    }
  }
  int32_t q[64];
#pragma unroll
  for (int r2 = 0; r2 < 64; ++r2) q[kOrder.at[r2]] = c[r2];
#pragma unroll
  for (int l = 0; l < 16; ++l) lift_inv(q[l], q[l + 16], q[l + 32], q[l + 48]);
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    const int b = 16 * (l >> 2) + (l & 3);
    lift_inv(q[b], q[b + 4], q[b + 8], q[b + 12]);
  }
#pragma unroll
  for (int r2 = 0; r2 < 16; ++r2) lift_inv(q[4 * r2], q[4 * r2 + 1], q[4 * r2 + 2], q[4 * r2 + 3]);
#pragma unroll
  for (int l = 0; l < 64; ++l) acc[l] = acc[l] + __builtin_ldexp((double)q[l], emax - 30);
}

// The high-half route straight from the slots of a residual component (W =
// 4 or 8): the pairs R[m] = (h(2m), h(2m+1)) that lift_dequant_add_hi16
// starts from, h(b) the high half of the coded-order word of block position
// b, are formed from the transposed words without the 32-bit words.  With
// slice X of that position (W bits, its negabinary mask bits M already
// flipped, see planes_slots) and sh = 32 - W - base >= 16 + (W == 4 ? 4 : 0)
// (base <= 8 here), the word is ((X - M) << sh) modulo 2^32, whose high half
// is ((X - M) << (sh - 16)) modulo 2^16.  One byte permute moves the byte
// holding each position's slice into the low byte of its half (W = 4: a
// mask then keeps the nibble), and one packed multiply-add forms X * 2^(sh -
// 16) - M * 2^(sh - 16) in both halves (a slice in a byte's upper nibble
// stands for 16 X and takes 2^(sh - 20)).  A float64 word's top 16 bits come
// out the same: its shift is sh + 32, of the same parity, and the top half
// of (X - M) << (sh + 32) modulo 2^64 is again (X - M) << (sh - 16).
template <int W, class R>
__device__ __forceinline__ void slots_hi16(R& r, int p, int zlead, const uint8_t* sq, v2s Rp[32]) {
  static_assert(W == 4 || W == 8, "byte-sized slices or smaller");
  uint32_t A[2 * W], n;
  // base <= 8 keeps sh - 16 >= 4 (W = 4) or >= 0 (W = 8); p <= 10 and a
  // block with zlead = 9 codes one plane, which slot 1 then holds
  const int base = zlead < 8 ? zlead : 8;
  read_slots_at<W>(r, A, base, p, zlead, sq, n);
  const int sh = 32 - W - base;
  const uint32_t MM = (sh & 1) ? 0x55555555u : 0xAAAAAAAAu;
#pragma unroll
  for (int i = 0; i < 2 * W; ++i) A[i] ^= MM;
  constexpr uint32_t kSlice = (1u << W) - 1u;
  const uint32_t d = (uint32_t)(sh - 16);
  const uint32_t off = (0u - ((MM & kSlice) << d)) & 0xFFFFu;  // -M * 2^(sh - 16) modulo 2^16
  const v2u offp = {(unsigned short)off, (unsigned short)off};
  // multipliers by the nibble each half takes: [lower][lower], [lower][upper], ...
  const unsigned short mlo = (unsigned short)(1u << d), mhi = (unsigned short)(W == 4 ? 1u << (d - 4) : 0u);
  const v2u mul[4] = {{mlo, mlo}, {mhi, mlo}, {mlo, mhi}, {mhi, mhi}};
#pragma unroll
  for (int m = 0; m < 32; ++m) {
    // coded positions of block positions 2m and 2m+1, and where their slices sit
    constexpr int kNone = 0x0C;  // v_perm selector of a zero byte
    const int j0 = kInvOrder.at[2 * m], j1 = kInvOrder.at[2 * m + 1];
    const int w0 = (j0 >> 5) * W + (j0 & 31) % W, g0 = (j0 & 31) / W;
    const int w1 = (j1 >> 5) * W + (j1 & 31) % W, g1 = (j1 & 31) / W;
    const int b0 = W == 4 ? g0 >> 1 : g0, b1 = W == 4 ? g1 >> 1 : g1;  // bytes
    const int u0 = W == 4 ? g0 & 1 : 0, u1 = W == 4 ? g1 & 1 : 0;      // upper nibbles
    // perm(x, y, sel): selector 0-3 picks a byte of y, 4-7 one of x
    const uint32_t sel = (uint32_t)b0 | ((uint32_t)kNone << 8) | ((uint32_t)(4 + b1) << 16) | ((uint32_t)kNone << 24);
    uint32_t v = __builtin_amdgcn_perm(A[w1], A[w0], sel);
    if constexpr (W == 4) v &= (u0 ? 0xF0u : 0x0Fu) | ((u1 ? 0xF0u : 0x0Fu) << 16);
    Rp[m] = (v2s)(__builtin_bit_cast(v2u, v) * mul[u0 + 2 * u1] + offp);
  }
}

// a coded float32 block decodes on the high-half route (lift_dequant_add_hi16)
// when its coded planes all lie in the top ten bit positions and its
// exponent keeps the scaled values normal
template <class T> __device__ __forceinline__ bool hi16_block(int p, int emax) {
  return sizeof(T) == 4 && p <= 10 && fast_dequant(emax);
}

// advance a reader over one block without reconstructing it; returns false
// on a malformed header.  full: set for a coded block outside the float32
// high-half route (hi16_block)
template <class T, class R>
__device__ __forceinline__ bool block_skip(R& r, int minexp, const uint8_t* sq, bool& full) {
  full = false;
  constexpr int P = FT<T>::P;
  if (!r.get(1)) return true;  // empty
  if (r.get(1)) {              // raw
    for (int l = 0; l < 64; ++l) r.get64((uint32_t)P);
    return true;
  }
  int delta = 0;
#pragma unroll 1
  while (r.get(1)) {
    if (++delta > P) return false;
  }
  const int emax = (int)r.get((uint32_t)FT<T>::EBITS) - FT<T>::BIAS;
  int p = emax - minexp + kGuard;
  p = (p < 0 ? 0 : (p > P ? P : p)) + delta;
  if (emax < 2 - FT<T>::BIAS || p < 1 || p > P) return false;
  full = sizeof(T) == 4 && !hi16_block<T>(p, emax);
  uint32_t n = 0;
  for (int t = 0; t < p; ++t) (void)plane_read(r, n, sq);
  return true;
}

// ===========================================================================
// Codec 1: prediction and uniform quantisation on the same 4x4x4 blocks (a
// second error-bounded compressor behind the multi-component driver, Sec.
// 6.2; prediction-based compressors, Sec. 5).  Per block and escalation step
// d: bin h_d = 2 tau 2^-d, q = rint(e / h_d) (as e * (1 / h_d) in double),
// the block-local Lorenzo prediction error of q (mixed first differences
// along x, y, z in wrapping P-bit integers) when it is narrower than q, and
// the zigzag values at one width w per block.  Block header: nonempty, coded
// / raw, d in unary, a "predicted" bit, w in 6 bits; then 64 x w bits.
constexpr int kPqMaxDelta = 63;

template <class S> __device__ __forceinline__ typename std::make_unsigned<S>::type zigzag(S r) {
  typedef typename std::make_unsigned<S>::type W;
  return ((W)r << 1) ^ (W)(r >> (8 * sizeof(S) - 1));
}
template <class S> __device__ __forceinline__ S unzigzag(typename std::make_unsigned<S>::type z) {
  typedef typename std::make_unsigned<S>::type W;
  return (S)((z >> 1) ^ ((W)0 - (z & 1u)));
}

// Lorenzo prediction errors in place: each sample minus its predecessor along
// x, then along y, then along z (wrapping); the mixed difference of q
template <class S> __device__ __forceinline__ void lorenzo_fwd(S q[64]) {
#pragma unroll
  for (int l = 63; l >= 0; --l)
    if (l & 3) q[l] = wsub(q[l], q[l - 1]);
#pragma unroll
  for (int l = 63; l >= 0; --l)
    if ((l >> 2) & 3) q[l] = wsub(q[l], q[l - 4]);
#pragma unroll
  for (int l = 63; l >= 0; --l)
    if (l >> 4) q[l] = wsub(q[l], q[l - 16]);
}
// its inverse: running sums along z, y and x (wrapping)
template <class S> __device__ __forceinline__ void lorenzo_inv(S q[64]) {
#pragma unroll
  for (int l = 16; l < 64; ++l) q[l] = wadd(q[l], q[l - 16]);
#pragma unroll
  for (int l = 0; l < 64; ++l)
    if ((l >> 2) & 3) q[l] = wadd(q[l], q[l - 4]);
#pragma unroll
  for (int l = 0; l < 64; ++l)
    if (l & 3) q[l] = wadd(q[l], q[l - 1]);
}

template <class U> __device__ __forceinline__ uint32_t bit_length(U v) {
  if constexpr (sizeof(U) == 4) return v ? 32u - (uint32_t)__builtin_clz(v) : 0u;
  else return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u;
}

// q of a residual block at escalation d: false when some |e * inv_d| is not
// below 2^(P-2) (too wide to code; also NaN)
template <class T>
__device__ __forceinline__ bool pq_quantize(const T e[64], double inv0, int delta, typename FT<T>::S q[64]) {
  typedef typename FT<T>::S S;
  const double inv = __builtin_ldexp(inv0, delta);
  const double lim = (double)((typename FT<T>::U)1 << (FT<T>::P - 2));
  bool ok = true;
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const double t = (double)opaque(e[l]) * inv;  // converted here, each candidate (not held as doubles)
    ok = ok && __builtin_fabs(t) < lim;
    q[l] = ok ? (S)__builtin_rint(t) : (S)0;
  }
  return ok;
}

// width and choice of a quantised block: the zigzag width of q itself and
// of its Lorenzo prediction errors; the predicted form only when narrower.
// Each prediction error is formed from its (up to) eight corner samples, the
// same mixed difference the separable passes give, so q stays as it is and
// no second array is held.
template <class S> __device__ __forceinline__ uint32_t pq_width(const S q[64], bool& pred) {
  typedef typename std::make_unsigned<S>::type W;
  W mq = 0, mp = 0;
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const int x = l & 3, y = (l >> 2) & 3, z = l >> 4;
    W r = (W)q[l];
    if (x) r -= (W)q[l - 1];
    if (y) r -= (W)q[l - 4];
    if (z) r -= (W)q[l - 16];
    if (x && y) r += (W)q[l - 5];
    if (x && z) r += (W)q[l - 17];
    if (y && z) r += (W)q[l - 20];
    if (x && y && z) r -= (W)q[l - 21];
    const W zq = zigzag(q[l]), zp = zigzag((S)r);
    mq = zq > mq ? zq : mq;
    mp = zp > mp ? zp : mp;
  }
  const uint32_t wq = bit_length(mq), wp = bit_length(mp);
  pred = wp < wq;
  return pred ? wp : wq;
}

template <class T> __device__ __forceinline__ uint32_t pq_bits(int delta, uint32_t w) {
  return 2u + (uint32_t)(delta + 1) + 1u + 6u + 64u * w;
}

// emit a coded block of codec 1 (its header bits included)
template <class T>
__device__ __forceinline__ void pq_emit(LdsBits& w, typename FT<T>::S q[64], int delta, bool pred, uint32_t width) {
  typedef typename FT<T>::U U;
  w.put(1, 2);  // nonempty, coded
  for (int t = 0; t < delta; ++t) w.put(1, 1);
  w.put(0, 1);
  w.put(pred ? 1u : 0u, 1);
  w.put(width, 6);
  if (pred) lorenzo_fwd(q);
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const U z = zigzag(q[l]);
    if constexpr (sizeof(U) == 4) w.put(z, width);
    else w.put64(z, width);
  }
}

// Alg. 2 for one block of codec 1: acc += x_i (left to right)
template <class T, class R>
__device__ __forceinline__ bool pq_decode_add(R& r, double h0, T acc[64]) {
  typedef typename FT<T>::U U;
  typedef typename FT<T>::S S;
  constexpr int P = FT<T>::P;
  const uint32_t h = r.peek32();
  if (!(h & 1u)) {  // empty
    r.skip(1);
    return true;
  }
  if (h & 2u) {  // raw block
    r.skip(2);
#pragma unroll
    for (int l = 0; l < 64; ++l) acc[l] = acc[l] + from_raw((U)r.get64((uint32_t)P), (T)0);
    return true;
  }
  int delta = (int)__builtin_ctz(~(h >> 2) | 0x40000000u);
  uint32_t pred, width;
  if (3 + delta + 7 <= 32) {
    pred = (h >> (3 + delta)) & 1u;
    width = (h >> (4 + delta)) & 63u;
    r.skip((uint32_t)(3 + delta + 7));
  } else {
    r.skip(2);
    delta = 0;
#pragma unroll 1
    while (r.get(1)) {
      if (++delta > kPqMaxDelta) return false;
    }
    pred = r.get(1);
    width = r.get(6);
  }
  if (width > (uint32_t)P) return false;  // a P-bit zigzag value needs at most P bits
  S q[64];
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    U z;
    if constexpr (sizeof(U) == 4) z = width ? r.get(width) : 0u;
    else z = width ? (U)r.get64nz(width) : (U)0;
    q[l] = unzigzag<S>(z);
  }
  if (pred) lorenzo_inv(q);
  const double hd = __builtin_ldexp(h0, -delta);
#pragma unroll
  for (int l = 0; l < 64; ++l) acc[l] = acc[l] + (T)((double)q[l] * hd);
  return true;
}

// advance over one block of codec 1 without reconstructing it
template <class T, class R> __device__ __forceinline__ bool pq_block_skip(R& r) {
  constexpr int P = FT<T>::P;
  if (!r.get(1)) return true;
  if (r.get(1)) {
    for (int l = 0; l < 64; ++l) r.get64((uint32_t)P);
    return true;
  }
  int delta = 0;
#pragma unroll 1
  while (r.get(1)) {
    if (++delta > kPqMaxDelta) return false;
  }
  r.get(1);
  const uint32_t width = r.get(6);
  if (width > (uint32_t)P) return false;  // a P-bit zigzag value needs at most P bits
  for (int l = 0; l < 64; ++l) r.get64(width);
  return true;
}

}  // namespace pmc
