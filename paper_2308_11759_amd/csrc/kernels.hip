// kernels.hip -- HIP kernels of the multi-component codec for gfx950, and the
// host-side launchers the C-ABI calls.
//
//  k_encode   one component of Alg. 1 (Sec. 4.1): residual, block coding,
//             decode-for-verify, the x~ update and the measured error
//             (Sec. 4.3); one lane per 4x4x4 block,
//             one wave per 4 chunks, chunk bitstreams assembled in LDS
//  k_tile_*   chunk word counts -> chunk offsets and stream size
//  k_pack     staging -> final stream (header, chunk index, payload)
//  k_decode   Alg. 2 (Sec. 4.2): decode components [k0, k1) of a block and
//             add them left to right into x~; one lane per block, located by
//             the chunk index plus a per-block bit offset written by k_encode
//  k_aux      rebuild those per-block offsets for streams written elsewhere
//  k_range    min / max / non-finite count (tau_0 = range, Sec. 5.1)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "codec_device.hpp"
#include "launch.hpp"

namespace pmc {

enum { MODE_EMPTY = 0, MODE_CODED = 1, MODE_RAW = 2 };

// ---------------------------------------------------------------------------
// block gather / scatter with edge replication for partial blocks
struct BlockPos {
  uint64_t x0, y0, z0;
  uint32_t vx, vy, vz;  // valid extents (1..4)
};

__device__ __forceinline__ BlockPos block_pos(const Geo& g, uint64_t blk) {
  BlockPos b;
  uint64_t bx = blk % g.nbx;
  uint64_t t = blk / g.nbx;
  uint64_t by = t % g.nby;
  uint64_t bz = t / g.nby;
  b.x0 = 4 * bx;
  b.y0 = 4 * by;
  b.z0 = 4 * bz;
  b.vx = (uint32_t)min<uint64_t>(4, g.nx - b.x0);
  b.vy = (uint32_t)min<uint64_t>(4, g.ny - b.y0);
  b.vz = (uint32_t)min<uint64_t>(4, g.nz - b.z0);
  return b;
}

__device__ __forceinline__ bool lvalid(const BlockPos& b, int l) {
  return (uint32_t)(l & 3) < b.vx && (uint32_t)((l >> 2) & 3) < b.vy && (uint32_t)(l >> 4) < b.vz;
}
// bit l set when sample l of the block lies inside the field
__device__ __forceinline__ uint64_t valid_mask(const BlockPos& b) {
  const uint64_t xm = (1ull << b.vx) - 1ull;                                               // a row
  const uint64_t ym = (xm | xm << 4 | xm << 8 | xm << 12) & ((1ull << (4 * b.vy)) - 1ull);  // a z slice
  const uint64_t zm = ym | ym << 16 | ym << 32 | ym << 48;
  return b.vz == 4 ? zm : zm & ((1ull << (16 * b.vz)) - 1ull);
}
// |v| for sample l, or +0 where the sample lies outside the field: the mask
// bit becomes an all-ones / all-zeros word applied to the double's bits, so
// no per-sample condition (a lane mask) has to stay live
__device__ __forceinline__ double masked_abs(uint64_t m, int l, double v) {
  const uint64_t keep = 0ull - ((m >> l) & 1ull);
  return __longlong_as_double((long long)((uint64_t)__double_as_longlong(v) & keep & 0x7FFFFFFFFFFFFFFFull));
}

// one block row (ly, lz): 4 consecutive x values; rows of partial blocks
// repeat their last valid sample (edge replication on load)
template <class T>
__device__ __forceinline__ const T* row_ptr(const T* f, const Geo& g, const BlockPos& b, int r) {
  const uint32_t ly = min<uint32_t>(r & 3, b.vy - 1), lz = min<uint32_t>(r >> 2, b.vz - 1);
  return f + b.x0 + g.nx * ((b.y0 + ly) + g.ny * (b.z0 + lz));
}

// A full block's rows start at block_base + row_step(r): the step depends only
// on the field's shape, so it is the same for every lane (scalar registers)
// and a lane keeps one address instead of one per row.
template <class T> __device__ __forceinline__ T* block_base(T* f, const Geo& g, const BlockPos& b) {
  return f + (b.x0 + g.nx * (b.y0 + g.ny * b.z0));
}
__device__ __forceinline__ uint64_t row_step(const Geo& g, int r) {
  return g.nx * (uint64_t)(r & 3) + g.nx * g.ny * (uint64_t)(r >> 2);
}

template <class T>
__device__ __forceinline__ void load_block(const T* __restrict__ f, const Geo& g, const BlockPos& b, T v[64]) {
  const bool vec = b.vx == 4 && g.rows_aligned;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const T* row = row_ptr(f, g, b, r);
    if (vec) {
      if constexpr (sizeof(T) == 4) {
        float4 q = *reinterpret_cast<const float4*>(row);
        v[4 * r] = q.x; v[4 * r + 1] = q.y; v[4 * r + 2] = q.z; v[4 * r + 3] = q.w;
      } else {
        double2 q0 = *reinterpret_cast<const double2*>(row);
        double2 q1 = *reinterpret_cast<const double2*>(row + 2);
        v[4 * r] = q0.x; v[4 * r + 1] = q0.y; v[4 * r + 2] = q1.x; v[4 * r + 3] = q1.y;
      }
    } else {
      const uint32_t m = b.vx - 1;
      v[4 * r] = row[0];
      v[4 * r + 1] = row[min<uint32_t>(1, m)];
      v[4 * r + 2] = row[min<uint32_t>(2, m)];
      v[4 * r + 3] = row[min<uint32_t>(3, m)];
    }
  }
}

// one 16-byte row piece written with the streaming (nt) cache policy: the
// partial sums a launch writes are read back only by a later launch, after far
// more than the L2 holds has passed through it, so keeping them in L2 would
// only push out lines this launch still reads
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ void store_row16_nt(T* row, T a, T b, T c, T d) {
  if constexpr (sizeof(T) == 4) {
    __builtin_nontemporal_store(nt_f4{a, b, c, d}, reinterpret_cast<nt_f4*>(row));
  } else {
    __builtin_nontemporal_store(nt_d2{a, b}, reinterpret_cast<nt_d2*>(row));
    __builtin_nontemporal_store(nt_d2{c, d}, reinterpret_cast<nt_d2*>(row + 2));
  }
}

template <class T>
__device__ __forceinline__ void store_block(T* __restrict__ f, const Geo& g, const BlockPos& b, const T v[64]) {
  const bool vec = b.vx == 4 && g.rows_aligned;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if ((uint32_t)(r & 3) >= b.vy || (uint32_t)(r >> 2) >= b.vz) continue;
    T* row = const_cast<T*>(row_ptr((const T*)f, g, b, r));
    if (vec) {
      store_row16_nt(row, v[4 * r], v[4 * r + 1], v[4 * r + 2], v[4 * r + 3]);
    } else {
      row[0] = v[4 * r];
      if (b.vx > 1) row[1] = v[4 * r + 1];
      if (b.vx > 2) row[2] = v[4 * r + 2];
      if (b.vx > 3) row[3] = v[4 * r + 3];
    }
  }
}

// store row r of a block (valid samples only); wfull: every lane of the wave
// has a full block of aligned rows (a wave-uniform flag), so the store needs
// no per-lane path
template <class T>
__device__ __forceinline__ void store_row(T* __restrict__ f, const Geo& g, const BlockPos& b, int r, const T v[4],
                                          bool wfull = false) {
  if (!wfull && ((uint32_t)(r & 3) >= b.vy || (uint32_t)(r >> 2) >= b.vz)) return;
  T* row = wfull ? block_base(f, g, b) + row_step(g, r) : const_cast<T*>(row_ptr((const T*)f, g, b, r));
  if (wfull || (b.vx == 4 && g.rows_aligned)) {
    store_row16_nt(row, v[0], v[1], v[2], v[3]);
  } else {
    row[0] = v[0];
    if (b.vx > 1) row[1] = v[1];
    if (b.vx > 2) row[2] = v[2];
    if (b.vx > 3) row[3] = v[3];
  }
}

// the samples of a block that lie in a box, read from / written to the box's
// own dense array (x fastest); samples outside the field are outside every
// box, and samples of the block outside the box are not touched (read as +0)
template <class T>
__device__ __forceinline__ void load_box(const T* __restrict__ f, const BoxArgs& bx, const BlockPos& b, T v[64]) {
  const uint64_t nx = bx.hi[0] - bx.lo[0], ny = bx.hi[1] - bx.lo[1];
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const uint64_t x = b.x0 + (l & 3), y = b.y0 + ((l >> 2) & 3), z = b.z0 + (l >> 4);
    v[l] = (x >= bx.lo[0] && x < bx.hi[0] && y >= bx.lo[1] && y < bx.hi[1] && z >= bx.lo[2] && z < bx.hi[2])
               ? f[(x - bx.lo[0]) + nx * ((y - bx.lo[1]) + ny * (z - bx.lo[2]))]
               : (T)0;
  }
}
template <class T>
__device__ __forceinline__ void store_box(T* __restrict__ f, const BoxArgs& bx, const BlockPos& b, const T v[64]) {
  const uint64_t nx = bx.hi[0] - bx.lo[0], ny = bx.hi[1] - bx.lo[1];
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const uint64_t x = b.x0 + (l & 3), y = b.y0 + ((l >> 2) & 3), z = b.z0 + (l >> 4);
    if (x >= bx.lo[0] && x < bx.hi[0] && y >= bx.lo[1] && y < bx.hi[1] && z >= bx.lo[2] && z < bx.hi[2])
      f[(x - bx.lo[0]) + nx * ((y - bx.lo[1]) + ny * (z - bx.lo[2]))] = v[l];
  }
}

// load row r of a block (edge replication as in load_block); a null field
// reads as +0
template <class T>
__device__ __forceinline__ void load_row(const T* f, const Geo& g, const BlockPos& b, int r, T v[4]) {
  if (!f) {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (T)0;
    return;
  }
  const T* row = row_ptr(f, g, b, r);
  if (b.vx == 4 && g.rows_aligned) {
    if constexpr (sizeof(T) == 4) {
      float4 q = *reinterpret_cast<const float4*>(row);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      double2 q0 = *reinterpret_cast<const double2*>(row);
      double2 q1 = *reinterpret_cast<const double2*>(row + 2);
      v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
    }
  } else {
    const uint32_t m = b.vx - 1;
    v[0] = row[0];
    v[1] = row[min<uint32_t>(1, m)];
    v[2] = row[min<uint32_t>(2, m)];
    v[3] = row[min<uint32_t>(3, m)];
  }
}

// rows [r0, r0 + R) of a block into v[4R].  When every lane of the wave has a
// full block of aligned rows (wfull, a wave-uniform flag) the R loads are
// plain 16-byte loads at the block base plus a uniform step, with no per-lane
// branch, so they are all in flight together; otherwise each row takes
// load_row's per-lane path.  A null field reads as +0.
template <class T, int R>
__device__ __forceinline__ void load_rows(const T* f, const Geo& g, const BlockPos& b, int r0, bool wfull,
                                          T v[4 * R]) {
  if (!f) {
#pragma unroll
    for (int k = 0; k < 4 * R; ++k) v[k] = (T)0;
    return;
  }
  if (wfull) {
    const T* const base = block_base(f, g, b);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const T* row = base + row_step(g, r0 + k);
      if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(row);
        v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
      } else {
        const double2 q0 = *reinterpret_cast<const double2*>(row);
        const double2 q1 = *reinterpret_cast<const double2*>(row + 2);
        v[4 * k] = q0.x; v[4 * k + 1] = q0.y; v[4 * k + 2] = q1.x; v[4 * k + 3] = q1.y;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) load_row(f, g, b, r0 + k, v + 4 * k);
  }
}


__device__ __forceinline__ BlockPos opaque_pos(BlockPos b) {
  b.x0 = opaque(b.x0);
  b.y0 = opaque(b.y0);
  b.z0 = opaque(b.z0);
  return b;
}

// a + v * scale where v * scale is exact: one fused multiply-add equals the
// plain sum of the (exact) product
__device__ __forceinline__ float fma_exact(float v, float scale, float a) { return __builtin_fmaf(v, scale, a); }
__device__ __forceinline__ double fma_exact(double v, double scale, double a) { return a + v * scale; }

// NaN-propagating max, matching "take a if not a <= m"
__device__ __forceinline__ double nmax(double m, double a) { return a <= m ? m : a; }
// the same maximum where no operand is NaN: one v_max_f64 instead of a
// compare and two selects.  The candidate checks take it: |x - x~_i| with
// x finite (an input with NaN or Inf fails the call whatever its streams)
// and x~_i finite or, on overflow, infinite (x~_{i-1} stays within tau of x)
__device__ __forceinline__ double nmax_num(double m, double a) { return __builtin_fmax(m, a); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = nmax(v, __shfl_xor(v, d, 64));
  return v;
}

// ---------------------------------------------------------------------------
// encode one component
constexpr uint32_t kEmitWords = 256;  // LDS window per chunk, in 32-bit words

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gmem_void_t;

// the block's x values in LDS, [row r][lane][4 values] (f32) or
// [row r][half h][lane][2 values] (f64): each 16-byte piece of a row is one
// direct global->LDS load (global_load_lds_dwordx4), so x never occupies
// VGPRs; partial or unaligned rows are written by plain loads
template <class T> struct XLds {
  T* base;  // s_x
  uint32_t lane;
  __device__ __forceinline__ T* slot(int r, int t) const {
    if constexpr (sizeof(T) == 4) return base + ((uint32_t)r * 64 + lane) * 4 + t;
    else return base + (((uint32_t)r * 2 + (t >> 1)) * 64 + lane) * 2 + (t & 1);
  }
  __device__ __forceinline__ T at(int l) const { return *slot(l >> 2, l & 3); }
};

// The encoder's own partial sums x~_i (its workspace, never seen outside
// compression) are not kept in the field's layout but in one tile per wave:
// the wave's 64 blocks as [row r][lane][16-byte piece] (float32: 4 values;
// float64: [row r][half][lane][2 values]), the layout XLds uses in LDS.
// Every row access of a wave is then one coalesced 1 KiB transfer at a
// uniform offset, with no per-lane paths for partial blocks; their padded
// samples hold values nothing reads (the residual is edge-replicated from
// the block's valid samples in registers instead).
constexpr uint64_t kTileValues = 64 * 64;  // values of one wave's tile
template <class T> __device__ __forceinline__ uint32_t tile_index(uint32_t lane, int r, int t) {
  if constexpr (sizeof(T) == 4) return ((uint32_t)r * 64 + lane) * 4 + (uint32_t)t;
  else return (((uint32_t)r * 2 + (uint32_t)(t >> 1)) * 64 + lane) * 2 + (uint32_t)(t & 1);
}
// rows [r0, r0 + R) of this lane's block from a wave's tile; a null tile reads as +0
template <class T, int R>
__device__ __forceinline__ void tile_load_rows(const T* tile, uint32_t lane, int r0, T v[4 * R]) {
  if (!tile) {
#pragma unroll
    for (int k = 0; k < 4 * R; ++k) v[k] = (T)0;
    return;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if constexpr (sizeof(T) == 4) {
      const float4 q = *reinterpret_cast<const float4*>(tile + tile_index<T>(lane, r0 + k, 0));
      v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
    } else {
      const double2 q0 = *reinterpret_cast<const double2*>(tile + tile_index<T>(lane, r0 + k, 0));
      const double2 q1 = *reinterpret_cast<const double2*>(tile + tile_index<T>(lane, r0 + k, 2));
      v[4 * k] = q0.x; v[4 * k + 1] = q0.y; v[4 * k + 2] = q1.x; v[4 * k + 3] = q1.y;
    }
  }
}
// row r of this lane's block into a wave's tile (streaming cache policy: the
// next reader is the next component's launch)
template <class T> __device__ __forceinline__ void tile_store_row(T* tile, uint32_t lane, int r, const T v[4]) {
  if constexpr (sizeof(T) == 4) {
    __builtin_nontemporal_store(nt_f4{v[0], v[1], v[2], v[3]}, reinterpret_cast<nt_f4*>(tile + tile_index<T>(lane, r, 0)));
  } else {
    __builtin_nontemporal_store(nt_d2{v[0], v[1]}, reinterpret_cast<nt_d2*>(tile + tile_index<T>(lane, r, 0)));
    __builtin_nontemporal_store(nt_d2{v[2], v[3]}, reinterpret_cast<nt_d2*>(tile + tile_index<T>(lane, r, 2)));
  }
}
// edge replication of a partial block's residual, in registers: each padded
// sample takes the value of the last valid sample on each axis (x, then y,
// then z), as the block gather of a partial block does
template <class T>
__device__ __forceinline__ void replicate_edges(T e[64], uint32_t vx, uint32_t vy, uint32_t vz) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int t = 1; t < 4; ++t) e[4 * r + t] = (uint32_t)t < vx ? e[4 * r + t] : e[4 * r + t - 1];
#pragma unroll
  for (int lz = 0; lz < 4; ++lz)
#pragma unroll
    for (int ly = 1; ly < 4; ++ly)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int l = 4 * ly + 16 * lz + t;
        e[l] = (uint32_t)ly < vy ? e[l] : e[l - 4];
      }
#pragma unroll
  for (int lz = 1; lz < 4; ++lz)
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int l = 16 * lz + m;
      e[l] = (uint32_t)lz < vz ? e[l] : e[l - 16];
    }
}

// (the direct loads are only issued here: the caller waits, s_waitcnt 0,
// before reading s_x, and may issue other loads first.  x is read from memory
// once per launch, so its loads take the streaming (nt) policy, cache-policy
// bit 1, leaving L2 to the x~ rows that the check pass reads a second time)
constexpr int kNt = 2;
template <class T>
__device__ __forceinline__ void load_block_lds(const T* __restrict__ f, const Geo& g, const BlockPos& b, T* s_x,
                                               uint32_t lane, bool wfull) {
  const bool vec = wfull || (b.vx == 4 && g.rows_aligned);
  XLds<T> X{s_x, lane};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const T* row = row_ptr(f, g, b, r);
    if (vec) {
      if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_global_load_lds((gmem_void_t*)row, (lds_void_t*)(s_x + r * 256), 16, 0, kNt);
      } else {
        __builtin_amdgcn_global_load_lds((gmem_void_t*)row, (lds_void_t*)(s_x + (r * 2) * 128), 16, 0, kNt);
        __builtin_amdgcn_global_load_lds((gmem_void_t*)(row + 2), (lds_void_t*)(s_x + (r * 2 + 1) * 128), 16, 0,
                                         kNt);
      }
    } else {
      const uint32_t m = b.vx - 1;
#pragma unroll
      for (int t = 0; t < 4; ++t) *X.slot(r, t) = row[min<uint32_t>(t, m)];
    }
  }
}

// the candidate check of a codec-1 block: x~_i = x~_{i-1} + x_i row by row
// in the field precision, each integer q = rint(e * inv_d) formed again and
// turned into q * h_d as its row comes (so no array of integers or decoded
// values is held across the check), the rows stored as they come (a
// rejected candidate is overwritten later), and the largest |x - x~_i| in
// double over the block's valid samples
template <class T>
__device__ __forceinline__ double check_rows_pq(const XLds<T>& XL, const T* tin, T* tout, uint32_t lane,
                                                uint64_t vmask, const T e[64], double inv, double h) {
  double ea = 0.0;
  constexpr int RB = 8;
#pragma unroll
  for (int r0 = 0; r0 < 16; r0 += RB) {
    T tr[4 * RB];
    tile_load_rows<T, RB>(tin, lane, r0, tr);
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int r = r0 + k;
      T row[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int l = 4 * r + t;
        const typename FT<T>::S q = (typename FT<T>::S)__builtin_rint((double)opaque(e[l]) * inv);
        row[t] = tr[4 * k + t] + (T)((double)q * h);  // x~_{i-1} + x_i in the field precision
        ea = nmax_num(ea, masked_abs(vmask, l, (double)XL.at(l) - (double)row[t]));
      }
      if (tout) tile_store_row(tout, lane, r, row);
    }
  }
  return ea;
}

// one wave = 64 consecutive blocks = 4 chunks; `wave` numbers these groups
// within the field.  s_x: 64 * 64 values of LDS owned by this wave.  kFull:
// the caller guarantees that every block is full and rows are aligned (all
// three dimensions multiples of 4), so the per-lane edge paths of the x
// loads and of the residual compile away and their conditions hold no
// registers.  x~_{i-1} / x~_i are the wave's tiles (see tile_index).
// kCodec: 0 the block-transform codec, 1 prediction and quantisation (its
// residual block stays in registers for the candidates and the emission)
// kHiCheck: float64 candidates may be checked on the high-word route (the
// batched kernel leaves it out: it holds too many registers there)
template <class T, bool kFull = false, int kCodec = 0, bool kHiCheck = true>
__device__ __forceinline__ void encode_wave(const EncArgs<T> a, uint32_t wave, T* s_x, const uint16_t* unsq) {
  typedef typename FT<T>::U U;
  typedef typename FT<T>::S S;
  constexpr int P = FT<T>::P;
  constexpr int CAP = chunk_cap_words<T>();
  // LDS: the block's x values while deciding; once x is dead the same bytes
  // hold the emission windows and the plane words
  static_assert(64 * 64 * sizeof(T) >= 4 * (4 * kEmitWords + 32 * 64), "LDS reuse");
  uint32_t* const s_emit = reinterpret_cast<uint32_t*>(s_x);
  uint32_t* const s_planes = s_emit + 4 * kEmitWords;

  const uint32_t lane = threadIdx.x;
  uint32_t* pw = s_planes + lane;
  const uint64_t blk = (uint64_t)wave * 64 + lane;
  const bool active = blk < a.g.nblocks;

  BlockPos bp = block_pos(a.g, active ? blk : 0);
  if constexpr (kFull) {
    bp.vx = 4;
    bp.vy = 4;
    bp.vz = 4;
  }
  // every lane has a full block of aligned rows: row accesses without per-lane paths
  const bool wfull = kFull || __all(bp.vx == 4 && bp.vy == 4 && bp.vz == 4 && a.g.rows_aligned);
  // this wave's tiles of x~_{i-1} (none for the first component) and x~_i
  // (none for the last)
  const T* const tile_in = a.first ? nullptr : a.xt_in + (uint64_t)wave * kTileValues;
  T* const tile_out = a.last ? nullptr : a.xt_out + (uint64_t)wave * kTileValues;
  // x into LDS and x~_{i-1} into registers, all loads in flight together
  load_block_lds(a.x, a.g, bp, s_x, lane, wfull);
  T e[64];
  tile_load_rows<T, 16>(tile_in, lane, 0, e);
  __builtin_amdgcn_s_waitcnt(0);  // direct loads, LDS writes and the rows complete
  const XLds<T> X{s_x, lane};
  // row addresses are recomputed where used instead of kept in registers
  bp = opaque_pos(bp);
  const uint64_t vmask = kFull ? ~0ull : valid_mask(bp);

  // the residual e = x - x~_{i-1} (kept in registers), edge-replicated in a
  // partial block, and its largest magnitude (the block exponent, the
  // all-zero test).  The first component, where x~_0 = 0 and the residual is
  // x itself, also gives the largest |x| (non-finite input; x is the same for
  // every component, and the host combines the components' flags).
  U maxabs = 0, xmax = 0;  // largest |residual| and |x| bit patterns
  U u[64];                 // the residual's coefficients: every candidate and the emission use them
  int emax;
  {
#pragma unroll
    for (int l = 0; l < 64; ++l) e[l] = X.at(l) - e[l];
    if constexpr (!kFull) {
      if (!wfull) replicate_edges(e, bp.vx, bp.vy, bp.vz);
    }
#pragma unroll
    for (int l = 0; l < 64; ++l) {
      const U ab = abs_bits(e[l]);
      maxabs = ab > maxabs ? ab : maxabs;
    }
    if (a.first) xmax = maxabs;  // x - (+0) has the magnitude of x
    emax = block_emax<T>(maxabs);
    if constexpr (kCodec == 0) {
      if (active && maxabs != 0) forward_coeffs<T>(e, emax, u);
    }
  }
  // the error before this component, max |x - x~_{i-1}| in double over the
  // block's samples: the previous component left it per block; for the first
  // (x~_0 = 0) it is the largest |x| (edge samples repeat valid ones) unless a
  // NaN makes the running maximum order-dependent, then it is taken sample by
  // sample as everywhere else
  double eb = 0.0;
  if (!a.first) {
    if (active) eb = a.berr[blk];
  } else if (xmax <= abs_bits((T)__builtin_inf())) {
    eb = (double)from_raw(xmax, (T)0);
  } else {
#pragma unroll 4
    for (int l = 0; l < 64; ++l) eb = nmax(eb, masked_abs(vmask, l, (double)X.at(l) - 0.0));
  }
  int p = emax - a.minexp + kGuard;
  p = p < 0 ? 0 : (p > P ? P : p);
  int mode = MODE_EMPTY, delta = 0;
  uint32_t nbits = 1;
  double err = eb;

  // acceptance: smallest plane count p >= p0 whose block meets tau without
  // raising the error; else empty (already within tau) or raw
  if (active && maxabs != 0) {
    for (;;) {
      // re-derived each iteration so the loads below are not hoisted out of
      // the loop into 64 registers
      const XLds<T> XL{opaque(s_x), lane};
      const T* const tin = tile_in;
      const uint32_t ln = opaque(lane);  // tile addresses likewise
      bool feasible = false;
      uint32_t cb = 0;
      if constexpr (kCodec == 0) {
        if (p >= 1 && p <= P) {
          cb = 2u + (uint32_t)(delta + 1) + (uint32_t)FT<T>::EBITS + planes_cost_reg<T>(u, p);
          feasible = cb <= (uint32_t)FT<T>::RAW_BITS;
        }
        if (feasible) {
          const U m = plane_mask<U>(P, p);
          // decode, add and check one row at a time; x~_i rows are stored as
          // they come (a rejected candidate is overwritten below)
          T dv[64];
          T scale;
          if (sizeof(T) == 8 && kHiCheck && __all(p <= 26 && emax >= -992)) {
            // float64 with the top p <= 26 planes: the inverse transform on
            // the coefficients' high 32-bit words (see decode_hi32), the
            // same values
            int32_t h[64];
#pragma unroll
            for (int r = 0; r < 64; ++r) h[kOrder.at[r]] = (int32_t)((uint64_t)from_nb<T>(u[r] & m) >> 32);
#pragma unroll
            for (int l = 0; l < 16; ++l) lift_inv(h[l], h[l + 16], h[l + 32], h[l + 48]);
#pragma unroll
            for (int l = 0; l < 16; ++l) {
              const int b = 16 * (l >> 2) + (l & 3);
              lift_inv(h[b], h[b + 4], h[b + 8], h[b + 12]);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) lift_inv(h[4 * r], h[4 * r + 1], h[4 * r + 2], h[4 * r + 3]);
#pragma unroll
            for (int l = 0; l < 64; ++l) dv[l] = (T)__builtin_ldexp((double)h[l], emax - 30);
            scale = (T)1;
          } else {
            S c[64], q[64];
#pragma unroll
            for (int r = 0; r < 64; ++r) c[r] = from_nb<T>(u[r] & m);  // the top p planes
            inverse_zy_ints<T>(c, q);
            inverse_x<T>(q);
            scale = dequantize_block(q, emax, dv);
          }
          double ea = 0.0;
          // eight rows of x~_{i-1} in flight together
          constexpr int RB = 8;
#pragma unroll
          for (int r0 = 0; r0 < 16; r0 += RB) {
            T tr[4 * RB];
            tile_load_rows<T, RB>(tin, ln, r0, tr);
#pragma unroll
            for (int k = 0; k < RB; ++k) {
              const int r = r0 + k;
              T row[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int l = 4 * r + t;
                row[t] = fma_exact(dv[l], scale, tr[4 * k + t]);  // x~_{i-1} + x_i in the field precision
                const double dl = masked_abs(vmask, l, (double)XL.at(l) - (double)row[t]);
                ea = sizeof(T) == 4 ? nmax_num(ea, dl) : nmax(ea, dl);  // (float64: nmax holds fewer registers)
              }
              if (tile_out) tile_store_row(tile_out, ln, r, row);
            }
          }
          if (ea <= a.tau && ea <= eb) {
            mode = MODE_CODED;
            nbits = cb;
            err = ea;
            break;
          }
        }
      } else {
        // bin 2 tau 2^-delta; the block's integers, its code width, its size
        S q[64];
        if (delta <= kPqMaxDelta && pq_quantize<T>(e, a.inv0, delta, q)) {
          bool pred;
          cb = pq_bits<T>(delta, pq_width(q, pred));
          feasible = cb <= (uint32_t)FT<T>::RAW_BITS;
        }
        if (feasible) {
          const double ea = check_rows_pq<T>(XL, tin, tile_out, ln, vmask, e, __builtin_ldexp(a.inv0, delta),
                                             __builtin_ldexp(a.h0, -delta));
          if (ea <= a.tau && ea <= eb) {
            mode = MODE_CODED;
            nbits = cb;
            err = ea;
            break;
          }
        }
      }
      if (eb <= a.tau) {
        mode = MODE_EMPTY;
        nbits = 1;
        err = eb;
        break;
      }
      if (!feasible) {
        mode = MODE_RAW;
        nbits = (uint32_t)FT<T>::RAW_BITS;
        break;
      }
      ++p;
      ++delta;
    }
  }
  bool miss = false;
  if (active && mode == MODE_RAW) {
    double ea = 0.0;
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
      T tr[4], d[4];
      tile_load_rows<T, 1>(tile_in, lane, r, tr);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int l = 4 * r + t;
        const T xl = X.at(l);
        d[t] = tr[t] + (xl - tr[t]);
        ea = nmax(ea, masked_abs(vmask, l, (double)xl - (double)d[t]));
      }
      if (tile_out) tile_store_row(tile_out, lane, r, d);
    }
    err = ea;
    miss = !(ea <= a.tau && ea <= eb);
  } else if (active && mode == MODE_EMPTY) {
    miss = !(eb <= a.tau);
    // x~_i = x~_{i-1} + 0 (also over the rows of a rejected candidate)
    if (tile_out) {
#pragma unroll 1
      for (int r = 0; r < 16; ++r) {
        T tr[4], d[4];
        tile_load_rows<T, 1>(tile_in, lane, r, tr);
#pragma unroll
        for (int t = 0; t < 4; ++t) d[t] = tr[t] + (T)0;
        tile_store_row(tile_out, lane, r, d);
      }
    }
  }
  if (!active) {
    err = 0.0;
    miss = false;
    nbits = 0;
  }
  if (active && !a.last) a.berr[blk] = err;  // the next component's error before coding

  // per-component statistics
  {
    // every counter lives on one cache line, so the usual wave issues no
    // atomic at all: coded blocks are counted on the host as the remainder,
    // and the error maximum is only raised when this wave's exceeds it
    const unsigned long long be = __ballot(active && mode == MODE_EMPTY);
    const unsigned long long br = __ballot(active && mode == MODE_RAW);
    const unsigned long long bs = __ballot(active && mode == MODE_CODED && delta > 0);
    const unsigned long long bf =
        kCodec == 0 && sizeof(T) == 4 ? __ballot(active && mode == MODE_CODED && !hi16_block<T>(p, emax)) : 0ull;
    const unsigned long long bm = __ballot(miss);
    const bool nonfinite = xmax >= abs_bits((T)__builtin_inf());  // an infinite or NaN sample
    const unsigned long long bn = __ballot(active && nonfinite);
    const double wm = wave_max(err);
    if (lane == 0) {
      if (be) atomicAdd(&a.meta->nempty, (unsigned long long)__popcll(be));
      if (br) atomicAdd(&a.meta->nraw, (unsigned long long)__popcll(br));
      if (bs) atomicAdd(&a.meta->nesc, (unsigned long long)__popcll(bs));
      // a flag, read first: most waves of such a component would set it
      if (bf && *(volatile unsigned long long*)&a.meta->full == 0) atomicOr(&a.meta->full, 1ull);
      if (bm) atomicAdd(&a.meta->nmiss, (unsigned long long)__popcll(bm));
      if (bn) atomicOr(&a.meta->flags, (unsigned int)FLAG_NONFINITE);
      const unsigned long long wb = (unsigned long long)__double_as_longlong(wm);
      if (wb > *(volatile unsigned long long*)&a.meta->linf_bits) atomicMax(&a.meta->linf_bits, wb);
    }
  }

  __syncthreads();  // every lane is done with x: its LDS is reused below

  // offsets of the blocks inside their chunk (16 lanes = one chunk)
  uint32_t incl = nbits;
#pragma unroll
  for (int s = 1; s < 16; s <<= 1) {
    uint32_t y = __shfl_up(incl, s, 16);
    if ((lane & 15) >= (uint32_t)s) incl += y;
  }
  const uint32_t off = incl - nbits;
  if (active) a.aux[blk] = off;
  uint32_t cwords[4];
  uint32_t maxw = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cwords[c] = (__shfl(incl, 16 * c + 15, 64) + 31) / 32;
    maxw = cwords[c] > maxw ? cwords[c] : maxw;
  }

  // emit the four chunk bitstreams through LDS windows of kEmitWords words
  for (uint32_t w0 = 0; w0 < maxw; w0 += kEmitWords) {
    for (uint32_t i = lane; i < 4 * kEmitWords; i += 64) s_emit[i] = 0;
    __syncthreads();
    const uint64_t lo_bit = (uint64_t)w0 * 32, hi_bit = (uint64_t)(w0 + kEmitWords) * 32;
    if (active && (uint64_t)off < hi_bit && (uint64_t)off + nbits > lo_bit) {
      LdsBits w;
      w.init(&s_emit[(lane >> 4) * kEmitWords], off, w0, kEmitWords);
      if (mode == MODE_EMPTY) {
        w.put(0, 1);
      } else if (mode == MODE_RAW) {  // the residual's bits, x and x~_{i-1} re-read
        w.put(3, 2);
#pragma unroll 1
        for (int r = 0; r < 16; ++r) {
          T xr[4];
          load_row(a.x, a.g, bp, r, xr);  // x of the sample the edge replication picks
          const uint32_t ly = min<uint32_t>(r & 3, bp.vy - 1), lz = min<uint32_t>(r >> 2, bp.vz - 1);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            // x~_{i-1} of the same sample, from the tile
            const T tr = tile_in ? tile_in[tile_index<T>(lane, (int)(ly + 4 * lz), (int)min<uint32_t>(t, bp.vx - 1))]
                                 : (T)0;
            w.put64((uint64_t)raw_bits_lo((T)(xr[t] - tr)), (uint32_t)P);
          }
        }
      } else if constexpr (kCodec == 0) {
        w.put(1, 2);  // nonempty, coded
        for (int t = 0; t < delta; ++t) w.put(1, 1);
        w.put(0, 1);
        w.put((uint64_t)(emax + FT<T>::BIAS), (uint32_t)FT<T>::EBITS);
        planes_emit<T>(w, u, p, pw, unsq);
      } else {
        // the accepted candidate's integers again (the same arithmetic)
        S q[64];
        (void)pq_quantize<T>(e, a.inv0, delta, q);
        bool pred;
        const uint32_t width = pq_width(q, pred);
        pq_emit<T>(w, q, delta, pred, width);
      }
      w.flush();
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint64_t chunk = (uint64_t)wave * 4 + c;
      if (chunk < a.g.nchunks && cwords[c] > w0) {
        const uint32_t nw = cwords[c] - w0 < kEmitWords ? cwords[c] - w0 : kEmitWords;
        uint32_t* dst = a.staging + chunk * (uint64_t)CAP + w0;
        for (uint32_t i = lane; i < nw; i += 64) dst[i] = s_emit[c * kEmitWords + i];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint64_t chunk = (uint64_t)wave * 4 + c;
    if (lane == 0 && chunk < a.g.nchunks) a.chunk_words[chunk] = cwords[c];
  }
}

template <class T, bool kFull, int kCodec>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void k_encode(EncArgs<T> a) {
  __shared__ T s_x[64 * 64];
  __shared__ uint16_t s_unsq[256];
  unsqueeze_table(s_unsq);
  encode_wave<T, kFull, kCodec>(a, blockIdx.x, s_x, s_unsq);
}

// ---------------------------------------------------------------------------
// chunk offsets: exclusive prefix sum of chunk word counts in two passes
// over tiles of kScanTile chunks (tile sums; then per tile the sum of the
// tile sums before it plus the scan inside it, with the stream size
// bookkeeping in the first tile's workgroup).  The batched path keeps three
// passes (tile sums, their scan per field, per-tile scans)
__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v, uint32_t lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long y = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += y;
  }
  return v;
}

// block-wide inclusive scan of one value per thread (1024 threads)
__device__ __forceinline__ unsigned long long block_incl_scan(unsigned long long v, unsigned long long* sh) {
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  v = wave_incl_scan(v, lane);
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  if (wave == 0) {
    unsigned long long w = lane < 16 ? sh[lane] : 0ull;
    w = wave_incl_scan(w, lane);
    if (lane < 16) sh[lane] = w;
  }
  __syncthreads();
  if (wave > 0) v += sh[wave - 1];
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(1024) void k_tile_sums(ScanArgs a) {
  __shared__ unsigned long long sh[16];
  const uint64_t i = (uint64_t)blockIdx.x * kScanTile + threadIdx.x;
  unsigned long long v = i < a.nchunks ? a.chunk_words[i] : 0ull;
  v = block_incl_scan(v, sh);
  if (threadIdx.x == kScanTile - 1) a.tile_sums[blockIdx.x] = v;
}

// chunk offsets of one tile: the words of the tiles before it (from the
// tile sums) plus the exclusive scan inside the tile; workgroup 0 also
// records the stream's size and where the next component's stream starts
__global__ __launch_bounds__(1024) void k_tile_offsets(ScanArgs a) {
  __shared__ unsigned long long sh[16];
  const uint64_t ntiles = (a.nchunks + kScanTile - 1) / kScanTile;
  unsigned long long before = 0, total = 0;
  for (uint64_t base = 0; base < ntiles; base += 1024) {
    const uint64_t j = base + threadIdx.x;
    const unsigned long long v = j < ntiles ? a.tile_sums[j] : 0ull;
    before += j < blockIdx.x ? v : 0ull;
    total += v;
  }
  (void)block_incl_scan(before, sh);
  before = sh[15];  // the workgroup's sum (sh is stable until the next scan writes it)
  __syncthreads();
  (void)block_incl_scan(total, sh);
  total = sh[15];
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * kScanTile + threadIdx.x;
  const unsigned long long v = i < a.nchunks ? a.chunk_words[i] : 0ull;
  const unsigned long long inc = block_incl_scan(v, sh);
  if (i < a.nchunks) a.offsets[i] = (uint32_t)(before + inc - v);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CompMeta* m = &a.meta[a.comp];
    const unsigned long long words = total;
    const unsigned long long bytes = (unsigned long long)kHeaderBytes + 4ull * a.nchunks + 4ull * words;
    m->payload_words = words;
    m->stream_bytes = bytes;
    const unsigned long long end = m->stream_offset + bytes;
    if (end > a.streams_cap) m->flags |= FLAG_OVERFLOW;
    if (words > 0xFFFFFFFFull) m->flags |= FLAG_INDEX;
    if (a.comp + 1 < a.ncomp) a.meta[a.comp + 1].stream_offset = (end + 255ull) & ~255ull;
  }
}

// ---------------------------------------------------------------------------
// copy the four chunks [c0, c0 + 4) from their staging slots (cap words
// apart) into the payload.  They are consecutive in the payload (the offsets
// are a prefix sum), so their words form one output range that all lanes copy
// together, each word fetched from its chunk's slot.  Returns the range's
// length in words (the chunks' decode-wave span).
__device__ __forceinline__ uint32_t pack_quad(const uint32_t* __restrict__ staging, uint64_t cap,
                                              const uint32_t* chunk_words, const uint32_t* offsets, uint64_t nchunks,
                                              uint64_t c0, uint32_t* __restrict__ payload, uint32_t* index) {
  const uint32_t lane = threadIdx.x;
  uint32_t cum[5];
  cum[0] = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) cum[c + 1] = cum[c] + (c0 + c < nchunks ? chunk_words[c0 + c] : 0u);
  const uint32_t o0 = offsets[c0];
  const uint32_t span = cum[4];
  const uint32_t* __restrict__ src = staging + c0 * cap;
  uint32_t* __restrict__ dst = payload + o0;
  for (uint32_t j0 = 0; j0 < span; j0 += 256) {
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // four loads in flight per lane
      const uint32_t j = j0 + 64 * k + lane;
      const uint32_t c = (j >= cum[1] ? 1u : 0u) + (j >= cum[2] ? 1u : 0u) + (j >= cum[3] ? 1u : 0u);
      const uint32_t start = c == 0 ? 0u : c == 1 ? cum[1] : c == 2 ? cum[2] : cum[3];
      v[k] = j < span ? src[c * cap + (j - start)] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t j = j0 + 64 * k + lane;
      if (j < span) dst[j] = v[k];
    }
  }
  if (lane < 4 && c0 + lane < nchunks)
    index[c0 + lane] = o0 + (lane == 0 ? 0u : lane == 1 ? cum[1] : lane == 2 ? cum[2] : cum[3]);
  return span;
}

// staging -> stream: header, index, payload (one wave per four chunks)
template <class T>
__global__ __launch_bounds__(64) void k_pack(PackArgs a) {
  constexpr int CAP = chunk_cap_words<T>();
  const CompMeta* m = &a.meta[a.comp];
  if (m->flags & (FLAG_OVERFLOW | FLAG_INDEX)) return;
  uint8_t* base = a.streams + m->stream_offset;
  uint32_t* index = reinterpret_cast<uint32_t*>(base + kHeaderBytes);
  uint32_t* payload = index + a.nchunks;
  const uint32_t lane = threadIdx.x;
  // a grid-stride loop over the chunk quads: few, longer-lived waves
  const uint64_t nquads = (a.nchunks + 3) / 4;
  uint32_t span = 0;
  for (uint64_t q = blockIdx.x; q < nquads; q += gridDim.x) {
    const uint32_t s = pack_quad(a.staging, CAP, a.chunk_words, a.offsets, a.nchunks, q * 4, payload, index);
    span = s > span ? s : span;
  }
  // most waves see a maximum already recorded: read before the atomic
  if (lane == 0 && span > *(volatile unsigned long long*)&a.meta[a.comp].max_span)
    atomicMax(&a.meta[a.comp].max_span, (unsigned long long)span);
  if (blockIdx.x == 0 && lane < 16) {
    uint32_t* h = reinterpret_cast<uint32_t*>(base);
    const uint64_t taub = (uint64_t)__double_as_longlong(a.tau);
    uint32_t v = 0;
    switch (lane) {
      case 0: v = kMagic; break;
      case 1: v = (uint32_t)kVersion | ((uint32_t)a.codec << 8) | ((uint32_t)FT<T>::CODE << 16) | (3u << 24); break;
      case 2: v = (uint32_t)a.g.nx; break;
      case 3: v = (uint32_t)(a.g.nx >> 32); break;
      case 4: v = (uint32_t)a.g.ny; break;
      case 5: v = (uint32_t)(a.g.ny >> 32); break;
      case 6: v = (uint32_t)a.g.nz; break;
      case 7: v = (uint32_t)(a.g.nz >> 32); break;
      case 8: v = (uint32_t)taub; break;
      case 9: v = (uint32_t)(taub >> 32); break;
      case 10: v = (uint32_t)a.minexp; break;
      case 11: v = (uint32_t)kChunkBlocks; break;
      case 12: v = (uint32_t)a.nchunks; break;
      case 13: v = (uint32_t)(a.nchunks >> 32); break;
      case 14: v = (uint32_t)m->payload_words; break;
      case 15: v = (uint32_t)(m->payload_words >> 32); break;
    }
    h[lane] = v;
  }
}

// ---------------------------------------------------------------------------
// Alg. 2 over one block per lane: x~ = (((x~_in or +0) + x_1) + x_2) ... in
// the field precision; the block's bits start at its chunk's word offset plus
// the block's bit offset from the per-block index
// routes of the inverse transform: kRouteAuto picks per wave (float64: the
// high-word route where it applies); kRouteFull the plain route; kRouteHi16
// the float32 high-half route, for components whose every block has p <= 10
// and fast_dequant(emax) (the caller guarantees it)
constexpr int kRouteAuto = 0, kRouteFull = 1, kRouteHi16 = 2;
template <class T, int kRoute = kRouteAuto, class R>
__device__ __forceinline__ bool decode_block_add(R& r, int minexp, T acc[64], const uint8_t* sq, bool rel) {
  typedef typename FT<T>::U U;
  constexpr int P = FT<T>::P;
  constexpr int EB = FT<T>::EBITS;
  const uint32_t h = r.peek32();
  if (!(h & 1u)) {  // empty: x_i = 0 leaves x~ unchanged
    r.skip(1);
    return true;
  }
  if (h & 2u) {  // raw block
    r.skip(2);
#pragma unroll
    for (int l = 0; l < 64; ++l) {
      T v = from_raw((U)r.get64((uint32_t)P), (T)0);
      acc[l] = acc[l] + v;
    }
    return true;
  }
  // unary escalation count, then the biased block exponent
  int delta = (int)__builtin_ctz(~(h >> 2) | 0x40000000u);
  int emax;
  if (3 + delta + EB <= 32) {
    emax = (int)((h >> (3 + delta)) & ((1u << EB) - 1u)) - FT<T>::BIAS;
    r.skip((uint32_t)(3 + delta + EB));
  } else {
    r.skip(2);
    delta = 0;
#pragma unroll 1
    while (r.get(1)) {  // (rare: a long escalation; kept as a loop)
      if (++delta > P) return false;
    }
    emax = (int)r.get((uint32_t)EB) - FT<T>::BIAS;
  }
  int p = emax - minexp + kGuard;
  p = (p < 0 ? 0 : (p > P ? P : p)) + delta;
  if (emax < 2 - FT<T>::BIAS || p < 1 || p > P) return false;
  // Leading empty planes: until a coefficient is significant, a plane
  // without a new one is a single 0 (its negative group test), so the first
  // zeros of the block's plane data are that many empty planes, skipped at once.
  const int z0 = (int)__builtin_ctz(r.peek32() | 0x80000000u);
  const int zlead = z0 < p ? z0 : p;
  r.skip((uint32_t)zlead);
  if constexpr (sizeof(T) == 8 && kRoute == kRouteAuto) {
    // residual components whose coded planes all lie in the top ten bit
    // positions and keep every result normal: the lifting on the words' top
    // 16 bits, two per register, from 4 or 8 slots (wave-uniform choices)
    if (rel && __all(p <= 10 && emax >= -1008)) {
      const int np = p - zlead;
      v2s R2[32];
      if (__all(np <= 4)) {
        slots_hi16<4>(r, p, zlead, sq, R2);
        lift_dequant_add_hi16(R2, emax, acc);
        return true;
      }
      if (__all(np <= 8)) {
        slots_hi16<8>(r, p, zlead, sq, R2);
        lift_dequant_add_hi16(R2, emax, acc);
        return true;
      }
    }
    // every coded plane in the top 26 bit positions and every result
    // normal: the lifting on the coefficients' high words (a wave-uniform
    // choice; both routes give the same sums)
    if (__all(p <= 26 && emax >= -992)) {
      const int np = p - zlead;
      if (__all(np <= 4)) decode_hi32<4>(r, p, zlead, emax, acc, sq, rel);
      else if (__all(np <= 8)) decode_hi32<8>(r, p, zlead, emax, acc, sq, rel);
      else decode_hi32<16>(r, p, zlead, emax, acc, sq, rel);
      return true;
    }
  }
  if constexpr (sizeof(T) == 4 && kRoute == kRouteHi16) {
    // residual components (rel): the packed pairs straight from 4 or 8
    // slots, else from the 32-bit words of 16
    v2s R2[32];
    const int np = p - zlead;
    if (__all(np <= 4)) {
      slots_hi16<4>(r, p, zlead, sq, R2);
    } else if (__all(np <= 8)) {
      slots_hi16<8>(r, p, zlead, sq, R2);
    } else {
      typename FT<T>::S c[64];
      planes_slots<T, 16>(r, c, p, zlead, sq, rel);
      pack_hi16(c, R2);
    }
    lift_dequant_add_hi16(R2, emax, acc);
    return true;
  }
  typename FT<T>::S c[64], q[64];
  planes_read<T>(r, c, p, zlead, sq, rel);
  inverse_zy_ints<T>(c, q);
  inverse_x<T>(q);
  dequant_add(q, emax, acc);
  return true;
}

// words of one wave's four chunks staged in LDS per component (13.3 KB, so
// that 12 one-wave workgroups fit a CU's LDS); spans larger than this use
// the global-memory reader (the host picks the variant from the largest span
// of the streams it decodes)
constexpr uint32_t kStageWords = 3326;
// The staging buffer is double-buffered while spans are small: two halves of
// kHalfWords data words (64-word multiples, since a copy writes whole 64-word
// rows) plus 3 spare words each for the reader's look-ahead.  The next
// component's words load into one half while the wave decodes from the other.
// A component whose span exceeds a half uses the whole buffer and is staged
// without overlap.
constexpr uint32_t kHalfWords = 1600;
constexpr uint32_t kHalf1 = kHalfWords + 3;  // word offset of the second half
static_assert(kHalf1 + kHalfWords + 3 <= kStageWords + 3, "halves fit the buffer");

// the wave's span of payload words of one component: its chunks [4w, 4w + 4)
// are consecutive in the payload
struct Span {
  uint64_t s0, s1;
  bool ok;
};
__device__ __forceinline__ Span wave_span(const uint32_t* index, uint64_t nchunks, uint64_t words, uint64_t w) {
  const uint64_t c0 = w * 4, c1 = min<uint64_t>(c0 + 4, nchunks);
  Span sp;
  sp.s0 = index[c0];
  sp.s1 = c1 < nchunks ? (uint64_t)index[c1] : words;
  sp.ok = sp.s0 <= sp.s1 && sp.s1 <= words && sp.s1 - sp.s0 <= kStageWords;
  return sp;
}
// issue (not wait for) the copy of a span into the staging words at `base`
__device__ __forceinline__ void stage_span(const uint32_t* payload, const Span& sp, uint32_t* stage, uint32_t base) {
  const uint32_t lane = threadIdx.x;
  const uint32_t span = (uint32_t)(sp.s1 - sp.s0);
  for (uint32_t k = 0; k < span; k += 64) {
    const uint32_t j = k + lane < span ? k + lane : span - 1;
    __builtin_amdgcn_global_load_lds((gmem_void_t*)(payload + sp.s0 + j), (lds_void_t*)(stage + base + k), 4, 0, 0);
  }
}

// decode the wave's 64 blocks [64 w, 64 w + 64) of a field: x~ = in (or +0)
// plus components [0, ncomp) of the given streams, left to right.  Every lane
// runs the component loop (the staging copies are shared); false on a
// malformed stream.  kFull: every block of the field is full and rows are
// aligned (all dimensions multiples of 4): no per-lane edge paths.
// one block of one component, codec 0 (minexp) or codec 1 (step = 2 tau)
template <class T, int kCodec, int kRoute = kRouteAuto, class R>
__device__ __forceinline__ bool decode_block_codec(R& r, int minexp, double step, T acc[64], const uint8_t* sq,
                                                   bool rel) {
  if constexpr (kCodec == 0) return decode_block_add<T, kRoute>(r, minexp, acc, sq, rel);
  else return pq_decode_add<T>(r, step, acc);
}

template <class T, bool kStaged, bool kBox = false, bool kFull = false, int kCodec = 0, bool kHiRes = false>
__device__ __forceinline__ bool decode_wave(const Geo& g, const uint8_t* const* s, const uint32_t* const* aux,
                                            const uint64_t* words, const int* minexp, const double* step, int ncomp,
                                            uint32_t relmask, const T* in, T* out, uint64_t w, const uint8_t* sq,
                                            uint32_t* stage, const BoxArgs* box = nullptr) {
  const uint32_t lane = threadIdx.x;
  const uint64_t blk = w * 64 + lane;
  bool active = blk < g.nblocks;
  BlockPos bp = block_pos(g, active ? blk : 0);
  if constexpr (kFull) {
    bp.vx = 4;
    bp.vy = 4;
    bp.vz = 4;
  }
  if constexpr (kBox) {  // only this row's blocks in the box are decoded (each by
                         // one workgroup); the wave still stages its chunks,
                         // whose bit offsets locate every block
    active = active && blk >= box->row_first && blk <= box->row_last;
  }
  const uint64_t chunk = blk / kChunkBlocks;
  T acc[64];
  if (in && active) {
    if constexpr (kBox) load_box(in, *box, bp, acc);
    else if constexpr (kFull) load_rows<T, 16>(in, g, opaque_pos(bp), 0, true, acc);
    else load_block(in, g, opaque_pos(bp), acc);
  } else {
#pragma unroll
    for (int l = 0; l < 64; ++l) acc[l] = (T)0;
  }
  bool ok = true;
  if constexpr (kStaged) {
    // component i: its span, where it sits in LDS, and this lane's chunk range
    // and bit offset (loaded together with the span's words)
    Span cur{0, 0, false};
    uint32_t cur_base = 0, cur_cap = kStageWords;
    uint32_t start = 0, stop = 0, off = 0;  // word offsets (a payload has < 2^32 words) and bit offset
    if (ncomp > 0) {
      const uint32_t* index = reinterpret_cast<const uint32_t*>(s[0] + kHeaderBytes);
      cur = wave_span(index, g.nchunks, words[0], w);
      cur_cap = cur.s1 - cur.s0 <= kHalfWords ? kHalfWords : kStageWords;
      if (cur.ok) stage_span(index + g.nchunks, cur, stage, 0);
      if (active) {
        start = index[chunk];
        stop = chunk + 1 < g.nchunks ? index[chunk + 1] : (uint32_t)min<uint64_t>(words[0], 0xFFFFFFFFull);
        off = aux[0][blk];
      }
    }
    auto component = [&](int i, auto route) {
        __builtin_amdgcn_s_waitcnt(0);  // component i's words and lane values
        __syncthreads();
        // the next component: into the other half while this one decodes, when
        // both fit a half
        Span nxt{0, 0, false};
        uint32_t nxt_base = 0, nxt_cap = kStageWords;
        uint32_t nstart = 0, nstop = 0, noff = 0;
        bool pre = false;
        const uint32_t* nindex = nullptr;
        if (i + 1 < ncomp) {
          nindex = reinterpret_cast<const uint32_t*>(s[i + 1] + kHeaderBytes);
          nxt = wave_span(nindex, g.nchunks, words[i + 1], w);
          pre = nxt.ok && cur.ok && cur.s1 - cur.s0 <= kHalfWords && nxt.s1 - nxt.s0 <= kHalfWords;
          if (pre) {
            nxt_base = cur_base == 0 ? kHalf1 : 0;
            nxt_cap = kHalfWords;
            stage_span(nindex + g.nchunks, nxt, stage, nxt_base);
            if (active) {
              nstart = nindex[chunk];
              nstop = chunk + 1 < g.nchunks ? nindex[chunk + 1] : (uint32_t)min<uint64_t>(words[i + 1], 0xFFFFFFFFull);
              noff = aux[i + 1][blk];
            }
          }
        }
        if (active && ok) {
          if (!cur.ok || words[i] > 0xFFFFFFFFull || start > stop || stop > words[i] ||
              off >= (uint64_t)(stop - start) * 32 || start < cur.s0 || stop > cur.s1) {
            ok = false;
          } else {
            const uint32_t s0 = (uint32_t)cur.s0;
            LBits r;
            r.init(stage + cur_base, start - s0 + (off >> 5), stop - s0, cur_cap);
            r.skip((uint32_t)(off & 31));
            ok = decode_block_codec<T, kCodec, decltype(route)::value>(r, minexp[i], step[i], acc, sq,
                                                                        (relmask >> i) & 1u) && !r.bad();
          }
        }
        if (i + 1 < ncomp && !pre) {  // staged after this component, into the whole buffer's first half or all of it
          __syncthreads();  // every lane is done with this component's words
          nxt_base = 0;
          nxt_cap = nxt.s1 - nxt.s0 <= kHalfWords ? kHalfWords : kStageWords;
          if (nxt.ok) stage_span(nindex + g.nchunks, nxt, stage, 0);
          if (active) {
            nstart = nindex[chunk];
            nstop = chunk + 1 < g.nchunks ? nindex[chunk + 1] : (uint32_t)min<uint64_t>(words[i + 1], 0xFFFFFFFFull);
            noff = aux[i + 1][blk];
          }
        }
        cur = nxt;
        cur_base = nxt_base;
        cur_cap = nxt_cap;
        start = nstart;
        stop = nstop;
        off = noff;
    };
    if constexpr (kHiRes) {
      // the store's first component (if decoded here) on the full route,
      // the residual ones on the high-half route only
      int i = 0;
      if (ncomp > 0 && !(relmask & 1u)) {
        component(0, std::integral_constant<int, kRouteFull>{});
        i = 1;
      }
      for (; i < ncomp; ++i) component(i, std::integral_constant<int, kRouteHi16>{});
    } else {
      for (int i = 0; i < ncomp; ++i) component(i, std::integral_constant<int, kRouteAuto>{});
    }
  } else {
    for (int i = 0; i < ncomp; ++i) {
      if (!active || !ok) continue;
      const uint32_t* index = reinterpret_cast<const uint32_t*>(s[i] + kHeaderBytes);
      const uint32_t* payload = index + g.nchunks;
      const uint64_t start = index[chunk];
      const uint64_t stop = chunk + 1 < g.nchunks ? (uint64_t)index[chunk + 1] : words[i];
      const uint64_t off = aux[i][blk];
      if (start > stop || stop > words[i] || stop > 0xFFFFFFFFull || off >= (stop - start) * 32) {
        ok = false;
        continue;
      }
      GBits r;
      r.init(payload, (uint32_t)(start + (off >> 5)), (uint32_t)stop);
      r.skip((uint32_t)(off & 31));
      ok = decode_block_codec<T, kCodec>(r, minexp[i], step[i], acc, sq, (relmask >> i) & 1u) && !r.bad();
    }
  }
  // a block whose stream did not parse is written as quiet NaNs, so the
  // output never keeps stale memory (the status word reports it as well)
  if (active && !ok) {
#pragma unroll
    for (int l = 0; l < 64; ++l) acc[l] = (T)__builtin_nan("");
  }
  // the block position is recomputed here rather than kept in registers
  if (active) {
    if constexpr (kBox) {
      store_box(out, *box, block_pos(g, opaque(w) * 64 + lane), acc);
    } else if constexpr (kFull) {
      const BlockPos bo = block_pos(g, opaque(w) * 64 + lane);
#pragma unroll
      for (int r = 0; r < 16; ++r) store_row(out, g, bo, r, acc + 4 * r, true);
    } else {
      store_block(out, g, block_pos(g, opaque(w) * 64 + lane), acc);
    }
  }
  return ok || !active;
}

// kHiRes: the launch's residual components decode on the float32 high-half
// route alone (the host has checked that every block of them qualifies)
template <class T, bool kStaged, bool kFull, int kCodec, bool kHiRes = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_decode(DecArgs<T> a) {
  __shared__ uint8_t s_squeeze[256];
  __shared__ uint32_t s_stage[kStaged ? kStageWords + 3 : 1];
  squeeze_table(s_squeeze);
  if (!decode_wave<T, kStaged, false, kFull, kCodec, kHiRes>(a.g, a.s, a.aux, a.words, a.minexp, a.step, a.ncomp, a.relmask,
                                                     a.in, a.out, blockIdx.x, s_squeeze, s_stage))
    atomicOr(a.status, 1u);
}

// region retrieval: workgroup (row, i) decodes the i-th wave of the box's
// block row `row` (rows in y-then-z order); waves past the row's last block
// exit.  a.in / a.out are box arrays (a.in: the box after earlier components).
// A wave whose blocks span several box rows (narrow fields) is staged once
// per row, and each row's workgroup decodes only that row's blocks.
template <class T, bool kStaged, int kCodec>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_decode_box(
    DecArgs<T> a, BoxArgs b) {
  __shared__ uint8_t s_squeeze[256];
  __shared__ uint32_t s_stage[kStaged ? kStageWords + 3 : 1];
  const uint32_t row = blockIdx.x / b.waves_per_row, i = blockIdx.x % b.waves_per_row;
  const uint64_t nry = b.bhi[1] - b.blo[1];
  const uint64_t by = b.blo[1] + row % nry, bz = b.blo[2] + row / nry;
  b.row_first = (bz * a.g.nby + by) * a.g.nbx + b.blo[0];
  b.row_last = (bz * a.g.nby + by) * a.g.nbx + b.bhi[0] - 1;
  const uint64_t w = b.row_first / 64 + i;
  if (w > b.row_last / 64) return;  // uniform over the workgroup
  squeeze_table(s_squeeze);
  if (!decode_wave<T, kStaged, true, false, kCodec>(a.g, a.s, a.aux, a.words, a.minexp, a.step, a.ncomp, a.relmask,
                                                    a.in, a.out, w, s_squeeze, s_stage, &b))
    atomicOr(a.status, 1u);
}

// many retrieval queries in one launch: wave w belongs to the query q with
// wave_prefix[q] <= w < wave_prefix[q + 1]
template <class T, bool kStaged, int kCodec, bool kHiRes = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_decode_queries(ServeArgs a) {
  __shared__ uint8_t s_squeeze[256];
  __shared__ uint32_t s_stage[kStaged ? kStageWords + 3 : 1];
  squeeze_table(s_squeeze);
  const uint32_t w = blockIdx.x;
  uint32_t lo = 0, hi = a.nq;  // largest q with wave_prefix[q] <= w
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (a.wave_prefix[mid] <= w) lo = mid;
    else hi = mid;
  }
  // the query table is read-only for the launch: read through the constant
  // address space, so its values can be loaded again where needed instead of
  // being held across the wave's work
  typedef __attribute__((address_space(4))) const QueryDev CQueryDev;
  const CQueryDev& q = ((const CQueryDev*)a.q)[lo];
  Geo g;
  g.nx = q.g.nx;
  g.ny = q.g.ny;
  g.nz = q.g.nz;
  g.nbx = q.g.nbx;
  g.nby = q.g.nby;
  g.nbz = q.g.nbz;
  g.nblocks = q.g.nblocks;
  g.nchunks = q.g.nchunks;
  g.rows_aligned = q.g.rows_aligned;
  g.pad = 0;
  if (!decode_wave<T, kStaged, false, false, kCodec, kHiRes>(
          g, (const uint8_t* const*)q.s, (const uint32_t* const*)q.aux, (const uint64_t*)q.words,
          (const int*)q.minexp, (const double*)q.step, q.ncomp, q.relmask, reinterpret_cast<const T*>(q.in),
          reinterpret_cast<T*>(q.out), w - a.wave_prefix[lo], s_squeeze, s_stage))
    atomicOr(a.status, 1u);
}

// per-block bit offsets of a stream written elsewhere: parse each chunk
template <class T, int kCodec>
__global__ __launch_bounds__(64) void k_aux(AuxArgs a) {
  __shared__ uint8_t s_squeeze[256];
  squeeze_table(s_squeeze);
  const uint64_t chunk = (uint64_t)blockIdx.x * 64 + threadIdx.x;
  if (chunk >= a.g.nchunks) return;
  const uint32_t* index = reinterpret_cast<const uint32_t*>(a.s + kHeaderBytes);
  const uint32_t* payload = index + a.g.nchunks;
  const uint64_t start = index[chunk];
  const uint64_t stop = chunk + 1 < a.g.nchunks ? (uint64_t)index[chunk + 1] : a.words;
  // a chunk holds at least one block, hence at least one bit
  bool ok = start < stop && stop <= a.words && stop <= 0xFFFFFFFFull;
  GBits r;
  r.init(payload, (uint32_t)start, (uint32_t)(ok ? stop : start));
  const uint64_t b0 = chunk * kChunkBlocks, b1 = min<uint64_t>(a.g.nblocks, b0 + kChunkBlocks);
  bool any_full = false;
  for (uint64_t blk = b0; blk < b1; ++blk) {
    a.aux[blk] = ok ? (uint32_t)r.consumed((uint32_t)start) : 0u;
    bool full = false;
    if (ok) ok = (kCodec == 0 ? block_skip<T>(r, a.minexp, s_squeeze, full) : pq_block_skip<T>(r)) && !r.bad();
    any_full = any_full || full;
  }
  if (!ok && a.status) atomicOr(a.status, 1u);
  if (any_full && a.full && *(volatile unsigned long long*)a.full == 0) atomicOr(a.full, 1ull);
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ordered(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// min / max over the finite samples and the count of the others.  Keys are
// the samples' bits mapped to unsigned integers of the same order (sign and
// zero sign included), so the reduction is exact integer min / max in the
// field's own width; the per-wave result is widened to the double key of the
// same value for the device-wide atomics.  16-byte loads when aligned.
template <class T> struct RangeKey;
template <> struct RangeKey<float> {
  typedef uint32_t K;
  static __device__ __forceinline__ K key(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b >> 31) ? ~b : (b | 0x80000000u);
  }
  static __device__ __forceinline__ bool finite(float v) { return (__float_as_uint(v) & 0x7F800000u) != 0x7F800000u; }
  static __device__ __forceinline__ double value(K k) {
    return (double)__uint_as_float((k >> 31) ? (k & 0x7FFFFFFFu) : ~k);
  }
};
template <> struct RangeKey<double> {
  typedef unsigned long long K;
  static __device__ __forceinline__ K key(double v) { return ordered(v); }
  static __device__ __forceinline__ bool finite(double v) {
    return ((unsigned long long)__double_as_longlong(v) & 0x7FF0000000000000ull) != 0x7FF0000000000000ull;
  }
  static __device__ __forceinline__ double value(K k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k));
  }
};

template <class T>
__global__ __launch_bounds__(256) void k_range(const T* __restrict__ x, uint64_t n, unsigned long long* out) {
  typedef RangeKey<T> RK;
  typedef typename RK::K K;
  K lo = ~(K)0, hi = 0;
  uint32_t bad = 0;
  auto take = [&](T v) {
    const K k = RK::key(v);
    const bool fin = RK::finite(v);
    lo = fin && k < lo ? k : lo;
    hi = fin && k > hi ? k : hi;
    bad += fin ? 0u : 1u;
  };
  const uint64_t tid = (uint64_t)blockIdx.x * 256 + threadIdx.x, stride = (uint64_t)gridDim.x * 256;
  constexpr uint64_t V = 16 / sizeof(T);  // samples per 16-byte load
  uint64_t done = 0;
  if (((uintptr_t)x & 15) == 0) {
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V16;
    const V16* xv = reinterpret_cast<const V16*>(x);
    auto take16 = [&](const V16& v) {
      if constexpr (sizeof(T) == 4) {
        take(v.x);
        take(v.y);
        take(v.z);
        take(v.w);
      } else {
        take(v.x);
        take(v.y);
      }
    };
    const uint64_t nv = n / V;
    uint64_t i = tid;
    for (; i + 3 * stride < nv; i += 4 * stride) {  // four 16-byte loads in flight
      const V16 a0 = xv[i], a1 = xv[i + stride], a2 = xv[i + 2 * stride], a3 = xv[i + 3 * stride];
      take16(a0);
      take16(a1);
      take16(a2);
      take16(a3);
    }
    for (; i < nv; i += stride) take16(xv[i]);
    done = nv * V;
  }
  for (uint64_t i = done + tid; i < n; i += stride) take(x[i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const K a = __shfl_xor(lo, d, 64), b = __shfl_xor(hi, d, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
    bad += __shfl_xor(bad, d, 64);
  }
  // the workgroup's four waves, then one set of atomics per workgroup (each
  // skipped when the device-wide value is already at least as extreme)
  __shared__ K s_lo[4], s_hi[4];
  __shared__ uint32_t s_bad[4];
  const uint32_t wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wv] = lo;
    s_hi[wv] = hi;
    s_bad[wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      lo = s_lo[k] < lo ? s_lo[k] : lo;
      hi = s_hi[k] > hi ? s_hi[k] : hi;
      bad += s_bad[k];
    }
    if (lo != ~(K)0) {  // this workgroup saw a finite sample
      const unsigned long long ol = ordered(RK::value(lo)), oh = ordered(RK::value(hi));
      if (ol < *(volatile unsigned long long*)&out[0]) atomicMin(&out[0], ol);
      if (oh > *(volatile unsigned long long*)&out[1]) atomicMax(&out[1], oh);
    }
    if (bad) atomicAdd(&out[2], (unsigned long long)bad);
  }
}

// p[0, n) = v, except p[j] = vj (j >= n: none)
__global__ void k_fill64(unsigned long long* p, uint64_t n, unsigned long long v, uint64_t j, unsigned long long vj) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i == j ? vj : v;
}

// ---------------------------------------------------------------------------
// batches: many fields of mixed size and type in persistent launches.  Work
// is listed as items; each workgroup walks the list with a static stride, so
// a field's bytes depend only on its own blocks, never on the schedule.
template <class T, class F> __device__ __forceinline__ EncArgs<T> field_enc_args(const F& f, int comp) {
  EncArgs<T> a;
  a.x = reinterpret_cast<const T*>(f.x);
  a.xt_in = reinterpret_cast<const T*>(comp > 0 ? f.xt[(comp - 1) & 1] : nullptr);
  a.xt_out = reinterpret_cast<T*>(f.xt[comp & 1]);
  // member by member: F may live in the constant address space
  a.g.nx = f.g.nx;
  a.g.ny = f.g.ny;
  a.g.nz = f.g.nz;
  a.g.nbx = f.g.nbx;
  a.g.nby = f.g.nby;
  a.g.nbz = f.g.nbz;
  a.g.nblocks = f.g.nblocks;
  a.g.nchunks = f.g.nchunks;
  a.g.rows_aligned = f.g.rows_aligned;
  a.g.pad = 0;
  a.tau = f.tau[comp];
  a.minexp = f.minexp[comp];
  a.first = comp == 0;
  a.last = comp == f.ncomp - 1;
  a.staging = f.staging;
  a.chunk_words = f.chunk_words;
  a.aux = f.aux0 + (uint64_t)comp * f.aux_stride;
  a.meta = f.meta0 + comp;
  a.berr = f.berr;
  return a;
}

template <class T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void k_encode_batch(BatchArgs b) {
  __shared__ T s_x[64 * 64];
  __shared__ uint16_t s_unsq[256];
  unsqueeze_table(s_unsq);
  // the field table is read-only for the launch: read through the constant
  // address space, so its values can be loaded again where needed instead of
  // being held across the wave's work
  typedef __attribute__((address_space(4))) const FieldDev CFieldDev;
  const CFieldDev* const fields = (const CFieldDev*)b.fields;
  for (uint32_t it = blockIdx.x; it < b.nitems; it += gridDim.x) {
    const Item w = b.items[it];
    const CFieldDev& f = fields[w.field];
    if (b.comp < f.ncomp) encode_wave<T, false, 0, false>(field_enc_args<T>(f, b.comp), w.index, s_x, s_unsq);
    __syncthreads();  // the next item reuses s_x
  }
}

// stream bookkeeping at the start: component 0's stream follows the field's
// block indexes
__global__ void k_batch_init(const FieldDev* fields, uint32_t nfields) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfields) return;
  const FieldDev& d = fields[f];
  for (int i = 0; i < d.ncomp; ++i) {
    unsigned long long* m = reinterpret_cast<unsigned long long*>(d.meta0 + i);
    for (int w = 0; w < (int)(sizeof(CompMeta) / 8); ++w) m[w] = 0ull;
  }
  d.meta0[0].stream_offset = (unsigned long long)d.ncomp * d.aux_stride * 4ull;
}

__global__ __launch_bounds__(1024) void k_btile_sums(BatchArgs b) {
  __shared__ unsigned long long sh[16];
  const Item t = b.items[blockIdx.x];
  const FieldDev& f = b.fields[t.field];
  if (b.comp >= f.ncomp) return;  // uniform across the workgroup
  const uint64_t i = (uint64_t)t.index * kScanTile + threadIdx.x;
  unsigned long long v = i < f.g.nchunks ? f.chunk_words[i] : 0ull;
  v = block_incl_scan(v, sh);
  if (threadIdx.x == kScanTile - 1) f.tile_sums[t.index] = v;
}

__global__ __launch_bounds__(1024) void k_btile_scan(BatchArgs b) {
  __shared__ unsigned long long sh[16];
  const FieldDev& f = b.fields[blockIdx.x];
  if (b.comp >= f.ncomp) return;
  unsigned long long carry = 0;
  for (uint64_t base = 0; base < f.ntiles; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    unsigned long long v = i < f.ntiles ? f.tile_sums[i] : 0ull;
    unsigned long long inc = block_incl_scan(v, sh);
    if (i < f.ntiles) f.tile_sums[i] = carry + inc - v;
    carry += sh[15];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    CompMeta* m = f.meta0 + b.comp;
    const unsigned long long words = carry;
    const unsigned long long bytes = (unsigned long long)kHeaderBytes + 4ull * f.g.nchunks + 4ull * words;
    m->payload_words = words;
    m->stream_bytes = bytes;
    const unsigned long long end = m->stream_offset + bytes;
    if (end > f.region_cap) m->flags |= FLAG_OVERFLOW;
    if (words > 0xFFFFFFFFull) m->flags |= FLAG_INDEX;
    if (b.comp + 1 < f.ncomp) f.meta0[b.comp + 1].stream_offset = (end + 255ull) & ~255ull;
  }
}

__global__ __launch_bounds__(1024) void k_btile_offsets(BatchArgs b) {
  __shared__ unsigned long long sh[16];
  const Item t = b.items[blockIdx.x];
  const FieldDev& f = b.fields[t.field];
  if (b.comp >= f.ncomp) return;
  const uint64_t i = (uint64_t)t.index * kScanTile + threadIdx.x;
  unsigned long long v = i < f.g.nchunks ? f.chunk_words[i] : 0ull;
  unsigned long long inc = block_incl_scan(v, sh);
  if (i < f.g.nchunks) f.offsets[i] = (uint32_t)(f.tile_sums[t.index] + inc - v);
}

__global__ __launch_bounds__(64) void k_bpack(BatchArgs b) {
  const Item q = b.items[blockIdx.x];
  const FieldDev& f = b.fields[q.field];
  if (b.comp >= f.ncomp) return;
  const CompMeta* m = f.meta0 + b.comp;
  if (m->flags & (FLAG_OVERFLOW | FLAG_INDEX)) return;
  const uint64_t cap = f.dtype == 1 ? (uint64_t)chunk_cap_words<float>() : (uint64_t)chunk_cap_words<double>();
  uint8_t* base = f.region + m->stream_offset;
  uint32_t* index = reinterpret_cast<uint32_t*>(base + kHeaderBytes);
  uint32_t* payload = index + f.g.nchunks;
  const uint32_t lane = threadIdx.x;
  const uint32_t span =
      pack_quad(f.staging, cap, f.chunk_words, f.offsets, f.g.nchunks, (uint64_t)q.index * 4, payload, index);
  if (lane == 0 && span > *(volatile unsigned long long*)&f.meta0[b.comp].max_span)
    atomicMax(&f.meta0[b.comp].max_span, (unsigned long long)span);
  if (q.index == 0 && lane < 16) {
    uint32_t* h = reinterpret_cast<uint32_t*>(base);
    const double tau = f.tau[b.comp];
    const uint64_t taub = (uint64_t)__double_as_longlong(tau);
    uint32_t v = 0;
    switch (lane) {
      case 0: v = kMagic; break;
      case 1: v = (uint32_t)kVersion | ((uint32_t)f.dtype << 16) | (3u << 24); break;
      case 2: v = (uint32_t)f.g.nx; break;
      case 3: v = (uint32_t)(f.g.nx >> 32); break;
      case 4: v = (uint32_t)f.g.ny; break;
      case 5: v = (uint32_t)(f.g.ny >> 32); break;
      case 6: v = (uint32_t)f.g.nz; break;
      case 7: v = (uint32_t)(f.g.nz >> 32); break;
      case 8: v = (uint32_t)taub; break;
      case 9: v = (uint32_t)(taub >> 32); break;
      case 10: v = (uint32_t)f.minexp[b.comp]; break;
      case 11: v = (uint32_t)kChunkBlocks; break;
      case 12: v = (uint32_t)f.g.nchunks; break;
      case 13: v = (uint32_t)(f.g.nchunks >> 32); break;
      case 14: v = (uint32_t)m->payload_words; break;
      case 15: v = (uint32_t)(m->payload_words >> 32); break;
    }
    h[lane] = v;
  }
}

// ---------------------------------------------------------------------------
// host launchers
template <class T> hipError_t launch_encode(const EncArgs<T>& a, int codec, hipStream_t s) {
  const uint64_t wgs = (a.g.nblocks + 63) / 64;
  // every block full and every row aligned: the kernel without edge paths
  const bool full = a.g.nx % 4 == 0 && a.g.ny % 4 == 0 && a.g.nz % 4 == 0 && a.g.rows_aligned;
  const dim3 grid((uint32_t)wgs), wg(64);
  if (codec == 0) {
    if (full) hipLaunchKernelGGL((k_encode<T, true, 0>), grid, wg, 0, s, a);
    else hipLaunchKernelGGL((k_encode<T, false, 0>), grid, wg, 0, s, a);
  } else {
    if (full) hipLaunchKernelGGL((k_encode<T, true, 1>), grid, wg, 0, s, a);
    else hipLaunchKernelGGL((k_encode<T, false, 1>), grid, wg, 0, s, a);
  }
  return hipGetLastError();
}
hipError_t launch_scan(const ScanArgs& a, hipStream_t s) {
  const uint64_t tiles = (a.nchunks + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_tile_sums, dim3((uint32_t)tiles), dim3(kScanTile), 0, s, a);
  hipLaunchKernelGGL(k_tile_offsets, dim3((uint32_t)tiles), dim3(kScanTile), 0, s, a);
  return hipGetLastError();
}
template <class T> hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  const uint64_t quads = (a.nchunks + 3) / 4;
  const uint64_t wgs = quads < 8192 ? quads : 8192;
  hipLaunchKernelGGL(k_pack<T>, dim3((uint32_t)wgs), dim3(64), 0, s, a);
  return hipGetLastError();
}
uint64_t stage_words() { return kStageWords; }
template <class T, int kCodec>
void launch_decode_codec(const DecArgs<T>& a, uint64_t max_span, bool hires, hipStream_t s) {
  const uint64_t wgs = (a.g.nblocks + 63) / 64;
  const dim3 grid((uint32_t)wgs), wg(64);
  // every block full and every row aligned: the kernel without edge paths
  const bool full = a.g.nx % 4 == 0 && a.g.ny % 4 == 0 && a.g.nz % 4 == 0 && a.g.rows_aligned;
  if constexpr (sizeof(T) == 4 && kCodec == 0) {
    if (hires && max_span <= kStageWords) {
      if (full) hipLaunchKernelGGL((k_decode<T, true, true, kCodec, true>), grid, wg, 0, s, a);
      else hipLaunchKernelGGL((k_decode<T, true, false, kCodec, true>), grid, wg, 0, s, a);
      return;
    }
  }
  if (max_span <= kStageWords) {
    if (full) hipLaunchKernelGGL((k_decode<T, true, true, kCodec>), grid, wg, 0, s, a);
    else hipLaunchKernelGGL((k_decode<T, true, false, kCodec>), grid, wg, 0, s, a);
  } else {
    if (full) hipLaunchKernelGGL((k_decode<T, false, true, kCodec>), grid, wg, 0, s, a);
    else hipLaunchKernelGGL((k_decode<T, false, false, kCodec>), grid, wg, 0, s, a);
  }
}
template <class T>
hipError_t launch_decode(const DecArgs<T>& a, uint64_t max_span, int codec, bool hires, hipStream_t s) {
  if (codec == 0) launch_decode_codec<T, 0>(a, max_span, hires, s);
  else launch_decode_codec<T, 1>(a, max_span, false, s);
  return hipGetLastError();
}
template <class T>
hipError_t launch_decode_box(const DecArgs<T>& a, const BoxArgs& b, uint64_t max_span, int codec, hipStream_t s) {
  const uint64_t rows = (b.bhi[1] - b.blo[1]) * (b.bhi[2] - b.blo[2]);
  const uint64_t wgs = rows * b.waves_per_row;
  if (wgs == 0) return hipSuccess;
  const dim3 grid((uint32_t)wgs), wg(64);
  const bool staged = max_span <= kStageWords;
  if (codec == 0) {
    if (staged) hipLaunchKernelGGL((k_decode_box<T, true, 0>), grid, wg, 0, s, a, b);
    else hipLaunchKernelGGL((k_decode_box<T, false, 0>), grid, wg, 0, s, a, b);
  } else {
    if (staged) hipLaunchKernelGGL((k_decode_box<T, true, 1>), grid, wg, 0, s, a, b);
    else hipLaunchKernelGGL((k_decode_box<T, false, 1>), grid, wg, 0, s, a, b);
  }
  return hipGetLastError();
}
template <class T>
hipError_t launch_decode_queries(const ServeArgs& a, uint64_t max_span, int codec, bool hires, hipStream_t s) {
  if (a.nwaves == 0) return hipSuccess;
  const dim3 grid(a.nwaves), wg(64);
  const bool staged = max_span <= kStageWords;
  if constexpr (sizeof(T) == 4) {
    if (codec == 0 && hires && staged) {
      hipLaunchKernelGGL((k_decode_queries<T, true, 0, true>), grid, wg, 0, s, a);
      return hipGetLastError();
    }
  }
  if (codec == 0) {
    if (staged) hipLaunchKernelGGL((k_decode_queries<T, true, 0>), grid, wg, 0, s, a);
    else hipLaunchKernelGGL((k_decode_queries<T, false, 0>), grid, wg, 0, s, a);
  } else {
    if (staged) hipLaunchKernelGGL((k_decode_queries<T, true, 1>), grid, wg, 0, s, a);
    else hipLaunchKernelGGL((k_decode_queries<T, false, 1>), grid, wg, 0, s, a);
  }
  return hipGetLastError();
}
// ---------------------------------------------------------------------------
// sums of d = a - b - shift and of d^2 in float64 over a field (b NULL: 0),
// for the accuracy gain of Sec. 5.1.1 (standard deviation of the data,
// root-mean-square error of a reconstruction).  Deterministic: each
// workgroup reduces a fixed grid-stride share in a fixed order into its own
// partial pair, and one workgroup then adds the partials in index order.
constexpr int kSumGroups = 1024;  // workgroups of the first stage (the partials)

__device__ __forceinline__ void block_sum2(double& s, double& q, double* sh) {
  const uint32_t t = threadIdx.x;
  sh[t] = s;
  sh[256 + t] = q;
  __syncthreads();
  for (uint32_t h = 128; h > 0; h >>= 1) {
    if (t < h) {
      sh[t] = sh[t] + sh[t + h];
      sh[256 + t] = sh[256 + t] + sh[256 + t + h];
    }
    __syncthreads();
  }
  s = sh[0];
  q = sh[256];
}

template <class T>
__global__ __launch_bounds__(256) void k_sum_sq(const T* __restrict__ a, const T* __restrict__ b, double shift,
                                                uint64_t n, double* partials) {
  __shared__ double sh[512];
  double s = 0.0, q = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const double d = ((double)a[i] - (b ? (double)b[i] : 0.0)) - shift;
    s = s + d;
    q = q + d * d;
  }
  block_sum2(s, q, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s;
    partials[2 * blockIdx.x + 1] = q;
  }
}

__global__ __launch_bounds__(256) void k_sum_sq_final(const double* partials, uint32_t groups, double* out) {
  __shared__ double sh[512];
  double s = 0.0, q = 0.0;
  for (uint32_t g = threadIdx.x; g < groups; g += 256) {
    s = s + partials[2 * g];
    q = q + partials[2 * g + 1];
  }
  block_sum2(s, q, sh);
  if (threadIdx.x == 0) {
    out[0] = s;
    out[1] = q;
  }
}

template <class T>
hipError_t launch_sum_sq(const T* a, const T* b, double shift, uint64_t n, double* ws, double* out, hipStream_t s) {
  uint64_t groups = (n + 255) / 256;
  if (groups > kSumGroups) groups = kSumGroups;
  if (groups == 0) groups = 1;
  hipLaunchKernelGGL(k_sum_sq<T>, dim3((uint32_t)groups), dim3(256), 0, s, a, b, shift, n, ws);
  hipLaunchKernelGGL(k_sum_sq_final, dim3(1), dim3(256), 0, s, ws, (uint32_t)groups, out);
  return hipGetLastError();
}
uint64_t sum_sq_ws_bytes() { return (uint64_t)kSumGroups * 16 + 256; }

// ---------------------------------------------------------------------------
// Sec. 3's scalar special case as a second compressor behind the same
// driver: C(e) = fl32(e) (round to nearest even float32), D(y) = y in the
// field's type.  One thread per value runs all n components of Alg. 1 in
// registers: e = x - x~ in the field's type, y = fl32(e), x~ = x~ + y; the
// measured errors max |x - x~_i| (float64) are raised per wave with atomics on
// their bit patterns (non-negative doubles order like their bits).
// (NC: a compile-time bound on n, so that the per-component maxima have fixed
// registers; launched with the smallest of 4, 8, 32 that holds n)
template <class T, int NC>
__global__ __launch_bounds__(256) void k_cast_encode(const T* __restrict__ x, uint64_t N, int n,
                                                     float* __restrict__ comps, unsigned long long* linf_bits) {
  double mx[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) mx[i] = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < N; j += stride) {
    const T xj = x[j];
    T xt = (T)0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      if (i < n) {
        const float y = (float)(xj - xt);  // the residual in the field's type, then rounded once
        comps[(uint64_t)i * N + j] = y;
        xt = xt + (T)y;
        const double err = __builtin_fabs((double)xj - (double)xt);
        mx[i] = err > mx[i] ? err : mx[i];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    if (i < n) {
      const double wm = wave_max(mx[i]);
      const unsigned long long wb = (unsigned long long)__double_as_longlong(wm);
      if ((threadIdx.x & 63) == 0 && wb > *(volatile unsigned long long*)&linf_bits[i]) atomicMax(&linf_bits[i], wb);
    }
  }
}
// x~_k = (...((+0 + y_1) + y_2) ...) + y_k in the field's type
template <class T>
__global__ __launch_bounds__(256) void k_cast_decode(const float* __restrict__ comps, uint64_t N, int k,
                                                     T* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < N; j += stride) {
    T acc = (T)0;
    for (int i = 0; i < k; ++i) acc = acc + (T)comps[(uint64_t)i * N + j];
    out[j] = acc;
  }
}
template <class T>
hipError_t launch_cast_encode(const T* x, uint64_t N, int n, float* comps, unsigned long long* linf, hipStream_t s) {
  uint64_t wgs = (N + 255) / 256;
  if (wgs > 4096) wgs = 4096;
  if (wgs == 0) wgs = 1;
  if (n <= 4) hipLaunchKernelGGL((k_cast_encode<T, 4>), dim3((uint32_t)wgs), dim3(256), 0, s, x, N, n, comps, linf);
  else if (n <= 8) hipLaunchKernelGGL((k_cast_encode<T, 8>), dim3((uint32_t)wgs), dim3(256), 0, s, x, N, n, comps, linf);
  else hipLaunchKernelGGL((k_cast_encode<T, kMaxComps>), dim3((uint32_t)wgs), dim3(256), 0, s, x, N, n, comps, linf);
  return hipGetLastError();
}
template <class T> hipError_t launch_cast_decode(const float* comps, uint64_t N, int k, T* out, hipStream_t s) {
  uint64_t wgs = (N + 255) / 256;
  if (wgs > 4096) wgs = 4096;
  if (wgs == 0) wgs = 1;
  hipLaunchKernelGGL(k_cast_decode<T>, dim3((uint32_t)wgs), dim3(256), 0, s, comps, N, k, out);
  return hipGetLastError();
}
template hipError_t launch_cast_encode<float>(const float*, uint64_t, int, float*, unsigned long long*, hipStream_t);
template hipError_t launch_cast_encode<double>(const double*, uint64_t, int, float*, unsigned long long*, hipStream_t);
template hipError_t launch_cast_decode<float>(const float*, uint64_t, int, float*, hipStream_t);
template hipError_t launch_cast_decode<double>(const float*, uint64_t, int, double*, hipStream_t);

template <class T> hipError_t launch_aux(const AuxArgs& a, int codec, hipStream_t s) {
  const uint64_t wgs = (a.g.nchunks + 63) / 64;
  if (codec == 0) hipLaunchKernelGGL((k_aux<T, 0>), dim3((uint32_t)wgs), dim3(64), 0, s, a);
  else hipLaunchKernelGGL((k_aux<T, 1>), dim3((uint32_t)wgs), dim3(64), 0, s, a);
  return hipGetLastError();
}
template <class T> hipError_t launch_range(const T* x, uint64_t n, unsigned long long* out, hipStream_t s) {
  uint64_t wgs = (n + 255) / 256;
  if (wgs > 2048) wgs = 2048;
  if (wgs == 0) wgs = 1;
  hipLaunchKernelGGL(k_range<T>, dim3((uint32_t)wgs), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}
template <class T> hipError_t launch_encode_batch(const BatchArgs& a, uint32_t grid, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode_batch<T>, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_batch_scan(const BatchArgs& tiles, uint32_t nfields, hipStream_t s) {
  hipLaunchKernelGGL(k_btile_sums, dim3(tiles.nitems), dim3(kScanTile), 0, s, tiles);
  hipLaunchKernelGGL(k_btile_scan, dim3(nfields), dim3(1024), 0, s, tiles);
  hipLaunchKernelGGL(k_btile_offsets, dim3(tiles.nitems), dim3(kScanTile), 0, s, tiles);
  return hipGetLastError();
}
hipError_t launch_batch_pack(const BatchArgs& quads, hipStream_t s) {
  hipLaunchKernelGGL(k_bpack, dim3(quads.nitems), dim3(64), 0, s, quads);
  return hipGetLastError();
}
hipError_t launch_batch_init(const FieldDev* fields, uint32_t nfields, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3((nfields + 63) / 64), dim3(64), 0, s, fields, nfields);
  return hipGetLastError();
}
hipError_t launch_fill64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s) {
  return launch_fill64_one(p, n, v, n, v, s);
}
hipError_t launch_fill64_one(unsigned long long* p, uint64_t n, unsigned long long v, uint64_t j,
                             unsigned long long vj, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill64, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n, v, j, vj);
  return hipGetLastError();
}

template hipError_t launch_encode_batch<float>(const BatchArgs&, uint32_t, hipStream_t);
template hipError_t launch_encode_batch<double>(const BatchArgs&, uint32_t, hipStream_t);
template hipError_t launch_encode<float>(const EncArgs<float>&, int, hipStream_t);
template hipError_t launch_encode<double>(const EncArgs<double>&, int, hipStream_t);
template hipError_t launch_pack<float>(const PackArgs&, hipStream_t);
template hipError_t launch_pack<double>(const PackArgs&, hipStream_t);
template hipError_t launch_decode<float>(const DecArgs<float>&, uint64_t, int, bool, hipStream_t);
template hipError_t launch_decode<double>(const DecArgs<double>&, uint64_t, int, bool, hipStream_t);
template hipError_t launch_decode_queries<float>(const ServeArgs&, uint64_t, int, bool, hipStream_t);
template hipError_t launch_decode_queries<double>(const ServeArgs&, uint64_t, int, bool, hipStream_t);
template hipError_t launch_aux<float>(const AuxArgs&, int, hipStream_t);
template hipError_t launch_aux<double>(const AuxArgs&, int, hipStream_t);
template hipError_t launch_range<float>(const float*, uint64_t, unsigned long long*, hipStream_t);
template hipError_t launch_range<double>(const double*, uint64_t, unsigned long long*, hipStream_t);
template hipError_t launch_decode_box<float>(const DecArgs<float>&, const BoxArgs&, uint64_t, int, hipStream_t);
template hipError_t launch_decode_box<double>(const DecArgs<double>&, const BoxArgs&, uint64_t, int, hipStream_t);
template hipError_t launch_sum_sq<float>(const float*, const float*, double, uint64_t, double*, double*, hipStream_t);
template hipError_t launch_sum_sq<double>(const double*, const double*, double, uint64_t, double*, double*,
                                          hipStream_t);

}  // namespace pmc
