// Device-side helpers shared by the solver's HIP kernels: brick addressing,
// wavefront shuffles, buffer access and the solve's device-resident scalars.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfmg {

constexpr int kWave = 64;          // CDNA wavefront = one 4^3 brick
constexpr int kBlock = 256;        // 4 bricks per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int32_t dWall = -1;
constexpr int32_t dCoarseBase = -2;

__device__ __forceinline__ int32_t dev_decode_coarse(int32_t v) { return dCoarseBase - v; }

__device__ __forceinline__ int dev_morton(int x, int y, int z) {
  return (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((x & 2) << 2) | ((y & 2) << 3) |
         ((z & 2) << 4);
}
__device__ __forceinline__ int dev_cx(int m) { return (m & 1) | ((m >> 2) & 2); }
__device__ __forceinline__ int dev_cy(int m) { return ((m >> 1) & 1) | ((m >> 3) & 2); }
__device__ __forceinline__ int dev_cz(int m) { return ((m >> 2) & 1) | ((m >> 4) & 2); }
__device__ __forceinline__ int dev_coord(int m, int a) {
  return a == 0 ? dev_cx(m) : (a == 1 ? dev_cy(m) : dev_cz(m));
}

// Lane of the neighbour of cell m across direction d (axis d/2, + if d odd)
// inside the brick, or, when the neighbour lies in the next brick, the
// index of that cell in the next brick (the same bit pattern).
__device__ __forceinline__ int dev_partner(int m, int d) {
  int low = 1 << (d >> 1);
  int both = low | (low << 3);
  if (d & 1) return (m & low) ? (m ^ both) : (m ^ low);
  return (m & low) ? (m ^ low) : (m ^ both);
}
__device__ __forceinline__ bool dev_outside(int m, int d) {
  int low = 1 << (d >> 1);
  int both = low | (low << 3);
  return (d & 1) ? ((m & both) == both) : ((m & both) == 0);
}
// Index (0..15) of a face cell in the face normal to axis a: the two other
// local coordinates in increasing axis order, the lower one fastest.
__device__ __forceinline__ int dev_face_index(int m, int a) {
  int o0 = a == 0 ? 1 : 0;
  int o1 = a == 2 ? 1 : 2;
  return dev_coord(m, o0) + 4 * dev_coord(m, o1);
}

template <class T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, kWave);
}
template <class T>
__device__ __forceinline__ T shfl_xor(T v, int mask) {
  return __shfl_xor(v, mask, kWave);
}

// Value of v in the lane whose byte address (4 x lane) is addr.
template <class T>
__device__ __forceinline__ T bperm(T v, int addr) {
  if constexpr (sizeof(T) == 8) {
    uint64_t x = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(uint32_t(x))));
    uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(uint32_t(x >> 32))));
    return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
  } else {
    static_assert(sizeof(T) == 4, "4- or 8-byte values");
    return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
  }
}

// Sum over the 8 lanes of an aligned sibling group (identical in every lane:
// the xor butterfly adds the same operands in every lane).
template <class T>
__device__ __forceinline__ T group8_sum(T v) {
  v = v + shfl_xor(v, 1);
  v = v + shfl_xor(v, 2);
  v = v + shfl_xor(v, 4);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 1; o < kWave; o <<= 1) v = v + shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// Raw buffer access: a per-lane element offset (voffset) plus a wave-uniform
// element base (soffset), both 32-bit, against a wave-uniform resource
// descriptor.  The per-brick part of an address is then scalar arithmetic
// and the per-lane part a loop-invariant register.  Every buffer accessed
// this way is below 4 GiB (checked on the host).
// ---------------------------------------------------------------------------
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped, unswizzled) buffer, gfx9 family
constexpr uint64_t kMaxBufferBytes = 0xffffffffull;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint64_t bytes) {
  uint32_t n = bytes >= kMaxBufferBytes ? uint32_t(kMaxBufferBytes) : uint32_t(bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, int(n), kRsrcWord3);
}

// Cache-policy operand of a buffer load (gfx950): 0 = default, 2 = nt
// (non-temporal: the line is a first candidate for eviction from L2).
constexpr int kCpolDefault = 0;
constexpr int kCpolStream = 2;
// Level-kernel policy (not an operand value): the coefficient arrays load
// non-temporal, the right-hand side and the plus-face table with the
// default policy.  coef_pol / side_pol give the operand of each kind of
// load for a level policy (kCpolDefault, kCpolStream or this).
constexpr int kCpolStreamCoef = 0x100;
constexpr int coef_pol(int cp) { return cp == kCpolStreamCoef ? kCpolStream : cp; }
constexpr int side_pol(int cp) { return cp == kCpolStreamCoef ? kCpolDefault : cp; }

// Load of element `lane` of the array at element offset `base` (the lane
// offset goes to voffset, the uniform base to soffset).
template <class T, int CPOL = kCpolDefault>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t base) {
  constexpr uint32_t n = sizeof(T);
  if constexpr (n == 8)
    return __builtin_bit_cast(
        T, __builtin_amdgcn_raw_buffer_load_b64(r, int(lane * n), int(base * n), CPOL));
  else if constexpr (n == 4)
    return __builtin_bit_cast(
        T, __builtin_amdgcn_raw_buffer_load_b32(r, int(lane * n), int(base * n), CPOL));
  else
    return __builtin_bit_cast(
        T, __builtin_amdgcn_raw_buffer_load_b16(r, int(lane * n), int(base * n), CPOL));
}

template <class T, int CPOL = kCpolDefault>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t base,
                                       T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "bstore: 4- or 8-byte values");
  if constexpr (sizeof(T) == 8) {
    typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, int(lane * 8u),
                                          int(base * 8u), CPOL);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(lane * 4u),
                                          int(base * 4u), CPOL);
  }
}

// Scalars of one PCG solve, resident in device memory.
struct Scalars {
  double rr0;    // ||r_0||^2
  double rr;     // ||r_k||^2
  double rz;     // (r_k, z_k)
  double pAp;    // (p_k, A p_k)
  double alpha;
  double beta;
  double tol2;   // rtol^2 ||r_0||^2
  double sum;    // scratch: sum for the null-space mean
  double cnt;    // scratch: active count
  double tr;     // ||rhs - A x||^2 of the true residual
  double rscale; // power of two the cycle's input (the residual) is scaled by
  int done;      // 1: stop iterating (converged or failed)
  int status;    // 0 running/converged, -5 breakdown
  int iters;
  int xpend;     // 1: x still lacks alpha p of the last residual update
};

}  // namespace mfmg
