// Device-side helpers shared by the solver's HIP kernels: brick addressing,
// wavefront shuffles and deterministic block reductions.
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
  int done;      // 1: stop iterating (converged or failed)
  int status;    // 0 running/converged, -5 breakdown
  int iters;
  int pad;
  unsigned int ticket[4];  // last-block counters of the reductions
};

// Deterministic two-stage sum: every block stores its partial, the last
// block to finish adds all partials in index order and calls fin(total).
template <class Fin>
__device__ __forceinline__ void block_reduce_finish(double v, double *partials,
                                                    unsigned int *ticket, Fin fin) {
  __shared__ double red[kWavesPerBlock];
  __shared__ bool last;
  v = wave_sum(v);
  int lane = threadIdx.x & (kWave - 1);
  int w = threadIdx.x / kWave;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kWavesPerBlock; ++i) s += red[i];
    partials[blockIdx.x] = s;
    __threadfence();
    unsigned int t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double s = 0.0;
  for (unsigned int i = threadIdx.x; i < gridDim.x; i += blockDim.x) {
    s += partials[i];
  }
  // fixed-order combination across the block
  s = wave_sum(s);
  if (lane == 0) red[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int i = 0; i < kWavesPerBlock; ++i) tot += red[i];
    *ticket = 0u;
    fin(tot);
  }
}

}  // namespace mfmg
