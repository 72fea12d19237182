// HIP kernels of the solver: coefficient assembly (Section 2.1, Eq. 3),
// coarsening (Algorithm 3), the brick stencil with T-junction ghosts
// (Section 3.1, Eq. 10), red-black Gauss-Seidel, the FAS-style cycle steps
// (Algorithm 4) and the PCG vector kernels (Algorithm 1).
//
// Layout: a brick is 4x4x4 cells = one wavefront; lane m is the cell with
// local Morton index m.  Bricks have global ids (leaf bricks first, in
// canonical order, then inner bricks).  Per-brick arrays of 64 values are
// indexed brick * 64 + m; coefficient arrays hold [c | kx | ky | kz] per
// brick (256 values).
#pragma once

#include <type_traits>

#include "device.hpp"

namespace mfmg {

struct Topo {
  int64_t nlb;             // leaf bricks
  int64_t nb;              // all bricks
  const int32_t *nbr;      // 6 per brick
  const int32_t *coord;    // 3 per brick
  const int32_t *parent;   // per brick
  const int32_t *child;    // 8 per brick
  const int32_t *tplus;    // per leaf brick
  const uint64_t *act;     // per brick: active-cell mask
  const uint32_t *flags;   // per brick: face kinds, see kFlag*
};

// Per-brick face flags: bit d (d = 0..5) the face is a T-junction (coarser
// leaf beyond), bit 8 + d the same-level neighbour is an inner brick, bit
// 16 + d the face is a domain wall.
constexpr uint32_t kFlagT = 0x3fu;
constexpr uint32_t kFlagInner = 0x3fu << 8;
constexpr uint32_t kFlagWall = 0x3fu << 16;

// Coefficient access for one multigrid level: leaf bricks read CL values,
// inner bricks read CI values multiplied by iscale (FP16 inner coefficients
// are stored divided by the cell size of their level).
template <class V, class CL, class CI>
struct Coefs {
  const CL *leaf;   // nlb * 256
  const CI *inner;  // (nb - nlb) * 256
  const CL *tc;     // plus-side T-face coefficients, 48 per slot
  int64_t nlb;
  V iscale;
  // When CL == CI the inner coefficients directly follow the leaf ones
  // (one array over all bricks) and no branch is needed.
  __device__ __forceinline__ V get(uint32_t b, int comp, int m) const {
    if constexpr (std::is_same<CL, CI>::value) {
      return V(leaf[b * 256u + comp * 64 + m]);
    } else {
      if (b < nlb) return V(leaf[b * 256u + comp * 64 + m]);
      return V(inner[(b - uint32_t(nlb)) * 256u + comp * 64 + m]) * iscale;
    }
  }
  __device__ __forceinline__ V tplus(int32_t slot, int a, int fidx) const {
    return V(tc[uint32_t(slot) * 48u + a * 16 + fidx]);
  }
};

template <class T>
__device__ __forceinline__ T to_v(double x) { return T(x); }

// Coarse cell (local Morton index inside the coarse leaf brick J) seen from
// cell m of brick b across direction d at a T-junction.
__device__ __forceinline__ int coarse_local(const Topo &T, uint32_t b, int m, int d,
                                            int32_t J) {
  int a = d >> 1;
  int s = (d & 1) ? 1 : -1;
  int loc[3] = {dev_cx(m), dev_cy(m), dev_cz(m)};
  int c[3];
  for (int ax = 0; ax < 3; ++ax) {
    int64_t g = int64_t(T.coord[3 * b + ax]) * 4 + loc[ax] + (ax == a ? s : 0);
    c[ax] = int((g >> 1) - int64_t(T.coord[3 * int64_t(J) + ax]) * 4) & 3;
  }
  return dev_morton(c[0], c[1], c[2]);
}

// ---------------------------------------------------------------------------
// Level operator at one cell (every lane of the wave executes this for its
// own cell of brick b):  (A u)_m = c u_m - sum_d k_d v_d  with v_d the
// same-level neighbour value, 0 at a wall, or at a T-junction the ghost
// u_m + (u_J - mean_active_siblings(u)) / 2, u_J read from the coarser level.
// All neighbour loads are issued before any arithmetic; the T-junction work
// sits behind a wave-uniform branch on the brick's face flags.
// ---------------------------------------------------------------------------
template <class V, class CL, class CI>
__device__ __forceinline__ V level_Au(const Topo &T, const Coefs<V, CL, CI> &cf,
                                      const V *__restrict__ U, uint32_t b, int m, V u,
                                      V c, V k0, V k1, V k2, uint64_t amask, uint32_t flags,
                                      const int32_t (&nb6)[6]) {
  V v[6], k[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    V kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    v[d] = shfl(u, p);
    k[d] = (d & 1) ? shfl(kown, p) : kown;
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int p = dev_partner(m, d);
    if (dev_outside(m, d) && nb6[d] >= 0) {
      v[d] = U[uint32_t(nb6[d]) * 64u + p];
      if (d & 1) k[d] = cf.get(nb6[d], 1 + (d >> 1), p);
    }
  }
#pragma unroll
  for (int d = 0; d < 6; ++d)
    if (dev_outside(m, d) && ((flags >> (16 + d)) & 1u)) v[d] = V(0);
  if (flags & kFlagT) {
    bool act = (amask >> m) & 1ull;
    V s = group8_sum(act ? u : V(0));
    int cnt = __popcll((amask >> (m & 56)) & 0xffull);
    V ubar = cnt ? s / V(cnt) : V(0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (((flags >> d) & 1u) && dev_outside(m, d)) {
        int32_t J = dev_decode_coarse(nb6[d]);
        V uJ = U[uint32_t(J) * 64u + coarse_local(T, b, m, d, J)];
        v[d] = u + (uJ - ubar) * V(0.5);
        if (d & 1) k[d] = cf.tplus(T.tplus[b], d >> 1, dev_face_index(m, d >> 1));
      }
    }
  }
  V acc = c * u;
#pragma unroll
  for (int d = 0; d < 6; ++d) acc -= k[d] * v[d];
  return acc;
}

// Composite leaf operator (the PCG operator, FP64), forward.  X and C cover
// all bricks: where a leaf's same-level neighbour is an inner cell P, X holds
// the mean of P's active children (written by k_average_up) and C holds P's
// Algorithm 3 coefficients, whose face coefficient is the sum of the fine
// sub-face coefficients over 2, i.e. the coarse side of the T-junction
// (Section 3.1).  The fine side uses the ghost of Eq. (10).
__device__ __forceinline__ double composite_Au(const Topo &T, const double *__restrict__ C,
                                               const double *__restrict__ TC,
                                               const double *__restrict__ X, uint32_t b,
                                               int m, double u, double c, double k0,
                                               double k1, double k2, uint64_t amask,
                                               uint32_t flags, const int32_t (&nb6)[6]) {
  double v[6], k[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    double kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    v[d] = shfl(u, p);
    k[d] = (d & 1) ? shfl(kown, p) : kown;
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int p = dev_partner(m, d);
    if (dev_outside(m, d) && nb6[d] >= 0) {
      v[d] = X[uint32_t(nb6[d]) * 64u + p];
      if (d & 1) k[d] = C[uint32_t(nb6[d]) * 256u + (1 + (d >> 1)) * 64 + p];
    }
  }
#pragma unroll
  for (int d = 0; d < 6; ++d)
    if (dev_outside(m, d) && ((flags >> (16 + d)) & 1u)) v[d] = 0.0;
  bool act = (amask >> m) & 1ull;
  if (flags & kFlagT) {
    double s = group8_sum(act ? u : 0.0);
    int cnt = __popcll((amask >> (m & 56)) & 0xffull);
    double ubar = cnt ? s / double(cnt) : 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (((flags >> d) & 1u) && dev_outside(m, d)) {
        int32_t J = dev_decode_coarse(nb6[d]);
        double uJ = X[uint32_t(J) * 64u + coarse_local(T, b, m, d, J)];
        v[d] = u + (uJ - ubar) * 0.5;
        if (d & 1)
          k[d] = TC[uint32_t(T.tplus[b]) * 48u + (d >> 1) * 16 + dev_face_index(m, d >> 1)];
      }
    }
  }
  double acc = c * u;
#pragma unroll
  for (int d = 0; d < 6; ++d) acc -= k[d] * v[d];
  return act ? acc : 0.0;
}

// Transposed composite operator (adjoint path).  Its T-junction blocks are
// the transposes of the rank-one blocks of A: a fine cell's row gets, for
// every sibling, (1/n) sum over the sibling group's T-faces of
// (k/2)(x_i - x_J); a coarse leaf's row gets - sum_f (k_f/2) x_f over the
// fine face cells f instead of K_F times their parent's mean.  X is a leaf
// vector; inner neighbours are read through their children.
__device__ __forceinline__ double composite_AuT(const Topo &T, const double *__restrict__ C,
                                                const double *__restrict__ TC,
                                                const double *__restrict__ X, uint32_t b,
                                                int m, double u, double c, double k0,
                                                double k1, double k2, uint64_t amask,
                                                uint32_t flags, const int32_t (&nb6)[6]) {
  bool act = (amask >> m) & 1ull;
  int cnt = __popcll((amask >> (m & 56)) & 0xffull);
  double acc = c * u;
  double tpart = 0.0;  // this cell's sum of (k/2)(u_m - u_J) over its T-faces
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    double kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    double v = shfl(u, p);
    double kp = shfl(kown, p);
    double k = (d & 1) ? kp : kown;
    if (dev_outside(m, d)) {
      int32_t nb = nb6[d];
      if (nb >= 0 && nb < T.nlb) {
        v = X[uint32_t(nb) * 64u + p];
        if (d & 1) k = C[uint32_t(nb) * 256u + (1 + a) * 64 + p];
      } else if (nb >= 0) {
        // inner neighbour P: - sum over P's children on the face toward this
        // cell of (k_f / 2) x_f
        int32_t cb = T.child[8 * int64_t(nb) + (p >> 3)];
        int base = (p & 7) << 3;
        int facebit = (d & 1) ? 0 : 1;
        double sumkv = 0.0;
        for (int t = 0; t < 8; ++t) {
          if (((t >> a) & 1) != facebit) continue;
          int q = base | t;
          double kc = (d & 1) ? C[uint32_t(cb) * 256u + (1 + a) * 64 + q]
                              : TC[uint32_t(T.tplus[cb]) * 48u + a * 16 + dev_face_index(q, a)];
          sumkv += kc * 0.5 * X[uint32_t(cb) * 64u + q];
        }
        acc -= sumkv;
        continue;
      } else if (nb == dWall) {
        v = 0.0;
      } else {
        int32_t J = dev_decode_coarse(nb);
        double uJ = X[uint32_t(J) * 64u + coarse_local(T, b, m, d, J)];
        if (d & 1) k = TC[uint32_t(T.tplus[b]) * 48u + a * 16 + dev_face_index(m, a)];
        acc -= k * u;
        tpart += k * 0.5 * (u - uJ);
        continue;
      }
    }
    acc -= k * v;
  }
  double S = group8_sum(tpart);
  if (act && cnt) acc += S / double(cnt);
  return act ? acc : 0.0;
}

// Mean of the active cells of each aligned sibling group of a leaf brick
// with a T-face, written to the parent cells' slots of a full-size vector
// (the value the composite operator reads for an inner neighbour).
__device__ __forceinline__ void average_up(const Topo &T, double *__restrict__ X, uint32_t b,
                                           int m, double x, uint64_t amask) {
  bool act = (amask >> m) & 1ull;
  double s = group8_sum(act ? x : 0.0);
  int cnt = __popcll((amask >> (m & 56)) & 0xffull);
  if ((m & 7) == 0) {
    uint32_t P = uint32_t(T.parent[b]);
    int32_t bx = T.coord[3 * b], by = T.coord[3 * b + 1], bz = T.coord[3 * b + 2];
    int oct = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
    X[P * 64u + ((oct << 3) | (m >> 3))] = cnt ? s / double(cnt) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
struct AssembleArgs {
  Topo T;
  const int64_t *fbase;
  const uint8_t *fmask;
  const double *beta;
  const int8_t *blevel;
  int bc[6];
  double theta;
  double *coef;   // nb * 256 (leaf part written)
  double *tc;     // n_tplus * 48
};

__device__ __forceinline__ int64_t face_id(const AssembleArgs &A, int64_t cell, int d) {
  return A.fbase[cell] + __popc(unsigned(A.fmask[cell]) & ((1u << d) - 1u));
}

__global__ void __launch_bounds__(kBlock) k_assemble(AssembleArgs A) {
  int64_t b = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  if (b >= A.T.nlb) return;
  int l = A.blevel[b];
  double h = ldexp(1.0, -l);
  double hf = ldexp(1.0, -(l + 1));
  double dk[6];
  int64_t cell = b * 64 + m;
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    double k = 0.0;
    if (!dev_outside(m, d)) {
      // same brick: same-level neighbour
      if (d & 1) {
        k = A.beta[face_id(A, b * 64 + p, d - 1)] * h;
      } else {
        k = A.beta[face_id(A, cell, d)] * h;
      }
    } else {
      int32_t nb = A.T.nbr[6 * b + d];
      if (nb == dWall) {
        k = A.bc[d] == 1 ? A.beta[face_id(A, cell, d)] * (h / A.theta) : 0.0;
      } else if (nb >= 0 && nb < A.T.nlb) {
        if (d & 1) {
          k = A.beta[face_id(A, uint32_t(nb) * 64u + p, d - 1)] * h;
        } else {
          k = A.beta[face_id(A, cell, d)] * h;
        }
      } else if (nb >= 0) {
        // finer neighbours: sum of the 4 fine sub-face coefficients over 2
        int32_t cb = A.T.child[8 * int64_t(nb) + (p >> 3)];
        int base = (p & 7) << 3;
        int o0 = a == 0 ? 1 : 0;
        int o1 = a == 2 ? 1 : 2;
        int abit = (d & 1) ? 0 : 1;
        double acc = 0.0;
        for (int n = 0; n < 4; ++n) {
          int t = (abit << a) | ((n & 1) << o0) | ((n >> 1) << o1);
          acc = acc + A.beta[face_id(A, uint32_t(cb) * 64u + (base | t), d ^ 1)] * hf / 2.0;
        }
        k = acc;
      } else {
        // coarser neighbour: this cell owns the T-face
        k = A.beta[face_id(A, cell, d)] * h;
        if (d & 1) A.tc[int64_t(A.T.tplus[b]) * 48 + a * 16 + dev_face_index(m, a)] = k;
      }
    }
    dk[d] = k;
  }
  double c = dk[0] + dk[1] + dk[2] + dk[3] + dk[4] + dk[5];
  double *cf = A.coef + b * 256;
  cf[m] = c;
  cf[64 + m] = dk[0];
  cf[128 + m] = dk[2];
  cf[192 + m] = dk[4];
}

// active-cell masks: one bit per cell with c != 0
__global__ void __launch_bounds__(kBlock) k_active_mask(const double *coef, const int32_t *list,
                                                        int64_t n, uint64_t *act) {
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  if (i >= n) return;
  int64_t b = list ? list[i] : i;
  uint64_t mask = __ballot(coef[b * 256 + m] != 0.0);
  if (m == 0) act[b] = mask;
}

// Algorithm 3: coarse coefficients of the inner bricks of one level.
__global__ void __launch_bounds__(kBlock) k_coarsen(const int32_t *list, int64_t n, Topo T,
                                                    double *coef, double alpha) {
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int q = threadIdx.x & (kWave - 1);
  if (i >= n) return;
  int64_t b = list[i];
  int32_t cb = T.child[8 * b + (q >> 3)];
  const double *cc = coef + uint32_t(cb) * 256u;
  int base = (q & 7) << 3;
  double c = 0.0, kx = 0.0, ky = 0.0, kz = 0.0;
  int cnt = 0;
  for (int t = 0; t < 8; ++t) {
    int ch = base | t;
    double ci = cc[ch];
    bool on = ci != 0.0;
    if (on) {
      ++cnt;
      c = c + ci / alpha;
    }
    double kk[3] = {cc[64 + ch], cc[128 + ch], cc[192 + ch]};
    for (int a = 0; a < 3; ++a) {
      if ((t >> a) & 1) {
        int sib = base | (t ^ (1 << a));
        if (on && cc[sib] != 0.0) c = c + 2.0 / alpha * (-kk[a]);
      } else {
        if (a == 0) kx = kx + kk[0] / alpha;
        if (a == 1) ky = ky + kk[1] / alpha;
        if (a == 2) kz = kz + kk[2] / alpha;
      }
    }
  }
  if (cnt == 0) c = 0.0;
  double *o = coef + b * 256;
  o[q] = c;
  o[64 + q] = kx;
  o[128 + q] = ky;
  o[192 + q] = kz;
}

// FP64 coefficients -> FP32 leaf copies and FP16 inner copies scaled by 1/h
__global__ void k_convert_leaf(const double *src, float *dst, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}
__global__ void __launch_bounds__(kBlock) k_convert_inner(const double *coef, const int8_t *blevel,
                                                          int64_t nlb, int64_t nb, __half *dst) {
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  int64_t b = nlb + i;
  if (b >= nb) return;
  double inv_h = ldexp(1.0, int(blevel[b]));
  for (int comp = 0; comp < 4; ++comp)
    dst[i * 256 + comp * 64 + m] = __float2half_rn(float(coef[b * 256 + comp * 64 + m] * inv_h));
}

// ---------------------------------------------------------------------------
// multigrid cycle kernels (one wave per brick of a level list)
// ---------------------------------------------------------------------------
template <class V, class CL, class CI>
struct LevelArgs {
  Topo T;
  Coefs<V, CL, CI> cf;
  V *U;              // iterate, nb * 64
  V *B;              // right-hand side, nb * 64 (leaf part: PCG residual)
  V *Ustar;          // FAS initial guess of inner cells, (nb - nlb) * 64
  const int32_t *list;
  int64_t n;
  const int *done;   // skip when the solve has stopped
};

template <class V, class CL, class CI>
__device__ __forceinline__ void load_cell(const LevelArgs<V, CL, CI> &A, uint32_t b, int m, V &c,
                                          V &k0, V &k1, V &k2) {
  c = A.cf.get(b, 0, m);
  k0 = A.cf.get(b, 1, m);
  k1 = A.cf.get(b, 2, m);
  k2 = A.cf.get(b, 3, m);
}

__device__ __forceinline__ void load_nbr(const Topo &T, uint32_t b, int32_t (&nb6)[6]) {
#pragma unroll
  for (int d = 0; d < 6; ++d) nb6[d] = T.nbr[6 * b + d];
}

// One colour half-sweep: u_m += (b_m - (A u)_m) / c_m on cells of the colour.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_smooth(LevelArgs<V, CL, CI> A, int colour) {
  if (A.done && *A.done) return;
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.n) return;
  uint32_t b = uint32_t(A.list[i]);
  V c, k0, k1, k2;
  load_cell(A, b, m, c, k0, k1, k2);
  V u = A.U[b * 64u + m];
  V rhs = A.B[b * 64u + m];
  uint64_t amask = A.T.act[b];
  int32_t nb6[6];
  load_nbr(A.T, b, nb6);
  V Au = level_Au(A.T, A.cf, A.U, b, m, u, c, k0, k1, k2, amask, A.T.flags[b], nb6);
  bool act = (amask >> m) & 1ull;
  int col = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
  if (act && col == colour) A.U[b * 64u + m] = u + (rhs - Au) / c;
}

// Residual, restriction and FAS initial guess from level l to its parents:
//   b_P = beta_mg (1/alpha) sum_children r,  u_P = u*_P = mean of active
//   children (the FAS coarse right-hand side is completed by k_fas_rhs).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_restrict(LevelArgs<V, CL, CI> A, V scale) {
  if (A.done && *A.done) return;
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.n) return;
  uint32_t b = uint32_t(A.list[i]);
  V c, k0, k1, k2;
  load_cell(A, b, m, c, k0, k1, k2);
  V u = A.U[b * 64u + m];
  V rhs = A.B[b * 64u + m];
  uint64_t amask = A.T.act[b];
  int32_t nb6[6];
  load_nbr(A.T, b, nb6);
  V Au = level_Au(A.T, A.cf, A.U, b, m, u, c, k0, k1, k2, amask, A.T.flags[b], nb6);
  bool act = (amask >> m) & 1ull;
  V r = act ? rhs - Au : V(0);
  V rs = group8_sum(r);
  V us = group8_sum(act ? u : V(0));
  int cnt = __popcll((amask >> (m & 56)) & 0xffull);
  if ((m & 7) == 0) {
    uint32_t P = uint32_t(A.T.parent[b]);
    // octant of this brick inside its parent
    int32_t bx = A.T.coord[3 * b], by = A.T.coord[3 * b + 1], bz = A.T.coord[3 * b + 2];
    int oct = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
    int q = (oct << 3) | (m >> 3);
    V ust = cnt ? us / V(cnt) : V(0);
    A.B[P * 64u + q] = rs * scale;
    A.U[P * 64u + q] = ust;
    A.Ustar[(P - uint32_t(A.T.nlb)) * 64u + q] = ust;
  }
}

// FAS coarse right-hand side on inner bricks: b += A^{l-1} u*.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_fas_rhs(LevelArgs<V, CL, CI> A) {
  if (A.done && *A.done) return;
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.n) return;
  uint32_t b = uint32_t(A.list[i]);
  V c, k0, k1, k2;
  load_cell(A, b, m, c, k0, k1, k2);
  V u = A.U[b * 64u + m];
  uint64_t amask = A.T.act[b];
  int32_t nb6[6];
  load_nbr(A.T, b, nb6);
  V Au = level_Au(A.T, A.cf, A.U, b, m, u, c, k0, k1, k2, amask, A.T.flags[b], nb6);
  bool act = (amask >> m) & 1ull;
  V rhs = A.B[b * 64u + m];
  A.B[b * 64u + m] = act ? rhs + Au : V(0);
}

// Prolongation of the FAS correction: u += u_P - u*_P on active cells.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_prolong(LevelArgs<V, CL, CI> A) {
  if (A.done && *A.done) return;
  int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.n) return;
  uint32_t b = uint32_t(A.list[i]);
  uint64_t amask = A.T.act[b];
  if (!((amask >> m) & 1ull)) return;
  uint32_t P = uint32_t(A.T.parent[b]);
  int32_t bx = A.T.coord[3 * b], by = A.T.coord[3 * b + 1], bz = A.T.coord[3 * b + 2];
  int oct = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
  int q = (oct << 3) | (m >> 3);
  V corr = A.U[P * 64u + q] - A.Ustar[(P - uint32_t(A.T.nlb)) * 64u + q];
  A.U[b * 64u + m] += corr;
}

// Coarsest level: nu_coarse RBGS iterations in one workgroup, (R,B) for the
// first half of the iterations and (B,R) for the rest.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(1024) k_coarsest(LevelArgs<V, CL, CI> A, int nu) {
  if (A.done && *A.done) return;
  int w = threadIdx.x / kWave;
  int nw = blockDim.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  int half = nu / 2;
  for (int it = 0; it < nu; ++it) {
    for (int h2 = 0; h2 < 2; ++h2) {
      int colour = it < half ? h2 : 1 - h2;
      for (int64_t i = w; i < A.n; i += nw) {
        uint32_t b = uint32_t(A.list[i]);
        V c, k0, k1, k2;
        load_cell(A, b, m, c, k0, k1, k2);
        V u = A.U[b * 64u + m];
        V rhs = A.B[b * 64u + m];
        uint64_t amask = A.T.act[b];
        int32_t nb6[6];
        load_nbr(A.T, b, nb6);
        V Au = level_Au(A.T, A.cf, A.U, b, m, u, c, k0, k1, k2, amask, A.T.flags[b], nb6);
        bool act = (amask >> m) & 1ull;
        int col = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
        if (act && col == colour) A.U[b * 64u + m] = u + (rhs - Au) / c;
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

template <class V>
__global__ void k_fill(V *x, int64_t n, V v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace mfmg
