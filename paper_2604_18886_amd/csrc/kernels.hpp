// HIP kernels of the solver: coefficient assembly (Section 2.1, Eq. 3),
// coarsening (Algorithm 3), the brick stencil with T-junction ghosts
// (Section 3.1, Eq. 10), red-black Gauss-Seidel and the steps of the
// FAS-style cycle (Algorithm 4).
//
// Layout: a brick is 4x4x4 cells = one wavefront; lane m is the cell with
// local Morton index m.  Device brick ids are level-major: leaf bricks first
// (finest level first, Morton order inside a level), then inner bricks
// (finest level first, Morton order), so the bricks of one level form two
// contiguous ranges.  Per-brick arrays of 64 values are indexed
// brick * 64 + m; coefficient arrays hold [c | kx | ky | kz] per brick.
#pragma once

#include <type_traits>

#include "device.hpp"

namespace mfmg {

// One brick's topology in a single 64-byte record (one scalar load).
struct alignas(64) BrickMeta {
  int32_t nbr[6];    // >= 0 same-level brick, -1 wall, <= -2 coarser leaf (T)
  uint32_t flags;    // see kFlag*
  int32_t parent;    // parent brick, -1 at the coarsest stored level
  int32_t tplus;     // slot of plus-side T-face coefficients, -1 if none
  int32_t coord[3];  // brick coordinates at its level
  uint32_t act[2];   // active-cell mask (bit m: cell m has c != 0)
  int32_t level;     // cell level
  int32_t pad;
};
static_assert(sizeof(BrickMeta) == 64, "brick record must be 64 bytes");

// Face flags: bit d (d = 0..5) T-junction (coarser leaf beyond), bit 8 + d
// same-level neighbour is an inner brick, bit 16 + d domain wall.
constexpr uint32_t kFlagT = 0x3fu;
constexpr uint32_t kFlagInner = 0x3fu << 8;
constexpr uint32_t kFlagWall = 0x3fu << 16;

struct Topo {
  uint32_t nlb;            // leaf bricks (device ids 0 .. nlb-1)
  uint32_t nb;             // all bricks
  const BrickMeta *meta;   // nb records
  const int32_t *child;    // 8 per brick (octant dx + 2 dy + 4 dz), -1 for leaves
};

// Bricks of one level: a leaf range followed by an inner range.
struct Range {
  uint32_t leaf_lo, n_leaf, inner_lo, n_inner;
  __device__ __forceinline__ uint32_t brick(uint32_t i) const {
    return i < n_leaf ? leaf_lo + i : inner_lo + (i - n_leaf);
  }
  __host__ __device__ uint32_t n() const { return n_leaf + n_inner; }
};

__device__ __forceinline__ uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}
__device__ __forceinline__ uint64_t act_mask(const BrickMeta &M) {
  return uint64_t(M.act[0]) | (uint64_t(M.act[1]) << 32);
}
__device__ __forceinline__ int octant_of(const BrickMeta &M) {
  return (M.coord[0] & 1) | ((M.coord[1] & 1) << 1) | ((M.coord[2] & 1) << 2);
}

// Coefficient access for one multigrid level: leaf bricks read CL values,
// inner bricks read CI values multiplied by iscale (FP16 inner coefficients
// are stored divided by the cell size of their level).  When CL == CI the
// inner coefficients directly follow the leaf ones in one array.
template <class V, class CL, class CI>
struct Coefs {
  const CL *leaf;
  const CI *inner;
  const CL *tc;  // plus-side T-face coefficients, 48 per slot
  uint32_t nlb;
  V iscale;
  __device__ __forceinline__ V get(uint32_t b, int comp, int m) const {
    if constexpr (std::is_same<CL, CI>::value) {
      return V(leaf[b * 256u + comp * 64 + m]);
    } else {
      if (b < nlb) return V(leaf[b * 256u + comp * 64 + m]);
      return V(inner[(b - nlb) * 256u + comp * 64 + m]) * iscale;
    }
  }
  __device__ __forceinline__ V tplus(int32_t slot, int a, int fidx) const {
    return V(tc[uint32_t(slot) * 48u + a * 16 + fidx]);
  }
};

template <class V>
__device__ __forceinline__ V div_by(V a, V c) {
  if constexpr (std::is_same<V, float>::value) {
    return a * __builtin_amdgcn_rcpf(c);  // v_rcp_f32, 1 ulp: enough for a smoother
  } else {
    return a / c;
  }
}

// Coarse cell (local Morton index inside the coarse leaf brick J) seen from
// cell m of brick M across direction d at a T-junction.
__device__ __forceinline__ int coarse_local(const BrickMeta &M, int m, int d,
                                            const BrickMeta &MJ) {
  int a = d >> 1;
  int s = (d & 1) ? 1 : -1;
  int loc[3] = {dev_cx(m), dev_cy(m), dev_cz(m)};
  int c[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    int g = M.coord[ax] * 4 + loc[ax] + (ax == a ? s : 0);
    c[ax] = ((g >> 1) - MJ.coord[ax] * 4) & 3;
  }
  return dev_morton(c[0], c[1], c[2]);
}

// ---------------------------------------------------------------------------
// Neighbour sum of the level operator at one cell (every lane of the wave
// executes this for its own cell of brick b):
//   S_m = sum_d k_d v_d,   (A u)_m = c_m u_m - S_m,
// v_d the same-level neighbour value, 0 at a wall, or at a T-junction the
// ghost u_m + (u_J - mean_active_siblings(u)) / 2 with u_J read from the
// coarser level.  All neighbour loads are issued before any arithmetic; the
// T-junction work sits behind a wave-uniform branch on the face flags.
// ---------------------------------------------------------------------------
template <class V, class CL, class CI>
__device__ __forceinline__ V neighbour_sum(const Topo &T, const Coefs<V, CL, CI> &cf,
                                           const V *__restrict__ U, const BrickMeta &M,
                                           int m, V u, V k0, V k1, V k2) {
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
    if (dev_outside(m, d) && M.nbr[d] >= 0) {
      v[d] = U[uint32_t(M.nbr[d]) * 64u + p];
      if (d & 1) k[d] = cf.get(uint32_t(M.nbr[d]), 1 + (d >> 1), p);
    }
  }
#pragma unroll
  for (int d = 0; d < 6; ++d)
    if (dev_outside(m, d) && ((M.flags >> (16 + d)) & 1u)) v[d] = V(0);
  if (M.flags & kFlagT) {
    uint64_t amask = act_mask(M);
    bool act = (amask >> m) & 1ull;
    V s = group8_sum(act ? u : V(0));
    int cnt = __popcll((amask >> (m & 56)) & 0xffull);
    V ubar = cnt ? s / V(cnt) : V(0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (((M.flags >> d) & 1u) && dev_outside(m, d)) {
        int32_t J = dev_decode_coarse(M.nbr[d]);
        const BrickMeta MJ = T.meta[J];
        V uJ = U[uint32_t(J) * 64u + coarse_local(M, m, d, MJ)];
        v[d] = u + (uJ - ubar) * V(0.5);
        if (d & 1) k[d] = cf.tplus(M.tplus, d >> 1, dev_face_index(m, d >> 1));
      }
    }
  }
  V acc = V(0);
#pragma unroll
  for (int d = 0; d < 6; ++d) acc += k[d] * v[d];
  return acc;
}

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
struct AssembleArgs {
  Topo T;
  const int64_t *fbase;  // per device leaf cell: canonical id of its first owned face
  const uint8_t *fmask;  // per device leaf cell: owned directions
  const double *beta;    // canonical face order
  int bc[6];
  double theta;
  double *coef;          // nlb * 256
  double *tc;            // n_tplus * 48
};

__device__ __forceinline__ int64_t face_id(const AssembleArgs &A, uint32_t cell, int d) {
  return A.fbase[cell] + __popc(unsigned(A.fmask[cell]) & ((1u << d) - 1u));
}

// Leaf coefficients (Eq. 3): per direction the face coefficient
// beta S / h (same level or the fine side of a T-junction), beta S/(theta h)
// at a Dirichlet wall, 0 at a Neumann wall, and for a finer neighbour the
// sum of its 4 sub-face coefficients over 2; c is the sum over directions.
__global__ void __launch_bounds__(kBlock) k_assemble(AssembleArgs A) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= A.T.nlb) return;
  const BrickMeta M = A.T.meta[b];
  double h = ldexp(1.0, -M.level);
  double hf = ldexp(1.0, -(M.level + 1));
  double dk[6];
  uint32_t cell = b * 64u + m;
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    double k = 0.0;
    if (!dev_outside(m, d)) {
      k = (d & 1) ? A.beta[face_id(A, b * 64u + p, d - 1)] * h
                  : A.beta[face_id(A, cell, d)] * h;
    } else {
      int32_t nb = M.nbr[d];
      if (nb == dWall) {
        k = A.bc[d] == 1 ? A.beta[face_id(A, cell, d)] * (h / A.theta) : 0.0;
      } else if (nb >= 0 && uint32_t(nb) < A.T.nlb) {
        k = (d & 1) ? A.beta[face_id(A, uint32_t(nb) * 64u + p, d - 1)] * h
                    : A.beta[face_id(A, cell, d)] * h;
      } else if (nb >= 0) {
        // finer neighbours: the leaf children of inner cell p of brick nb
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
        if (d & 1) A.tc[uint32_t(M.tplus) * 48u + a * 16 + dev_face_index(m, a)] = k;
      }
    }
    dk[d] = k;
  }
  double c = dk[0] + dk[1] + dk[2] + dk[3] + dk[4] + dk[5];
  double *cf = A.coef + b * 256u;
  cf[m] = c;
  cf[64 + m] = dk[0];
  cf[128 + m] = dk[2];
  cf[192 + m] = dk[4];
}

// Active-cell masks of bricks [lo, lo + n): bit m set when c_m != 0.
__global__ void __launch_bounds__(kBlock) k_active_mask(const double *coef, uint32_t lo,
                                                        uint32_t n, BrickMeta *meta) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= n) return;
  uint32_t b = lo + i;
  uint64_t mask = __ballot(coef[b * 256u + m] != 0.0);
  if (m == 0) {
    meta[b].act[0] = uint32_t(mask);
    meta[b].act[1] = uint32_t(mask >> 32);
  }
}

// Algorithm 3: coarse coefficients of the inner bricks [lo, lo + n) from
// their children, one lane per coarse cell.
__global__ void __launch_bounds__(kBlock) k_coarsen(uint32_t lo, uint32_t n, Topo T,
                                                    double *coef, double alpha) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int q = threadIdx.x & (kWave - 1);
  if (i >= n) return;
  uint32_t b = lo + i;
  int32_t cb = T.child[8 * int64_t(b) + (q >> 3)];
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
  double *o = coef + b * 256u;
  o[q] = c;
  o[64 + q] = kx;
  o[128 + q] = ky;
  o[192 + q] = kz;
}

// FP64 coefficients -> FP32 copies (leaf bricks, T-face table)
__global__ void k_convert_leaf(const double *src, float *dst, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}
// FP64 inner coefficients -> FP16 copies of c / h_l
__global__ void __launch_bounds__(kBlock) k_convert_inner(const double *coef, Topo T,
                                                          __half *dst) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  uint32_t b = T.nlb + i;
  if (b >= T.nb) return;
  double inv_h = ldexp(1.0, T.meta[b].level);
  for (int comp = 0; comp < 4; ++comp)
    dst[i * 256u + comp * 64 + m] =
        __float2half_rn(float(coef[b * 256u + comp * 64 + m] * inv_h));
}

// ---------------------------------------------------------------------------
// multigrid cycle kernels (one wave per brick of a level)
// ---------------------------------------------------------------------------
template <class V, class CL, class CI>
struct LevelArgs {
  Topo T;
  Coefs<V, CL, CI> cf;
  V *U;              // iterate, nb * 64
  V *B;              // right-hand side, nb * 64 (leaf part: the PCG residual)
  V *Ustar;          // FAS initial guess of inner cells, (nb - nlb) * 64
  Range R;
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

// One colour half-sweep of red-black Gauss-Seidel: on the cells of the
// colour, u_m = (b_m + S_m) / c_m, i.e. u_m += (b - A u)_m / c_m with every
// read taken from the values before the sweep.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_smooth(LevelArgs<V, CL, CI> A, int colour) {
  if (A.done && *A.done) return;
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  V c, k0, k1, k2;
  load_cell(A, b, m, c, k0, k1, k2);
  V u = A.U[b * 64u + m];
  V rhs = A.B[b * 64u + m];
  V S = neighbour_sum(A.T, A.cf, A.U, M, m, u, k0, k1, k2);
  bool act = (act_mask(M) >> m) & 1ull;
  int col = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
  if (act && col == colour) A.U[b * 64u + m] = div_by(rhs + S, c);
}

// Residual, restriction and FAS initial guess from level l to its parents:
//   b_P = beta_mg (1/alpha) sum_children r,  u_P = u*_P = mean of active
//   children (k_fas_rhs then adds A^{l-1} u* on inner cells).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_restrict(LevelArgs<V, CL, CI> A, V scale) {
  if (A.done && *A.done) return;
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  V c, k0, k1, k2;
  load_cell(A, b, m, c, k0, k1, k2);
  V u = A.U[b * 64u + m];
  V rhs = A.B[b * 64u + m];
  V S = neighbour_sum(A.T, A.cf, A.U, M, m, u, k0, k1, k2);
  uint64_t amask = act_mask(M);
  bool act = (amask >> m) & 1ull;
  V r = act ? rhs - (c * u - S) : V(0);
  V rs = group8_sum(r);
  V us = group8_sum(act ? u : V(0));
  int cnt = __popcll((amask >> (m & 56)) & 0xffull);
  if ((m & 7) == 0) {
    uint32_t P = uint32_t(M.parent);
    int q = (octant_of(M) << 3) | (m >> 3);
    V ust = cnt ? us / V(cnt) : V(0);
    A.B[P * 64u + q] = rs * scale;
    A.U[P * 64u + q] = ust;
    A.Ustar[(P - A.T.nlb) * 64u + q] = ust;
  }
}

// FAS coarse right-hand side on inner bricks: b += A^{l-1} u*.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_fas_rhs(LevelArgs<V, CL, CI> A) {
  if (A.done && *A.done) return;
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  V c, k0, k1, k2;
  load_cell(A, b, m, c, k0, k1, k2);
  V u = A.U[b * 64u + m];
  V S = neighbour_sum(A.T, A.cf, A.U, M, m, u, k0, k1, k2);
  bool act = (act_mask(M) >> m) & 1ull;
  V rhs = A.B[b * 64u + m];
  A.B[b * 64u + m] = act ? rhs + (c * u - S) : V(0);
}

// Prolongation of the FAS correction: u += u_P - u*_P on active cells.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_prolong(LevelArgs<V, CL, CI> A) {
  if (A.done && *A.done) return;
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  if (!((act_mask(M) >> m) & 1ull)) return;
  uint32_t P = uint32_t(M.parent);
  int q = (octant_of(M) << 3) | (m >> 3);
  V corr = A.U[P * 64u + q] - A.Ustar[(P - A.T.nlb) * 64u + q];
  A.U[b * 64u + m] += corr;
}

// Coarsest level: nu RBGS iterations in one workgroup, (R,B) for the first
// half of the iterations and (B,R) for the rest.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(1024) k_coarsest(LevelArgs<V, CL, CI> A, int nu) {
  if (A.done && *A.done) return;
  uint32_t w = wave_id();
  uint32_t nw = blockDim.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  int half = nu / 2;
  for (int it = 0; it < nu; ++it) {
    for (int h2 = 0; h2 < 2; ++h2) {
      int colour = it < half ? h2 : 1 - h2;
      for (uint32_t i = w; i < A.R.n(); i += nw) {
        uint32_t b = A.R.brick(i);
        const BrickMeta M = A.T.meta[b];
        V c, k0, k1, k2;
        load_cell(A, b, m, c, k0, k1, k2);
        V u = A.U[b * 64u + m];
        V rhs = A.B[b * 64u + m];
        V S = neighbour_sum(A.T, A.cf, A.U, M, m, u, k0, k1, k2);
        bool act = (act_mask(M) >> m) & 1ull;
        int col = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
        if (act && col == colour) A.U[b * 64u + m] = div_by(rhs + S, c);
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// transpose of the cycle (adjoint solves).  The cycle's linear steps are
// transposed and taken in reverse order; this gives a cycle for A^T in
// residual form: RHO (the adjoint of u) is a residual that is reduced, Y
// (the adjoint of b) accumulates the solution, W is a scratch level vector.
// ---------------------------------------------------------------------------
template <class V, class CL, class CI>
struct LevelArgsT {
  Topo T;
  Coefs<V, CL, CI> cf;
  V *RHO;    // nb * 64
  V *Y;      // nb * 64
  V *W;      // nb * 64
  V *SBAR;   // (nb - nlb) * 64
  V *YS;     // (nb - nlb) * 64
  Range R;
  V bscale;  // beta_mg / alpha
};

// Transposed level operator at one cell, applied to W:
//   (c_m - sum_{T faces of m} k) W_m - sum_{other faces} k W_nbr
//   + (1 / n_active siblings) sum over the sibling group's T-faces (k_i/2) W_i
// (the coupling to the coarser level, B^T, is applied by k_T_coupling).
template <class V, class CL, class CI>
__device__ __forceinline__ V level_AuT(const Coefs<V, CL, CI> &cf, const V *__restrict__ W,
                                       const BrickMeta &M, int m, V w, V c, V k0, V k1, V k2) {
  V v[6], k[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    V kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    v[d] = shfl(w, p);
    k[d] = (d & 1) ? shfl(kown, p) : kown;
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int p = dev_partner(m, d);
    if (dev_outside(m, d) && M.nbr[d] >= 0) {
      v[d] = W[uint32_t(M.nbr[d]) * 64u + p];
      if (d & 1) k[d] = cf.get(uint32_t(M.nbr[d]), 1 + (d >> 1), p);
    }
  }
#pragma unroll
  for (int d = 0; d < 6; ++d)
    if (dev_outside(m, d) && ((M.flags >> (16 + d)) & 1u)) v[d] = V(0);
  uint64_t amask = act_mask(M);
  bool act = (amask >> m) & 1ull;
  V acc = c * w;
  if (M.flags & kFlagT) {
    V tpart = V(0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (((M.flags >> d) & 1u) && dev_outside(m, d)) {
        V kt = (d & 1) ? cf.tplus(M.tplus, d >> 1, dev_face_index(m, d >> 1)) : k[d];
        acc -= kt * w;
        tpart += kt * V(0.5) * w;
        k[d] = V(0);
      }
    }
    V Ssum = group8_sum(tpart);
    int cnt = __popcll((amask >> (m & 56)) & 0xffull);
    if (act && cnt) acc += Ssum / V(cnt);
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) acc -= k[d] * v[d];
  return act ? acc : V(0);
}

// First half of a transposed half-sweep: w = RHO / c on the cells of the
// colour (0 elsewhere), Y += w, W = w.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_sweep_w(LevelArgsT<V, CL, CI> A, int colour) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  bool act = (act_mask(M) >> m) & 1ull;
  int col = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
  V w = V(0);
  if (act && col == colour) w = div_by(A.RHO[b * 64u + m], A.cf.get(b, 0, m));
  A.W[b * 64u + m] = w;
  if (w != V(0)) A.Y[b * 64u + m] += w;
}

// RHO -= A^T W on the bricks of the range.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_apply(LevelArgsT<V, CL, CI> A) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  V c = A.cf.get(b, 0, m), k0 = A.cf.get(b, 1, m), k1 = A.cf.get(b, 2, m),
    k2 = A.cf.get(b, 3, m);
  V t = level_AuT(A.cf, A.W, M, m, A.W[b * 64u + m], c, k0, k1, k2);
  A.RHO[b * 64u + m] -= t;
}

// Coupling of level l to the coarser leaves, transposed: on the leaf bricks
// of level l-1 (the range), RHO_J += sum over the fine T-face cells f next
// to J of (k_f / 2) W_f (the fine cells are children of J's inner neighbour).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_coupling(LevelArgsT<V, CL, CI> A) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  if (!(M.flags & kFlagInner)) return;
  if (!((act_mask(M) >> m) & 1ull)) return;
  V acc = V(0);
  for (int d = 0; d < 6; ++d) {
    if (!((M.flags >> (8 + d)) & 1u) || !dev_outside(m, d)) continue;
    int a = d >> 1;
    int p = dev_partner(m, d);
    int32_t cb = A.T.child[8 * int64_t(M.nbr[d]) + (p >> 3)];
    int32_t slot = A.T.meta[cb].tplus;
    int base = (p & 7) << 3;
    int facebit = (d & 1) ? 0 : 1;
    for (int t = 0; t < 8; ++t) {
      if (((t >> a) & 1) != facebit) continue;
      int q = base | t;
      V kc = (d & 1) ? A.cf.get(uint32_t(cb), 1 + a, q) : A.cf.tplus(slot, a, dev_face_index(q, a));
      acc += kc * V(0.5) * A.W[uint32_t(cb) * 64u + q];
    }
  }
  A.RHO[b * 64u + m] += acc;
}

// Transposed prolongation input: the children's residual sums move to the
// parents, RHO_P += sum_active_children RHO, SBAR_P = -(that sum).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_restrict(LevelArgsT<V, CL, CI> A) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  bool act = (act_mask(M) >> m) & 1ull;
  V s = group8_sum(act ? A.RHO[b * 64u + m] : V(0));
  if ((m & 7) == 0) {
    uint32_t P = uint32_t(M.parent);
    int q = (octant_of(M) << 3) | (m >> 3);
    A.RHO[P * 64u + q] += s;
    A.SBAR[(P - A.T.nlb) * 64u + q] = -s;
  }
}

// After the coarse recursion, on the bricks of level l-1: inner cells move
// RHO into SBAR and zero it, keep Y (active) in YS and W, zero Y; leaf
// bricks set W = 0.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_coarse(LevelArgsT<V, CL, CI> A) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  if (b < A.T.nlb) {
    A.W[b * 64u + m] = V(0);
    return;
  }
  const BrickMeta M = A.T.meta[b];
  bool act = (act_mask(M) >> m) & 1ull;
  uint32_t j = (b - A.T.nlb) * 64u + m;
  A.SBAR[j] += A.RHO[b * 64u + m];
  A.RHO[b * 64u + m] = V(0);
  V yb = act ? A.Y[b * 64u + m] : V(0);
  A.YS[j] = yb;
  A.W[b * 64u + m] = yb;
  A.Y[b * 64u + m] = V(0);
}

// On the bricks of level l-1: t = (A^{l-1})^T W (W = YS on inner cells, 0 on
// leaves); inner cells SBAR += t, leaf cells RHO += t.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_fas(LevelArgsT<V, CL, CI> A) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  V c = A.cf.get(b, 0, m), k0 = A.cf.get(b, 1, m), k1 = A.cf.get(b, 2, m),
    k2 = A.cf.get(b, 3, m);
  V t = level_AuT(A.cf, A.W, M, m, A.W[b * 64u + m], c, k0, k1, k2);
  if (b < A.T.nlb)
    A.RHO[b * 64u + m] += t;
  else
    A.SBAR[(b - A.T.nlb) * 64u + m] += t;
}

// On the bricks of level l: active cells RHO += SBAR_P / n_active(P),
// tbar = (beta_mg / alpha) YS_P, Y += tbar, W = tbar (0 on inactive cells).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_prolong(LevelArgsT<V, CL, CI> A) {
  uint32_t i = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (i >= A.R.n()) return;
  uint32_t b = A.R.brick(i);
  const BrickMeta M = A.T.meta[b];
  uint64_t amask = act_mask(M);
  bool act = (amask >> m) & 1ull;
  V tb = V(0);
  if (act) {
    uint32_t P = uint32_t(M.parent);
    int q = (octant_of(M) << 3) | (m >> 3);
    int cnt = __popcll((amask >> (m & 56)) & 0xffull);
    uint32_t j = (P - A.T.nlb) * 64u + q;
    A.RHO[b * 64u + m] += A.SBAR[j] / V(cnt);
    tb = A.bscale * A.YS[j];
    A.Y[b * 64u + m] += tb;
  }
  A.W[b * 64u + m] = tb;
}

// Coarsest level, transposed: the half-sweeps of k_coarsest in reverse
// order, each as w = RHO / c on the colour, Y += w, RHO -= A^T w.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(1024) k_T_coarsest(LevelArgsT<V, CL, CI> A, int nu) {
  uint32_t w = wave_id();
  uint32_t nw = blockDim.x / kWave;
  int m = threadIdx.x & (kWave - 1);
  int half = nu / 2;
  for (int it = 0; it < nu; ++it) {
    for (int h2 = 0; h2 < 2; ++h2) {
      int colour = it < nu - half ? h2 : 1 - h2;
      for (uint32_t i = w; i < A.R.n(); i += nw) {
        uint32_t b = A.R.brick(i);
        const BrickMeta M = A.T.meta[b];
        bool act = (act_mask(M) >> m) & 1ull;
        int col = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
        V x = V(0);
        if (act && col == colour) x = div_by(A.RHO[b * 64u + m], A.cf.get(b, 0, m));
        A.W[b * 64u + m] = x;
        A.Y[b * 64u + m] += x;
      }
      __threadfence_block();
      __syncthreads();
      for (uint32_t i = w; i < A.R.n(); i += nw) {
        uint32_t b = A.R.brick(i);
        const BrickMeta M = A.T.meta[b];
        V c = A.cf.get(b, 0, m), k0 = A.cf.get(b, 1, m), k1 = A.cf.get(b, 2, m),
          k2 = A.cf.get(b, 3, m);
        V t = level_AuT(A.cf, A.W, M, m, A.W[b * 64u + m], c, k0, k1, k2);
        A.RHO[b * 64u + m] -= t;
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// leaf part of the transposed cycle's residual from an FP64 leaf vector
template <class V>
__global__ void k_T_load(const double *src, V *dst, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = V(src[i]);
}

template <class V>
__global__ void k_fill(V *x, int64_t n, V v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace mfmg
