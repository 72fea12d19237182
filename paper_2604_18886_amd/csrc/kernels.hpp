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

// Per brick: for each axis a, the parent brick's same-level neighbour on the
// brick's side of the parent along a (the parent's nbr[2 a + bit a of the
// brick's octant]); -1 where there is none or the brick has no parent.  The
// brick across face d of axis a has that brick as its parent when the face
// lies on the parent's face, and the brick's own parent otherwise.
struct alignas(16) ParentNbrs {
  int32_t across[3];
  int32_t pad;
};

struct Topo {
  uint32_t nlb;            // leaf bricks (device ids 0 .. nlb-1)
  uint32_t nb;             // all bricks
  const BrickMeta *meta;   // nb records
  const int32_t *child;    // 8 per brick (octant dx + 2 dy + 4 dz), -1 for leaves
  const ParentNbrs *pnb;   // nb entries (hierarchies only; null elsewhere)
};

// Bricks of one level: a leaf range followed by an inner range.
struct Range {
  uint32_t leaf_lo, n_leaf, inner_lo, n_inner;
  __device__ __forceinline__ uint32_t brick(uint32_t i) const {
    return i < n_leaf ? leaf_lo + i : inner_lo + (i - n_leaf);
  }
  __host__ __device__ uint32_t n() const { return n_leaf + n_inner; }
};

// Brick records are never written by a kernel that reads them: loading them
// through the constant address space lets a wave-uniform load be a scalar
// load even after the kernel has stored to other arrays.
__device__ __forceinline__ BrickMeta load_meta(const BrickMeta *meta, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) BrickMeta *)meta)[b];
#else
  return meta[b];  // host pass: never executed
#endif
}

__device__ __forceinline__ ParentNbrs load_parent_nbrs(const ParentNbrs *pnb, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) ParentNbrs *)pnb)[b];
#else
  return pnb[b];  // host pass: never executed
#endif
}

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
// cell m of brick M across direction d at a T-junction: the coarse cell
// holding the fine position next to m, i.e. that position's global
// coordinates halved.  J's cells start at a multiple of 4 on every axis, so
// the local index is the halved coordinate modulo 4 and J's own record is
// not needed.
__device__ __forceinline__ int coarse_local(const BrickMeta &M, int m, int d) {
  int a = d >> 1;
  int s = (d & 1) ? 1 : -1;
  int loc[3] = {dev_cx(m), dev_cy(m), dev_cz(m)};
  int c[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    int g = M.coord[ax] * 4 + loc[ax] + (ax == a ? s : 0);
    c[ax] = (g >> 1) & 3;
  }
  return dev_morton(c[0], c[1], c[2]);
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

// The parent-neighbour table (ParentNbrs), one thread per brick.
__global__ void __launch_bounds__(kBlock) k_parent_nbrs(Topo T, ParentNbrs *out) {
  uint32_t b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= T.nb) return;
  const BrickMeta &M = T.meta[b];
  ParentNbrs r;
  r.pad = 0;
  for (int a = 0; a < 3; ++a) {
    r.across[a] = -1;
    if (M.parent >= 0) {
      int side = (octant_of(M) >> a) & 1;
      r.across[a] = T.meta[M.parent].nbr[2 * a + side];
    }
  }
  out[b] = r;
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
// FP16 copy of an inner coefficient scaled to c / h_l (through FP32, round to
// nearest even).  A non-zero value that would land below FP16's normal range
// (2^-14) is stored as 2^-14 with its sign: a sliver face keeps a small
// positive coupling instead of vanishing, so no cell that is active in FP64
// gets a zero diagonal in the mixed-precision cycle.
__device__ __forceinline__ __half half_coef(double v) {
  __half q = __float2half_rn(float(v));
  if (v != 0.0 && fabsf(__half2float(q)) < 0x1p-14f)
    q = __float2half_rn(v < 0.0 ? -0x1p-14f : 0x1p-14f);
  return q;
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
    dst[i * 256u + comp * 64 + m] = half_coef(coef[b * 256u + comp * 64 + m] * inv_h);
}

// Plus-face coefficients of every brick, for the level kernels: entry
// a * 16 + f is the coefficient of the face between the brick's cell on its
// +a side with face index f and what lies beyond it -- the same-level
// neighbour's k_a (in mixed precision rounded exactly as the neighbour's own
// coefficients are stored), or the T-face coefficient K_F.  At a +a domain
// wall it is the part of the cell's diagonal not carried by its other five
// faces (the wall's coefficient; 0 at a Neumann wall), so that for every cell
// the diagonal is the sum of the six face coefficients the stencil sees
// (Eq. 3; Algorithm 3 keeps this on every level).  A cell on several +walls
// carries that part on the first of them.
template <class CL>
__global__ void __launch_bounds__(kBlock) k_plus_faces(Topo T, const double *coef,
                                                       const double *tc, CL *pf, int half_inner) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int e = threadIdx.x & (kWave - 1);
  if (b >= T.nb || e >= 48) return;
  int a = e >> 4, f = e & 15;
  int c[3];
  c[a] = 3;
  c[a == 0 ? 1 : 0] = f & 3;
  c[a == 2 ? 1 : 2] = f >> 2;
  int m = dev_morton(c[0], c[1], c[2]);
  const BrickMeta M = T.meta[b];
  const double *own = coef + uint64_t(b) * 256u;
  double kp[3];
  bool wall[3];
  bool inner_nbr = false;
  for (int ax = 0; ax < 3; ++ax) {
    int dd = 2 * ax + 1;
    kp[ax] = 0.0;
    wall[ax] = false;
    int p = dev_partner(m, dd);
    if (!dev_outside(m, dd)) {
      kp[ax] = own[(1 + ax) * 64 + p];
      continue;
    }
    int32_t n = M.nbr[dd];
    if (n >= 0) {
      kp[ax] = coef[uint64_t(n) * 256u + (1 + ax) * 64 + p];
      if (ax == a) inner_nbr = uint32_t(n) >= T.nlb;
    } else if ((M.flags >> dd) & 1u) {
      kp[ax] = tc[uint32_t(M.tplus) * 48u + ax * 16 + dev_face_index(m, ax)];
    } else {
      wall[ax] = true;
    }
  }
  double v = kp[a];
  if (wall[a]) {
    int first = wall[0] ? 0 : (wall[1] ? 1 : 2);
    v = first == a ? own[m] - (own[64 + m] + own[128 + m] + own[192 + m]) -
                         (kp[0] + kp[1] + kp[2])
                   : 0.0;
  } else if (half_inner && inner_nbr) {
    float hv = __half2float(half_coef(v * ldexp(1.0, M.level)));
    v = double(hv * ldexpf(1.0f, -M.level));
  }
  pf[b * 48u + e] = CL(v);
}

// ---------------------------------------------------------------------------
// multigrid cycle kernels.  A wave processes one brick at a time and loops
// over the bricks of a level; everything that depends only on the lane is
// computed once, outside the loop, and every per-brick address is scalar
// arithmetic (buffer loads with a uniform base).
// ---------------------------------------------------------------------------
template <class V, class CL, class CI>
struct LevelArgs {
  Topo T;
  Coefs<V, CL, CI> cf;
  const CL *pf;      // plus-face coefficients, 48 per brick (k_plus_faces)
  V *U;              // iterate, nb * 64
  V *B;              // right-hand side, nb * 64 (leaf part: the PCG residual)
  V *Ustar;          // FAS initial guess of inner cells, (nb - nlb) * 64
  Range R;
  const int *done;   // skip when the solve has stopped
};

// A voffset at or above this is out of range for every buffer the level
// kernels read (all are below 2 GiB): such a load returns 0.
constexpr uint32_t kOutOfRange = 0x80000000u;

// Lane constants: the lane's cell, its partners across the six directions,
// and the byte offsets the stencil's loads use.
template <class V, class CL>
struct LaneC {
  uint32_t m;        // local Morton index
  int p[6];          // partner cell across direction d (this brick or the next)
  bool out[6];       // the partner lies in the neighbouring brick
  uint32_t poff[6];  // out[d] ? p * sizeof(V) : kOutOfRange
  uint32_t foff[3];  // plus-face slot of the cell on axis a, in bytes
  int colour;        // (x + y + z) & 1
  int esrc[6];       // fused prolongation: lane holding the correction of the
                     // parent of the neighbour across d (prolong_gather)
  // FP64 only: gathered face loads of the full stencil (see stencil_sum)
  uint32_t goff[2];  // lane k < 48 of gather h: byte offset of its value in the brick
  int gdir[2];       //   across face 3h + k / 16 (that face; 6 for k >= 48)
  int gsrc[6];       // 4 x the lane holding the value across face d (gather d / 3)
  int psrc[6];       // 4 x p[d]
  uint32_t pfoff;    // lane k < 48: byte offset of plus-face entry k
  int pfsrc[3];      // 4 x the lane holding the lane's plus-face entry of axis a
};

template <class V, class CL>
__device__ __forceinline__ LaneC<V, CL> lane_consts() {
  LaneC<V, CL> L;
  L.m = threadIdx.x & (kWave - 1);
  int m = int(L.m);
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    L.p[d] = dev_partner(m, d);
    L.out[d] = dev_outside(m, d);
    L.poff[d] = L.out[d] ? uint32_t(L.p[d]) * uint32_t(sizeof(V)) : kOutOfRange;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    L.foff[a] = uint32_t(a * 16 + dev_face_index(m, a)) * uint32_t(sizeof(CL));
  L.colour = (dev_cx(m) + dev_cy(m) + dev_cz(m)) & 1;
#pragma unroll
  for (int d = 0; d < 6; ++d) L.esrc[d] = (L.out[d] ? 8 * (1 + d) : 0) + (L.p[d] >> 3);
  if constexpr (sizeof(V) == 8) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      L.gdir[h] = 6;
      L.goff[h] = kOutOfRange;
      if (m < 48) {
        int d = 3 * h + (m >> 4), a = d >> 1;
        int o0 = a == 0 ? 1 : 0;
        int o1 = a == 2 ? 1 : 2;
        int f = m & 15;
        int xyz[3];
        xyz[a] = (d & 1) ? 3 : 0;
        xyz[o0] = f & 3;
        xyz[o1] = f >> 2;
        L.gdir[h] = d;
        L.goff[h] = uint32_t(dev_partner(dev_morton(xyz[0], xyz[1], xyz[2]), d)) *
                    uint32_t(sizeof(V));
      }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      L.gsrc[d] = 4 * (16 * (d % 3) + dev_face_index(m, d >> 1));
      L.psrc[d] = 4 * L.p[d];
    }
    L.pfoff = m < 48 ? uint32_t(m) * uint32_t(sizeof(CL)) : kOutOfRange;
#pragma unroll
    for (int a = 0; a < 3; ++a) L.pfsrc[a] = 4 * (a * 16 + dev_face_index(m, a));
  }
  return L;
}

// Bricks of a level range for this wave.  Workgroups are dispatched to the
// eight XCDs in turn (workgroup g on XCD g mod 8); each XCD takes one
// contiguous eighth of the range, so bricks that are close in Morton order,
// and hence mostly each other's neighbours, share that XCD's L2.  The grid
// is a multiple of 8 workgroups.
struct WaveLoop {
  uint32_t first, end, step;
};
// The loop of workgroup `block` of a grid of `blocks` (a multiple of 8).
__device__ __forceinline__ WaveLoop wave_loop_of(uint32_t n, uint32_t block, uint32_t blocks) {
  uint32_t x = block & 7u;
  uint32_t j = (block >> 3) * kWavesPerBlock + wave_id();
  uint32_t chunk = (n + 7u) >> 3;
  uint32_t lo = x * chunk;
  uint32_t hi = lo + chunk < n ? lo + chunk : n;
  return {lo + j, hi, (blocks >> 3) * kWavesPerBlock};
}
__device__ __forceinline__ WaveLoop wave_loop(uint32_t n) {
  return wave_loop_of(n, blockIdx.x, gridDim.x);
}

// CP: cache policy of the loads whose data a launch uses once (coefficient
// arrays, plus-face table, right-hand side).  On a level larger than the
// Infinity Cache these are loaded non-temporal, so that the iterate -- the
// only array read again for neighbouring bricks -- keeps the L2; on smaller
// levels everything stays cached for the next half-sweep.  kCpolStreamCoef
// streams only the coefficients: the FP32 cycle's finest level then keeps
// its iterate, right-hand side and plus-face table (216 MB on the large
// workload) in the 256 MB Infinity Cache from one half-sweep to the next.
template <class V, class CL, class CI, int CP = kCpolDefault>
struct LevelView {
  __amdgpu_buffer_rsrc_t u, b, us, cl, ci, pf;
  const BrickMeta *meta;
  const ParentNbrs *pnb;
  uint32_t nlb;
  V iscale;
};

template <int CP = kCpolDefault, class V, class CL, class CI>
__device__ __forceinline__ LevelView<V, CL, CI, CP> level_view(const LevelArgs<V, CL, CI> &A) {
  LevelView<V, CL, CI, CP> X;
  uint64_t nb = A.T.nb, nlb = A.T.nlb;
  X.u = make_rsrc(A.U, nb * 64 * sizeof(V));
  X.b = make_rsrc(A.B, nb * 64 * sizeof(V));
  X.us = make_rsrc(A.Ustar, (nb - nlb) * 64 * sizeof(V));
  X.cl = make_rsrc(A.cf.leaf, nlb * 256 * sizeof(CL));
  X.ci = make_rsrc(A.cf.inner, (nb - nlb) * 256 * sizeof(CI));
  X.pf = make_rsrc(A.pf, nb * 48 * sizeof(CL));
  X.meta = A.T.meta;
  X.pnb = A.T.pnb;
  X.nlb = A.T.nlb;
  X.iscale = A.cf.iscale;
  return X;
}

// Coefficient comp (0 = c, 1 + a = k_a) of the lane's cell of brick b;
// INNER selects the inner-brick array (FP16 in mixed precision, stored
// divided by the cell size).
template <bool INNER, class V, class CL, class CI, int CP>
__device__ __forceinline__ V own_coef(const LevelView<V, CL, CI, CP> &X, uint32_t b, int comp,
                                      uint32_t m) {
  if constexpr (INNER) {
    V v = V(bload<CI, coef_pol(CP)>(X.ci, m, (b - X.nlb) * 256u + uint32_t(comp) * 64u));
    if constexpr (std::is_same<CL, CI>::value) return v;
    else return v * X.iscale;
  } else {
    return V(bload<CL, coef_pol(CP)>(X.cl, m, b * 256u + uint32_t(comp) * 64u));
  }
}

template <class T, int CPOL = kCpolDefault>
__device__ __forceinline__ T bload_bytes(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(
        T, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), CPOL));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(
        T, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), CPOL));
  else
    return __builtin_bit_cast(
        T, __builtin_amdgcn_raw_buffer_load_b16(r, int(voff), int(soff), CPOL));
}

// Neighbour sum of the level operator at the lane's cell of brick b:
//   S_m = sum_d k_d v_d,   (A u)_m = c_m u_m - S_m,
// v_d the same-level neighbour value (a lane shuffle inside the brick, a
// load from the neighbouring brick across its faces), 0 at a wall, or at a
// T-junction (Eq. 10) the ghost u_m + (u_J - mean of the active siblings)/2
// with u_J read from the coarser leaf.  k_d is the cell's own k_a on the
// minus side and the neighbour's k_a on the plus side (a shuffle inside
// the brick, the brick's plus-face array across its faces).  The loads
// across a face are issued by every lane with an offset that is out of
// range for the inner lanes and, at a wall or T-face, for all lanes, so
// the only branch is a scalar one around the T-junction ghosts.  diag
// returns c_m as the sum of the six face coefficients (see k_plus_faces),
// so the diagonal is not streamed from memory.
// Values across the six faces of the lane's cell and their coefficients:
// v[d] the same-level neighbour's entry of the vector in buffer x (0 at a
// wall or T-face, where the load is out of range), k[d] the face
// coefficient (own k_a on the minus side, the neighbour's on the plus side).
template <int CP, class V, class CL>
__device__ __forceinline__ void face_values(__amdgpu_buffer_rsrc_t x, __amdgpu_buffer_rsrc_t pf,
                                            const LaneC<V, CL> &L, uint32_t b,
                                            const BrickMeta &M, V u, V k0, V k1, V k2, V (&v)[6],
                                            V (&k)[6]) {
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    V kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    int32_t n = M.nbr[d];
    uint32_t sb = n >= 0 ? uint32_t(n) * uint32_t(64 * sizeof(V)) : kOutOfRange;
    V vl = bload_bytes<V>(x, L.poff[d] + sb, 0);
    V vs = shfl(u, L.p[d]);
    v[d] = L.out[d] ? vl : vs;
    if (d & 1) {
      V kl = V(bload_bytes<CL, side_pol(CP)>(pf, L.foff[a], b * uint32_t(48 * sizeof(CL))));
      V ks = shfl(kown, L.p[d]);
      k[d] = L.out[d] ? kl : ks;
    } else {
      k[d] = kown;
    }
  }
}

// FP64 form of face_values: the brick's 96 face cells take their values
// from two gathered loads (lane k < 48 of gather h fetches the value across
// face 3h + k / 16 for the face cell with face index k % 16) and its 48
// plus-face coefficients from one (lane k: entry k), each cell reading its
// entries by lane exchange.  The face loads of face_values are full-wave
// loads with only the face lanes in range; for 8-byte values the texture
// units' per-lane work on them, not HBM, bounded the stencils.
template <int CP, class V, class CL>
__device__ __forceinline__ void face_values_gathered(__amdgpu_buffer_rsrc_t x,
                                                     __amdgpu_buffer_rsrc_t pf,
                                                     const LaneC<V, CL> &L, uint32_t b,
                                                     const BrickMeta &M, V u, V k0, V k1, V k2,
                                                     V (&v)[6], V (&k)[6]) {
  uint32_t gb0 = 0u, gb1 = 0u;  // bytes to the brick across each gather's face
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    uint32_t sb = M.nbr[d] >= 0 ? uint32_t(M.nbr[d]) * uint32_t(64 * sizeof(V)) : kOutOfRange;
    gb0 = L.gdir[0] == d ? sb : gb0;
    gb1 = L.gdir[1] == d ? sb : gb1;
  }
  V g0 = bload_bytes<V>(x, L.goff[0] + gb0, 0);
  V g1 = bload_bytes<V>(x, L.goff[1] + gb1, 0);
  CL pfv = bload_bytes<CL, side_pol(CP)>(pf, L.pfoff, b * uint32_t(48 * sizeof(CL)));
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    V kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    V vl = bperm(d < 3 ? g0 : g1, L.gsrc[d]);
    V vs = bperm(u, L.psrc[d]);
    v[d] = L.out[d] ? vl : vs;
    if (d & 1) {
      V kl = V(bperm(pfv, L.pfsrc[a]));
      V ks = bperm(kown, L.psrc[d]);
      k[d] = L.out[d] ? kl : ks;
    } else {
      k[d] = kown;
    }
  }
}

// The FAS correction u_P - u*_P of the parent cell of the lane's cell
// (Algorithm 4, prolongation): the brick covers octant o of its parent
// brick, whose cells o * 8 .. o * 8 + 7 are the parents of its 2^3 blocks.
template <class V, class CL, class CI, int CP>
__device__ __forceinline__ V own_correction(const LevelView<V, CL, CI, CP> &X,
                                            const LaneC<V, CL> &L, const BrickMeta &M) {
  uint32_t base = uint32_t(M.parent) * 64u + uint32_t(octant_of(M)) * 8u;
  uint32_t q = L.m >> 3;
  return bload<V>(X.u, q, base) - bload<V>(X.us, q, base - X.nlb * 64u);
}

// Prolongation folded into the first post-smoothing half-sweep of a level.
// Algorithm 4 adds u_P - u*_P to every active cell of the level before the
// post-smoothing; a colour-c half-sweep reads only the colour-c cells' own
// values and their neighbours, so it can add the corrections to what it
// reads instead, and store the corrected colour-c cells it updates.  The
// other colour's cells are left uncorrected in memory: the next half-sweep
// overwrites the active ones without reading their old values, except in
// the T-junction ghosts, where it adds the correction itself (mode 2 of
// smooth_brick).  Inactive cells are not corrected (as before); their face
// coefficients are zero, so a correction added to them changes no sum.
//
// The corrections one brick needs lie in at most seven parent octants: its
// own and those of the bricks across its six faces (octant o ^ (1 << a) of
// the same parent, or of the parent's neighbour when the face lies on the
// parent's face; ParentNbrs).  Lane k < 56 fetches entry k & 7 of octant
// slot k >> 3 (0: the brick's own, 1 + d: across face d) in one load of
// each vector; a face without a same-level brick beyond it (wall,
// T-junction) is out of range and gets a zero correction.  Each lane then
// takes the correction of its own parent cell from lane m >> 3 and that of
// its neighbour across face d (in the brick or beyond it) from lane
// L.esrc[d].
template <class V, class CL, class CI, int CP>
__device__ __forceinline__ V prolong_gather(const LevelView<V, CL, CI, CP> &X,
                                            const LaneC<V, CL> &L, const BrickMeta &M,
                                            const ParentNbrs &PN) {
  // every brick above the coarsest level has a parent
  const bool has_parent = M.parent >= 0;
  const uint32_t P = uint32_t(M.parent);
  const uint32_t o = uint32_t(octant_of(M));
  const uint32_t slot = L.m >> 3;
  uint32_t pb = P, oc = o;
  bool valid = slot == 0u;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int a = d >> 1;
    const uint32_t bit = 1u << a;
    const bool across = ((o & bit) != 0u) == ((d & 1) != 0);
    const int32_t nb = across ? PN.across[a] : int32_t(P);
    if (slot == uint32_t(1 + d)) {
      pb = uint32_t(nb);
      oc = o ^ bit;
      valid = M.nbr[d] >= 0 && nb >= 0;
    }
  }
  valid = valid && has_parent;
  const uint32_t cell = pb * 64u + oc * 8u + (L.m & 7u);
  const uint32_t ou = valid ? cell * uint32_t(sizeof(V)) : kOutOfRange;
  const uint32_t os = valid ? (cell - X.nlb * 64u) * uint32_t(sizeof(V)) : kOutOfRange;
  return bload_bytes<V>(X.u, ou, 0) - bload_bytes<V>(X.us, os, 0);
}

// T-junction ghosts (Eq. 10) of a brick with T-faces: across each T-face d
// the lane's value becomes u_m + (u_J - mean of the active siblings) / 2,
// u_J read from the coarser leaf.  The coarse values of all T-faces are
// requested before any is used, so a brick with several T-faces waits for
// one round trip.  PR as in stencil_sum: the own values get the FAS
// correction first (1: corr from prolong_gather; 2: the not yet stored
// correction of the colour-`colour` cells).
template <int PR, class V, class CL, class CI, int CP>
__device__ __forceinline__ void t_ghosts(const LevelView<V, CL, CI, CP> &X, const LaneC<V, CL> &L,
                                         const BrickMeta &M, V u, V (&v)[6], V corr,
                                         int colour) {
  V uJ[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    uJ[d] = V(0);
    if ((M.flags >> d) & 1u) {
      uint32_t J = uint32_t(dev_decode_coarse(M.nbr[d]));
      uJ[d] = bload<V>(X.u, uint32_t(coarse_local(M, int(L.m), d)), J * 64u);
    }
  }
  uint64_t amask = act_mask(M);
  bool act = (amask >> L.m) & 1ull;
  if constexpr (PR == 1) {
    // every lane takes part in the exchange (a lane exchange in a
    // conditional would read inactive lanes)
    const V eo = shfl(corr, int(L.m >> 3));
    u = act ? u + eo : u;
  }
  if constexpr (PR == 2) u = act && L.colour == colour ? u + own_correction(X, L, M) : u;
  V s = group8_sum(act ? u : V(0));
  int cnt = __popcll((amask >> (L.m & 56u)) & 0xffull);
  V ubar = cnt ? s / V(cnt) : V(0);
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if ((M.flags >> d) & 1u) {
      V g = u + (uJ[d] - ubar) * V(0.5);
      v[d] = L.out[d] ? g : v[d];
    }
  }
}

// PR: 0 the plain stencil; 1 the first post-smoothing half-sweep with the
// prolongation folded in (corr from prolong_gather: every neighbour value
// gets the correction of its parent cell, the T-junction ghosts use the
// corrected own and sibling values); 2 the half-sweep after it (the
// ghosts of the colour-`colour` cells add their own, not yet stored,
// correction).
template <int PR = 0, class V, class CL, class CI, int CP>
__device__ __forceinline__ V stencil_sum(const LevelView<V, CL, CI, CP> &X, const LaneC<V, CL> &L,
                                         uint32_t b, const BrickMeta &M, V u, V k0, V k1,
                                         V k2, V &diag, V corr = V(0), int colour = 0) {
  V v[6], k[6];
  if constexpr (sizeof(V) == 8)
    face_values_gathered<CP>(X.u, X.pf, L, b, M, u, k0, k1, k2, v, k);
  else
    face_values<CP>(X.u, X.pf, L, b, M, u, k0, k1, k2, v, k);
  if constexpr (PR == 1) {
#pragma unroll
    for (int d = 0; d < 6; ++d) v[d] = v[d] + shfl(corr, L.esrc[d]);
  }
  if (M.flags & kFlagT) {
    if constexpr (sizeof(V) == 8) {
      t_ghosts<PR>(X, L, M, u, v, corr, colour);
    } else {
      // FP32: the ghosts face by face (each coarse value waited for before
      // the next is requested); the hoisted form of t_ghosts made the
      // compiler schedule the whole FP32 stencil worse (finest half-sweep
      // 114 -> 119 us), while it speeds up the FP64 one
      uint64_t amask = act_mask(M);
      bool act = (amask >> L.m) & 1ull;
      if constexpr (PR == 1) {
        // every lane takes part in the exchange (a lane exchange in a
        // conditional would read inactive lanes)
        const V eo = shfl(corr, int(L.m >> 3));
        u = act ? u + eo : u;
      }
      if constexpr (PR == 2) u = act && L.colour == colour ? u + own_correction(X, L, M) : u;
      V s = group8_sum(act ? u : V(0));
      int cnt = __popcll((amask >> (L.m & 56u)) & 0xffull);
      V ubar = cnt ? s / V(cnt) : V(0);
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if ((M.flags >> d) & 1u) {
          uint32_t J = uint32_t(dev_decode_coarse(M.nbr[d]));
          V uJ = bload<V>(X.u, uint32_t(coarse_local(M, int(L.m), d)), J * 64u);
          V g = u + (uJ - ubar) * V(0.5);
          v[d] = L.out[d] ? g : v[d];
        }
      }
    }
  }
  diag = ((k[0] + k[1]) + (k[2] + k[3])) + (k[4] + k[5]);
  V acc = V(0);
#pragma unroll
  for (int d = 0; d < 6; ++d) acc += k[d] * v[d];
  return acc;
}

// One brick of a colour half-sweep of red-black Gauss-Seidel: on the cells
// of the colour u_m = (b_m + S_m) / c_m, every read taken before the write
// (the neighbours of a cell all have the other colour).  PR = 1: the first
// post-smoothing half-sweep with the prolongation folded in; PR = 2: the
// one after it (see prolong_gather).
template <bool INNER, int PR, class V, class CL, class CI, int CP>
__device__ __forceinline__ void smooth_brick(const LevelView<V, CL, CI, CP> &X, const LaneC<V, CL> &L,
                                             uint32_t b, int colour) {
  const BrickMeta M = load_meta(X.meta, b);
  V corr = V(0);
  if constexpr (PR == 1) corr = prolong_gather(X, L, M, load_parent_nbrs(X.pnb, b));
  V k0 = own_coef<INNER>(X, b, 1, L.m);
  V k1 = own_coef<INNER>(X, b, 2, L.m);
  V k2 = own_coef<INNER>(X, b, 3, L.m);
  V u = bload<V>(X.u, L.m, b * 64u);
  V rhs = bload<V, side_pol(CP)>(X.b, L.m, b * 64u);
  V c;
  V S = stencil_sum<PR>(X, L, b, M, u, k0, k1, k2, c, corr, colour);
  bool act = (act_mask(M) >> L.m) & 1ull;
  if (act && L.colour == colour) bstore<V>(X.u, L.m, b * 64u, div_by(rhs + S, c));
}

// Gathered face loads of an FP64 colour-c half-sweep.  The loads of the
// stencil are limited by the texture units' per-lane work, and the six face
// loads of stencil_sum are full-wave loads of which only the face lanes are
// in range.  The brick's colour-c cells on its six faces need 48 values from
// the neighbouring bricks (8 per face); lane k = 8 d + j (k < 48) fetches the
// one for the j-th such cell of face d in a single load and each cell takes
// its value from that lane with a lane exchange.  Likewise one load brings
// the brick's 48 plus-face coefficients (lane k: entry k).  A face's cells
// are numbered by their face index f (dev_face_index); cells f = 2j and
// 2j + 1 have opposite colours, and the colour-c one is the j-th.  (For FP32
// the exchanges cost more than the loads they save, and the six face loads
// stay.)
struct HalfGather {
  uint32_t goff;   // k < 48: byte offset of lane k's value in the brick across face k / 8
  int gdir;        // k / 8 for k < 48, 6 (no load) otherwise
  int gsrc[6];     // 4 x the lane holding the value across face d for the lane's cell
  int psrc[6];     // 4 x the lane's partner lane across direction d
  uint32_t pfoff;  // k < 48: byte offset of plus-face entry k, else out of range
  int pfsrc[3];    // 4 x the lane holding the lane's plus-face entry of axis a
};

template <class V, class CL>
__device__ __forceinline__ HalfGather half_gather(const LaneC<V, CL> &L, int colour) {
  HalfGather G;
  int k = int(L.m);
  G.gdir = k < 48 ? k >> 3 : 6;
  G.goff = kOutOfRange;
  if (k < 48) {
    int d = k >> 3, a = d >> 1;
    int o0 = a == 0 ? 1 : 0;
    int o1 = a == 2 ? 1 : 2;
    int side = (d & 1) ? 3 : 0;
    int f = 2 * (k & 7);
    if (((side + (f & 3) + (f >> 2)) & 1) != colour) f += 1;
    int xyz[3];
    xyz[a] = side;
    xyz[o0] = f & 3;
    xyz[o1] = f >> 2;
    int p = dev_partner(dev_morton(xyz[0], xyz[1], xyz[2]), d);
    G.goff = uint32_t(p) * uint32_t(sizeof(V));
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    G.gsrc[d] = 4 * (8 * d + (dev_face_index(k, d >> 1) >> 1));
    G.psrc[d] = 4 * L.p[d];
  }
  G.pfoff = k < 48 ? uint32_t(k) * uint32_t(sizeof(CL)) : kOutOfRange;
#pragma unroll
  for (int a = 0; a < 3; ++a) G.pfsrc[a] = 4 * (a * 16 + dev_face_index(k, a));
  return G;
}

// One brick of a colour half-sweep with gathered face loads: the values,
// ghosts and sums of smooth_brick, term for term.
template <bool INNER, int PR, class V, class CL, class CI, int CP>
__device__ __forceinline__ void smooth_brick_gathered(const LevelView<V, CL, CI, CP> &X,
                                                      const LaneC<V, CL> &L, const HalfGather &G,
                                                      uint32_t b, int colour) {
  const BrickMeta M = load_meta(X.meta, b);
  V k0 = own_coef<INNER>(X, b, 1, L.m);
  V k1 = own_coef<INNER>(X, b, 2, L.m);
  V k2 = own_coef<INNER>(X, b, 3, L.m);
  V u = bload<V>(X.u, L.m, b * 64u);
  V rhs = bload<V, side_pol(CP)>(X.b, L.m, b * 64u);
  const bool act = (act_mask(M) >> L.m) & 1ull;
  V corr = V(0);
  if constexpr (PR == 1) corr = prolong_gather(X, L, M, load_parent_nbrs(X.pnb, b));
  uint32_t gb = 0u;  // byte offset of the brick across the lane's gather face
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    uint32_t sb = M.nbr[d] >= 0 ? uint32_t(M.nbr[d]) * uint32_t(64 * sizeof(V)) : kOutOfRange;
    gb = G.gdir == d ? sb : gb;
  }
  V gv = bload_bytes<V>(X.u, G.goff + gb, 0);
  CL pfv = bload_bytes<CL, side_pol(CP)>(X.pf, G.pfoff, b * uint32_t(48 * sizeof(CL)));
  V v[6], k[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    V kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    V vl = bperm(gv, G.gsrc[d]);
    V vs = bperm(u, G.psrc[d]);
    v[d] = L.out[d] ? vl : vs;
    if constexpr (PR == 1) v[d] = v[d] + shfl(corr, L.esrc[d]);
    if (d & 1) {
      V kl = V(bperm(pfv, G.pfsrc[a]));
      V ks = bperm(kown, G.psrc[d]);
      k[d] = L.out[d] ? kl : ks;
    } else {
      k[d] = kown;
    }
  }
  if (M.flags & kFlagT) t_ghosts<PR>(X, L, M, u, v, corr, colour);
  V c = ((k[0] + k[1]) + (k[2] + k[3])) + (k[4] + k[5]);
  V S = V(0);
#pragma unroll
  for (int d = 0; d < 6; ++d) S += k[d] * v[d];
  if (act && L.colour == colour) bstore<V>(X.u, L.m, b * 64u, div_by(rhs + S, c));
}

// PR: 0 a plain half-sweep, 1 the first post-smoothing half-sweep with the
// prolongation folded in, 2 the half-sweep after it (smooth_brick).
template <class V, class CL, class CI, int CP = kCpolDefault, int PR = 0>
__global__ void __launch_bounds__(kBlock) k_smooth(LevelArgs<V, CL, CI> A, int colour) {
  if (A.done && *A.done) return;
  if constexpr (sizeof(V) == 8) {
    const LaneC<V, CL> L = lane_consts<V, CL>();
    const HalfGather G = half_gather(L, colour);
    const LevelView<V, CL, CI, CP> X = level_view<CP>(A);
    const WaveLoop W = wave_loop(A.R.n());
    for (uint32_t i = W.first; i < W.end; i += W.step) {
      if (i < A.R.n_leaf) smooth_brick_gathered<false, PR>(X, L, G, A.R.leaf_lo + i, colour);
      else smooth_brick_gathered<true, PR>(X, L, G, A.R.inner_lo + (i - A.R.n_leaf), colour);
    }
  } else {
    const LaneC<V, CL> L = lane_consts<V, CL>();
    const LevelView<V, CL, CI, CP> X = level_view<CP>(A);
    const WaveLoop W = wave_loop(A.R.n());
    for (uint32_t i = W.first; i < W.end; i += W.step) {
      if (i < A.R.n_leaf) smooth_brick<false, PR>(X, L, A.R.leaf_lo + i, colour);
      else smooth_brick<true, PR>(X, L, A.R.inner_lo + (i - A.R.n_leaf), colour);
    }
  }
}

// The first half-sweep of a level whose bricks are all leaves, from a zero
// iterate: every neighbour, ghost and wall value is 0, so the sweep sets
// u = b / c on the cells of the colour and 0 on all others (which also
// clears the iterate).
template <class V, class CL, class CI, int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_smooth_zero(LevelArgs<V, CL, CI> A, int colour) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI, CP> X = level_view<CP>(A);
  const WaveLoop W = wave_loop(A.R.n_leaf);
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    uint32_t b = A.R.leaf_lo + i;
    const BrickMeta M = load_meta(X.meta, b);
    bool act = (act_mask(M) >> L.m) & 1ull;
    V c = own_coef<false>(X, b, 0, L.m);
    V rhs = bload<V, side_pol(CP)>(X.b, L.m, b * 64u);
    bstore<V>(X.u, L.m, b * 64u, act && L.colour == colour ? div_by(rhs, c) : V(0));
  }
}

// Residual, restriction and FAS initial guess from one brick of level l to
// its parent cells:  b_P = beta_mg (1/alpha) sum_children r,
// u_P = u*_P = mean of the active children (k_fas_rhs then adds
// A^{l-1} u* on inner cells).
template <bool INNER, class V, class CL, class CI, int CP>
__device__ __forceinline__ void restrict_brick(const LevelView<V, CL, CI, CP> &X,
                                               const LaneC<V, CL> &L,
                                               uint32_t b, V scale) {
  const BrickMeta M = load_meta(X.meta, b);
  V k0 = own_coef<INNER>(X, b, 1, L.m);
  V k1 = own_coef<INNER>(X, b, 2, L.m);
  V k2 = own_coef<INNER>(X, b, 3, L.m);
  V u = bload<V>(X.u, L.m, b * 64u);
  V rhs = bload<V, side_pol(CP)>(X.b, L.m, b * 64u);
  V c;
  V S = stencil_sum(X, L, b, M, u, k0, k1, k2, c);
  uint64_t amask = act_mask(M);
  bool act = (amask >> L.m) & 1ull;
  V r = act ? rhs - (c * u - S) : V(0);
  V rs = group8_sum(r);
  V us = group8_sum(act ? u : V(0));
  int cnt = __popcll((amask >> (L.m & 56u)) & 0xffull);
  if ((L.m & 7u) == 0) {
    uint32_t base = uint32_t(M.parent) * 64u + uint32_t(octant_of(M)) * 8u;
    uint32_t q = L.m >> 3;
    V ust = cnt ? div_by(us, V(cnt)) : V(0);
    bstore<V>(X.b, q, base, rs * scale);
    bstore<V>(X.u, q, base, ust);
    bstore<V>(X.us, q, base - X.nlb * 64u, ust);
  }
}

template <class V, class CL, class CI, int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_restrict(LevelArgs<V, CL, CI> A, V scale) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI, CP> X = level_view<CP>(A);
  const WaveLoop W = wave_loop(A.R.n());
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    if (i < A.R.n_leaf) restrict_brick<false>(X, L, A.R.leaf_lo + i, scale);
    else restrict_brick<true>(X, L, A.R.inner_lo + (i - A.R.n_leaf), scale);
  }
}

// FAS coarse right-hand side on inner bricks: b += A^{l-1} u*.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_fas_rhs(LevelArgs<V, CL, CI> A) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI> X = level_view(A);
  const WaveLoop W = wave_loop(A.R.n_inner);
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    uint32_t b = A.R.inner_lo + i;
    const BrickMeta M = load_meta(X.meta, b);
    V k0 = own_coef<true>(X, b, 1, L.m);
    V k1 = own_coef<true>(X, b, 2, L.m);
    V k2 = own_coef<true>(X, b, 3, L.m);
    V u = bload<V>(X.u, L.m, b * 64u);
    V rhs = bload<V>(X.b, L.m, b * 64u);
    V c;
    V S = stencil_sum(X, L, b, M, u, k0, k1, k2, c);
    bool act = (act_mask(M) >> L.m) & 1ull;
    bstore<V>(X.b, L.m, b * 64u, act ? rhs + (c * u - S) : V(0));
  }
}

// The first pre-smoothing half-sweep of a level with the FAS right-hand
// side folded in, for a level with no leaf at or below it (all its bricks
// are inner, none has a T-face).  Right after the restriction u = u* on
// every cell, so one neighbour sum S of u* gives both b += c u* - S (stored
// on every cell, as k_fas_rhs) and, on the cells of the colour,
// u = (b + S) / c (as k_smooth).  The sum is read from the u* array, which
// this launch does not write, so no brick's sum can see another brick's
// update; values and sums are those of k_fas_rhs and k_smooth.  A
// neighbour that is not an inner brick (none, on such a level) would read
// as a wall.
template <class V, class CL, class CI, int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_smooth_fas(LevelArgs<V, CL, CI> A, int colour) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI, CP> X = level_view<CP>(A);
  LevelView<V, CL, CI, CP> Xs = X;  // u = u*, indexed by brick id - nlb
  Xs.u = X.us;
  const WaveLoop W = wave_loop(A.R.n_inner);
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    uint32_t b = A.R.inner_lo + i;
    const BrickMeta M = load_meta(X.meta, b);
    BrickMeta Ms = M;
#pragma unroll
    for (int d = 0; d < 6; ++d)
      Ms.nbr[d] = M.nbr[d] >= int32_t(X.nlb) ? M.nbr[d] - int32_t(X.nlb) : -1;
    Ms.flags = M.flags & ~uint32_t(kFlagT);
    V k0 = own_coef<true>(X, b, 1, L.m);
    V k1 = own_coef<true>(X, b, 2, L.m);
    V k2 = own_coef<true>(X, b, 3, L.m);
    V u = bload<V>(X.us, L.m, (b - X.nlb) * 64u);
    V rhs = bload<V, side_pol(CP)>(X.b, L.m, b * 64u);
    V c;
    V S = stencil_sum(Xs, L, b, Ms, u, k0, k1, k2, c);
    bool act = (act_mask(M) >> L.m) & 1ull;
    V rf = act ? rhs + (c * u - S) : V(0);
    bstore<V>(X.b, L.m, b * 64u, rf);
    if (act && L.colour == colour) bstore<V>(X.u, L.m, b * 64u, div_by(rf + S, c));
  }
}

// Prolongation of the FAS correction: u += u_P - u*_P on active cells.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_prolong(LevelArgs<V, CL, CI> A) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI> X = level_view(A);
  const WaveLoop W = wave_loop(A.R.n());
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    uint32_t b = A.R.brick(i);
    const BrickMeta M = load_meta(X.meta, b);
    uint32_t base = uint32_t(M.parent) * 64u + uint32_t(octant_of(M)) * 8u;
    uint32_t q = L.m >> 3;
    V corr = bload<V>(X.u, q, base) - bload<V>(X.us, q, base - X.nlb * 64u);
    V u = bload<V>(X.u, L.m, b * 64u);
    if ((act_mask(M) >> L.m) & 1ull) bstore<V>(X.u, L.m, b * 64u, u + corr);
  }
}

// Coarsest level: nu RBGS iterations in one workgroup, (R,B) for the first
// half of the iterations and (B,R) for the rest.  The level is a complete
// grid of at most kCoarsestBricks bricks (no T-junctions), so its iterate
// stays in LDS and each wave keeps the coefficients of its bricks (at most
// kCoarsestSlots) in registers for all 2 nu half-sweeps; every value read,
// and the order of every sum, is that of the global-memory half-sweep.
constexpr int kCoarsestBricks = 64;
constexpr int kCoarsestSlots = kCoarsestBricks / (1024 / kWave);

template <class V, class CL, class CI>
__global__ void __launch_bounds__(1024) k_coarsest(LevelArgs<V, CL, CI> A, int nu) {
  if (A.done && *A.done) return;
  __shared__ V su[kCoarsestBricks * 64];
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI> X = level_view(A);
  const uint32_t w = wave_id();
  const uint32_t nw = blockDim.x / kWave;
  const uint32_t n = A.R.n();
  const int m = int(L.m);
  V rhs[kCoarsestSlots], kown[kCoarsestSlots][3], kpl[kCoarsestSlots][3];
  int32_t nbl[kCoarsestSlots][6];
  uint64_t amask[kCoarsestSlots];
#pragma unroll
  for (int j = 0; j < kCoarsestSlots; ++j) {
    uint32_t i = w + uint32_t(j) * nw;
    if (i >= n) continue;
    bool inner = i >= A.R.n_leaf;
    uint32_t b = A.R.brick(i);
    const BrickMeta M = load_meta(X.meta, b);
    amask[j] = act_mask(M);
    for (int a = 0; a < 3; ++a) {
      kown[j][a] = inner ? own_coef<true>(X, b, 1 + a, L.m) : own_coef<false>(X, b, 1 + a, L.m);
      kpl[j][a] = V(bload_bytes<CL>(X.pf, L.foff[a], b * uint32_t(48 * sizeof(CL))));
    }
    for (int d = 0; d < 6; ++d) {
      int32_t nb = M.nbr[d];
      nbl[j][d] = nb < 0 ? -1
                  : uint32_t(nb) < X.nlb ? nb - int32_t(A.R.leaf_lo)
                                          : int32_t(A.R.n_leaf) + nb - int32_t(A.R.inner_lo);
    }
    rhs[j] = bload<V>(X.b, L.m, b * 64u);
    su[i * 64u + uint32_t(m)] = bload<V>(X.u, L.m, b * 64u);
  }
  __syncthreads();
  int half = nu / 2;
  for (int it = 0; it < nu; ++it) {
    for (int h2 = 0; h2 < 2; ++h2) {
      int colour = it < half ? h2 : 1 - h2;
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i >= n) continue;
        V v[6], k[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          int a = d >> 1;
          int p = L.p[d];
          int32_t nbase = L.out[d] ? (nbl[j][d] >= 0 ? nbl[j][d] * 64 : -1) : int32_t(i) * 64;
          v[d] = nbase >= 0 ? su[nbase + p] : V(0);
          if (d & 1) {
            V ks = shfl(kown[j][a], p);
            k[d] = L.out[d] ? kpl[j][a] : ks;
          } else {
            k[d] = kown[j][a];
          }
        }
        V c = ((k[0] + k[1]) + (k[2] + k[3])) + (k[4] + k[5]);
        V S = V(0);
#pragma unroll
        for (int d = 0; d < 6; ++d) S += k[d] * v[d];
        bool act = (amask[j] >> m) & 1ull;
        if (act && L.colour == colour) su[i * 64u + uint32_t(m)] = div_by(rhs[j] + S, c);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < kCoarsestSlots; ++j) {
    uint32_t i = w + uint32_t(j) * nw;
    if (i < n) bstore<V>(X.u, L.m, A.R.brick(i) * 64u, su[i * 64u + uint32_t(m)]);
  }
}

// The FAS step of level f = lc + 1 in one workgroup (Algorithm 4 on that
// level: FAS right-hand side, pre-smoothing, residual restriction, mu
// coarsest solves, prolongation, post-smoothing) when level f is a complete
// grid of at most kCoarsestBricks bricks without T-junctions and the
// coarsest level has at most kBottomCoarse bricks.  Both iterates stay in
// LDS and each wave keeps the coefficients of its bricks in registers, so
// the dozen launches of a few microseconds each that the separate kernels
// take become one.  Every value read and the order of every sum are those
// of k_fas_rhs, k_smooth, k_restrict, k_coarsest and k_prolong, and the
// arrays in memory end as those kernels leave them.  MULTI: the kernel
// takes `visits` consecutive FAS steps of level f (the level above's mu),
// both iterates staying in LDS from one to the next; otherwise one step per
// launch.  fas = 0 skips the FAS right-hand side of the first step (a
// W-cycle's later visits: it is already in B).  The FP64 cycle takes one
// step per launch: with the loop its registers spill further (120 against
// 88 bytes per lane) and the W-cycle got slower.
constexpr int kBottomCoarse = 1024 / kWave;

// Six local neighbour indices in [-1, 63] packed as bytes (-1: wall).
__device__ __forceinline__ uint64_t pack_nbr(const BrickMeta &M, const Range &R, uint32_t nlb) {
  uint64_t v = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int32_t nb = M.nbr[d];
    int32_t loc = nb < 0 ? -1
                  : uint32_t(nb) < nlb ? nb - int32_t(R.leaf_lo)
                                       : int32_t(R.n_leaf) + nb - int32_t(R.inner_lo);
    v |= uint64_t(uint8_t(int8_t(loc))) << (8 * d);
  }
  return v;
}
__device__ __forceinline__ int32_t unpack_nbr(uint64_t v, int d) {
  return int32_t(int8_t(uint8_t(v >> (8 * d))));
}

// Fixed part of the stencil of one brick (slot index i of its level) in
// k_bottom: the six face coefficients as the stencil sees them (own k_a on
// the minus side, the partner's or the plus-face table's on the plus side),
// their sum in the stencil's order, and the LDS index of each neighbour
// value (partner p in this brick or in the neighbouring one; at a wall the
// index `zero`: an LDS entry that holds 0, or kBottomWall), two 16-bit
// indices per word.
template <class V, class CL>
__device__ __forceinline__ void bottom_faces(const LaneC<V, CL> &L, uint32_t i, uint64_t nbr,
                                             const V (&kown)[3], const V (&kpl)[3],
                                             uint32_t zero, V (&k)[6], V &c,
                                             uint32_t (&lds)[3]) {
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = L.p[d];
    int32_t nl = unpack_nbr(nbr, d);
    int32_t nbase = L.out[d] ? (nl >= 0 ? nl * 64 : -1) : int32_t(i) * 64;
    uint32_t idx = nbase >= 0 ? uint32_t(nbase + p) : zero;
    if (d & 1) {
      V ks = shfl(kown[a], p);
      k[d] = L.out[d] ? kpl[a] : ks;
      lds[a] |= idx << 16;
    } else {
      k[d] = kown[a];
      lds[a] = idx;
    }
  }
  c = ((k[0] + k[1]) + (k[2] + k[3])) + (k[4] + k[5]);
}

// Neighbour sum of k_bottom's stencil over an LDS iterate (bottom_faces).
// FP64: a wall reads the zero entry, so the six reads take no branch (mixed
// W-cycle of the large workload, FP64: 9.98 -> 9.69 ms); FP32: a wall's
// index is kBottomWall and its read is skipped (reading the zero entry made
// the FP32 half-sweeps slower: W-cycle 6.24 -> 6.34 ms).  The sums are the
// same either way.
constexpr uint32_t kBottomWall = 0xffffu;
template <class V>
__device__ __forceinline__ V bottom_sum(const V *su, const V (&k)[6], const uint32_t (&lds)[3]) {
  V S = V(0);
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    uint32_t idx = (lds[d >> 1] >> (16 * (d & 1))) & 0xffffu;
    V v;
    if constexpr (sizeof(V) == 8) v = su[idx];
    else v = idx != kBottomWall ? su[idx] : V(0);
    S += k[d] * v;
  }
  return S;
}

// k_bottom's set-up loads of a brick's own face coefficients (axes 1-3),
// raw: the store that does not hold the brick is addressed out of range and
// reads 0, so the loads of all slots issue without a branch between them.
template <class V, class CL, class CI, int CP>
__device__ __forceinline__ void own_coef_raw(const LevelView<V, CL, CI, CP> &X, uint32_t b,
                                             bool inner, uint32_t m, CI (&ri)[3],
                                             CL (&rl)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uint32_t comp = uint32_t(1 + a);
    uint32_t oi = inner ? ((b - X.nlb) * 256u + comp * 64u) * uint32_t(sizeof(CI)) : kOutOfRange;
    uint32_t ol = inner ? kOutOfRange : (b * 256u + comp * 64u) * uint32_t(sizeof(CL));
    ri[a] = bload_bytes<CI, coef_pol(CP)>(X.ci, m * uint32_t(sizeof(CI)), oi);
    rl[a] = bload_bytes<CL, coef_pol(CP)>(X.cl, m * uint32_t(sizeof(CL)), ol);
  }
}
// The coefficient own_coef gives, from own_coef_raw's values.
template <class V, class CL, class CI, int CP>
__device__ __forceinline__ V own_coef_of(const LevelView<V, CL, CI, CP> &X, bool inner, CI ri,
                                         CL rl) {
  if (inner) {
    V v = V(ri);
    if constexpr (std::is_same<CL, CI>::value) return v;
    else return v * X.iscale;
  }
  return V(rl);
}

template <class V, class CL, class CI, bool MULTI>
__global__ void __launch_bounds__(1024) k_bottom(LevelArgs<V, CL, CI> Af, LevelArgs<V, CL, CI> Ac,
                                                 int nu_pre, int nu_post, int nu_coarse, int mu,
                                                 int fas, int visits, V scale) {
  if (Af.done && *Af.done) return;
  // the iterates of level f and of the coarsest level, each with a zero
  // entry after it that FP64's wall reads take (bottom_sum)
  constexpr uint32_t kZf = kCoarsestBricks * 64, kZc = kBottomCoarse * 64;
  constexpr uint32_t kWf = sizeof(V) == 8 ? kZf : kBottomWall;
  constexpr uint32_t kWc = sizeof(V) == 8 ? kZc : kBottomWall;
  __shared__ V uf[kZf + 1];
  __shared__ V uc[kZc + 1];
  __shared__ V bc[kBottomCoarse * 64];    // restricted residual of its inner cells
  __shared__ V sc[kBottomCoarse * 64];    // u* of its inner cells
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelView<V, CL, CI> Xf = level_view(Af);
  const LevelView<V, CL, CI> Xc = level_view(Ac);
  const uint32_t w = wave_id();
  const uint32_t nw = blockDim.x / kWave;
  const uint32_t nf = Af.R.n(), nc = Ac.R.n();
  const uint32_t m = L.m;
  // FP32: the set-up issues every slot's loads before it uses any (set-up
  // of a V-cycle's launch 12.2 -> 8.5 us; before, each inner coefficient
  // load waited in a branch of its own), and the half-sweeps read every
  // slot's neighbours before any slot writes.  FP64 goes slot by slot: the
  // values held would add to its register spills.
  constexpr bool kBatch = sizeof(V) == 4;
  if (threadIdx.x == 0) {
    uf[kZf] = V(0);
    uc[kZc] = V(0);
  }
  // per slot: right-hand side, the six face coefficients as the stencil
  // sees them and their sum (the diagonal), and the LDS index of each of the
  // six neighbour values (two 16-bit indices per word); all fixed for the
  // whole kernel, so the half-sweeps only read LDS and add
  V rf[kCoarsestSlots], kf[kCoarsestSlots][6], cf[kCoarsestSlots];
  uint32_t lf[kCoarsestSlots][3];
  uint64_t af[kCoarsestSlots];
  uint32_t parf[kCoarsestSlots];  // 64 x (parent's local index) + 8 x octant
  if constexpr (kBatch) {
    CI ri[kCoarsestSlots][3];
    CL rl[kCoarsestSlots][3], rp[kCoarsestSlots][3];
    V ru[kCoarsestSlots];
#pragma unroll
    for (int j = 0; j < kCoarsestSlots; ++j) {
      uint32_t i = w + uint32_t(j) * nw;
      if (i >= nf) continue;
      uint32_t b = Af.R.brick(i);
      own_coef_raw(Xf, b, i >= Af.R.n_leaf, m, ri[j], rl[j]);
#pragma unroll
      for (int a = 0; a < 3; ++a)
        rp[j][a] = bload_bytes<CL>(Xf.pf, L.foff[a], b * uint32_t(48 * sizeof(CL)));
      rf[j] = bload<V>(Xf.b, m, b * 64u);
      ru[j] = bload<V>(Xf.u, m, b * 64u);
    }
#pragma unroll
    for (int j = 0; j < kCoarsestSlots; ++j) {
      uint32_t i = w + uint32_t(j) * nw;
      if (i >= nf) continue;
      bool inner = i >= Af.R.n_leaf;
      const BrickMeta M = load_meta(Xf.meta, Af.R.brick(i));
      af[j] = act_mask(M);
      V kown[3], kpl[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        kown[a] = own_coef_of(Xf, inner, ri[j][a], rl[j][a]);
        kpl[a] = V(rp[j][a]);
      }
      bottom_faces(L, i, pack_nbr(M, Af.R, Xf.nlb), kown, kpl, kWf, kf[j], cf[j], lf[j]);
      parf[j] = (Ac.R.n_leaf + uint32_t(M.parent) - Ac.R.inner_lo) * 64u +
                uint32_t(octant_of(M)) * 8u;
      uf[i * 64u + m] = ru[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kCoarsestSlots; ++j) {
      uint32_t i = w + uint32_t(j) * nw;
      if (i >= nf) continue;
      bool inner = i >= Af.R.n_leaf;
      uint32_t b = Af.R.brick(i);
      const BrickMeta M = load_meta(Xf.meta, b);
      af[j] = act_mask(M);
      V kown[3], kpl[3];
      for (int a = 0; a < 3; ++a) {
        kown[a] = inner ? own_coef<true>(Xf, b, 1 + a, m) : own_coef<false>(Xf, b, 1 + a, m);
        kpl[a] = V(bload_bytes<CL>(Xf.pf, L.foff[a], b * uint32_t(48 * sizeof(CL))));
      }
      bottom_faces(L, i, pack_nbr(M, Af.R, Xf.nlb), kown, kpl, kWf, kf[j], cf[j], lf[j]);
      parf[j] = (Ac.R.n_leaf + uint32_t(M.parent) - Ac.R.inner_lo) * 64u +
                uint32_t(octant_of(M)) * 8u;
      rf[j] = bload<V>(Xf.b, m, b * 64u);
      uf[i * 64u + m] = bload<V>(Xf.u, m, b * 64u);
    }
  }
  // the coarsest level: coefficients (loaded now, used after the
  // restriction); its leaf bricks keep their iterate and right-hand side
  V rc = V(0);
  V kc[6], cc = V(0);
  uint32_t lc[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
  uint64_t ac = 0;
  bool cin = false;
  if (w < nc) {
    cin = w >= Ac.R.n_leaf;
    uint32_t b = Ac.R.brick(w);
    const BrickMeta M = load_meta(Xc.meta, b);
    ac = act_mask(M);
    V kown[3], kpl[3];
    for (int a = 0; a < 3; ++a) {
      kown[a] = cin ? own_coef<true>(Xc, b, 1 + a, m) : own_coef<false>(Xc, b, 1 + a, m);
      kpl[a] = V(bload_bytes<CL>(Xc.pf, L.foff[a], b * uint32_t(48 * sizeof(CL))));
    }
    bottom_faces(L, w, pack_nbr(M, Ac.R, Xc.nlb), kown, kpl, kWc, kc, cc, lc);
    if (!cin) {
      rc = bload<V>(Xc.b, m, b * 64u);
      uc[w * 64u + m] = bload<V>(Xc.u, m, b * 64u);
    }
  }
  __syncthreads();

  // neighbour sum and diagonal of slot j of level f from the LDS iterate
  auto stencil_f = [&](int j, uint32_t i, V &c) {
    (void)i;
    c = cf[j];
    return bottom_sum(uf, kf[j], lf[j]);
  };
  // (FP32: every slot's neighbour sum is read before any slot writes: a
  // cell of the colour reads only cells of the other colour, which no lane
  // writes in this half-sweep; the other lanes' sums are not used.)
  auto half_sweep_f = [&](int colour) {
    if constexpr (kBatch) {
      V S[kCoarsestSlots];
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i < nf) S[j] = bottom_sum(uf, kf[j], lf[j]);
      }
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i >= nf) continue;
        bool act = (af[j] >> m) & 1ull;
        if (act && L.colour == colour) uf[i * 64u + m] = div_by(rf[j] + S[j], cf[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i >= nf) continue;
        V c;
        V S = stencil_f(j, i, c);
        bool act = (af[j] >> m) & 1ull;
        if (act && L.colour == colour) uf[i * 64u + m] = div_by(rf[j] + S, c);
      }
    }
    __syncthreads();
  };

  auto stencil_c = [&](V &c) {
    c = cc;
    return bottom_sum(uc, kc, lc);
  };
  for (int visit = 0; visit < (MULTI ? visits : 1); ++visit) {
    // FAS right-hand side of the inner bricks: b += A u*
    if (visit == 0 && fas) {
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i >= nf || i < Af.R.n_leaf) continue;
        V c;
        V S = stencil_f(j, i, c);
        V u = uf[i * 64u + m];
        bool act = (af[j] >> m) & 1ull;
        rf[j] = act ? rf[j] + (c * u - S) : V(0);
        bstore<V>(Xf.b, m, Af.R.brick(i) * 64u, rf[j]);
      }
      __syncthreads();  // every wave's reads of uf before the first writes
    }
    for (int it = 0; it < nu_pre; ++it) {
      half_sweep_f(0);
      half_sweep_f(1);
    }
    // residual restriction and u* to the coarsest level
#pragma unroll
    for (int j = 0; j < kCoarsestSlots; ++j) {
      uint32_t i = w + uint32_t(j) * nw;
      if (i >= nf) continue;
      V c;
      V S = stencil_f(j, i, c);
      V u = uf[i * 64u + m];
      bool act = (af[j] >> m) & 1ull;
      V r = act ? rf[j] - (c * u - S) : V(0);
      V rs = group8_sum(r);
      V us = group8_sum(act ? u : V(0));
      int cnt = __popcll((af[j] >> (m & 56u)) & 0xffull);
      if ((m & 7u) == 0) {
        uint32_t q = parf[j] + (m >> 3);
        V ust = cnt ? div_by(us, V(cnt)) : V(0);
        bc[q] = rs * scale;
        uc[q] = ust;
        sc[q] = ust;
      }
    }
    __syncthreads();

    // the coarsest level: FAS right-hand side, mu solves
    if (w < nc && cin) {
      V c;
      V S = stencil_c(c);
      V u = uc[w * 64u + m];
      bool act = (ac >> m) & 1ull;
      rc = act ? bc[w * 64u + m] + (c * u - S) : V(0);
    }
    __syncthreads();
    int half = nu_coarse / 2;
    for (int rep = 0; rep < mu; ++rep)
      for (int it = 0; it < nu_coarse; ++it)
        for (int h2 = 0; h2 < 2; ++h2) {
          int colour = it < half ? h2 : 1 - h2;
          if (w < nc) {
            V c;
            V S = stencil_c(c);
            bool act = (ac >> m) & 1ull;
            if (act && L.colour == colour) uc[w * 64u + m] = div_by(rc + S, c);
          }
          __syncthreads();
        }

    // prolongation of the correction (FP32: every slot's reads before the
    // writes), post-smoothing
    if constexpr (kBatch) {
      V un[kCoarsestSlots];
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i >= nf) continue;
        uint32_t q = parf[j] + (m >> 3);
        un[j] = uf[i * 64u + m] + (uc[q] - sc[q]);
      }
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i < nf && ((af[j] >> m) & 1ull)) uf[i * 64u + m] = un[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < kCoarsestSlots; ++j) {
        uint32_t i = w + uint32_t(j) * nw;
        if (i >= nf) continue;
        uint32_t q = parf[j] + (m >> 3);
        V corr = uc[q] - sc[q];
        if ((af[j] >> m) & 1ull) uf[i * 64u + m] = uf[i * 64u + m] + corr;
      }
    }
    __syncthreads();
    for (int it = 0; it < nu_post; ++it) {
      half_sweep_f(1);
      half_sweep_f(0);
    }
  }

  // the arrays as the separate kernels leave them
#pragma unroll
  for (int j = 0; j < kCoarsestSlots; ++j) {
    uint32_t i = w + uint32_t(j) * nw;
    if (i < nf) bstore<V>(Xf.u, m, Af.R.brick(i) * 64u, uf[i * 64u + m]);
  }
  if (w < nc) {
    uint32_t b = Ac.R.brick(w);
    bstore<V>(Xc.u, m, b * 64u, uc[w * 64u + m]);
    if (cin) {
      bstore<V>(Xc.b, m, b * 64u, rc);
      bstore<V>(Xc.us, m, (b - Xc.nlb) * 64u, sc[w * 64u + m]);
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
  V *W2;     // nb * 64: the next transposed half-sweep's W (written by k_T_apply)
  V *SBAR;   // (nb - nlb) * 64
  V *YS;     // (nb - nlb) * 64
  Range R;
  V bscale;  // beta_mg / alpha
  const int *done;  // skip when the solve has stopped (may be null)
  const CL *pf;     // plus-face coefficients (as LevelArgs::pf)
};

// Buffer view of the transposed cycle's arrays on one level.
template <class V, class CL, class CI, int CP = kCpolDefault>
struct LevelViewT {
  LevelView<V, CL, CI, CP> c;  // coefficients and plus faces (u = W)
  __amdgpu_buffer_rsrc_t rho, y, w, w2, sbar, ys;
};

template <int CP = kCpolDefault, class V, class CL, class CI>
__device__ __forceinline__ LevelViewT<V, CL, CI, CP> level_view_T(const LevelArgsT<V, CL, CI> &A) {
  LevelViewT<V, CL, CI, CP> X;
  uint64_t nb = A.T.nb, nlb = A.T.nlb;
  X.rho = make_rsrc(A.RHO, nb * 64 * sizeof(V));
  X.y = make_rsrc(A.Y, nb * 64 * sizeof(V));
  X.w = make_rsrc(A.W, nb * 64 * sizeof(V));
  X.w2 = make_rsrc(A.W2, nb * 64 * sizeof(V));
  X.sbar = make_rsrc(A.SBAR, (nb - nlb) * 64 * sizeof(V));
  X.ys = make_rsrc(A.YS, (nb - nlb) * 64 * sizeof(V));
  X.c.u = X.w;
  X.c.b = X.w;
  X.c.us = X.w;
  X.c.cl = make_rsrc(A.cf.leaf, nlb * 256 * sizeof(CL));
  X.c.ci = make_rsrc(A.cf.inner, (nb - nlb) * 256 * sizeof(CI));
  X.c.pf = make_rsrc(A.pf, nb * 48 * sizeof(CL));
  X.c.meta = A.T.meta;
  X.c.nlb = A.T.nlb;
  X.c.iscale = A.cf.iscale;
  return X;
}

// Transposed level operator at the lane's cell, applied to W (w its own
// entry):
//   (c_m - sum_{T faces of m} k) w_m - sum_{other faces} k W_nbr
//   + (1 / n_active siblings) sum over the sibling group's T-faces (k_i/2) w_i
// (the coupling to the coarser level, B^T, is applied by coupling_brick).  The
// loads across T-faces are out of range, so those faces drop out of the
// neighbour sum by themselves.
template <bool INNER, class V, class CL, class CI, int CP>
__device__ __forceinline__ V level_AuT(const LevelViewT<V, CL, CI, CP> &X, const LaneC<V, CL> &L,
                                       uint32_t b, const BrickMeta &M, V w, V &diag) {
  V k0 = own_coef<INNER>(X.c, b, 1, L.m);
  V k1 = own_coef<INNER>(X.c, b, 2, L.m);
  V k2 = own_coef<INNER>(X.c, b, 3, L.m);
  V v[6], k[6];
  if constexpr (sizeof(V) == 8)
    face_values_gathered<CP>(X.w, X.c.pf, L, b, M, w, k0, k1, k2, v, k);
  else
    face_values<CP>(X.w, X.c.pf, L, b, M, w, k0, k1, k2, v, k);
  V c = ((k[0] + k[1]) + (k[2] + k[3])) + (k[4] + k[5]);
  diag = c;
  uint64_t amask = act_mask(M);
  bool act = (amask >> L.m) & 1ull;
  V acc = c * w;
  if (M.flags & kFlagT) {
    V tpart = V(0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if ((M.flags >> d) & 1u) {
        V kt = L.out[d] ? k[d] : V(0);
        acc -= kt * w;
        tpart += kt * V(0.5) * w;
      }
    }
    V Ssum = group8_sum(tpart);
    int cnt = __popcll((amask >> (L.m & 56u)) & 0xffull);
    if (act && cnt) acc += Ssum / V(cnt);
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) acc -= k[d] * v[d];
  return act ? acc : V(0);
}

// First half of a transposed half-sweep: W = RHO / c on the active cells of
// the colour, 0 elsewhere.
template <bool INNER, class V, class CL, class CI, int CP>
__device__ __forceinline__ void sweep_w_brick(const LevelViewT<V, CL, CI, CP> &X,
                                              const LaneC<V, CL> &L, uint32_t b, int colour) {
  const BrickMeta M = load_meta(X.c.meta, b);
  bool act = (act_mask(M) >> L.m) & 1ull;
  // the diagonal the forward half-sweep divides by: the sum of the six face
  // coefficients the stencil sees (own k on the minus faces, the partner's
  // or the plus-face table's on the plus faces), summed in the same order
  V kd[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    V kown = own_coef<INNER>(X.c, b, 1 + a, L.m);
    V kl = V(bload_bytes<CL, side_pol(CP)>(X.c.pf, L.foff[a], b * uint32_t(48 * sizeof(CL))));
    V ks = shfl(kown, L.p[2 * a + 1]);
    kd[2 * a] = kown;
    kd[2 * a + 1] = L.out[2 * a + 1] ? kl : ks;
  }
  V c = ((kd[0] + kd[1]) + (kd[2] + kd[3])) + (kd[4] + kd[5]);
  V x = V(0);
  if (act && L.colour == colour) x = div_by(bload<V>(X.rho, L.m, b * 64u), c);
  bstore<V>(X.w, L.m, b * 64u, x);
}

template <class V, class CL, class CI, int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_T_sweep_w(LevelArgsT<V, CL, CI> A, int colour) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelViewT<V, CL, CI, CP> X = level_view_T<CP>(A);
  const WaveLoop W = wave_loop(A.R.n());
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    if (i < A.R.n_leaf) sweep_w_brick<false>(X, L, A.R.leaf_lo + i, colour);
    else sweep_w_brick<true>(X, L, A.R.inner_lo + (i - A.R.n_leaf), colour);
  }
}

// RHO -= A^T W on the bricks of the range; with colour >= 0 (a transposed
// half-sweep) also Y += W on that colour's cells (W is zero elsewhere).
// With next >= 0 the first step of the following half-sweep is taken too:
// W2 = RHO / c on the active cells of colour next (own cells only, so no
// other wave needs them during this launch), 0 elsewhere.
template <bool INNER, class V, class CL, class CI, int CP>
__device__ __forceinline__ void apply_T_brick(const LevelViewT<V, CL, CI, CP> &X,
                                              const LaneC<V, CL> &L, uint32_t b, int colour,
                                              int next) {
  const BrickMeta M = load_meta(X.c.meta, b);
  V w = bload<V>(X.w, L.m, b * 64u);
  V c;
  V t = level_AuT<INNER>(X, L, b, M, w, c);
  V rho = bload<V>(X.rho, L.m, b * 64u) - t;
  bstore<V>(X.rho, L.m, b * 64u, rho);
  // FP32: Y passes the caches non-temporal (its next use is two half-sweeps
  // later; mixed adjoint 95.3 -> 94.3 ms); FP64 keeps it cached (148.2
  // against 149.2 ms)
  constexpr int yp = sizeof(V) == 4 ? kCpolStream : kCpolDefault;
  if (L.colour == colour)
    bstore<V, yp>(X.y, L.m, b * 64u, bload<V, yp>(X.y, L.m, b * 64u) + w);
  if (next >= 0) {
    bool act = (act_mask(M) >> L.m) & 1ull;
    bstore<V>(X.w2, L.m, b * 64u, act && L.colour == next ? div_by(rho, c) : V(0));
  }
}

template <class V, class CL, class CI, int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_T_apply(LevelArgsT<V, CL, CI> A, int colour,
                                                    int next) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelViewT<V, CL, CI, CP> X = level_view_T<CP>(A);
  const WaveLoop W = wave_loop(A.R.n());
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    if (i < A.R.n_leaf) apply_T_brick<false>(X, L, A.R.leaf_lo + i, colour, next);
    else apply_T_brick<true>(X, L, A.R.inner_lo + (i - A.R.n_leaf), colour, next);
  }
}

// Coupling of level l to the coarser leaves, transposed: on the leaf bricks
// of level l-1 that have an inner neighbour (a list), RHO_J += sum over the
// fine T-face cells f next to J of (k_f / 2) W_f (the fine cells are
// children of J's inner neighbour); this is one listed brick b (lane m).
template <class V, class CL, class CI>
__device__ __forceinline__ void coupling_brick(const LevelArgsT<V, CL, CI> &A, uint32_t b,
                                               int m) {
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

// A transposed half-sweep's apply step on level l (workgroups [0, g_apply),
// as k_T_apply) and, in the same launch, the coupling of its w to the
// coarser leaves (the workgroups after, one wave per listed brick): the coupling reads
// only w, which the apply step does not write, and writes the residual of
// level l-1 leaf bricks, which the apply step does not touch.
template <class V, class CL, class CI, int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_T_apply_couple(LevelArgsT<V, CL, CI> A, int colour,
                                                           int next, LevelArgsT<V, CL, CI> C,
                                                           const uint32_t *list, uint32_t n,
                                                           uint32_t g_apply) {
  if (A.done && *A.done) return;
  if (blockIdx.x < g_apply) {
    const LaneC<V, CL> L = lane_consts<V, CL>();
    const LevelViewT<V, CL, CI, CP> X = level_view_T<CP>(A);
    const WaveLoop W = wave_loop_of(A.R.n(), blockIdx.x, g_apply);
    for (uint32_t i = W.first; i < W.end; i += W.step) {
      if (i < A.R.n_leaf) apply_T_brick<false>(X, L, A.R.leaf_lo + i, colour, next);
      else apply_T_brick<true>(X, L, A.R.inner_lo + (i - A.R.n_leaf), colour, next);
    }
  } else {
    uint32_t i = (blockIdx.x - g_apply) * kWavesPerBlock + wave_id();
    int m = threadIdx.x & (kWave - 1);
    if (i < n) coupling_brick(C, list[i], m);
  }
}

// Transposed prolongation input: the children's residual sums move to the
// parents, RHO_P += sum_active_children RHO, SBAR_P = -(that sum).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_restrict(LevelArgsT<V, CL, CI> A) {
  if (A.done && *A.done) return;
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
  if (A.done && *A.done) return;
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
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelViewT<V, CL, CI> X = level_view_T(A);
  const WaveLoop W = wave_loop(A.R.n());
  for (uint32_t i = W.first; i < W.end; i += W.step) {
    if (i < A.R.n_leaf) {
      uint32_t b = A.R.leaf_lo + i;
      const BrickMeta M = load_meta(X.c.meta, b);
      V c;
      V t = level_AuT<false>(X, L, b, M, bload<V>(X.w, L.m, b * 64u), c);
      bstore<V>(X.rho, L.m, b * 64u, bload<V>(X.rho, L.m, b * 64u) + t);
    } else {
      uint32_t b = A.R.inner_lo + (i - A.R.n_leaf);
      const BrickMeta M = load_meta(X.c.meta, b);
      V c;
      V t = level_AuT<true>(X, L, b, M, bload<V>(X.w, L.m, b * 64u), c);
      uint32_t j = (b - X.c.nlb) * 64u;
      bstore<V>(X.sbar, L.m, j, bload<V>(X.sbar, L.m, j) + t);
    }
  }
}

// On the bricks of level l: active cells RHO += SBAR_P / n_active(P),
// tbar = (beta_mg / alpha) YS_P, Y += tbar, W = tbar (0 on inactive cells).
template <class V, class CL, class CI>
__global__ void __launch_bounds__(kBlock) k_T_prolong(LevelArgsT<V, CL, CI> A) {
  if (A.done && *A.done) return;
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
// order, each as w = RHO / c on the colour, then RHO -= A^T w, Y += w.
template <class V, class CL, class CI>
__global__ void __launch_bounds__(1024) k_T_coarsest(LevelArgsT<V, CL, CI> A, int nu) {
  if (A.done && *A.done) return;
  const LaneC<V, CL> L = lane_consts<V, CL>();
  const LevelViewT<V, CL, CI> X = level_view_T(A);
  uint32_t w = wave_id();
  uint32_t nw = blockDim.x / kWave;
  int half = nu / 2;
  for (int it = 0; it < nu; ++it) {
    for (int h2 = 0; h2 < 2; ++h2) {
      int colour = it < nu - half ? h2 : 1 - h2;
      for (uint32_t i = w; i < A.R.n(); i += nw) {
        if (i < A.R.n_leaf) sweep_w_brick<false>(X, L, A.R.leaf_lo + i, colour);
        else sweep_w_brick<true>(X, L, A.R.inner_lo + (i - A.R.n_leaf), colour);
      }
      __threadfence_block();
      __syncthreads();
      for (uint32_t i = w; i < A.R.n(); i += nw) {
        if (i < A.R.n_leaf) apply_T_brick<false>(X, L, A.R.leaf_lo + i, colour, -1);
        else apply_T_brick<true>(X, L, A.R.inner_lo + (i - A.R.n_leaf), colour, -1);
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// flag[b] = leaf brick b has an inner (finer-refined) face neighbour
__global__ void k_couple_flag(const BrickMeta *meta, uint32_t nlb, int64_t *flag) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nlb) flag[b] = (meta[b].flags & kFlagInner) ? 1 : 0;
}

// list[pos[b]] = b for the flagged bricks (pos: exclusive scan of the flags)
__global__ void k_couple_list(const BrickMeta *meta, uint32_t nlb, const int64_t *pos,
                              uint32_t *list) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nlb && (meta[b].flags & kFlagInner)) list[pos[b]] = b;
}

// dst = V(src * scale): the transposed cycle's input (scale: the power of
// two of the solve's scalars, or null for 1)
template <class V>
__global__ void k_T_load(const double *src, V *dst, int64_t n, const double *scale) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = V(scale ? src[i] * *scale : src[i]);
}

template <class V>
__global__ void k_fill(V *x, int64_t n, V v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace mfmg
