// Octree construction on the device: the same octree as the host builder
// (Section 3: leaf and inner cells, face-neighbouring leaves at most one
// level apart; Section 4.1: a node meeting the surface is split), built
// with dense per-level tables so that no step needs a sort or a hash.
//
// The nodes of level l are the 4^3-cell bricks of that level, indexed by
// their Morton key over the level's brick grid (8^(l-2) keys; brick
// coordinates of at most 10 bits per axis, x in the least significant
// bit).  Two tables per level describe the whole tree:
//   split[l][k]  node k exists and has children (levels below the uniform
//                grid level are complete and split);
//   id[l][k]     device brick id of node k, or -1.
// Node k of level l exists iff l <= min_level or split[l-1][k >> 3].
//
// Device brick order (as the solver expects it): leaf bricks level-major,
// finest level first, Morton order within a level; then inner bricks
// level-major from max_level-1 down to level 2, Morton order within a
// level.  The canonical order of the leaf bricks (faces, leaves and ABI
// vectors) is the Morton order of their first cell at the finest level.
#pragma once

#include "kernels.hpp"
#include "topology.hpp"

namespace mfmg {

constexpr int kOctLevels = kMaxLevel + 1;
constexpr int kOctTile = 4096;    // keys per workgroup of the counting passes
constexpr int kOctThreads = 256;  // 16 consecutive keys per thread

struct OctTables {
  uint8_t *split;
  int32_t *id;
  uint64_t split_off[kOctLevels];
  uint64_t id_off[kOctLevels];
  int min_level, max_level;
};

__host__ __device__ inline uint64_t oct_keys(int l) { return uint64_t(1) << (3 * (l - 2)); }

__device__ __forceinline__ uint32_t oct_spread(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}
__device__ __forceinline__ uint32_t oct_compact(uint32_t x) {
  x &= 0x09249249u;
  x = (x | (x >> 2)) & 0x030c30c3u;
  x = (x | (x >> 4)) & 0x0300f00fu;
  x = (x | (x >> 8)) & 0x030000ffu;
  x = (x | (x >> 16)) & 0x3ffu;
  return x;
}
__device__ __forceinline__ uint32_t oct_key(uint32_t a, uint32_t b, uint32_t c) {
  return oct_spread(a) | (oct_spread(b) << 1) | (oct_spread(c) << 2);
}
__device__ __forceinline__ void oct_coords(uint32_t k, int32_t &a, int32_t &b, int32_t &c) {
  a = int32_t(oct_compact(k));
  b = int32_t(oct_compact(k >> 1));
  c = int32_t(oct_compact(k >> 2));
}

__device__ __forceinline__ bool oct_exists(const OctTables &T, int l, uint64_t k) {
  return l <= T.min_level || T.split[T.split_off[l - 1] + (k >> 3)] != 0;
}
__device__ __forceinline__ bool oct_split(const OctTables &T, int l, uint64_t k) {
  return l < T.max_level && T.split[T.split_off[l] + k] != 0;
}

// Refinement predicates of the grid generator on the closed node box,
// evaluated operation by operation without contraction, so that every
// decision is the IEEE one the host builder takes.
__device__ inline bool oct_sphere_meets(const Prim &p, const double lo[3], const double hi[3]) {
#pragma clang fp contract(off)
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double t = lo[ax] - p.center[ax];
    if (0.0 > t) t = 0.0;
    double t2 = p.center[ax] - hi[ax];
    if (t2 > t) t = t2;
    dmin2 = dmin2 + t * t;
    double u1 = fabs(lo[ax] - p.center[ax]);
    double u2 = fabs(hi[ax] - p.center[ax]);
    double u = u1 > u2 ? u1 : u2;
    dmax2 = dmax2 + u * u;
  }
  double ro = p.radius + p.band;
  double ri = p.radius - p.band;
  if (dmin2 > ro * ro) return false;
  if (ri > 0.0 && dmax2 < ri * ri) return false;
  return true;
}
__device__ inline bool oct_box_meets(const Prim &p, const double lo[3], const double hi[3]) {
  bool inter = true, inside = true;
  for (int ax = 0; ax < 3; ++ax) {
    inter = inter && lo[ax] <= p.hi[ax] && p.lo[ax] <= hi[ax];
    inside = inside && p.lo[ax] < lo[ax] && hi[ax] < p.hi[ax];
  }
  return inter && !inside;
}

// Predicate refinement of level l (levels in increasing order): an
// existing node is split when its box meets a primitive; levels below the
// uniform grid level are split everywhere.
__global__ void k_oct_refine(OctTables T, int l, const Prim *prims, int n_prims) {
  uint64_t nk = oct_keys(l);
  double s = double(kBrick) * ldexp(1.0, -l);
  for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < nk;
       k += uint64_t(gridDim.x) * blockDim.x) {
    uint8_t v = 0;
    if (l < T.min_level) {
      v = 1;
    } else if (oct_exists(T, l, k)) {
      int32_t a, b, c;
      oct_coords(uint32_t(k), a, b, c);
      double lo[3] = {a * s, b * s, c * s};
      double hi[3] = {(a + 1) * s, (b + 1) * s, (c + 1) * s};
      for (int i = 0; i < n_prims; ++i) {
        const Prim &p = prims[i];
        if (p.kind == 0 ? oct_sphere_meets(p, lo, hi) : oct_box_meets(p, lo, hi)) {
          v = 1;
          break;
        }
      }
    }
    T.split[T.split_off[l] + k] = v;
  }
}

// 2:1 balance of level l (levels in decreasing order, l >= min_level + 2):
// every existing node needs, across each face, the node of level l-1 that
// contains its neighbour; a missing one is created with its siblings by
// splitting its parent.  (That parent's own existence is the constraint of
// the new node towards its siblings, taken in the pass of level l-1.)
// Concurrent writers store the same byte.
__global__ void k_oct_balance(OctTables T, int l) {
  uint64_t nk = oct_keys(l);
  int32_t per = int32_t(1) << (l - 2);
  for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < nk;
       k += uint64_t(gridDim.x) * blockDim.x) {
    if (!oct_exists(T, l, k)) continue;
    int32_t a, b, c;
    oct_coords(uint32_t(k), a, b, c);
    for (int d = 0; d < 6; ++d) {
      int32_t s = (d & 1) ? 1 : -1;
      int32_t na = a + (d >> 1 == 0 ? s : 0);
      int32_t nb = b + (d >> 1 == 1 ? s : 0);
      int32_t nc = c + (d >> 1 == 2 ? s : 0);
      if (na < 0 || nb < 0 || nc < 0 || na >= per || nb >= per || nc >= per) continue;
      uint32_t r = oct_key(uint32_t(na) >> 1, uint32_t(nb) >> 1, uint32_t(nc) >> 1);
      uint8_t *q = T.split + T.split_off[l - 2] + (r >> 3);
      if (*q == 0) *q = 1;
    }
  }
}

// leaf (bit 0) / inner (bit 1) class of key k at level l
__device__ __forceinline__ uint32_t oct_class(const OctTables &T, int l, uint64_t k) {
  if (!oct_exists(T, l, k)) return 0;
  return oct_split(T, l, k) ? 2u : 1u;
}

// Per workgroup of kOctTile keys: number of leaf and inner nodes.
__global__ void __launch_bounds__(kOctThreads) k_oct_count(OctTables T, int l, uint32_t *cnt) {
  uint64_t nk = oct_keys(l);
  uint64_t k0 = uint64_t(blockIdx.x) * kOctTile + uint64_t(threadIdx.x) * 16;
  uint32_t nl = 0, ni = 0;
  for (int j = 0; j < 16; ++j) {
    uint64_t k = k0 + j;
    if (k >= nk) break;
    uint32_t c = oct_class(T, l, k);
    nl += c == 1;
    ni += c == 2;
  }
  __shared__ uint32_t s[2][kOctThreads];
  s[0][threadIdx.x] = nl;
  s[1][threadIdx.x] = ni;
  __syncthreads();
  for (int w = kOctThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cnt[2 * blockIdx.x] = s[0][0];
    cnt[2 * blockIdx.x + 1] = s[1][0];
  }
}

// Exclusive scan of n pairs in place (one workgroup of 1024 threads,
// chunk by chunk); the totals go to tot[0..1].
__global__ void __launch_bounds__(1024) k_oct_scan_pairs(uint32_t *cnt, uint64_t n,
                                                         uint32_t *tot) {
  __shared__ uint32_t s[2][1024];
  uint32_t carry0 = 0, carry1 = 0;
  for (uint64_t base = 0; base < n; base += 1024) {
    uint64_t i = base + threadIdx.x;
    uint32_t v0 = i < n ? cnt[2 * i] : 0u, v1 = i < n ? cnt[2 * i + 1] : 0u;
    s[0][threadIdx.x] = v0;
    s[1][threadIdx.x] = v1;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
      uint32_t a0 = threadIdx.x >= unsigned(w) ? s[0][threadIdx.x - w] : 0u;
      uint32_t a1 = threadIdx.x >= unsigned(w) ? s[1][threadIdx.x - w] : 0u;
      __syncthreads();
      s[0][threadIdx.x] += a0;
      s[1][threadIdx.x] += a1;
      __syncthreads();
    }
    if (i < n) {
      cnt[2 * i] = carry0 + s[0][threadIdx.x] - v0;
      cnt[2 * i + 1] = carry1 + s[1][threadIdx.x] - v1;
    }
    carry0 += s[0][1023];
    carry1 += s[1][1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tot[0] = carry0;
    tot[1] = carry1;
  }
}

// Brick ids of level l: leaf node of rank r -> leaf_lo + r, inner node of
// rank r -> inner_lo + r (ranks in Morton order); records each brick's key
// and level.  cnt holds the scanned per-workgroup counts of k_oct_count.
__global__ void __launch_bounds__(kOctThreads) k_oct_assign(OctTables T, int l,
                                                            const uint32_t *cnt,
                                                            uint32_t leaf_lo, uint32_t inner_lo,
                                                            uint32_t *bkey, int8_t *blev) {
  uint64_t nk = oct_keys(l);
  uint64_t k0 = uint64_t(blockIdx.x) * kOctTile + uint64_t(threadIdx.x) * 16;
  uint32_t cls[16];
  uint32_t nl = 0, ni = 0;
  for (int j = 0; j < 16; ++j) {
    uint64_t k = k0 + j;
    cls[j] = k < nk ? oct_class(T, l, k) : 0u;
    nl += cls[j] == 1;
    ni += cls[j] == 2;
  }
  __shared__ uint32_t s[2][kOctThreads];
  s[0][threadIdx.x] = nl;
  s[1][threadIdx.x] = ni;
  __syncthreads();
  for (int w = 1; w < kOctThreads; w <<= 1) {
    uint32_t a0 = threadIdx.x >= unsigned(w) ? s[0][threadIdx.x - w] : 0u;
    uint32_t a1 = threadIdx.x >= unsigned(w) ? s[1][threadIdx.x - w] : 0u;
    __syncthreads();
    s[0][threadIdx.x] += a0;
    s[1][threadIdx.x] += a1;
    __syncthreads();
  }
  uint32_t rl = cnt[2 * blockIdx.x] + s[0][threadIdx.x] - nl;
  uint32_t ri = cnt[2 * blockIdx.x + 1] + s[1][threadIdx.x] - ni;
  for (int j = 0; j < 16; ++j) {
    uint64_t k = k0 + j;
    if (k >= nk) break;
    int32_t id = -1;
    if (cls[j] == 1) id = int32_t(leaf_lo + rl++);
    else if (cls[j] == 2) id = int32_t(inner_lo + ri++);
    T.id[T.id_off[l] + k] = id;
    if (id >= 0) {
      bkey[id] = uint32_t(k);
      blev[id] = int8_t(l);
    }
  }
}

struct OctLevels {
  uint32_t leaf_lo[kOctLevels];
  uint32_t n_leaf[kOctLevels];
};

// number of entries of the sorted keys[0, n) below x
__device__ inline uint32_t oct_lower_bound(const uint32_t *keys, uint32_t n, uint64_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (uint64_t(keys[mid]) < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Canonical position of each leaf brick: the number of leaf bricks whose
// first finest-level cell precedes its own in Morton order, counted level
// by level with one binary search in each level's sorted keys (leaves do
// not overlap, so a coarser leaf precedes iff it precedes the ancestor, a
// finer one iff it precedes the first descendant).
// inv must be -1 on entry; k_oct_check_perm then flags a position no leaf
// took (so canon is a permutation before anything indexes with it).
__global__ void k_oct_canon(OctTables T, OctLevels LV, uint32_t nlb, const uint32_t *bkey,
                            const int8_t *blev, int32_t *canon, int32_t *inv, int *err) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlb) return;
  int l = blev[i];
  uint64_t k = bkey[i];
  uint32_t r = 0;
  for (int q = T.min_level; q <= T.max_level; ++q) {
    if (LV.n_leaf[q] == 0) continue;
    if (q == l) {
      r += i - LV.leaf_lo[q];
      continue;
    }
    uint64_t x = q < l ? (k >> (3 * (l - q))) : (k << (3 * (q - l)));
    r += oct_lower_bound(bkey + LV.leaf_lo[q], LV.n_leaf[q], x);
  }
  if (r >= nlb) {
    *err = 1;
    r = 0;
  }
  canon[i] = int32_t(r);
  inv[r] = int32_t(i);
}

__global__ void k_oct_check_perm(const int32_t *inv, uint32_t nlb, int *err) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nlb && inv[j] < 0) *err = 1;
}

// Brick records and child table (tplus and act are filled later).  Sets
// *err when the tree breaks an invariant the solver relies on.
__global__ void k_oct_meta(OctTables T, uint32_t nlb, uint32_t nb, const uint32_t *bkey,
                           const int8_t *blev, BrickMeta *meta, int32_t *child, int *err) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int l = blev[i];
  uint32_t k = bkey[i];
  int32_t a, b, c;
  oct_coords(k, a, b, c);
  int32_t per = int32_t(1) << (l - 2);
  BrickMeta M;
  M.flags = 0;
  for (int d = 0; d < 6; ++d) {
    int32_t s = (d & 1) ? 1 : -1;
    int32_t na = a + (d >> 1 == 0 ? s : 0);
    int32_t nbb = b + (d >> 1 == 1 ? s : 0);
    int32_t nc = c + (d >> 1 == 2 ? s : 0);
    int32_t v;
    if (na < 0 || nbb < 0 || nc < 0 || na >= per || nbb >= per || nc >= per) {
      v = kWall;
      M.flags |= 1u << (16 + d);
    } else {
      uint32_t kn = oct_key(uint32_t(na), uint32_t(nbb), uint32_t(nc));
      int32_t j = T.id[T.id_off[l] + kn];
      if (j >= 0) {
        v = j;
        if (uint32_t(j) >= nlb) M.flags |= 1u << (8 + d);
      } else {
        int32_t J = l > kMinLevel ? T.id[T.id_off[l - 1] + (kn >> 3)] : -1;
        if (J < 0 || uint32_t(J) >= nlb || i >= nlb) {
          *err = 1;
          J = 0;  // keeps every later index in range; the build fails
        }
        v = kCoarseBase - J;
        M.flags |= 1u << d;
      }
    }
    M.nbr[d] = v;
  }
  int32_t par = -1;
  if (l > kMinLevel) {
    par = T.id[T.id_off[l - 1] + (k >> 3)];
    if (par < 0 || uint32_t(par) < nlb) *err = 1;
  }
  M.parent = par;
  M.tplus = -1;
  M.coord[0] = a;
  M.coord[1] = b;
  M.coord[2] = c;
  M.act[0] = 0;
  M.act[1] = 0;
  M.level = l;
  M.pad = 0;
  meta[i] = M;
  for (int o = 0; o < 8; ++o) {
    int32_t ch = -1;
    if (i >= nlb) {
      ch = l < T.max_level ? T.id[T.id_off[l + 1] + 8ull * k + o] : -1;
      if (ch < 0) *err = 1;
    }
    child[8ull * i + o] = ch;
  }
}

// flag[j] = leaf brick at canonical position j has a T-face on a plus side
__global__ void k_oct_tflag(const BrickMeta *meta, const int32_t *inv, uint32_t nlb,
                            int64_t *flag) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlb) return;
  flag[j] = (meta[inv[j]].flags & 0x2au) ? 1 : 0;
}

__global__ void k_oct_tplus(BrickMeta *meta, const int32_t *inv, uint32_t nlb,
                            const int64_t *pos) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlb) return;
  BrickMeta *M = meta + inv[j];
  M->tplus = (M->flags & 0x2au) ? int32_t(pos[j]) : -1;
}

// Directions whose face a leaf cell owns: a wall, a coarser neighbour, or a
// same-level leaf neighbour on the minus side (finer neighbours own the
// split faces).
__device__ __forceinline__ uint32_t oct_owned(const BrickMeta &M, uint32_t nlb, int m) {
  int p[3] = {dev_cx(m), dev_cy(m), dev_cz(m)};
  uint32_t mask = 0;
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    bool inside = (d & 1) ? p[a] < kBrick - 1 : p[a] > 0;
    bool own;
    if (inside) {
      own = (d & 1) == 0;
    } else {
      int32_t n = M.nbr[d];
      if (n == kWall || n <= kCoarseBase) own = true;
      else own = uint32_t(n) < nlb && (d & 1) == 0;
    }
    if (own) mask |= 1u << d;
  }
  return mask;
}

// One wave per device leaf brick: owned-face masks and the brick's face
// count at its canonical position.
__global__ void __launch_bounds__(kBlock) k_oct_fmask(const BrickMeta *meta, const int32_t *canon,
                                                      uint32_t nlb, uint8_t *fmask,
                                                      int64_t *bcount) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= nlb) return;
  uint32_t mask = oct_owned(meta[b], nlb, m);
  fmask[uint64_t(b) * 64 + m] = uint8_t(mask);
  uint32_t n = wave_sum(uint32_t(__popc(mask)));
  if (m == 0) bcount[canon[b]] = int64_t(n);
}

// first face id of each cell: the brick's base plus the faces of the lanes
// before it
__global__ void __launch_bounds__(kBlock) k_oct_fbase(const uint8_t *fmask, const int32_t *canon,
                                                      uint32_t nlb, const int64_t *bbase,
                                                      int64_t *fbase) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= nlb) return;
  uint32_t n = __popc(fmask[uint64_t(b) * 64 + m]);
  uint32_t incl = n;
  for (int w = 1; w < kWave; w <<= 1) {
    uint32_t t = __shfl_up(incl, w, kWave);
    if (m >= w) incl += t;
  }
  fbase[uint64_t(b) * 64 + m] = bbase[canon[b]] + int64_t(incl - n);
}

// ---------------------------------------------------------------------------
// exclusive scan of int64 (three passes; one workgroup adds the tile sums)
// ---------------------------------------------------------------------------
constexpr int kScanTile = 1024;

__global__ void __launch_bounds__(256) k_scan_tiles(int64_t *x, int64_t n, int64_t *tiles) {
  __shared__ int64_t s[256];
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * 4;
  int64_t v[4], t = 0;
  for (int j = 0; j < 4; ++j) {
    v[j] = base + j < n ? x[base + j] : 0;
    t += v[j];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int w = 1; w < 256; w <<= 1) {
    int64_t a = threadIdx.x >= unsigned(w) ? s[threadIdx.x - w] : 0;
    __syncthreads();
    s[threadIdx.x] += a;
    __syncthreads();
  }
  int64_t run = s[threadIdx.x] - t;
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) x[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 255) tiles[blockIdx.x] = s[255];
}

__global__ void __launch_bounds__(1024) k_scan_top(int64_t *tiles, int64_t n, int64_t *total) {
  __shared__ int64_t s[1024];
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < n ? tiles[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
      int64_t a = threadIdx.x >= unsigned(w) ? s[threadIdx.x - w] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < n) tiles[i] = carry + s[threadIdx.x] - v;
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_scan_add(int64_t *x, int64_t n, const int64_t *tiles) {
  int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t off = tiles[blockIdx.x];
  for (int j = threadIdx.x; j < kScanTile; j += 256)
    if (base + j < n) x[base + j] += off;
}

// ---------------------------------------------------------------------------
// canonical-order outputs of a device topology
// ---------------------------------------------------------------------------
// leaves: level and (i, j, k) of every leaf cell at its canonical index
__global__ void __launch_bounds__(kBlock) k_oct_leaves(const BrickMeta *meta, const int32_t *canon,
                                                       uint32_t nlb, uint8_t *level,
                                                       int32_t *ijk) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= nlb) return;
  const BrickMeta M = meta[b];
  int64_t c = int64_t(canon[b]) * 64 + m;
  level[c] = uint8_t(M.level);
  ijk[3 * c] = M.coord[0] * kBrick + dev_cx(m);
  ijk[3 * c + 1] = M.coord[1] * kBrick + dev_cy(m);
  ijk[3 * c + 2] = M.coord[2] * kBrick + dev_cz(m);
}

// faces in canonical order: owner cell, direction, the leaf cell on the
// other side (-1 at a wall) and the kind (0 wall, 1 same level, 2 coarser)
__global__ void __launch_bounds__(kBlock) k_oct_faces(const BrickMeta *meta, const int32_t *canon,
                                                      const int64_t *fbase, const uint8_t *fmask,
                                                      uint32_t nlb, int64_t *owner, int8_t *dir,
                                                      int64_t *other, int8_t *kind) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= nlb) return;
  const BrickMeta M = meta[b];
  int64_t c = int64_t(canon[b]) * 64 + m;
  int64_t f = fbase[uint64_t(b) * 64 + m];
  uint32_t mask = fmask[uint64_t(b) * 64 + m];
  int p[3] = {dev_cx(m), dev_cy(m), dev_cz(m)};
  for (int d = 0; d < 6; ++d) {
    if (!((mask >> d) & 1u)) continue;
    int a = d >> 1;
    int q[3] = {p[0], p[1], p[2]};
    q[a] += (d & 1) ? 1 : -1;
    int64_t o;
    int k;
    if (q[a] >= 0 && q[a] < kBrick) {
      o = int64_t(canon[b]) * 64 + dev_morton(q[0], q[1], q[2]);
      k = 1;
    } else {
      int32_t n = M.nbr[d];
      if (n == kWall) {
        o = -1;
        k = 0;
      } else if (n >= 0) {
        o = int64_t(canon[n]) * 64 + dev_morton(q[0] & 3, q[1] & 3, q[2] & 3);
        k = 1;
      } else {
        int32_t J = kCoarseBase - n;
        const BrickMeta &MJ = meta[J];
        int cc[3];
        for (int e = 0; e < 3; ++e) {
          int64_t g = int64_t(M.coord[e]) * kBrick + q[e];
          cc[e] = int((g >> 1) - int64_t(MJ.coord[e]) * kBrick);
        }
        o = int64_t(canon[J]) * 64 + dev_morton(cc[0], cc[1], cc[2]);
        k = 2;
      }
    }
    owner[f] = c;
    dir[f] = int8_t(d);
    other[f] = o;
    kind[f] = int8_t(k);
    ++f;
  }
}

// level of each leaf brick at its canonical position
__global__ void k_oct_canon_level(const BrickMeta *meta, const int32_t *canon, uint32_t nlb,
                                  int8_t *out) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nlb) out[canon[b]] = int8_t(meta[b].level);
}

}  // namespace mfmg
