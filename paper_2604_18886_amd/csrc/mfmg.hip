// C ABI and host driver of the matrix-free octree multigrid PCG solver.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mfmg.h"
#include "kernels.hpp"
#include "octree_kernels.hpp"
#include "pcg_kernels.hpp"
#include "projection_kernels.hpp"
#include "topology.hpp"

using namespace mfmg;

// --------------------------------------------------------------------------
// errors and device buffers
// --------------------------------------------------------------------------
namespace {
thread_local std::string g_err;

mfmg_status fail(mfmg_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

struct HipError {
  hipError_t e;
  const char *what;
};

#define HIP_CHECK(x)                                   \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) throw HipError{e_, #x};      \
  } while (0)

mfmg_status hip_fail(const HipError &e) {
  return fail(e.e == hipErrorOutOfMemory ? MFMG_ERR_OOM : MFMG_ERR_HIP,
              std::string(e.what) + ": " + hipGetErrorString(e.e));
}

template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t count) {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = count;
    if (count == 0) return;
    HIP_CHECK(hipMalloc(&p, count * sizeof(T)));
  }
  void upload(const std::vector<T> &v, hipStream_t s) {
    alloc(v.size());
    if (!v.empty())
      HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

inline unsigned grid_for(int64_t bricks) {
  int64_t g = (bricks + kWavesPerBlock - 1) / kWavesPerBlock;
  return unsigned(g > 0 ? g : 1);
}
// Grid of the level kernels (wave_loop): a multiple of 8 workgroups, at
// most waves_per_xcd waves per XCD, each looping over its share of bricks.
// Measured on the large workload: the FP32 stencils and the reductions over
// the leaves are fastest with 3072 waves per XCD looping (mixed solve 42.35
// -> 41.62 ms against 2048; 4096 and 6144 gave 41.85 ms); the FP64
// stencils (more registers, five waves resident per SIMD) with 1920, three
// rounds of them (FP64 half-sweep 207 -> 192 us against one brick per
// wave).  One workgroup of k_finish adds the reductions' partials, however
// many.  Levels of fewer than 65536 bricks (the small workloads' leaf
// levels, every coarse level) take 2048 waves per XCD in FP32, so that each
// wave gets four or more bricks rather than two or three (leaf half-sweep of
// the 2.3 M-leaf cut-sphere workload 11.7 -> 10.8 us, its mixed solve 6.92
// -> 6.72 ms; the large workload's mixed solve 41.52 -> 41.48 ms).
// MFMG_WAVES_PER_XCD (read once) overrides the cap, for tuning.
constexpr int64_t kWavesPerXcd32 = 3072;
constexpr int64_t kWavesPerXcdSmall32 = 2048;
constexpr int64_t kSmallLevelBricks = 65536;
constexpr int64_t kWavesPerXcd64 = 1920;
inline int64_t waves_override() {
  static const int64_t v = [] {
    const char *e = std::getenv("MFMG_WAVES_PER_XCD");
    long long x = e ? std::atoll(e) : 0;
    return x > 0 ? int64_t(x) : int64_t(0);
  }();
  return v;
}
inline unsigned grid_waves(int64_t bricks, int64_t cap) {
  int64_t chunk = (bricks + 7) / 8;
  int64_t waves = std::min<int64_t>(std::max<int64_t>(chunk, 1), cap);
  return unsigned(8 * ((waves + kWavesPerBlock - 1) / kWavesPerBlock));
}
inline int64_t cap32(int64_t bricks) {
  return bricks < kSmallLevelBricks ? kWavesPerXcdSmall32 : kWavesPerXcd32;
}
// reductions and FP32 stencils
inline unsigned level_grid(int64_t bricks) {
  return grid_waves(bricks, waves_override() ? waves_override() : cap32(bricks));
}
// stencils on values of type V
template <class V>
inline unsigned stencil_grid(int64_t bricks) {
  if (waves_override()) return grid_waves(bricks, waves_override());
  return grid_waves(bricks, sizeof(V) == 8 ? kWavesPerXcd64 : cap32(bricks));
}
// The transposed cycle's stencils (adjoint solves) keep one brick per wave
// in FP64: they do not use the gathered face loads, and looping made them
// slower.  In FP32 they loop with 2048 waves per XCD (3072 made the mixed
// adjoint solve slower, 93.8 -> 94.6 ms).
constexpr int64_t kWavesPerXcdT32 = 2048;
template <class V>
inline unsigned stencil_grid_T(int64_t bricks) {
  if (waves_override()) return grid_waves(bricks, waves_override());
  return grid_waves(bricks, sizeof(V) == 8 ? int64_t(1) << 30 : kWavesPerXcdT32);
}
// A stencil launch whose single-use streams (coefficients, plus faces,
// right-hand side) and iterate together exceed the 256 MB Infinity Cache
// gains nothing from caching those streams for the next launch, and they
// only push the iterate's lines out of L2: such launches load them
// non-temporal (kCpolStream; the FP32 cycle streams only the coefficients,
// Cycle::kCpolLevel).  Measured on the large workload: the finest
// mixed half-sweep (about 415 MB) runs 11% faster that way, the next
// level (about 140 MB, re-read from the Infinity Cache by the following
// half-sweep) 20% slower.  MFMG_STREAM_BYTES (read once) overrides the
// threshold, for tuning.
inline double stream_threshold() {
  static const double v = [] {
    const char *e = std::getenv("MFMG_STREAM_BYTES");
    double x = e ? std::atof(e) : -1.0;
    return x >= 0 ? x : 256.0 * 1024 * 1024;
  }();
  return v;
}
inline unsigned grid_elems(int64_t n, int t) { return unsigned(std::max<int64_t>(1, (n + t - 1) / t)); }

// grid of the Krylov kernels (grid-stride over leaf bricks, one partial sum
// per workgroup)
constexpr int64_t kMaxReduceBlocks = 2048;
inline unsigned grid_reduce(int64_t bricks) {
  int64_t g = (bricks + kWavesPerBlock - 1) / kWavesPerBlock;
  return unsigned(std::max<int64_t>(1, std::min(g, kMaxReduceBlocks)));
}
}  // namespace

// --------------------------------------------------------------------------
// objects
// --------------------------------------------------------------------------
// Device view of the topology.  Device brick ids are level-major (leaf bricks
// by descending level then Morton order; inner bricks likewise).
struct DeviceTopology {
  DevBuf<BrickMeta> meta;             // act = 0
  DevBuf<int32_t> child;              // 8 per device brick
  DevBuf<int64_t> fbase;              // per device leaf cell
  DevBuf<uint8_t> fmask;              // per device leaf cell
  DevBuf<int32_t> canon;              // device leaf brick -> canonical leaf brick
  std::vector<Range> range;           // per level
  uint32_t nlb = 0, nb = 0;
};

// An octree built on the host keeps its host topology (and makes its device
// tables at first use); one built on the device has only the device tables.
struct mfmg_octree {
  Topology topo;  // host-built octrees only
  bool on_host = true;
  int min_level = 0, max_level = 0;
  int64_t nlb = 0, nb = 0, n_faces = 0, n_tplus = 0;
  mutable std::shared_ptr<DeviceTopology> dt;
};

struct mfmg_coeffs {
  const mfmg_octree *tree = nullptr;
  std::shared_ptr<DeviceTopology> dt;
  DevBuf<double> coef;  // nlb * 256, FP64 leaf coefficients (device order)
  DevBuf<double> tc;    // n_tplus * 48
  mfmg_bc bc{};
  int has_dirichlet = 0;
};

struct mfmg_hierarchy {
  const mfmg_coeffs *co = nullptr;
  mfmg_mg_params prm{};
  int L = 0, lc = 0;
  DevBuf<BrickMeta> meta;  // topology records with this hierarchy's activity masks
  DevBuf<ParentNbrs> pnb;  // parent-neighbour table (fused prolongation)
  DevBuf<double> coef64;   // nb * 256 (leaf part = assembled, inner = Algorithm 3)
  DevBuf<float> coef32;    // nlb * 256 (mixed)
  DevBuf<__half> coef16;   // (nb - nlb) * 256 (mixed)
  DevBuf<float> tc32;      // mixed
  DevBuf<double> pf64;     // plus-face coefficients, nb * 48 (FP64 cycle, composite operator)
  DevBuf<float> pf32;      // plus-face coefficients, nb * 48 (mixed cycle)
  double n_active = 0;     // active leaf cells
  std::vector<char> stream_lv;  // per level: the cycle's stencils stream their coefficients
  bool stream_composite = false;  // the same for the composite operator
  bool fuse_bottom = false;       // level lc + 1 and the coarsest level in one kernel (k_bottom)
  bool fuse_prolong = true;       // prolongation folded into the post-smoothing (k_smooth PR)
  std::vector<char> fold_fas;     // per level: FAS right-hand side folded into k_smooth_fas
  // work vectors (device order)
  DevBuf<double> U64, B64, S64;  // FP64 cycle: nb*64, nb*64, (nb-nlb)*64
  DevBuf<float> U32, B32, S32;   // mixed cycle
  DevBuf<double> r;              // PCG residual (mixed; aliases B64 in FP64 mode)
  DevBuf<double> x;              // PCG iterate (leaf size)
  DevBuf<double> pd;             // search direction (full size: parent means of T bricks)
  DevBuf<double> Ap;             // leaf size
  DevBuf<double> Xf;             // full-size scratch for operator applications
  DevBuf<double> partials;
  DevBuf<Scalars> S;
  DevBuf<double> hist;
  // transposed cycle (allocated on first use): residual, solution, scratch
  DevBuf<double> T64[6];  // RHO, Y, W (nb*64), SBAR, YS ((nb-nlb)*64), W2 (nb*64)
  // leaf bricks with an inner neighbour (level-major), per level [lo, lo + n)
  DevBuf<uint32_t> couple;
  std::vector<uint32_t> couple_lo, couple_n;
  DevBuf<float> T32[6];
  DevBuf<double> rA;              // adjoint PCG residual
  // face arrays for the per-face gradient (allocated on first use)
  DevBuf<int64_t> f_owner, f_other;
  DevBuf<int8_t> f_dir, f_kind, leaf_level;
  DevBuf<uint64_t> canon_act;
  Scalars *hostS = nullptr;      // pinned: the scalars read back after a solve
  int *host_done = nullptr;      // pinned, mapped: stop flag written by k_finish
  int *host_done_dev = nullptr;  // its device address
  hipEvent_t iter_ev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;                 // capture-only stream of the graphs
  hipGraphExec_t iter_graph[2] = {nullptr, nullptr};  // PCG loop body [null space]
  void drop_graphs() {
    for (hipGraphExec_t &g : iter_graph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
  ~mfmg_hierarchy() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hostS) (void)hipHostFree(hostS);
    if (host_done) (void)hipHostFree(host_done);
    for (hipEvent_t e : iter_ev)
      if (e) (void)hipEventDestroy(e);
  }
};

extern "C" const char *mfmg_last_error(void) { return g_err.c_str(); }

// --------------------------------------------------------------------------
// octree
// --------------------------------------------------------------------------
static mfmg_status convert_prims(const mfmg_refine_spec *spec, std::vector<Prim> &prims) {
  if (spec->n_prims < 0 || (spec->n_prims > 0 && !spec->prims))
    return fail(MFMG_ERR_INVALID_ARG, "bad primitive list");
  prims.assign(size_t(spec->n_prims), Prim{});
  for (int i = 0; i < spec->n_prims; ++i) {
    const mfmg_prim &p = spec->prims[i];
    Prim &q = prims[i];
    q.kind = p.kind;
    for (int a = 0; a < 3; ++a) {
      q.center[a] = p.center[a];
      q.lo[a] = p.lo[a];
      q.hi[a] = p.hi[a];
    }
    q.radius = p.radius;
    q.band = p.band;
    if (!(p.band >= 0.0)) return fail(MFMG_ERR_INVALID_ARG, "negative band");
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_build_octree(const mfmg_refine_spec *spec, mfmg_octree **out) {
  if (!spec || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  std::vector<Prim> prims;
  mfmg_status pst = convert_prims(spec, prims);
  if (pst != MFMG_OK) return pst;
  std::unique_ptr<mfmg_octree> t(new (std::nothrow) mfmg_octree());
  if (!t) return fail(MFMG_ERR_OOM, "host allocation failed");
  std::string err;
  try {
    err = build_topology(spec->min_level, spec->max_level, spec->node_size, prims, t->topo);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  if (!err.empty())
    return fail(err.find("balanced") != std::string::npos ? MFMG_ERR_TOPOLOGY
                                                          : MFMG_ERR_INVALID_ARG,
                err);
  t->on_host = true;
  t->min_level = t->topo.min_level;
  t->max_level = t->topo.max_level;
  t->nlb = t->topo.n_leaf_bricks;
  t->nb = t->topo.n_bricks;
  t->n_faces = t->topo.n_faces;
  t->n_tplus = t->topo.n_tplus;
  *out = t.release();
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_octree_info(const mfmg_octree *t, int64_t *n_leaves,
                                        int64_t *n_faces, int64_t *n_leaf_bricks) {
  if (!t) return fail(MFMG_ERR_INVALID_ARG, "NULL octree");
  if (n_leaves) *n_leaves = t->nlb * kCells;
  if (n_faces) *n_faces = t->n_faces;
  if (n_leaf_bricks) *n_leaf_bricks = t->nlb;
  return MFMG_OK;
}

static mfmg_status leaves_from_device(const mfmg_octree *t, uint8_t *level, int32_t *ijk);
static mfmg_status faces_from_device(const mfmg_octree *t, int64_t *owner, int8_t *dir,
                                     int64_t *other, int8_t *kind);

extern "C" mfmg_status mfmg_octree_leaves(const mfmg_octree *t, uint8_t *level, int32_t *ijk) {
  if (!t || !level || !ijk) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (!t->on_host) return leaves_from_device(t, level, ijk);
  const Topology &T = t->topo;
  for (int64_t b = 0; b < T.n_leaf_bricks; ++b)
    for (int m = 0; m < kCells; ++m) {
      int x, y, z;
      local_coords(m, x, y, z);
      int64_t c = b * kCells + m;
      level[c] = uint8_t(T.level[b]);
      ijk[3 * c] = T.coord[3 * b] * kBrick + x;
      ijk[3 * c + 1] = T.coord[3 * b + 1] * kBrick + y;
      ijk[3 * c + 2] = T.coord[3 * b + 2] * kBrick + z;
    }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_octree_faces(const mfmg_octree *t, int64_t *owner, int8_t *dir,
                                         int64_t *other, int8_t *kind) {
  if (!t || !owner || !dir || !other || !kind)
    return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (!t->on_host) return faces_from_device(t, owner, dir, other, kind);
  const Topology &T = t->topo;
  for (int64_t b = 0; b < T.n_leaf_bricks; ++b)
    for (int m = 0; m < kCells; ++m) {
      int64_t c = b * kCells + m;
      int64_t f = T.cell_fbase[c];
      for (int d = 0; d < 6; ++d) {
        if (!((T.cell_fmask[c] >> d) & 1)) continue;
        int64_t o;
        int k = T.cell_neighbour(b, m, d, &o);
        owner[f] = c;
        dir[f] = int8_t(d);
        other[f] = o;
        kind[f] = int8_t(k);
        ++f;
      }
    }
  return MFMG_OK;
}

extern "C" void mfmg_destroy_octree(mfmg_octree *t) { delete t; }

// --------------------------------------------------------------------------
// device topology and coefficients
// --------------------------------------------------------------------------
// From the host topology: perm maps a host brick id (canonical leaf order,
// then inner bricks) to its device id.
static void build_device_topology(const Topology &T, DeviceTopology &D, hipStream_t s) {
  int64_t nlb = T.n_leaf_bricks, nb = T.n_bricks;
  D.nlb = uint32_t(nlb);
  D.nb = uint32_t(nb);
  std::vector<int32_t> perm(nb, -1);
  std::vector<int32_t> order(nlb);
  for (int64_t i = 0; i < nlb; ++i) order[i] = int32_t(i);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return T.level[a] > T.level[b]; });
  std::vector<int32_t> canon(nlb);
  for (int64_t i = 0; i < nlb; ++i) {
    perm[order[i]] = int32_t(i);
    canon[i] = order[i];
  }
  for (int64_t b = nlb; b < nb; ++b) perm[b] = int32_t(b);  // inner ids already level-major
  int L = T.max_level;
  D.range.assign(L + 1, Range{0, 0, 0, 0});
  for (int64_t i = 0; i < nlb; ++i) {
    Range &R = D.range[T.level[order[i]]];
    if (R.n_leaf == 0) R.leaf_lo = uint32_t(i);
    R.n_leaf++;
  }
  for (int l = kMinLevel; l <= L; ++l)
    if (!T.level_inner[l].empty()) {
      D.range[l].inner_lo = uint32_t(T.level_inner[l].front());
      D.range[l].n_inner = uint32_t(T.level_inner[l].size());
    }
  std::vector<BrickMeta> meta_host(nb, BrickMeta{});
  std::vector<int32_t> child(8 * nb, -1);
  for (int64_t b = 0; b < nb; ++b) {
    BrickMeta &M = meta_host[perm[b]];
    std::memset(&M, 0, sizeof(M));
    M.flags = 0;
    for (int d = 0; d < 6; ++d) {
      int32_t n = T.nbr[6 * b + d];
      if (n <= kCoarseBase) {
        M.nbr[d] = encode_coarse(perm[decode_coarse(n)]);
        M.flags |= 1u << d;
      } else if (n == kWall) {
        M.nbr[d] = kWall;
        M.flags |= 1u << (16 + d);
      } else {
        M.nbr[d] = perm[n];
        if (n >= nlb) M.flags |= 1u << (8 + d);
      }
    }
    M.parent = T.parent[b] >= 0 ? perm[T.parent[b]] : -1;
    M.tplus = b < nlb ? T.tplus[b] : -1;
    for (int a = 0; a < 3; ++a) M.coord[a] = T.coord[3 * b + a];
    M.level = T.level[b];
    for (int o = 0; o < 8; ++o) {
      int32_t c = T.child[8 * b + o];
      child[8 * int64_t(perm[b]) + o] = c >= 0 ? perm[c] : -1;
    }
  }
  std::vector<int64_t> fbase(nlb * kCells);
  std::vector<uint8_t> fmask(nlb * kCells);
  for (int64_t b = 0; b < nlb; ++b)
    for (int m = 0; m < kCells; ++m) {
      fbase[int64_t(perm[b]) * kCells + m] = T.cell_fbase[b * kCells + m];
      fmask[int64_t(perm[b]) * kCells + m] = T.cell_fmask[b * kCells + m];
    }
  D.meta.upload(meta_host, s);
  D.child.upload(child, s);
  D.fbase.upload(fbase, s);
  D.fmask.upload(fmask, s);
  D.canon.upload(canon, s);
  HIP_CHECK(hipStreamSynchronize(s));
}

static Topo make_topo(const DeviceTopology &D, const BrickMeta *meta) {
  Topo t;
  t.nlb = D.nlb;
  t.nb = D.nb;
  t.meta = meta;
  t.child = D.child.p;
  t.pnb = nullptr;
  return t;
}

// Device tables of an octree: built with it on the device, or made from the
// host topology at first use (not thread-safe for one octree).
static std::shared_ptr<DeviceTopology> device_topology(const mfmg_octree *t, hipStream_t s) {
  if (!t->dt) {
    std::shared_ptr<DeviceTopology> d(new DeviceTopology());
    build_device_topology(t->topo, *d, s);
    t->dt = d;
  }
  return t->dt;
}

// exclusive scan of x[0, n) in place on stream s; *total (device) = sum
static void scan_exclusive(int64_t *x, int64_t n, int64_t *total, hipStream_t s) {
  int64_t tiles = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  DevBuf<int64_t> t;
  t.alloc(size_t(tiles));
  hipLaunchKernelGGL(k_scan_tiles, dim3(unsigned(tiles)), dim3(256), 0, s, x, n, t.p);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, t.p, tiles, total);
  hipLaunchKernelGGL(k_scan_add, dim3(unsigned(tiles)), dim3(256), 0, s, x, n,
                     (const int64_t *)t.p);
  HIP_CHECK(hipStreamSynchronize(s));  // t is freed on return
}

static unsigned key_grid(uint64_t nk) {
  return unsigned(std::min<uint64_t>((nk + 255) / 256, 65535));
}

// The octree of the spec built on the device (see octree_kernels.hpp);
// returns "" or an error message.
static std::string build_octree_device(const mfmg_refine_spec *spec,
                                       const std::vector<Prim> &prims, hipStream_t s,
                                       mfmg_octree &t) {
  if (spec->node_size != kBrick) return "node_size must be 4";
  int lmin = spec->min_level, lmax = spec->max_level;
  if (lmin < kMinLevel || lmax > kMaxLevel || lmin > lmax)
    return "levels out of range (2 <= min_level <= max_level <= 12)";
  for (const Prim &p : prims)
    if (p.kind != 0 && p.kind != 1) return "unknown primitive kind";
  OctTables T;
  T.min_level = lmin;
  T.max_level = lmax;
  uint64_t ns = 0, ni = 0;
  for (int l = 0; l < kOctLevels; ++l) T.split_off[l] = T.id_off[l] = 0;
  for (int l = kMinLevel; l <= lmax; ++l) {
    if (l < lmax) {
      T.split_off[l] = ns;
      ns += oct_keys(l);
    }
    T.id_off[l] = ni;
    ni += oct_keys(l);
  }
  DevBuf<uint8_t> split;
  DevBuf<int32_t> id;
  split.alloc(std::max<uint64_t>(ns, 1));
  id.alloc(ni);
  T.split = split.p;
  T.id = id.p;
  DevBuf<Prim> dprims;
  dprims.upload(prims, s);
  // refinement by the predicates, then 2:1 balance from the finest level down
  for (int l = kMinLevel; l < lmax; ++l)
    hipLaunchKernelGGL(k_oct_refine, dim3(key_grid(oct_keys(l))), dim3(256), 0, s, T, l,
                       (const Prim *)dprims.p, int(prims.size()));
  for (int l = lmax; l >= lmin + 2; --l)
    hipLaunchKernelGGL(k_oct_balance, dim3(key_grid(oct_keys(l))), dim3(256), 0, s, T, l);
  // leaf and inner counts per level
  uint64_t boff[kOctLevels + 1] = {0};
  for (int l = kMinLevel; l <= lmax; ++l)
    boff[l + 1] = boff[l] + (oct_keys(l) + kOctTile - 1) / kOctTile;
  for (int l = 0; l < kMinLevel; ++l) boff[l + 1] = 0;
  DevBuf<uint32_t> cnt, tot;
  cnt.alloc(2 * boff[lmax + 1]);
  tot.alloc(2 * kOctLevels);
  for (int l = kMinLevel; l <= lmax; ++l) {
    uint64_t nblk = boff[l + 1] - boff[l];
    hipLaunchKernelGGL(k_oct_count, dim3(unsigned(nblk)), dim3(kOctThreads), 0, s, T, l,
                       cnt.p + 2 * boff[l]);
    hipLaunchKernelGGL(k_oct_scan_pairs, dim3(1), dim3(1024), 0, s, cnt.p + 2 * boff[l], nblk,
                       tot.p + 2 * l);
  }
  std::vector<uint32_t> th(2 * kOctLevels, 0);
  HIP_CHECK(hipMemcpyAsync(th.data() + 2 * kMinLevel, tot.p + 2 * kMinLevel,
                           2 * (lmax + 1 - kMinLevel) * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  // device ids: leaves finest level first, then inner bricks finest first
  OctLevels LV;
  uint32_t inner_lo[kOctLevels] = {0};
  for (int l = 0; l < kOctLevels; ++l) LV.leaf_lo[l] = LV.n_leaf[l] = 0;
  uint64_t nlb = 0;
  for (int l = lmax; l >= kMinLevel; --l) {
    LV.leaf_lo[l] = uint32_t(nlb);
    LV.n_leaf[l] = th[2 * l];
    nlb += th[2 * l];
  }
  uint64_t nb = nlb;
  for (int l = lmax; l >= kMinLevel; --l) {
    inner_lo[l] = uint32_t(nb);
    nb += th[2 * l + 1];
  }
  if (nb >= (uint64_t(1) << 31) / kCells) return "octree too large";
  DevBuf<uint32_t> bkey;
  DevBuf<int8_t> blev;
  bkey.alloc(nb);
  blev.alloc(nb);
  for (int l = kMinLevel; l <= lmax; ++l)
    hipLaunchKernelGGL(k_oct_assign, dim3(unsigned(boff[l + 1] - boff[l])), dim3(kOctThreads),
                       0, s, T, l, (const uint32_t *)cnt.p + 2 * boff[l], LV.leaf_lo[l],
                       inner_lo[l], bkey.p, blev.p);
  std::shared_ptr<DeviceTopology> dp(new DeviceTopology());
  DeviceTopology &D = *dp;
  D.nlb = uint32_t(nlb);
  D.nb = uint32_t(nb);
  D.range.assign(lmax + 1, Range{0, 0, 0, 0});
  for (int l = kMinLevel; l <= lmax; ++l)
    D.range[l] = Range{th[2 * l] ? LV.leaf_lo[l] : 0u, th[2 * l],
                       th[2 * l + 1] ? inner_lo[l] : 0u, th[2 * l + 1]};
  D.meta.alloc(nb);
  D.child.alloc(8 * nb);
  D.canon.alloc(nlb);
  D.fbase.alloc(nlb * kCells);
  D.fmask.alloc(nlb * kCells);
  DevBuf<int32_t> inv;
  DevBuf<int> err;
  inv.alloc(nlb);
  err.alloc(1);
  HIP_CHECK(hipMemsetAsync(err.p, 0, sizeof(int), s));
  HIP_CHECK(hipMemsetAsync(inv.p, 0xff, size_t(nlb) * sizeof(int32_t), s));
  int eh = 0;
  if (nlb) {
    hipLaunchKernelGGL(k_oct_canon, dim3(grid_elems(int64_t(nlb), 256)), dim3(256), 0, s, T,
                       LV, uint32_t(nlb), (const uint32_t *)bkey.p, (const int8_t *)blev.p,
                       D.canon.p, inv.p, err.p);
    hipLaunchKernelGGL(k_oct_check_perm, dim3(grid_elems(int64_t(nlb), 256)), dim3(256), 0, s,
                       (const int32_t *)inv.p, uint32_t(nlb), err.p);
    HIP_CHECK(hipMemcpyAsync(&eh, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (eh) return "canonical leaf order is not a permutation";
  }
  hipLaunchKernelGGL(k_oct_meta, dim3(grid_elems(int64_t(nb), 256)), dim3(256), 0, s, T,
                     uint32_t(nlb), uint32_t(nb), (const uint32_t *)bkey.p,
                     (const int8_t *)blev.p, D.meta.p, D.child.p, err.p);
  // plus-side T-face slots and face numbering, both in canonical order
  DevBuf<int64_t> work, totals;
  work.alloc(std::max<uint64_t>(nlb, 1));
  totals.alloc(2);
  hipLaunchKernelGGL(k_oct_tflag, dim3(grid_elems(int64_t(nlb), 256)), dim3(256), 0, s,
                     (const BrickMeta *)D.meta.p, (const int32_t *)inv.p, uint32_t(nlb), work.p);
  scan_exclusive(work.p, int64_t(nlb), totals.p, s);
  hipLaunchKernelGGL(k_oct_tplus, dim3(grid_elems(int64_t(nlb), 256)), dim3(256), 0, s,
                     D.meta.p, (const int32_t *)inv.p, uint32_t(nlb), (const int64_t *)work.p);
  hipLaunchKernelGGL(k_oct_fmask, dim3(grid_for(int64_t(nlb))), dim3(kBlock), 0, s,
                     (const BrickMeta *)D.meta.p, (const int32_t *)D.canon.p, uint32_t(nlb),
                     D.fmask.p, work.p);
  scan_exclusive(work.p, int64_t(nlb), totals.p + 1, s);
  hipLaunchKernelGGL(k_oct_fbase, dim3(grid_for(int64_t(nlb))), dim3(kBlock), 0, s,
                     (const uint8_t *)D.fmask.p, (const int32_t *)D.canon.p, uint32_t(nlb),
                     (const int64_t *)work.p, D.fbase.p);
  int64_t th2[2];
  HIP_CHECK(hipMemcpyAsync(th2, totals.p, sizeof(th2), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&eh, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(s));
  if (eh) return "octree is not 2:1 balanced";
  t.on_host = false;
  t.min_level = lmin;
  t.max_level = lmax;
  t.nlb = int64_t(nlb);
  t.nb = int64_t(nb);
  t.n_tplus = th2[0];
  t.n_faces = th2[1];
  t.dt = dp;
  return "";
}

static mfmg_status leaves_to(const mfmg_octree *t, uint8_t *level, int32_t *ijk,
                             hipStream_t s) {
  std::shared_ptr<DeviceTopology> D = device_topology(t, s);
  if (D->nlb)
    hipLaunchKernelGGL(k_oct_leaves, dim3(grid_for(D->nlb)), dim3(kBlock), 0, s,
                       (const BrickMeta *)D->meta.p, (const int32_t *)D->canon.p, D->nlb, level,
                       ijk);
  HIP_CHECK(hipGetLastError());
  return MFMG_OK;
}

static mfmg_status faces_to(const mfmg_octree *t, int64_t *owner, int8_t *dir, int64_t *other,
                            int8_t *kind, hipStream_t s) {
  std::shared_ptr<DeviceTopology> D = device_topology(t, s);
  if (D->nlb)
    hipLaunchKernelGGL(k_oct_faces, dim3(grid_for(D->nlb)), dim3(kBlock), 0, s,
                       (const BrickMeta *)D->meta.p, (const int32_t *)D->canon.p,
                       (const int64_t *)D->fbase.p, (const uint8_t *)D->fmask.p, D->nlb, owner,
                       dir, other, kind);
  HIP_CHECK(hipGetLastError());
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_build_octree_device(const mfmg_refine_spec *spec, void *stream,
                                                mfmg_octree **out) {
  if (!spec || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  std::vector<Prim> prims;
  mfmg_status st = convert_prims(spec, prims);
  if (st != MFMG_OK) return st;
  std::unique_ptr<mfmg_octree> t(new (std::nothrow) mfmg_octree());
  if (!t) return fail(MFMG_ERR_OOM, "host allocation failed");
  std::string err;
  try {
    err = build_octree_device(spec, prims, (hipStream_t)stream, *t);
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  if (!err.empty())
    return fail(err.find("balanced") != std::string::npos ? MFMG_ERR_TOPOLOGY
                                                          : MFMG_ERR_INVALID_ARG,
                err);
  *out = t.release();
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_octree_leaves_device(const mfmg_octree *t, uint8_t *level,
                                                 int32_t *ijk, void *stream) {
  if (!t || !level || !ijk) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  try {
    return leaves_to(t, level, ijk, (hipStream_t)stream);
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
}

extern "C" mfmg_status mfmg_octree_faces_device(const mfmg_octree *t, int64_t *owner,
                                                int8_t *dir, int64_t *other, int8_t *kind,
                                                void *stream) {
  if (!t || !owner || !dir || !other || !kind)
    return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  try {
    return faces_to(t, owner, dir, other, kind, (hipStream_t)stream);
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
}

// host outputs of a device-built octree: the device outputs, copied back
static mfmg_status leaves_from_device(const mfmg_octree *t, uint8_t *level, int32_t *ijk) {
  try {
    hipStream_t s = nullptr;
    int64_t n = t->nlb * kCells;
    DevBuf<uint8_t> lv;
    DevBuf<int32_t> c;
    lv.alloc(size_t(std::max<int64_t>(n, 1)));
    c.alloc(size_t(std::max<int64_t>(3 * n, 1)));
    mfmg_status st = leaves_to(t, lv.p, c.p, s);
    if (st != MFMG_OK) return st;
    HIP_CHECK(hipMemcpyAsync(level, lv.p, size_t(n), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(ijk, c.p, size_t(3 * n) * sizeof(int32_t), hipMemcpyDeviceToHost,
                             s));
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

static mfmg_status faces_from_device(const mfmg_octree *t, int64_t *owner, int8_t *dir,
                                     int64_t *other, int8_t *kind) {
  try {
    hipStream_t s = nullptr;
    size_t n = size_t(std::max<int64_t>(t->n_faces, 1));
    DevBuf<int64_t> ow, ot;
    DevBuf<int8_t> di, ki;
    ow.alloc(n);
    ot.alloc(n);
    di.alloc(n);
    ki.alloc(n);
    mfmg_status st = faces_to(t, ow.p, di.p, ot.p, ki.p, s);
    if (st != MFMG_OK) return st;
    size_t nf = size_t(t->n_faces);
    HIP_CHECK(hipMemcpyAsync(owner, ow.p, nf * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(other, ot.p, nf * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(dir, di.p, nf, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(kind, ki.p, nf, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_assemble_coeffs(const mfmg_octree *tree, const double *face_beta,
                                            const mfmg_bc *bc, void *stream,
                                            mfmg_coeffs **out) {
  if (!tree || !face_beta || !bc || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  for (int d = 0; d < 6; ++d)
    if (bc->bc[d] != MFMG_NEUMANN && bc->bc[d] != MFMG_DIRICHLET)
      return fail(MFMG_ERR_INVALID_ARG, "bad boundary condition");
  if (!(bc->theta > 0.0 && bc->theta <= 1.0))
    return fail(MFMG_ERR_INVALID_ARG, "theta must be in (0, 1]");
  hipStream_t s = (hipStream_t)stream;
  try {
    std::unique_ptr<mfmg_coeffs> co(new mfmg_coeffs());
    co->tree = tree;
    co->bc = *bc;
    for (int d = 0; d < 6; ++d) co->has_dirichlet |= bc->bc[d] == MFMG_DIRICHLET;
    co->dt = device_topology(tree, s);
    co->coef.alloc(size_t(tree->nlb) * 256);
    co->tc.alloc(size_t(tree->n_tplus) * 48 + 1);
    AssembleArgs A;
    A.T = make_topo(*co->dt, co->dt->meta.p);
    A.fbase = co->dt->fbase.p;
    A.fmask = co->dt->fmask.p;
    A.beta = face_beta;
    for (int d = 0; d < 6; ++d) A.bc[d] = bc->bc[d];
    A.theta = bc->theta;
    A.coef = co->coef.p;
    A.tc = co->tc.p;
    if (tree->nlb)
      hipLaunchKernelGGL(k_assemble, dim3(grid_for(tree->nlb)), dim3(kBlock), 0, s, A);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
    *out = co.release();
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

// leaf coefficients (device order) -> [c | kx | ky | kz], each canonical
__global__ void k_coef_to_canonical(const double *coef, const int32_t *canon, uint32_t nlb,
                                    double *out) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= nlb) return;
  uint64_t N = uint64_t(nlb) * 64u;
  for (int comp = 0; comp < 4; ++comp)
    out[comp * N + uint64_t(canon[b]) * 64u + m] = coef[b * 256u + comp * 64 + m];
}

extern "C" mfmg_status mfmg_coeffs_leaf(const mfmg_coeffs *co, double *out, void *stream) {
  if (!co || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  try {
    hipLaunchKernelGGL(k_coef_to_canonical, dim3(grid_for(co->dt->nlb)), dim3(kBlock), 0, s,
                       (const double *)co->coef.p, (const int32_t *)co->dt->canon.p,
                       co->dt->nlb, out);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

extern "C" void mfmg_destroy_coeffs(mfmg_coeffs *co) { delete co; }

// --------------------------------------------------------------------------
// hierarchy
// --------------------------------------------------------------------------
extern "C" mfmg_status mfmg_build_hierarchy(const mfmg_coeffs *co, const mfmg_mg_params *prm,
                                            void *stream, mfmg_hierarchy **out) {
  if (!co || !prm || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  const mfmg_octree &T = *co->tree;
  if (prm->coarsest_level < kMinLevel || prm->coarsest_level > T.min_level)
    return fail(MFMG_ERR_INVALID_ARG, "coarsest_level must be in [2, min_level]");
  if (prm->nu_pre < 0 || prm->nu_post < 0 || prm->nu_coarse < 0 || prm->mu < 1 || prm->mu > 4)
    return fail(MFMG_ERR_INVALID_ARG, "bad smoothing counts or cycle index");
  if (!(prm->alpha > 0.0) || !std::isfinite(prm->beta_mg))
    return fail(MFMG_ERR_INVALID_ARG, "bad alpha or beta_mg");
  if (prm->precision != MFMG_FP64 && prm->precision != MFMG_MIXED)
    return fail(MFMG_ERR_INVALID_ARG, "bad precision");
  int64_t nlc = (int64_t(1) << prm->coarsest_level) / kBrick;
  if (nlc * nlc * nlc > 64) return fail(MFMG_ERR_INVALID_ARG, "coarsest level too large");
  {
    // The stencil kernels address their arrays with 32-bit byte offsets:
    // coefficient and plus-face arrays must stay within 4 GiB, the vectors
    // they read across faces below 2 GiB (an offset with bit 31 set is the
    // out-of-range load of a wall or T-face).  The FP64 composite operator
    // of the outer iteration runs in both precisions.
    const DeviceTopology &D = *co->dt;
    uint64_t nb = D.nb, nlb = D.nlb;
    uint64_t big = std::max(nlb * 256 * sizeof(double), nb * 48 * sizeof(double));
    uint64_t vec = nb * 64 * sizeof(double);
    if (prm->precision == MFMG_FP64)
      big = std::max(big, nb * 256 * sizeof(double));
    else
      big = std::max({big, nlb * 256 * sizeof(float), (nb - nlb) * 256 * sizeof(__half)});
    if (big > kMaxBufferBytes || vec >= kOutOfRange)
      return fail(MFMG_ERR_INVALID_ARG, "level arrays exceed the 32-bit offset range");
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    std::unique_ptr<mfmg_hierarchy> h(new mfmg_hierarchy());
    const DeviceTopology &D = *co->dt;
    h->co = co;
    h->prm = *prm;
    h->lc = prm->coarsest_level;
    h->L = 0;
    for (int l = kMinLevel; l <= T.max_level; ++l)
      if (D.range[l].n() > 0) h->L = l;
    int64_t nb = D.nb, nlb = D.nlb, N = nlb * 64;
    h->meta.alloc(D.nb);
    HIP_CHECK(hipMemcpyAsync(h->meta.p, D.meta.p, size_t(D.nb) * sizeof(BrickMeta),
                             hipMemcpyDeviceToDevice, s));
    h->coef64.alloc(size_t(nb) * 256);
    HIP_CHECK(hipMemcpyAsync(h->coef64.p, co->coef.p, size_t(nlb) * 256 * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_active_mask, dim3(grid_for(nlb)), dim3(kBlock), 0, s,
                       (const double *)h->coef64.p, 0u, uint32_t(nlb), h->meta.p);
    Topo topo = make_topo(D, h->meta.p);
    h->pnb.alloc(size_t(nb));
    if (nb > 0)
      hipLaunchKernelGGL(k_parent_nbrs, dim3(unsigned((nb + kBlock - 1) / kBlock)), dim3(kBlock),
                         0, s, topo, h->pnb.p);
    for (int l = T.max_level - 1; l >= kMinLevel; --l) {
      const Range &R = D.range[l];
      if (R.n_inner == 0) continue;
      hipLaunchKernelGGL(k_coarsen, dim3(grid_for(R.n_inner)), dim3(kBlock), 0, s, R.inner_lo,
                         R.n_inner, topo, h->coef64.p, prm->alpha);
      hipLaunchKernelGGL(k_active_mask, dim3(grid_for(R.n_inner)), dim3(kBlock), 0, s,
                         (const double *)h->coef64.p, R.inner_lo, R.n_inner, h->meta.p);
    }
    HIP_CHECK(hipGetLastError());
    h->pf64.alloc(size_t(nb) * 48);
    hipLaunchKernelGGL(k_plus_faces<double>, dim3(grid_for(nb)), dim3(kBlock), 0, s, topo,
                       (const double *)h->coef64.p, (const double *)co->tc.p, h->pf64.p, 0);
    if (prm->precision == MFMG_MIXED) {
      h->coef32.alloc(size_t(nlb) * 256);
      h->coef16.alloc(size_t(nb - nlb) * 256 + 1);
      h->tc32.alloc(co->tc.n);
      hipLaunchKernelGGL(k_convert_leaf, dim3(grid_elems(nlb * 256, 256)), dim3(256), 0, s,
                         (const double *)h->coef64.p, h->coef32.p, nlb * 256);
      hipLaunchKernelGGL(k_convert_leaf, dim3(grid_elems(int64_t(co->tc.n), 256)), dim3(256),
                         0, s, (const double *)co->tc.p, h->tc32.p, int64_t(co->tc.n));
      if (nb > nlb)
        hipLaunchKernelGGL(k_convert_inner, dim3(grid_for(nb - nlb)), dim3(kBlock), 0, s,
                           (const double *)h->coef64.p, topo, h->coef16.p);
      h->pf32.alloc(size_t(nb) * 48);
      hipLaunchKernelGGL(k_plus_faces<float>, dim3(grid_for(nb)), dim3(kBlock), 0, s, topo,
                         (const double *)h->coef64.p, (const double *)co->tc.p, h->pf32.p, 1);
      h->U32.alloc(size_t(nb) * 64);
      h->B32.alloc(size_t(nb) * 64);
      h->S32.alloc(size_t(nb - nlb) * 64 + 1);
      h->r.alloc(size_t(N));
    } else {
      h->U64.alloc(size_t(nb) * 64);
      h->B64.alloc(size_t(nb) * 64);
      h->S64.alloc(size_t(nb - nlb) * 64 + 1);
    }
    h->x.alloc(size_t(N));
    h->pd.alloc(size_t(nb) * 64);
    h->Xf.alloc(size_t(nb) * 64);
    h->Ap.alloc(size_t(N));
    h->partials.alloc(std::max<int64_t>({kMaxReduceBlocks, int64_t(grid_for(nlb)) + 8,
                                         int64_t(level_grid(nlb))}));
    h->S.alloc(1);
    HIP_CHECK(hipMemsetAsync(h->S.p, 0, sizeof(Scalars), s));
    HIP_CHECK(hipHostMalloc(&h->hostS, sizeof(Scalars), hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc(&h->host_done, sizeof(int), hipHostMallocMapped));
    HIP_CHECK(hipHostGetDevicePointer((void **)&h->host_done_dev, h->host_done, 0));
    *h->host_done = 0;
    for (hipEvent_t &e : h->iter_ev)
      HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // active leaf count (for the null-space mean)
    std::vector<BrickMeta> mh(nlb);
    HIP_CHECK(hipMemcpyAsync(mh.data(), h->meta.p, size_t(nlb) * sizeof(BrickMeta),
                             hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
    int64_t na = 0;
    for (const BrickMeta &M : mh) na += __builtin_popcount(M.act[0]) + __builtin_popcount(M.act[1]);
    h->n_active = double(na);
    {
      // bytes one half-sweep of a level touches: iterate and right-hand
      // side, four coefficients' worth of face data, the brick records
      bool mixed = prm->precision == MFMG_MIXED;
      double V = mixed ? 4.0 : 8.0, CL = mixed ? 4.0 : 8.0, CI = mixed ? 2.0 : 8.0;
      h->stream_lv.assign(size_t(T.max_level) + 1, 0);
      for (int l = kMinLevel; l <= T.max_level; ++l) {
        const Range &R = D.range[l];
        double ws = double(R.n_leaf) * (64 * (2 * V + 3.75 * CL) + 64) +
                    double(R.n_inner) * (64 * (2 * V + 3.75 * CI) + 64);
        h->stream_lv[size_t(l)] = ws > stream_threshold();
      }
      h->stream_composite = double(nlb) * (64 * (2 * 8.0 + 3.75 * 8.0) + 64) > stream_threshold();
    }
    {
      // k_bottom takes level lc + 1 (below the finest) and the coarsest
      // level when the former is a grid of at most kCoarsestBricks bricks
      // without T-junctions and the latter has at most kBottomCoarse bricks.
      // MFMG_FUSE_BOTTOM=0 (read at each build) keeps the separate kernels.
      const char *e = std::getenv("MFMG_FUSE_BOTTOM");
      int f = h->lc + 1;
      bool ok = !(e && e[0] == '0') && f < h->L && D.range[f].n() <= uint32_t(kCoarsestBricks) &&
                D.range[h->lc].n() <= uint32_t(kBottomCoarse);
      if (ok) {
        const Range &R = D.range[f];
        for (uint32_t i = 0; i < R.n_leaf; ++i)
          if (mh[R.leaf_lo + i].flags & kFlagT) ok = false;
        std::vector<BrickMeta> mi(R.n_inner);
        if (R.n_inner) {
          HIP_CHECK(hipMemcpyAsync(mi.data(), h->meta.p + R.inner_lo,
                                   size_t(R.n_inner) * sizeof(BrickMeta), hipMemcpyDeviceToHost,
                                   s));
          HIP_CHECK(hipStreamSynchronize(s));
        }
        for (const BrickMeta &M : mi)
          if (M.flags & kFlagT) ok = false;
      }
      h->fuse_bottom = ok;
    }
    {
      // MFMG_FUSE_PROLONG=0 (read at each build) keeps the separate
      // prolongation kernel.
      const char *e = std::getenv("MFMG_FUSE_PROLONG");
      h->fuse_prolong = !(e && e[0] == '0');
    }
    {
      // A level above the coarsest with no leaf at or below it takes its FAS
      // right-hand side in its first pre-smoothing half-sweep (k_smooth_fas).
      // MFMG_FUSE_FAS=0 (read at each build) keeps k_fas_rhs.
      const char *e = std::getenv("MFMG_FUSE_FAS");
      bool on = !(e && e[0] == '0');
      h->fold_fas.assign(D.range.size(), 0);
      bool leaf_below = false;
      for (size_t l = 0; l < D.range.size(); ++l) {
        leaf_below = leaf_below || D.range[l].n_leaf > 0;
        h->fold_fas[l] = on && int(l) > h->lc && int(l) < h->L && !leaf_below &&
                         D.range[l].n_inner > 0;
      }
    }
    *out = h.release();
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

// Device ids of the bricks of a level in Morton order at that level (leaf
// and inner bricks merged by their coordinates), with their records.
static void level_order(const mfmg_hierarchy *h, int level, std::vector<int32_t> &ids,
                        std::vector<BrickMeta> &recs, hipStream_t s) {
  const DeviceTopology &D = *h->co->dt;
  const Range &R = D.range[size_t(level)];
  std::vector<BrickMeta> leaf(R.n_leaf), inner(R.n_inner);
  if (R.n_leaf)
    HIP_CHECK(hipMemcpyAsync(leaf.data(), D.meta.p + R.leaf_lo, R.n_leaf * sizeof(BrickMeta),
                             hipMemcpyDeviceToHost, s));
  if (R.n_inner)
    HIP_CHECK(hipMemcpyAsync(inner.data(), D.meta.p + R.inner_lo,
                             R.n_inner * sizeof(BrickMeta), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  auto key = [](const BrickMeta &M) {
    uint64_t k = 0;
    for (int i = 0; i < 21; ++i)
      for (int a = 0; a < 3; ++a) k |= uint64_t((M.coord[a] >> i) & 1) << (3 * i + a);
    return k;
  };
  // both ranges are in Morton order already: merge them
  ids.clear();
  recs.clear();
  size_t i = 0, j = 0;
  while (i < leaf.size() || j < inner.size()) {
    bool take_leaf = j == inner.size() || (i < leaf.size() && key(leaf[i]) < key(inner[j]));
    if (take_leaf) {
      ids.push_back(int32_t(R.leaf_lo + i));
      recs.push_back(leaf[i++]);
    } else {
      ids.push_back(int32_t(R.inner_lo + j));
      recs.push_back(inner[j++]);
    }
  }
}

extern "C" mfmg_status mfmg_hierarchy_level_bricks(const mfmg_hierarchy *h, int level,
                                                   int64_t *count, int32_t *coords,
                                                   uint8_t *is_leaf) {
  if (!h || !count) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (level < kMinLevel || level > h->co->tree->max_level)
    return fail(MFMG_ERR_INVALID_ARG, "bad level");
  try {
    std::vector<int32_t> ids;
    std::vector<BrickMeta> recs;
    level_order(h, level, ids, recs, nullptr);
    *count = int64_t(ids.size());
    uint32_t nlb = h->co->dt->nlb;
    for (size_t i = 0; i < ids.size(); ++i) {
      if (coords)
        for (int a = 0; a < 3; ++a) coords[3 * i + a] = recs[i].coord[a];
      if (is_leaf) is_leaf[i] = uint32_t(ids[i]) < nlb;
    }
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_hierarchy_level_coeffs(const mfmg_hierarchy *h, int level,
                                                   double *out, void *stream) {
  if (!h || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (level < kMinLevel || level > h->co->tree->max_level)
    return fail(MFMG_ERR_INVALID_ARG, "bad level");
  hipStream_t s = (hipStream_t)stream;
  try {
    std::vector<int32_t> ids;
    std::vector<BrickMeta> recs;
    level_order(h, level, ids, recs, s);
    for (size_t i = 0; i < ids.size(); ++i)
      HIP_CHECK(hipMemcpyAsync(out + i * 256, h->coef64.p + int64_t(ids[i]) * 256,
                               256 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

extern "C" void mfmg_destroy_hierarchy(mfmg_hierarchy *h) { delete h; }

// --------------------------------------------------------------------------
// cycle driver
// --------------------------------------------------------------------------
namespace {

template <class V, class CL, class CI>
struct Cycle {
  const mfmg_hierarchy *h;
  const CL *leafc;
  const CI *innerc;
  const CL *pf;
  V *U, *B, *Ust;
  const int *done;
  hipStream_t s;
  // Policy of a streamed level's single-use loads.  FP32 cycle: only the
  // coefficients stream, so the finest level's iterate, right-hand side and
  // plus-face table stay in the Infinity Cache between half-sweeps (large
  // workload: finest half-sweep 114 -> 106 us, cycle 1.82 -> 1.77 ms).
  // FP64: all of them stream; its finest level's iterate, right-hand side
  // and plus faces alone exceed the cache, and keeping them cached made the
  // cycle slower (2.98 -> 3.14 ms).
  static constexpr int kCpolLevel = sizeof(V) == 4 ? kCpolStreamCoef : kCpolStream;

  V iscale(int l) const {
    return std::is_same<CI, __half>::value ? V(std::ldexp(1.0, -l)) : V(1);
  }
  LevelArgs<V, CL, CI> args(int l, bool inner_only) const {
    const DeviceTopology &D = *h->co->dt;
    LevelArgs<V, CL, CI> A;
    A.T = make_topo(D, h->meta.p);
    A.T.pnb = h->pnb.p;
    A.cf.leaf = leafc;
    A.cf.inner = innerc;
    A.cf.tc = nullptr;
    A.cf.nlb = D.nlb;
    A.cf.iscale = iscale(l);
    A.pf = pf;
    A.U = U;
    A.B = B;
    A.Ustar = Ust;
    A.R = D.range[l];
    if (inner_only) {
      A.R.n_leaf = 0;
      A.R.leaf_lo = 0;
    }
    A.done = done;
    return A;
  }

  bool stream(int l) const { return h->stream_lv[size_t(l)]; }
  template <int PR>
  void half_sweep_pr(int l, const LevelArgs<V, CL, CI> &A, int colour) const {
    dim3 g(stencil_grid<V>(A.R.n()));
    if (stream(l))
      hipLaunchKernelGGL((k_smooth<V, CL, CI, kCpolLevel, PR>), g, dim3(kBlock), 0, s, A,
                         colour);
    else
      hipLaunchKernelGGL((k_smooth<V, CL, CI, kCpolDefault, PR>), g, dim3(kBlock), 0, s, A,
                         colour);
  }
  // pr: 0 a plain half-sweep; 1 and 2 the first two half-sweeps of a
  // post-smoothing that takes the prolongation with it (k_smooth).
  void half_sweep(int l, const LevelArgs<V, CL, CI> &A, int colour, int pr = 0) const {
    if (pr == 1) half_sweep_pr<1>(l, A, colour);
    else if (pr == 2) half_sweep_pr<2>(l, A, colour);
    else half_sweep_pr<0>(l, A, colour);
  }
  // prolong: the level's FAS correction is still to be added (the first
  // two half-sweeps fold it in; nu >= 1).
  // fold: the level's FAS right-hand side is still to be formed, by its
  // first half-sweep (k_smooth_fas; the level has no leaves, nu >= 1).
  void smooth(int l, int first, int nu, bool zero_start = false, bool prolong = false,
              bool fold = false) const {
    auto A = args(l, false);
    if (A.R.n() == 0) return;
    for (int it = 0; it < nu; ++it)
      for (int c = 0; c < 2; ++c) {
        int colour = c == 0 ? first : 1 - first;
        dim3 g(stencil_grid<V>(A.R.n()));
        if (zero_start && it == 0 && c == 0) {
          if (stream(l))
            hipLaunchKernelGGL((k_smooth_zero<V, CL, CI, kCpolLevel>), g, dim3(kBlock), 0, s,
                               A, colour);
          else
            hipLaunchKernelGGL((k_smooth_zero<V, CL, CI>), g, dim3(kBlock), 0, s, A, colour);
        } else if (fold && it == 0 && c == 0) {
          dim3 gi(stencil_grid<V>(A.R.n_inner));
          if (stream(l))
            hipLaunchKernelGGL((k_smooth_fas<V, CL, CI, kCpolLevel>), gi, dim3(kBlock), 0, s,
                               A, colour);
          else
            hipLaunchKernelGGL((k_smooth_fas<V, CL, CI>), gi, dim3(kBlock), 0, s, A, colour);
        } else {
          half_sweep(l, A, colour, prolong && it == 0 ? 1 + c : 0);
        }
      }
  }

  // zero_start: the level's iterate is zero and its bricks are all leaves
  // (the finest level at the start of a cycle), so the first half-sweep
  // needs no neighbour values and also clears the iterate.
  // fold: as for smooth (the first visit of a level of fold_fas).
  void fas(int l, bool zero_start = false, bool fold = false) const {
    const mfmg_mg_params &p = h->prm;
    if (l == h->lc) {
      auto A = args(l, false);
      int threads = int(std::min<int64_t>(16, A.R.n())) * kWave;
      hipLaunchKernelGGL((k_coarsest<V, CL, CI>), dim3(1), dim3(threads), 0, s, A,
                         p.nu_coarse);
      return;
    }
    smooth(l, 0, p.nu_pre, zero_start, false, fold);
    auto A = args(l, false);
    V scale = V(p.beta_mg / p.alpha);
    if (stream(l))
      hipLaunchKernelGGL((k_restrict<V, CL, CI, kCpolLevel>), dim3(stencil_grid<V>(A.R.n())),
                         dim3(kBlock), 0, s, A, scale);
    else
      hipLaunchKernelGGL((k_restrict<V, CL, CI>), dim3(stencil_grid<V>(A.R.n())), dim3(kBlock),
                         0, s, A, scale);
    if (l - 1 == h->lc + 1 && h->fuse_bottom) {
      auto F = args(l - 1, false);
      auto Cc = args(h->lc, false);
      if constexpr (sizeof(V) == 4)
        hipLaunchKernelGGL((k_bottom<V, CL, CI, true>), dim3(1), dim3(1024), 0, s, F, Cc,
                           p.nu_pre, p.nu_post, p.nu_coarse, p.mu, 1, p.mu, scale);
      else
        for (int k = 0; k < p.mu; ++k)
          hipLaunchKernelGGL((k_bottom<V, CL, CI, false>), dim3(1), dim3(1024), 0, s, F, Cc,
                             p.nu_pre, p.nu_post, p.nu_coarse, p.mu, int(k == 0), 1, scale);
    } else {
      auto C = args(l - 1, true);
      bool fold = h->fold_fas[size_t(l - 1)] && p.nu_pre > 0;
      if (C.R.n() && !fold)
        hipLaunchKernelGGL((k_fas_rhs<V, CL, CI>), dim3(stencil_grid<V>(C.R.n_inner)),
                           dim3(kBlock), 0, s, C);
      for (int k = 0; k < p.mu; ++k) fas(l - 1, false, fold && k == 0);
    }
    if (h->fuse_prolong && p.nu_post > 0) {
      smooth(l, 1, p.nu_post, false, true);
    } else {
      hipLaunchKernelGGL((k_prolong<V, CL, CI>), dim3(stencil_grid<V>(A.R.n())), dim3(kBlock),
                         0, s, A);
      smooth(l, 1, p.nu_post);
    }
  }

  void run() const {
    const Range &RL = h->co->dt->range[h->L];
    bool zero_start = h->L > h->lc && h->prm.nu_pre > 0 && RL.n_inner == 0 && RL.leaf_lo == 0;
    int64_t lo = zero_start ? int64_t(RL.n_leaf) * 64 : 0;
    int64_t N = int64_t(h->co->dt->nlb) * 64 - lo;
    if (N > 0)
      hipLaunchKernelGGL((k_fill<V>), dim3(grid_elems(N, 256)), dim3(256), 0, s, U + lo, N,
                         V(0));
    fas(h->L, zero_start);
  }
};

void run_cycle(const mfmg_hierarchy *h, hipStream_t s, const int *done) {
  if (h->prm.precision == MFMG_MIXED) {
    Cycle<float, float, __half> c{h, h->coef32.p, h->coef16.p, h->pf32.p,
                                  h->U32.p, h->B32.p, h->S32.p, done, s};
    c.run();
  } else {
    // FP64 inner coefficients directly follow the leaf ones in coef64
    Cycle<double, double, double> c{h, h->coef64.p, h->coef64.p + int64_t(h->co->dt->nlb) * 256,
                                    h->pf64.p, h->U64.p, h->B64.p, h->S64.p, done, s};
    c.run();
  }
}

// Transpose of the cycle (exact adjoint of run_cycle's linear map), in
// residual form: RHO leaf part = input, output = Y leaf part.
template <class V, class CL, class CI>
struct CycleT {
  const mfmg_hierarchy *h;
  const CL *leafc;
  const CI *innerc;
  const CL *tc;
  const CL *pf;
  V *RHO, *Y, *W, *SBAR, *YS, *W2;
  hipStream_t s;
  const int *done;

  V iscale(int l) const {
    return std::is_same<CI, __half>::value ? V(std::ldexp(1.0, -l)) : V(1);
  }
  LevelArgsT<V, CL, CI> args(int l, int part) const {  // part: 0 all, 1 leaf only
    const DeviceTopology &D = *h->co->dt;
    LevelArgsT<V, CL, CI> A;
    A.T = make_topo(D, h->meta.p);
    A.T.pnb = h->pnb.p;
    A.cf.leaf = leafc;
    A.cf.inner = innerc;
    A.cf.tc = tc;
    A.cf.nlb = D.nlb;
    A.cf.iscale = iscale(l);
    A.RHO = RHO;
    A.Y = Y;
    A.W = W;
    A.W2 = W2;
    A.SBAR = SBAR;
    A.YS = YS;
    A.R = D.range[l];
    if (part == 1) {
      A.R.n_inner = 0;
      A.R.inner_lo = 0;
    }
    A.bscale = V(h->prm.beta_mg / h->prm.alpha);
    A.done = done;
    A.pf = pf;
    return A;
  }
  // RHO -= A^T w, w in buffer win, and the coupling of w to the coarser
  // level's leaves; colour >= 0: the apply step of a transposed half-sweep
  // of that colour; next >= 0: also the next half-sweep's w, into wout
  void launch_apply(int l, int colour, V *win, int next = -1, V *wout = nullptr) const {
    auto A = args(l, 0);
    A.W = win;
    A.W2 = wout ? wout : win;
    uint32_t nc = l > h->lc ? h->couple_n[size_t(l - 1)] : 0;
    if (nc) {
      // the apply step and the coupling in one launch
      auto C = args(l - 1, 1);
      C.W = win;
      const uint32_t *list = (const uint32_t *)h->couple.p + h->couple_lo[size_t(l - 1)];
      unsigned ga = stencil_grid_T<V>(A.R.n());
      dim3 g(ga + grid_for(nc));
      if (h->stream_lv[size_t(l)])
        hipLaunchKernelGGL((k_T_apply_couple<V, CL, CI, kCpolStream>), g, dim3(kBlock), 0, s, A,
                           colour, next, C, list, nc, ga);
      else
        hipLaunchKernelGGL((k_T_apply_couple<V, CL, CI>), g, dim3(kBlock), 0, s, A, colour,
                           next, C, list, nc, ga);
      return;
    }
    if (h->stream_lv[size_t(l)])
      hipLaunchKernelGGL((k_T_apply<V, CL, CI, kCpolStream>), dim3(stencil_grid_T<V>(A.R.n())),
                         dim3(kBlock), 0, s, A, colour, next);
    else
      hipLaunchKernelGGL((k_T_apply<V, CL, CI>), dim3(stencil_grid_T<V>(A.R.n())), dim3(kBlock),
                         0, s, A, colour, next);
  }
  // Transpose of smooth(l, (c0, 1 - c0), nu): 2 nu half-sweeps with the
  // colours in reversed order.  Each apply step also forms the w of the
  // half-sweep after it, alternating between W2 and W: the first w is in
  // W2 and the last in W (2 nu - 1 is odd).  w_ready: the caller's last
  // apply already put the first w in W2.
  void smooth_T(int l, int first, int nu, bool w_ready = false) const {
    auto A = args(l, 0);
    if (A.R.n() == 0 || nu == 0) return;
    if (!w_ready) {
      A.W = W2;
      if (h->stream_lv[size_t(l)])
        hipLaunchKernelGGL((k_T_sweep_w<V, CL, CI, kCpolStream>), dim3(stencil_grid_T<V>(A.R.n())),
                           dim3(kBlock), 0, s, A, first);
      else
        hipLaunchKernelGGL((k_T_sweep_w<V, CL, CI>), dim3(stencil_grid_T<V>(A.R.n())),
                           dim3(kBlock), 0, s, A, first);
    }
    V *buf[2] = {W2, W};
    for (int k = 0; k < 2 * nu; ++k) {
      int colour = (k & 1) ? 1 - first : first;
      int next = k + 1 < 2 * nu ? 1 - colour : -1;
      launch_apply(l, colour, buf[k & 1], next, buf[(k & 1) ^ 1]);
    }
  }
  void fas_T(int l) const {
    const mfmg_mg_params &p = h->prm;
    if (l == h->lc) {
      auto A = args(l, 0);
      int threads = int(std::min<int64_t>(16, A.R.n())) * kWave;
      hipLaunchKernelGGL((k_T_coarsest<V, CL, CI>), dim3(1), dim3(threads), 0, s, A,
                         p.nu_coarse);
      return;
    }
    smooth_T(l, 0, p.nu_post);  // forward post-smoothing is (B,R)^nu
    auto A = args(l, 0);
    hipLaunchKernelGGL((k_T_restrict<V, CL, CI>), dim3(grid_for(A.R.n())), dim3(kBlock), 0, s,
                       A);
    for (int k = 0; k < p.mu; ++k) fas_T(l - 1);
    auto C = args(l - 1, 0);
    hipLaunchKernelGGL((k_T_coarse<V, CL, CI>), dim3(grid_for(C.R.n())), dim3(kBlock), 0, s, C);
    hipLaunchKernelGGL((k_T_fas<V, CL, CI>), dim3(stencil_grid_T<V>(C.R.n())), dim3(kBlock), 0,
                       s, C);
    hipLaunchKernelGGL((k_T_prolong<V, CL, CI>), dim3(grid_for(A.R.n())), dim3(kBlock), 0, s,
                       A);
    // forward pre-smoothing is (R,B)^nu; its transpose starts with colour 1
    if (p.nu_pre > 0) {
      launch_apply(l, -1, W, 1, W2);
      smooth_T(l, 1, p.nu_pre, true);
    } else {
      launch_apply(l, -1, W);
    }
  }
  // input: an FP64 leaf vector in device order, multiplied by *scale on
  // loading (scale may be null)
  void run(const double *in, const double *scale) const {
    const DeviceTopology &D = *h->co->dt;
    int64_t nb64 = int64_t(D.nb) * 64, N = int64_t(D.nlb) * 64;
    hipLaunchKernelGGL((k_fill<V>), dim3(grid_elems(nb64, 256)), dim3(256), 0, s, Y, nb64, V(0));
    hipLaunchKernelGGL((k_fill<V>), dim3(grid_elems(nb64 - N, 256)), dim3(256), 0, s, RHO + N,
                       nb64 - N, V(0));
    hipLaunchKernelGGL((k_T_load<V>), dim3(grid_elems(N, 256)), dim3(256), 0, s, in, RHO, N,
                       scale);
    fas_T(h->L);
  }
};

template <class V>
void alloc_transpose(const mfmg_hierarchy *hc, DevBuf<V> (&T)[6]) {
  if (T[0].p) return;
  int64_t nb = hc->co->dt->nb, nlb = hc->co->dt->nlb;
  for (int i = 0; i < 3; ++i) T[i].alloc(size_t(nb) * 64);
  for (int i = 3; i < 5; ++i) T[i].alloc(size_t(nb - nlb) * 64 + 1);
  T[5].alloc(size_t(nb) * 64);
}

// The leaf bricks whose coarse cells take the transposed T-junction coupling
// (those with an inner face neighbour), per level, made at first use.
static void ensure_coupling_lists(mfmg_hierarchy *h, hipStream_t s) {
  if (!h->couple_n.empty()) return;
  const DeviceTopology &D = *h->co->dt;
  uint32_t nlb = D.nlb;
  std::vector<int64_t> pos(size_t(nlb) + 1, 0);
  DevBuf<int64_t> work, total;
  work.alloc(std::max<size_t>(nlb, 1));
  total.alloc(1);
  hipLaunchKernelGGL(k_couple_flag, dim3(grid_elems(nlb, 256)), dim3(256), 0, s,
                     (const BrickMeta *)D.meta.p, nlb, work.p);
  scan_exclusive(work.p, int64_t(nlb), total.p, s);
  HIP_CHECK(hipMemcpyAsync(pos.data(), work.p, size_t(nlb) * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(pos.data() + nlb, total.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  h->couple.alloc(std::max<size_t>(size_t(pos[nlb]), 1));
  hipLaunchKernelGGL(k_couple_list, dim3(grid_elems(nlb, 256)), dim3(256), 0, s,
                     (const BrickMeta *)D.meta.p, nlb, (const int64_t *)work.p, h->couple.p);
  HIP_CHECK(hipGetLastError());
  h->couple_lo.assign(D.range.size(), 0);
  h->couple_n.assign(D.range.size(), 0);
  for (size_t l = 0; l < D.range.size(); ++l) {
    const Range &R = D.range[l];
    if (!R.n_leaf) continue;
    h->couple_lo[l] = uint32_t(pos[R.leaf_lo]);
    h->couple_n[l] = uint32_t(pos[R.leaf_lo + R.n_leaf] - pos[R.leaf_lo]);
  }
  HIP_CHECK(hipStreamSynchronize(s));  // work is freed on return
}

// z = M^T r: r, z FP64 leaf vectors in device order; returns the z buffer
// (the Y leaf part, of the cycle's value type).  In mixed precision the
// solve passes its scalars' residual scale (scale), so z is M^T (scale r).
void run_cycle_T(mfmg_hierarchy *h, const double *r, hipStream_t s,
                 const int *done = nullptr, const double *scale = nullptr) {
  ensure_coupling_lists(h, s);
  if (h->prm.precision == MFMG_MIXED) {
    alloc_transpose(h, h->T32);
    CycleT<float, float, __half> c{h, h->coef32.p, h->coef16.p, h->tc32.p, h->pf32.p,
                                   h->T32[0].p, h->T32[1].p, h->T32[2].p, h->T32[3].p,
                                   h->T32[4].p, h->T32[5].p, s, done};
    c.run(r, scale);
  } else {
    alloc_transpose(h, h->T64);
    CycleT<double, double, double> c{h, h->coef64.p,
                                     h->coef64.p + int64_t(h->co->dt->nlb) * 256,
                                     h->co->tc.p, h->pf64.p, h->T64[0].p, h->T64[1].p,
                                     h->T64[2].p, h->T64[3].p, h->T64[4].p, h->T64[5].p, s,
                                     done};
    c.run(r, nullptr);
  }
}

PcgArgs pcg_args(mfmg_hierarchy *h) {
  PcgArgs P;
  P.T = make_topo(*h->co->dt, h->meta.p);
  P.C = h->coef64.p;
  P.TC = h->co->tc.p;
  P.PF = h->pf64.p;
  P.canon = h->co->dt->canon.p;
  P.S = h->S.p;
  P.partials = h->partials.p;
  P.hist = h->hist.p;
  P.host_done = h->host_done_dev;
  P.scale_low = h->prm.precision == MFMG_MIXED ? 1 : 0;
  return P;
}

}  // namespace

// --------------------------------------------------------------------------
// component entry points
// --------------------------------------------------------------------------
extern "C" mfmg_status mfmg_apply_operator(mfmg_hierarchy *h, const double *x, double *y,
                                           int transpose, void *stream) {
  if (!h || !x || !y) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  unsigned G = grid_for(h->co->dt->nlb);
  try {
    PcgArgs P = pcg_args(h);
    hipLaunchKernelGGL(k_full, dim3(G), dim3(kBlock), 0, s, P, x, h->Xf.p, 1);
    if (transpose)
      hipLaunchKernelGGL(k_applyT, dim3(G), dim3(kBlock), 0, s, P, (const double *)h->Xf.p,
                         h->Ap.p);
    else
      hipLaunchKernelGGL(k_apply, dim3(level_grid(h->co->dt->nlb)), dim3(kBlock), 0, s, P,
                         (const double *)h->Xf.p, h->Ap.p);
    hipLaunchKernelGGL(k_to_canonical<double>, dim3(G), dim3(kBlock), 0, s, P,
                       (const double *)h->Ap.p, y);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_apply_precond(mfmg_hierarchy *h, const double *r, double *z,
                                          int transpose, void *stream) {
  if (!h || !r || !z) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  unsigned G = grid_for(h->co->dt->nlb);
  try {
    PcgArgs P = pcg_args(h);
    if (transpose) {
      if (!h->rA.p) h->rA.alloc(size_t(h->co->dt->nlb) * 64);
      hipLaunchKernelGGL(k_from_canonical<double>, dim3(G), dim3(kBlock), 0, s, P, r, h->rA.p);
      run_cycle_T(h, h->rA.p, s);
      if (h->prm.precision == MFMG_MIXED)
        hipLaunchKernelGGL(k_to_canonical<float>, dim3(G), dim3(kBlock), 0, s, P,
                           (const float *)h->T32[1].p, z);
      else
        hipLaunchKernelGGL(k_to_canonical<double>, dim3(G), dim3(kBlock), 0, s, P,
                           (const double *)h->T64[1].p, z);
    } else if (h->prm.precision == MFMG_MIXED) {
      hipLaunchKernelGGL(k_from_canonical<float>, dim3(G), dim3(kBlock), 0, s, P, r, h->B32.p);
      run_cycle(h, s, nullptr);
      hipLaunchKernelGGL(k_to_canonical<float>, dim3(G), dim3(kBlock), 0, s, P,
                         (const float *)h->U32.p, z);
    } else {
      hipLaunchKernelGGL(k_from_canonical<double>, dim3(G), dim3(kBlock), 0, s, P, r, h->B64.p);
      run_cycle(h, s, nullptr);
      hipLaunchKernelGGL(k_to_canonical<double>, dim3(G), dim3(kBlock), 0, s, P,
                         (const double *)h->U64.p, z);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

// --------------------------------------------------------------------------
// PCG (Algorithm 1)
// --------------------------------------------------------------------------
// Reductions of the PCG: the kernel stores one partial per workgroup and
// k_finish adds them in fixed order and updates the scalars.
struct Reduce {
  PcgArgs P;
  hipStream_t s;
  unsigned G;  // grid of the flat leaf kernels

  Reduce(mfmg_hierarchy *h, hipStream_t s_) : P(pcg_args(h)), s(s_) {
    G = grid_reduce(h->co->dt->nlb);
  }
  void finish(unsigned n, int op, int arg = 0, double rtol = 0.0) const {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, P, int64_t(n), op, arg, rtol);
  }
  template <class V>
  void init(const double *rhs, double *r, V *r_low, double *x, double rtol) const {
    hipLaunchKernelGGL(k_pcg_init<V>, dim3(G), dim3(kBlock), 0, s, P, rhs, r, r_low, x);
    finish(G, kFinInit, 0, rtol);
  }
  // v -= mean over active cells (Section 2.2); mode as k_shift_mean
  template <class V>
  void shift_mean(double *v, V *v_low, double na, int mode, double rtol) const {
    hipLaunchKernelGGL(k_sum_active, dim3(G), dim3(kBlock), 0, s, P, (const double *)v);
    finish(G, kFinSum);
    hipLaunchKernelGGL(k_shift_mean<V>, dim3(G), dim3(kBlock), 0, s, P, v, v_low, na, mode);
    if (mode != 3) finish(G, kFinShift, mode, rtol);
  }
  // sum over the active cells of v (canonical order) or of |v|, on the host
  double active_sum(const double *v, int absval, const double *dev_sum) const {
    hipLaunchKernelGGL(k_sum_active_canon, dim3(G), dim3(kBlock), 0, s, P, v, absval);
    finish(G, kFinSum);
    double x = 0.0;
    HIP_CHECK(hipMemcpyAsync(&x, dev_sum, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return x;
  }
  void true_resid(const double *rhs, const double *X, uint32_t nlb) const {
    unsigned g = level_grid(nlb);
    hipLaunchKernelGGL(k_true_resid, dim3(g), dim3(kBlock), 0, s, P, rhs, X);
    finish(g, kFinTrue);
  }
};

// The canonical face list with the per-brick levels and activity masks in
// canonical order (for per-face kernels), made at first use and kept.
static void ensure_face_list(mfmg_hierarchy *h, hipStream_t s) {
  if (h->f_owner.p) return;
  const DeviceTopology &D = *h->co->dt;
  size_t nf = size_t(std::max<int64_t>(h->co->tree->n_faces, 1));
  h->f_owner.alloc(nf);
  h->f_other.alloc(nf);
  h->f_dir.alloc(nf);
  h->f_kind.alloc(nf);
  h->leaf_level.alloc(size_t(D.nlb));
  h->canon_act.alloc(size_t(D.nlb));
  if (D.nlb) {
    hipLaunchKernelGGL(k_oct_faces, dim3(grid_for(D.nlb)), dim3(kBlock), 0, s,
                       (const BrickMeta *)D.meta.p, (const int32_t *)D.canon.p,
                       (const int64_t *)D.fbase.p, (const uint8_t *)D.fmask.p, D.nlb,
                       h->f_owner.p, h->f_dir.p, h->f_other.p, h->f_kind.p);
    hipLaunchKernelGGL(k_oct_canon_level, dim3(grid_elems(D.nlb, 256)), dim3(256), 0, s,
                       (const BrickMeta *)D.meta.p, (const int32_t *)D.canon.p, D.nlb,
                       h->leaf_level.p);
    hipLaunchKernelGGL(k_canonical_act, dim3(grid_elems(D.nlb, 256)), dim3(256), 0, s,
                       (const BrickMeta *)h->meta.p, (const int32_t *)D.canon.p, D.nlb,
                       h->canon_act.p);
  }
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(s));
}

// Without a Dirichlet face A is singular on the constants of the active
// cells (Section 2.2); with the null-space shift off, a right-hand side whose
// active sum is not zero (relative to the sum of its magnitudes) has no
// solution.
static bool incompatible_rhs(mfmg_hierarchy *h, const double *rhs, hipStream_t s) {
  Reduce R(h, s);
  const double *dev_sum = &h->S.p->sum;
  double sum = R.active_sum(rhs, 0, dev_sum);
  double mag = R.active_sum(rhs, 1, dev_sum);
  return std::fabs(sum) > 1e-10 * mag;
}

// Launch helpers of one Krylov iteration (Algorithm 1).
template <class V>
struct Krylov {
  mfmg_hierarchy *h;
  PcgArgs P;
  hipStream_t s;
  unsigned G;   // grid of the flat vector kernels
  unsigned GB;  // one wave per leaf brick (transposed operator)
  unsigned GA;  // wave_loop grid of the forward operator
  int64_t n2;   // leaf entries / 2

  Krylov(mfmg_hierarchy *h_, hipStream_t s_) : h(h_), s(s_) {
    P = pcg_args(h);
    G = grid_reduce(h->co->dt->nlb);
    GB = grid_for(h->co->dt->nlb);
    GA = level_grid(h->co->dt->nlb);
    n2 = int64_t(h->co->dt->nlb) * 32;
  }
  void rz(const double *r, const V *z, int first) const {
    hipLaunchKernelGGL(k_pcg_rz<V>, dim3(GA), dim3(kBlock), 0, s, P, r, z);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, P, int64_t(GA), int(kFinRz), first,
                       0.0);
  }
  void pupdate(const V *z, int first) const {
    hipLaunchKernelGGL(k_pcg_p<V>, dim3(GA), dim3(kBlock), 0, s, P, z, h->pd.p, h->x.p, first);
  }
  void Ap(bool trans) const {
    if (trans)
      hipLaunchKernelGGL(k_pcg_ApT, dim3(GB), dim3(kBlock), 0, s, P, (const double *)h->pd.p,
                         h->Ap.p);
    else if (h->stream_composite)
      hipLaunchKernelGGL(k_pcg_Ap<kCpolStream>, dim3(GA), dim3(kBlock), 0, s, P,
                         (const double *)h->pd.p, h->Ap.p);
    else
      hipLaunchKernelGGL(k_pcg_Ap<>, dim3(GA), dim3(kBlock), 0, s, P, (const double *)h->pd.p,
                         h->Ap.p);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, P, int64_t(trans ? GB : GA),
                       int(kFinAlpha), 0, 0.0);
  }
  void update(double *r, V *r_low, int defer) const {
    hipLaunchKernelGGL(k_pcg_update<V>, dim3(G), dim3(kBlock), 0, s, P, r, r_low,
                       (const double *)h->Ap.p, defer, n2);
    if (!defer)
      hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, P, int64_t(G), int(kFinUpdate),
                         0, 0.0);
  }
  // after the loop: the iterate's last step, if the solve stopped between a
  // residual update and the k_pcg_p that takes it
  void finish_x() const {
    hipLaunchKernelGGL(k_pcg_x, dim3(G), dim3(kBlock), 0, s, P, h->x.p,
                       (const double *)h->pd.p);
  }
};

// Loop body of Algorithm 1 (from A p to the next search direction).
template <class V>
static void iteration_body(mfmg_hierarchy *h, double *r, V *r_low, V *z, bool null_space,
                           hipStream_t s) {
  Reduce R(h, s);
  Krylov<V> K(h, s);
  K.Ap(false);
  K.update(r, r_low, int(null_space));
  if (null_space) R.shift_mean<V>(r, r_low, std::max(1.0, h->n_active), 1, 0.0);
  run_cycle(h, s, &h->S.p->done);
  K.rz(r, z, 0);
  K.pupdate(z, 0);
}

// Launch graphs can be switched off with MFMG_GRAPHS=0 (read once).
inline bool graphs_enabled() {
  static const bool on = [] {
    const char *e = std::getenv("MFMG_GRAPHS");
    return !(e && e[0] == '0');
  }();
  return on;
}

// The loop body as one HIP graph, captured once per hierarchy: about a
// hundred launches, the coarse-level ones only a few microseconds long --
// shorter than the host needs to issue them one at a time.  Every argument
// is a pointer or size fixed for the hierarchy (the residual history buffer
// only grows, and drops the graphs when it does); the body records no
// memset or copy.  Captured on a private stream, launched on the caller's.
template <class V>
static hipGraphExec_t iteration_graph(mfmg_hierarchy *h, double *r, V *r_low, V *z,
                                      bool null_space) {
  hipGraphExec_t &ge = h->iter_graph[null_space ? 1 : 0];
  if (ge) return ge;
  if (!h->cap_stream) HIP_CHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIP_CHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    iteration_body<V>(h, r, r_low, z, null_space, h->cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(h->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_CHECK(hipStreamEndCapture(h->cap_stream, &g));
  hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ge = nullptr;
    HIP_CHECK(e);
  }
  return ge;
}

// The stop test of Algorithm 1 is taken on the recursively updated residual;
// after it fires the FP64 true residual ||rhs - A x|| is formed.  While that
// exceeds the tolerance and iterations are left, the iteration starts again
// from x with r = rhs - A x (tolerance and iteration budget unchanged), so a
// solve reported as converged meets rtol in its true residual.  A restart that
// does not lower the true residual ends the solve (not converged).
// Status of a finished solve from its scalars: breakdown, not converged
// (recurrence or true residual above the tolerance), or OK.
static mfmg_status solve_status(const Scalars &S) {
  if (S.status == -5) return MFMG_ERR_BREAKDOWN;
  if (S.rr0 > 0.0 && (!(S.rr <= S.tol2) || !(S.tr <= S.tol2))) return MFMG_NOT_CONVERGED;
  return MFMG_OK;
}

static bool restart_wanted(const Scalars &S, int max_iter, double prev_tr) {
  return S.status == 0 && S.rr0 > 0.0 && S.rr <= S.tol2 && S.tr > S.tol2 &&
         S.iters < max_iter && S.tr < prev_tr;
}

// Queue up to n iterations of the loop body; returns when the stop flag is
// seen or n have been queued.
template <class V>
static void run_iterations(mfmg_hierarchy *h, double *r, V *r_low, V *z, bool null_space,
                           int n, hipGraphExec_t body, hipStream_t s) {
  for (int it = 0; it < n; ++it) {
    if (body)
      HIP_CHECK(hipGraphLaunch(body, s));
    else
      iteration_body<V>(h, r, r_low, z, null_space, s);
    // The stop flag of iteration it is read on the host only after
    // iteration it + 1 is queued, so the GPU never idles on the round trip;
    // every kernel of an iteration queued after the stop returns at once.
    // k_finish mirrors the flag into mapped host memory (no copy launch).
    HIP_CHECK(hipEventRecord(h->iter_ev[it & 1], s));
    if (it > 0) {
      HIP_CHECK(hipEventSynchronize(h->iter_ev[(it - 1) & 1]));
      if (__atomic_load_n(h->host_done, __ATOMIC_ACQUIRE)) break;
    }
  }
}

template <class V>
static void pcg_iterate(mfmg_hierarchy *h, const double *rhs, double *r, V *r_low, V *z,
                        const mfmg_solve_params *sp, bool null_space, hipStream_t s,
                        const double *x0) {
  PcgArgs P = pcg_args(h);
  unsigned G = grid_reduce(h->co->dt->nlb);
  unsigned GL = level_grid(h->co->dt->nlb);
  Reduce R(h, s);
  const int *done = &h->S.p->done;
  double na = std::max(1.0, h->n_active);
  double *x = h->x.p;
  __atomic_store_n(h->host_done, 0, __ATOMIC_RELEASE);  // the stream is idle here
  R.init<V>(rhs, r, (V *)nullptr, x, sp->rtol);
  if (null_space) R.shift_mean<V>(r, (V *)nullptr, na, 0, sp->rtol);
  if (x0) {
    // r = rhs - A x0; the tolerance stays rtol ||rhs|| from the step above
    hipLaunchKernelGGL(k_full, dim3(G), dim3(kBlock), 0, s, P, x0, h->Xf.p, 1);
    hipLaunchKernelGGL(k_residual_vec, dim3(GL), dim3(kBlock), 0, s, P, rhs,
                       (const double *)h->Xf.p, r);
    hipLaunchKernelGGL(k_warm_start<V>, dim3(G), dim3(kBlock), 0, s, P, x0, x,
                       (const double *)r, (V *)nullptr);
    R.finish(G, kFinWarm);
  }
  if (r_low) hipLaunchKernelGGL(k_scale_low<V>, dim3(G), dim3(kBlock), 0, s, P, r, r_low);
  Krylov<V> K(h, s);
  run_cycle(h, s, done);
  K.rz(r, z, 1);
  K.pupdate(z, 1);
  hipGraphExec_t body = graphs_enabled() && sp->max_iter > 0
                           ? iteration_graph<V>(h, r, r_low, z, null_space)
                           : nullptr;
  double prev_tr = INFINITY;
  int left = sp->max_iter;
  for (;;) {
    run_iterations<V>(h, r, r_low, z, null_space, left, body, s);
    K.finish_x();
    // zero-mean solution, then the true residual (shifted to zero mean)
    if (null_space) R.shift_mean<double>(x, (double *)nullptr, na, 3, 0.0);
    hipLaunchKernelGGL(k_full, dim3(G), dim3(kBlock), 0, s, P, (const double *)x, h->Xf.p, 0);
    if (null_space) {
      hipLaunchKernelGGL(k_residual_vec, dim3(GL), dim3(kBlock), 0, s, P, rhs,
                         (const double *)h->Xf.p, h->Ap.p);
      R.shift_mean<double>(h->Ap.p, (double *)nullptr, na, 2, 0.0);
    } else {
      R.true_resid(rhs, (const double *)h->Xf.p, h->co->dt->nlb);
    }
    HIP_CHECK(hipMemcpyAsync(h->hostS, h->S.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    const Scalars S = *h->hostS;
    if (!restart_wanted(S, sp->max_iter, prev_tr)) break;
    prev_tr = S.tr;
    left = sp->max_iter - S.iters;
    // r = rhs - A x (the null-space form is already in Ap)
    if (!null_space)
      hipLaunchKernelGGL(k_residual_vec, dim3(GL), dim3(kBlock), 0, s, P, rhs,
                         (const double *)h->Xf.p, h->Ap.p);
    hipLaunchKernelGGL(k_restart, dim3(G), dim3(kBlock), 0, s, P, (const double *)h->Ap.p, r);
    R.finish(G, kFinRestart);
    if (r_low) hipLaunchKernelGGL(k_scale_low<V>, dim3(G), dim3(kBlock), 0, s, P, r, r_low);
    run_cycle(h, s, done);
    K.rz(r, z, 1);
    K.pupdate(z, 1);
  }
  HIP_CHECK(hipGetLastError());
}

extern "C" mfmg_status mfmg_pcg_solve(mfmg_hierarchy *h, const double *rhs, double *p,
                                      const mfmg_solve_params *sp, void *stream,
                                      mfmg_solve_stats *stats, double *hist) {
  if (!h || !rhs || !p || !sp) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (!(sp->rtol >= 0.0) || sp->max_iter < 0) return fail(MFMG_ERR_INVALID_ARG, "bad params");
  if (sp->null_space < -1 || sp->null_space > 1)
    return fail(MFMG_ERR_INVALID_ARG, "null_space must be -1, 0 or 1");
  bool ns = sp->null_space == 1 || (sp->null_space == -1 && !h->co->has_dirichlet);
  if (sp->warm_start != 0 && sp->warm_start != 1)
    return fail(MFMG_ERR_INVALID_ARG, "warm_start must be 0 or 1");
  if (sp->warm_start && ns)
    return fail(MFMG_ERR_INVALID_ARG, "warm start is not available with the null-space shift");
  hipStream_t s = (hipStream_t)stream;
  mfmg_status st = MFMG_OK;
  try {
    if (h->hist.n < size_t(sp->max_iter) + 2) {
      h->drop_graphs();  // they hold the old history pointer
      h->hist.alloc(std::max<size_t>(size_t(sp->max_iter) + 2, 1024));
    }
    if (!ns && !h->co->has_dirichlet && incompatible_rhs(h, rhs, s))
      return fail(MFMG_ERR_INCOMPATIBLE_RHS,
                  "no Dirichlet face and the null-space shift is off, but the right-hand "
                  "side does not sum to zero over the active cells");
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    HIP_CHECK(hipEventRecord(e0, s));
    if (h->prm.precision == MFMG_MIXED)
      pcg_iterate<float>(h, rhs, h->r.p, h->B32.p, h->U32.p, sp, ns, s,
                         sp->warm_start ? (const double *)p : nullptr);
    else
      pcg_iterate<double>(h, rhs, h->B64.p, (double *)nullptr, h->U64.p, sp, ns, s,
                          sp->warm_start ? (const double *)p : nullptr);
    PcgArgs P = pcg_args(h);
    hipLaunchKernelGGL(k_to_canonical<double>, dim3(grid_for(h->co->dt->nlb)), dim3(kBlock), 0,
                       s, P, (const double *)h->x.p, p);
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipMemcpyAsync(h->hostS, h->S.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const Scalars &S = *h->hostS;
    st = solve_status(S);
    if (stats) {
      stats->iters = S.iters;
      stats->status = st;
      stats->rel_resid_recur = S.rr0 > 0.0 ? std::sqrt(S.rr / S.rr0) : 0.0;
      stats->rel_resid_true = S.rr0 > 0.0 ? std::sqrt(S.tr / S.rr0) : 0.0;
      stats->seconds = ms * 1e-3;
    }
    if (hist)
      HIP_CHECK(hipMemcpy(hist, h->hist.p, (size_t(sp->max_iter) + 1) * sizeof(double),
                          hipMemcpyDeviceToHost));
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  if (st == MFMG_ERR_BREAKDOWN) return fail(st, "PCG breakdown: (r,z) or (p,Ap) not positive");
  if (st == MFMG_NOT_CONVERGED)
    g_err = "not converged: the residual (recursive or true) is above rtol after max_iter "
            "iterations or at the rounding floor";
  return st;
}

// Adjoint PCG: A^T lambda = g preconditioned by M^T (Algorithm 1 with the
// transposed operator and cycle), with the same restart rule as the forward
// solve.  On return Xf holds the true residual g - A^T lambda in device
// order (shifted to zero mean with the null space) and S->tr its norm.
template <class V>
static void pcg_adjoint_iterate(mfmg_hierarchy *h, const double *g, V *z,
                                const mfmg_solve_params *sp, bool null_space, hipStream_t s) {
  PcgArgs P = pcg_args(h);
  unsigned G = grid_reduce(h->co->dt->nlb);
  Reduce R(h, s);
  double na = std::max(1.0, h->n_active);
  double *x = h->x.p, *r = h->rA.p;
  const int *done = &h->S.p->done;
  const double *scale = &h->S.p->rscale;  // 1 in FP64
  __atomic_store_n(h->host_done, 0, __ATOMIC_RELEASE);  // the stream is idle here
  R.init<V>(g, r, (V *)nullptr, x, sp->rtol);
  if (null_space) R.shift_mean<V>(r, (V *)nullptr, na, 0, sp->rtol);
  Krylov<V> K(h, s);
  run_cycle_T(h, r, s, done, scale);
  K.rz(r, z, 1);
  K.pupdate(z, 1);
  double prev_tr = INFINITY;
  int left = sp->max_iter;
  for (;;) {
    for (int it = 0; it < left; ++it) {
      K.Ap(true);
      K.update(r, (V *)nullptr, int(null_space));
      if (null_space) R.shift_mean<V>(r, (V *)nullptr, na, 1, sp->rtol);
      run_cycle_T(h, r, s, done, scale);
      K.rz(r, z, 0);
      K.pupdate(z, 0);
      // stop flag of iteration it read after iteration it + 1 is queued (as in
      // the forward solve); kernels queued after the stop return at once
      HIP_CHECK(hipEventRecord(h->iter_ev[it & 1], s));
      if (it > 0) {
        HIP_CHECK(hipEventSynchronize(h->iter_ev[(it - 1) & 1]));
        if (__atomic_load_n(h->host_done, __ATOMIC_ACQUIRE)) break;
      }
    }
    K.finish_x();
    if (null_space) R.shift_mean<double>(x, (double *)nullptr, na, 3, 0.0);
    // true residual g - A^T lambda (into Xf) and its norm
    hipLaunchKernelGGL(k_full, dim3(G), dim3(kBlock), 0, s, P, (const double *)x, h->Xf.p, 0);
    hipLaunchKernelGGL(k_applyT, dim3(G), dim3(kBlock), 0, s, P, (const double *)h->Xf.p,
                       h->Ap.p);
    hipLaunchKernelGGL(k_resid_T, dim3(G), dim3(kBlock), 0, s, P, g, (const double *)h->Ap.p,
                       h->Xf.p);
    R.finish(G, kFinTrue);
    if (null_space) R.shift_mean<double>(h->Xf.p, (double *)nullptr, na, 2, 0.0);
    HIP_CHECK(hipMemcpyAsync(h->hostS, h->S.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    const Scalars S = *h->hostS;
    if (!restart_wanted(S, sp->max_iter, prev_tr)) break;
    prev_tr = S.tr;
    left = sp->max_iter - S.iters;
    hipLaunchKernelGGL(k_restart, dim3(G), dim3(kBlock), 0, s, P, (const double *)h->Xf.p, r);
    R.finish(G, kFinRestart);
    run_cycle_T(h, r, s, done, scale);
    K.rz(r, z, 1);
    K.pupdate(z, 1);
  }
  HIP_CHECK(hipGetLastError());
}

extern "C" mfmg_status mfmg_pcg_solve_adjoint(mfmg_hierarchy *h, const double *p,
                                              const double *dL_dp, double *lambda,
                                              double *dL_dbeta,
                                              const mfmg_solve_params *sp, void *stream,
                                              mfmg_solve_stats *stats) {
  if (!h || !p || !dL_dp || !lambda || !dL_dbeta || !sp)
    return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (!(sp->rtol >= 0.0) || sp->max_iter < 0) return fail(MFMG_ERR_INVALID_ARG, "bad params");
  if (sp->null_space < -1 || sp->null_space > 1)
    return fail(MFMG_ERR_INVALID_ARG, "null_space must be -1, 0 or 1");
  bool ns = sp->null_space == 1 || (sp->null_space == -1 && !h->co->has_dirichlet);
  if (sp->warm_start) return fail(MFMG_ERR_INVALID_ARG, "the adjoint solve starts from zero");
  hipStream_t s = (hipStream_t)stream;
  const mfmg_octree &T = *h->co->tree;
  const DeviceTopology &D = *h->co->dt;
  mfmg_status st = MFMG_OK;
  try {
    if (h->hist.n < size_t(sp->max_iter) + 2) {
      h->drop_graphs();  // they hold the old history pointer
      h->hist.alloc(std::max<size_t>(size_t(sp->max_iter) + 2, 1024));
    }
    if (!ns && !h->co->has_dirichlet && incompatible_rhs(h, dL_dp, s))
      return fail(MFMG_ERR_INCOMPATIBLE_RHS,
                  "no Dirichlet face and the null-space shift is off, but dL/dp does not "
                  "sum to zero over the active cells");
    if (!h->rA.p) h->rA.alloc(size_t(D.nlb) * 64);
    ensure_face_list(h, s);
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    HIP_CHECK(hipEventRecord(e0, s));
    if (h->prm.precision == MFMG_MIXED) {
      alloc_transpose(h, h->T32);
      pcg_adjoint_iterate<float>(h, dL_dp, h->T32[1].p, sp, ns, s);
    } else {
      alloc_transpose(h, h->T64);
      pcg_adjoint_iterate<double>(h, dL_dp, h->T64[1].p, sp, ns, s);
    }
    PcgArgs P = pcg_args(h);
    unsigned G = grid_for(D.nlb);
    hipLaunchKernelGGL(k_to_canonical<double>, dim3(G), dim3(kBlock), 0, s, P,
                       (const double *)h->x.p, lambda);
    GradArgs A;
    A.owner = h->f_owner.p;
    A.other = h->f_other.p;
    A.dir = h->f_dir.p;
    A.kind = h->f_kind.p;
    A.level = h->leaf_level.p;
    A.act = h->canon_act.p;
    A.lam = lambda;
    A.p = p;
    for (int d = 0; d < 6; ++d) A.bc[d] = h->co->bc.bc[d];
    A.theta = h->co->bc.theta;
    A.n_faces = T.n_faces;
    A.g = dL_dbeta;
    hipLaunchKernelGGL(k_face_gradient, dim3(grid_elems(T.n_faces, 256)), dim3(256), 0, s, A);
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipMemcpyAsync(h->hostS, h->S.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const Scalars &S = *h->hostS;
    st = solve_status(S);
    if (stats) {
      stats->iters = S.iters;
      stats->status = st;
      stats->rel_resid_recur = S.rr0 > 0.0 ? std::sqrt(S.rr / S.rr0) : 0.0;
      stats->rel_resid_true = S.rr0 > 0.0 ? std::sqrt(S.tr / S.rr0) : 0.0;
      stats->seconds = ms * 1e-3;
    }
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  if (st == MFMG_ERR_BREAKDOWN) return fail(st, "PCG breakdown: (r,z) or (p,Ap) not positive");
  if (st == MFMG_NOT_CONVERGED)
    g_err = "not converged: the residual (recursive or true) is above rtol after max_iter "
            "iterations or at the rounding floor";
  return st;
}

// --------------------------------------------------------------------------
// measurement
// --------------------------------------------------------------------------
namespace {

// Algorithmic bytes of one half-sweep over the bricks of level l.
double smooth_bytes(const mfmg_hierarchy *h, int l) {
  const DeviceTopology &D = *h->co->dt;
  bool mixed = h->prm.precision == MFMG_MIXED;
  double V = mixed ? 4.0 : 8.0;
  double CL = mixed ? 4.0 : 8.0, CI = mixed ? 2.0 : 8.0;
  double n_in = double(D.range[l].n_inner) * 64, n_leaf = double(D.range[l].n_leaf) * 64;
  auto per = [&](double C) { return V + 0.5 * V + 0.5 * C + 3.0 * C + 0.5 * V; };
  return n_leaf * per(CL) + n_in * per(CI);
}

// Algorithmic bytes of one whole cycle (all kernels of all levels).
double cycle_bytes(const mfmg_hierarchy *h) {
  const DeviceTopology &D = *h->co->dt;
  const mfmg_mg_params &p = h->prm;
  bool mixed = p.precision == MFMG_MIXED;
  double V = mixed ? 4.0 : 8.0;
  double CL = mixed ? 4.0 : 8.0, CI = mixed ? 2.0 : 8.0;
  double total = double(h->co->dt->nlb) * 64 * V;  // zero the leaf iterate
  // visits of each level per cycle: mu^(L - l)
  for (int l = h->L; l >= h->lc; --l) {
    double visits = std::pow(double(p.mu), double(h->L - l));
    double n_in = double(D.range[l].n_inner) * 64, n_leaf = double(D.range[l].n_leaf) * 64;
    double n_all = n_in + n_leaf;
    double cells_coef = n_leaf * 4.0 * CL + n_in * 4.0 * CI;  // 4 coefficients
    if (l == h->lc) {
      total += visits * 2.0 * p.nu_coarse * smooth_bytes(h, l);
      continue;
    }
    double lvl = 2.0 * (p.nu_pre + p.nu_post) * smooth_bytes(h, l);
    lvl += n_all * (2.0 * V + 3.0 * V / 8.0) + cells_coef;  // residual + restriction
    double c_in = double(D.range[l - 1].n_inner) * 64;        // FAS right-hand side
    double c_coef = c_in * 4.0 * CI;
    // (folded into the first half-sweep of level l - 1: only its store of b)
    bool fold = l - 1 > h->lc && h->fold_fas[size_t(l - 1)] && p.nu_pre > 0 &&
                !(l - 1 == h->lc + 1 && h->fuse_bottom);
    lvl += fold ? c_in * V : c_in * 3.0 * V + c_coef;
    // prolongation: the parent values, plus the level's iterate unless the
    // post-smoothing takes the prolongation with it
    bool fused = h->fuse_prolong && p.nu_post > 0;
    lvl += n_all * ((fused ? 0.0 : 2.0 * V) + 2.0 * V / 8.0);
    total += visits * lvl;
  }
  return total;
}

}  // namespace

constexpr size_t kCopyBytes = size_t(1) << 30;

extern "C" mfmg_status mfmg_profile(mfmg_hierarchy *h, int what, int level, int reps,
                                    void *stream, double *ms_per_launch,
                                    double *bytes_per_launch) {
  if (!h || !ms_per_launch || reps < 1) return fail(MFMG_ERR_INVALID_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  if (what == MFMG_PROFILE_SMOOTH && (level < h->lc || level > h->L))
    return fail(MFMG_ERR_INVALID_ARG, "level out of range");
  if (what < MFMG_PROFILE_SMOOTH || what > MFMG_PROFILE_COPY)
    return fail(MFMG_ERR_INVALID_ARG, "unknown profile step");
  try {
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    bool mixed = h->prm.precision == MFMG_MIXED;
    DevBuf<char> copy_src, copy_dst;  // 1 GiB each, only for the copy
    if (what == MFMG_PROFILE_COPY) {
      copy_src.alloc(kCopyBytes);
      copy_dst.alloc(kCopyBytes);
      HIP_CHECK(hipMemsetAsync(copy_src.p, 1, kCopyBytes, s));
    }
    auto launch = [&]() {
      if (what == MFMG_PROFILE_SMOOTH) {
        if (mixed) {
          Cycle<float, float, __half> c{h, h->coef32.p, h->coef16.p, h->pf32.p,
                                        h->U32.p, h->B32.p, h->S32.p, nullptr, s};
          c.half_sweep(level, c.args(level, false), 0);
        } else {
          Cycle<double, double, double> c{h, h->coef64.p,
                                          h->coef64.p + int64_t(h->co->dt->nlb) * 256,
                                          h->pf64.p, h->U64.p, h->B64.p, h->S64.p,
                                          nullptr, s};
          c.half_sweep(level, c.args(level, false), 0);
        }
      } else if (what == MFMG_PROFILE_CYCLE) {
        run_cycle(h, s, nullptr);
      } else {
        int64_t n16 = int64_t(kCopyBytes / 16);
        hipLaunchKernelGGL(k_stream_copy, dim3(grid_elems(n16, 1024)), dim3(256), 0, s,
                           (const f32x4 *)copy_src.p, (f32x4 *)copy_dst.p, n16);
      }
    };
    launch();  // warm
    HIP_CHECK(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) launch();
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = double(ms) / reps;
    if (bytes_per_launch)
      *bytes_per_launch = what == MFMG_PROFILE_SMOOTH ? smooth_bytes(h, level)
                          : what == MFMG_PROFILE_CYCLE ? cycle_bytes(h)
                                                       : 2.0 * double(kCopyBytes);
  } catch (const HipError &e) {
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return MFMG_OK;
}

// --------------------------------------------------------------------------
// projection of a face velocity field
// --------------------------------------------------------------------------
extern "C" mfmg_status mfmg_divergence(mfmg_hierarchy *h, const double *face_beta,
                                       const double *face_u, double *div, void *stream) {
  if (!h || !face_beta || !face_u || !div) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  try {
    const DeviceTopology &D = *h->co->dt;
    DivArgs A;
    A.T = make_topo(D, h->meta.p);
    A.fbase = D.fbase.p;
    A.fmask = D.fmask.p;
    A.canon = D.canon.p;
    A.beta = face_beta;
    A.u = face_u;
    A.div = div;
    if (D.nlb) hipLaunchKernelGGL(k_divergence, dim3(grid_for(D.nlb)), dim3(kBlock), 0, s, A);
    HIP_CHECK(hipGetLastError());
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_project_velocity(mfmg_hierarchy *h, const double *face_beta,
                                             const double *p, double *face_u, void *stream) {
  if (!h || !face_beta || !p || !face_u) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  try {
    ensure_face_list(h, s);
    FluxArgs A;
    A.owner = h->f_owner.p;
    A.other = h->f_other.p;
    A.dir = h->f_dir.p;
    A.kind = h->f_kind.p;
    A.level = h->leaf_level.p;
    A.act = h->canon_act.p;
    A.beta = face_beta;
    A.p = p;
    for (int d = 0; d < 6; ++d) A.bc[d] = h->co->bc.bc[d];
    A.theta = h->co->bc.theta;
    A.n_faces = h->co->tree->n_faces;
    A.u = face_u;
    if (A.n_faces)
      hipLaunchKernelGGL(k_project_velocity, dim3(grid_elems(A.n_faces, 256)), dim3(256), 0, s,
                         A);
    HIP_CHECK(hipGetLastError());
  } catch (const HipError &e) {
    return hip_fail(e);
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_divergence_rms(mfmg_hierarchy *h, const double *div, double *rms,
                                           void *stream) {
  if (!h || !div || !rms) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  try {
    Reduce R(h, s);
    const double *dev_sum = &h->S.p->sum;
    double part[2];
    for (int what = 0; what < 2; ++what) {
      hipLaunchKernelGGL(k_div_rms_part, dim3(R.G), dim3(kBlock), 0, s, R.P, div, what);
      R.finish(R.G, kFinSum);
      HIP_CHECK(hipMemcpyAsync(&part[what], dev_sum, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_CHECK(hipStreamSynchronize(s));
    *rms = part[1] > 0.0 ? std::sqrt(part[0] / part[1]) : 0.0;
  } catch (const HipError &e) {
    return hip_fail(e);
  }
  return MFMG_OK;
}

// --------------------------------------------------------------------------
// allocation-free form of mfmg_divergence_rms (callers that cannot allocate)
// --------------------------------------------------------------------------
namespace {

// The partial sums of the two reductions (sum V (div/V)^2 and sum V), one
// slot per workgroup of the reduction grid (at most kMaxReduceBlocks each),
// in a fixed device array: 32 KiB that every device the library runs on
// holds until the process ends.  Every slot a call reads is written by the
// same call, so nothing needs clearing; calls that overlap on one device
// race on it.
constexpr int64_t kNoAllocSlots = 2 * kMaxReduceBlocks;
__device__ __align__(256) double scratch[kNoAllocSlots];

// Device address of `scratch` per device ordinal, looked up once per device
// with that device current (in host code the array's name is only a
// host-side stand-in).
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_dev;

hipError_t scratch_address(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (size_t(dev) >= g_scratch_dev.size()) g_scratch_dev.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_dev[size_t(dev)]) {
    double *ptr = nullptr;
    e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[size_t(dev)] = ptr;
  }
  *out = g_scratch_dev[size_t(dev)];
  return hipSuccess;
}

// rms = sqrt(a / b) from the n partials of each sum (a at parts, b at
// parts + kMaxReduceBlocks), added in the order k_finish adds them.
__global__ void __launch_bounds__(1024) k_rms_finish(const double *parts, int64_t n,
                                                     double *rms) {
  __shared__ double red[2][16];
  double s[2];
  for (int k = 0; k < 2; ++k) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v += parts[k * kMaxReduceBlocks + i];
    s[k] = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = s[k];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[2] = {0.0, 0.0};
  for (int k = 0; k < 2; ++k)
    for (unsigned w = 0; w < blockDim.x / 64; ++w) tot[k] += red[k][w];
  rms[0] = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : 0.0;
}

}  // namespace

extern "C" mfmg_status mfmg_divergence_rms_noalloc(mfmg_hierarchy *h, const double *div,
                                                   double *rms, void *stream) {
  if (!h || !div || !rms) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  double *parts = nullptr;
  hipError_t e = scratch_address(&parts);
  if (e != hipSuccess)
    return fail(MFMG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  PcgArgs P = pcg_args(h);
  unsigned G = grid_reduce(h->co->dt->nlb);
  if (int64_t(G) > kMaxReduceBlocks)
    return fail(MFMG_ERR_INVALID_ARG, "reduction grid larger than the fixed partial-sum array");
  for (int what = 0; what < 2; ++what) {
    P.partials = parts + what * kMaxReduceBlocks;
    hipLaunchKernelGGL(k_div_rms_part, dim3(G), dim3(kBlock), 0, s, P, div, what);
  }
  hipLaunchKernelGGL(k_rms_finish, dim3(1), dim3(1024), 0, s, (const double *)parts,
                     int64_t(G), rms);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(MFMG_ERR_HIP, hipGetErrorString(e));
  return MFMG_OK;
}
