// C ABI and host driver of the matrix-free octree multigrid PCG solver.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mfmg.h"
#include "kernels.hpp"
#include "topology.hpp"

using namespace mfmg;

// --------------------------------------------------------------------------
// errors
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
    if (!v.empty()) HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T),
                                             hipMemcpyHostToDevice, s));
  }
};

inline unsigned grid_for(int64_t bricks) {
  int64_t g = (bricks + kWavesPerBlock - 1) / kWavesPerBlock;
  return unsigned(g > 0 ? g : 1);
}
inline unsigned grid_elems(int64_t n, int t) { return unsigned((n + t - 1) / t); }

// grid of the reduction kernels (grid-stride over leaf bricks)
inline unsigned grid_reduce(int64_t bricks) {
  int64_t g = (bricks + kWavesPerBlock - 1) / kWavesPerBlock;
  if (g > 2048) g = 2048;
  return unsigned(g > 0 ? g : 1);
}
}  // namespace

// --------------------------------------------------------------------------
// objects
// --------------------------------------------------------------------------
struct mfmg_octree {
  Topology topo;
};

struct DeviceTopology {
  DevBuf<int32_t> nbr, coord, parent, child, tplus;
  DevBuf<int8_t> level;
  DevBuf<int64_t> fbase;
  DevBuf<uint8_t> fmask;
  DevBuf<uint64_t> act;
  DevBuf<uint32_t> flags;              // per-brick face flags
  DevBuf<int32_t> lists;               // concatenated per-level lists
  std::vector<int64_t> all_off, all_n; // per level: offset/count of all bricks
  std::vector<int64_t> in_off, in_n;   // per level: inner bricks
  DevBuf<int32_t> leaf_list;           // 0..nlb-1 (identity)
};

struct mfmg_coeffs {
  const mfmg_octree *tree = nullptr;
  std::unique_ptr<DeviceTopology> dt;
  DevBuf<double> coef;  // nlb * 256, FP64 leaf coefficients
  DevBuf<double> tc;    // n_tplus * 48
  mfmg_bc bc{};
  int has_dirichlet = 0;
};

struct mfmg_hierarchy {
  const mfmg_coeffs *co = nullptr;
  mfmg_mg_params prm{};
  int L = 0, lc = 0;
  DevBuf<double> coef64;  // nb * 256 (leaf part = assembled, inner = Algorithm 3)
  DevBuf<float> coef32;   // nlb * 256 (mixed)
  DevBuf<__half> coef16;  // (nb - nlb) * 256 (mixed)
  DevBuf<float> tc32;     // mixed
  DevBuf<uint64_t> act;   // nb
  // work vectors
  DevBuf<double> U64, B64, S64;  // FP64 cycle: nb*64, nb*64, (nb-nlb)*64
  DevBuf<float> U32, B32, S32;   // mixed cycle
  DevBuf<double> r, pd, Ap;      // PCG (r aliases B64 in FP64 mode); pd is full-size
  DevBuf<double> Xf;             // full-size scratch for operator applications
  DevBuf<double> partials;
  DevBuf<Scalars> S;
  DevBuf<double> hist;
  Scalars *hostS = nullptr;      // pinned
  ~mfmg_hierarchy() {
    if (hostS) (void)hipHostFree(hostS);
  }
};

extern "C" const char *mfmg_last_error(void) { return g_err.c_str(); }

// --------------------------------------------------------------------------
// octree
// --------------------------------------------------------------------------
extern "C" mfmg_status mfmg_build_octree(const mfmg_refine_spec *spec, mfmg_octree **out) {
  if (!spec || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (spec->n_prims < 0 || (spec->n_prims > 0 && !spec->prims))
    return fail(MFMG_ERR_INVALID_ARG, "bad primitive list");
  std::vector<Prim> prims(spec->n_prims);
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
  *out = t.release();
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_octree_info(const mfmg_octree *t, int64_t *n_leaves,
                                        int64_t *n_faces, int64_t *n_leaf_bricks) {
  if (!t) return fail(MFMG_ERR_INVALID_ARG, "NULL octree");
  if (n_leaves) *n_leaves = t->topo.n_leaves();
  if (n_faces) *n_faces = t->topo.n_faces;
  if (n_leaf_bricks) *n_leaf_bricks = t->topo.n_leaf_bricks;
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_octree_leaves(const mfmg_octree *t, uint8_t *level, int32_t *ijk) {
  if (!t || !level || !ijk) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
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
static void upload_topology(const Topology &T, DeviceTopology &D, hipStream_t s) {
  D.nbr.upload(T.nbr, s);
  D.coord.upload(T.coord, s);
  D.parent.upload(T.parent, s);
  D.child.upload(T.child, s);
  D.tplus.upload(T.tplus, s);
  D.level.upload(T.level, s);
  D.fbase.upload(T.cell_fbase, s);
  D.fmask.upload(T.cell_fmask, s);
  std::vector<uint32_t> flags(T.n_bricks, 0u);
  for (int64_t b = 0; b < T.n_bricks; ++b)
    for (int d = 0; d < 6; ++d) {
      int32_t n = T.nbr[6 * b + d];
      if (n <= kCoarseBase) flags[b] |= 1u << d;
      else if (n == kWall) flags[b] |= 1u << (16 + d);
      else if (n >= T.n_leaf_bricks) flags[b] |= 1u << (8 + d);
    }
  D.flags.upload(flags, s);
  std::vector<int32_t> lists;
  int L = T.max_level;
  D.all_off.assign(L + 1, 0);
  D.all_n.assign(L + 1, 0);
  D.in_off.assign(L + 1, 0);
  D.in_n.assign(L + 1, 0);
  for (int l = kMinLevel; l <= L; ++l) {
    D.all_off[l] = int64_t(lists.size());
    D.all_n[l] = int64_t(T.level_bricks[l].size());
    lists.insert(lists.end(), T.level_bricks[l].begin(), T.level_bricks[l].end());
    D.in_off[l] = int64_t(lists.size());
    D.in_n[l] = int64_t(T.level_inner[l].size());
    lists.insert(lists.end(), T.level_inner[l].begin(), T.level_inner[l].end());
  }
  std::vector<int32_t> leaf(T.n_leaf_bricks);
  for (int64_t i = 0; i < T.n_leaf_bricks; ++i) leaf[i] = int32_t(i);
  D.lists.upload(lists, s);
  D.leaf_list.upload(leaf, s);
  D.act.alloc(T.n_bricks);
  HIP_CHECK(hipStreamSynchronize(s));
}

static Topo make_topo(const Topology &T, const DeviceTopology &D, const uint64_t *act) {
  Topo t;
  t.nlb = T.n_leaf_bricks;
  t.nb = T.n_bricks;
  t.nbr = D.nbr.p;
  t.coord = D.coord.p;
  t.parent = D.parent.p;
  t.child = D.child.p;
  t.tplus = D.tplus.p;
  t.act = act;
  t.flags = D.flags.p;
  return t;
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
  const Topology &T = tree->topo;
  try {
    std::unique_ptr<mfmg_coeffs> co(new mfmg_coeffs());
    co->tree = tree;
    co->bc = *bc;
    for (int d = 0; d < 6; ++d) co->has_dirichlet |= bc->bc[d] == MFMG_DIRICHLET;
    co->dt.reset(new DeviceTopology());
    upload_topology(T, *co->dt, s);
    co->coef.alloc(size_t(T.n_leaf_bricks) * 256);
    co->tc.alloc(size_t(T.n_tplus) * 48 + 1);
    AssembleArgs A;
    A.T = make_topo(T, *co->dt, co->dt->act.p);
    A.fbase = co->dt->fbase.p;
    A.fmask = co->dt->fmask.p;
    A.beta = face_beta;
    A.blevel = co->dt->level.p;
    for (int d = 0; d < 6; ++d) A.bc[d] = bc->bc[d];
    A.theta = bc->theta;
    A.coef = co->coef.p;
    A.tc = co->tc.p;
    hipLaunchKernelGGL(k_assemble, dim3(grid_for(T.n_leaf_bricks)), dim3(kBlock), 0, s, A);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
    *out = co.release();
  } catch (const HipError &e) {
    return fail(e.e == hipErrorOutOfMemory ? MFMG_ERR_OOM : MFMG_ERR_HIP,
                std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_coeffs_leaf(const mfmg_coeffs *co, double *out, void *stream) {
  if (!co || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Topology &T = co->tree->topo;
  int64_t N = T.n_leaves();
  try {
    for (int comp = 0; comp < 4; ++comp)
      HIP_CHECK(hipMemcpy2DAsync(out + comp * N + 0, 64 * sizeof(double),
                                 co->coef.p + comp * 64, 256 * sizeof(double),
                                 64 * sizeof(double), size_t(T.n_leaf_bricks),
                                 hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return MFMG_OK;
}

extern "C" void mfmg_destroy_coeffs(mfmg_coeffs *co) { delete co; }

// --------------------------------------------------------------------------
// hierarchy
// --------------------------------------------------------------------------
template <class V, class CL, class CI>
static LevelArgs<V, CL, CI> level_args(const mfmg_hierarchy *h, int l, bool inner_only,
                                       const CL *leafc, const CI *innerc, const CL *tc,
                                       V *U, V *B, V *Ust, V iscale, const int *done) {
  const Topology &T = h->co->tree->topo;
  const DeviceTopology &D = *h->co->dt;
  LevelArgs<V, CL, CI> A;
  A.T = make_topo(T, D, h->act.p);
  A.cf.leaf = leafc;
  A.cf.inner = innerc;
  A.cf.tc = tc;
  A.cf.nlb = T.n_leaf_bricks;
  A.cf.iscale = iscale;
  A.U = U;
  A.B = B;
  A.Ustar = Ust;
  if (inner_only) {
    A.list = D.lists.p + D.in_off[l];
    A.n = D.in_n[l];
  } else {
    A.list = D.lists.p + D.all_off[l];
    A.n = D.all_n[l];
  }
  A.done = done;
  return A;
}

extern "C" mfmg_status mfmg_build_hierarchy(const mfmg_coeffs *co, const mfmg_mg_params *prm,
                                            void *stream, mfmg_hierarchy **out) {
  if (!co || !prm || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  const Topology &T = co->tree->topo;
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
  hipStream_t s = (hipStream_t)stream;
  try {
    std::unique_ptr<mfmg_hierarchy> h(new mfmg_hierarchy());
    h->co = co;
    h->prm = *prm;
    h->lc = prm->coarsest_level;
    h->L = 0;
    for (int l = kMinLevel; l <= T.max_level; ++l)
      if (!co->dt->all_n.empty() && co->dt->all_n[l] > 0) h->L = l;
    const DeviceTopology &D = *co->dt;
    int64_t nb = T.n_bricks, nlb = T.n_leaf_bricks, N = T.n_leaves();
    h->coef64.alloc(size_t(nb) * 256);
    h->act.alloc(size_t(nb));
    HIP_CHECK(hipMemcpyAsync(h->coef64.p, co->coef.p, size_t(nlb) * 256 * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_active_mask, dim3(grid_for(nlb)), dim3(kBlock), 0, s,
                       (const double *)h->coef64.p, (const int32_t *)nullptr, nlb, h->act.p);
    Topo topo = make_topo(T, D, h->act.p);
    for (int l = T.max_level - 1; l >= kMinLevel; --l) {
      int64_t n = D.in_n[l];
      if (n == 0) continue;
      const int32_t *list = D.lists.p + D.in_off[l];
      hipLaunchKernelGGL(k_coarsen, dim3(grid_for(n)), dim3(kBlock), 0, s, list, n, topo,
                         h->coef64.p, prm->alpha);
      hipLaunchKernelGGL(k_active_mask, dim3(grid_for(n)), dim3(kBlock), 0, s,
                         (const double *)h->coef64.p, list, n, h->act.p);
    }
    HIP_CHECK(hipGetLastError());
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
                           (const double *)h->coef64.p, (const int8_t *)D.level.p, nlb, nb,
                           h->coef16.p);
      h->U32.alloc(size_t(nb) * 64);
      h->B32.alloc(size_t(nb) * 64);
      h->S32.alloc(size_t(nb - nlb) * 64 + 1);
      h->r.alloc(size_t(N));
    } else {
      h->U64.alloc(size_t(nb) * 64);
      h->B64.alloc(size_t(nb) * 64);
      h->S64.alloc(size_t(nb - nlb) * 64 + 1);
    }
    h->pd.alloc(size_t(nb) * 64);
    h->Xf.alloc(size_t(nb) * 64);
    h->Ap.alloc(size_t(N));
    h->partials.alloc(4096);
    h->S.alloc(1);
    HIP_CHECK(hipMemsetAsync(h->S.p, 0, sizeof(Scalars), s));
    HIP_CHECK(hipHostMalloc(&h->hostS, sizeof(Scalars), hipHostMallocDefault));
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
    *out = h.release();
  } catch (const HipError &e) {
    return fail(e.e == hipErrorOutOfMemory ? MFMG_ERR_OOM : MFMG_ERR_HIP,
                std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc &) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_hierarchy_level_bricks(const mfmg_hierarchy *h, int level,
                                                   int64_t *count, int32_t *coords,
                                                   uint8_t *is_leaf) {
  if (!h || !count) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  const Topology &T = h->co->tree->topo;
  if (level < kMinLevel || level > T.max_level) return fail(MFMG_ERR_INVALID_ARG, "bad level");
  const auto &lst = T.level_bricks[level];
  *count = int64_t(lst.size());
  for (size_t i = 0; i < lst.size(); ++i) {
    int32_t b = lst[i];
    if (coords)
      for (int a = 0; a < 3; ++a) coords[3 * i + a] = T.coord[3 * int64_t(b) + a];
    if (is_leaf) is_leaf[i] = b < T.n_leaf_bricks;
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_hierarchy_level_coeffs(const mfmg_hierarchy *h, int level,
                                                   double *out, void *stream) {
  if (!h || !out) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  const Topology &T = h->co->tree->topo;
  if (level < kMinLevel || level > T.max_level) return fail(MFMG_ERR_INVALID_ARG, "bad level");
  hipStream_t s = (hipStream_t)stream;
  try {
    const auto &lst = T.level_bricks[level];
    for (size_t i = 0; i < lst.size(); ++i)
      HIP_CHECK(hipMemcpyAsync(out + i * 256, h->coef64.p + int64_t(lst[i]) * 256,
                               256 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
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
  const CL *tc;
  V *U, *B, *Ust;
  const int *done;
  hipStream_t s;

  V iscale(int l) const {
    return std::is_same<CI, __half>::value ? V(std::ldexp(1.0, -l)) : V(1);
  }
  LevelArgs<V, CL, CI> args(int l, bool inner_only) const {
    return level_args<V, CL, CI>(h, l, inner_only, leafc, innerc, tc, U, B, Ust, iscale(l),
                                 done);
  }

  void smooth(int l, int first, int nu) const {
    auto A = args(l, false);
    if (A.n == 0) return;
    for (int it = 0; it < nu; ++it)
      for (int c = 0; c < 2; ++c)
        hipLaunchKernelGGL((k_smooth<V, CL, CI>), dim3(grid_for(A.n)), dim3(kBlock), 0, s, A,
                           c == 0 ? first : 1 - first);
  }

  void fas(int l) const {
    const mfmg_mg_params &p = h->prm;
    if (l == h->lc) {
      auto A = args(l, false);
      int threads = int(std::min<int64_t>(16, A.n)) * kWave;
      hipLaunchKernelGGL((k_coarsest<V, CL, CI>), dim3(1), dim3(threads), 0, s, A,
                         p.nu_coarse);
      return;
    }
    smooth(l, 0, p.nu_pre);
    auto A = args(l, false);
    V scale = V(p.beta_mg / p.alpha);
    hipLaunchKernelGGL((k_restrict<V, CL, CI>), dim3(grid_for(A.n)), dim3(kBlock), 0, s, A,
                       scale);
    auto C = args(l - 1, true);
    if (C.n)
      hipLaunchKernelGGL((k_fas_rhs<V, CL, CI>), dim3(grid_for(C.n)), dim3(kBlock), 0, s, C);
    for (int k = 0; k < p.mu; ++k) fas(l - 1);
    hipLaunchKernelGGL((k_prolong<V, CL, CI>), dim3(grid_for(A.n)), dim3(kBlock), 0, s, A);
    smooth(l, 1, p.nu_post);
  }

  void run() const {
    const Topology &T = h->co->tree->topo;
    int64_t N = T.n_leaves();
    hipLaunchKernelGGL((k_fill<V>), dim3(grid_elems(N, 256)), dim3(256), 0, s, U, N, V(0));
    fas(h->L);
  }
};

void run_cycle(const mfmg_hierarchy *h, hipStream_t s, const int *done) {
  if (h->prm.precision == MFMG_MIXED) {
    Cycle<float, float, __half> c{h, h->coef32.p, h->coef16.p, h->tc32.p,
                                  h->U32.p, h->B32.p, h->S32.p, done, s};
    c.run();
  } else {
    Cycle<double, double, double> c{h, h->coef64.p, h->coef64.p + 0, h->co->tc.p,
                                    h->U64.p, h->B64.p, h->S64.p, done, s};
    // FP64 inner coefficients live in the same array, after the leaf bricks
    c.innerc = h->coef64.p + h->co->tree->topo.n_leaf_bricks * 256;
    c.run();
  }
}

}  // namespace

// --------------------------------------------------------------------------
// PCG kernels
// --------------------------------------------------------------------------
namespace mfmg {

struct PcgArgs {
  Topo T;
  const double *C;   // FP64 coefficients, leaf bricks first
  const double *TC;  // FP64 plus-side T coefficients
  Scalars *S;
  double *partials;
  double *hist;
};

__device__ __forceinline__ void leaf_cell(const PcgArgs &P, uint32_t b, int m, double &c,
                                          double &k0, double &k1, double &k2) {
  const double *cf = P.C + b * 256u;
  c = cf[m];
  k0 = cf[64 + m];
  k1 = cf[128 + m];
  k2 = cf[192 + m];
}

#define BRICK_LOOP(P)                                                               \
  int m = threadIdx.x & (kWave - 1);                                                \
  for (uint32_t b = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;              \
       b < uint32_t((P).T.nlb); b += gridDim.x * kWavesPerBlock)

// r = rhs on active cells, x = 0, ||r||^2
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_init(PcgArgs P, const double *rhs, double *r,
                                                     V *r_low, double *x, double rtol) {
  double part = 0.0;
  BRICK_LOOP(P) {
    bool act = (P.T.act[b] >> m) & 1ull;
    double v = act ? rhs[b * 64u + m] : 0.0;
    r[b * 64u + m] = v;
    if (r_low) r_low[b * 64u + m] = V(v);
    x[b * 64u + m] = 0.0;
    part += v * v;
  }
  Scalars *S = P.S;
  block_reduce_finish(part, P.partials, &S->ticket[0], [&](double tot) {
    S->rr0 = tot;
    S->rr = tot;
    S->tol2 = rtol * rtol * tot;
    S->iters = 0;
    S->status = 0;
    S->done = (tot == 0.0) || !(tot < INFINITY);
    if (!(tot < INFINITY)) S->status = -5;
    S->rz = 0.0;
    P.hist[0] = tot > 0.0 ? 1.0 : 0.0;
  });
}

// (r, z) and beta = (r, z) / (r, z)_old (beta = 0 on the first call)
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_rz(PcgArgs P, const double *r, const V *z,
                                                   int first) {
  if (P.S->done) return;
  double part = 0.0;
  BRICK_LOOP(P) { part += r[b * 64u + m] * double(z[b * 64u + m]); }
  Scalars *S = P.S;
  block_reduce_finish(part, P.partials, &S->ticket[1], [&](double tot) {
    if (!(tot > 0.0) || !(tot < INFINITY)) {
      S->status = -5;
      S->done = 1;
      return;
    }
    S->beta = first ? 0.0 : tot / S->rz;
    S->rz = tot;
  });
}

// p = z + beta p (p = z on the first call)
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_p(PcgArgs P, const V *z, double *p, int first) {
  if (P.S->done) return;
  double beta = P.S->beta;
  BRICK_LOOP(P) {
    uint64_t amask = P.T.act[b];
    bool act = (amask >> m) & 1ull;
    double v = double(z[b * 64u + m]);
    if (!first) v = v + beta * p[b * 64u + m];
    v = act ? v : 0.0;
    p[b * 64u + m] = v;
    if (P.T.flags[b] & kFlagT) average_up(P.T, p, b, m, v, amask);
  }
}

// Ap = A p (composite operator) and alpha = (r, z) / (p, Ap)
__global__ void __launch_bounds__(kBlock) k_pcg_Ap(PcgArgs P, const double *p, double *Ap) {
  if (P.S->done) return;
  double part = 0.0;
  BRICK_LOOP(P) {
    double c, k0, k1, k2;
    leaf_cell(P, b, m, c, k0, k1, k2);
    double u = p[b * 64u + m];
    int32_t nb6[6];
    load_nbr(P.T, b, nb6);
    double y = composite_Au(P.T, P.C, P.TC, p, b, m, u, c, k0, k1, k2, P.T.act[b],
                            P.T.flags[b], nb6);
    Ap[b * 64u + m] = y;
    part += u * y;
  }
  Scalars *S = P.S;
  block_reduce_finish(part, P.partials, &S->ticket[2], [&](double tot) {
    S->pAp = tot;
    if (!(tot > 0.0) || !(tot < INFINITY)) {
      S->status = -5;
      S->done = 1;
      return;
    }
    S->alpha = S->rz / tot;
  });
}

// x += alpha p, r -= alpha Ap, ||r||^2, stop test
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_update(PcgArgs P, double *x, double *r,
                                                       V *r_low, const double *p,
                                                       const double *Ap) {
  if (P.S->done) return;
  double alpha = P.S->alpha;
  double part = 0.0;
  BRICK_LOOP(P) {
    uint32_t i = b * 64u + m;
    x[i] = x[i] + alpha * p[i];
    double v = r[i] - alpha * Ap[i];
    r[i] = v;
    if (r_low) r_low[i] = V(v);
    part += v * v;
  }
  Scalars *S = P.S;
  block_reduce_finish(part, P.partials, &S->ticket[3], [&](double tot) {
    S->rr = tot;
    S->iters += 1;
    P.hist[S->iters] = S->rr0 > 0.0 ? sqrt(tot / S->rr0) : 0.0;
    if (!(tot < INFINITY)) {
      S->status = -5;
      S->done = 1;
    } else if (tot <= S->tol2) {
      S->done = 1;
    }
  });
}

// copy a leaf vector into the leaf part of a full-size vector and write the
// parent means that the composite operator reads for inner neighbours
__global__ void __launch_bounds__(kBlock) k_full(PcgArgs P, const double *x, double *X) {
  BRICK_LOOP(P) {
    uint64_t amask = P.T.act[b];
    double v = ((amask >> m) & 1ull) ? x[b * 64u + m] : 0.0;
    X[b * 64u + m] = v;
    if (P.T.flags[b] & kFlagT) average_up(P.T, X, b, m, v, amask);
  }
}

// y = A X (X full-size, from k_full) or y = A^T x (x a leaf vector)
template <bool TRANS>
__global__ void __launch_bounds__(kBlock) k_apply(PcgArgs P, const double *x, double *y) {
  BRICK_LOOP(P) {
    double c, k0, k1, k2;
    leaf_cell(P, b, m, c, k0, k1, k2);
    int32_t nb6[6];
    load_nbr(P.T, b, nb6);
    if (TRANS)
      y[b * 64u + m] = composite_AuT(P.T, P.C, P.TC, x, b, m, x[b * 64u + m], c, k0, k1, k2,
                                    P.T.act[b], P.T.flags[b], nb6);
    else
      y[b * 64u + m] = composite_Au(P.T, P.C, P.TC, x, b, m, x[b * 64u + m], c, k0, k1, k2,
                                   P.T.act[b], P.T.flags[b], nb6);
  }
}

// ||rhs - A x||^2 over active cells
__global__ void __launch_bounds__(kBlock) k_true_resid(PcgArgs P, const double *rhs,
                                                       const double *x) {
  double part = 0.0;
  BRICK_LOOP(P) {
    double c, k0, k1, k2;
    leaf_cell(P, b, m, c, k0, k1, k2);
    int32_t nb6[6];
    load_nbr(P.T, b, nb6);
    double y = composite_Au(P.T, P.C, P.TC, x, b, m, x[b * 64u + m], c, k0, k1, k2,
                            P.T.act[b], P.T.flags[b], nb6);
    bool act = (P.T.act[b] >> m) & 1ull;
    double t = act ? rhs[b * 64u + m] - y : 0.0;
    part += t * t;
  }
  Scalars *S = P.S;
  block_reduce_finish(part, P.partials, &S->ticket[0], [&](double tot) { S->tr = tot; });
}

// copy a leaf vector into the low-precision right-hand side of the cycle
template <class V>
__global__ void k_to_low(const double *src, V *dst, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = V(src[i]);
}
template <class V>
__global__ void k_from_low(const V *src, double *dst, const uint64_t *act, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = ((act[i >> 6] >> (i & 63)) & 1ull) ? double(src[i]) : 0.0;
}

}  // namespace mfmg

static PcgArgs pcg_args(mfmg_hierarchy *h) {
  const Topology &T = h->co->tree->topo;
  PcgArgs P;
  P.T = make_topo(T, *h->co->dt, h->act.p);
  P.C = h->coef64.p;
  P.TC = h->co->tc.p;
  P.S = h->S.p;
  P.partials = h->partials.p;
  P.hist = h->hist.p;
  return P;
}

extern "C" mfmg_status mfmg_apply_operator(mfmg_hierarchy *h, const double *x, double *y,
                                           int transpose, void *stream) {
  if (!h || !x || !y) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Topology &T = h->co->tree->topo;
  try {
    PcgArgs P = pcg_args(h);
    if (transpose) {
      hipLaunchKernelGGL(k_apply<true>, dim3(grid_for(T.n_leaf_bricks)), dim3(kBlock), 0, s, P,
                         x, y);
    } else {
      hipLaunchKernelGGL(k_full, dim3(grid_for(T.n_leaf_bricks)), dim3(kBlock), 0, s, P, x,
                         h->Xf.p);
      hipLaunchKernelGGL(k_apply<false>, dim3(grid_for(T.n_leaf_bricks)), dim3(kBlock), 0, s,
                         P, (const double *)h->Xf.p, y);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return MFMG_OK;
}

extern "C" mfmg_status mfmg_apply_precond(mfmg_hierarchy *h, const double *r, double *z,
                                          int transpose, void *stream) {
  if (!h || !r || !z) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (transpose) return fail(MFMG_ERR_INVALID_ARG, "transposed cycle not available");
  hipStream_t s = (hipStream_t)stream;
  const Topology &T = h->co->tree->topo;
  int64_t N = T.n_leaves();
  try {
    if (h->prm.precision == MFMG_MIXED) {
      hipLaunchKernelGGL(k_to_low<float>, dim3(grid_elems(N, 256)), dim3(256), 0, s, r,
                         h->B32.p, N);
      run_cycle(h, s, nullptr);
      hipLaunchKernelGGL(k_from_low<float>, dim3(grid_elems(N, 256)), dim3(256), 0, s,
                         (const float *)h->U32.p, z, (const uint64_t *)h->act.p, N);
    } else {
      hipLaunchKernelGGL(k_to_low<double>, dim3(grid_elems(N, 256)), dim3(256), 0, s, r,
                         h->B64.p, N);
      run_cycle(h, s, nullptr);
      hipLaunchKernelGGL(k_from_low<double>, dim3(grid_elems(N, 256)), dim3(256), 0, s,
                         (const double *)h->U64.p, z, (const uint64_t *)h->act.p, N);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
  } catch (const HipError &e) {
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return MFMG_OK;
}

template <class V>
static void pcg_iterate(mfmg_hierarchy *h, const double *rhs, double *x, double *r, V *r_low,
                        V *z, const mfmg_solve_params *sp, hipStream_t s) {
  const Topology &T = h->co->tree->topo;
  PcgArgs P = pcg_args(h);
  unsigned G = grid_reduce(T.n_leaf_bricks);
  const int *done = &h->S.p->done;
  hipLaunchKernelGGL(k_pcg_init<V>, dim3(G), dim3(kBlock), 0, s, P, rhs, r, r_low, x,
                     sp->rtol);
  run_cycle(h, s, done);
  hipLaunchKernelGGL(k_pcg_rz<V>, dim3(G), dim3(kBlock), 0, s, P, (const double *)r,
                     (const V *)z, 1);
  hipLaunchKernelGGL(k_pcg_p<V>, dim3(G), dim3(kBlock), 0, s, P, (const V *)z, h->pd.p, 1);
  for (int it = 0; it < sp->max_iter; ++it) {
    hipLaunchKernelGGL(k_pcg_Ap, dim3(G), dim3(kBlock), 0, s, P, (const double *)h->pd.p,
                       h->Ap.p);
    hipLaunchKernelGGL(k_pcg_update<V>, dim3(G), dim3(kBlock), 0, s, P, x, r, r_low,
                       (const double *)h->pd.p, (const double *)h->Ap.p);
    run_cycle(h, s, done);
    hipLaunchKernelGGL(k_pcg_rz<V>, dim3(G), dim3(kBlock), 0, s, P, (const double *)r,
                       (const V *)z, 0);
    hipLaunchKernelGGL(k_pcg_p<V>, dim3(G), dim3(kBlock), 0, s, P, (const V *)z, h->pd.p, 0);
    HIP_CHECK(hipMemcpyAsync(h->hostS, h->S.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (h->hostS->done) break;
  }
  hipLaunchKernelGGL(k_full, dim3(grid_for(T.n_leaf_bricks)), dim3(kBlock), 0, s, P,
                     (const double *)x, h->Xf.p);
  hipLaunchKernelGGL(k_true_resid, dim3(G), dim3(kBlock), 0, s, P, rhs, (const double *)h->Xf.p);
  HIP_CHECK(hipGetLastError());
}

extern "C" mfmg_status mfmg_pcg_solve(mfmg_hierarchy *h, const double *rhs, double *p,
                                      const mfmg_solve_params *sp, void *stream,
                                      mfmg_solve_stats *stats, double *hist) {
  if (!h || !rhs || !p || !sp) return fail(MFMG_ERR_INVALID_ARG, "NULL argument");
  if (!(sp->rtol >= 0.0) || sp->max_iter < 0) return fail(MFMG_ERR_INVALID_ARG, "bad params");
  if (sp->null_space == 1 || (sp->null_space == -1 && !h->co->has_dirichlet))
    return fail(MFMG_ERR_INVALID_ARG, "null-space projection not available in this build");
  hipStream_t s = (hipStream_t)stream;
  mfmg_status st = MFMG_OK;
  try {
    h->hist.alloc(size_t(sp->max_iter) + 2);
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    HIP_CHECK(hipEventRecord(e0, s));
    if (h->prm.precision == MFMG_MIXED)
      pcg_iterate<float>(h, rhs, p, h->r.p, h->B32.p, h->U32.p, sp, s);
    else
      pcg_iterate<double>(h, rhs, p, h->B64.p, (double *)nullptr, h->U64.p, sp, s);
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipMemcpyAsync(h->hostS, h->S.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const Scalars &S = *h->hostS;
    if (S.status == -5)
      st = MFMG_ERR_BREAKDOWN;
    else if (S.rr0 > 0.0 && !(S.rr <= S.tol2))
      st = MFMG_NOT_CONVERGED;
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
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  if (st == MFMG_ERR_BREAKDOWN) return fail(st, "PCG breakdown: (r,z) or (p,Ap) not positive");
  if (st == MFMG_NOT_CONVERGED) g_err = "not converged within max_iter";
  return st;
}

extern "C" mfmg_status mfmg_pcg_solve_adjoint(mfmg_hierarchy *h, const double *p,
                                              const double *dL_dp, double *lambda,
                                              double *dL_dbeta,
                                              const mfmg_solve_params *sp, void *stream,
                                              mfmg_solve_stats *stats) {
  (void)h; (void)p; (void)dL_dp; (void)lambda; (void)dL_dbeta; (void)sp; (void)stream;
  (void)stats;
  return fail(MFMG_ERR_INVALID_ARG, "adjoint solve not available in this build");
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
  double n_in = double(D.in_n[l]) * 64, n_all = double(D.all_n[l]) * 64;
  double n_leaf = n_all - n_in;
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
  double total = double(h->co->tree->topo.n_leaves()) * V;  // zero the leaf iterate
  // visits of each level per cycle: mu^(L - l)
  for (int l = h->L; l >= h->lc; --l) {
    double visits = std::pow(double(p.mu), double(h->L - l));
    double n_in = double(D.in_n[l]) * 64, n_all = double(D.all_n[l]) * 64;
    double n_leaf = n_all - n_in;
    double cells_coef = n_leaf * 4.0 * CL + n_in * 4.0 * CI;  // 4 coefficients
    if (l == h->lc) {
      total += visits * 2.0 * p.nu_coarse * smooth_bytes(h, l);
      continue;
    }
    double lvl = 2.0 * (p.nu_pre + p.nu_post) * smooth_bytes(h, l);
    lvl += n_all * (2.0 * V + 3.0 * V / 8.0) + cells_coef;  // residual + restriction
    double c_in = double(D.in_n[l - 1]) * 64;                 // FAS right-hand side
    double c_coef = c_in * 4.0 * CI;
    lvl += c_in * 3.0 * V + c_coef;
    lvl += n_all * (2.0 * V + 2.0 * V / 8.0);                 // prolongation
    total += visits * lvl;
  }
  return total;
}

}  // namespace

extern "C" mfmg_status mfmg_profile(mfmg_hierarchy *h, int what, int level, int reps,
                                    void *stream, double *ms_per_launch,
                                    double *bytes_per_launch) {
  if (!h || !ms_per_launch || reps < 1) return fail(MFMG_ERR_INVALID_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const Topology &T = h->co->tree->topo;
  if (what == MFMG_PROFILE_SMOOTH && (level < h->lc || level > h->L))
    return fail(MFMG_ERR_INVALID_ARG, "level out of range");
  try {
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    bool mixed = h->prm.precision == MFMG_MIXED;
    auto launch = [&]() {
      if (what == MFMG_PROFILE_SMOOTH) {
        if (mixed) {
          Cycle<float, float, __half> c{h, h->coef32.p, h->coef16.p, h->tc32.p,
                                        h->U32.p, h->B32.p, h->S32.p, nullptr, s};
          auto A = c.args(level, false);
          hipLaunchKernelGGL((k_smooth<float, float, __half>), dim3(grid_for(A.n)),
                             dim3(kBlock), 0, s, A, 0);
        } else {
          Cycle<double, double, double> c{h, h->coef64.p,
                                          h->coef64.p + T.n_leaf_bricks * 256,
                                          h->co->tc.p, h->U64.p, h->B64.p, h->S64.p,
                                          nullptr, s};
          auto A = c.args(level, false);
          hipLaunchKernelGGL((k_smooth<double, double, double>), dim3(grid_for(A.n)),
                             dim3(kBlock), 0, s, A, 0);
        }
      } else {
        run_cycle(h, s, nullptr);
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
      *bytes_per_launch = what == MFMG_PROFILE_SMOOTH ? smooth_bytes(h, level) : cycle_bytes(h);
  } catch (const HipError &e) {
    return fail(MFMG_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return MFMG_OK;
}
