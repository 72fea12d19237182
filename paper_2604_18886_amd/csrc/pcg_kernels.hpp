// HIP kernels of the outer Krylov solver (Algorithm 1, FP64): the composite
// leaf operator with its T-junction rows (Section 3.1) and its transpose,
// the PCG vector updates with fused deterministic dot products, and the
// gather/scatter between the canonical leaf order of the C ABI and the
// level-major device order.
#pragma once

#include "kernels.hpp"

namespace mfmg {

struct PcgArgs {
  Topo T;
  const double *C;       // FP64 coefficients of all bricks (device order)
  const double *TC;      // FP64 plus-side T-face coefficients
  const double *PF;      // FP64 plus-face coefficients of all bricks, 48 per brick
  const int32_t *canon;  // device leaf brick -> canonical leaf brick
  Scalars *S;
  double *partials;
  double *hist;
  int *host_done;        // pinned host copy of S->done (mapped), or null
  int scale_low;         // 1: the cycle reads an FP32 copy of the residual, scaled
                         // by the power of two S->rscale (0: FP64, unscaled)
};

// Scale of the cycle's FP32 input: the power of two that brings the mean
// square of a residual with squared norm rr over n entries to [1, 4).  The
// cycle is linear, so z = M r is recovered exactly by the inverse power of
// two; FP32's range then holds the residual whatever the scale of the
// right-hand side.
__device__ __forceinline__ double low_scale(const PcgArgs &P, double rr) {
  if (!P.scale_low || !(rr > 0.0) || !(rr < INFINITY)) return 1.0;
  int e = ilogb(rr / (64.0 * double(P.T.nlb)));
  return ldexp(1.0, -(e / 2));
}

__device__ __forceinline__ void leaf_cell(const PcgArgs &P, uint32_t b, int m, double &c,
                                          double &k0, double &k1, double &k2) {
  const double *cf = P.C + b * 256u;
  c = cf[m];
  k0 = cf[64 + m];
  k1 = cf[128 + m];
  k2 = cf[192 + m];
}

// Transposed composite operator (adjoint path).  Its T-junction blocks are
// the transposes of the rank-one blocks of A: a fine cell's row gets, for
// every active sibling, (1/n) sum over the sibling group's T-faces of
// (k/2)(x_i - x_J); a coarse leaf's row gets - sum_f (k_f/2) x_f over the
// fine face cells f in place of K_F times their parent's mean.  X is a
// leaf-sized vector in device order; inner neighbours are read through
// their children.
__device__ __forceinline__ double composite_AuT(const Topo &T, const double *__restrict__ C,
                                                const double *__restrict__ TC,
                                                const double *__restrict__ X,
                                                const BrickMeta &M, int m, double u, double c,
                                                double k0, double k1, double k2) {
  uint64_t amask = act_mask(M);
  bool act = (amask >> m) & 1ull;
  int cnt = __popcll((amask >> (m & 56)) & 0xffull);
  double acc = c * u;
  double tpart = 0.0;  // this cell's sum of (k/2)(x_m - x_J) over its T-faces
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    double kown = a == 0 ? k0 : (a == 1 ? k1 : k2);
    double v = shfl(u, p);
    double kp = shfl(kown, p);
    double k = (d & 1) ? kp : kown;
    if (dev_outside(m, d)) {
      int32_t nb = M.nbr[d];
      if (nb >= 0 && uint32_t(nb) < T.nlb) {
        v = X[uint32_t(nb) * 64u + p];
        if (d & 1) k = C[uint32_t(nb) * 256u + (1 + a) * 64 + p];
      } else if (nb >= 0) {
        int32_t cb = T.child[8 * int64_t(nb) + (p >> 3)];
        int32_t slot = T.meta[cb].tplus;
        int base = (p & 7) << 3;
        int facebit = (d & 1) ? 0 : 1;  // children on P's face toward this cell
        double sumkv = 0.0;
        for (int t = 0; t < 8; ++t) {
          if (((t >> a) & 1) != facebit) continue;
          int q = base | t;
          double kc = (d & 1) ? C[uint32_t(cb) * 256u + (1 + a) * 64 + q]
                              : TC[uint32_t(slot) * 48u + a * 16 + dev_face_index(q, a)];
          sumkv += kc * 0.5 * X[uint32_t(cb) * 64u + q];
        }
        acc -= sumkv;
        continue;
      } else if (nb == dWall) {
        v = 0.0;
      } else {
        int32_t J = dev_decode_coarse(nb);
        double uJ = X[uint32_t(J) * 64u + coarse_local(M, m, d)];
        if (d & 1) k = TC[uint32_t(M.tplus) * 48u + a * 16 + dev_face_index(m, a)];
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
// with a T-face, written to the parent cells' slots of a full-size vector:
// the value the forward composite operator reads for an inner neighbour.
__device__ __forceinline__ void average_up(double *__restrict__ X, const BrickMeta &M, int m,
                                           double x) {
  uint64_t amask = act_mask(M);
  bool act = (amask >> m) & 1ull;
  double s = group8_sum(act ? x : 0.0);
  int cnt = __popcll((amask >> (m & 56)) & 0xffull);
  if ((m & 7) == 0)
    X[uint32_t(M.parent) * 64u + ((octant_of(M) << 3) | (m >> 3))] = cnt ? s / double(cnt) : 0.0;
}

// The forward composite operator is the finest-level stencil applied to a
// full-size vector whose inner cells hold the mean of their active children
// (average_up): an inner neighbour's plus-face coefficient is its Algorithm 3
// k, the sum of the fine sub-face coefficients over 2 (the coarse side of a
// T-junction), and the fine side takes the ghost of Eq. (10).  It therefore
// runs through stencil_sum, on the FP64 coefficient arrays.
template <int CP = kCpolDefault>
__device__ __forceinline__ LevelView<double, double, double, CP> composite_view(const PcgArgs &P,
                                                                                const double *X) {
  LevelView<double, double, double, CP> V;
  uint64_t nb = P.T.nb, nlb = P.T.nlb;
  V.u = make_rsrc(X, nb * 64 * sizeof(double));
  V.b = V.u;
  V.us = V.u;
  V.cl = make_rsrc(P.C, nlb * 256 * sizeof(double));
  V.ci = make_rsrc(P.C + nlb * 256, (nb - nlb) * 256 * sizeof(double));
  V.pf = make_rsrc(P.PF, nb * 48 * sizeof(double));
  V.meta = P.T.meta;
  V.nlb = P.T.nlb;
  V.iscale = 1.0;
  return V;
}

// y = (A X)_m at the lane's cell of leaf brick b (0 on inactive cells); u = X_m.
template <int CP>
__device__ __forceinline__ double composite_row(const LevelView<double, double, double, CP> &V,
                                                const LaneC<double, double> &L, uint32_t b,
                                                double &u) {
  const BrickMeta M = load_meta(V.meta, b);
  double k0 = own_coef<false>(V, b, 1, L.m);
  double k1 = own_coef<false>(V, b, 2, L.m);
  double k2 = own_coef<false>(V, b, 3, L.m);
  u = bload<double>(V.u, L.m, b * 64u);
  double c;
  double S = stencil_sum(V, L, b, M, u, k0, k1, k2, c);
  bool act = (act_mask(M) >> L.m) & 1ull;
  return act ? c * u - S : 0.0;
}

// per-workgroup partial of a wave-private sum, in fixed order
__device__ __forceinline__ void block_partial(double part, double *partials) {
  __shared__ double red[kWavesPerBlock];
  part = wave_sum(part);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) s += red[w];
    partials[blockIdx.x] = s;
  }
}

// grid-stride loop of one wave over the leaf bricks
#define LEAF_LOOP(P)                                                     \
  int m = threadIdx.x & (kWave - 1);                                     \
  for (uint32_t b = blockIdx.x * kWavesPerBlock + wave_id(); b < (P).T.nlb; \
       b += gridDim.x * kWavesPerBlock)

// r = rhs (canonical order) on active cells, x = 0, ||r||^2
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_init(PcgArgs P, const double *rhs, double *r,
                                                     V *r_low, double *x) {
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    bool act = (act_mask(M) >> m) & 1ull;
    double v = act ? rhs[uint32_t(P.canon[b]) * 64u + m] : 0.0;
    r[b * 64u + m] = v;
    if (r_low) r_low[b * 64u + m] = V(v);
    x[b * 64u + m] = 0.0;
    part += v * v;
  }
  block_partial(part, P.partials);
}

// Warm start (Algorithm 1 from an initial guess): r already holds rhs - A x0;
// x = x0 (canonical input) on active cells, the FP32 copy of r, ||r||^2.
template <class V>
__global__ void __launch_bounds__(kBlock) k_warm_start(PcgArgs P, const double *x0, double *x,
                                                       const double *r, V *r_low) {
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    bool act = (act_mask(M) >> m) & 1ull;
    x[b * 64u + m] = act ? x0[uint32_t(P.canon[b]) * 64u + m] : 0.0;
    double v = r[b * 64u + m];
    if (r_low) r_low[b * 64u + m] = V(v);
    part += v * v;
  }
  block_partial(part, P.partials);
}

// r_low = V(r * S->rscale): the cycle's input after the residual was set
// outside the iteration (start, warm start, restart)
template <class V>
__global__ void __launch_bounds__(kBlock) k_scale_low(PcgArgs P, const double *r, V *r_low) {
  double sc = P.S->rscale;
  LEAF_LOOP(P) { r_low[b * 64u + m] = V(r[b * 64u + m] * sc); }
}

// Restart from the true residual t (device order, already zero on inactive
// cells): r = t and ||r||^2 (the stop test's reference ||r_0|| is kept)
__global__ void __launch_bounds__(kBlock) k_restart(PcgArgs P, const double *t, double *r) {
  double part = 0.0;
  LEAF_LOOP(P) {
    double v = t[b * 64u + m];
    r[b * 64u + m] = v;
    part += v * v;
  }
  block_partial(part, P.partials);
}

// (r, z) over the leaf bricks (wave_loop grid); z is the cycle's output for
// the scaled residual
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_rz(PcgArgs P, const double *r, const V *z) {
  if (P.S->done) return;
  double zs = 1.0 / P.S->rscale;  // a power of two: exact
  uint32_t m = threadIdx.x & (kWave - 1);
  const __amdgpu_buffer_rsrc_t rr = make_rsrc(r, uint64_t(P.T.nlb) * 64 * sizeof(double));
  const __amdgpu_buffer_rsrc_t zr = make_rsrc(z, uint64_t(P.T.nlb) * 64 * sizeof(V));
  const WaveLoop W = wave_loop(P.T.nlb);
  double part = 0.0;
  for (uint32_t b = W.first; b < W.end; b += W.step)
    part += bload<double, kCpolStream>(rr, m, b * 64u) * (double(bload<V>(zr, m, b * 64u)) * zs);
  block_partial(part, P.partials);
}

// p = z + beta p (p = z on the first call) over the leaf bricks, and for
// bricks with a T-face the mean of each active sibling group written to the
// parent's slot of the full-size p: the value the forward composite operator
// reads for an inner neighbour.  After the first call it also takes the
// iterate's step x += alpha p of the residual update before (Algorithm 1's
// x update, moved here because this kernel reads p anyway); k_pcg_x adds it
// when the solve stopped before this kernel ran.
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_p(PcgArgs P, const V *z, double *p, double *x,
                                                  int first) {
  if (P.S->done) return;
  double beta = first ? 0.0 : P.S->beta;
  double alpha = P.S->alpha;
  double zs = 1.0 / P.S->rscale;
  uint32_t m = threadIdx.x & (kWave - 1);
  const __amdgpu_buffer_rsrc_t zr = make_rsrc(z, uint64_t(P.T.nlb) * 64 * sizeof(V));
  const __amdgpu_buffer_rsrc_t pr = make_rsrc(p, uint64_t(P.T.nb) * 64 * sizeof(double));
  const __amdgpu_buffer_rsrc_t xr = make_rsrc(x, uint64_t(P.T.nlb) * 64 * sizeof(double));
  const WaveLoop W = wave_loop(P.T.nlb);
  if (!first && blockIdx.x == 0 && threadIdx.x == 0) P.S->xpend = 0;
  for (uint32_t b = W.first; b < W.end; b += W.step) {
    double v = double(bload<V, kCpolStream>(zr, m, b * 64u)) * zs;
    if (!first) {
      double po = bload<double, kCpolStream>(pr, m, b * 64u);
      bstore<double, kCpolStream>(xr, m, b * 64u,
                                  bload<double, kCpolStream>(xr, m, b * 64u) + alpha * po);
      v += beta * po;
    }
    bstore<double>(pr, m, b * 64u, v);
    const BrickMeta M = load_meta(P.T.meta, b);
    if (M.flags & kFlagT) average_up(p, M, int(m), v);
  }
}

// Ap = A p over the leaf bricks (wave_loop grid); each workgroup stores its
// partial (p, Ap), k_finish_alpha adds them in fixed order.
template <int CP = kCpolDefault>
__global__ void __launch_bounds__(kBlock) k_pcg_Ap(PcgArgs P, const double *p, double *Ap) {
  if (P.S->done) return;
  const LevelView<double, double, double, CP> V = composite_view<CP>(P, p);
  const LaneC<double, double> L = lane_consts<double, double>();
  const __amdgpu_buffer_rsrc_t out = make_rsrc(Ap, uint64_t(P.T.nlb) * 64 * sizeof(double));
  const WaveLoop W = wave_loop(P.T.nlb);
  double part = 0.0;
  for (uint32_t b = W.first; b < W.end; b += W.step) {
    double u;
    double y = composite_row(V, L, b, u);
    bstore<double>(out, L.m, b * 64u, y);
    part += u * y;
  }
  block_partial(part, P.partials);
}

// Ap = A^T p (adjoint solves), one wave per leaf brick.
__global__ void __launch_bounds__(kBlock) k_pcg_ApT(PcgArgs P, const double *p, double *Ap) {
  if (P.S->done) return;
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  double part = 0.0;
  if (b < P.T.nlb) {
    const BrickMeta M = P.T.meta[b];
    double c, k0, k1, k2;
    leaf_cell(P, b, m, c, k0, k1, k2);
    double u = p[b * 64u + m];
    double y = composite_AuT(P.T, P.C, P.TC, p, M, m, u, c, k0, k1, k2);
    Ap[b * 64u + m] = y;
    part = u * y;
  }
  block_partial(part, P.partials);
}

// Second stage of every PCG reduction: the per-workgroup partials of the
// preceding kernel (n of them) are added in fixed order by one workgroup,
// which then updates the solve's scalars.  (A grid-wide "last workgroup"
// scheme needs a device-scope release per workgroup, which writes back the
// XCD's L2 each time; a kernel boundary is cheaper.)
enum FinishOp : int {
  kFinInit = 0,   // ||r_0||^2: tolerance, first history entry
  kFinRz = 1,     // (r, z): beta (arg = 1 on the first iteration)
  kFinAlpha = 2,  // (p, Ap): alpha
  kFinUpdate = 3, // ||r_k||^2: stop test
  kFinTrue = 4,   // ||rhs - A x||^2
  kFinSum = 5,    // sum over active cells (null-space mean)
  kFinShift = 6,  // ||v||^2 after the mean shift, arg = mode of k_shift_mean
  kFinWarm = 7,   // ||rhs - A x0||^2 of a warm start (tolerance kept from ||rhs||)
  kFinRestart = 8,// ||r||^2 of a restart from the true residual (tolerance kept)
};

__device__ __forceinline__ void finish_iteration(const PcgArgs &P, double tot) {
  Scalars *S = P.S;
  S->xpend = 1;  // the residual update of this iteration is done
  S->rr = tot;
  S->iters += 1;
  P.hist[S->iters] = S->rr0 > 0.0 ? sqrt(tot / S->rr0) : 0.0;
  if (!(tot < INFINITY)) {
    S->status = -5;
    S->done = 1;
  } else if (tot <= S->tol2) {
    S->done = 1;
  }
}

__device__ __forceinline__ void finish_initial(const PcgArgs &P, double tot, double rtol) {
  Scalars *S = P.S;
  S->rr0 = tot;
  S->rr = tot;
  S->tol2 = rtol * rtol * tot;
  S->iters = 0;
  S->xpend = 0;
  S->status = 0;
  S->done = (tot == 0.0) || !(tot < INFINITY);
  if (!(tot < INFINITY)) S->status = -5;
  S->rz = 0.0;
  S->rscale = low_scale(P, tot);
  P.hist[0] = tot > 0.0 ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(1024) k_finish(PcgArgs P, int64_t n, int op, int arg,
                                                 double rtol) {
  Scalars *S = P.S;
  // the reductions of a stopped solve were skipped by their kernels
  bool gated = op == kFinRz || op == kFinAlpha || op == kFinUpdate ||
               (op == kFinShift && arg == 1);
  if (gated && S->done) return;
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += P.partials[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (unsigned w = 0; w < blockDim.x / 64; ++w) tot += red[w];
  switch (op) {
    case kFinInit:
      finish_initial(P, tot, rtol);
      break;
    case kFinRz:
      if (!(tot > 0.0) || !(tot < INFINITY)) {
        S->status = -5;
        S->done = 1;
      } else {
        S->beta = arg ? 0.0 : tot / S->rz;
        S->rz = tot;
      }
      break;
    case kFinAlpha:
      S->pAp = tot;
      if (!(tot > 0.0) || !(tot < INFINITY)) {
        S->status = -5;
        S->done = 1;
      } else {
        S->alpha = S->rz / tot;
      }
      // scale of the residual the update is about to write, from the last
      // norm (a PCG residual changes by modest factors per iteration)
      S->rscale = low_scale(P, S->rr);
      break;
    case kFinUpdate:
      finish_iteration(P, tot);
      break;
    case kFinTrue:
      S->tr = tot;
      break;
    case kFinSum:
      S->sum = tot;
      break;
    case kFinShift:
      if (arg == 0) finish_initial(P, tot, rtol);
      else if (arg == 1) finish_iteration(P, tot);
      else if (arg == 2) S->tr = tot;
      break;
    case kFinWarm:
      S->rr = tot;
      S->rscale = low_scale(P, tot);
      P.hist[0] = S->rr0 > 0.0 ? sqrt(tot / S->rr0) : 0.0;
      if (!(tot < INFINITY)) {
        S->status = -5;
        S->done = 1;
      } else if (tot <= S->tol2) {
        S->done = 1;
      }
      break;
    case kFinRestart:
      S->rr = tot;
      S->rscale = low_scale(P, tot);
      S->xpend = 0;
      S->done = !(tot > S->tol2) || !(tot < INFINITY);
      if (!(tot < INFINITY)) S->status = -5;
      break;
  }
  // the host polls the stop flag here instead of copying the scalars back
  if (P.host_done) __hip_atomic_store(P.host_done, S->done, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_SYSTEM);
}

// r -= alpha Ap, ||r||^2 and the stop test (the iterate's x += alpha p is
// taken by the next k_pcg_p, or by k_pcg_x after the loop)
template <class V>
__global__ void __launch_bounds__(kBlock) k_pcg_update(PcgArgs P, double *r, V *r_low,
                                                       const double *Ap, int defer,
                                                       int64_t n2) {
  if (P.S->done) return;
  double alpha = P.S->alpha;
  double sc = P.S->rscale;
  double part = 0.0;
  double2 *r2 = reinterpret_cast<double2 *>(r);
  const double2 *a2 = reinterpret_cast<const double2 *>(Ap);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    typedef double d2a __attribute__((ext_vector_type(2)));
    d2a av = __builtin_nontemporal_load(reinterpret_cast<const d2a *>(a2 + i));
    if (r_low) {
      // mixed: the cycle reads the FP32 copy next, r only in the next
      // (r, z), after the whole cycle: r passes the caches non-temporal
      typedef double d2 __attribute__((ext_vector_type(2)));
      d2 rv = __builtin_nontemporal_load(reinterpret_cast<d2 *>(r2 + i));
      rv.x -= alpha * av.x;
      rv.y -= alpha * av.y;
      __builtin_nontemporal_store(rv, reinterpret_cast<d2 *>(r2 + i));
      r_low[2 * i] = V(rv.x * sc);
      r_low[2 * i + 1] = V(rv.y * sc);
      part += rv.x * rv.x + rv.y * rv.y;
    } else {
      double2 rv = r2[i];
      rv.x -= alpha * av.x;
      rv.y -= alpha * av.y;
      r2[i] = rv;
      part += rv.x * rv.x + rv.y * rv.y;
    }
  }
  if (defer) return;  // the null-space shift completes this step
  block_partial(part, P.partials);
}

// x += alpha p when the solve stopped after a residual update and before
// the k_pcg_p that would have taken the iterate's step.
__global__ void __launch_bounds__(kBlock) k_pcg_x(PcgArgs P, double *x, const double *p) {
  if (!P.S->xpend) return;
  double alpha = P.S->alpha;
  LEAF_LOOP(P) { x[b * 64u + m] += alpha * p[b * 64u + m]; }
}

// X (full size, device order) from a leaf vector x; canonical = 1 when x is
// in canonical order.  Inactive cells are zeroed; bricks with T-faces write
// the sibling-group means into the parent slots.
__global__ void __launch_bounds__(kBlock) k_full(PcgArgs P, const double *x, double *X,
                                                 int canonical) {
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    uint32_t src = (canonical ? uint32_t(P.canon[b]) : b) * 64u + m;
    double v = ((act_mask(M) >> m) & 1ull) ? x[src] : 0.0;
    X[b * 64u + m] = v;
    if (M.flags & kFlagT) average_up(X, M, m, v);
  }
}

// y = A X (X from k_full), y in device order (wave_loop grid)
__global__ void __launch_bounds__(kBlock) k_apply(PcgArgs P, const double *X, double *y) {
  const LevelView<double, double, double> V = composite_view(P, X);
  const LaneC<double, double> L = lane_consts<double, double>();
  const __amdgpu_buffer_rsrc_t out = make_rsrc(y, uint64_t(P.T.nlb) * 64 * sizeof(double));
  const WaveLoop W = wave_loop(P.T.nlb);
  for (uint32_t b = W.first; b < W.end; b += W.step) {
    double u;
    double v = composite_row(V, L, b, u);
    bstore<double>(out, L.m, b * 64u, v);
  }
}

// y = A^T X, y in device order
__global__ void __launch_bounds__(kBlock) k_applyT(PcgArgs P, const double *X, double *y) {
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    double c, k0, k1, k2;
    leaf_cell(P, b, m, c, k0, k1, k2);
    double u = X[b * 64u + m];
    y[b * 64u + m] = composite_AuT(P.T, P.C, P.TC, X, M, m, u, c, k0, k1, k2);
  }
}

// ||rhs - A X||^2 over active cells, rhs in canonical order (wave_loop grid)
__global__ void __launch_bounds__(kBlock) k_true_resid(PcgArgs P, const double *rhs,
                                                       const double *X) {
  const LevelView<double, double, double> V = composite_view(P, X);
  const LaneC<double, double> L = lane_consts<double, double>();
  const WaveLoop W = wave_loop(P.T.nlb);
  double part = 0.0;
  for (uint32_t b = W.first; b < W.end; b += W.step) {
    double u;
    double y = composite_row(V, L, b, u);
    const BrickMeta M = load_meta(P.T.meta, b);
    bool act = (act_mask(M) >> L.m) & 1ull;
    double t = act ? rhs[uint32_t(P.canon[b]) * 64u + L.m] - y : 0.0;
    part += t * t;
  }
  block_partial(part, P.partials);
}

// t = g - y on active cells (g canonical, y and t device order) and ||t||^2
// (true residual of the adjoint system with y = A^T lambda)
__global__ void __launch_bounds__(kBlock) k_resid_T(PcgArgs P, const double *g, const double *y,
                                                    double *t) {
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    bool act = (act_mask(M) >> m) & 1ull;
    double v = act ? g[uint32_t(P.canon[b]) * 64u + m] - y[b * 64u + m] : 0.0;
    t[b * 64u + m] = v;
    part += v * v;
  }
  block_partial(part, P.partials);
}

// device-order leaf vector of type V -> canonical FP64 (inactive cells 0)
template <class V>
__global__ void __launch_bounds__(kBlock) k_to_canonical(PcgArgs P, const V *src, double *dst) {
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    double v = ((act_mask(M) >> m) & 1ull) ? double(src[b * 64u + m]) : 0.0;
    dst[uint32_t(P.canon[b]) * 64u + m] = v;
  }
}

// canonical FP64 -> device-order leaf vector of type V
template <class V>
__global__ void __launch_bounds__(kBlock) k_from_canonical(PcgArgs P, const double *src, V *dst) {
  LEAF_LOOP(P) { dst[b * 64u + m] = V(src[uint32_t(P.canon[b]) * 64u + m]); }
}

// ---------------------------------------------------------------------------
// null space (no Dirichlet face): the residual is shifted to zero mean over
// the active cells after it is formed (Section 2.2)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_sum_active(PcgArgs P, const double *v) {
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    if ((act_mask(M) >> m) & 1ull) part += v[b * 64u + m];
  }
  block_partial(part, P.partials);
}

// sum of v (canonical order) over the active cells, or of |v| (absval)
__global__ void __launch_bounds__(kBlock) k_sum_active_canon(PcgArgs P, const double *v,
                                                             int absval) {
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    if ((act_mask(M) >> m) & 1ull) {
      double x = v[int64_t(P.canon[b]) * 64 + m];
      part += absval ? fabs(x) : x;
    }
  }
  block_partial(part, P.partials);
}

// v -= sum / n_active on active cells and ||v||^2; mode 0: initial residual
// (sets rr0, tolerance, done), 1: iteration residual (stop test), 2: true
// residual (tr), 3: solution (no norm)
template <class V>
__global__ void __launch_bounds__(kBlock) k_shift_mean(PcgArgs P, double *v, V *v_low,
                                                       double n_active, int mode) {
  if (mode == 1 && P.S->done) return;
  double mean = P.S->sum / n_active;
  double sc = P.S->rscale;
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    uint32_t i = b * 64u + m;
    double x = ((act_mask(M) >> m) & 1ull) ? v[i] - mean : 0.0;
    v[i] = x;
    if (v_low) v_low[i] = V(x * sc);
    part += x * x;
  }
  block_partial(part, P.partials);
}

// t = rhs - A X over active cells (device order), rhs canonical (wave_loop grid)
__global__ void __launch_bounds__(kBlock) k_residual_vec(PcgArgs P, const double *rhs,
                                                         const double *X, double *t) {
  const LevelView<double, double, double> V = composite_view(P, X);
  const LaneC<double, double> L = lane_consts<double, double>();
  const WaveLoop W = wave_loop(P.T.nlb);
  for (uint32_t b = W.first; b < W.end; b += W.step) {
    double u;
    double y = composite_row(V, L, b, u);
    const BrickMeta M = load_meta(P.T.meta, b);
    bool act = (act_mask(M) >> L.m) & 1ull;
    t[b * 64u + L.m] = act ? rhs[uint32_t(P.canon[b]) * 64u + L.m] - y : 0.0;
  }
}

// Streaming copy (measurement of the achievable HBM bandwidth): 16-byte
// nontemporal accesses, each thread issuing its four loads before its four
// stores.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_stream_copy(const f32x4 *__restrict__ src,
                                                     f32x4 *__restrict__ dst, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  f32x4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i + k * 256 < n) v[k] = __builtin_nontemporal_load(src + i + k * 256);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i + k * 256 < n) __builtin_nontemporal_store(v[k], dst + i + k * 256);
}

// ---------------------------------------------------------------------------
// per-face gradient of the adjoint: dL/dbeta_f = -lambda^T (dA/dbeta_f) p
// (canonical face and leaf order)
// ---------------------------------------------------------------------------
struct GradArgs {
  const int64_t *owner;
  const int64_t *other;
  const int8_t *dir;
  const int8_t *kind;         // 0 wall, 1 same level, 2 T-junction (owner finer)
  const int8_t *level;        // per canonical leaf brick
  const uint64_t *act;        // per canonical leaf brick
  const double *lam;
  const double *p;
  int bc[6];
  double theta;
  int64_t n_faces;
  double *g;
};

__device__ __forceinline__ bool canon_active(const GradArgs &A, int64_t cell) {
  return (A.act[cell >> 6] >> (cell & 63)) & 1ull;
}

__global__ void k_face_gradient(GradArgs A) {
  int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= A.n_faces) return;
  int64_t o = A.owner[f];
  int64_t t = A.other[f];
  int k = A.kind[f];
  double h = ldexp(1.0, -int(A.level[o >> 6]));
  double g = 0.0;
  bool ao = canon_active(A, o);
  if (k == 0) {
    if (ao && A.bc[A.dir[f]] == 1) g = -(h / A.theta) * A.lam[o] * A.p[o];
  } else if (ao && canon_active(A, t)) {
    if (k == 1) {
      g = -h * (A.lam[o] - A.lam[t]) * (A.p[o] - A.p[t]);
    } else {
      // mean of p over the active siblings of the fine owner
      int64_t base = o & ~int64_t(7);
      double s = 0.0;
      int n = 0;
      for (int q = 0; q < 8; ++q)
        if (canon_active(A, base + q)) {
          s += A.p[base + q];
          ++n;
        }
      double pbar = n ? s / double(n) : 0.0;
      g = -(h / 2.0) * (A.lam[o] - A.lam[t]) * (pbar - A.p[t]);
    }
  }
  A.g[f] = g;
}

// activity masks in canonical leaf-brick order
__global__ void k_canonical_act(const BrickMeta *meta, const int32_t *canon, uint32_t nlb,
                                uint64_t *out) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nlb) out[canon[b]] = act_mask(meta[b]);
}

}  // namespace mfmg
