// Projection of a face velocity field around the solve (Section 2.1's flux
// form of the pressure equation; the static projection test of Section 4.4):
// the integrated divergence of MAC face velocities weighted by the faces'
// fluid fractions (the solve's right-hand side), the velocity update with the
// operator's own face fluxes, and the volume-weighted RMS of a divergence
// (Section 4.2).
//
// Velocities u_f are normal components along the + axis of each canonical
// face; a face's fluid area is beta_f h_o^2 (h_o of its owner, the finer
// side).  With the pressure flux
//   F_f = k_f (p_o - p_t)               same level,
//   F_f = k_f (mean of p over the active siblings of o - p_t) / 2
//                                       T-junction (o the fine owner),
//   F_f = k_f p_o                       Dirichlet wall (k_f = beta h / theta),
//   F_f = 0                             Neumann wall or an inactive side,
// (A p)_i sums +F_f over the faces leaf i owns and -F_f over the others, and
// u_f <- u_f - s_o F_f / (beta_f h_o^2) (s_o = +1 where the + axis points out
// of the owner) makes div(u_new) = div(u) - A p.
#pragma once

#include "kernels.hpp"
#include "pcg_kernels.hpp"

namespace mfmg {

struct DivArgs {
  Topo T;
  const int64_t *fbase;   // per device leaf cell: first owned face
  const uint8_t *fmask;   // per device leaf cell: owned directions
  const int32_t *canon;   // device leaf brick -> canonical leaf brick
  const double *beta;     // canonical face order
  const double *u;        // canonical face order
  double *div;            // canonical leaf order
};

__device__ __forceinline__ int64_t div_face(const DivArgs &A, uint32_t cell, int d) {
  return A.fbase[cell] + __popc(unsigned(A.fmask[cell]) & ((1u << d) - 1u));
}

// flow along the + axis through face f of area h^2
__device__ __forceinline__ double div_flow(const DivArgs &A, int64_t f, double h2) {
  return A.beta[f] * h2 * A.u[f];
}

// One wave per device leaf brick, one lane per cell: the outflow through
// each of its six sides, summed in direction order (a side towards finer
// leaves adds its four sub-faces in a fixed order).
__global__ void __launch_bounds__(kBlock) k_divergence(DivArgs A) {
  uint32_t b = blockIdx.x * kWavesPerBlock + wave_id();
  int m = threadIdx.x & (kWave - 1);
  if (b >= A.T.nlb) return;
  const BrickMeta M = A.T.meta[b];
  double h = ldexp(1.0, -M.level);
  double hf = ldexp(1.0, -(M.level + 1));
  uint32_t cell = b * 64u + m;
  double div = 0.0;
  for (int d = 0; d < 6; ++d) {
    int a = d >> 1;
    int p = dev_partner(m, d);
    double sgn = (d & 1) ? 1.0 : -1.0;
    double flow;
    if (!dev_outside(m, d)) {
      flow = (d & 1) ? div_flow(A, div_face(A, b * 64u + p, d - 1), h * h)
                     : div_flow(A, div_face(A, cell, d), h * h);
    } else {
      int32_t nb = M.nbr[d];
      if (nb == dWall || nb <= dCoarseBase) {
        flow = div_flow(A, div_face(A, cell, d), h * h);
      } else if (uint32_t(nb) < A.T.nlb) {
        flow = (d & 1) ? div_flow(A, div_face(A, uint32_t(nb) * 64u + p, d - 1), h * h)
                       : div_flow(A, div_face(A, cell, d), h * h);
      } else {
        // finer neighbours: the leaf children of inner cell p of brick nb
        int32_t cb = A.T.child[8 * int64_t(nb) + (p >> 3)];
        int base = (p & 7) << 3;
        int o0 = a == 0 ? 1 : 0;
        int o1 = a == 2 ? 1 : 2;
        int abit = (d & 1) ? 0 : 1;
        flow = 0.0;
        for (int n = 0; n < 4; ++n) {
          int t = (abit << a) | ((n & 1) << o0) | ((n >> 1) << o1);
          flow = flow + div_flow(A, div_face(A, uint32_t(cb) * 64u + (base | t), d ^ 1), hf * hf);
        }
      }
    }
    div = div + sgn * flow;
  }
  A.div[int64_t(A.canon[b]) * 64 + m] = div;
}

struct FluxArgs {
  const int64_t *owner, *other;  // canonical face list
  const int8_t *dir, *kind;
  const int8_t *level;           // per canonical leaf brick
  const uint64_t *act;           // per canonical leaf brick
  const double *beta;
  const double *p;               // canonical leaf order
  int bc[6];
  double theta;
  int64_t n_faces;
  double *u;                     // canonical face order, updated in place
};

__device__ __forceinline__ bool flux_active(const FluxArgs &A, int64_t cell) {
  return (A.act[cell >> 6] >> (cell & 63)) & 1ull;
}

// One thread per canonical face: u_f -= s_o F_f / (beta_f h_o^2).
__global__ void k_project_velocity(FluxArgs A) {
  int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= A.n_faces) return;
  double beta = A.beta[f];
  if (!(beta > 0.0)) return;
  int64_t o = A.owner[f];
  int64_t t = A.other[f];
  int k = A.kind[f];
  int d = A.dir[f];
  double h = ldexp(1.0, -int(A.level[o >> 6]));
  double F = 0.0;
  if (flux_active(A, o)) {
    if (k == 0) {
      if (A.bc[d] == 1) F = beta * (h / A.theta) * A.p[o];
    } else if (flux_active(A, t)) {
      if (k == 1) {
        F = beta * h * (A.p[o] - A.p[t]);
      } else {
        int64_t base = o & ~int64_t(7);
        double s = 0.0;
        int n = 0;
        for (int q = 0; q < 8; ++q)
          if (flux_active(A, base + q)) {
            s += A.p[base + q];
            ++n;
          }
        double pbar = n ? s / double(n) : 0.0;
        F = beta * h * (pbar - A.p[t]) / 2.0;
      }
    }
  }
  double sgn = (d & 1) ? 1.0 : -1.0;
  A.u[f] -= sgn * F / (beta * h * h);
}

// Parts of RMS_V over the active leaves of a canonical-order divergence:
// what = 0: sum of div_i^2 / V_i (= V_i (div_i / V_i)^2), 1: sum of V_i.
__global__ void __launch_bounds__(kBlock) k_div_rms_part(PcgArgs P, const double *div,
                                                         int what) {
  double part = 0.0;
  LEAF_LOOP(P) {
    const BrickMeta M = P.T.meta[b];
    if ((act_mask(M) >> m) & 1ull) {
      double V = ldexp(1.0, -3 * M.level);
      double x = div[int64_t(P.canon[b]) * 64 + m];
      part += what ? V : x * x / V;
    }
  }
  block_partial(part, P.partials);
}

}  // namespace mfmg
