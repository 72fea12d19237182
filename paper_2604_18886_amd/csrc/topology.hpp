// Host-side octree topology of the solver: node refinement, 2:1 face
// balance, canonical Morton brick order, per-level brick lists, brick
// neighbour tables and the canonical face numbering.
//
// The refinement unit is a brick of 4x4x4 cells (a node).  Refinement and
// balance follow Section 3 of the paper (leaf, inner and ghost cells;
// face-neighbouring leaves differ by at most one level) with the grid
// generator's rule of Section 4.1 (a node meeting the surface is split).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mfmg {

constexpr int kBrick = 4;       // cells per brick edge
constexpr int kCells = 64;      // cells per brick
constexpr int kMaxLevel = 12;   // finest supported cell level
constexpr int kMinLevel = 2;    // a 4^3 brick needs at least 4 cells per axis

struct Prim {
  int kind;  // 0 sphere, 1 box
  double center[3];
  double radius;
  double band;
  double lo[3];
  double hi[3];
};

// Neighbour encoding of a brick face: >= 0 same-level brick id, kWall for
// the domain boundary, <= kCoarseBase: the region is covered by the coarser
// leaf brick id = kCoarseBase - value (a T-junction face).
constexpr int32_t kWall = -1;
constexpr int32_t kCoarseBase = -2;

inline int32_t encode_coarse(int32_t brick) { return kCoarseBase - brick; }
inline int32_t decode_coarse(int32_t v) { return kCoarseBase - v; }

// Local Morton index of cell (x, y, z) inside a brick (x in bit 0).
inline int local_morton(int x, int y, int z) {
  return (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((x & 2) << 2) |
         ((y & 2) << 3) | ((z & 2) << 4);
}
inline void local_coords(int m, int &x, int &y, int &z) {
  x = (m & 1) | ((m >> 2) & 2);
  y = ((m >> 1) & 1) | ((m >> 3) & 2);
  z = ((m >> 2) & 1) | ((m >> 4) & 2);
}

struct Topology {
  int min_level = 0, max_level = 0;
  int64_t n_leaf_bricks = 0;  // leaf bricks come first, in canonical order
  int64_t n_bricks = 0;       // leaf + inner bricks (levels kMinLevel..max)
  std::vector<int8_t> level;   // per brick
  std::vector<int32_t> coord;  // 3 per brick, brick coordinates at its level
  std::vector<int32_t> nbr;    // 6 per brick
  std::vector<int32_t> parent; // per brick, -1 at level kMinLevel
  std::vector<int32_t> child;  // 8 per brick (octant dx + 2 dy + 4 dz), -1 for leaves
  // bricks of each level (leaf and inner), in Morton order at that level
  std::vector<std::vector<int32_t>> level_bricks;
  std::vector<std::vector<int32_t>> level_inner;  // inner bricks only

  // canonical faces
  int64_t n_faces = 0;
  std::vector<int64_t> cell_fbase;  // per leaf cell: id of its first owned face
  std::vector<uint8_t> cell_fmask;  // per leaf cell: bitmask of owned directions
  // per leaf brick: slot in the table of plus-side T-face coefficients
  // (3 faces x 16 cells per slot), -1 when the brick has no + T-face
  std::vector<int32_t> tplus;
  int64_t n_tplus = 0;

  int64_t n_leaves() const { return n_leaf_bricks * kCells; }

  // Face kind of leaf cell (brick b, local m) across direction d and the
  // leaf cell on the other side: 0 wall, 1 same level, 2 coarser leaf,
  // 3 finer leaves (the face is split and owned by the finer cells).
  int cell_neighbour(int64_t b, int m, int d, int64_t *other) const;
};

// Build the topology; returns an empty string or an error message.
std::string build_topology(int min_level, int max_level, int node_size,
                           const std::vector<Prim> &prims, Topology &out);

}  // namespace mfmg
