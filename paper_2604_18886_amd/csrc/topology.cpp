// Host octree topology: refinement, balance, brick tables, face numbering.
// Compiled with -ffp-contract=off so that the refinement predicates take the
// same IEEE decisions as any other straightforward evaluation of them.
#include "topology.hpp"

#include <algorithm>
#include <cmath>
#include <unordered_map>
#include <unordered_set>

namespace mfmg {
namespace {

const int kDir[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                        {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};

inline uint64_t node_key(int l, int64_t a, int64_t b, int64_t c) {
  return (uint64_t(l) << 48) | (uint64_t(a) << 32) | (uint64_t(b) << 16) |
         uint64_t(c);
}

// Interleave the low `bits` bits of x, y, z (x least significant).
uint64_t morton(uint64_t x, uint64_t y, uint64_t z, int bits) {
  uint64_t k = 0;
  for (int i = 0; i < bits; ++i) {
    k |= ((x >> i) & 1u) << (3 * i);
    k |= ((y >> i) & 1u) << (3 * i + 1);
    k |= ((z >> i) & 1u) << (3 * i + 2);
  }
  return k;
}

// Closed node box meets the shell radius - band <= |x - c| <= radius + band.
// Squared distances only: no square root enters the decision.
bool sphere_meets(const Prim &p, const double lo[3], const double hi[3]) {
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double t = lo[ax] - p.center[ax];
    if (0.0 > t) t = 0.0;
    double t2 = p.center[ax] - hi[ax];
    if (t2 > t) t = t2;
    dmin2 = dmin2 + t * t;
    double u1 = std::fabs(lo[ax] - p.center[ax]);
    double u2 = std::fabs(hi[ax] - p.center[ax]);
    double u = u1 > u2 ? u1 : u2;
    dmax2 = dmax2 + u * u;
  }
  double ro = p.radius + p.band;
  double ri = p.radius - p.band;
  if (dmin2 > ro * ro) return false;
  if (ri > 0.0 && dmax2 < ri * ri) return false;
  return true;
}

// Closed node box meets the boundary of the closed obstacle box.
bool box_meets_surface(const Prim &p, const double lo[3], const double hi[3]) {
  bool inter = true, inside = true;
  for (int ax = 0; ax < 3; ++ax) {
    inter = inter && lo[ax] <= p.hi[ax] && p.lo[ax] <= hi[ax];
    inside = inside && p.lo[ax] < lo[ax] && hi[ax] < p.hi[ax];
  }
  return inter && !inside;
}

bool meets(const Prim &p, const double lo[3], const double hi[3]) {
  return p.kind == 0 ? sphere_meets(p, lo, hi) : box_meets_surface(p, lo, hi);
}

struct Node {
  int l;
  int32_t a, b, c;
};

using NodeSet = std::unordered_set<uint64_t>;

void split(NodeSet &leaves, const Node &n) {
  leaves.erase(node_key(n.l, n.a, n.b, n.c));
  for (int o = 0; o < 8; ++o)
    leaves.insert(node_key(n.l + 1, 2 * n.a + (o & 1), 2 * n.b + ((o >> 1) & 1),
                           2 * n.c + ((o >> 2) & 1)));
}

Node unpack(uint64_t k) {
  return Node{int(k >> 48), int32_t((k >> 32) & 0xffff),
              int32_t((k >> 16) & 0xffff), int32_t(k & 0xffff)};
}

// Least 2:1 face-balanced refinement: split every leaf that has a face
// neighbour two or more levels finer, until none is left.
void balance(NodeSet &leaves, int min_level) {
  for (;;) {
    std::vector<uint64_t> todo;
    for (uint64_t k : leaves) {
      Node n = unpack(k);
      int64_t per = (int64_t(1) << n.l) / kBrick;
      for (int d = 0; d < 6; ++d) {
        int64_t a = n.a + kDir[d][0], b = n.b + kDir[d][1], c = n.c + kDir[d][2];
        if (a < 0 || b < 0 || c < 0 || a >= per || b >= per || c >= per) continue;
        for (int q = n.l; q >= min_level; --q) {
          int s = n.l - q;
          uint64_t ck = node_key(q, a >> s, b >> s, c >> s);
          if (leaves.count(ck)) {
            if (q <= n.l - 2) todo.push_back(ck);
            break;
          }
        }
      }
    }
    if (todo.empty()) return;
    std::sort(todo.begin(), todo.end());
    todo.erase(std::unique(todo.begin(), todo.end()), todo.end());
    for (uint64_t k : todo)
      if (leaves.count(k)) split(leaves, unpack(k));
  }
}

}  // namespace

int Topology::cell_neighbour(int64_t b, int m, int d, int64_t *other) const {
  int x, y, z;
  local_coords(m, x, y, z);
  int nx = x + kDir[d][0], ny = y + kDir[d][1], nz = z + kDir[d][2];
  if (nx >= 0 && ny >= 0 && nz >= 0 && nx < kBrick && ny < kBrick && nz < kBrick) {
    *other = b * kCells + local_morton(nx, ny, nz);
    return 1;
  }
  int32_t n = nbr[6 * b + d];
  if (n == kWall) {
    *other = -1;
    return 0;
  }
  if (n >= 0) {
    if (n >= n_leaf_bricks) {
      *other = -1;
      return 3;
    }
    *other = int64_t(n) * kCells + local_morton(nx & 3, ny & 3, nz & 3);
    return 1;
  }
  int32_t J = decode_coarse(n);
  // global coordinates of the neighbour position at this level, halved
  int64_t gx = int64_t(coord[3 * b]) * kBrick + nx;
  int64_t gy = int64_t(coord[3 * b + 1]) * kBrick + ny;
  int64_t gz = int64_t(coord[3 * b + 2]) * kBrick + nz;
  int cx = int((gx >> 1) - int64_t(coord[3 * J]) * kBrick);
  int cy = int((gy >> 1) - int64_t(coord[3 * J + 1]) * kBrick);
  int cz = int((gz >> 1) - int64_t(coord[3 * J + 2]) * kBrick);
  *other = int64_t(J) * kCells + local_morton(cx, cy, cz);
  return 2;
}

std::string build_topology(int min_level, int max_level, int node_size,
                           const std::vector<Prim> &prims, Topology &T) {
  if (node_size != kBrick) return "node_size must be 4";
  if (min_level < kMinLevel || max_level > kMaxLevel || min_level > max_level)
    return "levels out of range (2 <= min_level <= max_level <= 12)";
  for (const Prim &p : prims)
    if (p.kind != 0 && p.kind != 1) return "unknown primitive kind";

  // ---- predicate refinement
  NodeSet leaves;
  int64_t n0 = (int64_t(1) << min_level) / kBrick;
  for (int64_t a = 0; a < n0; ++a)
    for (int64_t b = 0; b < n0; ++b)
      for (int64_t c = 0; c < n0; ++c) leaves.insert(node_key(min_level, a, b, c));
  for (int l = min_level; l < max_level; ++l) {
    std::vector<uint64_t> cur;
    for (uint64_t k : leaves)
      if (int(k >> 48) == l) cur.push_back(k);
    double s = double(kBrick) * std::ldexp(1.0, -l);
    for (uint64_t k : cur) {
      Node n = unpack(k);
      double lo[3] = {n.a * s, n.b * s, n.c * s};
      double hi[3] = {(n.a + 1) * s, (n.b + 1) * s, (n.c + 1) * s};
      for (const Prim &p : prims)
        if (meets(p, lo, hi)) {
          split(leaves, n);
          break;
        }
    }
  }
  balance(leaves, min_level);

  // ---- leaf bricks in canonical order
  int L = 0;
  for (uint64_t k : leaves) L = std::max(L, int(k >> 48));
  T.min_level = min_level;
  T.max_level = max_level;
  struct Rec {
    uint64_t key;
    Node n;
  };
  std::vector<Rec> recs;
  recs.reserve(leaves.size());
  for (uint64_t k : leaves) {
    Node n = unpack(k);
    int s = max_level - n.l;
    uint64_t mk = morton(uint64_t(n.a) * kBrick << s, uint64_t(n.b) * kBrick << s,
                         uint64_t(n.c) * kBrick << s, max_level);
    recs.push_back({mk, n});
  }
  std::sort(recs.begin(), recs.end(),
            [](const Rec &x, const Rec &y) { return x.key < y.key; });
  T.n_leaf_bricks = int64_t(recs.size());

  std::unordered_map<uint64_t, int32_t> id;
  id.reserve(recs.size() * 2);
  for (size_t i = 0; i < recs.size(); ++i)
    id[node_key(recs[i].n.l, recs[i].n.a, recs[i].n.b, recs[i].n.c)] = int32_t(i);
  std::vector<Node> nodes;
  for (auto &r : recs) nodes.push_back(r.n);

  // ---- inner bricks: every ancestor of a leaf brick down to kMinLevel
  T.level_bricks.assign(max_level + 1, {});
  T.level_inner.assign(max_level + 1, {});
  for (int l = max_level - 1; l >= kMinLevel; --l) {
    std::vector<Rec> inner;
    std::unordered_set<uint64_t> seen;
    for (const Node &n : nodes) {
      if (n.l <= l) continue;
      int s = n.l - l;
      uint64_t k = node_key(l, n.a >> s, n.b >> s, n.c >> s);
      if (seen.insert(k).second) {
        Node p = unpack(k);
        inner.push_back({morton(p.a, p.b, p.c, max_level), p});
      }
    }
    std::sort(inner.begin(), inner.end(),
              [](const Rec &x, const Rec &y) { return x.key < y.key; });
    for (auto &r : inner) {
      uint64_t k = node_key(r.n.l, r.n.a, r.n.b, r.n.c);
      if (id.count(k)) return "inner brick coincides with a leaf brick";
      int32_t bid = int32_t(nodes.size());
      id[k] = bid;
      nodes.push_back(r.n);
      T.level_inner[l].push_back(bid);
    }
  }
  T.n_bricks = int64_t(nodes.size());
  if (T.n_bricks >= (int64_t(1) << 31) / kCells) return "octree too large";

  // ---- per-level brick lists in Morton order at that level
  {
    std::vector<std::vector<Rec>> per(max_level + 1);
    for (size_t i = 0; i < nodes.size(); ++i) {
      const Node &n = nodes[i];
      per[n.l].push_back({morton(n.a, n.b, n.c, max_level), Node{int(i), 0, 0, 0}});
    }
    for (int l = kMinLevel; l <= max_level; ++l) {
      std::sort(per[l].begin(), per[l].end(),
                [](const Rec &x, const Rec &y) { return x.key < y.key; });
      for (auto &r : per[l]) T.level_bricks[l].push_back(r.n.l);
    }
  }

  // ---- brick tables
  T.level.resize(T.n_bricks);
  T.coord.resize(3 * T.n_bricks);
  T.nbr.resize(6 * T.n_bricks);
  T.parent.assign(T.n_bricks, -1);
  T.child.assign(8 * T.n_bricks, -1);
  for (int64_t i = 0; i < T.n_bricks; ++i) {
    const Node &n = nodes[i];
    T.level[i] = int8_t(n.l);
    T.coord[3 * i] = n.a;
    T.coord[3 * i + 1] = n.b;
    T.coord[3 * i + 2] = n.c;
    int64_t per = (int64_t(1) << n.l) / kBrick;
    for (int d = 0; d < 6; ++d) {
      int64_t a = n.a + kDir[d][0], b = n.b + kDir[d][1], c = n.c + kDir[d][2];
      int32_t v;
      if (a < 0 || b < 0 || c < 0 || a >= per || b >= per || c >= per) {
        v = kWall;
      } else {
        auto it = id.find(node_key(n.l, a, b, c));
        if (it != id.end()) {
          v = it->second;
        } else {
          auto jt = id.find(node_key(n.l - 1, a >> 1, b >> 1, c >> 1));
          if (jt == id.end() || jt->second >= T.n_leaf_bricks)
            return "octree is not 2:1 balanced";
          if (i >= T.n_leaf_bricks) return "inner brick at a T-junction";
          v = encode_coarse(jt->second);
        }
      }
      T.nbr[6 * i + d] = v;
    }
    if (n.l > kMinLevel) {
      auto it = id.find(node_key(n.l - 1, n.a >> 1, n.b >> 1, n.c >> 1));
      if (it == id.end() || it->second < T.n_leaf_bricks) return "missing parent brick";
      T.parent[i] = it->second;
      int o = (n.a & 1) | ((n.b & 1) << 1) | ((n.c & 1) << 2);
      T.child[8 * int64_t(it->second) + o] = int32_t(i);
    }
  }
  for (int64_t i = T.n_leaf_bricks; i < T.n_bricks; ++i)
    for (int o = 0; o < 8; ++o)
      if (T.child[8 * i + o] < 0) return "inner brick with a missing child";

  // ---- plus-side T-face coefficient slots
  T.tplus.assign(T.n_leaf_bricks, -1);
  T.n_tplus = 0;
  for (int64_t i = 0; i < T.n_leaf_bricks; ++i) {
    bool any = false;
    for (int d = 1; d < 6; d += 2) any = any || T.nbr[6 * i + d] <= kCoarseBase;
    if (any) T.tplus[i] = int32_t(T.n_tplus++);
  }

  // ---- canonical faces: (owner, direction); owned = wall, coarser
  // neighbour, or same-level neighbour on the - side
  int64_t N = T.n_leaves();
  T.cell_fbase.resize(N);
  T.cell_fmask.resize(N);
  int64_t f = 0;
  for (int64_t b = 0; b < T.n_leaf_bricks; ++b)
    for (int m = 0; m < kCells; ++m) {
      uint8_t mask = 0;
      for (int d = 0; d < 6; ++d) {
        int64_t other;
        int kind = T.cell_neighbour(b, m, d, &other);
        bool own = kind == 0 || kind == 2 || (kind == 1 && (d & 1) == 0);
        if (own) mask |= uint8_t(1u << d);
      }
      T.cell_fbase[b * kCells + m] = f;
      T.cell_fmask[b * kCells + m] = mask;
      f += __builtin_popcount(mask);
    }
  T.n_faces = f;
  return "";
}

}  // namespace mfmg
