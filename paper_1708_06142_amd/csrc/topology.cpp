// Host-side amr-tree topology (Sec. 2): validation that the leaf blocks tile
// the domain, the set of all blocks (leaves and their ancestors), their order
// by (level, Morton key) and the child links.  Integer work only.
#include <algorithm>
#include <unordered_map>

#include "ctx.hpp"

namespace ot {

namespace {

// spread the low 21 bits of v to every third bit
uint64_t part1by2(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

uint64_t morton3(uint64_t x, uint64_t y, uint64_t z) {
  return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

struct Node {
  int32_t lev;
  int32_t c[3];
  uint64_t key;
  int64_t leaf;
};

uint64_t pack(int lev, const int32_t c[3]) {
  return ((uint64_t)lev << 60) | ((uint64_t)c[0] << 40) | ((uint64_t)c[1] << 20) | (uint64_t)c[2];
}

}  // namespace

std::string build_topology(const int32_t nroot[3], int64_t nb, const int32_t *level,
                           const int32_t *coord, Topology &t) {
  if (nb <= 0) return "no blocks";
  for (int k = 0; k < 3; ++k)
    if (nroot[k] < 1 || nroot[k] > 64) return "nroot out of range";
  int lmax = 1;
  for (int64_t b = 0; b < nb; ++b) {
    if (level[b] < 1 || level[b] > 15) return "block level out of range";
    for (int k = 0; k < 3; ++k) {
      int64_t nmax = (int64_t)nroot[k] << (level[b] - 1);
      if (coord[3 * b + k] < 0 || coord[3 * b + k] >= nmax) return "block coordinate out of range";
    }
    lmax = std::max(lmax, (int)level[b]);
  }
  // every leaf and its ancestors, keyed by (level, coord)
  std::unordered_map<uint64_t, int64_t> index;  // key -> position in nodes
  std::vector<Node> nodes;
  nodes.reserve(nb * 2);
  for (int64_t b = 0; b < nb; ++b) {
    int32_t c[3] = {coord[3 * b], coord[3 * b + 1], coord[3 * b + 2]};
    uint64_t k0 = pack(level[b], c);
    auto it = index.find(k0);
    if (it != index.end()) {
      if (nodes[it->second].leaf >= 0) return "duplicate leaf block";
      return "leaf block overlaps a coarser block";
    }
    index.emplace(k0, (int64_t)nodes.size());
    nodes.push_back(Node{level[b], {c[0], c[1], c[2]}, 0, b});
    for (int l = level[b] - 1; l >= 1; --l) {
      for (int k = 0; k < 3; ++k) c[k] >>= 1;
      uint64_t kk = pack(l, c);
      auto jt = index.find(kk);
      if (jt != index.end()) {
        if (nodes[jt->second].leaf >= 0) return "leaf block overlaps a coarser block";
        break;  // ancestors above are present already
      }
      index.emplace(kk, (int64_t)nodes.size());
      nodes.push_back(Node{l, {c[0], c[1], c[2]}, 0, -1});
    }
  }
  for (auto &n : nodes) {
    int sh = lmax - n.lev;
    n.key = morton3((uint64_t)n.c[0] << sh, (uint64_t)n.c[1] << sh, (uint64_t)n.c[2] << sh);
  }
  std::sort(nodes.begin(), nodes.end(), [](const Node &a, const Node &b) {
    return a.lev != b.lev ? a.lev < b.lev : a.key < b.key;
  });
  int64_t na = (int64_t)nodes.size();
  index.clear();
  for (int64_t i = 0; i < na; ++i) index.emplace(pack(nodes[i].lev, nodes[i].c), i);

  t = Topology();
  t.nb = nb;
  t.na = na;
  t.lmax = lmax;
  t.blev.assign(level, level + nb);
  t.bcoord.assign(coord, coord + 3 * nb);
  t.alev.resize(na);
  t.acoord.resize(3 * na);
  t.akey.resize(na);
  t.aleaf.resize(na);
  t.achild.assign(8 * na, -1);
  t.bamr.assign(nb, -1);
  t.level_begin.assign(lmax + 2, na);
  for (int64_t i = na - 1; i >= 0; --i) t.level_begin[nodes[i].lev] = i;
  for (int l = lmax; l >= 1; --l)
    if (t.level_begin[l] > t.level_begin[l + 1]) t.level_begin[l] = t.level_begin[l + 1];
  for (int64_t i = 0; i < na; ++i) {
    const Node &n = nodes[i];
    t.alev[i] = n.lev;
    for (int k = 0; k < 3; ++k) t.acoord[3 * i + k] = n.c[k];
    t.akey[i] = n.key;
    t.aleaf[i] = n.leaf;
    if (n.leaf >= 0) {
      t.bamr[n.leaf] = i;
      continue;
    }
    for (int o = 0; o < 8; ++o) {
      int32_t c[3];
      for (int k = 0; k < 3; ++k) c[k] = 2 * n.c[k] + ((o >> k) & 1);
      auto it = index.find(pack(n.lev + 1, c));
      if (it == index.end()) return "hole: a block is neither a leaf nor fully refined";
      t.achild[8 * i + o] = it->second;
      if (it->second != t.achild[8 * i] + o) return "internal: children not contiguous";
    }
  }
  int64_t nr = t.level_begin[2] - t.level_begin[1];
  if (nr != (int64_t)nroot[0] * nroot[1] * nroot[2]) return "hole: a root block is missing";
  t.nroots = nr;
  return std::string();
}

}  // namespace ot
