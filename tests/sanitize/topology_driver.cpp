// Drives the library's host-side amr-tree topology (validation, ancestors,
// (level, Morton key) order, child links) on seeded random AMR grids and on
// invalid ones, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (see tests/test_sanitize.py).  Exit status 0 on
// success.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../paper_1708_06142_amd/csrc/ctx.hpp"

static int failures = 0;
#define CHECK(c)                                                               \
  do {                                                                         \
    if (!(c)) {                                                                \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                              \
    }                                                                          \
  } while (0)

struct Grid {
  int32_t nroot[3];
  std::vector<int32_t> level, coord;
};

// every root refined recursively with probability p per block, up to lmax
static Grid random_grid(std::mt19937_64 &rng, const int32_t nroot[3], double p, int lmax) {
  Grid g{{nroot[0], nroot[1], nroot[2]}, {}, {}};
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<std::tuple<int, int, int, int>> todo;
  for (int z = 0; z < nroot[2]; ++z)
    for (int y = 0; y < nroot[1]; ++y)
      for (int x = 0; x < nroot[0]; ++x) todo.emplace_back(1, x, y, z);
  while (!todo.empty()) {
    auto [l, x, y, z] = todo.back();
    todo.pop_back();
    if (l < lmax && u(rng) < p) {
      for (int o = 0; o < 8; ++o) todo.emplace_back(l + 1, 2 * x + (o & 1), 2 * y + ((o >> 1) & 1), 2 * z + (o >> 2));
      continue;
    }
    g.level.push_back(l);
    g.coord.insert(g.coord.end(), {x, y, z});
  }
  // input order must not matter: shuffle the leaves
  std::vector<int64_t> perm(g.level.size());
  for (size_t i = 0; i < perm.size(); ++i) perm[i] = (int64_t)i;
  std::shuffle(perm.begin(), perm.end(), rng);
  Grid s{{nroot[0], nroot[1], nroot[2]}, {}, {}};
  for (int64_t i : perm) {
    s.level.push_back(g.level[i]);
    s.coord.insert(s.coord.end(), {g.coord[3 * i], g.coord[3 * i + 1], g.coord[3 * i + 2]});
  }
  return s;
}

static std::string build(const Grid &g, ot::Topology &t) {
  return ot::build_topology(g.nroot, (int64_t)g.level.size(), g.level.data(), g.coord.data(), t);
}

static void check_valid(const Grid &g) {
  ot::Topology t;
  const std::string why = build(g, t);
  CHECK(why.empty());
  if (!why.empty()) {
    std::fprintf(stderr, "  reason: %s\n", why.c_str());
    return;
  }
  const int64_t nb = (int64_t)g.level.size();
  CHECK(t.nb == nb && t.nroots == (int64_t)g.nroot[0] * g.nroot[1] * g.nroot[2]);
  // ancestors: every distinct (level, coord) on the way up from the leaves
  std::set<std::tuple<int, int, int, int>> all;
  for (int64_t b = 0; b < nb; ++b) {
    int c[3] = {g.coord[3 * b], g.coord[3 * b + 1], g.coord[3 * b + 2]};
    for (int l = g.level[b]; l >= 1; --l) {
      all.emplace(l, c[0], c[1], c[2]);
      for (int k = 0; k < 3; ++k) c[k] >>= 1;
    }
  }
  CHECK(t.na == (int64_t)all.size());
  // (level, key) order and per-level ranges
  for (int64_t i = 1; i < t.na; ++i)
    CHECK(t.alev[i - 1] < t.alev[i] || (t.alev[i - 1] == t.alev[i] && t.akey[i - 1] < t.akey[i]));
  for (int l = 1; l <= t.lmax; ++l) {
    CHECK(t.level_begin[l] <= t.level_begin[l + 1]);
    for (int64_t i = t.level_begin[l]; i < t.level_begin[l + 1]; ++i) CHECK(t.alev[i] == l);
  }
  // leaves map both ways; internal nodes have 8 contiguous children one level down
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t a = t.bamr[b];
    CHECK(a >= 0 && a < t.na && t.aleaf[a] == b && t.alev[a] == g.level[b]);
  }
  for (int64_t i = 0; i < t.na; ++i) {
    if (t.aleaf[i] >= 0) {
      for (int o = 0; o < 8; ++o) CHECK(t.achild[8 * i + o] == -1);
      continue;
    }
    for (int o = 0; o < 8; ++o) {
      const int64_t c = t.achild[8 * i + o];
      CHECK(c == t.achild[8 * i] + o && c >= 0 && c < t.na && t.alev[c] == t.alev[i] + 1);
      for (int k = 0; k < 3; ++k) CHECK(t.acoord[3 * c + k] == 2 * t.acoord[3 * i + k] + ((o >> k) & 1));
    }
  }
}

static void check_invalid(Grid g, const char *what) {
  ot::Topology t;
  const std::string why = build(g, t);
  CHECK(!why.empty());
  if (why.empty()) std::fprintf(stderr, "  accepted an invalid grid: %s\n", what);
}

int main() {
  std::mt19937_64 rng(7);
  const int32_t shapes[4][3] = {{1, 1, 1}, {2, 1, 3}, {1, 1, 4}, {3, 2, 1}};
  for (int trial = 0; trial < 24; ++trial) {
    const int32_t *nr = shapes[trial % 4];
    check_valid(random_grid(rng, nr, 0.15 + 0.03 * (trial % 8), 2 + trial % 5));
  }
  // deepest supported level: the corner block refined at every level down to 15
  {
    Grid g{{1, 1, 1}, {}, {}};
    for (int l = 2; l <= 15; ++l)
      for (int o = 1; o < 8; ++o) {
        g.level.push_back(l);
        g.coord.insert(g.coord.end(), {o & 1, (o >> 1) & 1, o >> 2});
      }
    g.level.push_back(15);
    g.coord.insert(g.coord.end(), {0, 0, 0});
    check_valid(g);
  }
  const int32_t one[3] = {1, 1, 1};
  Grid base{{1, 1, 1}, {}, {}};  // the unit root refined once
  for (int o = 0; o < 8; ++o) {
    base.level.push_back(2);
    base.coord.insert(base.coord.end(), {o & 1, (o >> 1) & 1, o >> 2});
  }
  check_valid(base);
  {
    Grid g = base;  // duplicate
    g.level.push_back(2);
    g.coord.insert(g.coord.end(), {0, 0, 0});
    check_invalid(g, "duplicate");
  }
  {
    Grid g = base;  // a child of an existing leaf
    g.level.push_back(3);
    g.coord.insert(g.coord.end(), {0, 0, 0});
    check_invalid(g, "overlap");
  }
  {
    Grid g = base;  // a hole
    g.level.pop_back();
    g.coord.resize(g.coord.size() - 3);
    check_invalid(g, "hole");
  }
  {
    Grid g = base;
    g.level[0] = 0;
    check_invalid(g, "level 0");
    g.level[0] = 16;
    check_invalid(g, "level 16");
  }
  {
    Grid g = base;
    g.coord[0] = 2;
    check_invalid(g, "coordinate past the root");
    g.coord[0] = -1;
    check_invalid(g, "negative coordinate");
  }
  {
    Grid g = base;
    g.nroot[1] = 0;
    check_invalid(g, "nroot 0");
    g.nroot[1] = 65;
    check_invalid(g, "nroot 65");
  }
  {
    Grid g{{2, 1, 1}, {}, {}};  // a root block missing
    g.level.push_back(1);
    g.coord.insert(g.coord.end(), {0, 0, 0});
    check_invalid(g, "missing root");
  }
  {
    ot::Topology t;
    CHECK(!ot::build_topology(one, 0, nullptr, nullptr, t).empty());
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("topology driver: all checks passed\n");
  return 0;
}
