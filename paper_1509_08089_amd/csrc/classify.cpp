// Motif classification tables for the sampling kernels.
//
// Motif ids follow the paper's numbering, which is fixed by the constants it
// prints for each class (phi^(1), phi^(2) of Section 4.1.2 for 4 nodes; Table 2
// for 5 nodes).  A connected graph on 4 or 5 nodes is identified here by its
// sorted degree sequence together with its number of triangles, which separates
// all 6 four-node and all 21 five-node classes; the key of each id below is the
// one of the graph whose Table 2 constants carry that id.
//
// A kernel knows which edges its sample contains by construction and probes the
// remaining pairs; the probe bits index a table built here.
#include <algorithm>
#include <array>
#include <cstring>
#include <stdexcept>

#include "internal.h"

namespace moss {
namespace {

struct ClassKey {
  int id;
  std::array<int, 5> deg;  // descending, unused entries 0
  int triangles;
};

// 4 nodes: M1 3-path, M2 3-star, M3 4-cycle, M4 triangle with a pendant, M5 diamond, M6 K4.
constexpr ClassKey kKeys4[6] = {
    {1, {2, 2, 1, 1, 0}, 0}, {2, {3, 1, 1, 1, 0}, 0}, {3, {2, 2, 2, 2, 0}, 0},
    {4, {3, 2, 2, 1, 0}, 1}, {5, {3, 3, 2, 2, 0}, 2}, {6, {3, 3, 3, 3, 0}, 4},
};

// 5 nodes (Table 2 columns 1..21).
constexpr ClassKey kKeys5[21] = {
    {1, {2, 2, 2, 1, 1}, 0},  {2, {4, 1, 1, 1, 1}, 0},  {3, {3, 2, 1, 1, 1}, 0},  {4, {3, 2, 2, 2, 1}, 1},
    {5, {3, 2, 2, 2, 1}, 0},  {6, {2, 2, 2, 2, 2}, 0},  {7, {3, 3, 2, 1, 1}, 1},  {8, {4, 2, 2, 1, 1}, 1},
    {9, {3, 3, 3, 2, 1}, 2},  {10, {3, 3, 2, 2, 2}, 1}, {11, {4, 3, 2, 2, 1}, 2}, {12, {4, 2, 2, 2, 2}, 2},
    {13, {3, 3, 2, 2, 2}, 0}, {14, {4, 3, 3, 2, 2}, 3}, {15, {4, 3, 3, 3, 1}, 4}, {16, {4, 4, 2, 2, 2}, 3},
    {17, {3, 3, 3, 3, 2}, 2}, {18, {4, 3, 3, 3, 3}, 4}, {19, {4, 4, 3, 3, 2}, 5}, {20, {4, 4, 4, 3, 3}, 7},
    {21, {4, 4, 4, 4, 4}, 10},
};

int class_of_adjacency(int k, const bool adj[5][5]) {
  std::array<int, 5> deg{0, 0, 0, 0, 0};
  int tri = 0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      if (adj[i][j]) ++deg[i];
  for (int a = 0; a < k; ++a)
    for (int b = a + 1; b < k; ++b)
      for (int c = b + 1; c < k; ++c)
        if (adj[a][b] && adj[b][c] && adj[a][c]) ++tri;
  std::sort(deg.begin(), deg.end(), [](int x, int y) { return x > y; });
  const ClassKey* keys = k == 4 ? kKeys4 : kKeys5;
  const int nk = k == 4 ? 6 : 21;
  for (int i = 0; i < nk; ++i)
    if (keys[i].deg == deg && keys[i].triangles == tri) return keys[i].id;
  return -1;
}

struct Pair {
  int a, b;
};

// Builds a table: `known` edges are present in every sample, `probe[i]` is the pair
// tested by bit i of the kernel's mask.
void build_lut(int k, const Pair* known, int nknown, const Pair* probe, int nprobe, uint8_t* lut) {
  for (int mask = 0; mask < (1 << nprobe); ++mask) {
    bool adj[5][5] = {};
    for (int i = 0; i < nknown; ++i) adj[known[i].a][known[i].b] = adj[known[i].b][known[i].a] = true;
    for (int i = 0; i < nprobe; ++i)
      if (mask >> i & 1) adj[probe[i].a][probe[i].b] = adj[probe[i].b][probe[i].a] = true;
    const int c = class_of_adjacency(k, adj);
    if (c < 1) throw std::logic_error("sample structure is not a connected motif");
    lut[mask] = (uint8_t)c;
  }
}

}  // namespace

// Node order in every sample: v = 0, u = 1, w = 2, r = 3, t = 4.
void class_luts(uint8_t lut4[8], uint8_t lut5t[64], uint8_t lut5p[64]) {
  // MOSS-4: known v-u, v-w, u-r; probes u~w, v~r, w~r
  const Pair k4[] = {{0, 1}, {0, 2}, {1, 3}};
  const Pair p4[] = {{1, 2}, {0, 3}, {2, 3}};
  build_lut(4, k4, 3, p4, 3, lut4);
  // T-5: known v-u, v-w, v-r, u-t; probes u~w, u~r, w~r, v~t, w~t, r~t
  const Pair kt[] = {{0, 1}, {0, 2}, {0, 3}, {1, 4}};
  const Pair pt[] = {{1, 2}, {1, 3}, {2, 3}, {0, 4}, {2, 4}, {3, 4}};
  build_lut(5, kt, 4, pt, 6, lut5t);
  // Path-5: known v-u, v-w, u-r, w-t; probes v~r, v~t, u~w, u~t, w~r, r~t
  const Pair kp[] = {{0, 1}, {0, 2}, {1, 3}, {2, 4}};
  const Pair pp[] = {{0, 3}, {0, 4}, {1, 2}, {1, 4}, {2, 3}, {3, 4}};
  build_lut(5, kp, 4, pp, 6, lut5p);
}

}  // namespace moss

extern "C" moss_status moss_class_lut(int32_t sampler, uint8_t* out, int32_t len) {
  if (!out) return MOSS_E_ARG;
  uint8_t l4[8], lt[64], lp[64];
  try {
    moss::class_luts(l4, lt, lp);
  } catch (...) {
    return MOSS_E_ARG;
  }
  if ((sampler == MOSS_SAMPLER_MOSS4 || sampler == MOSS_SAMPLER_MOSS4MIN) && len == 8) std::memcpy(out, l4, 8);
  else if (sampler == MOSS_SAMPLER_T5 && len == 64) std::memcpy(out, lt, 64);
  else if (sampler == MOSS_SAMPLER_PATH5 && len == 64) std::memcpy(out, lp, 64);
  else return MOSS_E_ARG;
  return MOSS_OK;
}
