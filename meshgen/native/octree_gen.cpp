// Native core of the seeded octree mesh generator (input generation only).
//
// Given the refined-cell grids of a 2:1-balanced octree (one byte per cell and
// level), it lists the leaves along the Morton curve, finds the nodes (cell
// corners, mid-edge nodes where a finer cell has a corner, face centres by
// the face rule of the mesh format), numbers nodes in first-touch order along
// the leaf sequence and writes the natural-order connectivity.
//
// Two calls: og_build() does the work and keeps the result; og_fetch() copies
// it into caller arrays sized from the counts og_build() returned.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace {

const int CORNER[8][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1},
                          {-1, -1, 1},  {1, -1, 1},  {-1, 1, 1},  {1, 1, 1}};
const int EDGE[12][3] = {{0, -1, -1}, {0, 1, -1}, {0, -1, 1}, {0, 1, 1}, {-1, 0, -1}, {1, 0, -1},
                         {-1, 0, 1},  {1, 0, 1},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 1, 0}};
const int FACE[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

struct State {
  int lmax = 0;
  int64_t ext[3] = {0, 0, 0};  // lattice extent per axis (points = ext + 1)
  std::vector<uint8_t> level;
  std::vector<int32_t> lat;    // 3 per cell
  std::vector<uint32_t> slots;
  std::vector<int64_t> ptr;
  std::vector<int32_t> conn;
  std::vector<int32_t> node_lat;
};

State g;

inline int64_t lidx(int64_t x, int64_t y, int64_t z) { return (x * (g.ext[1] + 1) + y) * (g.ext[2] + 1) + z; }

uint32_t face_bits(uint32_t e) {
  uint32_t out = 0;
  for (int f = 0; f < 6; ++f) {
    int a = FACE[f][0] ? 0 : (FACE[f][1] ? 1 : 2);
    int nh = 0, axes[4], bits[4], n = 0;
    for (int k = 0; k < 12; ++k)
      if (EDGE[k][a] == FACE[f][a]) {
        bits[n] = (e >> k) & 1;
        axes[n] = EDGE[k][0] == 0 ? 0 : (EDGE[k][1] == 0 ? 1 : 2);
        nh += bits[n];
        ++n;
      }
    bool opp = false;
    if (nh == 2)
      for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
          if (axes[i] == axes[j] && bits[i] && bits[j]) opp = true;
    if (nh > 0 && !opp) out |= 1u << f;
  }
  return out;
}

}  // namespace

extern "C" {

// roots: root-cube counts; refined[l] (l < lmax): byte grid of shape roots*2^l (C order).
// Returns 0 and fills counts = {n_cells, n_nodes, n_conn}.
int og_build(const int64_t* roots, int lmax, const uint8_t* const* refined, int64_t* counts) {
  g = State();
  g.lmax = lmax;
  for (int a = 0; a < 3; ++a) g.ext[a] = roots[a] << lmax;

  // leaves along the Morton curve: roots in Morton order of their index, children in z-order
  std::vector<int64_t> roots_order;
  for (int64_t x = 0; x < roots[0]; ++x)
    for (int64_t y = 0; y < roots[1]; ++y)
      for (int64_t z = 0; z < roots[2]; ++z) roots_order.push_back((x << 42) | (y << 21) | z);
  auto morton = [](int64_t k) {
    uint64_t x = k >> 42, y = (k >> 21) & 0x1FFFFF, z = k & 0x1FFFFF, m = 0;
    for (int b = 0; b < 21; ++b)
      m |= (((x >> b) & 1) << (3 * b)) | (((y >> b) & 1) << (3 * b + 1)) | (((z >> b) & 1) << (3 * b + 2));
    return m;
  };
  std::sort(roots_order.begin(), roots_order.end(), [&](int64_t a, int64_t b) { return morton(a) < morton(b); });

  struct Item { int64_t x, y, z; int l; };
  std::vector<Item> stack;
  for (auto it = roots_order.rbegin(); it != roots_order.rend(); ++it)
    stack.push_back({*it >> 42, (*it >> 21) & 0x1FFFFF, *it & 0x1FFFFF, 0});
  while (!stack.empty()) {
    Item c = stack.back();
    stack.pop_back();
    bool ref = false;
    if (c.l < lmax) {
      const int64_t n1 = roots[1] << c.l, n2 = roots[2] << c.l;
      ref = refined[c.l][(c.x * n1 + c.y) * n2 + c.z] != 0;
    }
    if (ref) {
      for (int ch = 7; ch >= 0; --ch)
        stack.push_back({2 * c.x + (ch & 1), 2 * c.y + ((ch >> 1) & 1), 2 * c.z + ((ch >> 2) & 1), c.l + 1});
    } else {
      const int64_t s = 1ll << (lmax - c.l);
      g.level.push_back((uint8_t)c.l);
      g.lat.push_back((int32_t)(c.x * s));
      g.lat.push_back((int32_t)(c.y * s));
      g.lat.push_back((int32_t)(c.z * s));
    }
  }
  const int64_t C = (int64_t)g.level.size();
  const int64_t npts = (g.ext[0] + 1) * (g.ext[1] + 1) * (g.ext[2] + 1);

  // corner nodes
  std::vector<uint8_t> flag(npts, 0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < C; ++c) {
    const int64_t s = 1ll << (lmax - g.level[c]);
    for (int k = 0; k < 8; ++k)
      flag[lidx(g.lat[3 * c] + (CORNER[k][0] + 1) / 2 * s, g.lat[3 * c + 1] + (CORNER[k][1] + 1) / 2 * s,
                g.lat[3 * c + 2] + (CORNER[k][2] + 1) / 2 * s)] = 1;
  }
  // edge masks from the corners, then face centres
  g.slots.assign(C, 0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < C; ++c) {
    if (g.level[c] == lmax) continue;
    const int64_t h = (1ll << (lmax - g.level[c])) / 2;
    uint32_t e = 0;
    for (int k = 0; k < 12; ++k)
      if (flag[lidx(g.lat[3 * c] + (EDGE[k][0] + 1) * h, g.lat[3 * c + 1] + (EDGE[k][1] + 1) * h,
                    g.lat[3 * c + 2] + (EDGE[k][2] + 1) * h)])
        e |= 1u << k;
    g.slots[c] = e;
  }
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < C; ++c) {
    if (g.level[c] == lmax) continue;
    const uint32_t fb = face_bits(g.slots[c]);
    g.slots[c] |= fb << 12;
    const int64_t h = (1ll << (lmax - g.level[c])) / 2;
    for (int f = 0; f < 6; ++f)
      if ((fb >> f) & 1)
        flag[lidx(g.lat[3 * c] + (FACE[f][0] + 1) * h, g.lat[3 * c + 1] + (FACE[f][1] + 1) * h,
                  g.lat[3 * c + 2] + (FACE[f][2] + 1) * h)] = 1;
  }
  flag.clear();
  flag.shrink_to_fit();

  // connectivity pointers
  g.ptr.assign(C + 1, 0);
  for (int64_t c = 0; c < C; ++c) g.ptr[c + 1] = g.ptr[c] + 8 + __builtin_popcount(g.slots[c]);
  g.conn.assign(g.ptr[C], -1);

  // first-touch node numbering along the leaf sequence
  std::vector<int32_t> id(npts, -1);
  int32_t next = 0;
  for (int64_t c = 0; c < C; ++c) {
    const int64_t s = 1ll << (lmax - g.level[c]);
    const int64_t h = s / 2;
    int64_t q = g.ptr[c];
    auto touch = [&](int64_t x, int64_t y, int64_t z) {
      int32_t& v = id[lidx(x, y, z)];
      if (v < 0) {
        v = next++;
        g.node_lat.push_back((int32_t)x);
        g.node_lat.push_back((int32_t)y);
        g.node_lat.push_back((int32_t)z);
      }
      g.conn[q++] = v;
    };
    const int64_t x0 = g.lat[3 * c], y0 = g.lat[3 * c + 1], z0 = g.lat[3 * c + 2];
    for (int k = 0; k < 8; ++k)
      touch(x0 + (CORNER[k][0] + 1) / 2 * s, y0 + (CORNER[k][1] + 1) / 2 * s, z0 + (CORNER[k][2] + 1) / 2 * s);
    for (int k = 0; k < 12; ++k)
      if ((g.slots[c] >> k) & 1) touch(x0 + (EDGE[k][0] + 1) * h, y0 + (EDGE[k][1] + 1) * h, z0 + (EDGE[k][2] + 1) * h);
    for (int f = 0; f < 6; ++f)
      if ((g.slots[c] >> (12 + f)) & 1)
        touch(x0 + (FACE[f][0] + 1) * h, y0 + (FACE[f][1] + 1) * h, z0 + (FACE[f][2] + 1) * h);
  }
  counts[0] = C;
  counts[1] = next;
  counts[2] = g.ptr[C];
  return 0;
}

int og_fetch(uint8_t* level, int32_t* lat, uint32_t* slots, int64_t* ptr, int32_t* conn, int32_t* node_lat) {
  const size_t C = g.level.size();
  memcpy(level, g.level.data(), C);
  memcpy(lat, g.lat.data(), 12 * C);
  memcpy(slots, g.slots.data(), 4 * C);
  memcpy(ptr, g.ptr.data(), 8 * (C + 1));
  memcpy(conn, g.conn.data(), 4 * g.conn.size());
  if (node_lat) memcpy(node_lat, g.node_lat.data(), 4 * g.node_lat.size());
  g = State();
  return 0;
}

}  // extern "C"
