// Host set-up of the owner-tile layout (see kernels.h, OwnerTile).
//
// Nodes carry internal ids in first-touch order along the cell sequence, so a
// run of consecutive ids is a spatially compact set.  Tile t owns the ids
// [t*T, (t+1)*T).  Its work is every regular 8-node cell (a pattern with a Walsh table, identity
// orientation) that touches an owned node; for each such cell only the rows of
// owned corners are accumulated.  Hanging-node cells are not staged here: they
// have a pass of their own, whose rows reach the owning tiles as (dof, result)
// pairs (set up with the mesh).
//
// The regular cells form the items: one scale class (Walsh table, level, material) per item
// so the pre-scaled Walsh table is uniform in a wave, full waves of cells in
// cell (Morton) order (the item's mask is the union of the cells' owned-corner
// masks), and the eight local node indices of a cell stored together (16 bytes,
// lane-major).
#include <algorithm>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tiling.h"

namespace sbfem {

namespace {

template <class F>
void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 64) nt = 1;
  std::vector<std::thread> th;
  for (unsigned w = 0; w < nt; ++w)
    th.emplace_back([&, w] {
      for (int64_t i = w; i < n; i += nt) f(i);
    });
  for (auto& t : th) t.join();
}

struct TileOut {
  std::vector<int32_t> local;      // global ids of local nodes (owned first)
  std::vector<CellItem> items;     // offsets relative to this tile
  std::vector<uint16_t> lidx;
  std::vector<LoadEntry> loads;
  bool pure8 = true;  // no hanging-node cell
};

}  // namespace

bool build_owner_tiles(const TilingInput& in, int32_t tile_nodes, TilingOutput& out) {
  const int64_t N = in.n_nodes, C = in.n_cells;
  // node -> cells (internal ids), cells in increasing order
  std::vector<int64_t> nptr(N + 1, 0);
  for (int64_t i = 0; i < in.cptr[C]; ++i) nptr[in.conn[i] + 1]++;
  for (int64_t n = 0; n < N; ++n) nptr[n + 1] += nptr[n];
  std::vector<int32_t> ncell(nptr[N]);
  {
    std::vector<int64_t> pos(nptr.begin(), nptr.end() - 1);
    for (int64_t c = 0; c < C; ++c)
      for (int64_t i = in.cptr[c]; i < in.cptr[c + 1]; ++i) ncell[pos[in.conn[i]]++] = (int32_t)c;
  }
  // scale class of every regular cell: (Walsh table, level, material) in order of first use
  auto is_regular = [&](int64_t c) { return in.regular && in.regular[in.pattern[c]] >= 0; };
  std::vector<int32_t> cls(in.regular ? C : 0, -1);
  out = TilingOutput();
  if (in.regular) {
    std::unordered_map<int32_t, int32_t> seen;
    for (int64_t c = 0; c < C; ++c) {
      if (!is_regular(c)) continue;
      const int32_t key = ((int32_t)in.regular[in.pattern[c]] << 16) | ((int32_t)in.level[c] << 8) | in.material[c];
      auto it = seen.find(key);
      if (it == seen.end()) {
        it = seen.emplace(key, (int32_t)out.scale_keys.size()).first;
        out.scale_keys.push_back(key);
      }
      cls[c] = it->second;
    }
  }
  // load entries by node
  std::unordered_map<int64_t, double> bmap;
  for (size_t i = 0; i < in.load_dof.size(); ++i) bmap[in.load_dof[i]] += in.load_val[i];

  const int64_t n_tiles = (N + tile_nodes - 1) / tile_nodes;
  std::vector<TileOut> res(n_tiles);
  parallel_for(n_tiles, [&](int64_t t) {
    TileOut& r = res[t];
    const int64_t own0 = t * tile_nodes, own1 = std::min<int64_t>(N, own0 + tile_nodes);
    std::vector<int32_t> cells;
    for (int64_t n = own0; n < own1; ++n)
      for (int64_t i = nptr[n]; i < nptr[n + 1]; ++i) cells.push_back(ncell[i]);
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    // local numbering: owned nodes first (in id order), then others on first sight
    for (int64_t n = own0; n < own1; ++n) r.local.push_back((int32_t)n);
    std::unordered_map<int32_t, int32_t> other;
    struct CellRec { int32_t c; uint32_t mask; int32_t pattern; };
    std::vector<CellRec> recs;
    std::vector<uint16_t> li_flat;
    std::vector<int64_t> li_off(cells.size() + 1, 0);
    for (size_t j = 0; j < cells.size(); ++j) {
      const int32_t c = cells[j];
      uint32_t mask = 0;
      if (!is_regular(c)) {  // hanging-node cell: not staged in this tile
        r.pure8 = false;
        li_off[j + 1] = (int64_t)li_flat.size();
        continue;
      }
      for (int64_t i = in.cptr[c]; i < in.cptr[c + 1]; ++i) {
        const int32_t g = in.conn[i];
        int32_t l;
        if (g >= own0 && g < own1) {
          l = (int32_t)(g - own0);
          mask |= 1u << (i - in.cptr[c]);
        } else {
          auto it = other.find(g);
          if (it == other.end()) {
            l = (int32_t)r.local.size();
            other.emplace(g, l);
            r.local.push_back(g);
          } else {
            l = it->second;
          }
        }
        li_flat.push_back((uint16_t)l);
      }
      li_off[j + 1] = (int64_t)li_flat.size();
      recs.push_back({(int32_t)j, mask, (int32_t)in.pattern[c]});
    }
    // regular 8-node cells: items of one scale class in cell (Morton) order, so that the lanes
    // of a wave hold neighbouring cells and their corner nodes spread over the LDS banks; full
    // waves with the union of the cells' owned-corner masks.  The other cells of the tile
    // (hanging-node cells) are handled by the hanging-cell pass.
    std::vector<CellRec> r8;
    for (const auto& rc : recs) r8.push_back({rc.c, rc.mask, cls[cells[rc.c]]});
    std::stable_sort(r8.begin(), r8.end(), [](const CellRec& a, const CellRec& b) { return a.pattern < b.pattern; });
    size_t i0 = 0;
    while (i0 < r8.size()) {
      size_t i1 = i0;
      while (i1 < r8.size() && i1 - i0 < (size_t)kWave && r8[i1].pattern == r8[i0].pattern) ++i1;
      CellItem it{};
      it.lidx0 = (int64_t)r.lidx.size();
      it.koff = (int64_t)kWalshC * r8[i0].pattern;
      it.count = (int32_t)(i1 - i0);
      it.mask = 0;
      for (size_t b = i0; b < i1; ++b) {
        it.mask |= r8[b].mask;
        for (int k = 0; k < 8; ++k) r.lidx.push_back(li_flat[li_off[r8[b].c] + k]);
      }
      r.items.push_back(it);
      i0 = i1;
    }
    for (int64_t n = own0; n < own1; ++n)
      for (int a = 0; a < 3; ++a) {
        auto it = bmap.find(3 * n + a);
        if (it != bmap.end()) r.loads.push_back({(int32_t)(3 * (n - own0) + a), 0, it->second});
      }
  });

  // concatenate in tile order.  Halo lists at a fixed stride (the largest halo) when the
  // padding costs at most half the lists again: then a block finds its halo ids from its
  // tile index alone, without waiting for the tile record.
  out.tile_nodes = tile_nodes;
  int64_t halo_max = 0, halo_sum = 0;
  for (int64_t t = 0; t < n_tiles; ++t) {
    const int64_t n_own = std::min<int64_t>(tile_nodes, N - t * tile_nodes);
    const int64_t h = (int64_t)res[t].local.size() - n_own;
    halo_max = std::max(halo_max, h);
    halo_sum += h;
  }
  const int64_t stride = std::max<int64_t>(1, halo_max);
  out.halo_stride = n_tiles * stride <= halo_sum + halo_sum / 2 + (1 << 20) ? stride : 0;
  out.local_entries = halo_sum + N;
  for (int64_t t = 0; t < n_tiles; ++t) {
    TileOut& r = res[t];
    OwnerTile ot{};
    ot.own0 = t * tile_nodes;
    ot.n_own = (int32_t)std::min<int64_t>(tile_nodes, N - ot.own0);
    ot.node0 = out.halo_stride ? t * out.halo_stride : (int64_t)out.nodelist.size();
    ot.n_local = (int32_t)r.local.size();
    ot.item0 = (int64_t)out.items.size();
    ot.n_items = (int32_t)r.items.size();
    ot.load0 = (int32_t)out.loads.size();
    ot.n_load = (int32_t)r.loads.size();
    out.max_local = std::max<int64_t>(out.max_local, ot.n_local);
    if (ot.n_local > 65535) return false;
    const int64_t lbase = (int64_t)out.lidx.size();
    for (auto it : r.items) {
      it.lidx0 += lbase;
      out.items.push_back(it);
    }
    // owned nodes are implicit (own0 + i); only the others are listed
    out.nodelist.insert(out.nodelist.end(), r.local.begin() + ot.n_own, r.local.end());
    if (out.halo_stride) out.nodelist.resize((size_t)((t + 1) * out.halo_stride), -1);
    out.lidx.insert(out.lidx.end(), r.lidx.begin(), r.lidx.end());
    out.loads.insert(out.loads.end(), r.loads.begin(), r.loads.end());
    out.tiles.push_back(ot);
    if (r.pure8)
      out.n_pure8++;
    else
      out.n_mixed++;
    r = TileOut();
  }
  return true;
}

}  // namespace sbfem
