"""The owner-tile layout (host index work of the tiled assembly), checked exactly on the CPU.

The library's tiling code is compiled here with g++ (with a small harness,
`tests/native/tiling_probe.cpp`) and run on generated meshes.  Every output is
index work, so every check is exact:

* tile t owns nodes [t T, (t + 1) T) (the last tile up to the end);
* its halo lists name nodes it does not own, once each, padded with -1 to the
  fixed stride when one is used;
* the regular 8-node cells of tile t's items are exactly the regular cells that
  touch a node of t, once each, in corner order, in increasing cell order
  within an item, one scale class (level, material) per item, at most a wave
  per item, and the item mask is the union of the cells' owned corners;
* over all tiles every corner of every regular cell is owned exactly once (so
  no force row is dropped or added twice), and hanging-node cells appear in no
  item (they have a pass of their own);
* load entries sit in the tile that owns their dof, with the summed value.
"""

import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from meshgen import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2103_09100_amd", "csrc")

TILE = np.dtype([("node0", "<i8"), ("own0", "<i8"), ("item0", "<i8"), ("hpair0", "<i8"), ("n_own", "<i4"),
                 ("n_local", "<i4"), ("n_items", "<i4"), ("load0", "<i4"), ("n_load", "<i4"), ("n_hpair", "<i4")])
ITEM = np.dtype([("lidx0", "<i8"), ("koff", "<i8"), ("count", "<i4"), ("mask", "<u4")])
LOAD = np.dtype([("ldof", "<i4"), ("pad", "<i4"), ("val", "<f8")])


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    d = tmp_path_factory.mktemp("tiling")
    so = str(d / "libtiling_probe.so")
    cmd = ["g++", "-std=c++17", "-O2", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + CSRC, os.path.join(ROOT, "tests", "native", "tiling_probe.cpp"), os.path.join(CSRC, "tiling.cpp"),
           "-o", so, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = C.CDLL(so)
    sizes = (C.c_int64 * 3)()
    lib.tiling_struct_sizes(sizes)
    assert list(sizes) == [TILE.itemsize, ITEM.itemsize, LOAD.itemsize]
    return lib


def internal_mesh(mesh):
    """First-touch node numbering along the cell order (what the library does), cells of
    the 8-node pattern marked; arrays as the tiling takes them."""
    conn = np.asarray(mesh.conn, dtype=np.int64)
    ptr = np.asarray(mesh.conn_ptr, dtype=np.int64)
    N = int(mesh.n_nodes)
    first = np.full(N, -1, dtype=np.int64)
    order = []
    for g in conn:
        if first[g] < 0:
            first[g] = len(order)
            order.append(g)
    for g in range(N):
        if first[g] < 0:
            first[g] = len(order)
            order.append(g)
    iconn = first[conn].astype(np.int32)
    nn = np.diff(ptr)
    pattern = np.where(nn == 8, 0, 1).astype(np.uint16)  # 0: regular 8-node cell
    load_dof = np.asarray(mesh.load_dof, dtype=np.int64)
    load_dof = 3 * first[load_dof // 3] + load_dof % 3
    return dict(N=N, ptr=ptr, conn=iconn, pattern=pattern, level=np.asarray(mesh.cell_level, dtype=np.uint8),
                material=np.asarray(mesh.cell_mat, dtype=np.uint8), load_dof=load_dof,
                load_val=np.asarray(mesh.load_val, dtype=np.float64))


def run_tiling(lib, m, tile_nodes):
    P = C.c_void_p
    ok = lib.tiling_run(C.c_int64(m["N"]), C.c_int64(len(m["ptr"]) - 1), P(m["ptr"].ctypes.data),
                        P(m["conn"].ctypes.data), P(m["pattern"].ctypes.data), P(m["level"].ctypes.data),
                        P(m["material"].ctypes.data), C.c_int32(0), C.c_int64(len(m["load_dof"])),
                        P(m["load_dof"].ctypes.data), P(m["load_val"].ctypes.data), C.c_int32(tile_nodes))
    assert ok == 1
    s = (C.c_int64 * 12)()
    lib.tiling_sizes(s)
    s = list(s)
    out = dict(tiles=np.zeros(s[0], TILE), items=np.zeros(s[1], ITEM), lidx=np.zeros(s[2], np.uint16),
               nodelist=np.zeros(s[3], np.int32), loads=np.zeros(s[4], LOAD), scale_keys=np.zeros(s[5], np.int32))
    lib.tiling_copy(*[P(out[k].ctypes.data) for k in ("tiles", "items", "lidx", "nodelist", "loads", "scale_keys")])
    out.update(halo_stride=s[6], tile_nodes=s[7], max_local=s[8], local_entries=s[9], n_pure8=s[10], n_mixed=s[11])
    return out


def check_tiling(m, out, tn):
    N, ptr, conn = m["N"], m["ptr"], m["conn"]
    tiles, items, lidx, nodelist = out["tiles"], out["items"], out["lidx"], out["nodelist"]
    H = out["halo_stride"]
    n_tiles = -(-N // tn)
    assert out["tile_nodes"] == tn and len(tiles) == n_tiles
    assert out["n_pure8"] + out["n_mixed"] == n_tiles
    regular = np.flatnonzero(m["pattern"] == 0)
    cell_of = {tuple(conn[ptr[c]:ptr[c + 1]]): c for c in regular}
    # node -> regular cells touching it
    touching = [[] for _ in range(N)]
    for c in regular:
        for g in conn[ptr[c]:ptr[c + 1]]:
            touching[g].append(c)
    owned_rows = np.zeros(len(ptr) - 1, dtype=np.int64)
    key = m["level"].astype(np.int64) * 256 + m["material"]
    assert out["max_local"] == tiles["n_local"].max() and out["local_entries"] == tiles["n_local"].sum()
    for t in range(n_tiles):
        T = tiles[t]
        own0, n_own = int(T["own0"]), int(T["n_own"])
        assert own0 == t * tn and n_own == min(tn, N - own0)
        assert T["n_hpair"] == 0
        n_halo = int(T["n_local"]) - n_own
        if H:
            assert T["node0"] == t * H and n_halo <= H
            assert np.all(nodelist[t * H + n_halo:(t + 1) * H] == -1)
        halo = nodelist[T["node0"]:T["node0"] + n_halo].astype(np.int64)
        assert np.all((halo >= 0) & (halo < N)) and not np.any((halo >= own0) & (halo < own0 + n_own))
        assert len(np.unique(halo)) == n_halo
        local = np.concatenate([np.arange(own0, own0 + n_own), halo])
        expect = set()
        for g in range(own0, own0 + n_own):
            expect.update(touching[g])
        seen = []
        for it in items[T["item0"]:T["item0"] + T["n_items"]]:
            cnt = int(it["count"])
            assert 1 <= cnt <= 64 and it["lidx0"] % 8 == 0 and it["koff"] % 32 == 0
            k_cls = out["scale_keys"][it["koff"] // 32]
            cells, mask = [], 0
            for j in range(cnt):
                li = lidx[it["lidx0"] + 8 * j:it["lidx0"] + 8 * j + 8].astype(np.int64)
                g = local[li]
                c = cell_of[tuple(g)]
                cells.append(c)
                own = (g >= own0) & (g < own0 + n_own)
                mask |= int(sum(1 << k for k in range(8) if own[k]))
                owned_rows[c] += int(own.sum())
                assert key[c] == k_cls
            assert cells == sorted(cells)
            assert int(it["mask"]) == mask
            seen.extend(cells)
        assert len(seen) == len(set(seen)) and set(seen) == expect
        # loads of the tile
        ld = out["loads"][T["load0"]:T["load0"] + T["n_load"]]
        dofs = m["load_dof"]
        mine = (dofs >= 3 * own0) & (dofs < 3 * (own0 + n_own))
        want = {}
        for d_, v in zip(dofs[mine], m["load_val"][mine]):
            want[int(d_ - 3 * own0)] = want.get(int(d_ - 3 * own0), 0.0) + v
        got = {int(e["ldof"]): float(e["val"]) for e in ld}
        assert got.keys() == want.keys()
        for k in want:
            assert got[k] == want[k]  # summed in input order on both sides
    # every corner of every regular cell owned exactly once; hanging cells in no item
    assert np.all(owned_rows[regular] == 8)
    assert np.all(owned_rows[m["pattern"] != 0] == 0)


@pytest.mark.parametrize("which,tn", [("cfg1", 512), ("cfg1", 100), ("zoo", 512), ("zoo", 64), ("zoo", 200)])
def test_owner_tiles_exact(probe, which, tn):
    mesh = configs.cfg1() if which == "cfg1" else configs.small_zoo()
    m = internal_mesh(mesh)
    out = run_tiling(probe, m, tn)
    check_tiling(m, out, tn)
    if which == "zoo":
        assert out["n_mixed"] > 0 and np.any(m["pattern"] != 0)
