// Internal interface between the C-ABI host code and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbfem {

constexpr int kTile = 256;  // cells per block (one cell per thread)
constexpr int kWave = 64;

struct LoadParams {
  int32_t kind;
  int32_t cycles;
  double t1;
  double P0;
  const double* table;  // kind 3: P(t_n) per step n (device), n < n_table
  int64_t n_table;
  double dt;            // kind 3: step of the table (t_n = n dt)
};

// Owner tile: a block updates the nodes [own0, own0 + n_own) (internal ids).
// Its local nodes are the owned ones (local i < n_own is node own0 + i) followed
// by the other nodes its regular cells touch (local i >= n_own is
// nodelist[node0 + i - n_own]); u of all of them is staged in LDS.  The forces of
// hanging-node cells on its owned dofs arrive as n_hpair (owned dof, result)
// pairs at hpairs[hpair0...] into the hanging-cell pass's results.
struct OwnerTile {
  int64_t node0;
  int64_t own0;
  int64_t item0;
  int64_t hpair0;
  int32_t n_own;
  int32_t n_local;
  int32_t n_items;
  int32_t load0;
  int32_t n_load;
  int32_t n_hpair;
};

// A force of a hanging-node cell on an owned dof of a tile: hres[res] added to local dof ldof.
struct HangPair {
  int32_t ldof;
  uint32_t res;
};

// Hanging-node cells (every cell that is not a regular 8-node cell), each once, in items of
// up to a wave of cells of one pattern: cell i of the item is hanging cell cell0 + i, its
// node k is hconn[conn0 + k * count + i] (internal ids); the force of its master row r
// (oriented, scaled) goes to hres[res0 + r * 64 + i].
struct HangItem {
  int64_t cell0;
  int64_t conn0;
  int64_t koff;     // master matrix offset
  int64_t res0;
  int32_t nn;
  int32_t count;
};

// Up to one wave of regular 8-node cells of one scale class (identity orientation) in an owner
// tile; rows of owned corners are accumulated (mask: union of the cells' owned corners).
// Local node indices lane-major, lidx[lidx0 + 8*lane + k] (lidx0 a multiple of 8),
// koff = kWalshC * scale class.
struct CellItem {
  int64_t lidx0;
  int64_t koff;
  int32_t count;
  uint32_t mask;
};

// Entries per scale class of the structured Walsh table of the 8-node cell (31 used).
constexpr int kWalshC = 32;

struct LoadEntry {
  int32_t ldof;    // 3 * local owned node + axis
  int32_t pad;
  double val;
};

struct TiledArgs {
  const OwnerTile* tiles;
  int64_t n_tiles;
  const CellItem* items;
  const uint16_t* lidx;
  const int32_t* nodelist;
  const LoadEntry* loads;
  const double* matE;
  double h0;
  const double* K64;
  const float* K32;     // FP32 products: K in FP32; 16-bit products: K rounded to FP16 / BF16, held in FP32
  const double* Ws64;   // 8-node cell: structured Walsh table times s_e, kWalshC per scale class
  const float* Ws32;    // (16-bit products: the unscaled table rounded to 16 bits, s_e in the last entry)
  const void* u;        // u_n        (state storage, see `state`)
  void* um1;            // u_{n-1} in, u_{n+1} out (owned nodes)
  const void* minv;     // inverse lumped mass per dof (FP64, or FP32 with FP32 state; 0 on fixed dofs)
  double* f;            // force-only mode: R_int of owned dofs written here
  unsigned long long* flag;    // smallest step n whose update gave a non-finite u_{n+1} (~0: none)
  // probe histories (n_probes = 0: none): tile t records the entries [probe_ptr[t], probe_ptr[t+1])
  // of `probes` (x: 3 * local owned node + axis, y: probe slot); step n's u_{n+1} and
  // (u_{n+1} - 2 u_n + u_{n-1}) / dt^2 go to row n - probe_step0 (< probe_rows) of probe_u, probe_a
  const int32_t* probe_ptr;
  const int2* probes;
  double* probe_u;
  double* probe_a;
  int64_t probe_step0;
  int64_t probe_rows;
  int32_t n_probes;
  const HangItem* hitems;      // hanging-cell pass
  const int32_t* hconn;
  const uint8_t* horient;
  const uint8_t* hlevel;
  const uint8_t* hmaterial;
  const HangPair* hpairs;      // per tile, its (owned dof, result) pairs
  void* hres;                  // forces of the hanging cells' rows, rewritten every step (FP64 for
                               // FP64 products, else FP32)
  int64_t ndof;         // dofs of the mesh (offset of the low parts of compensated state)
  int32_t state;        // 0 FP64, 1 FP32, 2 compensated FP32 pair (hi at u[i], lo at u[ndof + i])
  int32_t round16;      // 16-bit product operands: 0 none, 1 FP16 (per-cell power-of-two scale), 2 BF16
  LoadParams L;         // P(t) of the load vector
  double dt;
  double dt2;
  double c;             // alpha dt / 2
  int32_t lds_bytes;    // dynamic LDS: 3 FP64 forces per owned node + 3 u values per local node
  int64_t tile_nodes;   // tile t owns nodes [t tile_nodes, (t + 1) tile_nodes) (the last: up to the end)
  int64_t halo_stride;  // > 0: the halo ids of tile t start at nodelist[t halo_stride], -1 padded
  int32_t block_threads;        // owner-tile pass: 64..512, multiple of 64
  int32_t block_threads_mixed;  // hanging-cell pass (one wave per item)
};

// A block's work: up to kTile consecutive cells of one pattern segment.
struct Tile {
  int64_t cell0;   // first cell (index into the sorted per-cell arrays)
  int64_t conn0;   // conn index of slot 0 of the first cell
  int64_t stride;  // cells in the segment (distance between slots of one cell)
  int64_t koff;    // offset of the pattern's master matrix (entries)
  int32_t count;   // cells in this tile (1..kTile)
  int32_t nn;      // nodes per cell of the pattern
};

// Tiles of one launch group: n_fixed8 tiles of 8-node cells, then n_mixed tiles of larger cells.
struct TileRange {
  int64_t first;
  int64_t n_fixed8;
  int64_t n_mixed;
};

struct ElementArgs {
  const Tile* tiles;
  const double* u;
  double* f;
  const int32_t* conn;
  const uint8_t* orient;
  const uint8_t* level;
  const uint8_t* material;
  const double* matE;
  double h0;
  const double* K64;
  const float* K32;
};

// Optional per-class event hook: called before (begin=true) and after each launch.
struct LaunchHook {
  void (*fn)(void* ctx, int cls, bool begin, hipStream_t s) = nullptr;
  void* ctx = nullptr;
  void operator()(int cls, bool begin, hipStream_t s) const {
    if (fn) fn(ctx, cls, begin, s);
  }
};

hipError_t launch_ebe(const ElementArgs& a, const TileRange& r, bool fp32, bool atomic, hipStream_t s,
                      const LaunchHook& hook = LaunchHook());
// A mesh in a tiled launch: its two argument blocks (u and u_prev swap roles every step),
// the step number of the launch and which block holds the current roles.
struct MeshRef {
  const TiledArgs* args;  // device, 2 entries
  int64_t step;
  int32_t parity;
  int32_t pad;
};
// (mesh, tile) of a batched launch
struct TileWork {
  int32_t mesh;
  int32_t pad;
  int64_t tile;
};

// Launch description: one mesh (work lists null; its ref is `single`, or refs[0] on the
// device when refs is set) or a batch (refs + work lists).  A step is two passes: the
// hanging-node cells (items [0, n_hang)), then every owner tile (tiles [0, n_tiles)).  In a
// batch, TileWork::tile is the item or tile index.  Launches read step and parity of the
// ref plus k; refs on the device (not `single`) let a captured graph replay at any step.
struct TiledLaunch {
  MeshRef single;
  const MeshRef* refs = nullptr;
  const TileWork* work8 = nullptr;     // batch: every owner tile of every mesh
  const TileWork* work_hang = nullptr; // batch: every hanging-cell item of every mesh
  int64_t n_tiles = 0, n_hang = 0;
  int64_t k = 0;                       // batch: steps since the refs were recorded
  bool fp32 = false;
  bool reduced = false;                // FP32 or compensated state, or 16-bit products
  int32_t prec = 0;                    // hanging-cell pass: sbfem_prod of the products
  int32_t state = 0;                   // hanging-cell pass: sbfem_state of u
  bool hang_mma = true;                // hanging-cell pass on the matrix cores (else one lane per cell)
  bool force_only = false;
  int32_t threads8 = 512, threads_mixed = 256;
  size_t lds = 0;                      // owner-tile pass
  size_t lds_hang = 0;                 // hanging-cell pass
};

hipError_t launch_tiled(const TiledLaunch& L, hipStream_t s, const LaunchHook& hook = LaunchHook());
// per-unit launchers
void ebe8_launch(const ElementArgs& a, const Tile* tiles, int64_t n, bool fp32, bool atomic, hipStream_t s);
void ebe_mixed_fp64_launch(const ElementArgs& a, const Tile* tiles, int64_t n, bool atomic, hipStream_t s);
void ebe_mixed_fp32_launch(const ElementArgs& a, const Tile* tiles, int64_t n, bool atomic, hipStream_t s);
void owner_pass_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
// owner-tile pass per product precision (one translation unit each), the state storage by L.state
void owner_fp64_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void owner_fp32_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void owner_fp16_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void owner_bf16_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void tiled_hang_fp64_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void tiled_hang_fp32_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void tiled_hang_fp64r_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
void tiled_hang_fp32r_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s);
// hanging-cell pass on the matrix cores, one translation unit per product precision
void hang_mma_fp64_launch(const TiledLaunch& L, const TileWork* work, int64_t count, hipStream_t s);
void hang_mma_fp32_launch(const TiledLaunch& L, const TileWork* work, int64_t count, hipStream_t s);
void hang_mma_fp16_launch(const TiledLaunch& L, const TileWork* work, int64_t count, hipStream_t s);
void hang_mma_bf16_launch(const TiledLaunch& L, const TileWork* work, int64_t count, hipStream_t s);
// LDS bytes of a matrix-core hanging-pass block for a master of nd dofs in precision prec
int hang_mma_lds_bytes(int prec, int nd);

hipError_t launch_load(double* f, const int64_t* idx, const double* val, int64_t nnz, const LoadParams& L,
                       double t, hipStream_t s);
// u_{n+1} = (dt2 M^-1 (-f) + 2 u_n - (1 - c) u_{n-1}) / (1 + c) over u_{n-1}, f cleared; a non-finite
// result lowers *flag to `step` (atomic minimum)
hipError_t launch_update(const double* un, double* unm1, double* f, const double* minv, int64_t ndof,
                         double dt2, double c, unsigned long long* flag, int64_t step, hipStream_t s);
hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t s);
// refs[0..n): step += steps, parity flipped when steps is odd (graph-safe: a kernel)
hipError_t launch_refs_advance(MeshRef* refs, int32_t n, int64_t steps, hipStream_t s);
hipError_t launch_ref_set(MeshRef* ref, const MeshRef& v, hipStream_t s);

// Dense kernels of the eigenvalue solver: n x p blocks stored column after column, FP64;
// reductions in a fixed order.
hipError_t launch_gram(const double* X, const double* Y, int64_t n, int p, double* G, hipStream_t s);  // G = X^T Y
hipError_t launch_gemm_small(const double* X, int64_t n, int p, const double* Q, int q, double* Y,
                             hipStream_t s);                                                      // Y = X Q
hipError_t launch_scale_cols(const double* S, const double* X, double* Y, int64_t n, int p, hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n, hipStream_t s);
hipError_t launch_axpbypcz(double a, const double* x, double b, const double* y, double c, double* z, int64_t n,
                           hipStream_t s);
hipError_t launch_vmul(const double* sc, const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_ritz_residual(const double* X, const double* AX, int64_t n, int p, const double* theta,
                                double* out, hipStream_t s);  // out[j] = |AX_j - theta_j X_j|^2

}  // namespace sbfem
