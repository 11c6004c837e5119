// C-ABI host implementation of the explicit octree-SBFEM stepper (see include/sbfem.h).
//
// Set-up (Alg. 1, initialisation): validate the mesh, optionally colour the
// cells (no two cells of a colour share a node), sort cells by (colour,
// pattern) into segments, lay the node ids of each segment out slot-major,
// assemble the lumped diagonal mass and the start-up point (eq. D0), and upload
// everything once.  Time loop: per step a load kernel, the element kernels of
// each colour, and the central-difference update (eq. DnMdiag).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbfem.h"
#include "kernels.h"
#include "tiling.h"

namespace {

thread_local std::string g_err;

sbfem_status fail(sbfem_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(e_ == hipErrorOutOfMemory ? SBFEM_ENOMEM : SBFEM_EDEVICE, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                     \
  } while (0)

// Device memory: hipMalloc/hipFree, or the caller's allocator (sbfem_set_allocator).  Each
// object keeps the allocator it was created with and returns its memory through it.
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* user = nullptr;
};
Allocator g_alloc;

hipError_t dalloc_bytes(const Allocator& A, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  if (A.alloc) {
    *p = A.alloc(bytes, A.user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

template <class T>
hipError_t dalloc(const Allocator& A, T** p, size_t n) {
  void* q = nullptr;
  const hipError_t e = dalloc_bytes(A, &q, n * sizeof(T));
  *p = (T*)q;
  return e;
}

template <class T>
void dfree(const Allocator& A, T*& p) {
  if (p) {
    if (A.release)
      A.release((void*)p, A.user);
    else
      (void)hipFree((void*)p);
  }
  p = nullptr;
}

// orientation code -> (pi, s), the same decoding as the device code
void decode(int code, int pi[3], double s[3]) {
  const int p = code >> 3;
  pi[0] = p >> 1;
  const int lo = (pi[0] == 0) ? 1 : 0;
  const int hi = (pi[0] == 2) ? 1 : 2;
  pi[1] = (p & 1) ? hi : lo;
  pi[2] = (p & 1) ? lo : hi;
  for (int a = 0; a < 3; ++a) s[a] = ((code >> a) & 1) ? -1.0 : 1.0;
}

// corner k = i + 2j + 4l of the master (at (2i-1, 2j-1, 2l-1)) is corner corner_image(k) of a cell
// in orientation (pi, s): the cell position q has q[pi(a)] = s_a p[a]
int corner_image(int k, const int pi[3], const double s[3]) {
  int n = 0;
  for (int a = 0; a < 3; ++a) {
    const int pa = ((k >> a) & 1) ? 1 : -1;
    const int q = s[a] > 0 ? pa : -pa;
    if (q > 0) n |= 1 << pi[a];
  }
  return n;
}

// 16-bit operand rounding on the host (round to nearest even), as the device does it
float round_fp16(float x) { return (float)(_Float16)x; }
float round_bf16(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  b &= 0xFFFF0000u;
  float y;
  std::memcpy(&y, &b, 4);
  return y;
}

// State arrays in device storage form (sbfem_state): FP64; FP32; compensated FP32 pair with
// hi = fl32(v) in [0, n) and lo = fl32(v - hi) in [n, 2n).
int64_t state_bytes(int mode, int64_t n) { return n * (mode == SBFEM_STATE_FP32 ? 4 : 8); }
std::vector<char> pack_state(int mode, const double* v, int64_t n) {
  std::vector<char> raw(state_bytes(mode, n));
  if (mode == SBFEM_STATE_FP64) {
    std::memcpy(raw.data(), v, n * 8);
  } else {
    float* q = (float*)raw.data();
    for (int64_t i = 0; i < n; ++i) {
      q[i] = (float)v[i];
      if (mode == SBFEM_STATE_KAHAN32) q[n + i] = (float)(v[i] - (double)q[i]);
    }
  }
  return raw;
}
void unpack_state(int mode, const char* raw, int64_t n, double* v) {
  if (mode == SBFEM_STATE_FP64) {
    std::memcpy(v, raw, n * 8);
    return;
  }
  const float* q = (const float*)raw;
  for (int64_t i = 0; i < n; ++i) v[i] = (double)q[i] + (mode == SBFEM_STATE_KAHAN32 ? (double)q[n + i] : 0.0);
}

double load_time_host(const sbfem::LoadParams& L, double t) {
  if (L.kind == SBFEM_LOAD_RICKER) {
    const double tau = (t - L.t1) / (L.t1 / 5.0);
    return (1.0 - tau * tau) * std::exp(-0.5 * tau * tau) * L.P0;
  }
  if (L.kind == SBFEM_LOAD_TRIANGLE) {
    if (t < 0.0 || t > 2.0 * L.t1) return 0.0;
    return (1.0 - std::fabs(t / L.t1 - 1.0)) * L.P0;
  }
  if (t < 0.0 || t > L.t1) return 0.0;
  const double pi = 3.14159265358979323846;
  const double w = std::sin(pi * t / L.t1);
  return std::sin(2.0 * pi * L.cycles * t / L.t1) * w * w * L.P0;
}

}  // namespace

struct sbfem_patterns {
  Allocator alloc;
  int32_t n = 0;
  int device = 0;
  std::vector<int32_t> ndof;
  std::vector<int64_t> koff, moff;
  std::vector<double> K, m, omega;
  double* dK64 = nullptr;
  float* dK32 = nullptr;
  float* dK16 = nullptr;   // K rounded to FP16, held in FP32 (16-bit product operands)
  float* dKb16 = nullptr;  // K rounded to BF16, held in FP32
  // 8-node patterns (one per Poisson-ratio library) whose matrix has the block structure of the
  // corner Walsh basis and is invariant under the 48 cube transformations: their cells are
  // mapped onto them in identity orientation and take the Walsh path with a structured table
  // (sbfem::kWalshC entries, layout as in the device code).  walsh_id[pattern]: index of the
  // pattern's table in Wcs, -1 for every other pattern.
  std::vector<int16_t> walsh_id;
  std::vector<std::vector<double>> Wcs;
};

struct sbfem_mesh {
  Allocator alloc;
  const sbfem_patterns* P = nullptr;
  int device = 0;
  int64_t N = 0, C = 0, ndof = 0;
  double h0 = 1.0, dt = 0.0, alpha = 0.0;
  int prod = 0, state_mode = 0, assembly = 0;
  sbfem::LoadParams L{};
  void* u = nullptr;     // state storage per state_mode: FP64, FP32 or compensated FP32 pair
  void* um1 = nullptr;
  double* f = nullptr;
  double* load_table = nullptr;  // P(t_n) per step (load kind TABLE)
  void* minv = nullptr;  // per dof: FP64, or FP32 with FP32 state
  double* matE = nullptr;
  int32_t* conn = nullptr;
  uint8_t* orient = nullptr;
  uint8_t* level = nullptr;
  uint8_t* material = nullptr;
  sbfem::Tile* tiles = nullptr;
  int64_t* load_idx = nullptr;
  double* load_val = nullptr;
  int64_t nnz = 0;
  unsigned long long* flag_d = nullptr;  // first step with a non-finite update (~0: none), device
  unsigned long long* flag_h = nullptr;  // its copy in pinned host memory
  hipEvent_t flag_ev = nullptr;
  bool flag_pending = false;
  int64_t check_every = 0;  // step_n: examine the record every this many steps (0: next call)
  std::vector<sbfem::TileRange> groups;  // one per colour
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (class, index of the begin event)
  int64_t step = 0;
  int64_t bytes = 0;
  int n_colours = 1;
  // internal node numbering (first touch along the cell order)
  std::vector<int32_t> int2ext;
  std::vector<double> mdiag;  // lumped diagonal mass (internal numbering), for read_state
  std::vector<bool> fixed;    // Dirichlet dofs (internal numbering)
  double lambda_bound = 0.0;  // max over cells of omega_max,e^2: bounds the spectrum of M^-1 K (eq. tcr)
  int64_t n_res = 0;          // hanging-cell row-force slots
  // probe histories (sbfem_set_probes)
  int32_t* probe_ptr = nullptr;
  int2* probes = nullptr;
  double* probe_u = nullptr;
  double* probe_a = nullptr;
  int64_t probe_step0 = 0, probe_rows = 0;
  int32_t n_probes = 0;
  // owner tiles
  sbfem::OwnerTile* otiles = nullptr;
  sbfem::CellItem* items = nullptr;
  uint16_t* lidx = nullptr;
  int32_t* nodelist = nullptr;
  sbfem::LoadEntry* tloads = nullptr;
  int64_t n_pure8 = 0, n_mixed = 0;
  int32_t lds_bytes = 0;
  sbfem::TiledArgs* d_args = nullptr;   // two argument blocks: (u=buf0, prev=buf1) and swapped
  sbfem::HangItem* hitems = nullptr;    // hanging-cell pass
  int32_t* hconn = nullptr;
  uint8_t* horient = nullptr;
  uint8_t* hlevel = nullptr;
  uint8_t* hmaterial = nullptr;
  sbfem::HangPair* hpairs = nullptr;    // per owner tile: (owned dof, result index) of hanging rows
  void* hres = nullptr;                 // row forces of the hanging cells (hanging-cell pass output)
  bool hang_mma = true;                 // hanging-cell pass on the matrix cores
  int64_t n_hang = 0;
  int64_t lds_hang = 0;                 // LDS of a hanging-pass block (its pattern's matrix)
  int32_t tile_nodes = 0;
  int64_t halo_stride = 0;              // tile halo lists at a fixed stride (0: packed)
  double* dWs64 = nullptr;              // Walsh blocks times s_e per scale class (pure 8-node tiles)
  float* dWs32 = nullptr;
  void* buf0 = nullptr;
  int32_t block_threads = 512;        // 8-node owner tiles
  int32_t block_threads_mixed = 256;  // owner tiles with larger cells
  bool walsh = true;
  int64_t layout[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // step loops captured in HIP graphs (owner-tile assembly): graph_steps per graph, 0 = off
  int32_t graph_steps = 0;
  sbfem::MeshRef* d_ref = nullptr;  // the mesh's ref on the device, read by graph replays
  hipGraphExec_t gexec = nullptr;   // graph of graph_steps steps (built on first use)
};

namespace {

constexpr int32_t kOwnerTileNodes = 512;  // nodes owned by one block in the tiled assembly

sbfem_status validate_desc(const sbfem_patterns* p, const sbfem_mesh_desc* d) {
  if (!p || !d) return fail(SBFEM_EINVAL, "null patterns or descriptor");
  if (d->n_nodes <= 0 || d->n_cells <= 0) return fail(SBFEM_EINVAL, "empty mesh");
  if (3 * d->n_nodes > (int64_t)INT32_MAX * 3) return fail(SBFEM_EINVAL, "too many nodes for int32 ids");
  if (!d->conn || !d->pattern || !d->orient || !d->level || !d->material)
    return fail(SBFEM_EINVAL, "missing cell arrays");
  if (d->n_materials <= 0 || d->n_materials > 256 || !d->E || !d->rho)
    return fail(SBFEM_EINVAL, "bad material table");
  for (int i = 0; i < d->n_materials; ++i)
    if (!(d->E[i] > 0) || !(d->rho[i] > 0)) return fail(SBFEM_EINVAL, "material %d: E and rho must be > 0", i);
  if (!(d->h0 > 0)) return fail(SBFEM_EINVAL, "h0 must be > 0");
  if (!(d->dt > 0) || !std::isfinite(d->dt)) return fail(SBFEM_EINVAL, "dt must be > 0");
  if (d->load_nnz < 0 || (d->load_nnz > 0 && (!d->load_dof || !d->load_val)))
    return fail(SBFEM_EINVAL, "bad load vector");
  if (d->load_kind < 0 || d->load_kind > 3) return fail(SBFEM_EINVAL, "unknown load kind");
  if (d->load_kind == SBFEM_LOAD_TABLE && (d->load_table_n < 1 || !d->load_table))
    return fail(SBFEM_EINVAL, "a load table needs at least one entry");
  if (d->prod < SBFEM_PROD_FP64 || d->prod > SBFEM_PROD_BF16)
    return fail(SBFEM_EINVAL, "unknown product precision %d", d->prod);
  if (d->state < SBFEM_STATE_FP64 || d->state > SBFEM_STATE_KAHAN32)
    return fail(SBFEM_EINVAL, "unknown state storage %d", d->state);
  if ((d->prod >= SBFEM_PROD_FP16 || d->state != SBFEM_STATE_FP64) && d->assembly != SBFEM_ASM_TILED)
    return fail(SBFEM_EINVAL, "16-bit products and FP32 or compensated state need the tiled assembly");
  if (d->assembly != SBFEM_ASM_ATOMIC && d->assembly != SBFEM_ASM_COLOUR && d->assembly != SBFEM_ASM_TILED)
    return fail(SBFEM_EINVAL, "unknown assembly mode");
  if (d->tile_nodes < 0 || d->block_threads < 0 || d->block_threads_mixed < 0 ||
      (d->block_threads && (d->block_threads % 64 || d->block_threads > 512)) ||
      (d->block_threads_mixed && (d->block_threads_mixed % 64 || d->block_threads_mixed > 512)))
    return fail(SBFEM_EINVAL, "bad owner-tile shape");
  for (int64_t c = 0; c < d->n_cells; ++c) {
    if (d->pattern[c] >= p->n) return fail(SBFEM_EINVAL, "cell %lld: pattern %d out of range", (long long)c, d->pattern[c]);
    if (d->orient[c] >= 48) return fail(SBFEM_EINVAL, "cell %lld: orientation %d >= 48", (long long)c, d->orient[c]);
    if (d->material[c] >= d->n_materials) return fail(SBFEM_EINVAL, "cell %lld: material out of range", (long long)c);
    if (d->level[c] > 40) return fail(SBFEM_EINVAL, "cell %lld: level %d too deep", (long long)c, d->level[c]);
  }
  return SBFEM_OK;
}

// Host plan of a mesh (Alg. 1 set-up): internal numbering, normalised orientations, lumped
// mass, load vector, and the layout of the chosen assembly, with every device buffer's size.
// create_mesh uploads a plan; mesh_footprint returns the bytes of the same buffers.
struct MeshPlan {
  int64_t N = 0, C = 0, ndof = 0;
  std::vector<int64_t> cptr;          // offsets into conn per cell (input order)
  std::vector<int32_t> int2ext;       // internal node -> caller node
  std::vector<int32_t> iconn;         // internal node ids per cell (master order)
  std::vector<uint8_t> orient;        // orientation per cell (8-node cells re-listed in identity)
  std::vector<double> mdiag, minv;    // lumped mass and its inverse (0 on fixed dofs), internal dofs
  std::vector<bool> fixed;            // Dirichlet dofs, internal numbering
  double lambda_bound = 0.0;          // max over cells of omega_max,e^2
  std::vector<int64_t> bidx;          // load vector, internal dofs, duplicates merged
  std::vector<double> bval;
  std::vector<double> matE;           // 256 entries
  bool force_array = false;           // an FP64 force array over all dofs is allocated
  // owner tiles
  sbfem::TilingOutput to;
  int32_t lds_bytes = 0, block_threads = 512, block_threads_mixed = 256;
  bool walsh = true;
  bool hang_mma = true;               // hanging-cell pass on the matrix cores
  std::vector<sbfem::HangItem> hitems;
  std::vector<int32_t> hconn;
  std::vector<uint8_t> hor, hlev, hmat;
  std::vector<sbfem::HangPair> hpairs;
  int64_t n_res = 0, lds_hang = 0;
  std::vector<double> ws64;
  std::vector<float> ws32;
  int64_t layout[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // classic assemblies
  std::vector<int32_t> sconn;
  std::vector<uint8_t> sorient, slevel, smat;
  std::vector<sbfem::Tile> tiles;
  std::vector<sbfem::TileRange> groups;
  int n_colours = 1;
};

// Every device buffer of a mesh with its size in bytes, in allocation order: f(slot, bytes),
// where slot is the mesh member that holds it (null when m is null, for the footprint).
template <class F>
void for_each_buffer(const MeshPlan& P, const sbfem_mesh_desc* d, sbfem_mesh* m, F f) {
  auto slot = [&](auto member) -> void** { return m ? (void**)&(m->*member) : nullptr; };
  const int64_t ndof = P.ndof;
  f(slot(&sbfem_mesh::u), (size_t)state_bytes(d->state, ndof));
  f(slot(&sbfem_mesh::um1), (size_t)state_bytes(d->state, ndof));
  f(slot(&sbfem_mesh::minv), (size_t)ndof * (d->state == SBFEM_STATE_FP32 ? 4 : 8));
  if (P.force_array) f(slot(&sbfem_mesh::f), (size_t)(ndof * 8));
  f(slot(&sbfem_mesh::matE), 256 * 8);
  f(slot(&sbfem_mesh::flag_d), sizeof(unsigned long long));
  if (d->load_kind == SBFEM_LOAD_TABLE) f(slot(&sbfem_mesh::load_table), (size_t)d->load_table_n * 8);
  if (d->assembly == SBFEM_ASM_TILED) {
    const auto& to = P.to;
    f(slot(&sbfem_mesh::otiles), to.tiles.size() * sizeof(sbfem::OwnerTile));
    f(slot(&sbfem_mesh::items), to.items.size() * sizeof(sbfem::CellItem));
    f(slot(&sbfem_mesh::lidx), to.lidx.size() * 2);
    f(slot(&sbfem_mesh::nodelist), to.nodelist.size() * 4);
    f(slot(&sbfem_mesh::tloads), to.loads.size() * sizeof(sbfem::LoadEntry));
    f(slot(&sbfem_mesh::hitems), P.hitems.size() * sizeof(sbfem::HangItem));
    f(slot(&sbfem_mesh::hconn), P.hconn.size() * 4);
    f(slot(&sbfem_mesh::horient), P.hor.size());
    f(slot(&sbfem_mesh::hlevel), P.hlev.size());
    f(slot(&sbfem_mesh::hmaterial), P.hmat.size());
    f(slot(&sbfem_mesh::hpairs), std::max<size_t>(1, P.hpairs.size()) * sizeof(sbfem::HangPair));
    f(slot(&sbfem_mesh::hres), (size_t)std::max<int64_t>(1, P.n_res) * (d->prod == SBFEM_PROD_FP64 ? 8 : 4));
    f(slot(&sbfem_mesh::d_args), 2 * sizeof(sbfem::TiledArgs));
    f(slot(&sbfem_mesh::d_ref), sizeof(sbfem::MeshRef));
    f(slot(&sbfem_mesh::dWs64), P.ws64.size() * 8);
    f(slot(&sbfem_mesh::dWs32), P.ws32.size() * 4);
  } else {
    f(slot(&sbfem_mesh::conn), P.iconn.size() * 4);
    f(slot(&sbfem_mesh::orient), (size_t)P.C);
    f(slot(&sbfem_mesh::level), (size_t)P.C);
    f(slot(&sbfem_mesh::material), (size_t)P.C);
    f(slot(&sbfem_mesh::tiles), P.tiles.size() * sizeof(sbfem::Tile));
    f(slot(&sbfem_mesh::load_idx), P.bidx.size() * 8);
    f(slot(&sbfem_mesh::load_val), P.bval.size() * 8);
  }
}

int64_t plan_bytes(const MeshPlan& P, const sbfem_mesh_desc* d) {
  int64_t b = 0;
  for_each_buffer(P, d, nullptr, [&](void**, size_t bytes) { b += (int64_t)bytes; });
  return b;
}

sbfem_status plan_mesh(const sbfem_patterns* p, const sbfem_mesh_desc* d, MeshPlan& P) {
  sbfem_status st = validate_desc(p, d);
  if (st != SBFEM_OK) return st;
  const int64_t N = d->n_nodes, C = d->n_cells, ndof = 3 * N;
  P.N = N;
  P.C = C;
  P.ndof = ndof;
  // per-cell node counts and offsets into conn (input order)
  P.cptr.assign(C + 1, 0);
  for (int64_t c = 0; c < C; ++c) P.cptr[c + 1] = P.cptr[c] + p->ndof[d->pattern[c]] / 3;
  const std::vector<int64_t>& cptr = P.cptr;
  const int64_t total = cptr[C];
  for (int64_t i = 0; i < total; ++i)
    if (d->conn[i] < 0 || d->conn[i] >= N)
      return fail(SBFEM_EINVAL, "node id %d at conn[%lld] out of range", d->conn[i], (long long)i);

  // internal numbering: first touch along the cell order (nodes used by no cell go last)
  std::vector<int32_t> ext2int(N, -1);
  P.int2ext.resize(N);
  {
    int32_t next = 0;
    for (int64_t i = 0; i < total; ++i) {
      const int32_t g = d->conn[i];
      if (ext2int[g] < 0) {
        ext2int[g] = next;
        P.int2ext[next++] = g;
      }
    }
    for (int64_t g = 0; g < N; ++g)
      if (ext2int[g] < 0) {
        ext2int[g] = next;
        P.int2ext[next++] = (int32_t)g;
      }
  }
  P.iconn.resize(total);
  std::vector<int32_t>& iconn = P.iconn;
  for (int64_t i = 0; i < total; ++i) iconn[i] = ext2int[d->conn[i]];
  // Cells of the 8-node pattern, whose matrix (and lumped mass) is invariant under the
  // 48 cube transformations, are re-listed in identity orientation: the master matrix
  // applies to the cell's own corner order and no transformation is needed per step.
  P.orient.assign(d->orient, d->orient + C);
  std::vector<uint8_t>& orient = P.orient;
  if (!p->Wcs.empty()) {
    for (int64_t c = 0; c < C; ++c) {
      if (p->walsh_id[d->pattern[c]] < 0 || orient[c] == 0) continue;
      int pi[3], nat[8];
      double sg[3];
      decode(orient[c], pi, sg);
      for (int k = 0; k < 8; ++k) nat[corner_image(k, pi, sg)] = iconn[cptr[c] + k];
      for (int k = 0; k < 8; ++k) iconn[cptr[c] + k] = nat[k];
      orient[c] = 0;
    }
  }

  // lumped diagonal mass in internal numbering (summation order fixed: cell order)
  P.mdiag.assign(ndof, 0.0);
  for (int64_t c = 0; c < C; ++c) {
    const int pid = d->pattern[c];
    const double h = std::ldexp(d->h0, -(int)d->level[c]);
    const double sc = d->rho[d->material[c]] * h * h * h;
    int pi[3];
    double sg[3];
    decode(orient[c], pi, sg);
    const double* mp = p->m.data() + p->moff[pid];
    for (int64_t k = 0; k < cptr[c + 1] - cptr[c]; ++k)
      for (int a = 0; a < 3; ++a) P.mdiag[3 * (int64_t)iconn[cptr[c] + k] + pi[a]] += sc * mp[3 * k + a];
  }
  P.minv.resize(ndof);
  P.fixed.assign(ndof, false);
  for (int64_t i = 0; i < ndof; ++i) {
    const int64_t e = 3 * (int64_t)P.int2ext[i / 3] + i % 3;
    if (d->fixed_dof && d->fixed_dof[e]) {
      P.fixed[i] = true;
      P.minv[i] = 0.0;
    } else {
      if (!(P.mdiag[i] > 0))
        return fail(SBFEM_EINVAL, "free dof %lld has no mass (node not used by any cell?)", (long long)e);
      P.minv[i] = 1.0 / P.mdiag[i];
    }
  }

  // element bound of the spectrum: omega_max,e = omega_p sqrt(E/rho) / h (eqs. tcr, tcr_scale)
  for (int64_t c = 0; c < C; ++c) {
    const double h = std::ldexp(d->h0, -(int)d->level[c]);
    const double w = p->omega[d->pattern[c]];
    P.lambda_bound = std::max(P.lambda_bound, w * w * d->E[d->material[c]] / (d->rho[d->material[c]] * h * h));
  }

  // load vector (internal dofs) with merged duplicates
  std::map<int64_t, double> bmap;
  for (int64_t i = 0; i < d->load_nnz; ++i) {
    if (d->load_dof[i] < 0 || d->load_dof[i] >= ndof)
      return fail(SBFEM_EINVAL, "load dof %lld out of range", (long long)d->load_dof[i]);
    const int64_t e = d->load_dof[i];
    bmap[3 * (int64_t)ext2int[e / 3] + e % 3] += d->load_val[i];
  }
  for (auto& kv : bmap) {
    P.bidx.push_back(kv.first);
    P.bval.push_back(kv.second);
  }
  std::vector<int32_t>().swap(ext2int);
  P.matE.assign(256, 0.0);
  for (int i = 0; i < d->n_materials; ++i) P.matE[i] = d->E[i];
  // the owner-tile step keeps no force array; the start-up with u0 needs one (K u0)
  P.force_array = d->assembly != SBFEM_ASM_TILED || d->u0 != nullptr;
  if (d->assembly == SBFEM_ASM_TILED) {
    sbfem::TilingInput ti;
    ti.n_nodes = N;
    ti.n_cells = C;
    ti.cptr = cptr.data();
    ti.conn = iconn.data();
    ti.pattern = d->pattern;
    ti.orient = orient.data();
    ti.level = d->level;
    ti.material = d->material;
    ti.pattern_ndof = p->ndof.data();
    ti.pattern_koff = p->koff.data();
    ti.load_dof = P.bidx;
    ti.load_val = P.bval;
    sbfem::TilingOutput& to = P.to;
    // tile size: env SBFEM_TILE_NODES or the default; halved until one block's LDS
    // (u of its local nodes + f of its owned ones) fits the per-block limit
    int device = 0, lds_max = 65536;
    (void)hipGetDevice(&device);
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (lds_max < 16384) lds_max = 65536;
    int32_t tn0 = kOwnerTileNodes;
    if (const char* ev = std::getenv("SBFEM_TILE_NODES")) tn0 = std::max(32, std::atoi(ev));
    auto threads_env = [](const char* name, int32_t& v) {
      if (const char* ev = std::getenv(name)) {
        const int bt = std::atoi(ev);
        if (bt >= 64 && bt <= 512 && bt % 64 == 0) v = bt;
      }
    };
    threads_env("SBFEM_BLOCK_THREADS", P.block_threads);
    threads_env("SBFEM_BLOCK_THREADS_MIXED", P.block_threads_mixed);
    // explicit descriptor values win over the defaults and the environment
    auto threads_desc = [](int32_t v, int32_t& out) {
      if (v >= 64 && v <= 512 && v % 64 == 0) out = v;
    };
    threads_desc(d->block_threads, P.block_threads);
    threads_desc(d->block_threads_mixed, P.block_threads_mixed);
    if (d->tile_nodes > 0) tn0 = std::max(32, d->tile_nodes);
    if (const char* ev = std::getenv("SBFEM_DENSE8")) P.walsh = std::atoi(ev) == 0;
    ti.regular = P.walsh && !p->Wcs.empty() ? p->walsh_id.data() : nullptr;
    auto regular = [&](int64_t c) { return ti.regular && ti.regular[d->pattern[c]] >= 0; };
    bool ok = false;
    // LDS per block: FP64 forces of the owned nodes, u of the local nodes (FP64: 24 B per node;
    // FP32: 16-byte float4 nodes)
    const int64_t node_bytes = d->prod != SBFEM_PROD_FP64 ? 16 : 24;
    for (int32_t tn = tn0; tn >= 32; tn /= 2) {
      if (!sbfem::build_owner_tiles(ti, tn, to)) continue;
      // forces of the owned nodes rounded up to an even number of doubles (16-byte aligned u)
      const int64_t fbytes = 8 * ((3 * (int64_t)to.tile_nodes + 1) & ~(int64_t)1);
      if (node_bytes * to.max_local + fbytes <= lds_max) {
        P.lds_bytes = (int32_t)(node_bytes * to.max_local + fbytes);
        ok = true;
        break;
      }
    }
    if (!ok) return fail(SBFEM_EINVAL, "no owner-tile size fits the on-chip memory of a block");
    // hanging-node cells (every cell that is not a regular 8-node cell), each once: items of up
    // to a wave of cells of one pattern, in cell order within a pattern; node ids slot-major
    std::vector<int64_t> hcells;
    for (int64_t c = 0; c < C; ++c)
      if (!regular(c)) hcells.push_back(c);
    std::stable_sort(hcells.begin(), hcells.end(),
                     [&](int64_t x, int64_t y) { return d->pattern[x] < d->pattern[y]; });
    // the items of one block of the VALU hanging pass share a pattern: each pattern's items are
    // padded with empty items to whole blocks, and the block stages that pattern's matrix in
    // LDS (the matrix-core pass takes one item per block and needs no padding)
    if (const char* ev = std::getenv("SBFEM_HANG")) P.hang_mma = std::strcmp(ev, "valu") != 0;
    const int per_block = P.hang_mma ? 1 : P.block_threads_mixed / sbfem::kWave;
    std::vector<std::pair<int64_t, sbfem::HangPair>> tpairs;  // (tile, pair)
    int64_t kl_max = 0;  // entries of the largest staged matrix (rows padded to 4)
    for (size_t i0 = 0; i0 < hcells.size();) {
      const int pid = d->pattern[hcells[i0]];
      size_t i1 = i0;
      while (i1 < hcells.size() && i1 - i0 < (size_t)sbfem::kWave && d->pattern[hcells[i1]] == pid) ++i1;
      sbfem::HangItem it{};
      it.res0 = P.n_res;
      it.cell0 = (int64_t)P.hor.size();
      it.conn0 = (int64_t)P.hconn.size();
      it.koff = p->koff[pid];
      it.nn = p->ndof[pid] / 3;
      it.count = (int32_t)(i1 - i0);
      for (int k = 0; k < it.nn; ++k)
        for (size_t j = i0; j < i1; ++j) P.hconn.push_back(iconn[cptr[hcells[j]] + k]);
      for (size_t j = i0; j < i1; ++j) {
        P.hor.push_back(orient[hcells[j]]);
        P.hlev.push_back(d->level[hcells[j]]);
        P.hmat.push_back(d->material[hcells[j]]);
      }
      P.hitems.push_back(it);
      const int64_t nd = p->ndof[pid];
      // row r of lane j: dof 3 g_k + pi(a) (r = 3k + a) of the tile that owns node g_k
      for (size_t j = i0; j < i1; ++j) {
        const int64_t c = hcells[j];
        int pi[3];
        double sg[3];
        decode(orient[c], pi, sg);
        for (int r = 0; r < nd; ++r) {
          const int64_t g = iconn[cptr[c] + r / 3];
          const int64_t t = g / to.tile_nodes;
          const int64_t ri = P.n_res + (int64_t)r * sbfem::kWave + (int64_t)(j - i0);
          tpairs.push_back({t, {(int32_t)(3 * (g - t * to.tile_nodes) + pi[r % 3]), (uint32_t)ri}});
        }
      }
      P.n_res += nd * sbfem::kWave;
      kl_max = std::max<int64_t>(kl_max, nd * ((nd + 3) & ~3));
      i0 = i1;
      if (i0 == hcells.size() || d->pattern[hcells[i0]] != pid) {
        sbfem::HangItem pad = it;
        pad.count = 0;
        while (P.hitems.size() % per_block) P.hitems.push_back(pad);
      }
    }
    if (P.hang_mma) {
      P.lds_hang = 0;
      for (const auto& it : P.hitems) P.lds_hang = std::max<int64_t>(P.lds_hang, sbfem::hang_mma_lds_bytes(d->prod, 3 * it.nn));
    } else {
      P.lds_hang = kl_max * (d->prod == SBFEM_PROD_FP64 ? 8 : 4);
    }
    if (P.n_res > (int64_t)UINT32_MAX) return fail(SBFEM_EINVAL, "too many hanging-node cells for 32-bit result indices");
    // pairs grouped by owner tile (each tile's pairs in result order)
    std::stable_sort(tpairs.begin(), tpairs.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    P.hpairs.resize(tpairs.size());
    for (size_t i = 0; i < tpairs.size(); ++i) {
      P.hpairs[i] = tpairs[i].second;
      auto& ot = to.tiles[tpairs[i].first];
      if (ot.n_hpair == 0) ot.hpair0 = (int64_t)i;
      ot.n_hpair++;
    }
    std::vector<std::pair<int64_t, sbfem::HangPair>>().swap(tpairs);
    P.layout[0] = to.n_pure8;
    P.layout[1] = to.n_mixed;
    P.layout[2] = (int64_t)to.items.size();
    P.layout[3] = to.local_entries;
    P.layout[4] = (int64_t)hcells.size();  // regular cell entries over all tiles, plus the hanging cells
    for (const auto& it : to.items) P.layout[4] += it.count;
    P.layout[5] = to.tile_nodes;
    // algorithmic bytes per step of each pass (the method's own traffic, whatever the layout):
    // the owner-tile pass reads u_n, u_{n-1}, M^-1 and writes u_{n+1} of every dof (in the
    // state storage: 8 B per value for FP64 and the compensated pair, 4 B for FP32, with M^-1
    // in FP32 beside FP32 state), the node ids (4 B each) and orientation, level, material
    // (1 B each) of the regular 8-node cells, and the load entries (16 B); the hanging-cell
    // pass the same per-cell bytes of the other cells
    {
      const int64_t bs = d->state == SBFEM_STATE_FP32 ? 4 : 8;
      int64_t b8 = 4 * bs * ndof + 16 * (int64_t)P.bidx.size(), bo = 0;
      for (int64_t c = 0; c < C; ++c) (regular(c) ? b8 : bo) += 4 * (cptr[c + 1] - cptr[c]) + 3;
      P.layout[6] = b8;
      P.layout[7] = bo;
    }
    P.layout[8] = to.max_local;
    P.layout[9] = P.lds_bytes;
    // structured Walsh table pre-multiplied by s_e = E h of each scale class (one rounding per entry)
    const size_t ncls = to.scale_keys.size();
    const int WC = sbfem::kWalshC;
    P.ws64.assign(std::max<size_t>(1, ncls) * WC, 0.0);
    P.ws32.assign(P.ws64.size(), 0.0f);
    for (size_t c = 0; c < ncls; ++c) {
      const int wid = to.scale_keys[c] >> 16, lev = (to.scale_keys[c] >> 8) & 255, mat = to.scale_keys[c] & 255;
      const std::vector<double>& Wc = p->Wcs[wid];
      const double se = d->E[mat] * std::ldexp(d->h0, -lev);
      for (int i = 0; i < WC; ++i) {
        P.ws64[WC * c + i] = se * Wc[i];
        P.ws32[WC * c + i] = (float)P.ws64[WC * c + i];
      }
      if (d->prod == SBFEM_PROD_FP16 || d->prod == SBFEM_PROD_BF16) {
        // 16-bit operands: the unscaled coefficients rounded to 16 bits, s_e applied after
        for (int i = 0; i < WC - 1; ++i)
          P.ws32[WC * c + i] = d->prod == SBFEM_PROD_FP16 ? round_fp16((float)Wc[i]) : round_bf16((float)Wc[i]);
        P.ws32[WC * c + WC - 1] = (float)se;
      }
    }
    return SBFEM_OK;
  }

  // classic assemblies: colours greedy in input order, per-node mask of the colours already
  // touching it
  std::vector<uint8_t> colour(C, 0);
  int n_colours = 1;
  if (d->assembly == SBFEM_ASM_COLOUR) {
    std::vector<uint64_t> used(N, 0);
    for (int64_t c = 0; c < C; ++c) {
      uint64_t forb = 0;
      for (int64_t i = cptr[c]; i < cptr[c + 1]; ++i) forb |= used[iconn[i]];
      if (forb == ~0ull) return fail(SBFEM_EINVAL, "cell %lld needs more than 64 colours", (long long)c);
      int col = 0;
      while ((forb >> col) & 1) ++col;
      colour[c] = (uint8_t)col;
      n_colours = std::max(n_colours, col + 1);
      for (int64_t i = cptr[c]; i < cptr[c + 1]; ++i) used[iconn[i]] |= 1ull << col;
    }
  }
  P.n_colours = n_colours;
  // order: colour, 8-node class first, pattern; stable in input order (counting sort)
  const int64_t n_keys = (int64_t)n_colours * 2 * p->n;
  auto key = [&](int64_t c) -> int64_t {
    const int pid = d->pattern[c];
    const int mixed = p->ndof[pid] == 24 ? 0 : 1;
    return ((int64_t)colour[c] * 2 + mixed) * p->n + pid;
  };
  std::vector<int64_t> order(C);
  {
    std::vector<int64_t> start(n_keys + 1, 0);
    for (int64_t c = 0; c < C; ++c) start[key(c) + 1]++;
    for (int64_t k = 0; k < n_keys; ++k) start[k + 1] += start[k];
    for (int64_t c = 0; c < C; ++c) order[start[key(c)]++] = c;
  }
  // segments, tiles and slot-major node ids
  P.sconn.resize(total);
  P.sorient.resize(C);
  P.slevel.resize(C);
  P.smat.resize(C);
  P.groups.assign(n_colours, sbfem::TileRange{-1, 0, 0});
  int64_t cpos = 0, i0 = 0;
  while (i0 < C) {
    int64_t i1 = i0;
    const int64_t k0 = key(order[i0]);
    while (i1 < C && key(order[i1]) == k0) ++i1;
    const int pid = d->pattern[order[i0]];
    const int nn = p->ndof[pid] / 3;
    const int col = colour[order[i0]];
    const int64_t cnt = i1 - i0;
    for (int64_t j = 0; j < cnt; ++j) {
      const int64_t c = order[i0 + j];
      for (int k = 0; k < nn; ++k) P.sconn[cpos + (int64_t)k * cnt + j] = iconn[cptr[c] + k];
      P.sorient[i0 + j] = orient[c];
      P.slevel[i0 + j] = d->level[c];
      P.smat[i0 + j] = d->material[c];
    }
    auto& g = P.groups[col];
    if (g.first < 0) g.first = (int64_t)P.tiles.size();
    for (int64_t j = 0; j < cnt; j += sbfem::kTile) {
      sbfem::Tile t;
      t.cell0 = i0 + j;
      t.conn0 = cpos + j;
      t.stride = cnt;
      t.koff = p->koff[pid];
      t.count = (int32_t)std::min<int64_t>(sbfem::kTile, cnt - j);
      t.nn = nn;
      P.tiles.push_back(t);
      if (nn == 8)
        g.n_fixed8++;
      else
        g.n_mixed++;
    }
    cpos += cnt * nn;
    i0 = i1;
  }
  for (auto& g : P.groups)
    if (g.first < 0) g.first = 0;
  return SBFEM_OK;
}

}  // namespace

extern "C" {

const char* sbfem_last_error(void) { return g_err.c_str(); }

sbfem_status sbfem_set_allocator(void* (*alloc)(size_t bytes, void* user), void (*release)(void* ptr, void* user),
                                 void* user) {
  if ((alloc == nullptr) != (release == nullptr)) return fail(SBFEM_EINVAL, "give both alloc and release, or neither");
  g_alloc.alloc = alloc;
  g_alloc.release = release;
  g_alloc.user = user;
  return SBFEM_OK;
}

sbfem_status sbfem_upload_patterns(sbfem_patterns** out, int32_t n_patterns, const int32_t* ndof,
                                   const double* K, const double* m, const double* omega, void* hip_stream) {
  if (!out) return fail(SBFEM_EINVAL, "null output handle");
  *out = nullptr;
  if (n_patterns <= 0 || n_patterns > 65535 || !ndof || !K || !m || !omega)
    return fail(SBFEM_EINVAL, "bad pattern library arguments");
  auto* p = new sbfem_patterns();
  p->alloc = g_alloc;
  p->n = n_patterns;
  int64_t ko = 0, mo = 0;
  for (int i = 0; i < n_patterns; ++i) {
    if (ndof[i] < 24 || ndof[i] > 78 || ndof[i] % 3) {
      delete p;
      return fail(SBFEM_EINVAL, "pattern %d: ndof %d not in 24..78 or not a multiple of 3", i, ndof[i]);
    }
    p->ndof.push_back(ndof[i]);
    p->koff.push_back(ko);
    p->moff.push_back(mo);
    ko += (int64_t)ndof[i] * ndof[i];
    mo += ndof[i];
  }
  p->K.assign(K, K + ko);
  p->m.assign(m, m + mo);
  p->omega.assign(omega, omega + n_patterns);
  for (int64_t i = 0; i < mo; ++i)
    if (!(p->m[i] > 0)) {
      delete p;
      return fail(SBFEM_EINVAL, "non-positive lumped mass in the library");
    }
  for (int i = 0; i < n_patterns; ++i)
    if (!(p->omega[i] > 0)) {
      delete p;
      return fail(SBFEM_EINVAL, "pattern %d: non-positive frequency", i);
    }
  std::vector<float> K32(p->K.begin(), p->K.end());
  // Walsh blocks of the 8-node pattern: Khat[(a',s'),(a,s)] = 1/64 sum_{k,k'} chi_s'(k) K[3k+a'][3k'+a] chi_s(k'),
  // corner k = i + 2j + 4l at (2i-1, 2j-1, 2l-1), chi_s(k) = prod_b p_b^(s_b); used only if every
  // entry outside the blocks s' = t^(1<<a'), s = t^(1<<a) vanishes to roundoff.
  p->walsh_id.assign(n_patterns, -1);
  for (int pid = 0; pid < n_patterns; ++pid) {
    if (p->ndof[pid] != 24) continue;
    std::vector<double> W(72, 0.0);
    const double* Kp = p->K.data() + p->koff[pid];
    auto chi = [](int k, int s) {
      double v = 1.0;
      for (int b = 0; b < 3; ++b)
        if ((s >> b) & 1) v *= ((k >> b) & 1) ? 1.0 : -1.0;
      return v;
    };
    double kmax = 0.0, off = 0.0;
    for (int i = 0; i < 576; ++i) kmax = std::max(kmax, std::fabs(Kp[i]));
    for (int a2 = 0; a2 < 3; ++a2)
      for (int s2 = 0; s2 < 8; ++s2)
        for (int a = 0; a < 3; ++a)
          for (int s1 = 0; s1 < 8; ++s1) {
            double v = 0.0;
            for (int k = 0; k < 8; ++k)
              for (int k2 = 0; k2 < 8; ++k2) v += chi(k, s2) * Kp[(3 * k + a2) * 24 + 3 * k2 + a] * chi(k2, s1);
            v /= 64.0;
            const int t = s1 ^ (1 << a);
            if ((s2 ^ (1 << a2)) == t)
              W[t * 9 + a2 * 3 + a] = v;
            else
              off = std::max(off, std::fabs(v));
          }
    const bool blocks = off <= 1e-12 * kmax / 8.0;
    // invariance under every transformation g:  K[3k+a][3k'+a'] = s_a s_a' K[3n(k)+pi(a)][3n(k')+pi(a')],
    // where corner k of the master sits at corner n(k) of the cell (Sec. 3.2.2)
    double dev = 0.0;
    for (int code = 0; code < 48; ++code) {
      int pi[3], nk[8];
      double sg[3];
      decode(code, pi, sg);
      for (int k = 0; k < 8; ++k) nk[k] = corner_image(k, pi, sg);
      for (int k = 0; k < 8; ++k)
        for (int a = 0; a < 3; ++a)
          for (int k2 = 0; k2 < 8; ++k2)
            for (int a2 = 0; a2 < 3; ++a2) {
              const double v = sg[a] * sg[a2] * Kp[(3 * nk[k] + pi[a]) * 24 + 3 * nk[k2] + pi[a2]];
              dev = std::max(dev, std::fabs(v - Kp[(3 * k + a) * 24 + 3 * k2 + a2]));
            }
    }
    // structured table: translation modes carry no force, block 1 << m couples only the axes
    // other than m, block 7 ^ (1 << m) keeps axis m on its own, blocks 0 and 7 are (d - o) I + o J
    auto Wb = [&](int t, int a2, int a) { return W[t * 9 + a2 * 3 + a]; };
    double wmax = 0.0, werr = 0.0;
    for (double v : W) wmax = std::max(wmax, std::fabs(v));
    for (int t = 0; t < 8; ++t)
      for (int a2 = 0; a2 < 3; ++a2)
        for (int a = 0; a < 3; ++a) {
          bool zero = (t == (1 << a2)) || (t == (1 << a));
          if (t == 3 || t == 5 || t == 6) {
            const int m = t == 3 ? 2 : (t == 5 ? 1 : 0);
            zero = zero || ((a2 == m) != (a == m));
          }
          if (zero) werr = std::max(werr, std::fabs(Wb(t, a2, a)));
          if (t == 0 || t == 7)
            werr = std::max(werr, std::fabs(Wb(t, a2, a) - (a2 == a ? Wb(t, 0, 0) : Wb(t, 0, 1))));
        }
    std::vector<double> Wc(sbfem::kWalshC, 0.0);
    Wc[0] = Wb(0, 0, 0) - Wb(0, 0, 1);
    Wc[1] = Wb(0, 0, 1);
    Wc[2] = Wb(7, 0, 0) - Wb(7, 0, 1);
    Wc[3] = Wb(7, 0, 1);
    for (int mm = 0; mm < 3; ++mm) {
      const int i = mm == 0 ? 1 : 0, j = mm == 2 ? 1 : 2;
      const int t1 = 1 << mm, t2 = 7 ^ (1 << mm);
      const double b1[4] = {Wb(t1, i, i), Wb(t1, i, j), Wb(t1, j, i), Wb(t1, j, j)};
      const double b2[5] = {Wb(t2, i, i), Wb(t2, i, j), Wb(t2, j, i), Wb(t2, j, j), Wb(t2, mm, mm)};
      for (int q = 0; q < 4; ++q) Wc[4 + 4 * mm + q] = b1[q];
      for (int q = 0; q < 5; ++q) Wc[16 + 5 * mm + q] = b2[q];
    }
    if (blocks && dev <= 1e-12 * kmax && werr <= 1e-12 * wmax && p->Wcs.size() < 32767) {
      p->walsh_id[pid] = (int16_t)p->Wcs.size();
      p->Wcs.push_back(Wc);
    }
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = dalloc(p->alloc, &p->dK64, ko);
  if (e == hipSuccess) e = dalloc(p->alloc, &p->dK32, ko);
  if (e == hipSuccess) e = dalloc(p->alloc, &p->dK16, ko);
  if (e == hipSuccess) e = dalloc(p->alloc, &p->dKb16, ko);
  std::vector<float> K16(ko), Kb16(ko);
  for (int64_t i = 0; i < ko; ++i) {
    K16[i] = round_fp16(K32[i]);
    Kb16[i] = round_bf16(K32[i]);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(p->dK64, p->K.data(), ko * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->dK32, K32.data(), ko * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->dK16, K16.data(), ko * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->dKb16, Kb16.data(), ko * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dfree(p->alloc, p->dK64);
    dfree(p->alloc, p->dK32);
    dfree(p->alloc, p->dK16);
    dfree(p->alloc, p->dKb16);
    delete p;
    return fail(e == hipErrorOutOfMemory ? SBFEM_ENOMEM : SBFEM_EDEVICE, "pattern upload: %s", hipGetErrorString(e));
  }
  *out = p;
  return SBFEM_OK;
}

void sbfem_destroy_patterns(sbfem_patterns* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  dfree(p->alloc, p->dK64);
  dfree(p->alloc, p->dK32);
  dfree(p->alloc, p->dK16);
  dfree(p->alloc, p->dKb16);
  delete p;
}

sbfem_status sbfem_mesh_footprint(const sbfem_patterns* p, const sbfem_mesh_desc* d, int64_t* bytes) {
  if (!p || !d || !bytes) return fail(SBFEM_EINVAL, "null argument");
  MeshPlan P;
  sbfem_status st = plan_mesh(p, d, P);
  if (st != SBFEM_OK) return st;
  *bytes = plan_bytes(P, d);
  return SBFEM_OK;
}

sbfem_status sbfem_critical_dt(const sbfem_patterns* p, const sbfem_mesh_desc* d, double* dt_cr) {
  if (!dt_cr) return fail(SBFEM_EINVAL, "null output");
  // only what the limit needs: the cell arrays it reads and the material table (the time step
  // itself need not be set yet)
  if (!p || !d) return fail(SBFEM_EINVAL, "null patterns or descriptor");
  if (d->n_cells <= 0) return fail(SBFEM_EINVAL, "empty mesh");
  if (!d->pattern || !d->level || !d->material) return fail(SBFEM_EINVAL, "missing cell arrays");
  if (d->n_materials <= 0 || d->n_materials > 256 || !d->E || !d->rho)
    return fail(SBFEM_EINVAL, "bad material table");
  for (int i = 0; i < d->n_materials; ++i)
    if (!(d->E[i] > 0) || !(d->rho[i] > 0)) return fail(SBFEM_EINVAL, "material %d: E and rho must be > 0", i);
  if (!(d->h0 > 0)) return fail(SBFEM_EINVAL, "h0 must be > 0");
  double best = INFINITY;
  for (int64_t c = 0; c < d->n_cells; ++c) {
    const int pid = d->pattern[c];
    if (pid >= p->n || d->material[c] >= d->n_materials) return fail(SBFEM_EINVAL, "cell %lld out of range", (long long)c);
    const double h = std::ldexp(d->h0, -(int)d->level[c]);
    const double w = p->omega[pid] * std::sqrt(d->E[d->material[c]] / d->rho[d->material[c]]) / h;
    best = std::min(best, 2.0 / w);
  }
  *dt_cr = best;
  return SBFEM_OK;
}

// Device work lists of a batch for one set of active meshes, and the graph of a chunk of
// steps over them; kept between calls while graphs are on, so that a serving loop that
// steps the same set repeatedly replays the same graph.
struct BatchLists {
  std::vector<sbfem_mesh*> meshes;  // active meshes; index = ref index
  int32_t graph_steps = 0;
  Allocator alloc;
  sbfem::MeshRef* d_refs = nullptr;
  sbfem::TileWork* d_w8 = nullptr;
  sbfem::TileWork* d_wm = nullptr;
  int64_t n8 = 0, nm = 0;
  hipGraphExec_t gexec = nullptr;
  uint64_t stamp = 0;
};
static std::mutex g_batch_mu;  // guards the cache
static std::vector<BatchLists*> g_batch_cache;
static uint64_t g_batch_clock = 0;
constexpr size_t kBatchCacheMax = 16;

static void free_lists(BatchLists* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  dfree(b->alloc, b->d_refs);
  dfree(b->alloc, b->d_w8);
  dfree(b->alloc, b->d_wm);
  delete b;
}

// drop every cached batch that steps this mesh (its graphs name the mesh's buffers)
static void forget_batch_graphs(const sbfem_mesh* m) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t i = 0; i < g_batch_cache.size();) {
    const auto& v = g_batch_cache[i]->meshes;
    if (std::find(v.begin(), v.end(), m) != v.end()) {
      (void)hipDeviceSynchronize();
      free_lists(g_batch_cache[i]);
      g_batch_cache.erase(g_batch_cache.begin() + (std::ptrdiff_t)i);
    } else {
      ++i;
    }
  }
}

void sbfem_destroy_mesh(sbfem_mesh* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  forget_batch_graphs(m);
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  dfree(m->alloc, m->d_ref);
  for (auto e : m->ev_pool) (void)hipEventDestroy(e);
  if (m->flag_ev) (void)hipEventDestroy(m->flag_ev);
  if (m->flag_h) (void)hipHostFree(m->flag_h);
  dfree(m->alloc, m->u);
  dfree(m->alloc, m->um1);
  dfree(m->alloc, m->f);
  dfree(m->alloc, m->minv);
  dfree(m->alloc, m->matE);
  dfree(m->alloc, m->conn);
  dfree(m->alloc, m->orient);
  dfree(m->alloc, m->level);
  dfree(m->alloc, m->material);
  dfree(m->alloc, m->tiles);
  dfree(m->alloc, m->load_idx);
  dfree(m->alloc, m->load_val);
  dfree(m->alloc, m->flag_d);
  dfree(m->alloc, m->otiles);
  dfree(m->alloc, m->items);
  dfree(m->alloc, m->lidx);
  dfree(m->alloc, m->nodelist);
  dfree(m->alloc, m->tloads);
  dfree(m->alloc, m->d_args);
  dfree(m->alloc, m->hitems);
  dfree(m->alloc, m->hconn);
  dfree(m->alloc, m->horient);
  dfree(m->alloc, m->hlevel);
  dfree(m->alloc, m->hmaterial);
  dfree(m->alloc, m->hpairs);
  dfree(m->alloc, m->hres);
  dfree(m->alloc, m->dWs64);
  dfree(m->alloc, m->dWs32);
  dfree(m->alloc, m->load_table);
  dfree(m->alloc, m->probe_ptr);
  dfree(m->alloc, m->probes);
  dfree(m->alloc, m->probe_u);
  dfree(m->alloc, m->probe_a);
  delete m;
}

static sbfem::ElementArgs element_args(const sbfem_mesh* m) {
  sbfem::ElementArgs a;
  a.tiles = m->tiles;
  a.u = (const double*)m->u;  // the classic assemblies keep FP64 state
  a.f = m->f;
  a.conn = m->conn;
  a.orient = m->orient;
  a.level = m->level;
  a.material = m->material;
  a.matE = m->matE;
  a.h0 = m->h0;
  a.K64 = m->P->dK64;
  a.K32 = m->P->dK32;
  return a;
}

static void profile_hook(void* ctx, int cls, bool begin, hipStream_t s) {
  auto* m = (sbfem_mesh*)ctx;
  if (m->ev_used == m->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    m->ev_pool.push_back(e);
  }
  if (begin) m->ev_marks.push_back({cls, m->ev_used});
  (void)hipEventRecord(m->ev_pool[m->ev_used++], s);
}

static sbfem::LaunchHook hook_of(sbfem_mesh* m) {
  sbfem::LaunchHook h;
  if (m->profiling) {
    h.fn = profile_hook;
    h.ctx = m;
  }
  return h;
}

// f += R_int(u) over all colours (f must hold what it should be added to)
static sbfem::TiledArgs tiled_args_for(const sbfem_mesh* m, const void* u, void* um1) {
  sbfem::TiledArgs a{};
  a.tiles = m->otiles;
  a.n_tiles = m->n_pure8 + m->n_mixed;
  a.hitems = m->hitems;
  a.hconn = m->hconn;
  a.horient = m->horient;
  a.hlevel = m->hlevel;
  a.hmaterial = m->hmaterial;
  a.hpairs = m->hpairs;
  a.hres = m->hres;
  a.items = m->items;
  a.lidx = m->lidx;
  a.nodelist = m->nodelist;
  a.tile_nodes = m->tile_nodes;
  a.halo_stride = m->halo_stride;
  a.loads = m->tloads;
  a.matE = m->matE;
  a.h0 = m->h0;
  a.K64 = m->P->dK64;
  a.K32 = m->prod == SBFEM_PROD_FP16 ? m->P->dK16 : (m->prod == SBFEM_PROD_BF16 ? m->P->dKb16 : m->P->dK32);
  a.Ws64 = m->dWs64;
  a.Ws32 = m->dWs32;
  a.u = u;
  a.um1 = um1;
  a.minv = m->minv;
  a.f = m->f;
  a.flag = m->flag_d;
  a.probe_ptr = m->probe_ptr;
  a.probes = m->probes;
  a.probe_u = m->probe_u;
  a.probe_a = m->probe_a;
  a.probe_step0 = m->probe_step0;
  a.probe_rows = m->probe_rows;
  a.n_probes = m->n_probes;
  a.ndof = m->ndof;
  a.state = m->state_mode;
  a.round16 = m->prod == SBFEM_PROD_FP16 ? 1 : (m->prod == SBFEM_PROD_BF16 ? 2 : 0);
  a.L = m->L;
  a.dt = m->dt;
  a.dt2 = m->dt * m->dt;
  a.c = 0.5 * m->alpha * m->dt;
  a.lds_bytes = m->lds_bytes;
  a.block_threads = m->block_threads;
  a.block_threads_mixed = m->block_threads_mixed;
  return a;
}

static int tiled_parity(const sbfem_mesh* m) { return m->u == m->buf0 ? 0 : 1; }

static sbfem::TiledLaunch tiled_launch(const sbfem_mesh* m, bool force_only) {
  sbfem::TiledLaunch L;
  L.single.args = m->d_args;
  L.single.step = m->step;
  L.single.parity = tiled_parity(m);
  L.n_tiles = m->n_pure8 + m->n_mixed;
  L.n_hang = m->n_hang;
  L.lds_hang = (size_t)m->lds_hang;
  L.fp32 = m->prod != SBFEM_PROD_FP64;  // FP32 kernels also carry the 16-bit product forms
  L.reduced = m->state_mode != SBFEM_STATE_FP64 || m->prod == SBFEM_PROD_FP16 || m->prod == SBFEM_PROD_BF16;
  L.force_only = force_only;
  L.prec = m->prod;
  L.state = m->state_mode;
  L.hang_mma = m->hang_mma;
  L.threads8 = m->block_threads;
  L.threads_mixed = m->block_threads_mixed;
  L.lds = (size_t)m->lds_bytes;
  return L;
}

static sbfem_status internal_force(sbfem_mesh* m, hipStream_t s) {
  if (m->assembly == SBFEM_ASM_TILED) {
    HIP_TRY(sbfem::launch_tiled(tiled_launch(m, true), s, hook_of(m)));
    return SBFEM_OK;
  }
  sbfem::ElementArgs a = element_args(m);
  const bool atomic = m->assembly == SBFEM_ASM_ATOMIC;
  const sbfem::LaunchHook h = hook_of(m);
  for (const auto& g : m->groups) HIP_TRY(sbfem::launch_ebe(a, g, m->prod == SBFEM_PROD_FP32, atomic, s, h));
  return SBFEM_OK;
}

// The device mesh from its host plan (consumed: its tables move into the mesh or die here).
static sbfem_status create_from_plan(sbfem_mesh** out, MeshPlan& P, const sbfem_patterns* p,
                                     const sbfem_mesh_desc* d, void* hip_stream) {
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t ndof = P.ndof;

  auto* m = new sbfem_mesh();
  m->alloc = g_alloc;
  m->P = p;
  (void)hipGetDevice(&m->device);
  m->N = P.N;
  m->C = P.C;
  m->ndof = ndof;
  m->h0 = d->h0;
  m->dt = d->dt;
  m->alpha = d->alpha;
  m->prod = d->prod;
  m->state_mode = d->state;
  m->assembly = d->assembly;
  m->L.kind = d->load_kind;
  m->L.cycles = d->load_cycles;
  m->L.t1 = d->load_t1;
  m->L.P0 = d->load_P0;
  m->L.dt = d->dt;
  m->nnz = (int64_t)P.bidx.size();
  m->n_colours = P.n_colours;
  m->groups = P.groups;
  m->n_pure8 = P.to.n_pure8;
  m->n_mixed = P.to.n_mixed;
  m->tile_nodes = P.to.tile_nodes;
  m->halo_stride = P.to.halo_stride;
  m->n_hang = (int64_t)P.hitems.size();
  m->lds_hang = P.lds_hang;
  m->lds_bytes = P.lds_bytes;
  m->block_threads = P.block_threads;
  m->block_threads_mixed = P.block_threads_mixed;
  m->walsh = P.walsh;
  m->hang_mma = P.hang_mma;
  for (int i = 0; i < 10; ++i) m->layout[i] = P.layout[i];

  hipError_t e = hipSuccess;
  int64_t bytes = 0;
  for_each_buffer(P, d, m, [&](void** slot, size_t b) {
    if (e == hipSuccess) e = dalloc_bytes(m->alloc, slot, b);
    bytes += (int64_t)b;
  });
  m->bytes = bytes;
  auto H2D = [&](void* dst, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
  };
  if (d->assembly == SBFEM_ASM_TILED) {
    const auto& to = P.to;
    H2D(m->otiles, to.tiles.data(), to.tiles.size() * sizeof(sbfem::OwnerTile));
    H2D(m->items, to.items.data(), to.items.size() * sizeof(sbfem::CellItem));
    H2D(m->lidx, to.lidx.data(), to.lidx.size() * 2);
    H2D(m->nodelist, to.nodelist.data(), to.nodelist.size() * 4);
    H2D(m->tloads, to.loads.data(), to.loads.size() * sizeof(sbfem::LoadEntry));
    H2D(m->hitems, P.hitems.data(), P.hitems.size() * sizeof(sbfem::HangItem));
    H2D(m->hconn, P.hconn.data(), P.hconn.size() * 4);
    H2D(m->horient, P.hor.data(), P.hor.size());
    H2D(m->hlevel, P.hlev.data(), P.hlev.size());
    H2D(m->hmaterial, P.hmat.data(), P.hmat.size());
    H2D(m->hpairs, P.hpairs.data(), P.hpairs.size() * sizeof(sbfem::HangPair));
    H2D(m->dWs64, P.ws64.data(), P.ws64.size() * 8);
    H2D(m->dWs32, P.ws32.data(), P.ws32.size() * 4);
  } else {
    H2D(m->conn, P.sconn.data(), P.sconn.size() * 4);
    H2D(m->orient, P.sorient.data(), P.sorient.size());
    H2D(m->level, P.slevel.data(), P.slevel.size());
    H2D(m->material, P.smat.data(), P.smat.size());
    H2D(m->tiles, P.tiles.data(), P.tiles.size() * sizeof(sbfem::Tile));
    H2D(m->load_idx, P.bidx.data(), P.bidx.size() * 8);
    H2D(m->load_val, P.bval.data(), P.bval.size() * 8);
  }
  std::vector<float> minv32;
  if (d->state == SBFEM_STATE_FP32) {
    minv32.assign(P.minv.begin(), P.minv.end());
    H2D(m->minv, minv32.data(), ndof * 4);
  } else {
    H2D(m->minv, P.minv.data(), ndof * 8);
  }
  H2D(m->matE, P.matE.data(), 256 * 8);
  if (d->load_kind == SBFEM_LOAD_TABLE) {
    H2D(m->load_table, d->load_table, (size_t)d->load_table_n * 8);
    m->L.table = m->load_table;
    m->L.n_table = d->load_table_n;
  }
  const unsigned long long no_flag = ~0ull;
  H2D(m->flag_d, &no_flag, sizeof(no_flag));
  if (e == hipSuccess && m->f) e = sbfem::launch_fill(m->f, ndof, 0.0, s);
  if (e == hipSuccess) e = hipHostMalloc((void**)&m->flag_h, sizeof(unsigned long long), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->flag_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the plan's host buffers die with this call
  if (e != hipSuccess) {
    sbfem_destroy_mesh(m);
    return fail(e == hipErrorOutOfMemory ? SBFEM_ENOMEM : SBFEM_EDEVICE, "create_mesh upload: %s",
                hipGetErrorString(e));
  }
  *m->flag_h = no_flag;
  m->buf0 = m->u;
  if (d->assembly == SBFEM_ASM_TILED) {
    const sbfem::TiledArgs ta[2] = {tiled_args_for(m, m->u, m->um1), tiled_args_for(m, m->um1, m->u)};
    H2D(m->d_args, ta, sizeof(ta));
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }

  // start-up point (eq. D0): u_-1 = u0 - dt v0 + dt^2/2 a0,  a0 = M^-1 (P(0) b - K u0) - alpha v0
  const std::vector<double>& minv = P.minv;
  std::vector<double> u0(ndof, 0.0), v0(ndof, 0.0), ku0(ndof, 0.0);
  for (int64_t i = 0; i < ndof; ++i) {
    const int64_t ex = 3 * (int64_t)P.int2ext[i / 3] + i % 3;
    if (d->u0) u0[i] = d->u0[ex];
    if (d->v0) v0[i] = d->v0[ex];
    if (minv[i] == 0.0) u0[i] = v0[i] = 0.0;
  }
  const std::vector<char> u0raw = pack_state(d->state, u0.data(), ndof);
  H2D(m->u, u0raw.data(), u0raw.size());
  if (e == hipSuccess && d->u0) {
    sbfem_status fs = internal_force(m, s);
    if (fs != SBFEM_OK) {
      sbfem_destroy_mesh(m);
      return fs;
    }
    e = hipMemcpyAsync(ku0.data(), m->f, ndof * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = sbfem::launch_fill(m->f, ndof, 0.0, s);
  }
  const double P0t = d->load_kind == SBFEM_LOAD_TABLE ? d->load_table[0] : load_time_host(m->L, 0.0);
  std::vector<double> um1(ndof);
  std::vector<double> fext(ndof, 0.0);
  for (size_t i = 0; i < P.bidx.size(); ++i) fext[P.bidx[i]] = P0t * P.bval[i];
  for (int64_t i = 0; i < ndof; ++i) {
    const double a0 = minv[i] * (fext[i] - ku0[i]) - (minv[i] != 0.0 ? d->alpha * v0[i] : 0.0);
    um1[i] = u0[i] - d->dt * v0[i] + 0.5 * d->dt * d->dt * a0;
  }
  const std::vector<char> um1raw = pack_state(d->state, um1.data(), ndof);
  H2D(m->um1, um1raw.data(), um1raw.size());
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    sbfem_destroy_mesh(m);
    return fail(SBFEM_EDEVICE, "create_mesh initial state: %s", hipGetErrorString(e));
  }
  m->int2ext.swap(P.int2ext);
  m->mdiag.swap(P.mdiag);
  m->fixed.swap(P.fixed);
  m->lambda_bound = P.lambda_bound;
  m->n_res = P.n_res;
  *out = m;
  return SBFEM_OK;
}

sbfem_status sbfem_create_mesh(sbfem_mesh** out, const sbfem_patterns* p, const sbfem_mesh_desc* d,
                               void* hip_stream) {
  if (!out) return fail(SBFEM_EINVAL, "null output handle");
  *out = nullptr;
  MeshPlan P;
  sbfem_status st = plan_mesh(p, d, P);
  if (st != SBFEM_OK) return st;
  return create_from_plan(out, P, p, d, hip_stream);
}

// A host plan kept between sbfem_plan_mesh and sbfem_create_mesh_planned.
struct sbfem_plan {
  MeshPlan P;
  const sbfem_patterns* p = nullptr;
  const sbfem_mesh_desc* d = nullptr;
  int64_t n_cells = 0, n_nodes = 0;
  bool used = false;
};

sbfem_status sbfem_plan_mesh(sbfem_plan** out, const sbfem_patterns* p, const sbfem_mesh_desc* d,
                             int64_t* device_bytes) {
  if (!out) return fail(SBFEM_EINVAL, "null output handle");
  *out = nullptr;
  auto* pl = new sbfem_plan();
  sbfem_status st = plan_mesh(p, d, pl->P);
  if (st != SBFEM_OK) {
    delete pl;
    return st;
  }
  pl->p = p;
  pl->d = d;
  pl->n_cells = d->n_cells;
  pl->n_nodes = d->n_nodes;
  if (device_bytes) *device_bytes = plan_bytes(pl->P, d);
  *out = pl;
  return SBFEM_OK;
}

sbfem_status sbfem_create_mesh_planned(sbfem_mesh** out, sbfem_plan* plan, void* hip_stream) {
  if (!out) return fail(SBFEM_EINVAL, "null output handle");
  *out = nullptr;
  if (!plan || plan->used) return fail(SBFEM_EINVAL, "null or already used plan");
  if (plan->d->n_cells != plan->n_cells || plan->d->n_nodes != plan->n_nodes)
    return fail(SBFEM_EINVAL, "the descriptor changed since the plan was made");
  plan->used = true;
  return create_from_plan(out, plan->P, plan->p, plan->d, hip_stream);
}

void sbfem_destroy_plan(sbfem_plan* plan) { delete plan; }

// Argument blocks of the owner-tile launches re-uploaded after a change of the mesh's buffers.
static sbfem_status upload_tiled_args(sbfem_mesh* m, hipStream_t s) {
  const bool swapped = m->u != m->buf0;
  void* b0 = m->buf0;
  void* b1 = swapped ? m->u : m->um1;
  const sbfem::TiledArgs ta[2] = {tiled_args_for(m, b0, b1), tiled_args_for(m, b1, b0)};
  HIP_TRY(hipMemcpyAsync(m->d_args, ta, sizeof(ta), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SBFEM_OK;
}

// The FP64 force array over all dofs, allocated on first use by a mesh that has none (the
// owner-tile step needs none; the force-only evaluation writes it).
static sbfem_status ensure_force_array(sbfem_mesh* m, hipStream_t s) {
  if (m->f) return SBFEM_OK;
  HIP_TRY(dalloc(m->alloc, &m->f, (size_t)m->ndof));
  m->bytes += m->ndof * 8;
  if (m->assembly == SBFEM_ASM_TILED) return upload_tiled_args(m, s);
  return SBFEM_OK;
}

static sbfem_status check_flag(sbfem_mesh* m) {
  if (!m->flag_pending) return SBFEM_OK;
  hipError_t q = hipEventQuery(m->flag_ev);
  if (q == hipErrorNotReady) return SBFEM_OK;
  m->flag_pending = false;
  if (q != hipSuccess) return fail(SBFEM_EDEVICE, "finite check: %s", hipGetErrorString(q));
  if (*m->flag_h != ~0ull)
    return fail(SBFEM_EUNSTABLE, "displacement became non-finite at step %llu (time step above the stability limit?)",
                *m->flag_h + 1);
  return SBFEM_OK;
}

static sbfem_status enqueue_step(sbfem_mesh* m, hipStream_t s) {
  const double t = (double)m->step * m->dt;
  const sbfem::LaunchHook h = hook_of(m);
  if (m->assembly == SBFEM_ASM_TILED) {
    (void)t;
    HIP_TRY(sbfem::launch_tiled(tiled_launch(m, false), s, h));
    std::swap(m->u, m->um1);
    m->step++;
    return SBFEM_OK;
  }
  h(0, true, s);
  HIP_TRY(sbfem::launch_load(m->f, m->load_idx, m->load_val, m->nnz, m->L, t, s));
  h(0, false, s);
  sbfem_status st = internal_force(m, s);
  if (st != SBFEM_OK) return st;
  h(3, true, s);
  HIP_TRY(sbfem::launch_update((const double*)m->u, (double*)m->um1, m->f, (const double*)m->minv, m->ndof,
                               m->dt * m->dt, 0.5 * m->alpha * m->dt, m->flag_d, m->step, s));
  h(3, false, s);
  std::swap(m->u, m->um1);
  m->step++;
  return SBFEM_OK;
}

// The update kernels record the first step whose result is not finite; its value is copied
// to the host behind the call's work and examined by the next call on the mesh.
static sbfem_status finish_steps(sbfem_mesh* m, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(m->flag_h, m->flag_d, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(m->flag_ev, s));
  m->flag_pending = true;
  return SBFEM_OK;
}

// Graph of `steps` steps over the launch L whose refs live on the device (d_refs[0..n)):
// launch k of the chunk reads step + k; a last kernel advances the refs by `steps`, so the
// graph replays at whatever step the refs hold.  Captured on a private stream.
static hipError_t capture_steps(sbfem::TiledLaunch L, sbfem::MeshRef* d_refs, int32_t n, int32_t steps,
                                hipGraphExec_t* out) {
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t le = hipSuccess;
    for (int32_t k = 0; k < steps && le == hipSuccess; ++k) {
      L.k = k;
      le = sbfem::launch_tiled(L, cs);
    }
    if (le == hipSuccess) le = sbfem::launch_refs_advance(d_refs, n, steps, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);  // always ends the capture
    if (e == hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipStreamDestroy(cs);
  return e;
}

static sbfem::MeshRef ref_of(const sbfem_mesh* m, int64_t ahead) {
  sbfem::MeshRef r{};
  r.args = m->d_args;
  r.step = m->step + ahead;
  r.parity = (int32_t)((tiled_parity(m) + ahead) & 1);
  return r;
}

// Whole graphs of the mesh's step chunk; `left` keeps the steps still to take.
static sbfem_status graph_steps_single(sbfem_mesh* m, int64_t& left, hipStream_t s) {
  const int32_t G = m->graph_steps;
  if (G <= 0 || m->assembly != SBFEM_ASM_TILED || m->profiling || left < G) return SBFEM_OK;
  if (!m->gexec) {
    sbfem::TiledLaunch L = tiled_launch(m, false);
    L.refs = m->d_ref;
    HIP_TRY(capture_steps(L, m->d_ref, 1, G, &m->gexec));
  }
  HIP_TRY(sbfem::launch_ref_set(m->d_ref, ref_of(m, 0), s));
  for (; left >= G; left -= G) {
    HIP_TRY(hipGraphLaunch(m->gexec, s));
    m->step += G;
    if (G & 1) std::swap(m->u, m->um1);
  }
  return SBFEM_OK;
}

sbfem_status sbfem_set_graph_steps(sbfem_mesh* m, int32_t steps) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  if (steps < 0 || steps > 4096) return fail(SBFEM_EINVAL, "graph steps must be in [0, 4096]");
  if (steps > 0 && m->assembly != SBFEM_ASM_TILED) return fail(SBFEM_EINVAL, "step graphs need the owner-tile assembly");
  if (steps == m->graph_steps) return SBFEM_OK;
  HIP_TRY(hipSetDevice(m->device));
  forget_batch_graphs(m);
  if (m->gexec) {
    HIP_TRY(hipDeviceSynchronize());  // the old graph may still run
    (void)hipGraphExecDestroy(m->gexec);
    m->gexec = nullptr;
  }
  m->graph_steps = steps;
  return SBFEM_OK;
}

// n steps launched (graph chunks first, then one by one), the non-finite record copied behind them
static sbfem_status launch_steps(sbfem_mesh* m, int64_t n, hipStream_t s) {
  int64_t left = n;
  sbfem_status st = graph_steps_single(m, left, s);
  if (st != SBFEM_OK) return st;
  for (int64_t k = 0; k < left; ++k) {
    st = enqueue_step(m, s);
    if (st != SBFEM_OK) return st;
  }
  return n > 0 ? finish_steps(m, s) : SBFEM_OK;
}

sbfem_status sbfem_step_n(sbfem_mesh* m, int64_t n_steps, void* hip_stream) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  if (n_steps < 0) return fail(SBFEM_EINVAL, "negative step count");
  HIP_TRY(hipSetDevice(m->device));
  sbfem_status st = check_flag(m);
  if (st != SBFEM_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  if (m->check_every <= 0) return launch_steps(m, n_steps, s);
  // chunks of check_every steps, each examined before the next is launched
  for (int64_t left = n_steps; left > 0;) {
    const int64_t k = std::min(left, m->check_every);
    st = launch_steps(m, k, s);
    if (st != SBFEM_OK) return st;
    left -= k;
    HIP_TRY(hipEventSynchronize(m->flag_ev));
    st = check_flag(m);
    if (st != SBFEM_OK) return st;
  }
  return SBFEM_OK;
}

sbfem_status sbfem_set_check_interval(sbfem_mesh* m, int64_t steps) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  if (steps < 0) return fail(SBFEM_EINVAL, "negative check interval");
  m->check_every = steps;
  return SBFEM_OK;
}

// Owner-tile meshes that share a pattern library and a product precision advance together:
// one launch per step and pass covers the tiles of every mesh that still has steps to take
// (a segment of steps per set of active meshes).  With graphs on (every mesh of the group
// has graph_steps > 0; the smallest is used) the segment's whole chunks replay a cached
// graph and the rest is launched directly.  Other meshes step one by one.
static hipError_t build_lists(BatchLists* b, hipStream_t s) {
  std::vector<sbfem::TileWork> w8, wm;
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    const sbfem_mesh* m = b->meshes[i];
    for (int64_t t = 0; t < m->n_pure8 + m->n_mixed; ++t) w8.push_back({(int32_t)i, 0, t});
    for (int64_t t = 0; t < m->n_hang; ++t) wm.push_back({(int32_t)i, 0, t});
  }
  b->n8 = (int64_t)w8.size();
  b->nm = (int64_t)wm.size();
  hipError_t e = dalloc(b->alloc, &b->d_refs, b->meshes.size());
  if (e == hipSuccess) e = dalloc(b->alloc, &b->d_w8, std::max<size_t>(1, w8.size()));
  if (e == hipSuccess) e = dalloc(b->alloc, &b->d_wm, std::max<size_t>(1, wm.size()));
  if (e == hipSuccess && !w8.empty())
    e = hipMemcpyAsync(b->d_w8, w8.data(), w8.size() * sizeof(sbfem::TileWork), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !wm.empty())
    e = hipMemcpyAsync(b->d_wm, wm.data(), wm.size() * sizeof(sbfem::TileWork), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host lists die here
  return e;
}

// cached lists of this active set (the caller holds g_batch_mu); null on failure
static BatchLists* cached_lists(const std::vector<sbfem_mesh*>& act, int32_t G, hipStream_t s, hipError_t& e) {
  for (auto* b : g_batch_cache)
    if (b->graph_steps == G && b->meshes == act) {
      b->stamp = ++g_batch_clock;
      return b;
    }
  if (g_batch_cache.size() >= kBatchCacheMax) {
    e = hipStreamSynchronize(s);  // the least recently used entry may still be in flight
    if (e != hipSuccess) return nullptr;
    auto lru = std::min_element(g_batch_cache.begin(), g_batch_cache.end(),
                                [](const BatchLists* x, const BatchLists* y) { return x->stamp < y->stamp; });
    free_lists(*lru);
    g_batch_cache.erase(lru);
  }
  auto* b = new BatchLists();
  b->meshes = act;
  b->graph_steps = G;
  b->alloc = act[0]->alloc;
  b->stamp = ++g_batch_clock;
  e = build_lists(b, s);
  if (e != hipSuccess) {
    free_lists(b);
    return nullptr;
  }
  g_batch_cache.push_back(b);
  return b;
}

// Bytes of the work lists of one batched segment over these meshes in a scratch buffer:
// refs, then the owner-tile list, then the hanging-cell item list (each 256-byte aligned).
static size_t scratch_list_bytes(const std::vector<sbfem_mesh*>& act, size_t* off8, size_t* offm) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  int64_t n8 = 0, nm = 0;
  for (const auto* m : act) {
    n8 += m->n_pure8 + m->n_mixed;
    nm += m->n_hang;
  }
  const size_t o8 = up(act.size() * sizeof(sbfem::MeshRef));
  const size_t om = o8 + up((size_t)n8 * sizeof(sbfem::TileWork));
  if (off8) *off8 = o8;
  if (offm) *offm = om;
  return om + (size_t)nm * sizeof(sbfem::TileWork);
}

// scratch != null: the work lists go into that device buffer (no allocation, no graphs)
static sbfem_status batch_tiled(const std::vector<sbfem_mesh*>& g, const std::vector<int64_t>& steps,
                                hipStream_t s, char* scratch = nullptr) {
  const size_t n = g.size();
  int64_t most = 0;
  int32_t G = g[0]->graph_steps;
  for (size_t i = 0; i < n; ++i) {
    most = std::max(most, steps[i]);
    G = std::min(G, g[i]->graph_steps);
  }
  if (scratch) G = 0;
  std::vector<std::vector<sbfem::TileWork>> keep_work;  // host lists of the async copies
  sbfem::TiledLaunch L0 = tiled_launch(g[0], false);
  for (auto* m : g) {
    L0.lds = std::max(L0.lds, (size_t)m->lds_bytes);
    L0.lds_hang = std::max(L0.lds_hang, (size_t)m->lds_hang);
  }
  std::unique_lock<std::mutex> lk(g_batch_mu, std::defer_lock);
  if (G > 0) lk.lock();
  std::vector<std::vector<sbfem::MeshRef>> keep;  // host refs of the async copies
  hipError_t e = hipSuccess;
  for (int64_t k = 0; k < most && e == hipSuccess;) {
    // the segment [k, end): meshes with steps left, until the first of them finishes
    std::vector<sbfem_mesh*> act;
    int64_t end = most;
    for (size_t i = 0; i < n; ++i)
      if (steps[i] > k) {
        act.push_back(g[i]);
        end = std::min(end, steps[i]);
      }
    BatchLists* b = nullptr;
    if (G > 0) {
      b = cached_lists(act, G, s, e);
    } else if (scratch) {
      // the lists of this segment written into the scratch buffer, behind the work of the
      // previous segment on the same stream
      b = new BatchLists();
      b->meshes = act;
      size_t o8 = 0, om = 0;
      (void)scratch_list_bytes(act, &o8, &om);
      keep_work.emplace_back();
      keep_work.emplace_back();
      auto& w8 = keep_work[keep_work.size() - 2];
      auto& wm = keep_work.back();
      for (size_t i = 0; i < act.size(); ++i) {
        for (int64_t t = 0; t < act[i]->n_pure8 + act[i]->n_mixed; ++t) w8.push_back({(int32_t)i, 0, t});
        for (int64_t t = 0; t < act[i]->n_hang; ++t) wm.push_back({(int32_t)i, 0, t});
      }
      b->d_refs = (sbfem::MeshRef*)scratch;
      b->d_w8 = (sbfem::TileWork*)(scratch + o8);
      b->d_wm = (sbfem::TileWork*)(scratch + om);
      b->n8 = (int64_t)w8.size();
      b->nm = (int64_t)wm.size();
      if (!w8.empty())
        e = hipMemcpyAsync(b->d_w8, w8.data(), w8.size() * sizeof(sbfem::TileWork), hipMemcpyHostToDevice, s);
      if (e == hipSuccess && !wm.empty())
        e = hipMemcpyAsync(b->d_wm, wm.data(), wm.size() * sizeof(sbfem::TileWork), hipMemcpyHostToDevice, s);
    } else {
      b = new BatchLists();
      b->meshes = act;
      b->alloc = act[0]->alloc;
      e = build_lists(b, s);
    }
    if (e == hipSuccess) {
      keep.emplace_back(act.size());
      for (size_t j = 0; j < act.size(); ++j) keep.back()[j] = ref_of(act[j], k);
      e = hipMemcpyAsync(b->d_refs, keep.back().data(), act.size() * sizeof(sbfem::MeshRef),
                         hipMemcpyHostToDevice, s);
    }
    sbfem::TiledLaunch L = L0;
    L.refs = b ? b->d_refs : nullptr;
    L.work8 = b ? b->d_w8 : nullptr;
    L.work_hang = b ? b->d_wm : nullptr;
    L.n_tiles = b ? b->n8 : 0;
    L.n_hang = b ? b->nm : 0;
    int64_t j = k;
    if (e == hipSuccess && G > 0 && end - k >= G) {
      if (!b->gexec) e = capture_steps(L, b->d_refs, (int32_t)act.size(), G, &b->gexec);
      for (; e == hipSuccess && end - j >= G; j += G) e = hipGraphLaunch(b->gexec, s);
    }
    const int64_t ref_k = j;  // the device refs now hold step offset ref_k
    for (; e == hipSuccess && j < end; ++j) {
      L.k = j - ref_k;
      e = sbfem::launch_tiled(L, s);
    }
    if (scratch && b) {
      delete b;  // points into the scratch buffer; nothing to free
    } else if (G == 0 && b) {
      const hipError_t q = hipStreamSynchronize(s);  // the lists are in use until here
      if (e == hipSuccess) e = q;
      free_lists(b);
    }
    k = end;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (lk.owns_lock()) lk.unlock();
  if (e != hipSuccess) return fail(SBFEM_EDEVICE, "batched step: %s", hipGetErrorString(e));
  for (size_t i = 0; i < n; ++i) {
    if (steps[i] & 1) std::swap(g[i]->u, g[i]->um1);
    g[i]->step += steps[i];
    sbfem_status st = finish_steps(g[i], s);
    if (st != SBFEM_OK) return st;
  }
  return SBFEM_OK;
}

// Batched stepping (sbfem_step_batch); scratch != null: the work lists of the owner-tile groups
// go into that device buffer of scratch_bytes (checked up front), with no allocation and no graphs.
static sbfem_status step_batch_impl(sbfem_mesh* const* ms, int32_t n, const int64_t* n_steps, void* hip_stream,
                                    char* scratch, size_t scratch_bytes) {
  if (n < 0 || (n > 0 && (!ms || !n_steps))) return fail(SBFEM_EINVAL, "bad batch arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  for (int i = 0; i < n; ++i) {
    if (!ms[i] || n_steps[i] < 0) return fail(SBFEM_EINVAL, "bad batch entry %d", i);
    for (int j = 0; j < i; ++j)
      if (ms[j] == ms[i]) return fail(SBFEM_EINVAL, "mesh %d appears twice in the batch", i);
    sbfem_status st = check_flag(ms[i]);
    if (st != SBFEM_OK) return st;
  }
  // groups of owner-tile meshes with one library and one precision
  std::vector<std::vector<sbfem_mesh*>> groups;
  std::vector<std::vector<int64_t>> group_steps;
  std::vector<char> used(n, 0);
  for (int i = 0; i < n; ++i) {
    if (used[i] || ms[i]->assembly != SBFEM_ASM_TILED || ms[i]->profiling) continue;
    std::vector<sbfem_mesh*> g;
    std::vector<int64_t> st;
    for (int j = i; j < n; ++j)
      if (!used[j] && ms[j]->assembly == SBFEM_ASM_TILED && !ms[j]->profiling && ms[j]->P == ms[i]->P &&
          ms[j]->prod == ms[i]->prod && ms[j]->state_mode == ms[i]->state_mode &&
          ms[j]->block_threads == ms[i]->block_threads &&
          ms[j]->block_threads_mixed == ms[i]->block_threads_mixed && ms[j]->hang_mma == ms[i]->hang_mma &&
          n_steps[j] > 0) {
        g.push_back(ms[j]);
        st.push_back(n_steps[j]);
        used[j] = 1;
      }
    if (!g.empty()) {
      groups.push_back(g);
      group_steps.push_back(st);
    }
  }
  if (scratch) {
    // every mesh of a group is active in its first segment: the largest lists
    for (const auto& g : groups) {
      const size_t need = scratch_list_bytes(g, nullptr, nullptr);
      if (need > scratch_bytes)
        return fail(SBFEM_EINVAL, "the batch needs %zu bytes of work lists, more than the %zu-byte scratch buffer",
                    need, scratch_bytes);
    }
  }
  for (size_t i = 0; i < groups.size(); ++i) {
    HIP_TRY(hipSetDevice(groups[i][0]->device));
    sbfem_status r = batch_tiled(groups[i], group_steps[i], s, scratch);
    if (r != SBFEM_OK) return r;
  }
  // the rest, interleaved step by step
  int64_t most = 0;
  for (int i = 0; i < n; ++i)
    if (!used[i]) most = std::max(most, n_steps[i]);
  for (int64_t k = 0; k < most; ++k)
    for (int i = 0; i < n; ++i)
      if (!used[i] && k < n_steps[i]) {
        sbfem_status st = enqueue_step(ms[i], s);
        if (st != SBFEM_OK) return st;
      }
  for (int i = 0; i < n; ++i)
    if (!used[i] && n_steps[i] > 0) {
      sbfem_status st = finish_steps(ms[i], s);
      if (st != SBFEM_OK) return st;
    }
  return SBFEM_OK;
}

sbfem_status sbfem_step_batch(sbfem_mesh* const* ms, int32_t n, const int64_t* n_steps, void* hip_stream) {
  return step_batch_impl(ms, n, n_steps, hip_stream, nullptr, 0);
}

}  // extern "C"

// Per-device work-list buffer of sbfem_step_batch_noalloc.  In host code `scratch` names a
// host-side stand-in: its device address comes from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) char scratch[SBFEM_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;

extern "C" {

static sbfem_status scratch_of_device(int dev, char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    HIP_TRY(hipSetDevice(dev));
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    it = g_scratch_ptr.emplace(dev, (char*)ptr).first;
  }
  *out = it->second;
  return SBFEM_OK;
}

sbfem_status sbfem_step_batch_noalloc(sbfem_mesh* const* ms, int32_t n, const int64_t* n_steps, void* hip_stream) {
  if (n < 0 || (n > 0 && (!ms || !n_steps))) return fail(SBFEM_EINVAL, "bad batch arguments");
  int dev = -1;
  for (int i = 0; i < n; ++i) {
    if (!ms[i]) return fail(SBFEM_EINVAL, "bad batch entry %d", i);
    if (dev < 0) dev = ms[i]->device;
    if (ms[i]->device != dev) return fail(SBFEM_EINVAL, "the meshes of a batch must share one device");
  }
  if (n == 0) return SBFEM_OK;
  char* ptr = nullptr;
  sbfem_status st = scratch_of_device(dev, &ptr);
  if (st != SBFEM_OK) return st;
  return step_batch_impl(ms, n, n_steps, hip_stream, ptr, SBFEM_NOALLOC_SCRATCH_BYTES);
}

sbfem_status sbfem_read_state(sbfem_mesh* m, int32_t which, double* host_out, int64_t* step, void* hip_stream) {
  if (!m || !host_out) return fail(SBFEM_EINVAL, "null argument");
  if (which < 0 || which > 3) return fail(SBFEM_EINVAL, "which must be 0, 1, 2 or 3");
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<double> tmp(m->ndof);
  if (which == 3) {
    tmp = m->mdiag;
  } else if (which == 2) {
    sbfem_status st = ensure_force_array(m, s);
    if (st != SBFEM_OK) return st;
    st = internal_force(m, s);
    if (st != SBFEM_OK) return st;
    HIP_TRY(hipMemcpyAsync(tmp.data(), m->f, m->ndof * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(sbfem::launch_fill(m->f, m->ndof, 0.0, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    std::vector<char> raw(state_bytes(m->state_mode, m->ndof));
    HIP_TRY(hipMemcpyAsync(raw.data(), which == 0 ? m->u : m->um1, raw.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    unpack_state(m->state_mode, raw.data(), m->ndof, tmp.data());
  }
  for (int64_t i = 0; i < m->ndof; ++i) host_out[3 * (int64_t)m->int2ext[i / 3] + i % 3] = tmp[i];
  if (step) *step = m->step;
  return check_flag(m);
}

sbfem_status sbfem_write_state(sbfem_mesh* m, const double* u_n, const double* u_nm1, int64_t step,
                               void* hip_stream) {
  if (!m || !u_n || !u_nm1) return fail(SBFEM_EINVAL, "null argument");
  if (step < 0) return fail(SBFEM_EINVAL, "negative step");
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<double> a(m->ndof), b(m->ndof);
  for (int64_t i = 0; i < m->ndof; ++i) {
    const int64_t e = 3 * (int64_t)m->int2ext[i / 3] + i % 3;
    a[i] = u_n[e];
    b[i] = u_nm1[e];
  }
  const std::vector<char> ra = pack_state(m->state_mode, a.data(), m->ndof);
  const std::vector<char> rb = pack_state(m->state_mode, b.data(), m->ndof);
  HIP_TRY(hipMemcpyAsync(m->u, ra.data(), ra.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(m->um1, rb.data(), rb.size(), hipMemcpyHostToDevice, s));
  const unsigned long long no_flag = ~0ull;
  HIP_TRY(hipMemcpyAsync(m->flag_d, &no_flag, sizeof(no_flag), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  m->step = step;
  m->flag_pending = false;
  *m->flag_h = no_flag;
  return SBFEM_OK;
}

sbfem_status sbfem_profile(sbfem_mesh* m, int32_t enable) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  m->profiling = enable != 0;
  return SBFEM_OK;
}

sbfem_status sbfem_profile_read(sbfem_mesh* m, double* ms, int64_t* launches) {
  if (!m || !ms || !launches) return fail(SBFEM_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(m->device));
  for (int c = 0; c < SBFEM_N_KERNEL_CLASSES; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (auto& mk : m->ev_marks) {
    HIP_TRY(hipEventSynchronize(m->ev_pool[mk.second + 1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, m->ev_pool[mk.second], m->ev_pool[mk.second + 1]));
    ms[mk.first] += t;
    launches[mk.first] += 1;
  }
  m->ev_marks.clear();
  m->ev_used = 0;
  return SBFEM_OK;
}

sbfem_status sbfem_mesh_layout(const sbfem_mesh* m, int64_t* vals, int32_t n_vals) {
  if (!m || (n_vals > 0 && !vals)) return fail(SBFEM_EINVAL, "null argument");
  for (int i = 0; i < n_vals; ++i) vals[i] = i < 10 ? m->layout[i] : 0;
  return SBFEM_OK;
}

sbfem_status sbfem_mesh_info(const sbfem_mesh* m, int64_t* device_bytes, int64_t* n_dof, int32_t* n_colours) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  if (device_bytes) *device_bytes = m->bytes;
  if (n_dof) *n_dof = m->ndof;
  if (n_colours) *n_colours = m->n_colours;
  return SBFEM_OK;
}

}  // extern "C"

extern "C" sbfem_status sbfem_set_probes(sbfem_mesh* m, int32_t n_probes, const int64_t* dofs, int64_t capacity,
                                         void* hip_stream) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  if (n_probes < 0 || capacity < 0 || (n_probes > 0 && !dofs)) return fail(SBFEM_EINVAL, "bad probe arguments");
  if (n_probes > 0 && m->assembly != SBFEM_ASM_TILED) return fail(SBFEM_EINVAL, "probes need the owner-tile assembly");
  for (int32_t i = 0; i < n_probes; ++i)
    if (dofs[i] < 0 || dofs[i] >= m->ndof) return fail(SBFEM_EINVAL, "probe %d: dof out of range", i);
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipStreamSynchronize(s));  // launches in flight may still read the old buffers
  dfree(m->alloc, m->probe_ptr);
  dfree(m->alloc, m->probes);
  dfree(m->alloc, m->probe_u);
  dfree(m->alloc, m->probe_a);
  m->n_probes = 0;
  m->probe_rows = 0;
  if (n_probes > 0) {
    std::vector<int32_t> ext2int(m->N);
    for (int64_t i = 0; i < m->N; ++i) ext2int[m->int2ext[i]] = (int32_t)i;
    const int64_t n_tiles = m->n_pure8 + m->n_mixed;
    std::vector<std::vector<int2>> per(n_tiles);
    for (int32_t i = 0; i < n_probes; ++i) {
      const int64_t node = ext2int[dofs[i] / 3];
      const int64_t t = node / m->tile_nodes;
      per[t].push_back(make_int2((int)(3 * (node - t * m->tile_nodes) + dofs[i] % 3), i));
    }
    std::vector<int32_t> ptr(n_tiles + 1, 0);
    std::vector<int2> ent;
    for (int64_t t = 0; t < n_tiles; ++t) {
      ent.insert(ent.end(), per[t].begin(), per[t].end());
      ptr[t + 1] = (int32_t)ent.size();
    }
    const size_t hist = (size_t)std::max<int64_t>(1, capacity) * n_probes;
    hipError_t e = dalloc(m->alloc, &m->probe_ptr, ptr.size());
    if (e == hipSuccess) e = dalloc(m->alloc, &m->probes, ent.size());
    if (e == hipSuccess) e = dalloc(m->alloc, &m->probe_u, hist);
    if (e == hipSuccess) e = dalloc(m->alloc, &m->probe_a, hist);
    if (e == hipSuccess) e = hipMemcpyAsync(m->probe_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(m->probes, ent.data(), ent.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      dfree(m->alloc, m->probe_ptr);
      dfree(m->alloc, m->probes);
      dfree(m->alloc, m->probe_u);
      dfree(m->alloc, m->probe_a);
      return fail(e == hipErrorOutOfMemory ? SBFEM_ENOMEM : SBFEM_EDEVICE, "probes: %s", hipGetErrorString(e));
    }
    m->n_probes = n_probes;
    m->probe_rows = capacity;
    m->probe_step0 = m->step;
  }
  return upload_tiled_args(m, s);
}

extern "C" sbfem_status sbfem_read_probes(sbfem_mesh* m, double* host_u, double* host_a, int64_t* rows,
                                          int64_t* step0, void* hip_stream) {
  if (!m) return fail(SBFEM_EINVAL, "null mesh");
  const int64_t r = std::max<int64_t>(0, std::min(m->probe_rows, m->step - m->probe_step0));
  if (rows) *rows = m->n_probes ? r : 0;
  if (step0) *step0 = m->probe_step0;
  if (m->n_probes == 0 || r == 0) return SBFEM_OK;
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t bytes = (size_t)r * m->n_probes * 8;
  if (host_u) HIP_TRY(hipMemcpyAsync(host_u, m->probe_u, bytes, hipMemcpyDeviceToHost, s));
  if (host_a) HIP_TRY(hipMemcpyAsync(host_a, m->probe_a, bytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return check_flag(m);
}

// ---------------------------------------------------------------------------------------------
// Lowest eigenfrequencies of the free vibration K phi = omega^2 M phi (Sec. 5.1): Chebyshev-
// filtered subspace iteration on A = S K S, S = diag(M^-1/2) with S = 0 on fixed dofs, whose
// eigenvalues over the free dofs are omega^2.  K is applied by the owner-tile pass in force-only
// mode to a whole block of vectors in one batched launch (one argument block per vector).

namespace {

// Symmetric eigen-decomposition of a small dense matrix by cyclic Jacobi rotations.  A is n x n
// row-major and is overwritten; w receives the eigenvalues ascending and V (row-major) the
// eigenvectors as columns in the same order.
void jacobi_eigen(std::vector<double> A, int n, std::vector<double>& w, std::vector<double>& V) {
  std::vector<double> Q(n * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * (size_t)n + i] = 1.0;
  double total = 0.0;
  for (double v : A) total += v * v;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * (size_t)n + j] * A[i * (size_t)n + j];
    if (off <= 1e-32 * total) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * (size_t)n + q];
        if (apq == 0.0) continue;
        const double app = A[p * (size_t)n + p], aqq = A[q * (size_t)n + q];
        // rotation angle that zeroes A[p][q]: tan(2 phi) = 2 apq / (aqq - app)
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(tau * tau + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[k * (size_t)n + p], akq = A[k * (size_t)n + q];
          A[k * (size_t)n + p] = c * akp - s * akq;
          A[k * (size_t)n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[p * (size_t)n + k], aqk = A[q * (size_t)n + k];
          A[p * (size_t)n + k] = c * apk - s * aqk;
          A[q * (size_t)n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[k * (size_t)n + p], qkq = Q[k * (size_t)n + q];
          Q[k * (size_t)n + p] = c * qkp - s * qkq;
          Q[k * (size_t)n + q] = s * qkp + c * qkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * (size_t)n + a] < A[b * (size_t)n + b]; });
  w.resize(n);
  V.assign(n * (size_t)n, 0.0);
  for (int j = 0; j < n; ++j) {
    w[j] = A[idx[j] * (size_t)n + idx[j]];
    for (int i = 0; i < n; ++i) V[i * (size_t)n + j] = Q[i * (size_t)n + idx[j]];
  }
}

}  // namespace

// Work of one eigenvalue solve: p argument blocks (one per column of the block), the work
// lists of the batched force-only launches over (column, tile) and (column, item), and the
// dense blocks (n x p, column-major) of the iteration.
struct EigenWork {
  Allocator alloc;
  int64_t n = 0;
  int p = 0;
  sbfem::TiledArgs* d_args = nullptr;  // p argument blocks
  sbfem::MeshRef* d_refs = nullptr;
  sbfem::TileWork* d_w8 = nullptr;
  sbfem::TileWork* d_wm = nullptr;
  int64_t n8 = 0, nm = 0;
  double* S = nullptr;                 // M^-1/2 per dof, 0 on fixed dofs
  double *X = nullptr, *AX = nullptr, *Y0 = nullptr, *Y1 = nullptr, *W = nullptr, *F = nullptr;
  void* hres = nullptr;                // hanging-cell row forces, one slice per column
  double *G = nullptr, *H = nullptr, *Q = nullptr, *theta = nullptr, *res = nullptr;
  ~EigenWork() {
    for (void** q : {(void**)&d_args, (void**)&d_refs, (void**)&d_w8, (void**)&d_wm, (void**)&S, (void**)&X,
                     (void**)&AX, (void**)&Y0, (void**)&Y1, (void**)&W, (void**)&F, (void**)&hres, (void**)&G,
                     (void**)&H, (void**)&Q, (void**)&theta, (void**)&res})
      if (*q) {
        if (alloc.release)
          alloc.release(*q, alloc.user);
        else
          (void)hipFree(*q);
        *q = nullptr;
      }
  }
};

// y = S .* x for every column of an n x p block; the operator's element pass in between
static hipError_t eigen_apply(EigenWork& W, const sbfem::TiledLaunch& L, const double* X, double* Y, hipStream_t s) {
  hipError_t e = sbfem::launch_scale_cols(W.S, X, W.W, W.n, W.p, s);
  if (e == hipSuccess) e = sbfem::launch_tiled(L, s);
  if (e == hipSuccess) e = sbfem::launch_scale_cols(W.S, W.F, Y, W.n, W.p, s);
  return e;
}

extern "C" sbfem_status sbfem_eigen_lowest(sbfem_mesh* m, int32_t k, int32_t block, int32_t degree, int32_t max_iter,
                                           double tol, double* host_omega, double* host_resid, int32_t* iterations,
                                           void* hip_stream) {
  if (!m || !host_omega) return fail(SBFEM_EINVAL, "null argument");
  if (m->assembly != SBFEM_ASM_TILED || m->prod != SBFEM_PROD_FP64 || m->state_mode != SBFEM_STATE_FP64)
    return fail(SBFEM_EINVAL, "the eigenvalue solver needs the owner-tile assembly with FP64 products and state");
  if (k < 1 || max_iter < 1 || !(tol > 0)) return fail(SBFEM_EINVAL, "bad k, max_iter or tol");
  const int64_t n = m->ndof;
  int64_t n_free = 0;
  for (int64_t i = 0; i < n; ++i) n_free += m->fixed[i] ? 0 : 1;
  const int p = block > 0 ? block : k + std::max(16, k / 2);
  if (p < k || p > n_free || p > 512) return fail(SBFEM_EINVAL, "block %d must lie in [k, min(free dofs, 512)]", p);
  const int d = degree > 0 ? degree : 20;
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)hip_stream;
  EigenWork W;
  W.alloc = m->alloc;
  W.n = n;
  W.p = p;
  const int64_t np = n * p;
  const int64_t n_tiles = m->n_pure8 + m->n_mixed;
  const size_t rbytes = (size_t)std::max<int64_t>(1, m->n_res) * 8;
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = dalloc_bytes(W.alloc, ptr, bytes);
  };
  A((void**)&W.d_args, p * sizeof(sbfem::TiledArgs));
  A((void**)&W.d_refs, p * sizeof(sbfem::MeshRef));
  A((void**)&W.d_w8, std::max<int64_t>(1, p * n_tiles) * sizeof(sbfem::TileWork));
  A((void**)&W.d_wm, std::max<int64_t>(1, p * m->n_hang) * sizeof(sbfem::TileWork));
  A((void**)&W.S, n * 8);
  for (double** b : {&W.X, &W.AX, &W.Y0, &W.Y1, &W.W, &W.F}) A((void**)b, np * 8);
  A(&W.hres, rbytes * p);
  A((void**)&W.G, (size_t)p * p * 8);
  A((void**)&W.H, (size_t)p * p * 8);
  A((void**)&W.Q, (size_t)p * p * 8);
  A((void**)&W.theta, p * 8);
  A((void**)&W.res, p * 8);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? SBFEM_ENOMEM : SBFEM_EDEVICE, "eigen work: %s",
                                   hipGetErrorString(e));
  // argument blocks: column j reads u from W_j, writes R_int to F_j, hanging rows to its slice
  std::vector<sbfem::TiledArgs> args(p);
  std::vector<sbfem::MeshRef> refs(p);
  std::vector<sbfem::TileWork> w8, wm;
  for (int j = 0; j < p; ++j) {
    args[j] = tiled_args_for(m, W.W + (int64_t)j * n, nullptr);
    args[j].f = W.F + (int64_t)j * n;
    args[j].hres = (char*)W.hres + rbytes * j;
    refs[j] = sbfem::MeshRef{W.d_args + j, 0, 0, 0};
    for (int64_t t = 0; t < n_tiles; ++t) w8.push_back({j, 0, t});
    for (int64_t t = 0; t < m->n_hang; ++t) wm.push_back({j, 0, t});
  }
  std::vector<double> S(n);
  for (int64_t i = 0; i < n; ++i) S[i] = m->fixed[i] ? 0.0 : 1.0 / std::sqrt(m->mdiag[i]);
  // seeded start block, zero on fixed dofs
  std::vector<double> X0(np);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  for (int64_t i = 0; i < np; ++i) {
    st ^= st << 13, st ^= st >> 7, st ^= st << 17;  // xorshift64
    X0[i] = m->fixed[i % n] ? 0.0 : (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  auto H2D = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  H2D(W.d_args, args.data(), p * sizeof(sbfem::TiledArgs));
  H2D(W.d_refs, refs.data(), p * sizeof(sbfem::MeshRef));
  H2D(W.d_w8, w8.data(), w8.size() * sizeof(sbfem::TileWork));
  H2D(W.d_wm, wm.data(), wm.size() * sizeof(sbfem::TileWork));
  H2D(W.S, S.data(), n * 8);
  H2D(W.X, X0.data(), np * 8);
  if (e != hipSuccess) return fail(SBFEM_EDEVICE, "eigen set-up: %s", hipGetErrorString(e));
  sbfem::TiledLaunch L = tiled_launch(m, true);
  L.refs = W.d_refs;
  L.work8 = W.d_w8;
  L.work_hang = W.d_wm;
  L.n_tiles = p * n_tiles;
  L.n_hang = p * m->n_hang;
  L.k = 0;

  const double lam_hi = 1.01 * m->lambda_bound;  // above the spectrum of A (element bound, eq. tcr)
  std::vector<double> G(p * (size_t)p), H(p * (size_t)p), lam, U, Qf(p * (size_t)p), th(p, 0.0), rs(p, 0.0);
  double a_cut = 0.0;
  int it = 0;
  bool done = false;
  for (; it < max_iter && !done; ++it) {
    if (it > 0) {
      // Chebyshev filter of degree d damping [a_cut, lam_hi] (Y_{j+1} = 2 (A - c)/e Y_j - Y_{j-1})
      const double c = 0.5 * (lam_hi + a_cut), eh = 0.5 * (lam_hi - a_cut);
      // the filter amplifies the lowest Ritz direction by T_d(x0); the degree is held so that
      // this stays below 1e8 and the block keeps its rank in FP64
      const double x0 = (c - th[0]) / eh;
      int dg = d;
      if (x0 > 1.0) dg = std::max(1, std::min(d, (int)(std::log(1e8) / std::log(x0 + std::sqrt(x0 * x0 - 1.0)))));
      double* y0 = W.X;
      double* y1 = W.Y1;
      e = eigen_apply(W, L, y0, W.AX, s);
      if (e == hipSuccess) e = sbfem::launch_axpby(1.0 / eh, W.AX, -c / eh, y0, y1, np, s);
      for (int j = 2; j <= dg && e == hipSuccess; ++j) {
        // y_j = 2/e (A - c) y_{j-1} - y_{j-2}, written over y_{j-2}
        e = eigen_apply(W, L, y1, W.AX, s);
        if (e == hipSuccess) e = sbfem::launch_axpbypcz(2.0 / eh, W.AX, -2.0 * c / eh, y1, -1.0, y0, np, s);
        std::swap(y0, y1);
      }
      // the filtered block (y1) becomes X; y0 is free again
      W.X = y1;
      W.Y1 = y0;
    }
    // two orthonormalisation passes X <- X U Lambda^-1/2 (G = X^T X = U Lambda U^T); directions
    // whose Gram eigenvalue falls below 1e-14 of the largest are replaced by fresh seeded
    // vectors between the passes
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      e = sbfem::launch_gram(W.X, W.X, n, p, W.G, s);
      if (e == hipSuccess) e = hipMemcpyAsync(G.data(), W.G, G.size() * 8, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) break;
      jacobi_eigen(G, p, lam, U);
      const double thr = 1e-14 * lam.back();
      std::fill(Qf.begin(), Qf.end(), 0.0);
      int r = 0;
      for (int j = 0; j < p; ++j) {
        if (!(lam[j] > thr)) continue;
        for (int i = 0; i < p; ++i) Qf[i * (size_t)p + r] = U[i * (size_t)p + j] / std::sqrt(lam[j]);
        ++r;
      }
      if (r == 0) return fail(SBFEM_EDEVICE, "eigen iteration: the block has no independent column");
      H2D(W.Q, Qf.data(), Qf.size() * 8);
      if (e == hipSuccess) e = sbfem::launch_gemm_small(W.X, n, p, W.Q, p, W.Y0, s);
      std::swap(W.X, W.Y0);
      if (r < p) {
        for (int64_t i = 0; i < (int64_t)(p - r) * n; ++i) {
          st ^= st << 13, st ^= st >> 7, st ^= st << 17;
          X0[i] = m->fixed[i % n] ? 0.0 : (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        H2D(W.X + (int64_t)r * n, X0.data(), (size_t)(p - r) * n * 8);
      }
    }
    // Rayleigh-Ritz: H = X^T A X = Q Theta Q^T, X <- X Q, AX <- AX Q
    if (e == hipSuccess) e = eigen_apply(W, L, W.X, W.AX, s);
    if (e == hipSuccess) e = sbfem::launch_gram(W.X, W.AX, n, p, W.H, s);
    if (e == hipSuccess) e = hipMemcpyAsync(H.data(), W.H, H.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(SBFEM_EDEVICE, "eigen iteration: %s", hipGetErrorString(e));
    for (int i = 0; i < p; ++i)  // symmetrise (rounding of the products)
      for (int j = i + 1; j < p; ++j) H[i * (size_t)p + j] = H[j * (size_t)p + i] = 0.5 * (H[i * (size_t)p + j] + H[j * (size_t)p + i]);
    jacobi_eigen(H, p, th, Qf);
    H2D(W.Q, Qf.data(), Qf.size() * 8);
    H2D(W.theta, th.data(), p * 8);
    if (e == hipSuccess) e = sbfem::launch_gemm_small(W.X, n, p, W.Q, p, W.Y0, s);
    if (e == hipSuccess) e = sbfem::launch_gemm_small(W.AX, n, p, W.Q, p, W.Y1, s);
    std::swap(W.X, W.Y0);
    std::swap(W.AX, W.Y1);
    const int r = p;
    if (e == hipSuccess) e = sbfem::launch_ritz_residual(W.X, W.AX, n, std::min(r, p), W.theta, W.res, s);
    if (e == hipSuccess) e = hipMemcpyAsync(rs.data(), W.res, p * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(SBFEM_EDEVICE, "eigen iteration: %s", hipGetErrorString(e));
    done = true;
    for (int j = 0; j < k; ++j) done = done && std::sqrt(std::max(rs[j], 0.0)) <= tol * th[j];
    a_cut = th[r - 1];
  }
  for (int j = 0; j < k; ++j) {
    host_omega[j] = std::sqrt(std::max(th[j], 0.0));
    if (host_resid) host_resid[j] = std::sqrt(std::max(rs[j], 0.0)) / std::max(th[j], 1e-300);
  }
  if (iterations) *iterations = it;
  if (!done) return fail(SBFEM_ENOTCONV, "eigenvalues not converged to %g in %d iterations", tol, max_iter);
  return SBFEM_OK;
}
