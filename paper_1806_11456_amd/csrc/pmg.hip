// pmg: MI355X (gfx950) implementation of the C-ABI declared in include/pmg.h.
// One translation unit: device helpers and kernels are included below, then the host library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/pmg.h"
#include "device.h"
#include "kernels_elem.inc"
#include "kernels_face.inc"
#include "kernels_setup.inc"
#include "kernels_mg.inc"
#include "host_basis.inc"

// Scratch of the allocation-free entry points (pmg_wall_force_noalloc): one copy per device, held until the
// process ends.  Block partials of the wall-force sum (PMG_SCRATCH_BLOCKS blocks of 256 wall nodes, 6 values
// each) followed by the 6 summed values.  Host code reaches it only through the address that pmg_ctx_create
// takes with hipGetSymbolAddress (pmg_ctx_s::scratch).
#define PMG_SCRATCH_BLOCKS 8192
#define PMG_SCRATCH_DOUBLES (6 * PMG_SCRATCH_BLOCKS + 8)
static __device__ __align__(256) double scratch[PMG_SCRATCH_DOUBLES];

// ------------------------------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------------------------------
namespace {
thread_local std::string g_err;

struct PmgError : std::runtime_error {
  pmg_status st;
  PmgError(pmg_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

#define HIPCHECK(x)                                                                          \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess)                                                                    \
      throw PmgError(e_ == hipErrorOutOfMemory ? PMG_ERR_OOM : PMG_ERR_HIP,                  \
                     std::string(#x) + ": " + hipGetErrorString(e_));                        \
  } while (0)

#define REQUIRE(c, msg) \
  do {                  \
    if (!(c)) throw PmgError(PMG_ERR_INVALID_ARG, msg); \
  } while (0)

template <class F>
pmg_status guard(F&& f) {
  try {
    f();
    return PMG_OK;
  } catch (const PmgError& e) {
    g_err = e.what();
    return e.st;
  } catch (const std::exception& e) {
    g_err = e.what();
    return PMG_ERR_INVALID_ARG;
  } catch (...) {
    g_err = "unknown error";
    return PMG_ERR_INVALID_ARG;
  }
}

inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

// device allocations owned by a level / solver
// Bytes the library has requested from hipMalloc and not yet freed (all handles, all devices).
std::atomic<long long> g_dev_bytes{0};

// Debug mode (environment PMG_POISON=1, read at every allocation): fresh device allocations are filled with
// all-ones bytes, a NaN in FP64 and FP32, so a kernel that reads memory nothing has written yet turns its
// results non-finite instead of silently using whatever the allocator left there.
static bool poison_allocations() {
  const char* e = getenv("PMG_POISON");
  return e && e[0] == '1';
}

struct DevArena {
  std::vector<void*> ptrs;
  long long bytes = 0;
  template <class T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    HIPCHECK(hipMalloc(&p, n * sizeof(T)));
    if (poison_allocations()) HIPCHECK(hipMemset(p, 0xff, n * sizeof(T)));
    ptrs.push_back(p);
    bytes += (long long)(n * sizeof(T));
    g_dev_bytes += (long long)(n * sizeof(T));
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  ~DevArena() {
    for (void* p : ptrs) (void)hipFree(p);
    g_dev_bytes -= bytes;
  }
};

inline int pack3(int a, int b, int c) { return a | (b << 8) | (c << 16); }

}  // namespace

// ------------------------------------------------------------------------------------------------
// Handles
// ------------------------------------------------------------------------------------------------
struct pmg_ctx_s {
  int device = 0;
  int lds_max = 65536;  // LDS bytes one workgroup may allocate on the device
  double* scratch = nullptr;  // device address of this device's copy of 'scratch' (hipGetSymbolAddress)
  DevArena arena;
  double* T[2] = {nullptr, nullptr};  // transfer tables per family
  std::map<std::string, int> tile_cache;  // autotuned tile targets keyed by level structure
};

struct pmg_mesh_s {
  pmg_ctx ctx;
  int64_t K;
  int M[3];
  std::vector<double> gnodes;
  std::vector<int64_t> nbr;
  std::vector<int32_t> nbrf, orient, bc;
  DevArena arena;
  double* d_gnodes = nullptr;
};

enum { PREC_F64 = 0, PREC_F32 = 1 };

// Work arrays of the operator stages in a level's precision.
template <class T>
struct Work {
  T *qf = nullptr, *Ws = nullptr, *gW = nullptr, *gf = nullptr, *Phi = nullptr;
  T* fvn = nullptr;  // [4][nf] each side's F^v . n on conforming and boundary faces
};

// LDS of the gradient kernel in values: W and the metric terms at the tile's nodes, W* and the normals at
// its face nodes.
static int grad_lds_words(int nodes, int face_nodes) { return 13 * nodes + 7 * face_nodes; }
// LDS of the divergence kernel: the nodal fluxes, and Phi at the face nodes (or the updated state at the nodes).
static int div_lds_words(int nodes, int face_nodes) { return 15 * nodes + 5 * std::max(nodes, face_nodes); }

// A range of a level's element tiles launched with one block size: the smallest of 64, 128, 256, 512 threads
// that holds the range's largest tile, one node per thread.
struct TileClass {
  int first = 0, count = 0, block = PMG_BLOCK, npt = 1, max_tile = 1, grad_words = 1, div_words = 1;
};

struct Level {
  int K = 0, nn = 0, nf = 0, nm = 0, fam = 0;
  int prec = PREC_F64;  // working precision of the operator and smoother on this level
  std::vector<int> ord, off, fo;
  int ntiles = 0, nftiles = 0, max_tile = 0, tile_target = 256;
  int grad_words = 0;                      // largest LDS of the gradient kernel over the tiles, in values
  int div_words = 0;                       // the same for the divergence kernel
  int nf1tiles = 0;                        // face tiles of p-nonconforming interfaces (mortar passes)
  int nfctiles = 0;                        // face tiles of conforming interfaces and boundaries
  int64_t nfl_conf = 0, nfl_bnd = 0, nfl_nc = 0;  // face nodes on conforming / boundary / mortar faces
  // launch ranges of the element tiles: 'all' holds every tile; with tile_split != 0 the tiles are ordered by
  // size class (tcls, one per block size) and, within a class, by problem, and the gradient (bit 0) and the
  // divergence (bit 1) launch once per class; the other kernels always launch once over every tile
  std::vector<TileClass> tcls;
  TileClass all;
  int tile_split = 0;
  DevArena arena;
  DevArena tile_arena;  // element tiles (rebuilt by the autotuner)
  int *d_ord, *d_off, *d_fo, *d_node_elem, *d_elist, *d_mface, *d_ftile, *d_ftprob;
  int *d_eoff = nullptr, *d_efo = nullptr;  // per elist entry
  int *d_wlink = nullptr, *d_mlink = nullptr, *d_f1list = nullptr;
  int4* d_fcrec = nullptr;  // conforming / boundary face tiles: {first mortar node, end, problem, 0}
  int2* d_cmap = nullptr;
  // quadrature of the no-slip wall faces: mortar node and Gauss weight w_s w_t of every wall node (host),
  // uploaded on the first wall-force evaluation
  std::vector<int> wall_mn;
  std::vector<double> wall_w;
  int* d_wall_mn = nullptr;
  double* d_wall_w = nullptr;
  int* d_ptile = nullptr;  // [tcls.size()][nprob + 1]: the element tiles of each problem within each class
  int4* d_tiles;
  FaceRec* d_faces;
  double *d_Ja, *d_invJ, *d_J, *d_Nout, *d_mgeo;  // geometry in FP64 (always kept)
  double* d_hfac = nullptr;                        // [2][nn] geometric factors of the CFL step
  Work<double> w64;
  Work<float> w32;
  LevelDevT<double> dev;
  LevelDevT<float> dev32;  // FP32 copies of the geometry (FP32 levels)
  template <class T>
  const LevelDevT<T>& devT() const {
    if constexpr (std::is_same<T, float>::value) return dev32; else return dev;
  }
  template <class T>
  const Work<T>& work() const {
    if constexpr (std::is_same<T, float>::value) return w32; else return w64;
  }
  size_t wsize() const { return prec == PREC_F32 ? sizeof(float) : sizeof(double); }
  size_t lds_trace(const TileClass& c) const { return (size_t)5 * c.max_tile * wsize(); }
  size_t lds_grad(const TileClass& c) const { return (size_t)c.grad_words * wsize(); }
  size_t lds_div(const TileClass& c) const { return (size_t)c.div_words * wsize(); }
};

struct XferTiles {
  DevArena arena;
  int4* d_restrict = nullptr;  // from the finer level to the coarser one
  int4* d_prolong = nullptr;   // from the coarser level to the finer one
  int* d_elist = nullptr;
  int ntiles = 0, lds_stride = 0;
};

struct Hier {
  int dir = -1;
  std::vector<std::shared_ptr<Level>> lv;  // 0 = coarsest
  std::vector<int> caps;                   // per level index
  std::vector<void*> Q, Q0, S, r, Sp, G, R;  // [5][nn] per level, in that level's precision
  std::vector<std::unique_ptr<XferTiles>> xf;  // xf[l]: pair (l, l+1)
  DevArena arena;
  int top() const { return (int)lv.size() - 1; }
};

// Event timing of selected kernel kinds (pmg_profile_enable / pmg_profile_read).
enum { PK_TRACE = 0, PK_FACE1 = 1, PK_GRAD = 2, PK_FACE2 = 3, PK_DIV = 4, PK_DT = 5, PK_XFER = 6, PK_N = 7 };

struct Prof {
  uint32_t mask = 0;
  int stride = 1;                 // time every stride-th launch of each selected kind
  int64_t count[PK_N] = {0};      // launches of each kind seen while selected
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  struct Rec {
    int kind;
    size_t ev;     // first of the two events
    double bytes;  // compulsory bytes of the launch
  };
  std::vector<Rec> recs;
  ~Prof() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  size_t begin(int kind, hipStream_t st) {
    if (!((mask >> kind) & 1u)) return SIZE_MAX;
    if (count[kind]++ % stride != 0) return SIZE_MAX;
    while (pool.size() < next + 2) {
      hipEvent_t e;
      // device-scope release only: the timer does not need a system-wide fence around each kernel
      HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      pool.push_back(e);
    }
    size_t i = next;
    next += 2;
    HIPCHECK(hipEventRecord(pool[i], st));
    return i;
  }
  void end(int kind, size_t i, double bytes, hipStream_t st) {
    HIPCHECK(hipEventRecord(pool[i + 1], st));
    recs.push_back({kind, i, bytes});
  }
  void read(int kind, double* ms, int64_t* n, double* bytes) {
    double tot = 0.0, b = 0.0;
    int64_t cnt = 0;
    std::vector<Rec> keep;
    for (auto& r : recs) {
      if (r.kind != kind) {
        keep.push_back(r);
        continue;
      }
      HIPCHECK(hipEventSynchronize(pool[r.ev + 1]));
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, pool[r.ev], pool[r.ev + 1]));
      tot += t;
      b += r.bytes;
      cnt++;
    }
    recs.swap(keep);
    if (recs.empty()) next = 0;
    *ms = tot;
    *n = cnt;
    if (bytes) *bytes = b;
  }
};

// Launch bracketed by events when its kind is selected; 'bytes' is the launch's compulsory traffic.
#define PROF_LAUNCH(s, kind, st, bytes, ...)                                     \
  do {                                                                           \
    size_t pi_ = (s)->prof->begin((kind), (st));                                 \
    __VA_ARGS__;                                                                 \
    if (pi_ != SIZE_MAX) (s)->prof->end((kind), pi_, (double)(bytes), (st));     \
  } while (0)

// Captured V-cycles / truncation-error cycles, replayed with hipGraphLaunch.
struct GraphKey {
  int kind;  // 0 isotropic V-cycle, 1 anisotropic 3V tau cycle, 2 FP64 isotropic V-cycle of a mixed solver
  const void *Q, *S, *tau, *act;
  int isolated;
  bool operator<(const GraphKey& o) const {
    return std::tie(kind, Q, S, tau, act, isolated) < std::tie(o.kind, o.Q, o.S, o.tau, o.act, o.isolated);
  }
};

struct pmg_solver_s {
  std::unique_ptr<Prof> prof = std::make_unique<Prof>();
  pmg_ctx ctx = nullptr;
  const pmg_mesh_s* mesh = nullptr;          // the (union) mesh
  std::unique_ptr<pmg_mesh_s> own_mesh;      // union mesh of a batch
  int nprob = 1;
  int family = 0;
  std::vector<Phys> phys;                    // per problem
  std::vector<int> eprob;                    // problem of each element
  std::vector<int> prob_elem;                // first element of each problem (nprob+1)
  pmg_mg_params mg;
  std::vector<int> orders;
  std::shared_ptr<Level> top;
  Hier iso;
  std::unique_ptr<Hier> aniso[3];
  DevArena arena;
  Phys* d_ptab = nullptr;
  int* d_eprob = nullptr;
  int* d_ones = nullptr;                     // per problem: all 1 (every problem active, nothing skipped)
  int* d_act[2] = {nullptr, nullptr};        // per problem: the problems a batched cycle advances
  std::unique_ptr<Hier> iso64;               // FP64 isotropic hierarchy of a mixed-precision solver
  std::vector<int> fp32_cycles;              // per problem: cycles of the last solve with FP32 coarse levels
  std::vector<int> halvings;                 // per problem: step-constant halvings by the divergence guard
  double* d_Qbak = nullptr;                  // [5][nn] the state at the last accepted check (divergence guard)
  double* d_Qstart = nullptr;                // [5][nn] the state at the start of the guarded solve call
  // the shared face-trace array holds the traces of this state on this level (launch-order bookkeeping:
  // k_trace is skipped when the next evaluation is of the same state on the same level)
  mutable const Level* qf_level = nullptr;
  mutable const void* qf_src = nullptr;
  mutable const int* qf_act = nullptr;  // the active-problem array of that evaluation (nullptr: all problems)
  std::vector<int> iso_caps;                 // order caps of the isotropic levels, finest first
  double* d_taumap = nullptr;                // scratch tau map of pmg_tau_nodal
  std::vector<double> history;               // residual checks of the last pmg_solve
  int64_t cycles_total = 0;                  // V-cycles run on the state since creation or restore
  unsigned long long* d_red = nullptr;       // reduction slots [NSLOTS][nprob]
  unsigned long long* d_part = nullptr;      // [K] per-tile partials of a reduction (at most K tiles)
  double* d_zero = nullptr;                  // [5][nn] zeros (absent source)
  double* d_R = nullptr;                     // [5][nn] top-level scratch residual
  double* d_G = nullptr;                     // [5][nn] top-level RK register
  int nmax = 1;
  int use_graph = 0;
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
  ~pmg_solver_s() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

enum { SLOT_DT = 0, SLOT_NORM = 1, SLOT_NORM2 = 2, NSLOTS = 3 };

static unsigned long long* slot_ptr(const pmg_solver_s* s, int slot) { return s->d_red + (size_t)slot * s->nprob; }

// ------------------------------------------------------------------------------------------------
// Level construction (Sec. 2 geometry; tiles and faces)
// ------------------------------------------------------------------------------------------------
// Element tiles: elements bucketed by (problem, order triple), packed to about 'target' nodes (one element
// when larger), so every tile has one order triple and one problem.  'split' (bit 0 the gradient, bit 1 the
// divergence): that kernel is launched per class of tiles by size (at most 64, 128, 256 nodes, larger), each
// with its own block size and LDS, so that a small tile does not hold the idle lanes of the level's largest
// block; otherwise it is one launch over every tile.
static void build_tiles(const pmg_solver_s* s, Level& L, int target, int split = 0) {
  std::map<std::pair<int, int>, std::vector<int>> buckets;
  for (int e = 0; e < L.K; e++)
    buckets[{s->eprob[e], pack3(L.ord[3 * e] + 1, L.ord[3 * e + 1] + 1, L.ord[3 * e + 2] + 1)}].push_back(e);
  std::vector<int> elist;
  std::vector<int4> tiles;
  std::vector<int> tgw, tdw;  // LDS words of each tile (gradient, divergence)
  int max_tile = 1, grad_words = 1, div_words = 1;
  for (auto& kv : buckets) {
    int key = kv.first.second;
    int n1 = key & 255, n2 = (key >> 8) & 255, n3 = key >> 16;
    int npe = n1 * n2 * n3;
    int fpe = 2 * (n2 * n3 + n1 * n3 + n1 * n2);
    int per = std::max(1, std::min(PMG_MAX_TILE_ELEMS, target / npe));
    auto lds_fits = [&](int c) {
      return (size_t)std::max(grad_lds_words(c * npe, c * fpe), div_lds_words(c * npe, c * fpe)) * L.wsize() <=
             (size_t)s->ctx->lds_max;
    };
    while (per > 1 && (per * npe > PMG_TILE_MAX || !lds_fits(per))) per--;
    const auto& es = kv.second;
    for (size_t i = 0; i < es.size(); i += per) {
      int cnt = (int)std::min<size_t>(per, es.size() - i);
      tiles.push_back(make_int4((int)elist.size(), cnt, key, cnt * npe));
      tgw.push_back(grad_lds_words(cnt * npe, cnt * fpe));
      tdw.push_back(div_lds_words(cnt * npe, cnt * fpe));
      grad_words = std::max(grad_words, tgw.back());
      div_words = std::max(div_words, tdw.back());
      max_tile = std::max(max_tile, cnt * npe);
      for (int c = 0; c < cnt; c++) elist.push_back(es[i + c]);
    }
  }
  REQUIRE(max_tile <= PMG_TILE_MAX, "element tile too large");
  REQUIRE((size_t)std::max(grad_words, div_words) * L.wsize() <= (size_t)s->ctx->lds_max,
          "element tile too large for the device's LDS");
  // launch classes; a stable reorder by class keeps each class's tiles grouped by problem
  auto block_of = [](int nodes) { return nodes <= 64 ? 0 : (nodes <= 128 ? 1 : (nodes <= PMG_BLOCK ? 2 : 3)); };
  const int ncls = split ? 4 : 1;  // tiles ordered by class whenever a kernel launches per class
  std::vector<int> tcl(tiles.size(), 0);
  if (split)
    for (size_t t = 0; t < tiles.size(); t++) tcl[t] = block_of(tiles[t].w);
  std::vector<int> order;
  order.reserve(tiles.size());
  std::vector<TileClass> cls(ncls);
  for (int c = 0; c < ncls; c++) {
    TileClass& C = cls[c];
    C.first = (int)order.size();
    for (size_t t = 0; t < tiles.size(); t++)
      if (tcl[t] == c) {
        order.push_back((int)t);
        C.max_tile = std::max(C.max_tile, tiles[t].w);
        C.grad_words = std::max(C.grad_words, tgw[t]);
        C.div_words = std::max(C.div_words, tdw[t]);
      }
    C.count = (int)order.size() - C.first;
    const int b = block_of(C.max_tile);
    C.block = b == 0 ? 64 : (b == 1 ? 128 : (b == 2 ? PMG_BLOCK : PMG_TILE_MAX));
    C.npt = 1;
  }
  std::vector<int4> otiles(tiles.size());
  for (size_t t = 0; t < order.size(); t++) otiles[t] = tiles[order[t]];
  tiles.swap(otiles);
  std::vector<int> tprob(tiles.size()), eoff(elist.size()), efo(elist.size()), ptile((size_t)ncls * (s->nprob + 1), 0);
  for (size_t t = 0; t < tiles.size(); t++) tprob[t] = s->eprob[elist[tiles[t].x]];
  // buckets are ordered by problem first: within a class each problem's tiles are one range
  for (int c = 0; c < ncls; c++) {
    int* pt = ptile.data() + (size_t)c * (s->nprob + 1);
    const int t0 = cls[c].first, t1 = cls[c].first + cls[c].count;
    for (int p = 0; p <= s->nprob; p++) pt[p] = t0;
    for (int t = t0; t < t1; t++) pt[tprob[t] + 1] = t + 1;
    for (int p = 0; p < s->nprob; p++) pt[p + 1] = std::max(pt[p + 1], pt[p]);
    for (int t = t0 + 1; t < t1; t++) REQUIRE(tprob[t] >= tprob[t - 1], "element tiles not grouped by problem");
  }
  REQUIRE((int)tiles.size() <= L.K, "more element tiles than elements");
  for (size_t k = 0; k < elist.size(); k++) {
    eoff[k] = L.off[elist[k]];
    efo[k] = L.fo[6 * elist[k]];
  }
  // tile records: {first elist entry, elements, packed node counts, nodes} and {problem, first node, first
  // face node, 0}, the bases -1 unless the tile's elements are consecutive in the node and face arrays
  std::vector<int4> rec(2 * tiles.size());
  for (size_t t = 0; t < tiles.size(); t++) {
    const int4 T = tiles[t];
    const int n1 = T.z & 255, n2 = (T.z >> 8) & 255, n3 = T.z >> 16;
    const int npe = n1 * n2 * n3, fpe = 2 * (n2 * n3 + n1 * n3 + n1 * n2);
    bool contiguous = true;
    for (int c = 0; c < T.y; c++)
      contiguous = contiguous && eoff[T.x + c] == eoff[T.x] + c * npe && efo[T.x + c] == efo[T.x] + c * fpe;
    rec[2 * t] = T;
    rec[2 * t + 1] = make_int4(tprob[t], contiguous ? eoff[T.x] : -1, contiguous ? efo[T.x] : -1, 0);
  }
  L.tile_arena.~DevArena();
  new (&L.tile_arena) DevArena();
  L.d_elist = L.tile_arena.upload(elist);
  L.d_tiles = L.tile_arena.upload(rec);
  L.d_eoff = L.tile_arena.upload(eoff);
  L.d_efo = L.tile_arena.upload(efo);
  L.d_ptile = L.tile_arena.upload(ptile);
  L.ntiles = (int)tiles.size();
  L.max_tile = max_tile;
  L.grad_words = grad_words;
  L.div_words = div_words;
  L.tile_target = target;
  L.tile_split = split;
  L.tcls = cls;
  TileClass A;
  A.first = 0;
  A.count = (int)tiles.size();
  A.max_tile = max_tile;
  A.grad_words = grad_words;
  A.div_words = div_words;
  const int ba = block_of(max_tile);
  A.block = ba == 0 ? 64 : (ba == 1 ? 128 : (ba == 2 ? PMG_BLOCK : PMG_TILE_MAX));
  A.npt = 1;
  L.all = A;
  L.dev.tiles = L.dev32.tiles = L.d_tiles;
  L.dev.elist = L.dev32.elist = L.d_elist;
  L.dev.eoff = L.dev32.eoff = L.d_eoff;
  L.dev.efo = L.dev32.efo = L.d_efo;
}

static std::shared_ptr<Level> build_level(pmg_solver_s* s, const std::vector<int>& ord, int prec = PREC_F64) {
  const pmg_mesh_s* m = s->mesh;
  auto L = std::make_shared<Level>();
  const int K = (int)m->K;
  L->K = K;
  L->fam = s->family;
  L->prec = prec;
  L->ord = ord;
  L->off.assign(K + 1, 0);
  L->fo.assign(6 * K, 0);
  int64_t nn = 0, nf = 0;
  for (int e = 0; e < K; e++) {
    int n1 = ord[3 * e] + 1, n2 = ord[3 * e + 1] + 1, n3 = ord[3 * e + 2] + 1;
    L->off[e] = (int)nn;
    nn += (int64_t)n1 * n2 * n3;
    const int fs[3] = {n2 * n3, n1 * n3, n1 * n2};
    for (int f = 0; f < 6; f++) {
      L->fo[6 * e + f] = (int)nf;
      nf += fs[f / 2];
    }
  }
  REQUIRE(12 * nn < (1ll << 31) && 12 * nf < (1ll << 31), "mesh too large for 32-bit node indexing");
  L->off[K] = (int)nn;
  L->nn = (int)nn;
  L->nf = (int)nf;

  // faces: one record per interface (master side) and per boundary face
  std::vector<FaceRec> faces;
  std::vector<int> fprob;
  for (int e = 0; e < K; e++)
    for (int f = 0; f < 6; f++) {
      int64_t g = m->nbr[6 * e + f];
      int h = m->nbrf[6 * e + f];
      bool master = g < 0 || e < g || (e == g && f < h);
      if (!master) continue;
      FaceRec F;
      memset(&F, 0, sizeof(F));
      int d = f / 2, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      F.eM = e; F.fM = f; F.o = g >= 0 ? m->orient[6 * e + f] : 0; F.bc = m->bc[6 * e + f];
      F.foM = L->fo[6 * e + f];
      F.nMs = ord[3 * e + t1] + 1;
      F.nMt = ord[3 * e + t2] + 1;
      if (g >= 0) {
        F.eS = (int)g; F.fS = h;
        int dg = h / 2, s1 = dg == 0 ? 1 : 0, s2 = dg == 2 ? 1 : 2;
        F.foS = L->fo[6 * g + h];
        F.nS1 = ord[3 * g + s1] + 1;
        F.nS2 = ord[3 * g + s2] + 1;
        int slave_s = (F.o & 4) ? F.nS2 : F.nS1, slave_t = (F.o & 4) ? F.nS1 : F.nS2;
        F.ms = std::max(F.nMs, slave_s);
        F.mt = std::max(F.nMt, slave_t);
        int m1 = (F.o & 4) ? F.mt : F.ms, m2 = (F.o & 4) ? F.ms : F.mt;
        F.flags = ((F.ms == F.nMs && F.mt == F.nMt) ? 1 : 0) | ((m1 == F.nS1 && m2 == F.nS2) ? 2 : 0);
      } else {
        F.eS = -1; F.fS = -1; F.foS = 0;
        F.ms = F.nMs; F.mt = F.nMt;
        F.flags = 1;
      }
      faces.push_back(F);
    }
  // faces ordered by (problem, p-nonconforming first, mortar size) and packed into tiles of <= PMG_FACE_TILE
  // lanes that never split a face nor mix problems or conforming with p-nonconforming interfaces
  auto mortar = [](const FaceRec& F) { return F.eS >= 0 && F.flags != 3; };
  std::stable_sort(faces.begin(), faces.end(), [&](const FaceRec& a, const FaceRec& b) {
    int pa = s->eprob[a.eM], pb = s->eprob[b.eM];
    if (pa != pb) return pa < pb;
    if (mortar(a) != mortar(b)) return mortar(a);
    return a.ms * a.mt > b.ms * b.mt;
  });
  std::vector<int> ftile{0}, mface, f1list;
  int cur = 0, cur_prob = faces.empty() ? 0 : s->eprob[faces[0].eM];
  bool cur_mortar = !faces.empty() && mortar(faces[0]);
  for (size_t i = 0; i < faces.size(); i++) {
    int nmf = faces[i].ms * faces[i].mt;
    int p = s->eprob[faces[i].eM];
    if (cur > 0 && (cur + nmf > PMG_FACE_TILE || p != cur_prob || mortar(faces[i]) != cur_mortar)) {
      if (cur_mortar) f1list.push_back((int)ftile.size() - 1);
      ftile.push_back((int)mface.size());
      cur = 0;
    }
    cur_prob = p;
    cur_mortar = mortar(faces[i]);
    faces[i].mbase = (int)mface.size();
    for (int k = 0; k < nmf; k++) mface.push_back((int)i);
    cur += nmf;
  }
  if (ftile.back() != (int)mface.size()) {
    if (cur_mortar) f1list.push_back((int)ftile.size() - 1);
    ftile.push_back((int)mface.size());
  }
  L->nftiles = (int)ftile.size() - 1;
  L->nf1tiles = (int)f1list.size();
  std::vector<int> fclist;
  for (int t = 0, k = 0; t < L->nftiles; t++) {
    if (k < L->nf1tiles && f1list[k] == t) k++;
    else fclist.push_back(t);
  }
  L->nfctiles = (int)fclist.size();
  std::vector<int> ftprob(std::max(L->nftiles, 1), 0);
  for (int t = 0; t < L->nftiles; t++) ftprob[t] = s->eprob[faces[mface[ftile[t]]].eM];
  L->nm = (int)mface.size();
  REQUIRE(8ll * L->nm + 16 < (1ll << 31), "mesh too large for 32-bit mortar indexing");

  // source of the BR1 interface state of every face node (the gradient kernel's wlink)
  // and the face nodes of each mortar node of conforming and boundary faces (the flat flux pass's cmap)
  std::vector<int> wlink(nf, PMG_WLINK_MORTAR), mlink(nf, -1);
  std::vector<int2> cmap(std::max(L->nm, 1), make_int2(-1, -1));
  for (const FaceRec& F : faces) {
    if (F.eS < 0) {
      for (int k = 0; k < F.nMs * F.nMt; k++) {
        wlink[F.foM + k] = -2 - (8 * (F.mbase + k) + F.bc);
        cmap[F.mbase + k] = make_int2(F.foM + k, -1 - F.bc);
      }
      L->nfl_bnd += F.nMs * F.nMt;
    } else if (!mortar(F)) {
      // conforming: mortar node (al, be) is master node al + nMs be and slave node i1 + nS1 i2
      for (int be = 0; be < F.mt; be++)
        for (int al = 0; al < F.ms; al++) {
          int i1, i2;
          if (F.o & 4) {
            i1 = (F.o & 1) ? F.mt - 1 - be : be;
            i2 = (F.o & 2) ? F.ms - 1 - al : al;
          } else {
            i1 = (F.o & 1) ? F.ms - 1 - al : al;
            i2 = (F.o & 2) ? F.mt - 1 - be : be;
          }
          const int fm = F.foM + al + F.nMs * be, fs = F.foS + i1 + F.nS1 * i2;
          wlink[fm] = fs;
          wlink[fs] = fm;
          mlink[fm] = mlink[fs] = F.mbase + al + F.ms * be;
          cmap[F.mbase + al + F.ms * be] = make_int2(fm, fs);
        }
      L->nfl_conf += 2 * F.ms * F.mt;
    } else {
      L->nfl_nc += F.nMs * F.nMt + F.nS1 * F.nS2;
    }
  }
  REQUIRE(L->nfl_conf + L->nfl_bnd + L->nfl_nc == nf, "face nodes not covered by the interfaces");
  for (const FaceRec& F : faces)
    if (F.eS < 0 && F.bc == 1) {
      double xs[PMG_MAXN], ws[PMG_MAXN], xt[PMG_MAXN], wt[PMG_MAXN];
      hb::nodes(F.nMs, L->fam, xs, ws);
      hb::nodes(F.nMt, L->fam, xt, wt);
      for (int b = 0; b < F.nMt; b++)
        for (int a = 0; a < F.nMs; a++) {
          L->wall_mn.push_back(F.mbase + a + F.nMs * b);
          L->wall_w.push_back(ws[a] * wt[b]);
        }
    }

  std::vector<int> node_elem(nn);
  for (int e = 0; e < K; e++)
    for (int p = L->off[e]; p < L->off[e + 1]; p++) node_elem[p] = e;

  DevArena& A = L->arena;
  L->d_ord = A.upload(ord);
  L->d_off = A.upload(L->off);
  L->d_fo = A.upload(L->fo);
  L->d_node_elem = A.upload(node_elem);
  L->d_faces = A.upload(faces);
  L->d_mface = A.upload(mface);
  L->d_ftile = A.upload(ftile);
  L->d_ftprob = A.upload(ftprob);
  L->d_wlink = A.upload(wlink);
  L->d_mlink = A.upload(mlink);
  L->d_f1list = f1list.empty() ? nullptr : A.upload(f1list);
  std::vector<int4> fcrec;
  for (int t : fclist) fcrec.push_back(make_int4(ftile[t], ftile[t + 1], ftprob[t], 0));
  L->d_fcrec = fcrec.empty() ? nullptr : A.upload(fcrec);
  L->d_cmap = A.upload(cmap);
  L->d_Ja = A.alloc<double>(9 * nn);
  L->d_invJ = A.alloc<double>(nn);
  L->d_J = A.alloc<double>(nn);
  L->d_Nout = A.alloc<double>(3 * nf);
  L->d_mgeo = A.alloc<double>(4 * (size_t)std::max(L->nm, 1));
  // Operator work arrays live only during one evaluation on one level, and every level of a solver runs on
  // one stream: the finest level allocates them (FP64) and every coarser level of every hierarchy aliases
  // them, never larger (capped orders give fewer nodes, face nodes and mortar nodes per element), FP32
  // levels in half the bytes.
  if (!s->top) {
    REQUIRE(prec == PREC_F64, "the finest level is FP64");
    Work<double>& W = L->w64;
    W.qf = A.alloc<double>(5 * nf);
    W.Ws = A.alloc<double>(4 * nf);
    W.gW = A.alloc<double>(12 * nn);
    W.gf = A.alloc<double>(12 * nf);
    W.fvn = A.alloc<double>(4 * nf);
    W.Phi = A.alloc<double>(5 * nf);
  } else {
    const Work<double>& T = s->top->w64;
    REQUIRE(nn <= s->top->nn && nf <= s->top->nf, "coarse level larger than the finest");
    if (prec == PREC_F32)
      L->w32 = Work<float>{(float*)T.qf, (float*)T.Ws, (float*)T.gW, (float*)T.gf, (float*)T.Phi, (float*)T.fvn};
    else
      L->w64 = T;
  }

  LevelDev& D = L->dev;
  memset(&D, 0, sizeof(D));
  D.K = K; D.nn = (int)nn; D.nf = (int)nf; D.nm = L->nm; D.fam = L->fam;
  D.ptab = s->d_ptab; D.eprob = s->d_eprob; D.node_elem = L->d_node_elem;
  D.dt = (const double*)slot_ptr(s, SLOT_DT);
  D.active = s->d_ones;
  D.ord = L->d_ord; D.off = L->d_off; D.fo = L->d_fo;
  D.Ja = L->d_Ja; D.invJ = L->d_invJ; D.J = L->d_J; D.Nout = L->d_Nout;
  D.faces = L->d_faces; D.mface = L->d_mface; D.ftile = L->d_ftile; D.ftprob = L->d_ftprob; D.mgeo = L->d_mgeo;
  D.wlink = L->d_wlink;
  D.mlink = L->d_mlink;
  D.cmap = L->d_cmap;
  D.T_ = s->ctx->T[L->fam];
  build_tiles(s, *L, 256);

  // geometry on the device
  DevArena tmp;
  GeoArgs G;
  G.gnodes = m->d_gnodes;
  G.M1 = m->M[0]; G.M2 = m->M[1]; G.M3 = m->M[2];
  G.node_elem = L->d_node_elem;
  G.X = tmp.alloc<double>(3 * nn);
  G.dX = tmp.alloc<double>(9 * nn);
  G.Ja = L->d_Ja; G.invJ = L->d_invJ; G.J = L->d_J;
  int nb = cdiv(nn, 256);
  k_geo_x<<<nb, 256>>>(D, G);
  k_geo_dx<<<nb, 256>>>(D, G);
  k_geo_metric<<<nb, 256>>>(D, G);
  k_geo_faces<<<L->ntiles, PMG_BLOCK>>>(D, L->d_Nout);
  if (L->nm > 0) k_mortar_geo<<<cdiv(L->nm, 256), 256>>>(D, L->d_mgeo);
  L->d_hfac = A.alloc<double>(2 * nn);
  k_hfac<<<nb, 256>>>(D, L->d_hfac);
  if (prec == PREC_F32) {
    // FP32 copies of the metric terms, each rounded once from the FP64 geometry
    LevelDevT<float>& F = L->dev32;
    memset(&F, 0, sizeof(F));
    F.K = D.K; F.nn = D.nn; F.nf = D.nf; F.nm = D.nm; F.fam = D.fam;
    F.ptab = D.ptab; F.eprob = D.eprob; F.node_elem = D.node_elem; F.dt = D.dt; F.active = D.active;
    F.ord = D.ord; F.off = D.off; F.fo = D.fo; F.faces = D.faces; F.mface = D.mface; F.ftile = D.ftile;
    F.ftprob = D.ftprob;
    F.wlink = D.wlink;
    F.mlink = D.mlink;
    F.cmap = D.cmap;
    F.T_ = D.T_;
    F.tiles = D.tiles; F.elist = D.elist; F.eoff = D.eoff; F.efo = D.efo;
    auto down = [&](const double* src, size_t n) {
      float* dst = A.alloc<float>(n);
      k_copy<<<cdiv(n, 256), 256>>>(dst, src, n);
      return (const float*)dst;
    };
    F.Ja = down(L->d_Ja, 9 * nn);
    F.invJ = down(L->d_invJ, nn);
    F.J = down(L->d_J, nn);
    F.Nout = down(L->d_Nout, 3 * nf);
    F.mgeo = down(L->d_mgeo, 4 * (size_t)std::max(L->nm, 1));
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipDeviceSynchronize());
  return L;
}

static std::unique_ptr<XferTiles> build_xfer(const pmg_solver_s* s, const Level& fine, const Level& coarse) {
  auto X = std::make_unique<XferTiles>();
  std::map<std::tuple<int, int, int>, std::vector<int>> buckets;
  for (int e = 0; e < fine.K; e++) {
    int a = pack3(fine.ord[3 * e] + 1, fine.ord[3 * e + 1] + 1, fine.ord[3 * e + 2] + 1);
    int b = pack3(coarse.ord[3 * e] + 1, coarse.ord[3 * e + 1] + 1, coarse.ord[3 * e + 2] + 1);
    buckets[{s->eprob[e], a, b}].push_back(e);
  }
  std::vector<int> elist;
  std::vector<int4> tr, tp;
  int stride = 1;
  for (auto& kv : buckets) {
    int a = std::get<1>(kv.first), b = std::get<2>(kv.first);
    const int a0 = a & 255, a1 = (a >> 8) & 255, a2 = a >> 16, b0 = b & 255, b1 = (b >> 8) & 255, b2 = b >> 16;
    const int na = a0 * a1 * a2, nb = b0 * b1 * b2;
    // largest stage of either sweep's tensor product (an order that rises in one direction and falls in
    // another can exceed both ends; between levels of one hierarchy it is max(na, nb))
    const int big = std::max({na, nb, b0 * a1 * a2, b0 * b1 * a2, a0 * b1 * b2, a0 * a1 * b2});
    int per = std::max(1, 256 / big);
    const auto& es = kv.second;
    for (size_t i = 0; i < es.size(); i += per) {
      int cnt = (int)std::min<size_t>(per, es.size() - i);
      // direct node bases when the tile's elements are consecutive on a level
      bool cf = true, cc = true;
      for (int c = 0; c < cnt; c++) {
        cf = cf && fine.off[es[i + c]] == fine.off[es[i]] + c * na;
        cc = cc && coarse.off[es[i + c]] == coarse.off[es[i]] + c * nb;
      }
      const int bf = cf ? fine.off[es[i]] : -1, bc = cc ? coarse.off[es[i]] : -1;
      tr.push_back(make_int4((int)elist.size(), cnt, a, b));
      tr.push_back(make_int4(bf, bc, 0, 0));
      tp.push_back(make_int4((int)elist.size(), cnt, b, a));
      tp.push_back(make_int4(bc, bf, 0, 0));
      stride = std::max(stride, cnt * big);
      for (int c = 0; c < cnt; c++) elist.push_back(es[i + c]);
    }
  }
  X->ntiles = (int)tr.size() / 2;
  X->lds_stride = stride;
  X->d_restrict = X->arena.upload(tr);
  X->d_prolong = X->arena.upload(tp);
  X->d_elist = X->arena.upload(elist);
  return X;
}

// ------------------------------------------------------------------------------------------------
// Operator, smoother, transfers
// ------------------------------------------------------------------------------------------------
template <class T>
static DivArgs<T> div_args(int mode) {
  DivArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.mode = mode;
  return a;
}

// Element-tile launches: per launch class of the level's tiles, the kernel instance of the class's block size
// (and, for the gradient and the divergence, one node per thread unless a tile is larger than the block),
// the tile records and per-tile outputs offset to the class's first tile.
template <class T>
static LevelDevT<T> class_dev(const LevelDevT<T>& D, const TileClass& c) {
  LevelDevT<T> Dc = D;
  Dc.tiles = D.tiles + 2 * (size_t)c.first;
  return Dc;
}

// The launch ranges of one kernel: the size classes when its bit of the level's split is set, else all tiles.
static std::vector<TileClass> launch_ranges(const Level& L, int bit) {
  if (L.tile_split & bit) return L.tcls;
  return std::vector<TileClass>(1, L.all);
}

template <class T>
static void launch_trace(const Level& L, const LevelDevT<T>& D, const T* Q, T* qf, hipStream_t st) {
  for (const TileClass& c : launch_ranges(L, 0)) {
    if (!c.count) continue;
    const LevelDevT<T> Dc = class_dev(D, c);
    const size_t lds = L.lds_trace(c);
    if (c.block == 64) k_trace<T, 64><<<c.count, 64, lds, st>>>(Dc, Q, qf);
    else if (c.block == 128) k_trace<T, 128><<<c.count, 128, lds, st>>>(Dc, Q, qf);
    else if (c.block == PMG_BLOCK) k_trace<T, PMG_BLOCK><<<c.count, PMG_BLOCK, lds, st>>>(Dc, Q, qf);
    else k_trace<T, PMG_TILE_MAX><<<c.count, PMG_TILE_MAX, lds, st>>>(Dc, Q, qf);
  }
}

template <class T>
static void launch_grad(const Level& L, const LevelDevT<T>& D, const T* Q, const T* qf, const T* Ws, int isolated,
                        T* gW, T* gf, T* fvn, T* phi, hipStream_t st) {
  for (const TileClass& c : launch_ranges(L, 1)) {
    if (!c.count) continue;
    const LevelDevT<T> Dc = class_dev(D, c);
    const size_t lds = L.lds_grad(c);
    if (c.block == 64) k_grad<T, 1, 64><<<c.count, 64, lds, st>>>(Dc, Q, qf, Ws, isolated, gW, gf, fvn, phi);
    else if (c.block == 128)
      k_grad<T, 1, 128><<<c.count, 128, lds, st>>>(Dc, Q, qf, Ws, isolated, gW, gf, fvn, phi);
    else if (c.block == PMG_BLOCK)
      k_grad<T, 1, PMG_BLOCK><<<c.count, PMG_BLOCK, lds, st>>>(Dc, Q, qf, Ws, isolated, gW, gf, fvn, phi);
    else k_grad<T, 1, PMG_TILE_MAX><<<c.count, PMG_TILE_MAX, lds, st>>>(Dc, Q, qf, Ws, isolated, gW, gf, fvn, phi);
  }
}

template <class T>
static void launch_div(const Level& L, const LevelDevT<T>& D, const T* Q, const T* gW, const T* Phi,
                       const DivArgs<T>& a, hipStream_t st) {
  for (const TileClass& c : launch_ranges(L, 2)) {
    if (!c.count) continue;
    const LevelDevT<T> Dc = class_dev(D, c);
    DivArgs<T> ac = a;
    if (ac.norm) ac.norm += c.first;
    const size_t lds = L.lds_div(c);
    if (c.block == 64) k_div<T, 1, 64><<<c.count, 64, lds, st>>>(Dc, Q, gW, Phi, ac);
    else if (c.block == 128) k_div<T, 1, 128><<<c.count, 128, lds, st>>>(Dc, Q, gW, Phi, ac);
    else if (c.block == PMG_BLOCK) k_div<T, 1, PMG_BLOCK><<<c.count, PMG_BLOCK, lds, st>>>(Dc, Q, gW, Phi, ac);
    else k_div<T, 1, PMG_TILE_MAX><<<c.count, PMG_TILE_MAX, lds, st>>>(Dc, Q, gW, Phi, ac);
  }
}

template <class T>
static void launch_dt(const Level& L, const LevelDevT<T>& D, const T* Q, unsigned long long* out, hipStream_t st) {
  for (const TileClass& c : launch_ranges(L, 0)) {
    if (!c.count) continue;
    const LevelDevT<T> Dc = class_dev(D, c);
    if (c.block == 64) k_dt<T, 64><<<c.count, 64, 0, st>>>(Dc, Q, L.d_hfac, out + c.first);
    else if (c.block == 128) k_dt<T, 128><<<c.count, 128, 0, st>>>(Dc, Q, L.d_hfac, out + c.first);
    else if (c.block == PMG_BLOCK) k_dt<T, PMG_BLOCK><<<c.count, PMG_BLOCK, 0, st>>>(Dc, Q, L.d_hfac, out + c.first);
    else k_dt<T, PMG_TILE_MAX><<<c.count, PMG_TILE_MAX, 0, st>>>(Dc, Q, L.d_hfac, out + c.first);
  }
}

// A(Q) through the stages: q traces, interface state + Roe flux, gradient (+ gradient traces), viscous
// numerical flux, divergence (the epilogue in 'a' decides what is written).  T is the level's precision.
// 'act' (nullable): the problems advanced by a cycle; tiles of the others return at once and leave their
// outputs untouched (a frozen problem's state and correction stay exactly as they are).
// The shared trace array no longer describes any state (called whenever a state or the array may change
// outside op_eval: transfers, copies, graph replays, every entry point).
static void traces_stale(const pmg_solver_s* s) {
  s->qf_level = nullptr;
  s->qf_src = nullptr;
  s->qf_act = nullptr;
}

template <class T>
static void op_eval(const pmg_solver_s* s, Level& L, const T* Q, bool isolated, const DivArgs<T>& a_in,
                    hipStream_t st, const int* act = nullptr) {
  LevelDevT<T> D = L.devT<T>();
  if (act) D.active = D.skip = act;
  const Work<T>& W = L.work<T>();
  const double nn = L.nn, nf = L.nf, nm = L.nm, w = sizeof(T);
  DivArgs<T> a = a_in;
  if (a.mode == EPI_RK) a.qf_out = W.qf;  // the stage leaves the traces of the state it writes
  // traces written for every problem serve any later evaluation; traces written with frozen problems
  // skipped serve only evaluations over the same problems
  const bool fresh = s->qf_level == &L && s->qf_src == (const void*)Q && (s->qf_act == nullptr || s->qf_act == act);
  if (!fresh)
    PROF_LAUNCH(s, PK_TRACE, st, (5 * nn + 5 * nf) * w,
                launch_trace(L, D, Q, W.qf, st));
  // BR1 interface state: the mortar pass on p-nonconforming interfaces only; the gradient kernel forms it
  // on conforming and boundary faces (and everywhere when isolated) from the traces
  const double ncf = L.nfl_nc, cf = L.nfl_conf, bf = L.nfl_bnd;
  if (!isolated && L.nf1tiles > 0)
    PROF_LAUNCH(s, PK_FACE1, st, (5 * ncf + 4 * ncf) * w,
                k_face1<T><<<L.nf1tiles, PMG_FACE_TILE, 0, st>>>(D, L.d_f1list, W.qf, W.Ws));
  // gradient: Q, J a, 1/J, N in; grad W and its traces out; W* from the traces (own and facing node, the
  // link table, the boundary normal) or from the mortar pass
  // face values of the gradient: the trace on mortar faces, F^v . n (own trace again, interface normal and
  // link) elsewhere
  const double wsrc = isolated ? 5 * nf : 10 * cf + 8 * bf + 4 * ncf + nf * 4.0 / w;
  // (isolated: the flux itself from the own trace and N_out)
  const double gout = isolated ? 5 * nf + 5 * nf : 12 * ncf + (cf + bf) * (5 + 3 + 4) + cf * 4.0 / w;
  PROF_LAUNCH(s, PK_GRAD, st, (15 * nn + 3 * nf + wsrc + 12 * nn + gout) * w,
              launch_grad(L, D, Q, (const T*)W.qf, (const T*)W.Ws, isolated ? 1 : 0, W.gW, W.gf, W.fvn, W.Phi, st));
  if (!isolated) {
    // numerical flux: the flat pass on conforming and boundary faces, the mortar pass on the others
    const double cbf = cf + bf, cm = cf / 2 + bf;  // face nodes and mortar nodes there
    if (L.nfctiles > 0)
      PROF_LAUNCH(s, PK_FACE2, st, (9 * cbf + 4 * cm + 5 * cbf) * w + 8 * cm,
                  k_face2c<T><<<L.nfctiles, PMG_FACE_TILE, 0, st>>>(D, L.d_fcrec, W.qf, W.fvn, W.Phi));
    if (L.nf1tiles > 0)
      PROF_LAUNCH(s, PK_FACE2, st, (17 * ncf + 4 * (nm - cm) + 5 * ncf) * w,
                  k_face2<T><<<L.nf1tiles, PMG_FACE_TILE, 17 * PMG_FACE_TILE * sizeof(T), st>>>(D, L.d_f1list, W.qf,
                                                                                           W.gf, W.Phi));
  }
  // divergence: Q, grad W, J a, 1/J, Phi in; the epilogue's own arrays
  double epi = 0.0;
  switch (a.mode) {
    case EPI_R: epi = (a.S ? 5 : 0) * nn + 5 * nn; break;
    case EPI_RK: epi = (a.S ? 5 : 0) * nn + (a.a != 0.0 ? 5 : 0) * nn + 10 * nn; break;
    case EPI_SRC: epi = 10 * nn + ((a.tau_map && a.Sphys) ? 5 * nn : 0); break;
    case EPI_TAU: epi = a.Sphys ? 5 * nn : 0; break;
    default: epi = 5 * nn;
  }
  if (a.mode == EPI_RK) epi += 5 * nf;  // the fused traces
  PROF_LAUNCH(s, PK_DIV, st, (27 * nn + 5 * nf + epi) * w,
              launch_div(L, D, Q, (const T*)W.gW, (const T*)W.Phi, a, st));
  s->qf_level = &L;
  s->qf_src = a.mode == EPI_RK ? (const void*)a.Qrk : (const void*)Q;
  s->qf_act = fresh && s->qf_act == nullptr ? nullptr : act;
}

static const double RK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

static void reset_slot(const pmg_solver_s* s, int slot, double v, hipStream_t st) {
  unsigned long long bits;
  memcpy(&bits, &v, sizeof(bits));
  k_fill_u64<<<cdiv(s->nprob, 64), 64, 0, st>>>(slot_ptr(s, slot), s->nprob, bits);
}

// per-problem values of a slot (waits for the stream)
static std::vector<double> read_slots(const pmg_solver_s* s, int slot, hipStream_t st) {
  std::vector<unsigned long long> bits(s->nprob);
  HIPCHECK(hipMemcpyAsync(bits.data(), slot_ptr(s, slot), bits.size() * sizeof(bits[0]), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  HIPCHECK(hipGetLastError());
  std::vector<double> v(s->nprob);
  memcpy(v.data(), bits.data(), v.size() * sizeof(double));
  return v;
}

// max over problems (NaN wins)
static double read_slot(const pmg_solver_s* s, int slot, hipStream_t st) {
  double m = 0.0;
  for (double x : read_slots(s, slot, st)) m = (x > m || x != x) ? x : m;
  return m;
}

// Per-problem min (dt) or max (norms) of the per-tile partials a kernel of level L left in d_part, into a slot.
static void reduce_tiles(const pmg_solver_s* s, const Level& L, int slot, bool take_max, const int* act,
                         hipStream_t st) {
  const double init = take_max ? 0.0 : INFINITY;
  unsigned long long bits;
  memcpy(&bits, &init, sizeof(bits));
  k_tile_reduce<<<s->nprob, 256, 0, st>>>(s->d_part, L.d_ptile, (int)L.tcls.size(), s->nprob, act,
                                           take_max ? 1 : 0, bits, slot_ptr(s, slot));
}

template <class T>
static void timestep(const pmg_solver_s* s, Level& L, const T* Q, hipStream_t st, const int* act = nullptr) {
  LevelDevT<T> D = L.devT<T>();
  if (act) D.active = D.skip = act;
  PROF_LAUNCH(s, PK_DT, st, L.nn * (5.0 * sizeof(T) + 16.0),
              launch_dt(L, D, Q, s->d_part, st));
  reduce_tiles(s, L, SLOT_DT, false, act, st);
}

template <class T>
static void smooth(const pmg_solver_s* s, Level& L, T* Q, const T* S, T* G, int sweeps, hipStream_t st,
                   const int* act = nullptr, const T* R1 = nullptr) {
  for (int it = 0; it < sweeps; it++) {
    timestep(s, L, (const T*)Q, st, act);
    for (int k = 0; k < 3; k++) {
      if (it == 0 && k == 0 && R1) {
        // the first stage's residual at this state is R1 (formed with the coarse source from the same
        // evaluation, bitwise what the stage's own evaluation would give): the update alone, then the traces
        // of the new state, which the next stage's evaluation takes as its own
        LevelDevT<T> D = L.devT<T>();
        if (act) D.active = D.skip = act;
        k_rk_first<T><<<cdiv(L.nn, 256), 256, 0, st>>>(D, R1, Q, G, RK_B[0]);
        launch_trace(L, D, (const T*)Q, L.work<T>().qf, st);
        s->qf_level = &L;
        s->qf_src = (const void*)Q;
        s->qf_act = act;
        continue;
      }
      DivArgs<T> a = div_args<T>(EPI_RK);
      a.S = S;
      a.Qrk = Q;
      a.G = G;
      a.a = RK_A[k];
      a.b = RK_B[k];
      op_eval(s, L, (const T*)Q, false, a, st, act);
    }
  }
}

// out = S - A(Q); optional per-problem max-norm into a slot
template <class T>
static void residual(const pmg_solver_s* s, Level& L, const T* Q, const T* S, T* out, bool isolated, int norm_slot,
                     hipStream_t st, const int* act = nullptr) {
  DivArgs<T> a = div_args<T>(EPI_R);
  a.S = S;
  a.out = out;
  if (norm_slot >= 0) a.norm = s->d_part;
  op_eval(s, L, Q, isolated, a, st, act);
  if (norm_slot >= 0) reduce_tiles(s, L, norm_slot, true, act, st);
}

// The same on buffers held in the level's own precision.
static void smooth_any(const pmg_solver_s* s, Level& L, void* Q, const void* S, void* G, int sweeps, hipStream_t st,
                       const int* act = nullptr, const void* R1 = nullptr) {
  if (L.prec == PREC_F32) smooth(s, L, (float*)Q, (const float*)S, (float*)G, sweeps, st, act, (const float*)R1);
  else smooth(s, L, (double*)Q, (const double*)S, (double*)G, sweeps, st, act, (const double*)R1);
}

static void residual_any(const pmg_solver_s* s, Level& L, const void* Q, const void* S, void* out, bool isolated,
                         int norm_slot, hipStream_t st, const int* act = nullptr) {
  if (L.prec == PREC_F32)
    residual(s, L, (const float*)Q, (const float*)S, (float*)out, isolated, norm_slot, st, act);
  else
    residual(s, L, (const double*)Q, (const double*)S, (double*)out, isolated, norm_slot, st, act);
}

template <class TU, class TV>
static void xfer_t(const pmg_solver_s* s, const Level& from, const Level& to, const XferTiles& X, bool prolong,
                   const TU* U, const TU* U0, TV* V, bool accumulate, hipStream_t st, TV* V0 = nullptr,
                   const TU* U2 = nullptr, TV* V2 = nullptr) {
  traces_stale(s);  // V may be a state whose traces are held
  XferArgs<TU, TV> a;
  a.tiles = prolong ? X.d_prolong : X.d_restrict;
  a.elist = X.d_elist;
  a.off_from = from.d_off;
  a.off_to = to.d_off;
  a.nn_from = from.nn;
  a.nn_to = to.nn;
  a.T = from.dev.T_;
  a.U = U;
  a.U0 = U0;
  a.V = V;
  a.V0 = V0;
  a.U2 = U2;
  a.V2 = V2;
  a.accumulate = accumulate ? 1 : 0;
  a.lds_stride = X.lds_stride;
  const double bytes = 5.0 * from.nn * ((U0 ? 2 : 1) + (U2 ? 1 : 0)) * sizeof(TU) +
                       5.0 * to.nn * ((accumulate ? 2 : 1) + (V0 ? 1 : 0) + (V2 ? 1 : 0)) * sizeof(TV);
  if (U2)
    PROF_LAUNCH(s, PK_XFER, st, bytes,
                k_transfer<TU, TV, 10><<<X.ntiles, PMG_BLOCK, (size_t)20 * X.lds_stride * sizeof(double), st>>>(a));
  else
    PROF_LAUNCH(s, PK_XFER, st, bytes,
                k_transfer<TU, TV, 5><<<X.ntiles, PMG_BLOCK, (size_t)10 * X.lds_stride * sizeof(double), st>>>(a));
}

// Transfer between two levels; 'U', 'U0' (and 'U2') in the precision of 'from', 'V' ('V0', 'V2') in that of 'to'.
static void xfer(const pmg_solver_s* s, const Level& from, const Level& to, const XferTiles& X, bool prolong,
                 const void* U, const void* U0, void* V, bool accumulate, hipStream_t st, void* V0 = nullptr,
                 const void* U2 = nullptr, void* V2 = nullptr) {
  const bool f32 = from.prec == PREC_F32, t32 = to.prec == PREC_F32;
  if (f32 && t32)
    xfer_t(s, from, to, X, prolong, (const float*)U, (const float*)U0, (float*)V, accumulate, st, (float*)V0,
           (const float*)U2, (float*)V2);
  else if (f32)
    xfer_t(s, from, to, X, prolong, (const float*)U, (const float*)U0, (double*)V, accumulate, st, (double*)V0,
           (const float*)U2, (double*)V2);
  else if (t32)
    xfer_t(s, from, to, X, prolong, (const double*)U, (const double*)U0, (float*)V, accumulate, st, (float*)V0,
           (const double*)U2, (float*)V2);
  else
    xfer_t(s, from, to, X, prolong, (const double*)U, (const double*)U0, (double*)V, accumulate, st, (double*)V0,
           (const double*)U2, (double*)V2);
}

// Transfer of caller-owned FP64 fields, whatever the levels' working precision.
static void xfer64(const pmg_solver_s* s, const Level& from, const Level& to, const XferTiles& X, bool prolong,
                   const double* U, double* V, hipStream_t st) {
  xfer_t(s, from, to, X, prolong, U, (const double*)nullptr, V, false, st);
}

template <class TD, class TS>
static void copy(TD* dst, const TS* src, size_t n, hipStream_t st) {
  k_copy<<<cdiv(n, 256), 256, 0, st>>>(dst, src, n);
}

// copy of 5 x nn values held in a level's precision
static void copy_level(const Level& L, void* dst, const void* src, hipStream_t st) {
  size_t n = 5 * (size_t)L.nn;
  if (L.prec == PREC_F32) copy((float*)dst, (const float*)src, n, st);
  else copy((double*)dst, (const double*)src, n, st);
}

// ------------------------------------------------------------------------------------------------
// Tile autotuner: per level, the element-tile size with the fastest operator evaluation
// ------------------------------------------------------------------------------------------------
static std::string level_key(const pmg_solver_s* s, const Level& L) {
  // structure = histogram of (order triple) buckets; the tile choice depends only on it
  std::map<int, int> h;
  for (int e = 0; e < L.K; e++) h[pack3(L.ord[3 * e], L.ord[3 * e + 1], L.ord[3 * e + 2])]++;
  std::string k = std::to_string(L.fam) + ":" + std::to_string(L.prec) + ":" + std::to_string(s->nprob);
  for (auto& kv : h) k += "," + std::to_string(kv.first) + "x" + std::to_string(kv.second);
  return k;
}

static void autotune_level(pmg_solver_s* s, Level& L, hipStream_t st) {
  traces_stale(s);
  std::string key = level_key(s, L);
  // cached choice: target | split << 16
  auto it = s->ctx->tile_cache.find(key);
  if (it != s->ctx->tile_cache.end()) {
    const int tg = it->second & 0xffff, sp = it->second >> 16;
    if (tg != L.tile_target || sp != L.tile_split) build_tiles(s, L, tg, sp);
    return;
  }
  DevArena tmp;
  void* Q = tmp.alloc<char>(5 * (size_t)L.nn * L.wsize());
  void* R = tmp.alloc<char>(5 * (size_t)L.nn * L.wsize());
  if (L.prec == PREC_F32) k_freestream<<<cdiv(L.nn, 256), 256, 0, st>>>(L.dev32, (float*)Q);
  else k_freestream<<<cdiv(L.nn, 256), 256, 0, st>>>(L.dev, (double*)Q);
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  uint32_t mask = s->prof->mask;
  s->prof->mask = 0;
  int best = L.tile_target, best_split = L.tile_split;
  float best_t = 1e30f;
  for (int cand = 0; cand < 20; cand++) {
    const int target = 32 << (cand >> 2), split = cand & 3;
    build_tiles(s, L, target, split);
    if (split) {
      int used = 0;
      for (const TileClass& c : L.tcls) used += c.count > 0;
      if (used < 2) continue;  // one class: the same launches as without the split
    }
    // warm-up, then enough residuals for about 4 ms of timing (at least 3, at most 64)
    HIPCHECK(hipEventRecord(e0, st));
    residual_any(s, L, Q, nullptr, R, false, -1, st);
    HIPCHECK(hipEventRecord(e1, st));
    HIPCHECK(hipEventSynchronize(e1));
    float t1 = 0.f;
    HIPCHECK(hipEventElapsedTime(&t1, e0, e1));
    const int reps = std::max(3, std::min(64, (int)(4.0f / std::max(t1, 1e-3f))));
    HIPCHECK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; r++) residual_any(s, L, Q, nullptr, R, false, -1, st);
    HIPCHECK(hipEventRecord(e1, st));
    HIPCHECK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHECK(hipEventElapsedTime(&t, e0, e1));
    t /= (float)reps;
    if (t < best_t) {
      best_t = t;
      best = target;
      best_split = split;
    }
  }
  s->prof->mask = mask;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  traces_stale(s);  // the timing state is freed
  if (best != L.tile_target || best_split != L.tile_split) build_tiles(s, L, best, best_split);
  s->ctx->tile_cache[key] = best | best_split << 16;
}

// ------------------------------------------------------------------------------------------------
// Hierarchies and the FAS V-cycle (Sec. 3.1, Algorithm "FAS: V-Cycle"; Sec. 3.3.1 anisotropic cycle)
// ------------------------------------------------------------------------------------------------
// Levels below the top run in 'coarse_prec' (FP32 in the mixed-precision cycle); the top level is FP64.
static void build_hier(pmg_solver_s* s, Hier& H, int dir, const std::vector<int>& caps_finest_first,
                       int coarse_prec = PREC_F64) {
  H.dir = dir;
  const int nlev = (int)caps_finest_first.size();
  const int K = (int)s->mesh->K;
  H.lv.resize(nlev);
  H.caps.resize(nlev);
  for (int l = 0; l < nlev; l++) {
    int cap = caps_finest_first[nlev - 1 - l];
    H.caps[l] = cap;
    if (l == nlev - 1) {
      H.lv[l] = s->top;
      continue;
    }
    std::vector<int> o(3 * K);
    for (int e = 0; e < K; e++)
      for (int d = 0; d < 3; d++) {
        int p = s->orders[3 * e + d];
        o[3 * e + d] = ((dir < 0 || dir == d) && p > cap) ? cap : p;
      }
    H.lv[l] = build_level(s, o, coarse_prec);
  }
  H.Q.assign(nlev, nullptr); H.Q0.assign(nlev, nullptr); H.S.assign(nlev, nullptr); H.r.assign(nlev, nullptr);
  H.Sp.assign(nlev, nullptr); H.G.assign(nlev, nullptr); H.R.assign(nlev, nullptr);
  for (int l = 0; l < nlev; l++) {
    size_t n = 5 * (size_t)H.lv[l]->nn * H.lv[l]->wsize();
    if (l < nlev - 1) H.Q[l] = H.arena.alloc<char>(n);  // the top state is the caller's buffer
    H.Q0[l] = H.arena.alloc<char>(n);
    H.S[l] = H.arena.alloc<char>(n);
    H.r[l] = H.arena.alloc<char>(n);
    H.Sp[l] = H.arena.alloc<char>(n);
    H.G[l] = H.arena.alloc<char>(n);
    H.R[l] = H.arena.alloc<char>(n);
  }
  H.xf.clear();
  for (int l = 0; l + 1 < nlev; l++) H.xf.push_back(build_xfer(s, *H.lv[l + 1], *H.lv[l]));
}

struct TauRec {
  double* map;
  int nt;
  int isolated;
  double* nodal = nullptr;  // optional pointwise tau of one (direction, cap) level
  int nodal_dir = -1, nodal_cap = 0;
};

struct CycleCtx {
  pmg_solver_s* s;
  Hier* H;
  hipStream_t st;
  const TauRec* tau;
  const int* act;  // nullable: the problems this cycle advances (batched solves)
};

static void restrict_to(CycleCtx& c, int l, const void* Uf, void* Uc) {
  Hier& H = *c.H;
  xfer(c.s, *H.lv[l], *H.lv[l - 1], *H.xf[l - 1], false, Uf, nullptr, Uc, false, c.st);
}

static void absmax(CycleCtx& c, const Level& L, const void* U, int slot) {
  size_t n = 5 * (size_t)L.nn;
  reset_slot(c.s, slot, 0.0, c.st);
  if (L.prec == PREC_F32)
    k_absmax<<<std::min(cdiv(n, 256), 2048), 256, 0, c.st>>>((const float*)U, n, slot_ptr(c.s, slot));
  else
    k_absmax<<<std::min(cdiv(n, 256), 2048), 256, 0, c.st>>>((const double*)U, n, slot_ptr(c.s, slot));
}

// pre-smoothing; leaves R[l] = S - A(Q) and returns ||R||_inf when tuning (else 0)
static double pre_smooth(CycleCtx& c, int l, int top) {
  pmg_solver_s* s = c.s;
  Hier& H = *c.H;
  Level& L = *H.lv[l];
  const pmg_mg_params& P = s->mg;
  // below the top, the coarse source left the first stage's residual in R[l] (not with tuning)
  const void* R1 = (l < top && !P.tuning) ? H.R[l] : nullptr;
  if (l == 0) {
    smooth_any(s, L, H.Q[l], H.S[l], H.G[l], P.beta_coarse, c.st, c.act, R1);
    return 0.0;
  }
  if (!P.tuning) {
    smooth_any(s, L, H.Q[l], H.S[l], H.G[l], P.beta_pre, c.st, c.act, R1);
    residual_any(s, L, H.Q[l], H.S[l], H.R[l], false, -1, c.st, c.act);
    return 0.0;
  }
  double rf = 0.0;
  for (int rep = 0; rep < std::max(1, P.max_repeats); rep++) {
    smooth_any(s, L, H.Q[l], H.S[l], H.G[l], P.beta_pre, c.st, c.act);
    residual_any(s, L, H.Q[l], H.S[l], H.R[l], false, SLOT_NORM, c.st, c.act);
    restrict_to(c, l, H.R[l], H.r[l - 1]);
    absmax(c, *H.lv[l - 1], H.r[l - 1], SLOT_NORM2);
    rf = read_slot(s, SLOT_NORM, c.st);
    double rc = read_slot(s, SLOT_NORM2, c.st);
    if (rf != rf) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual during pre-smoothing");
    if (rf < P.eta * rc) break;
  }
  return rf;
}

static void post_smooth(CycleCtx& c, int l, double rpre) {
  pmg_solver_s* s = c.s;
  Hier& H = *c.H;
  Level& L = *H.lv[l];
  const pmg_mg_params& P = s->mg;
  if (!P.tuning) {
    smooth_any(s, L, H.Q[l], H.S[l], H.G[l], P.beta_post, c.st, c.act);
    return;
  }
  for (int rep = 0; rep < std::max(1, P.max_repeats); rep++) {
    smooth_any(s, L, H.Q[l], H.S[l], H.G[l], P.beta_post, c.st, c.act);
    residual_any(s, L, H.Q[l], H.S[l], H.R[l], false, SLOT_NORM, c.st, c.act);
    double r = read_slot(s, SLOT_NORM, c.st);
    if (r != r) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual during post-smoothing");
    if (r <= rpre) break;
  }
}

// coarse source S = A(Q~) + r (eq. FAScoarseSource) in the level's precision; in FP64 levels the truncation
// error of the anisotropic cycle is taken from the same evaluation (or from an extra isolated one)
template <class T>
static void coarse_source(CycleCtx& c, int l) {
  pmg_solver_s* s = c.s;
  Hier& H = *c.H;
  Level& L = *H.lv[l];
  DivArgs<T> a = div_args<T>(EPI_SRC);
  a.S = (const T*)H.r[l];
  a.out = (T*)H.S[l];
  if (!s->mg.tuning) a.out2 = (T*)H.R[l];  // the first pre-smoothing stage's residual (pre_smooth)
  const bool rec = c.tau != nullptr;
  T* nodal = nullptr;
  if (rec && c.tau->nodal && H.dir == c.tau->nodal_dir && H.caps[l] == c.tau->nodal_cap) {
    if constexpr (std::is_same<T, double>::value) nodal = c.tau->nodal;
  }
  if (rec && !c.tau->isolated) {
    a.tau_out = nodal;
    a.Sphys = (const T*)H.Sp[l];
    a.tau_map = c.tau->map;
    a.tau_dir = H.dir;
    a.tau_cap = H.caps[l];
    a.tau_nt = c.tau->nt;
    a.tau_top_ord = s->top->d_ord;
  }
  op_eval(s, L, (const T*)H.Q[l], false, a, c.st, c.act);
  if (rec && c.tau->isolated) {
    DivArgs<T> t = div_args<T>(EPI_TAU);
    t.tau_out = nodal;
    t.Sphys = (const T*)H.Sp[l];
    t.tau_map = c.tau->map;
    t.tau_dir = H.dir;
    t.tau_cap = H.caps[l];
    t.tau_nt = c.tau->nt;
    t.tau_top_ord = s->top->d_ord;
    op_eval(s, L, (const T*)H.Q[l], true, t, c.st, c.act);
  }
}

static void vcycle_rec(CycleCtx& c, int l, int top) {
  pmg_solver_s* s = c.s;
  Hier& H = *c.H;
  Level& L = *H.lv[l];
  if (l < top) {
    if (L.prec == PREC_F32) {
      if (c.tau) throw PmgError(PMG_ERR_INVALID_ARG, "truncation errors are recorded on FP64 levels only");
      coarse_source<float>(c, l);
    } else {
      coarse_source<double>(c, l);
    }
  }
  // Q~0: the restricted state (on an FP32 level, the FP64 restriction rounded once), written by the
  // restriction with Q~; the correction Q~ - Q~0 is formed in the level's precision and added to the finer
  // level in its precision
  double rpre = pre_smooth(c, l, top);
  if (l > 0) {
    Level& Lc = *H.lv[l - 1];
    // the state and the residual restricted in one launch
    xfer(s, L, Lc, *H.xf[l - 1], false, H.Q[l], nullptr, H.Q[l - 1], false, c.st, H.Q0[l - 1],
         s->mg.tuning ? nullptr : H.R[l], s->mg.tuning ? nullptr : H.r[l - 1]);
    vcycle_rec(c, l - 1, top);
    // Q <- Q + I (Q~c - Q~c_0)   (eqs. FASIterError, FASCorrectSol)
    xfer(s, Lc, L, *H.xf[l - 1], true, H.Q[l - 1], H.Q0[l - 1], H.Q[l], true, c.st);
    post_smooth(c, l, rpre);
  }
}

// physical source on every level: the top one as given (zero when absent), restricted level by level
static void set_sources(CycleCtx& c, const double* S) {
  Hier& H = *c.H;
  int top = H.top();
  size_t n = 5 * (size_t)H.lv[top]->nn;
  copy((double*)H.Sp[top], S ? S : c.s->d_zero, n, c.st);
  for (int l = top; l > 0; l--) restrict_to(c, l, H.Sp[l], H.Sp[l - 1]);
}

static void run_vcycles(pmg_solver_s* s, Hier& H, double* Q, const double* S, int ncycles, const TauRec* tau,
                        hipStream_t st, const int* act = nullptr) {
  traces_stale(s);
  CycleCtx c{s, &H, st, tau, act};
  int top = H.top();
  H.Q[top] = Q;
  set_sources(c, S);
  copy((double*)H.S[top], (const double*)H.Sp[top], 5 * (size_t)H.lv[top]->nn, st);
  for (int k = 0; k < ncycles; k++) vcycle_rec(c, top, top);
  H.Q[top] = nullptr;
}

static Hier& aniso_hier(pmg_solver_s* s, int d) {
  if (!s->aniso[d]) {
    int pmax = 1;
    for (int64_t e = 0; e < s->mesh->K; e++) pmax = std::max(pmax, s->orders[3 * e + d]);
    std::vector<int> caps;
    for (int c = pmax; c >= 1; c--) caps.push_back(c);
    s->aniso[d] = std::make_unique<Hier>();
    build_hier(s, *s->aniso[d], d, caps);  // truncation errors are FP64 quantities: FP64 levels
  }
  return *s->aniso[d];
}

// The FP64 isotropic hierarchy: the solver's own one, or for a mixed-precision solver a second one with
// FP64 coarse levels, built on first use (outside any graph capture).
static Hier& iso_f64(pmg_solver_s* s) {
  if (s->mg.precision != 1) return s->iso;
  if (!s->iso64) {
    auto H = std::make_unique<Hier>();
    build_hier(s, *H, -1, s->iso_caps, PREC_F64);
    s->iso64 = std::move(H);
  }
  return *s->iso64;
}

static void tau_cycles(pmg_solver_s* s, double* Q, const double* S, const TauRec& tau, hipStream_t st) {
  size_t n = (size_t)s->mesh->K * 3 * tau.nt;
  k_fill<<<cdiv(n, 256), 256, 0, st>>>(tau.map, n, (double)NAN);
  for (int d = 0; d < 3; d++) {
    Hier& H = aniso_hier(s, d);
    if (H.lv.size() < 2) continue;
    run_vcycles(s, H, Q, S, 1, &tau, st);
  }
}

// Replays a captured graph of 'body' (a fixed launch sequence without host synchronisation) on 'st'.
template <class F>
static void run_graph(pmg_solver_s* s, const GraphKey& key, int repeats, hipStream_t st, F&& body) {
  auto it = s->graphs.find(key);
  if (it == s->graphs.end()) {
    if (!s->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    uint32_t mask = s->prof->mask;
    s->prof->mask = 0;  // no timing events inside a graph
    HIPCHECK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      body(s->cap_stream);
    } catch (...) {
      (void)hipStreamEndCapture(s->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      s->prof->mask = mask;
      throw;
    }
    HIPCHECK(hipStreamEndCapture(s->cap_stream, &g));
    s->prof->mask = mask;
    hipGraphExec_t ex = nullptr;
    HIPCHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    it = s->graphs.emplace(key, ex).first;
  }
  for (int r = 0; r < repeats; r++) HIPCHECK(hipGraphLaunch(it->second, st));
  traces_stale(s);  // the replay rewrote the trace array
}

// ------------------------------------------------------------------------------------------------
// Solver construction (one problem or a batch)
// ------------------------------------------------------------------------------------------------
static void set_phys(Phys& P, const pmg_physics* ph) {
  P.gamma = ph->gamma;
  P.gm1 = ph->gamma - 1.0;
  P.gM2 = ph->gamma * ph->mach * ph->mach;
  P.Re = ph->reynolds;
  P.invRe = 1.0 / ph->reynolds;
  P.kcoef = 1.0 / ((ph->gamma - 1.0) * ph->prandtl * ph->mach * ph->mach);
  P.suth = ph->sutherland;
  P.suth1 = 1.0 + ph->sutherland;
  P.cfl_adv = ph->cfl_adv;
  P.cfl_visc = ph->cfl_visc;
  P.pinf = 1.0 / (ph->gamma * ph->mach * ph->mach);
  P.rhoE_inf = P.pinf / (ph->gamma - 1.0) + 0.5;
  P.visc_const = ph->viscosity_model == 1;
  P.family = ph->node_family;
}

// Mapping of one mesh raised to higher orders M' >= M (exact: its polynomial sampled at the new nodes).
static void elevate_mapping(const pmg_mesh_s* m, const int Mn[3], std::vector<double>& out) {
  const int M1 = m->M[0], M2 = m->M[1], M3 = m->M[2];
  const size_t per_old = (size_t)(M1 + 1) * (M2 + 1) * (M3 + 1) * 3;
  auto lag = [](int M, int a, double x) {
    double v = 1.0;
    for (int k = 0; k <= M; k++)
      if (k != a) v *= (x - (-1.0 + 2.0 * k / M)) / ((-1.0 + 2.0 * a / M) - (-1.0 + 2.0 * k / M));
    return v;
  };
  for (int64_t e = 0; e < m->K; e++) {
    const double* g = m->gnodes.data() + e * per_old;
    for (int k = 0; k <= Mn[2]; k++)
      for (int j = 0; j <= Mn[1]; j++)
        for (int i = 0; i <= Mn[0]; i++) {
          double x[3] = {-1.0 + 2.0 * i / Mn[0], -1.0 + 2.0 * j / Mn[1], -1.0 + 2.0 * k / Mn[2]};
          double p[3] = {0, 0, 0};
          for (int c3 = 0; c3 <= M3; c3++)
            for (int c2 = 0; c2 <= M2; c2++)
              for (int c1 = 0; c1 <= M1; c1++) {
                double wgt = lag(M1, c1, x[0]) * lag(M2, c2, x[1]) * lag(M3, c3, x[2]);
                const double* q = g + ((c3 * (M2 + 1) + c2) * (M1 + 1) + c1) * 3;
                for (int c = 0; c < 3; c++) p[c] += wgt * q[c];
              }
          for (int c = 0; c < 3; c++) out.push_back(p[c]);
        }
  }
}

static pmg_solver_s* create_solver(pmg_ctx ctx, const std::vector<const pmg_mesh_s*>& meshes,
                                   const std::vector<const int32_t*>& orders, const pmg_physics* phys,
                                   const pmg_mg_params* mg) {
  REQUIRE(!meshes.empty(), "no problems");
  HIPCHECK(hipSetDevice(ctx->device));
  auto s = std::make_unique<pmg_solver_s>();
  s->ctx = ctx;
  const int n = (int)meshes.size();
  s->nprob = n;
  s->family = phys[0].node_family;
  for (int p = 0; p < n; p++) {
    REQUIRE(meshes[p] && orders[p], "NULL mesh or orders");
    REQUIRE(meshes[p]->ctx == ctx, "mesh belongs to another context");
    const pmg_physics* ph = &phys[p];
    REQUIRE(ph->node_family == 0 || ph->node_family == 1, "node_family must be 0 or 1");
    REQUIRE(ph->node_family == s->family, "every problem of a batch must use the same node family");
    REQUIRE(ph->mach > 0 && ph->reynolds > 0 && ph->gamma > 1 && ph->prandtl > 0, "bad physics parameters");
    REQUIRE(ph->cfl_adv > 0 && ph->cfl_visc > 0, "CFL constants must be positive");
    Phys P;
    set_phys(P, ph);
    s->phys.push_back(P);
  }
  // the (union) mesh
  if (n == 1) {
    s->mesh = meshes[0];
  } else {
    auto um = std::make_unique<pmg_mesh_s>();
    um->ctx = ctx;
    um->K = 0;
    for (int d = 0; d < 3; d++) {
      um->M[d] = 1;
      for (auto* m : meshes) um->M[d] = std::max(um->M[d], m->M[d]);
    }
    for (auto* m : meshes) {
      int64_t base = um->K;
      if (m->M[0] == um->M[0] && m->M[1] == um->M[1] && m->M[2] == um->M[2])
        um->gnodes.insert(um->gnodes.end(), m->gnodes.begin(), m->gnodes.end());
      else
        elevate_mapping(m, um->M, um->gnodes);
      for (int64_t v : m->nbr) um->nbr.push_back(v < 0 ? v : v + base);
      um->nbrf.insert(um->nbrf.end(), m->nbrf.begin(), m->nbrf.end());
      um->orient.insert(um->orient.end(), m->orient.begin(), m->orient.end());
      um->bc.insert(um->bc.end(), m->bc.begin(), m->bc.end());
      um->K += m->K;
    }
    REQUIRE(um->K < (1 << 30), "batch too large");
    um->d_gnodes = um->arena.upload(um->gnodes);
    s->own_mesh = std::move(um);
    s->mesh = s->own_mesh.get();
  }
  const int K = (int)s->mesh->K;
  s->prob_elem.push_back(0);
  int pmax_first = -1;
  for (int p = 0; p < n; p++) {
    int pmax = 1;
    for (int64_t e = 0; e < meshes[p]->K; e++)
      for (int d = 0; d < 3; d++) {
        int v = orders[p][3 * e + d];
        REQUIRE(v >= 1 && v <= PMG_MAXN - 1, "orders must be 1..7");
        s->orders.push_back(v);
        pmax = std::max(pmax, v);
      }
    if (p == 0) pmax_first = pmax;
    // equal maximum orders keep every problem's level sequence identical to its own solve
    REQUIRE(pmax == pmax_first, "every problem of a batch must have the same maximum order");
    for (int64_t e = 0; e < meshes[p]->K; e++) s->eprob.push_back(p);
    s->prob_elem.push_back(s->prob_elem.back() + (int)meshes[p]->K);
  }
  s->nmax = pmax_first;
  pmg_mg_params d;
  memset(&d, 0, sizeof(d));
  d.beta_pre = d.beta_post = d.beta_coarse = 3;
  d.eta = 1.1;
  d.max_repeats = 10;
  d.fmg_threshold = 0.1;
  s->mg = mg ? *mg : d;
  REQUIRE(s->mg.beta_pre >= 0 && s->mg.beta_post >= 0 && s->mg.beta_coarse >= 0, "negative sweep count");
  REQUIRE(!(n > 1 && s->mg.tuning), "residual-based smoothing tuning is per problem: not available in a batch");
  s->d_ptab = s->arena.upload(s->phys);
  s->d_eprob = s->arena.upload(s->eprob);
  s->d_ones = s->arena.upload(std::vector<int>(n, 1));
  s->d_act[0] = s->arena.upload(std::vector<int>(n, 1));
  s->d_act[1] = s->arena.upload(std::vector<int>(n, 1));
  s->d_red = s->arena.alloc<unsigned long long>((size_t)NSLOTS * n);
  s->d_part = s->arena.alloc<unsigned long long>((size_t)K);
  s->top = build_level(s.get(), s->orders);
  if (!s->top->wall_mn.empty()) {
    // quadrature lists of the no-slip walls of the finest level (read by the wall-force entry points)
    s->top->d_wall_mn = s->top->arena.upload(s->top->wall_mn);
    s->top->d_wall_w = s->top->arena.upload(s->top->wall_w);
  }
  std::vector<int> caps;
  if (mg && mg->n_levels > 0 && mg->level_caps) {
    caps.assign(mg->level_caps, mg->level_caps + mg->n_levels);
    for (size_t i = 1; i < caps.size(); i++) REQUIRE(caps[i] < caps[i - 1] && caps[i] >= 1, "level caps must decrease");
  } else {
    int nl = (mg && mg->n_levels > 0) ? mg->n_levels : s->nmax;
    for (int c = s->nmax; c >= 1 && (int)caps.size() < nl; c--) caps.push_back(c);
  }
  REQUIRE(s->mg.precision == 0 || s->mg.precision == 1, "precision must be 0 (FP64) or 1 (mixed)");
  REQUIRE(s->mg.mixed_patience >= 0, "negative mixed_patience");
  s->mg.level_caps = nullptr;
  s->iso_caps = caps;
  s->fp32_cycles.assign(n, 0);
  s->halvings.assign(n, 0);
  REQUIRE(s->mg.guard >= 0, "negative guard");
  build_hier(s.get(), s->iso, -1, caps, s->mg.precision == 1 ? PREC_F32 : PREC_F64);
  size_t nq = 5 * (size_t)s->top->nn;
  s->d_zero = s->arena.alloc<double>(nq);
  s->d_R = s->arena.alloc<double>(nq);
  s->d_G = s->arena.alloc<double>(nq);
  k_fill<<<cdiv(nq, 256), 256>>>(s->d_zero, nq, 0.0);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipDeviceSynchronize());
  (void)K;
  return s.release();
}

// ------------------------------------------------------------------------------------------------
// Device footprint of a solver, counted on the host from the connectivity and the orders (the same
// allocations as the level, hierarchy and solver construction above; the anisotropic truncation-error
// hierarchies are built on first use and are not included).
// ------------------------------------------------------------------------------------------------
struct LevelCount {
  double nn = 0, nf = 0, nm = 0, nfaces = 0, ntiles = 0, nwall = 0;
};

static LevelCount count_level(const pmg_mesh_s* m, const std::vector<int>& ord, const std::vector<int>& eprob) {
  LevelCount c;
  const int64_t K = m->K;
  std::map<std::pair<int, int>, int> buckets;
  for (int64_t e = 0; e < K; e++) {
    int n1 = ord[3 * e] + 1, n2 = ord[3 * e + 1] + 1, n3 = ord[3 * e + 2] + 1;
    c.nn += (double)n1 * n2 * n3;
    c.nf += 2.0 * (n2 * n3 + n1 * n3 + n1 * n2);
    buckets[{eprob[e], pack3(n1, n2, n3)}]++;
    for (int f = 0; f < 6; f++) {
      int64_t g = m->nbr[6 * e + f];
      int h = m->nbrf[6 * e + f];
      if (!(g < 0 || e < g || (e == g && f < h))) continue;
      int d = f / 2, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      int ms = ord[3 * e + t1] + 1, mt = ord[3 * e + t2] + 1;
      if (g >= 0) {
        int o = m->orient[6 * e + f], dg = h / 2, s1 = dg == 0 ? 1 : 0, s2 = dg == 2 ? 1 : 2;
        int nS1 = ord[3 * g + s1] + 1, nS2 = ord[3 * g + s2] + 1;
        ms = std::max(ms, (o & 4) ? nS2 : nS1);
        mt = std::max(mt, (o & 4) ? nS1 : nS2);
      }
      c.nm += (double)ms * mt;
      c.nfaces += 1;
      if (g < 0 && m->bc[6 * e + f] == 1) c.nwall += (double)ms * mt;
    }
  }
  for (auto& kv : buckets) {
    int key = kv.first.second, n1 = key & 255, n2 = (key >> 8) & 255, n3 = key >> 16, npe = n1 * n2 * n3;
    int fpe = 2 * (n2 * n3 + n1 * n3 + n1 * n2);
    int per = std::max(1, std::min(PMG_MAX_TILE_ELEMS, 256 / npe));
    while (per > 1 && (per * npe > PMG_TILE_MAX ||
                       std::max(grad_lds_words(per * npe, per * fpe), div_lds_words(per * npe, per * fpe)) * 8.0 >
                           m->ctx->lds_max))
      per--;
    c.ntiles += (kv.second + per - 1) / per;
  }
  return c;
}

// Bytes of one level (arena + element tiles) and of its hierarchy arrays ('top': the state is the caller's).
static double level_bytes(const LevelCount& c, int64_t K, int prec, bool top) {
  const double w = prec == PREC_F32 ? 4.0 : 8.0;
  double b = 4.0 * (3 * K + (K + 1) + 6 * K + c.nn + c.nm + c.nm / 64.0 + 2) + sizeof(FaceRec) * c.nfaces;
  b += 8.0 * (9 * c.nn + c.nn + c.nn + 3 * c.nf + 4 * std::max(c.nm, 1.0) + 2 * c.nn);  // FP64 geometry
  if (top) b += 8.0 * (5 * c.nf + 4 * c.nf + 12 * c.nn + 12 * c.nf + 5 * c.nf + 4 * c.nf);  // shared work arrays
  if (top) b += 12.0 * c.nwall;  // wall quadrature lists
  if (prec == PREC_F32) b += 4.0 * (9 * c.nn + c.nn + c.nn + 3 * c.nf + 4 * std::max(c.nm, 1.0));
  b += 3 * 4.0 * K + 32.0 * c.ntiles + 4.0 * (c.nm / 64.0 + 2);  // element tiles (+ offsets), face-tile problems
  b += 8.0 * c.nf + 16.0 * (c.nm / 64.0 + 2);  // interface links (state, mortar node), face-tile list and records
  b += 8.0 * std::max(c.nm, 1.0);              // face nodes of the conforming mortar nodes
  b += 4.0 * 2;                                // tile range of the problem
  b += (top ? 6.0 : 7.0) * 5 * c.nn * w;           // Q (not on top), Q0, S, r, Sp, G, R
  b += 4.0 * K + 2 * 32.0 * K;                     // transfer tiles towards this level (upper bound)
  return b;
}

// Footprint of one problem's solver as constructed; 'transient' receives the extra bytes held while a
// level's geometry is being built, 'switch_extra' the FP64 coarse hierarchy a mixed-precision solver builds
// when it switches precision.
static double solver_footprint(const pmg_mesh_s* m, const int32_t* orders, const pmg_mg_params* mg,
                               double* transient, double* switch_extra) {
  const int64_t K = m->K;
  std::vector<int> ord(orders, orders + 3 * K), eprob(K, 0);
  int pmax = 1;
  for (int v : ord) pmax = std::max(pmax, v);
  std::vector<int> caps;
  if (mg && mg->n_levels > 0 && mg->level_caps) caps.assign(mg->level_caps, mg->level_caps + mg->n_levels);
  else
    for (int c = pmax; c >= 1 && (int)caps.size() < ((mg && mg->n_levels > 0) ? mg->n_levels : pmax); c--)
      caps.push_back(c);
  const bool mixed = mg && mg->precision == 1;
  double b = 0.0, nn_top = 0.0, extra = 0.0;
  for (size_t l = 0; l < caps.size(); l++) {
    std::vector<int> o(ord);
    if (l > 0)
      for (auto& v : o) v = std::min(v, caps[l]);
    LevelCount c = count_level(m, o, eprob);
    if (l == 0) {
      nn_top = c.nn;
      b += level_bytes(c, K, PREC_F64, true);
    } else {
      b += level_bytes(c, K, mixed ? PREC_F32 : PREC_F64, false);
      if (mixed) extra += level_bytes(c, K, PREC_F64, false);  // the FP64 hierarchy of the precision switch
    }
  }
  b += sizeof(Phys) + 4.0 * K + 3 * 4.0 + 8.0 * NSLOTS + 8.0 * K + 3 * 5 * 8.0 * nn_top;  // solver arrays
  if (mg && mg->guard > 0) b += 2 * 5 * 8.0 * nn_top;  // the divergence guard's two state copies
  if (transient) *transient = 12.0 * 8.0 * nn_top;
  if (switch_extra) *switch_extra = extra;
  return b;
}

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------
extern "C" {

const char* pmg_last_error(void) { return g_err.c_str(); }

pmg_status pmg_ctx_create(int hip_device, pmg_ctx* out) {
  return guard([&] {
    REQUIRE(out, "out is NULL");
    int n = 0;
    HIPCHECK(hipGetDeviceCount(&n));
    REQUIRE(hip_device >= 0 && hip_device < n, "no such HIP device");
    HIPCHECK(hipSetDevice(hip_device));
    auto c = std::make_unique<pmg_ctx_s>();
    c->device = hip_device;
    HIPCHECK(hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device));
    BasisTables B[2];
    std::vector<double> T(TMAT_STRIDE);
    for (int fam = 0; fam < 2; fam++) {
      hb::build_family(fam, B[fam], T.data());
      c->T[fam] = c->arena.upload(T);
    }
    HIPCHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_tab), B, sizeof(B)));
    // this device's copy of the static scratch array of the allocation-free entry points: host code uses
    // only the address returned here, never the array's name
    void* sp = nullptr;
    HIPCHECK(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
    REQUIRE(sp != nullptr, "no device address for the scratch array");
    c->scratch = (double*)sp;
    *out = c.release();
  });
}

void pmg_ctx_destroy(pmg_ctx ctx) { delete ctx; }

pmg_status pmg_mesh_create(pmg_ctx ctx, int64_t K, const int32_t M[3], const double* geom_nodes,
                           const int64_t* nbr_elem, const int32_t* nbr_face, const int32_t* orient,
                           const int32_t* bc, pmg_mesh* out) {
  return guard([&] {
    REQUIRE(ctx && out && M && geom_nodes && nbr_elem && nbr_face && orient && bc, "NULL argument");
    REQUIRE(K > 0 && K < (1 << 30), "K out of range");
    for (int d = 0; d < 3; d++) REQUIRE(M[d] >= 1 && M[d] <= 4, "mapping order must be 1..4");
    for (int64_t e = 0; e < K; e++)
      for (int f = 0; f < 6; f++) {
        int64_t g = nbr_elem[6 * e + f];
        if (g < 0) {
          REQUIRE(bc[6 * e + f] >= 1 && bc[6 * e + f] <= 4, "boundary face without a boundary tag (1..4)");
          continue;
        }
        REQUIRE(g < K, "neighbour index out of range");
        int h = nbr_face[6 * e + f];
        REQUIRE(h >= 0 && h < 6, "neighbour face out of range");
        REQUIRE(orient[6 * e + f] >= 0 && orient[6 * e + f] < 8, "orientation code out of range");
        REQUIRE(nbr_elem[6 * g + h] == e && nbr_face[6 * g + h] == f, "neighbour does not point back");
      }
    HIPCHECK(hipSetDevice(ctx->device));
    auto m = std::make_unique<pmg_mesh_s>();
    m->ctx = ctx;
    m->K = K;
    for (int d = 0; d < 3; d++) m->M[d] = M[d];
    size_t ng = (size_t)K * (M[0] + 1) * (M[1] + 1) * (M[2] + 1) * 3;
    m->gnodes.assign(geom_nodes, geom_nodes + ng);
    m->nbr.assign(nbr_elem, nbr_elem + 6 * K);
    m->nbrf.assign(nbr_face, nbr_face + 6 * K);
    m->orient.assign(orient, orient + 6 * K);
    m->bc.assign(bc, bc + 6 * K);
    m->d_gnodes = m->arena.upload(m->gnodes);
    *out = m.release();
  });
}

void pmg_mesh_destroy(pmg_mesh mesh) { delete mesh; }

pmg_status pmg_solver_create(pmg_ctx ctx, pmg_mesh mesh, const int32_t* orders, const pmg_physics* ph,
                             const pmg_mg_params* mg, pmg_solver* out) {
  return guard([&] {
    REQUIRE(ctx && mesh && orders && ph && out, "NULL argument");
    *out = create_solver(ctx, {mesh}, {orders}, ph, mg);
  });
}

pmg_status pmg_batch_create(pmg_ctx ctx, int n, const pmg_mesh* meshes, const int32_t* const* orders,
                            const pmg_physics* phys, const pmg_mg_params* mg, pmg_solver* out) {
  return guard([&] {
    REQUIRE(ctx && meshes && orders && phys && out && n >= 1, "bad argument");
    std::vector<const pmg_mesh_s*> ms(meshes, meshes + n);
    std::vector<const int32_t*> os(orders, orders + n);
    *out = create_solver(ctx, ms, os, phys, mg);
  });
}

void pmg_solver_destroy(pmg_solver s) { delete s; }

pmg_status pmg_state_layout(pmg_solver s, int64_t* n_nodes, int64_t* elem_node_offset) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    if (n_nodes) *n_nodes = s->top->nn;
    if (elem_node_offset)
      for (int e = 0; e <= s->top->K; e++) elem_node_offset[e] = s->top->off[e];
  });
}

pmg_status pmg_batch_layout(pmg_solver s, int* n_problems, int64_t* problem_node_offset) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    if (n_problems) *n_problems = s->nprob;
    if (problem_node_offset)
      for (int p = 0; p <= s->nprob; p++) problem_node_offset[p] = s->top->off[s->prob_elem[p]];
  });
}

pmg_status pmg_init_freestream(pmg_solver s, double* Q_dev, void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev, "NULL argument");
    traces_stale(s);
    k_freestream<<<cdiv(s->top->nn, 256), 256, 0, (hipStream_t)stream>>>(s->top->dev, Q_dev);
    HIPCHECK(hipGetLastError());
  });
}

pmg_status pmg_residual(pmg_solver s, int op, const double* Q_dev, const double* S_dev, double* R_dev,
                        double* res_inf_host, void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && R_dev, "NULL argument");
    traces_stale(s);
    REQUIRE(op == 0 || op == 1, "op must be 0 (DG) or 1 (isolated)");
    hipStream_t st = (hipStream_t)stream;
    residual(s, *s->top, Q_dev, S_dev, R_dev, op == 1, res_inf_host ? SLOT_NORM : -1, st);
    HIPCHECK(hipGetLastError());
    if (res_inf_host) {
      *res_inf_host = read_slot(s, SLOT_NORM, st);
      if (*res_inf_host != *res_inf_host) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual");
    }
  });
}

pmg_status pmg_batch_norms(pmg_solver s, const double* Q_dev, const double* S_dev, double* res_inf_host,
                           void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && res_inf_host, "NULL argument");
    traces_stale(s);
    hipStream_t st = (hipStream_t)stream;
    residual(s, *s->top, Q_dev, S_dev, s->d_R, false, SLOT_NORM, st);
    std::vector<double> v = read_slots(s, SLOT_NORM, st);
    for (int p = 0; p < s->nprob; p++) res_inf_host[p] = v[p];
  });
}

pmg_status pmg_timestep(pmg_solver s, const double* Q_dev, double* dt_host, void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && dt_host, "NULL argument");
    traces_stale(s);
    hipStream_t st = (hipStream_t)stream;
    timestep(s, *s->top, Q_dev, st);
    std::vector<double> v = read_slots(s, SLOT_DT, st);
    double m = INFINITY;
    for (double x : v) m = std::min(m, x);
    *dt_host = m;
  });
}

pmg_status pmg_smooth(pmg_solver s, double* Q_dev, const double* S_dev, int sweeps, void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && sweeps >= 0, "bad argument");
    traces_stale(s);
    smooth(s, *s->top, Q_dev, S_dev, s->d_G, sweeps, (hipStream_t)stream);
    HIPCHECK(hipGetLastError());
  });
}

static Hier& pick_hier(pmg_solver s, int hierarchy) {
  REQUIRE(hierarchy >= -1 && hierarchy <= 2, "hierarchy must be -1, 0, 1 or 2");
  return hierarchy < 0 ? s->iso : aniso_hier(s, hierarchy);
}

pmg_status pmg_level_info(pmg_solver s, int hierarchy, int level, int32_t* n_levels, int64_t* n_nodes,
                          int32_t* orders) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    Hier& H = pick_hier(s, hierarchy);
    if (n_levels) *n_levels = (int32_t)H.lv.size();
    if (level < 0) return;
    REQUIRE(level < (int)H.lv.size(), "level out of range");
    if (n_nodes) *n_nodes = H.lv[level]->nn;
    if (orders) memcpy(orders, H.lv[level]->ord.data(), sizeof(int32_t) * 3 * s->mesh->K);
  });
}

pmg_status pmg_restrict(pmg_solver s, int hierarchy, int level, const double* Uf, double* Uc, void* stream) {
  return guard([&] {
    REQUIRE(s && Uf && Uc, "NULL argument");
    traces_stale(s);
    Hier& H = pick_hier(s, hierarchy);
    REQUIRE(level >= 1 && level < (int)H.lv.size(), "level out of range");
    xfer64(s, *H.lv[level], *H.lv[level - 1], *H.xf[level - 1], false, Uf, Uc, (hipStream_t)stream);
    HIPCHECK(hipGetLastError());
  });
}

pmg_status pmg_prolong(pmg_solver s, int hierarchy, int level, const double* Uc, double* Uf, void* stream) {
  return guard([&] {
    REQUIRE(s && Uf && Uc, "NULL argument");
    traces_stale(s);
    Hier& H = pick_hier(s, hierarchy);
    REQUIRE(level >= 0 && level + 1 < (int)H.lv.size(), "level out of range");
    xfer64(s, *H.lv[level], *H.lv[level + 1], *H.xf[level], true, Uc, Uf, (hipStream_t)stream);
    HIPCHECK(hipGetLastError());
  });
}

pmg_status pmg_set_graph(pmg_solver s, int enable) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    s->use_graph = enable ? 1 : 0;
  });
}

pmg_status pmg_autotune(pmg_solver s, void* stream) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    traces_stale(s);
    hipStream_t st = (hipStream_t)stream;
    std::vector<Level*> done;
    auto tune = [&](Hier& H) {
      for (auto& l : H.lv)
        if (std::find(done.begin(), done.end(), l.get()) == done.end()) {
          autotune_level(s, *l, st);
          done.push_back(l.get());
        }
    };
    tune(s->iso);
    if (s->iso64) tune(*s->iso64);
    for (int d = 0; d < 3; d++)
      if (s->aniso[d]) tune(*s->aniso[d]);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);  // tiles changed: recapture
    s->graphs.clear();
    HIPCHECK(hipStreamSynchronize(st));
  });
}

pmg_status pmg_set_tiles(pmg_solver s, int hierarchy, int level, int tile_target, int split) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    REQUIRE(tile_target == 32 || tile_target == 64 || tile_target == 128 || tile_target == 256 || tile_target == 512,
            "tile_target must be 32, 64, 128, 256 or 512");
    REQUIRE(split >= 0 && split <= 3, "split must be 0..3");
    Hier& H = pick_hier(s, hierarchy);
    REQUIRE(level >= 0 && level < (int)H.lv.size(), "level out of range");
    HIPCHECK(hipDeviceSynchronize());  // launches in flight read the tile arrays that are replaced
    traces_stale(s);
    build_tiles(s, *H.lv[level], tile_target, split);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);  // tiles changed: recapture
    s->graphs.clear();
  });
}

pmg_status pmg_level_tiles(pmg_solver s, int hierarchy, int level, int32_t* tile_target, int32_t* split) {
  return guard([&] {
    REQUIRE(s && tile_target, "NULL argument");
    Hier& H = pick_hier(s, hierarchy);
    REQUIRE(level >= 0 && level < (int)H.lv.size(), "level out of range");
    *tile_target = H.lv[level]->tile_target;
    if (split) *split = H.lv[level]->tile_split;
  });
}

pmg_status pmg_vcycle(pmg_solver s, double* Q_dev, const double* S_dev, int n_cycles, double* res_inf_host,
                      void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && n_cycles >= 0, "bad argument");
    traces_stale(s);
    hipStream_t st = (hipStream_t)stream;
    if (s->use_graph && !s->mg.tuning && n_cycles > 0) {
      // sources once eagerly, then the captured cycle (its sources are re-derived inside; identical work)
      GraphKey key{0, Q_dev, S_dev, nullptr, nullptr, 0};
      run_graph(s, key, n_cycles, st, [&](hipStream_t cs) { run_vcycles(s, s->iso, Q_dev, S_dev, 1, nullptr, cs); });
    } else {
      run_vcycles(s, s->iso, Q_dev, S_dev, n_cycles, nullptr, st);
    }
    s->cycles_total += n_cycles;
    HIPCHECK(hipGetLastError());
    if (res_inf_host) {
      residual(s, *s->top, Q_dev, S_dev, s->d_R, false, SLOT_NORM, st);
      *res_inf_host = read_slot(s, SLOT_NORM, st);
      if (*res_inf_host != *res_inf_host) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual");
    }
  });
}

// One batched V-cycle of hierarchy H that advances the problems flagged in 'act' (device array).
static void cycle_once(pmg_solver_s* s, Hier& H, int kind, double* Q, const double* S, const int* act,
                       hipStream_t st) {
  if (s->use_graph && !s->mg.tuning) {
    GraphKey key{kind, Q, S, nullptr, act, 0};
    run_graph(s, key, 1, st, [&](hipStream_t cs) { run_vcycles(s, H, Q, S, 1, nullptr, cs, act); });
  } else {
    run_vcycles(s, H, Q, S, 1, nullptr, st, act);
  }
}

// Stopping and precision bookkeeping of one problem: FP32 coarse levels are kept while the residual keeps
// reaching new minima; after 'patience' stalled cycles (the FP32 round-off floor of the coarse correction)
// the problem continues with FP64 coarse levels.  At a round-off floor the residual hovers at its minimum,
// up one cycle and down the next; a start-up transient raises it cycle after cycle.  So a cycle counts as
// stalled only when it reaches no new minimum, the residual has fallen below its first value, stays within
// twice its best value and did not rise over the cycle.  A cycle the divergence guard rolled back is no
// evidence either way and restarts the count.
struct MixedState {
  int f32 = 0, stall = 0;
  double best = INFINITY, first = -1.0, prev = INFINITY;
  void update(double r, int patience) {
    if (!f32) return;
    if (first < 0.0) first = r;
    if (r < best) {
      best = r;
      stall = 0;
    } else if (best < first && r <= 2.0 * best && r <= prev && ++stall >= patience) {
      f32 = 0;
    }
    prev = r;
  }
  void rolled_back() {
    stall = 0;
    prev = INFINITY;
  }
};

// Divergence guard of the solve drivers (mg.guard > 0).  At every residual check, a problem whose residual is
// no longer finite, or grew more than 1e4-fold over the last cycle, gets back its state of the previous check
// (or, when it fails again before any accepted check, its state at the start of the call) and continues with
// both explicit step constants halved, at most mg.guard times; a problem that still fails then keeps its last
// accepted state and is reported as failed (pmg_solve fails; pmg_batch_solve freezes it and carries on with
// the others).  The halved constants stay with the solver.  The state of every problem is copied at each
// accepted check (one device copy of the finest state; a V-cycle costs far more).
struct DivGuard {
  pmg_solver_s* s;
  hipStream_t st;
  std::vector<double> r_ok, r_start;  // residuals at the last accepted check and at the start of the call
  std::vector<int> fails;             // per problem: failures since its last accepted check
  std::vector<int> rolled;            // per problem: restored at the last check
  bool first = true;
  DivGuard(pmg_solver_s* s_, hipStream_t st_)
      : s(s_), st(st_), r_ok(s_->nprob, 0.0), r_start(s_->nprob, 0.0), fails(s_->nprob, 0), rolled(s_->nprob, 0) {
    if (s->mg.guard > 0 && !s->d_Qbak) {
      s->d_Qbak = s->arena.alloc<double>(5 * (size_t)s->top->nn);
      s->d_Qstart = s->arena.alloc<double>(5 * (size_t)s->top->nn);
    }
  }
  void restore(int p, const double* from, double* Q) {
    const Level& T = *s->top;
    const size_t n0 = T.off[s->prob_elem[p]], n1 = T.off[s->prob_elem[p + 1]];
    for (int v = 0; v < 5; v++)
      HIPCHECK(hipMemcpyAsync(Q + (size_t)v * T.nn + n0, from + (size_t)v * T.nn + n0, (n1 - n0) * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
  }
  // r: this check's residuals (restored problems get the residual of the state they got back); advanced: the
  // problems the last cycle moved.  Returns the problems that used up their halvings (restored to their last
  // accepted state).
  std::vector<int> check(std::vector<double>& r, const std::vector<int>& advanced, double* Q) {
    std::vector<int> failed;
    std::fill(rolled.begin(), rolled.end(), 0);
    if (s->mg.guard <= 0) return failed;
    const Level& T = *s->top;
    bool restored = false;
    for (int p = 0; p < s->nprob && !first; p++) {
      if (!advanced[p]) continue;
      if (r[p] == r[p] && !(r[p] > 1e4 * r_ok[p])) {
        fails[p] = 0;
        continue;
      }
      restored = true;
      rolled[p] = 1;
      if (s->halvings[p] >= s->mg.guard) {
        restore(p, s->d_Qbak, Q);
        r[p] = r_ok[p];
        failed.push_back(p);
        continue;
      }
      s->halvings[p]++;
      const bool again = ++fails[p] >= 2;
      restore(p, again ? s->d_Qstart : s->d_Qbak, Q);
      r[p] = again ? r_start[p] : r_ok[p];
      s->phys[p].cfl_adv *= 0.5;
      s->phys[p].cfl_visc *= 0.5;
      HIPCHECK(hipStreamSynchronize(st));
      HIPCHECK(hipMemcpy(s->d_ptab + p, &s->phys[p], sizeof(Phys), hipMemcpyHostToDevice));
    }
    if (restored) traces_stale(s);
    if (first) {
      r_start = r;
      copy(s->d_Qstart, (const double*)Q, 5 * (size_t)T.nn, st);
    }
    for (int p = 0; p < s->nprob; p++) r_ok[p] = r[p];
    first = false;
    copy(s->d_Qbak, (const double*)Q, 5 * (size_t)T.nn, st);
    return failed;
  }
};

pmg_status pmg_solve(pmg_solver s, double* Q_dev, const double* S_dev, double tol, int max_cycles, int* cycles_out,
                     double* res_inf_out, void* stream) {
  pmg_status rc = guard([&] {
    REQUIRE(s && Q_dev && max_cycles >= 0, "bad argument");
    traces_stale(s);  // the caller may have changed Q in place since the last evaluation
    hipStream_t st = (hipStream_t)stream;
    const bool mixed = s->mg.precision == 1;
    const int patience = s->mg.mixed_patience > 0 ? s->mg.mixed_patience : 4;
    Hier* H = &s->iso;
    CycleCtx c{s, H, st, nullptr, nullptr};
    const int top = H->top();
    H->Q[top] = Q_dev;
    set_sources(c, S_dev);
    int cycles = 0, c32 = 0;
    double r = 0.0;
    if (s->mg.fmg) {
      for (int l = top; l > 0; l--) restrict_to(c, l, H->Q[l], H->Q[l - 1]);
      for (int l = 0; l < top; l++) {
        Level& L = *H->lv[l];
        copy_level(L, H->S[l], H->Sp[l], st);
        for (;;) {
          residual_any(s, L, H->Q[l], H->Sp[l], H->R[l], false, SLOT_NORM, st);
          r = read_slot(s, SLOT_NORM, st);
          if (r != r) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual in the FMG start");
          if (r < s->mg.fmg_threshold || cycles >= max_cycles) break;
          vcycle_rec(c, l, l);
          cycles++;
          c32 += mixed;
        }
        xfer(s, L, *H->lv[l + 1], *H->xf[l], true, H->Q[l], nullptr, H->Q[l + 1], false, st);
      }
    }
    H->Q[top] = nullptr;
    MixedState ms;
    ms.f32 = mixed;
    s->history.clear();
    DivGuard dg(s, st);
    const std::vector<int> all(s->nprob, 1);  // a batch handle: every problem advances with the others
    for (;;) {
      residual(s, *s->top, (const double*)Q_dev, S_dev, s->d_R, false, SLOT_NORM, st);
      std::vector<double> rv = read_slots(s, SLOT_NORM, st);  // per problem
      if (!dg.check(rv, all, Q_dev).empty()) throw PmgError(PMG_ERR_NONPHYSICAL, "diverged after every step halving");
      r = 0.0;
      bool rolled = false;
      for (int p = 0; p < s->nprob; p++) {
        r = (rv[p] > r || rv[p] != rv[p]) ? rv[p] : r;  // max over problems, NaN wins
        rolled = rolled || dg.rolled[p];
      }
      s->history.push_back(r);
      if (r != r) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual");
      if (r < tol || cycles >= max_cycles) break;
      if (rolled) ms.rolled_back();
      else ms.update(r, patience);
      if (s->mg.tuning) {
        // residual-based tuning reads norms inside the cycle: eager launches
        Hier& Hc = ms.f32 ? s->iso : iso_f64(s);
        run_vcycles(s, Hc, Q_dev, S_dev, 1, nullptr, st);
      } else {
        cycle_once(s, ms.f32 ? s->iso : iso_f64(s), ms.f32 ? 0 : 2, Q_dev, S_dev, nullptr, st);
      }
      cycles++;
      s->cycles_total++;
      c32 += ms.f32;
    }
    s->fp32_cycles.assign(s->nprob, c32);
    if (cycles_out) *cycles_out = cycles;
    if (res_inf_out) *res_inf_out = r;
    if (r >= tol) throw PmgError(PMG_ERR_NOT_CONVERGED, "max_cycles reached before the tolerance");
  });
  if (s) s->iso.Q[s->iso.top()] = nullptr;
  return rc;
}

pmg_status pmg_batch_solve(pmg_solver s, double* Q_dev, const double* S_dev, double tol, int max_cycles,
                           int32_t* cycles_out, double* res_inf_out, void* stream) {
  pmg_status rc = guard([&] {
    REQUIRE(s && Q_dev && max_cycles >= 0, "bad argument");
    traces_stale(s);  // the caller may have changed Q in place since the last evaluation
    hipStream_t st = (hipStream_t)stream;
    const int n = s->nprob;
    const bool mixed = s->mg.precision == 1;
    const int patience = s->mg.mixed_patience > 0 ? s->mg.mixed_patience : 4;
    std::vector<int> active(n, 1), cyc(n, 0), c32(n, 0), a32(n, 0), a64(n, 0);
    std::vector<MixedState> ms(n);
    for (auto& m : ms) m.f32 = mixed;
    std::vector<double> r(n, 0.0);
    DivGuard dg(s, st);
    std::vector<int> dead(n, 0);  // problems the guard gave up on: frozen at their last accepted state
    for (;;) {
      residual(s, *s->top, (const double*)Q_dev, S_dev, s->d_R, false, SLOT_NORM, st);  // every problem
      r = read_slots(s, SLOT_NORM, st);
      for (int p : dg.check(r, active, Q_dev)) dead[p] = 1;
      int n32 = 0, n64 = 0;
      for (int p = 0; p < n; p++) {
        if (dead[p]) active[p] = 0;
        if (r[p] != r[p]) throw PmgError(PMG_ERR_NONPHYSICAL, "non-finite residual in problem " + std::to_string(p));
        if (active[p] && (r[p] < tol || cyc[p] >= max_cycles)) active[p] = 0;  // converged problems freeze
        if (active[p] && dg.rolled[p]) ms[p].rolled_back();
        else if (active[p]) ms[p].update(r[p], patience);
        a32[p] = active[p] && ms[p].f32;
        a64[p] = active[p] && !ms[p].f32;
        n32 += a32[p];
        n64 += a64[p];
      }
      if (n32 + n64 == 0) break;
      // the previous iteration's reads synchronised the stream: the flag arrays are free to rewrite
      if (n32) {
        HIPCHECK(hipMemcpyAsync(s->d_act[0], a32.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        cycle_once(s, s->iso, 0, Q_dev, S_dev, s->d_act[0], st);
      }
      if (n64) {
        HIPCHECK(hipMemcpyAsync(s->d_act[1], a64.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        cycle_once(s, iso_f64(s), mixed ? 2 : 0, Q_dev, S_dev, s->d_act[1], st);
      }
      for (int p = 0; p < n; p++) {
        cyc[p] += active[p];
        c32[p] += a32[p];
      }
    }
    s->fp32_cycles = c32;
    bool all = true;
    std::string gave_up;
    for (int p = 0; p < n; p++) {
      if (cycles_out) cycles_out[p] = cyc[p];
      if (res_inf_out) res_inf_out[p] = dead[p] ? (double)NAN : r[p];
      all = all && r[p] < tol;
      if (dead[p]) gave_up += (gave_up.empty() ? "" : ", ") + std::to_string(p);
    }
    if (!gave_up.empty())
      throw PmgError(PMG_ERR_NONPHYSICAL, "diverged after every step halving (frozen at their last accepted "
                                          "state, residual reported as NaN): problems " + gave_up);
    if (!all) throw PmgError(PMG_ERR_NOT_CONVERGED, "max_cycles reached before the tolerance in some problem");
  });
  return rc;
}

pmg_status pmg_guard_stats(pmg_solver s, int32_t* halvings, double* cfl_host) {
  return guard([&] {
    REQUIRE(s && halvings, "NULL argument");
    for (int p = 0; p < s->nprob; p++) {
      halvings[p] = s->halvings[p];
      if (cfl_host) {
        cfl_host[2 * p] = s->phys[p].cfl_adv;
        cfl_host[2 * p + 1] = s->phys[p].cfl_visc;
      }
    }
  });
}

pmg_status pmg_solve_stats(pmg_solver s, int32_t* fp32_cycles) {
  return guard([&] {
    REQUIRE(s && fp32_cycles, "NULL argument");
    for (int p = 0; p < s->nprob; p++) fp32_cycles[p] = s->fp32_cycles[p];
  });
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Serving: continuous batching of steady solves at V-cycle granularity
// ------------------------------------------------------------------------------------------------
// Each admitted request owns a solver (its levels stay resident until it retires) and runs on one of the
// server's streams.  One worker thread loops: admit queued requests whose footprint fits the budget,
// launch one V-cycle of every resident request that is not done, launch every resident request's residual
// norm with its copy to pinned host memory, wait for the streams once, then retire converged (or failed)
// requests and free their memory.  Every request sees the launch sequence of pmg_solve (residual, test,
// cycle), so its result does not depend on what else is resident.
struct ServerReq {
  uint64_t ticket = 0;
  const pmg_mesh_s* mesh = nullptr;
  std::vector<int32_t> orders;
  pmg_physics phys;
  pmg_mg_params mg;
  std::vector<int32_t> caps;
  double tol = 0.0;
  int max_cycles = 0;
  double* Q = nullptr;
  double est = 0.0;  // admitted bytes (steady footprint + construction transient)
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  pmg_solver_s* s = nullptr;
  hipStream_t st = nullptr;
  double* h_norm = nullptr;  // pinned
  int cycles = 0, fp32 = 0, status = -1, done = 0;
  bool cycle_next = false;
  MixedState ms;
  double r = 0.0;
  std::string err;
};

struct pmg_server_s {
  pmg_ctx ctx = nullptr;
  double budget = 0.0;
  int graph = 1;
  int batched = 0;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<ServerReq>> queue;
  std::vector<std::shared_ptr<ServerReq>> resident;  // the worker thread's own list (no lock)
  std::map<uint64_t, std::shared_ptr<ServerReq>> all;
  // the fields below are read and written under mu
  double used = 0.0, peak = 0.0;
  uint64_t next_ticket = 1;
  int64_t completed = 0, iterations = 0;
  int n_resident = 0, max_resident = 0;  // published by the worker after each change of 'resident'
  bool stop = false;
  std::string fatal;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

static void server_retire(pmg_server_s* sv, const std::shared_ptr<ServerReq>& r, int status) {
  delete r->s;
  r->s = nullptr;
  if (r->h_norm) (void)hipHostFree(r->h_norm);
  r->h_norm = nullptr;
  std::lock_guard<std::mutex> lk(sv->mu);
  r->status = status;
  r->t_done = sv->now();
  r->done = 1;
  sv->used -= r->est;
  sv->completed++;
}

static void server_loop(pmg_server_s* sv) {
  if (hipSetDevice(sv->ctx->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->fatal = "hipSetDevice failed in the server thread";
    return;
  }
  size_t rr = 0;
  for (;;) {
    std::vector<std::shared_ptr<ServerReq>> admit;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->resident.empty()) sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop) break;
      // first come, first served: a request waits until everything submitted before it is admitted
      while (!sv->queue.empty() && sv->used + sv->queue.front()->est <= sv->budget) {
        auto r = sv->queue.front();
        sv->queue.pop_front();
        sv->used += r->est;
        sv->peak = std::max(sv->peak, sv->used);
        r->t_admit = sv->now();
        admit.push_back(r);
      }
    }
    for (auto& r : admit) {
      pmg_status rc = guard([&] {
        r->mg.level_caps = r->caps.empty() ? nullptr : r->caps.data();
        r->s = create_solver(sv->ctx, {r->mesh}, {r->orders.data()}, &r->phys, &r->mg);
        r->s->use_graph = sv->graph;
        r->st = sv->streams[rr++ % sv->streams.size()];
        HIPCHECK(hipHostMalloc((void**)&r->h_norm, sizeof(double), hipHostMallocDefault));
        r->ms.f32 = r->s->mg.precision == 1;
      });
      if (rc != PMG_OK) {
        r->err = g_err;
        server_retire(sv, r, rc);
        continue;
      }
      sv->resident.push_back(r);
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->n_resident = (int)sv->resident.size();
      sv->max_resident = std::max(sv->max_resident, sv->n_resident);
    }
    if (sv->resident.empty()) continue;
    // one iteration: the decided cycle, then the residual norm, for every resident request
    for (auto& r : sv->resident) {
      pmg_status rc = guard([&] {
        pmg_solver_s* s = r->s;
        if (r->cycle_next) {
          cycle_once(s, r->ms.f32 ? s->iso : iso_f64(s), r->ms.f32 ? 0 : 2, r->Q, nullptr, nullptr, r->st);
          r->cycles++;
          r->fp32 += r->ms.f32;
        }
        residual(s, *s->top, (const double*)r->Q, (const double*)nullptr, s->d_R, false, SLOT_NORM, r->st);
        HIPCHECK(hipMemcpyAsync(r->h_norm, slot_ptr(s, SLOT_NORM), sizeof(double), hipMemcpyDeviceToHost, r->st));
      });
      if (rc != PMG_OK) {
        r->err = g_err;
        r->status = rc;
      }
    }
    for (hipStream_t st : sv->streams) (void)hipStreamSynchronize(st);
    std::vector<std::shared_ptr<ServerReq>> keep;
    for (auto& r : sv->resident) {
      int status = r->status >= 0 ? r->status : -1;
      if (status < 0) {
        r->r = *r->h_norm;
        if (r->r != r->r) {
          r->err = "non-finite residual";
          status = PMG_ERR_NONPHYSICAL;
        } else if (r->r < r->tol) {
          status = PMG_OK;
        } else if (r->cycles >= r->max_cycles) {
          status = PMG_ERR_NOT_CONVERGED;
        } else {
          r->ms.update(r->r, r->s->mg.mixed_patience > 0 ? r->s->mg.mixed_patience : 4);
          r->cycle_next = true;
        }
      }
      if (status >= 0) server_retire(sv, r, status);
      else keep.push_back(r);
    }
    sv->resident.swap(keep);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->iterations++;
    sv->n_resident = (int)sv->resident.size();
  }
  for (auto& r : sv->resident) server_retire(sv, r, PMG_ERR_BUSY);
  sv->resident.clear();
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->n_resident = 0;
}

// Batched serving: the resident requests that can share a solver (same multigrid parameters, node family and
// maximum order) advance together in one union solver (the batch solver of pmg_batch_create) on one stream,
// one batched V-cycle per iteration for the requests on FP32 coarse levels and one for those on FP64 ones,
// then one residual launch for every member.  The union holds the members' states; it is rebuilt when its
// membership changes (each remaining member's state copied out, the new union built, the states copied in)
// and a retiring member's state is copied back before it is reported done.  Per-problem arithmetic in a union
// is that of the problem's own solver, so results stay bitwise those of solving each request alone.
struct ServerGroup {
  std::string key;
  std::vector<std::shared_ptr<ServerReq>> reqs;  // members, in union order
  pmg_solver_s* u = nullptr;
  double* Qu = nullptr;     // union state [5][nn] (u's arena)
  std::vector<size_t> off;  // first union node of each member
  size_t nn = 0;
  bool dirty = true;
  hipStream_t st = nullptr;
};

static std::string server_group_key(const ServerReq& r) {
  int pmax = 1;
  for (int v : r.orders) pmax = std::max(pmax, v);
  const pmg_mg_params& m = r.mg;
  std::string k = std::to_string(pmax) + ":" + std::to_string(r.phys.node_family);
  k += ":" + std::to_string(m.beta_pre) + "," + std::to_string(m.beta_post) + "," + std::to_string(m.beta_coarse);
  k += ":" + std::to_string(m.precision) + "," + std::to_string(m.mixed_patience) + "," + std::to_string(m.n_levels);
  for (int c : r.caps) k += "," + std::to_string(c);
  return k;
}

// member p's range of the union state <-> its own state
static void group_copy(ServerGroup& g, size_t p, bool to_union) {
  const ServerReq& r = *g.reqs[p];
  const size_t n = g.off[p + 1] - g.off[p];  // the member's own node count
  for (int v = 0; v < 5; v++) {
    double* a = g.Qu + (size_t)v * g.nn + g.off[p];
    double* b = r.Q + (size_t)v * n;
    HIPCHECK(hipMemcpyAsync(to_union ? a : b, to_union ? b : a, n * sizeof(double), hipMemcpyDeviceToDevice, g.st));
  }
}

static void group_release(ServerGroup& g) {
  if (!g.u) return;
  for (size_t p = 0; p < g.reqs.size(); p++) group_copy(g, p, false);
  HIPCHECK(hipStreamSynchronize(g.st));
  delete g.u;
  g.u = nullptr;
  g.Qu = nullptr;
}

static void group_build(pmg_server_s* sv, ServerGroup& g) {
  std::vector<const pmg_mesh_s*> meshes;
  std::vector<const int32_t*> orders;
  std::vector<pmg_physics> phys;
  for (auto& r : g.reqs) {
    meshes.push_back(r->mesh);
    orders.push_back(r->orders.data());
    phys.push_back(r->phys);
  }
  pmg_mg_params mg = g.reqs[0]->mg;
  mg.level_caps = g.reqs[0]->caps.empty() ? nullptr : g.reqs[0]->caps.data();
  g.u = create_solver(sv->ctx, meshes, orders, phys.data(), &mg);
  g.u->use_graph = sv->graph;
  const Level& T = *g.u->top;
  g.nn = (size_t)T.nn;
  g.off.assign(g.reqs.size() + 1, 0);
  for (size_t p = 0; p <= g.reqs.size(); p++) g.off[p] = (size_t)T.off[g.u->prob_elem[p]];
  g.Qu = g.u->arena.alloc<double>(5 * g.nn);
  for (size_t p = 0; p < g.reqs.size(); p++) group_copy(g, p, true);
  g.dirty = false;
}

static void server_loop_batched(pmg_server_s* sv) {
  if (hipSetDevice(sv->ctx->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->fatal = "hipSetDevice failed in the server thread";
    return;
  }
  std::vector<ServerGroup> groups;
  auto n_resident = [&] {
    size_t n = 0;
    for (auto& g : groups) n += g.reqs.size();
    return n;
  };
  for (;;) {
    std::vector<std::shared_ptr<ServerReq>> admit;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (n_resident() == 0) sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop) break;
      while (!sv->queue.empty() && sv->used + sv->queue.front()->est <= sv->budget) {
        auto r = sv->queue.front();
        sv->queue.pop_front();
        sv->used += r->est;
        sv->peak = std::max(sv->peak, sv->used);
        r->t_admit = sv->now();
        admit.push_back(r);
      }
    }
    for (auto& r : admit) {
      const std::string key = server_group_key(*r);
      ServerGroup* g = nullptr;
      for (auto& x : groups)
        if (x.key == key) g = &x;
      if (!g) {
        groups.emplace_back();
        g = &groups.back();
        g->key = key;
        g->st = sv->streams[(groups.size() - 1) % sv->streams.size()];
      }
      if (g->u) {
        // the union is rebuilt with the new member: the current members' states go back to them first
        pmg_status rc = guard([&] { group_release(*g); });
        if (rc != PMG_OK) {
          std::lock_guard<std::mutex> lk(sv->mu);
          sv->fatal = "server: " + g_err;
        }
      }
      r->ms.f32 = r->mg.precision == 1;
      g->reqs.push_back(r);
      g->dirty = true;
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->n_resident = (int)n_resident();
      sv->max_resident = std::max(sv->max_resident, sv->n_resident);
      if (!sv->fatal.empty()) break;
    }
    for (auto& g : groups) {
      if (g.reqs.empty()) continue;
      if (g.dirty) {
        pmg_status rc = guard([&] { group_build(sv, g); });
        if (rc != PMG_OK) {
          // the union could not be built: every member fails with the error
          for (auto& r : g.reqs) {
            r->err = g_err;
            server_retire(sv, r, rc);
          }
          g.reqs.clear();
          g.u = nullptr;
          continue;
        }
      }
      // one iteration: the decided cycles, then every member's residual norm (the launch sequence of
      // pmg_batch_solve: problems not advanced skip their tiles)
      const int n = (int)g.reqs.size();
      pmg_solver_s* u = g.u;
      std::vector<int> a32(n, 0), a64(n, 0);
      int n32 = 0, n64 = 0;
      for (int p = 0; p < n; p++) {
        a32[p] = g.reqs[p]->cycle_next && g.reqs[p]->ms.f32;
        a64[p] = g.reqs[p]->cycle_next && !g.reqs[p]->ms.f32;
        n32 += a32[p];
        n64 += a64[p];
      }
      std::vector<double> r;
      pmg_status rc = guard([&] {
        traces_stale(u);
        if (n32) {
          HIPCHECK(hipMemcpyAsync(u->d_act[0], a32.data(), n * sizeof(int), hipMemcpyHostToDevice, g.st));
          cycle_once(u, u->iso, 0, g.Qu, nullptr, u->d_act[0], g.st);
        }
        if (n64) {
          HIPCHECK(hipMemcpyAsync(u->d_act[1], a64.data(), n * sizeof(int), hipMemcpyHostToDevice, g.st));
          cycle_once(u, iso_f64(u), u->mg.precision == 1 ? 2 : 0, g.Qu, nullptr, u->d_act[1], g.st);
        }
        residual(u, *u->top, (const double*)g.Qu, (const double*)nullptr, u->d_R, false, SLOT_NORM, g.st);
        r = read_slots(u, SLOT_NORM, g.st);  // waits for the stream
      });
      if (rc != PMG_OK) {
        for (auto& q : g.reqs) {
          q->err = g_err;
          q->status = rc;
        }
        r.assign(n, (double)NAN);
      }
      std::vector<std::shared_ptr<ServerReq>> keep;
      std::vector<size_t> keep_p;
      for (int p = 0; p < n; p++) {
        auto& q = g.reqs[p];
        if (a32[p] || a64[p]) {
          q->cycles++;
          q->fp32 += a32[p];
        }
        int status = q->status >= 0 ? q->status : -1;
        if (status < 0) {
          q->r = r[p];
          if (q->r != q->r) {
            q->err = "non-finite residual";
            status = PMG_ERR_NONPHYSICAL;
          } else if (q->r < q->tol) {
            status = PMG_OK;
          } else if (q->cycles >= q->max_cycles) {
            status = PMG_ERR_NOT_CONVERGED;
          } else {
            q->ms.update(q->r, q->mg.mixed_patience > 0 ? q->mg.mixed_patience : 4);
            q->cycle_next = true;
          }
        }
        if (status >= 0) {
          // the member's state goes back to it before it is reported done
          pmg_status rc2 = guard([&] {
            group_copy(g, (size_t)p, false);
            HIPCHECK(hipStreamSynchronize(g.st));
          });
          if (rc2 != PMG_OK && status == PMG_OK) {
            q->err = g_err;
            status = rc2;
          }
          server_retire(sv, q, status);
          g.dirty = true;
        } else {
          keep.push_back(q);
          keep_p.push_back((size_t)p);
        }
      }
      if (g.dirty) {
        // membership changed: the remaining members' states go back to them; the union is rebuilt next time
        for (size_t i = 0; i < keep.size(); i++) {
          pmg_status rc3 = guard([&] { group_copy(g, keep_p[i], false); });
          (void)rc3;
        }
        (void)hipStreamSynchronize(g.st);
        delete g.u;
        g.u = nullptr;
        g.Qu = nullptr;
      }
      g.reqs.swap(keep);
    }
    groups.erase(std::remove_if(groups.begin(), groups.end(), [](const ServerGroup& g) { return g.reqs.empty(); }),
                 groups.end());
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->iterations++;
    sv->n_resident = (int)n_resident();
  }
  for (auto& g : groups) {
    (void)guard([&] { group_release(g); });
    for (auto& r : g.reqs) server_retire(sv, r, PMG_ERR_BUSY);
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->n_resident = 0;
}

extern "C" {

pmg_status pmg_footprint(pmg_mesh mesh, const int32_t* orders, const pmg_mg_params* mg, int64_t* bytes,
                         int64_t* transient_bytes, int64_t* switch_bytes) {
  return guard([&] {
    REQUIRE(mesh && orders && bytes, "NULL argument");
    for (int64_t i = 0; i < 3 * mesh->K; i++) REQUIRE(orders[i] >= 1 && orders[i] <= PMG_MAXN - 1, "orders must be 1..7");
    double tr = 0.0, sw = 0.0;
    *bytes = (int64_t)std::ceil(solver_footprint(mesh, orders, mg, &tr, &sw));
    if (transient_bytes) *transient_bytes = (int64_t)std::ceil(tr);
    if (switch_bytes) *switch_bytes = (int64_t)std::ceil(sw);
  });
}

pmg_status pmg_device_bytes(int64_t* bytes) {
  return guard([&] {
    REQUIRE(bytes, "NULL argument");
    *bytes = g_dev_bytes.load();
  });
}

pmg_status pmg_server_create(pmg_ctx ctx, int64_t hbm_budget_bytes, int n_streams, int use_graph, int batched,
                             pmg_server* out) {
  return guard([&] {
    REQUIRE(ctx && out, "NULL argument");
    REQUIRE(hbm_budget_bytes > 0, "the HBM budget must be positive");
    REQUIRE(n_streams >= 1 && n_streams <= 64, "n_streams must be 1..64");
    HIPCHECK(hipSetDevice(ctx->device));
    auto sv = std::make_unique<pmg_server_s>();
    sv->ctx = ctx;
    sv->budget = (double)hbm_budget_bytes;
    sv->graph = use_graph ? 1 : 0;
    REQUIRE(batched == 0 || batched == 1, "batched must be 0 or 1");
    sv->batched = batched;
    for (int i = 0; i < n_streams; i++) {
      hipStream_t st;
      HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      sv->streams.push_back(st);
    }
    pmg_server_s* p = sv.get();
    if (batched) sv->worker = std::thread([p] { server_loop_batched(p); });
    else sv->worker = std::thread([p] { server_loop(p); });
    *out = sv.release();
  });
}

pmg_status pmg_server_submit(pmg_server sv, pmg_mesh mesh, const int32_t* orders, const pmg_physics* phys,
                             const pmg_mg_params* mg, double* Q_dev, double tol, int max_cycles, uint64_t* ticket) {
  return guard([&] {
    REQUIRE(sv && mesh && orders && phys && Q_dev && ticket, "NULL argument");
    REQUIRE(mesh->ctx == sv->ctx, "mesh belongs to another context");
    REQUIRE(max_cycles >= 0, "negative max_cycles");
    REQUIRE(!mg || (!mg->tuning && !mg->fmg), "served solves use fixed sweep counts and no FMG start");
    REQUIRE(!mg || mg->guard == 0, "the divergence guard belongs to pmg_solve / pmg_batch_solve, not to served solves");
    for (int64_t i = 0; i < 3 * mesh->K; i++) REQUIRE(orders[i] >= 1 && orders[i] <= PMG_MAXN - 1, "orders must be 1..7");
    auto r = std::make_shared<ServerReq>();
    r->mesh = mesh;
    r->orders.assign(orders, orders + 3 * mesh->K);
    r->phys = *phys;
    if (mg) {
      r->mg = *mg;
      if (mg->n_levels > 0 && mg->level_caps) r->caps.assign(mg->level_caps, mg->level_caps + mg->n_levels);
    } else {
      memset(&r->mg, 0, sizeof(r->mg));
      r->mg.beta_pre = r->mg.beta_post = r->mg.beta_coarse = 3;
      r->mg.eta = 1.1;
      r->mg.max_repeats = 10;
      r->mg.fmg_threshold = 0.1;
    }
    r->mg.level_caps = nullptr;
    r->tol = tol;
    r->max_cycles = max_cycles;
    r->Q = Q_dev;
    double tr = 0.0, sw = 0.0;
    pmg_mg_params m = r->mg;
    m.level_caps = r->caps.empty() ? nullptr : r->caps.data();
    r->est = solver_footprint(mesh, orders, &m, &tr, &sw) + tr + sw;
    std::lock_guard<std::mutex> lk(sv->mu);
    REQUIRE(sv->fatal.empty(), "server stopped: " + sv->fatal);
    if (r->est > sv->budget)
      throw PmgError(PMG_ERR_OOM, "request footprint " + std::to_string((long long)r->est) +
                                      " B exceeds the server's HBM budget");
    r->ticket = sv->next_ticket++;
    r->t_submit = sv->now();
    sv->queue.push_back(r);
    sv->all[r->ticket] = r;
    *ticket = r->ticket;
    sv->cv.notify_one();
  });
}

pmg_status pmg_server_poll(pmg_server sv, uint64_t ticket, int* done, int* status, int* cycles, int* fp32_cycles,
                           double* res_inf, double* latency_s, double* queue_s) {
  return guard([&] {
    REQUIRE(sv && done, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    REQUIRE(it != sv->all.end(), "unknown ticket");
    const ServerReq& r = *it->second;
    *done = r.done;
    if (!r.done) return;
    if (status) *status = r.status;
    if (cycles) *cycles = r.cycles;
    if (fp32_cycles) *fp32_cycles = r.fp32;
    if (res_inf) *res_inf = r.r;
    if (latency_s) *latency_s = r.t_done - r.t_submit;
    if (queue_s) *queue_s = r.t_admit - r.t_submit;
  });
}

pmg_status pmg_server_stats(pmg_server sv, int* resident, int* queued, int64_t* completed, int64_t* iterations,
                            int64_t* bytes_in_use, int64_t* peak_bytes, int* max_resident) {
  return guard([&] {
    REQUIRE(sv, "NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (resident) *resident = sv->n_resident;
    if (queued) *queued = (int)sv->queue.size();
    if (completed) *completed = sv->completed;
    if (iterations) *iterations = sv->iterations;
    if (bytes_in_use) *bytes_in_use = (int64_t)sv->used;
    if (peak_bytes) *peak_bytes = (int64_t)sv->peak;
    if (max_resident) *max_resident = sv->max_resident;
    REQUIRE(sv->fatal.empty(), "server stopped: " + sv->fatal);
  });
}

void pmg_server_destroy(pmg_server sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
  delete sv;
}

pmg_status pmg_tau_estimate(pmg_solver s, double* Q_dev, const double* S_dev, int isolated, double* tau_map_dev,
                            void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && tau_map_dev, "NULL argument");
    traces_stale(s);
    hipStream_t st = (hipStream_t)stream;
    const int nt = std::max(s->nmax - 1, 1);
    TauRec tau{tau_map_dev, nt, isolated ? 1 : 0};
    for (int d = 0; d < 3; d++) aniso_hier(s, d);  // built before any capture
    if (s->use_graph) {
      GraphKey key{1, Q_dev, S_dev, tau_map_dev, nullptr, tau.isolated};
      run_graph(s, key, 1, st, [&](hipStream_t cs) { tau_cycles(s, Q_dev, S_dev, tau, cs); });
    } else {
      tau_cycles(s, Q_dev, S_dev, tau, st);
    }
    HIPCHECK(hipGetLastError());
  });
}

// ------------------------------------------------------------------------------------------------
// Residual history, checkpoint and restore
// ------------------------------------------------------------------------------------------------
pmg_status pmg_solve_history(pmg_solver s, double* out, int32_t capacity, int32_t* n) {
  return guard([&] {
    REQUIRE(s && n, "NULL argument");
    REQUIRE(capacity >= 0 && (capacity == 0 || out), "bad output buffer");
    *n = (int32_t)s->history.size();
    for (int i = 0; i < std::min<int>(capacity, (int)s->history.size()); i++) out[i] = s->history[i];
  });
}

static uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
  for (size_t i = 0; i < n; i++) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

static const char kCkptMagic[8] = {'P', 'M', 'G', 'C', 'K', 'P', 'T', '1'};

pmg_status pmg_checkpoint(pmg_solver s, const char* path, const double* Q_dev, void* stream) {
  return guard([&] {
    REQUIRE(s && path && Q_dev, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t K = s->mesh->K, nn = s->top->nn, nh = (int64_t)s->history.size();
    std::vector<unsigned char> buf;
    auto put = [&](const void* p, size_t n) {
      const unsigned char* c = (const unsigned char*)p;
      buf.insert(buf.end(), c, c + n);
    };
    put(kCkptMagic, 8);
    put(&K, 8);
    put(&nn, 8);
    put(&s->nprob, 4);
    put(s->orders.data(), sizeof(int) * s->orders.size());
    put(&s->cycles_total, 8);
    put(&nh, 8);
    put(s->history.data(), sizeof(double) * nh);
    std::vector<double> Q(5 * (size_t)nn);
    HIPCHECK(hipMemcpyAsync(Q.data(), Q_dev, Q.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    put(Q.data(), Q.size() * sizeof(double));
    uint64_t h = fnv1a(buf.data(), buf.size());
    put(&h, 8);
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    REQUIRE(f, std::string("cannot open ") + tmp);
    size_t w = fwrite(buf.data(), 1, buf.size(), f);
    int cl = fclose(f);
    REQUIRE(w == buf.size() && cl == 0, std::string("short write to ") + tmp);
    REQUIRE(rename(tmp.c_str(), path) == 0, std::string("cannot rename to ") + path);
  });
}

pmg_status pmg_restore(pmg_solver s, const char* path, double* Q_dev, void* stream) {
  return guard([&] {
    REQUIRE(s && path && Q_dev, "NULL argument");
    traces_stale(s);
    FILE* f = fopen(path, "rb");
    REQUIRE(f, std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = fread(chunk, 1, sizeof(chunk), f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    fclose(f);
    size_t pos = 0;
    auto take = [&](void* p, size_t n) {
      REQUIRE(pos + n <= buf.size(), "checkpoint file is truncated");
      memcpy(p, buf.data() + pos, n);
      pos += n;
    };
    REQUIRE(buf.size() >= 16, "checkpoint file is truncated");
    uint64_t h_file;
    memcpy(&h_file, buf.data() + buf.size() - 8, 8);
    REQUIRE(fnv1a(buf.data(), buf.size() - 8) == h_file, "checkpoint checksum mismatch");
    char magic[8];
    take(magic, 8);
    REQUIRE(memcmp(magic, kCkptMagic, 8) == 0, "not a checkpoint of this library");
    int64_t K, nn, cyc, nh;
    int32_t np;
    take(&K, 8);
    take(&nn, 8);
    take(&np, 4);
    REQUIRE(K == s->mesh->K && nn == s->top->nn && np == s->nprob, "checkpoint is of another problem");
    std::vector<int> ord(s->orders.size());
    take(ord.data(), sizeof(int) * ord.size());
    REQUIRE(ord == s->orders, "checkpoint has other orders");
    take(&cyc, 8);
    take(&nh, 8);
    REQUIRE(nh >= 0 && nh < (1ll << 40), "bad history length");
    std::vector<double> hist((size_t)nh);
    take(hist.data(), sizeof(double) * nh);
    std::vector<double> Q(5 * (size_t)nn);
    take(Q.data(), Q.size() * sizeof(double));
    REQUIRE(pos + 8 == buf.size(), "checkpoint has trailing bytes");
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipMemcpyAsync(Q_dev, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    s->cycles_total = cyc;
    s->history = hist;
  });
}

pmg_status pmg_cycle_count(pmg_solver s, int64_t* cycles) {
  return guard([&] {
    REQUIRE(s && cycles, "NULL argument");
    *cycles = s->cycles_total;
  });
}

pmg_status pmg_tau_nodal(pmg_solver s, int dir, int order, double* Q_dev, const double* S_dev, int isolated,
                         double* tau_dev, void* stream) {
  return guard([&] {
    REQUIRE(s && Q_dev && tau_dev, "NULL argument");
    traces_stale(s);
    REQUIRE(dir >= 0 && dir <= 2, "dir must be 0, 1 or 2");
    Hier& H = aniso_hier(s, dir);
    int lev = -1;
    for (int l = 0; l + 1 < (int)H.lv.size(); l++)
      if (H.caps[l] == order) lev = l;
    REQUIRE(lev >= 0, "no coarse level with that order in that direction (1 <= order < max order in dir)");
    hipStream_t st = (hipStream_t)stream;
    if (!s->d_taumap) s->d_taumap = s->arena.alloc<double>((size_t)s->mesh->K * 3 * std::max(s->nmax - 1, 1));
    TauRec tau{s->d_taumap, std::max(s->nmax - 1, 1), isolated ? 1 : 0};
    tau.nodal = tau_dev;
    tau.nodal_dir = dir;
    tau.nodal_cap = order;
    run_vcycles(s, H, Q_dev, S_dev, 1, &tau, st);
    HIPCHECK(hipGetLastError());
  });
}

pmg_status pmg_profile_enable(pmg_solver s, uint32_t mask) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    REQUIRE((mask >> PK_N) == 0, "unknown kernel kind in mask");
    s->prof->mask = mask;
  });
}

pmg_status pmg_profile_stride(pmg_solver s, int32_t stride) {
  return guard([&] {
    REQUIRE(s, "NULL solver");
    REQUIRE(stride >= 1, "stride must be at least 1");
    s->prof->stride = stride;
    for (auto& c : s->prof->count) c = 0;
  });
}

pmg_status pmg_profile_read(pmg_solver s, int kind, double* total_ms, int64_t* launches, double* alg_bytes) {
  return guard([&] {
    REQUIRE(s && total_ms && launches, "NULL argument");
    REQUIRE(kind >= 0 && kind < PK_N, "unknown kernel kind");
    s->prof->read(kind, total_ms, launches, alg_bytes);
  });
}

}  // extern "C"

#include "adapt.inc"
#include "functionals.inc"
