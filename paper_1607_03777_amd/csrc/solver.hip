// Problem setup and solver orchestration behind the C ABI (include/sdg.h).
//
// A problem object holds nbatch independent problems on one mesh (same nx,
// ny, k, boundary sides and options; own viscosity, force and solution).
// Device vectors are stored problem after problem; Krylov scalars are
// per-problem device arrays and each problem leaves the iteration when it
// converges (its updates are masked) while the others continue.
//
// Setup (Sections 4 and 6): element viscosity -> deduplicated diagonal
// blocks of A (eq. smoother) and their inverses; A_{1,c} = P_cd^T A_1 P_cd
// (Section 6.1.2) from element-local matrices; the Galerkin h-hierarchy;
// the dense inverse of the coarsest operator; Chebyshev bounds
// [cheb_lo, cheb_hi] * lambda* with lambda* the largest Ritz value of
// eig_steps Arnoldi steps on M^{-1} A (Section 6).
//
// Solve: the two-level cycle of Algorithm 1 (Chebyshev with element-block
// Jacobi before and after; the coarse solve is one h-cycle with
// Chebyshev/point-Jacobi smoothing and the dense coarsest inverse; the
// small h-levels run in one workgroup per problem), preconditioning CG
// (Section 8.1) or FGMRES for the viscous block, and right-preconditioned
// FGMRES with the upper block-triangular preconditioner for Stokes
// (Section 5).  The Krylov loops run on the host and read one short array of
// per-problem scalars back per step; all vector work runs in the library's
// kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <array>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "sdg_common.h"
#include "sdg_kernels.h"
#include "ext_kernels.h"
#include "runtime.h"

struct SdgCombiner;  // combined launches of concurrent CG iterations (serving)

// A context is freed when it has been destroyed and its last problem is
// gone, so problems destroyed after their context stay valid.
struct sdg_ctx {
  SdgCombiner* comb = nullptr;  // set while a request server runs on the context
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  int live = 0;
  bool closing = false;
  std::mutex mu;  // used, live, closing (problems may be created and destroyed from several threads)
  // kernel tracing
  struct TraceRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  bool trace = false;
  std::mutex trace_mu;
  std::vector<hipEvent_t> ev_pool;
  std::vector<TraceRec> pending;
  int64_t tr_n[SDG_TRACE_CLASSES] = {};
  double tr_ms[SDG_TRACE_CLASSES] = {};
  double tr_bytes[SDG_TRACE_CLASSES] = {};
  // device blocks released by finished problems and temporaries, kept for
  // reuse by size (hipFree synchronises the whole device, hipMalloc is slow;
  // batched and served groups of one shape ask for the same sizes again).
  // A block enters the cache only once no queued work uses it.  Guarded by mu.
  std::multimap<size_t, void*> cache;
  size_t cached = 0;
  // unit-block tables of the extended-precision residual, per (k, nx, ny,
  // lx, ly, side kinds); device arrays live until the context is freed.
  // Guarded by mu.
  struct ExtEntry {
    sdg::ExtTables T;
    void* mem = nullptr;
  };
  std::map<std::string, ExtEntry> ext;
  ~sdg_ctx() {
    for (auto& kv : ext) (void)hipFree(kv.second.mem);
    for (auto& r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& kv : cache) (void)hipFree(kv.second);
  }
};

// ---------------------------------------------------------------------------
// Allocation-free form of sdg_get_blocks: the element list it hands to the
// block kernel lives in this file-scope device array instead of a buffer
// allocated per call.  Its device address is taken once per device, with
// that device current, when a context is created (sdg_create); host code
// uses only that address.  Every call on one device shares the array.
// ---------------------------------------------------------------------------
static constexpr int64_t NOALLOC_MAX_ELEMS = 1 << 20;  // elements x batch (4 MiB)
static __device__ __align__(256) int scratch[NOALLOC_MAX_ELEMS];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

namespace sdg {
int ctx_device(const sdg_ctx* c) { return c ? c->device : 0; }
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
const char* get_error() { return g_err.c_str(); }
}  // namespace sdg

using namespace sdg;

namespace {

// address of `scratch` on the current device (once per device)
int scratch_setup(int device) {
  if (device < 0 || device >= 64) {
    set_error("device index beyond the allocation-free scratch table (64 devices)");
    return SDG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return SDG_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
    return SDG_ERR_DEVICE;
  }
  g_scratch_ptr[device] = ptr;
  return SDG_OK;
}
void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return (device >= 0 && device < 64) ? g_scratch_ptr[device] : nullptr;
}
__global__ void iota_kernel(int64_t n, int* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) out[i] = (int)i;
}

constexpr double BF16_LAMBDA_MAX = 4.0;  // see the BF16 check in sdg_problem_create_batch
constexpr int TAIL_NODES = 17 * 17;  // h-levels with at most this many nodes run in the tail kernel
constexpr int RED_SCRATCH = 512 * 64;

// Tile shapes chosen by sdg_autotune, per (k, nx, ny, nbatch, kernel,
// precision), shared by every later problem of that shape in the process.
std::mutex g_tune_mu;
std::map<std::array<int, 6>, int> g_tune;

hipEvent_t trace_event(sdg_ctx* c) {
  hipEvent_t e = nullptr;
  {
    std::lock_guard<std::mutex> g(c->trace_mu);
    if (!c->ev_pool.empty()) {
      e = c->ev_pool.back();
      c->ev_pool.pop_back();
    }
  }
  if (!e && hipEventCreate(&e) != hipSuccess) e = nullptr;
  return e;
}

// Runs launch() and, while tracing is on, brackets it with events.
template <typename F>
int traced(sdg_ctx* c, hipStream_t s, int cls, double bytes, F&& launch) {
  if (!c->trace) return launch();
  hipEvent_t a = trace_event(c), b = trace_event(c);
  if (!a || !b) {
    set_error("hipEventCreate failed while tracing");
    return SDG_ERR_DEVICE;
  }
  SDG_HIP(hipEventRecord(a, s));
  const int rc = launch();
  SDG_HIP(hipEventRecord(b, s));
  std::lock_guard<std::mutex> g(c->trace_mu);
  c->pending.push_back(sdg_ctx::TraceRec{cls, a, b, bytes});
  return rc;
}

struct CLevel {
  int nx = 0, ny = 0, nn = 0;
  double* st = nullptr;
  double* dinv = nullptr;
  double *b = nullptr, *x = nullptr, *xalt = nullptr, *r = nullptr, *d = nullptr;
  double* dense = nullptr;
  double* ab = nullptr;  // [smooth_h][nbatch][2]
  std::vector<double> lmin, lmax;
  bool coarsest = false;
};

// Workspace of a GCR solve: m search directions p_j (P) and their images
// q_j = K p_j (Q), both [m][total]; the residual r and the cycle's
// correction c ([total]); device coefficients and the done mask.
struct GcrWork {
  double *Q = nullptr, *Pd = nullptr, *r = nullptr, *c = nullptr;
  double* coef = nullptr;  // [4 (m + 1) + 4][nb]
  int* done = nullptr;     // [nb]
  int m = 0;
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct sdg_problem {
  sdg_ctx* ctx = nullptr;
  sdg_mesh mesh{};
  sdg_options opt{};
  MeshDev M{};
  hipStream_t s = nullptr;
  int nb = 1;  // batch size
  int k = 0, K1 = 0, NB = 0, NPE = 0;
  int nel = 0;
  int64_t nu = 0, np = 0;  // per problem
  std::vector<std::pair<void*, size_t>> allocs;
  size_t bytes = 0;
  double* eta = nullptr;   // [nb][nel]
  double* etap = nullptr;  // [nb][np], eta over the pressure modes
  std::vector<double> eta_host;
  // block Jacobi
  int nuniq = 0;
  BjPlan bj{};  // elements grouped by unique block
  double* scale = nullptr;
  double* binv = nullptr;
  float* binv32 = nullptr;
  uint16_t* binv16 = nullptr;
  double* xpacked = nullptr;  // packed FP64 factors X = L^{-1} (low precision)
  double* binvq = nullptr;    // quad-packed FP64 inverses (streamed smoother plans)
  std::vector<int> reps;
  // DG cycle
  double *vr = nullptr, *vd = nullptr;
  float *fb = nullptr, *fx = nullptr, *fr = nullptr, *fd = nullptr;
  std::vector<double> lmin0, lmax0;
  double* ab0 = nullptr;  // [smooth_dg][nb][2]
  std::vector<CLevel> lev;
  int tail_start = 0;
  TailArgs tail{};
  // Krylov
  double* red = nullptr;
  double* dsc = nullptr;  // device scalars (see SC_* offsets)
  double* hsc = nullptr;  // pinned host mirror
  int64_t nsc = 0;        // its size in doubles (that of dsc)
  // published CG scalars: pinned copy, sequence number written by the
  // device after them, the device-side counter and the host's count
  double* hpub = nullptr;
  unsigned* hseq = nullptr;
  unsigned* dcount = nullptr;
  unsigned seq = 0;
  int* active = nullptr;  // device [nb]
  int nact_host = 0;      // ones in the last upload of `active`
  // pinned staging ring of the small uploads made between launches (active
  // flags, coefficients): a slot is reused once its copy has completed
  static constexpr int STAGE_SLOTS = 8;
  static constexpr size_t STAGE_BYTES = 8192;
  char* hstage = nullptr;
  hipEvent_t stage_ev[STAGE_SLOTS] = {};
  int stage_next = 0;
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr;
  double *gV = nullptr, *gZ = nullptr, *gw = nullptr, *gt = nullptr;
  double* gcoef = nullptr;  // FGMRES coefficients on the device
  int* gdone = nullptr;     // FGMRES: problems finished within the cycle
  int64_t gn = 0;  // per-problem length of the FGMRES vectors
  bool neumann = false;
  double setup_ms = 0;
  // per-problem statistics of the last solve
  std::vector<int> inner_total, inner_max;
  // tile shape of the SIP kernels: [apply, residual][FP64, FP32]
  int tile[2][2] = {{0, 0}, {0, 0}};
  // the dense inverse of the coarsest level runs on a side stream beside the
  // eigenvalue estimates: ds_ev = {fork, join}; dense_stat: its flags of
  // positive definiteness, checked when setup joins it
  hipStream_t ds = nullptr;
  hipEvent_t ds_ev[2] = {nullptr, nullptr};
  int* dense_stat = nullptr;
  // captured CG iteration (two graphs: the roles of the two r.z slots alternate)
  hipStream_t gs = nullptr;  // private stream used only to capture
  hipGraphExec_t cg_graph[2] = {nullptr, nullptr};
  double* cg_x = nullptr;  // fixed iterate buffer of the captured iteration
  // extended-precision residual tables (from the context's cache)
  const ExtTables* ext = nullptr;
  // GCR workspace of the inner viscous solve
  GcrWork gi;
};

namespace {

// device scalar layout: each slot holds nb doubles; SC_H holds [nb][restart+4]
enum { SC_RZ = 0, SC_RZ2, SC_PQ, SC_RR, SC_BN, SC_H, SC_COUNT_FIXED };
inline double* sc(sdg_problem* P, int slot) { return P->dsc + (int64_t)slot * P->nb; }
inline double* sc_h(sdg_problem* P) { return P->dsc + (int64_t)SC_H * P->nb; }

// Device memory through the context's cache: a released block of the same
// (256-byte rounded) size is reused; otherwise hipMalloc, and on failure the
// cache is emptied and the allocation tried once more.
size_t cache_size(size_t bytes) { return (bytes + 255) & ~size_t(255); }
int ctx_get(sdg_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  {
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->cache.find(bytes);
    if (it != c->cache.end()) {
      *out = it->second;
      c->cache.erase(it);
      c->cached -= bytes;
      return SDG_OK;
    }
  }
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    std::multimap<size_t, void*> drop;
    {
      std::lock_guard<std::mutex> g(c->mu);
      drop.swap(c->cache);
      c->cached = 0;
    }
    for (auto& kv : drop) (void)hipFree(kv.second);
    e = hipMalloc(out, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    *out = nullptr;
    return SDG_ERR_NOMEM;
  }
  return SDG_OK;
}
// The caller guarantees that no queued work still uses the block.
void ctx_put(sdg_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> g(c->mu);
  c->cache.emplace(bytes, p);
  c->cached += bytes;
}

int palloc(sdg_problem* P, void** out, size_t bytes) {
  *out = nullptr;
  if (bytes == 0) return SDG_OK;
  bytes = cache_size(bytes);
  {
    std::lock_guard<std::mutex> g(P->ctx->mu);
    if (P->ctx->budget && P->ctx->used + bytes > P->ctx->budget) {
      set_error("device memory budget exceeded");
      return SDG_ERR_NOMEM;
    }
    P->ctx->used += bytes;  // reserved before the allocation
  }
  if (ctx_get(P->ctx, bytes, out) < 0) {
    std::lock_guard<std::mutex> g(P->ctx->mu);
    P->ctx->used -= std::min(P->ctx->used, bytes);
    return SDG_ERR_NOMEM;
  }
  P->allocs.push_back({*out, bytes});
  P->bytes += bytes;
  return SDG_OK;
}
// Temporaries of one call: from the cache, returned after the problem's
// stream has drained (all work that used them is done).
template <typename T>
int tmp_get(sdg_problem* P, T** out, int64_t n) {
  void* p = nullptr;
  const int rc = ctx_get(P->ctx, cache_size((size_t)std::max<int64_t>(n, 1) * sizeof(T)), &p);
  *out = (T*)p;
  return rc;
}
template <typename T>
void tmp_put(sdg_problem* P, T* p, int64_t n) {
  if (!p) return;
  (void)hipStreamSynchronize(P->s);
  ctx_put(P->ctx, (void*)p, cache_size((size_t)std::max<int64_t>(n, 1) * sizeof(T)));
}

template <typename T>
int palloc_t(sdg_problem* P, T** out, int64_t n) {
  void* p = nullptr;
  int rc = palloc(P, &p, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
  *out = (T*)p;
  return rc;
}

bool mesh_ok(const sdg_mesh* m) {
  if (!m) return false;
  if (m->nx < 1 || m->ny < 1 || m->k < 1 || m->k > SDG_KMAX) return false;
  if (!(m->lx > 0) || !(m->ly > 0)) return false;
  for (int i = 0; i < 4; ++i)
    if (m->bc[i] < 0 || m->bc[i] > 2) return false;
  return true;
}

int to_host(sdg_problem* P, void* dst, const void* src, size_t bytes) {
  SDG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, P->s));
  SDG_HIP(hipStreamSynchronize(P->s));
  return SDG_OK;
}
// host -> device through the pinned mirror when it fits (the source may be
// reused right after the call returns)
int to_dev(sdg_problem* P, void* dst, const void* src, size_t bytes) {
  SDG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, P->s));
  SDG_HIP(hipStreamSynchronize(P->s));
  return SDG_OK;
}
// Enqueue the publication of n device scalars; returns the sequence number
// the host waits for.
int publish(sdg_problem* P, const double* src, int n, unsigned* seq_out) {
  SDG_TRY(publish_scalars(src, n, P->hpub, P->dcount, P->hseq, P->s));
  *seq_out = ++P->seq;
  return SDG_OK;
}
// Wait until the device has published sequence number `seq` (spinning on
// the pinned flag, then copy the scalars out).  A wait beyond a few seconds
// falls back to a stream synchronisation, which reports device errors.
int wait_published(sdg_problem* P, unsigned seq, int n, double* out) {
  volatile unsigned* flag = P->hseq;
  const auto t0 = std::chrono::steady_clock::now();
  int spins = 0;
  while (*flag != seq) {
    if (++spins % 1024 == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::seconds(5)) {
      SDG_HIP(hipStreamSynchronize(P->s));
      if (*flag != seq) {
        set_error("published scalars did not arrive");
        return SDG_ERR_DEVICE;
      }
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  std::memcpy(out, const_cast<const double*>(P->hpub), n * sizeof(double));
  return SDG_OK;
}
int read_dev(sdg_problem* P, const double* src, int n, double* out) {
  if (n > P->nsc) return to_host(P, out, src, (size_t)n * sizeof(double));  // beyond the pinned mirror
  SDG_HIP(hipMemcpyAsync(P->hsc, src, n * sizeof(double), hipMemcpyDeviceToHost, P->s));
  SDG_HIP(hipStreamSynchronize(P->s));
  std::memcpy(out, P->hsc, n * sizeof(double));
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// dedup keys: face kinds and neighbour/self viscosity ratios
// ---------------------------------------------------------------------------
struct BlockKey {
  int kind[4];
  double ratio[4];
  bool operator==(const BlockKey& o) const {
    for (int i = 0; i < 4; ++i)
      if (kind[i] != o.kind[i] || ratio[i] != o.ratio[i]) return false;
    return true;
  }
};
struct BlockKeyHash {
  size_t operator()(const BlockKey& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 4; ++i) {
      uint64_t v;
      std::memcpy(&v, &k.ratio[i], 8);
      h = (h ^ (uint64_t)k.kind[i]) * 1099511628211ull;
      h = (h ^ v) * 1099511628211ull;
    }
    return (size_t)h;
  }
};

// The diagonal block of element e of one problem (viscosity et) is eta_e
// times a block fixed by the kinds of its four faces and the face
// viscosities of eq. (eta_face) relative to eta_e: the key of that block.
BlockKey block_key(const sdg_mesh& m, const double* et, int e) {
  const int nx = m.nx, ny = m.ny, ix = e % nx, iy = e / nx;
  const double ee = et[e];
  BlockKey key;
  const int nbs[4] = {ix > 0 ? e - 1 : -1, ix < nx - 1 ? e + 1 : -1, iy > 0 ? e - nx : -1,
                      iy < ny - 1 ? e + nx : -1};
  for (int f = 0; f < 4; ++f) {
    if (nbs[f] >= 0) {
      key.kind[f] = F_INTERIOR;
      const double r = et[nbs[f]] / ee;
      key.ratio[f] = r > 1.0 ? r : 1.0;
    } else {
      key.kind[f] = m.bc[f];
      key.ratio[f] = 1.0;
    }
  }
  return key;
}

int setup_blocks(sdg_problem* P) {
  const int nel = P->nel;
  const int64_t ntot = (int64_t)nel * P->nb;
  std::vector<int> ids(ntot);
  std::vector<double> scale(ntot);
  P->reps.clear();
  std::unordered_map<BlockKey, int, BlockKeyHash> map;
  BlockKey prev_key{};
  int prev_id = -1;
  for (int64_t ge = 0; ge < ntot; ++ge) {
    const int64_t pb = ge / nel;
    const int e = (int)(ge - pb * nel);
    const double* et = P->eta_host.data() + pb * nel;
    const double ee = et[e];
    const BlockKey key = block_key(P->mesh, et, e);
    int id;
    if (P->opt.dedup && ge > 0 && key == prev_key) {
      id = prev_id;  // neighbouring elements mostly share a block: no hashing
    } else if (P->opt.dedup) {
      auto it = map.find(key);
      if (it == map.end()) {
        id = (int)P->reps.size();
        map.emplace(key, id);
        P->reps.push_back((int)ge);
      } else {
        id = it->second;
      }
    } else {
      id = (int)P->reps.size();
      P->reps.push_back((int)ge);
    }
    ids[ge] = id;
    scale[ge] = P->eta_host[P->reps[id]] / ee;
    prev_key = key;
    prev_id = id;
  }
  P->nuniq = (int)P->reps.size();
  // group the elements by block (counting sort, element order kept inside
  // a group) and cut each group into work items of at most G elements
  // 16 elements per work item: one wavefront's matrix-core columns
  const int G = bj_group_size(P->NB);
  std::vector<int> first(P->nuniq + 1, 0);
  for (int64_t ge = 0; ge < ntot; ++ge) ++first[ids[ge] + 1];
  for (int u = 0; u < P->nuniq; ++u) first[u + 1] += first[u];
  std::vector<int> perm(ntot), fill(first.begin(), first.end() - 1), work;
  for (int64_t ge = 0; ge < ntot; ++ge) perm[fill[ids[ge]]++] = (int)ge;
  for (int u = 0; u < P->nuniq; ++u)
    for (int st = first[u]; st < first[u + 1]; st += G) {
      work.push_back(u);
      work.push_back(st);
      work.push_back(std::min(G, first[u + 1] - st));
    }
  int *dperm = nullptr, *dwork = nullptr;
  SDG_TRY(palloc_t(P, &dperm, ntot));
  SDG_TRY(palloc_t(P, &dwork, (int64_t)work.size()));
  SDG_TRY(palloc_t(P, &P->scale, ntot));
  SDG_TRY(to_dev(P, dperm, perm.data(), ntot * sizeof(int)));
  SDG_TRY(to_dev(P, dwork, work.data(), work.size() * sizeof(int)));
  SDG_TRY(to_dev(P, P->scale, scale.data(), ntot * sizeof(double)));
  P->bj = BjPlan{P->NB, G, (int)(work.size() / 3), P->nel, dperm, dwork, P->scale};
  // fewer than two elements per work item on average (a viscosity that
  // varies per element): the smoother is bound by reading the blocks, which
  // the streaming kernels read once, coalesced, from a packed triangle
  // (k <= 4; above, the matrix-core kernels measured faster)
  P->bj.stream = P->k <= 4 && ntot < 2 * (int64_t)P->bj.nwork;
  int* dreps = nullptr;
  int* dstat = nullptr;
  SDG_TRY(palloc_t(P, &dreps, P->nuniq));
  SDG_TRY(palloc_t(P, &dstat, P->nuniq));
  SDG_TRY(to_dev(P, dreps, P->reps.data(), P->nuniq * sizeof(int)));
  const int64_t nbb = (int64_t)P->NB * P->NB;
  const int64_t npk = (int64_t)P->NB * (P->NB + 1) / 2;
  const bool low = P->opt.prec_apply == SDG_FP32 || P->opt.prec_smoother != SDG_FP64;
  double* packed = nullptr;
  if (low) SDG_TRY(palloc_t(P, &packed, (int64_t)P->nuniq * npk));
  SDG_TRY(palloc_t(P, &P->binv, (int64_t)P->nuniq * nbb));
  SDG_TRY(sip_block_list(P->M, P->k, P->eta, dreps, P->nuniq, P->binv, P->s));
  SDG_TRY(spd_inverse(P->binv, P->NB, P->nuniq, dstat, P->s, packed));
  if (P->bj.stream) {
    SDG_TRY(palloc_t(P, &P->binvq, (int64_t)P->nuniq * tri_quad_size(P->NB)));
    SDG_TRY(sym_quad_f64(P->binv, P->NB, P->nuniq, P->binvq, P->s));
  }
  std::vector<int> st(P->nuniq);
  SDG_TRY(to_host(P, st.data(), dstat, P->nuniq * sizeof(int)));
  for (int i = 0; i < P->nuniq; ++i)
    if (st[i]) {
      set_error("element block " + std::to_string(P->reps[i]) + " is not positive definite");
      return SDG_ERR_UNSUPPORTED;
    }
  // low precision: the inverse Cholesky factor X = L^{-1} in FP32 or BF16,
  // once per block as a packed lower triangle of 2 x 2 quads; the smoother
  // applies X^T X
  P->xpacked = packed;
  if (low && P->opt.prec_smoother == SDG_BF16) {
    SDG_TRY(palloc_t(P, &P->binv16, (int64_t)P->nuniq * tri_quad_size(P->NB)));
    SDG_TRY(tri_quad_bf16(packed, P->NB, P->nuniq, P->binv16, P->s));
  } else if (low) {
    SDG_TRY(palloc_t(P, &P->binv32, (int64_t)P->nuniq * tri_quad_size(P->NB)));
    SDG_TRY(tri_quad_f32(packed, P->NB, P->nuniq, P->binv32, P->s));
  }
  return SDG_OK;
}

int q0_stencil(sdg_problem* P, double* st);

// the problem's stream waits for the coarsest level's inverse, whose flags
// are then checked
int join_dense(sdg_problem* P) {
  if (!P->dense_stat) return SDG_OK;
  SDG_HIP(hipStreamWaitEvent(P->s, P->ds_ev[1], 0));
  std::vector<int> st(P->nb);
  SDG_TRY(to_host(P, st.data(), P->dense_stat, P->nb * sizeof(int)));
  P->dense_stat = nullptr;
  for (int i = 0; i < P->nb; ++i)
    if (st[i]) {
      set_error("coarsest operator is not positive definite (a rigid motion is not restrained)");
      return SDG_ERR_UNSUPPORTED;
    }
  return SDG_OK;
}

int setup_coarse(sdg_problem* P) {
  const int nx = P->mesh.nx, ny = P->mesh.ny, nb = P->nb;
  const bool q0 = P->opt.coarse_space == 1;
  double* clocal = nullptr;
  if (!q0) {
    SDG_TRY(palloc_t(P, &clocal, (int64_t)P->nel * nb * 64));
    SDG_TRY(sip_coarse_local(P->M, P->k, nb, P->eta, clocal, P->s));
  }
  // Q_1: the (nx + 1) x (ny + 1) vertices; Q_0: the nx x ny element centres,
  // a node grid of nx - 1 by ny - 1 intervals
  int cx = q0 ? nx - 1 : nx, cy = q0 ? ny - 1 : ny;
  P->lev.clear();
  while (true) {
    CLevel L;
    L.nx = cx;
    L.ny = cy;
    L.nn = (cx + 1) * (cy + 1);
    const int64_t nv = (int64_t)2 * L.nn * nb;
    SDG_TRY(palloc_t(P, &L.st, (int64_t)36 * L.nn * nb));
    for (double** v : {&L.b, &L.x, &L.xalt, &L.r, &L.d}) SDG_TRY(palloc_t(P, v, nv));
    if (P->lev.empty()) {
      if (q0) SDG_TRY(q0_stencil(P, L.st));
      else SDG_TRY(coarse_stencil_from_local(cx, cy, nb, clocal, L.st, P->s));
    } else {
      const CLevel& F = P->lev.back();
      SDG_TRY(galerkin_coarsen(F.nx, F.ny, nb, F.st, L.st, P->s));
    }
    const bool more = (cx % 2 == 0) && (cy % 2 == 0) && cx > P->opt.coarsest_n && cy > P->opt.coarsest_n;
    L.coarsest = !more;
    if (L.coarsest) {
      const int n2 = 2 * L.nn;
      if (n2 > 2048) {
        set_error("coarsest level too large for the dense solve (more than 2048 unknowns); use element "
                  "counts with more factors of two");
        return SDG_ERR_UNSUPPORTED;
      }
      int* dstat = nullptr;
      SDG_TRY(palloc_t(P, &L.dense, (int64_t)n2 * n2 * nb));
      SDG_TRY(palloc_t(P, &dstat, nb));
      SDG_TRY(stencil_to_dense(cx, cy, nb, L.st, L.dense, P->s));
      // one workgroup per problem (about 4 ms for 16 problems of 9 x 9
      // nodes): on the side stream it overlaps the eigenvalue estimates,
      // which do not read it; join_dense ends setup with it
      if (!P->ds) SDG_HIP(hipStreamCreateWithFlags(&P->ds, hipStreamNonBlocking));
      for (hipEvent_t& e : P->ds_ev)
        if (!e) SDG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      SDG_HIP(hipEventRecord(P->ds_ev[0], P->s));
      SDG_HIP(hipStreamWaitEvent(P->ds, P->ds_ev[0], 0));
      SDG_TRY(spd_inverse(L.dense, n2, nb, dstat, P->ds));
      SDG_HIP(hipEventRecord(P->ds_ev[1], P->ds));
      P->dense_stat = dstat;
    } else {
      SDG_TRY(palloc_t(P, &L.dinv, nv));
      SDG_TRY(stencil_diag_inv(cx, cy, nb, L.st, L.dinv, P->s));
      SDG_TRY(palloc_t(P, &L.ab, (int64_t)P->opt.smooth_h * nb * 2));
    }
    P->lev.push_back(L);
    if (L.coarsest) break;
    cx /= 2;
    cy /= 2;
  }
  // the tail: the suffix of levels with few nodes (always includes the coarsest)
  const int nl = (int)P->lev.size();
  int ts = nl - 1;
  while (ts > 0 && P->lev[ts - 1].nn <= TAIL_NODES && nl - (ts - 1) <= TAIL_MAXLEV) --ts;
  P->tail_start = ts;
  return SDG_OK;
}

// traced launches of the hot kernels (algorithmic bytes: vectors once each)
// problems the traced launch works on: inside a CG iteration the converged
// ones are skipped
double traced_problems(const sdg_problem* P) { return P->M.active ? P->nact_host : P->nb; }
double vec_bytes(const sdg_problem* P, int w) { return (double)P->nel * traced_problems(P) * P->NB * w; }
double elem_bytes(const sdg_problem* P, int w) { return (double)P->nel * traced_problems(P) * w; }
int run_sip_apply(sdg_problem* P, const double* u, double* y) {
  return traced(P->ctx, P->s, SDG_TRACE_SIP_APPLY, 2 * vec_bytes(P, 8) + elem_bytes(P, 8),
                [&] { return sip_apply(P->M, P->k, P->nb, P->eta, u, y, P->s, P->tile[0][0]); });
}
// A_0 = (P_k^0)^T A P_k^0 (Section 6.1.1) by probing: A applied to the unit
// (0, 0) mode of one component on every element of one colour of a 3 x 3
// colouring (18 applies); the (0, 0) responses are the stencil entries.
int q0_stencil(sdg_problem* P, double* st) {
  const int nx = P->mesh.nx, ny = P->mesh.ny, nb = P->nb;
  const int64_t U = P->nu * nb;
  double *v = nullptr, *y = nullptr;
  if (tmp_get(P, &v, U) < 0 || tmp_get(P, &y, U) < 0) {
    tmp_put(P, v, U);
    set_error("allocation of the Q_0 probe vectors failed");
    return SDG_ERR_NOMEM;
  }
  int rc = SDG_OK;
  if (hipMemsetAsync(st, 0, (size_t)36 * P->nel * nb * sizeof(double), P->s) != hipSuccess) rc = SDG_ERR_DEVICE;
  for (int c = 0; c < 9 && rc >= 0; ++c)
    for (int d = 0; d < 2 && rc >= 0; ++d) {
      rc = q0_probe_vec(nx, ny, nb, P->k, c % 3, c / 3, d, v, P->s);
      if (rc >= 0) rc = sip_apply(P->M, P->k, nb, P->eta, v, y, P->s, 0);
      if (rc >= 0) rc = q0_probe_gather(nx, ny, nb, P->k, c % 3, c / 3, d, y, st, P->s);
    }
  tmp_put(P, v, U);  // synchronises the stream first
  tmp_put(P, y, U);
  return rc;
}

// y = A u and out[pb] = u.y.  With the wavefront kernel the product is
// summed inside the operator kernel (per-tile partials, then a fixed-order
// sum), which saves a pass over u and y; otherwise apply, then dot.
int run_sip_apply_dot(sdg_problem* P, const double* u, double* y, double* out) {
  const int parts = sip_apply_dot_parts(P->M, P->k, P->nb);
  if (P->tile[0][0] != 0 || parts <= 0 || parts > RED_SCRATCH) {
    SDG_TRY(run_sip_apply(P, u, y));
    return bmulti_dot(P->nu, P->nb, 1, u, 0, y, out, P->red, P->s);
  }
  SDG_TRY(traced(P->ctx, P->s, SDG_TRACE_SIP_APPLY, 2 * vec_bytes(P, 8) + elem_bytes(P, 8), [&] {
    return sip_apply_dot(P->M, P->k, P->nb, P->eta, u, y, P->red, RED_SCRATCH, P->s);
  }));
  return reduce_parts(parts / P->nb, P->nb, P->red, out, P->s);
}
// y = A u and the partial sums of u.y, *nparts per problem in P->red (at
// most cap in all): the operator kernel's per-tile partials, or a first
// reduction stage after a plain apply
int run_sip_apply_dot_parts(sdg_problem* P, const double* u, double* y, int cap, int* nparts) {
  const int parts = sip_apply_dot_parts(P->M, P->k, P->nb);
  if (P->tile[0][0] != 0 || parts <= 0 || parts > cap) {
    SDG_TRY(run_sip_apply(P, u, y));
    return bdot_parts(P->nu, P->nb, u, y, P->red, cap, nparts, P->s, P->M.active);
  }
  SDG_TRY(traced(P->ctx, P->s, SDG_TRACE_SIP_APPLY, 2 * vec_bytes(P, 8) + elem_bytes(P, 8), [&] {
    return sip_apply_dot(P->M, P->k, P->nb, P->eta, u, y, P->red, cap, P->s);
  }));
  *nparts = parts / P->nb;
  return SDG_OK;
}
int run_sip_residual(sdg_problem* P, const double* b, const double* u, double* r) {
  return traced(P->ctx, P->s, SDG_TRACE_SIP_RESIDUAL, 3 * vec_bytes(P, 8) + elem_bytes(P, 8),
                [&] { return sip_residual(P->M, P->k, P->nb, P->eta, b, u, r, P->s, P->tile[1][0]); });
}
int run_sip_apply_f32(sdg_problem* P, const float* u, float* y) {
  return traced(P->ctx, P->s, SDG_TRACE_SIP_APPLY, 2 * vec_bytes(P, 4) + elem_bytes(P, 8),
                [&] { return sip_apply_f32(P->M, P->k, P->nb, P->eta, u, y, P->s, P->tile[0][1]); });
}
int run_sip_residual_f32(sdg_problem* P, const float* b, const float* u, float* r) {
  return traced(P->ctx, P->s, SDG_TRACE_SIP_RESIDUAL, 3 * vec_bytes(P, 4) + elem_bytes(P, 8),
                [&] { return sip_residual_f32(P->M, P->k, P->nb, P->eta, b, u, r, P->s, P->tile[1][1]); });
}
// Unit-block tables of the extended-precision residual for the problem's
// mesh: integrated on the host in long double once per context and mesh.
int ensure_ext(sdg_problem* P) {
  if (P->ext) return SDG_OK;
  sdg_ctx* c = P->ctx;
  const sdg_mesh& m = P->mesh;
  char key[160];
  std::snprintf(key, sizeof(key), "%d/%d/%d/%.17g/%.17g/%d%d%d%d", m.k, m.nx, m.ny, m.lx, m.ly, m.bc[0], m.bc[1],
                m.bc[2], m.bc[3]);
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->ext.find(key);
  if (it == c->ext.end()) {
    std::vector<double2> TA, TBu, TBp;
    sdg_ctx::ExtEntry E;
    ext_unit_blocks(m.k, m.lx, m.ly, m.nx, m.ny, m.bc, TA, TBu, TBp, E.T.cpen);
    const size_t na = TA.size() * sizeof(double2), nbu = TBu.size() * sizeof(double2);
    const size_t bytes = na + 2 * nbu;
    if (hipMalloc(&E.mem, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("allocation of the extended-precision operator tables failed");
      return SDG_ERR_NOMEM;
    }
    char* base = (char*)E.mem;
    if (hipMemcpy(base, TA.data(), na, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + na, TBu.data(), nbu, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + na + nbu, TBp.data(), nbu, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(E.mem);
      set_error("upload of the extended-precision operator tables failed");
      return SDG_ERR_DEVICE;
    }
    E.T.A = (const double2*)base;
    E.T.Bu = (const double2*)(base + na);
    E.T.Bp = (const double2*)(base + na + nbu);
    it = c->ext.emplace(key, E).first;
  }
  P->ext = &it->second.T;
  return SDG_OK;
}
// r = b - K (xh + xl) in double-FP64 (stokes: velocity then pressure block
// of the stacked vectors); abs_mode: r = |K||xh|
int run_ext(sdg_problem* P, bool stokes, bool abs_mode, const double* b, const double* xh, const double* xl,
            double* r) {
  SDG_TRY(ensure_ext(P));
  const int64_t U = P->nu * P->nb;
  const bool st = stokes && P->np > 0;
  return ext_residual(P->M, P->k, P->nb, abs_mode, P->eta, b, xh, xl, st ? xh + U : nullptr,
                      (st && xl) ? xl + U : nullptr, st ? b + U : nullptr, *P->ext, r, st ? r + U : nullptr, P->s);
}
// effective unit roundoff of the true residual: FP64 evaluation, or the
// extended one (coefficients exact to the 64-bit mantissa of long double)
double resid_eps(const sdg_problem* P) { return P->opt.refine ? 0x1p-63 : 0x1p-53; }

std::array<int, 6> tune_key(const sdg_problem* P, int kernel, int prec) {
  return {P->k, P->mesh.nx, P->mesh.ny, P->nb, kernel, prec};
}
void drop_graphs(sdg_problem* P) {
  for (hipGraphExec_t& g : P->cg_graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}
double smoother_bytes(const sdg_problem* P, int flags, int w) {
  const int nvec = 2 + !!(flags & BJ_READ_X) + !!(flags & BJ_READ_D) + !!(flags & BJ_WRITE_D);
  double b = nvec * vec_bytes(P, w) + elem_bytes(P, 12);  // + scale and permutation
  // streamed plans: every block read once from HBM (packed triangle)
  if (P->bj.stream)
    b += (double)P->nuniq * tri_quad_size(P->NB) * (P->binv16 ? 2 : w == 4 ? 4 : 8) * traced_problems(P) / P->nb;
  return b;
}
// the FP64 smoother's operand: quad-packed inverses for streamed plans
const double* bj_inverses(const sdg_problem* P) { return P->bj.stream ? P->binvq : P->binv; }

// Chebyshev coefficients: step 0 -> (0, 1/theta); step s >= 1 ->
// (rho_s rho_{s-1}, 2 rho_s / delta) with rho_0 = 1/sigma,
// rho_s = 1/(2 sigma - rho_{s-1})
void cheb_coefs(double lmin, double lmax, int steps, std::vector<double>& out, int nb, int pb) {
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  for (int s = 0; s < steps; ++s) {
    double a, b;
    if (s == 0) {
      a = 0.0;
      b = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      a = rn * rho;
      b = 2.0 * rn / delta;
      rho = rn;
    }
    out[((size_t)s * nb + pb) * 2] = a;
    out[((size_t)s * nb + pb) * 2 + 1] = b;
  }
}

int upload_cheb(sdg_problem* P) {
  const int nb = P->nb;
  std::vector<double> c0((size_t)P->opt.smooth_dg * nb * 2);
  for (int pb = 0; pb < nb; ++pb) cheb_coefs(P->lmin0[pb], P->lmax0[pb], P->opt.smooth_dg, c0, nb, pb);
  SDG_TRY(to_dev(P, P->ab0, c0.data(), c0.size() * sizeof(double)));
  for (auto& L : P->lev) {
    if (L.coarsest) continue;
    std::vector<double> c((size_t)P->opt.smooth_h * nb * 2);
    for (int pb = 0; pb < nb; ++pb) cheb_coefs(L.lmin[pb], L.lmax[pb], P->opt.smooth_h, c, nb, pb);
    SDG_TRY(to_dev(P, L.ab, c.data(), c.size() * sizeof(double)));
  }
  TailArgs& T = P->tail;
  T.nlev = (int)P->lev.size() - P->tail_start;
  T.nbatch = nb;
  T.steps = P->opt.smooth_h;
  for (int i = 0; i < T.nlev; ++i) {
    const CLevel& L = P->lev[P->tail_start + i];
    T.lev[i] = TailLevel{L.nx, L.ny, L.st, L.dinv, L.b, L.x, L.r, L.d, L.ab};
  }
  T.dense = P->lev.back().dense;
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// multigrid cycle
// ---------------------------------------------------------------------------
const double* ab0_step(sdg_problem* P, int s) { return P->ab0 + (int64_t)s * P->nb * 2; }

// Update flags of Chebyshev step s of m on the DG level.  From a zero start
// the first direction equals the first iterate, so step 1 takes it from x
// (BJ_FOLD) and step 0 stores no direction; the last step stores none.
int bj_flags(int s, int m, bool zero) {
  int f = 0;
  if (s > 0 || !zero) f |= BJ_READ_X;
  if (s == 1 && zero) f |= BJ_FOLD;
  else if (s > 0) f |= BJ_READ_D;
  if (s < m - 1 && !(s == 0 && zero)) f |= BJ_WRITE_D;
  return f;
}
int bj_step64(sdg_problem* P, const double* r, int s, double* x, bool zero) {
  const int f = bj_flags(s, P->opt.smooth_dg, zero);
  return traced(P->ctx, P->s, SDG_TRACE_SMOOTHER, smoother_bytes(P, f, 8),
                [&] { return bj_cheb_f64(P->bj, bj_inverses(P), r, ab0_step(P, s), P->vd, x, f, P->s); });
}
int bj_step32(sdg_problem* P, const float* r, int s, float* x, bool zero) {
  const int f = bj_flags(s, P->opt.smooth_dg, zero);
  return traced(P->ctx, P->s, SDG_TRACE_SMOOTHER, smoother_bytes(P, f, 4), [&] {
    if (P->binv16) return bj_tri_cheb_bf16(P->bj, P->binv16, r, ab0_step(P, s), P->fd, x, f, P->s);
    return bj_tri_cheb_f32(P->bj, P->binv32, r, ab0_step(P, s), P->fd, x, f, P->s);
  });
}
int bj_apply32(sdg_problem* P, const float* r, float* z) {
  return traced(P->ctx, P->s, SDG_TRACE_SMOOTHER, smoother_bytes(P, BJ_APPLY, 4), [&] {
    if (P->binv16) return bj_tri_apply_bf16(P->bj, P->binv16, r, z, P->s);
    return bj_tri_apply_f32(P->bj, P->binv32, r, z, P->s);
  });
}
int bj_apply64(sdg_problem* P, const double* r, double* z) {
  return traced(P->ctx, P->s, SDG_TRACE_SMOOTHER, smoother_bytes(P, BJ_APPLY, 8),
                [&] { return bj_apply_f64(P->bj, bj_inverses(P), r, z, P->s); });
}

int cheb_dg64(sdg_problem* P, const double* b, double* x, bool zero) {
  for (int s = 0; s < P->opt.smooth_dg; ++s) {
    const double* r = b;
    if (!(s == 0 && zero)) {
      SDG_TRY(run_sip_residual(P, b, x, P->vr));
      r = P->vr;
    }
    SDG_TRY(bj_step64(P, r, s, x, zero));
  }
  return SDG_OK;
}
int cheb_dg32(sdg_problem* P, const float* b, float* x, bool zero) {
  for (int s = 0; s < P->opt.smooth_dg; ++s) {
    const float* r = b;
    if (!(s == 0 && zero)) {
      SDG_TRY(run_sip_residual_f32(P, b, x, P->fr));
      r = P->fr;
    }
    SDG_TRY(bj_step32(P, r, s, x, zero));
  }
  return SDG_OK;
}

// Chebyshev steps s0 .. smooth_h - 1 of an h-level (steps before s0 were
// done by a fused kernel, which leaves its result in L.xalt for the swap)
int cheb_h(sdg_problem* P, CLevel& L, bool zero, int s0 = 0) {
  for (int s = s0; s < P->opt.smooth_h; ++s) {
    const int mode = s == 0 ? (zero ? 1 : 2) : 0;
    const double* ab = L.ab + (int64_t)s * P->nb * 2;
    SDG_TRY(hcheb_step(L.nx, L.ny, P->nb, L.st, L.dinv, L.b, L.x, L.xalt, L.d, ab, mode, P->s));
    std::swap(L.x, L.xalt);
  }
  return SDG_OK;
}

// first_done: the level's first Chebyshev step (from zero) was fused into
// the kernel that restricted its right-hand side.  The coarse level's first
// pre-smoothing step rides on the restriction (same arithmetic, one launch
// fewer per level; the fused step still swaps x and xalt, so every cycle
// swaps an even number of times and captured graphs see the same buffers on
// every replay).  (Folding the prolongation into the first post-smoothing
// step as well, forming x + P e at the nine stencil nodes, took the
// headline step from 289 to 333 ms: far dearer than the launch it saved.)
int hcycle(sdg_problem* P, int li, bool first_done = false) {
  if (li >= P->tail_start)
    return traced(P->ctx, P->s, SDG_TRACE_COARSE_TAIL, 0.0, [&] { return coarse_tail(P->tail, P->s); });
  CLevel& L = P->lev[li];
  CLevel& C = P->lev[li + 1];
  const bool steps = P->opt.smooth_h > 0;
  SDG_TRY(cheb_h(P, L, true, first_done ? 1 : 0));
  SDG_TRY(stencil_residual(L.nx, L.ny, P->nb, L.st, L.b, L.x, L.r, P->s));
  const bool fuse_c = steps && li + 1 < P->tail_start;  // the tail smooths its levels itself
  if (fuse_c) {
    SDG_TRY(h_restrict_first(C.nx, C.ny, P->nb, L.r, C.b, C.dinv, C.ab, C.xalt, C.d, P->s));
    std::swap(C.x, C.xalt);
  } else {
    SDG_TRY(h_restrict(C.nx, C.ny, P->nb, L.r, C.b, P->s));
  }
  SDG_TRY(hcycle(P, li + 1, fuse_c));
  SDG_TRY(h_prolong_add(C.nx, C.ny, P->nb, C.x, L.x, P->s));
  SDG_TRY(cheb_h(P, L, false));
  return SDG_OK;
}

// the operands of level 0's zero-start step when the p-restriction can do it
// (level 0 smoothed by the per-level kernels, not by the tail)
bool first_step(sdg_problem* P, FirstStep& fs) {
  if (P->tail_start == 0 || P->opt.smooth_h <= 0) return false;
  CLevel& L = P->lev[0];
  fs = FirstStep{L.dinv, L.ab, L.xalt, L.d};
  return true;
}
int vcycle64(sdg_problem* P, const double* b, double* x) {
  SDG_TRY(cheb_dg64(P, b, x, true));
  // only the Q1 modes of the residual reach the coarse space: the operator
  // kernel writes just those (8 values per element, laid out as a k = 1
  // vector) and the restriction reads them with k = 1
  // algorithmic bytes: u, eta, the Q1 modes of b, the 8 values written
  SDG_TRY(traced(P->ctx, P->s, SDG_TRACE_SIP_RESIDUAL, vec_bytes(P, 8) + 17 * elem_bytes(P, 8),
                 [&] { return sip_residual_q1(P->M, P->k, P->nb, P->eta, b, x, P->vr, P->s); }));
  const int64_t nelt = (int64_t)P->nel * P->nb;
  bool first_done = false;
  if (P->opt.coarse_space == 1) {
    SDG_TRY(q0_restrict(nelt, P->vr, P->lev[0].b, P->s));
  } else {
    FirstStep fs;
    first_done = first_step(P, fs);
    SDG_TRY(p_restrict(P->M, 1, P->nb, P->vr, P->lev[0].b, P->s, first_done ? &fs : nullptr));
  }
  if (first_done) std::swap(P->lev[0].x, P->lev[0].xalt);
  SDG_TRY(hcycle(P, 0, first_done));
  if (P->opt.coarse_space == 1) SDG_TRY(q0_prolong_add(nelt, P->k, P->lev[0].x, x, P->s));
  else SDG_TRY(p_prolong_add(P->M, P->k, P->nb, P->lev[0].x, x, P->s));
  SDG_TRY(cheb_dg64(P, b, x, false));
  return SDG_OK;
}

// fine level in FP32 (FP64 in and out); the coarse Q1 hierarchy stays FP64
int vcycle32(sdg_problem* P, const double* b, double* x) {
  const int64_t n = P->nu * P->nb;
  SDG_TRY(d2f(n, b, P->fb, P->s));
  SDG_TRY(cheb_dg32(P, P->fb, P->fx, true));
  // the residual's Q1 modes only (as in the FP64 cycle)
  SDG_TRY(traced(P->ctx, P->s, SDG_TRACE_SIP_RESIDUAL, vec_bytes(P, 4) + 9 * elem_bytes(P, 8),
                 [&] { return sip_residual_q1_f32(P->M, P->k, P->nb, P->eta, P->fb, P->fx, P->fr, P->s); }));
  const int64_t nelt = (int64_t)P->nel * P->nb;
  bool first_done = false;
  if (P->opt.coarse_space == 1) {
    SDG_TRY(q0_restrict_f32(nelt, P->fr, P->lev[0].b, P->s));
  } else {
    FirstStep fs;
    first_done = first_step(P, fs);
    SDG_TRY(p_restrict_f32(P->M, 1, P->nb, P->fr, P->lev[0].b, P->s, first_done ? &fs : nullptr));
  }
  if (first_done) std::swap(P->lev[0].x, P->lev[0].xalt);
  SDG_TRY(hcycle(P, 0, first_done));
  if (P->opt.coarse_space == 1) SDG_TRY(q0_prolong_add_f32(nelt, P->k, P->lev[0].x, P->fx, P->s));
  else SDG_TRY(p_prolong_add_f32(P->M, P->k, P->nb, P->lev[0].x, P->fx, P->s));
  SDG_TRY(cheb_dg32(P, P->fb, P->fx, false));
  SDG_TRY(f2d(n, P->fx, x, P->s));
  return SDG_OK;
}

bool low_precision(const sdg_problem* P) {
  return P->opt.prec_apply == SDG_FP32 || P->opt.prec_smoother != SDG_FP64;
}

int vcycle(sdg_problem* P, const double* b, double* x) {
  return low_precision(P) ? vcycle32(P, b, x) : vcycle64(P, b, x);
}

// ---------------------------------------------------------------------------
// batched vector helpers over one or two segments per problem (Stokes
// vectors: all velocities, then all pressures)
// ---------------------------------------------------------------------------
struct Seg {
  int64_t off;  // offset of the segment block
  int64_t n;    // per-problem length
};
struct VSpec {
  Seg seg[2];
  int nseg;
  int64_t total;  // length of one batched vector
};
VSpec viscous_spec(const sdg_problem* P) {
  VSpec v;
  v.seg[0] = {0, P->nu};
  v.seg[1] = {0, 0};
  v.nseg = 1;
  v.total = P->nu * P->nb;
  return v;
}
VSpec stokes_spec(const sdg_problem* P) {
  VSpec v;
  v.seg[0] = {0, P->nu};
  v.seg[1] = {P->nu * P->nb, P->np};
  v.nseg = P->np > 0 ? 2 : 1;
  v.total = (P->nu + P->np) * P->nb;
  return v;
}

// out[pb * m + j] = <V_j[pb], w[pb]> summed over the segments (host array)
int vs_dots(sdg_problem* P, const VSpec& S, int m, const double* V, int64_t ldv, const double* w,
            std::vector<double>& out) {
  const int nb = P->nb;
  out.assign((size_t)nb * m, 0.0);
  std::vector<double> part((size_t)nb * m);
  for (int q = 0; q < S.nseg; ++q) {
    SDG_TRY(bmulti_dot(S.seg[q].n, nb, m, V + S.seg[q].off, ldv, w + S.seg[q].off, sc_h(P), P->red, P->s));
    SDG_TRY(read_dev(P, sc_h(P), nb * m, part.data()));
    for (size_t i = 0; i < part.size(); ++i) out[i] += part[i];
  }
  return SDG_OK;
}
int vs_axpy(sdg_problem* P, const VSpec& S, int m, const double* V, int64_t ldv, const double* hdev, double* w) {
  for (int q = 0; q < S.nseg; ++q)
    SDG_TRY(bmulti_axpy(S.seg[q].n, P->nb, m, V + S.seg[q].off, ldv, hdev, w + S.seg[q].off, P->s));
  return SDG_OK;
}
int vs_combine(sdg_problem* P, const VSpec& S, int m, const double* V, int64_t ldv, const double* hdev, double* y) {
  for (int q = 0; q < S.nseg; ++q)
    SDG_TRY(bmulti_combine(S.seg[q].n, P->nb, m, V + S.seg[q].off, ldv, hdev, y + S.seg[q].off, P->s));
  return SDG_OK;
}
// y = x / a[pb] (a in device memory; a = 0 -> 0)
int vs_div(sdg_problem* P, const VSpec& S, const double* adev, const double* x, double* y) {
  for (int q = 0; q < S.nseg; ++q)
    SDG_TRY(bscale(S.seg[q].n, P->nb, adev, x + S.seg[q].off, y + S.seg[q].off, 1, P->s));
  return SDG_OK;
}
int vs_norms(sdg_problem* P, const VSpec& S, const double* x, std::vector<double>& out) {
  SDG_TRY(vs_dots(P, S, 1, x, 0, x, out));
  for (auto& v : out) v = std::sqrt(v > 0 ? v : 0.0);
  return SDG_OK;
}
// host -> device without waiting: the bytes are copied into a slot of the
// pinned staging ring and the copy is queued on the problem's stream, ahead
// of the launches that read dst (larger uploads wait, as to_dev)
int to_dev_async(sdg_problem* P, void* dst, const void* src, size_t bytes) {
  if (!P->hstage || bytes > sdg_problem::STAGE_BYTES) return to_dev(P, dst, src, bytes);
  const int k = P->stage_next;
  P->stage_next = (k + 1) % sdg_problem::STAGE_SLOTS;
  SDG_HIP(hipEventSynchronize(P->stage_ev[k]));  // the slot's previous copy is done
  char* slot = P->hstage + (size_t)k * sdg_problem::STAGE_BYTES;
  std::memcpy(slot, src, bytes);
  SDG_HIP(hipMemcpyAsync(dst, slot, bytes, hipMemcpyHostToDevice, P->s));
  SDG_HIP(hipEventRecord(P->stage_ev[k], P->s));
  return SDG_OK;
}
int upload_scalars(sdg_problem* P, double* dst, const std::vector<double>& v) {
  return to_dev_async(P, dst, v.data(), v.size() * sizeof(double));
}
int upload_active(sdg_problem* P, const std::vector<int>& act) {
  P->nact_host = (int)std::count(act.begin(), act.end(), 1);
  return to_dev_async(P, P->active, act.data(), act.size() * sizeof(int));
}

// ---------------------------------------------------------------------------
// Chebyshev bounds: Arnoldi (classical Gram-Schmidt twice) on M^{-1} A for
// every problem of the batch; level -1 = DG level, li >= 0 = CG level li
// ---------------------------------------------------------------------------
int vs_dots_dev(sdg_problem* P, const VSpec& S, int mj, const double* V, int64_t ldv, const double* w,
                double* dst, double* segb);
int arnoldi(sdg_problem* P, int li, std::vector<double>& lambda, std::vector<double>* hess_out) {
  const int m = P->opt.eig_steps, nb = P->nb;
  const int64_t n = li < 0 ? P->nu : 2 * (int64_t)P->lev[li].nn;
  VSpec S;
  S.seg[0] = {0, n};
  S.seg[1] = {0, 0};
  S.nseg = 1;
  S.total = n * nb;
  double *V = nullptr, *w = nullptr, *dH = nullptr, *lam = nullptr, *hb = nullptr;
  int *dms = nullptr, *dstop = nullptr;
  const int64_t nV = (int64_t)(m + 1) * S.total, nH = (int64_t)(m + 1) * m * nb;
  // hb: the two passes' coefficients [2][nb][m], ||w||^2 [nb], divisors [nb]
  const int64_t nhb = (int64_t)(2 * m + 2) * nb;
  auto release = [&] {
    tmp_put(P, V, nV);
    tmp_put(P, w, S.total);
    tmp_put(P, dH, nH);
    tmp_put(P, lam, nb);
    tmp_put(P, dms, nb);
    tmp_put(P, hb, nhb);
    tmp_put(P, dstop, nb);
  };
  if (tmp_get(P, &V, nV) < 0 || tmp_get(P, &w, S.total) < 0 || tmp_get(P, &dH, nH) < 0 ||
      tmp_get(P, &lam, nb) < 0 || tmp_get(P, &dms, nb) < 0 || tmp_get(P, &hb, nhb) < 0 ||
      tmp_get(P, &dstop, nb) < 0) {
    release();
    set_error("allocation of the Arnoldi workspace failed");
    return SDG_ERR_NOMEM;
  }
  double* hsq = hb + (int64_t)2 * m * nb;
  double* hs = hsq + nb;
  const uint64_t seed = P->opt.seed + ((uint64_t)(li + 1) << 32);
  int rc = SDG_OK;
  // The whole iteration stays on the device (coefficients, norms, the
  // Hessenberg matrices and each problem's stopping test); the host reads
  // the largest eigenvalues once at the end.
  do {
    // every problem starts from the same vector
    if ((rc = uniform_pm1(seed, n, V, P->s, nb)) < 0) break;
    const std::vector<int> ms0(nb, m);
    if (hipMemsetAsync(dH, 0, nH * sizeof(double), P->s) != hipSuccess ||
        hipMemsetAsync(dstop, 0, nb * sizeof(int), P->s) != hipSuccess) {
      set_error("clearing the Arnoldi workspace failed");
      rc = SDG_ERR_DEVICE;
      break;
    }
    if ((rc = to_dev_async(P, dms, ms0.data(), nb * sizeof(int))) < 0) break;
    // v_0 = v / ||v||
    if ((rc = vs_dots_dev(P, S, 1, V, 0, V, hsq, nullptr)) < 0) break;
    if ((rc = norm_mask(nb, hsq, dstop, hs, P->s)) < 0) break;
    if ((rc = vs_div(P, S, hs, V, V)) < 0) break;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (int64_t)j * S.total;
      if (li < 0 && low_precision(P)) {
        // bounds of the operator the smoother applies: FP32 apply, FP32/BF16 inverses
        if ((rc = d2f(S.total, vj, P->fb, P->s)) < 0) break;
        if ((rc = run_sip_apply_f32(P, P->fb, P->fr)) < 0) break;
        if ((rc = bj_apply32(P, P->fr, P->fd)) < 0) break;
        if ((rc = f2d(S.total, P->fd, w, P->s)) < 0) break;
      } else if (li < 0) {
        if ((rc = run_sip_apply(P, vj, P->vr)) < 0) break;
        if ((rc = bj_apply64(P, P->vr, w)) < 0) break;
      } else {
        CLevel& L = P->lev[li];
        if ((rc = stencil_apply(L.nx, L.ny, nb, L.st, vj, L.r, P->s)) < 0) break;
        if ((rc = vec_mul(S.total, L.dinv, L.r, w, P->s)) < 0) break;
      }
      // classical Gram-Schmidt twice, then column j of H and the next basis
      // vector (zero for a problem that has stopped)
      const int mj = j + 1;
      for (int pass = 0; pass < 2 && rc >= 0; ++pass) {
        double* hp = hb + (int64_t)pass * m * nb;
        if ((rc = vs_dots_dev(P, S, mj, V, S.total, w, hp, nullptr)) < 0) break;
        rc = vs_axpy(P, S, mj, V, S.total, hp, w);
      }
      if (rc < 0) break;
      if ((rc = vs_dots_dev(P, S, 1, w, 0, w, hsq, nullptr)) < 0) break;
      if ((rc = arnoldi_col(nb, j, m, hb, hb + (int64_t)m * nb, hsq, dstop, dms, dH, hs, P->s)) < 0) break;
      if ((rc = vs_div(P, S, hs, w, V + (int64_t)(j + 1) * S.total)) < 0) break;
    }
    if (rc < 0) break;
    if ((rc = bhessenberg_max_eig(nb, dH, dms, m + 1, (int64_t)(m + 1) * m, lam, P->s)) < 0) break;
    lambda.resize(nb);
    if ((rc = read_dev(P, lam, nb, lambda.data())) < 0) break;
    if (hess_out) {
      hess_out->resize((size_t)nH);
      if ((rc = read_dev(P, dH, (int)nH, hess_out->data())) < 0) break;
    }
  } while (0);
  release();  // synchronises the stream first
  return rc < 0 ? rc : SDG_OK;
}

// ---------------------------------------------------------------------------
// Krylov methods
// ---------------------------------------------------------------------------
// Batched preconditioned CG with x0 = 0; problem pb stops when
// ||r||_2 < rtol ||b||_2 (unpreconditioned, recursively updated residual).
// status[pb]: SDG_OK, SDG_NOT_CONVERGED or SDG_BREAKDOWN.
// The part of a CG iteration between two readbacks of the scalars: the
// V-cycle z = B r, r.z, p = z + beta p, q = A p, p.q, the x/r update and
// ||r||^2, then the copy of (p.q, ||r||^2) to the pinned mirror.  rzA holds
// the previous r.z, rzB receives the new one.
// While a CG iteration is issued (or captured), the operator kernels, the
// smoother, the dot products and the updates skip the problems whose active
// flag is 0: they have converged, their x and r stay as they are, and their
// other vectors are not read again in this solve.
struct CgMask {
  sdg_problem* P;
  explicit CgMask(sdg_problem* p) : P(p) {
    P->M.active = P->active;
    P->bj.active = P->active;
  }
  ~CgMask() {
    P->M.active = nullptr;
    P->bj.active = nullptr;
  }
};
int cg_body(sdg_problem* P, double* x, double* rzA, double* rzB) {
  const CgMask mask(P);
  const int nb = P->nb;
  const int64_t n = P->nu;
  // partial sums live in the two halves of the reduction scratch: r.z and
  // p.q in the first, ||r||^2 in the second (written while p.q's are read)
  constexpr int HALF = RED_SCRATCH / 2;
  double* part_rr = P->red + HALF;
  SDG_TRY(vcycle(P, P->cg_r, P->cg_z));
  int nrz = 0, npq = 0, nrr = 0;
  SDG_TRY(bdot_parts(n, nb, P->cg_r, P->cg_z, P->red, HALF, &nrz, P->s, P->active));
  SDG_TRY(cg_update2_red(n, nb, P->cg_z, P->cg_p, P->red, nrz, rzB, rzA, P->active, P->s));
  SDG_TRY(run_sip_apply_dot_parts(P, P->cg_p, P->cg_q, HALF, &npq));
  SDG_TRY(cg_update1_red(n, nb, P->cg_p, P->cg_q, x, P->cg_r, rzB, P->red, npq, sc(P, SC_PQ), P->active, part_rr,
                         HALF, &nrr, P->s));
  // (p.q, ||r||^2) to the pinned mirror; the host counts the publications
  return publish_red(part_rr, nrr, nb, sc(P, SC_RR), sc(P, SC_PQ), 2 * nb, P->hpub, P->dcount, P->hseq, P->s);
}

// Captures cg_body (on the fixed iterate buffer) as a graph, once per parity.
int cg_graph(sdg_problem* P, int parity, hipGraphExec_t* out) {
  if (P->cg_graph[parity]) {
    *out = P->cg_graph[parity];
    return SDG_OK;
  }
  if (!P->gs) SDG_HIP(hipStreamCreateWithFlags(&P->gs, hipStreamNonBlocking));
  double* rz = sc(P, SC_RZ);
  double* rz2 = sc(P, SC_RZ2);
  hipStream_t user = P->s;
  P->s = P->gs;
  hipGraph_t g = nullptr;
  int rc = SDG_OK;
  if (hipStreamBeginCapture(P->gs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = SDG_ERR_DEVICE;
  } else {
    rc = parity == 0 ? cg_body(P, P->cg_x, rz, rz2) : cg_body(P, P->cg_x, rz2, rz);
    if (hipStreamEndCapture(P->gs, &g) != hipSuccess && rc >= 0) rc = SDG_ERR_DEVICE;
  }
  P->s = user;
  if (rc >= 0 && hipGraphInstantiate(&P->cg_graph[parity], g, nullptr, nullptr, 0) != hipSuccess) {
    P->cg_graph[parity] = nullptr;
    rc = SDG_ERR_DEVICE;
  }
  if (g) (void)hipGraphDestroy(g);
  if (rc < 0) {
    (void)hipGetLastError();
    set_error("capture of the CG iteration as a HIP graph failed");
    return rc;
  }
  *out = P->cg_graph[parity];
  return SDG_OK;
}

// State of one batched CG solve, split so that several problems (of
// different shapes) can be advanced in lockstep: cg_start runs the first
// iteration up to the publication of its scalars; cg_poll waits for a
// publication and decides per problem (converged, breakdown, limit);
// cg_body_launch enqueues the next iteration (a graph replay, or eager
// launches while tracing); cg_finish drains the stream and copies the
// iterate out.  rtol_pb (optional): a tolerance per problem.
struct CgRun {
  sdg_problem* P = nullptr;
  const double* b = nullptr;
  double* x_out = nullptr;
  double* x = nullptr;
  double rtol = 0;
  int maxit = 0;
  const std::vector<double>* rtol_pb = nullptr;
  bool graphs = false;
  std::vector<int> its, status, act;
  std::vector<double> rel, bn;
  int nact = 0, it = 0, parity = 0;
  unsigned expect = 0;
  bool running = false;  // an iteration is queued whose scalars are not yet read
  bool combine = false;  // iterations go through the context's combiner (serving)
};
// the context's combiner (defined below)
int comb_submit(sdg_ctx* c, CgRun& R);
void comb_enter(sdg_ctx* c);
void comb_leave(sdg_ctx* c);

int cg_start(CgRun& R, sdg_problem* P, const double* b, double* x_out, double rtol, int maxit,
             const std::vector<double>* rtol_pb) {
  R.P = P;
  R.b = b;
  R.x_out = x_out;
  R.rtol = rtol;
  R.maxit = maxit;
  R.rtol_pb = rtol_pb;
  const int nb = P->nb;
  const int64_t n = P->nu;
  const VSpec S = viscous_spec(P);
  // replayed iterations work on a fixed iterate buffer (graph arguments)
  R.graphs = P->opt.graphs && !P->ctx->trace;
  R.x = R.graphs ? P->cg_x : x_out;
  SDG_TRY(vs_norms(P, S, b, R.bn));  // synchronises the stream
  P->seq = *const_cast<volatile unsigned*>(P->hseq);  // the device's count of publications so far
  SDG_HIP(hipMemsetAsync(R.x, 0, S.total * sizeof(double), P->s));
  R.its.assign(nb, 0);
  R.rel.assign(nb, 0.0);
  R.status.assign(nb, SDG_OK);
  R.act.assign(nb, 0);
  R.nact = 0;
  R.it = 0;
  R.parity = 0;
  R.running = false;
  for (int pb = 0; pb < nb; ++pb) {
    if (!std::isfinite(R.bn[pb])) {
      R.status[pb] = SDG_BREAKDOWN;
      R.rel[pb] = NAN;
    } else if (R.bn[pb] > 0.0) {
      R.act[pb] = 1;
      R.rel[pb] = 1.0;
      R.status[pb] = SDG_NOT_CONVERGED;
      ++R.nact;
    }
  }
  if (R.nact == 0) return SDG_OK;
  SDG_TRY(upload_active(P, R.act));
  SDG_TRY(vec_copy(S.total, b, P->cg_r, P->s));
  SDG_TRY(vcycle(P, P->cg_r, P->cg_z));
  SDG_TRY(vec_copy(S.total, P->cg_z, P->cg_p, P->s));
  double* rz = sc(P, SC_RZ);
  SDG_TRY(bmulti_dot(n, nb, 1, P->cg_r, 0, P->cg_z, rz, P->red, P->s));
  // first iteration: q = A p, p.q, update, readback
  SDG_TRY(run_sip_apply_dot(P, P->cg_p, P->cg_q, sc(P, SC_PQ)));
  SDG_TRY(cg_update1(n, nb, P->cg_p, P->cg_q, R.x, P->cg_r, rz, sc(P, SC_PQ), P->active, sc(P, SC_RR), P->red,
                     P->s));
  SDG_TRY(publish(P, sc(P, SC_PQ), 2 * nb, &R.expect));
  R.running = true;
  return SDG_OK;
}

// Reads the queued iteration's scalars; *more: the solve needs another
// iteration (the active flags on the device are refreshed if they changed).
int cg_poll(CgRun& R, bool* more) {
  *more = false;
  if (!R.running) return SDG_OK;
  sdg_problem* P = R.P;
  const int nb = P->nb;
  std::vector<double> both(2 * (size_t)nb);
  SDG_TRY(wait_published(P, R.expect, 2 * nb, both.data()));
  R.running = false;
  bool changed = false;
  for (int pb = 0; pb < nb; ++pb) {
    if (!R.act[pb]) continue;
    const double pq = both[pb], rr = both[nb + pb];
    if (!(pq > 0.0) || !std::isfinite(pq)) {
      R.status[pb] = SDG_BREAKDOWN;
      R.act[pb] = 0;
      --R.nact;
      changed = true;
      continue;
    }
    ++R.its[pb];
    R.rel[pb] = std::sqrt(rr > 0 ? rr : 0.0) / R.bn[pb];
    if (!std::isfinite(R.rel[pb])) {
      R.status[pb] = SDG_BREAKDOWN;
      R.act[pb] = 0;
      --R.nact;
      changed = true;
    } else if (R.rel[pb] < (R.rtol_pb ? (*R.rtol_pb)[pb] : R.rtol)) {
      R.status[pb] = SDG_OK;
      R.act[pb] = 0;
      --R.nact;
      changed = true;
    }
  }
  ++R.it;
  if (R.nact == 0 || R.it >= R.maxit) return SDG_OK;
  if (changed) SDG_TRY(upload_active(P, R.act));
  *more = true;
  return SDG_OK;
}

// the next iteration on the problem's stream (graph or eager); a caller that
// launched it inside a combined graph passes launched = true
int cg_body_launch(CgRun& R, bool launched) {
  sdg_problem* P = R.P;
  double* rz = sc(P, SC_RZ);
  double* rz2 = sc(P, SC_RZ2);
  if (!launched) {
    if (R.graphs && P->ctx->comb && R.combine) {
      SDG_TRY(comb_submit(P->ctx, R));
    } else if (R.graphs) {
      hipGraphExec_t ge = nullptr;
      SDG_TRY(cg_graph(P, R.parity, &ge));
      SDG_HIP(hipGraphLaunch(ge, P->s));
    } else {
      SDG_TRY(R.parity == 0 ? cg_body(P, R.x, rz, rz2) : cg_body(P, R.x, rz2, rz));
    }
  }
  R.expect = ++P->seq;  // the iteration ends with one publication
  R.parity ^= 1;
  R.running = true;
  return SDG_OK;
}

int cg_finish(CgRun& R) {
  sdg_problem* P = R.P;
  SDG_HIP(hipStreamSynchronize(P->s));
  if (R.graphs) SDG_TRY(vec_copy(P->nu * P->nb, R.x, R.x_out, P->s));
  return SDG_OK;
}

int cg_solve(sdg_problem* P, const double* b, double* x_out, double rtol, int maxit, std::vector<int>& its,
             std::vector<double>& rel, std::vector<int>& status, const std::vector<double>* rtol_pb = nullptr) {
  CgRun R;
  SDG_TRY(cg_start(R, P, b, x_out, rtol, maxit, rtol_pb));
  R.combine = R.graphs && P->ctx->comb != nullptr;
  if (R.combine) comb_enter(P->ctx);
  int rc = SDG_OK;
  while (true) {
    bool more = false;
    if ((rc = cg_poll(R, &more)) < 0 || !more) break;
    if ((rc = cg_body_launch(R, false)) < 0) break;
  }
  if (R.combine) comb_leave(P->ctx);
  SDG_TRY(rc);
  SDG_TRY(cg_finish(R));
  its = R.its;
  rel = R.rel;
  status = R.status;
  return SDG_OK;
}

// Several batched CG solves (problems of different meshes and orders, all
// on one stream) advanced in lockstep.  With graphs, one iteration of every
// running solve is a single replay of a combined HIP graph: a fork from a
// private capture stream, one parallel branch per solve (its V-cycle,
// updates, operator apply and the publication of its scalars) and a join,
// so that a single launch covers every shape and the solves overlap on the
// device.  The combined graph is captured once per set of running solves
// and parity and reused; a solve that has converged leaves the set.  With a
// single solve the problem's own captured iteration is replayed.
// The cache holds at most MAX_CACHED graphs: the set of running solves and
// their parities changes as solves start, finish and (in the server) miss
// a launch window, and every new combination is a new graph.  A full cache
// is emptied after the streams its graphs were launched on have drained.
struct MultiGraphs {
  static constexpr size_t MAX_CACHED = 64;
  hipStream_t cs = nullptr;
  std::vector<hipEvent_t> ev;
  std::map<std::string, hipGraphExec_t> cache;
  std::vector<hipStream_t> launched_on;  // streams the cached graphs were launched on
  int64_t built = 0;                     // graphs instantiated so far
  ~MultiGraphs() {
    for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (cs) (void)hipStreamDestroy(cs);
  }
  void note_launch(hipStream_t s) {
    if (std::find(launched_on.begin(), launched_on.end(), s) == launched_on.end()) launched_on.push_back(s);
  }
  int flush() {
    for (hipStream_t s : launched_on) SDG_HIP(hipStreamSynchronize(s));
    for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
    cache.clear();
    launched_on.clear();
    return SDG_OK;
  }
};

// The graph for one iteration of the solves A (with their parities); the
// caller launches it on a stream it passes to note_launch.
int multi_graph(MultiGraphs& G, std::vector<CgRun*>& A, hipGraphExec_t* out) {
  std::string key;
  for (CgRun* r : A) key += std::to_string((uintptr_t)r->P) + ":" + std::to_string(r->parity) + ";";
  auto it = G.cache.find(key);
  if (it != G.cache.end()) {
    *out = it->second;
    return SDG_OK;
  }
  if (G.cache.size() >= MultiGraphs::MAX_CACHED) SDG_TRY(G.flush());
  if (!G.cs) SDG_HIP(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
  while (G.ev.size() < A.size() + 1) {
    hipEvent_t e;
    SDG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    G.ev.push_back(e);
  }
  for (CgRun* r : A)
    if (!r->P->gs) SDG_HIP(hipStreamCreateWithFlags(&r->P->gs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  int rc = SDG_OK;
  if (hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = SDG_ERR_DEVICE;
  } else {
    if (hipEventRecord(G.ev[0], G.cs) != hipSuccess) rc = SDG_ERR_DEVICE;
    for (size_t i = 0; i < A.size() && rc >= 0; ++i) {
      sdg_problem* P = A[i]->P;
      if (hipStreamWaitEvent(P->gs, G.ev[0], 0) != hipSuccess) {
        rc = SDG_ERR_DEVICE;  // this branch was not forked: nothing to join
        break;
      }
      hipStream_t user = P->s;
      P->s = P->gs;
      double* rz = sc(P, SC_RZ);
      double* rz2 = sc(P, SC_RZ2);
      rc = A[i]->parity == 0 ? cg_body(P, A[i]->x, rz, rz2) : cg_body(P, A[i]->x, rz2, rz);
      P->s = user;
      // every forked branch joins the capture stream, also after a failure,
      // so that the capture can end with no stream left in it
      if (hipEventRecord(G.ev[i + 1], P->gs) != hipSuccess || hipStreamWaitEvent(G.cs, G.ev[i + 1], 0) != hipSuccess)
        rc = rc < 0 ? rc : SDG_ERR_DEVICE;
    }
    if (hipStreamEndCapture(G.cs, &g) != hipSuccess && rc >= 0) rc = SDG_ERR_DEVICE;
  }
  hipGraphExec_t ge = nullptr;
  if (rc >= 0 && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) rc = SDG_ERR_DEVICE;
  if (g) (void)hipGraphDestroy(g);
  if (rc < 0) {
    (void)hipGetLastError();
    set_error("capture of the combined CG iteration as a HIP graph failed");
    return rc;
  }
  G.cache[key] = ge;
  ++G.built;
  *out = ge;
  return SDG_OK;
}

// runs[i] already started (cg_start); advances all to completion.  A single
// solve on a context with a running request server goes through the
// server's combined launches.
int cg_multi(std::vector<CgRun>& runs, MultiGraphs& G) {
  const bool via_comb = runs.size() == 1 && runs[0].graphs && runs[0].P->ctx->comb;
  if (via_comb) {
    runs[0].combine = true;
    comb_enter(runs[0].P->ctx);
  }
  int rc = SDG_OK;
  while (rc >= 0) {
    std::vector<CgRun*> A;
    for (CgRun& r : runs) {
      bool more = false;
      if ((rc = cg_poll(r, &more)) < 0) break;
      if (more) A.push_back(&r);
    }
    if (rc < 0 || A.empty()) break;
    const bool combined = A.size() > 1 && A[0]->graphs;
    if (combined) {
      hipGraphExec_t ge = nullptr;
      if ((rc = multi_graph(G, A, &ge)) < 0) break;
      G.note_launch(A[0]->P->s);
      if (hipGraphLaunch(ge, A[0]->P->s) != hipSuccess) {
        set_error("hipGraphLaunch of the combined CG iteration failed");
        rc = SDG_ERR_DEVICE;
        break;
      }
    }
    for (CgRun* r : A)
      if ((rc = cg_body_launch(*r, combined)) < 0) break;
  }
  if (via_comb) comb_leave(runs[0].P->ctx);
  SDG_TRY(rc);
  for (CgRun& r : runs) SDG_TRY(cg_finish(r));
  return SDG_OK;
}

}  // namespace

// Continuous batching at the iteration level.  While a request server runs,
// every CG solve of the context (one per server slot, each on its own host
// thread and stream) hands its next iteration to the context's combiner
// instead of launching it: the first thread to arrive waits a short window
// for the other slots that are inside a CG solve, then launches one combined
// graph (one parallel branch per waiting solve, with event dependencies on
// every slot's stream) and releases them.  A request admitted into a free
// slot thus joins the running launches at its first iteration boundary, and
// the iterations of requests of different shapes overlap on the device in
// one launch.  The combined graphs are cached per set of solves and
// parities and dropped with their problems.
struct SdgCombiner {
  std::mutex mu;
  std::condition_variable cv;
  int members = 0;  // CG solves in progress
  struct Entry {
    CgRun* R;
    bool launched = false;
    int rc = 0;
  };
  std::vector<Entry*> pending;
  bool leader = false;
  MultiGraphs G;
  hipStream_t ls = nullptr;
  std::vector<hipEvent_t> ev;
  hipEvent_t done = nullptr;
  int64_t launches = 0, combined = 0;
  int max_width = 0;
  ~SdgCombiner() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (done) (void)hipEventDestroy(done);
    if (ls) (void)hipStreamDestroy(ls);
  }
};

namespace {

constexpr auto COMBINE_WINDOW = std::chrono::microseconds(150);

void comb_enter(sdg_ctx* c) {
  SdgCombiner* C = c->comb;
  std::lock_guard<std::mutex> g(C->mu);
  ++C->members;
}
void comb_leave(sdg_ctx* c) {
  SdgCombiner* C = c->comb;
  {
    std::lock_guard<std::mutex> g(C->mu);
    --C->members;
  }
  C->cv.notify_all();
}

// the launch of one set of iterations (caller holds C->mu; the owners of
// these solves wait in comb_submit, so their problems may be used here)
int comb_launch(SdgCombiner* C, std::vector<CgRun*>& A) {
  std::sort(A.begin(), A.end(), [](CgRun* a, CgRun* b) { return (uintptr_t)a->P < (uintptr_t)b->P; });
  ++C->launches;
  C->max_width = std::max(C->max_width, (int)A.size());
  if (A.size() == 1) {
    hipGraphExec_t ge = nullptr;
    SDG_TRY(cg_graph(A[0]->P, A[0]->parity, &ge));
    SDG_HIP(hipGraphLaunch(ge, A[0]->P->s));
    return SDG_OK;
  }
  ++C->combined;
  if (!C->ls) SDG_HIP(hipStreamCreateWithFlags(&C->ls, hipStreamNonBlocking));
  hipGraphExec_t ge = nullptr;
  SDG_TRY(multi_graph(C->G, A, &ge));
  C->G.note_launch(C->ls);
  if (!C->done) SDG_HIP(hipEventCreateWithFlags(&C->done, hipEventDisableTiming));
  while (C->ev.size() < A.size()) {
    hipEvent_t e;
    SDG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    C->ev.push_back(e);
  }
  for (size_t i = 0; i < A.size(); ++i) {
    SDG_HIP(hipEventRecord(C->ev[i], A[i]->P->s));
    SDG_HIP(hipStreamWaitEvent(C->ls, C->ev[i], 0));
  }
  SDG_HIP(hipGraphLaunch(ge, C->ls));
  SDG_HIP(hipEventRecord(C->done, C->ls));
  for (CgRun* r : A) SDG_HIP(hipStreamWaitEvent(r->P->s, C->done, 0));
  return SDG_OK;
}

int comb_submit(sdg_ctx* c, CgRun& R) {
  SdgCombiner* C = c->comb;
  std::unique_lock<std::mutex> lk(C->mu);
  SdgCombiner::Entry e{&R};
  C->pending.push_back(&e);
  C->cv.notify_all();
  while (!e.launched) {
    if (!C->leader) {
      C->leader = true;
      C->cv.wait_for(lk, COMBINE_WINDOW, [&] { return (int)C->pending.size() >= C->members; });
      std::vector<SdgCombiner::Entry*> take;
      take.swap(C->pending);
      std::vector<CgRun*> A;
      for (auto* x : take) A.push_back(x->R);
      const int rc = comb_launch(C, A);
      for (auto* x : take) {
        x->launched = true;
        x->rc = rc;
      }
      C->leader = false;
      C->cv.notify_all();
    } else {
      C->cv.wait(lk);
    }
  }
  return e.rc;
}

// drop cached combined graphs that contain problem P (it is being destroyed)
void comb_drop(sdg_ctx* c, const sdg_problem* P) {
  SdgCombiner* C = c->comb;
  if (!C) return;
  std::lock_guard<std::mutex> g(C->mu);
  // keys are "P:parity;" tokens: match P at the start or after a separator
  const std::string tag = std::to_string((uintptr_t)P) + ":";
  for (auto it = C->G.cache.begin(); it != C->G.cache.end();) {
    if (it->first.compare(0, tag.size(), tag) == 0 || it->first.find(";" + tag) != std::string::npos) {
      (void)hipGraphExecDestroy(it->second);
      it = C->G.cache.erase(it);
    } else {
      ++it;
    }
  }
}

// Viscous solves by CG with iterative refinement in extended precision
// (opts.refine with viscous_krylov = 0), for one or several batched
// problems (in lockstep, see cg_multi): the iterate is the double-FP64 pair
// (xh, xl); each step solves A d = r by CG in FP64 to a tolerance relative
// to its right-hand side chosen so that the step reaches rtol (at most 1e-6
// per step, where FP64 CG stays far from its own floor), adds d in
// double-FP64 and forms the true residual r = F - A (xh + xl) in extended
// precision.  Converged problems get a zero right-hand side and stay put.
// its[pb] counts CG iterations over all steps.
struct RefineState {
  sdg_problem* P = nullptr;
  const double* F = nullptr;
  double *xh = nullptr, *xl = nullptr, *r = nullptr, *d = nullptr;
  std::vector<double> bn, tol;
  std::vector<char> act;
  std::vector<double> prev;
  std::vector<int> gaps;
  std::vector<int> its, status;
  std::vector<double> rel;
};

int cg_refine_multi(std::vector<RefineState>& G, double rtol, int maxit, MultiGraphs& MG) {
  int rc = SDG_OK;
  for (RefineState& R : G) {
    sdg_problem* P = R.P;
    const int nb = P->nb;
    const VSpec S = viscous_spec(P);
    if (tmp_get(P, &R.r, S.total) < 0 || tmp_get(P, &R.d, S.total) < 0) {
      set_error("allocation of the refinement vectors failed");
      rc = SDG_ERR_NOMEM;
      break;
    }
    R.its.assign(nb, 0);
    R.rel.assign(nb, 1.0);
    R.status.assign(nb, SDG_NOT_CONVERGED);
    R.act.assign(nb, 1);
    R.prev.assign(nb, 1.0);
    R.gaps.assign(nb, 0);
    if ((rc = vs_norms(P, S, R.F, R.bn)) < 0) break;
    if (hipMemsetAsync(R.xh, 0, S.total * sizeof(double), P->s) != hipSuccess ||
        hipMemsetAsync(R.xl, 0, S.total * sizeof(double), P->s) != hipSuccess) {
      rc = SDG_ERR_DEVICE;
      break;
    }
    if ((rc = vec_copy(S.total, R.F, R.r, P->s)) < 0) break;
  }
  for (int step = 0; step < 64 && rc >= 0; ++step) {
    std::vector<CgRun> runs;
    std::vector<RefineState*> stepping;
    runs.reserve(G.size());
    for (RefineState& R : G) {
      sdg_problem* P = R.P;
      const int nb = P->nb;
      const VSpec S = viscous_spec(P);
      std::vector<double> rn;
      if ((rc = vs_norms(P, S, R.r, rn)) < 0) break;
      std::vector<char> stag(nb, 0);
      bool any_stag = false;
      int used = 0;
      for (int pb = 0; pb < nb; ++pb) {
        used = std::max(used, R.its[pb]);
        if (!R.act[pb]) continue;
        if (!(R.bn[pb] > 0.0)) {
          R.rel[pb] = std::isfinite(R.bn[pb]) ? 0.0 : NAN;
          R.status[pb] = std::isfinite(R.bn[pb]) ? SDG_OK : SDG_BREAKDOWN;
          R.act[pb] = 0;
          continue;
        }
        R.rel[pb] = rn[pb] / R.bn[pb];
        if (!std::isfinite(R.rel[pb])) {
          R.status[pb] = SDG_BREAKDOWN;
          R.act[pb] = 0;
        } else if (R.rel[pb] < rtol) {
          R.status[pb] = SDG_OK;
          R.act[pb] = 0;
        } else if (step > 0) {
          R.gaps[pb] = R.rel[pb] > 0.5 * R.prev[pb] ? R.gaps[pb] + 1 : 0;
          if (R.gaps[pb] >= 2) {
            stag[pb] = 1;
            any_stag = true;
          } else if (R.its[pb] >= maxit) {
            R.act[pb] = 0;  // NOT_CONVERGED
          }
        }
        R.prev[pb] = R.rel[pb];
      }
      if (any_stag) {
        std::vector<double> kx;
        if ((rc = run_ext(P, false, true, nullptr, R.xh, nullptr, R.d)) < 0) break;
        if ((rc = vs_norms(P, S, R.d, kx)) < 0) break;
        for (int pb = 0; pb < nb; ++pb)
          if (stag[pb]) {
            R.status[pb] = R.rel[pb] <= 4.0 * resid_eps(P) * kx[pb] / R.bn[pb] ? SDG_FLOOR : SDG_NOT_CONVERGED;
            R.act[pb] = 0;
          }
      }
      int nact = 0;
      std::vector<double> keep(nb, 0.0);
      R.tol.assign(nb, 0.5);
      for (int pb = 0; pb < nb; ++pb) {
        if (!R.act[pb]) continue;
        ++nact;
        keep[pb] = 1.0;
        R.tol[pb] = std::min(0.5, std::max(1e-6, 0.5 * rtol * R.bn[pb] / rn[pb]));
      }
      if (nact == 0 || used >= maxit) continue;
      // converged problems: zero right-hand side (the CG leaves them at 0)
      if ((rc = upload_scalars(P, sc(P, SC_BN), keep)) < 0) break;
      if ((rc = vs_div(P, S, sc(P, SC_BN), R.r, R.r)) < 0) break;
      runs.emplace_back();
      if ((rc = cg_start(runs.back(), P, R.r, R.d, rtol, maxit - used, &R.tol)) < 0) break;
      stepping.push_back(&R);
    }
    if (rc < 0 || runs.empty()) break;
    if ((rc = cg_multi(runs, MG)) < 0) break;
    for (size_t i = 0; i < runs.size() && rc >= 0; ++i) {
      RefineState& R = *stepping[i];
      sdg_problem* P = R.P;
      for (int pb = 0; pb < P->nb; ++pb) {
        if (!R.act[pb]) continue;
        R.its[pb] += runs[i].its[pb];
        if (runs[i].status[pb] == SDG_BREAKDOWN) {
          R.status[pb] = SDG_BREAKDOWN;
          R.act[pb] = 0;
        }
      }
      const int64_t tot = P->nu * P->nb;
      if ((rc = dd_accumulate(tot, R.d, R.xh, R.xl, P->s)) < 0) break;
      if ((rc = run_ext(P, false, false, R.F, R.xh, R.xl, R.r)) < 0) break;
    }
  }
  for (RefineState& R : G) {
    const int64_t tot = R.P->nu * R.P->nb;
    tmp_put(R.P, R.r, tot);  // synchronises the stream first
    tmp_put(R.P, R.d, tot);
    R.r = R.d = nullptr;
  }
  return rc;
}

int cg_refine(sdg_problem* P, const double* F, double* xh, double* xl, double rtol, int maxit,
              std::vector<int>& its, std::vector<double>& rel, std::vector<int>& status) {
  std::vector<RefineState> G(1);
  G[0].P = P;
  G[0].F = F;
  G[0].xh = xh;
  G[0].xl = xl;
  MultiGraphs MG;
  SDG_TRY(cg_refine_multi(G, rtol, maxit, MG));
  its = G[0].its;
  rel = G[0].rel;
  status = G[0].status;
  return SDG_OK;
}

int ensure_gmres(sdg_problem* P, int64_t n_per_problem) {
  if (P->gV && P->gn == n_per_problem) return SDG_OK;
  if (P->gV) {
    set_error("FGMRES workspace was sized for the other system (viscous vs Stokes)");
    return SDG_ERR_INVALID;
  }
  const int m = P->opt.restart;
  const int64_t tot = n_per_problem * P->nb;
  SDG_TRY(palloc_t(P, &P->gV, (int64_t)(m + 1) * tot));
  SDG_TRY(palloc_t(P, &P->gZ, (int64_t)m * tot));
  SDG_TRY(palloc_t(P, &P->gw, tot));
  SDG_TRY(palloc_t(P, &P->gt, P->nu * P->nb));
  // two passes of m + 1 coefficients, the masked norm, and the per-segment
  // partials (two segments of m + 1 values)
  SDG_TRY(palloc_t(P, &P->gcoef, (int64_t)(4 * (m + 1) + 4) * P->nb));
  SDG_TRY(palloc_t(P, &P->gdone, P->nb));
  P->gn = n_per_problem;
  return SDG_OK;
}

// dst[pb][i] = V_i . w per problem for i < mj, on the device, summed over
// the segments of S in order (segb: scratch of S.nseg * nb * mj values)
int vs_dots_dev(sdg_problem* P, const VSpec& S, int mj, const double* V, int64_t ldv, const double* w,
                double* dst, double* segb) {
  const int nb = P->nb;
  if (S.nseg == 1)
    return bmulti_dot(S.seg[0].n, nb, mj, V + S.seg[0].off, ldv, w + S.seg[0].off, dst, P->red, P->s);
  for (int q = 0; q < S.nseg; ++q)
    SDG_TRY(bmulti_dot(S.seg[q].n, nb, mj, V + S.seg[q].off, ldv, w + S.seg[q].off,
                       segb + (int64_t)q * nb * mj, P->red, P->s));
  return seg_sum((int64_t)nb * mj, S.nseg, segb, dst, P->s);
}

// Batched right-preconditioned FGMRES(restart), classical Gram-Schmidt
// applied twice, x0 = 0; each problem stops on its own true residual.
//
// Each restart is a step of iterative refinement: the cycle solves for a
// correction from the current true residual.  resid(x, xlo, w) forms that
// residual, w = b - K x; with xlo != nullptr (opts.refine) the iterate is
// the double-FP64 pair (x, xlo), the correction is accumulated into it in
// double-FP64 and resid evaluates the residual in extended precision, so
// the restarts drive the residual below the FP64 floor.  abs_apply(x, y)
// forms y = |K||x| for the floor estimate of a stagnating problem.
template <typename MV, typename PC, typename PJ, typename RS, typename AB>
int fgmres(sdg_problem* P, const VSpec& S, const double* b_in, double* x, double* xlo, double rtol, int maxit,
           MV matvec, PC prec, PJ project, RS resid, AB abs_apply, std::vector<int>& its, std::vector<double>& rel,
           std::vector<int>& status) {
  const int m = P->opt.restart, nb = P->nb;
  SDG_TRY(ensure_gmres(P, S.total / nb));
  double* V = P->gV;
  double* Z = P->gZ;
  double* w = P->gw;
  const int64_t ldv = S.total;
  SDG_TRY(vec_copy(S.total, b_in, w, P->s));
  SDG_TRY(project(w));
  std::vector<double> bn, beta;
  SDG_TRY(vs_norms(P, S, w, bn));
  SDG_HIP(hipMemsetAsync(x, 0, S.total * sizeof(double), P->s));
  if (xlo) SDG_HIP(hipMemsetAsync(xlo, 0, S.total * sizeof(double), P->s));
  its.assign(nb, 0);
  rel.assign(nb, 0.0);
  status.assign(nb, SDG_OK);
  std::vector<char> act(nb, 0);
  for (int pb = 0; pb < nb; ++pb) {
    if (!std::isfinite(bn[pb])) {
      status[pb] = SDG_BREAKDOWN;
    } else if (bn[pb] > 0.0) {
      act[pb] = 1;
      rel[pb] = 1.0;
      status[pb] = SDG_NOT_CONVERGED;
    }
  }
  beta = bn;
  std::vector<double> H((size_t)nb * (m + 1) * m), cs((size_t)nb * m), sn((size_t)nb * m);
  std::vector<double> g((size_t)nb * (m + 1)), y((size_t)nb * m);
  std::vector<int> jd(nb), gaps(nb, 0);
  std::vector<char> done(nb), est_conv(nb);
  std::vector<double> prev_rel(nb, 1.0);
  int total = 0;
  while (true) {
    bool any = false;
    for (int pb = 0; pb < nb; ++pb) any = any || act[pb];
    if (!any || total >= maxit) break;
    std::vector<double> bsc(nb);
    for (int pb = 0; pb < nb; ++pb) bsc[pb] = act[pb] ? beta[pb] : 0.0;
    SDG_TRY(upload_scalars(P, sc(P, SC_BN), bsc));
    SDG_TRY(vs_div(P, S, sc(P, SC_BN), w, V));
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int pb = 0; pb < nb; ++pb) {
      g[(size_t)pb * (m + 1)] = beta[pb];
      jd[pb] = 0;
      done[pb] = !act[pb];
      est_conv[pb] = 0;
    }
    bool done_changed = true;  // the device copy of `done` is refreshed before use
    for (int j = 0; j < m; ++j) {
      double* zj = Z + (int64_t)j * ldv;
      SDG_TRY(prec(V + (int64_t)j * ldv, zj));
      SDG_TRY(project(zj));
      SDG_TRY(matvec(zj, w));
      // classical Gram-Schmidt twice and the new vector's norm, with the
      // coefficients kept on the device: hbuf = [pass 0 | pass 1 | norms],
      // read back once per iteration
      const int mj = j + 1;
      double* hbuf = P->gcoef;
      double* segb = P->gcoef + (int64_t)(2 * (m + 1) + 2) * nb;
      for (int pass = 0; pass < 2; ++pass) {
        double* hp = hbuf + (int64_t)pass * nb * mj;
        SDG_TRY(vs_dots_dev(P, S, mj, V, ldv, w, hp, segb));
        SDG_TRY(vs_axpy(P, S, mj, V, ldv, hp, w));
      }
      double* hsq = hbuf + (int64_t)(2 * (m + 1) + 1) * nb;  // w.w per problem
      double* hs_dev = hbuf + (int64_t)2 * nb * mj;
      if (done_changed) {
        std::vector<int> di(nb);
        for (int pb = 0; pb < nb; ++pb) di[pb] = done[pb] ? 1 : 0;
        SDG_TRY(to_dev_async(P, P->gdone, di.data(), nb * sizeof(int)));
        done_changed = false;
      }
      SDG_TRY(vs_dots_dev(P, S, 1, w, 0, w, hsq, segb));
      SDG_TRY(norm_mask(nb, hsq, P->gdone, hs_dev, P->s));
      SDG_TRY(vs_div(P, S, hs_dev, w, V + (int64_t)(j + 1) * ldv));
      std::vector<double> hb((size_t)2 * nb * mj + nb);
      SDG_TRY(read_dev(P, hbuf, (int)hb.size(), hb.data()));
      std::vector<double> h((size_t)nb * mj), hn(nb);
      for (size_t i = 0; i < h.size(); ++i) h[i] = (0.0 + hb[i]) + hb[(size_t)nb * mj + i];
      for (int pb = 0; pb < nb; ++pb) hn[pb] = hb[(size_t)2 * nb * mj + pb];
      bool all_done = true;
      for (int pb = 0; pb < nb; ++pb) {
        if (done[pb]) continue;
        double* col = H.data() + ((size_t)pb * m + j) * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = h[(size_t)pb * (j + 1) + i];
        col[j + 1] = hn[pb];
        double* c = cs.data() + (size_t)pb * m;
        double* s_ = sn.data() + (size_t)pb * m;
        double* gg = g.data() + (size_t)pb * (m + 1);
        for (int i = 0; i < j; ++i) {
          const double t = c[i] * col[i] + s_[i] * col[i + 1];
          col[i + 1] = -s_[i] * col[i] + c[i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        if (!(den > 0.0) || !std::isfinite(den)) {
          status[pb] = SDG_BREAKDOWN;
          act[pb] = 0;
          done[pb] = 1;
          done_changed = true;
          continue;
        }
        c[j] = col[j] / den;
        s_[j] = col[j + 1] / den;
        col[j] = den;
        col[j + 1] = 0.0;
        gg[j + 1] = -s_[j] * gg[j];
        gg[j] = c[j] * gg[j];
        ++its[pb];
        jd[pb] = j + 1;
        const double est = std::fabs(gg[j + 1]) / bn[pb];
        if (est < rtol) est_conv[pb] = 1;
        if (est < rtol || hn[pb] == 0.0 || its[pb] >= maxit) {
          done[pb] = 1;
          done_changed = true;
        }
        all_done = all_done && done[pb];
      }
      ++total;
      if (all_done || total >= maxit) break;
    }
    // y = H^{-1} g per problem, x += Z y
    std::fill(y.begin(), y.end(), 0.0);
    int jmax = 0;
    for (int pb = 0; pb < nb; ++pb) {
      const int jj = jd[pb];
      jmax = std::max(jmax, jj);
      const double* Hp = H.data() + (size_t)pb * m * (m + 1);
      const double* gg = g.data() + (size_t)pb * (m + 1);
      double* yy = y.data() + (size_t)pb * m;
      for (int i = jj - 1; i >= 0; --i) {
        double s = gg[i];
        for (int l = i + 1; l < jj; ++l) s -= Hp[(size_t)l * (m + 1) + i] * yy[l];
        yy[i] = s / Hp[(size_t)i * (m + 1) + i];
      }
    }
    if (jmax > 0) {
      std::vector<double> yc((size_t)nb * jmax);
      for (int pb = 0; pb < nb; ++pb)
        for (int i = 0; i < jmax; ++i) yc[(size_t)pb * jmax + i] = y[(size_t)pb * m + i];
      SDG_TRY(upload_scalars(P, sc_h(P), yc));
      if (xlo) {
        // the correction Z y, accumulated into the double-FP64 iterate
        SDG_HIP(hipMemsetAsync(w, 0, S.total * sizeof(double), P->s));
        SDG_TRY(vs_combine(P, S, jmax, Z, ldv, sc_h(P), w));
        SDG_TRY(dd_accumulate(S.total, w, x, xlo, P->s));
      } else {
        SDG_TRY(vs_combine(P, S, jmax, Z, ldv, sc_h(P), x));
      }
    }
    // true residual (the next cycle's right-hand side)
    SDG_TRY(resid(x, xlo, w));
    SDG_TRY(project(w));
    SDG_TRY(vs_norms(P, S, w, beta));
    std::vector<char> stag(nb, 0);
    bool any_stag = false;
    for (int pb = 0; pb < nb; ++pb) {
      if (bn[pb] > 0.0 && std::isfinite(bn[pb])) rel[pb] = beta[pb] / bn[pb];
      if (!act[pb]) continue;
      if (rel[pb] < rtol) {
        status[pb] = SDG_OK;
        act[pb] = 0;
        continue;
      }
      // stagnation: the Arnoldi estimate fell below rtol but the true
      // residual did not follow, twice without halving
      if (est_conv[pb] && rel[pb] > 0.5 * prev_rel[pb]) ++gaps[pb];
      else gaps[pb] = 0;
      prev_rel[pb] = rel[pb];
      if (gaps[pb] >= 2) {
        stag[pb] = 1;
        any_stag = true;
      } else if (its[pb] >= maxit) {
        status[pb] = SDG_NOT_CONVERGED;
        act[pb] = 0;
      }
    }
    if (any_stag) {
      // a stagnation is the rounding floor of the residual's evaluation only
      // if the residual lies within a small factor of eps |K||x| / |b|;
      // otherwise the iteration failed to converge.  Z is free between
      // cycles and holds |K||x|.
      std::vector<double> kx;
      SDG_TRY(abs_apply(x, Z));
      SDG_TRY(vs_norms(P, S, Z, kx));
      for (int pb = 0; pb < nb; ++pb) {
        if (!stag[pb]) continue;
        const double fl = resid_eps(P) * kx[pb] / bn[pb];
        status[pb] = rel[pb] <= 4.0 * fl ? SDG_FLOOR : SDG_NOT_CONVERGED;
        act[pb] = 0;
      }
    }
  }
  return SDG_OK;
}

// Batched GCR(m) with right preconditioning (the generalised conjugate
// residual method; flexible, so the preconditioner may change between
// iterations), x0 = 0.  Iteration j: p = M^{-1} r, q = K p, q and p
// orthogonalised against the earlier q (classical Gram-Schmidt twice, the
// same coefficients applied to p), normalised by |q|, then alpha = r.q,
// x += alpha p, r -= alpha q: |r| is the exact residual norm of the
// iteration in exact arithmetic and is read back once per iteration.  A
// problem whose |r| falls below rtol |b| stops (its q and p are masked to
// zero from then on).  After m iterations, or when every problem stopped,
// the cycle's correction is added to the iterate and the true residual is
// formed by resid(x, xlo, r) (extended precision with xlo, as in fgmres):
// restarts are steps of iterative refinement, and the stagnation and
// floor logic is that of fgmres.  The paper runs GCR for both loops of its
// six-inclusion experiment (Section 8.3).
template <typename MV, typename PC, typename PJ, typename RS, typename AB>
int gcr(sdg_problem* P, const VSpec& S, const GcrWork& W, const double* b_in, double* x, double* xlo, double rtol,
        int maxit, MV matvec, PC prec, PJ project, RS resid, AB abs_apply, std::vector<int>& its,
        std::vector<double>& rel, std::vector<int>& status) {
  const int m = W.m, nb = P->nb;
  const int64_t ldv = S.total;
  double* hsq = W.coef;
  double* hs = W.coef + nb;
  double* rr = W.coef + 2 * (int64_t)nb;
  double* alpha = W.coef + 3 * (int64_t)nb;
  double* gsc = W.coef + 4 * (int64_t)nb;                // [nb][m] Gram-Schmidt coefficients
  double* segb = W.coef + (4 + (int64_t)m) * nb;         // per-segment partials
  SDG_TRY(vec_copy(S.total, b_in, W.r, P->s));
  SDG_TRY(project(W.r));
  std::vector<double> bn;
  SDG_TRY(vs_norms(P, S, W.r, bn));
  SDG_HIP(hipMemsetAsync(x, 0, S.total * sizeof(double), P->s));
  if (xlo) SDG_HIP(hipMemsetAsync(xlo, 0, S.total * sizeof(double), P->s));
  its.assign(nb, 0);
  rel.assign(nb, 0.0);
  status.assign(nb, SDG_OK);
  std::vector<char> act(nb, 0);
  for (int pb = 0; pb < nb; ++pb) {
    if (!std::isfinite(bn[pb])) {
      status[pb] = SDG_BREAKDOWN;
    } else if (bn[pb] > 0.0) {
      act[pb] = 1;
      rel[pb] = 1.0;
      status[pb] = SDG_NOT_CONVERGED;
    }
  }
  std::vector<int> gaps(nb, 0);
  std::vector<double> prev_rel(nb, 1.0);
  std::vector<char> est_conv(nb, 0);
  int total = 0;
  while (true) {
    bool any = false;
    for (int pb = 0; pb < nb; ++pb) any = any || act[pb];
    if (!any || total >= maxit) break;
    // the correction of this cycle (x itself when not refining)
    double* xc = xlo ? W.c : x;
    if (xlo) SDG_HIP(hipMemsetAsync(W.c, 0, S.total * sizeof(double), P->s));
    std::vector<int> di(nb);
    for (int pb = 0; pb < nb; ++pb) {
      di[pb] = act[pb] ? 0 : 1;
      est_conv[pb] = 0;
    }
    SDG_TRY(to_dev_async(P, W.done, di.data(), nb * sizeof(int)));
    bool all_done = false;
    for (int j = 0; j < m && !all_done && total < maxit; ++j) {
      double* pj = W.Pd + (int64_t)j * ldv;
      double* qj = W.Q + (int64_t)j * ldv;
      SDG_TRY(prec(W.r, pj));
      SDG_TRY(project(pj));
      SDG_TRY(matvec(pj, qj));
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        SDG_TRY(vs_dots_dev(P, S, j, W.Q, ldv, qj, gsc, segb));
        SDG_TRY(vs_axpy(P, S, j, W.Q, ldv, gsc, qj));
        SDG_TRY(vs_axpy(P, S, j, W.Pd, ldv, gsc, pj));
      }
      // |q| (zero for problems that stopped: their q and p become zero, so
      // their alpha is zero and x, r stay put)
      SDG_TRY(vs_dots_dev(P, S, 1, qj, 0, qj, hsq, segb));
      SDG_TRY(norm_mask(nb, hsq, W.done, hs, P->s));
      SDG_TRY(vs_div(P, S, hs, qj, qj));
      SDG_TRY(vs_div(P, S, hs, pj, pj));
      SDG_TRY(vs_dots_dev(P, S, 1, qj, 0, W.r, alpha, segb));
      SDG_TRY(vs_combine(P, S, 1, pj, 0, alpha, xc));
      SDG_TRY(vs_axpy(P, S, 1, qj, 0, alpha, W.r));
      SDG_TRY(vs_dots_dev(P, S, 1, W.r, 0, W.r, rr, segb));
      std::vector<double> hb(2 * (size_t)nb);
      SDG_TRY(read_dev(P, hs, nb, hb.data()));
      SDG_TRY(read_dev(P, rr, nb, hb.data() + nb));
      ++total;
      all_done = true;
      bool changed = false;
      for (int pb = 0; pb < nb; ++pb) {
        if (di[pb]) continue;
        ++its[pb];
        const double est = std::sqrt(std::max(hb[nb + pb], 0.0)) / bn[pb];
        if (!(hb[pb] > 0.0) || !std::isfinite(hb[pb]) || !std::isfinite(est)) {
          status[pb] = SDG_BREAKDOWN;
          act[pb] = 0;
          di[pb] = 1;
          changed = true;
          continue;
        }
        if (est < rtol) est_conv[pb] = 1;
        if (est < rtol || its[pb] >= maxit) {
          di[pb] = 1;
          changed = true;
        }
        all_done = all_done && di[pb];
      }
      if (changed) SDG_TRY(to_dev_async(P, W.done, di.data(), nb * sizeof(int)));
    }
    if (xlo) SDG_TRY(dd_accumulate(S.total, W.c, x, xlo, P->s));
    // true residual, the next cycle's start
    SDG_TRY(resid(x, xlo, W.r));
    SDG_TRY(project(W.r));
    std::vector<double> beta;
    SDG_TRY(vs_norms(P, S, W.r, beta));
    std::vector<char> stag(nb, 0);
    bool any_stag = false;
    for (int pb = 0; pb < nb; ++pb) {
      if (bn[pb] > 0.0 && std::isfinite(bn[pb])) rel[pb] = beta[pb] / bn[pb];
      if (!act[pb]) continue;
      if (rel[pb] < rtol) {
        status[pb] = SDG_OK;
        act[pb] = 0;
        continue;
      }
      if (est_conv[pb] && rel[pb] > 0.5 * prev_rel[pb]) ++gaps[pb];
      else gaps[pb] = 0;
      prev_rel[pb] = rel[pb];
      if (gaps[pb] >= 2) {
        stag[pb] = 1;
        any_stag = true;
      } else if (its[pb] >= maxit) {
        status[pb] = SDG_NOT_CONVERGED;
        act[pb] = 0;
      }
    }
    if (any_stag) {
      std::vector<double> kx;
      SDG_TRY(abs_apply(x, W.Q));
      SDG_TRY(vs_norms(P, S, W.Q, kx));
      for (int pb = 0; pb < nb; ++pb) {
        if (!stag[pb]) continue;
        status[pb] = rel[pb] <= 4.0 * resid_eps(P) * kx[pb] / bn[pb] ? SDG_FLOOR : SDG_NOT_CONVERGED;
        act[pb] = 0;
      }
    }
  }
  return SDG_OK;
}

// GCR workspace of the inner viscous solve (separate from the outer
// solve's Krylov vectors, which are in use while the preconditioner runs)
int ensure_gcr_inner(sdg_problem* P) {
  if (P->gi.Q) return SDG_OK;
  const int m = P->opt.restart;
  const int64_t tot = P->nu * P->nb;
  GcrWork& W = P->gi;
  W.m = m;
  SDG_TRY(palloc_t(P, &W.Q, (int64_t)m * tot));
  SDG_TRY(palloc_t(P, &W.Pd, (int64_t)m * tot));
  SDG_TRY(palloc_t(P, &W.r, tot));
  SDG_TRY(palloc_t(P, &W.c, tot));
  SDG_TRY(palloc_t(P, &W.coef, (int64_t)(4 * (m + 1) + 4) * P->nb));
  SDG_TRY(palloc_t(P, &W.done, P->nb));
  return SDG_OK;
}
// the outer solve's GCR workspace lives in the FGMRES buffers
GcrWork outer_gcr_work(sdg_problem* P) {
  GcrWork W;
  W.m = P->opt.restart;
  const int64_t tot = P->gn * P->nb;
  W.Q = P->gV;
  W.r = P->gV + (int64_t)W.m * tot;
  W.Pd = P->gZ;
  W.c = P->gw;
  W.coef = P->gcoef;
  W.done = P->gdone;
  return W;
}

// Stokes operator K = [A B; B^T 0] on x = [u (all problems); p (all problems)]
int stokes_matvec(sdg_problem* P, const double* x, double* y) {
  const int64_t U = P->nu * P->nb;
  SDG_TRY(run_sip_apply(P, x, y));
  SDG_TRY(grad_apply(P->M, P->k, P->nb, x + U, P->gt, P->s));
  SDG_TRY(vec_axpy(U, 1.0, P->gt, y, P->s));
  SDG_TRY(div_apply(P->M, P->k, P->nb, x, y + U, P->s));
  return SDG_OK;
}

// upper block-triangular preconditioner [A B; 0 S] (eq. discretestokespc)
// with S = -diag(1/eta_K), the viscosity-scaled pressure mass matrix taken
// as an approximation of the (negative definite) Schur complement
// -B^T A^{-1} B:  z_p = S^{-1} v_p = -eta v_p, z_u = (inner CG)(v_u - B z_p)
int stokes_prec(sdg_problem* P, const double* v, double* z) {
  const int64_t U = P->nu * P->nb, Pn = P->np * P->nb;
  SDG_TRY(vec_mul(Pn, P->etap, v + U, z + U, P->s));
  SDG_TRY(vec_scale_copy(Pn, -1.0, z + U, z + U, P->s));
  SDG_TRY(grad_apply(P->M, P->k, P->nb, z + U, P->gt, P->s));
  SDG_TRY(vec_axpby(U, 1.0, v, -1.0, P->gt, P->s));
  std::vector<int> its, st;
  std::vector<double> rel;
  if (P->opt.viscous_krylov == 2) {
    // GCR for the inner solve (the paper's six-inclusion setting)
    SDG_TRY(ensure_gcr_inner(P));
    const VSpec S = viscous_spec(P);
    auto mv = [&](const double* xx, double* yy) { return run_sip_apply(P, xx, yy); };
    auto pc = [&](const double* vv, double* zz) { return vcycle(P, vv, zz); };
    auto pj = [&](double*) { return SDG_OK; };
    auto rs = [&](const double* xx, const double*, double* w) { return run_sip_residual(P, P->gt, xx, w); };
    auto ab = [&](const double* xx, double* yy) { return run_ext(P, false, true, nullptr, xx, nullptr, yy); };
    SDG_TRY(gcr(P, S, P->gi, P->gt, z, nullptr, P->opt.inner_rtol, P->opt.inner_max_it, mv, pc, pj, rs, ab, its,
                rel, st));
  } else {
    SDG_TRY(cg_solve(P, P->gt, z, P->opt.inner_rtol, P->opt.inner_max_it, its, rel, st));
  }
  for (int pb = 0; pb < P->nb; ++pb) {
    P->inner_total[pb] += its[pb];
    P->inner_max[pb] = std::max(P->inner_max[pb], its[pb]);
  }
  return SDG_OK;
}

int stokes_project(sdg_problem* P, double* x) {
  if (P->neumann || P->np == 0) return SDG_OK;
  return bpressure_project(P->nel, P->NPE, P->nb, P->np, x + P->nu * P->nb, P->red, P->s);
}

int fill_stats(sdg_problem* P, sdg_stats* st, const std::vector<int>& status, const std::vector<int>& its,
               const std::vector<double>& rel, double t0, bool stokes) {
  // aggregate outcome: breakdown > not converged > rounding floor > ok
  auto rank = [](int s) { return s == SDG_BREAKDOWN ? 3 : s == SDG_NOT_CONVERGED ? 2 : s == SDG_FLOOR ? 1 : 0; };
  int worst = SDG_OK;
  for (int pb = 0; pb < P->nb; ++pb) {
    if (rank(status[pb]) > rank(worst)) worst = status[pb];
    if (!st) continue;
    st[pb].status = status[pb];
    st[pb].outer_its = its[pb];
    st[pb].inner_its_total = stokes ? P->inner_total[pb] : 0;
    st[pb].inner_its_max = stokes ? P->inner_max[pb] : 0;
    st[pb].rel_residual = rel[pb];
    st[pb].setup_ms = P->setup_ms;
    st[pb].solve_ms = now_ms() - t0;
  }
  return worst;
}

}  // namespace

namespace sdg {
// Device bytes of a batched problem whose element blocks are nuniq distinct
// matrices after deduplication (at most nel * nbatch).
size_t required_bytes_blocks(const sdg_mesh* mesh, const sdg_options* opts, int stokes, int nbatch, int64_t nuniq) {
  const int64_t nb = nbatch;
  const int64_t nel = (int64_t)mesh->nx * mesh->ny;
  const int64_t NB = 2 * (int64_t)(mesh->k + 1) * (mesh->k + 1);
  const int64_t nu = nel * NB, np = nel * mesh->k * mesh->k;
  size_t b = 0;
  b += nb * (nel * 8 * 2 + nel * 4 + np * 8);  // eta, scale, element permutation, etap
  nuniq = std::max<int64_t>(1, std::min<int64_t>(nuniq, nel * nb));
  b += nuniq * NB * NB * 8 + nuniq * 8;
  b += 12 * (nel * nb / 16 + nuniq + 1);  // smoother work list (16 elements per item at least)
  const bool low = opts->prec_apply == SDG_FP32 || opts->prec_smoother != SDG_FP64;
  // low precision: the packed FP64 factor and the quad-packed factor in the
  // storage type (BF16 factors may be replaced by FP32 ones at setup: both
  // counted)
  if (low) b += nuniq * (NB * (NB + 1) / 2 * 8 + NB * (NB + 2) / 2 * (opts->prec_smoother == SDG_BF16 ? 2 + 4 : 4));
  // quad-packed FP64 inverses of a streamed smoother plan (k <= 4)
  if (mesh->k <= 4) b += nuniq * NB * (NB + 2) / 2 * 8;
  const bool q0 = opts->coarse_space == 1;
  if (q0) b += nb * nu * 8 * 2;  // probe vectors of A_0
  else b += nb * nel * 64 * 8;    // coarse local matrices
  int cx = q0 ? mesh->nx - 1 : mesh->nx, cy = q0 ? mesh->ny - 1 : mesh->ny;
  while (true) {
    const int64_t nn = (int64_t)(cx + 1) * (cy + 1);
    b += nb * nn * (36 + 14) * 8 + opts->smooth_h * nb * 16;
    const bool more = cx % 2 == 0 && cy % 2 == 0 && cx > opts->coarsest_n && cy > opts->coarsest_n;
    if (!more) {
      b += nb * 4 * nn * nn * 8 + nb * 8;
      break;
    }
    cx /= 2;
    cy /= 2;
  }
  b += nb * nu * 8 * 2 + opts->smooth_dg * nb * 16;  // DG cycle vectors
  if (low) b += nb * nu * 4 * 4;
  b += RED_SCRATCH * 8 + (SC_COUNT_FIXED + std::max(opts->restart, opts->eig_steps) + 4) * nb * 8 * 2 + nb * 4;
  b += nb * nu * 8 * 4;  // CG
  const int64_t n = stokes ? nu + np : nu;
  // the call's assembled right-hand side and iterate copies: F and G
  // (viscous), or b, x and the low part (Stokes)
  b += stokes ? nb * 3 * n * 8 : nb * (nu + np) * 8;
  if (stokes || opts->viscous_krylov >= 1) b += nb * ((2 * (int64_t)opts->restart + 2) * n + nu) * 8;
  if (stokes && opts->viscous_krylov == 2) b += nb * (2 * (int64_t)opts->restart + 2) * nu * 8;  // inner GCR
  b += nb * (int64_t)(opts->eig_steps + 2) * std::max<int64_t>(nu, 1) * 8;  // transient Arnoldi
  b += nb * (int64_t)(2 * opts->eig_steps + 2) * 8 + nb * 4;  // its coefficients and stopping flags
  if (opts->refine) b += nb * 3 * n * 8;  // low part of the iterate, refinement residual and correction
  return b;
}


int64_t unique_blocks(const sdg_mesh& m, const double* eta, int nbatch, bool dedup) {
  const int64_t nel = (int64_t)m.nx * m.ny, ntot = nel * nbatch;
  if (!dedup) return ntot;
  std::unordered_set<BlockKey, BlockKeyHash> seen;
  for (int64_t ge = 0; ge < ntot; ++ge) {
    const int64_t pb = ge / nel;
    seen.insert(block_key(m, eta + pb * nel, (int)(ge - pb * nel)));
  }
  return (int64_t)seen.size();
}
}  // namespace sdg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sdg_last_error(void) { return get_error(); }

void sdg_options_default(sdg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-8;
  o->inner_rtol = 1e-3;
  o->max_it = 1000;
  o->inner_max_it = 500;
  o->restart = 30;
  o->smooth_dg = 2;
  o->smooth_h = 3;
  o->coarsest_n = 8;
  o->eig_steps = 10;
  o->cheb_lo = 0.1;
  o->cheb_hi = 1.1;
  o->prec_smoother = SDG_FP64;
  o->prec_apply = SDG_FP64;
  o->viscous_krylov = 0;
  o->dedup = 1;
  o->seed = 0;
  o->graphs = 1;
}

int sdg_create(int device, size_t mem_budget, sdg_ctx** out) {
  if (!out) {
    set_error("NULL output pointer");
    return SDG_ERR_INVALID;
  }
  *out = nullptr;
  int ndev = 0;
  SDG_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) {
    set_error("device index out of range");
    return SDG_ERR_INVALID;
  }
  SDG_HIP(hipSetDevice(device));
  SDG_TRY(scratch_setup(device));
  sdg_ctx* c = new sdg_ctx();
  c->device = device;
  c->budget = mem_budget;
  *out = c;
  return SDG_OK;
}

void sdg_destroy(sdg_ctx* ctx) {
  if (!ctx) return;
  bool del;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    del = ctx->live == 0;
    ctx->closing = true;
  }
  if (del) delete ctx;
}

static bool opts_ok(const sdg_options* o) {
  if (!o) return false;
  if (!(o->rtol > 0) || !(o->inner_rtol > 0) || o->max_it < 1 || o->inner_max_it < 1) return false;
  if (o->restart < 1 || o->restart > 200 || o->smooth_dg < 1 || o->smooth_h < 1) return false;
  if (o->coarsest_n < 1 || o->eig_steps < 1 || o->eig_steps > 30) return false;
  if (!(o->cheb_lo > 0) || !(o->cheb_hi > o->cheb_lo)) return false;
  if (o->prec_smoother < 0 || o->prec_smoother > 2 || o->prec_apply < 0 || o->prec_apply > 1) return false;
  if (o->refine < 0 || o->refine > 1 || o->viscous_krylov < 0 || o->viscous_krylov > 2) return false;
  if (o->outer_krylov < 0 || o->outer_krylov > 1) return false;
  if (o->coarse_space < 0 || o->coarse_space > 1) return false;
  return true;
}

size_t sdg_required_bytes_batch(const sdg_mesh* mesh, const sdg_options* opts, int stokes, int nbatch) {
  if (!mesh_ok(mesh) || !opts_ok(opts) || nbatch < 1) return 0;
  return required_bytes_blocks(mesh, opts, stokes, nbatch, (int64_t)mesh->nx * mesh->ny * nbatch);
}

size_t sdg_required_bytes(const sdg_mesh* mesh, const sdg_options* opts, int stokes) {
  return sdg_required_bytes_batch(mesh, opts, stokes, 1);
}

void sdg_problem_destroy(sdg_problem* P);

int sdg_problem_create_batch(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, int nbatch,
                             const double* eta_dev, void* stream, sdg_problem** out) {
  if (!out) {
    set_error("NULL output pointer");
    return SDG_ERR_INVALID;
  }
  *out = nullptr;
  if (!ctx || !eta_dev || nbatch < 1 || nbatch > 4096) {
    set_error("NULL context or viscosity, or batch size outside 1..4096");
    return SDG_ERR_INVALID;
  }
  if (!mesh_ok(mesh)) {
    set_error("invalid mesh (need nx, ny >= 1, 1 <= k <= 6, lx, ly > 0, bc in 0..2)");
    return SDG_ERR_INVALID;
  }
  sdg_options o;
  if (opts) o = *opts;
  else sdg_options_default(&o);
  if (!opts_ok(&o)) {
    set_error("invalid options");
    return SDG_ERR_INVALID;
  }
  bool all_neumann = true, any_neumann = false;
  for (int i = 0; i < 4; ++i) {
    all_neumann = all_neumann && mesh->bc[i] == SDG_NEUMANN;
    any_neumann = any_neumann || mesh->bc[i] == SDG_NEUMANN;
  }
  if (all_neumann) {
    set_error("all-Neumann viscous problem is singular (rigid motions)");
    return SDG_ERR_UNSUPPORTED;
  }
  SDG_HIP(hipSetDevice(ctx->device));
  const double t0 = now_ms();
  sdg_problem* P = new sdg_problem();
  P->ctx = ctx;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->live++;
  }
  P->mesh = *mesh;
  P->opt = o;
  P->s = (hipStream_t)stream;
  P->nb = nbatch;
  P->k = mesh->k;
  P->K1 = mesh->k + 1;
  P->NB = 2 * P->K1 * P->K1;
  P->NPE = mesh->k * mesh->k;
  P->nel = mesh->nx * mesh->ny;
  P->nu = (int64_t)P->nel * P->NB;
  P->np = (int64_t)P->nel * P->NPE;
  P->neumann = any_neumann;
  P->M.nx = mesh->nx;
  P->M.ny = mesh->ny;
  P->M.hx = mesh->lx / mesh->nx;
  P->M.hy = mesh->ly / mesh->ny;
  for (int i = 0; i < 4; ++i) P->M.bc[i] = mesh->bc[i];
  P->inner_total.assign(nbatch, 0);
  P->inner_max.assign(nbatch, 0);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (int kern = 0; kern < 2; ++kern)
      for (int pr = 0; pr < 2; ++pr) {
        auto it = g_tune.find(tune_key(P, kern, pr));
        P->tile[kern][pr] = it != g_tune.end() ? it->second : sip_tile_default(P->k, pr == 1);
      }
  }
  auto fail = [&](int rc) {
    sdg_problem_destroy(P);
    return rc;
  };
  const int64_t ntot = (int64_t)P->nel * nbatch;
  int rc;
  if ((rc = palloc_t(P, &P->eta, ntot)) < 0) return fail(rc);
  P->eta_host.resize(ntot);
  if (hipMemcpyAsync(P->eta_host.data(), eta_dev, ntot * sizeof(double), hipMemcpyDeviceToHost, P->s) != hipSuccess ||
      hipStreamSynchronize(P->s) != hipSuccess) {
    (void)hipGetLastError();
    set_error("copy of the viscosity failed (device pointer expected)");
    return fail(SDG_ERR_DEVICE);
  }
  for (int64_t e = 0; e < ntot; ++e)
    if (!(P->eta_host[e] > 0.0) || !std::isfinite(P->eta_host[e])) {
      set_error("viscosity must be positive and finite (element " + std::to_string(e % P->nel) + " of problem " +
                std::to_string(e / P->nel) + ")");
      return fail(SDG_ERR_INVALID);
    }
  // the viscosity per element and per pressure mode, copied and expanded on
  // the device
  if ((rc = vec_copy(ntot, eta_dev, P->eta, P->s)) < 0) return fail(rc);
  if ((rc = palloc_t(P, &P->etap, (int64_t)P->np * nbatch)) < 0) return fail(rc);
  if ((rc = vec_expand(ntot, P->NPE, P->eta, P->etap, P->s)) < 0) return fail(rc);
  // the Q_1 hierarchy does not read the blocks: its kernels run while the
  // host groups the elements by block
  const bool coarse_first = o.coarse_space == 0;
  if (coarse_first && (rc = setup_coarse(P)) < 0) return fail(rc);
  if ((rc = setup_blocks(P)) < 0) return fail(rc);
  if (!coarse_first && (rc = setup_coarse(P)) < 0) return fail(rc);
  const int64_t U = P->nu * nbatch;
  for (double** v : {&P->vr, &P->vd, &P->cg_r, &P->cg_z, &P->cg_p, &P->cg_q, &P->cg_x})
    if ((rc = palloc_t(P, v, U)) < 0) return fail(rc);
  if (low_precision(P))
    for (float** v : {&P->fb, &P->fx, &P->fr, &P->fd})
      if ((rc = palloc_t(P, v, U)) < 0) return fail(rc);
  if ((rc = palloc_t(P, &P->ab0, (int64_t)o.smooth_dg * nbatch * 2)) < 0) return fail(rc);
  if ((rc = palloc_t(P, &P->red, RED_SCRATCH)) < 0) return fail(rc);
  const int64_t nsc = (int64_t)(SC_COUNT_FIXED + std::max(o.restart, o.eig_steps) + 4) * nbatch * 2;
  if ((rc = palloc_t(P, &P->dsc, nsc)) < 0) return fail(rc);
  P->nsc = nsc;
  if ((rc = palloc_t(P, &P->active, nbatch)) < 0) return fail(rc);
  if (hipHostMalloc((void**)&P->hsc, nsc * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&P->hpub, (2 * nbatch + 2) * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("pinned allocation failed");
    return fail(SDG_ERR_NOMEM);
  }
  P->hseq = reinterpret_cast<unsigned*>(P->hpub + 2 * nbatch);
  *P->hseq = 0u;
  if (hipHostMalloc((void**)&P->hstage, sdg_problem::STAGE_SLOTS * sdg_problem::STAGE_BYTES) != hipSuccess) {
    (void)hipGetLastError();
    set_error("pinned allocation failed");
    return fail(SDG_ERR_NOMEM);
  }
  for (hipEvent_t& e : P->stage_ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      set_error("event creation failed");
      return fail(SDG_ERR_DEVICE);
    }
    if (hipEventRecord(e, P->s) != hipSuccess) return fail(SDG_ERR_DEVICE);
  }
  if ((rc = palloc_t(P, &P->dcount, 1)) < 0) return fail(rc);
  SDG_HIP(hipMemsetAsync(P->dcount, 0, sizeof(unsigned), P->s));
  // Chebyshev bounds
  std::vector<double> lam;
  if ((rc = arnoldi(P, -1, lam, nullptr)) < 0) return fail(rc);
  // With exact block inverses the largest eigenvalue of the smoothed DG
  // operator is about 2 at every order.  BF16 factors of a block whose
  // condition is near the reciprocal of the BF16 unit (10^7 and more at
  // viscosity jumps of 10^6) overshoot by an order of magnitude and stall
  // the cycle: such a batch gets FP32 factors instead.
  if (P->binv16 && *std::max_element(lam.begin(), lam.end()) > BF16_LAMBDA_MAX) {
    if ((rc = palloc_t(P, &P->binv32, (int64_t)P->nuniq * tri_quad_size(P->NB))) < 0) return fail(rc);
    if ((rc = tri_quad_f32(P->xpacked, P->NB, P->nuniq, P->binv32, P->s)) < 0) return fail(rc);
    P->binv16 = nullptr;
    if ((rc = arnoldi(P, -1, lam, nullptr)) < 0) return fail(rc);
  }
  P->lmin0.resize(nbatch);
  P->lmax0.resize(nbatch);
  for (int pb = 0; pb < nbatch; ++pb) {
    P->lmin0[pb] = o.cheb_lo * lam[pb];
    P->lmax0[pb] = o.cheb_hi * lam[pb];
  }
  for (size_t li = 0; li < P->lev.size(); ++li) {
    CLevel& L = P->lev[li];
    if (L.coarsest) continue;
    if ((rc = arnoldi(P, (int)li, lam, nullptr)) < 0) return fail(rc);
    L.lmin.resize(nbatch);
    L.lmax.resize(nbatch);
    for (int pb = 0; pb < nbatch; ++pb) {
      L.lmin[pb] = o.cheb_lo * lam[pb];
      L.lmax[pb] = o.cheb_hi * lam[pb];
    }
  }
  if ((rc = join_dense(P)) < 0) return fail(rc);
  if ((rc = upload_cheb(P)) < 0) return fail(rc);
  if (hipStreamSynchronize(P->s) != hipSuccess) {
    (void)hipGetLastError();
    set_error("setup failed on the device");
    return fail(SDG_ERR_DEVICE);
  }
  P->setup_ms = now_ms() - t0;
  *out = P;
  return SDG_OK;
}

int sdg_problem_create(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta_dev,
                       void* stream, sdg_problem** out) {
  return sdg_problem_create_batch(ctx, mesh, opts, 1, eta_dev, stream, out);
}

void sdg_problem_destroy(sdg_problem* P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->s);
  if (P->ds) {  // a setup that failed before joining the side stream
    (void)hipStreamSynchronize(P->ds);
    (void)hipStreamDestroy(P->ds);
  }
  for (hipEvent_t e : P->ds_ev)
    if (e) (void)hipEventDestroy(e);
  drop_graphs(P);
  if (P->ctx) comb_drop(P->ctx, P);
  if (P->gs) (void)hipStreamDestroy(P->gs);
  // the stream has drained: the blocks go back to the context's cache
  if (P->ctx)
    for (auto& a : P->allocs) ctx_put(P->ctx, a.first, a.second);
  else
    for (auto& a : P->allocs) (void)hipFree(a.first);
  if (P->hsc) (void)hipHostFree(P->hsc);
  if (P->hpub) (void)hipHostFree(P->hpub);
  for (hipEvent_t e : P->stage_ev)
    if (e) (void)hipEventDestroy(e);
  if (P->hstage) (void)hipHostFree(P->hstage);
  if (sdg_ctx* c = P->ctx) {
    bool del;
    {
      std::lock_guard<std::mutex> g(c->mu);
      c->used -= std::min(c->used, P->bytes);
      c->live--;
      del = c->closing && c->live == 0;
    }
    if (del) delete c;
  }
  delete P;
}

int sdg_problem_smoother_precision(const sdg_problem* P, int* prec) {
  if (!P || !prec) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  *prec = P->binv16 ? SDG_BF16 : P->binv32 ? SDG_FP32 : SDG_FP64;
  return SDG_OK;
}

int sdg_problem_batch(const sdg_problem* P, int* nbatch) {
  if (!P || !nbatch) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  *nbatch = P->nb;
  return SDG_OK;
}

int sdg_problem_levels(const sdg_problem* P, int* nlevels) {
  if (!P || !nlevels) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  *nlevels = 1 + (int)P->lev.size();
  return SDG_OK;
}

int sdg_get_bounds(const sdg_problem* P, double* b) {
  if (!P || !b) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  const int nl = 1 + (int)P->lev.size();
  for (int pb = 0; pb < P->nb; ++pb) {
    double* o = b + (size_t)pb * nl * 2;
    o[0] = P->lmin0[pb];
    o[1] = P->lmax0[pb];
    for (size_t i = 0; i < P->lev.size(); ++i) {
      const bool c = P->lev[i].coarsest;
      o[2 + 2 * i] = c ? 0.0 : P->lev[i].lmin[pb];
      o[3 + 2 * i] = c ? 0.0 : P->lev[i].lmax[pb];
    }
  }
  return SDG_OK;
}

int sdg_set_bounds(sdg_problem* P, const double* b) {
  if (!P || !b) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  const int nl = 1 + (int)P->lev.size();
  for (int pb = 0; pb < P->nb; ++pb) {
    const double* o = b + (size_t)pb * nl * 2;
    P->lmin0[pb] = o[0];
    P->lmax0[pb] = o[1];
    for (size_t i = 0; i < P->lev.size(); ++i) {
      if (P->lev[i].coarsest) continue;
      P->lev[i].lmin[pb] = o[2 + 2 * i];
      P->lev[i].lmax[pb] = o[3 + 2 * i];
    }
  }
  return upload_cheb(P);
}

int sdg_eig_estimate(sdg_problem* P, int level, double* lambda_out, double* hess) {
  if (!P || !lambda_out || level < 0 || level > (int)P->lev.size()) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  if (level > 0 && P->lev[level - 1].coarsest) {
    set_error("the coarsest level is solved directly and has no smoother");
    return SDG_ERR_INVALID;
  }
  std::vector<double> lam, H;
  SDG_TRY(arnoldi(P, level - 1, lam, &H));
  for (int pb = 0; pb < P->nb; ++pb) lambda_out[pb] = lam[pb];
  if (hess) std::memcpy(hess, H.data(), H.size() * sizeof(double));
  return SDG_OK;
}

#define PCHECK(...)                         \
  do {                                      \
    if (!P) {                               \
      set_error("NULL problem");            \
      return SDG_ERR_INVALID;               \
    }                                       \
    const void* _ptrs[] = {__VA_ARGS__};    \
    for (const void* _p : _ptrs)            \
      if (!_p) {                            \
        set_error("NULL pointer argument"); \
        return SDG_ERR_INVALID;             \
      }                                     \
  } while (0)

int sdg_apply_viscous(sdg_problem* P, const double* u, double* y) {
  PCHECK(u, y);
  return run_sip_apply(P, u, y);
}
int sdg_residual_viscous(sdg_problem* P, const double* b, const double* u, double* r) {
  PCHECK(b, u, r);
  return run_sip_residual(P, b, u, r);
}
int sdg_apply_viscous_f32(sdg_problem* P, const float* u, float* y) {
  PCHECK(u, y);
  return run_sip_apply_f32(P, u, y);
}
int sdg_apply_div(sdg_problem* P, const double* u, double* q) {
  PCHECK(u, q);
  return div_apply(P->M, P->k, P->nb, u, q, P->s);
}
int sdg_apply_grad(sdg_problem* P, const double* p, double* v) {
  PCHECK(p, v);
  return grad_apply(P->M, P->k, P->nb, p, v, P->s);
}
int sdg_apply_blockjacobi(sdg_problem* P, const double* r, double* z) {
  PCHECK(r, z);
  if (P->opt.prec_smoother == SDG_FP64) return bj_apply64(P, r, z);
  if (!P->fr) {
    set_error("low-precision smoother storage missing");
    return SDG_ERR_INVALID;
  }
  SDG_TRY(d2f(P->nu * P->nb, r, P->fr, P->s));
  SDG_TRY(bj_apply32(P, P->fr, P->fd));
  return f2d(P->nu * P->nb, P->fd, z, P->s);
}
int sdg_get_blocks(sdg_problem* P, double* blocks) {
  PCHECK(blocks);
  const int64_t ntot = (int64_t)P->nel * P->nb;
  std::vector<int> all(ntot);
  for (int64_t e = 0; e < ntot; ++e) all[e] = (int)e;
  int* d = nullptr;
  SDG_HIP(hipMalloc((void**)&d, ntot * sizeof(int)));
  int rc = SDG_OK;
  if (hipMemcpyAsync(d, all.data(), ntot * sizeof(int), hipMemcpyHostToDevice, P->s) != hipSuccess) rc = SDG_ERR_DEVICE;
  if (rc == SDG_OK) rc = sip_block_list(P->M, P->k, P->eta, d, (int)ntot, blocks, P->s);
  (void)hipStreamSynchronize(P->s);
  (void)hipFree(d);
  return rc;
}
int sdg_get_blocks_noalloc(sdg_problem* P, double* blocks) {
  PCHECK(blocks);
  const int64_t ntot = (int64_t)P->nel * P->nb;
  if (ntot > NOALLOC_MAX_ELEMS) {
    set_error("sdg_get_blocks_noalloc: " + std::to_string(ntot) + " elements (all problems of the batch) exceed " +
              "its limit of " + std::to_string(NOALLOC_MAX_ELEMS));
    return SDG_ERR_INVALID;
  }
  int* list = (int*)scratch_ptr(P->ctx->device);
  if (!list) {
    set_error("sdg_get_blocks_noalloc: scratch address not set up for this device");
    return SDG_ERR_DEVICE;
  }
  const int grid = (int)std::min<int64_t>((ntot + 255) / 256, 4096);
  hipLaunchKernelGGL(iota_kernel, dim3(grid), dim3(256), 0, P->s, ntot, list);
  SDG_CHECK_LAUNCH();
  return sip_block_list(P->M, P->k, P->eta, list, (int)ntot, blocks, P->s);
}
int sdg_p_restrict(sdg_problem* P, const double* r, double* rc) {
  PCHECK(r, rc);
  if (P->opt.coarse_space == 1) return q0_restrict_full((int64_t)P->nel * P->nb, P->k, r, rc, P->s);
  return p_restrict(P->M, P->k, P->nb, r, rc, P->s);
}
int sdg_p_prolong_add(sdg_problem* P, const double* ec, double* u) {
  PCHECK(ec, u);
  if (P->opt.coarse_space == 1) return q0_prolong_add((int64_t)P->nel * P->nb, P->k, ec, u, P->s);
  return p_prolong_add(P->M, P->k, P->nb, ec, u, P->s);
}
int sdg_get_coarse_stencil(sdg_problem* P, int level, double* st, int* nx_out, int* ny_out) {
  PCHECK(st);
  if (level < 0 || level >= (int)P->lev.size()) {
    set_error("level out of range");
    return SDG_ERR_INVALID;
  }
  const CLevel& L = P->lev[level];
  SDG_HIP(hipMemcpyAsync(st, L.st, (size_t)36 * L.nn * P->nb * sizeof(double), hipMemcpyDeviceToDevice, P->s));
  if (nx_out) *nx_out = L.nx;
  if (ny_out) *ny_out = L.ny;
  return SDG_OK;
}
int sdg_vcycle(sdg_problem* P, const double* b, double* x) {
  PCHECK(b, x);
  return vcycle(P, b, x);
}
int sdg_assemble_rhs(sdg_problem* P, const double* f, const double* g, double* F, double* G) {
  PCHECK(f, F, G);
  return rhs_assemble(P->M, P->k, P->nb, P->eta, f, g, F, G, P->s);
}

}  // extern "C"

namespace {

// Viscous solve behind sdg_solve_viscous_dev / _ext_dev: u (and, for
// opts.refine, the low part ulo; may be null) of u = A^{-1} F.
int solve_viscous_impl(sdg_problem* P, const double* f, const double* g, double* u, double* ulo, sdg_stats* st) {
  const double t0 = now_ms();
  const int64_t U = P->nu * P->nb;
  const bool refine = P->opt.refine != 0;
  double* F = nullptr;
  double* G = nullptr;
  double* xl = nullptr;
  const int64_t nG = std::max<int64_t>(P->np * P->nb, 1);
  const bool own_lo = refine && !ulo;
  if (tmp_get(P, &F, U) < 0 || tmp_get(P, &G, nG) < 0 || (own_lo && tmp_get(P, &xl, U) < 0)) {
    tmp_put(P, F, U);
    tmp_put(P, G, nG);
    tmp_put(P, xl, U);
    set_error("allocation failed");
    return SDG_ERR_NOMEM;
  }
  if (!own_lo) xl = ulo;
  std::vector<int> its, status;
  std::vector<double> rel;
  const VSpec S = viscous_spec(P);
  int rc = rhs_assemble(P->M, P->k, P->nb, P->eta, f, g, F, G, P->s);
  if (rc >= 0) {
    if (P->opt.viscous_krylov == 2) {
      rc = ensure_gmres(P, P->nu);
      auto mv = [&](const double* x, double* y) { return run_sip_apply(P, x, y); };
      auto pc = [&](const double* v, double* z) { return vcycle(P, v, z); };
      auto pj = [&](double*) { return SDG_OK; };
      auto rs = [&](const double* x, const double* lo, double* w) {
        if (refine) return run_ext(P, false, false, F, x, lo, w);
        return run_sip_residual(P, F, x, w);
      };
      auto ab = [&](const double* x, double* y) { return run_ext(P, false, true, nullptr, x, nullptr, y); };
      if (rc >= 0)
        rc = gcr(P, S, outer_gcr_work(P), F, u, refine ? xl : nullptr, P->opt.rtol, P->opt.max_it, mv, pc, pj, rs,
                 ab, its, rel, status);
    } else if (P->opt.viscous_krylov == 1) {
      auto mv = [&](const double* x, double* y) { return run_sip_apply(P, x, y); };
      auto pc = [&](const double* v, double* z) { return vcycle(P, v, z); };
      auto pj = [&](double*) { return SDG_OK; };
      auto rs = [&](const double* x, const double* lo, double* w) {
        if (refine) return run_ext(P, false, false, F, x, lo, w);
        return run_sip_residual(P, F, x, w);
      };
      auto ab = [&](const double* x, double* y) { return run_ext(P, false, true, nullptr, x, nullptr, y); };
      rc = fgmres(P, S, F, u, refine ? xl : nullptr, P->opt.rtol, P->opt.max_it, mv, pc, pj, rs, ab, its, rel,
                  status);
    } else if (refine) {
      rc = cg_refine(P, F, u, xl, P->opt.rtol, P->opt.max_it, its, rel, status);
    } else {
      rc = cg_solve(P, F, u, P->opt.rtol, P->opt.max_it, its, rel, status);
    }
  }
  // true residual ||F - A u|| / ||F|| per problem (extended precision with
  // the low part when refining)
  if (rc >= 0) {
    std::vector<double> fn, rn;
    rc = vs_norms(P, S, F, fn);
    if (rc >= 0) rc = refine ? run_ext(P, false, false, F, u, xl, P->vr) : run_sip_residual(P, F, u, P->vr);
    if (rc >= 0) rc = vs_norms(P, S, P->vr, rn);
    if (rc >= 0)
      for (int pb = 0; pb < P->nb; ++pb) rel[pb] = fn[pb] > 0 ? rn[pb] / fn[pb] : 0.0;
  }
  if (rc >= 0 && ulo && !refine && hipMemsetAsync(ulo, 0, U * sizeof(double), P->s) != hipSuccess)
    rc = SDG_ERR_DEVICE;
  tmp_put(P, F, U);  // synchronises the stream first
  tmp_put(P, G, nG);
  if (own_lo) tmp_put(P, xl, U);
  if (rc < 0) return rc;
  return fill_stats(P, st, status, its, rel, t0, false);
}

int solve_stokes_impl(sdg_problem* P, const double* f, const double* g, double* u, double* ulo, double* p,
                      double* plo, sdg_stats* st) {
  const double t0 = now_ms();
  const VSpec S = stokes_spec(P);
  const int64_t U = P->nu * P->nb;
  const bool refine = P->opt.refine != 0;
  double* b = nullptr;
  double* x = nullptr;
  double* xl = nullptr;
  if (tmp_get(P, &b, S.total) < 0 || tmp_get(P, &x, S.total) < 0 || tmp_get(P, &xl, S.total) < 0) {
    tmp_put(P, b, S.total);
    tmp_put(P, x, S.total);
    tmp_put(P, xl, S.total);
    set_error("allocation failed");
    return SDG_ERR_NOMEM;
  }
  std::fill(P->inner_total.begin(), P->inner_total.end(), 0);
  std::fill(P->inner_max.begin(), P->inner_max.end(), 0);
  std::vector<int> its, status;
  std::vector<double> rel;
  int rc = rhs_assemble(P->M, P->k, P->nb, P->eta, f, g, b, b + U, P->s);
  if (rc >= 0) rc = ensure_gmres(P, P->nu + P->np);
  if (rc >= 0) {
    auto mv = [&](const double* xx, double* yy) { return stokes_matvec(P, xx, yy); };
    auto pc = [&](const double* v, double* z) { return stokes_prec(P, v, z); };
    auto pj = [&](double* v) { return stokes_project(P, v); };
    auto rs = [&](const double* xx, const double* lo, double* w) {
      if (refine) return run_ext(P, true, false, b, xx, lo, w);
      SDG_TRY(stokes_matvec(P, xx, w));
      return vec_axpby(S.total, 1.0, b, -1.0, w, P->s);
    };
    auto ab = [&](const double* xx, double* yy) { return run_ext(P, true, true, nullptr, xx, nullptr, yy); };
    if (P->opt.outer_krylov == 1)
      rc = gcr(P, S, outer_gcr_work(P), b, x, refine ? xl : nullptr, P->opt.rtol, P->opt.max_it, mv, pc, pj, rs, ab,
               its, rel, status);
    else
      rc = fgmres(P, S, b, x, refine ? xl : nullptr, P->opt.rtol, P->opt.max_it, mv, pc, pj, rs, ab, its, rel,
                  status);
  }
  if (rc >= 0) {
    // the pressure of the pair: the constant is fixed on its high part
    rc = stokes_project(P, x);
    if (rc >= 0 && hipMemcpyAsync(u, x, U * sizeof(double), hipMemcpyDeviceToDevice, P->s) != hipSuccess) rc = SDG_ERR_DEVICE;
    if (rc >= 0 && P->np > 0 &&
        hipMemcpyAsync(p, x + U, P->np * P->nb * sizeof(double), hipMemcpyDeviceToDevice, P->s) != hipSuccess)
      rc = SDG_ERR_DEVICE;
    if (rc >= 0 && ulo) {
      if (refine) {
        if (hipMemcpyAsync(ulo, xl, U * sizeof(double), hipMemcpyDeviceToDevice, P->s) != hipSuccess) rc = SDG_ERR_DEVICE;
      } else if (hipMemsetAsync(ulo, 0, U * sizeof(double), P->s) != hipSuccess) {
        rc = SDG_ERR_DEVICE;
      }
    }
    if (rc >= 0 && plo && P->np > 0) {
      if (refine) {
        if (hipMemcpyAsync(plo, xl + U, P->np * P->nb * sizeof(double), hipMemcpyDeviceToDevice, P->s) != hipSuccess)
          rc = SDG_ERR_DEVICE;
      } else if (hipMemsetAsync(plo, 0, P->np * P->nb * sizeof(double), P->s) != hipSuccess) {
        rc = SDG_ERR_DEVICE;
      }
    }
  }
  tmp_put(P, b, S.total);  // synchronises the stream first
  tmp_put(P, x, S.total);
  tmp_put(P, xl, S.total);
  if (rc < 0) return rc;
  return fill_stats(P, st, status, its, rel, t0, true);
}

}  // namespace

extern "C" {

int sdg_solve_viscous_dev(sdg_problem* P, const double* f, const double* g, double* u, sdg_stats* st) {
  PCHECK(f, u);
  return solve_viscous_impl(P, f, g, u, nullptr, st);
}
int sdg_solve_viscous_ext_dev(sdg_problem* P, const double* f, const double* g, double* u, double* ulo,
                              sdg_stats* st) {
  PCHECK(f, u);
  return solve_viscous_impl(P, f, g, u, ulo, st);
}
int sdg_solve_stokes_dev(sdg_problem* P, const double* f, const double* g, double* u, double* p, sdg_stats* st) {
  PCHECK(f, u, p);
  return solve_stokes_impl(P, f, g, u, nullptr, p, nullptr, st);
}
int sdg_solve_stokes_ext_dev(sdg_problem* P, const double* f, const double* g, double* u, double* ulo, double* p,
                             double* plo, sdg_stats* st) {
  PCHECK(f, u, p);
  return solve_stokes_impl(P, f, g, u, ulo, p, plo, st);
}
int sdg_residual_ext(sdg_problem* P, int stokes, const double* b, const double* xh, const double* xl, double* r) {
  PCHECK(b, xh, r);
  return run_ext(P, stokes != 0, false, b, xh, xl, r);
}
int sdg_abs_apply(sdg_problem* P, int stokes, const double* x, double* y) {
  PCHECK(x, y);
  return run_ext(P, stokes != 0, true, nullptr, x, nullptr, y);
}

static int host_solve(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta,
                      const double* f, const double* g, double* u, double* p, sdg_stats* st, bool stokes) {
  if (!ctx || !mesh_ok(mesh) || !eta || !f || !u || (stokes && !p)) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  SDG_HIP(hipSetDevice(ctx->device));
  const int64_t nel = (int64_t)mesh->nx * mesh->ny;
  const int64_t NB = 2 * (int64_t)(mesh->k + 1) * (mesh->k + 1);
  const int64_t nu = nel * NB, np = nel * mesh->k * mesh->k;
  const int64_t ng = (int64_t)(2 * mesh->nx + 2 * mesh->ny) * 2 * (mesh->k + 1);
  double *de = nullptr, *df = nullptr, *dg = nullptr, *du = nullptr, *dp = nullptr;
  int rc = SDG_OK;
  // staging arrays from the context's cache (returned below, after the
  // synchronous copies and the problem's own drain)
  auto bytes_of = [](int64_t n) { return cache_size((size_t)std::max<int64_t>(n, 1) * sizeof(double)); };
  auto al = [&](double** q, int64_t n) {
    if (rc < 0) return;
    void* v = nullptr;
    if (ctx_get(ctx, bytes_of(n), &v) < 0) {
      set_error("allocation failed");
      rc = SDG_ERR_NOMEM;
    }
    *q = (double*)v;
  };
  al(&de, nel);
  al(&df, nu);
  al(&du, nu);
  if (stokes) al(&dp, np);
  if (g) al(&dg, ng);
  if (rc >= 0) {
    if (hipMemcpy(de, eta, nel * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(df, f, nu * 8, hipMemcpyHostToDevice) != hipSuccess ||
        (g && hipMemcpy(dg, g, ng * 8, hipMemcpyHostToDevice) != hipSuccess)) {
      (void)hipGetLastError();
      set_error("host to device copy failed");
      rc = SDG_ERR_DEVICE;
    }
  }
  sdg_problem* P = nullptr;
  if (rc >= 0) rc = sdg_problem_create(ctx, mesh, opts, de, nullptr, &P);
  if (rc >= 0) {
    rc = stokes ? sdg_solve_stokes_dev(P, df, dg, du, dp, st) : sdg_solve_viscous_dev(P, df, dg, du, st);
    if (rc >= 0) {
      if (hipMemcpy(u, du, nu * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          (stokes && np > 0 && hipMemcpy(p, dp, np * 8, hipMemcpyDeviceToHost) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("device to host copy failed");
        rc = SDG_ERR_DEVICE;
      }
    }
  }
  sdg_problem_destroy(P);  // drains the problem's stream; the copies above are synchronous
  const int64_t ns[5] = {nel, nu, ng, nu, np};
  double* qs[5] = {de, df, dg, du, dp};
  for (int i = 0; i < 5; ++i)
    if (qs[i]) ctx_put(ctx, qs[i], bytes_of(ns[i]));
  return rc;
}

int sdg_solve_viscous_batch(sdg_ctx* ctx, int n, const sdg_mesh* meshes, const sdg_options* opts,
                            const double* const* eta, const double* const* f, double* const* u,
                            double* const* u_lo, sdg_stats* stats) {
  if (!ctx || n < 0 || (n > 0 && (!meshes || !eta || !f || !u))) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  if (n == 0) return SDG_OK;
  sdg_options o;
  if (opts) o = *opts;
  else sdg_options_default(&o);
  for (int i = 0; i < n; ++i)
    if (!mesh_ok(&meshes[i]) || !eta[i] || !f[i] || !u[i]) {
      set_error("invalid mesh or NULL array of request " + std::to_string(i));
      return SDG_ERR_INVALID;
    }
  SDG_HIP(hipSetDevice(ctx->device));
  const double t0 = now_ms();
  // requests of identical mesh and order form one batched problem
  std::map<std::string, std::vector<int>> bykey;
  for (int i = 0; i < n; ++i) {
    const sdg_mesh& m = meshes[i];
    char key[160];
    std::snprintf(key, sizeof(key), "%d/%d/%d/%.17g/%.17g/%d%d%d%d", m.k, m.nx, m.ny, m.lx, m.ly, m.bc[0], m.bc[1],
                  m.bc[2], m.bc[3]);
    bykey[key].push_back(i);
  }
  struct Grp {
    std::vector<int> idx;
    sdg_problem* P = nullptr;
    double *de = nullptr, *df = nullptr, *dF = nullptr, *dG = nullptr, *du = nullptr, *dul = nullptr;
    int64_t ne = 0, nu = 0, np = 0;
  };
  std::vector<Grp> G;
  for (auto& kv : bykey) {
    G.emplace_back();
    G.back().idx = kv.second;
  }
  hipStream_t s = nullptr;
  SDG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  auto bytes_of = [](int64_t cnt) { return cache_size((size_t)std::max<int64_t>(cnt, 1) * sizeof(double)); };
  // The groups are set up from up to 8 host threads, each group on a stream
  // of its own, so that the host parts of setup (block grouping, the reads
  // of the eigenvalue estimates) of different groups overlap, and so do
  // their kernels.  Every group then joins s, on which the solve runs.
  auto setup_group = [&](Grp& g, hipStream_t gst) -> int {
    const sdg_mesh& m = meshes[g.idx[0]];
    const int nb = (int)g.idx.size();
    g.ne = (int64_t)m.nx * m.ny;
    g.nu = g.ne * 2 * (m.k + 1) * (m.k + 1);
    g.np = g.ne * m.k * m.k;
    int grc = SDG_OK;
    for (double** q : {&g.de}) grc = grc < 0 ? grc : ctx_get(ctx, bytes_of(nb * g.ne), (void**)q);
    for (double** q : {&g.df, &g.dF, &g.du, &g.dul}) grc = grc < 0 ? grc : ctx_get(ctx, bytes_of(nb * g.nu), (void**)q);
    if (grc >= 0) grc = ctx_get(ctx, bytes_of(nb * g.np), (void**)&g.dG);
    for (int i = 0; i < nb && grc >= 0; ++i) {
      const int r = g.idx[i];
      if (hipMemcpyAsync(g.de + i * g.ne, eta[r], g.ne * 8, hipMemcpyHostToDevice, gst) != hipSuccess ||
          hipMemcpyAsync(g.df + i * g.nu, f[r], g.nu * 8, hipMemcpyHostToDevice, gst) != hipSuccess) {
        (void)hipGetLastError();
        set_error("host to device copy failed");
        grc = SDG_ERR_DEVICE;
      }
    }
    if (grc >= 0) grc = sdg_problem_create_batch(ctx, &m, &o, nb, g.de, gst, &g.P);
    if (grc >= 0) grc = rhs_assemble(g.P->M, g.P->k, nb, g.P->eta, g.df, nullptr, g.dF, g.dG, gst);
    return grc;
  };
  int rc = SDG_OK;
  std::vector<hipStream_t> gstr(G.size(), nullptr);
  for (hipStream_t& q : gstr)
    if (rc >= 0 && hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      q = nullptr;
      set_error("stream creation failed");
      rc = SDG_ERR_DEVICE;
    }
  if (rc >= 0) {
    std::vector<int> grc(G.size(), SDG_OK);
    std::vector<std::string> gerr(G.size());
    std::atomic<size_t> next{0};
    auto work = [&] {
      const bool dev_ok = hipSetDevice(ctx->device) == hipSuccess;
      for (size_t gi; (gi = next.fetch_add(1)) < G.size();) {
        grc[gi] = dev_ok ? setup_group(G[gi], gstr[gi]) : SDG_ERR_DEVICE;
        if (grc[gi] < 0) gerr[gi] = dev_ok ? std::string(sdg_last_error()) : std::string("hipSetDevice failed");
      }
    };
    std::vector<std::thread> th;
    for (size_t t = 1; t < std::min<size_t>(G.size(), 8); ++t) th.emplace_back(work);
    work();
    for (std::thread& t : th) t.join();
    for (size_t gi = 0; gi < G.size() && rc >= 0; ++gi)
      if (grc[gi] < 0) {
        rc = grc[gi];
        set_error(gerr[gi]);  // the message was set on the worker's thread
      }
  }
  // s waits for every group's setup; the groups' problems then run on s
  hipEvent_t joined = nullptr;
  if (rc >= 0 && hipEventCreateWithFlags(&joined, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    joined = nullptr;
    set_error("event creation failed");
    rc = SDG_ERR_DEVICE;
  }
  for (size_t gi = 0; gi < G.size() && rc >= 0; ++gi) {
    if (hipEventRecord(joined, gstr[gi]) != hipSuccess || hipStreamWaitEvent(s, joined, 0) != hipSuccess) {
      (void)hipGetLastError();
      set_error("joining the groups' streams failed");
      rc = SDG_ERR_DEVICE;
      break;
    }
    G[gi].P->s = s;
  }
  // solve: CG groups in lockstep (combined graph per iteration); other
  // Krylov choices group after group
  std::vector<std::vector<int>> its(G.size()), status(G.size());
  std::vector<std::vector<double>> rel(G.size());
  if (rc >= 0) {
    MultiGraphs MG;
    if (o.viscous_krylov == 0 && o.refine) {
      std::vector<RefineState> R(G.size());
      for (size_t i = 0; i < G.size(); ++i) {
        R[i].P = G[i].P;
        R[i].F = G[i].dF;
        R[i].xh = G[i].du;
        R[i].xl = G[i].dul;
      }
      rc = cg_refine_multi(R, o.rtol, o.max_it, MG);
      for (size_t i = 0; i < G.size() && rc >= 0; ++i) {
        its[i] = R[i].its;
        rel[i] = R[i].rel;
        status[i] = R[i].status;
      }
    } else if (o.viscous_krylov == 0) {
      std::vector<CgRun> runs(G.size());
      for (size_t i = 0; i < G.size() && rc >= 0; ++i) {
        rc = cg_start(runs[i], G[i].P, G[i].dF, G[i].du, o.rtol, o.max_it, nullptr);
        if (rc >= 0 && hipMemsetAsync(G[i].dul, 0, G[i].idx.size() * G[i].nu * 8, s) != hipSuccess) rc = SDG_ERR_DEVICE;
      }
      if (rc >= 0) rc = cg_multi(runs, MG);
      for (size_t i = 0; i < G.size() && rc >= 0; ++i) {
        its[i] = runs[i].its;
        status[i] = runs[i].status;
      }
    } else {
      for (size_t i = 0; i < G.size() && rc >= 0; ++i) {
        std::vector<sdg_stats> st(G[i].idx.size());
        rc = solve_viscous_impl(G[i].P, G[i].df, nullptr, G[i].du, G[i].dul, st.data());
        for (size_t j = 0; j < st.size() && rc >= 0; ++j) {
          its[i].push_back(st[j].outer_its);
          status[i].push_back(st[j].status);
        }
      }
    }
  }
  // true residuals (extended with refinement), results to the host
  for (size_t i = 0; i < G.size() && rc >= 0; ++i) {
    Grp& g = G[i];
    sdg_problem* P = g.P;
    const VSpec S = viscous_spec(P);
    std::vector<double> fn, rn;
    rc = vs_norms(P, S, g.dF, fn);
    if (rc >= 0)
      rc = o.refine ? run_ext(P, false, false, g.dF, g.du, g.dul, P->vr) : run_sip_residual(P, g.dF, g.du, P->vr);
    if (rc >= 0) rc = vs_norms(P, S, P->vr, rn);
    if (rc < 0) break;
    rel[i].assign(g.idx.size(), 0.0);
    for (size_t j = 0; j < g.idx.size(); ++j) rel[i][j] = fn[j] > 0 ? rn[j] / fn[j] : 0.0;
    std::vector<sdg_stats> st(g.idx.size());
    fill_stats(P, st.data(), status[i], its[i], rel[i], t0, false);
    for (size_t j = 0; j < g.idx.size() && rc >= 0; ++j) {
      const int r = g.idx[j];
      if (stats) stats[r] = st[j];
      if (hipMemcpyAsync(u[r], g.du + j * g.nu, g.nu * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          (u_lo && u_lo[r] &&
           hipMemcpyAsync(u_lo[r], g.dul + j * g.nu, g.nu * 8, hipMemcpyDeviceToHost, s) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("device to host copy failed");
        rc = SDG_ERR_DEVICE;
      }
    }
    if (rc >= 0 && hipStreamSynchronize(s) != hipSuccess) rc = SDG_ERR_DEVICE;
  }
  int worst = SDG_OK;
  auto rank = [](int v) { return v == SDG_BREAKDOWN ? 3 : v == SDG_NOT_CONVERGED ? 2 : v == SDG_FLOOR ? 1 : 0; };
  for (auto& sv : status)
    for (int v : sv)
      if (rank(v) > rank(worst)) worst = v;
  (void)hipStreamSynchronize(s);
  for (hipStream_t q : gstr)  // a group whose setup failed may still have work there
    if (q) (void)hipStreamSynchronize(q);
  for (Grp& g : G) {
    sdg_problem_destroy(g.P);  // drains the stream
    const int nb = (int)g.idx.size();
    if (g.de) ctx_put(ctx, g.de, bytes_of(nb * g.ne));
    for (double* q : {g.df, g.dF, g.du, g.dul})
      if (q) ctx_put(ctx, q, bytes_of(nb * g.nu));
    if (g.dG) ctx_put(ctx, g.dG, bytes_of(nb * g.np));
  }
  if (joined) (void)hipEventDestroy(joined);
  for (hipStream_t q : gstr)
    if (q) (void)hipStreamDestroy(q);
  (void)hipStreamDestroy(s);
  return rc < 0 ? rc : worst;
}

int sdg_solve_viscous(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta,
                      const double* f, const double* g, double* u, sdg_stats* st) {
  return host_solve(ctx, mesh, opts, eta, f, g, u, nullptr, st, false);
}
int sdg_solve_stokes(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta,
                     const double* f, const double* g, double* u, double* p, sdg_stats* st) {
  return host_solve(ctx, mesh, opts, eta, f, g, u, p, st, true);
}

int sdg_tile_variants(int k, int* count) {
  if (!count || k < 1 || k > 6) {
    set_error("NULL output or order k out of range");
    return SDG_ERR_INVALID;
  }
  *count = sip_tile_variants(k);
  return SDG_OK;
}

int sdg_tile_shape(int k, int variant, int* tx, int* ty) {
  if (!tx || !ty || k < 1 || k > 6 || variant < 0 || variant >= sip_tile_variants(k)) {
    set_error("NULL output, order k or tile variant out of range");
    return SDG_ERR_INVALID;
  }
  sip_tile_shape(k, variant, tx, ty);
  return SDG_OK;
}

int sdg_get_tile(const sdg_problem* P, int kernel, int precision, int* variant) {
  if (!P || !variant || kernel < 0 || kernel > 1 || (precision != SDG_FP64 && precision != SDG_FP32)) {
    set_error("invalid problem, kernel or precision");
    return SDG_ERR_INVALID;
  }
  *variant = P->tile[kernel][precision == SDG_FP64 ? 0 : 1];
  return SDG_OK;
}

int sdg_set_tile(sdg_problem* P, int kernel, int precision, int variant) {
  if (!P || kernel < 0 || kernel > 1 || (precision != SDG_FP64 && precision != SDG_FP32) || variant < 0 ||
      variant >= sip_tile_variants(P->k)) {
    set_error("invalid problem, kernel, precision or tile variant");
    return SDG_ERR_INVALID;
  }
  P->tile[kernel][precision == SDG_FP64 ? 0 : 1] = variant;
  drop_graphs(P);
  return SDG_OK;
}

int sdg_autotune(sdg_problem* P, int reps, int* variants, double* us) {
  if (!P || reps < 1) {
    set_error("invalid problem or repetition count");
    return SDG_ERR_INVALID;
  }
  const int64_t U = P->nu * P->nb;
  const int nv = sip_tile_variants(P->k);
  SDG_TRY(uniform_pm1(P->opt.seed ^ 0x5eedull, U, P->cg_r, P->s));
  SDG_TRY(uniform_pm1(P->opt.seed ^ 0xb0bull, U, P->cg_z, P->s));
  const bool f32 = low_precision(P);
  if (f32) {
    SDG_TRY(d2f(U, P->cg_r, P->fx, P->s));
    SDG_TRY(d2f(U, P->cg_z, P->fb, P->s));
  }
  hipEvent_t e0, e1;
  SDG_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return SDG_ERR_DEVICE;
  }
  int rc = SDG_OK;
  for (int kern = 0; kern < 2 && rc >= 0; ++kern)
    for (int pr = 0; pr < (f32 ? 2 : 1) && rc >= 0; ++pr) {
      double best = 1e300;
      int bestv = 0;
      for (int v = 0; v < nv && rc >= 0; ++v) {
        auto launch = [&]() {
          if (pr == 0)
            return kern == 0 ? sip_apply(P->M, P->k, P->nb, P->eta, P->cg_r, P->cg_p, P->s, v)
                             : sip_residual(P->M, P->k, P->nb, P->eta, P->cg_z, P->cg_r, P->cg_p, P->s, v);
          return kern == 0 ? sip_apply_f32(P->M, P->k, P->nb, P->eta, P->fx, P->fr, P->s, v)
                           : sip_residual_f32(P->M, P->k, P->nb, P->eta, P->fb, P->fx, P->fr, P->s, v);
        };
        for (int w = 0; w < 2 && rc >= 0; ++w) rc = launch();
        if (rc < 0) break;
        if (hipEventRecord(e0, P->s) != hipSuccess) rc = SDG_ERR_DEVICE;
        for (int r = 0; r < reps && rc >= 0; ++r) rc = launch();
        if (rc < 0) break;
        float ms = 0.f;
        if (hipEventRecord(e1, P->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          set_error("event timing failed during autotuning");
          rc = SDG_ERR_DEVICE;
          break;
        }
        const double t = 1e3 * ms / reps;
        if (t < best) {
          best = t;
          bestv = v;
        }
      }
      if (rc < 0) break;
      P->tile[kern][pr] = bestv;
      drop_graphs(P);
      if (variants) variants[kern * 2 + pr] = bestv;
      if (us) us[kern * 2 + pr] = best;
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tune[tune_key(P, kern, pr)] = bestv;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!f32 && rc >= 0) {
    if (variants) variants[1] = variants[3] = -1;
    if (us) us[1] = us[3] = 0.0;
  }
  return rc;
}

int sdg_trace_enable(sdg_ctx* ctx, int on) {
  if (!ctx) {
    set_error("NULL context");
    return SDG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(ctx->trace_mu);
  if (on) {
    for (auto& r : ctx->pending) {
      ctx->ev_pool.push_back(r.a);
      ctx->ev_pool.push_back(r.b);
    }
    ctx->pending.clear();
    for (int c = 0; c < SDG_TRACE_CLASSES; ++c) {
      ctx->tr_n[c] = 0;
      ctx->tr_ms[c] = ctx->tr_bytes[c] = 0.0;
    }
  }
  ctx->trace = on != 0;
  return SDG_OK;
}

int sdg_trace_read(sdg_ctx* ctx, int kclass, int64_t* launches, double* total_ms, double* bytes) {
  if (!ctx || kclass < 0 || kclass >= SDG_TRACE_CLASSES) {
    set_error("invalid context or kernel class");
    return SDG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(ctx->trace_mu);
  for (auto& r : ctx->pending) {
    SDG_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    SDG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    ctx->tr_n[r.cls] += 1;
    ctx->tr_ms[r.cls] += ms;
    ctx->tr_bytes[r.cls] += r.bytes;
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->pending.clear();
  if (launches) *launches = ctx->tr_n[kclass];
  if (total_ms) *total_ms = ctx->tr_ms[kclass];
  if (bytes) *bytes = ctx->tr_bytes[kclass];
  return SDG_OK;
}

int sdg_uniform_pm1(sdg_ctx* ctx, uint64_t seed, int64_t n, double* out, void* stream) {
  if (!ctx || !out || n < 0) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  return uniform_pm1(seed, n, out, (hipStream_t)stream);
}

}  // extern "C"

namespace sdg {
int ctx_combine(sdg_ctx* c, int on) {
  if (on) {
    if (!c->comb) c->comb = new SdgCombiner();
    return SDG_OK;
  }
  delete c->comb;  // no solve may be running (the server's workers have stopped)
  c->comb = nullptr;
  return SDG_OK;
}
void ctx_combine_stats(sdg_ctx* c, int64_t* launches, int64_t* combined, int* max_width, int64_t* graphs) {
  SdgCombiner* C = c->comb;
  if (!C) return;
  std::lock_guard<std::mutex> g(C->mu);
  if (launches) *launches = C->launches;
  if (combined) *combined = C->combined;
  if (max_width) *max_width = C->max_width;
  if (graphs) *graphs = C->G.built;
}
void* ctx_alloc(sdg_ctx* c, size_t bytes) {
  void* p = nullptr;
  return ctx_get(c, cache_size(bytes), &p) < 0 ? nullptr : p;
}
void ctx_release(sdg_ctx* c, void* p, size_t bytes) { ctx_put(c, p, cache_size(bytes)); }
}  // namespace sdg
