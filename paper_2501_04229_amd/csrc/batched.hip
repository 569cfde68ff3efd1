// Batched (alpha, omega) sweep: many systems of uneven size times up to 16
// parameter trials each, solved in one persistent launch captured in a HIP
// graph.  Each block pulls (system, trial) units from a device queue, largest
// systems first, and runs the whole refinement loop of Algorithm 1 on that
// unit with block-local synchronisation (solve_body.h with BlockRed): no
// device-wide barrier, no host round trip, per-unit iteration records.  This
// is the parameter sweep behind the predictor's training set (Section 3.3.2
// generates its training set from small systems of the same structure).
//
// The threads per block are chosen by a short timed trial of each candidate
// (one sweep of every unit) and cached per batch shape.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <numeric>
#include <vector>

#include "solve_body.h"

namespace gadi {

gadi_status ensure_workspace(System& s);
gadi_status ensure_fp32_public(System& s);

struct BatchSys {
  int n, npad;
  const int32_t* slice_ptr;
  const int32_t* col;
  const int32_t* slice_dia;
  const int32_t* dia_off;
  const double* a_off;
  const double* a_diag;
  const void* h_off;
  const void* s_off;
  const void* h_diag;
  const double* b;    // [npad], zero padded
  long long xoff;     // offset of trial 0's solution in the output buffer, -1 if not wanted
};

struct BatchArgs {
  const BatchSys* sys;
  const int* order;   // unit ids, largest systems first
  int nunits, ntrial, nsys;
  int grid_per_system;
  const double* alpha;
  const double* omega;
  double tol, eps;
  int maxit_out, maxit_in;
  char* ws;           // per-block workspace
  size_t ws_stride;
  int* queue;
  DevInfo* info;      // [nunits], indexed by unit id
  double* xout;
  unsigned long long* best_work;  // [nsys] or null: prune dominated trials
};

static __host__ __device__ inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <class Mode, int BLOCK>
__global__ void __launch_bounds__(BLOCK) batched_kernel(BatchArgs ba) {
  __shared__ int sh_k;
  char* ws = ba.ws + ba.ws_stride * blockIdx.x;
  for (;;) {
    if (threadIdx.x == 0) sh_k = atomicAdd(ba.queue, 1);
    __syncthreads();
    const int k = sh_k;
    __syncthreads();
    if (k >= ba.nunits) break;
    const int u = ba.order[k];
    const int si = u / ba.ntrial, ti = u % ba.ntrial;
    const BatchSys S = ba.sys[si];
    const size_t vb = align256((size_t)S.npad * sizeof(double));
    SolveArgs a{};
    a.n = S.n;
    a.npad = S.npad;
    a.ntiles = S.npad / BLOCK;
    a.maxit_out = ba.maxit_out;
    a.maxit_in = ba.maxit_in;
    a.hist_cap = 0;
    a.slice_ptr = S.slice_ptr;
    a.col = S.col;
    a.slice_dia = S.slice_dia;
    a.dia_off = S.dia_off;
    a.a_off = S.a_off;
    a.a_diag = S.a_diag;
    a.h_off = S.h_off;
    a.s_off = S.s_off;
    a.h_diag = S.h_diag;
    a.b = S.b;
    double* const xw = (double*)ws;
    a.x = xw;
    a.r = ws + vb;
    a.z = ws + 2 * vb;
    a.w = ws + 3 * vb;
    for (int v = 0; v < 8; ++v) a.v[v] = ws + (4 + v) * vb;
    const int gi = ba.grid_per_system ? u : ti;
    a.alpha = ba.alpha[gi];
    a.omega = ba.omega[gi];
    a.tol = ba.tol;
    a.eps_h = ba.eps;
    a.eps_s = ba.eps;
    a.hist = nullptr;
    a.prune = ba.best_work ? ba.best_work + si : nullptr;
    for (int i = threadIdx.x; i < S.npad; i += BLOCK) xw[i] = 0.0;
    __syncthreads();
    const long long t_start = wall_clock64();
    BlockRed<BLOCK> red;
    DevInfo r{};
    const PatGeneric pat{Pattern{a.slice_ptr, a.col, a.slice_dia, a.dia_off, a.n - 1}};
    (void)solve_body<Mode, BLOCK, false, 1>(a, red, pat, 0, S.npad / BLOCK, r);
    if (threadIdx.x == 0) {
      r.barriers = red.barriers;
      r.barrier_ticks = wall_clock64() - t_start;  // the unit's wall-clock ticks
      ba.info[u] = r;
    }
    if (ti == 0 && S.xoff >= 0)
      for (int i = threadIdx.x; i < S.n; i += BLOCK) ba.xout[S.xoff + i] = xw[i];
    __syncthreads();
  }
}

// Queue and pruning bounds start fresh in every launch (a kernel, not a memset,
// so the launch can be captured in a graph).
__global__ void reset_batch_kernel(int* queue, unsigned long long* best, int nsys) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
  if (best)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nsys; i += gridDim.x * blockDim.x) best[i] = ~0ull;
}

template <class Mode, int BLOCK>
static gadi_status occupancy_t(int* nb) {
  GADI_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, batched_kernel<Mode, BLOCK>, BLOCK, 0));
  if (*nb < 1) *nb = 1;
  return GADI_OK;
}

// Resident blocks of the batched kernel for a block size, bounded by `cap`.
static gadi_status batched_blocks(int prec, int block, int cap, int cus, int* G) {
  int nb = 1;
  gadi_status st = GADI_EINVAL;
#define OCC(M)                                                 \
  switch (block) {                                             \
    case 256: st = occupancy_t<M, 256>(&nb); break;            \
    case 512: st = occupancy_t<M, 512>(&nb); break;            \
    case 1024: st = occupancy_t<M, 1024>(&nb); break;          \
  }
  if (prec == GADI_PREC_FP16_IR) {
    OCC(ModeF16)
  } else if (prec == GADI_PREC_FP32_IR) {
    OCC(ModeF32)
  } else {
    OCC(ModeF64)
  }
#undef OCC
  if (st != GADI_OK) return st;
  long long g = (long long)nb * cus;
  if (g > cap) g = cap;
  *G = (int)(g < 1 ? 1 : g);
  return GADI_OK;
}

template <class Mode, int BLOCK>
static gadi_status launch_batched_t(const BatchArgs& ba, int G, hipStream_t stream) {
  hipLaunchKernelGGL(reset_batch_kernel, dim3(1), dim3(256), 0, stream, ba.queue, ba.best_work, ba.nsys);
  hipLaunchKernelGGL((batched_kernel<Mode, BLOCK>), dim3((unsigned)G), dim3(BLOCK), 0, stream, ba);
  GADI_HIP_CHECK(hipGetLastError());
  return GADI_OK;
}

template <class Mode>
static gadi_status launch_batched_mode(const BatchArgs& ba, int block, int G, hipStream_t st) {
  switch (block) {
    case 256: return launch_batched_t<Mode, 256>(ba, G, st);
    case 512: return launch_batched_t<Mode, 512>(ba, G, st);
    case 1024: return launch_batched_t<Mode, 1024>(ba, G, st);
  }
  return GADI_EINVAL;
}

static gadi_status launch_batched(int prec, const BatchArgs& ba, int block, int G, hipStream_t st) {
  if (prec == GADI_PREC_FP16_IR) return launch_batched_mode<ModeF16>(ba, block, G, st);
  if (prec == GADI_PREC_FP32_IR) return launch_batched_mode<ModeF32>(ba, block, G, st);
  return launch_batched_mode<ModeF64>(ba, block, G, st);
}

// Record + launch through a HIP graph (captured once per call).
static gadi_status run_graph(int prec, const BatchArgs& ba, int block, int G, hipStream_t stream) {
  hipStream_t cs = stream;
  bool own = false;
  if (!cs) {
    GADI_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    own = true;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  gadi_status st = GADI_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = launch_batched(prec, ba, block, G, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (st == GADI_OK && e2 != hipSuccess) st = fail_hip(e2, "hipStreamEndCapture", __FILE__, __LINE__);
  } else {
    st = fail_hip(e, "hipStreamBeginCapture", __FILE__, __LINE__);
  }
  if (st == GADI_OK) {
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (e != hipSuccess) st = fail_hip(e, "graph launch", __FILE__, __LINE__);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (own) (void)hipStreamDestroy(cs);
  return st;
}

static std::map<std::tuple<int, int, int>, int> g_batched_block;  // (prec, log2 max npad, nunits bucket)

}  // namespace gadi

using namespace gadi;

extern "C" gadi_status gadi_ir_solve_batched(gadi_handle* const* hs, int32_t nsys, const double* const* b,
                                             double* const* x, const double* alpha, const double* omega,
                                             int32_t ntrial, double tol, const gadi_options* opts,
                                             gadi_solve_info* info) {
  if (!hs || !b || !alpha || !omega || !info || nsys < 1 || ntrial < 1 || ntrial > 16 || !(tol >= 0.0))
    return GADI_EINVAL;
  gadi_options o;
  if (opts) o = *opts;
  else gadi_default_options(&o, GADI_PREC_FP16_IR);
  const int ngrid = o.grid_per_system ? nsys * ntrial : ntrial;
  for (int t = 0; t < ngrid; ++t)
    if (!(alpha[t] > 0.0) || !std::isfinite(alpha[t]) || !(omega[t] >= 0.0 && omega[t] < 2.0)) return GADI_EINVAL;
  if (o.prec < GADI_PREC_FP64 || o.prec > GADI_PREC_FP32_IR || !(o.eps_inner > 0.0) || o.eps_inner >= 1.0 ||
      o.maxit_outer < 0 || o.maxit_inner < 1 || o.on_device)
    return GADI_EINVAL;
  for (int s = 0; s < nsys; ++s)
    if (!hs[s] || !b[s]) return GADI_EINVAL;
  hipStream_t stream = hs[0]->sys.stream;
  const int nunits = nsys * ntrial;
  std::vector<BatchSys> hsys(nsys);
  int max_npad = 0;
  long long xtotal = 0;
  std::vector<long long> nsl(nsys);
  for (int s = 0; s < nsys; ++s) {
    System& S = hs[s]->sys;
    if (o.prec == GADI_PREC_FP32_IR) {
      gadi_status st = ensure_fp32_public(S);
      if (st != GADI_OK) return st;
    }
    BatchSys& d = hsys[s];
    d.n = S.n;
    d.npad = S.npad;
    d.slice_ptr = S.slice_ptr;
    d.col = S.col;
    d.slice_dia = S.slice_dia;
    d.dia_off = S.dia_off;
    d.a_off = S.a_off;
    d.a_diag = S.a_diag;
    if (o.prec == GADI_PREC_FP16_IR) {
      d.h_off = S.h_off16;
      d.s_off = S.s_off16;
      d.h_diag = S.h_diag16;
    } else if (o.prec == GADI_PREC_FP32_IR) {
      d.h_off = S.h_off32;
      d.s_off = S.s_off32;
      d.h_diag = S.h_diag32;
    } else {
      d.h_off = S.h_off64;
      d.s_off = S.s_off64;
      d.h_diag = S.h_diag64;
    }
    d.xoff = (x && x[s]) ? xtotal : -1;
    if (x && x[s]) xtotal += S.n;
    max_npad = std::max(max_npad, S.npad);
    nsl[s] = S.nslots + S.npad;
  }
  // right-hand sides, zero padded, in one device buffer
  std::vector<size_t> boff(nsys);
  size_t btotal = 0;
  for (int s = 0; s < nsys; ++s) {
    boff[s] = btotal;
    btotal += (size_t)hsys[s].npad;
  }
  // units largest system first; trials of a system stay together
  std::vector<int> sys_order(nsys);
  std::iota(sys_order.begin(), sys_order.end(), 0);
  std::stable_sort(sys_order.begin(), sys_order.end(), [&](int p, int q) { return nsl[p] > nsl[q]; });
  std::vector<int> order;
  order.reserve(nunits);
  for (int s : sys_order)
    for (int t = 0; t < ntrial; ++t) order.push_back(s * ntrial + t);

  const size_t vb = align256((size_t)max_npad * sizeof(double));
  const size_t ws_stride = 12 * vb;
  int cus = 0, dev = 0;
  GADI_HIP_CHECK(hipGetDevice(&dev));
  GADI_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // resident blocks: bounded by 8 per compute unit, the unit count and a
  // 16 GiB workspace budget
  const long long budget = 16ll << 30;
  const int cap = (int)std::max(1ll, std::min<long long>({(long long)nunits, (long long)cus * 8,
                                                          budget / (long long)ws_stride}));

  double *db = nullptr, *dal = nullptr, *dom = nullptr, *dx = nullptr;
  BatchSys* dsys = nullptr;
  int *dorder = nullptr, *dq = nullptr;
  unsigned long long* dbest = nullptr;
  DevInfo* dinfo = nullptr;
  char* dws = nullptr;
  gadi_status st = GADI_OK;
  auto cleanup = [&]() {
    void* ps[] = {db, dal, dom, dx, dsys, dorder, dq, dinfo, dws, dbest};
    for (void* p : ps)
      if (p) (void)hipFree(p);
  };
#define BCHECK(expr)                                                \
  do {                                                              \
    hipError_t e_ = (expr);                                         \
    if (e_ != hipSuccess) {                                         \
      st = fail_hip(e_, #expr, __FILE__, __LINE__);                 \
      cleanup();                                                    \
      return st;                                                    \
    }                                                               \
  } while (0)
  BCHECK(hipMalloc((void**)&db, sizeof(double) * btotal));
  BCHECK(hipMemset(db, 0, sizeof(double) * btotal));
  for (int s = 0; s < nsys; ++s) {
    BCHECK(hipMemcpy(db + boff[s], b[s], sizeof(double) * hsys[s].n, hipMemcpyHostToDevice));
    hsys[s].b = db + boff[s];
  }
  BCHECK(hipMalloc((void**)&dsys, sizeof(BatchSys) * nsys));
  BCHECK(hipMemcpy(dsys, hsys.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice));
  BCHECK(hipMalloc((void**)&dorder, sizeof(int) * nunits));
  BCHECK(hipMemcpy(dorder, order.data(), sizeof(int) * nunits, hipMemcpyHostToDevice));
  BCHECK(hipMalloc((void**)&dal, sizeof(double) * ngrid));
  BCHECK(hipMalloc((void**)&dom, sizeof(double) * ngrid));
  BCHECK(hipMemcpy(dal, alpha, sizeof(double) * ngrid, hipMemcpyHostToDevice));
  BCHECK(hipMemcpy(dom, omega, sizeof(double) * ngrid, hipMemcpyHostToDevice));
  BCHECK(hipMalloc((void**)&dq, sizeof(int)));
  if (o.prune_dominated) BCHECK(hipMalloc((void**)&dbest, sizeof(unsigned long long) * nsys));
  BCHECK(hipMalloc((void**)&dinfo, sizeof(DevInfo) * nunits));
  BCHECK(hipMemset(dinfo, 0, sizeof(DevInfo) * nunits));
  BCHECK(hipMalloc((void**)&dx, sizeof(double) * (xtotal ? xtotal : 1)));
  BCHECK(hipMalloc((void**)&dws, ws_stride * cap));

  BatchArgs ba{};
  ba.sys = dsys;
  ba.order = dorder;
  ba.nunits = nunits;
  ba.ntrial = ntrial;
  ba.nsys = nsys;
  ba.grid_per_system = o.grid_per_system ? 1 : 0;
  ba.alpha = dal;
  ba.omega = dom;
  ba.tol = tol;
  ba.eps = o.eps_inner;
  ba.maxit_out = o.maxit_outer;
  ba.maxit_in = o.maxit_inner;
  ba.ws = dws;
  ba.ws_stride = ws_stride;
  ba.queue = dq;
  ba.info = dinfo;
  ba.xout = dx;
  ba.best_work = dbest;

  // threads per block: env override, cached choice, or a timed one-sweep trial
  int lg = 0;
  while ((1 << lg) < max_npad) ++lg;
  const auto key = std::make_tuple((int)o.prec, lg, nunits >= 256 ? 2 : (nunits >= 32 ? 1 : 0));
  int block = 0;
  if (const char* eb = std::getenv("GADI_BATCH_BLOCK")) block = std::atoi(eb);
  if (!block) {
    auto it = g_batched_block.find(key);
    if (it != g_batched_block.end()) block = it->second;
  }
  if (!block) {
    hipEvent_t e0, e1;
    BCHECK(hipEventCreate(&e0));
    BCHECK(hipEventCreate(&e1));
    BatchArgs probe = ba;
    probe.maxit_out = ba.maxit_out < 1 ? ba.maxit_out : 1;
    double best = 1e300;
    for (int cand : {256, 512, 1024}) {
      int G = 1;
      if ((st = batched_blocks(o.prec, cand, cap, cus, &G)) != GADI_OK) break;
      BCHECK(hipEventRecord(e0, stream));
      st = launch_batched(o.prec, probe, cand, G, stream);
      if (st != GADI_OK) break;
      BCHECK(hipEventRecord(e1, stream));
      BCHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      BCHECK(hipEventElapsedTime(&ms, e0, e1));
      if (std::getenv("GADI_DEBUG")) std::fprintf(stderr, "gadi: batched tune block %d: %.3f ms\n", cand, ms);
      if (ms < best) {
        best = ms;
        block = cand;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GADI_OK) {
      cleanup();
      return st;
    }
    g_batched_block[key] = block;
  }

  hipEvent_t t0, t1;
  BCHECK(hipEventCreate(&t0));
  BCHECK(hipEventCreate(&t1));
  int G = 1;
  if ((st = batched_blocks(o.prec, block, cap, cus, &G)) != GADI_OK) {
    cleanup();
    return st;
  }
  BCHECK(hipEventRecord(t0, stream));
  st = run_graph(o.prec, ba, block, G, stream);
  BCHECK(hipEventRecord(t1, stream));
  BCHECK(hipEventSynchronize(t1));
  float total_ms = 0.f;
  BCHECK(hipEventElapsedTime(&total_ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != GADI_OK) {
    cleanup();
    return st;
  }
  std::vector<DevInfo> hinfo(nunits);
  BCHECK(hipMemcpy(hinfo.data(), dinfo, sizeof(DevInfo) * nunits, hipMemcpyDeviceToHost));
  for (int s = 0; s < nsys; ++s)
    if (hsys[s].xoff >= 0)
      BCHECK(hipMemcpy(x[s], dx + hsys[s].xoff, sizeof(double) * hsys[s].n, hipMemcpyDeviceToHost));
  int rate = 0;
  BCHECK(hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev));
  gadi_status worst = GADI_OK;
  for (int u = 0; u < nunits; ++u) {
    const DevInfo& r = hinfo[u];
    gadi_solve_info& out = info[u];
    out.status = r.status;
    out.outer_sweeps = r.sweeps;
    out.inner_H = r.inner_h;
    out.inner_S = r.inner_s;
    out.relres = r.relres;
    out.seconds = (double)r.barrier_ticks / ((rate > 0 ? rate : 100000) * 1000.0);
    out.alpha = alpha[o.grid_per_system ? u : u % ntrial];
    out.omega = omega[o.grid_per_system ? u : u % ntrial];
    out.fell_back = 0;
    out.barriers = r.barriers;
    out.barrier_seconds = total_ms * 1e-3;  // whole batch: device time of the graph launch
    if (r.status == GADI_EMAXIT && worst == GADI_OK) worst = GADI_EMAXIT;
  }
  cleanup();
#undef BCHECK
  return worst;
}
