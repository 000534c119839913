// Host runtime and C ABI (include/lbm.h) of the adaptive D2Q21 step (and of
// the reference model, D2Q49 with 13 constraints, on the same framework).
//
// A context owns no device memory: it carves the caller's workspace into two
// population buffers (A/B, 2 x 21 or 2 x 49 planes each), two lattice-tag arrays, the
// diagnostics record and the reduction partials, and enqueues every kernel
// on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "lbm.h"
#include "reference49.hpp"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxBatch = 1024;  // contexts per lbm_step_batched call
static_assert(kMaxBatch <= kMaxJobs, "the batched rebuild's job table holds kMaxJobs");

// Initial-guess table: |u'_x|, |u'_y| in [0, 2] (step 1/32), 1/T in
// [0.5, 1/0.3] (35 levels), 8 floats per point (4.7 MB; 16 floats, 9.5 MB,
// for the 13-constraint set; the states of a flow touch a small part of it).
constexpr int kTabU = 65;
constexpr int kTabS = 35;
constexpr float kTabUmax = 2.0f;
constexpr float kTabSmin = 0.5f;
constexpr float kTabSmax = 1.0f / 0.3f;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Velocities of a constraint set's lattice: D2Q49 for the 13-constraint
// reference model, D2Q21 otherwise.
int lattice_q(int constraints) { return constraints == kM13 ? kQ49 : kQ; }

// Bytes of the initial-guess table of a constraint set (8 floats per grid
// point, 16 for the 13-constraint set).
size_t table_bytes_of(int constraints) {
  return static_cast<size_t>(kTabU) * kTabU * kTabS * (constraints == kM13 ? kRec13 : 8) *
         sizeof(float);
}

// The flexible-Prandtl collision (eq. Shakhov) is on for Pr other than 1
// (0 also means BGK).
bool shakhov_on(const lbm_config* c) { return c->prandtl != 0.0 && c->prandtl != 1.0; }

struct Layout {
  size_t pop_bytes;  // one buffer: f and g, Q planes each
  size_t tag_bytes;
  size_t diag_off, part_off, sums_off, table_off, total;
  size_t off_pop[2], off_tag[2];
  size_t mac_off, mask_off, list_off, count_off;  // carried from step to step
  size_t seen_off, pair_off;                      // the rebuild queue (D2Q21)
  long long pair_cap;
  size_t batch_off;                               // job table of a batched call
  size_t keys_off;                                // failure words of a batched call
  int nparts;
};

bool config_ok(const lbm_config* c) {
  if (!c) return false;
  const long long N = static_cast<long long>(c->nx) * c->ny;
  const long long es = c->precision == LBM_FP64 ? 8 : 4;
  return c->nx >= 1 && c->ny >= 1 && N < (1ll << 31) && N * es < (1ll << 32) &&
         (c->precision == LBM_FP64 || c->precision == LBM_FP32_STORE) && c->gamma > 1.0 &&
         std::isfinite(c->gamma) && c->nu >= 0.0 && std::isfinite(c->nu) &&
         c->shift_mode >= 0 && c->shift_mode <= 3 && c->shift_halfwidth >= 0.5 &&
         (c->shift_mode != LBM_SHIFT_NEIGHBOURHOOD ||
          (c->shift_halfwidth < 1.0 && c->constraints == kM)) &&
         c->shift_halfwidth < 8.0 && c->newton_tol > 0.0 && c->newton_max_iter >= 1 &&
         c->newton_max_iter <= 1000 && c->max_abs_shift >= 0 && c->max_abs_shift <= 12 &&
         std::abs(c->fixed_ux) <= c->max_abs_shift && std::abs(c->fixed_uy) <= c->max_abs_shift &&
         (c->constraints == kM || c->constraints == 4 ||
          (c->constraints == kM13 && c->precision == LBM_FP64 &&
           c->shift_mode != LBM_SHIFT_NEIGHBOURHOOD)) &&
         c->prandtl >= 0.0 && c->prandtl < 1e3 &&
         (!shakhov_on(c) || (c->prandtl >= 1e-2 && c->constraints != 4 &&
                             c->shift_mode != LBM_SHIFT_NEIGHBOURHOOD)) &&
         (c->fallback == 0 || (c->fallback == 1 && !shakhov_on(c)));
}

Layout layout(const lbm_config* c) {
  Layout L{};
  const size_t N = static_cast<size_t>(c->nx) * c->ny;
  const size_t es = c->precision == LBM_FP64 ? sizeof(double) : sizeof(float);
  const size_t Q = static_cast<size_t>(lattice_q(c->constraints));
  L.pop_bytes = align_up(2 * Q * N * es);
  L.tag_bytes = align_up(N * sizeof(int));
  L.nparts = static_cast<int>((N + kBlock - 1) / kBlock);
  size_t off = 0;
  for (int b = 0; b < 2; ++b) {
    L.off_pop[b] = off;
    off += L.pop_bytes;
  }
  for (int b = 0; b < 2; ++b) {
    L.off_tag[b] = off;
    off += L.tag_bytes;
  }
  L.mac_off = off;
  off += align_up(4 * N * (LBM_CARRY_FP64 ? sizeof(double) : es));
  L.mask_off = off;  // one link bit per velocity
  off += align_up(N * (Q > 32 ? sizeof(unsigned long long) : sizeof(unsigned)));
  L.list_off = off;
  off += align_up(N * sizeof(int));
  L.count_off = off;
  off += align_up(4 * sizeof(unsigned));  // list and pair-queue lengths
  // rebuild queue: a seen mask per node and room for the (source, lattice)
  // pairs: 21 N on grids below 65536 nodes (a pair per link at most, so it
  // cannot fill), else 4 N (four pairs per node on average; the flows here
  // queue about 0.01-0.05 per node)
  L.seen_off = off;
  off += align_up(N * sizeof(unsigned long long));
  L.pair_cap = static_cast<long long>(N < 65536 ? 21 * N : 4 * N);
  L.pair_off = off;
  off += align_up(static_cast<size_t>(L.pair_cap) * sizeof(unsigned long long));
  L.batch_off = off;
  off += align_up(kMaxBatch * sizeof(JobArgs));
  L.keys_off = off;
  off += align_up(kMaxBatch * sizeof(unsigned long long));
  L.diag_off = off;
  off += align_up(sizeof(DevDiag));
  L.part_off = off;
  off += align_up(static_cast<size_t>(L.nparts) * 4 * sizeof(double));
  L.sums_off = off;
  off += align_up(4 * sizeof(double));
  L.table_off = off;
  off += align_up(table_bytes_of(c->constraints));
  L.total = off;
  return L;
}

}  // namespace

// A chunk of steps recorded as a HIP graph: kernel nodes only, for one
// buffer parity (the chunk is even, so replays keep it).
struct StepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int chunk = 0;
  int cur = -1;     // buffer holding the state when a replay starts
  int parity = -1;  // steps done mod 2 when a replay starts
  std::vector<StepArgs> step_args;  // kernel arguments of the nodes
  std::vector<RebuildArgs> rebuild_args;

  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    chunk = 0;
    cur = parity = -1;
    step_args.clear();
    rebuild_args.clear();
  }
};

// The launches of a batched quantum recorded as a HIP graph (kernel nodes
// only), kept by the batch's first context.  The kernels read the job
// table at a fixed device address, so a replay needs only a fresh table;
// the graph is rebuilt when the launch shape changes (job count, steps of
// the quantum, grid sizes, schedule).
struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* jobs = nullptr;
  int njobs = -1, most = -1, B = 0, remap = -1;
  unsigned step_grid = 0, rebuild_grid = 0;
  const void* step_fn = nullptr;
  const void* rebuild_fn = nullptr;
  std::vector<int> s_args;
  int builds = 0, replays = 0;

  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    njobs = most = remap = -1;
  }
};

struct lbm_ctx {
  lbm_config cfg;
  Layout lay;
  hipStream_t stream;
  int device;
  char* ws;
  int cur;  // buffer holding the current state
  bool initialized;
  int64_t steps_done;
  Grid grid;
  Phys phys;
  GuessTable table;
  int nblocks;       // 256-lane blocks (init, exports, reductions)
  lbm_schedule sched;  // step_block, tiles, remap, rebuild workgroups (resolved)
  StepGraph graphs[2];  // by buffer parity
  BatchGraph batch_graph;  // quanta of batches this context leads

  ~lbm_ctx() {
    for (auto& g : graphs) g.reset();
    batch_graph.reset();
  }
  int step_tiles() const {
    return static_cast<int>((grid.N + sched.step_block - 1) / sched.step_block);
  }

  void* f(int b) const { return ws + lay.off_pop[b]; }
  void* g(int b) const {
    const size_t es = cfg.precision == LBM_FP64 ? sizeof(double) : sizeof(float);
    return ws + lay.off_pop[b] + lattice_q(cfg.constraints) * static_cast<size_t>(grid.N) * es;
  }
  int* tag(int b) const { return reinterpret_cast<int*>(ws + lay.off_tag[b]); }
  Carry carry() const {
    Carry k;
    k.mask = reinterpret_cast<unsigned*>(ws + lay.mask_off);
    k.mac = ws + lay.mac_off;
    k.list = reinterpret_cast<int*>(ws + lay.list_off);
    k.counters = reinterpret_cast<unsigned*>(ws + lay.count_off);
    k.seen = reinterpret_cast<unsigned long long*>(ws + lay.seen_off);
    k.pairs = reinterpret_cast<unsigned long long*>(ws + lay.pair_off);
    k.pair_cap = lay.pair_cap;
    return k;
  }
  DevDiag* diag() const { return reinterpret_cast<DevDiag*>(ws + lay.diag_off); }
  double* parts() const { return reinterpret_cast<double*>(ws + lay.part_off); }
  double* sums() const { return reinterpret_cast<double*>(ws + lay.sums_off); }
};

#define HIP_TRY(expr)                       \
  do {                                      \
    if ((expr) != hipSuccess) return LBM_ERR_HIP; \
  } while (0)

namespace {

// Device-side clean diagnostics record (fail_key = ~0, counters 0) and
// empty rebuild lists and queues.
__global__ void diag_reset_kernel(DevDiag* d, unsigned* list_counters) {
  const int i = threadIdx.x;
  unsigned long long* w = reinterpret_cast<unsigned long long*>(d);
  const int n = static_cast<int>(sizeof(DevDiag) / sizeof(unsigned long long));
  if (i < n) w[i] = (i == 0) ? ~0ull : 0ull;
  if (i < 4) list_counters[i] = 0u;
}

// Device entry of the step kernel for a storage type, pass and block size;
// nullptr for a combination that is not built.
template <typename S, int B>
const void* step_fn_of(bool tiled) {
  return tiled ? reinterpret_cast<const void*>(&step_kernel<S, true, B, true>)
               : reinterpret_cast<const void*>(&step_kernel<S, true, B, false>);
}

// Device entry of the step kernel for a storage type, pass, block size,
// tiling and constraint count; nullptr for a combination that is not built
// (the four-constraint set is built for 64-lane untiled blocks only).
const void* step_kernel_fn(int precision, bool stream_pass, int block, bool tiled, int M,
                           bool nbh = false, bool pr = false) {
  const bool f64 = precision == LBM_FP64;
  if (pr && M != kM13) {  // flexible Prandtl number: default schedule, 8 constraints
    if (block != 64 || tiled || M != kM || nbh) return nullptr;
    if (f64)
      return stream_pass
                 ? reinterpret_cast<const void*>(&step_kernel<double, true, 64, false, kM, false, true>)
                 : reinterpret_cast<const void*>(&step_kernel<double, false, 64, false, kM, false, true>);
    return stream_pass
               ? reinterpret_cast<const void*>(&step_kernel<float, true, 64, false, kM, false, true>)
               : reinterpret_cast<const void*>(&step_kernel<float, false, 64, false, kM, false, true>);
  }
  if (M == kM13) {  // reference model: FP64, 64-lane untiled blocks
    if (!f64 || block != 64 || tiled || nbh) return nullptr;
    if (pr)
      return stream_pass ? reinterpret_cast<const void*>(&step49_kernel<true, true>)
                         : reinterpret_cast<const void*>(&step49_kernel<false, true>);
    return stream_pass ? reinterpret_cast<const void*>(&step49_kernel<true>)
                       : reinterpret_cast<const void*>(&step49_kernel<false>);
  }
  if (nbh) {  // shift mode 3: default schedule, 8 constraints
    if (block != 64 || tiled || M != kM) return nullptr;
    if (f64)
      return stream_pass ? reinterpret_cast<const void*>(&step_kernel<double, true, 64, false, kM, true>)
                         : reinterpret_cast<const void*>(&step_kernel<double, false, 64, false, kM, true>);
    return stream_pass ? reinterpret_cast<const void*>(&step_kernel<float, true, 64, false, kM, true>)
                       : reinterpret_cast<const void*>(&step_kernel<float, false, 64, false, kM, true>);
  }
  if (M == 4) {
    if (block != 64 || tiled) return nullptr;
    if (f64)
      return stream_pass ? reinterpret_cast<const void*>(&step_kernel<double, true, 64, false, 4>)
                         : reinterpret_cast<const void*>(&step_kernel<double, false, 64, false, 4>);
    return stream_pass ? reinterpret_cast<const void*>(&step_kernel<float, true, 64, false, 4>)
                       : reinterpret_cast<const void*>(&step_kernel<float, false, 64, false, 4>);
  }
  if (M != kM) return nullptr;
  if (f64) {
    if (!stream_pass)
      return block == 64 && !tiled ? reinterpret_cast<const void*>(&step_kernel<double, false, 64, false>)
                                   : nullptr;
    switch (block) {
      case 64: return step_fn_of<double, 64>(tiled);
      case 128: return step_fn_of<double, 128>(tiled);
    }
  } else {
    if (!stream_pass)
      return block == 64 && !tiled ? reinterpret_cast<const void*>(&step_kernel<float, false, 64, false>)
                                   : nullptr;
    switch (block) {
      case 64: return step_fn_of<float, 64>(tiled);
      case 128: return step_fn_of<float, 128>(tiled);
      case 256: return step_fn_of<float, 256>(tiled);
    }
  }
  return nullptr;
}

const void* step_batched_fn(int precision, int block, int M) {
  const bool f64 = precision == LBM_FP64;
  if (M == 4) {
    if (block != 64) return nullptr;
    return f64 ? reinterpret_cast<const void*>(&step_batched_kernel<double, 64, 4>)
               : reinterpret_cast<const void*>(&step_batched_kernel<float, 64, 4>);
  }
  if (M != kM) return nullptr;
  if (f64) {
    switch (block) {
      case 64: return reinterpret_cast<const void*>(&step_batched_kernel<double, 64>);
      case 128: return reinterpret_cast<const void*>(&step_batched_kernel<double, 128>);
    }
  } else {
    switch (block) {
      case 64: return reinterpret_cast<const void*>(&step_batched_kernel<float, 64>);
      case 128: return reinterpret_cast<const void*>(&step_batched_kernel<float, 128>);
      case 256: return reinterpret_cast<const void*>(&step_batched_kernel<float, 256>);
    }
  }
  return nullptr;
}

const void* rebuild_fn(int precision, int M, bool pr = false) {
  const bool f64 = precision == LBM_FP64;
  if (M == kM13)
    return !f64 ? nullptr
                : pr ? reinterpret_cast<const void*>(&rebuild49_kernel<true>)
                     : reinterpret_cast<const void*>(&rebuild49_kernel<false>);
  if (pr)
    return M != kM ? nullptr
                   : f64 ? reinterpret_cast<const void*>(&rebuild_kernel<double, kM, true>)
                         : reinterpret_cast<const void*>(&rebuild_kernel<float, kM, true>);
  if (M == 4)
    return f64 ? reinterpret_cast<const void*>(&rebuild_kernel<double, 4>)
               : reinterpret_cast<const void*>(&rebuild_kernel<float, 4>);
  return f64 ? reinterpret_cast<const void*>(&rebuild_kernel<double>)
             : reinterpret_cast<const void*>(&rebuild_kernel<float>);
}

const void* rebuild_batched_fn(int precision, int M) {
  const bool f64 = precision == LBM_FP64;
  if (M == 4)
    return f64 ? reinterpret_cast<const void*>(&rebuild_batched_kernel<double, 4>)
               : reinterpret_cast<const void*>(&rebuild_batched_kernel<float, 4>);
  return f64 ? reinterpret_cast<const void*>(&rebuild_batched_kernel<double>)
             : reinterpret_cast<const void*>(&rebuild_batched_kernel<float>);
}

// One launch of a single-argument kernel, as a direct launch or a graph node.
template <typename Args>
struct Launch {
  const void* fn = nullptr;
  dim3 grid, block;
  Args args;
};

// The step from buffer src into dst; the collide-only pass of the initial
// condition (stream_pass false) always runs one 64-lane tile per workgroup.
Launch<StepArgs> step_launch(const lbm_ctx* c, int src, int dst, bool stream_pass, int step) {
  Launch<StepArgs> L;
  StepArgs& a = L.args;
  a.fin = c->f(src);
  a.gin = c->g(src);
  a.fout = c->f(dst);
  a.gout = c->g(dst);
  a.tin = c->tag(src);
  a.tout = c->tag(dst);
  a.carry = c->carry();
  a.grid = c->grid;
  a.phys = c->phys;
  a.table = c->table;
  a.step = step;
  a.diag = c->diag();
  const int B = stream_pass ? c->sched.step_block : 64;
  a.ntiles = static_cast<int>((c->grid.N + B - 1) / B);
  a.tiles = stream_pass ? c->sched.tiles_per_block : 1;
  a.remap = stream_pass ? c->sched.xcd_remap : 1;
  L.fn = step_kernel_fn(c->cfg.precision, stream_pass, B, a.tiles > 1, c->cfg.constraints,
                        c->cfg.shift_mode == LBM_SHIFT_NEIGHBOURHOOD, shakhov_on(&c->cfg));
  L.grid = dim3(static_cast<unsigned>((a.ntiles + a.tiles - 1) / a.tiles));
  L.block = dim3(B);
  return L;
}

// Rebuilds the mismatched links of step `step` (pulling from buffer src)
// into buffer dst: the queue pass (queue = true), then the rebuild pass.
// No launch (fn nullptr) with one lattice for all nodes.
Launch<RebuildArgs> rebuild_launch(const lbm_ctx* c, int src, int dst, int step, bool queue) {
  Launch<RebuildArgs> L;
  if (c->cfg.shift_mode == LBM_SHIFT_FIXED) return L;
  RebuildArgs& a = L.args;
  a.fout = c->f(dst);
  a.gout = c->g(dst);
  a.tags = c->tag(src);
  a.carry = c->carry();
  a.grid = c->grid;
  a.phys = c->phys;
  a.table = c->table;
  a.step = step;
  a.diag = c->diag();
  // the 49-velocity rebuild takes its receiver list directly
  if (queue)
    L.fn = c->cfg.constraints == kM13 ? nullptr : reinterpret_cast<const void*>(&queue_kernel);
  else
    L.fn = rebuild_fn(c->cfg.precision, c->cfg.constraints, shakhov_on(&c->cfg));
  L.grid = dim3(static_cast<unsigned>(c->sched.rebuild_blocks));
  L.block = dim3(kBlock);
  return L;
}

template <typename Args>
lbm_status enqueue(const Launch<Args>& L, hipStream_t stream) {
  if (!L.fn) return LBM_OK;
  Args a = L.args;
  void* params[] = {&a};
  if (hipLaunchKernel(L.fn, L.grid, L.block, params, 0, stream) != hipSuccess) return LBM_ERR_HIP;
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status launch_step(lbm_ctx* c, int src, int dst, bool stream_pass, int step) {
  const Launch<StepArgs> L = step_launch(c, src, dst, stream_pass, step);
  if (!L.fn) return LBM_ERR_ARG;
  return enqueue(L, c->stream);
}

lbm_status launch_rebuild(lbm_ctx* c, int src, int dst, int step) {
  const lbm_status st = enqueue(rebuild_launch(c, src, dst, step, true), c->stream);
  return st ? st : enqueue(rebuild_launch(c, src, dst, step, false), c->stream);
}

__global__ void set_step_base_kernel(DevDiag* d, unsigned long long base) {
  if (threadIdx.x == 0) d->step_base = base;
}

__global__ void advance_step_base_kernel(DevDiag* d, unsigned long long by) {
  if (threadIdx.x == 0) d->step_base += by;
}

template <typename Args>
lbm_status add_node(hipGraph_t g, hipGraphNode_t* prev, const Launch<Args>& L, Args* stored) {
  hipKernelNodeParams p{};
  void* params[] = {stored};
  p.func = const_cast<void*>(L.fn);
  p.gridDim = L.grid;
  p.blockDim = L.block;
  p.sharedMemBytes = 0;
  p.kernelParams = params;
  p.extra = nullptr;
  hipGraphNode_t node = nullptr;
  if (hipGraphAddKernelNode(&node, g, *prev ? prev : nullptr, *prev ? 1 : 0, &p) != hipSuccess)
    return LBM_ERR_HIP;
  *prev = node;
  return LBM_OK;
}

// Records `chunk` steps starting from the context's current buffer and step
// parity: per step the rebuild (if any) and the step, then the node that
// advances the failure step base by the chunk.  Steps are recorded as
// parity + 1 .. parity + chunk; a replay adds the base set before it.
lbm_status build_graph(lbm_ctx* c, int chunk, StepGraph& G) {
  G.reset();
  const int parity = static_cast<int>(c->steps_done & 1);
  G.step_args.reserve(chunk);
  G.rebuild_args.reserve(2 * chunk);
  if (hipGraphCreate(&G.graph, 0) != hipSuccess) return LBM_ERR_HIP;
  hipGraphNode_t prev = nullptr;
  int cur = c->cur;
  lbm_status st = LBM_OK;
  for (int k = 1; k <= chunk && st == LBM_OK; ++k) {
    const int src = cur, dst = 1 - cur;
    for (int pass = 0; pass < 2 && st == LBM_OK; ++pass) {
      const Launch<RebuildArgs> R = rebuild_launch(c, src, dst, parity + k, pass == 0);
      if (R.fn) {
        G.rebuild_args.push_back(R.args);
        st = add_node(G.graph, &prev, R, &G.rebuild_args.back());
      }
    }
    const Launch<StepArgs> S = step_launch(c, src, dst, true, parity + k);
    if (st == LBM_OK && !S.fn) st = LBM_ERR_ARG;
    if (st == LBM_OK) {
      G.step_args.push_back(S.args);
      st = add_node(G.graph, &prev, S, &G.step_args.back());
    }
    cur = dst;
  }
  if (st == LBM_OK) {
    hipKernelNodeParams p{};
    DevDiag* d = c->diag();
    unsigned long long by = static_cast<unsigned long long>(chunk);
    void* params[] = {&d, &by};
    p.func = reinterpret_cast<void*>(&advance_step_base_kernel);
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.kernelParams = params;
    hipGraphNode_t node = nullptr;
    if (hipGraphAddKernelNode(&node, G.graph, &prev, 1, &p) != hipSuccess) st = LBM_ERR_HIP;
  }
  if (st == LBM_OK && hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0) != hipSuccess)
    st = LBM_ERR_HIP;
  if (st != LBM_OK) {
    G.reset();
    return st;
  }
  G.chunk = chunk;
  G.cur = c->cur;
  G.parity = parity;
  return LBM_OK;
}

// Field by field (padding bytes of caller-built structs are not compared).
bool same_config(const lbm_config& a, const lbm_config& b) {
  return a.nx == b.nx && a.ny == b.ny && a.precision == b.precision && a.gamma == b.gamma &&
         a.nu == b.nu && a.shift_mode == b.shift_mode && a.fixed_ux == b.fixed_ux &&
         a.fixed_uy == b.fixed_uy && a.shift_halfwidth == b.shift_halfwidth &&
         a.newton_tol == b.newton_tol && a.newton_max_iter == b.newton_max_iter &&
         a.max_abs_shift == b.max_abs_shift && a.sensor == b.sensor &&
         a.collect_stats == b.collect_stats && a.constraints == b.constraints &&
         a.prandtl == b.prandtl && a.fallback == b.fallback;
}

// Default and checked schedules.
int default_rebuild_blocks(long long N) {
  return static_cast<int>(std::min<long long>((N + kBlock - 1) / kBlock, 4096));
}

bool schedule_ok(const lbm_ctx* c, const lbm_schedule* s) {
  if (!s) return false;
  const bool tiled = s->tiles_per_block > 1;
  if (!step_kernel_fn(c->cfg.precision, true, s->step_block, tiled, c->cfg.constraints,
                      c->cfg.shift_mode == LBM_SHIFT_NEIGHBOURHOOD, shakhov_on(&c->cfg)))
    return false;
  if (c->cfg.constraints != kM13 && !shakhov_on(&c->cfg) &&
      !step_batched_fn(c->cfg.precision, s->step_block, c->cfg.constraints))
    return false;
  const long long tiles = (c->grid.N + s->step_block - 1) / s->step_block;
  return s->tiles_per_block >= 1 && s->tiles_per_block <= 64 && tiles < (1ll << 31) &&
         (s->xcd_remap == 0 || s->xcd_remap == 1) && s->rebuild_blocks >= 0 &&
         s->rebuild_blocks <= 65535;
}

// Status of a recorded failure word's code.
lbm_status status_of_code(unsigned long long key) {
  const unsigned code = static_cast<unsigned>(key & 7ull);
  if (code == kCodeNewton) return LBM_ERR_NEWTON;
  if (code == kCodeQueueFull) return LBM_ERR_WORKSPACE;
  return LBM_ERR_NONPHYSICAL;
}

lbm_status read_status(lbm_ctx* c, unsigned long long* key_out) {
  unsigned long long key = ~0ull;
  HIP_TRY(hipMemcpyAsync(&key, &c->diag()->fail_key, sizeof key, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (key_out) *key_out = key;
  if (key == ~0ull) return LBM_OK;
  return status_of_code(key);
}

lbm_status init_common(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
                       const double* T, const int8_t* sux, const int8_t* suy) {
  if (!c || !rho || !ux || !uy || !T) return LBM_ERR_ARG;
  if (c->cfg.shift_mode == LBM_SHIFT_STATIC && (!sux || !suy)) return LBM_ERR_ARG;
  hipLaunchKernelGGL(diag_reset_kernel, dim3(1), dim3(64), 0, c->stream, c->diag(),
                     c->carry().counters);
  HIP_TRY(hipMemsetAsync(c->ws + c->lay.seen_off, 0,
                         static_cast<size_t>(c->grid.N) * sizeof(unsigned long long), c->stream));
  InitArgs a;
  a.rho = rho;
  a.ux = ux;
  a.uy = uy;
  a.T = T;
  a.sux = sux;
  a.suy = suy;
  a.fout = c->f(0);
  a.gout = c->g(0);
  a.tout = c->tag(0);
  a.grid = c->grid;
  a.phys = c->phys;
  a.table = c->table;
  a.diag = c->diag();
  if (c->cfg.constraints == kM13) {
    hipLaunchKernelGGL(init49_kernel, dim3(c->nblocks), dim3(kBlock), 0, c->stream, a);
  } else if (c->cfg.constraints == 4) {
    if (c->cfg.precision == LBM_FP64)
      hipLaunchKernelGGL((init_kernel<double, 4>), dim3(c->nblocks), dim3(kBlock), 0, c->stream, a);
    else
      hipLaunchKernelGGL((init_kernel<float, 4>), dim3(c->nblocks), dim3(kBlock), 0, c->stream, a);
  } else if (c->cfg.precision == LBM_FP64) {
    hipLaunchKernelGGL(init_kernel<double>, dim3(c->nblocks), dim3(kBlock), 0, c->stream, a);
  } else {
    hipLaunchKernelGGL(init_kernel<float>, dim3(c->nblocks), dim3(kBlock), 0, c->stream, a);
  }
  HIP_TRY(hipGetLastError());
  lbm_status st = launch_step(c, 0, 1, false, 0);
  if (st) return st;
  c->cur = 1;
  c->steps_done = 0;
  st = read_status(c, nullptr);
  c->initialized = (st == LBM_OK);
  return st;
}

// One queue launch, one rebuild launch and one step launch per step for
// every context of a batch.  dev_jobs / dev_keys: device memory for the job table and the
// failure words (n entries each); host_jobs / host_keys: host staging of
// the same size.
// Records (or reuses) the graph of a quantum's launches in ctxs[0]'s
// batch graph and replays it once.
lbm_status replay_batch_graph(lbm_ctx* c0, JobArgs* dev_jobs, int njobs, int most,
                              const void* step_fn, dim3 step_grid, int B, int remap,
                              const void* rebuild_fn, dim3 rebuild_grid, bool any_rebuild) {
  BatchGraph& G = c0->batch_graph;
  const void* rfn = any_rebuild ? rebuild_fn : nullptr;
  if (!G.exec || G.jobs != dev_jobs || G.njobs != njobs || G.most != most || G.B != B ||
      G.remap != remap || G.step_grid != step_grid.x || G.rebuild_grid != rebuild_grid.x ||
      G.step_fn != step_fn || G.rebuild_fn != rfn) {
    G.reset();
    if (hipGraphCreate(&G.graph, 0) != hipSuccess) return LBM_ERR_HIP;
    G.s_args.resize(most);
    hipGraphNode_t prev = nullptr;
    lbm_status st = LBM_OK;
    JobArgs* jobs = dev_jobs;
    int nj = njobs, rm = remap;
    for (int k = 0; k < most && st == LBM_OK; ++k) {
      G.s_args[k] = k;
      // queue, rebuild, step
      for (int pass = rfn ? 0 : 2; pass < 3 && st == LBM_OK; ++pass) {
        hipKernelNodeParams p{};
        void* rparams[] = {&jobs, &nj, &G.s_args[k]};
        void* sparams[] = {&jobs, &nj, &G.s_args[k], &rm};
        p.func = pass == 0   ? reinterpret_cast<void*>(&queue_batched_kernel)
                 : pass == 1 ? const_cast<void*>(rfn)
                             : const_cast<void*>(step_fn);
        p.gridDim = pass < 2 ? rebuild_grid : step_grid;
        p.blockDim = dim3(pass < 2 ? kBlock : B);
        p.sharedMemBytes = 0;
        p.kernelParams = pass < 2 ? rparams : sparams;
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        if (hipGraphAddKernelNode(&node, G.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) !=
            hipSuccess)
          st = LBM_ERR_HIP;
        prev = node;
      }
    }
    if (st == LBM_OK && hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0) != hipSuccess)
      st = LBM_ERR_HIP;
    if (st != LBM_OK) {
      G.reset();
      return st;
    }
    G.jobs = dev_jobs;
    G.njobs = njobs;
    G.most = most;
    G.B = B;
    G.remap = remap;
    G.step_grid = step_grid.x;
    G.rebuild_grid = rebuild_grid.x;
    G.step_fn = step_fn;
    G.rebuild_fn = rfn;
    G.builds += 1;
  }
  if (hipGraphLaunch(G.exec, c0->stream) != hipSuccess) return LBM_ERR_HIP;
  G.replays += 1;
  return LBM_OK;
}

lbm_status step_batched_common(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n,
                               JobArgs* dev_jobs, unsigned long long* dev_keys,
                               JobArgs* host_jobs, unsigned long long* host_keys,
                               bool graph = false) {
  int32_t most = 0;
  bool any_rebuild = false;
  long long nodes = 0;
  for (int32_t k = 0; k < n; ++k) {
    lbm_ctx* c = ctxs[k];
    if (!c || nsteps[k] < 0) return LBM_ERR_ARG;
    if (c->cfg.shift_mode == LBM_SHIFT_NEIGHBOURHOOD || c->cfg.constraints == kM13 ||
        shakhov_on(&c->cfg))
      return LBM_ERR_ARG;
    if (c->cfg.precision != ctxs[0]->cfg.precision ||
        c->cfg.constraints != ctxs[0]->cfg.constraints || c->stream != ctxs[0]->stream ||
        c->device != ctxs[0]->device)
      return LBM_ERR_ARG;
    for (int32_t m = 0; m < k; ++m)
      if (ctxs[m] == c) return LBM_ERR_ARG;
    if (!c->initialized) return LBM_ERR_STATE;
    most = std::max(most, nsteps[k]);
    any_rebuild = any_rebuild || c->cfg.shift_mode != LBM_SHIFT_FIXED;
    nodes += c->grid.N;
  }
  // job table, blocks of the step launch in job order
  const int B = ctxs[0]->sched.step_block;
  const void* step_fn = step_batched_fn(ctxs[0]->cfg.precision, B, ctxs[0]->cfg.constraints);
  if (!step_fn) return LBM_ERR_ARG;
  long long blocks = 0;
  for (int32_t k = 0; k < n; ++k) {
    lbm_ctx* c = ctxs[k];
    JobArgs& j = host_jobs[k];
    for (int b = 0; b < 2; ++b) {
      j.pop[b] = c->f(b);
      j.tag[b] = c->tag(b);
    }
    j.carry = c->carry();
    j.grid = c->grid;
    j.phys = c->phys;
    j.table = c->table;
    j.diag = c->diag();
    j.cur = c->cur;
    j.step0 = static_cast<int>(c->steps_done);
    j.nsteps = nsteps[k];
    j.block0 = static_cast<int>(blocks);
    j.nblocks = static_cast<int>((c->grid.N + B - 1) / B);
    blocks += j.nblocks;
  }
  if (blocks >= (1ll << 31)) return LBM_ERR_ARG;
  lbm_ctx* c0 = ctxs[0];
  HIP_TRY(hipMemcpyAsync(dev_jobs, host_jobs, n * sizeof(JobArgs), hipMemcpyHostToDevice,
                         c0->stream));
  const dim3 step_grid(static_cast<unsigned>(blocks));
  // queue and rebuild: each workgroup first sums the jobs' counts, so the
  // grid follows the batch's size (one 256-lane workgroup per 2048 nodes)
  // between two and four workgroups per CU
  const dim3 rebuild_grid(
      static_cast<unsigned>(std::clamp<long long>((nodes + 2047) / 2048, 512, 1024)));
  const void* rebuild_batched = rebuild_batched_fn(c0->cfg.precision, c0->cfg.constraints);
  int remap = c0->sched.xcd_remap;
  if (graph && most > 0) {
    const lbm_status gs = replay_batch_graph(c0, dev_jobs, n, most, step_fn, step_grid, B, remap,
                                             rebuild_batched, rebuild_grid, any_rebuild);
    if (gs) return gs;
  } else {
    for (int32_t st = 0; st < most; ++st) {
      int njobs = n, s_arg = st;
      void* rebuild_params[] = {&dev_jobs, &njobs, &s_arg};
      void* step_params[] = {&dev_jobs, &njobs, &s_arg, &remap};
      if (any_rebuild) {
        HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&queue_batched_kernel), rebuild_grid,
                                dim3(kBlock), rebuild_params, 0, c0->stream));
        HIP_TRY(hipLaunchKernel(rebuild_batched, rebuild_grid, dim3(kBlock), rebuild_params, 0,
                                c0->stream));
      }
      HIP_TRY(hipLaunchKernel(step_fn, step_grid, dim3(B), step_params, 0, c0->stream));
      HIP_TRY(hipGetLastError());
    }
  }
  for (int32_t k = 0; k < n; ++k) {
    ctxs[k]->cur ^= (nsteps[k] & 1);
    ctxs[k]->steps_done += nsteps[k];
  }
  // every job's failure word in one copy
  hipLaunchKernelGGL(gather_fail_keys_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     c0->stream, dev_jobs, n, dev_keys);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host_keys, dev_keys, n * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, c0->stream));
  HIP_TRY(hipStreamSynchronize(c0->stream));
  for (int32_t k = 0; k < n; ++k)
    if (host_keys[k] != ~0ull) return status_of_code(host_keys[k]);
  return LBM_OK;
}

// ------------------------------------------------- allocation-free batches
// lbm_step_batched_noalloc keeps its job table and failure words in this
// file-scope device array instead of the first context's workspace; every
// device the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: the device address
// of each device's copy comes from hipGetSymbolAddress, taken once per
// device with that device current.
constexpr size_t kScratchJobsBytes =
    (kMaxBatch * sizeof(JobArgs) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kScratchJobsBytes + kMaxBatch * sizeof(unsigned long long);
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// host staging of the allocation-free batch (one batch at a time per process)
std::mutex g_noalloc_host_mu;
JobArgs g_noalloc_host_jobs[kMaxBatch];
unsigned long long g_noalloc_host_keys[kMaxBatch];

lbm_status scratch_of_device(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return LBM_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBM_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_default_config(lbm_config* c, int32_t nx, int32_t ny) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->nx = nx;
  c->ny = ny;
  c->precision = LBM_FP64;
  c->gamma = 1.4;
  c->nu = 0.0;
  c->shift_mode = LBM_SHIFT_ADAPTIVE;
  c->shift_halfwidth = 0.5;
  c->newton_tol = 1e-12;
  c->newton_max_iter = 30;
  c->max_abs_shift = 6;
  c->sensor = 0;
  c->collect_stats = 0;
  c->constraints = kM;
  c->prandtl = 1.0;
  c->fallback = 0;
}

size_t lbm_workspace_bytes(const lbm_config* cfg) {
  if (!config_ok(cfg)) return 0;
  return layout(cfg).total;
}

namespace {

lbm_status create_common(const lbm_ctx* like, const lbm_config* cfg, void* ws, size_t bytes,
                         void* stream, lbm_ctx** out) {
  if (!out) return LBM_ERR_ARG;
  *out = nullptr;
  if (!config_ok(cfg)) return LBM_ERR_ARG;
  const Layout L = layout(cfg);
  if (!ws || bytes < L.total || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
    return LBM_ERR_WORKSPACE;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ws) != hipSuccess || attr.type != hipMemoryTypeDevice)
    return LBM_ERR_WORKSPACE;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ERR_ARG;
  c->cfg = *cfg;
  c->lay = L;
  c->stream = static_cast<hipStream_t>(stream);
  HIP_TRY(hipGetDevice(&c->device));
  c->ws = static_cast<char*>(ws);
  c->cur = 0;
  c->initialized = false;
  c->steps_done = 0;
  c->grid.N = static_cast<long long>(cfg->nx) * cfg->ny;
  c->grid.nx = cfg->nx;
  c->grid.ny = cfg->ny;
  const int reach = 4 + cfg->max_abs_shift;  // pull offset plus gradient stencil
  c->grid.fast_x = cfg->nx >= reach;
  c->grid.fast_y = cfg->ny >= reach;
  const double Cv = 1.0 / (cfg->gamma - 1.0);
  c->phys.nu = cfg->nu;
  c->phys.Cv = Cv;
  c->phys.Cp = cfg->gamma * Cv;
  c->phys.halfwidth = cfg->shift_halfwidth;
  c->phys.tol = cfg->newton_tol;
  c->phys.max_iter = cfg->newton_max_iter;
  c->phys.shift_mode = cfg->shift_mode;
  c->phys.fixed_ux = cfg->fixed_ux;
  c->phys.fixed_uy = cfg->fixed_uy;
  c->phys.max_abs_shift = cfg->max_abs_shift;
  c->phys.sensor = cfg->sensor;
  c->phys.stats = cfg->collect_stats;
  c->phys.fallback = cfg->fallback;
  c->phys.inv_pr = shakhov_on(cfg) ? 1.0 / cfg->prandtl : 1.0;
  c->nblocks = L.nparts;
  c->sched.step_block = cfg->precision == LBM_FP64 ? step_block<double>() : step_block<float>();
  c->sched.tiles_per_block = 1;
  c->sched.xcd_remap = 1;
  c->sched.rebuild_blocks = default_rebuild_blocks(c->grid.N);
  c->table.data = reinterpret_cast<const float*>(c->ws + L.table_off);
  c->table.nu = kTabU;
  c->table.ns = kTabS;
  c->table.umax = kTabUmax;
  c->table.smin = kTabSmin;
  c->table.smax = kTabSmax;
  c->table.inv_hu = (kTabU - 1) / kTabUmax;
  c->table.inv_hs = (kTabS - 1) / (kTabSmax - kTabSmin);
  hipLaunchKernelGGL(diag_reset_kernel, dim3(1), dim3(64), 0, c->stream, c->diag(),
                     c->carry().counters);
  const size_t table_bytes = table_bytes_of(cfg->constraints);
  if (like && like->cfg.constraints == cfg->constraints) {
    if (hipMemcpyAsync(c->ws + L.table_off, like->ws + like->lay.table_off, table_bytes,
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
      delete c;
      return LBM_ERR_HIP;
    }
  } else {
    // the table of the context's constraint set, built on the device
    const int pts = kTabU * kTabU * kTabS;
    float* tab = reinterpret_cast<float*>(c->ws + L.table_off);
    if (cfg->constraints == kM13)
      hipLaunchKernelGGL(table13_kernel, dim3((pts + 255) / 256), dim3(256), 0, c->stream, tab,
                         kTabU, kTabS, kTabUmax, kTabSmin, kTabSmax, 1e-13, 100);
    else if (cfg->constraints == 4)
      hipLaunchKernelGGL(table4_kernel, dim3((pts + 255) / 256), dim3(256), 0, c->stream, tab,
                         kTabU, kTabS, kTabUmax, kTabSmin, kTabSmax, 1e-13, 100);
    else
      hipLaunchKernelGGL(table_kernel, dim3((pts + 255) / 256), dim3(256), 0, c->stream, tab,
                         kTabU, kTabS, kTabUmax, kTabSmin, kTabSmax, 1e-13, 100);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return LBM_ERR_HIP;
  }
  *out = c;
  return LBM_OK;
}

}  // namespace

lbm_status lbm_create(const lbm_config* cfg, void* ws, size_t bytes, void* stream,
                      lbm_ctx** out) {
  return create_common(nullptr, cfg, ws, bytes, stream, out);
}

lbm_status lbm_create_like(const lbm_ctx* like, const lbm_config* cfg, void* ws, size_t bytes,
                           void* stream, lbm_ctx** out) {
  if (!like) {
    if (out) *out = nullptr;
    return LBM_ERR_ARG;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBM_ERR_HIP;
  if (dev != like->device) {
    if (out) *out = nullptr;
    return LBM_ERR_ARG;
  }
  return create_common(like, cfg, ws, bytes, stream, out);
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
                           const double* T) {
  if (!c) return LBM_ERR_ARG;
  if (c->cfg.shift_mode == LBM_SHIFT_STATIC) return LBM_ERR_STATE;
  return init_common(c, rho, ux, uy, T, nullptr, nullptr);
}

lbm_status lbm_init_fields_static(lbm_ctx* c, const double* rho, const double* ux,
                                  const double* uy, const double* T, const int8_t* Ux,
                                  const int8_t* Uy) {
  if (!c) return LBM_ERR_ARG;
  if (c->cfg.shift_mode != LBM_SHIFT_STATIC) return LBM_ERR_STATE;
  return init_common(c, rho, ux, uy, T, Ux, Uy);
}

lbm_status lbm_step_async(lbm_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return LBM_ERR_ARG;
  if (!c->initialized) return LBM_ERR_STATE;
  for (int32_t k = 0; k < nsteps; ++k) {
    const int src = c->cur, dst = 1 - c->cur;
    const int step = static_cast<int>(c->steps_done + 1);
    lbm_status st = launch_rebuild(c, src, dst, step);
    if (st) return st;
    st = launch_step(c, src, dst, true, step);
    if (st) return st;
    c->cur = dst;
    c->steps_done += 1;
  }
  return LBM_OK;
}

lbm_status lbm_step_profiled(lbm_ctx* c, int32_t nsteps, double* ms_rebuild, double* ms_step) {
  if (!c || nsteps < 1 || !ms_rebuild || !ms_step) return LBM_ERR_ARG;
  if (!c->initialized) return LBM_ERR_STATE;
  *ms_rebuild = 0.0;
  *ms_step = 0.0;
  std::vector<hipEvent_t> ev(2 * static_cast<size_t>(nsteps) + 1, nullptr);
  lbm_status st = LBM_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      st = LBM_ERR_HIP;
    }
  if (st == LBM_OK && hipEventRecord(ev[0], c->stream) != hipSuccess) st = LBM_ERR_HIP;
  for (int32_t k = 0; k < nsteps && st == LBM_OK; ++k) {
    const int src = c->cur, dst = 1 - c->cur;
    const int step = static_cast<int>(c->steps_done + 1);
    st = launch_rebuild(c, src, dst, step);
    if (st == LBM_OK && hipEventRecord(ev[2 * k + 1], c->stream) != hipSuccess) st = LBM_ERR_HIP;
    if (st == LBM_OK) st = launch_step(c, src, dst, true, step);
    if (st == LBM_OK && hipEventRecord(ev[2 * k + 2], c->stream) != hipSuccess) st = LBM_ERR_HIP;
    if (st == LBM_OK) {
      c->cur = dst;
      c->steps_done += 1;
    }
  }
  if (st == LBM_OK && hipEventSynchronize(ev.back()) != hipSuccess) st = LBM_ERR_HIP;
  for (int32_t k = 0; k < nsteps && st == LBM_OK; ++k) {
    float a = 0.0f, b = 0.0f;
    if (hipEventElapsedTime(&a, ev[2 * k], ev[2 * k + 1]) != hipSuccess ||
        hipEventElapsedTime(&b, ev[2 * k + 1], ev[2 * k + 2]) != hipSuccess)
      st = LBM_ERR_HIP;
    *ms_rebuild += a;
    *ms_step += b;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st) return st;
  return read_status(c, nullptr);
}

lbm_status lbm_copy_state(lbm_ctx* dst, const lbm_ctx* src) {
  if (!dst || !src || dst == src) return LBM_ERR_ARG;
  if (!same_config(dst->cfg, src->cfg) || dst->device != src->device) return LBM_ERR_ARG;
  if (!src->initialized) return LBM_ERR_STATE;
  // every region before the table: buffers, tags, carried arrays, diagnostics
  HIP_TRY(hipStreamSynchronize(src->stream));
  HIP_TRY(hipMemcpyAsync(dst->ws, src->ws, src->lay.table_off, hipMemcpyDeviceToDevice,
                         dst->stream));
  HIP_TRY(hipStreamSynchronize(dst->stream));
  dst->cur = src->cur;
  dst->steps_done = src->steps_done;
  dst->initialized = true;
  return LBM_OK;
}

lbm_status lbm_set_schedule(lbm_ctx* c, const lbm_schedule* sched) {
  if (!c || !schedule_ok(c, sched)) return LBM_ERR_ARG;
  c->sched = *sched;
  if (c->sched.rebuild_blocks == 0) c->sched.rebuild_blocks = default_rebuild_blocks(c->grid.N);
  for (auto& g : c->graphs) g.reset();
  return LBM_OK;
}

lbm_status lbm_get_schedule(const lbm_ctx* c, lbm_schedule* sched) {
  if (!c || !sched) return LBM_ERR_ARG;
  *sched = c->sched;
  return LBM_OK;
}

lbm_status lbm_step_graph_async(lbm_ctx* c, int32_t nsteps, int32_t chunk) {
  if (!c || nsteps < 0 || chunk < 2 || chunk > 1024 || (chunk & 1)) return LBM_ERR_ARG;
  if (!c->initialized) return LBM_ERR_STATE;
  const int32_t reps = nsteps / chunk;
  if (reps > 0) {
    StepGraph& G = c->graphs[c->cur];
    const int parity = static_cast<int>(c->steps_done & 1);
    if (!G.exec || G.chunk != chunk || G.cur != c->cur || G.parity != parity) {
      const lbm_status st = build_graph(c, chunk, G);
      if (st) return st;
    }
    hipLaunchKernelGGL(set_step_base_kernel, dim3(1), dim3(64), 0, c->stream, c->diag(),
                       static_cast<unsigned long long>(c->steps_done - parity));
    HIP_TRY(hipGetLastError());
    // the base goes back to 0 even if a replay fails to enqueue, so that
    // plain launches afterwards record their own step numbers
    int32_t done = 0;
    while (done < reps && hipGraphLaunch(G.exec, c->stream) == hipSuccess) ++done;
    hipLaunchKernelGGL(set_step_base_kernel, dim3(1), dim3(64), 0, c->stream, c->diag(), 0ull);
    c->steps_done += static_cast<int64_t>(done) * chunk;
    if (done < reps) return LBM_ERR_HIP;
    HIP_TRY(hipGetLastError());
  }
  return lbm_step_async(c, nsteps - reps * chunk);
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_ERR_ARG;
  return read_status(c, nullptr);
}

lbm_status lbm_step(lbm_ctx* c, int32_t nsteps) {
  lbm_status st = lbm_step_async(c, nsteps);
  if (st) return st;
  return read_status(c, nullptr);
}

lbm_status lbm_get_macros(lbm_ctx* c, double* rho, double* ux, double* uy, double* T,
                          int8_t* Ux, int8_t* Uy) {
  if (!c || !rho || !ux || !uy || !T) return LBM_ERR_ARG;
  if (!c->initialized) return LBM_ERR_STATE;
  const int b = c->cur;
  if (c->cfg.constraints == kM13)
    hipLaunchKernelGGL(macros49_kernel, dim3(c->nblocks), dim3(kBlock), 0, c->stream,
                       static_cast<const double*>(c->f(b)), static_cast<const double*>(c->g(b)),
                       c->tag(b), c->grid.N, c->phys.Cv, rho, ux, uy, T, Ux, Uy);
  else if (c->cfg.precision == LBM_FP64)
    hipLaunchKernelGGL(macros_kernel<double>, dim3(c->nblocks), dim3(kBlock), 0, c->stream,
                       static_cast<const double*>(c->f(b)), static_cast<const double*>(c->g(b)),
                       c->tag(b), c->grid.N, c->phys.Cv, rho, ux, uy, T, Ux, Uy);
  else
    hipLaunchKernelGGL(macros_kernel<float>, dim3(c->nblocks), dim3(kBlock), 0, c->stream,
                       static_cast<const float*>(c->f(b)), static_cast<const float*>(c->g(b)),
                       c->tag(b), c->grid.N, c->phys.Cv, rho, ux, uy, T, Ux, Uy);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, double* f, double* g) {
  if (!c || !f || !g) return LBM_ERR_ARG;
  if (!c->initialized) return LBM_ERR_STATE;
  const int b = c->cur;
  const long long cnt = lattice_q(c->cfg.constraints) * c->grid.N;
  if (c->cfg.precision == LBM_FP64) {
    HIP_TRY(hipMemcpyAsync(f, c->f(b), cnt * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(g, c->g(b), cnt * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  } else {
    const dim3 grid(static_cast<unsigned>((cnt + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(widen_kernel<float>, grid, dim3(kBlock), 0, c->stream,
                       static_cast<const float*>(c->f(b)), f, cnt);
    hipLaunchKernelGGL(widen_kernel<float>, grid, dim3(kBlock), 0, c->stream,
                       static_cast<const float*>(c->g(b)), g, cnt);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

void lbm_velocities(int32_t* cx, int32_t* cy) {
  for (int k = 0; k < kQ; ++k) {
    if (cx) cx[k] = plane_cx(k);
    if (cy) cy[k] = plane_cy(k);
  }
}

int32_t lbm_lattice_velocities(int32_t constraints, int32_t* cx, int32_t* cy) {
  if (constraints != kM && constraints != 4 && constraints != kM13) return 0;
  const int Q = lattice_q(constraints);
  for (int k = 0; k < Q; ++k) {
    if (cx) cx[k] = Q == kQ49 ? cx49(k) : plane_cx(k);
    if (cy) cy[k] = Q == kQ49 ? cy49(k) : plane_cy(k);
  }
  return Q;
}

lbm_status lbm_get_diag(lbm_ctx* c, lbm_diag* out) {
  if (!c || !out) return LBM_ERR_ARG;
  std::memset(out, 0, sizeof *out);
  DevDiag d;
  HIP_TRY(hipMemcpyAsync(&d, c->diag(), sizeof d, hipMemcpyDeviceToHost, c->stream));
  double sums[4] = {0, 0, 0, 0};
  if (c->initialized || c->steps_done == 0) {
    const int b = c->cur;
    if (c->cfg.constraints == kM13)
      hipLaunchKernelGGL(conserved49_kernel, dim3(c->nblocks), dim3(kBlock), 0, c->stream,
                         static_cast<const double*>(c->f(b)),
                         static_cast<const double*>(c->g(b)), c->tag(b), c->grid.N, c->parts());
    else if (c->cfg.precision == LBM_FP64)
      hipLaunchKernelGGL(conserved_kernel<double>, dim3(c->nblocks), dim3(kBlock), 0, c->stream,
                         static_cast<const double*>(c->f(b)),
                         static_cast<const double*>(c->g(b)), c->tag(b), c->grid.N, c->parts());
    else
      hipLaunchKernelGGL(conserved_kernel<float>, dim3(c->nblocks), dim3(kBlock), 0, c->stream,
                         static_cast<const float*>(c->f(b)), static_cast<const float*>(c->g(b)),
                         c->tag(b), c->grid.N, c->parts());
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kBlock), 0, c->stream, c->parts(),
                       c->nblocks, c->sums());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(sums, c->sums(), sizeof sums, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  out->steps_done = c->steps_done;
  if (d.fail_key == ~0ull) {
    out->status = LBM_OK;
    out->fail_step = -1;
    out->fail_node = -1;
  } else {
    out->status = status_of_code(d.fail_key);
    out->fail_step = static_cast<int32_t>(d.fail_key >> 34);
    out->fail_node = static_cast<int64_t>((d.fail_key >> 3) & ((1ull << 31) - 1));
  }
  out->newton_calls = static_cast<int64_t>(d.newton_calls);
  out->newton_iters = static_cast<int64_t>(d.newton_iters);
  out->mismatched_links = static_cast<int64_t>(d.mismatched);
  for (int i = 0; i < LBM_HIST_BINS; ++i) out->iter_hist[i] = static_cast<int64_t>(d.hist[i]);
  for (int i = 0; i < 4; ++i) out->conserved[i] = sums[i];
  out->fallback_solves = static_cast<int64_t>(d.fallbacks);
  return LBM_OK;
}

lbm_status lbm_step_batched(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n) {
  if (!ctxs || !nsteps || n < 0 || n > kMaxBatch || (n > 0 && !ctxs[0])) return LBM_ERR_ARG;
  if (n == 0) return LBM_OK;
  std::vector<JobArgs> jobs(n);
  std::vector<unsigned long long> keys(n, ~0ull);
  lbm_ctx* c0 = ctxs[0];
  return step_batched_common(ctxs, nsteps, n,
                             reinterpret_cast<JobArgs*>(c0->ws + c0->lay.batch_off),
                             reinterpret_cast<unsigned long long*>(c0->ws + c0->lay.keys_off),
                             jobs.data(), keys.data());
}

lbm_status lbm_step_batched_graph(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n,
                                  int32_t* graph_built) {
  if (!ctxs || !nsteps || n < 0 || n > kMaxBatch || (n > 0 && !ctxs[0])) return LBM_ERR_ARG;
  if (graph_built) *graph_built = 0;
  if (n == 0) return LBM_OK;
  std::vector<JobArgs> jobs(n);
  std::vector<unsigned long long> keys(n, ~0ull);
  lbm_ctx* c0 = ctxs[0];
  const int before = c0->batch_graph.builds;
  const lbm_status st =
      step_batched_common(ctxs, nsteps, n, reinterpret_cast<JobArgs*>(c0->ws + c0->lay.batch_off),
                          reinterpret_cast<unsigned long long*>(c0->ws + c0->lay.keys_off),
                          jobs.data(), keys.data(), true);
  if (graph_built) *graph_built = c0->batch_graph.builds - before;
  return st;
}

lbm_status lbm_step_batched_noalloc(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n) {
  if (!ctxs || !nsteps || n < 0 || n > kMaxBatch || (n > 0 && !ctxs[0])) return LBM_ERR_ARG;
  if (n == 0) return LBM_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBM_ERR_HIP;
  if (dev != ctxs[0]->device) return LBM_ERR_ARG;
  char* sp = nullptr;
  const lbm_status st = scratch_of_device(dev, &sp);
  if (st) return st;
  // one batch at a time per process: the host staging below is shared
  std::lock_guard<std::mutex> lock(g_noalloc_host_mu);
  return step_batched_common(ctxs, nsteps, n, reinterpret_cast<JobArgs*>(sp),
                             reinterpret_cast<unsigned long long*>(sp + kScratchJobsBytes),
                             g_noalloc_host_jobs, g_noalloc_host_keys);
}

lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (bytes == 0) return LBM_OK;
  if (!src || !dst) return LBM_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return LBM_ERR_ARG;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const long long words = static_cast<long long>(bytes / 16);
  if (words > 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return LBM_ERR_HIP;
    // eight workgroups per compute unit, enough passes to amortise the tail
    const long long per_pass = static_cast<long long>(kBlock) * kCopyUnroll;
    const long long need = (words + per_pass - 1) / per_pass;
    const unsigned blocks = static_cast<unsigned>(std::min<long long>(need, 8ll * cus));
    hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                       static_cast<const CopyWord*>(src), static_cast<CopyWord*>(dst), words);
  }
  const long long tail = static_cast<long long>(bytes % 16);
  if (tail) {
    const long long off = words * 16;
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(kBlock), 0, stream,
                       static_cast<const unsigned char*>(src) + off,
                       static_cast<unsigned char*>(dst) + off, tail);
  }
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

void lbm_destroy(lbm_ctx* c) { delete c; }

const char* lbm_status_str(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_ARG: return "invalid argument";
    case LBM_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_STATE: return "call out of order";
    case LBM_ERR_NEWTON: return "equilibrium solve did not converge";
    case LBM_ERR_NONPHYSICAL: return "non-physical state or lattice shift out of range";
  }
  return "unknown status";
}

}  // extern "C"
