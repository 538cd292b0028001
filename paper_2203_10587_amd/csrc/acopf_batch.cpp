// Batched evaluation: many instances (N-1 contingencies, scenarios, served
// requests) in one kernel launch.  The batch owns
//   - per-instance offsets into the caller's packed buffers,
//   - a device descriptor table (one InstOff per instance),
//   - a tile list over all instances, ordered so that each instance's tiles
//     land on one XCD (workgroup b runs on XCD b mod 8, so tiles at list
//     positions p = q (mod 8) form XCD queue q) and instances are spread over
//     the eight queues largest-first,
//   - the f-reduction scratch, and
//   - a small cache of instantiated HIP graphs keyed by the buffer set.
#include <algorithm>
#include <array>
#include <cstring>
#include <list>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "acopf.h"
#include "acopf_host.h"

namespace acopf {
constexpr int kXcds = 8;
constexpr size_t kGraphCache = 8;

struct GraphKey {
  unsigned variant;
  std::array<const void*, 13> ptrs;
  bool operator==(const GraphKey& o) const { return variant == o.variant && ptrs == o.ptrs; }
};

}  // namespace acopf

struct acopf_batch_s {
  std::vector<acopf_net> nets;
  int32_t count = 0;
  acopf_sched sched{};
  std::vector<int64_t> xo, co, jo, ho;
  int device = 0;
  void* mem = nullptr;
  acopf::InstOff* d_table = nullptr;
  acopf::Tile* d_tiles = nullptr;
  double* d_fpart = nullptr;
  int ntiles = 0;
  int grid = 0;  // 0: one workgroup per tile
  acopf::Tile* d_tiles_inst = nullptr;  // the same tiles, instance after instance
  std::vector<int32_t> inst_tile_off;   // count + 1
  int max_len = 0;                      // max n + m over instances
  hipStream_t cap_stream = nullptr;
  std::list<std::pair<acopf::GraphKey, hipGraphExec_t>> graphs;  // most recent first
};

using namespace acopf;

namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

int cu_count(int device, int* cus) {
  hipDeviceProp_t p;
  hipError_t e = hipGetDeviceProperties(&p, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  *cus = p.multiProcessorCount;
  return ACOPF_OK;
}

void free_batch(acopf_batch_s* b) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->mem) (void)hipFree(b->mem);
  (void)hipSetDevice(cur);
  for (acopf_net n : b->nets) n->refs.fetch_sub(1);
  delete b;
}

unsigned variant_of(unsigned what) {
  if ((what & ~unsigned(ACOPF_F | ACOPF_GRADF | ACOPF_C)) == 0) return K_FG;
  if (what == ACOPF_J) return K_J;
  if (what == ACOPF_H) return K_H;
  return K_ALL;
}

// The evaluation kernel, then (if f is wanted) the f reduction.
hipError_t enqueue(acopf_batch_s* b, unsigned variant, const Bufs& bufs, hipStream_t s) {
  const InstOff none{};
  hipError_t e = launch_eval(variant, b->sched.tile_be, bufs, b->d_table, none, b->d_tiles,
                             b->ntiles, b->grid, s);
  if (e == hipSuccess && bufs.f) e = launch_fsum(b->d_table, none, 0, b->count, bufs.fpart, bufs.f, s);
  return e;
}

int run_batch(acopf_batch_s* b, unsigned variant, const Bufs& bufs, hipStream_t stream) {
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  if (b->sched.no_graph) {
    e = enqueue(b, variant, bufs, stream);
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    return ACOPF_OK;
  }
  GraphKey key{variant,
               {bufs.x, bufs.lam, bufs.wc, bufs.sigma, bufs.wf, bufs.f, bufs.gradf, bufs.c,
                bufs.jac, bufs.hess, bufs.u, bufs.dir, bufs.out}};
  hipGraphExec_t exec = nullptr;
  for (auto it = b->graphs.begin(); it != b->graphs.end(); ++it) {
    if (it->first == key) {
      exec = it->second;
      b->graphs.splice(b->graphs.begin(), b->graphs, it);
      break;
    }
  }
  if (!exec) {
    if (!b->cap_stream) {
      e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = enqueue(b, variant, bufs, b->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(le, "batch kernel capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    b->graphs.emplace_front(key, exec);
    if (b->graphs.size() > kGraphCache) {
      (void)hipGraphExecDestroy(b->graphs.back().second);
      b->graphs.pop_back();
    }
  }
  e = hipGraphLaunch(exec, stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ACOPF_OK;
}

}  // namespace

extern "C" {

int acopf_batch_create(const acopf_net* nets, int32_t count, const acopf_sched* sched,
                       acopf_batch* out) {
  if (!out) return fail(ACOPF_EINVAL, "null output handle");
  *out = nullptr;
  if (!nets || count < 1) return fail(ACOPF_EINVAL, "need at least one net");
  acopf_sched s{kDefaultTileBe, 0, 1, 0};
  if (sched) s = *sched;
  TileCaps caps;
  if (!caps_for(s.tile_be, &caps)) return fail(ACOPF_EINVAL, "tile_be must be 64, 128, 256 or 512");
  if (s.xcd_group < 0 || s.xcd_group > 1 || s.no_graph < 0 || s.no_graph > 1)
    return fail(ACOPF_EINVAL, "xcd_group and no_graph must be 0 or 1");
  if (s.grid_mult < 0 || s.grid_mult > 64) return fail(ACOPF_EINVAL, "grid_mult must be in [0, 64]");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (int k = 0; k < count; ++k) {
    if (!nets[k]) return fail(ACOPF_EINVAL, "null net at index " + std::to_string(k));
    if (nets[k]->base->device != dev)
      return fail(ACOPF_EINVAL, "net " + std::to_string(k) + " lives on another device");
  }
  acopf_batch_s* b = nullptr;
  try {
    b = new acopf_batch_s();
    b->nets.assign(nets, nets + count);
    for (acopf_net n : b->nets) n->refs.fetch_add(1);
    b->count = count;
    b->sched = s;
    b->device = dev;
    b->xo.assign(count + 1, 0);
    b->co.assign(count + 1, 0);
    b->jo.assign(count + 1, 0);
    b->ho.assign(count + 1, 0);
    std::vector<int32_t> fpo(count + 1, 0);
    for (int k = 0; k < count; ++k) {
      const acopf_dims& d = nets[k]->dims;
      b->xo[k + 1] = b->xo[k] + d.n;
      b->co[k + 1] = b->co[k] + d.m;
      b->jo[k + 1] = b->jo[k] + d.nnz_jac;
      b->ho[k + 1] = b->ho[k] + d.nnz_hess;
      fpo[k + 1] = fpo[k] + nets[k]->base->topo.nchunks;
    }
    // per-base schedule (outage children share their base's)
    struct PerBase {
      Schedule sch;
      size_t work_off = 0;   // into the batch's work array
    };
    std::map<const Base*, PerBase> per_base;
    size_t work_total = 0;
    for (int k = 0; k < count; ++k) {
      const Base* B = nets[k]->base.get();
      if (per_base.count(B)) continue;
      PerBase pb;
      int rc = make_tiles(B->topo, s.tile_be, &pb.sch);
      if (rc) {
        free_batch(b);
        return rc;
      }
      pb.work_off = work_total;
      work_total += pb.sch.work.size();
      per_base.emplace(B, std::move(pb));
    }
    // XCD queues, largest instances first (LPT on tile counts)
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    auto ntile = [&](int k) { return int(per_base[nets[k]->base.get()].sch.tiles.size()); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return ntile(a) > ntile(c); });
    std::vector<std::vector<Tile>> queue(s.xcd_group ? kXcds : 1);
    std::vector<int64_t> load(queue.size(), 0);
    for (int k : order) {
      const size_t qi = std::min_element(load.begin(), load.end()) - load.begin();
      for (Tile t : per_base[nets[k]->base.get()].sch.tiles) {
        t.inst = k;
        queue[qi].push_back(t);
      }
      load[qi] += ntile(k);
    }
    std::vector<Tile> tiles_inst;
    b->inst_tile_off.assign(count + 1, 0);
    for (int k = 0; k < count; ++k) {
      for (Tile t : per_base[nets[k]->base.get()].sch.tiles) {
        t.inst = k;
        tiles_inst.push_back(t);
      }
      b->inst_tile_off[k + 1] = int32_t(tiles_inst.size());
      const acopf_dims& d = nets[k]->dims;
      b->max_len = std::max<int>(b->max_len, int(d.n + d.m));
    }
    std::vector<Tile> tiles;
    size_t total = 0;
    for (auto& q : queue) total += q.size();
    tiles.reserve(total);
    std::vector<size_t> pos(queue.size(), 0);
    while (tiles.size() < total) {
      for (size_t qi = 0; qi < queue.size(); ++qi)
        if (pos[qi] < queue[qi].size()) tiles.push_back(queue[qi][pos[qi]++]);
    }
    b->ntiles = int(tiles.size());
    int cus = 256;
    int rc = cu_count(dev, &cus);
    if (rc) {
      free_batch(b);
      return rc;
    }
    b->grid = s.grid_mult > 0 ? std::min(b->ntiles, s.grid_mult * cus) : 0;
    // device table, tiles, work items, scratch
    const size_t s_table = align_up(size_t(count) * sizeof(InstOff));
    const size_t s_tiles = align_up(tiles.size() * sizeof(Tile));
    const size_t s_tinst = align_up(tiles_inst.size() * sizeof(Tile));
    const size_t s_work = align_up(std::max<size_t>(work_total, 1) * sizeof(WorkItem));
    const size_t s_fpart = align_up(size_t(fpo[count]) * sizeof(double));
    e = hipMalloc(&b->mem, s_table + s_tiles + s_work + s_fpart + s_tinst);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b->mem = nullptr;
      free_batch(b);
      return fail(ACOPF_ENOMEM, std::string("hipMalloc of batch tables: ") + hipGetErrorString(e));
    }
    char* base = static_cast<char*>(b->mem);
    b->d_table = reinterpret_cast<InstOff*>(base);
    b->d_tiles = reinterpret_cast<Tile*>(base + s_table);
    WorkItem* d_work = reinterpret_cast<WorkItem*>(base + s_table + s_tiles);
    b->d_fpart = reinterpret_cast<double*>(base + s_table + s_tiles + s_work);
    b->d_tiles_inst = reinterpret_cast<Tile*>(base + s_table + s_tiles + s_work + s_fpart);
    std::vector<InstOff> table(count);
    for (int k = 0; k < count; ++k) {
      InstOff I = net_inst(nets[k]);
      I.work = d_work + per_base[nets[k]->base.get()].work_off;
      I.xo = b->xo[k];
      I.co = b->co[k];
      I.jo = b->jo[k];
      I.ho = b->ho[k];
      I.k = k;
      I.fpo = fpo[k];
      table[k] = I;
    }
    e = hipMemcpy(b->d_table, table.data(), table.size() * sizeof(InstOff), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice);
    for (auto& kv : per_base) {
      const Schedule& sc = kv.second.sch;
      if (e == hipSuccess && !sc.work.empty())
        e = hipMemcpy(d_work + kv.second.work_off, sc.work.data(), sc.work.size() * sizeof(WorkItem),
                      hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
      e = hipMemcpy(b->d_tiles_inst, tiles_inst.data(), tiles_inst.size() * sizeof(Tile),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_fpart, 0, s_fpart);
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e, "batch table upload");
    }
    *out = b;
    t_err.clear();
    return ACOPF_OK;
  } catch (const std::bad_alloc&) {
    if (b) free_batch(b);
    return fail(ACOPF_ENOMEM, "host allocation failed");
  }
}

int acopf_batch_destroy(acopf_batch batch) {
  if (!batch) return ACOPF_OK;
  free_batch(batch);
  return ACOPF_OK;
}

int acopf_batch_offsets(acopf_batch b, int64_t* x_off, int64_t* c_off, int64_t* j_off,
                        int64_t* h_off) {
  if (!b) return fail(ACOPF_EINVAL, "null batch");
  const size_t n = (b->count + 1) * sizeof(int64_t);
  if (x_off) std::memcpy(x_off, b->xo.data(), n);
  if (c_off) std::memcpy(c_off, b->co.data(), n);
  if (j_off) std::memcpy(j_off, b->jo.data(), n);
  if (h_off) std::memcpy(h_off, b->ho.data(), n);
  return ACOPF_OK;
}

int acopf_batch_eval(acopf_batch b, const double* x, const double* sigma, const double* lambda,
                     double* f, double* grad_f, double* c, double* jac_val, double* hess_val,
                     unsigned what, hipStream_t stream) {
  if (!b || !x) return fail(ACOPF_EINVAL, "null batch or x");
  if (what & ~unsigned(ACOPF_ALL)) return fail(ACOPF_EINVAL, "unknown bits in what");
  if (((what & ACOPF_F) && !f) || ((what & ACOPF_GRADF) && !grad_f) || ((what & ACOPF_C) && !c) ||
      ((what & ACOPF_J) && !jac_val) ||
      ((what & ACOPF_H) && (!hess_val || !lambda || !sigma)))
    return fail(ACOPF_EINVAL, "a selected output (or lambda/sigma for ACOPF_H) is null");
  if (!what) return ACOPF_OK;
  Bufs bufs{};
  bufs.x = x;
  bufs.lam = (what & ACOPF_H) ? lambda : nullptr;
  bufs.sigma = (what & ACOPF_H) ? sigma : nullptr;
  bufs.f = (what & ACOPF_F) ? f : nullptr;
  bufs.gradf = (what & ACOPF_GRADF) ? grad_f : nullptr;
  bufs.c = (what & ACOPF_C) ? c : nullptr;
  bufs.jac = (what & ACOPF_J) ? jac_val : nullptr;
  bufs.hess = (what & ACOPF_H) ? hess_val : nullptr;
  bufs.fpart = b->d_fpart;
  return run_batch(b, variant_of(what), bufs, stream);
}

int acopf_batch_hvp(acopf_batch b, const double* x, const double* sigma, const double* lambda,
                    const double* d, double* out, hipStream_t stream) {
  if (!b || !x || !sigma || !lambda || !d || !out) return fail(ACOPF_EINVAL, "null argument");
  Bufs bufs{};
  bufs.x = x;
  bufs.sigma = sigma;
  bufs.lam = lambda;
  bufs.dir = d;
  bufs.out = out;
  bufs.fpart = b->d_fpart;
  return run_batch(b, K_HVP, bufs, stream);
}

int acopf_batch_jvp(acopf_batch b, const double* x, const double* d, double* out,
                    hipStream_t stream) {
  if (!b || !x || !d || !out) return fail(ACOPF_EINVAL, "null argument");
  Bufs bufs{};
  bufs.x = x;
  bufs.dir = d;
  bufs.out = out;
  bufs.fpart = b->d_fpart;
  return run_batch(b, K_JVP, bufs, stream);
}

int acopf_batch_eval_range(acopf_batch b, int32_t first, int32_t count, const double* x,
                           const double* sigma, const double* lambda, double* f, double* grad_f,
                           double* c, double* jac_val, double* hess_val, unsigned what,
                           hipStream_t stream) {
  if (!b || !x) return fail(ACOPF_EINVAL, "null batch or x");
  if (first < 0 || count < 1 || first > b->count - count)
    return fail(ACOPF_EINVAL, "instance window out of range");
  if (what & ~unsigned(ACOPF_ALL)) return fail(ACOPF_EINVAL, "unknown bits in what");
  if (((what & ACOPF_F) && !f) || ((what & ACOPF_GRADF) && !grad_f) || ((what & ACOPF_C) && !c) ||
      ((what & ACOPF_J) && !jac_val) ||
      ((what & ACOPF_H) && (!hess_val || !lambda || !sigma)))
    return fail(ACOPF_EINVAL, "a selected output (or lambda/sigma for ACOPF_H) is null");
  if (!what) return ACOPF_OK;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  Bufs bufs{};
  bufs.x = x;
  bufs.lam = (what & ACOPF_H) ? lambda : nullptr;
  bufs.sigma = (what & ACOPF_H) ? sigma : nullptr;
  bufs.f = (what & ACOPF_F) ? f : nullptr;
  bufs.gradf = (what & ACOPF_GRADF) ? grad_f : nullptr;
  bufs.c = (what & ACOPF_C) ? c : nullptr;
  bufs.jac = (what & ACOPF_J) ? jac_val : nullptr;
  bufs.hess = (what & ACOPF_H) ? hess_val : nullptr;
  bufs.fpart = b->d_fpart;
  const int t0 = b->inst_tile_off[first], t1 = b->inst_tile_off[first + count];
  const InstOff none{};
  e = launch_eval(variant_of(what), b->sched.tile_be, bufs, b->d_table, none, b->d_tiles_inst + t0,
                  t1 - t0, 0, stream);
  if (e == hipSuccess && bufs.f) e = launch_fsum(b->d_table, none, first, count, bufs.fpart, bufs.f, stream);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  return ACOPF_OK;
}

int acopf_batch_draw_iterates(acopf_batch b, int32_t first, int32_t count, const uint64_t* seeds,
                              double pmin, double pmax, double qmin, double qmax, double* x,
                              double* lambda, hipStream_t stream) {
  if (!b || !seeds || !x || !lambda) return fail(ACOPF_EINVAL, "null argument");
  if (first < 0 || count < 1 || first > b->count - count)
    return fail(ACOPF_EINVAL, "instance window out of range");
  if (count > 65535) return fail(ACOPF_EINVAL, "at most 65535 instances per draw");
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  e = launch_draw(b->d_table, first, count, b->max_len, seeds, pmin, pmax, qmin, qmax, x, lambda,
                  stream);
  if (e != hipSuccess) return hip_fail(e, "draw kernel launch");
  return ACOPF_OK;
}

int acopf_batch_vjp(acopf_batch b, const double* x, const double* w_f, const double* w_c,
                    double* u, hipStream_t stream) {
  if (!b || !x || !w_f || !w_c || !u) return fail(ACOPF_EINVAL, "null argument");
  Bufs bufs{};
  bufs.x = x;
  bufs.wf = w_f;
  bufs.wc = w_c;
  bufs.u = u;
  bufs.fpart = b->d_fpart;
  return run_batch(b, K_VJP, bufs, stream);
}

}  // extern "C"
