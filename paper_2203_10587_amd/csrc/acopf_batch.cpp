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
#include <atomic>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
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
  int32_t form = ACOPF_POLAR;  // shared by every instance
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
  // product tiles: instances of one base in groups of kProdInst ([0]) or
  // of the JVP's size ([1]), as prod_group() gives per product
  acopf::Tile* d_ptiles[2] = {nullptr, nullptr};
  int nptiles[2] = {0, 0};
  acopf::WorkItem* d_work = nullptr;    // work items of every distinct base, back to back
  std::vector<int32_t> inst_tile_off;   // count + 1
  int max_len = 0;                      // max n + m over instances
  int max_chunks = 1;                   // f partials per instance, at most
  int64_t nparts = 0;                   // f partials of the whole batch
  hipStream_t cap_stream = nullptr;
  std::list<std::pair<acopf::GraphKey, hipGraphExec_t>> graphs;  // most recent first
  std::atomic<int> refs{0};             // couplings built on this batch
};

// Coupling rows over a batch: per row the child and the parent column of the
// packed x; per coupled column the rows touching it (row << 1 | parent).
struct acopf_couple_s {
  acopf_batch batch = nullptr;
  int64_t rows = 0;
  std::vector<int64_t> cols;   // 2 per row: child column, parent column
  int32_t ncols = 0;
  void* mem = nullptr;
  int64_t* d_cols = nullptr;
  int64_t* d_tcol = nullptr;
  int32_t* d_tptr = nullptr;
  int32_t* d_tent = nullptr;
};

using namespace acopf;

// Scratch of acopf_batch_eval_noalloc: the objective partials of the
// instances with several cost-item chunks live in this file-scope device
// array instead of the batch's own allocation.  Each device holds its own
// copy.  In host code the name is only a host-side stand-in, so its device
// address is taken once per device with hipGetSymbolAddress (from
// acopf_batch_create, which runs with the device current) and only that
// address is handed to kernels.
static constexpr int64_t kScratchParts = int64_t(1) << 15;  // 32,768 doubles, 256 KiB
static __device__ __align__(256) double scratch[kScratchParts];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current.
static int scratch_address(int dev, double** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ACOPF_EINVAL, "device index " + std::to_string(dev) + " beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return hip_fail(e, "hipGetSymbolAddress of the scratch array");
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return ACOPF_OK;
}

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

bool is_product(unsigned variant) { return (variant & (W_VJP | W_HVP | W_JVP)) != 0; }

// The evaluation kernel, then (if f is wanted) the f reduction.  The
// products walk their own tile lists, whose bus tiles serve several
// instances of one base network at a time.
hipError_t enqueue(acopf_batch_s* b, unsigned variant, const Bufs& bufs, hipStream_t s) {
  InstOff none{};
  none.work = b->d_work;  // the tiles' w0 index this array
  const bool prod = is_product(variant);
  const int pl = prod_group(variant) == kProdInst ? 0 : 1;
  const Tile* tiles = prod ? b->d_ptiles[pl] : b->d_tiles;
  const int nt = prod ? b->nptiles[pl] : b->ntiles;
  const int grid = b->grid > 0 ? std::min(b->grid, nt) : 0;
  hipError_t e = launch_eval(variant, b->sched.tile_be, bufs, b->d_table, none, tiles, nt, grid, s);
  // a single-chunk instance has its f written by its generator tile
  if (e == hipSuccess && bufs.f && b->max_chunks > 1)
    e = launch_fsum(b->d_table, none, 0, b->count, bufs.fpart, bufs.f, s);
  return e;
}

int run_batch(acopf_batch_s* b, unsigned variant, const Bufs& bufs, hipStream_t stream) {
  if (b->form == ACOPF_CARTESIAN) variant |= W_CART;
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

int enqueue_range(acopf_batch_s* b, int32_t first, int32_t count, const double* x,
                  const double* sigma, const double* lambda, double* f, double* grad_f, double* c,
                  double* jac_val, double* hess_val, unsigned what, hipStream_t stream);

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
    if (nets[k]->base->topo.form != nets[0]->base->topo.form)
      return fail(ACOPF_EINVAL, "net " + std::to_string(k) +
                                    " uses another representation than net 0");
  }
  acopf_batch_s* b = nullptr;
  try {
    b = new acopf_batch_s();
    b->nets.assign(nets, nets + count);
    for (acopf_net n : b->nets) n->refs.fetch_add(1);
    b->count = count;
    b->form = nets[0]->base->topo.form;
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
      b->max_chunks = std::max(b->max_chunks, nets[k]->base->topo.nchunks);
    }
    b->nparts = fpo[count];
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
      if (work_total > size_t(INT32_MAX)) {
        free_batch(b);
        return fail(ACOPF_EINVAL, "the batch's work items exceed 2^31");
      }
      per_base.emplace(B, std::move(pb));
    }
    // XCD queues, largest instances first (LPT on tile counts)
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    auto ntile = [&](int k) { return int(per_base[nets[k]->base.get()].sch.tiles.size()); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return ntile(a) > ntile(c); });
    // A queue ends with its instances' generator chunks (a pure generator
    // chunk is short work), so that the launch's last workgroups are short
    // ones; slack chunks, which are not, stay with their instance.
    auto short_tail = [](const Tile& t, int ng) {
      return (t.kind_aux & 3) == TILE_GEN && t.a1 <= ng;
    };
    auto close_queues = [](std::vector<std::vector<Tile>>& qs, std::vector<std::vector<Tile>>& tails) {
      for (size_t qi = 0; qi < qs.size(); ++qi)
        qs[qi].insert(qs[qi].end(), tails[qi].begin(), tails[qi].end());
    };
    std::vector<std::vector<Tile>> queue(s.xcd_group ? kXcds : 1), qtail(queue.size());
    std::vector<int64_t> load(queue.size(), 0);
    for (int k : order) {
      const size_t qi = std::min_element(load.begin(), load.end()) - load.begin();
      const PerBase& pb = per_base[nets[k]->base.get()];
      const int ng = nets[k]->base->topo.ng;
      for (Tile t : pb.sch.tiles) {
        t.inst = k;
        t.w0 += int32_t(pb.work_off);
        (short_tail(t, ng) ? qtail : queue)[qi].push_back(t);
      }
      load[qi] += ntile(k);
    }
    close_queues(queue, qtail);
    std::vector<Tile> tiles_inst;
    b->inst_tile_off.assign(count + 1, 0);
    for (int k = 0; k < count; ++k) {
      const PerBase& pb = per_base[nets[k]->base.get()];
      for (Tile t : pb.sch.tiles) {
        t.inst = k;
        t.w0 += int32_t(pb.work_off);
        tiles_inst.push_back(t);
      }
      b->inst_tile_off[k + 1] = int32_t(tiles_inst.size());
      const acopf_dims& d = nets[k]->dims;
      b->max_len = std::max<int>(b->max_len, int(d.n + d.m));
    }
    // interleave XCD queues: list position p runs on XCD p mod 8
    auto interleave = [](const std::vector<std::vector<Tile>>& qs) {
      std::vector<Tile> out;
      size_t total = 0;
      for (auto& q : qs) total += q.size();
      out.reserve(total);
      std::vector<size_t> pos(qs.size(), 0);
      while (out.size() < total) {
        for (size_t qi = 0; qi < qs.size(); ++qi)
          if (pos[qi] < qs[qi].size()) out.push_back(qs[qi][pos[qi]++]);
      }
      return out;
    };
    std::vector<Tile> tiles = interleave(queue);
    b->ntiles = int(tiles.size());
    // product tiles: the instances of each base network in groups of up to
    // `group` (instance order), a group's bus tiles once with all of its
    // instances, each instance's generator tiles on their own; groups spread
    // over the XCD queues largest-first like the instances above
    std::map<const Base*, std::vector<int>> by_base;
    std::vector<const Base*> base_order;
    for (int k = 0; k < count; ++k) {
      const Base* B = nets[k]->base.get();
      if (!by_base.count(B)) base_order.push_back(B);
      by_base[B].push_back(k);
    }
    auto product_tiles = [&](int group) {
      struct Unit {
        int inst[kProdInst];
        int n;
      };
      std::vector<Unit> units;
      for (const Base* B : base_order) {
        const std::vector<int>& ks = by_base[B];
        for (size_t j = 0; j < ks.size(); j += group) {
          Unit u{};
          u.n = int(std::min<size_t>(group, ks.size() - j));
          for (int q = 0; q < kProdInst; ++q) u.inst[q] = q < u.n ? ks[j + q] : -1;
          units.push_back(u);
        }
      }
      std::stable_sort(units.begin(), units.end(), [&](const Unit& a, const Unit& c) {
        return ntile(a.inst[0]) > ntile(c.inst[0]);
      });
      std::vector<std::vector<Tile>> pq(s.xcd_group ? kXcds : 1), ptail(pq.size());
      std::vector<int64_t> pload(pq.size(), 0);
      for (const Unit& u : units) {
        const size_t qi = std::min_element(pload.begin(), pload.end()) - pload.begin();
        const PerBase& pb = per_base[nets[u.inst[0]]->base.get()];
        const int ng = nets[u.inst[0]]->base->topo.ng;
        for (Tile t : pb.sch.tiles) {
          t.inst = u.inst[0];
          t.w0 += int32_t(pb.work_off);
          if ((t.kind_aux & 3) == TILE_BUS) {
            for (int q = 1; q < kProdInst; ++q) t.more[q - 1] = u.inst[q];
            pq[qi].push_back(t);
          } else {
            for (int q = 0; q < u.n; ++q) {
              t.inst = u.inst[q];
              (short_tail(t, ng) ? ptail : pq)[qi].push_back(t);
            }
          }
        }
        pload[qi] += ntile(u.inst[0]);
      }
      close_queues(pq, ptail);
      return interleave(pq);
    };
    const std::vector<Tile> ptiles[2] = {product_tiles(kProdInst), product_tiles(prod_group(W_JVP))};
    for (int q = 0; q < 2; ++q) b->nptiles[q] = int(ptiles[q].size());
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
    const size_t s_ptiles0 = align_up(ptiles[0].size() * sizeof(Tile));
    const size_t s_ptiles1 = align_up(ptiles[1].size() * sizeof(Tile));
    e = hipMalloc(&b->mem,
                  s_table + s_tiles + s_work + s_fpart + s_tinst + s_ptiles0 + s_ptiles1);
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
    b->d_work = d_work;
    b->d_fpart = reinterpret_cast<double*>(base + s_table + s_tiles + s_work);
    b->d_tiles_inst = reinterpret_cast<Tile*>(base + s_table + s_tiles + s_work + s_fpart);
    b->d_ptiles[0] = reinterpret_cast<Tile*>(base + s_table + s_tiles + s_work + s_fpart + s_tinst);
    b->d_ptiles[1] = reinterpret_cast<Tile*>(reinterpret_cast<char*>(b->d_ptiles[0]) + s_ptiles0);
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
    for (int q = 0; q < 2; ++q)
      if (e == hipSuccess)
        e = hipMemcpy(b->d_ptiles[q], ptiles[q].data(), ptiles[q].size() * sizeof(Tile),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_fpart, 0, s_fpart);
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e, "batch table upload");
    }
    // set-up of the allocation-free entry point on this device; a failure
    // here is reported by that entry point, not by the batch
    double* sp = nullptr;
    if (scratch_address(dev, &sp) != ACOPF_OK) t_err.clear();
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
  if (batch->refs.load() != 0)
    return fail(ACOPF_ESTATE, "batch still has couplings; destroy them first");
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

int acopf_batch_eval_noalloc(acopf_batch b, const double* x, const double* sigma,
                             const double* lambda, double* f, double* grad_f, double* c,
                             double* jac_val, double* hess_val, unsigned what,
                             hipStream_t stream) {
  if (!b || !x) return fail(ACOPF_EINVAL, "null batch or x");
  if (what & ~unsigned(ACOPF_ALL)) return fail(ACOPF_EINVAL, "unknown bits in what");
  if (((what & ACOPF_F) && !f) || ((what & ACOPF_GRADF) && !grad_f) || ((what & ACOPF_C) && !c) ||
      ((what & ACOPF_J) && !jac_val) ||
      ((what & ACOPF_H) && (!hess_val || !lambda || !sigma)))
    return fail(ACOPF_EINVAL, "a selected output (or lambda/sigma for ACOPF_H) is null");
  if (b->nparts > kScratchParts)
    return fail(ACOPF_EINVAL, "the batch needs " + std::to_string(b->nparts) +
                                  " objective partials; the allocation-free evaluation holds at most " +
                                  std::to_string(kScratchParts));
  if (!what) return ACOPF_OK;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  double* sp = nullptr;
  int rc = scratch_address(cur, &sp);
  if (rc) return rc;
  Bufs bufs{};
  bufs.x = x;
  bufs.lam = (what & ACOPF_H) ? lambda : nullptr;
  bufs.sigma = (what & ACOPF_H) ? sigma : nullptr;
  bufs.f = (what & ACOPF_F) ? f : nullptr;
  bufs.gradf = (what & ACOPF_GRADF) ? grad_f : nullptr;
  bufs.c = (what & ACOPF_C) ? c : nullptr;
  bufs.jac = (what & ACOPF_J) ? jac_val : nullptr;
  bufs.hess = (what & ACOPF_H) ? hess_val : nullptr;
  bufs.fpart = sp;
  // always a direct launch: capturing and instantiating a graph allocates
  const unsigned variant = variant_of(what) | (b->form == ACOPF_CARTESIAN ? W_CART : 0u);
  e = enqueue(b, variant, bufs, stream);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  return ACOPF_OK;
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
  return enqueue_range(b, first, count, x, sigma, lambda, f, grad_f, c, jac_val, hess_val, what,
                       stream);
}

int acopf_batch_serve_window(acopf_batch b, int32_t first, int32_t count, const uint64_t* seeds,
                             double pmin, double pmax, double qmin, double qmax, double* x,
                             double* lambda, double* sigma, double* f, double* grad_f, double* c,
                             double* jac_val, double* hess_val, hipStream_t stream) {
  if (!b || !seeds || !x || !lambda || !sigma || !f || !grad_f || !c || !jac_val || !hess_val)
    return fail(ACOPF_EINVAL, "null argument");
  if (first < 0 || count < 1 || first > b->count - count)
    return fail(ACOPF_EINVAL, "instance window out of range");
  if (count > kWindowSeeds)
    return fail(ACOPF_EINVAL, "at most " + std::to_string(kWindowSeeds) + " instances per window");
  if (b->form != ACOPF_POLAR) return fail(ACOPF_EINVAL, "iterates are drawn for the polar representation only");
  for (int32_t k = first; k < first + count; ++k)
    if (b->nets[k]->base->topo.sl.ns) return fail(ACOPF_EINVAL, "iterates are not drawn for nets with slack variables");
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  e = launch_draw_window(b->d_table, first, count, b->max_len, seeds, pmin, pmax, qmin, qmax, x,
                         lambda, sigma, stream);
  if (e != hipSuccess) return hip_fail(e, "draw kernel launch");
  return enqueue_range(b, first, count, x, sigma, lambda, f, grad_f, c, jac_val, hess_val,
                       ACOPF_ALL, stream);
}

}  // extern "C"

namespace {

int enqueue_range(acopf_batch_s* b, int32_t first, int32_t count, const double* x,
                  const double* sigma, const double* lambda, double* f, double* grad_f, double* c,
                  double* jac_val, double* hess_val, unsigned what, hipStream_t stream) {
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
  hipError_t e;
  const int t0 = b->inst_tile_off[first], t1 = b->inst_tile_off[first + count];
  InstOff none{};
  none.work = b->d_work;  // the tiles' w0 index this array
  const unsigned variant = variant_of(what) | (b->form == ACOPF_CARTESIAN ? W_CART : 0u);
  e = launch_eval(variant, b->sched.tile_be, bufs, b->d_table, none, b->d_tiles_inst + t0,
                  t1 - t0, 0, stream);
  if (e == hipSuccess && bufs.f && b->max_chunks > 1)
    e = launch_fsum(b->d_table, none, first, count, bufs.fpart, bufs.f, stream);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  return ACOPF_OK;
}

}  // namespace

extern "C" {

int acopf_batch_draw_iterates(acopf_batch b, int32_t first, int32_t count, const uint64_t* seeds,
                              double pmin, double pmax, double qmin, double qmax, double* x,
                              double* lambda, hipStream_t stream) {
  if (!b || !seeds || !x || !lambda) return fail(ACOPF_EINVAL, "null argument");
  if (first < 0 || count < 1 || first > b->count - count)
    return fail(ACOPF_EINVAL, "instance window out of range");
  if (count > 65535) return fail(ACOPF_EINVAL, "at most 65535 instances per draw");
  if (b->form != ACOPF_POLAR) return fail(ACOPF_EINVAL, "iterates are drawn for the polar representation only");
  for (acopf_net n : b->nets)
    if (n->base->topo.sl.ns) return fail(ACOPF_EINVAL, "iterates are not drawn for nets with slack variables");
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

int acopf_batch_xdot(acopf_batch b, const double* a, const double* v, double* out,
                     hipStream_t stream) {
  if (!b || !a || !v || !out) return fail(ACOPF_EINVAL, "null argument");
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  e = launch_xdot(b->d_table, b->count, a, v, out, stream);
  if (e != hipSuccess) return hip_fail(e, "dot kernel launch");
  return ACOPF_OK;
}

// ---------------------------------------------------------------------------
// coupling rows

int acopf_couple_create(acopf_batch b, const int32_t* child, const int32_t* parent,
                        int32_t nlinks, acopf_couple* out) {
  if (!out) return fail(ACOPF_EINVAL, "null output handle");
  *out = nullptr;
  if (!b || nlinks < 0 || (nlinks > 0 && (!child || !parent)))
    return fail(ACOPF_EINVAL, "null batch or link arrays");
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(ACOPF_EINVAL, "batch lives on another device");
  acopf_couple cp = nullptr;
  try {
    cp = new acopf_couple_s;
    cp->batch = b;
    for (int32_t l = 0; l < nlinks; ++l) {
      const int32_t a = child[l], p = parent[l];
      if (a < 0 || a >= b->count || p < 0 || p >= b->count)
        return delete cp, fail(ACOPF_EINVAL, "link " + std::to_string(l) + ": instance out of range");
      if (a == p)
        return delete cp, fail(ACOPF_EINVAL, "link " + std::to_string(l) + " joins an instance to itself");
      const acopf_dims &da = b->nets[a]->dims, &dp = b->nets[p]->dims;
      if (da.ngen != dp.ngen)
        return delete cp, fail(ACOPF_EINVAL, "link " + std::to_string(l) +
                                                  ": the instances have different generator counts");
      // Pg block of x: [theta; v; Pg; Qg]
      for (int32_t k = 0; k < da.ngen; ++k) {
        cp->cols.push_back(b->xo[a] + 2 * int64_t(da.nbus) + k);
        cp->cols.push_back(b->xo[p] + 2 * int64_t(dp.nbus) + k);
      }
    }
    cp->rows = int64_t(cp->cols.size() / 2);
    if (cp->rows >= (int64_t(1) << 30))
      return delete cp, fail(ACOPF_EINVAL, "more than 2^30 coupling rows");
    // the transposed product: rows touching each coupled column, in row order
    std::vector<std::pair<int64_t, int32_t>> ent;
    ent.reserve(cp->cols.size());
    for (int64_t r = 0; r < cp->rows; ++r) {
      ent.push_back({cp->cols[2 * r], int32_t(r << 1)});
      ent.push_back({cp->cols[2 * r + 1], int32_t((r << 1) | 1)});
    }
    std::sort(ent.begin(), ent.end());
    std::vector<int64_t> tcol;
    std::vector<int32_t> tptr, tent;
    for (size_t q = 0; q < ent.size(); ++q) {
      if (q == 0 || ent[q].first != ent[q - 1].first) {
        tcol.push_back(ent[q].first);
        tptr.push_back(int32_t(q));
      }
      tent.push_back(ent[q].second);
    }
    tptr.push_back(int32_t(ent.size()));
    cp->ncols = int32_t(tcol.size());
    const size_t s_cols = align_up(std::max<size_t>(cp->cols.size(), 1) * sizeof(int64_t));
    const size_t s_tcol = align_up(std::max<size_t>(tcol.size(), 1) * sizeof(int64_t));
    const size_t s_tptr = align_up(tptr.size() * sizeof(int32_t));
    const size_t s_tent = align_up(std::max<size_t>(tent.size(), 1) * sizeof(int32_t));
    e = hipMalloc(&cp->mem, s_cols + s_tcol + s_tptr + s_tent);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      cp->mem = nullptr;
      delete cp;
      return fail(ACOPF_ENOMEM, std::string("hipMalloc of coupling rows: ") + hipGetErrorString(e));
    }
    char* base = static_cast<char*>(cp->mem);
    cp->d_cols = reinterpret_cast<int64_t*>(base);
    cp->d_tcol = reinterpret_cast<int64_t*>(base + s_cols);
    cp->d_tptr = reinterpret_cast<int32_t*>(base + s_cols + s_tcol);
    cp->d_tent = reinterpret_cast<int32_t*>(base + s_cols + s_tcol + s_tptr);
    if (!cp->cols.empty())
      e = hipMemcpy(cp->d_cols, cp->cols.data(), cp->cols.size() * sizeof(int64_t),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess && !tcol.empty())
      e = hipMemcpy(cp->d_tcol, tcol.data(), tcol.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(cp->d_tptr, tptr.data(), tptr.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tent.empty())
      e = hipMemcpy(cp->d_tent, tent.data(), tent.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(cp->mem);
      delete cp;
      return hip_fail(e, "coupling upload");
    }
  } catch (const std::bad_alloc&) {
    if (cp) {
      if (cp->mem) (void)hipFree(cp->mem);
      delete cp;
    }
    return fail(ACOPF_ENOMEM, "host allocation failed");
  }
  b->refs.fetch_add(1);
  *out = cp;
  t_err.clear();
  return ACOPF_OK;
}

int acopf_couple_destroy(acopf_couple cp) {
  if (!cp) return ACOPF_OK;
  if (cp->mem) (void)hipFree(cp->mem);
  cp->batch->refs.fetch_sub(1);
  delete cp;
  return ACOPF_OK;
}

int acopf_couple_dims(acopf_couple cp, int64_t* rows, int64_t* nnz) {
  if (!cp) return fail(ACOPF_EINVAL, "null coupling");
  if (rows) *rows = cp->rows;
  if (nnz) *nnz = 2 * cp->rows;
  return ACOPF_OK;
}

int acopf_couple_pattern(acopf_couple cp, int64_t* rowptr, int64_t* col) {
  if (!cp || !rowptr || !col) return fail(ACOPF_EINVAL, "null coupling or output array");
  for (int64_t r = 0; r <= cp->rows; ++r) rowptr[r] = 2 * r;
  for (int64_t r = 0; r < cp->rows; ++r) {
    const int64_t a = cp->cols[2 * r], p = cp->cols[2 * r + 1];
    col[2 * r] = std::min(a, p);
    col[2 * r + 1] = std::max(a, p);
  }
  return ACOPF_OK;
}

static int couple_device(acopf_couple cp) {
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != cp->batch->device) return fail(ACOPF_EINVAL, "coupling lives on another device");
  return ACOPF_OK;
}

int acopf_couple_eval(acopf_couple cp, const double* x, double* c, double* jac_val,
                      hipStream_t stream) {
  if (!cp || !x) return fail(ACOPF_EINVAL, "null coupling or x");
  if (int rc = couple_device(cp)) return rc;
  hipError_t e = launch_couple_rows(cp->d_cols, cp->rows, x, c, jac_val, stream);
  return e == hipSuccess ? ACOPF_OK : hip_fail(e, "coupling rows launch");
}

int acopf_couple_vjp(acopf_couple cp, const double* w, double* u, hipStream_t stream) {
  if (!cp || !w || !u) return fail(ACOPF_EINVAL, "null coupling, w or u");
  if (int rc = couple_device(cp)) return rc;
  hipError_t e = launch_couple_vjp(cp->d_tcol, cp->d_tptr, cp->d_tent, cp->ncols, w, u, stream);
  return e == hipSuccess ? ACOPF_OK : hip_fail(e, "coupling VJP launch");
}

int acopf_couple_jvp(acopf_couple cp, const double* d, double* out, hipStream_t stream) {
  if (!cp || !d || !out) return fail(ACOPF_EINVAL, "null coupling, d or out");
  if (int rc = couple_device(cp)) return rc;
  hipError_t e = launch_couple_rows(cp->d_cols, cp->rows, d, out, nullptr, stream);
  return e == hipSuccess ? ACOPF_OK : hip_fail(e, "coupling JVP launch");
}

}  // extern "C"
