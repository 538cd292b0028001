// Host-side objects behind the C ABI handles.
#pragma once

#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "acopf.h"
#include "acopf_internal.h"

namespace acopf {

// Host copy of a base network and everything derived from it.
struct Topology {
  int32_t nb = 0, nl = 0, ng = 0, nchunks = 1;
  int32_t gchunks = 0;  // generator chunks; slack chunks follow up to nchunks
  int32_t form = ACOPF_POLAR;  // ACOPF_POLAR or ACOPF_CARTESIAN
  SlackDev sl{};               // slack blocks (their columns follow Qg)
  double base = 100.0;
  std::vector<int2> ft;
  std::vector<BranchY> y;
  std::vector<BranchY6> y6;        // y without (gtf, btf)
  std::vector<double2> tf;         // (gtf, btf)
  std::vector<uint8_t> shifted;    // 1 where (gtf, btf) is not (gft, bft) bit for bit
  std::vector<double4> bus;
  std::vector<double> rate;       // apparent-power limit per branch (<= 0: none)
  std::vector<int32_t> gen_bus;
  std::vector<double> c2, c1, c0;
  std::vector<int32_t> be_ptr, be;
  std::vector<int2> acnt;
  std::vector<int4> rows;
  std::vector<int32_t> gen_ptr, gen_list;
  int64_t nnz_jac = 0, nnz_hess = 0;
  int32_t jflow = 0, hpg = 0;
};

// Tiles and work items of one schedule (tile size) for a network.
struct Schedule {
  std::vector<Tile> tiles;        // [bus tiles][gen tiles]
  std::vector<WorkItem> work;
  int counts[2] = {0, 0};
};

// A base network resident on one device; shared by its outage children.
struct Base {
  Topology topo;
  int device = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  NetDev* d_net = nullptr;
  Tile* d_tiles = nullptr;           // plain-path schedule on the device
  WorkItem* d_work = nullptr;
  Schedule plain;
  ~Base();
};

}  // namespace acopf

struct acopf_net_s {
  std::shared_ptr<acopf::Base> base;
  acopf_net_s* parent = nullptr;
  int32_t out_l = -1, out_p = -1, out_q = -1, out_rm = 0;
  int32_t rj[8] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX,
                   INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  int32_t rh[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  acopf_dims dims{};
  void* scratch = nullptr;           // f partials of the plain path
  double* d_fpart = nullptr;
  std::atomic<int> refs{0};          // outage children and batches using this net
};

namespace acopf {

extern thread_local std::string t_err;
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
int build_topology(const acopf_net_desc* d, const acopf_net_opts* o, Topology* T);
int outage_info(const Topology& T, int32_t l, int32_t* p, int32_t* q, int32_t* rm);
void fill_dims(const Topology& T, int32_t outage, int32_t rm, acopf_dims* d);
void flow_limits(const Topology& T, int32_t outage, double* hmax);
void build_pattern(const Topology& T, int32_t outage, std::vector<int32_t>* jp,
                   std::vector<int32_t>* jc, std::vector<int32_t>* hp, std::vector<int32_t>* hc);
int make_tiles(const Topology& T, int tile_be, Schedule* S);
void removed_slots(const Topology& T, int32_t p, int32_t q, int32_t rm, int32_t rj[8],
                   int32_t rh[4]);
int upload_base(Base* B);
int net_init_scratch(acopf_net_s* net);
InstOff net_inst(const acopf_net_s* net);
int check_device(const acopf_net_s* net);

// Seeds of one served window, passed by value in the draw kernel's arguments.
constexpr int kWindowSeeds = 64;
struct WindowSeeds {
  uint64_t s[kWindowSeeds];
};

// Draw the iterates of instances [first, first + count) from host seeds and
// set their sigma to 1 (count <= kWindowSeeds).
hipError_t launch_draw_window(const InstOff* table, int first, int count, int max_len,
                              const uint64_t* host_seeds, double pmin, double pmax, double qmin,
                              double qmax, double* x, double* lam, double* sigma,
                              hipStream_t stream);

// Per-instance dot products over the packed x layout of a batch table:
// out[k] = a_k . b_k (fixed summation order).
hipError_t launch_xdot(const InstOff* table, int count, const double* a, const double* b,
                       double* out, hipStream_t stream);

}  // namespace acopf
