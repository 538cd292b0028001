// Internal layout shared by the host code and the gfx950 kernels.
//
// Everything a kernel reads about a network lives in one NetDev record in
// device memory; everything about one evaluation instance (which net, which
// outage, where its slices of the packed buffers start) in one InstOff.
// Work is cut into tiles of two kinds:
//   bus tile  a contiguous range of buses: every branch touching them is
//             evaluated once (a host-built work list names the branch, its
//             endpoints and the LDS slots of its ends inside the tile); the
//             tile writes the power-balance rows of c and J, the theta/v rows
//             of the Hessian (or the VJP's theta/v entries), and the flow-limit
//             rows of the branches whose from-bus it owns
//   gen tile  a fixed chunk of generators: f, grad f, the Pg diagonal of H
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace acopf {

constexpr int kGenChunk = 256;   // generators per gen tile; fixes the f reduction tree
constexpr uint32_t kNoSlot = 0xFFFFu;

enum TileKind : int32_t { TILE_BUS = 1, TILE_GEN = 2 };

// A unit of work.  Bus tile: buses [a0, a1), branch ends [e0, e0 + ne) of the
// adjacency, work items [w0, w0 + nw).  Gen tile: generators [a0, a1);
// kind_aux = (chunk << 2) | kind.
struct Tile {
  int32_t inst, kind_aux, a0, a1, e0, ne, w0, nw;
};

// One branch evaluated by a bus tile: branch id, its from and to bus, and
// the tile-local branch-end slots of the two ends (kNoSlot if that end's bus
// is outside the tile), packed as slot_from | slot_to << 16.
struct WorkItem {
  int32_t l, f, t;
  uint32_t slots;
};

// Admittances of one branch (pi model, from-side ideal transformer).
struct BranchY {
  double gff, bff, gft, bft, gtf, btf, gtt, btt;
};

struct NetDev {
  int32_t nb, nl, ng, nchunks;
  const BranchY* br_y;      // [nl]
  const double4* bus;       // [nb] (pd, qd, gs, bs)
  const int32_t* be_ptr;    // [nb + 1] branch ends of bus i: adjacency positions be_ptr[i] ..
  const int2* acnt;         // [nb] (|{i} u N(i)|, #distinct neighbours below i)
  const int4* rows;         // [nb + 1] base starts of (J P row, J Q row, H theta row, H v row)
  const int32_t* gen_ptr;   // [nb + 1] generators at bus i: gen_list[gen_ptr[i] .. gen_ptr[i+1])
  const int32_t* gen_list;  // [ng]
  const int32_t* gen_bus;   // [ng]
  const double* gen_c2;     // [ng]
  const double* gen_c1;
  const double* gen_c0;
  double base_mva;
  int32_t jflow;            // base start of the flow rows in J
  int32_t hpg;              // base start of the Pg rows in H
};

// One evaluation instance.  Offsets index the packed buffers of Bufs.
struct InstOff {
  const NetDev* net;
  const WorkItem* work;     // work items of the schedule in use
  int32_t out_l;            // removed branch, -1 for none
  int32_t out_p, out_q;     // its endpoints, p < q
  int32_t out_rm;           // 1 if no parallel branch keeps the (p, q) slots
  int64_t xo;               // x, grad f, u
  int64_t co;               // lambda, c, w_c
  int64_t jo;               // Jacobian values
  int64_t ho;               // Hessian values
  int32_t k;                // instance index: f, sigma, w_f, ticket
  int32_t fpo;              // first f partial of this instance
};

struct Bufs {
  const double* x;
  const double* lam;
  const double* wc;
  const double* sigma;      // per-instance array or nullptr (then sigma_v)
  const double* wf;         // per-instance array or nullptr (then wf_v)
  double sigma_v, wf_v;
  double* f;
  double* gradf;
  double* c;
  double* jac;
  double* hess;
  double* u;
  double* fpart;            // f partial sums, one per generator chunk
  uint32_t* ticket;         // per instance: gen chunks finished in this launch
};

enum : unsigned {
  W_F = 1u, W_GRADF = 2u, W_C = 4u, W_J = 8u, W_H = 16u, W_VJP = 32u,
};

// Tile capacities of one schedule: workgroup size, branch ends per bus tile
// and the LDS staging capacity (doubles) for the tile's J and H row segments.
struct TileCaps {
  int32_t wg, be, stage;
};

// Staging of ~10 doubles per branch end covers grids of mean degree ~3; the
// tiler closes a tile early when a dense patch would overflow it.
constexpr TileCaps kCaps64 = {64, 64, 640};
constexpr TileCaps kCaps128 = {128, 128, 1280};
constexpr TileCaps kCaps256 = {256, 256, 2560};
constexpr int kDefaultTileBe = 128;

inline bool caps_for(int tile_be, TileCaps* out) {
  switch (tile_be) {
    case 64: *out = kCaps64; return true;
    case 128: *out = kCaps128; return true;
    case 256: *out = kCaps256; return true;
    default: return false;
  }
}

// Kernel variants (compile-time `what`).
enum : unsigned {
  K_FG = W_F | W_GRADF | W_C,
  K_J = W_J,
  K_H = W_H,
  K_ALL = W_F | W_GRADF | W_C | W_J | W_H,
  K_VJP = W_VJP,
};

// Enqueue one evaluation kernel over `ntiles` tiles.  grid = 0 launches one
// workgroup per tile; otherwise a persistent grid of `grid` workgroups
// strides over the tile list.
hipError_t launch_eval(unsigned kvariant, int tile_be, const Bufs& b, const InstOff* table,
                       const InstOff& one, const Tile* tiles, int ntiles, int grid,
                       hipStream_t stream);

}  // namespace acopf
