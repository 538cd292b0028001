// Internal layout shared by the host code and the gfx950 kernels.
//
// Everything a kernel reads about a network lives in one NetDev record in
// device memory; everything about one evaluation instance (which net, which
// outage, where its slices of the packed buffers start) in one InstOff.
// Work is cut into tiles of two kinds:
//   bus tile  a contiguous range of buses.  A host-built work list names
//             every branch touching the tile (branch, endpoints, LDS slots of
//             its ends); each is evaluated once into per-branch-end LDS
//             records.  A host-built slot map then describes every output
//             entry of the tile's CSR row segments as a signed sum of a
//             contiguous range of records (branch ends are sorted by bus and
//             far bus, so a diagonal entry sums a bus's ends and an
//             off-diagonal entry the ends of one parallel-branch group), so
//             one lane computes and stores one output entry.  The tile also
//             writes the balance rows of c, and the flow-limit rows of the
//             branches whose from-bus it owns.
//   gen tile  a fixed chunk of generators: f, grad f, the Pg diagonal of H
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace acopf {

constexpr int kGenChunk = 256;   // generators per gen tile; fixes the f reduction tree
constexpr uint32_t kNoSlot = 0xFFFFu;

enum TileKind : int32_t { TILE_BUS = 1, TILE_GEN = 2 };

// A unit of work.  Bus tile: buses [a0, a1), branch ends [e0, e0 + ne) of the
// adjacency, work items [w0, w0 + nw), slot map [sm0, sm0 + nP + nT + nV) for
// the J P rows (the J Q rows share it), the H theta rows and the H v rows,
// whose base starts are jP0, jQ0, hT0, hV0.  Gen tile: generators [a0, a1);
// kind_aux = (chunk << 2) | kind.
struct Tile {
  int32_t inst, kind_aux, a0, a1, e0, ne, w0, nw;
  int32_t sm0, nP, nT, nV, jP0, jQ0, hT0, hV0;
};

// One branch evaluated by a bus tile: branch id, its from and to bus, and
// the tile-local branch-end slots of the two ends (kNoSlot if that end's bus
// is outside the tile), packed as slot_from | slot_to << 16.
struct WorkItem {
  int32_t l, f, t;
  uint32_t slots;
};

// One output entry, packed in 32 bits: value = (-1)^neg * sum of record
// field `field` over branch ends [ea, ea + cnt) of the tile, plus the bus
// extra of `kind` for tile-local bus `bl`:
//   ea (9 bits) | cnt << 9 (10) | field << 19 (2) | neg << 21 | kind << 22 (2) | bl << 24 (8)
enum SlotKind : int32_t {
  SK_SUM = 0,      // plain signed sum
  SK_JDIAG_V = 1,  // J diagonal d/dv_i: + 2 gs v_i (P row) or - 2 bs v_i (Q row)
  SK_GEN = 2,      // generator column: the constant -1
  SK_HDIAG_V = 3,  // H (v_i, v_i): + 2 (lP_i gs - lQ_i bs)
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

// One evaluation instance.  Offsets index the packed buffers of Bufs.  An
// N-1 instance whose removed branch had no parallel twin loses 8 Jacobian
// and 4 Hessian slots; their base positions, ascending, are rj and rh
// (INT32_MAX when nothing is removed), and every later entry moves down by
// the number of removed positions before it.
struct InstOff {
  const NetDev* net;
  const WorkItem* work;     // work items of the schedule in use
  const uint32_t* slots;    // slot map of the schedule in use
  int32_t out_l;            // removed branch, -1 for none
  int32_t out_rm;           // 1 if the removal drops the (p, q) slots
  int32_t rj[8];
  int32_t rh[4];
  int64_t xo;               // x, grad f, u
  int64_t co;               // lambda, c, w_c
  int64_t jo;               // Jacobian values
  int64_t ho;               // Hessian values
  int32_t k;                // instance index: f, sigma, w_f
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
  const double* dir;        // direction of a Hessian- or Jacobian-vector product
  double* out;              // H dir (length n) or J dir (length m)
  double* fpart;            // f partial sums, one per generator chunk
};

enum : unsigned {
  W_F = 1u, W_GRADF = 2u, W_C = 4u, W_J = 8u, W_H = 16u, W_VJP = 32u, W_HVP = 64u, W_JVP = 128u,
};

// Tile capacities of one schedule: workgroup size, branch ends per bus tile
// (LDS records), buses per bus tile (LDS bus terms) and slot-map entries per
// lane (prefetched into registers at the start of the tile).
struct TileCaps {
  int32_t wg, be, nbus, spl;
};

constexpr TileCaps kCaps64 = {64, 64, 32, 8};
constexpr TileCaps kCaps128 = {128, 128, 64, 8};
constexpr TileCaps kCaps256 = {256, 256, 128, 8};
constexpr TileCaps kCaps512 = {256, 512, 256, 12};
constexpr int kDefaultTileBe = 256;

inline bool caps_for(int tile_be, TileCaps* out) {
  switch (tile_be) {
    case 64: *out = kCaps64; return true;
    case 128: *out = kCaps128; return true;
    case 256: *out = kCaps256; return true;
    case 512: *out = kCaps512; return true;
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
  K_HVP = W_HVP,
  K_JVP = W_JVP,
};

// Enqueue the f reduction for instances [first, first + count) (table) or
// the one instance `one` (table == nullptr, first = 0, count = 1).
hipError_t launch_fsum(const InstOff* table, const InstOff& one, int first, int count,
                       const double* fpart, double* f, hipStream_t stream);

// Enqueue one evaluation kernel over `ntiles` tiles.  grid = 0 launches one
// workgroup per tile; otherwise a persistent grid of `grid` workgroups
// strides over the tile list.
hipError_t launch_eval(unsigned kvariant, int tile_be, const Bufs& b, const InstOff* table,
                       const InstOff& one, const Tile* tiles, int ntiles, int grid,
                       hipStream_t stream);

// Enqueue the random-iterate draw for instances [first, first + count) of a
// batch table; max_len bounds n + m over those instances.
hipError_t launch_draw(const InstOff* table, int first, int count, int max_len,
                       const uint64_t* seeds, double pmin, double pmax, double qmin, double qmax,
                       double* x, double* lam, hipStream_t stream);

}  // namespace acopf
