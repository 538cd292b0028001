// Internal layout shared by the host code and the gfx950 kernels.
//
// Everything a kernel reads about a network lives in one NetDev record in
// device memory; everything about one evaluation instance (which net, which
// outage, where its slices of the packed buffers start) in one InstOff.
// Work is cut into tiles of two kinds:
//   bus tile  a contiguous range of buses.  A host-built work list names
//             every branch touching the tile (branch, endpoints, LDS slots of
//             its ends, and the base positions of the off-diagonal entries
//             it owns in the tile's rows); each is evaluated once.  The lane
//             places those off-diagonal entries in an LDS copy of the tile's
//             J and H row segments (a group of parallel branches sits in
//             consecutive lanes of one wave and its first lane places the
//             group's sum) and leaves per-branch-end records in LDS; after a
//             barrier, a lane per bus sums its ends' records into the bus's
//             diagonal entries (placed in the same copy) and balance rows;
//             after another, the workgroup stores the row segments with
//             consecutive lanes on consecutive entries.  The tile also writes
//             the flow-limit rows of the branches whose from-bus it owns.
//             A variant forming both J and H runs this twice in one tile:
//             flows and J (records, rows, store), then H in the same LDS.
//   gen tile  a fixed chunk of cost items (the generators, then the slack
//             variables of a net that has them): f, grad f, the Pg diagonal of H
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace acopf {

constexpr int kGenChunk = 256;   // reduction slots per gen tile; fixes the f reduction tree
constexpr int kGenPerSlot = 4;   // generators per reduction slot: a generator chunk holds 1024
constexpr int kSlackPerSlot = 8; // slack items per reduction slot: a slack chunk holds 2048
constexpr uint32_t kNoSlot = 0xFFFFu;

enum TileKind : int32_t { TILE_BUS = 1, TILE_GEN = 2 };

// A unit of work.  Bus tile: buses [a0, a1), branch ends [e0, e0 + ne) of the
// adjacency, work items [w0, w0 + nw) of the launch's work array (a batch
// holds every distinct base's items back to back), the largest parallel-branch group
// among them (gmax), and the tile's row segments as base positions: J P rows
// [jP0, jP0 + nP) (Q rows [jQ0, jQ0 + nP)), H theta rows [hT0, hT0 + nT),
// H v rows [hV0, hV0 + nV).  Gen tile: cost items [a0, a1) (item k >= ng is
// slack variable k - ng);
// kind_aux = (chunk << 2) | kind.
// A product bus tile may serve up to kProdInst - 1 further instances of the
// same base network (more[]; -1 past the last).
constexpr int kProdInst = 4;
struct Tile {
  int32_t inst, kind_aux, a0, a1, e0, ne, w0, nw;
  int32_t gmax, nP, nT, nV, jP0, jQ0, hT0, hV0;
  int32_t more[kProdInst - 1] = {-1, -1, -1};
};

// One branch evaluated by a bus tile, in 32 bytes.  l < 0 pads the list so
// that no parallel-branch group straddles two waves.  slots = slot_from |
// slot_to << 16: the tile-local branch-end records of the two ends (kNoSlot
// if that end's bus is outside the tile).  With lo < hi the end buses, the
// positions this tile stores, relative to the start of the tile's row
// segment of the same kind (kNoPos where the end's bus is outside the tile;
// Q rows at the same offsets in the Q segment):
//   jlo  J (P_lo, theta_hi); (P_lo, v_hi) at jlo + alo   (J P rows)
//   hvlo H (v_lo, theta_hi)                              (H v rows)
//   jhi  J (P_hi, theta_lo); (P_hi, v_lo) at jhi + ahi   (J P rows)
//   hvhi H (v_hi, theta_lo); (v_hi, v_lo) at hvhi + ahi  (H v rows)
//   hthi H (theta_hi, theta_lo)                          (H theta rows)
// a_e = |{e} u N(e)|, the length of the theta part of bus e's rows.
// grp: for the first branch of a group of parallel branches, the group size
// (1 for a branch without a twin); 0 for the other members, which follow in
// the next lanes.  shifted: the branch shifts phase, so the to side's
// off-diagonal admittances differ from the from side's (NetDev::br_tf).
constexpr uint32_t kNoPos = 0xFFFFu;
struct WorkItem {
  int32_t l, f, t;
  uint32_t slots;
  uint32_t j;    // jlo | jhi << 16
  uint32_t hv;   // hvlo | hvhi << 16
  uint32_t th;   // hthi | grp << 16 | shifted << 24
  uint32_t a;    // alo | ahi << 16
  __host__ __device__ uint32_t jlo() const { return j & 0xFFFFu; }
  __host__ __device__ uint32_t jhi() const { return j >> 16; }
  __host__ __device__ uint32_t hvlo() const { return hv & 0xFFFFu; }
  __host__ __device__ uint32_t hvhi() const { return hv >> 16; }
  __host__ __device__ uint32_t hthi() const { return th & 0xFFFFu; }
  __host__ __device__ int grp() const { return int((th >> 16) & 0xFFu); }
  __host__ __device__ bool shifted() const { return ((th >> 24) & 1u) != 0; }
  __host__ __device__ uint32_t alo() const { return a & 0xFFFFu; }
  __host__ __device__ uint32_t ahi() const { return a >> 16; }
};

// Feasibility slack blocks of a network (at most 6: dP+, dP-, dQ+, dQ-, Pl,
// Ql), each nb variables after Qg.  Block k: balance row row[k] (0 active,
// 1 reactive) with coefficient coef[k], penalty c2[k] (B s)^2 + c1[k] B s.
// nsp blocks go to each active row (the same number to each reactive row).
constexpr int kMaxSlack = 6;
struct SlackDev {
  int32_t ns, nsp;
  int32_t row[kMaxSlack];
  double coef[kMaxSlack], c2[kMaxSlack], c1[kMaxSlack];
};

// Admittances of one branch (pi model, from-side ideal transformer).
struct BranchY {
  double gff, bff, gft, bft, gtf, btf, gtt, btt;
};

// What the kernels load per branch: BranchY without (gtf, btf), which equal
// (gft, bft) unless the branch shifts phase; a shifting branch's pair is
// kept apart (NetDev::br_tf) and read only by the lanes that need it.
struct alignas(16) BranchY6 {
  double gff, bff, gft, bft, gtt, btt;
};

struct NetDev {
  int32_t nb, nl, ng, nchunks;
  const BranchY6* br_y;     // [nl]
  const double2* br_tf;     // [nl] (g_tf, b_tf), read for phase-shifting branches only
  const double4* bus;       // [nb] (pd, qd, gs, bs)
  const int32_t* be_ptr;    // [nb + 1] branch ends of bus i: adjacency positions be_ptr[i] ..
  const int32_t* gen_ptr;   // [nb + 1] generators at bus i: gen_list[gen_ptr[i] .. gen_ptr[i+1])
  const int32_t* gen_list;  // [ng]
  const int32_t* gen_bus;   // [ng]
  const double* gen_c2;     // [ng]
  const double* gen_c1;
  const double* gen_c0;
  const int4* rows;         // [nb + 1] base row starts: J P, J Q, H theta, H v
  const int2* acnt;         // [nb] |{i} u N(i)|, |{j in N(i) : j < i}|
  double base_mva;
  int32_t jflow;            // base start of the flow rows in J
  int32_t hpg;              // base start of the Pg rows in H
  int32_t qoff;             // J Q row of a bus minus its P row
  int32_t gen_ident;        // 1 if gen_list is the identity (generators numbered by bus)
  SlackDev sl;              // slack blocks (sl.ns = 0: none)
};

// One evaluation instance.  Offsets index the packed buffers of Bufs.  An
// N-1 instance whose removed branch had no parallel twin loses 8 Jacobian
// and 4 Hessian slots; their base positions, ascending, are rj and rh
// (INT32_MAX when nothing is removed), and every later entry moves down by
// the number of removed positions before it.
struct InstOff {
  const NetDev* net;
  const WorkItem* work;     // work items of the schedule in use; kernels read them through
                            // the launch's `one` argument (a batch's tiles index its array)
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
  double* fpart;            // f partial sums, one per cost-item chunk
};

enum : unsigned {
  W_F = 1u, W_GRADF = 2u, W_C = 4u, W_J = 8u, W_H = 16u, W_VJP = 32u, W_HVP = 64u, W_JVP = 128u,
  W_CART = 256u,  // power-balance-cartesian representation (x = [e; f; Pg; Qg])
};

// Instances of one base network per product bus tile: kProdInst for the VJP
// and the HVP; three for the JVP, whose tiles of four need more registers
// than four waves per SIMD leave.
__host__ __device__ constexpr int prod_group(unsigned what) {
  return (what & W_JVP) != 0 ? 3 : kProdInst;
}

// Tile capacities of one schedule class (the schedule's tile_be value):
// workgroup size, branch ends per bus tile (LDS records), buses per bus tile
// (one lane each) and entries of the tile's J and H row segments staged in
// LDS (the J rows, 2 nP, and afterwards the H rows, nT + nV, each within
// it).  The fused variant needs 6 record doubles per end plus the staged
// J rows (about 5.5 entries per end on power grids, the H rows about 3);
// classes 64, 128 and 256 are sized so that this stays within 160 KB of LDS
// at four waves per SIMD (10, 20 and 40 KB per workgroup), class 512 admits
// buses with up to 512 branch ends at lower occupancy.
struct TileCaps {
  int32_t cls, wg, be, nbus, stage;
};

constexpr TileCaps kCaps64 = {64, 64, 110, 55, 616};
constexpr TileCaps kCaps128 = {128, 128, 220, 110, 1232};
constexpr TileCaps kCaps256 = {256, 256, 440, 220, 2464};
constexpr TileCaps kCaps512 = {512, 256, 512, 256, 6144};
constexpr int kMaxGroup = 64;  // parallel branches between one bus pair
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

// Coupling rows: lane per row (values and +-1 Jacobian entries), and lane
// per coupled column for u += J' w.
hipError_t launch_couple_rows(const int64_t* cols, int64_t rows, const double* x, double* c,
                              double* jac, hipStream_t stream);
hipError_t launch_couple_vjp(const int64_t* tcol, const int32_t* tptr, const int32_t* tent,
                             int32_t ncols, const double* w, double* u, hipStream_t stream);

}  // namespace acopf
