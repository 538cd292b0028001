// gfx950 kernels for the polar ACOPF model evaluation (FP64).
//
// One kernel template covers every entry point; the compile-time variant
// selects which outputs a tile produces.  A workgroup walks a list of tiles
// (one tile per workgroup, or a persistent grid striding over the list).
//
//  bus tile  a contiguous range of buses.
//            Phase A, lane per branch touching the tile (uniform work): one
//            sincos of theta_f - theta_t, both end flows, their first
//            derivatives and the second derivatives of the branch's share of
//            the Lagrangian.  The lane stores the branch's off-diagonal
//            Jacobian and Hessian entries in the rows of the tile's buses at
//            host-computed positions (parallel branches share those entries:
//            a group sits in consecutive lanes of one wave and its first lane
//            stores the sum, added in lane order), and leaves, per end
//            inside the tile, that end's share of its own bus's rows and
//            diagonal entries in an LDS record.  A branch whose from-bus the
//            tile owns also writes its flow-limit rows: h = P^2 + Q^2 at both
//            ends and their Jacobian rows 2 (P dP + Q dQ) on (theta_f,
//            theta_t, v_f, v_t).
//            Phase B, lane per bus: the records of the bus's ends, summed in
//            adjacency order (by far bus, then branch), plus the bus's own
//            terms (shunt, load, generation) give its diagonal entries and
//            its balance rows.  No atomics: every sum has one owner and a
//            fixed order, so results are bitwise reproducible whatever the
//            tiling.
//  gen tile  a fixed chunk of cost items (1024 generators or 2048 slack
//            variables): grad f, the Pg (or slack) diagonal of H, those
//            columns of the VJP and HVP, and a fixed-tree partial sum of the
//            cost.  A net with one chunk has f written there; otherwise a
//            second small kernel adds each instance's partials in chunk order
//            (a kernel boundary instead of fences: an agent-scope release
//            fence per chunk writes back the whole L2).
//
// The model (paper: OPFLOW section, power-balance-polar representation; the
// formulation itself is the standard polar pi-model one the paper refers to):
// for a branch with from bus f and to bus t, theta = theta_f - theta_t,
//   P_f =  g_ff v_f^2 + v_f v_t (g_ft cos theta + b_ft sin theta)
//   Q_f = -b_ff v_f^2 + v_f v_t (g_ft sin theta - b_ft cos theta)
//   P_t =  g_tt v_t^2 + v_f v_t (g_tf cos theta - b_tf sin theta)
//   Q_t = -b_tt v_t^2 - v_f v_t (g_tf sin theta + b_tf cos theta)
// The branch's share of the Lagrangian is, over its two ends e,
//   lP_e P_e + lQ_e Q_e + mu_e (P_e^2 + Q_e^2)
// with lP, lQ the balance multipliers of the end buses and mu_e the
// multiplier of the end's flow-limit row.  All flows depend on the angles only
// through theta, so every d/dtheta_t is the negative of d/dtheta_f.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "acopf_internal.h"

namespace acopf {
namespace {

// Every output is written once and never read back by these kernels: stream
// it past the caches (a non-temporal store) so that x, the multipliers and
// the network data stay resident in L2.
__device__ __forceinline__ void put(double* p, double v) { __builtin_nontemporal_store(v, p); }

// A flow-limit Jacobian row (four consecutive entries): two 16-byte stores
// when the row is 16-byte aligned (so the L2 sees two pieces of each 32-byte
// row instead of four), else four 8-byte ones.
typedef double dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void put_row4(double* p, bool al16, double a, double b, double c,
                                         double d) {
  if (al16) {
    dbl2 lo, hi;
    lo.x = a;
    lo.y = b;
    hi.x = c;
    hi.y = d;
    __builtin_nontemporal_store(lo, reinterpret_cast<dbl2*>(p));
    __builtin_nontemporal_store(hi, reinterpret_cast<dbl2*>(p + 2));
  } else {
    put(&p[0], a);
    put(&p[1], b);
    put(&p[2], c);
    put(&p[3], d);
  }
}

// A branch's admittances: the 48-byte record, and for a phase-shifting
// branch its to side's off-diagonal pair.
__device__ __forceinline__ BranchY load_branch(const NetDev& N, const WorkItem& wi) {
  const BranchY6 a = N.br_y[wi.l];
  BranchY y{a.gff, a.bff, a.gft, a.bft, a.gft, a.bft, a.gtt, a.btt};
  if (wi.shifted()) {
    const double2 p = N.br_tf[wi.l];
    y.gtf = p.x;
    y.btf = p.y;
  }
  return y;
}

// ---------------------------------------------------------------------------
// one branch: both end flows; first derivatives with respect to
// (theta_f, v_f, v_t) are formed where they are used (members below)

struct Br {
  double vf, vt, w, cP, cQ, cPt, cQt;
  double gff, bff, gtt, btt;
  double Pf, Qf, Pt, Qt;
  // d/dtheta_f (a), d/dv_f (f), d/dv_t (t) of the from flow ...
  __device__ __forceinline__ double Pf_a() const { return -(w * cQ); }
  __device__ __forceinline__ double Pf_f() const { return fma(2.0 * gff, vf, vt * cP); }
  __device__ __forceinline__ double Pf_t() const { return vf * cP; }
  __device__ __forceinline__ double Qf_a() const { return w * cP; }
  __device__ __forceinline__ double Qf_f() const { return fma(-2.0 * bff, vf, vt * cQ); }
  __device__ __forceinline__ double Qf_t() const { return vf * cQ; }
  // ... and of the to flow
  __device__ __forceinline__ double Pt_a() const { return w * cQt; }
  __device__ __forceinline__ double Pt_f() const { return vt * cPt; }
  __device__ __forceinline__ double Pt_t() const { return fma(2.0 * gtt, vt, vf * cPt); }
  __device__ __forceinline__ double Qt_a() const { return -(w * cPt); }
  __device__ __forceinline__ double Qt_f() const { return vt * cQt; }
  __device__ __forceinline__ double Qt_t() const { return fma(-2.0 * btt, vt, vf * cQt); }
};

__device__ __forceinline__ void branch_eval(double thf, double tht, double vf, double vt,
                                            const BranchY& y, Br& o) {
  double sn, cs;
  sincos(thf - tht, &sn, &cs);
  const double w = vf * vt;
  o.vf = vf;
  o.vt = vt;
  o.w = w;
  o.cP = fma(y.gft, cs, y.bft * sn);
  o.cQ = fma(y.gft, sn, -(y.bft * cs));
  o.cPt = fma(y.gtf, cs, -(y.btf * sn));
  o.cQt = -fma(y.gtf, sn, y.btf * cs);
  o.gff = y.gff;
  o.bff = y.bff;
  o.gtt = y.gtt;
  o.btt = y.btt;
  o.Pf = fma(y.gff, vf * vf, w * o.cP);
  o.Qf = fma(-y.bff, vf * vf, w * o.cQ);
  o.Pt = fma(y.gtt, vt * vt, w * o.cPt);
  o.Qt = fma(-y.btt, vt * vt, w * o.cQt);
}

// ---------------------------------------------------------------------------
// one branch in the power-balance-cartesian representation: V = e + j f, so
// with A = e_f e_t + f_f f_t, B = f_f e_t - e_f f_t (the real and imaginary
// parts of V_f conj(V_t)) the flows are quadratic forms
//   P_f =  g_ff |V_f|^2 + g_ft A + b_ft B,   Q_f = -b_ff |V_f|^2 + g_ft B - b_ft A
//   P_t =  g_tt |V_t|^2 + g_tf A - b_tf B,   Q_t = -b_tt |V_t|^2 - g_tf B - b_tf A
// in the local variables z = (e_f, f_f, e_t, f_t); their gradients below are
// written out per component K, and their Hessians are constant.

struct BrC {
  double ef, ff, et, ft;
  double gff, bff, gft, bft, gtf, btf, gtt, btt;
  double Pf, Qf, Pt, Qt;
  template <int K>
  __device__ __forceinline__ double gPf() const {
    if constexpr (K == 0) return fma(2.0 * gff, ef, fma(gft, et, -(bft * ft)));
    if constexpr (K == 1) return fma(2.0 * gff, ff, fma(gft, ft, bft * et));
    if constexpr (K == 2) return fma(gft, ef, bft * ff);
    return fma(gft, ff, -(bft * ef));
  }
  template <int K>
  __device__ __forceinline__ double gQf() const {
    if constexpr (K == 0) return fma(-2.0 * bff, ef, -fma(bft, et, gft * ft));
    if constexpr (K == 1) return fma(-2.0 * bff, ff, fma(gft, et, -(bft * ft)));
    if constexpr (K == 2) return fma(gft, ff, -(bft * ef));
    return -fma(bft, ff, gft * ef);
  }
  template <int K>
  __device__ __forceinline__ double gPt() const {
    if constexpr (K == 0) return fma(gtf, et, btf * ft);
    if constexpr (K == 1) return fma(gtf, ft, -(btf * et));
    if constexpr (K == 2) return fma(2.0 * gtt, et, fma(gtf, ef, -(btf * ff)));
    return fma(2.0 * gtt, ft, fma(gtf, ff, btf * ef));
  }
  template <int K>
  __device__ __forceinline__ double gQt() const {
    if constexpr (K == 0) return fma(gtf, ft, -(btf * et));
    if constexpr (K == 1) return -fma(gtf, et, btf * ft);
    if constexpr (K == 2) return fma(-2.0 * btt, et, -fma(gtf, ff, btf * ef));
    return fma(-2.0 * btt, ft, fma(gtf, ef, -(btf * ff)));
  }
};

__device__ __forceinline__ void branch_eval_cart(double ef, double ff, double et, double ft,
                                                 const BranchY& y, BrC& o) {
  const double A = fma(ef, et, ff * ft), Bq = fma(ff, et, -(ef * ft));
  const double F = fma(ef, ef, ff * ff), Tm = fma(et, et, ft * ft);
  o.ef = ef;
  o.ff = ff;
  o.et = et;
  o.ft = ft;
  o.gff = y.gff;
  o.bff = y.bff;
  o.gft = y.gft;
  o.bft = y.bft;
  o.gtf = y.gtf;
  o.btf = y.btf;
  o.gtt = y.gtt;
  o.btt = y.btt;
  o.Pf = fma(y.gff, F, fma(y.gft, A, y.bft * Bq));
  o.Qf = fma(-y.bff, F, fma(y.gft, Bq, -(y.bft * A)));
  o.Pt = fma(y.gtt, Tm, fma(y.gtf, A, -(y.btf * Bq)));
  o.Qt = fma(-y.btt, Tm, -fma(y.gtf, Bq, y.btf * A));
}

// Record layout of phase A (structure of arrays in LDS, BE entries per
// field): for each branch end inside the tile, its share of its own bus's
// balance rows, diagonal Jacobian and Hessian entries and product rows.
template <unsigned WHAT>
struct Rec {
  static constexpr bool C = (WHAT & W_C) != 0;
  static constexpr bool J = (WHAT & W_J) != 0;
  static constexpr bool H = (WHAT & W_H) != 0;
  static constexpr bool V = (WHAT & W_VJP) != 0;
  static constexpr bool HV = (WHAT & W_HVP) != 0;
  static constexpr bool JV = (WHAT & W_JVP) != 0;
  static constexpr int oC = 0;                   // P_e, Q_e
  static constexpr int oJ = oC + (C ? 2 : 0);    // dP_e/dth_e, dP_e/dv_e, dQ_e/dth_e, dQ_e/dv_e
  static constexpr int nCJ = oJ + (J ? 4 : 0);
  // The fused variant walks the branches twice and lets the bus lanes
  // consume the balance and Jacobian records between the walks, so the
  // Hessian records of the second walk reuse their space.
  static constexpr bool REUSE = H && nCJ > 0;
  static constexpr int oH = REUSE ? 0 : nCJ;     // d2/dth_e2, d2/dv_e dth_e, d2/dv_e2
  static constexpr int eH = oH + (H ? 3 : 0);
  static constexpr int oV = eH > nCJ ? eH : nCJ; // u_th_e, u_v_e
  static constexpr int oHV = oV + (V ? 2 : 0);   // (H d)_th_e, (H d)_v_e
  static constexpr int oJV = oHV + (HV ? 2 : 0); // (J d) of P_e, of Q_e
  static constexpr int N = oJV + (JV ? 2 : 0);
};

// LDS of a bus tile, in doubles: the records, then the staged copy of the
// tile's row segments (J P rows and J Q rows, or H theta rows and H v rows;
// the fused variant stages the H rows in the same space once its J rows are
// stored).
template <unsigned WHAT, int BE, int STAGE>
struct Lds {
  // a product tile may hold the records of up to kProdInst instances
  static constexpr int kInst = (WHAT & (W_VJP | W_HVP | W_JVP)) != 0 ? prod_group(WHAT) : 1;
  static constexpr int kRec = Rec<WHAT>::N * BE * kInst;
  static constexpr int kStage = (Rec<WHAT>::J || Rec<WHAT>::H) ? STAGE : 0;
  static constexpr int kGen = kGenChunk;
  static constexpr int kMax = kRec + kStage > kGen ? kRec + kStage : kGen;
};

__device__ __forceinline__ int after_outage(int l, int ol) { return (ol >= 0 && l > ol) ? 1 : 0; }

// ---------------------------------------------------------------------------
// bus tile

// Position of a base entry in an instance that may have lost entries: -1 if
// the entry itself was removed, else the base position minus the removed
// positions before it.
template <int NR>
__device__ __forceinline__ int shifted(int gp, const int32_t (&r)[NR]) {
  int below = 0;
  bool gone = false;
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    below += r[m] < gp ? 1 : 0;
    gone = gone || r[m] == gp;
  }
  return gone ? -1 : gp - below;
}

// The same for a whole segment [s0, s0 + n) of base positions: when no
// removed position falls inside it, every entry moves by one constant.
struct SegShift {
  int below;
  bool inside;
  template <int NR>
  __device__ __forceinline__ SegShift(int s0, int n, const int32_t (&r)[NR]) : below(0), inside(false) {
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      below += r[m] < s0 ? 1 : 0;
      inside = inside || (r[m] >= s0 && r[m] < s0 + n);
    }
  }
};

// Sum over a parallel-branch group, left in its first lane: lanes
// [lane, lane + g) hold the members' values, added in lane order.  Every
// lane of the wave takes part (g = 0 or 1 leaves a lane's values as they
// are); the caller keeps control flow uniform.
template <int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV], int g, int gmax) {
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = v[q];
  for (int d = 1; d < gmax; ++d) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double o = __shfl_down(v[q], d, 64);
      if (d < g) acc[q] += o;
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = acc[q];
}

template <unsigned WHAT, int WG, int BE, int NBUS, int STAGE>
__device__ void bus_tile(const Bufs& B, const InstOff& I, const NetDev& N, const Tile& T,
                         const WorkItem* __restrict__ work, double* smem) {
  using R = Rec<WHAT>;
  using L = Lds<WHAT, BE, STAGE>;
  static_assert(NBUS <= WG, "one bus per lane");
  static_assert(WG % 64 == 0, "whole waves");
  static_assert(!(R::C && R::JV), "generator sums hold either x or the direction");
  constexpr bool CART = (WHAT & W_CART) != 0;
  constexpr bool DO_GF = (WHAT & W_GRADF) != 0 && !R::V;
  const int tid = threadIdx.x;
  const int nb = N.nb;
  const int ol = I.out_l;
  const int nll = N.nl - (ol >= 0 ? 1 : 0);
  const int b0 = T.a0, nbus = T.a1 - T.a0, e0 = T.e0;
  double* rec = smem;
  // staged row segments: tile-local index of a base position (J P rows,
  // J Q rows, H theta rows, H v rows)
  double* stg = smem + L::kRec;
  const int gmax = T.gmax;
  const int sP = -T.jP0, sQ = T.nP - T.jP0;
  // the fused variant stores its J rows before it stages the H rows, in
  // the same space
  const int h0 = (R::J && !R::REUSE) ? 2 * T.nP : 0;
  const int sT = h0 - T.hT0, sV = h0 + T.nT - T.hV0;
  const double* x = B.x + I.xo;
  const double* mul = (R::H || R::HV) ? B.lam + I.co : (R::V ? B.wc + I.co : nullptr);
  const bool hneed = R::V || R::HV || (R::H && B.hess != nullptr);
  const double* dir = (R::HV || R::JV) ? B.dir + I.xo : nullptr;
  double* cflow = (R::C && B.c) ? B.c + I.co + 2 * nb : nullptr;
  double* jflow = (R::J && B.jac) ? B.jac + I.jo + (N.jflow - 8 * I.out_rm) : nullptr;
  const bool jal = (reinterpret_cast<uintptr_t>(jflow) & 15) == 0;
  double* jac = (R::J && B.jac) ? B.jac + I.jo : nullptr;
  double* hess = (R::H && B.hess) ? B.hess + I.ho : nullptr;
  // Phase C's store of one staged row segment, consecutive lanes on
  // consecutive entries: the whole segment moves by one constant unless a
  // removed position of an N-1 instance falls inside it (then each entry is
  // looked up).
  auto seg = [&](double* out, int g0, int n, int s0, const auto& r) {
    const SegShift sh(g0, n, r);
    if (!sh.inside) {
      double* o = out + (g0 - sh.below);
      for (int k = tid; k < n; k += WG) put(&o[k], stg[s0 + k]);
    } else {
      for (int k = tid; k < n; k += WG) {
        const int p = shifted(g0 + k, r);
        if (p >= 0) put(&out[p], stg[s0 + k]);
      }
    }
  };

  // ---- phase A (1): lane per branch touching the tile.  Off-diagonal
  // entries go to the staged rows; each end's own-bus share goes to its
  // LDS record.  The loop bound is uniform so that whole waves meet at the
  // group sums.
  // A variant that forms both first and second derivatives walks the
  // branches twice (flows and Jacobian, then Hessian), recomputing the flows
  // from L2-resident inputs: the register peak is then the larger pass's,
  // not their union, which keeps more waves resident.  The bus lanes consume
  // the balance and Jacobian records between the two walks, so the Hessian
  // records reuse their LDS and a tile holds more branch ends (fewer tiles).
  auto branch_pass = [&](auto parts) {
    constexpr unsigned P = decltype(parts)::value;
    constexpr bool pC = (P & W_C) != 0, pJ = (P & W_J) != 0, pH = (P & W_H) != 0;
    constexpr bool pV = (P & W_VJP) != 0, pHV = (P & W_HVP) != 0, pJV = (P & W_JVP) != 0;
    constexpr bool FIRST = P == WHAT || (P & ~W_H) != 0 || R::REUSE;
    if constexpr (CART) {
    for (int k0 = 0; k0 < T.nw; k0 += WG) {
      const int k = k0 + tid;
      WorkItem wi{};
      wi.l = -2;  // lanes past the list: no branch, no group
      if (k < T.nw) wi = work[T.w0 + k];
      const int l = wi.l, f = wi.f, t = wi.t;
      const uint32_t sf = wi.slots & 0xFFFFu, st = wi.slots >> 16;
      const bool live = l >= 0 && l != ol;
      const bool fwd = f < t;
      if (FIRST && l >= 0 && !live) {
#pragma unroll
        for (int q = 0; q < R::N; ++q) {
          if (sf != kNoSlot) rec[q * BE + sf] = 0.0;
          if (st != kNoSlot) rec[q * BE + st] = 0.0;
        }
      }
      BrC b;
      int lp = 0;
      if (live) {
        const BranchY y = load_branch(N, wi);
        branch_eval_cart(x[f], x[nb + f], x[t], x[nb + t], y, b);
        lp = l - after_outage(l, ol);
        if constexpr (pC) {
          if (sf != kNoSlot) {
            rec[(R::oC + 0) * BE + sf] = b.Pf;
            rec[(R::oC + 1) * BE + sf] = b.Qf;
          }
          if (st != kNoSlot) {
            rec[(R::oC + 0) * BE + st] = b.Pt;
            rec[(R::oC + 1) * BE + st] = b.Qt;
          }
        }
        if constexpr (pJ) {  // own-bus columns (e_e, f_e) of the end's P and Q rows
          if (sf != kNoSlot) {
            rec[(R::oJ + 0) * BE + sf] = b.gPf<0>();
            rec[(R::oJ + 1) * BE + sf] = b.gPf<1>();
            rec[(R::oJ + 2) * BE + sf] = b.gQf<0>();
            rec[(R::oJ + 3) * BE + sf] = b.gQf<1>();
          }
          if (st != kNoSlot) {
            rec[(R::oJ + 0) * BE + st] = b.gPt<2>();
            rec[(R::oJ + 1) * BE + st] = b.gPt<3>();
            rec[(R::oJ + 2) * BE + st] = b.gQt<2>();
            rec[(R::oJ + 3) * BE + st] = b.gQt<3>();
          }
        }
        if constexpr (pJV) {
          const double d0 = dir[f], d1 = dir[nb + f], d2 = dir[t], d3 = dir[nb + t];
          const double jPf = fma(b.gPf<0>(), d0, fma(b.gPf<1>(), d1, fma(b.gPf<2>(), d2, b.gPf<3>() * d3)));
          const double jQf = fma(b.gQf<0>(), d0, fma(b.gQf<1>(), d1, fma(b.gQf<2>(), d2, b.gQf<3>() * d3)));
          const double jPt = fma(b.gPt<0>(), d0, fma(b.gPt<1>(), d1, fma(b.gPt<2>(), d2, b.gPt<3>() * d3)));
          const double jQt = fma(b.gQt<0>(), d0, fma(b.gQt<1>(), d1, fma(b.gQt<2>(), d2, b.gQt<3>() * d3)));
          if (sf != kNoSlot) {
            rec[(R::oJV + 0) * BE + sf] = jPf;
            rec[(R::oJV + 1) * BE + sf] = jQf;
            double* o = B.out + I.co + 2 * nb;
            put(&o[lp], 2.0 * fma(b.Pf, jPf, b.Qf * jQf));
            put(&o[nll + lp], 2.0 * fma(b.Pt, jPt, b.Qt * jQt));
          }
          if (st != kNoSlot) {
            rec[(R::oJV + 0) * BE + st] = jPt;
            rec[(R::oJV + 1) * BE + st] = jQt;
          }
        }
        if ((pC || pJ) && sf != kNoSlot) {  // the from-bus owner writes the flow-limit rows
          if (cflow) {
            put(&cflow[lp], fma(b.Pf, b.Pf, b.Qf * b.Qf));
            put(&cflow[nll + lp], fma(b.Pt, b.Pt, b.Qt * b.Qt));
          }
          if (jflow) {
            const double hf0 = 2.0 * fma(b.Pf, b.gPf<0>(), b.Qf * b.gQf<0>());
            const double hf1 = 2.0 * fma(b.Pf, b.gPf<1>(), b.Qf * b.gQf<1>());
            const double hf2 = 2.0 * fma(b.Pf, b.gPf<2>(), b.Qf * b.gQf<2>());
            const double hf3 = 2.0 * fma(b.Pf, b.gPf<3>(), b.Qf * b.gQf<3>());
            const double ht0 = 2.0 * fma(b.Pt, b.gPt<0>(), b.Qt * b.gQt<0>());
            const double ht1 = 2.0 * fma(b.Pt, b.gPt<1>(), b.Qt * b.gQt<1>());
            const double ht2 = 2.0 * fma(b.Pt, b.gPt<2>(), b.Qt * b.gQt<2>());
            const double ht3 = 2.0 * fma(b.Pt, b.gPt<3>(), b.Qt * b.gQt<3>());
            double* rf = jflow + 4 * lp;
            double* rt = jflow + 4 * nll + 4 * lp;
            // columns ascend: e_lo, e_hi, f_lo, f_hi
            put_row4(rf, jal, fwd ? hf0 : hf2, fwd ? hf2 : hf0, fwd ? hf1 : hf3, fwd ? hf3 : hf1);
            put_row4(rt, jal, fwd ? ht0 : ht2, fwd ? ht2 : ht0, fwd ? ht1 : ht3, fwd ? ht3 : ht1);
          }
        }
      }
      if constexpr (pJ) {
        // rows of the lo and hi end bus, columns (e, f) of the other end: P then Q
        double jv[8];
        if (live) {
          const double fP = b.gPf<2>(), fPf = b.gPf<3>(), fQ = b.gQf<2>(), fQf = b.gQf<3>();
          const double tP = b.gPt<0>(), tPf = b.gPt<1>(), tQ = b.gQt<0>(), tQf = b.gQt<1>();
          jv[0] = fwd ? fP : tP;
          jv[1] = fwd ? fPf : tPf;
          jv[2] = fwd ? fQ : tQ;
          jv[3] = fwd ? fQf : tQf;
          jv[4] = fwd ? tP : fP;
          jv[5] = fwd ? tPf : fPf;
          jv[6] = fwd ? tQ : fQ;
          jv[7] = fwd ? tQf : fQf;
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) jv[q] = 0.0;
        }
        if (gmax > 1) group_sum(jv, wi.grp(), gmax);
        if (wi.grp() > 0) {
          const uint32_t jlo = wi.jlo(), jhi = wi.jhi();
          if (jlo != kNoPos) {
            const int alo = int(wi.alo());
            stg[jlo] = jv[0];
            stg[jlo + alo] = jv[1];
            stg[T.nP + jlo] = jv[2];
            stg[T.nP + jlo + alo] = jv[3];
          }
          if (jhi != kNoPos) {
            const int ahi = int(wi.ahi());
            stg[jhi] = jv[4];
            stg[jhi + ahi] = jv[5];
            stg[T.nP + jhi] = jv[6];
            stg[T.nP + jhi + ahi] = jv[7];
          }
        }
      }
      if constexpr (pH || pV || pHV) {
        // (e_hi, e_lo), (f_lo, e_hi), (f_hi, e_lo), (f_hi, f_lo)
        double hv4[4] = {0.0, 0.0, 0.0, 0.0};
        if (live && hneed) {
          const double mf = mul[2 * nb + lp];
          const double mt = mul[2 * nb + nll + lp];
          const double oPf = fma(2.0 * mf, b.Pf, mul[f]);
          const double oQf = fma(2.0 * mf, b.Qf, mul[nb + f]);
          const double oPt = fma(2.0 * mt, b.Pt, mul[t]);
          const double oQt = fma(2.0 * mt, b.Qt, mul[nb + t]);
          if constexpr (pV) {  // u = sum of the weighted flow gradients
            const double u0 = fma(oPf, b.gPf<0>(), fma(oQf, b.gQf<0>(), fma(oPt, b.gPt<0>(), oQt * b.gQt<0>())));
            const double u1 = fma(oPf, b.gPf<1>(), fma(oQf, b.gQf<1>(), fma(oPt, b.gPt<1>(), oQt * b.gQt<1>())));
            const double u2 = fma(oPf, b.gPf<2>(), fma(oQf, b.gQf<2>(), fma(oPt, b.gPt<2>(), oQt * b.gQt<2>())));
            const double u3 = fma(oPf, b.gPf<3>(), fma(oQf, b.gQf<3>(), fma(oPt, b.gPt<3>(), oQt * b.gQt<3>())));
            if (sf != kNoSlot) {
              rec[(R::oV + 0) * BE + sf] = u0;
              rec[(R::oV + 1) * BE + sf] = u1;
            }
            if (st != kNoSlot) {
              rec[(R::oV + 0) * BE + st] = u2;
              rec[(R::oV + 1) * BE + st] = u3;
            }
          }
          if constexpr (pH || pHV) {
            // H = W + 2 mu_f (gPf gPf' + gQf gQf') + 2 mu_t (gPt gPt' + gQt gQt'),
            // W = sum of the weights times the constant flow Hessians:
            // W00 = W11 = 2 cf, W22 = W33 = 2 ct, W02 = W13 = cA, W12 = cB,
            // W03 = -cB, W01 = W23 = 0
            const double cf = fma(oPf, b.gff, -(oQf * b.bff));
            const double ct = fma(oPt, b.gtt, -(oQt * b.btt));
            const double cA = fma(oPf, b.gft, fma(-oQf, b.bft, fma(oPt, b.gtf, -(oQt * b.btf))));
            const double cB = fma(oPf, b.bft, fma(oQf, b.gft, -fma(oPt, b.btf, oQt * b.gtf)));
            const double m2f = 2.0 * mf, m2t = 2.0 * mt;
            const double pf0 = b.gPf<0>(), pf1 = b.gPf<1>(), pf2 = b.gPf<2>(), pf3 = b.gPf<3>();
            const double qf0 = b.gQf<0>(), qf1 = b.gQf<1>(), qf2 = b.gQf<2>(), qf3 = b.gQf<3>();
            const double pt0 = b.gPt<0>(), pt1 = b.gPt<1>(), pt2 = b.gPt<2>(), pt3 = b.gPt<3>();
            const double qt0 = b.gQt<0>(), qt1 = b.gQt<1>(), qt2 = b.gQt<2>(), qt3 = b.gQt<3>();
            auto gn = [&](double w, double pa, double pb, double qa, double qb, double sa,
                          double sb, double ra, double rb) {
              return fma(m2f, fma(pa, pb, qa * qb), fma(m2t, fma(sa, sb, ra * rb), w));
            };
            const double h00 = gn(2.0 * cf, pf0, pf0, qf0, qf0, pt0, pt0, qt0, qt0);
            const double h10 = gn(0.0, pf1, pf0, qf1, qf0, pt1, pt0, qt1, qt0);
            const double h11 = gn(2.0 * cf, pf1, pf1, qf1, qf1, pt1, pt1, qt1, qt1);
            const double h22 = gn(2.0 * ct, pf2, pf2, qf2, qf2, pt2, pt2, qt2, qt2);
            const double h32 = gn(0.0, pf3, pf2, qf3, qf2, pt3, pt2, qt3, qt2);
            const double h33 = gn(2.0 * ct, pf3, pf3, qf3, qf3, pt3, pt3, qt3, qt3);
            const double h02 = gn(cA, pf0, pf2, qf0, qf2, pt0, pt2, qt0, qt2);
            const double h03 = gn(-cB, pf0, pf3, qf0, qf3, pt0, pt3, qt0, qt3);
            const double h12 = gn(cB, pf1, pf2, qf1, qf2, pt1, pt2, qt1, qt2);
            const double h13 = gn(cA, pf1, pf3, qf1, qf3, pt1, pt3, qt1, qt3);
            if constexpr (pH) {
              if (sf != kNoSlot) {
                rec[(R::oH + 0) * BE + sf] = h00;
                rec[(R::oH + 1) * BE + sf] = h10;
                rec[(R::oH + 2) * BE + sf] = h11;
              }
              if (st != kNoSlot) {
                rec[(R::oH + 0) * BE + st] = h22;
                rec[(R::oH + 1) * BE + st] = h32;
                rec[(R::oH + 2) * BE + st] = h33;
              }
              hv4[0] = h02;
              hv4[1] = fwd ? h12 : h03;
              hv4[2] = fwd ? h03 : h12;
              hv4[3] = h13;
            }
            if constexpr (pHV) {
              const double d0 = dir[f], d1 = dir[nb + f], d2 = dir[t], d3 = dir[nb + t];
              if (sf != kNoSlot) {
                rec[(R::oHV + 0) * BE + sf] = fma(h00, d0, fma(h10, d1, fma(h02, d2, h03 * d3)));
                rec[(R::oHV + 1) * BE + sf] = fma(h10, d0, fma(h11, d1, fma(h12, d2, h13 * d3)));
              }
              if (st != kNoSlot) {
                rec[(R::oHV + 0) * BE + st] = fma(h02, d0, fma(h12, d1, fma(h22, d2, h32 * d3)));
                rec[(R::oHV + 1) * BE + st] = fma(h03, d0, fma(h13, d1, fma(h32, d2, h33 * d3)));
              }
            }
          }
        }
        if constexpr (pH) {
          if (gmax > 1) group_sum(hv4, wi.grp(), gmax);
          if (wi.grp() > 0) {
            const int v0 = h0 + T.nT;  // the H v rows follow the theta rows
            if (wi.jlo() != kNoPos) stg[v0 + wi.hvlo()] = hv4[1];
            if (wi.jhi() != kNoPos) {
              stg[h0 + wi.hthi()] = hv4[0];
              stg[v0 + wi.hvhi()] = hv4[2];
              stg[v0 + wi.hvhi() + wi.ahi()] = hv4[3];
            }
          }
        }
      }
    }
    } else {
    for (int k0 = 0; k0 < T.nw; k0 += WG) {
      const int k = k0 + tid;
      WorkItem wi{};
      wi.l = -2;  // lanes past the list: no branch, no group
      if (k < T.nw) wi = work[T.w0 + k];
      const int l = wi.l, f = wi.f, t = wi.t;
      const uint32_t sf = wi.slots & 0xFFFFu, st = wi.slots >> 16;
      const bool live = l >= 0 && l != ol;
      const bool fwd = f < t;  // the from bus is the lower-numbered end
      if (FIRST && l >= 0 && !live) {  // removed branch: its ends keep their places and add zero
  #pragma unroll
        for (int q = 0; q < R::N; ++q) {
          if (sf != kNoSlot) rec[q * BE + sf] = 0.0;
          if (st != kNoSlot) rec[q * BE + st] = 0.0;
        }
      }
      Br b;
      int lp = 0;
      if (live) {
        const BranchY y = load_branch(N, wi);
        branch_eval(x[f], x[t], x[nb + f], x[nb + t], y, b);
        lp = l - after_outage(l, ol);
        if constexpr (pC) {
          if (sf != kNoSlot) {
            rec[(R::oC + 0) * BE + sf] = b.Pf;
            rec[(R::oC + 1) * BE + sf] = b.Qf;
          }
          if (st != kNoSlot) {
            rec[(R::oC + 0) * BE + st] = b.Pt;
            rec[(R::oC + 1) * BE + st] = b.Qt;
          }
        }
        if constexpr (pJ) {
          if (sf != kNoSlot) {
            rec[(R::oJ + 0) * BE + sf] = b.Pf_a();
            rec[(R::oJ + 1) * BE + sf] = b.Pf_f();
            rec[(R::oJ + 2) * BE + sf] = b.Qf_a();
            rec[(R::oJ + 3) * BE + sf] = b.Qf_f();
          }
          if (st != kNoSlot) {  // to end: d/dtheta_t = -d/dtheta_f
            rec[(R::oJ + 0) * BE + st] = -b.Pt_a();
            rec[(R::oJ + 1) * BE + st] = b.Pt_t();
            rec[(R::oJ + 2) * BE + st] = -b.Qt_a();
            rec[(R::oJ + 3) * BE + st] = b.Qt_t();
          }
        }
        if constexpr (pJV) {  // J d: first derivatives along the direction
          const double da = dir[f] - dir[t], dvf = dir[nb + f], dvt = dir[nb + t];
          const double jPf = fma(b.Pf_a(), da, fma(b.Pf_f(), dvf, b.Pf_t() * dvt));
          const double jQf = fma(b.Qf_a(), da, fma(b.Qf_f(), dvf, b.Qf_t() * dvt));
          const double jPt = fma(b.Pt_a(), da, fma(b.Pt_f(), dvf, b.Pt_t() * dvt));
          const double jQt = fma(b.Qt_a(), da, fma(b.Qt_f(), dvf, b.Qt_t() * dvt));
          if (sf != kNoSlot) {
            rec[(R::oJV + 0) * BE + sf] = jPf;
            rec[(R::oJV + 1) * BE + sf] = jQf;
            double* o = B.out + I.co + 2 * nb;
            put(&o[lp], 2.0 * fma(b.Pf, jPf, b.Qf * jQf));
            put(&o[nll + lp], 2.0 * fma(b.Pt, jPt, b.Qt * jQt));
          }
          if (st != kNoSlot) {
            rec[(R::oJV + 0) * BE + st] = jPt;
            rec[(R::oJV + 1) * BE + st] = jQt;
          }
        }
        if ((pC || pJ) && sf != kNoSlot) {  // the from-bus owner writes the flow-limit rows
          if (cflow) {
            put(&cflow[lp], fma(b.Pf, b.Pf, b.Qf * b.Qf));
            put(&cflow[nll + lp], fma(b.Pt, b.Pt, b.Qt * b.Qt));
          }
          if (jflow) {
            const double hf_a = 2.0 * fma(b.Pf, b.Pf_a(), b.Qf * b.Qf_a());
            const double hf_f = 2.0 * fma(b.Pf, b.Pf_f(), b.Qf * b.Qf_f());
            const double hf_t = 2.0 * fma(b.Pf, b.Pf_t(), b.Qf * b.Qf_t());
            const double ht_a = 2.0 * fma(b.Pt, b.Pt_a(), b.Qt * b.Qt_a());
            const double ht_f = 2.0 * fma(b.Pt, b.Pt_f(), b.Qt * b.Qt_f());
            const double ht_t = 2.0 * fma(b.Pt, b.Pt_t(), b.Qt * b.Qt_t());
            double* rf = jflow + 4 * lp;
            double* rt = jflow + 4 * nll + 4 * lp;
            // columns ascend: theta_lo, theta_hi, v_lo, v_hi
            put_row4(rf, jal, fwd ? hf_a : -hf_a, fwd ? -hf_a : hf_a, fwd ? hf_f : hf_t,
                     fwd ? hf_t : hf_f);
            put_row4(rt, jal, fwd ? ht_a : -ht_a, fwd ? -ht_a : ht_a, fwd ? ht_f : ht_t,
                     fwd ? ht_t : ht_f);
          }
        }
      }
      if constexpr (pJ) {
        // rows of the lower (lo) and higher (hi) end bus, columns of the other:
        // d/dtheta and d/dv of P, then of Q
        double jv[8];
        if (live) {
          const double fP = -b.Pf_a(), fPv = b.Pf_t(), fQ = -b.Qf_a(), fQv = b.Qf_t();
          const double tP = b.Pt_a(), tPv = b.Pt_f(), tQ = b.Qt_a(), tQv = b.Qt_f();
          jv[0] = fwd ? fP : tP;
          jv[1] = fwd ? fPv : tPv;
          jv[2] = fwd ? fQ : tQ;
          jv[3] = fwd ? fQv : tQv;
          jv[4] = fwd ? tP : fP;
          jv[5] = fwd ? tPv : fPv;
          jv[6] = fwd ? tQ : fQ;
          jv[7] = fwd ? tQv : fQv;
        } else {
  #pragma unroll
          for (int q = 0; q < 8; ++q) jv[q] = 0.0;
        }
        if (gmax > 1) group_sum(jv, wi.grp(), gmax);
        if (wi.grp() > 0) {  // (entries of a removed branch without a twin are never stored)
          const uint32_t jlo = wi.jlo(), jhi = wi.jhi();
          if (jlo != kNoPos) {
            const int alo = int(wi.alo());
            stg[jlo] = jv[0];
            stg[jlo + alo] = jv[1];
            stg[T.nP + jlo] = jv[2];
            stg[T.nP + jlo + alo] = jv[3];
          }
          if (jhi != kNoPos) {
            const int ahi = int(wi.ahi());
            stg[jhi] = jv[4];
            stg[jhi + ahi] = jv[5];
            stg[T.nP + jhi] = jv[6];
            stg[T.nP + jhi + ahi] = jv[7];
          }
        }
      }
      if constexpr (pH || pV || pHV) {
        // (theta_hi, theta_lo), (v_lo, theta_hi), (v_hi, theta_lo), (v_hi, v_lo)
        double hv4[4] = {0.0, 0.0, 0.0, 0.0};
        if (live && hneed) {  // the full variant reads multipliers only when H is wanted
          const double mf = mul[2 * nb + lp];
          const double mt = mul[2 * nb + nll + lp];
          // weights of dP, dQ in  lP P + lQ Q + mu (P^2 + Q^2)
          const double oPf = fma(2.0 * mf, b.Pf, mul[f]);
          const double oQf = fma(2.0 * mf, b.Qf, mul[nb + f]);
          const double oPt = fma(2.0 * mt, b.Pt, mul[t]);
          const double oQt = fma(2.0 * mt, b.Qt, mul[nb + t]);
          // s, r: the weighted transfer terms; every second derivative and the
          // VJP are short expressions in them (the Gauss-Newton cross terms
          // Pt_f Pt_a + Qt_f Qt_a and Pf_t Pf_a + Qf_t Qf_a vanish identically)
          const double s = fma(oPf, b.cP, fma(oQf, b.cQ, fma(oPt, b.cPt, oQt * b.cQt)));
          const double r = fma(oQf, b.cP, fma(-oPf, b.cQ, fma(oPt, b.cQt, -(oQt * b.cPt))));
          if constexpr (pV) {
            const double u_a = b.w * r;  // d/dtheta_f; d/dtheta_t = -u_a
            const double u_f = fma(2.0 * b.vf, fma(oPf, b.gff, -(oQf * b.bff)), b.vt * s);
            const double u_t = fma(2.0 * b.vt, fma(oPt, b.gtt, -(oQt * b.btt)), b.vf * s);
            if (sf != kNoSlot) {
              rec[(R::oV + 0) * BE + sf] = u_a;
              rec[(R::oV + 1) * BE + sf] = u_f;
            }
            if (st != kNoSlot) {
              rec[(R::oV + 0) * BE + st] = -u_a;
              rec[(R::oV + 1) * BE + st] = u_t;
            }
          }
          if constexpr (pH || pHV) {
            const double m2f = 2.0 * mf, m2t = 2.0 * mt;
            const double ccf = fma(b.cP, b.cP, b.cQ * b.cQ), cct = fma(b.cPt, b.cPt, b.cQt * b.cQt);
            // d2L/dtheta_f^2
            const double a = fma(-b.w, s, (b.w * b.w) * fma(m2f, ccf, m2t * cct));
            // d2L/dv_f dtheta_f and d2L/dv_t dtheta_t
            const double beta_f =
                fma(b.vt, r, -(2.0 * m2f) * (b.vf * b.w) * fma(b.gff, b.cQ, b.bff * b.cP));
            const double beta_t =
                -fma(b.vf, r, (2.0 * m2t) * (b.vt * b.w) * fma(b.gtt, b.cQt, b.btt * b.cPt));
            const double pff = b.Pf_f(), qff = b.Qf_f(), ptt = b.Pt_t(), qtt = b.Qt_t();
            const double vv_ff = fma(2.0, fma(oPf, b.gff, -(oQf * b.bff)),
                                     fma(m2f, fma(pff, pff, qff * qff), m2t * (b.vt * b.vt) * cct));
            const double vv_tt = fma(2.0, fma(oPt, b.gtt, -(oQt * b.btt)),
                                     fma(m2f * (b.vf * b.vf), ccf, m2t * fma(ptt, ptt, qtt * qtt)));
            const double vv_ft =
                s + fma(m2f * b.vf, fma(2.0 * b.vf, fma(b.gff, b.cP, -(b.bff * b.cQ)), b.vt * ccf),
                        m2t * b.vt * fma(2.0 * b.vt, fma(b.gtt, b.cPt, -(b.btt * b.cQt)), b.vf * cct));
            if constexpr (pH) {
              if (sf != kNoSlot) {
                rec[(R::oH + 0) * BE + sf] = a;
                rec[(R::oH + 1) * BE + sf] = beta_f;
                rec[(R::oH + 2) * BE + sf] = vv_ff;
              }
              if (st != kNoSlot) {
                rec[(R::oH + 0) * BE + st] = a;
                rec[(R::oH + 1) * BE + st] = beta_t;
                rec[(R::oH + 2) * BE + st] = vv_tt;
              }
              // d/dtheta_t = -d/dtheta_f
              hv4[0] = -a;
              hv4[1] = fwd ? -beta_f : -beta_t;
              hv4[2] = fwd ? -beta_t : -beta_f;
              hv4[3] = vv_ft;
            }
            if constexpr (pHV) {
              // the branch's 4x4 block on (theta_f, theta_t, v_f, v_t) times d:
              // theta rows +-(a da + beta_f d_vf - beta_t d_vt), v rows below
              const double da = dir[f] - dir[t], dvf = dir[nb + f], dvt = dir[nb + t];
              const double h_a = fma(a, da, fma(beta_f, dvf, -(beta_t * dvt)));
              if (sf != kNoSlot) {
                rec[(R::oHV + 0) * BE + sf] = h_a;
                rec[(R::oHV + 1) * BE + sf] = fma(beta_f, da, fma(vv_ff, dvf, vv_ft * dvt));
              }
              if (st != kNoSlot) {
                rec[(R::oHV + 0) * BE + st] = -h_a;
                rec[(R::oHV + 1) * BE + st] = fma(-beta_t, da, fma(vv_ft, dvf, vv_tt * dvt));
              }
            }
          }
        }
        if constexpr (pH) {
          if (gmax > 1) group_sum(hv4, wi.grp(), gmax);
          if (wi.grp() > 0) {
            const int v0 = h0 + T.nT;  // the H v rows follow the theta rows
            if (wi.jlo() != kNoPos) stg[v0 + wi.hvlo()] = hv4[1];
            if (wi.jhi() != kNoPos) {
              stg[h0 + wi.hthi()] = hv4[0];
              stg[v0 + wi.hvhi()] = hv4[2];
              stg[v0 + wi.hvhi() + wi.ahi()] = hv4[3];
            }
          }
        }
      }
    }
    }
  };
  if constexpr (R::REUSE) {
    branch_pass(std::integral_constant<unsigned, WHAT & ~W_H>{});  // the Hessian walk follows phase B's first part
  } else {
    branch_pass(std::integral_constant<unsigned, WHAT>{});
  }

  // ---- phase A (2): lane per bus, the bus's own terms (kept in registers
  // across the barrier by the same lane)
  const bool has_bus = tid < nbus;
  const int i = b0 + tid;
  int ea = 0, eb = 0;
  int4 rw = make_int4(0, 0, 0, 0);
  int2 ac = make_int2(0, 0);
  int ngb = 0;
  double jbP = 0.0, jbQ = 0.0, hb = 0.0, cbP = 0.0, cbQ = 0.0, vb = 0.0, hvb = 0.0;
  double jvP = 0.0, jvQ = 0.0;
  // cartesian only: e_i, the shunt columns of e_i, and the magnitude row
  // e_i^2 + f_i^2 with its product rows
  double ei = 0.0, fi = 0.0, m2 = 0.0, jbPe = 0.0, jbQe = 0.0, hvbe = 0.0, vbe = 0.0, jvm = 0.0;
  double* c = (R::C && B.c) ? B.c + I.co : nullptr;
  if (has_bus) {
    ea = N.be_ptr[i] - e0;
    eb = N.be_ptr[i + 1] - e0;
    const double4 bd = N.bus[i];  // pd, qd, gs, bs
    const double vi = x[nb + i];  // v_i, or f_i in the cartesian representation
    // the squared magnitude |V_i|^2 and the weight of its row (cartesian)
    double lvm = 0.0;
    (void)lvm;
    if constexpr (CART) {
      ei = x[i];
      fi = vi;
      m2 = fma(ei, ei, vi * vi);
      if (R::H || R::V || R::HV) lvm = hneed ? mul[2 * nb + 2 * nll + i] : 0.0;
    }
    if constexpr (R::J || R::H) {
      rw = N.rows[i];
      ac = N.acnt[i];
    }
    if constexpr (R::J) {
      jbP = 2.0 * bd.z * vi;
      jbQ = -2.0 * bd.w * vi;
      if constexpr (CART) {
        jbPe = 2.0 * bd.z * ei;
        jbQe = -2.0 * bd.w * ei;
      }
      ngb = N.gen_ptr[i + 1] - N.gen_ptr[i];
    }
    if constexpr (R::H) {
      if (hess) {
        hb = CART ? 2.0 * (fma(mul[i], bd.z, -(mul[nb + i] * bd.w)) + lvm)
                  : 2.0 * fma(mul[i], bd.z, -(mul[nb + i] * bd.w));
      }
    }
    if constexpr (R::C) {
      if (c) {
        double pg = 0, qg = 0;
        for (int g = N.gen_ptr[i], g1 = N.gen_ptr[i + 1]; g < g1; ++g) {
          const int k = N.gen_ident ? g : N.gen_list[g];
          pg += x[2 * nb + k];
          qg += x[2 * nb + N.ng + k];
        }
        if constexpr (CART) {
          cbP = (bd.z * m2 - pg) + bd.x;
          cbQ = (-bd.w * m2 - qg) + bd.y;
        } else {
          cbP = (bd.z * vi * vi - pg) + bd.x;
          cbQ = (-bd.w * vi * vi - qg) + bd.y;
        }
        for (int k = 0; k < N.sl.ns; ++k) {  // slack blocks: +-1 in their row
          const double t = N.sl.coef[k] * x[2 * nb + 2 * N.ng + k * nb + i];
          if (N.sl.row[k] == 0) cbP += t; else cbQ += t;
        }
      }
    }
    if constexpr (R::V) {
      if constexpr (CART) {
        const double kap = 2.0 * (fma(mul[i], bd.z, -(mul[nb + i] * bd.w)) + lvm);
        vb = kap * vi;
        vbe = kap * ei;
      } else {
        vb = 2.0 * vi * fma(mul[i], bd.z, -(mul[nb + i] * bd.w));
      }
    }
    if constexpr (R::HV) {
      if constexpr (CART) {
        const double kap = 2.0 * (fma(mul[i], bd.z, -(mul[nb + i] * bd.w)) + lvm);
        hvb = kap * dir[nb + i];
        hvbe = kap * dir[i];
      } else {
        hvb = 2.0 * fma(mul[i], bd.z, -(mul[nb + i] * bd.w)) * dir[nb + i];
      }
    }
    if constexpr (R::JV) {
      double dpg = 0, dqg = 0;
      for (int g = N.gen_ptr[i], g1 = N.gen_ptr[i + 1]; g < g1; ++g) {
        const int k = N.gen_ident ? g : N.gen_list[g];
        dpg += dir[2 * nb + k];
        dqg += dir[2 * nb + N.ng + k];
      }
      if constexpr (CART) {  // d|V_i|^2 along the direction
        jvm = 2.0 * fma(ei, dir[i], vi * dir[nb + i]);
        jvP = bd.z * jvm - dpg;
        jvQ = -bd.w * jvm - dqg;
      } else {
        jvP = 2.0 * bd.z * vi * dir[nb + i] - dpg;
        jvQ = -2.0 * bd.w * vi * dir[nb + i] - dqg;
      }
      for (int k = 0; k < N.sl.ns; ++k) {
        const double t = N.sl.coef[k] * dir[2 * nb + 2 * N.ng + k * nb + i];
        if (N.sl.row[k] == 0) jvP += t; else jvQ += t;
      }
    }
  }
  __syncthreads();

  // ---- phase B: lane per bus, its ends' records summed in adjacency order
  // into the diagonal entries (staged) and the bus's rows
  if (has_bus) {
  if constexpr (R::C) {
    if (c) {
      double sp = 0.0, sq = 0.0;
      for (int e = ea; e < eb; ++e) {
        sp += rec[(R::oC + 0) * BE + e];
        sq += rec[(R::oC + 1) * BE + e];
      }
      put(&c[i], sp + cbP);
      put(&c[nb + i], sq + cbQ);
      if constexpr (CART) put(&c[2 * nb + 2 * nll + i], m2);
    }
  }
  if constexpr (DO_GF) {
    if (B.gradf) {
      double* gradf = B.gradf + I.xo;
      put(&gradf[i], 0.0);
      put(&gradf[nb + i], 0.0);
    }
  }
  if constexpr (R::J) {
    if (jac) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int e = ea; e < eb; ++e) {
        s0 += rec[(R::oJ + 0) * BE + e];
        s1 += rec[(R::oJ + 1) * BE + e];
        s2 += rec[(R::oJ + 2) * BE + e];
        s3 += rec[(R::oJ + 3) * BE + e];
      }
      // (theta_i), (v_i) of the P row, the same of the Q row, then the
      // generator columns (constant -1)
      const int pt = rw.x + ac.y, pv = rw.x + ac.x + ac.y;
      stg[sP + pt] = CART ? s0 + jbPe : s0;
      stg[sP + pv] = s1 + jbP;
      stg[sQ + pt] = CART ? s2 + jbQe : s2;
      stg[sQ + pv] = s3 + jbQ;
      if constexpr (CART) {  // the magnitude row (e_i, f_i), after the flow rows
        double* jm = jflow + 8 * nll + 2 * i;
        put(&jm[0], 2.0 * ei);
        put(&jm[1], 2.0 * fi);
      }
      for (int g = 0; g < ngb; ++g) {
        stg[sP + rw.x + 2 * ac.x + g] = -1.0;
        stg[sQ + rw.x + 2 * ac.x + g] = -1.0;
      }
      // slack columns after the generators, blocks in order within each row
      for (int k = 0, qp = 0, qq = 0; k < N.sl.ns; ++k) {
        if (N.sl.row[k] == 0)
          stg[sP + rw.x + 2 * ac.x + ngb + qp++] = N.sl.coef[k];
        else
          stg[sQ + rw.x + 2 * ac.x + ngb + qq++] = N.sl.coef[k];
      }
    }
  }
  }
  if constexpr (R::REUSE) {
    __syncthreads();  // balance and Jacobian records consumed, J rows complete
    if (jac) {
      seg(jac, T.jP0, T.nP, 0, I.rj);     // P rows
      seg(jac, T.jQ0, T.nP, T.nP, I.rj);  // Q rows
    }
    __syncthreads();  // the records and the staged rows are free again
    branch_pass(std::integral_constant<unsigned, W_H>{});
    __syncthreads();
  }
  if (has_bus) {
  if constexpr (R::H) {
    if (hess) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int e = ea; e < eb; ++e) {
        s0 += rec[(R::oH + 0) * BE + e];
        s1 += rec[(R::oH + 1) * BE + e];
        s2 += rec[(R::oH + 2) * BE + e];
      }
      stg[sT + rw.z + ac.y] = CART ? s0 + hb : s0;
      stg[sV + rw.w + ac.y] = s1;
      stg[sV + rw.w + ac.x + ac.y] = s2 + hb;
    }
  }
  if constexpr (R::V) {
    double ut = 0.0, uv = 0.0;
    for (int e = ea; e < eb; ++e) {
      ut += rec[(R::oV + 0) * BE + e];
      uv += rec[(R::oV + 1) * BE + e];
    }
    double* u = B.u + I.xo;
    put(&u[i], CART ? ut + vbe : ut);
    put(&u[nb + i], uv + vb);
  }
  if constexpr (R::HV) {
    double ht = 0.0, hv = 0.0;
    for (int e = ea; e < eb; ++e) {
      ht += rec[(R::oHV + 0) * BE + e];
      hv += rec[(R::oHV + 1) * BE + e];
    }
    double* o = B.out + I.xo;
    put(&o[i], CART ? ht + hvbe : ht);
    put(&o[nb + i], hv + hvb);
  }
  if constexpr (R::JV) {
    double jp = 0.0, jq = 0.0;
    for (int e = ea; e < eb; ++e) {
      jp += rec[(R::oJV + 0) * BE + e];
      jq += rec[(R::oJV + 1) * BE + e];
    }
    double* o = B.out + I.co;
    put(&o[i], jp + jvP);
    put(&o[nb + i], jq + jvQ);
    if constexpr (CART) put(&o[2 * nb + 2 * nll + i], jvm);
  }
  }

  // ---- phase C: the staged row segments, consecutive lanes on consecutive
  // entries; an N-1 instance skips the removed positions and shifts the rest
  if constexpr (R::J || R::H) {
    __syncthreads();
    if constexpr (R::J && !R::REUSE) {
      if (jac) {
        seg(jac, T.jP0, T.nP, 0, I.rj);      // P rows
        seg(jac, T.jQ0, T.nP, T.nP, I.rj);   // Q rows
      }
    }
    if constexpr (R::H) {
      if (hess) {
        seg(hess, T.hT0, T.nT, h0, I.rh);          // theta rows
        seg(hess, T.hV0, T.nV, h0 + T.nT, I.rh);   // v rows
      }
    }
  }
}

// ---------------------------------------------------------------------------
// product tile: a bus tile of the VJP, HVP or JVP for ni <= NI instances
// that share one base network (an N-1 batch groups its instances).  The work
// items, the branch admittances and the bus data are loaded once for all of
// them; each instance gathers its own x, multipliers and direction and keeps
// its own records.  Per instance the arithmetic and its order are those of a
// tile of one instance, so results do not depend on the grouping.
template <unsigned WHAT, int WG, int BE, int NI>
__device__ void prod_tile(const Bufs& B, const InstOff* __restrict__ table, const InstOff& I0,
                          const NetDev& N, const Tile& T, int ni,
                          const WorkItem* __restrict__ work, double* smem) {
  using R = Rec<WHAT>;
  static_assert(NI >= 1 && NI <= kProdInst, "instances per product tile");
  static_assert(!R::C && !R::J && !R::H, "products only");
  constexpr bool CART = (WHAT & W_CART) != 0;
  constexpr bool MUL = R::V || R::HV;   // weights: w_c (VJP) or lambda (HVP)
  constexpr bool DIR = R::HV || R::JV;
  const int tid = threadIdx.x;
  const int nb = N.nb;
  const int b0 = T.a0, nbus = T.a1 - T.a0, e0 = T.e0;
  int ol[NI], nll[NI];
  const double* xs[NI];
  const double* mul[NI];
  const double* dir[NI];
  int64_t xo[NI], co[NI];
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    if (ii >= ni) break;
    const InstOff& I = ii ? table[T.more[ii - 1]] : I0;
    ol[ii] = I.out_l;
    nll[ii] = N.nl - (I.out_l >= 0 ? 1 : 0);
    xo[ii] = I.xo;
    co[ii] = I.co;
    xs[ii] = B.x + I.xo;
    mul[ii] = MUL ? (R::HV ? B.lam + I.co : B.wc + I.co) : nullptr;
    dir[ii] = DIR ? B.dir + I.xo : nullptr;
  }

  // ---- phase A: lane per branch touching the tile
  for (int k0 = 0; k0 < T.nw; k0 += WG) {
    const int k = k0 + tid;
    WorkItem wi{};
    wi.l = -2;  // lanes past the list: no branch
    if (k < T.nw) wi = work[T.w0 + k];
    const int l = wi.l, f = wi.f, t = wi.t;
    const uint32_t sf = wi.slots & 0xFFFFu, st = wi.slots >> 16;
    BranchY y{};
    if (l >= 0) y = load_branch(N, wi);
    // each instance's inputs are gathered just before its arithmetic:
    // gathering every instance's first holds all the sets in registers,
    // which costs a wave per SIMD and measured slower in every product
    bool live[NI];
    int lp[NI];
    double gx[NI][4], gm[NI][6], gd[NI][4];
    auto gather = [&](int ii) {
      live[ii] = l >= 0 && l != ol[ii];
      lp[ii] = live[ii] ? l - after_outage(l, ol[ii]) : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) gx[ii][q] = gd[ii][q] = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) gm[ii][q] = 0.0;
      if (live[ii]) {
        const double* x = xs[ii];
        gx[ii][0] = x[f];
        gx[ii][1] = x[t];
        gx[ii][2] = x[nb + f];
        gx[ii][3] = x[nb + t];
        if constexpr (MUL) {
          const double* m = mul[ii];
          gm[ii][0] = m[2 * nb + lp[ii]];
          gm[ii][1] = m[2 * nb + nll[ii] + lp[ii]];
          gm[ii][2] = m[f];
          gm[ii][3] = m[nb + f];
          gm[ii][4] = m[t];
          gm[ii][5] = m[nb + t];
        }
        if constexpr (DIR) {
          const double* d = dir[ii];
          gd[ii][0] = d[f];
          gd[ii][1] = d[t];
          gd[ii][2] = d[nb + f];
          gd[ii][3] = d[nb + t];
        }
      }
    };
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      if (ii >= ni) break;
      gather(ii);
      double* rec = smem + ii * (R::N * BE);
      if (l >= 0 && !live[ii]) {  // removed branch: its ends keep their places and add zero
#pragma unroll
        for (int q = 0; q < R::N; ++q) {
          if (sf != kNoSlot) rec[q * BE + sf] = 0.0;
          if (st != kNoSlot) rec[q * BE + st] = 0.0;
        }
      }
      if (!live[ii]) continue;
      const int lpi = lp[ii], nl_i = nll[ii];
      if constexpr (CART) {
        BrC b;
        branch_eval_cart(gx[ii][0], gx[ii][2], gx[ii][1], gx[ii][3], y, b);
        if constexpr (R::JV) {
          const double d0 = gd[ii][0], d1 = gd[ii][2], d2 = gd[ii][1], d3 = gd[ii][3];
          const double jPf = fma(b.gPf<0>(), d0, fma(b.gPf<1>(), d1, fma(b.gPf<2>(), d2, b.gPf<3>() * d3)));
          const double jQf = fma(b.gQf<0>(), d0, fma(b.gQf<1>(), d1, fma(b.gQf<2>(), d2, b.gQf<3>() * d3)));
          const double jPt = fma(b.gPt<0>(), d0, fma(b.gPt<1>(), d1, fma(b.gPt<2>(), d2, b.gPt<3>() * d3)));
          const double jQt = fma(b.gQt<0>(), d0, fma(b.gQt<1>(), d1, fma(b.gQt<2>(), d2, b.gQt<3>() * d3)));
          if (sf != kNoSlot) {
            rec[(R::oJV + 0) * BE + sf] = jPf;
            rec[(R::oJV + 1) * BE + sf] = jQf;
            double* o = B.out + co[ii] + 2 * nb;
            put(&o[lpi], 2.0 * fma(b.Pf, jPf, b.Qf * jQf));
            put(&o[nl_i + lpi], 2.0 * fma(b.Pt, jPt, b.Qt * jQt));
          }
          if (st != kNoSlot) {
            rec[(R::oJV + 0) * BE + st] = jPt;
            rec[(R::oJV + 1) * BE + st] = jQt;
          }
        }
        if constexpr (MUL) {
          const double mf = gm[ii][0], mt = gm[ii][1];
          const double oPf = fma(2.0 * mf, b.Pf, gm[ii][2]);
          const double oQf = fma(2.0 * mf, b.Qf, gm[ii][3]);
          const double oPt = fma(2.0 * mt, b.Pt, gm[ii][4]);
          const double oQt = fma(2.0 * mt, b.Qt, gm[ii][5]);
          if constexpr (R::V) {
            const double u0 = fma(oPf, b.gPf<0>(), fma(oQf, b.gQf<0>(), fma(oPt, b.gPt<0>(), oQt * b.gQt<0>())));
            const double u1 = fma(oPf, b.gPf<1>(), fma(oQf, b.gQf<1>(), fma(oPt, b.gPt<1>(), oQt * b.gQt<1>())));
            const double u2 = fma(oPf, b.gPf<2>(), fma(oQf, b.gQf<2>(), fma(oPt, b.gPt<2>(), oQt * b.gQt<2>())));
            const double u3 = fma(oPf, b.gPf<3>(), fma(oQf, b.gQf<3>(), fma(oPt, b.gPt<3>(), oQt * b.gQt<3>())));
            if (sf != kNoSlot) {
              rec[(R::oV + 0) * BE + sf] = u0;
              rec[(R::oV + 1) * BE + sf] = u1;
            }
            if (st != kNoSlot) {
              rec[(R::oV + 0) * BE + st] = u2;
              rec[(R::oV + 1) * BE + st] = u3;
            }
          }
          if constexpr (R::HV) {
            // the branch's local Hessian (see the bus tile) times the direction
            const double cf = fma(oPf, b.gff, -(oQf * b.bff));
            const double ct = fma(oPt, b.gtt, -(oQt * b.btt));
            const double cA = fma(oPf, b.gft, fma(-oQf, b.bft, fma(oPt, b.gtf, -(oQt * b.btf))));
            const double cB = fma(oPf, b.bft, fma(oQf, b.gft, -fma(oPt, b.btf, oQt * b.gtf)));
            const double m2f = 2.0 * mf, m2t = 2.0 * mt;
            const double pf0 = b.gPf<0>(), pf1 = b.gPf<1>(), pf2 = b.gPf<2>(), pf3 = b.gPf<3>();
            const double qf0 = b.gQf<0>(), qf1 = b.gQf<1>(), qf2 = b.gQf<2>(), qf3 = b.gQf<3>();
            const double pt0 = b.gPt<0>(), pt1 = b.gPt<1>(), pt2 = b.gPt<2>(), pt3 = b.gPt<3>();
            const double qt0 = b.gQt<0>(), qt1 = b.gQt<1>(), qt2 = b.gQt<2>(), qt3 = b.gQt<3>();
            auto gn = [&](double w, double pa, double pb, double qa, double qb, double sa,
                          double sb, double ra, double rb) {
              return fma(m2f, fma(pa, pb, qa * qb), fma(m2t, fma(sa, sb, ra * rb), w));
            };
            const double h00 = gn(2.0 * cf, pf0, pf0, qf0, qf0, pt0, pt0, qt0, qt0);
            const double h10 = gn(0.0, pf1, pf0, qf1, qf0, pt1, pt0, qt1, qt0);
            const double h11 = gn(2.0 * cf, pf1, pf1, qf1, qf1, pt1, pt1, qt1, qt1);
            const double h22 = gn(2.0 * ct, pf2, pf2, qf2, qf2, pt2, pt2, qt2, qt2);
            const double h32 = gn(0.0, pf3, pf2, qf3, qf2, pt3, pt2, qt3, qt2);
            const double h33 = gn(2.0 * ct, pf3, pf3, qf3, qf3, pt3, pt3, qt3, qt3);
            const double h02 = gn(cA, pf0, pf2, qf0, qf2, pt0, pt2, qt0, qt2);
            const double h03 = gn(-cB, pf0, pf3, qf0, qf3, pt0, pt3, qt0, qt3);
            const double h12 = gn(cB, pf1, pf2, qf1, qf2, pt1, pt2, qt1, qt2);
            const double h13 = gn(cA, pf1, pf3, qf1, qf3, pt1, pt3, qt1, qt3);
            const double d0 = gd[ii][0], d1 = gd[ii][2], d2 = gd[ii][1], d3 = gd[ii][3];
            if (sf != kNoSlot) {
              rec[(R::oHV + 0) * BE + sf] = fma(h00, d0, fma(h10, d1, fma(h02, d2, h03 * d3)));
              rec[(R::oHV + 1) * BE + sf] = fma(h10, d0, fma(h11, d1, fma(h12, d2, h13 * d3)));
            }
            if (st != kNoSlot) {
              rec[(R::oHV + 0) * BE + st] = fma(h02, d0, fma(h12, d1, fma(h22, d2, h32 * d3)));
              rec[(R::oHV + 1) * BE + st] = fma(h03, d0, fma(h13, d1, fma(h32, d2, h33 * d3)));
            }
          }
        }
      } else {
        Br b;
        branch_eval(gx[ii][0], gx[ii][1], gx[ii][2], gx[ii][3], y, b);
        if constexpr (R::JV) {  // J d: first derivatives along the direction
          const double da = gd[ii][0] - gd[ii][1], dvf = gd[ii][2], dvt = gd[ii][3];
          const double jPf = fma(b.Pf_a(), da, fma(b.Pf_f(), dvf, b.Pf_t() * dvt));
          const double jQf = fma(b.Qf_a(), da, fma(b.Qf_f(), dvf, b.Qf_t() * dvt));
          const double jPt = fma(b.Pt_a(), da, fma(b.Pt_f(), dvf, b.Pt_t() * dvt));
          const double jQt = fma(b.Qt_a(), da, fma(b.Qt_f(), dvf, b.Qt_t() * dvt));
          if (sf != kNoSlot) {
            rec[(R::oJV + 0) * BE + sf] = jPf;
            rec[(R::oJV + 1) * BE + sf] = jQf;
            double* o = B.out + co[ii] + 2 * nb;
            put(&o[lpi], 2.0 * fma(b.Pf, jPf, b.Qf * jQf));
            put(&o[nl_i + lpi], 2.0 * fma(b.Pt, jPt, b.Qt * jQt));
          }
          if (st != kNoSlot) {
            rec[(R::oJV + 0) * BE + st] = jPt;
            rec[(R::oJV + 1) * BE + st] = jQt;
          }
        }
        if constexpr (MUL) {
          const double mf = gm[ii][0], mt = gm[ii][1];
          // weights of dP, dQ in  lP P + lQ Q + mu (P^2 + Q^2)
          const double oPf = fma(2.0 * mf, b.Pf, gm[ii][2]);
          const double oQf = fma(2.0 * mf, b.Qf, gm[ii][3]);
          const double oPt = fma(2.0 * mt, b.Pt, gm[ii][4]);
          const double oQt = fma(2.0 * mt, b.Qt, gm[ii][5]);
          // s, r: the weighted transfer terms (see the bus tile)
          const double s = fma(oPf, b.cP, fma(oQf, b.cQ, fma(oPt, b.cPt, oQt * b.cQt)));
          const double r = fma(oQf, b.cP, fma(-oPf, b.cQ, fma(oPt, b.cQt, -(oQt * b.cPt))));
          if constexpr (R::V) {
            const double u_a = b.w * r;  // d/dtheta_f; d/dtheta_t = -u_a
            const double u_f = fma(2.0 * b.vf, fma(oPf, b.gff, -(oQf * b.bff)), b.vt * s);
            const double u_t = fma(2.0 * b.vt, fma(oPt, b.gtt, -(oQt * b.btt)), b.vf * s);
            if (sf != kNoSlot) {
              rec[(R::oV + 0) * BE + sf] = u_a;
              rec[(R::oV + 1) * BE + sf] = u_f;
            }
            if (st != kNoSlot) {
              rec[(R::oV + 0) * BE + st] = -u_a;
              rec[(R::oV + 1) * BE + st] = u_t;
            }
          }
          if constexpr (R::HV) {
            const double m2f = 2.0 * mf, m2t = 2.0 * mt;
            const double ccf = fma(b.cP, b.cP, b.cQ * b.cQ), cct = fma(b.cPt, b.cPt, b.cQt * b.cQt);
            const double a = fma(-b.w, s, (b.w * b.w) * fma(m2f, ccf, m2t * cct));
            const double beta_f =
                fma(b.vt, r, -(2.0 * m2f) * (b.vf * b.w) * fma(b.gff, b.cQ, b.bff * b.cP));
            const double beta_t =
                -fma(b.vf, r, (2.0 * m2t) * (b.vt * b.w) * fma(b.gtt, b.cQt, b.btt * b.cPt));
            const double pff = b.Pf_f(), qff = b.Qf_f(), ptt = b.Pt_t(), qtt = b.Qt_t();
            const double vv_ff = fma(2.0, fma(oPf, b.gff, -(oQf * b.bff)),
                                     fma(m2f, fma(pff, pff, qff * qff), m2t * (b.vt * b.vt) * cct));
            const double vv_tt = fma(2.0, fma(oPt, b.gtt, -(oQt * b.btt)),
                                     fma(m2f * (b.vf * b.vf), ccf, m2t * fma(ptt, ptt, qtt * qtt)));
            const double vv_ft =
                s + fma(m2f * b.vf, fma(2.0 * b.vf, fma(b.gff, b.cP, -(b.bff * b.cQ)), b.vt * ccf),
                        m2t * b.vt * fma(2.0 * b.vt, fma(b.gtt, b.cPt, -(b.btt * b.cQt)), b.vf * cct));
            const double da = gd[ii][0] - gd[ii][1], dvf = gd[ii][2], dvt = gd[ii][3];
            const double h_a = fma(a, da, fma(beta_f, dvf, -(beta_t * dvt)));
            if (sf != kNoSlot) {
              rec[(R::oHV + 0) * BE + sf] = h_a;
              rec[(R::oHV + 1) * BE + sf] = fma(beta_f, da, fma(vv_ff, dvf, vv_ft * dvt));
            }
            if (st != kNoSlot) {
              rec[(R::oHV + 0) * BE + st] = -h_a;
              rec[(R::oHV + 1) * BE + st] = fma(-beta_t, da, fma(vv_ft, dvf, vv_tt * dvt));
            }
          }
        }
      }
    }
  }

  // ---- lane per bus: its own terms and its ends' records summed in
  // adjacency order.  The own terms of the first E instances are loaded
  // before the barrier (their loads overlap the wait), the others' after it,
  // one instance at a time: a tile of four holds one set across the barrier,
  // smaller tiles all of theirs.
  const bool has_bus = tid < nbus;
  const int i = b0 + tid;
  int ea = 0, eb = 0;
  double4 bd{};  // pd, qd, gs, bs
  auto own_terms = [&](int ii, double& o0, double& o1, double& o2) {
    o0 = o1 = o2 = 0.0;
    const double* x = xs[ii];
    const double vi = x[nb + i];  // v_i, or f_i in the cartesian representation
    double lvm = 0.0;
    (void)lvm;
    double ei = 0.0;
    (void)ei;
    if constexpr (CART) {
      ei = x[i];
      if constexpr (MUL) lvm = mul[ii][2 * nb + 2 * nll[ii] + i];
    }
    if constexpr (R::V) {
      const double* m = mul[ii];
      if constexpr (CART) {
        const double kap = 2.0 * (fma(m[i], bd.z, -(m[nb + i] * bd.w)) + lvm);
        o0 = kap * ei;   // theta (e) column
        o1 = kap * vi;   // v (f) column
      } else {
        o1 = 2.0 * vi * fma(m[i], bd.z, -(m[nb + i] * bd.w));
      }
    }
    if constexpr (R::HV) {
      const double* m = mul[ii];
      const double* d = dir[ii];
      if constexpr (CART) {
        const double kap = 2.0 * (fma(m[i], bd.z, -(m[nb + i] * bd.w)) + lvm);
        o0 = kap * d[i];
        o1 = kap * d[nb + i];
      } else {
        o1 = 2.0 * fma(m[i], bd.z, -(m[nb + i] * bd.w)) * d[nb + i];
      }
    }
    if constexpr (R::JV) {
      const double* d = dir[ii];
      double dpg = 0, dqg = 0;
      for (int g = N.gen_ptr[i], g1 = N.gen_ptr[i + 1]; g < g1; ++g) {
        const int kk = N.gen_ident ? g : N.gen_list[g];
        dpg += d[2 * nb + kk];
        dqg += d[2 * nb + N.ng + kk];
      }
      double jvP, jvQ;
      if constexpr (CART) {  // d|V_i|^2 along the direction
        const double jvm = 2.0 * fma(ei, d[i], vi * d[nb + i]);
        o2 = jvm;
        jvP = bd.z * jvm - dpg;
        jvQ = -bd.w * jvm - dqg;
      } else {
        jvP = 2.0 * bd.z * vi * d[nb + i] - dpg;
        jvQ = -2.0 * bd.w * vi * d[nb + i] - dqg;
      }
      for (int q = 0; q < N.sl.ns; ++q) {
        const double tt = N.sl.coef[q] * d[2 * nb + 2 * N.ng + q * nb + i];
        if (N.sl.row[q] == 0) jvP += tt; else jvQ += tt;
      }
      o0 = jvP;
      o1 = jvQ;
    }
  };
  constexpr int E = NI <= 3 ? NI : 1;
  double f0[NI], f1[NI], f2[NI];  // own terms of the first E instances
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) f0[ii] = f1[ii] = f2[ii] = 0.0;
  if (has_bus) {
    ea = N.be_ptr[i] - e0;
    eb = N.be_ptr[i + 1] - e0;
    bd = N.bus[i];
#pragma unroll
    for (int ii = 0; ii < E; ++ii) {
      if (ii >= ni) break;
      own_terms(ii, f0[ii], f1[ii], f2[ii]);
    }
  }
  __syncthreads();
  if (has_bus) {
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      if (ii >= ni) break;
      double own0 = f0[ii], own1 = f1[ii], own2 = f2[ii];
      if (ii >= E) own_terms(ii, own0, own1, own2);
      (void)own2;
      const double* rec = smem + ii * (R::N * BE);
      constexpr int o = R::V ? R::oV : (R::HV ? R::oHV : R::oJV);
      double s0 = 0.0, s1 = 0.0;
      for (int e = ea; e < eb; ++e) {
        s0 += rec[(o + 0) * BE + e];
        s1 += rec[(o + 1) * BE + e];
      }
      if constexpr (R::V || R::HV) {
        double* out = (R::V ? B.u : B.out) + xo[ii];
        put(&out[i], CART ? s0 + own0 : s0);
        put(&out[nb + i], s1 + own1);
      } else {
        double* out = B.out + co[ii];
        put(&out[i], s0 + own0);
        put(&out[nb + i], s1 + own1);
        if constexpr (CART) put(&out[2 * nb + 2 * nll[ii] + i], own2);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// gen tile: objective, its gradient, the Pg diagonal of H, the Pg/Qg part of
// the VJP, and this chunk's fixed-tree partial sum of the cost.  Its items
// are the generators, then (if the net has them) the slack variables, each
// with its own penalty term, gradient, H diagonal and VJP/HVP entries.

template <unsigned WHAT, int WG>
__device__ void gen_tile(const Bufs& B, const InstOff& I, const NetDev& N, int k0, int k1,
                         int chunk, double* smem) {
  constexpr bool DO_F = (WHAT & W_F) != 0;
  constexpr bool DO_GF = (WHAT & W_GRADF) != 0;
  constexpr bool DO_H = (WHAT & W_H) != 0;
  constexpr bool DO_V = (WHAT & W_VJP) != 0;
  constexpr bool DO_HV = (WHAT & W_HVP) != 0;
  const int tid = threadIdx.x;
  const int nb = N.nb, ng = N.ng;
  const double Bm = N.base_mva;
  const double* x = B.x + I.xo;
  double* gradf = (DO_GF && B.gradf) ? B.gradf + I.xo : nullptr;
  double* hess = (DO_H && B.hess) ? B.hess + I.ho : nullptr;
  const bool fout = DO_F && B.f != nullptr;
  const double sigma = B.sigma ? B.sigma[I.k] : B.sigma_v;
  const double wf = B.wf ? B.wf[I.k] : B.wf_v;
  const int hpg = N.hpg - 4 * I.out_rm;
  // each reduction slot sums its items in item order: kGenPerSlot
  // generators, or kSlackPerSlot slack variables
  const int per = k0 >= ng ? kSlackPerSlot : kGenPerSlot;
  for (int t = tid; t < kGenChunk; t += WG) {
    double term = 0.0;
    for (int r = 0; r < per; ++r) {
      const int k = k0 + t + r * kGenChunk;
      if (k >= k1) break;
      if (k >= ng) {  // slack variable j of block s at bus i
        const int j = k - ng, s = j / nb, i = j - s * nb;
        const int col = 2 * nb + 2 * ng + j;
        const double c2 = N.sl.c2[s], c1 = N.sl.c1[s];
        const double p = Bm * x[col];
        const double grad = Bm * fma(2.0 * c2, p, c1);
        if (gradf) put(&gradf[col], grad);
        if (hess) put(&hess[hpg + k], sigma * (2.0 * c2 * Bm * Bm));
        if constexpr (DO_V) {
          const double* w = B.wc + I.co;
          put(&B.u[I.xo + col], fma(wf, grad, N.sl.coef[s] * w[N.sl.row[s] * nb + i]));
        }
        if constexpr (DO_HV) {
          put(&B.out[I.xo + col], sigma * (2.0 * c2 * Bm * Bm) * B.dir[I.xo + col]);
        }
        if (fout) term += fma(c2, p, c1) * p;
      } else {
        const double pg = x[2 * nb + k];
        const double c2 = N.gen_c2[k], c1 = N.gen_c1[k];
        const double p = Bm * pg;
        const double grad = Bm * fma(2.0 * c2, p, c1);
        if (gradf) {
          put(&gradf[2 * nb + k], grad);
          put(&gradf[2 * nb + ng + k], 0.0);
        }
        if (hess) put(&hess[hpg + k], sigma * (2.0 * c2 * Bm * Bm));
        if constexpr (DO_V) {
          const double* w = B.wc + I.co;
          const int bus = N.gen_bus[k];
          put(&B.u[I.xo + 2 * nb + k], fma(wf, grad, -w[bus]));
          put(&B.u[I.xo + 2 * nb + ng + k], -w[nb + bus]);
        }
        if constexpr (DO_HV) {
          double* o = B.out + I.xo;
          put(&o[2 * nb + k], sigma * (2.0 * c2 * Bm * Bm) * B.dir[I.xo + 2 * nb + k]);
          put(&o[2 * nb + ng + k], 0.0);
        }
        if (fout) term += fma(fma(c2, p, c1), p, N.gen_c0[k]);
      }
    }
    if (fout) smem[t] = term;
  }
  if (!fout) return;
  // fixed pairwise tree over the chunk's 256 slots, whatever the WG size
  __syncthreads();
  for (int s = kGenChunk / 2; s > 0; s >>= 1) {
    for (int t = tid; t < s; t += WG) smem[t] = smem[t] + smem[t + s];
    __syncthreads();
  }
  if (tid == 0) {
    if (N.nchunks == 1)
      put(&B.f[I.k], smem[0]);  // the only partial is f (no k_fsum needed)
    else
      B.fpart[I.fpo + chunk] = smem[0];
  }
}

// f of each instance with several chunks: its chunk partials added in chunk
// order (a single-chunk instance has f written by its generator tile).  A
// kernel of its own, enqueued after the evaluation on the same stream, so
// the partials are visible without fences; the host skips it when no
// instance has more than one chunk.
__global__ __launch_bounds__(256) void k_fsum(const InstOff* __restrict__ table, InstOff one,
                                              int first, int count, const double* __restrict__ fpart,
                                              double* __restrict__ f) {
  const int k = first + static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (k >= first + count) return;
  const InstOff I = table ? table[k] : one;
  const int nch = I.net->nchunks;
  if (nch == 1) return;
  double s = 0.0;
  for (int ch = 0; ch < nch; ++ch) s += fpart[I.fpo + ch];
  put(&f[I.k], s);
}

// ---------------------------------------------------------------------------

// The products' kernel: bus tiles of up to kProdInst instances (prod_tile) and
// generator tiles, at the waves per SIMD their registers allow without
// spilling: three for the HVP, four otherwise.
template <unsigned WHAT>
struct ProdWaves {
  static constexpr int value = (WHAT & W_HVP) != 0 ? 3 : 4;
};

template <unsigned WHAT, int WG, int BE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(ProdWaves<WHAT>::value)))
void k_prod(Bufs B, const InstOff* __restrict__ table, InstOff one, const Tile* __restrict__ tiles,
            int ntiles) {
  __shared__ double smem[Lds<WHAT, BE, 0>::kMax];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile T = tiles[t];
    const InstOff I = table ? table[T.inst] : one;
    const NetDev& N = *I.net;
    if ((T.kind_aux & 3) == TILE_BUS) {
      if (T.more[0] >= 0) {
        constexpr int G = prod_group(WHAT);
        int ni = 2;
        while (ni < G && T.more[ni - 1] >= 0) ++ni;
        prod_tile<WHAT, WG, BE, G>(B, table, I, N, T, ni, one.work, smem);
      } else {
        prod_tile<WHAT, WG, BE, 1>(B, table, I, N, T, 1, one.work, smem);
      }
    } else {
      gen_tile<WHAT, WG>(B, I, N, T.a0, T.a1, T.kind_aux >> 2, smem);
    }
    __syncthreads();
  }
}

template <unsigned WHAT, int WG, int BE, int NBUS, int STAGE>
__global__ __launch_bounds__(WG) void k_eval(Bufs B, const InstOff* __restrict__ table,
                                             InstOff one, const Tile* __restrict__ tiles,
                                             int ntiles) {
  __shared__ double smem[Lds<WHAT, BE, STAGE>::kMax];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile T = tiles[t];
    const InstOff I = table ? table[T.inst] : one;
    const NetDev& N = *I.net;
    if ((T.kind_aux & 3) == TILE_BUS) {
      bus_tile<WHAT, WG, BE, NBUS, STAGE>(B, I, N, T, one.work, smem);
    } else {
      if constexpr ((WHAT & (W_F | W_GRADF | W_H | W_VJP | W_HVP)) != 0)
        gen_tile<WHAT, WG>(B, I, N, T.a0, T.a1, T.kind_aux >> 2, smem);
    }
    __syncthreads();
  }
}

template <unsigned WHAT>
hipError_t launch_caps(int tile_be, const Bufs& b, const InstOff* table, const InstOff& one,
                       const Tile* tiles, int ntiles, int grid, hipStream_t s) {
  const int blocks = grid > 0 ? (grid < ntiles ? grid : ntiles) : ntiles;
  if (blocks <= 0) return hipSuccess;
  switch (tile_be) {
#define ACOPF_CASE(C)                                                                      \
  case C.cls:                                                                              \
    if constexpr ((WHAT & (W_VJP | W_HVP | W_JVP)) != 0)                                   \
      k_prod<WHAT, C.wg, C.be><<<blocks, C.wg, 0, s>>>(b, table, one, tiles, ntiles);       \
    else                                                                                   \
      k_eval<WHAT, C.wg, C.be, C.nbus, C.stage><<<blocks, C.wg, 0, s>>>(b, table, one, tiles, ntiles); \
    break;
    ACOPF_CASE(kCaps64)
    ACOPF_CASE(kCaps128)
    ACOPF_CASE(kCaps256)
    ACOPF_CASE(kCaps512)
#undef ACOPF_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fsum(const InstOff* table, const InstOff& one, int first, int count,
                       const double* fpart, double* f, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  k_fsum<<<(count + 255) / 256, 256, 0, stream>>>(table, one, first, count, fpart, f);
  return hipGetLastError();
}

hipError_t launch_eval(unsigned kvariant, int tile_be, const Bufs& b, const InstOff* table,
                       const InstOff& one, const Tile* tiles, int ntiles, int grid,
                       hipStream_t stream) {
  constexpr unsigned C = W_CART;
  switch (kvariant) {
    case K_FG | C: return launch_caps<K_FG | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_J | C: return launch_caps<K_J | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_H | C: return launch_caps<K_H | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_ALL | C:
      return launch_caps<K_ALL | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_VJP | C:
      return launch_caps<K_VJP | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_HVP | C:
      return launch_caps<K_HVP | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_JVP | C:
      return launch_caps<K_JVP | C>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_FG: return launch_caps<K_FG>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_J: return launch_caps<K_J>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_H: return launch_caps<K_H>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_ALL: return launch_caps<K_ALL>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_VJP: return launch_caps<K_VJP>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_HVP: return launch_caps<K_HVP>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_JVP: return launch_caps<K_JVP>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace acopf
