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
//            the Lagrangian; per end inside the tile an LDS record (flows,
//            the six Jacobian terms, the four Hessian terms, or the two VJP
//            terms).  A branch whose from-bus the tile owns also writes its
//            flow-limit rows: h = P^2 + Q^2 at both ends and their Jacobian
//            rows 2 (P dP + Q dQ) on (theta_f, theta_t, v_f, v_t).  Lanes
//            also stage each bus's own terms (shunts, load, generation).
//            Phase B, lane per output entry: a host-built slot map gives each
//            entry of the tile's CSR row segments (J P and Q rows, H theta and
//            v rows) as a signed sum over a contiguous range of records --
//            branch ends are sorted by (bus, far bus, branch), so a diagonal
//            entry sums all of a bus's ends and an off-diagonal entry the ends
//            of one group of parallel branches -- plus a bus term; consecutive
//            lanes store consecutive entries.  No atomics: every sum has one
//            owner and a fixed order, so results are bitwise reproducible
//            whatever the tiling.
//  gen tile  a fixed chunk of 256 generators: grad f, the Pg diagonal of H,
//            the Pg/Qg part of the VJP and a fixed-tree partial sum of the
//            cost; the last chunk of an instance to finish (ticket counter)
//            adds the partials in chunk order into f and re-arms the counter.
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

#include "acopf_internal.h"

namespace acopf {
namespace {

// ---------------------------------------------------------------------------
// one branch: both end flows and first derivatives with respect to
// (theta_f, v_f, v_t)

struct Br {
  double vf, vt, w, cP, cQ, cPt, cQt;
  double Pf, Qf, Pt, Qt;
  double Pf_a, Pf_f, Pf_t, Qf_a, Qf_f, Qf_t;  // d/dtheta_f, d/dv_f, d/dv_t of the from flow
  double Pt_a, Pt_f, Pt_t, Qt_a, Qt_f, Qt_t;  // ... of the to flow
};

__device__ __forceinline__ void branch_eval(double thf, double tht, double vf, double vt,
                                            const BranchY& y, Br& o) {
  double sn, cs;
  sincos(thf - tht, &sn, &cs);
  const double w = vf * vt;
  const double cP = fma(y.gft, cs, y.bft * sn);
  const double cQ = fma(y.gft, sn, -(y.bft * cs));
  const double cPt = fma(y.gtf, cs, -(y.btf * sn));
  const double cQt = -fma(y.gtf, sn, y.btf * cs);
  o.vf = vf;
  o.vt = vt;
  o.w = w;
  o.cP = cP;
  o.cQ = cQ;
  o.cPt = cPt;
  o.cQt = cQt;
  const double vf2 = vf * vf, vt2 = vt * vt;
  o.Pf = fma(y.gff, vf2, w * cP);
  o.Qf = fma(-y.bff, vf2, w * cQ);
  o.Pt = fma(y.gtt, vt2, w * cPt);
  o.Qt = fma(-y.btt, vt2, w * cQt);
  o.Pf_a = -(w * cQ);
  o.Pf_f = fma(2.0 * y.gff, vf, vt * cP);
  o.Pf_t = vf * cP;
  o.Qf_a = w * cP;
  o.Qf_f = fma(-2.0 * y.bff, vf, vt * cQ);
  o.Qf_t = vf * cQ;
  o.Pt_a = w * cQt;
  o.Pt_f = vt * cPt;
  o.Pt_t = fma(2.0 * y.gtt, vt, vf * cPt);
  o.Qt_a = -(w * cPt);
  o.Qt_f = vt * cQt;
  o.Qt_t = fma(-2.0 * y.btt, vt, vf * cQt);
}

// Record layout of phase A (structure of arrays in LDS, BE entries per field).
template <unsigned WHAT>
struct Rec {
  static constexpr bool C = (WHAT & W_C) != 0;
  static constexpr bool J = (WHAT & W_J) != 0;
  static constexpr bool H = (WHAT & W_H) != 0;
  static constexpr bool V = (WHAT & W_VJP) != 0;
  static constexpr int oC = 0;                  // P_e, Q_e
  static constexpr int oJ = oC + (C ? 2 : 0);   // dP/dth_e, dP/dv_e, dP/dv_o, dQ/... (o = far end)
  static constexpr int oH = oJ + (J ? 6 : 0);   // d2/dth_e2, d2/dv_e dth_e, d2/dv_e2, d2/dv_e dv_o
  static constexpr int oV = oH + (H ? 4 : 0);   // u_th_e, u_v_e
  static constexpr int N = oV + (V ? 2 : 0);
};

// Bus terms staged by phase A (structure of arrays, NBUS entries per field).
template <unsigned WHAT>
struct BusRec {
  static constexpr bool C = (WHAT & W_C) != 0;
  static constexpr bool J = (WHAT & W_J) != 0;
  static constexpr bool H = (WHAT & W_H) != 0;
  static constexpr bool V = (WHAT & W_VJP) != 0;
  static constexpr int oJ = 0;                  // 2 gs v, -2 bs v
  static constexpr int oH = oJ + (J ? 2 : 0);   // 2 (lP gs - lQ bs)
  static constexpr int oC = oH + (H ? 1 : 0);   // (gs v^2 - Pg) + Pd, (-bs v^2 - Qg) + Qd
  static constexpr int oV = oC + (C ? 2 : 0);   // 2 v (wP gs - wQ bs)
  static constexpr int N = oV + (V ? 1 : 0);
};

template <unsigned WHAT, int BE, int NBUS>
struct Lds {
  static constexpr int kRec = Rec<WHAT>::N * BE;
  static constexpr int kBus = kRec + BusRec<WHAT>::N * NBUS + NBUS;  // + (first end, count) per bus
  static constexpr int kGen = kGenChunk;
  static constexpr int kMax = kBus > kGen ? kBus : kGen;
};

__device__ __forceinline__ int after_outage(int l, int ol) { return (ol >= 0 && l > ol) ? 1 : 0; }

// ---------------------------------------------------------------------------
// bus tile

// Position of a base slot in an instance that may have lost slots: -1 if
// the slot itself was removed, else the base position minus the removed
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

template <unsigned WHAT, int WG, int BE, int NBUS>
__device__ void bus_tile(const Bufs& B, const InstOff& I, const NetDev& N, const Tile& T,
                         double* smem) {
  using R = Rec<WHAT>;
  using U = BusRec<WHAT>;
  constexpr bool DO_GF = (WHAT & W_GRADF) != 0 && !R::V;
  const int tid = threadIdx.x;
  const int nb = N.nb;
  const int ol = I.out_l;
  const int nll = N.nl - (ol >= 0 ? 1 : 0);
  const int b0 = T.a0, nbus = T.a1 - T.a0, e0 = T.e0;
  double* rec = smem;
  double* bus = smem + Lds<WHAT, BE, NBUS>::kRec;
  int2* bus_e = reinterpret_cast<int2*>(bus + U::N * NBUS);
  const double* x = B.x + I.xo;
  const double* mul = R::H ? B.lam + I.co : (R::V ? B.wc + I.co : nullptr);
  const bool hneed = R::V || (R::H && B.hess != nullptr);
  double* cflow = (R::C && B.c) ? B.c + I.co + 2 * nb : nullptr;
  double* jflow = (R::J && B.jac) ? B.jac + I.jo + (N.jflow - 8 * I.out_rm) : nullptr;

  // ---- phase A (1): lane per branch touching the tile
  for (int k = tid; k < T.nw; k += WG) {
    const WorkItem wi = I.work[T.w0 + k];
    const int l = wi.l, f = wi.f, t = wi.t;
    const uint32_t sf = wi.slots & 0xFFFFu, st = wi.slots >> 16;
    if (l == ol) {  // removed branch: its ends keep their places and add zero
#pragma unroll
      for (int q = 0; q < R::N; ++q) {
        if (sf != kNoSlot) rec[q * BE + sf] = 0.0;
        if (st != kNoSlot) rec[q * BE + st] = 0.0;
      }
      continue;
    }
    const BranchY y = N.br_y[l];
    Br b;
    branch_eval(x[f], x[t], x[nb + f], x[nb + t], y, b);
    const int lp = l - after_outage(l, ol);
    if constexpr (R::C) {
      if (sf != kNoSlot) {
        rec[(R::oC + 0) * BE + sf] = b.Pf;
        rec[(R::oC + 1) * BE + sf] = b.Qf;
      }
      if (st != kNoSlot) {
        rec[(R::oC + 0) * BE + st] = b.Pt;
        rec[(R::oC + 1) * BE + st] = b.Qt;
      }
    }
    if constexpr (R::J) {
      if (sf != kNoSlot) {
        rec[(R::oJ + 0) * BE + sf] = b.Pf_a;
        rec[(R::oJ + 1) * BE + sf] = b.Pf_f;
        rec[(R::oJ + 2) * BE + sf] = b.Pf_t;
        rec[(R::oJ + 3) * BE + sf] = b.Qf_a;
        rec[(R::oJ + 4) * BE + sf] = b.Qf_f;
        rec[(R::oJ + 5) * BE + sf] = b.Qf_t;
      }
      if (st != kNoSlot) {  // to end: d/dtheta_t = -d/dtheta_f
        rec[(R::oJ + 0) * BE + st] = -b.Pt_a;
        rec[(R::oJ + 1) * BE + st] = b.Pt_t;
        rec[(R::oJ + 2) * BE + st] = b.Pt_f;
        rec[(R::oJ + 3) * BE + st] = -b.Qt_a;
        rec[(R::oJ + 4) * BE + st] = b.Qt_t;
        rec[(R::oJ + 5) * BE + st] = b.Qt_f;
      }
    }
    if (sf != kNoSlot) {  // the from-bus owner writes the flow-limit rows
      if (cflow) {
        cflow[lp] = fma(b.Pf, b.Pf, b.Qf * b.Qf);
        cflow[nll + lp] = fma(b.Pt, b.Pt, b.Qt * b.Qt);
      }
      if (jflow) {
        const double hf_a = 2.0 * fma(b.Pf, b.Pf_a, b.Qf * b.Qf_a);
        const double hf_f = 2.0 * fma(b.Pf, b.Pf_f, b.Qf * b.Qf_f);
        const double hf_t = 2.0 * fma(b.Pf, b.Pf_t, b.Qf * b.Qf_t);
        const double ht_a = 2.0 * fma(b.Pt, b.Pt_a, b.Qt * b.Qt_a);
        const double ht_f = 2.0 * fma(b.Pt, b.Pt_f, b.Qt * b.Qt_f);
        const double ht_t = 2.0 * fma(b.Pt, b.Pt_t, b.Qt * b.Qt_t);
        const bool asc = f < t;  // columns ascend: theta_lo, theta_hi, v_lo, v_hi
        double* rf = jflow + 4 * lp;
        double* rt = jflow + 4 * nll + 4 * lp;
        rf[0] = asc ? hf_a : -hf_a;
        rf[1] = asc ? -hf_a : hf_a;
        rf[2] = asc ? hf_f : hf_t;
        rf[3] = asc ? hf_t : hf_f;
        rt[0] = asc ? ht_a : -ht_a;
        rt[1] = asc ? -ht_a : ht_a;
        rt[2] = asc ? ht_f : ht_t;
        rt[3] = asc ? ht_t : ht_f;
      }
    }
    if constexpr (R::H || R::V) {
      if (!hneed) continue;  // the full variant reads multipliers only when H is wanted
      const double mf = mul[2 * nb + lp];
      const double mt = mul[2 * nb + nll + lp];
      // weights of dP, dQ in  lP P + lQ Q + mu (P^2 + Q^2)
      const double oPf = fma(2.0 * mf, b.Pf, mul[f]);
      const double oQf = fma(2.0 * mf, b.Qf, mul[nb + f]);
      const double oPt = fma(2.0 * mt, b.Pt, mul[t]);
      const double oQt = fma(2.0 * mt, b.Qt, mul[nb + t]);
      if constexpr (R::H) {
        // s: the weighted transfer terms; d2L/dv_f dv_t starts with s and
        // d2L/dtheta_f^2 with -w s
        const double s = fma(oPf, b.cP, fma(oQf, b.cQ, fma(oPt, b.cPt, oQt * b.cQt)));
        const double m2f = 2.0 * mf, m2t = 2.0 * mt;
        const double a = fma(-b.w, s,
                             fma(m2f, fma(b.Pf_a, b.Pf_a, b.Qf_a * b.Qf_a),
                                 m2t * fma(b.Pt_a, b.Pt_a, b.Qt_a * b.Qt_a)));
        // d2L/dv_f dtheta_f
        const double r = fma(oQf, b.cP, fma(-oPf, b.cQ, fma(oPt, b.cQt, -(oQt * b.cPt))));
        const double beta_f = fma(b.vt, r,
                                  fma(m2f, fma(b.Pf_f, b.Pf_a, b.Qf_f * b.Qf_a),
                                      m2t * fma(b.Pt_f, b.Pt_a, b.Qt_f * b.Qt_a)));
        // d2L/dv_t dtheta_t = -d2L/dv_t dtheta_f
        const double beta_t = -fma(b.vf, r,
                                   fma(m2f, fma(b.Pf_t, b.Pf_a, b.Qf_t * b.Qf_a),
                                       m2t * fma(b.Pt_t, b.Pt_a, b.Qt_t * b.Qt_a)));
        const double vv_ff = fma(2.0, fma(oPf, y.gff, -(oQf * y.bff)),
                                 fma(m2f, fma(b.Pf_f, b.Pf_f, b.Qf_f * b.Qf_f),
                                     m2t * fma(b.Pt_f, b.Pt_f, b.Qt_f * b.Qt_f)));
        const double vv_tt = fma(2.0, fma(oPt, y.gtt, -(oQt * y.btt)),
                                 fma(m2f, fma(b.Pf_t, b.Pf_t, b.Qf_t * b.Qf_t),
                                     m2t * fma(b.Pt_t, b.Pt_t, b.Qt_t * b.Qt_t)));
        const double vv_ft = s + fma(m2f, fma(b.Pf_f, b.Pf_t, b.Qf_f * b.Qf_t),
                                     m2t * fma(b.Pt_f, b.Pt_t, b.Qt_f * b.Qt_t));
        if (sf != kNoSlot) {
          rec[(R::oH + 0) * BE + sf] = a;
          rec[(R::oH + 1) * BE + sf] = beta_f;
          rec[(R::oH + 2) * BE + sf] = vv_ff;
          rec[(R::oH + 3) * BE + sf] = vv_ft;
        }
        if (st != kNoSlot) {
          rec[(R::oH + 0) * BE + st] = a;
          rec[(R::oH + 1) * BE + st] = beta_t;
          rec[(R::oH + 2) * BE + st] = vv_tt;
          rec[(R::oH + 3) * BE + st] = vv_ft;
        }
      }
      if constexpr (R::V) {
        const double u_a = fma(oPf, b.Pf_a, fma(oQf, b.Qf_a, fma(oPt, b.Pt_a, oQt * b.Qt_a)));
        if (sf != kNoSlot) {
          rec[(R::oV + 0) * BE + sf] = u_a;
          rec[(R::oV + 1) * BE + sf] =
              fma(oPf, b.Pf_f, fma(oQf, b.Qf_f, fma(oPt, b.Pt_f, oQt * b.Qt_f)));
        }
        if (st != kNoSlot) {
          rec[(R::oV + 0) * BE + st] = -u_a;
          rec[(R::oV + 1) * BE + st] =
              fma(oPf, b.Pf_t, fma(oQf, b.Qf_t, fma(oPt, b.Pt_t, oQt * b.Qt_t)));
        }
      }
    }
  }

  // ---- phase A (2): lane per bus, the bus's own terms
  const bool jout = R::J && B.jac != nullptr;
  const bool hout = R::H && B.hess != nullptr;
  double* c = (R::C && B.c) ? B.c + I.co : nullptr;
  for (int ib = tid; ib < nbus; ib += WG) {
    const int i = b0 + ib;
    const int ea = N.be_ptr[i];
    bus_e[ib] = make_int2(ea - e0, N.be_ptr[i + 1] - ea);
    const double4 bd = N.bus[i];  // pd, qd, gs, bs
    const double vi = x[nb + i];
    if constexpr (U::J) {
      bus[(U::oJ + 0) * NBUS + ib] = 2.0 * bd.z * vi;
      bus[(U::oJ + 1) * NBUS + ib] = -2.0 * bd.w * vi;
    }
    if constexpr (U::H) {
      if (hout) bus[U::oH * NBUS + ib] = 2.0 * fma(mul[i], bd.z, -(mul[nb + i] * bd.w));
    }
    if constexpr (U::C) {
      if (c) {
        double pg = 0, qg = 0;
        for (int g = N.gen_ptr[i], g1 = N.gen_ptr[i + 1]; g < g1; ++g) {
          const int k = N.gen_list[g];
          pg += x[2 * nb + k];
          qg += x[2 * nb + N.ng + k];
        }
        bus[(U::oC + 0) * NBUS + ib] = (bd.z * vi * vi - pg) + bd.x;
        bus[(U::oC + 1) * NBUS + ib] = (-bd.w * vi * vi - qg) + bd.y;
      }
    }
    if constexpr (U::V) {
      bus[U::oV * NBUS + ib] = 2.0 * vi * fma(mul[i], bd.z, -(mul[nb + i] * bd.w));
    }
  }
  __syncthreads();

  // ---- phase B: lane per output entry
  const int2* sm = I.slots + T.sm0;
  const bool shift = I.out_rm != 0;
  if (jout) {
    double* jac = B.jac + I.jo;
    for (int k = tid; k < T.nP; k += WG) {
      const int2 ent = sm[k];
      const int ea = ent.x & 0xFFFF, cnt = ent.x >> 16;
      const int fld = ent.y & 15, kind = (ent.y >> 5) & 7, bl = ent.y >> 8;
      double vp = 0.0, vq = 0.0;
      for (int e = ea; e < ea + cnt; ++e) {
        vp += rec[(R::oJ + fld) * BE + e];
        vq += rec[(R::oJ + 3 + fld) * BE + e];
      }
      if (ent.y & 16) {
        vp = -vp;
        vq = -vq;
      }
      if (kind == SK_JDIAG_V) {
        vp += bus[(U::oJ + 0) * NBUS + bl];
        vq += bus[(U::oJ + 1) * NBUS + bl];
      } else if (kind == SK_GEN) {
        vp = -1.0;
        vq = -1.0;
      }
      const int gp = shift ? shifted(T.jP0 + k, I.rj) : T.jP0 + k;
      const int gq = shift ? shifted(T.jQ0 + k, I.rj) : T.jQ0 + k;
      if (gp >= 0) jac[gp] = vp;
      if (gq >= 0) jac[gq] = vq;
    }
  }
  if (hout) {
    double* hess = B.hess + I.ho;
    const int2* smT = sm + T.nP;
    for (int k = tid; k < T.nT + T.nV; k += WG) {
      const int2 ent = smT[k];
      const int ea = ent.x & 0xFFFF, cnt = ent.x >> 16;
      const int fld = ent.y & 15, kind = (ent.y >> 5) & 7, bl = ent.y >> 8;
      double v = 0.0;
      for (int e = ea; e < ea + cnt; ++e) v += rec[(R::oH + fld) * BE + e];
      if (ent.y & 16) v = -v;
      if (kind == SK_HDIAG_V) v += bus[U::oH * NBUS + bl];
      const int base = k < T.nT ? T.hT0 + k : T.hV0 + (k - T.nT);
      const int gp = shift ? shifted(base, I.rh) : base;
      if (gp >= 0) hess[gp] = v;
    }
  }
  if constexpr (R::C || R::V || DO_GF) {
    double* gradf = (DO_GF && B.gradf) ? B.gradf + I.xo : nullptr;
    for (int ib = tid; ib < nbus; ib += WG) {
      const int i = b0 + ib;
      const int2 be = bus_e[ib];
      if constexpr (R::C) {
        if (c) {
          double sp = 0.0, sq = 0.0;
          for (int e = be.x; e < be.x + be.y; ++e) {
            sp += rec[(R::oC + 0) * BE + e];
            sq += rec[(R::oC + 1) * BE + e];
          }
          c[i] = sp + bus[(U::oC + 0) * NBUS + ib];
          c[nb + i] = sq + bus[(U::oC + 1) * NBUS + ib];
        }
      }
      if (gradf) {
        gradf[i] = 0.0;
        gradf[nb + i] = 0.0;
      }
      if constexpr (R::V) {
        double ut = 0.0, uv = 0.0;
        for (int e = be.x; e < be.x + be.y; ++e) {
          ut += rec[(R::oV + 0) * BE + e];
          uv += rec[(R::oV + 1) * BE + e];
        }
        double* u = B.u + I.xo;
        u[i] = ut;
        u[nb + i] = uv + bus[U::oV * NBUS + ib];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// gen tile: objective, its gradient, the Pg diagonal of H, the Pg/Qg part of
// the VJP

template <unsigned WHAT, int WG>
__device__ void gen_tile(const Bufs& B, const InstOff& I, const NetDev& N, int k0, int k1,
                         int chunk, double* smem) {
  constexpr bool DO_F = (WHAT & W_F) != 0;
  constexpr bool DO_GF = (WHAT & W_GRADF) != 0;
  constexpr bool DO_H = (WHAT & W_H) != 0;
  constexpr bool DO_V = (WHAT & W_VJP) != 0;
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
  for (int t = tid; t < kGenChunk; t += WG) {
    const int k = k0 + t;
    double term = 0.0;
    if (k < k1) {
      const double pg = x[2 * nb + k];
      const double c2 = N.gen_c2[k], c1 = N.gen_c1[k];
      const double p = Bm * pg;
      const double grad = Bm * fma(2.0 * c2, p, c1);
      if (gradf) {
        gradf[2 * nb + k] = grad;
        gradf[2 * nb + ng + k] = 0.0;
      }
      if (hess) hess[hpg + k] = sigma * (2.0 * c2 * Bm * Bm);
      if constexpr (DO_V) {
        const double* w = B.wc + I.co;
        const int bus = N.gen_bus[k];
        B.u[I.xo + 2 * nb + k] = fma(wf, grad, -w[bus]);
        B.u[I.xo + 2 * nb + ng + k] = -w[nb + bus];
      }
      if (fout) term = fma(fma(c2, p, c1), p, N.gen_c0[k]);
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
    double* fpart = B.fpart + I.fpo;
    __hip_atomic_store(&fpart[chunk], smem[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const uint32_t prev =
        __hip_atomic_fetch_add(&B.ticket[I.k], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == static_cast<uint32_t>(N.nchunks - 1)) {
      __threadfence();
      double f = 0.0;
      for (int ch = 0; ch < N.nchunks; ++ch)
        f += __hip_atomic_load(&fpart[ch], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      B.f[I.k] = f;
      __hip_atomic_store(&B.ticket[I.k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------

template <unsigned WHAT, int WG, int BE, int NBUS>
__global__ __launch_bounds__(WG) void k_eval(Bufs B, const InstOff* __restrict__ table,
                                             InstOff one, const Tile* __restrict__ tiles,
                                             int ntiles) {
  __shared__ double smem[Lds<WHAT, BE, NBUS>::kMax];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile T = tiles[t];
    const InstOff I = table ? table[T.inst] : one;
    const NetDev& N = *I.net;
    if ((T.kind_aux & 3) == TILE_BUS) {
      bus_tile<WHAT, WG, BE, NBUS>(B, I, N, T, smem);
    } else {
      if constexpr ((WHAT & (W_F | W_GRADF | W_H | W_VJP)) != 0)
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
  case C.be:                                                                               \
    k_eval<WHAT, C.wg, C.be, C.nbus><<<blocks, C.wg, 0, s>>>(b, table, one, tiles, ntiles); \
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

hipError_t launch_eval(unsigned kvariant, int tile_be, const Bufs& b, const InstOff* table,
                       const InstOff& one, const Tile* tiles, int ntiles, int grid,
                       hipStream_t stream) {
  switch (kvariant) {
    case K_FG: return launch_caps<K_FG>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_J: return launch_caps<K_J>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_H: return launch_caps<K_H>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_ALL: return launch_caps<K_ALL>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    case K_VJP: return launch_caps<K_VJP>(tile_be, b, table, one, tiles, ntiles, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace acopf
