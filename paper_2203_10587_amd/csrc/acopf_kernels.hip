// gfx950 kernels for the polar ACOPF model evaluation (FP64).
//
// One kernel template covers every entry point; the compile-time variant
// selects which outputs a tile produces.  A workgroup walks a list of tiles
// (one tile per workgroup, or a persistent grid striding over the list):
//
//  branch tile  lane per branch: one sincos of theta_f - theta_t, the four end
//               flows, h = P^2 + Q^2 at both ends and their Jacobian rows
//               (2 (P dP + Q dQ) on theta_f, theta_t, v_f, v_t).  The Jacobian
//               rows are staged in LDS and stored as one contiguous segment.
//  bus tile     a contiguous range of buses and all their branch ends.
//               Phase A, lane per branch end (uniform work): the branch seen
//               from bus i -- flows, first derivatives with respect to
//               (theta_i, v_i, v_j) and, for the Hessian, the four second
//               derivatives of this branch's share of the Lagrangian that
//               bus i's rows need -- into LDS records.
//               Phase B, lane per bus: a segmented sum over the bus's branch
//               ends in their fixed (neighbour, branch) order -- diagonal
//               entries over all of them, one off-diagonal entry per distinct
//               neighbour -- written into an LDS image of the tile's four
//               contiguous CSR row segments (J P rows, J Q rows, H theta rows,
//               H v rows).  No atomics: every sum has one owner and a fixed
//               order, so results are bitwise reproducible.
//               Phase C: the LDS image is streamed out with coalesced stores.
//  gen tile     a fixed chunk of 256 generators: grad f, the Pg diagonal of
//               H and a fixed-tree partial sum of the cost; the last chunk of
//               an instance to finish (ticket counter) adds the partials in
//               chunk order into f and re-arms the counter.
//
// The model (paper: OPFLOW section, power-balance-polar representation; the
// formulation itself is the standard polar pi-model one the paper refers to):
// for a branch seen from end i with other end j, theta = theta_i - theta_j,
// self admittance (g_ii, b_ii) and transfer admittance (g_ij, b_ij),
//   P_i =  g_ii v_i^2 + v_i v_j (g_ij cos theta + b_ij sin theta)
//   Q_i = -b_ii v_i^2 + v_i v_j (g_ij sin theta - b_ij cos theta)
// and symmetrically for end j with theta_j - theta_i.  The branch's share of
// the Lagrangian is  sum over its ends e of  lP_e P_e + lQ_e Q_e +
// mu_e (P_e^2 + Q_e^2),  with lP, lQ the balance multipliers of the end buses
// and mu_e the multiplier of the end's flow-limit row.
#include <hip/hip_runtime.h>

#include "acopf_internal.h"

namespace acopf {
namespace {

// ---------------------------------------------------------------------------
// The branch seen from end i (far end j): flows at both ends and their first
// derivatives with respect to (theta_i, v_i, v_j).  Flows depend on the
// angles only through their difference, so d/dtheta_j = -d/dtheta_i.
struct EndView {
  double vi, vj, w, cP, cQ, cPj, cQj;
  double Pi, Qi, Pj, Qj;
  double dPi_t, dPi_vi, dPi_vj, dQi_t, dQi_vi, dQi_vj;  // bus i's own end
  double dPj_t, dPj_vi, dPj_vj, dQj_t, dQj_vi, dQj_vj;  // the far end
};

__device__ __forceinline__ void end_view(double thi, double thj, double vi, double vj,
                                         double gii, double bii, double gij, double bij,
                                         double gjj, double bjj, double gji, double bji,
                                         EndView& o) {
  double sn, cs;
  sincos(thi - thj, &sn, &cs);
  const double w = vi * vj;
  const double cP = gij * cs + bij * sn;
  const double cQ = gij * sn - bij * cs;
  const double cPj = gji * cs - bji * sn;  // far end: sin(theta_j - theta_i) = -sn
  const double cQj = -gji * sn - bji * cs;
  o.vi = vi;
  o.vj = vj;
  o.w = w;
  o.cP = cP;
  o.cQ = cQ;
  o.cPj = cPj;
  o.cQj = cQj;
  o.Pi = gii * vi * vi + w * cP;
  o.Qi = -bii * vi * vi + w * cQ;
  o.Pj = gjj * vj * vj + w * cPj;
  o.Qj = -bjj * vj * vj + w * cQj;
  o.dPi_t = -w * cQ;
  o.dPi_vi = 2.0 * gii * vi + vj * cP;
  o.dPi_vj = vi * cP;
  o.dQi_t = w * cP;
  o.dQi_vi = -2.0 * bii * vi + vj * cQ;
  o.dQi_vj = vi * cQ;
  o.dPj_t = w * cQj;
  o.dPj_vi = vj * cPj;
  o.dPj_vj = 2.0 * gjj * vj + vi * cPj;
  o.dQj_t = -w * cPj;
  o.dQj_vi = vj * cQj;
  o.dQj_vj = -2.0 * bjj * vj + vi * cQj;
}

// Record layout of phase A (structure of arrays in LDS, BE entries per field).
template <unsigned WHAT>
struct Rec {
  static constexpr bool C = (WHAT & W_C) != 0;
  static constexpr bool J = (WHAT & W_J) != 0;
  static constexpr bool H = (WHAT & W_H) != 0;
  static constexpr bool V = (WHAT & W_VJP) != 0;
  static constexpr int oC = 0;                    // P_i, Q_i
  static constexpr int oJ = oC + (C ? 2 : 0);     // dP/dth_i, dP/dv_i, dP/dv_j, dQ/...
  static constexpr int oH = oJ + (J ? 6 : 0);     // a, beta, vv_ii, vv_ij
  static constexpr int oV = oH + (H ? 4 : 0);     // u_theta_i, u_v_i
  static constexpr int N = oV + (V ? 2 : 0);
};

template <unsigned WHAT, int WG, int BE, int STAGE>
struct Lds {
  static constexpr bool kStage = (WHAT & (W_J | W_H)) != 0;
  static constexpr int kBus = Rec<WHAT>::N * BE + BE / 2 + (kStage ? STAGE : 0);
  static constexpr int kBranch = (WHAT & W_J) ? 8 * WG : 1;
  static constexpr int kGen = kGenChunk;
  static constexpr int kA = kBus > kBranch ? kBus : kBranch;
  static constexpr int kMax = kA > kGen ? kA : kGen;
};

__device__ __forceinline__ int live_branches(const NetDev& N, const InstOff& I) {
  return N.nl - (I.out_l >= 0 ? 1 : 0);
}

__device__ __forceinline__ int after_outage(int l, int ol) {
  return (ol >= 0 && l > ol) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// branch tile: flow-limit rows

template <unsigned WHAT, int WG>
__device__ void branch_tile(const Bufs& B, const InstOff& I, const NetDev& N, int l0, int l1,
                            double* smem) {
  constexpr bool DO_C = (WHAT & W_C) != 0;
  constexpr bool DO_J = (WHAT & W_J) != 0;
  const int tid = threadIdx.x;
  const int nb = N.nb;
  const int nll = live_branches(N, I);
  const int ol = I.out_l;
  const int lp0 = l0 - after_outage(l0, ol);
  const int lp1 = l1 - after_outage(l1, ol);
  const double* x = B.x + I.xo;
  double* c = (DO_C && B.c) ? B.c + I.co : nullptr;
  const bool jout = DO_J && B.jac != nullptr;
  for (int l = l0 + tid; l < l1; l += WG) {
    if (l == ol) continue;
    const int lp = l - after_outage(l, ol);
    const int2 ft = N.br_ft[l];
    const BranchY y = N.br_y[l];
    EndView e;  // i = from end, j = to end
    end_view(x[ft.x], x[ft.y], x[nb + ft.x], x[nb + ft.y], y.gff, y.bff, y.gft, y.bft, y.gtt,
             y.btt, y.gtf, y.btf, e);
    if (c) {
      c[2 * nb + lp] = e.Pi * e.Pi + e.Qi * e.Qi;
      c[2 * nb + nll + lp] = e.Pj * e.Pj + e.Qj * e.Qj;
    }
    if (jout) {
      // d h / d(theta_f, v_f, v_t); d/dtheta_t = -d/dtheta_f
      const double hf_t = 2.0 * (e.Pi * e.dPi_t + e.Qi * e.dQi_t);
      const double hf_vf = 2.0 * (e.Pi * e.dPi_vi + e.Qi * e.dQi_vi);
      const double hf_vt = 2.0 * (e.Pi * e.dPi_vj + e.Qi * e.dQi_vj);
      const double ht_t = 2.0 * (e.Pj * e.dPj_t + e.Qj * e.dQj_t);
      const double ht_vf = 2.0 * (e.Pj * e.dPj_vi + e.Qj * e.dQj_vi);
      const double ht_vt = 2.0 * (e.Pj * e.dPj_vj + e.Qj * e.dQj_vj);
      const bool asc = ft.x < ft.y;  // columns ascend: theta_lo, theta_hi, v_lo, v_hi
      double* sf = smem + 4 * (lp - lp0);
      double* st = smem + 4 * WG + 4 * (lp - lp0);
      sf[0] = asc ? hf_t : -hf_t;
      sf[1] = asc ? -hf_t : hf_t;
      sf[2] = asc ? hf_vf : hf_vt;
      sf[3] = asc ? hf_vt : hf_vf;
      st[0] = asc ? ht_t : -ht_t;
      st[1] = asc ? -ht_t : ht_t;
      st[2] = asc ? ht_vf : ht_vt;
      st[3] = asc ? ht_vt : ht_vf;
    }
  }
  if (jout) {
    __syncthreads();
    const int n4 = 4 * (lp1 - lp0);
    double* jac = B.jac + I.jo;
    const int jflow = N.jflow - 8 * I.out_rm;
    double* df = jac + jflow + 4 * lp0;
    double* dt = jac + jflow + 4 * nll + 4 * lp0;
    for (int k = tid; k < n4; k += WG) {
      df[k] = smem[k];
      dt[k] = smem[4 * WG + k];
    }
  }
}

// ---------------------------------------------------------------------------
// bus tile: balance rows of c and J, theta/v rows of H, theta/v part of the VJP

// Row starts of an instance: the base pattern's, shifted for a removed
// (p, q) slot pair (p < q): rows p and q of the J balance blocks lose two
// entries each, row theta_q of H loses theta_p, row v_p loses theta_q and
// row v_q loses theta_p and v_p.
struct RowShift {
  int p, q, rm;
  __device__ __forceinline__ int below(int i) const { return (p < i ? 1 : 0) + (q < i ? 1 : 0); }
  __device__ __forceinline__ int jP(int4 r, int i) const { return r.x - 2 * rm * below(i); }
  __device__ __forceinline__ int jQ(int4 r, int i) const { return r.y - 4 * rm - 2 * rm * below(i); }
  __device__ __forceinline__ int hT(int4 r, int i) const { return r.z - rm * (q < i ? 1 : 0); }
  __device__ __forceinline__ int hV(int4 r, int i) const {
    return r.w - rm * (1 + (p < i ? 1 : 0) + 2 * (q < i ? 1 : 0));
  }
};

template <unsigned WHAT, int WG, int BE, int STAGE>
__device__ void bus_tile(const Bufs& B, const InstOff& I, const NetDev& N, int b0, int b1,
                         double* smem) {
  using R = Rec<WHAT>;
  constexpr bool DO_GF = (WHAT & W_GRADF) != 0 && !R::V;
  const int tid = threadIdx.x;
  const int nb = N.nb;
  const int nll = live_branches(N, I);
  const int ol = I.out_l;
  const int e0 = N.be_ptr[b0];
  const int ne = N.be_ptr[b1] - e0;
  double* rec = smem;
  int* nbr = reinterpret_cast<int*>(smem + R::N * BE);
  double* stage = smem + R::N * BE + BE / 2;
  const double* x = B.x + I.xo;
  const double* mul = R::H ? B.lam + I.co : (R::V ? B.wc + I.co : nullptr);

  // ---- phase A: lane per branch end
  for (int e = tid; e < ne; e += WG) {
    const int code = N.be[e0 + e];
    const int l = code >> 1;
    const bool ito = (code & 1) != 0;
    const int2 ft = N.br_ft[l];
    const int i = ito ? ft.y : ft.x;
    const int j = ito ? ft.x : ft.y;
    if (l == ol) {
      nbr[e] = -1 - j;  // removed branch: keeps its place in the order, adds nothing
      continue;
    }
    nbr[e] = j;
    const BranchY y = N.br_y[l];
    EndView v;
    end_view(x[i], x[j], x[nb + i], x[nb + j], ito ? y.gtt : y.gff, ito ? y.btt : y.bff,
             ito ? y.gtf : y.gft, ito ? y.btf : y.bft, ito ? y.gff : y.gtt, ito ? y.bff : y.btt,
             ito ? y.gft : y.gtf, ito ? y.bft : y.btf, v);
    if constexpr (R::C) {
      rec[(R::oC + 0) * BE + e] = v.Pi;
      rec[(R::oC + 1) * BE + e] = v.Qi;
    }
    if constexpr (R::J) {
      rec[(R::oJ + 0) * BE + e] = v.dPi_t;
      rec[(R::oJ + 1) * BE + e] = v.dPi_vi;
      rec[(R::oJ + 2) * BE + e] = v.dPi_vj;
      rec[(R::oJ + 3) * BE + e] = v.dQi_t;
      rec[(R::oJ + 4) * BE + e] = v.dQi_vi;
      rec[(R::oJ + 5) * BE + e] = v.dQi_vj;
    }
    if constexpr (R::H || R::V) {
      // the full-evaluation variant reads multipliers only when H is wanted
      if (!R::V && B.hess == nullptr) continue;
      const int lp = l - after_outage(l, ol);
      const double mf = mul[2 * nb + lp];
      const double mt = mul[2 * nb + nll + lp];
      const double mi = ito ? mt : mf;
      const double mj = ito ? mf : mt;
      // weights of dP, dQ in  lP P + lQ Q + mu (P^2 + Q^2)
      const double oPi = mul[i] + 2.0 * mi * v.Pi;
      const double oQi = mul[nb + i] + 2.0 * mi * v.Qi;
      const double oPj = mul[j] + 2.0 * mj * v.Pj;
      const double oQj = mul[nb + j] + 2.0 * mj * v.Qj;
      if constexpr (R::H) {
        const double s = oPi * v.cP + oQi * v.cQ + oPj * v.cPj + oQj * v.cQj;
        const double a =  // d2 / dtheta_i^2
            -v.w * s + 2.0 * mi * (v.dPi_t * v.dPi_t + v.dQi_t * v.dQi_t) +
            2.0 * mj * (v.dPj_t * v.dPj_t + v.dQj_t * v.dQj_t);
        const double beta =  // d2 / dv_i dtheta_i
            v.vj * (oQi * v.cP - oPi * v.cQ + oPj * v.cQj - oQj * v.cPj) +
            2.0 * mi * (v.dPi_vi * v.dPi_t + v.dQi_vi * v.dQi_t) +
            2.0 * mj * (v.dPj_vi * v.dPj_t + v.dQj_vi * v.dQj_t);
        const double b_self = ito ? y.btt : y.bff;
        const double g_self = ito ? y.gtt : y.gff;
        const double vvii =  // d2 / dv_i^2
            2.0 * (oPi * g_self - oQi * b_self) +
            2.0 * mi * (v.dPi_vi * v.dPi_vi + v.dQi_vi * v.dQi_vi) +
            2.0 * mj * (v.dPj_vi * v.dPj_vi + v.dQj_vi * v.dQj_vi);
        const double vvij =  // d2 / dv_i dv_j
            s + 2.0 * mi * (v.dPi_vi * v.dPi_vj + v.dQi_vi * v.dQi_vj) +
            2.0 * mj * (v.dPj_vi * v.dPj_vj + v.dQj_vi * v.dQj_vj);
        rec[(R::oH + 0) * BE + e] = a;
        rec[(R::oH + 1) * BE + e] = beta;
        rec[(R::oH + 2) * BE + e] = vvii;
        rec[(R::oH + 3) * BE + e] = vvij;
      }
      if constexpr (R::V) {
        rec[(R::oV + 0) * BE + e] = oPi * v.dPi_t + oQi * v.dQi_t + oPj * v.dPj_t + oQj * v.dQj_t;
        rec[(R::oV + 1) * BE + e] =
            oPi * v.dPi_vi + oQi * v.dQi_vi + oPj * v.dPj_vi + oQj * v.dQj_vi;
      }
    }
  }
  __syncthreads();

  // ---- phase B: lane per bus, segmented sums in (neighbour, branch) order
  const RowShift sh{I.out_p, I.out_q, I.out_rm};
  const int4 r0 = N.rows[b0];
  const int4 r1 = N.rows[b1];
  const int jP0 = sh.jP(r0, b0), jQ0 = sh.jQ(r0, b0), hT0 = sh.hT(r0, b0), hV0 = sh.hV(r0, b0);
  const int LP = sh.jP(r1, b1) - jP0, LQ = sh.jQ(r1, b1) - jQ0;
  const int LT = sh.hT(r1, b1) - hT0, LV = sh.hV(r1, b1) - hV0;
  double* sP = stage;
  double* sQ = sP + LP;
  double* sT = sQ + LQ;
  double* sV = sT + LT;
  const bool jout = R::J && B.jac != nullptr;
  const bool hout = R::H && B.hess != nullptr;
  double* c = (R::C && B.c) ? B.c + I.co : nullptr;
  double* gradf = (DO_GF && B.gradf) ? B.gradf + I.xo : nullptr;
  double* u = R::V ? B.u + I.xo : nullptr;

  for (int ib = tid; ib < b1 - b0; ib += WG) {
    const int i = b0 + ib;
    const int4 ri = N.rows[i];
    int2 ac = N.acnt[i];
    int a = ac.x, lo = ac.y;
    if (sh.rm) {
      if (i == sh.p) a -= 1;
      if (i == sh.q) { a -= 1; lo -= 1; }
    }
    const int oP = sh.jP(ri, i) - jP0, oQ = sh.jQ(ri, i) - jQ0;
    const int oT = sh.hT(ri, i) - hT0, oV = sh.hV(ri, i) - hV0;
    double sPi = 0, sQi = 0;
    double dP_t = 0, dP_v = 0, dQ_t = 0, dQ_v = 0;
    double ha = 0, hb = 0, hvv = 0;
    double ut = 0, uv = 0;
    int rank = 0;
    const int ebeg = N.be_ptr[i] - e0, eend = N.be_ptr[i + 1] - e0;
    int e = ebeg;
    while (e < eend) {
      const int key = nbr[e];
      const int j = key >= 0 ? key : -1 - key;
      bool live = false;
      double gPt = 0, gPv = 0, gQt = 0, gQv = 0, ga = 0, gb = 0, gvv = 0;
      for (; e < eend; ++e) {
        const int k2 = nbr[e];
        if ((k2 >= 0 ? k2 : -1 - k2) != j) break;
        if (k2 < 0) continue;
        live = true;
        if constexpr (R::C) {
          sPi += rec[(R::oC + 0) * BE + e];
          sQi += rec[(R::oC + 1) * BE + e];
        }
        if constexpr (R::J) {
          const double t0 = rec[(R::oJ + 0) * BE + e], t3 = rec[(R::oJ + 3) * BE + e];
          dP_t += t0;
          dP_v += rec[(R::oJ + 1) * BE + e];
          dQ_t += t3;
          dQ_v += rec[(R::oJ + 4) * BE + e];
          gPt += t0;
          gPv += rec[(R::oJ + 2) * BE + e];
          gQt += t3;
          gQv += rec[(R::oJ + 5) * BE + e];
        }
        if constexpr (R::H) {
          const double t0 = rec[(R::oH + 0) * BE + e], t1 = rec[(R::oH + 1) * BE + e];
          ha += t0;
          hb += t1;
          hvv += rec[(R::oH + 2) * BE + e];
          ga += t0;
          gb += t1;
          gvv += rec[(R::oH + 3) * BE + e];
        }
        if constexpr (R::V) {
          ut += rec[(R::oV + 0) * BE + e];
          uv += rec[(R::oV + 1) * BE + e];
        }
      }
      if (!live) continue;
      const int pos = rank + (j > i ? 1 : 0);
      if (jout) {
        sP[oP + pos] = -gPt;
        sP[oP + a + pos] = gPv;
        sQ[oQ + pos] = -gQt;
        sQ[oQ + a + pos] = gQv;
      }
      if (hout) {
        sV[oV + pos] = -gb;
        if (j < i) {
          sT[oT + pos] = -ga;
          sV[oV + a + pos] = gvv;
        }
      }
      ++rank;
    }
    const double4 bd = N.bus[i];  // pd, qd, gs, bs
    const double vi = x[nb + i];
    const int g0 = N.gen_ptr[i], g1 = N.gen_ptr[i + 1];
    if (jout) {
      sP[oP + lo] = dP_t;
      sP[oP + a + lo] = dP_v + 2.0 * bd.z * vi;
      sQ[oQ + lo] = dQ_t;
      sQ[oQ + a + lo] = dQ_v - 2.0 * bd.w * vi;
      for (int g = g0; g < g1; ++g) {
        sP[oP + 2 * a + (g - g0)] = -1.0;
        sQ[oQ + 2 * a + (g - g0)] = -1.0;
      }
    }
    if (hout) {
      const double* lam = B.lam + I.co;
      sT[oT + lo] = ha;
      sV[oV + lo] = hb;
      sV[oV + a + lo] = hvv + 2.0 * (lam[i] * bd.z - lam[nb + i] * bd.w);
    }
    if (c) {
      double pg = 0, qg = 0;
      for (int g = g0; g < g1; ++g) {
        const int k = N.gen_list[g];
        pg += x[2 * nb + k];
        qg += x[2 * nb + N.ng + k];
      }
      c[i] = sPi + bd.z * vi * vi - pg + bd.x;
      c[nb + i] = sQi - bd.w * vi * vi - qg + bd.y;
    }
    if (gradf) {
      gradf[i] = 0.0;
      gradf[nb + i] = 0.0;
    }
    if constexpr (R::V) {
      const double* w = B.wc + I.co;
      u[i] = ut;
      u[nb + i] = uv + 2.0 * (w[i] * bd.z - w[nb + i] * bd.w) * vi;
    }
  }

  // ---- phase C: stream the LDS image of the row segments out
  if (jout || hout) {
    __syncthreads();
    if (jout) {
      double* jac = B.jac + I.jo;
      for (int k = tid; k < LP; k += WG) jac[jP0 + k] = sP[k];
      for (int k = tid; k < LQ; k += WG) jac[jQ0 + k] = sQ[k];
    }
    if (hout) {
      double* hess = B.hess + I.ho;
      for (int k = tid; k < LT; k += WG) hess[hT0 + k] = sT[k];
      for (int k = tid; k < LV; k += WG) hess[hV0 + k] = sV[k];
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
      const double grad = 2.0 * c2 * Bm * p + c1 * Bm;
      if (gradf) {
        gradf[2 * nb + k] = grad;
        gradf[2 * nb + ng + k] = 0.0;
      }
      if (hess) hess[hpg + k] = sigma * (2.0 * c2 * Bm * Bm);
      if constexpr (DO_V) {
        const double* w = B.wc + I.co;
        const int bus = N.gen_bus[k];
        B.u[I.xo + 2 * nb + k] = wf * grad - w[bus];
        B.u[I.xo + 2 * nb + ng + k] = -w[nb + bus];
      }
      if (fout) term = c2 * p * p + c1 * p + N.gen_c0[k];
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

template <unsigned WHAT, int WG, int BE, int STAGE>
__global__ __launch_bounds__(WG) void k_eval(Bufs B, const InstOff* __restrict__ table,
                                             InstOff one, const Tile* __restrict__ tiles,
                                             int ntiles) {
  __shared__ double smem[Lds<WHAT, WG, BE, STAGE>::kMax];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile T = tiles[t];
    const InstOff I = table ? table[T.inst] : one;
    const NetDev& N = *I.net;
    const int kind = T.kind_aux & 3;
    if (kind == TILE_BUS) {
      bus_tile<WHAT, WG, BE, STAGE>(B, I, N, T.a0, T.a1, smem);
    } else if (kind == TILE_BRANCH) {
      if constexpr ((WHAT & (W_C | W_J)) != 0) branch_tile<WHAT, WG>(B, I, N, T.a0, T.a1, smem);
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
    case 64:
      k_eval<WHAT, 64, 64, kCaps64.stage><<<blocks, 64, 0, s>>>(b, table, one, tiles, ntiles);
      break;
    case 128:
      k_eval<WHAT, 128, 128, kCaps128.stage><<<blocks, 128, 0, s>>>(b, table, one, tiles, ntiles);
      break;
    case 256:
      k_eval<WHAT, 256, 256, kCaps256.stage><<<blocks, 256, 0, s>>>(b, table, one, tiles, ntiles);
      break;
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
