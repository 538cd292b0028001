// Host-only check of the bus-tile work lists: every position a work item or a
// bus lane stores must hold the column the CSR pattern puts there, and every
// Jacobian and Hessian entry before the flow and generator blocks must be
// stored exactly once per evaluation, and the gen tiles must cover every
// cost item (generators, then slack variables) once.  Compiled by
// tests/test_tiler.py.
#include "acopf_host.cpp"
#include <cstdio>
extern "C" int tile_check(const acopf_net_desc* d, int tile_be, unsigned slacks) {
  Topology T;
  acopf_net_opts o{};
  o.slacks = slacks;
  if (build_topology(d, &o, &T)) {
    printf("topology: %s\n", t_err.c_str());
    return 1;
  }
  std::vector<int32_t> jp, jc, hp, hc;
  build_pattern(T, -1, &jp, &jc, &hp, &hc);
  Schedule S;
  if (make_tiles(T, tile_be, &S)) {
    printf("tiles: %s\n", t_err.c_str());
    return 2;
  }
  const int nb = T.nb;
  const int qoff = T.rows[0].y - T.rows[0].x;
  std::vector<int> jcnt(T.jflow, 0), hcnt(T.hpg, 0);
  int bad = 0;
  auto chk = [&](bool c, const char* what, int a, int b) {
    if (!c && bad++ < 10) printf("FAIL %s (%d, %d)\n", what, a, b);
  };
  for (int ti = 0; ti < S.counts[0]; ++ti) {
    const Tile& tl = S.tiles[ti];
    for (int k = 0; k < tl.nw; ++k) {
      const WorkItem& wi = S.work[tl.w0 + k];
      if (wi.l < 0) continue;
      // absolute base positions from the tile-relative encoding
      struct {
        int l, f, t, grp, alo, ahi, jlo, jhi, hvlo, hvhi, hthi;
      } w{wi.l, wi.f, wi.t, wi.grp(), int(wi.alo()), int(wi.ahi()),
          wi.jlo() == kNoPos ? -1 : tl.jP0 + int(wi.jlo()),
          wi.jhi() == kNoPos ? -1 : tl.jP0 + int(wi.jhi()),
          wi.jlo() == kNoPos ? -1 : tl.hV0 + int(wi.hvlo()),
          wi.jhi() == kNoPos ? -1 : tl.hV0 + int(wi.hvhi()),
          wi.jhi() == kNoPos ? -1 : tl.hT0 + int(wi.hthi())};
      chk(wi.shifted() == (T.shifted[wi.l] != 0), "shifted flag", ti, k);
      chk(T.shifted[wi.l] != 0 || (T.y[wi.l].gtf == T.y[wi.l].gft && T.y[wi.l].btf == T.y[wi.l].bft),
          "unshifted pair", ti, k);
      if (w.grp > 1) {  // members follow, same lo/hi, same wave
        chk(k / 64 == (k + w.grp - 1) / 64, "group straddles a wave", ti, k);
        for (int m = 1; m < w.grp; ++m) {
          const WorkItem& o = S.work[tl.w0 + k + m];
          chk(o.grp() == 0 && std::min(o.f, o.t) == std::min(w.f, w.t) &&
                  std::max(o.f, o.t) == std::max(w.f, w.t) && o.l > w.l,
              "group member", ti, k + m);
        }
      }
      if (w.grp == 0) continue;
      const int lo = std::min(w.f, w.t), hi = std::max(w.f, w.t);
      if (w.jlo >= 0) {
        chk(jc[w.jlo] == hi && jc[w.jlo + w.alo] == nb + hi, "J lo P", w.jlo, hi);
        chk(jc[w.jlo + qoff] == hi && jc[w.jlo + w.alo + qoff] == nb + hi, "J lo Q", w.jlo, hi);
        chk(w.jlo >= jp[lo] && w.jlo < jp[lo + 1] && w.jlo + qoff >= jp[nb + lo] && w.jlo + qoff < jp[nb + lo + 1], "J lo row", w.jlo, lo);
        chk(hc[w.hvlo] == hi && w.hvlo >= hp[nb + lo] && w.hvlo < hp[nb + lo + 1], "H lo v-row theta", w.hvlo, hi);
        for (int p : {w.jlo, w.jlo + w.alo, w.jlo + qoff, w.jlo + w.alo + qoff}) jcnt[p]++;
        hcnt[w.hvlo]++;
      }
      if (w.jhi >= 0) {
        chk(jc[w.jhi] == lo && jc[w.jhi + w.ahi] == nb + lo, "J hi P", w.jhi, lo);
        chk(jc[w.jhi + qoff] == lo && jc[w.jhi + w.ahi + qoff] == nb + lo, "J hi Q", w.jhi, lo);
        chk(w.jhi >= jp[hi] && w.jhi < jp[hi + 1], "J hi row", w.jhi, hi);
        chk(hc[w.hthi] == lo && w.hthi >= hp[hi] && w.hthi < hp[hi + 1], "H hi theta-row", w.hthi, lo);
        chk(hc[w.hvhi] == lo && w.hvhi >= hp[nb + hi] && w.hvhi < hp[nb + hi + 1], "H hi v-row theta", w.hvhi, lo);
        chk(hc[w.hvhi + w.ahi] == nb + lo && w.hvhi + w.ahi < hp[nb + hi + 1], "H hi v-row v", w.hvhi, lo);
        for (int p : {w.jhi, w.jhi + w.ahi, w.jhi + qoff, w.jhi + w.ahi + qoff}) jcnt[p]++;
        hcnt[w.hthi]++;
        hcnt[w.hvhi]++;
        hcnt[w.hvhi + w.ahi]++;
      }
    }
    // bus diagonal and generator columns, as the kernel's phase B forms them
    for (int i = tl.a0; i < tl.a1; ++i) {
      const int4 rw = T.rows[i];
      const int a = T.acnt[i].x, blw = T.acnt[i].y;
      const int pt = rw.x + blw, pv = rw.x + a + blw;
      chk(jc[pt] == i && jc[pv] == nb + i && jc[pt + qoff] == i && jc[pv + qoff] == nb + i, "J diag", i, pt);
      for (int p : {pt, pv, pt + qoff, pv + qoff}) jcnt[p]++;
      const int g = T.gen_ptr[i + 1] - T.gen_ptr[i];
      for (int q = 0; q < g; ++q) {
        const int pg = rw.x + 2 * a + q;
        chk(jc[pg] == 2 * nb + T.gen_list[T.gen_ptr[i] + q], "J gen", i, pg);
        jcnt[pg]++;
        jcnt[pg + qoff]++;
      }
      // slack columns after the generators: the P-row blocks, then (at
      // +qoff) the Q-row blocks, each in block order
      for (int r = 0; r < 2; ++r) {
        int q = 0;
        for (int k = 0; k < T.sl.ns; ++k) {
          if (T.sl.row[k] != r) continue;
          const int ps = rw.x + 2 * a + g + q + (r ? qoff : 0);
          chk(jc[ps] == 2 * nb + 2 * T.ng + k * nb + i, "J slack", i, ps);
          chk(ps < jp[(r ? nb : 0) + i + 1], "J slack row", i, ps);
          jcnt[ps]++;
          ++q;
        }
        chk(q == T.sl.nsp, "slacks per row", i, q);
      }
      chk(hc[rw.z + blw] == i && hc[rw.w + blw] == i && hc[rw.w + a + blw] == nb + i, "H diag", i, rw.z);
      hcnt[rw.z + blw]++;
      hcnt[rw.w + blw]++;
      hcnt[rw.w + a + blw]++;
    }
  }
  for (int p = 0; p < T.jflow; ++p) chk(jcnt[p] == 1, "J coverage", p, jcnt[p]);
  for (int p = 0; p < T.hpg; ++p) chk(hcnt[p] == 1, "H coverage", p, hcnt[p]);
  {
    int next = 0;
    for (int ti = S.counts[0]; ti < S.counts[0] + S.counts[1]; ++ti) {
      const Tile& tl = S.tiles[ti];
      const bool slack = ti - S.counts[0] >= T.gchunks;
      chk(tl.a0 == next && tl.a1 - tl.a0 <= kGenChunk * (slack ? kSlackPerSlot : kGenPerSlot),
          "gen tile items", tl.a0, tl.a1);
      chk(slack ? tl.a0 >= T.ng : tl.a1 <= T.ng, "gen tile kind", tl.a0, tl.a1);
      chk((tl.kind_aux >> 2) == ti - S.counts[0], "gen tile chunk", ti, tl.kind_aux);
      next = tl.a1;
    }
    chk(next == T.ng + T.sl.ns * nb, "gen tiles end", next, T.ng + T.sl.ns * nb);
    chk(S.counts[1] == T.nchunks, "gen tile count", S.counts[1], T.nchunks);
  }
  if (bad) {
    printf("tile_be %d: %d tiles, %zu work items, %d failures\n", tile_be, S.counts[0],
           S.work.size(), bad);
    fflush(stdout);
  }
  return bad ? 3 : 0;
}
// The host code references the kernel launchers; this check never launches.
namespace acopf {
hipError_t launch_eval(unsigned, int, const Bufs&, const InstOff*, const InstOff&, const Tile*,
                       int, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fsum(const InstOff*, const InstOff&, int, int, const double*, double*,
                       hipStream_t) {
  return hipErrorInvalidValue;
}
}  // namespace acopf
