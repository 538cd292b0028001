// Host side of the C ABI: network validation, branch admittances, bus
// adjacency, CSR patterns, tiling, device residency and the single-instance
// evaluation entry points.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "acopf.h"
#include "acopf_host.h"

namespace acopf {

thread_local std::string t_err;

int fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(ACOPF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// validation and host-side derivation

static bool finite(double v) { return std::isfinite(v); }

// Representation and slack blocks of the options (nullptr: polar, none).
static int apply_opts(const acopf_net_opts* o, Topology* T) {
  T->form = ACOPF_POLAR;
  T->sl = SlackDev{};
  if (!o) return ACOPF_OK;
  if (o->form != ACOPF_POLAR && o->form != ACOPF_CARTESIAN)
    return fail(ACOPF_EINVAL, "form must be ACOPF_POLAR or ACOPF_CARTESIAN");
  if (o->slacks & ~unsigned(ACOPF_SLACK_IMBALANCE | ACOPF_SLACK_LOADLOSS))
    return fail(ACOPF_EINVAL, "unknown bits in slacks");
  if (!finite(o->imb_c2) || !finite(o->imb_c1) || !finite(o->loss_c2) || !finite(o->loss_c1))
    return fail(ACOPF_EINVAL, "non-finite slack penalty");
  T->form = o->form;
  SlackDev& s = T->sl;
  auto add = [&](int row, double coef, double c2, double c1) {
    s.row[s.ns] = row;
    s.coef[s.ns] = coef;
    s.c2[s.ns] = c2;
    s.c1[s.ns] = c1;
    ++s.ns;
  };
  if (o->slacks & ACOPF_SLACK_IMBALANCE) {
    add(0, -1.0, o->imb_c2, o->imb_c1);  // dP+: supplies power
    add(0, 1.0, o->imb_c2, o->imb_c1);   // dP-: absorbs it
    add(1, -1.0, o->imb_c2, o->imb_c1);  // dQ+
    add(1, 1.0, o->imb_c2, o->imb_c1);   // dQ-
  }
  if (o->slacks & ACOPF_SLACK_LOADLOSS) {
    add(0, -1.0, o->loss_c2, o->loss_c1);  // Pl: shed active load
    add(1, -1.0, o->loss_c2, o->loss_c1);  // Ql
  }
  s.nsp = s.ns / 2;
  return ACOPF_OK;
}

int build_topology(const acopf_net_desc* d, const acopf_net_opts* o, Topology* T) {
  if (!d) return fail(ACOPF_EINVAL, "null network description");
  {
    const int rc = apply_opts(o, T);
    if (rc) return rc;
  }
  if (d->nbus < 1) return fail(ACOPF_EINVAL, "nbus must be >= 1");
  if (d->nbranch < 0 || d->ngen < 0) return fail(ACOPF_EINVAL, "negative nbranch or ngen");
  if (!(d->base_mva > 0.0) || !finite(d->base_mva)) return fail(ACOPF_EINVAL, "base_mva must be > 0");
  const int nb = d->nbus, nl = d->nbranch, ng = d->ngen;
  if (nl > 0 && (!d->br_from || !d->br_to || !d->br_r || !d->br_x || !d->br_b || !d->br_tap ||
                 !d->br_shift || !d->br_rate))
    return fail(ACOPF_EINVAL, "null branch array");
  if (!d->bus_pd || !d->bus_qd || !d->bus_gs || !d->bus_bs) return fail(ACOPF_EINVAL, "null bus array");
  if (ng > 0 && (!d->gen_bus || !d->gen_c2 || !d->gen_c1 || !d->gen_c0))
    return fail(ACOPF_EINVAL, "null generator array");
  if (int64_t(nl) > (INT_MAX >> 2)) return fail(ACOPF_EINVAL, "too many branches");

  T->nb = nb;
  T->nl = nl;
  T->ng = ng;
  T->base = d->base_mva;
  T->ft.resize(nl);
  T->y.resize(nl);
  T->rate.resize(nl);
  for (int l = 0; l < nl; ++l) {
    const int f = d->br_from[l], t = d->br_to[l];
    if (f < 0 || f >= nb || t < 0 || t >= nb)
      return fail(ACOPF_EINVAL, "branch " + std::to_string(l) + ": bus id out of range");
    if (f == t) return fail(ACOPF_EINVAL, "branch " + std::to_string(l) + ": from == to");
    const double r = d->br_r[l], x = d->br_x[l], b = d->br_b[l];
    const double tap = d->br_tap[l], sh = d->br_shift[l];
    if (!finite(r) || !finite(x) || !finite(b) || !finite(tap) || !finite(sh) ||
        !finite(d->br_rate[l]))
      return fail(ACOPF_EINVAL, "branch " + std::to_string(l) + ": non-finite parameter");
    T->rate[l] = d->br_rate[l];
    if (r == 0.0 && x == 0.0)
      return fail(ACOPF_EINVAL, "branch " + std::to_string(l) + ": zero impedance");
    if (!(tap > 0.0)) return fail(ACOPF_EINVAL, "branch " + std::to_string(l) + ": tap must be > 0");
    // y_s = 1/(r + j x); N = tap e^{j shift}
    const double den = r * r + x * x;
    const double gs = r / den, bs = -x / den;
    const double cs = std::cos(sh), sn = std::sin(sh);
    BranchY& Y = T->y[l];
    Y.gff = gs / (tap * tap);
    Y.bff = (bs + 0.5 * b) / (tap * tap);
    // Y_ft = -y_s / conj(N) = -y_s e^{j shift} / tap
    Y.gft = -(gs * cs - bs * sn) / tap;
    Y.bft = -(gs * sn + bs * cs) / tap;
    // Y_tf = -y_s / N = -y_s e^{-j shift} / tap
    Y.gtf = -(gs * cs + bs * sn) / tap;
    Y.btf = -(bs * cs - gs * sn) / tap;
    Y.gtt = gs;
    Y.btt = bs + 0.5 * b;
    T->ft[l] = make_int2(f, t);
  }
  T->y6.resize(nl);
  T->tf.resize(nl);
  T->shifted.resize(nl);
  for (int l = 0; l < nl; ++l) {
    const BranchY& Y = T->y[l];
    T->y6[l] = BranchY6{Y.gff, Y.bff, Y.gft, Y.bft, Y.gtt, Y.btt};
    T->tf[l] = make_double2(Y.gtf, Y.btf);
    T->shifted[l] = (std::memcmp(&Y.gtf, &Y.gft, sizeof(double)) != 0 ||
                     std::memcmp(&Y.btf, &Y.bft, sizeof(double)) != 0) ? 1 : 0;
  }
  T->bus.resize(nb);
  for (int i = 0; i < nb; ++i) {
    const double v[4] = {d->bus_pd[i], d->bus_qd[i], d->bus_gs[i], d->bus_bs[i]};
    for (double z : v)
      if (!finite(z)) return fail(ACOPF_EINVAL, "bus " + std::to_string(i) + ": non-finite value");
    T->bus[i] = make_double4(v[0], v[1], v[2], v[3]);
  }
  T->gen_bus.resize(ng);
  T->c2.resize(ng);
  T->c1.resize(ng);
  T->c0.resize(ng);
  for (int k = 0; k < ng; ++k) {
    const int b = d->gen_bus[k];
    if (b < 0 || b >= nb) return fail(ACOPF_EINVAL, "generator " + std::to_string(k) + ": bus out of range");
    if (!finite(d->gen_c2[k]) || !finite(d->gen_c1[k]) || !finite(d->gen_c0[k]))
      return fail(ACOPF_EINVAL, "generator " + std::to_string(k) + ": non-finite cost");
    T->gen_bus[k] = b;
    T->c2[k] = d->gen_c2[k];
    T->c1[k] = d->gen_c1[k];
    T->c0[k] = d->gen_c0[k];
  }

  // branch ends sorted by (bus, other end, branch)
  std::vector<int32_t> cnt(nb + 1, 0);
  for (int l = 0; l < nl; ++l) {
    cnt[T->ft[l].x + 1]++;
    cnt[T->ft[l].y + 1]++;
  }
  T->be_ptr.assign(nb + 1, 0);
  for (int i = 0; i < nb; ++i) T->be_ptr[i + 1] = T->be_ptr[i] + cnt[i + 1];
  T->be.assign(2 * size_t(nl), 0);
  std::vector<int32_t> fill(T->be_ptr.begin(), T->be_ptr.end() - 1);
  for (int l = 0; l < nl; ++l) {
    T->be[fill[T->ft[l].x]++] = (l << 1);
    T->be[fill[T->ft[l].y]++] = (l << 1) | 1;
  }
  auto other = [&](int32_t code) {
    const int2 ft = T->ft[code >> 1];
    return (code & 1) ? ft.x : ft.y;
  };
  for (int i = 0; i < nb; ++i) {
    std::sort(T->be.begin() + T->be_ptr[i], T->be.begin() + T->be_ptr[i + 1],
              [&](int32_t a, int32_t b) {
                const int oa = other(a), ob = other(b);
                return oa != ob ? oa < ob : (a >> 1) < (b >> 1);
              });
  }
  // generators grouped by bus, index order within a bus
  T->gen_ptr.assign(nb + 1, 0);
  for (int k = 0; k < ng; ++k) T->gen_ptr[T->gen_bus[k] + 1]++;
  for (int i = 0; i < nb; ++i) T->gen_ptr[i + 1] += T->gen_ptr[i];
  T->gen_list.assign(ng, 0);
  {
    std::vector<int32_t> gf(T->gen_ptr.begin(), T->gen_ptr.end() - 1);
    for (int k = 0; k < ng; ++k) T->gen_list[gf[T->gen_bus[k]]++] = k;
  }
  // per-bus neighbour counts and base row starts
  T->acnt.resize(nb);
  T->rows.resize(nb + 1);
  int64_t jp = 0, ht = 0, hvsum = 0;
  std::vector<int64_t> jpv(nb + 1), htv(nb + 1), hvv(nb + 1);
  for (int i = 0; i < nb; ++i) {
    int distinct = 0, below = 0, prev = -1;
    for (int e = T->be_ptr[i]; e < T->be_ptr[i + 1]; ++e) {
      const int j = other(T->be[e]);
      if (j != prev) {
        ++distinct;
        if (j < i) ++below;
        prev = j;
      }
    }
    const int a = distinct + 1, g = T->gen_ptr[i + 1] - T->gen_ptr[i];
    T->acnt[i] = make_int2(a, below);
    jpv[i] = jp;
    htv[i] = ht;
    hvv[i] = hvsum;
    jp += 2 * a + g + T->sl.nsp;
    ht += below + 1;
    hvsum += a + below + 1;
  }
  jpv[nb] = jp;
  htv[nb] = ht;
  hvv[nb] = hvsum;
  const int64_t nslk = int64_t(T->sl.ns) * nb;
  const int64_t jflow = 2 * jp, nnzj = jflow + 8 * int64_t(nl);
  const int64_t hpg = ht + hvsum, nnzh = hpg + ng + nslk;
  if (nnzj + (T->form == ACOPF_CARTESIAN ? 2 * int64_t(nb) : 0) >= INT_MAX || nnzh >= INT_MAX ||
      2 * int64_t(nb) + 2 * int64_t(ng) + nslk >= INT_MAX)
    return fail(ACOPF_EINVAL, "pattern exceeds 2^31 entries");
  for (int i = 0; i <= nb; ++i)
    T->rows[i] = make_int4(int(jpv[i]), int(jp + jpv[i]), int(htv[i]), int(ht + hvv[i]));
  T->jflow = int(jflow);
  T->hpg = int(hpg);
  T->nnz_jac = nnzj;
  T->nnz_hess = nnzh;
  T->gchunks = int((ng + kGenChunk * kGenPerSlot - 1) / (kGenChunk * kGenPerSlot));
  constexpr int64_t kSlackChunk = int64_t(kGenChunk) * kSlackPerSlot;
  T->nchunks = std::max(1, T->gchunks + int((nslk + kSlackChunk - 1) / kSlackChunk));
  return ACOPF_OK;
}

int outage_info(const Topology& T, int32_t l, int32_t* p, int32_t* q, int32_t* rm) {
  if (l < 0 || l >= T.nl) return fail(ACOPF_EINVAL, "outage branch out of range");
  const int a = std::min(T.ft[l].x, T.ft[l].y), b = std::max(T.ft[l].x, T.ft[l].y);
  int others = 0;
  for (int e = T.be_ptr[a]; e < T.be_ptr[a + 1]; ++e) {
    const int code = T.be[e];
    const int2 ft = T.ft[code >> 1];
    const int o = (code & 1) ? ft.x : ft.y;
    if (o == b && (code >> 1) != l) ++others;
  }
  *p = a;
  *q = b;
  *rm = others == 0 ? 1 : 0;
  return ACOPF_OK;
}

void fill_dims(const Topology& T, int32_t outage, int32_t rm, acopf_dims* d) {
  const int live = T.nl - (outage >= 0 ? 1 : 0);
  const bool cart = T.form == ACOPF_CARTESIAN;
  d->n = 2 * int64_t(T.nb) + 2 * int64_t(T.ng) + int64_t(T.sl.ns) * T.nb;
  d->m = 2 * int64_t(T.nb) + 2 * int64_t(live) + (cart ? T.nb : 0);
  d->m_eq = 2 * int64_t(T.nb);
  d->nnz_jac = T.nnz_jac - (outage >= 0 ? 8 + 8 * rm : 0) + (cart ? 2 * int64_t(T.nb) : 0);
  d->nnz_hess = T.nnz_hess - (outage >= 0 ? 4 * rm : 0);
  d->nbus = T.nb;
  d->nbranch = live;
  d->ngen = T.ng;
  d->outage = outage;
}

// h+ of the live branches' flow rows: from ends, then to ends.
void flow_limits(const Topology& T, int32_t outage, double* hmax) {
  const int live = T.nl - (outage >= 0 ? 1 : 0);
  int r = 0;
  for (int l = 0; l < T.nl; ++l) {
    if (l == outage) continue;
    const double a = T.rate[l];
    hmax[r] = hmax[r + live] = a > 0.0 ? a * a : HUGE_VAL;
    ++r;
  }
}

// The structural pattern rule, applied to the live branches.
void build_pattern(const Topology& T, int32_t outage, std::vector<int32_t>* jp,
                   std::vector<int32_t>* jc, std::vector<int32_t>* hp, std::vector<int32_t>* hc) {
  const int nb = T.nb, ng = T.ng, nl = T.nl;
  std::vector<std::vector<int32_t>> S(nb);
  for (int i = 0; i < nb; ++i) {
    std::vector<int32_t>& s = S[i];
    bool self = false;
    for (int e = T.be_ptr[i]; e < T.be_ptr[i + 1]; ++e) {
      const int code = T.be[e];
      if ((code >> 1) == outage) continue;
      const int2 ft = T.ft[code >> 1];
      const int j = (code & 1) ? ft.x : ft.y;
      if (!self && j > i) {
        s.push_back(i);
        self = true;
      }
      if (s.empty() || s.back() != j) s.push_back(j);
    }
    if (!self) s.push_back(i);
  }
  jp->assign(1, 0);
  jc->clear();
  for (int blk = 0; blk < 2; ++blk) {
    for (int i = 0; i < nb; ++i) {
      for (int j : S[i]) jc->push_back(j);
      for (int j : S[i]) jc->push_back(nb + j);
      for (int g = T.gen_ptr[i]; g < T.gen_ptr[i + 1]; ++g)
        jc->push_back(2 * nb + (blk ? ng : 0) + T.gen_list[g]);
      for (int k = 0; k < T.sl.ns; ++k)  // slack columns of this row, blocks in order
        if (T.sl.row[k] == blk) jc->push_back(2 * nb + 2 * ng + k * nb + i);
      jp->push_back(int32_t(jc->size()));
    }
  }
  for (int blk = 0; blk < 2; ++blk) {
    for (int l = 0; l < nl; ++l) {
      if (l == outage) continue;
      const int a = std::min(T.ft[l].x, T.ft[l].y), b = std::max(T.ft[l].x, T.ft[l].y);
      jc->push_back(a);
      jc->push_back(b);
      jc->push_back(nb + a);
      jc->push_back(nb + b);
      jp->push_back(int32_t(jc->size()));
    }
  }
  if (T.form == ACOPF_CARTESIAN) {  // magnitude rows e_i^2 + f_i^2: columns e_i, f_i
    for (int i = 0; i < nb; ++i) {
      jc->push_back(i);
      jc->push_back(nb + i);
      jp->push_back(int32_t(jc->size()));
    }
  }
  hp->assign(1, 0);
  hc->clear();
  for (int i = 0; i < nb; ++i) {
    for (int j : S[i])
      if (j <= i) hc->push_back(j);
    hp->push_back(int32_t(hc->size()));
  }
  for (int i = 0; i < nb; ++i) {
    for (int j : S[i]) hc->push_back(j);
    for (int j : S[i])
      if (j <= i) hc->push_back(nb + j);
    hp->push_back(int32_t(hc->size()));
  }
  for (int k = 0; k < ng; ++k) {
    hc->push_back(2 * nb + k);
    hp->push_back(int32_t(hc->size()));
  }
  for (int k = 0; k < ng; ++k) hp->push_back(int32_t(hc->size()));
  for (int q = 0; q < T.sl.ns * nb; ++q) {  // slack rows: the diagonal
    hc->push_back(2 * nb + 2 * ng + q);
    hp->push_back(int32_t(hc->size()));
  }
}

// Position of bus j in the ascending set {i} u N(i).
static int rank_in(const Topology& T, int i, int j) {
  int r = (i < j) ? 1 : 0, prev = -1;
  for (int e = T.be_ptr[i]; e < T.be_ptr[i + 1]; ++e) {
    const int code = T.be[e];
    const int2 ft = T.ft[code >> 1];
    const int o = (code & 1) ? ft.x : ft.y;
    if (o != prev) {
      if (o < j) ++r;
      prev = o;
    }
  }
  return r;
}

int make_tiles(const Topology& T, int tile_be, Schedule* S) {
  TileCaps caps;
  if (!caps_for(tile_be, &caps)) return fail(ACOPF_EINVAL, "unsupported tile size");
  S->tiles.clear();
  S->work.clear();
  // adjacency position of each branch end
  std::vector<int32_t> pos_from(T.nl), pos_to(T.nl);
  for (int e = 0; e < int(T.be.size()); ++e) {
    const int code = T.be[e];
    ((code & 1) ? pos_to : pos_from)[code >> 1] = e;
  }
  // parallel-branch groups: every branch points at the smallest branch id
  // joining the same bus pair
  std::vector<int32_t> lead(T.nl);
  for (int i = 0; i < T.nb; ++i) {
    int prev = -1, first = -1;
    for (int e = T.be_ptr[i]; e < T.be_ptr[i + 1]; ++e) {
      const int code = T.be[e], l = code >> 1;
      const int2 ft = T.ft[l];
      const int o = (code & 1) ? ft.x : ft.y;
      if (o != prev) {
        prev = o;
        first = l;  // ends of one far bus are sorted by branch id
      }
      lead[l] = first;
    }
  }
  std::vector<int32_t> gsize(T.nl, 0);
  for (int l = 0; l < T.nl; ++l) gsize[lead[l]]++;
  for (int l = 0; l < T.nl; ++l)
    if (gsize[lead[l]] > kMaxGroup)
      return fail(ACOPF_EINVAL, "more than " + std::to_string(kMaxGroup) +
                                    " parallel branches join one bus pair");
  std::vector<int32_t> seen(T.nl, -1);
  std::vector<int32_t> items;
  bool tiler_error = false;
  auto close = [&](int b0, int b1) {
    const int e0 = T.be_ptr[b0], e1 = T.be_ptr[b1];
    const int4 r0 = T.rows[b0], r1 = T.rows[b1];
    items.clear();
    for (int e = e0; e < e1; ++e) {
      const int l = T.be[e] >> 1;
      if (seen[l] != b0) {
        seen[l] = b0;
        items.push_back(l);
      }
    }
    // groups together, in branch order, leaders first
    std::sort(items.begin(), items.end(), [&](int a, int b) {
      return lead[a] != lead[b] ? lead[a] < lead[b] : a < b;
    });
    const int w0 = int(S->work.size());
    int gmax = 1;
    auto in_tile = [&](int bus) { return bus >= b0 && bus < b1; };
    for (size_t k = 0; k < items.size();) {
      size_t k1 = k + 1;
      while (k1 < items.size() && lead[items[k1]] == lead[items[k]]) ++k1;
      const int g = int(k1 - k);
      gmax = std::max(gmax, g);
      // no group straddles two waves
      const int at = int(S->work.size()) - w0;
      if (g > 1 && at / 64 != (at + g - 1) / 64) {
        const int pad = 64 - at % 64;
        for (int q = 0; q < pad; ++q) {
          WorkItem d{};
          d.l = -2;
          d.j = d.hv = kNoPos | (kNoPos << 16);
          d.th = kNoPos;
          d.slots = kNoSlot | (kNoSlot << 16);
          S->work.push_back(d);
        }
      }
      for (size_t m = k; m < k1; ++m) {
        const int l = items[m];
        const int f = T.ft[l].x, t = T.ft[l].y;
        const int lo = std::min(f, t), hi = std::max(f, t);
        WorkItem w{};
        w.l = l;
        w.f = f;
        w.t = t;
        const uint32_t sf = in_tile(f) ? uint32_t(pos_from[l] - e0) : kNoSlot;
        const uint32_t st = in_tile(t) ? uint32_t(pos_to[l] - e0) : kNoSlot;
        w.slots = sf | (st << 16);
        // positions relative to the tile's segments (J P rows from r0.x,
        // H theta rows from r0.z, H v rows from r0.w)
        uint32_t jlo = kNoPos, hvlo = kNoPos, jhi = kNoPos, hvhi = kNoPos, hthi = kNoPos;
        if (in_tile(lo)) {
          const int r = rank_in(T, lo, hi);
          jlo = uint32_t(T.rows[lo].x + r - r0.x);
          hvlo = uint32_t(T.rows[lo].w + r - r0.w);
        }
        if (in_tile(hi)) {
          const int r = rank_in(T, hi, lo);
          jhi = uint32_t(T.rows[hi].x + r - r0.x);
          hvhi = uint32_t(T.rows[hi].w + r - r0.w);
          hthi = uint32_t(T.rows[hi].z + r - r0.z);
        }
        w.j = jlo | (jhi << 16);
        w.hv = hvlo | (hvhi << 16);
        w.th = hthi | (uint32_t((m == k) ? g : 0) << 16) | (uint32_t(T.shifted[l]) << 24);
        w.a = uint32_t(T.acnt[lo].x) | (uint32_t(T.acnt[hi].x) << 16);
        S->work.push_back(w);
      }
      k = k1;
    }
    // every stored position must lie in the tile's row segments
    // the J segments and the H segments are staged one after the other
    bool ok = e1 - e0 <= caps.be && b1 - b0 <= caps.nbus && 2 * (r1.x - r0.x) <= caps.stage &&
              (r1.z - r0.z) + (r1.w - r0.w) <= caps.stage;
    // (and fit the 16-bit relative encoding)
    ok = ok && r1.x - r0.x < int(kNoPos) && r1.z - r0.z < int(kNoPos) && r1.w - r0.w < int(kNoPos);
    for (size_t k = w0; ok && k < S->work.size(); ++k) {
      const WorkItem& w = S->work[k];
      if (w.l < 0) continue;
      if (w.jlo() != kNoPos)
        ok = ok && int(w.jlo() + w.alo()) < r1.x - r0.x && int(w.hvlo()) < r1.w - r0.w;
      if (w.jhi() != kNoPos)
        ok = ok && int(w.jhi() + w.ahi()) < r1.x - r0.x && int(w.hvhi() + w.ahi()) < r1.w - r0.w &&
             int(w.hthi()) < r1.z - r0.z;
    }
    if (!ok) {
      tiler_error = true;
      return;
    }
    Tile tl{};
    tl.inst = 0;
    tl.kind_aux = TILE_BUS;
    tl.a0 = b0;
    tl.a1 = b1;
    tl.e0 = e0;
    tl.ne = e1 - e0;
    tl.w0 = w0;
    tl.nw = int(S->work.size()) - w0;
    tl.gmax = gmax;
    tl.nP = r1.x - r0.x;
    tl.nT = r1.z - r0.z;
    tl.nV = r1.w - r0.w;
    tl.jP0 = r0.x;
    tl.jQ0 = r0.y;
    tl.hT0 = r0.z;
    tl.hV0 = r0.w;
    S->tiles.push_back(tl);
  };
  // staged entries of a bus: its J P and Q rows, then (in the same space,
  // after the J rows are stored) its H theta and v rows
  int b0 = 0, cur_be = 0, cur_j = 0, cur_h = 0;
  for (int i = 0; i < T.nb; ++i) {
    const int d = T.be_ptr[i + 1] - T.be_ptr[i];
    const int a = T.acnt[i].x, lo = T.acnt[i].y, g = T.gen_ptr[i + 1] - T.gen_ptr[i];
    const int sj = 2 * (2 * a + g + T.sl.nsp), sh = (lo + 1) + (a + lo + 1);
    if (d > caps.be || sj > caps.stage || sh > caps.stage)
      return fail(ACOPF_EINVAL, "bus " + std::to_string(i) + " has " + std::to_string(d) +
                                    " branch ends and " + std::to_string(std::max(sj, sh)) +
                                    " row entries; a bus tile of this schedule holds at most " +
                                    std::to_string(caps.be) + " and " +
                                    std::to_string(caps.stage));
    if (i > b0 && (cur_be + d > caps.be || cur_j + sj > caps.stage || cur_h + sh > caps.stage ||
                   i - b0 >= caps.nbus)) {
      close(b0, i);
      b0 = i;
      cur_be = 0;
      cur_j = 0;
      cur_h = 0;
    }
    cur_be += d;
    cur_j += sj;
    cur_h += sh;
  }
  close(b0, T.nb);
  if (tiler_error) return fail(ACOPF_EINVAL, "internal: work item positions outside the tile");
  S->counts[0] = int(S->tiles.size());
  // generator chunks of kGenChunk * kGenPerSlot items, then slack chunks of
  // kGenChunk * kSlackPerSlot items (item k >= ng is slack variable k - ng)
  const int nitems = T.ng + T.sl.ns * T.nb;
  for (int c = 0; c < T.nchunks; ++c) {
    Tile tl{};
    tl.kind_aux = (c << 2) | TILE_GEN;
    if (c < T.gchunks) {
      tl.a0 = c * kGenChunk * kGenPerSlot;
      tl.a1 = std::min(T.ng, (c + 1) * kGenChunk * kGenPerSlot);
    } else {
      const int span = kGenChunk * kSlackPerSlot;
      tl.a0 = std::min(nitems, T.ng + (c - T.gchunks) * span);
      tl.a1 = std::min(nitems, tl.a0 + span);
    }
    S->tiles.push_back(tl);
  }
  S->counts[1] = int(S->tiles.size()) - S->counts[0];
  return ACOPF_OK;
}

// Base positions of the 8 Jacobian and 4 Hessian slots an outage of a
// branch without a parallel twin removes (ascending), or INT32_MAX.
void removed_slots(const Topology& T, int32_t p, int32_t q, int32_t rm, int32_t rj[8],
                   int32_t rh[4]) {
  for (int k = 0; k < 8; ++k) rj[k] = INT_MAX;
  for (int k = 0; k < 4; ++k) rh[k] = INT_MAX;
  if (!rm) return;
  const int rpq = rank_in(T, p, q), rqp = rank_in(T, q, p);
  const int ap = T.acnt[p].x, aq = T.acnt[q].x;
  const int4 Rp = T.rows[p], Rq = T.rows[q];
  int32_t j[8] = {Rp.x + rpq, Rp.x + ap + rpq, Rq.x + rqp, Rq.x + aq + rqp,
                  Rp.y + rpq, Rp.y + ap + rpq, Rq.y + rqp, Rq.y + aq + rqp};
  int32_t h[4] = {Rq.z + rqp, Rp.w + rpq, Rq.w + rqp, Rq.w + aq + rqp};
  std::sort(j, j + 8);
  std::sort(h, h + 4);
  for (int k = 0; k < 8; ++k) rj[k] = j[k];
  for (int k = 0; k < 4; ++k) rh[k] = h[k];
}

// ---------------------------------------------------------------------------
// device residency

static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

Base::~Base() {
  if (mem) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    (void)hipFree(mem);
    (void)hipSetDevice(cur);
  }
}

int upload_base(Base* B) {
  const Topology& T = B->topo;
  int rc = make_tiles(T, kDefaultTileBe, &B->plain);
  if (rc) return rc;
  struct Part {
    const void* src;
    size_t bytes;
    size_t off;
  };
  std::vector<Part> parts = {
      {T.y6.data(), T.y6.size() * sizeof(BranchY6), 0},
      {T.bus.data(), T.bus.size() * sizeof(double4), 0},
      {T.be_ptr.data(), T.be_ptr.size() * sizeof(int32_t), 0},
      {T.gen_ptr.data(), T.gen_ptr.size() * sizeof(int32_t), 0},
      {T.gen_list.data(), T.gen_list.size() * sizeof(int32_t), 0},
      {T.gen_bus.data(), T.gen_bus.size() * sizeof(int32_t), 0},
      {T.c2.data(), T.c2.size() * sizeof(double), 0},
      {T.c1.data(), T.c1.size() * sizeof(double), 0},
      {T.c0.data(), T.c0.size() * sizeof(double), 0},
      {B->plain.tiles.data(), B->plain.tiles.size() * sizeof(Tile), 0},
      {B->plain.work.data(), B->plain.work.size() * sizeof(WorkItem), 0},
      {T.rows.data(), T.rows.size() * sizeof(int4), 0},
      {T.acnt.data(), T.acnt.size() * sizeof(int2), 0},
      {T.tf.data(), T.tf.size() * sizeof(double2), 0},
      {nullptr, sizeof(NetDev), 0},
  };
  size_t total = 0;
  for (Part& p : parts) {
    p.off = total;
    total += align_up(std::max<size_t>(p.bytes, 1));
  }
  hipError_t e = hipGetDevice(&B->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  void* mem = nullptr;
  e = hipMalloc(&mem, total);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? ACOPF_ENOMEM : ACOPF_EHIP,
                std::string("hipMalloc of network data: ") + hipGetErrorString(e));
  }
  B->mem = mem;
  B->bytes = total;
  char* base = static_cast<char*>(mem);
  auto at = [&](int k) { return static_cast<void*>(base + parts[k].off); };
  NetDev nd{};
  nd.nb = T.nb;
  nd.nl = T.nl;
  nd.ng = T.ng;
  nd.nchunks = T.nchunks;
  nd.br_y = static_cast<const BranchY6*>(at(0));
  nd.br_tf = static_cast<const double2*>(at(13));
  nd.bus = static_cast<const double4*>(at(1));
  nd.be_ptr = static_cast<const int32_t*>(at(2));
  nd.gen_ptr = static_cast<const int32_t*>(at(3));
  nd.gen_list = static_cast<const int32_t*>(at(4));
  nd.gen_bus = static_cast<const int32_t*>(at(5));
  nd.gen_c2 = static_cast<const double*>(at(6));
  nd.gen_c1 = static_cast<const double*>(at(7));
  nd.gen_c0 = static_cast<const double*>(at(8));
  nd.rows = static_cast<const int4*>(at(11));
  nd.acnt = static_cast<const int2*>(at(12));
  nd.base_mva = T.base;
  nd.jflow = T.jflow;
  nd.hpg = T.hpg;
  nd.qoff = T.rows[0].y - T.rows[0].x;
  nd.gen_ident = 1;
  for (int g = 0; g < T.ng; ++g)
    if (T.gen_list[g] != g) nd.gen_ident = 0;
  nd.sl = T.sl;
  B->d_tiles = static_cast<Tile*>(at(9));
  B->d_work = static_cast<WorkItem*>(at(10));
  B->d_net = static_cast<NetDev*>(at(14));
  parts[14].src = &nd;
  for (const Part& p : parts) {
    if (p.bytes == 0) continue;
    e = hipMemcpy(base + p.off, p.src, p.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of network data");
  }
  return ACOPF_OK;
}

}  // namespace acopf

using namespace acopf;

// ---------------------------------------------------------------------------
// C ABI: nets

extern "C" {

const char* acopf_last_error(void) { return t_err.c_str(); }

int acopf_version(void) { return 10400; }

static acopf_net_opts form_opts(int32_t form) {
  acopf_net_opts o{};
  o.form = form;
  return o;
}

int acopf_pattern_host(const acopf_net_desc* desc, int32_t outage, acopf_dims* dims,
                       int32_t* jac_rowptr, int32_t* jac_col, int32_t* hess_rowptr,
                       int32_t* hess_col) {
  return acopf_pattern_host_opts(desc, nullptr, outage, dims, jac_rowptr, jac_col, hess_rowptr,
                                 hess_col);
}

int acopf_flow_limits_host(const acopf_net_desc* desc, int32_t outage, double* hmax) {
  if (!hmax) return fail(ACOPF_EINVAL, "null hmax");
  try {
    Topology T;
    int rc = build_topology(desc, nullptr, &T);
    if (rc) return rc;
    if (outage < -1 || outage >= T.nl) return fail(ACOPF_EINVAL, "outage must be -1 or a branch index");
    flow_limits(T, outage, hmax);
    t_err.clear();
    return ACOPF_OK;
  } catch (const std::bad_alloc&) {
    return fail(ACOPF_ENOMEM, "host allocation failed");
  }
}

int acopf_flow_limits(acopf_net net, double* hmax) {
  if (!net || !hmax) return fail(ACOPF_EINVAL, "null net or hmax");
  flow_limits(net->base->topo, net->out_l, hmax);
  return ACOPF_OK;
}

int acopf_pattern_host_form(const acopf_net_desc* desc, int32_t form, int32_t outage,
                            acopf_dims* dims, int32_t* jac_rowptr, int32_t* jac_col,
                            int32_t* hess_rowptr, int32_t* hess_col) {
  const acopf_net_opts o = form_opts(form);
  return acopf_pattern_host_opts(desc, &o, outage, dims, jac_rowptr, jac_col, hess_rowptr,
                                 hess_col);
}

int acopf_pattern_host_opts(const acopf_net_desc* desc, const acopf_net_opts* opts,
                            int32_t outage, acopf_dims* dims, int32_t* jac_rowptr,
                            int32_t* jac_col, int32_t* hess_rowptr, int32_t* hess_col) {
  try {
    Topology T;
    int rc = build_topology(desc, opts, &T);
    if (rc) return rc;
    int32_t p = -1, q = -1, rm = 0;
    if (outage >= 0) {
      rc = outage_info(T, outage, &p, &q, &rm);
      if (rc) return rc;
    } else if (outage != -1) {
      return fail(ACOPF_EINVAL, "outage must be -1 or a branch index");
    }
    acopf_dims d;
    fill_dims(T, outage, rm, &d);
    if (dims) *dims = d;
    if (jac_rowptr || jac_col || hess_rowptr || hess_col) {
      std::vector<int32_t> jp, jc, hp, hc;
      build_pattern(T, outage, &jp, &jc, &hp, &hc);
      if (int64_t(jc.size()) != d.nnz_jac || int64_t(hc.size()) != d.nnz_hess)
        return fail(ACOPF_EINVAL, "internal: pattern size mismatch");
      if (jac_rowptr) std::memcpy(jac_rowptr, jp.data(), jp.size() * sizeof(int32_t));
      if (jac_col) std::memcpy(jac_col, jc.data(), jc.size() * sizeof(int32_t));
      if (hess_rowptr) std::memcpy(hess_rowptr, hp.data(), hp.size() * sizeof(int32_t));
      if (hess_col) std::memcpy(hess_col, hc.data(), hc.size() * sizeof(int32_t));
    }
    t_err.clear();
    return ACOPF_OK;
  } catch (const std::bad_alloc&) {
    return fail(ACOPF_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(ACOPF_EINVAL, "unexpected host error");
  }
}

int acopf_net_create(const acopf_net_desc* desc, acopf_net* out) {
  return acopf_net_create_opts(desc, nullptr, out);
}

int acopf_net_create_form(const acopf_net_desc* desc, int32_t form, acopf_net* out) {
  const acopf_net_opts o = form_opts(form);
  return acopf_net_create_opts(desc, &o, out);
}

int acopf_net_create_opts(const acopf_net_desc* desc, const acopf_net_opts* opts,
                          acopf_net* out) {
  if (!out) return fail(ACOPF_EINVAL, "null output handle");
  *out = nullptr;
  try {
    auto B = std::make_shared<Base>();
    int rc = build_topology(desc, opts, &B->topo);
    if (rc) return rc;
    rc = upload_base(B.get());
    if (rc) return rc;
    std::unique_ptr<acopf_net_s> net(new acopf_net_s());
    net->base = B;
    rc = net_init_scratch(net.get());
    if (rc) return rc;
    fill_dims(B->topo, -1, 0, &net->dims);
    *out = net.release();
    t_err.clear();
    return ACOPF_OK;
  } catch (const std::bad_alloc&) {
    return fail(ACOPF_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(ACOPF_EINVAL, "unexpected host error");
  }
}

int acopf_net_create_outage(acopf_net base, int32_t branch, acopf_net* out) {
  if (!base || !out) return fail(ACOPF_EINVAL, "null handle");
  *out = nullptr;
  if (base->parent) return fail(ACOPF_ESTATE, "an outage net cannot be the base of another");
  try {
    std::unique_ptr<acopf_net_s> net(new acopf_net_s());
    net->base = base->base;
    int rc = outage_info(base->base->topo, branch, &net->out_p, &net->out_q, &net->out_rm);
    if (rc) return rc;
    net->out_l = branch;
    removed_slots(base->base->topo, net->out_p, net->out_q, net->out_rm, net->rj, net->rh);
    net->parent = base;
    rc = net_init_scratch(net.get());
    if (rc) return rc;
    fill_dims(base->base->topo, branch, net->out_rm, &net->dims);
    base->refs.fetch_add(1);
    *out = net.release();
    t_err.clear();
    return ACOPF_OK;
  } catch (const std::bad_alloc&) {
    return fail(ACOPF_ENOMEM, "host allocation failed");
  }
}

int acopf_net_destroy(acopf_net net) {
  if (!net) return ACOPF_OK;
  if (net->refs.load() != 0)
    return fail(ACOPF_ESTATE, "net is still referenced by " + std::to_string(net->refs.load()) +
                                  " outage nets or batches");
  if (net->parent) net->parent->refs.fetch_sub(1);
  if (net->scratch) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(net->base->device);
    (void)hipFree(net->scratch);
    (void)hipSetDevice(cur);
  }
  delete net;
  return ACOPF_OK;
}

int acopf_dims_get(acopf_net net, acopf_dims* out) {
  if (!net || !out) return fail(ACOPF_EINVAL, "null argument");
  *out = net->dims;
  return ACOPF_OK;
}

int acopf_net_form(acopf_net net, int32_t* form) {
  if (!net || !form) return fail(ACOPF_EINVAL, "null argument");
  *form = net->base->topo.form;
  return ACOPF_OK;
}

int acopf_pattern(acopf_net net, int32_t* jac_rowptr, int32_t* jac_col, int32_t* hess_rowptr,
                  int32_t* hess_col) {
  if (!net) return fail(ACOPF_EINVAL, "null net");
  try {
    std::vector<int32_t> jp, jc, hp, hc;
    build_pattern(net->base->topo, net->out_l, &jp, &jc, &hp, &hc);
    if (jac_rowptr) std::memcpy(jac_rowptr, jp.data(), jp.size() * sizeof(int32_t));
    if (jac_col) std::memcpy(jac_col, jc.data(), jc.size() * sizeof(int32_t));
    if (hess_rowptr) std::memcpy(hess_rowptr, hp.data(), hp.size() * sizeof(int32_t));
    if (hess_col) std::memcpy(hess_col, hc.data(), hc.size() * sizeof(int32_t));
    return ACOPF_OK;
  } catch (const std::bad_alloc&) {
    return fail(ACOPF_ENOMEM, "host allocation failed");
  }
}

}  // extern "C"

namespace acopf {

int net_init_scratch(acopf_net_s* net) {
  const int nch = net->base->topo.nchunks;
  const size_t bytes = align_up(nch * sizeof(double));
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != net->base->device) return fail(ACOPF_EINVAL, "current device differs from the net's device");
  void* p = nullptr;
  e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ACOPF_ENOMEM, std::string("hipMalloc of scratch: ") + hipGetErrorString(e));
  }
  e = hipMemset(p, 0, bytes);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e, "hipMemset of scratch");
  }
  net->scratch = p;
  net->d_fpart = static_cast<double*>(p);
  return ACOPF_OK;
}

InstOff net_inst(const acopf_net_s* net) {
  InstOff I{};
  I.net = net->base->d_net;
  I.work = net->base->d_work;
  I.out_l = net->out_l;
  I.out_rm = net->out_rm;
  for (int k = 0; k < 8; ++k) I.rj[k] = net->rj[k];
  for (int k = 0; k < 4; ++k) I.rh[k] = net->rh[k];
  I.k = 0;
  I.fpo = 0;
  return I;
}

int check_device(const acopf_net_s* net) {
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != net->base->device)
    return fail(ACOPF_EINVAL, "net lives on device " + std::to_string(net->base->device) +
                                  ", current device is " + std::to_string(cur));
  return ACOPF_OK;
}

// Plain path: the net's own tile list [bus][gen], one workgroup per tile.
static int run_plain(const acopf_net_s* net, unsigned variant, Bufs b, bool bus, bool gen,
                     hipStream_t s) {
  int rc = check_device(net);
  if (rc) return rc;
  const Base& B = *net->base;
  b.fpart = net->d_fpart;
  const int nbu = B.plain.counts[0], ngt = B.plain.counts[1];
  if (!bus && !gen) return ACOPF_OK;
  const int t0 = bus ? 0 : nbu;
  const int t1 = gen ? nbu + ngt : nbu;
  const InstOff one = net_inst(net);
  if (B.topo.form == ACOPF_CARTESIAN) variant |= W_CART;
  hipError_t e = launch_eval(variant, kDefaultTileBe, b, nullptr, one, B.d_tiles + t0, t1 - t0, 0, s);
  if (e == hipSuccess && b.f && B.topo.nchunks > 1) e = launch_fsum(nullptr, one, 0, 1, b.fpart, b.f, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ACOPF_OK;
}

}  // namespace acopf

extern "C" {

int acopf_eval_f_g(acopf_net net, const double* x, double* f, double* grad_f, double* c,
                   hipStream_t stream) {
  if (!net || !x) return fail(ACOPF_EINVAL, "null net or x");
  Bufs b{};
  b.x = x;
  b.f = f;
  b.gradf = grad_f;
  b.c = c;
  return run_plain(net, K_FG, b, c != nullptr || grad_f != nullptr,
                   f != nullptr || grad_f != nullptr, stream);
}

int acopf_eval_jac(acopf_net net, const double* x, double* jac_val, hipStream_t stream) {
  if (!net || !x || !jac_val) return fail(ACOPF_EINVAL, "null net, x or jac_val");
  Bufs b{};
  b.x = x;
  b.jac = jac_val;
  return run_plain(net, K_J, b, true, false, stream);
}

int acopf_eval_hess(acopf_net net, const double* x, double sigma, const double* lambda,
                    double* hess_val, hipStream_t stream) {
  if (!net || !x || !lambda || !hess_val) return fail(ACOPF_EINVAL, "null net, x, lambda or hess_val");
  Bufs b{};
  b.x = x;
  b.lam = lambda;
  b.sigma_v = sigma;
  b.hess = hess_val;
  return run_plain(net, K_H, b, true, true, stream);
}

int acopf_vjp(acopf_net net, const double* x, double w_f, const double* w_c, double* u,
              hipStream_t stream) {
  if (!net || !x || !w_c || !u) return fail(ACOPF_EINVAL, "null net, x, w_c or u");
  Bufs b{};
  b.x = x;
  b.wc = w_c;
  b.wf_v = w_f;
  b.u = u;
  return run_plain(net, K_VJP, b, true, true, stream);
}

int acopf_hvp(acopf_net net, const double* x, double sigma, const double* lambda, const double* d,
              double* out, hipStream_t stream) {
  if (!net || !x || !lambda || !d || !out) return fail(ACOPF_EINVAL, "null argument");
  Bufs b{};
  b.x = x;
  b.lam = lambda;
  b.sigma_v = sigma;
  b.dir = d;
  b.out = out;
  return run_plain(net, K_HVP, b, true, true, stream);
}

int acopf_jvp(acopf_net net, const double* x, const double* d, double* out, hipStream_t stream) {
  if (!net || !x || !d || !out) return fail(ACOPF_EINVAL, "null argument");
  Bufs b{};
  b.x = x;
  b.dir = d;
  b.out = out;
  return run_plain(net, K_JVP, b, true, false, stream);
}

int acopf_eval_all(acopf_net net, const double* x, double sigma, const double* lambda, double* f,
                   double* grad_f, double* c, double* jac_val, double* hess_val, unsigned what,
                   hipStream_t stream) {
  if (!net || !x) return fail(ACOPF_EINVAL, "null net or x");
  if (what & ~unsigned(ACOPF_ALL)) return fail(ACOPF_EINVAL, "unknown bits in what");
  if (((what & ACOPF_F) && !f) || ((what & ACOPF_GRADF) && !grad_f) || ((what & ACOPF_C) && !c) ||
      ((what & ACOPF_J) && !jac_val) || ((what & ACOPF_H) && (!hess_val || !lambda)))
    return fail(ACOPF_EINVAL, "a selected output (or lambda for ACOPF_H) is null");
  Bufs b{};
  b.x = x;
  b.lam = lambda;
  b.sigma_v = sigma;
  b.f = (what & ACOPF_F) ? f : nullptr;
  b.gradf = (what & ACOPF_GRADF) ? grad_f : nullptr;
  b.c = (what & ACOPF_C) ? c : nullptr;
  b.jac = (what & ACOPF_J) ? jac_val : nullptr;
  b.hess = (what & ACOPF_H) ? hess_val : nullptr;
  if (!what) return ACOPF_OK;
  return run_plain(net, K_ALL, b, true, true, stream);
}

}  // extern "C"
