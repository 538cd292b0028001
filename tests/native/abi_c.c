/* A C (not C++) caller of the library: links libacopf.so through
 * include/acopf.h and checks, on the host only, the pattern of a 3-bus line
 * 0-1-2 with one generator at bus 0 against the pattern rule of the header,
 * written out by hand, plus one error path.  Compiled and run by
 * tests/test_abi_c.py.  Exit status 0 on success. */
#include <stdio.h>
#include <string.h>

#include "acopf.h"

static int same(const char* what, const int32_t* got, const int32_t* want, int n) {
  for (int i = 0; i < n; ++i)
    if (got[i] != want[i]) {
      printf("%s[%d] = %d, want %d\n", what, i, got[i], want[i]);
      return 0;
    }
  return 1;
}

int main(void) {
  const int32_t from[2] = {0, 1}, to[2] = {1, 2}, gen_bus[1] = {0};
  const double r[2] = {0.01, 0.02}, x[2] = {0.1, 0.2}, b[2] = {0.0, 0.05};
  const double tap[2] = {1.0, 1.0}, shift[2] = {0.0, 0.0}, rate[2] = {1.5, 0.0};
  const double pd[3] = {0.0, 0.5, 0.3}, qd[3] = {0.0, 0.1, 0.1};
  const double gs[3] = {0.0, 0.0, 0.0}, bs[3] = {0.0, 0.0, 0.0};
  const double c2[1] = {0.02}, c1[1] = {20.0}, c0[1] = {0.0};
  acopf_net_desc d;
  memset(&d, 0, sizeof d);
  d.nbus = 3;
  d.nbranch = 2;
  d.ngen = 1;
  d.base_mva = 100.0;
  d.br_from = from;
  d.br_to = to;
  d.br_r = r;
  d.br_x = x;
  d.br_b = b;
  d.br_tap = tap;
  d.br_shift = shift;
  d.br_rate = rate;
  d.bus_pd = pd;
  d.bus_qd = qd;
  d.bus_gs = gs;
  d.bus_bs = bs;
  d.gen_bus = gen_bus;
  d.gen_c2 = c2;
  d.gen_c1 = c1;
  d.gen_c0 = c0;

  if (acopf_version() < 10000) return 1;
  acopf_dims dims;
  if (acopf_pattern_host(&d, -1, &dims, NULL, NULL, NULL, NULL) != ACOPF_OK) {
    printf("pattern_host: %s\n", acopf_last_error());
    return 2;
  }
  /* x = [th0 th1 th2 v0 v1 v2 Pg0 Qg0]; c = [gP0..2 gQ0..2 hf0 hf1 ht0 ht1] */
  if (dims.n != 8 || dims.m != 10 || dims.m_eq != 6 || dims.nnz_jac != 46 ||
      dims.nnz_hess != 18 || dims.nbus != 3 || dims.nbranch != 2 || dims.ngen != 1 ||
      dims.outage != -1) {
    printf("dims n=%lld m=%lld m_eq=%lld nnz_jac=%lld nnz_hess=%lld\n", (long long)dims.n,
           (long long)dims.m, (long long)dims.m_eq, (long long)dims.nnz_jac,
           (long long)dims.nnz_hess);
    return 3;
  }
  /* h+ = rate^2 per flow row (from ends, then to ends); rate 0 is unlimited */
  double hmax[4];
  if (acopf_flow_limits_host(&d, -1, hmax) != ACOPF_OK) return 10;
  if (hmax[0] != 2.25 || hmax[2] != 2.25 || !(hmax[1] > 1e308) || !(hmax[3] > 1e308)) {
    printf("hmax %g %g %g %g\n", hmax[0], hmax[1], hmax[2], hmax[3]);
    return 11;
  }
  if (acopf_flow_limits_host(&d, 1, hmax) != ACOPF_OK || hmax[0] != 2.25 || hmax[1] != 2.25)
    return 12;
  int32_t jp[11], jc[46], hp[9], hc[18];
  if (acopf_pattern_host(&d, -1, NULL, jp, jc, hp, hc) != ACOPF_OK) return 4;
  const int32_t want_jp[11] = {0, 5, 11, 15, 20, 26, 30, 34, 38, 42, 46};
  const int32_t want_jc[46] = {0, 1, 3, 4, 6,    0, 1, 2, 3, 4, 5,    1, 2, 4, 5,
                               0, 1, 3, 4, 7,    0, 1, 2, 3, 4, 5,    1, 2, 4, 5,
                               0, 1, 3, 4,    1, 2, 4, 5,    0, 1, 3, 4,    1, 2, 4, 5};
  const int32_t want_hp[9] = {0, 1, 3, 5, 8, 13, 17, 18, 18};
  const int32_t want_hc[18] = {0,   0, 1,   1, 2,   0, 1, 3,   0, 1, 2, 3, 4,   1, 2, 4, 5,   6};
  if (!same("jac_rowptr", jp, want_jp, 11) || !same("jac_col", jc, want_jc, 46) ||
      !same("hess_rowptr", hp, want_hp, 9) || !same("hess_col", hc, want_hc, 18))
    return 5;
  /* an N-1 child of branch 0: bus 0 loses its neighbour, the flow rows of
     branch 0 go */
  if (acopf_pattern_host(&d, 0, &dims, NULL, NULL, NULL, NULL) != ACOPF_OK) return 6;
  if (dims.m != 8 || dims.m_eq != 6 || dims.nnz_jac != 46 - 8 - 8 || dims.nnz_hess != 18 - 4 ||
      dims.nbranch != 1 || dims.outage != 0)
    return 7;
  /* errors come back as codes with a message, never as exceptions */
  d.base_mva = 0.0;
  if (acopf_pattern_host(&d, -1, &dims, NULL, NULL, NULL, NULL) != ACOPF_EINVAL) return 8;
  if (strstr(acopf_last_error(), "base_mva") == NULL) return 9;
  printf("abi_c ok\n");
  return 0;
}
