// Host-side checks of libttm's argument validation and size planning, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code (the
// device code is compiled as usual) and run without a GPU: every call below
// returns before any HIP call that needs a device.  Exercises the size
// queries on seeded random shapes (mixed dimensions, bonds above the
// structural bound, every option), oversized and malformed descriptors, and
// the argument checks of every compute entry point.  Exit status 0 when
// every expected code came back and no sanitizer fired.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "ttm.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what, int line) {
  if (!ok) {
    fprintf(stderr, "host_checks: failed at line %d: %s\n", line, what);
    ++failures;
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

struct Train {
  std::vector<int32_t> phys, bonds;
  std::vector<int64_t> offs;
  ttm_tt view;
  Train(const std::vector<int32_t> &d, const std::vector<int32_t> &b) : phys(d), bonds(b) {
    int64_t pos = 0;
    for (size_t i = 0; i < d.size(); ++i) {
      offs.push_back(pos);
      pos += (int64_t)b[i] * d[i] * b[i + 1];
    }
    view.n_sites = (int32_t)d.size();
    view.phys = phys.data();
    view.bonds = bonds.data();
    view.offsets = offs.data();
    view.data = reinterpret_cast<const void *>(0x1000);
    view.dtype = TTM_F64;
  }
};

// SplitMix64 step (Steele, Lea, Flood): the random shapes only.
uint64_t next(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
int uniform(uint64_t &s, int lo, int hi) { return lo + (int)(next(s) % (uint64_t)(hi - lo + 1)); }

}  // namespace

int main() {
  // 1. size queries on random shapes, every option combination
  uint64_t seed = 20241025;
  for (int k = 0; k < 400; ++k) {
    const int n = uniform(seed, 1, 9);
    std::vector<int32_t> d(n), ba(n + 1, 1), bb(n + 1, 1);
    for (int i = 0; i < n; ++i) d[i] = uniform(seed, 1, 8);
    for (int i = 1; i < n; ++i) {
      ba[i] = uniform(seed, 1, 40);
      bb[i] = uniform(seed, 1, 40);
    }
    Train A(d, ba), B(d, bb);
    ttm_options o;
    ttm_default_options(&o);
    o.chi_mid = uniform(seed, -1, 64);
    o.final_round = uniform(seed, 0, 1);
    o.move_factor = uniform(seed, 0, 1);
    o.gauge = uniform(seed, 0, 1);
    o.contract_precision = uniform(seed, 0, 3);
    o.svd_mode = uniform(seed, 0, 1);
    o.rsvd_power = uniform(seed, 0, 12);
    o.rsvd_tol = uniform(seed, 0, 1) ? 1e-14 : 2e-8;
    const int chi = uniform(seed, 1, 80);
    size_t ws = 0;
    int64_t cap = 0;
    const int rc = ttm_query(&A.view, &B.view, chi, &o, &ws, &cap);
    EXPECT(rc == TTM_OK || rc == TTM_EUNSUPPORTED);
    if (rc == TTM_OK) EXPECT(ws > 0 && cap >= n);
    EXPECT(conventional_query(&A.view, &B.view, chi, &o, &ws, &cap) == TTM_OK);
    EXPECT(ttm_inner_grad_query(&A.view, &A.view, &B.view, &ws) == TTM_OK);
    {
      size_t plain = 0, ck = 0;
      EXPECT(ttm_inner_grad_query(&A.view, &A.view, &B.view, &plain) == TTM_OK);
      EXPECT(ttm_inner_grad_query_ex(&A.view, &A.view, &B.view, uniform(seed, 0, 12), &ck) == TTM_OK);
      EXPECT(ck > 0 && plain > 0);
      EXPECT(ttm_inner_grad_query_ex(&A.view, &A.view, &B.view, -3, &ck) == TTM_EINVAL);
    }
    // argument checks of the compute calls: all fail before any HIP call
    std::vector<int32_t> cb(n + 1);
    std::vector<int64_t> co(n);
    ttm_tt_out C = {cb.data(), co.data(), reinterpret_cast<void *>(0x2000), 0};
    EXPECT(ttm_multiply_ex(&A.view, &B.view, chi, -1.0, &C, nullptr, 0, nullptr, &o, nullptr) == TTM_EINVAL);
    EXPECT(ttm_multiply_ex(&A.view, &B.view, 0, 1e-12, &C, nullptr, 0, nullptr, &o, nullptr) == TTM_EINVAL);
    if (rc == TTM_OK) {
      EXPECT(ttm_multiply_ex(&A.view, &B.view, chi, 1e-12, &C, nullptr, 0, nullptr, &o, nullptr) == TTM_EWORKSPACE);
      EXPECT(ttm_multiply_static(&A.view, &B.view, chi, 1e-12, &C, nullptr, &o, nullptr) == TTM_ECAPACITY);
      EXPECT(strlen(ttm_last_error()) == 0);
    }
    EXPECT(conventional_multiply_ex(&A.view, &B.view, chi, NAN, &C, nullptr, 0, nullptr, &o, nullptr) ==
           TTM_EINVAL);
    double v = 0.0;
    EXPECT(ttm_inner_grad(&A.view, &A.view, &B.view, 9, &v, nullptr, nullptr, nullptr, 0, nullptr) == TTM_EINVAL);
    // the reverse mode: its sizes cover the product's, and its argument
    // checks come before any HIP call as well
    size_t vws = 0;
    int64_t vcap = 0;
    const int vrc = ttm_vjp_query(&A.view, &B.view, chi, &o, &vws, &vcap);
    EXPECT(vrc == ((o.gauge == TTM_GAUGE_RIGHT || o.svd_mode == TTM_SVD_RANDOMIZED) && rc == TTM_OK
                       ? TTM_EUNSUPPORTED : rc));
    if (vrc == TTM_OK) {
      size_t fws = 0;
      int64_t fcap = 0;
      EXPECT(ttm_query(&A.view, &B.view, chi, &o, &fws, &fcap) == TTM_OK);
      EXPECT(vws > fws && vcap == fcap);
      double *fake = reinterpret_cast<double *>(0x4000);
      EXPECT(ttm_multiply_vjp(&A.view, &B.view, chi, 1e-12, &o, &A.view, &C, fake, fake, nullptr, 0, nullptr,
                              nullptr) == TTM_EWORKSPACE);
      EXPECT(ttm_multiply_vjp(&A.view, &B.view, chi, NAN, &o, &A.view, &C, fake, fake, nullptr, 0, nullptr,
                              nullptr) == TTM_EINVAL);
    }
  }
  // 2. malformed descriptors and options
  {
    Train A({2, 3, 2}, {1, 2, 2, 1}), B({2, 3, 2}, {1, 2, 2, 1}), Bad({2, 2, 2}, {1, 2, 2, 1});
    Train Ends({2, 3, 2}, {2, 2, 2, 1});
    size_t ws = 0;
    int64_t cap = 0;
    EXPECT(ttm_query(&A.view, &Bad.view, 4, nullptr, &ws, &cap) == TTM_ESHAPE);
    EXPECT(ttm_query(&A.view, &Ends.view, 4, nullptr, &ws, &cap) == TTM_ESHAPE);
    EXPECT(ttm_query(nullptr, &B.view, 4, nullptr, &ws, &cap) == TTM_EINVAL);
    EXPECT(ttm_query(&A.view, &B.view, 0, nullptr, &ws, &cap) == TTM_EINVAL);
    ttm_options o;
    ttm_default_options(&o);
    o.gauge = 2;
    EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EINVAL);
    ttm_default_options(&o);
    o.move_factor = -1;
    EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EINVAL);
    ttm_default_options(&o);
    o.svd_mode = 2;
    EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EINVAL);
    ttm_default_options(&o);
    o.rsvd_power = 65;
    EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EINVAL);
    for (double bad_tol : {0.0, -1.0, 2.0, (double)NAN}) {
      ttm_default_options(&o);
      o.rsvd_tol = bad_tol;
      EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EINVAL);
    }
    ttm_default_options(&o);
    o.n_forced = 2;
    EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EINVAL);
    int32_t bad_rank[1] = {0};
    o.forced_ranks = bad_rank;
    o.n_forced = 1;
    EXPECT(ttm_query(&A.view, &B.view, 4, &o, &ws, &cap) == TTM_EFORCED);
    A.view.dtype = 7;
    EXPECT(ttm_query(&A.view, &B.view, 4, nullptr, &ws, &cap) == TTM_EUNSUPPORTED);
  }
  // 3. oversized shapes: sizes formed in 64 bits, rejected before use
  {
    const int big = 1 << 16;
    Train A({big, big}, {1, big, 1}), B({big, big}, {1, 1, 1});
    size_t ws = 0;
    int64_t cap = 0;
    EXPECT(ttm_query(&A.view, &B.view, 1 << 20, nullptr, &ws, &cap) == TTM_EINVAL);
    std::vector<int32_t> d(44, 2), b(45, 1 << 20);
    b[0] = b[44] = 1;
    Train W(d, b);
    EXPECT(conventional_query(&W.view, &W.view, big, nullptr, &ws, &cap) == TTM_EINVAL);
    Train G({big, big}, {1, 1 << 20, 1});
    EXPECT(ttm_inner_grad_query(&G.view, &G.view, &G.view, &ws) == TTM_EINVAL);
    Train S({8, 8, 8, 8, 8, 8, 8, 8}, {1, 8, 64, 128, 128, 128, 64, 8, 1});
    ttm_options o;
    ttm_default_options(&o);
    o.chi_mid = 0;
    EXPECT(ttm_query(&S.view, &S.view, 128, &o, &ws, &cap) == TTM_EUNSUPPORTED);
  }
  // 4. batch argument checks
  {
    Train A({2, 2, 2, 2}, {1, 2, 4, 2, 1});
    ttm_tt As[3] = {A.view, A.view, A.view};
    int32_t chis[3] = {4, 4, 4};
    double tols[3] = {1e-12, 1e-12, 1e-12};
    int32_t status[3];
    EXPECT(ttm_multiply_batch(3, As, As, chis, tols, nullptr, nullptr, nullptr, nullptr, nullptr, 2, nullptr,
                              status) == TTM_EINVAL);
    EXPECT(ttm_multiply_batch(-1, As, As, chis, tols, nullptr, nullptr, nullptr, nullptr, nullptr, 2, nullptr,
                              status) == TTM_EINVAL);
    EXPECT(ttm_multiply_batch(3, As, As, chis, tols, nullptr, nullptr, nullptr, nullptr, nullptr, 5, nullptr,
                              status) == TTM_EINVAL);
  }
  for (int c = 0; c >= -9; --c) EXPECT(ttm_strerror(c) != nullptr && strlen(ttm_strerror(c)) > 0);
  if (failures) {
    fprintf(stderr, "host_checks: %d failures\n", failures);
    return 1;
  }
  printf("host_checks: ok\n");
  return 0;
}
