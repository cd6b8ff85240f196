// Host-only paths of the C ABI under AddressSanitizer and UBSan: the BQP and
// Hermitian UCQP builders write into buffers of exactly the size the ABI
// documents, the options and argument checks run before any device work, and
// the sparse-A constructor rejects bad triplets on the host.  Calls nothing
// that touches a GPU.  Exit status 0 on success; a sanitizer report aborts.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "manidsdp.h"

#define EXPECT(cond)                                                 \
  do {                                                               \
    if (!(cond)) {                                                   \
      fprintf(stderr, "failed: %s (line %d): %s\n", #cond, __LINE__, \
              mdsdp_last_error());                                   \
      return 1;                                                      \
    }                                                                \
  } while (0)

static unsigned long long rng_state = 88172645463325252ull;
static double urand() {  // xorshift64, values in (-1, 1)
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) / (double)(1ull << 52) - 1.0;
}

int main() {
  // BQP builders, both basis orders
  for (int q = 1; q <= 24; ++q) {
    int32_t n = 0;
    int64_t m = 0;
    EXPECT(mdsdp_bqp_sizes(q, &n, &m) == MDSDP_OK);
    std::vector<int32_t> cls((size_t)n * (n + 1) / 2);
    for (int order = 0; order < 2; ++order) {
      EXPECT(mdsdp_bqp_classmap(q, order, cls.data()) == MDSDP_OK);
      for (int32_t id : cls) EXPECT(id >= 0 && id < m);
    }
    std::vector<double> Q((size_t)q * q), c(q), b(m);
    for (int i = 0; i < q; ++i)
      for (int j = i + 1; j < q; ++j) Q[i * q + j] = Q[j * q + i] = urand();
    for (double& x : c) x = urand();
    EXPECT(mdsdp_bqp_b(q, Q.data(), c.data(), b.data()) == MDSDP_OK);
    for (double x : b) EXPECT(isfinite(x));
  }
  EXPECT(mdsdp_bqp_sizes(0, nullptr, nullptr) == MDSDP_EINVAL);
  EXPECT(mdsdp_bqp_classmap(5, 7, nullptr) == MDSDP_EINVAL);

  // Hermitian UCQP builders
  for (int q = 1; q <= 10; ++q) {
    int32_t n = 0;
    int64_t m = 0;
    EXPECT(mdsdp_ucqp_sizes(q, &n, &m) == MDSDP_OK);
    std::vector<int32_t> cls((size_t)n * (n + 1) / 2);
    std::vector<int8_t> coef(cls.size());
    EXPECT(mdsdp_ucqp_structure(q, cls.data(), coef.data()) == MDSDP_OK);
    for (size_t e = 0; e < cls.size(); ++e) {
      EXPECT(coef[e] >= -1 && coef[e] <= 1);
      EXPECT(coef[e] == 0 || (cls[e] >= 0 && cls[e] < m));
    }
    std::vector<double> Qre((size_t)q * q), Qim((size_t)q * q), b(m);
    for (int i = 0; i < q; ++i) {
      Qre[i * q + i] = urand();
      for (int j = i + 1; j < q; ++j) {
        Qre[i * q + j] = Qre[j * q + i] = urand();
        Qim[i * q + j] = urand();
        Qim[j * q + i] = -Qim[i * q + j];
      }
    }
    EXPECT(mdsdp_ucqp_b(q, Qre.data(), Qim.data(), b.data()) == MDSDP_OK);
    for (double x : b) EXPECT(isfinite(x));
  }

  // options are validated before anything else
  mdsdp_options o;
  mdsdp_default_options(&o);
  mdsdp_result r;
  o.tol = 0.0;
  EXPECT(mdsdp_solve(nullptr, &o, 2, nullptr, &r, nullptr, 0, nullptr) == MDSDP_EINVAL);
  mdsdp_default_options(&o);
  o.round_gap = 2.0;
  EXPECT(mdsdp_solve(nullptr, &o, 2, nullptr, &r, nullptr, 0, nullptr) == MDSDP_EINVAL);
  mdsdp_default_options(&o);
  EXPECT(mdsdp_solve(nullptr, &o, 2, nullptr, &r, nullptr, 0, nullptr) == MDSDP_EINVAL);  // NULL problem
  EXPECT(mdsdp_sync_status(nullptr, nullptr) == MDSDP_EINVAL);
  double out[4];
  EXPECT(mdsdp_certificate_bound(nullptr, 2, nullptr, 1e-8, 10, 0, out, nullptr) == MDSDP_EINVAL);

  // sparse A with overlapping supports and with a coefficient other than +-1,
  // rejected on the host (n = 3, two classes)
  {
    const int32_t k[4] = {0, 0, 1, 1}, row[4] = {0, 1, 0, 0}, col[4] = {0, 1, 1, 1};
    const double v[4] = {1.0, 1.0, 1.0, 1.0}, b[2] = {1.0, 0.0};
    mdsdp_problem h = nullptr;
    EXPECT(mdsdp_create_sparse_A(3, 2, 4, k, row, col, v, b, nullptr, &h) == MDSDP_ENOTORTH);
    const double v2[3] = {1.0, 1.0, 2.0};
    EXPECT(mdsdp_create_sparse_A(3, 2, 3, k, row, col, v2, b, nullptr, &h) == MDSDP_EUNSUPPORTED);
    EXPECT(h == nullptr);
  }
  printf("host paths ok\n");
  return 0;
}
