// Host test driver for gabp_validate_csr, built with the address and undefined-behaviour
// sanitizers together with the library's host-only validate.cpp (no GPU). Every array is
// a heap allocation of exactly its stated length, so any read past it aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/gabp.h"

namespace {

struct Case {
  const char* name;
  int32_t n;
  std::vector<int32_t> rowptr, col, rev;
  std::vector<double> val;
  bool with_rev;
  int expect;
};

int run(const Case& c) {
  // exact-length heap copies (vector storage of exactly size() elements)
  std::vector<int32_t> rp(c.rowptr), cl(c.col), rv(c.rev);
  std::vector<double> vl(c.val);
  rp.shrink_to_fit();
  cl.shrink_to_fit();
  rv.shrink_to_fit();
  vl.shrink_to_fit();
  return gabp_validate_csr(c.n, static_cast<int64_t>(cl.size()), rp.data(), cl.data(),
                           vl.data(), c.with_rev ? rv.data() : nullptr);
}

}  // namespace

int main() {
  const double nan = std::nan("");
  const std::vector<Case> cases = {
      {"valid 3x3", 3, {0, 2, 5, 7}, {0, 1, 0, 1, 2, 1, 2}, {}, {4, -1, -1, 4, -1, -1, 4}, false, GABP_OK},
      {"valid with rev", 3, {0, 2, 5, 7}, {0, 1, 0, 1, 2, 1, 2}, {0, 2, 1, 3, 5, 4, 6},
       {4, -1, -1, 4, -1, -1, 4}, true, GABP_OK},
      {"one-way entry, rev -1", 2, {0, 2, 3}, {0, 1, 1}, {0, -1, 2}, {2, 1, 2}, true, GABP_OK},
      {"rowptr overshoots nnz inside", 2, {0, 5, 2}, {0, 1}, {}, {1, 1}, false, GABP_EINVAL},
      {"rowptr decreasing", 2, {0, 2, 1}, {0}, {}, {1}, false, GABP_EINVAL},
      {"rowptr[n] != nnz", 2, {0, 1, 3}, {0, 1}, {}, {1, 1}, false, GABP_EINVAL},
      {"nnz < n", 3, {0, 1, 2, 2}, {0, 1}, {}, {1, 1}, false, GABP_EINVAL},
      {"n = 0", 0, {0}, {}, {}, {}, false, GABP_EINVAL},
      {"column out of range", 2, {0, 1, 2}, {0, 7}, {}, {1, 1}, false, GABP_EINVAL},
      {"negative column", 2, {0, 2, 3}, {-1, 0, 1}, {}, {1, 1, 1}, false, GABP_EINVAL},
      {"columns not increasing", 2, {0, 2, 4}, {1, 0, 0, 1}, {}, {1, 2, 1, 2}, false, GABP_EINVAL},
      {"non-finite value", 2, {0, 1, 2}, {0, 1}, {}, {1, nan}, false, GABP_EINVAL},
      {"zero diagonal", 2, {0, 1, 2}, {0, 1}, {}, {1, 0}, false, GABP_EZERODIAG},
      {"missing diagonal", 2, {0, 2, 3}, {0, 1, 0}, {}, {1, 1, 1}, false, GABP_EZERODIAG},
      {"rev inconsistent", 2, {0, 2, 4}, {0, 1, 0, 1}, {0, 3, 2, 3}, {2, 1, 1, 2}, true, GABP_EINVAL},
      {"rev far out of range", 2, {0, 2, 4}, {0, 1, 0, 1}, {0, 1000000, 1, 3}, {2, 1, 1, 2}, true,
       GABP_EINVAL},
      {"rev of diagonal elsewhere", 2, {0, 2, 4}, {0, 1, 0, 1}, {1, 2, 1, 3}, {2, 1, 1, 2}, true,
       GABP_EINVAL},
  };
  int bad = 0;
  for (const auto& c : cases) {
    const int got = run(c);
    if (got != c.expect) {
      std::printf("FAIL %s: status %d, expected %d (%s)\n", c.name, got, c.expect,
                  gabp_last_error());
      ++bad;
    }
  }
  std::printf("%zu cases, %d failed\n", cases.size(), bad);
  return bad == 0 ? 0 : 1;
}
