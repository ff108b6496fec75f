// CPU check of the partial-sum table (paper_2506_09435_amd/csrc/partials.h): the capacity it gives
// holds every listed launch, including the grids the library uses, and the check made before each
// launch rejects one that would write past the buffer.  Prints "ok" on success.
#include <cstdio>
#include <cstdlib>

#include "partials.h"

using namespace fnpf;

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAILED line %d: %s\n", __LINE__, #c);          \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(int argc, char **argv) {
  // (colour blocks, owner blocks) pairs given on the command line, then some extremes
  std::vector<std::pair<long long, long long>> cases;
  for (int a = 1; a + 1 < argc; a += 2) cases.push_back({std::atoll(argv[a]), std::atoll(argv[a + 1])});
  cases.push_back({0, 0});
  cases.push_back({1, 1});
  cases.push_back({100000, 3});
  cases.push_back({3, 100000});
  for (auto [cb, ob] : cases) {
    const auto uses = partial_uses(cb, ob);
    const int64_t cap = partial_capacity(uses);
    CHECK(partial_layout_error(uses, cap).empty());
    for (const auto &u : uses) CHECK(partials_fit(cap, u.blocks, u.sums));
    // the grids the library launches: FP64 vector grid with up to three sums, FP32 grid with two
    CHECK(partials_fit(cap, kPartialVecBlocks, 3));
    CHECK(partials_fit(cap, 2 * kPartialVecBlocks, 2));
    CHECK(partials_fit(cap, cb, 1) && partials_fit(cap, ob, 1));
    // one more block than the buffer holds is rejected, and so is a capacity one short
    CHECK(!partials_fit(cap, cap + 1, 1));
    CHECK(!partial_layout_error(uses, cap - 1).empty());
  }
  CHECK(!partials_fit(10, -1, 1));
  CHECK(!partials_fit(10, 1, 0));
  if (fails == 0) std::printf("ok\n");
  return fails == 0 ? 0 : 1;
}
