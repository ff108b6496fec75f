// partials.h - capacity of a context's buffer of per-block partial sums (host logic only).
//
// Every reduction in the library is deterministic: each block of a launch writes its sums to
// partial[block * sums + k] and a one-block kernel adds them in block order.  One buffer per
// context serves all such launches, so it must hold the largest blocks x sums of any of them.
// partial_uses lists every kind of launch that writes partials, partial_capacity is the size
// that holds them all, and partials_fit is the check made before each launch.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fnpf {

constexpr int kPartialVecBlocks = 1024;   // grid of the grid-stride vector kernels (FP64 data)

struct PartialUse {
  const char *what;
  int64_t blocks;
  int sums;
};

// colour_blocks: blocks of the colour-scheduled apply summed over its colours (one partial each);
// owner_blocks: blocks of both passes of the owner-computes apply (one partial each).
inline std::vector<PartialUse> partial_uses(int64_t colour_blocks, int64_t owner_blocks) {
  const int64_t v64 = kPartialVecBlocks, v32 = 2 * kPartialVecBlocks;
  return {
      {"norm of b (k_bnorm)", v64, 1},
      {"PCG initial residual (k_pcg_init)", v64, 2},
      {"mixed outer residual (k_resid_to32)", v64, 3},
      {"PCG update (k_pcg_update)", v64, 2},
      {"p-multigrid update and dots, FP64 grid", v64, 2},
      {"p-multigrid update and dots, FP32 grid", v32, 2},
      {"Lanczos and power-iteration dots, FP32 grid", v32, 2},
      {"line-smoother B-norm (k_line_bnorm), FP32 grid", v32, 1},
      {"apply with dot product, colour schedule", colour_blocks, 1},
      {"apply with dot product, owner-computes", owner_blocks, 1},
  };
}

inline int64_t partial_capacity(const std::vector<PartialUse> &uses) {
  int64_t cap = 0;
  for (const auto &u : uses) cap = u.blocks * u.sums > cap ? u.blocks * u.sums : cap;
  return cap;
}

inline bool partials_fit(int64_t capacity, int64_t blocks, int sums) {
  return blocks >= 0 && sums > 0 && blocks * sums <= capacity;
}

// "" when every use fits the capacity, else the first use that does not
inline std::string partial_layout_error(const std::vector<PartialUse> &uses, int64_t capacity) {
  for (const auto &u : uses)
    if (!partials_fit(capacity, u.blocks, u.sums))
      return std::string("partial-sum buffer too small for ") + u.what;
  return "";
}

}  // namespace fnpf
