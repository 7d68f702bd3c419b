// Host-only checks of the level-major launch geometry and of the launchers'
// empty-range guards (no kernel is launched; runs without a GPU).
//  1. level_major_grid / level_major_item: for every level count, tile count
//     and mapping, each (tile, level) pair of the launch is produced by exactly
//     one workgroup and every other workgroup is idle; an empty level range or
//     an empty tile set gives an empty grid.
//  2. The launchers return success without launching for an empty level range
//     or no tiles (an empty range once reached an integer division by zero).
#include <cstdio>
#include <vector>

#include "../../paper_2304_10516_amd/csrc/dvnr_device.h"

using namespace dvnrk;

static int failures = 0;
#define CHECK(cond, ...)                \
  do {                                  \
    if (!(cond)) {                      \
      std::printf("FAIL: " __VA_ARGS__); \
      std::printf("\n");                \
      ++failures;                       \
    }                                   \
  } while (0)

int main() {
  const int tiles[] = {0, 1, 2, 3, 5, 7, 8, 9, 17, 100};
  for (int L = 0; L <= kMaxLevels; ++L)
    for (int nt : tiles)
      for (int xcd = 0; xcd <= 1; ++xcd) {
        const int grid = level_major_grid(L, nt, xcd);
        CHECK(grid >= 0, "negative grid L=%d nt=%d xcd=%d", L, nt, xcd);
        if (L == 0 || nt == 0) CHECK(grid == 0, "non-empty grid for an empty launch L=%d nt=%d", L, nt);
        const int l0 = 3;
        std::vector<int> seen((size_t)(L > 0 ? L : 1) * (nt > 0 ? nt : 1), 0);
        for (int wg = 0; wg < grid; ++wg) {
          int tile = -1, level = -1;
          if (!level_major_item(wg, l0, L, nt, xcd, tile, level)) continue;
          const bool in = tile >= 0 && tile < nt && level >= l0 && level < l0 + L;
          CHECK(in, "item out of range L=%d nt=%d xcd=%d wg=%d -> (%d, %d)", L, nt, xcd, wg, tile, level);
          if (in) seen[(size_t)tile * L + (level - l0)] += 1;
        }
        if (L > 0 && nt > 0)
          for (size_t i = 0; i < seen.size(); ++i)
            CHECK(seen[i] == 1, "pair %zu produced %d times L=%d nt=%d xcd=%d", i, seen[i], L, nt, xcd);
      }
  // empty level ranges and tile sets: success, nothing launched
  LevelDesc ld{};
  ld.L = 16;
  ld.F = 2;
  PartDesc pd{};
  pd.nl = 0;
  CHECK(launch_encode(Prec::MIXED, 1, ld, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr, 2, 2, 1,
                      nullptr, 5, 5) == hipSuccess, "encode, empty level range");
  CHECK(launch_encode(Prec::F32, 0, ld, nullptr, (const Tile*)8, 0, 0, nullptr, nullptr, nullptr, nullptr, 2, 2, 1,
                      nullptr, 0, 16) == hipSuccess, "encode, no tiles");
  CHECK(launch_scatter(Prec::F32, ld, 7, 7, nullptr, nullptr, 100, 0, nullptr, nullptr, nullptr, 2, 2, nullptr, 1, 1,
                       0, nullptr) == hipSuccess, "scatter, empty level range");
  CHECK(launch_scatter(Prec::F32, ld, 0, 16, nullptr, (const Tile*)8, 0, 0, nullptr, nullptr, nullptr, 2, 2, nullptr,
                       1, 1, 1, nullptr) == hipSuccess, "scatter, no tiles");
  CHECK(launch_scatter_priv(ld, 4, 4, 8, 1, nullptr, nullptr, nullptr, nullptr, nullptr, 2, nullptr, 0, 2, nullptr) ==
            hipSuccess, "privatized scatter, empty level range");
  CHECK(launch_encode_binned(Prec::MIXED, 1, ld, 9, 9, 8, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 2, 2,
                             nullptr) == hipSuccess, "binned encode, empty level range");
  CHECK(launch_part_bucket(ld, pd, nullptr, nullptr, 100, nullptr, nullptr, nullptr, nullptr, 2, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr) == hipSuccess, "partition pass 1, no levels");
  CHECK(launch_part_accum(ld, pd, nullptr, 4, 100, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr, nullptr) == hipSuccess, "partition pass 2, no levels");
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("launch guards ok\n");
  return 0;
}
