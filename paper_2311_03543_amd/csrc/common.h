// Device helpers shared by the gfx950 kernels of libcompar.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cmp {

constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, 32 CUs each

// Workgroups are dispatched round-robin over the XCDs (id % 8 lands on XCD
// id % 8).  Renumber so that each XCD receives one contiguous range of tile
// ids: neighbouring tiles then share that XCD's L2.  Bijective on [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = b % kXcds, idx = b / kXcds;
    return x * per + (x < rem ? x : rem) + idx;
}

// Tile coordinates from a linear id with "grouped" ordering: walk `group`
// tile-rows at a time, column by column, so consecutive ids reuse the same
// B column panel and a small set of A row panels.
__device__ __forceinline__ void grouped_tile(int id, int tiles_m, int tiles_n, int group,
                                             int& tm, int& tn) {
    const int per_group = group * tiles_n;
    const int g = id / per_group;
    const int first_m = g * group;
    const int gm = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
    const int local = id - g * per_group;
    tm = first_m + local % gm;
    tn = local / gm;
}

}  // namespace cmp
