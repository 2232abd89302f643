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

// Panel images: the operand layout the MFMA kernels stream.  An operand with
// Mp rows (a multiple of 256) and Kb bytes of K per row (a multiple of 64) is
// cut into blocks of 256 rows x 64 bytes (16 KiB); block (rb, kb) starts at
// byte (rb * nkb + kb) * 16 KiB, nkb = Kb / 64.  The K extent of one 256-row
// panel is therefore contiguous, and one block is exactly one LDS slab of one
// pipeline stage, copied linearly.  Inside a block, row r occupies bytes
// [64 r, 64 r + 64) and its 16-byte chunk c sits at position c ^ ((r / 4) % 4):
// the LDS bank swizzle, applied once by the writer of the image.
constexpr int kPanelRows = 256, kPanelRowBytes = 64, kPanelBlock = 16384;

__host__ __device__ __forceinline__ int64_t panel_offset(int64_t row, int64_t kbyte, int64_t nkb) {
    const int64_t rb = row >> 8, kb = kbyte >> 6;
    const int r = (int)(row & 255), c = (int)((kbyte >> 4) & 3);
    return ((rb * nkb + kb) << 14) + (r << 6) + ((c ^ ((r >> 2) & 3)) << 4) + (kbyte & 15);
}

// MX FP6 panel images (E2M3 codes packed 6 bits each, code j of a 32-value K
// half at bit 6 j, little endian): per operand three arrays, hi codes, lo
// codes and scales, cut like the panel images into blocks of 256 rows by one
// 64-value K block; block (rb, kb) is block number rb * nkb + kb of each array.
// A code block is 256 rows x 48 bytes (12 KiB); row r holds, at 48 r,
//   [half 0 bytes 0-15 | half 1 bytes 0-15 | half 0 bytes 16-23 | half 1 bytes 16-23]
// so that a lane's 24 bytes are one 16-byte and one 8-byte aligned read.  A
// scale block is 256 rows x 4 bytes (1 KiB): row r holds the E8M0 bytes
// (half 0 hi, half 0 lo, half 1 hi, half 1 lo) at 4 r, so one 16-bit read
// gives a lane both levels' scales of its half.
constexpr int kMx6RowBytes = 48, kMx6Block = kPanelRows * kMx6RowBytes, kMx6ScaleBlock = 1024;

__host__ __device__ __forceinline__ int64_t mx6_code_offset(int64_t row, int64_t kb, int h, int byte,
                                                            int64_t nkb) {
    const int64_t rb = row >> 8;
    const int r = (int)(row & 255);
    const int pos = byte < 16 ? 16 * h + byte : 32 + 8 * h + (byte - 16);
    return (rb * nkb + kb) * kMx6Block + r * kMx6RowBytes + pos;
}
__host__ __device__ __forceinline__ int64_t mx6_scale_offset(int64_t row, int64_t kb, int h, int level,
                                                             int64_t nkb) {
    return (((row >> 8) * nkb + kb) << 10) + (row & 255) * 4 + 2 * h + level;
}

// Workgroup `blk` of a launch that runs ta workgroups of one kind and tb of
// another (the operand pre-passes of A and B in one launch), spread evenly:
// the second kind sits at the blocks where floor(blk * tb / (ta + tb)) steps,
// so both kinds stream side by side in proportion for the whole launch.
// *index is the workgroup's number within its kind.
__device__ __forceinline__ bool second_kind(int64_t blk, int64_t ta, int64_t tb, int64_t* index) {
    const int64_t total = ta + tb;
    const int64_t before = blk * tb / total, upto = (blk + 1) * tb / total;
    *index = upto > before ? before : blk - before;
    return upto > before;
}

// The same over groups of eight consecutive workgroups, which the hardware
// hands to the eight XCDs in turn: every XCD gets its share of both kinds
// (a plain A, B, A, B order would put all of A on four XCDs).  A launch of
// paired_blocks(ta, tb) workgroups; returns 0 (first kind), 1 (second kind)
// or -1 for the few workgroups past the end of a kind's last group.
__host__ __device__ __forceinline__ int64_t paired_blocks(int64_t ta, int64_t tb) {
    return 8 * ((ta + 7) / 8 + (tb + 7) / 8);
}
__device__ __forceinline__ int paired_kind(int64_t blk, int64_t ta, int64_t tb, int64_t* index) {
    int64_t g;
    const bool second = second_kind(blk >> 3, (ta + 7) / 8, (tb + 7) / 8, &g);
    *index = 8 * g + (blk & 7);
    if (*index >= (second ? tb : ta)) return -1;
    return second ? 1 : 0;
}

}  // namespace cmp
