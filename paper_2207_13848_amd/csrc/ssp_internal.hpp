// Internal layout shared by the kernels and the host launch code.
#pragma once

#include <stdint.h>

#include "../../include/ssp.h"

namespace ssp {

// Row bins of the symbolic (distinct-count) kernels, by row FLOP.
//   bin 1: 1..128 products      -> one wave per row, LDS table <= 256 words
//   bin 2: 129..1024 products   -> 256 threads per row, LDS table <= 2048 words
//   bin 3: 1025..8192 products  -> 512 threads per row, LDS table <= 16384 words
//   bin 4: more                 -> 1024 threads, LDS bitmap per column window;
//                                  rows above kSplitTarget products are cut into
//                                  parts whose bitmaps a merge kernel ORs
constexpr uint64_t kBin1Max = 128, kBin2Max = 1024, kBin3Max = 8192;
constexpr int kBin1Words = 256, kBin2Words = 2048, kBin3Words = 16384;
constexpr int kBin1Team = 64, kBin2Team = 256, kBin3Team = 512, kBin4Team = 1024;

// Bin-4 bitmap window: at most 32768 words = 2^20 columns = 128 KiB of LDS.
constexpr int kWinWords = 32768;
constexpr uint64_t kSplitTarget = 1ull << 17; // products per part of a split row
constexpr int kMaxParts = 64;
constexpr int kMaxPartWindows = 1024;         // global part bitmaps (x window words)
constexpr int kMaxSplitWindows = 4;           // rows needing more windows are not split
constexpr int kMergeSlice = 1024;             // words per merge item

// Streaming FLOP kernels: 256 threads, tiles of kFlopTile merge-path items
// (rows + entries of A), at most kFlopTile + 3 < 2048 entries per tile.
constexpr int kFlopThreads = 256;
constexpr int kFlopChunk = 2048;
constexpr int64_t kFlopTile = 2040;

// Control block at the start of the workspace (device memory).
struct Ctl {
    ssp_stats stats;      // used when the caller passes no stats pointer
    uint32_t bin_cnt[8];  // items in bins 1..4 (index = bin), merge items at 5
    uint32_t pw_ctr;      // part windows handed out
    uint32_t pad_ctr;
    uint32_t fallback;    // 1: f* = 0, predict row FLOP
    uint32_t big_next;    // work queue of the long-row kernel
    uint32_t pad0[4];
    uint64_t div_dn, div_v; // Divisor of f*
    uint32_t div_shift, pad1;
    uint64_t ref_q_lo, ref_q_hi; // reference design: z* M
    uint64_t ref_d_lo, ref_d_hi; // reference design: n_s F
    uint64_t pad2[16];
    // distinct counts (z*, or the exact total) added by the symbolic kernels
    // into kAccSlots slots by workgroup: atomics on one address serialise,
    // atomics on distinct addresses do not; k_finalize sums the slots
    uint64_t zacc[64];
};
constexpr int kAccSlots = 64;

struct BinItem {  // bins 1..3
    int32_t row;
    uint32_t rf;
};

struct BigItem {  // bin 4: the A entries [e_lo, e_hi) of one long row
    int32_t row;
    int32_t slot;   // first part window of a split row, -1 when not split
    int32_t part;   // part index of a split row (0 when not split)
    int32_t nparts;
    int32_t e_lo, e_hi;
};

struct MergeItem {  // one slice of one window of a split row
    int32_t row;
    int32_t slot;
    int32_t nparts;
    int32_t window;
    int32_t slice;
    int32_t pad;
};

// Per-workgroup counters of the sampling passes.  k_sample_count writes
//   c[0..2] rows of bins 1..3, c[3] rows of bin 4, c[4] bin-4 items if its
//   split-eligible rows are split, c[5] their merge items, c[6] part windows
//   they request;
// k_sample_scan rewrites them in place as
//   c[0..2] offsets in bins 1..3, c[3] offset in bin 4, c[4] offset in the
//   merge list, c[5] first part window, c[6] 1 if the rows are split.
struct SampleCounts {
    uint32_t c[8];
    uint64_t ns, fs, as, pad; // sampled rows, their products, their A entries
};
constexpr int kSampleGroups = 512; // workgroups of the sampling passes (at most)

struct TileMeta {   // per streaming tile
    uint64_t head;  // products of its first row here, when that row began earlier
    uint64_t carry; // products of its last row here, when that row begins here and goes on
    uint64_t fsum;  // products of all its entries
    uint64_t pad;
};

// Workspace layout of one call (byte offsets, each 256-aligned).
struct Layout {
    size_t ctl, scratch, bin1, bin2, bin3, bin4, merge, tiles, meta, samp, rowtmp, total;
    int64_t cap13, cap4, cap5, ntiles;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int64_t flop_tiles(int64_t M, int64_t nnz)
{
    return (M + nnz + kFlopTile - 1) / kFlopTile;
}

inline Layout make_layout(int64_t nitems, int64_t M, int64_t nnzA, bool need_rowtmp)
{
    Layout L;
    L.cap13 = nitems > 0 ? nitems : 1;
    L.cap4 = L.cap13 + (int64_t)kMaxPartWindows;
    L.cap5 = (int64_t)kMaxPartWindows * (kWinWords / kMergeSlice) + 64;
    L.ntiles = flop_tiles(M, nnzA);
    size_t o = 0;
    L.ctl = o;     o = align256(o + sizeof(Ctl));
    L.scratch = o; o = align256(o + (size_t)kMaxPartWindows * kWinWords * sizeof(uint32_t));
    L.bin1 = o;    o = align256(o + (size_t)L.cap13 * sizeof(BinItem));
    L.bin2 = o;    o = align256(o + (size_t)L.cap13 * sizeof(BinItem));
    L.bin3 = o;    o = align256(o + (size_t)L.cap13 * sizeof(BinItem));
    L.bin4 = o;    o = align256(o + (size_t)L.cap4 * sizeof(BigItem));
    L.merge = o;   o = align256(o + (size_t)L.cap5 * sizeof(MergeItem));
    L.tiles = o;   o = align256(o + (size_t)(L.ntiles + 1) * sizeof(int32_t));
    L.meta = o;    o = align256(o + (size_t)(L.ntiles > 0 ? L.ntiles : 1) * sizeof(TileMeta));
    L.samp = o;    o = align256(o + (size_t)kSampleGroups * sizeof(SampleCounts));
    L.rowtmp = o;
    if (need_rowtmp) o = align256(o + (size_t)(M > 0 ? M : 1) * sizeof(int64_t));
    L.total = o;
    return L;
}

} // namespace ssp
