// Internal layout shared by the kernels and the host launch code.
#pragma once

#include <stdint.h>

#include "../../include/ssp.h"

namespace ssp {

// Row bins of the symbolic (distinct-count) kernels, by row FLOP.
//   bin 1: 1..128 products      -> one wave per row, LDS table <= 256 words
//   bin 2: 129..1024 products   -> 256 threads per row, LDS table <= 2048 words
//   bin 3: 1025..8192 products  -> 512 threads per row, LDS table <= 16384 words
//   bin 4: more                 -> 1024 threads, LDS bitmap over column windows,
//                                  long rows split across workgroups
constexpr uint64_t kBin1Max = 128, kBin2Max = 1024, kBin3Max = 8192;
constexpr int kBin1Words = 256, kBin2Words = 2048, kBin3Words = 16384;
constexpr int kBin1Team = 64, kBin2Team = 256, kBin3Team = 512, kBin4Team = 1024;

// Bin-4 bitmap window: 32768 words = 2^20 columns = 128 KiB of LDS.
constexpr int kWinWords = 32768;
constexpr int64_t kWinCols = (int64_t)kWinWords * 32;
// A bin-4 row with more products than kSplitTarget is cut into up to
// kMaxParts workgroups that merge their bitmaps in a global slot.
constexpr uint64_t kSplitTarget = 1ull << 16;
constexpr int kMaxParts = 64;
constexpr int kMaxSlots = 64;
constexpr int kSlotWindows = 4; // rows needing more windows are not split
constexpr int64_t kSlotWords = (int64_t)kSlotWindows * kWinWords + 64;

// Rows per tile of the streaming FLOP kernels (256 threads per tile).
constexpr int kFlopThreads = 256;
constexpr int kFlopChunk = 2048;

// Control block at the start of the workspace (device memory).
struct Ctl {
    ssp_stats stats;      // used when the caller passes no stats pointer
    uint32_t bin_cnt[8];  // items in bins 1..4 (index = bin)
    uint32_t slot_ctr;    // global bitmap slots handed out
    uint32_t fallback;    // 1: f* = 0, predict row FLOP
    uint32_t pad0[6];
    uint64_t div_dn, div_v; // Divisor of f*
    uint32_t div_shift, pad1;
    uint64_t ref_q_lo, ref_q_hi; // reference design: z* M
    uint64_t ref_d_lo, ref_d_hi; // reference design: n_s F
    uint64_t pad2[16];
};

struct BinItem {  // bins 1..3
    int32_t row;
    uint32_t rf;
};

struct BigItem {  // bin 4: one product range of one long row
    int32_t row;
    int32_t slot;   // global merge slot, -1 when the row is not split
    int32_t part;   // this item covers products [part, part+1) * rf / nparts
    int32_t nparts;
    uint64_t rf;    // products of the row
};

// Workspace layout of one call (byte offsets, each 256-aligned).
struct Layout {
    size_t ctl, bin1, bin2, bin3, bin4, slots, rowtmp, total;
    int64_t cap13, cap4;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline Layout make_layout(int64_t nitems, int64_t M, bool need_rowtmp)
{
    Layout L;
    L.cap13 = nitems > 0 ? nitems : 1;
    L.cap4 = L.cap13 + (int64_t)kMaxSlots * kMaxParts;
    size_t o = 0;
    // the slot region sits at a fixed offset: it is zero between calls (the
    // kernels that use a slot clear it again), whatever the other sizes are
    L.ctl = o;   o = align256(o + sizeof(Ctl));
    L.slots = o; o = align256(o + (size_t)kMaxSlots * kSlotWords * sizeof(uint32_t));
    L.bin1 = o;  o = align256(o + (size_t)L.cap13 * sizeof(BinItem));
    L.bin2 = o;  o = align256(o + (size_t)L.cap13 * sizeof(BinItem));
    L.bin3 = o;  o = align256(o + (size_t)L.cap13 * sizeof(BinItem));
    L.bin4 = o;  o = align256(o + (size_t)L.cap4 * sizeof(BigItem));
    L.rowtmp = o;
    if (need_rowtmp) o = align256(o + (size_t)(M > 0 ? M : 1) * sizeof(int64_t));
    L.total = o;
    return L;
}

} // namespace ssp
