// Internal layout shared by the kernels and the host launch code.
#pragma once

#include <stdint.h>

#include "../../include/ssp.h"

namespace ssp {

// Row bins of the symbolic (distinct-count) kernels, by row FLOP.
//   bin 1: 1..128 products      -> one wave per row, LDS table <= 256 words
//   bin 2: 129..1024 products   -> 256 threads (or one wave) per row, LDS table <= 2048 words
//   bin 3: 1025..8192 products  -> 512 threads per row, LDS table <= 16384 words
//   bin 4: more                 -> 1024 threads, LDS bitmap per column window;
//                                  rows above kSplitTarget products are cut into
//                                  parts whose bitmaps a merge kernel ORs
// Defaults of the bin limits (tunable, see ssp_tuning); a bin's limit times
// the hash-table multiplier may not exceed its table (kBin*Words).
constexpr uint64_t kBin1Max = 128, kBin2Max = 1024, kBin3Max = 8192;
constexpr int kBin1Words = 256, kBin2Words = 2048, kBin3Words = 16384;
constexpr int kBin1Team = 64, kBin2Team = 256, kBin3Team = 512, kBin4Team = 1024;
// Bin 2 runs one wave per row instead of kBin2Team threads when a call
// expects at least this many sampled rows: many rows then keep the chip busy,
// and a wave needs no barriers; few rows want the shorter chain of a team.
constexpr int64_t kBin2WaveRows = 8192;

// Bin-4 bitmap window: at most 32768 words = 2^20 columns = 128 KiB of LDS.
constexpr int kWinWords = 32768;
constexpr uint64_t kSplitTarget = 1ull << 19; // products per part of a split row (default)
constexpr uint32_t kLongLenDefault = 16;      // B rows walked in units by the long-row kernel
constexpr int kMaxParts = 64;
// Global part bitmaps of kWinWords words: a call holds kPartWindowsBase, a
// batch kPartWindowsBase per 32 cases up to kPartWindowsMax.
constexpr int kPartWindowsBase = 1024;
constexpr int kPartWindowsMax = 8192;
constexpr int kMaxSplitWindows = 4;           // rows needing more windows are not split
constexpr int kMergeSlice = 1024;             // words per merge item

// Words of the long-row bitmap for `cols` columns: whole 64-word rows (the
// bitmap's words are swizzled inside their row).
__host__ __device__ inline int64_t bitmap_words(int64_t cols)
{
    return (cols + 2047) / 2048 * 64;
}

// Streaming FLOP kernels: 256 threads, tiles of kFlopTile merge-path items
// (rows + entries of A), at most kFlopTile + 3 < 2048 entries per tile.
constexpr int kFlopThreads = 256;
constexpr int kFlopChunk = 2048;
constexpr int64_t kFlopTile = 2040;
// A.A tiles whose columns lie within kNearRows of their rows gather B's row
// pointers (A's, just streamed) instead of the separate row lengths.
constexpr int64_t kNearRows = 1 << 15;

// Distinct counts (z*, or the exact total) are added by the symbolic kernels
// into kAccSlots slots per case, chosen by workgroup: atomics on one address
// serialise, atomics on distinct addresses do not.  k_finalize sums them.
constexpr int kAccSlots = 64;

// Device code sees the arrays of a case as global-memory pointers.  Read from
// the case table (itself in global memory) they would otherwise be generic to
// the compiler, which then emits flat accesses; a flat load counts against the
// LDS counter as well, so every wait for an LDS result would also wait for it.
// The host sees plain pointers of the same size.
#ifndef SSP_GLOBAL
#ifdef __HIP_DEVICE_COMPILE__
#define SSP_GLOBAL __attribute__((address_space(1)))
#else
#define SSP_GLOBAL
#endif
#endif

struct Csr {
    const SSP_GLOBAL int32_t* rpt;
    const SSP_GLOBAL int32_t* col;
    int64_t nrows, ncols, nnz;
};

// One product of a call (a batch holds several).  Written by the host before
// the launches; the kernels find their case from the workgroup prefixes
// (wg_*: the first workgroup of the case in each kernel's grid) or from the
// case index an item carries.
struct CaseDesc {
    Csr A, B;
    SSP_GLOBAL int64_t* out;  // per-row output (prediction, reference or exact counts)
    SSP_GLOBAL int64_t* rf;   // per-row FLOP (the caller's array or workspace)
    ssp_stats* st;       // statistics (the caller's, or the case's workspace slot)
    SSP_GLOBAL uint16_t* blen;  // B's row lengths saturated at 0xFFFF (workspace; null:
                                // the streaming kernel reads B's row pointers)
    uint64_t seed, thresh;
    int64_t ncand;       // sampling candidates: rows (Bernoulli) or draws (paper)
    int64_t tile_base;   // first global tile of this case (tiles numbered case after case)
    int64_t ntiles;      // merge-path tiles of A (0 when A has no rows)
    int64_t group_base;  // first sampling group of this case
    int64_t group_size;  // candidates per sampling group (a multiple of 256)
    int64_t ngroups;
    int32_t win_words;   // long-row bitmap window, words (a multiple of 4)
    int32_t nwin;        // windows covering B's columns
    int32_t big3;        // bin-3 rows go to the long-row kernel
    int32_t merge_per_row;  // merge items of one split row
    int32_t paper;       // the paper's fixed-count sampler
    int32_t wg_tiles, wg_rows;
    // tuning (the same for every case of a call)
    uint32_t bin_max[3];    // product limits of bins 1..3
    uint32_t hash_mult;     // hash tables hold at least hash_mult x the distinct bound
    uint32_t long_len;      // long-row kernel: B rows of at least this many columns go in units
    uint32_t blen_own;      // this case writes blen (cases of one B share the array)
    uint64_t split_target;  // products per part of a split long row
    uint64_t est_max_rf;    // prediction: rows of fewer products take the estimated ceiling
};

// Per-case results written by the kernels.
struct CaseRes {
    uint64_t zacc[kAccSlots];
    uint32_t fallback, pad0;       // reference design: 1 when f* = 0 (predict row FLOP)
    uint64_t ref_q_lo, ref_q_hi;   // reference design: z* M
    uint64_t ref_d_lo, ref_d_hi;   // reference design: n_s F
    uint64_t pad[8];
};

// Control block at the start of the workspace (device memory): the shared
// lists of a call and their counters.
struct Ctl {
    uint32_t bin_cnt[8];  // items in bins 1..4 (index = bin; bin 4: the heavy items),
                          // merge items at 5, light bin-4 items at 6
    uint32_t pw_ctr;      // part windows handed out (exact path)
    uint32_t big_next;    // work queue of the long-row kernel
    uint32_t split_level; // the call's split level (sampling passes)
    uint32_t num_abort;   // numeric product: rows whose first-pass table filled up
    uint32_t num_next[2]; // numeric product: work queues of the dense passes
    uint32_t pad[18];
};

struct BinItem {  // bins 1..3
    int32_t row;
    uint32_t rf;
    int32_t cs;     // case
    int32_t pad;
};

struct BigItem {  // bin 4: entries e_lo + part + k nparts < e_hi of one long row
    int32_t row;
    int32_t slot;   // first part window of a split row, -1 when not split
    int32_t part;   // part index of a split row (0 when not split)
    int32_t nparts;
    int32_t e_lo, e_hi;
    int32_t cs;     // case
    int32_t pad;
};

struct MergeItem {  // one slice of one window of a split row
    int32_t row;
    int32_t slot;
    int32_t nparts;
    int32_t window;
    int32_t slice;
    int32_t cs;     // case
};

// Split levels: a call splits its eligible long rows at split_target << L,
// L the smallest level whose part windows all fit the scratch (the last level
// when none does; then a group's rows are split while the windows requested up
// to and including the group fit).  Rows above a quarter of the level's
// target are heavy.
constexpr int kSplitLevels = 4;
constexpr int kHeavyShift = 2;

// Per-group counters of the sampling passes.  k_sample_count writes the
// counts, k_sample_scan the offsets (and turns ns, fs, as into inclusive
// prefixes over all groups of the call).
struct SampleCounts {
    uint32_t n1, n2, n3, n4;   // sampled rows in bins 1..3 and bin 4
    uint32_t cs;               // case
    uint32_t split;            // (scan) 1 if the group's eligible rows are split
    // per level: bin-4 items, part windows, merge items of the eligible rows
    // (when split), heavy rows
    uint32_t lv[kSplitLevels][4];
    uint32_t o1, o2, o3;       // (scan) offsets in bins 1..3
    uint32_t oh, ol;           // (scan) offsets among the heavy and the light bin-4 items
    uint32_t om, ow;           // (scan) offset in the merge list, first part window
    uint32_t gfirst, glast;    // first and last group of the case
    uint32_t pad;
    uint64_t ns, fs, as;       // sampled rows, their products, their A entries
};
constexpr int kSampleTarget = 8192; // sampling groups of a call, about (at least 1 per case)

struct TileMeta {   // per streaming tile
    uint64_t head;  // products of its first row here, when that row began earlier
    uint64_t carry; // products of its last row here, when that row begins here and goes on
    uint64_t fsum;  // products of all its entries
    uint64_t pad;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int64_t flop_tiles(int64_t M, int64_t nnz)
{
    const int64_t t = (M + nnz + kFlopTile - 1) / kFlopTile;
    return t > 0 ? t : 1;
}

} // namespace ssp
