// HIP kernels of the prediction path for gfx950 (wave64).
//
// A call predicts one product or a batch of them (cases).  Launch order:
//   k_setup            clear counters, per-case results and statistics; the
//                      case table of small calls; merge-path tile starts
//   k_flop, k_flop_fixup
//                      products of every row (a pattern SpMV with the row
//                      lengths of B) into rf, and F
//   k_sample_count / _scan / _write
//                      the sampled rows (splitmix64), f*, n_s, and their bins
//                      (no scan launch for calls of few sampling groups)
//   k_sym, k_sym_big   exact distinct-column count of every binned row (LDS hash
//                      table or LDS bitmap); long rows are cut into parts that
//                      leave their bitmaps in global scratch
//   k_sym_merge        ORs the parts' bitmaps
//   k_pred_rows        z* per case, the empty-sample fallback and the per-row
//                      prediction
//   (exact structure and reference design: k_finalize, k_finalize_reference,
//   k_ref_rows)
// Kernels whose workgroups each serve one case find it by a binary search of
// the per-case workgroup prefixes; items of the shared bins carry their case.
#pragma once

#include "ssp_device.hpp"
#include "ssp_internal.hpp"

namespace ssp {

struct BinLists {
    BinItem* b1;
    BinItem* b2;
    BinItem* b3;
    BigItem* b4;
    MergeItem* merge;
    uint32_t* scratch; // part_windows windows of kWinWords words
    // Bin 4 holds its heavy items from the front (parts of split rows, and
    // rows above a quarter of the split target) and the light ones from the
    // back (light item i at cap4 - 1 - i): the long-row kernel takes the
    // heavy ones first, so the last items taken are short.
    uint32_t cap4;
    uint32_t part_windows;  // windows in scratch (the call's budget of split-row parts)
};

// Queue position k of the long-row kernel -> bin-4 list index, given the
// count of heavy items.
__device__ __forceinline__ uint32_t big_index(uint32_t k, uint32_t nheavy, uint32_t cap4)
{
    return k < nheavy ? k : cap4 - 1u - (k - nheavy);
}

// The case of workgroup `wg` in a grid whose workgroups serve one case each:
// the last case whose first workgroup (field F) is at or before wg.
template <int32_t CaseDesc::*F>
__device__ __forceinline__ int case_of_wg(const CaseDesc* __restrict__ cs, int n, int32_t wg)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cs[mid].*F <= wg) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Workgroups of case c in that grid (of `total` workgroups, the launch's
// grid by default).
template <int32_t CaseDesc::*F>
__device__ __forceinline__ int32_t wgs_of_case(const CaseDesc* __restrict__ cs, int n, int c,
                                               int32_t total = -1)
{
    const int32_t end = total >= 0 ? total : (int32_t)gridDim.x;
    return (c + 1 < n ? cs[c + 1].*F : end) - cs[c].*F;
}

typedef unsigned long long ull;

// A wave-uniform 64-bit value in scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ ull* as_ull(uint64_t* p) { return reinterpret_cast<ull*>(p); }

// ---------------------------------------------------------------- init

// Calls of at most kArgCases cases pass the case table in the kernel
// arguments of k_setup, which writes it to the workspace (kernel arguments are
// captured at launch, so the host buffer is free at once and no copy is
// queued on the stream).
constexpr int kArgCases = 8;
struct CaseArgs {
    CaseDesc d[kArgCases];
};

// ------------------------------------------------------------- binning

__device__ __forceinline__ int bin_of(uint64_t rf, const uint32_t (&lim)[3])
{
    return rf == 0 ? 0 : rf <= lim[0] ? 1 : rf <= lim[1] ? 2 : rf <= lim[2] ? 3 : 4;
}

// Bin of a row for the kernels: bin-3 rows go to the long-row kernel when all
// N columns fit one LDS bitmap window but not bin 3's table as a bitmap (bin 3
// would hash); the bitmap kernel then counts them far faster.
__device__ __forceinline__ int bin_route(uint64_t rf, const CaseDesc& cd)
{
    const int b = bin_of(rf, cd.bin_max);
    return (b == 3 && cd.big3) ? 4 : b;
}

// Merge items of a split row: one per (window, slice of kMergeSlice words).
__device__ inline void write_merge_items(MergeItem* dst, int32_t row, int32_t slot, int32_t nparts,
                                         int32_t ci, const CaseDesc& cd)
{
    const int64_t N = cd.B.ncols, wcols_full = (int64_t)cd.win_words * 32;
    int k = 0;
    for (int w = 0; w < cd.nwin; ++w) {
        const int64_t cols = (N - w * wcols_full) < wcols_full ? (N - w * wcols_full) : wcols_full;
        const int slices = (int)((bitmap_words(cols) + kMergeSlice - 1) / kMergeSlice);
        for (int sl = 0; sl < slices; ++sl) {
            MergeItem m;
            m.row = row;
            m.slot = slot;
            m.nparts = nparts;
            m.window = w;
            m.slice = sl;
            m.cs = ci;
            dst[k++] = m;
        }
    }
}

// Bin-4 items of one long row (single lane; the exact path, which appends
// with atomics).  A row above the split target, or with more entries than one
// chunk of the long-row kernel's workgroup, is cut into P parts (the split
// rule of the sampled path, split_info) when enough global part windows are
// left; part p takes the entries e0 + p,
// e0 + p + P, e0 + p + 2P, ...  In skewed rows the heavy entries (hub
// columns, long B rows) sit together, and a stride deals them out evenly, so
// the parts get near-equal product counts without a scan of the row.
// Unsplit rows are one part (P = 1).
__device__ inline void append_big(int32_t row, uint64_t rf, int32_t e0, int32_t e1, int32_t ci,
                                  const CaseDesc& cd, Ctl* ctl, const BinLists& L)
{
    const int64_t alen = (int64_t)e1 - e0;
    int32_t nparts = 1, slot = -1;
    const uint64_t T = cd.split_target;
    const uint64_t chunks = (uint64_t)((alen + kBin4Team - 1) / kBin4Team);
    if ((rf > T || chunks > 1) && cd.nwin <= kMaxSplitWindows && alen > 1 &&
        __hip_atomic_load(&ctl->pw_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
            L.part_windows) {  // (bounds the counter: it cannot wrap)
        uint64_t want = (rf + T - 1) / T;
        if (want < chunks) want = chunks;
        if (want > (uint64_t)kMaxParts) want = kMaxParts;
        if (want > (uint64_t)alen) want = (uint64_t)alen;
        const uint32_t need = (uint32_t)want * (uint32_t)cd.nwin;
        const uint32_t s = atomicAdd(&ctl->pw_ctr, need);
        if (s + need <= L.part_windows) {
            slot = (int32_t)s;
            nparts = (int32_t)want;
        }
    }
    const bool heavy = nparts > 1 || rf > (T >> kHeavyShift);
    const uint32_t base = heavy ? atomicAdd(&ctl->bin_cnt[4], (uint32_t)nparts)
                                : L.cap4 - 1u - atomicAdd(&ctl->bin_cnt[6], 1u);
    for (int32_t p = 0; p < nparts; ++p) {
        BigItem it;
        it.row = row;
        it.slot = slot;
        it.part = p;
        it.nparts = nparts;
        it.e_lo = e0;
        it.e_hi = e1;
        it.cs = ci;
        it.pad = 0;
        L.b4[base + p] = it;
    }
    if (slot >= 0) {
        const uint32_t mb = atomicAdd(&ctl->bin_cnt[5], (uint32_t)cd.merge_per_row);
        write_merge_items(L.merge + mb, row, slot, nparts, ci, cd);
    }
}

// Bins 1..3 of a wave's rows with one atomic per wave and bin (every lane
// calls it; b = 0 for lanes with nothing to append).
__device__ __forceinline__ void append_small_bins(int b, int32_t row, uint64_t rf, int32_t ci,
                                                  Ctl* ctl, const BinLists& L)
{
    const int lane = lane_id();
#pragma unroll
    for (int bb = 1; bb <= 3; ++bb) {
        const uint64_t m = __ballot(b == bb);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t pos = 0;
            if (lane == leader) pos = atomicAdd(&ctl->bin_cnt[bb], (uint32_t)__popcll(m));
            pos = __shfl(pos, leader, kWave);
            if (b == bb) {
                BinItem it;
                it.row = row;
                it.rf = (uint32_t)rf;
                it.cs = ci;
                it.pad = 0;
                (bb == 1 ? L.b1 : bb == 2 ? L.b2 : L.b3)[pos + rank_in(m)] = it;
            }
        }
    }
}

// The same over a whole workgroup of NT threads (every thread calls it): the
// three bins' counts are scanned in one pass (21-bit fields of one 64-bit
// value) and each bin's counter takes one atomic for the workgroup, from
// lanes 1..3 in parallel.  `sm` needs NT/64 entries, `s_base` 4.
template <int NT>
__device__ __forceinline__ void block_append_small_bins(int b, int32_t row, uint64_t rf, int32_t ci,
                                                        Ctl* ctl, const BinLists& L, uint64_t* sm,
                                                        uint32_t* s_base)
{
    const uint64_t flag = b == 1 ? 1ull : b == 2 ? (1ull << 21) : b == 3 ? (1ull << 42) : 0ull;
    uint64_t tot;
    const uint64_t pre = block_excl_scan<NT, uint64_t>(flag, sm, &tot);
    const int t = threadIdx.x;
    if (t >= 1 && t <= 3) {
        const uint32_t n = (uint32_t)((tot >> (21 * (t - 1))) & 0x1FFFFFu);
        s_base[t] = n ? atomicAdd(&ctl->bin_cnt[t], n) : 0u;
    }
    __syncthreads();
    if (b >= 1 && b <= 3) {
        BinItem it;
        it.row = row;
        it.rf = (uint32_t)rf;
        it.cs = ci;
        it.pad = 0;
        const uint32_t pos = s_base[b] + (uint32_t)((pre >> (21 * (b - 1))) & 0x1FFFFFu);
        (b == 1 ? L.b1 : b == 2 ? L.b2 : L.b3)[pos] = it;
    }
    __syncthreads();  // (s_base is rewritten by the next call)
}

// One row, appended by a single lane.
__device__ inline void append_row(int32_t row, uint64_t rf, int32_t e0, int32_t e1, int32_t ci,
                                  const CaseDesc& cd, Ctl* ctl, const BinLists& L)
{
    const int b = bin_route(rf, cd);
    if (b == 0) return;
    if (b == 4) {
        append_big(row, rf, e0, e1, ci, cd, ctl, L);
        return;
    }
    BinItem it;
    it.row = row;
    it.rf = (uint32_t)rf;
    it.cs = ci;
    it.pad = 0;
    const uint32_t i = atomicAdd(&ctl->bin_cnt[b], 1u);
    (b == 1 ? L.b1 : b == 2 ? L.b2 : L.b3)[i] = it;
}

// ------------------------------------------------------------ tiles

// Merge-path partition of the streaming FLOP pass: tile b of a case starts in
// row g when its first item b * kFlopTile lies in [rpt[g] + g, rpt[g+1] + g + 1),
// the span of row g's entries and end marker.  Writes the start row and the
// case of every global tile (tiles numbered case after case); `wg` is this
// workgroup's index in a tile grid of G_all workgroups (256 threads each).
__device__ __forceinline__ void tile_starts(const CaseDesc* __restrict__ tab, int n, int32_t wg,
                                            int32_t G_all, int32_t* __restrict__ tile_row,
                                            int32_t* __restrict__ tile_case)
{
    const int c = case_of_wg<&CaseDesc::wg_tiles>(tab, n, wg);
    const int64_t bl = (int64_t)wg - tab[c].wg_tiles;
    const int64_t G = wgs_of_case<&CaseDesc::wg_tiles>(tab, n, c, G_all);
    const Csr A = tab[c].A;
    const int64_t M = A.nrows, ntiles = tab[c].ntiles, base = tab[c].tile_base;
    const int64_t stride = G * 256;
    for (int64_t g = bl * 256 + threadIdx.x; g < M; g += stride) {
        const int64_t f0 = (int64_t)A.rpt[g] + g, f1 = (int64_t)A.rpt[g + 1] + g + 1;
        for (int64_t b = (f0 + kFlopTile - 1) / kFlopTile; b * kFlopTile < f1 && b < ntiles; ++b) {
            tile_row[base + b] = (int32_t)g;
            tile_case[base + b] = c;
        }
    }
    // B's row lengths in two bytes each (saturated): the streaming pass
    // gathers them instead of pairs of row pointers, a quarter of the bytes,
    // so they stay in L2 (a million rows: 2 MiB against 8)
    SSP_GLOBAL uint16_t* const blen = tab[c].blen;
    if (blen && tab[c].blen_own) {
        const Csr B = tab[c].B;
        for (int64_t k = bl * 256 + threadIdx.x; k < B.nrows; k += stride) {
            const int32_t l = B.rpt[k + 1] - B.rpt[k];
            blen[k] = (uint16_t)(l < 0xFFFF ? l : 0xFFFF);
        }
    }
}

// The first kernel of a call: workgroups [0, ninit) clear the cases' results,
// statistics and the control block (and with ARGS write the case table from
// the kernel arguments, for calls of at most kArgCases cases); the others
// write the merge-path tile starts (reading the case table from the kernel
// arguments with ARGS, else from the workspace, where the host copied it).
template <bool ARGS>
__global__ __launch_bounds__(256) void k_setup(Ctl* ctl, CaseDesc* __restrict__ cs,
                                              CaseRes* __restrict__ cr, int n, int ninit,
                                              int32_t* __restrict__ tile_row,
                                              int32_t* __restrict__ tile_case, CaseArgs args)
{
    const int t = threadIdx.x;
    if ((int)blockIdx.x >= ninit) {
        tile_starts(ARGS ? args.d : cs, n, (int32_t)blockIdx.x - ninit,
                    (int32_t)gridDim.x - ninit, tile_row, tile_case);
        return;
    }
    if (blockIdx.x == 0 && t < (int)(sizeof(Ctl) / 4)) reinterpret_cast<uint32_t*>(ctl)[t] = 0;
    for (int c = blockIdx.x; c < n; c += ninit) {
        const CaseDesc& d = ARGS ? args.d[c] : cs[c];
        if (ARGS) {
            static_assert(sizeof(CaseDesc) % 8 == 0, "copied as 64-bit words");
            const uint64_t* src = reinterpret_cast<const uint64_t*>(&args.d[c]);
            uint64_t* dst = reinterpret_cast<uint64_t*>(&cs[c]);
            for (int i = t; i < (int)(sizeof(CaseDesc) / 8); i += 256) dst[i] = src[i];
        }
        uint64_t* r = reinterpret_cast<uint64_t*>(&cr[c]);
        for (int i = t; i < (int)(sizeof(CaseRes) / 8); i += 256) r[i] = 0;
        if (t == 0) {
            ssp_stats* st = d.st;
            st->total_flop = 0;
            st->n_sampled = 0;
            st->sample_flop = 0;
            st->sample_nnz = 0;
            st->out_sum = 0;
            st->nrows = (uint64_t)d.A.nrows;
            st->flags = 0;
            st->a_sample_nnz = 0;
        }
    }
}

// --------------------------------------------------------- sampling

constexpr int kSampleThreads = 256;

// Sampler parameters of a case, in registers.
struct SamplerArgs {
    Csr A;
    const SSP_GLOBAL int64_t* rf;
    uint64_t seed, thresh;
    int64_t ncand;
    int32_t paper, nwin, big3, merge_per_row;
    uint32_t bin_max[3];
    uint64_t split_target;
};

__device__ __forceinline__ SamplerArgs sampler_args(const CaseDesc& cd)
{
    SamplerArgs a;
    a.A = cd.A;
    a.rf = cd.rf;
    a.seed = cd.seed;
    a.thresh = cd.thresh;
    a.ncand = cd.ncand;
    a.paper = cd.paper;
    a.nwin = cd.nwin;
    a.big3 = cd.big3;
    a.merge_per_row = cd.merge_per_row;
    a.bin_max[0] = cd.bin_max[0];
    a.bin_max[1] = cd.bin_max[1];
    a.bin_max[2] = cd.bin_max[2];
    a.split_target = cd.split_target;
    return a;
}

// Candidate i of a sampler: row i for the Bernoulli sampler (kept when the
// top 53 bits of splitmix64(seed, i) fall below the threshold), the i-th draw
// for the paper's (row floor(M u / 2^53) of the draw's top 53 bits u).
// Returns -1 for a candidate that is not sampled.
__device__ __forceinline__ int64_t candidate_row(int64_t i, const SamplerArgs& a)
{
    const uint64_t x = splitmix64_at(a.seed, (uint64_t)i) >> 11;
    if (a.paper) {
        const u128 p = mul_64x64((uint64_t)a.A.nrows, x);
        return (int64_t)((p.lo >> 53) | (p.hi << 11));
    }
    return x < a.thresh ? i : -1;
}

// What a sampled row contributes to the lists: its bin, and for bin 4
// whether it may be split and into how many parts.
struct SampledRow {
    int64_t g;
    uint64_t rf;
    int32_t e0, e1;
    int bin;
};

__device__ __forceinline__ SampledRow classify_row(int64_t g, const SamplerArgs& a)
{
    SampledRow r;
    r.g = g;
    r.rf = 0;
    r.e0 = r.e1 = 0;
    r.bin = 0;
    if (g < 0) return r;
    r.rf = (uint64_t)a.rf[g];
    r.e0 = a.A.rpt[g];
    r.e1 = a.A.rpt[g + 1];
    const int b = bin_of(r.rf, a.bin_max);
    r.bin = (b == 3 && a.big3) ? 4 : b;
    return r;
}

// How a bin-4 row splits at split level `lv`: eligible rows (above the
// level's target or with more entries than one chunk of the long-row
// kernel's workgroup, windows few enough, at least two entries) want one
// part per target's worth of products and at least one per chunk of
// entries (the chunks of one item run one after another), at most kMaxParts
// and one per entry; eligible rows and rows above a quarter of the target
// are heavy (a row's parts are written to the heavy list together).
struct SplitInfo {
    uint32_t want;  // parts when split (1 unless eligible)
    bool elig, heavy;
};

__device__ __forceinline__ SplitInfo split_info(const SampledRow& r, const SamplerArgs& a, int lv)
{
    SplitInfo si{1u, false, false};
    if (r.bin != 4) return si;
    const uint64_t T = a.split_target << lv;
    si.heavy = r.rf > (T >> kHeavyShift);
    const int64_t alen = (int64_t)r.e1 - r.e0;
    const uint64_t chunks = (uint64_t)((alen + kBin4Team - 1) / kBin4Team);
    if ((r.rf > T || chunks > 1) && a.nwin <= kMaxSplitWindows && alen > 1) {
        uint64_t want = (r.rf + T - 1) / T;
        if (want < chunks) want = chunks;
        if (want > (uint64_t)kMaxParts) want = kMaxParts;
        if (want > (uint64_t)alen) want = (uint64_t)alen;
        si.want = (uint32_t)want;
        si.elig = true;
        si.heavy = true;  // (the parts of a row go to the heavy list together)
    }
    return si;
}

// The case of sampling group `grp` (groups of a case are consecutive) and
// its candidates [lo, hi).
struct GroupRange {
    int c;
    int64_t lo, hi;
};

__device__ __forceinline__ GroupRange group_range(const CaseDesc* __restrict__ cs, int n,
                                                  int64_t grp)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cs[mid].group_base <= grp) lo = mid;
        else hi = mid;
    }
    GroupRange r;
    r.c = lo;
    const int64_t k = grp - cs[lo].group_base, C = cs[lo].group_size, nc = cs[lo].ncand;
    r.lo = k * C;
    r.hi = (r.lo + C) < nc ? (r.lo + C) : nc;
    return r;
}

// The sampled rows of a group, a round of NT * kCandPerThread candidates at a
// time, in candidate order: thread t draws candidates base + 8t .. base + 8t
// + 7 and a workgroup scan places the sampled ones in `rows` (LDS).  With a
// sparse sample a round yields few rows, and the per-row work of the passes
// (scans included) runs over those, not over every candidate.  Returns the
// count (uniform); ends with a barrier.
constexpr int kCandPerThread = 8;
template <int NT>
__device__ __forceinline__ int gather_sampled(int64_t base, int64_t hi, const SamplerArgs& a,
                                              int64_t* rows, uint64_t* s_red)
{
    int64_t g[kCandPerThread];
    uint32_t n = 0;
#pragma unroll
    for (int u = 0; u < kCandPerThread; ++u) {
        const int64_t i = base + (int64_t)threadIdx.x * kCandPerThread + u;
        g[u] = i < hi ? candidate_row(i, a) : -1;
        n += g[u] >= 0 ? 1u : 0u;
    }
    uint64_t tot;
    uint32_t pos = (uint32_t)block_excl_scan<NT, uint64_t>(n, s_red, &tot);
#pragma unroll
    for (int u = 0; u < kCandPerThread; ++u)
        if (g[u] >= 0) rows[pos++] = g[u];
    __syncthreads();
    return (int)tot;
}

// Pass 1: per group, the counts of SampleCounts (at every split level) and
// the sums of n_s, f* and the sample's A entries.  No atomics: the passes
// hand over per-group counters (same-address device atomics serialise on
// this part).
__global__ __launch_bounds__(kSampleThreads) void k_sample_count(const CaseDesc* __restrict__ cs,
                                                                int n,
                                                                SampleCounts* __restrict__ cnt)
{
    constexpr int NT = kSampleThreads, NC = 4 + 4 * kSplitLevels;
    __shared__ uint64_t s_red[NT / kWave + 1];
    __shared__ uint32_t s_tot[NT / kWave][NC];
    __shared__ int64_t s_rows[NT * kCandPerThread];
    const GroupRange gr = group_range(cs, n, blockIdx.x);
    const SamplerArgs a = sampler_args(cs[gr.c]);
    // c[0..3]: rows of bins 1..4; c[4 + 4 lv + j]: SampleCounts::lv[lv][j]
    uint32_t c[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) c[k] = 0;
    uint64_t ns = 0, fs = 0, as = 0;
    for (int64_t base = gr.lo; base < gr.hi; base += NT * kCandPerThread) {
        const int nr = gather_sampled<NT>(base, gr.hi, a, s_rows, s_red);
        for (int k = threadIdx.x; k < nr; k += NT) {
            const SampledRow r = classify_row(s_rows[k], a);
            ns += 1;
            fs += r.rf;
            as += (uint64_t)(r.e1 - r.e0);
            c[0] += r.bin == 1;  // (selects, not an index: c stays in registers)
            c[1] += r.bin == 2;
            c[2] += r.bin == 3;
            c[3] += r.bin == 4;
#pragma unroll
            for (int lv = 0; lv < kSplitLevels; ++lv) {
                const SplitInfo si = split_info(r, a, lv);
                c[4 + 4 * lv + 0] += r.bin == 4 ? si.want : 0u;
                c[4 + 4 * lv + 1] += si.elig ? si.want * (uint32_t)a.nwin : 0u;
                c[4 + 4 * lv + 2] += si.elig ? (uint32_t)a.merge_per_row : 0u;
                c[4 + 4 * lv + 3] += si.heavy ? 1u : 0u;
            }
        }
    }
    // the NC counts: wave sums, then one barrier and a column sum per count
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const uint32_t v = wave_sum(c[k]);
        if (lane_id() == 0) s_tot[wid][k] = v;
    }
    const uint64_t Ns = block_sum<NT, uint64_t>(ns, s_red);  // (its barrier covers s_tot)
    const uint64_t Fs = block_sum<NT, uint64_t>(fs, s_red);
    const uint64_t As = block_sum<NT, uint64_t>(as, s_red);
    SampleCounts* o = &cnt[blockIdx.x];
    if (threadIdx.x < NC) {
        uint32_t v = 0;
#pragma unroll
        for (int w = 0; w < NT / kWave; ++w) v += s_tot[w][threadIdx.x];
        const int k = threadIdx.x;
        if (k == 0) o->n1 = v;
        else if (k == 1) o->n2 = v;
        else if (k == 2) o->n3 = v;
        else if (k == 3) o->n4 = v;
        else o->lv[(k - 4) / 4][(k - 4) % 4] = v;
    }
    if (threadIdx.x == 0) {
        o->cs = (uint32_t)gr.c;
        o->gfirst = (uint32_t)cs[gr.c].group_base;
        o->glast = (uint32_t)(cs[gr.c].group_base + cs[gr.c].ngroups - 1);
        o->ns = Ns;
        o->fs = Fs;
        o->as = As;
    }
}

// Pass 2, one workgroup, the groups taken kScanThreads at a time.  First the
// call's split level: the part windows every level requests over all groups;
// the smallest level whose windows fit the scratch.  Then the exclusive
// offsets of every group in every list at that level, the split decision (a
// group's eligible rows are split when all part windows requested up to and
// including the group fit the scratch), the list sizes, and per case n_s, f*
// and the sample's A entries (one atomic per case and chunk of groups).  The
// first chunk's records are read with the first pass, the scans of a chunk go
// in two rounds (the second depends on the split decision) of one barrier
// pair each, and the records carry what the scan would otherwise look up in
// the case table (merge items, the case's groups).
constexpr int kScanThreads = 1024;

struct GroupRec {  // the counts of SampleCounts (k_sample_count's output)
    uint32_t n1, n2, n3, n4, cs, gfirst, glast;
    uint32_t lv[kSplitLevels][4];
    uint64_t ns, fs, as;
};

__device__ __forceinline__ GroupRec load_group(const SampleCounts* __restrict__ cnt, int64_t g,
                                               int64_t ngroups)
{
    GroupRec x{};
    if (g < ngroups) {
        const SampleCounts& y = cnt[g];
        x.n1 = y.n1;
        x.n2 = y.n2;
        x.n3 = y.n3;
        x.n4 = y.n4;
        x.cs = y.cs;
        x.gfirst = y.gfirst;
        x.glast = y.glast;
#pragma unroll
        for (int lv = 0; lv < kSplitLevels; ++lv)
#pragma unroll
            for (int j = 0; j < 4; ++j) x.lv[lv][j] = y.lv[lv][j];
        x.ns = y.ns;
        x.fs = y.fs;
        x.as = y.as;
    }
    return x;
}

// Offsets of one group in the lists (k_sample_scan's per-group output).
struct GroupOff {
    uint32_t o1, o2, o3, oh, ol, om, ow, split;
};

// The scan of pass 2 by one workgroup of NT threads.  all: every chunk of
// groups, with the statistics atomics and the list sizes; else only the chunks
// up to group gt's.  WRITE: every group's offsets stored in its record.  Group
// gt's offsets (gt >= 0) land in *s_go before the routine's last barrier.
// Returns the split level (every thread).  s_red: 5 NT/64 entries.
template <int NT, bool WRITE>
__device__ __forceinline__ int scan_groups(SampleCounts* __restrict__ cnt, int64_t ngroups,
                                           const CaseDesc* __restrict__ cs, Ctl* ctl,
                                           uint32_t budget, bool all, int64_t gt,
                                           uint64_t* s_red, uint64_t (*s_e)[NT], GroupOff* s_go)
{
    const int t = threadIdx.x;
    const GroupRec r0 = load_group(cnt, t, ngroups);
    uint64_t wsum[kSplitLevels];
#pragma unroll
    for (int lv = 0; lv < kSplitLevels; ++lv) wsum[lv] = r0.lv[lv][1];
    for (int64_t g = t + NT; g < ngroups; g += NT) {
#pragma unroll
        for (int lv = 0; lv < kSplitLevels; ++lv) wsum[lv] += cnt[g].lv[lv][1];
    }
    uint64_t wex[kSplitLevels], wtot[kSplitLevels];
    block_excl_scan_n<NT, kSplitLevels>(wsum, s_red, wex, wtot);
    int L = kSplitLevels - 1;
#pragma unroll
    for (int lv = kSplitLevels - 1; lv >= 0; --lv)
        if (uniform_u64(wtot[lv]) <= (uint64_t)budget) L = lv;
    uint64_t k01 = 0, k2w = 0, k4 = 0, km = 0;  // carries (k01, k2w, k4: two u32 fields)
    for (int64_t g0 = 0; g0 < ngroups && (all || g0 <= gt); g0 += NT) {
        const int64_t g = g0 + t;
        const GroupRec x = g0 == 0 ? r0 : load_group(cnt, g, ngroups);
        ssp_stats* const st = cs[x.cs].st;  // (issued now, used after the scans)
        // level L's counts (selected: the level is dynamic, an indexed
        // register array would live in scratch)
        uint32_t items = 0, wins = 0, me = 0, nh = 0;
#pragma unroll
        for (int lv = 0; lv < kSplitLevels; ++lv) {
            if (lv == L) {
                items = x.lv[lv][0];
                wins = x.lv[lv][1];
                me = x.lv[lv][2];
                nh = x.lv[lv][3];
            }
        }
        const uint64_t va[5] = {(uint64_t)x.n1 | ((uint64_t)x.n2 << 32),
                                (uint64_t)x.n3 | ((uint64_t)clamp_windows(wins, budget) << 32),
                                x.ns, x.fs, x.as};
        uint64_t ea[5], ta[5];
        block_excl_scan_n<NT, 5>(va, s_red, ea, ta);
        const uint64_t p01 = k01 + ea[0], p2w = k2w + ea[1];
        const uint64_t ens = ea[2], efs = ea[3], eas = ea[4];
        const uint32_t wpre = (uint32_t)(p2w >> 32);
        const bool split = wins != 0 && (uint64_t)wpre + wins <= (uint64_t)budget;
        // bin 4: heavy items (front: parts of split rows, heavy unsplit rows)
        // and light rows (back); eligible rows are heavy
        const uint32_t nf = split ? items - x.n4 + nh : nh;
        const uint32_t nb = x.n4 - nh;
        const uint32_t nm = split ? me : 0u;
        const uint64_t vb[2] = {(uint64_t)nf | ((uint64_t)nb << 32), (uint64_t)nm};
        uint64_t eb[2], tb[2];
        block_excl_scan_n<NT, 2>(vb, s_red, eb, tb);
        const uint64_t p4 = k4 + eb[0], pm = km + eb[1];
        s_e[0][t] = ens;
        s_e[1][t] = efs;
        s_e[2][t] = eas;
        __syncthreads();
        if (g < ngroups) {
            GroupOff go;
            go.o1 = (uint32_t)p01;
            go.o2 = (uint32_t)(p01 >> 32);
            go.o3 = (uint32_t)p2w;
            go.oh = (uint32_t)p4;
            go.ol = (uint32_t)(p4 >> 32);
            go.om = (uint32_t)pm;
            go.ow = wpre;
            go.split = split ? 1u : 0u;
            if (WRITE) {
                SampleCounts* o = &cnt[g];
                o->o1 = go.o1;
                o->o2 = go.o2;
                o->o3 = go.o3;
                o->oh = go.oh;
                o->ol = go.ol;
                o->om = go.om;
                o->ow = go.ow;
                o->split = go.split;
            }
            if (g == gt) *s_go = go;
            // the last group of its case in this chunk adds the case's part
            const int64_t first = x.gfirst, last = x.glast;
            if (all && (g == last || t == NT - 1 || g == ngroups - 1)) {
                const int k0 = first > g0 ? (int)(first - g0) : 0;
                const uint64_t dns = ens + x.ns - s_e[0][k0];
                const uint64_t dfs = efs + x.fs - s_e[1][k0];
                const uint64_t das = eas + x.as - s_e[2][k0];
                if (dns) atomicAdd(as_ull(&st->n_sampled), (ull)dns);
                if (dfs) atomicAdd(as_ull(&st->sample_flop), (ull)dfs);
                if (das) atomicAdd(as_ull(&st->a_sample_nnz), (ull)das);
            }
        }
        __syncthreads();  // s_e is rewritten by the next chunk
        k01 += ta[0];
        k2w = saturate_windows_hi(k2w + ta[1], budget);
        k4 += tb[0];
        km += tb[1];
    }
    if (all && t == 0) {
        ctl->bin_cnt[1] = (uint32_t)k01;
        ctl->bin_cnt[2] = (uint32_t)(k01 >> 32);
        ctl->bin_cnt[3] = (uint32_t)k2w;
        ctl->bin_cnt[4] = (uint32_t)k4;
        ctl->bin_cnt[5] = (uint32_t)km;
        ctl->bin_cnt[6] = (uint32_t)(k4 >> 32);
        ctl->split_level = (uint32_t)L;
    }
    return L;
}

__global__ __launch_bounds__(kScanThreads) void k_sample_scan(SampleCounts* __restrict__ cnt,
                                                             int64_t ngroups,
                                                             const CaseDesc* __restrict__ cs,
                                                             Ctl* ctl, uint32_t budget)
{
    constexpr int NT = kScanThreads;
    __shared__ uint64_t s_red[5 * (NT / kWave)];
    __shared__ uint64_t s_e[3][NT];  // exclusive prefixes of ns, fs, as in the chunk
    (void)scan_groups<NT, true>(cnt, ngroups, cs, ctl, budget, true, -1, s_red, s_e, nullptr);
}

// Pass 3: every group regenerates its candidates and writes its rows at its
// offsets (positions inside the group by workgroup scans, in candidate order).
// FUSED (calls of at most kFusedScanGroups groups, one chunk of the scan):
// pass 2 is not launched; every workgroup runs the scan itself, and
// workgroup 0 also adds the statistics and sets the list sizes.  Timed: a
// call of one group 0.047 -> 0.044 ms; with 512 groups (two chunks) no faster
// than the separate pass, with 1024 twice as slow (every workgroup scans).
constexpr int64_t kFusedScanGroups = kSampleThreads;

template <bool FUSED>
__global__ __launch_bounds__(kSampleThreads) void k_sample_write(const CaseDesc* __restrict__ cs,
                                                                int n,
                                                                SampleCounts* __restrict__ cnt,
                                                                Ctl* ctl, BinLists L,
                                                                int64_t ngroups, uint32_t budget)
{
    constexpr int NT = kSampleThreads;
    __shared__ uint64_t s_red[5 * (NT / kWave)];
    __shared__ int64_t s_rows[NT * kCandPerThread];
    __shared__ uint64_t s_e[FUSED ? 3 : 1][FUSED ? NT : 1];
    __shared__ GroupOff s_go;
    const int t = threadIdx.x;
    GroupOff o;
    int lvl;
    if constexpr (FUSED) {
        lvl = scan_groups<NT, false>(cnt, ngroups, cs, ctl, budget, blockIdx.x == 0,
                                     (int64_t)blockIdx.x, s_red,
                                     reinterpret_cast<uint64_t (*)[NT]>(&s_e[0][0]), &s_go);
        o = s_go;  // (written before the routine's last barrier)
    } else {
        const SampleCounts& y = cnt[blockIdx.x];
        o.o1 = y.o1;
        o.o2 = y.o2;
        o.o3 = y.o3;
        o.oh = y.oh;
        o.ol = y.ol;
        o.om = y.om;
        o.ow = y.ow;
        o.split = y.split;
        lvl = (int)ctl->split_level;
    }
    const GroupRange gr = group_range(cs, n, blockIdx.x);
    if (gr.lo >= gr.hi) return;  // (uniform over the workgroup)
    const SamplerArgs a = sampler_args(cs[gr.c]);
    const bool split = o.split != 0;
    uint32_t off1 = o.o1, off2 = o.o2, off3 = o.o3, off4 = o.oh, offm = o.om, offw = o.ow,
             offb = o.ol;
    for (int64_t base = gr.lo; base < gr.hi; base += NT * kCandPerThread) {
        const int nr = gather_sampled<NT>(base, gr.hi, a, s_rows, s_red);
        for (int k0 = 0; k0 < nr; k0 += NT) {  // same trip count in every lane (scans)
            const SampledRow r = classify_row(k0 + t < nr ? s_rows[k0 + t] : -1, a);
            const SplitInfo si = split_info(r, a, lvl);
            const bool sp = split && si.elig;
            const uint32_t n4 = r.bin == 4 ? (sp ? si.want : 1u) : 0u;
            const uint32_t nf = si.heavy ? n4 : 0u, nb = r.bin == 4 && !si.heavy ? 1u : 0u;
            const uint32_t nm = sp ? (uint32_t)a.merge_per_row : 0u;
            const uint32_t nw = sp ? si.want * (uint32_t)a.nwin : 0u;
            uint64_t t01, t34, tmw;
            // bins 1, 2 and light bin-4 rows in 21-bit fields (at most NT each)
            static_assert(NT < (1 << 21), "21-bit scan fields");
            const uint64_t f01 =
                (uint64_t)(r.bin == 1) | ((uint64_t)(r.bin == 2) << 21) | ((uint64_t)nb << 42);
            const uint64_t p01 = block_excl_scan<NT, uint64_t>(f01, s_red, &t01);
            const uint64_t p34 = block_excl_scan<NT, uint64_t>(
                (uint64_t)(r.bin == 3) | ((uint64_t)nf << 32), s_red, &t34);
            const uint64_t pmw = block_excl_scan<NT, uint64_t>((uint64_t)nm | ((uint64_t)nw << 32),
                                                               s_red, &tmw);
            if (r.bin >= 1 && r.bin <= 3) {
                BinItem it;
                it.row = (int32_t)r.g;
                it.rf = (uint32_t)r.rf;
                it.cs = gr.c;
                it.pad = 0;
                if (r.bin == 1) L.b1[off1 + (uint32_t)(p01 & 0x1FFFFF)] = it;
                else if (r.bin == 2) L.b2[off2 + (uint32_t)((p01 >> 21) & 0x1FFFFF)] = it;
                else L.b3[off3 + (uint32_t)p34] = it;
            } else if (r.bin == 4) {
                const uint32_t at = si.heavy ? off4 + (uint32_t)(p34 >> 32)
                                             : L.cap4 - 1u - (offb + (uint32_t)(p01 >> 42));
                const int32_t slot = sp ? (int32_t)(offw + (uint32_t)(pmw >> 32)) : -1;
                for (uint32_t p = 0; p < n4; ++p) {
                    BigItem it;
                    it.row = (int32_t)r.g;
                    it.slot = slot;
                    it.part = (int32_t)p;
                    it.nparts = (int32_t)n4;
                    it.e_lo = r.e0;
                    it.e_hi = r.e1;
                    it.cs = gr.c;
                    it.pad = 0;
                    L.b4[at + p] = it;
                }
                if (sp) write_merge_items(L.merge + offm + (uint32_t)pmw, (int32_t)r.g, slot,
                                          (int32_t)n4, gr.c, cs[gr.c]);
            }
            off1 += (uint32_t)(t01 & 0x1FFFFF);
            off2 += (uint32_t)((t01 >> 21) & 0x1FFFFF);
            offb += (uint32_t)(t01 >> 42);
            off3 += (uint32_t)t34;
            off4 += (uint32_t)(t34 >> 32);
            offm += (uint32_t)tmw;
            offw += (uint32_t)(tmw >> 32);
        }
    }
}

// ------------------------------------------------- distinct counting

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// Open addressing with linear probing on an LDS table of 2^lg words;
// returns 1 when `c` was not yet present.  Columns are < 2^31, so the
// all-ones word marks an empty slot.  Every probe is one compare-and-swap,
// whose returned word tells an insert, a repeat and an occupied slot apart
// (a plain read first, then the swap on an empty slot, took two dependent
// LDS round trips per new column: bins of uniform 2^20 d 32 90 -> 75 us).
__device__ __forceinline__ uint32_t hash_insert(uint32_t* tab, uint32_t c, int lg)
{
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t h = (c * 0x9E3779B1u) >> (32 - lg);
    for (;;) {
        const uint32_t prev = atomicCAS(&tab[h], kEmpty, c);
        if (prev == kEmpty) return 1u;
        if (prev == c) return 0u;
        h = (h + 1u) & mask;
    }
}

// Orders the LDS accesses of one wave (the LDS serves a wave's accesses in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronisation of a team: the workgroup, or its own wave for TEAM = 64.
template <int TEAM>
__device__ __forceinline__ void team_sync()
{
    if (TEAM == kWave) wave_sync();
    else __syncthreads();
}

// Bins 1..3: one team of TEAM threads per row (a workgroup, or one wave of
// one).  The row's products are enumerated chunk by chunk of TEAM entries of
// A: a scan of the B row lengths gives each product's owner, found by binary
// search in LDS, so every thread handles an equal share of products whatever
// the B row lengths.  Counting uses an LDS bitmap of all N columns when that
// is no larger than the hash table, else the hash table (size >= 2 x the
// row's distinct bound).  The team takes items first, first + stride, ...;
// `t` is its thread's index in the team, `slot` its distinct-count slot.
// MODE 0: add the count to the case's z*.  MODE 1: write it to out[row]
// (and to the case's total).
template <int TEAM, int WORDS, int MODE>
__device__ __forceinline__ void sym_rows(const CaseDesc* __restrict__ cs,
                                         const BinItem* __restrict__ items, uint32_t n,
                                         uint32_t first, uint32_t stride, int t, uint32_t* tab,
                                         int32_t* s_b0, uint32_t* s_off, uint32_t* s_red,
                                         CaseRes* __restrict__ cr, uint32_t slot)
{
    int zc = -1;  // case of zsum (items of a case are consecutive in the list)
    uint64_t zsum = 0;
    // The team's next row is prefetched in stages while the current one is
    // counted, so a row does not begin on its chain of dependent loads (item,
    // A row bounds, A columns, B row bounds): the item when a row begins, its
    // A row bounds after the table is cleared, the A columns of its first
    // chunk after the last products are issued, their B row bounds after the
    // count.
    uint32_t it = first;
    BinItem item{};
    int32_t ra0 = 0, ra1 = 0;  // the current row's A entries
    int32_t pb0 = 0;           // its first chunk's B row start and length,
    uint32_t plen = 0;         // for entry ra0 + t, when `staged`
    bool staged = false;
    if (it < n) {
        item = items[it];
        const Csr A = cs[item.cs].A;
        ra0 = A.rpt[item.row];
        ra1 = A.rpt[item.row + 1];
    }
    for (; it < n; it += stride) {
        const uint32_t itn = it + stride;
        const bool more = itn < n;
        BinItem nx{};
        if (more) nx = items[itn];
        if (item.cs != zc) {
            if (t == 0 && zsum) atomicAdd(as_ull(&cr[zc].zacc[slot]), (ull)zsum);
            zsum = 0;
            zc = item.cs;
        }
        const Csr A = cs[zc].A, B = cs[zc].B;
        const int64_t N = B.ncols;
        const uint32_t bound = (uint32_t)((int64_t)item.rf < N ? (int64_t)item.rf : N);
        uint32_t tsize = 64;
        const uint32_t mult = cs[zc].hash_mult;
        while (tsize < mult * bound && tsize < (uint32_t)WORDS) tsize <<= 1;
        const bool bitmap = N <= 32 * (int64_t)tsize;
        const uint32_t words = bitmap ? (uint32_t)((N + 31) / 32) : tsize;
        const int lg = __builtin_ctz(tsize);
        const uint32_t fill = bitmap ? 0u : kEmpty;
        for (uint32_t w = t; w < words; w += TEAM) tab[w] = fill;
        team_sync<TEAM>();
        // (the next row's A row bounds)
        int32_t na0 = 0, na1 = 0;
        if (more) {
            const Csr An = cs[nx.cs].A;
            na0 = An.rpt[nx.row];
            na1 = An.rpt[nx.row + 1];
        }
        uint32_t cnt = 0;
        int32_t nk = -1;  // (the next row's first-chunk column of this thread)
        for (int32_t a = ra0; a < ra1; a += TEAM) {
            const int32_t j = a + t;
            uint32_t len = 0;
            int32_t b0 = 0;
            if (staged && a == ra0) {
                b0 = pb0;
                len = plen;
            } else if (j < ra1) {
                const int32_t k = A.col[j];
                b0 = B.rpt[k];
                len = (uint32_t)(B.rpt[k + 1] - b0);
            }
            uint32_t tot;
            const uint32_t off = block_excl_scan<TEAM, uint32_t>(len, s_red, &tot);
            s_b0[t] = b0;
            s_off[t] = off;
            team_sync<TEAM>();
            const int na = (ra1 - a) < TEAM ? (ra1 - a) : TEAM;
            constexpr int U = 4;
            // same trip count in every lane; U independent loads in flight per lane
            // (software-pipelining the rounds, the next round's loads issued
            // before this round's inserts, was slower: registers)
            for (uint32_t p0 = 0; p0 < tot; p0 += TEAM * U) {
                uint32_t c[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // clamped product index, unconditional load, masked after
                    const uint32_t pr = p0 + u * TEAM + t;
                    const uint32_t p = pr < tot ? pr : tot - 1;
                    int lo = 0, hi = na;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_off[mid] <= p) lo = mid;
                        else hi = mid;
                    }
                    const uint32_t cv = (uint32_t)B.col[s_b0[lo] + (int32_t)(p - s_off[lo])];
                    c[u] = pr < tot ? cv : kNoWord;
                }
                // (the last chunk's last round: the next row's first-chunk columns)
                if (more && a + TEAM >= ra1 && p0 + TEAM * U >= tot && na0 + t < na1)
                    nk = cs[nx.cs].A.col[na0 + t];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (bitmap)
                        lds_bitmap_or(tab, c[u] == kNoWord ? kNoWord : (c[u] >> 5), 1u << (c[u] & 31));
                    else if (c[u] != kNoWord)
                        cnt += hash_insert(tab, c[u], lg);
                }
            }
            team_sync<TEAM>();
        }
        // (a row whose chunks issued no round: its columns now)
        if (more && nk < 0 && na0 + t < na1) nk = cs[nx.cs].A.col[na0 + t];
        if (bitmap)
            for (uint32_t w = t; w < words; w += TEAM) cnt += (uint32_t)__popc(tab[w]);
        const uint32_t total = block_sum<TEAM, uint32_t>(cnt, s_red);
        if (t == 0) {
            zsum += total;
            if (MODE == 1) cs[zc].out[item.row] = (int64_t)total;
        }
        // (the next row's first-chunk B row bounds)
        pb0 = 0;
        plen = 0;
        if (nk >= 0) {
            const Csr Bn = cs[nx.cs].B;
            pb0 = Bn.rpt[nk];
            plen = (uint32_t)(Bn.rpt[nk + 1] - pb0);
        }
        team_sync<TEAM>();
        item = nx;
        ra0 = na0;
        ra1 = na1;
        staged = more;
    }
    if (t == 0 && zsum) atomicAdd(as_ull(&cr[zc].zacc[slot]), (ull)zsum);
}

template <int TEAM, int WORDS, int MODE>
__global__ __launch_bounds__(TEAM) void k_sym(const CaseDesc* __restrict__ cs,
                                             const BinItem* __restrict__ items,
                                             const uint32_t* count, CaseRes* __restrict__ cr)
{
    __shared__ uint32_t tab[WORDS];
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ uint32_t s_red[TEAM / kWave + 1];
    sym_rows<TEAM, WORDS, MODE>(cs, items, *count, blockIdx.x, gridDim.x, threadIdx.x, tab, s_b0,
                                s_off, s_red, cr, blockIdx.x % kAccSlots);
}

// Bins 1 and 2 in one launch of 256-thread workgroups: the first g1 take
// bin-1 rows four at a time (one per wave), the others bin-2 rows (a
// workgroup per row), so the two bins' latency chains overlap.
constexpr int kBins12Threads = 256;

template <int MODE>
__global__ __launch_bounds__(kBins12Threads) void k_sym_bins12(const CaseDesc* __restrict__ cs,
                                                              const BinItem* __restrict__ b1,
                                                              const uint32_t* n1,
                                                              const BinItem* __restrict__ b2,
                                                              const uint32_t* n2, uint32_t g1,
                                                              CaseRes* __restrict__ cr)
{
    constexpr int NW = kBins12Threads / kWave;
    constexpr int W1 = kBin1Words + 2 * kWave + 2;  // per wave: table, owners, offsets, scan
    constexpr int W2 = kBin2Words + 2 * kBins12Threads + NW + 1;
    constexpr int WORDS = NW * W1 > W2 ? NW * W1 : W2;
    __shared__ uint32_t sm[WORDS];
    const int t = threadIdx.x, lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(t / kWave);
    const uint32_t slot = blockIdx.x % kAccSlots;
    if (blockIdx.x < g1) {
        uint32_t* base = sm + w * W1;
        sym_rows<kWave, kBin1Words, MODE>(cs, b1, *n1, blockIdx.x * NW + w, g1 * NW, lane, base,
                                          (int32_t*)(base + kBin1Words), base + kBin1Words + kWave,
                                          base + kBin1Words + 2 * kWave, cr, slot);
    } else {
        sym_rows<kBins12Threads, kBin2Words, MODE>(cs, b2, *n2, blockIdx.x - g1, gridDim.x - g1, t, sm,
                                                   (int32_t*)(sm + kBin2Words),
                                                   sm + kBin2Words + kBins12Threads,
                                                   sm + kBin2Words + 2 * kBins12Threads, cr, slot);
    }
}

// Bin 4: long rows, 1024 threads per item, an LDS bitmap per window of
// `win_words` words.  An item covers the A entries [e_lo, e_hi) of its row (all
// of them unless the row is split into parts).  The entries are taken 1024 at
// a time.  Those naming a B row of at least kLongLen columns are cut into
// units of kUnitCols columns; every wave walks its own contiguous range of the
// chunk's units, lane l reading columns [4l, 4l + 4) of a unit with one
// 16-byte load, kUnitsInFlight - 1 units ahead of the inserts.  The short B rows are
// flattened (owner by binary search in LDS) and shared out over the whole
// workgroup.  An unsplit item counts its bits; a part of a split row stores
// its window bitmap to global scratch for k_sym_merge.  Bitmap words are
// swizzled inside their 64-word rows (swz): neighbouring lanes striding a
// sorted B row would otherwise meet on one LDS bank every 64 words.
constexpr uint32_t kUnitCols = 4 * kWave;
constexpr int kUnitsInFlight = 4;  // 16-byte loads in flight per lane in the unit loop


template <int MODE, bool WIN1>
__global__ __launch_bounds__(kBin4Team) void k_sym_big(const CaseDesc* __restrict__ cs,
                                                       const BigItem* __restrict__ items,
                                                       const uint32_t* count, uint32_t* next,
                                                       BinLists L, CaseRes* __restrict__ cr)
{
    constexpr int TEAM = kBin4Team, NWAVE = TEAM / kWave;
    typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
    extern __shared__ __align__(16) uint32_t bm[];
    uint4* bm4 = reinterpret_cast<uint4*>(bm);
    // compacted entries of a chunk: short ones from the front, long ones from the back
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_len[TEAM];
    __shared__ uint64_t s_start[TEAM]; // short: first product; long: first unit
    __shared__ uint64_t s_red[2 * (TEAM / kWave)];
    __shared__ uint32_t s_it;
    // the next item, taken ahead by wave 0: ticket, descriptor, and the B row
    // bounds of the entries of its first chunk
    __shared__ uint32_t s_nt;
    __shared__ int32_t s_nx[8];
    __shared__ int32_t s_nb0[TEAM], s_nb1[TEAM];
    static_assert(sizeof(BigItem) == sizeof(s_nx), "descriptor words");
    const uint32_t nheavy = count[0], n = nheavy + count[2];  // heavy, light items
    const uint32_t near_end = 2u * gridDim.x;
    const int t = threadIdx.x, lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(t / kWave);
    int zc = -1;  // case of zsum
    uint64_t zsum = 0;
    // Work queue.  Far from its end, wave 0 takes the ticket of the next item
    // during the first chunk of the current one and stages what the next
    // item's first chunk reads (its other waves meanwhile take the chunk's
    // long entries), so an item does not begin on a chain of dependent global
    // loads.  Near the end (fewer than two items per workgroup left) the
    // ticket is taken as the last pass over the current item begins, so no
    // item waits on a busy workgroup while another is idle.
    if (t == 0) s_it = atomicAdd(next, 1u);
    __syncthreads();
    uint32_t it = __builtin_amdgcn_readfirstlane(s_it);
    bool staged = false;  // item `it` is staged in s_nx, s_nb0, s_nb1
    int clean4 = 0;       // leading 16-byte groups of the bitmap known to be zero
    for (;;) {
        if (it >= n) break;
        BigItem item;
        if (staged) {
            item.row = __builtin_amdgcn_readfirstlane(s_nx[0]);
            item.slot = __builtin_amdgcn_readfirstlane(s_nx[1]);
            item.part = __builtin_amdgcn_readfirstlane(s_nx[2]);
            item.nparts = __builtin_amdgcn_readfirstlane(s_nx[3]);
            item.e_lo = __builtin_amdgcn_readfirstlane(s_nx[4]);
            item.e_hi = __builtin_amdgcn_readfirstlane(s_nx[5]);
            item.cs = __builtin_amdgcn_readfirstlane(s_nx[6]);
        } else {
            item = items[big_index(it, nheavy, L.cap4)];
        }
        if (item.cs != zc) {
            if (t == 0 && zsum) atomicAdd(as_ull(&cr[zc].zacc[blockIdx.x % kAccSlots]), (ull)zsum);
            zsum = 0;
            zc = item.cs;
        }
        const Csr A = cs[zc].A, B = cs[zc].B;
        const int64_t N = B.ncols;
        const int32_t nwin = cs[zc].nwin;
        const int64_t wcols_full = (int64_t)cs[zc].win_words * 32;
        const uint32_t long_len = cs[zc].long_len;  // >= 8: a long row has a full 16-byte group
        // entries e0, e0 + P, e0 + 2P, ... below e_hi (P = 1 unless split)
        const int32_t e0 = item.e_lo + item.part, P = item.nparts;
        const int64_t cnt = item.e_hi > e0 ? ((int64_t)item.e_hi - e0 + P - 1) / P : 0;
        const bool ahead = it + near_end < n && cnt > 0;  // wave 0 stages the next item
        uint64_t total = 0;
        for (int w = 0; w < nwin; ++w) {
            const int64_t c_lo = w * wcols_full;
            const int64_t wcols = (N - c_lo) < wcols_full ? (N - c_lo) : wcols_full;
            const int words = (int)bitmap_words(wcols);
            const int w4 = words / 4;  // 16-byte groups (words: whole 64-word rows)
            // the bitmap is cleared when dirty; the pass that counts a window
            // zeroes every group it reads
            if (w4 > clean4) {
                for (int i = clean4 + t; i < w4; i += TEAM) bm4[i] = make_uint4(0u, 0u, 0u, 0u);
                clean4 = w4;
                __syncthreads();
            }
            const uint32_t clo32 = (uint32_t)c_lo, wc32 = (uint32_t)wcols;
            for (int64_t i0 = 0; i0 < cnt; i0 += TEAM) {
                const int64_t i = i0 + t;
                const bool live = i < cnt;
                const bool first = w == 0 && i0 == 0;
                int32_t b0, b1;
                if (staged && first) {
                    b0 = s_nb0[t];
                    b1 = s_nb1[t];
                } else {
                    const int32_t k = A.col[e0 + (int32_t)((live ? i : cnt - 1) * P)];
                    b0 = B.rpt[k];
                    b1 = B.rpt[k + 1];
                }
                const uint32_t len = live ? (uint32_t)(b1 - b0) : 0u;
                const bool lng = len >= long_len, shrt = !lng && len != 0;
                // short products (bits 0..19), short entries (20..39), long entries (40..)
                const uint64_t packed = (shrt ? (uint64_t)len | (1ull << 20) : 0ull) |
                                        (lng ? (1ull << 40) : 0ull);
                const uint64_t nunits = lng ? (len + kUnitCols - 1) / kUnitCols : 0u;
                uint64_t pk, uk, ptot, utot;
                block_excl_scan2<TEAM, uint64_t>(packed, nunits, s_red, &pk, &uk, &ptot, &utot);
                if (shrt) {
                    const int i = (int)((pk >> 20) & 0xFFFFF);
                    s_b0[i] = b0;
                    s_start[i] = pk & 0xFFFFF;
                }
                if (lng) {
                    const int i = TEAM - 1 - (int)(pk >> 40);
                    s_b0[i] = b0;
                    s_len[i] = len;
                    s_start[i] = uk;
                }
                __syncthreads();
                ptot = uniform_u64(ptot);
                utot = uniform_u64(utot);
                const uint32_t nsp = (uint32_t)(ptot & 0xFFFFF);
                const int nse = (int)((ptot >> 20) & 0xFFFFF), nle = (int)(ptot >> 40);
                // long entries: units [ub, ue) of this wave (wave 0 stages the
                // next item instead, during the first chunk of an `ahead` item)
                const bool stage = ahead && first;
                const int nwv = stage ? NWAVE - 1 : NWAVE, wv = stage ? wave - 1 : wave;
                const uint64_t ub = wv < 0 ? 0 : utot * (uint64_t)wv / nwv;
                const uint64_t ue = wv < 0 ? 0 : utot * (uint64_t)(wv + 1) / nwv;
                if (stage && wave == 0) {
                    uint32_t j = 0;
                    if (lane == 0) j = atomicAdd(next, 1u);
                    j = __builtin_amdgcn_readfirstlane(j);
                    if (lane == 0) s_nt = j;
                    if (j < n) {
                        // the descriptor's eight words, one per lane (a copy of
                        // the struct indexed by lane would go through scratch)
                        const int32_t* src =
                            reinterpret_cast<const int32_t*>(items + big_index(j, nheavy, L.cap4));
                        const int32_t wv = src[lane < 8 ? lane : 0];
                        if (lane < 8) s_nx[lane] = wv;
                        BigItem nx;
                        nx.row = __builtin_amdgcn_readlane(wv, 0);
                        nx.slot = __builtin_amdgcn_readlane(wv, 1);
                        nx.part = __builtin_amdgcn_readlane(wv, 2);
                        nx.nparts = __builtin_amdgcn_readlane(wv, 3);
                        nx.e_lo = __builtin_amdgcn_readlane(wv, 4);
                        nx.e_hi = __builtin_amdgcn_readlane(wv, 5);
                        nx.cs = __builtin_amdgcn_readlane(wv, 6);
                        nx.pad = 0;
                        const Csr A2 = cs[nx.cs].A, B2 = cs[nx.cs].B;
                        const int32_t ne0 = nx.e_lo + nx.part, nP = nx.nparts;
                        const int64_t ncnt =
                            nx.e_hi > ne0 ? ((int64_t)nx.e_hi - ne0 + nP - 1) / nP : 0;
                        const int m = (int)(ncnt < TEAM ? ncnt : TEAM);
                        // eight entries per lane in flight at a time
                        constexpr int PER = 8;
                        for (int q0 = 0; q0 < m; q0 += PER * kWave) {
                            int32_t kk[PER];
#pragma unroll
                            for (int u = 0; u < PER; ++u) {
                                const int q = q0 + lane + u * kWave;
                                kk[u] = A2.col[ne0 + (q < m ? q : m - 1) * nP];
                            }
#pragma unroll
                            for (int u = 0; u < PER; ++u) {
                                const int q = q0 + lane + u * kWave;
                                const i32x2u v = *(const SSP_GLOBAL i32x2u*)(B2.rpt + kk[u]);
                                if (q < m) {
                                    s_nb0[q] = v.x;
                                    s_nb1[q] = v.y;
                                }
                            }
                        }
                    }
                } else if (ub < ue) {
                    // owner of unit ub: the last long entry starting at or before it
                    int lo = 0, hi = nle;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_start[TEAM - 1 - mid] <= ub) lo = mid;
                        else hi = mid;
                    }
                    // Issue cursor, wave-uniform: long entry r, unit ui of its nu
                    // units; `left` units of this wave still to issue.  At the last
                    // unit the cursor stays, so prefetches past the end re-read it.
                    int r = __builtin_amdgcn_readfirstlane(lo);
                    uint32_t elen, nu, ui;
                    int32_t eb0;
                    auto load_entry = [&]() {
                        const int e = TEAM - 1 - r;
                        elen = __builtin_amdgcn_readfirstlane(s_len[e]);
                        eb0 = __builtin_amdgcn_readfirstlane(s_b0[e]);
                        nu = (elen + kUnitCols - 1) / kUnitCols;
                    };
                    load_entry();
                    ui = (uint32_t)(ub - uniform_u64(s_start[TEAM - 1 - r]));
                    uint32_t left = (uint32_t)(ue - ub);  // < 2^29: per-wave share
                    // kUnitsInFlight units in flight in registers of fixed roles (the
                    // loop is unrolled by that depth so no loaded register is moved
                    // before use, which would make the compiler wait for every load).
                    constexpr int D = kUnitsInFlight;
                    i32x4 v[D];
                    bool ok[D];
                    auto issue = [&](i32x4& v, bool& ok) {
                        const uint32_t base = ui * kUnitCols + 4u * lane;
                        const uint32_t off = base < elen - 4u ? base : elen - 4u;
                        v = *(const SSP_GLOBAL i32x4u*)(B.col + eb0 + off);
                        ok = base < elen;
                        __builtin_amdgcn_sched_barrier(0);  // keep the load ahead of the inserts
                    };
                    auto advance = [&]() {
                        if (left > 1) {
                            --left;
                            if (ui + 1 < nu) {
                                ++ui;
                            } else {
                                ++r;
                                ui = 0;
                                load_entry();
                            }
                        }
                    };
                    auto insert = [&](const i32x4& v, bool ok) {
                        if (WIN1) {
                            if (ok) lane_bitmap_insert4(bm, v);
                        } else {
                            const uint32_t c[4] = {ok ? (uint32_t)v.x : kNoWord,
                                                   ok ? (uint32_t)v.y : kNoWord,
                                                   ok ? (uint32_t)v.z : kNoWord,
                                                   ok ? (uint32_t)v.w : kNoWord};
                            lane_bitmap_insert<4>(bm, c, clo32, wc32);
                        }
                    };
                    const uint32_t n = left;
#pragma unroll
                    for (int k = 0; k < D - 1; ++k) {  // units 0 .. D-2
                        if (k) advance();
                        issue(v[k], ok[k]);
                    }
                    for (uint32_t u = 0; u < n; u += D) {
#pragma unroll
                        for (int k = 0; k < D; ++k) {  // issue unit u+k+D-1, insert unit u+k
                            advance();
                            issue(v[(k + D - 1) % D], ok[(k + D - 1) % D]);
                            if (k == 0 || u + k < n) insert(v[k], ok[k]);
                        }
                    }
                }
                // short entries: products flattened over the workgroup
                constexpr int US = 4;
                for (uint32_t q0 = 0; q0 < nsp; q0 += TEAM * US) {
                    uint32_t c[US];
#pragma unroll
                    for (int u = 0; u < US; ++u) {
                        const uint32_t qr = q0 + u * TEAM + t;
                        const uint32_t q = qr < nsp ? qr : nsp - 1;
                        int lo = 0, hi = nse;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (s_start[mid] <= q) lo = mid;
                            else hi = mid;
                        }
                        const uint32_t cv =
                            (uint32_t)B.col[s_b0[lo] + (int32_t)(q - (uint32_t)s_start[lo])];
                        c[u] = qr < nsp ? cv : kNoWord;
                    }
                    if (WIN1) lane_bitmap_insert_all<US>(bm, c);
                    else lane_bitmap_insert<US>(bm, c, clo32, wc32);
                }
                __syncthreads();
            }
            if (w == nwin - 1 && !ahead && t == 0)
                s_it = atomicAdd(next, 1u);  // read after the barrier below
            // 16-byte LDS reads, eight issued before any is used (a loop of
            // single reads would wait on each)
            constexpr int UR = 8;
            const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
            if (item.slot < 0) {
                uint32_t cnt = 0;
                for (int i0 = t; i0 < w4; i0 += UR * TEAM) {
                    uint4 x[UR];
#pragma unroll
                    for (int u = 0; u < UR; ++u) {
                        const int i = i0 + u * TEAM;
                        x[u] = bm4[i < w4 ? i : w4 - 1];
                    }
#pragma unroll
                    for (int u = 0; u < UR; ++u)
                        if (i0 + u * TEAM < w4) {
                            bm4[i0 + u * TEAM] = z4;
                            cnt += __popc(x[u].x) + __popc(x[u].y) + __popc(x[u].z) + __popc(x[u].w);
                        }
                }
                total += block_sum<TEAM, uint64_t>(cnt, s_red);
            } else {
                uint4* g = reinterpret_cast<uint4*>(
                    L.scratch + ((int64_t)item.slot + (int64_t)item.part * nwin + w) *
                                    (int64_t)kWinWords);
                for (int i0 = t; i0 < w4; i0 += UR * TEAM) {
                    uint4 x[UR];
#pragma unroll
                    for (int u = 0; u < UR; ++u) {
                        const int i = i0 + u * TEAM;
                        x[u] = bm4[i < w4 ? i : w4 - 1];
                    }
#pragma unroll
                    for (int u = 0; u < UR; ++u)
                        if (i0 + u * TEAM < w4) g[i0 + u * TEAM] = x[u];
                }
                clean4 = 0;  // (this pass leaves the bitmap as it is)
            }
            __syncthreads();
        }
        if (t == 0 && total) {
            zsum += total;
            if (MODE == 1) atomicAdd(reinterpret_cast<ull*>(&cs[zc].out[item.row]), (ull)total);
        }
        it = __builtin_amdgcn_readfirstlane(ahead ? s_nt : s_it);
        staged = ahead && it < n;
    }
    if (t == 0 && zsum) atomicAdd(as_ull(&cr[zc].zacc[blockIdx.x % kAccSlots]), (ull)zsum);
}

// ORs the part bitmaps of split rows, one slice of a window per item, and
// adds the distinct counts (sixteen parts' 16-byte groups in flight per
// thread: the parts' windows are read once, from L2 or MALL).
template <int MODE>
__global__ __launch_bounds__(256) void k_sym_merge(const CaseDesc* __restrict__ cs,
                                                  const MergeItem* __restrict__ items,
                                                  const uint32_t* count, BinLists L,
                                                  CaseRes* __restrict__ cr)
{
    __shared__ uint64_t s_red[256 / kWave + 1];
    const uint32_t n = *count;
    const int t = threadIdx.x;
    int zc = -1;
    uint64_t zsum = 0;
    static_assert(kMergeSlice == 4 * 256, "one 16-byte group per thread and slice");
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const MergeItem m = items[it];
        if (m.cs != zc) {
            if (t == 0 && zsum) atomicAdd(as_ull(&cr[zc].zacc[blockIdx.x % kAccSlots]), (ull)zsum);
            zsum = 0;
            zc = m.cs;
        }
        const int64_t N = cs[zc].B.ncols;
        const int32_t nwin = cs[zc].nwin;
        const int64_t wcols_full = (int64_t)cs[zc].win_words * 32;
        const int64_t c_lo = (int64_t)m.window * wcols_full;
        const int64_t wcols = (N - c_lo) < wcols_full ? (N - c_lo) : wcols_full;
        const int w4 = (int)(bitmap_words(wcols) / 4);  // 16-byte groups of this window
        const int g4 = m.slice * (kMergeSlice / 4) + t;
        uint32_t cnt = 0;
        if (g4 < w4) {
            // the parts' groups, sixteen 16-byte loads in flight, then OR
            constexpr int PF = 16;
            const int64_t stride4 = (int64_t)nwin * kWinWords / 4;
            const uint4* src = reinterpret_cast<const uint4*>(
                                   L.scratch + ((int64_t)m.slot + m.window) * (int64_t)kWinWords) +
                               g4;
            uint4 x = make_uint4(0u, 0u, 0u, 0u);
            for (int p0 = 0; p0 < m.nparts; p0 += PF) {
                uint4 v[PF];
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int pp = p0 + u < m.nparts ? p0 + u : m.nparts - 1;
                    v[u] = src[(int64_t)pp * stride4];
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    x.x |= v[u].x;
                    x.y |= v[u].y;
                    x.z |= v[u].z;
                    x.w |= v[u].w;
                }
            }
            cnt = __popc(x.x) + __popc(x.y) + __popc(x.z) + __popc(x.w);
        }
        const uint64_t total = block_sum<256, uint64_t>(cnt, s_red);
        if (t == 0 && total) {
            zsum += total;
            if (MODE == 1) atomicAdd(reinterpret_cast<ull*>(&cs[zc].out[m.row]), (ull)total);
        }
    }
    if (t == 0 && zsum) atomicAdd(as_ull(&cr[zc].zacc[blockIdx.x % kAccSlots]), (ull)zsum);
}

// ---------------------------------------------------------- finalize

// One workgroup of kAccSlots threads per case after the symbolic kernels of
// the reference design (MODE 0) or the exact structure (MODE 1): sums the
// case's distinct-count slots into z* or the exact total.  (The prediction
// kernel sums z* itself.)
template <int MODE>
__global__ __launch_bounds__(kAccSlots) void k_finalize(const CaseDesc* __restrict__ cs,
                                                       CaseRes* __restrict__ cr, int n)
{
    __shared__ uint64_t s_red[kAccSlots / kWave + 1];
    for (int c = blockIdx.x; c < n; c += gridDim.x) {
        const uint64_t z = block_sum<kAccSlots, uint64_t>(cr[c].zacc[threadIdx.x], s_red);
        if (threadIdx.x != 0) continue;
        ssp_stats* st = cs[c].st;
        if (MODE == 1) {
            st->out_sum = z;
            continue;
        }
        st->sample_nnz = z;
    }
}

// Reference design constants per case (Eq. (2)): z* M and n_s F.
__global__ void k_finalize_reference(const CaseDesc* __restrict__ cs, CaseRes* __restrict__ cr,
                                     int n)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        ssp_stats* st = cs[c].st;
        if (st->sample_flop == 0) {
            cr[c].fallback = 1;
            st->flags |= SSP_FLAG_EMPTY_SAMPLE;
            continue;
        }
        cr[c].fallback = 0;
        const u128 q = mul_64x64(st->sample_nnz, (uint64_t)cs[c].A.nrows);
        const u128 d = mul_64x64(st->n_sampled, st->total_flop);
        cr[c].ref_q_lo = q.lo;
        cr[c].ref_q_hi = q.hi;
        cr[c].ref_d_lo = d.lo;
        cr[c].ref_d_hi = d.hi;
    }
}

// -------------------------------------------------------------- k_flop

enum { FLOP_ONLY = 1, FLOP_EXACT_BIN = 2 };

// Output of one finished row of case c: its product count, or its bin.
template <int MODE>
__device__ __forceinline__ void emit_row(const CaseDesc* __restrict__ cs, int c, int64_t row,
                                         uint64_t rf, Ctl* ctl, const BinLists& L)
{
    if (MODE == FLOP_ONLY) {
        cs[c].rf[row] = (int64_t)rf;
    } else {
        const CaseDesc& cd = cs[c];
        const int b = bin_route(rf, cd);
        if (b == 0 || b == 4) cd.out[row] = 0;
        if (b != 0) append_row((int32_t)row, rf, cd.A.rpt[row], cd.A.rpt[row + 1], c, cd, ctl, L);
    }
}

// Merge-path tile b of a case covers the items [b T, (b+1) T) of the sequence
// that interleaves A's entries with one end marker per row (Merrill &
// Garland, SC16), so every tile has at most T = kFlopTile rows + entries
// whatever the row lengths.  A tile's entries are loaded four consecutive
// ones per lane with 16-byte loads (fully coalesced, non-temporal so the
// stream does not evict B's row lengths from L2), put in entry order across
// the lanes through LDS, and each contributes the length of the B row it
// names (one gather per entry, consecutive entries in consecutive lanes).  An exclusive scan of these lengths (in 32 bits when the
// lengths allow) gives the running product count at every row boundary, and a
// row's count is the difference of its two boundaries.  Rows that begin in an
// earlier tile or end in a later one leave their partial counts in the tile's
// metadata for k_flop_fixup.
//
// Tiles are numbered case after case (global tile g belongs to case
// tile_case[g]).  The kernel is persistent: workgroup w takes the global tiles
// w, w + G, w + 2G, ..., so at any time the device works on one or two
// neighbouring cases and their B row pointers stay in L2 (a batch that gave
// every case its own workgroups at once would gather from all of them
// together).  It software-pipelines its tiles: while tile g's gathers are in
// flight it issues the loads of tile g + G, and the starts of the tiles after
// that are staged in LDS.
struct FlopTileRegs {
    int64_t g;        // global tile
    int32_t c;        // its case
    const SSP_GLOBAL int32_t* Arpt;
    const SSP_GLOBAL int32_t* Brpt;
    const SSP_GLOBAL uint16_t* blen;
    SSP_GLOBAL int64_t* out;
    int64_t M, nnzA, K;
    int64_t i0, i1, j0, j1, a0;
    // entry q HALF + 256 wave + 64 l + lane in col[4 q + l] (VEC: as loaded,
    // entry q HALF + 256 wave + 4 lane + l, until the tile is processed)
    int32_t col[8];
    int32_t rp[kFlopTile / kFlopThreads + 1];  // (VEC: rows 4 NT u + 4 t + k in rp[4 u + k])
};

// Issues the loads of global tile g of case c, whose rows are [i0, i1].
template <int MODE, bool VEC>
__device__ __forceinline__ void flop_issue_tile(const CaseDesc* __restrict__ cs, int64_t g, int c,
                                                int64_t i0, int64_t i1, FlopTileRegs& R)
{
    constexpr int NT = kFlopThreads, HALF = kFlopChunk / 2, NRP = kFlopTile / kFlopThreads + 1;
    const int t = threadIdx.x;
    // the tile scalars are uniform: keep them in scalar registers
    c = __builtin_amdgcn_readfirstlane(c);
    const CaseDesc& cd = cs[c];
    R.g = g;
    R.c = c;
    R.Arpt = cd.A.rpt;
    R.Brpt = cd.B.rpt;
    R.blen = cd.blen;
    R.out = MODE == FLOP_ONLY ? cd.rf : cd.out;
    const SSP_GLOBAL int32_t* Acol = cd.A.col;
    const int64_t M = cd.A.nrows, nnzA = cd.A.nnz;
    R.M = M;
    R.nnzA = nnzA;
    R.K = cd.B.nrows;
    const int64_t d0 = (g - cd.tile_base) * kFlopTile;
    const int64_t d1 = (d0 + kFlopTile) < (M + nnzA) ? (d0 + kFlopTile) : (M + nnzA);
    i0 = (int64_t)__builtin_amdgcn_readfirstlane((int)i0);
    i1 = (int64_t)__builtin_amdgcn_readfirstlane((int)i1);
    R.i0 = i0;
    R.i1 = i1;
    R.j0 = d0 - i0;
    R.j1 = d1 - i1;
    R.a0 = R.j0 & ~(int64_t)3;
    const int64_t rlast = i1 < M ? i1 : M - 1;
    const int nb = (int)(rlast - i0 + 2);
    if (VEC) {
        // buffer loads: the row bounds past the tile's read 0 (no clamps)
        const __amdgpu_buffer_rsrc_t rr = buffer_rsrc(R.Arpt + i0, 4 * (uint64_t)nb);
#pragma unroll
        for (int u = 0; u < 2; ++u) {  // rows 4 NT u + 4 t .. + 3, one 16-byte load
            typedef int32_t v4i __attribute__((ext_vector_type(4)));
            const v4i v = __builtin_amdgcn_raw_buffer_load_b128(
                rr, 16u * (uint32_t)t + 16u * (uint32_t)NT * u, 0, 0);
            R.rp[4 * u + 0] = v.x;
            R.rp[4 * u + 1] = v.y;
            R.rp[4 * u + 2] = v.z;
            R.rp[4 * u + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < NRP; ++u) {
            const int k = t + u * NT;
            R.rp[u] = R.Arpt[i0 + (k < nb ? k : nb - 1)];
        }
    }
    // Loads are unconditional (masked later): a load under a lane condition
    // becomes a branch, and loads in separate branches are not kept in flight
    // together.  The fast form (VEC) reads through buffer resources, whose
    // lanes past the end read 0 (per 4-byte word: a 16-byte load that
    // straddles the end still returns the words before it), the other form
    // from clamped addresses.  VEC: each wave loads its 256 entries of a half
    // with one 16-byte load per lane and the tile's row bounds with two per
    // thread, the fewest load instructions for the address units (nine 4-byte
    // loads of row bounds and four of entries per half before: stencil 95 ->
    // 91 us); the other form loads four runs of 64 consecutive entries.  Either
    // way the gathers see consecutive entries in consecutive lanes: in banded
    // and stencil-like rows those name nearby B rows, whose row pointers then
    // share few cache lines per instruction (the first-level cache looks up
    // one line per clock).
    const int lane = t & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(t / kWave);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int64_t sb = R.a0 + q * HALF + 4 * kWave * wv;  // uniform
        if (VEC) {
            // a buffer over the wave's segment: entries past the last read 0;
            // four consecutive entries per lane in one 16-byte load (put in
            // entry order across the lanes through LDS before the gathers)
            // (non-temporal: the stream should not evict B's row pointers)
            const __amdgpu_buffer_rsrc_t rc =
                buffer_rsrc(Acol + (sb < nnzA ? sb : 0), sb < nnzA ? 4 * (uint64_t)(nnzA - sb) : 0);
            typedef int32_t v4i __attribute__((ext_vector_type(4)));
            const v4i v = __builtin_amdgcn_raw_buffer_load_b128(rc, 16u * (uint32_t)lane, 0, 2);
            R.col[4 * q + 0] = v.x;
            R.col[4 * q + 1] = v.y;
            R.col[4 * q + 2] = v.z;
            R.col[4 * q + 3] = v.w;
        } else {
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int64_t p = sb + kWave * l + lane;
                int32_t v = 0;
                if (nnzA > 0)  // A may have no entries (and no column array) at all
                    v = Acol[p < nnzA ? p : nnzA - 1];
                R.col[4 * q + l] = v;
            }
        }
    }
}

// Start row of the tile after global tile g (the case's M after its last tile).
__device__ __forceinline__ int32_t tile_end_row(const CaseDesc* __restrict__ cs,
                                                const int32_t* __restrict__ tile_row,
                                                const int32_t* __restrict__ tile_case,
                                                int64_t ntiles_all, int64_t g)
{
    const int c = tile_case[g];
    return (g + 1 < ntiles_all && tile_case[g + 1] == c) ? tile_row[g + 1]
                                                         : (int32_t)cs[c].A.nrows;
}

template <int MODE, bool VEC>
// (at least six waves per SIMD: the gathers need the waves in flight)
__global__ __launch_bounds__(kFlopThreads) __attribute__((amdgpu_waves_per_eu(6)))
void k_flop(const CaseDesc* __restrict__ cs,
                                                      const int32_t* __restrict__ tile_row,
                                                      const int32_t* __restrict__ tile_case,
                                                      int64_t ntiles_all, TileMeta* meta,
                                                      Ctl* ctl, BinLists L)
{
    constexpr int NT = kFlopThreads, CH = kFlopChunk, HALF = CH / 2;
    constexpr int T = (int)kFlopTile, NRP = kFlopTile / kFlopThreads + 1;
    // the tile's row bounds (T + 2 at most; VEC fills all 8 NT: two 16-byte loads per thread)
    static_assert(T + 2 <= 8 * NT, "row bounds of a tile fit two 16-byte loads per thread");
    __shared__ __align__(16) int32_t s_bnd[8 * NT];
    __shared__ __align__(16) uint32_t s_x[CH];
    __shared__ uint64_t s_pre0[NT], s_pre1[NT];
    __shared__ uint64_t s_w[2 * (NT / kWave)];
    __shared__ uint32_t s_base[4];  // (binning: the bins' offsets of a round of rows)

    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
    const int64_t G = gridDim.x;

    // Start row, case and end row of this workgroup's tiles, staged in LDS
    // kTrow at a time: reading them from LDS does not wait on the vector loads
    // in flight.  Past the last tile: the last tile's case with an empty row
    // range at its M, so the loads of the pipeline's extra issue stay in range.
    constexpr int kTrow = 64;
    __shared__ int32_t s_trow[kTrow + 1], s_tcase[kTrow + 1], s_next[kTrow + 1];
    int64_t b = blockIdx.x;
    if (b >= ntiles_all) return;
    auto stage_all = [&](int64_t bfirst) {  // tiles bfirst + k G, k <= kTrow
        for (int k = t; k <= kTrow; k += NT) {
            const int64_t bk = bfirst + (int64_t)k * G;
            if (bk < ntiles_all) {
                s_trow[k] = tile_row[bk];
                s_tcase[k] = tile_case[bk];
                s_next[k] = tile_end_row(cs, tile_row, tile_case, ntiles_all, bk);
            } else {
                const int cl = tile_case[ntiles_all - 1];
                s_tcase[k] = cl;
                s_trow[k] = s_next[k] = (int32_t)cs[cl].A.nrows;
            }
        }
        __syncthreads();
    };
    int64_t stage_base = b;
    stage_all(stage_base);
    int kk = 0;  // index of tile b in the staged window
    FlopTileRegs cur, nxt;
    flop_issue_tile<MODE, VEC>(cs, b, s_tcase[0], s_trow[0], s_next[0], cur);
    for (;;) {
        const int64_t bn = b + G;
        // 1. gathers of the current tile
        const int64_t i0 = cur.i0, i1 = cur.i1, j0 = cur.j0, j1 = cur.j1, a0 = cur.a0;
        const int64_t M = cur.M;
        const SSP_GLOBAL int32_t* __restrict__ Brpt = cur.Brpt;
        uint32_t x[8];  // (entry q HALF + 256 wave + 64 l + lane in x[4 q + l])
        // VEC: B has fewer than 2^30 rows (the host checks) and its row
        // lengths are in blen, two bytes each, read through a buffer resource
        // at 32-bit byte offsets (one address register per lane; masked lanes
        // read past the end: 0); a saturated length (a row of 65535 entries
        // or more) is read again from the row pointers.  Entry j is live when
        // j0 <= j < j1; relative to a0 both bounds are small (j0 - a0 < 4,
        // j1 - a0 <= kFlopChunk).
        const int rlo = (int)(j0 - a0), rhi = (int)(j1 - a0);
        if (VEC) {
            // the wave's entries, loaded four consecutive per lane, into entry
            // q HALF + 256 wave + 64 l + lane in col[4 q + l] (the wave's own
            // segment of s_x, free until the lengths are written there)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                *reinterpret_cast<uint4*>(&s_x[q * HALF + 4 * kWave * wid + 4 * lane]) =
                    make_uint4((uint32_t)cur.col[4 * q], (uint32_t)cur.col[4 * q + 1],
                               (uint32_t)cur.col[4 * q + 2], (uint32_t)cur.col[4 * q + 3]);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int l = 0; l < 4; ++l)
                    cur.col[4 * q + l] = (int32_t)s_x[q * HALF + kWave * (4 * wid + l) + lane];
            __builtin_amdgcn_wave_barrier();
        }
        // (VEC: 0 or 1, the half of the loaded word that is the length; 2:
        // the length itself)
        uint32_t xodd[8];
        if (VEC) {
            // A.A whose columns stay near the tile's rows (banded,
            // stencil-like): B's row pointers are A's, which the stream has
            // just brought in, so the gathers read them; otherwise the
            // two-byte lengths, whose smaller footprint stays in L2
            // (judged per wave from two of its columns, lane 0's first and
            // lane 63's last: near when both lie within kNearRows of the
            // tile's rows; the choice changes no result)
            bool near = false;
            if (cur.Brpt == cur.Arpt) {
                const int64_t c0 = __builtin_amdgcn_readlane(cur.col[0], 0);
                const int64_t c7 = __builtin_amdgcn_readlane(cur.col[7], kWave - 1);
                near = c0 >= i0 - kNearRows && c0 <= i1 + kNearRows && c7 >= i0 - kNearRows &&
                       c7 <= i1 + kNearRows;
            }
            if (near) {
                const __amdgpu_buffer_rsrc_t brs = buffer_rsrc(Brpt, 4 * (uint64_t)(cur.K + 1));
#pragma unroll
                for (int q = 0; q < 2; ++q) {
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int rel = q * HALF + kWave * (4 * wid + l) + lane;
                        const bool in = rel >= rlo && rel < rhi;
                        typedef int32_t v2i __attribute__((ext_vector_type(2)));
                        const v2i v = __builtin_amdgcn_raw_buffer_load_b64(
                            brs, in ? 4u * (uint32_t)cur.col[4 * q + l] : 0xFFFFFFF8u, 0, 0);
                        x[4 * q + l] = (uint32_t)(v.y - v.x);
                        xodd[4 * q + l] = 2u;
                    }
                }
            } else {
                const __amdgpu_buffer_rsrc_t bls =
                    buffer_rsrc(cur.blen, (2 * (uint64_t)cur.K + 3) & ~3ull);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int rel = q * HALF + kWave * (4 * wid + l) + lane;
                        const bool in = rel >= rlo && rel < rhi;
                        const uint32_t cc = (uint32_t)cur.col[4 * q + l];
                        // (the aligned 4-byte word holding the length: dword
                        // loads run at the full rate of the address unit)
                        x[4 * q + l] = __builtin_amdgcn_raw_buffer_load_b32(
                            bls, in ? 4u * (cc >> 1) : 0xFFFFFFF0u, 0, 0);
                        xodd[4 * q + l] = cc & 1u;
                    }
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const int rel = q * HALF + kWave * (4 * wid + l) + lane;
                    const bool in = rel >= rlo && rel < rhi;
                    const int32_t cc = in ? cur.col[4 * q + l] : 0;
                    uint32_t len = 0;
                    // row 0 of B when masked; with no entries at all (then K
                    // may be 0 and B's row pointers hold one value) nothing is read
                    if (cur.nnzA > 0) len = csr_row_len(Brpt, cc);
                    x[4 * q + l] = in ? len : 0u;
                }
            }
        }
        // 2. loads of the next tile, unconditionally (a branch here would make
        //    the compiler drain every load in flight at its join)
        flop_issue_tile<MODE, VEC>(cs, bn, s_tcase[kk + 1], s_trow[kk + 1], s_next[kk + 1], nxt);
        // 3. the current tile (VEC: the halves of the loaded words; a
        //    saturated length is read from the row pointers, after the next
        //    tile's loads were issued: a lane branch waits for the loads)
        if (VEC) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (xodd[u] == 2u) continue;
                x[u] = xodd[u] ? (x[u] >> 16) : (x[u] & 0xFFFFu);
                if (x[u] == 0xFFFFu) x[u] = csr_row_len(Brpt, cur.col[u]);
            }
        }
        const int64_t rlast = i1 < M ? i1 : M - 1;
        const int nb = (int)(rlast - i0 + 2);
        if (VEC) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
                *reinterpret_cast<int4*>(&s_bnd[4 * NT * u + 4 * t]) =
                    make_int4(cur.rp[4 * u], cur.rp[4 * u + 1], cur.rp[4 * u + 2], cur.rp[4 * u + 3]);
        } else {
#pragma unroll
            for (int u = 0; u < NRP; ++u) {
                const int k = t + u * NT;
                if (u * NT < nb && k < nb) s_bnd[k] = cur.rp[u];
            }
        }
        // the lengths in entry order; each thread then takes its four
        // consecutive entries of each half (the wave's own segment of s_x:
        // LDS operations of a wave complete in order, no barrier needed)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int l = 0; l < 4; ++l) s_x[q * HALF + kWave * (4 * wid + l) + lane] = x[4 * q + l];
        __builtin_amdgcn_wave_barrier();
        const uint4 xq0 = *reinterpret_cast<const uint4*>(&s_x[4 * t]);
        const uint4 xq1 = *reinterpret_cast<const uint4*>(&s_x[HALF + 4 * t]);
        const uint64_t s0 = (uint64_t)xq0.x + xq0.y + xq0.z + xq0.w;
        const uint64_t s1 = (uint64_t)xq1.x + xq1.y + xq1.z + xq1.w;
        // exclusive scans of the two halves, in lockstep; in 32 bits when
        // every length the wave holds is below 2^21 (its sums then stay below
        // 2^29), the usual case
        const uint32_t orx = xq0.x | xq0.y | xq0.z | xq0.w | xq1.x | xq1.y | xq1.z | xq1.w;
        uint64_t i0s, i1s;
        if (!__any(orx >= (1u << 21))) {
            i0s = wave_incl_scan<uint32_t>((uint32_t)s0);
            i1s = wave_incl_scan<uint32_t>((uint32_t)s1);
        } else {
            i0s = wave_incl_scan(s0);
            i1s = wave_incl_scan(s1);
        }
        if (lane == kWave - 1) {
            s_w[wid] = i0s;
            s_w[NT / kWave + wid] = i1s;
        }
        __syncthreads();
        uint64_t w0 = 0, w1 = 0, tot0 = 0, tot1 = 0;
#pragma unroll
        for (int w = 0; w < NT / kWave; ++w) {
            const uint64_t x0 = s_w[w], x1 = s_w[NT / kWave + w];
            w0 += (w < wid) ? x0 : 0;
            w1 += (w < wid) ? x1 : 0;
            tot0 += x0;
            tot1 += x1;
        }
        s_pre0[t] = w0 + i0s - s0;
        s_pre1[t] = tot0 + w1 + i1s - s1;
        __syncthreads();
        const uint64_t tile_total = tot0 + tot1;

        // running product count before entry position `pos` (a0 <= pos <= a0 + CH)
        auto prefix = [&](int64_t pos) -> uint64_t {
            const int d = (int)(pos - a0);
            if (d >= CH) return tile_total;
            const int q = d >> 10, tt = (d & (HALF - 1)) >> 2, l = d & 3;
            uint64_t v = q ? s_pre1[tt] : s_pre0[tt];
            const int base = q * HALF + 4 * tt;
            for (int m = 0; m < l; ++m) v += s_x[base + m];
            return v;
        };

        const int nrows_t = (int)(rlast - i0 + 1);
        for (int base = 0; base < nrows_t; base += NT) {  // same trip count in every lane
            const int k = base + t;
            bool emit = false;
            int64_t r = 0;
            uint64_t sum = 0;
            if (k < nrows_t) {
                r = i0 + k;
                const int64_t rs = s_bnd[k], re = s_bnd[k + 1];
                const bool open = (r == i1);
                if (!(open && rs >= j1)) {
                    const int64_t st_ = rs > j0 ? rs : j0;
                    const int64_t en = re < j1 ? re : j1;
                    sum = prefix(en) - prefix(st_);
                    if (rs < j0) meta[cur.g].head = sum;
                    else if (open) meta[cur.g].carry = sum;
                    else emit = true;
                }
            }
            if (MODE == FLOP_EXACT_BIN) {
                const CaseDesc& cd = cs[cur.c];
                const int bn_ = emit ? bin_route(sum, cd) : 0;
                // (s_w is free here: the tile's scans are done)
                block_append_small_bins<NT>(bn_, (int32_t)r, sum, cur.c, ctl, L, s_w, s_base);
                if (emit && (bn_ == 0 || bn_ == 4)) cur.out[r] = 0;
                if (emit && bn_ == 4)
                    append_big((int32_t)r, sum, s_bnd[k], s_bnd[k + 1], cur.c, cd, ctl, L);
            } else if (emit) {
                __builtin_nontemporal_store((int64_t)sum, cur.out + r);
            }
        }
        if (t == 0) meta[cur.g].fsum = tile_total;
        __syncthreads();  // s_bnd, s_x and the prefixes are rewritten for the next tile
        if (bn >= ntiles_all) break;
        b = bn;
        cur = nxt;
        if (++kk == kTrow) {  // restage; k = 0..kTrow are staged, so kk + 1 always is
                              // (the barrier above ends every read of the staged window)
            stage_base = b;
            stage_all(stage_base);
            kk = 0;
        }
    }
}

// One thread per global tile: a row that begins in tile g and goes on (its
// partial is g's carry) collects the heads of the case's following tiles up to
// the tile holding its end marker, then gets its output.  Adds each case's F:
// one atomic for the workgroup's first case, one per tile of any other case.
template <int MODE>
__global__ __launch_bounds__(256) void k_flop_fixup(const CaseDesc* __restrict__ cs,
                                                   const int32_t* __restrict__ tile_row,
                                                   const int32_t* __restrict__ tile_case,
                                                   int64_t ntiles_all, const TileMeta* meta,
                                                   Ctl* ctl, BinLists L)
{
    __shared__ uint64_t s_red[256 / kWave + 1];
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t g_first = (int64_t)blockIdx.x * 256;
    const int c0 = tile_case[g_first];  // (the grid covers ntiles_all, so g_first is a tile)
    uint64_t F = 0;
    int bin = 0;  // (binning: a small-bin row that ends here, appended by the whole wave)
    int32_t brow = 0, bcase = 0;
    uint64_t brf = 0;
    if (g < ntiles_all) {
        const int c = tile_case[g];
        const CaseDesc& cd = cs[c];
        const int64_t M = cd.A.nrows, nnzA = cd.A.nnz;
        const int64_t last = cd.tile_base + cd.ntiles;  // one past the case's last tile
        const int64_t d0 = (g - cd.tile_base) * kFlopTile;
        const int64_t d1 = (d0 + kFlopTile) < (M + nnzA) ? (d0 + kFlopTile) : (M + nnzA);
        const int64_t i1 = tile_end_row(cs, tile_row, tile_case, ntiles_all, g);
        const int64_t j0 = d0 - tile_row[g], j1 = d1 - i1;
        if (i1 < M) {
            const int64_t rs = cd.A.rpt[i1];
            if (rs >= j0 && rs < j1) {
                // the tile holding the row's end marker, item i1 + rpt[i1 + 1]
                // of the merged sequence; the heads up to it are independent
                // loads, eight in flight
                const int64_t e = cd.tile_base + (i1 + (int64_t)cd.A.rpt[i1 + 1]) / kFlopTile;
                const int64_t bend = e < last - 1 ? e : last - 1;
                uint64_t total = meta[g].carry;
                for (int64_t bb = g + 1; bb <= bend; bb += 8) {
                    uint64_t hd[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) hd[u] = bb + u <= bend ? meta[bb + u].head : 0;
#pragma unroll
                    for (int u = 0; u < 8; ++u) total += hd[u];
                }
                if (MODE == FLOP_ONLY) {
                    emit_row<MODE>(cs, c, i1, total, ctl, L);
                } else {
                    const int b = bin_route(total, cd);
                    if (b == 0 || b == 4) cd.out[i1] = 0;
                    if (b == 4)
                        append_big((int32_t)i1, total, cd.A.rpt[i1], cd.A.rpt[i1 + 1], c, cd, ctl, L);
                    bin = b == 4 ? 0 : b;
                    brow = (int32_t)i1;
                    bcase = c;
                    brf = total;
                }
            }
        }
        if (c == c0) F = meta[g].fsum;
        else if (meta[g].fsum) atomicAdd(as_ull(&cd.st->total_flop), (ull)meta[g].fsum);
    }
    if (MODE != FLOP_ONLY) append_small_bins(bin, brow, brf, bcase, ctl, L);  // (every lane)
    const uint64_t Fs = block_sum<256, uint64_t>(F, s_red);
    if (threadIdx.x == 0 && Fs) atomicAdd(as_ull(&cs[c0].st->total_flop), (ull)Fs);
}

// ------------------------------------------------------ prediction rows

constexpr int kRowsThreads = 1024;

// nnz_pred[i] = ceil(rf_i z* / f*) (Eq. (4) per row), rf_i when the sample has
// no products.  Grid-stride (at least one workgroup per case, rows or not):
// a step covers U G blocks of kRowsThreads rows and workgroup bl takes the
// blocks bl, bl + G, ..., so even a case of few rows spreads over every
// workgroup it is given; each adds its part of the output total with one
// atomic.  Every wave sums its case's distinct-count slots into z* itself (no
// barrier before the rows); the case's first workgroup records z* and the
// empty-sample flag in the statistics.  Rows of fewer than est_max_rf (at
// most 2^48) products take the double-precision estimate with an integer
// correction (exact, see ceil_mul_div_est), the others the 128-bit division,
// with the divisor derived where it is needed.
__global__ __launch_bounds__(kRowsThreads) void k_pred_rows(const CaseDesc* __restrict__ cs, int n,
                                                            const CaseRes* __restrict__ cr)
{
    __shared__ uint64_t s_red[kRowsThreads / kWave + 1];
    const int c = case_of_wg<&CaseDesc::wg_rows>(cs, n, blockIdx.x);
    const int64_t bl = (int64_t)blockIdx.x - cs[c].wg_rows;
    const int64_t G = wgs_of_case<&CaseDesc::wg_rows>(cs, n, c);
    const SSP_GLOBAL int64_t* __restrict__ rf_in = cs[c].rf;
    SSP_GLOBAL int64_t* __restrict__ out = cs[c].out;
    const int64_t M = cs[c].A.nrows;
    ssp_stats* st = cs[c].st;
    static_assert(kAccSlots == kWave, "one slot per lane");
    // Loads issued at once: the case's f*, its distinct-count slots, and the
    // first step's row products (none of them waits on another).
    const uint64_t fs = uniform_u64(st->sample_flop);
    const uint64_t z_ld = cr[c].zacc[lane_id()];
    constexpr int U = 4;  // rows per thread and step, loaded together
    const int64_t bstride = G * kRowsThreads, stride = bstride * U;
    uint64_t rf[U];
    auto load_rows = [&](int64_t i0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * bstride;
            rf[u] = i < M ? (uint64_t)__builtin_nontemporal_load(rf_in + i) : 0;
        }
    };
    const int64_t first = bl * kRowsThreads + threadIdx.x;
    load_rows(first);
    const uint64_t zs = wave_sum(z_ld);
    const bool fallback = fs == 0;
    const bool est = fs < kEstMaxD;  // (z* <= f*: a row has no more columns than products)
    const uint64_t est_max = cs[c].est_max_rf;  // (at most kEstMaxA)
    const double ratio = fallback ? 0.0 : (double)zs / (double)fs;
    if (bl == 0 && threadIdx.x == 0) {
        st->sample_nnz = zs;
        if (fallback) atomicOr(as_ull(&st->flags), (ull)SSP_FLAG_EMPTY_SAMPLE);
    }
    uint64_t osum = 0;
    for (int64_t i0 = first; i0 < M; i0 += stride) {
        if (i0 != first) load_rows(i0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * bstride;
            if (i < M) {
                const uint64_t a = rf[u];
                const uint64_t pred = fallback ? a
                                      : a == 0 ? 0
                                      : (est && a < est_max) ? ceil_mul_div_est(a, zs, fs, ratio)
                                                              : ceil_mul_div(a, zs, make_divisor(fs));
                __builtin_nontemporal_store((int64_t)pred, out + i);
                osum += pred;
            }
        }
    }
    const uint64_t O = block_sum<kRowsThreads, uint64_t>(osum, s_red);
    if (threadIdx.x == 0 && O) atomicAdd(as_ull(&st->out_sum), (ull)O);
}

// --------------------------------------------------- reference rows

// nnz_ref[i] = ceil(rf_i * (z* M) / (n_s F)).  The value is at most M N <
// 2^62 (z* <= n_s N, rf_i <= F) but the numerator can exceed 128 bits (rf_i <
// 2^62, z* M < 2^93): such rows divide the 192-bit product.  Grid-stride like
// k_pred_rows.
__global__ __launch_bounds__(kRowsThreads) void k_ref_rows(const CaseDesc* __restrict__ cs, int n,
                                                           const CaseRes* __restrict__ cr)
{
    __shared__ uint64_t s_red[kRowsThreads / kWave + 1];
    const int c = case_of_wg<&CaseDesc::wg_rows>(cs, n, blockIdx.x);
    const int64_t bl = (int64_t)blockIdx.x - cs[c].wg_rows;
    const int64_t G = wgs_of_case<&CaseDesc::wg_rows>(cs, n, c);
    const SSP_GLOBAL int64_t* __restrict__ rf_in = cs[c].rf;
    SSP_GLOBAL int64_t* __restrict__ out = cs[c].out;
    const int64_t M = cs[c].A.nrows;
    ssp_stats* st = cs[c].st;
    const uint32_t fallback = cr[c].fallback;
    const u128 Q = {cr[c].ref_q_lo, cr[c].ref_q_hi};
    const u128 Dd = {cr[c].ref_d_lo, cr[c].ref_d_hi};
    uint64_t osum = 0;
    const int64_t stride = G * kRowsThreads;
    for (int64_t i = bl * kRowsThreads + threadIdx.x; i < M; i += stride) {
        const uint64_t rf = (uint64_t)rf_in[i];
        uint64_t v = rf;
        if (!fallback && rf != 0) {
            // rf Q = (l2, l1, p0.lo)
            const u128 p0 = mul_64x64(rf, Q.lo), p1 = mul_64x64(rf, Q.hi);
            const uint64_t l1 = p0.hi + p1.lo;
            const uint64_t l2 = p1.hi + (l1 < p0.hi);
            v = l2 == 0 ? u128_ceil_div(u128{p0.lo, l1}, Dd).lo
                        : ceil_div_192_by_128(l2, l1, p0.lo, Dd);
        }
        out[i] = (int64_t)v;
        osum += v;
    }
    const uint64_t O = block_sum<kRowsThreads, uint64_t>(osum, s_red);
    if (threadIdx.x == 0 && O) atomicAdd(as_ull(&st->out_sum), (ull)O);
}

// ------------------------------------------------------------ validate

__global__ void k_zero_i64(int64_t* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ __launch_bounds__(256) void k_validate(Csr m, int64_t* n_bad)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    uint64_t bad = 0;
    for (int64_t i = g; i <= m.nrows; i += stride) {
        if (i == 0 && m.rpt[0] != 0) ++bad;
        if (i == m.nrows && (int64_t)m.rpt[m.nrows] != m.nnz) ++bad;
        if (i < m.nrows && m.rpt[i + 1] < m.rpt[i]) ++bad;
    }
    for (int64_t j = g; j < m.nnz; j += stride) {
        const int32_t c = m.col[j];
        if (c < 0 || (int64_t)c >= m.ncols) ++bad;
    }
    bad = wave_sum(bad);
    if (lane_id() == 0 && bad) atomicAdd(reinterpret_cast<ull*>(n_bad), (ull)bad);
}

} // namespace ssp
