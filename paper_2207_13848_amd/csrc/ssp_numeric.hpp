// Kernels of the numeric product C = A.B that consumes a predicted structure
// (Sec. I: the output structure is predicted so that C's memory can be
// allocated, and the numeric phase balanced, without a symbolic pass).
//
// Layout.  Row i of C gets a slot of s_i entries, s_i from the caller's
// per-row capacity (normally the prediction of Eq. (4)) and a margin; the
// slots are laid out by an exclusive scan of s_i.  One numeric pass
// accumulates every row once, counts its nonzeros and writes the row (columns
// increasing) into its slot when it fits.  The exact counts then give C's row
// offsets; a copy pass packs the rows that fitted and a fallback pass
// recomputes the rows that overflowed straight into their final place.
//
// Rows are binned by their product count (the row-FLOP pass of Alg. 1 routes
// them): up to kNumBin3Max products an LDS hash table of (column, value)
// pairs, more a dense accumulator of N values in global memory with a column
// bitmap, one per workgroup of a persistent grid.
#pragma once

#include "ssp_kernels.hpp"

namespace ssp {

// Product limits of the numeric bins and their LDS tables (slots of a 4-byte
// key and an 8-byte value; a table holds at least twice the row's bound on
// its distinct columns).
constexpr uint64_t kNumBin1Max = 128, kNumBin2Max = 1024, kNumBin3Max = 2048;
constexpr int kNumSlots1 = 256, kNumSlots2 = 2048, kNumSlots3 = 4096;
constexpr int kNumTeam1 = 64, kNumTeam2 = 256, kNumTeam3 = 512, kNumDenseTeam = 1024;
// Device-wide scans: kNumScanThreads threads x kNumScanRows rows per workgroup.
constexpr int kNumScanThreads = 1024, kNumScanRows = 8;
constexpr int64_t kNumScanBlock = (int64_t)kNumScanThreads * kNumScanRows;
constexpr int32_t kNumMarginMax = 10000;  // percent
constexpr int kNumCopyRows = 256;         // rows per workgroup of the copy pass

// A run of a row's entries kept in the overflow area: `n` entries from
// position `pos` of the row (in column order) at offset `off` of the area.
struct SpillRec {
    int64_t off;
    int32_t row, pos, n, pad;
};

// Overflow area: the rows share it through one 64-bit counter (agg[6]) that
// holds the records taken above bit kSpillShift and the area's entries taken
// below.  A longer row takes the area in chunks of sp_chunk entries (at most
// kSpillChunk; smaller when the area is small for the workgroups that may
// hold a chunk each) for its workgroup, so its entries past the slot form few
// runs.
constexpr int kSpillShift = 40;
constexpr int64_t kSpillChunk = 1 << 16;
constexpr int64_t kSpillCapMax = 1LL << 38;   // area entries, at most
constexpr int64_t kSpillRecMax = 1LL << 23;   // records, at most

// Arguments of the numeric kernels (one product per call; its CSR arrays are
// in the case table).
struct NumArgs {
    const SSP_GLOBAL double* Aval;
    const SSP_GLOBAL double* Bval;
    const SSP_GLOBAL int64_t* cap;  // per-row capacities (the caller's)
    SSP_GLOBAL int64_t* slot_off;   // M + 1: exclusive prefix of the slot sizes
    SSP_GLOBAL int64_t* cnt;        // M: nonzeros of every row (numeric pass)
    SSP_GLOBAL int32_t* slot_col;   // slot area: columns
    SSP_GLOBAL double* slot_val;    //            values
    SSP_GLOBAL int64_t* C_rpt;      // M + 1: row offsets of C (the caller's)
    SSP_GLOBAL int32_t* C_col;      // C (the caller's; copy pass)
    SSP_GLOBAL double* C_val;
    int64_t capacity;               // entries of C_col / C_val
    int64_t M, N;
    SSP_GLOBAL double* pool;        // dense accumulators: pool_slots x N values, zero between rows
    SSP_GLOBAL uint32_t* pool_mask; // their column bitmaps: pool_slots x mask_words, zero between rows
    int64_t mask_words;
    int32_t pool_slots;
    int32_t margin;                 // percent added to each capacity
    SSP_GLOBAL int64_t* part;       // per-block partials of the scans: 5 x blocks
    // [0] NNZ(C) [1] overflow rows [2] their nonzeros [3] slot entries [4] longest A row of
    // a long row [5] B unsorted [6] overflow-area counter [8] rows the area holds [9] their
    // entries there
    SSP_GLOBAL uint64_t* agg;
    SSP_GLOBAL int32_t* sp_col;     // overflow area (sp_cap entries): columns
    SSP_GLOBAL double* sp_val;      //                                 values
    SSP_GLOBAL SpillRec* sp_rec;    // its records (rec_cap)
    SSP_GLOBAL uint8_t* sp_state;   // M: 0 the row is not in the area, 1 its first s_i entries
                                    // are in its slot and the rest in records, 2 all in records
    int64_t sp_cap, rec_cap, sp_chunk;
};
constexpr int kNumAgg = 16;

// Takes n entries of the overflow area and, with `rec`, one record: their
// offsets, or false when the area or the records are used up.  The counter
// is read first, so calls after the area has run out leave it unchanged (it
// overshoots by at most the calls in flight: no carry into the record field).
// Every record below the final record count is written: one taken by a call
// that then fails (the area ran out meanwhile) is written empty (row -1).
__device__ __forceinline__ bool spill_take(const NumArgs& na, int64_t n, bool rec, int64_t* off,
                                           int64_t* r)
{
    constexpr uint64_t kLow = (1ull << kSpillShift) - 1;
    SSP_GLOBAL uint64_t* ctr = &na.agg[6];
    const uint64_t cur = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int64_t)(cur & kLow) + n > na.sp_cap || (rec && (int64_t)(cur >> kSpillShift) >= na.rec_cap))
        return false;
    const uint64_t add = (rec ? (1ull << kSpillShift) : 0ull) + (uint64_t)n;
    const uint64_t old = __hip_atomic_fetch_add(ctr, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *off = (int64_t)(old & kLow);
    *r = (int64_t)(old >> kSpillShift);
    const bool rec_ok = rec && *r < na.rec_cap;
    if (*off + n <= na.sp_cap && (!rec || rec_ok)) return true;
    if (rec_ok) {  // (a record below the final count: written, empty)
        SpillRec x;
        x.off = 0;
        x.row = -1;
        x.pos = 0;
        x.n = 0;
        x.pad = 0;
        na.sp_rec[*r] = x;
    }
    return false;
}

// Records a run of a row (false when the records are used up).
__device__ __forceinline__ bool spill_record(const NumArgs& na, int64_t row, int64_t pos,
                                             int64_t off, int64_t n)
{
    int64_t o, r;
    if (!spill_take(na, 0, true, &o, &r)) return false;
    SpillRec x;
    x.off = off;
    x.row = (int32_t)row;
    x.pos = (int32_t)pos;
    x.n = (int32_t)n;
    x.pad = 0;
    na.sp_rec[r] = x;
    return true;
}

// The area for a whole row of c entries, with its record: the offset in *off.
__device__ __forceinline__ bool spill_take_row(const NumArgs& na, int64_t row, int64_t c,
                                               int64_t* off)
{
    int64_t o, r;
    if (!spill_take(na, c, true, &o, &r)) return false;
    SpillRec x;
    x.off = o;
    x.row = (int32_t)row;
    x.pos = 0;
    x.n = (int32_t)c;
    x.pad = 0;
    na.sp_rec[r] = x;
    *off = o;
    return true;
}

// Slot size of a row: its capacity clamped to [0, N], plus ceil(margin %),
// at most N (a row of C has at most N entries).
__device__ __forceinline__ int64_t num_slot_size(int64_t cap, int32_t margin, int64_t N)
{
    const int64_t c = cap < 0 ? 0 : (cap > N ? N : cap);
    const int64_t s = c + (c * margin + 99) / 100;
    return s < N ? s : N;
}

// Whether row i's nonzeros fit its slot (decided after the numeric pass).
__device__ __forceinline__ bool num_fits(const NumArgs& na, int64_t i, int64_t c)
{
    return c <= na.slot_off[i + 1] - na.slot_off[i];
}

// ------------------------------------------------------------------ scans

// Value of row i in scan KIND: 0 the slot size, 1 the row's nonzeros.  KIND 1
// also counts the overflowing rows and their nonzeros.
template <int KIND>
__device__ __forceinline__ int64_t num_scan_value(const NumArgs& na, int64_t i, int64_t* o)
{
    if (KIND == 0) return num_slot_size(na.cap[i], na.margin, na.N);
    const int64_t c = na.cnt[i];
    if (!num_fits(na, i, c)) {
        o[0] += 1;
        o[1] += c;
        const int st = na.sp_state[i];
        if (st) {
            o[2] += 1;
            o[3] += st == 1 ? c - (na.slot_off[i + 1] - na.slot_off[i]) : c;
        }
    }
    return c;
}

// Pass 1 of a scan: the sums of every block of kNumScanBlock rows.
template <int KIND>
__global__ __launch_bounds__(kNumScanThreads) void k_num_scan_part(NumArgs na)
{
    __shared__ int64_t s_red[kNumScanThreads / kWave + 1];
    const int64_t nblk = (na.M + kNumScanBlock - 1) / kNumScanBlock;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        int64_t sum = 0, o[4] = {0, 0, 0, 0};
        const int64_t r0 = b * kNumScanBlock + (int64_t)threadIdx.x * kNumScanRows;
#pragma unroll
        for (int u = 0; u < kNumScanRows; ++u)
            if (r0 + u < na.M) sum += num_scan_value<KIND>(na, r0 + u, o);
        sum = block_sum<kNumScanThreads, int64_t>(sum, s_red);
        if (KIND == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = block_sum<kNumScanThreads, int64_t>(o[q], s_red);
        }
        if (threadIdx.x == 0) {
            na.part[b] = sum;
            if (KIND == 1) {
#pragma unroll
                for (int q = 0; q < 4; ++q) na.part[(q + 1) * nblk + b] = o[q];
            }
        }
    }
}

// Pass 2 (one workgroup): exclusive scan of the block sums in place, the
// total at out[M], the aggregates.
template <int KIND>
__global__ __launch_bounds__(kNumScanThreads) void k_num_scan_top(NumArgs na)
{
    __shared__ int64_t s_red[kNumScanThreads / kWave + 1];
    const int64_t nblk = (na.M + kNumScanBlock - 1) / kNumScanBlock;
    SSP_GLOBAL int64_t* out = KIND == 0 ? na.slot_off : na.C_rpt;
    int64_t run = 0, o[4] = {0, 0, 0, 0};
    for (int64_t b0 = 0; b0 < nblk; b0 += kNumScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nblk ? na.part[b] : 0;
        if (KIND == 1 && b < nblk) {
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] += na.part[(q + 1) * nblk + b];
        }
        int64_t tot;
        const int64_t ex = block_excl_scan<kNumScanThreads, int64_t>(v, s_red, &tot);
        if (b < nblk) na.part[b] = run + ex;
        run += tot;
    }
    if (KIND == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = block_sum<kNumScanThreads, int64_t>(o[q], s_red);
    }
    if (threadIdx.x == 0) {
        out[na.M] = run;
        if (KIND == 0) {
            na.agg[3] = (uint64_t)run;
        } else {
            na.agg[0] = (uint64_t)run;
            na.agg[1] = (uint64_t)o[0];
            na.agg[2] = (uint64_t)o[1];
            na.agg[8] = (uint64_t)o[2];
            na.agg[9] = (uint64_t)o[3];
        }
    }
}

// Pass 3: every row's exclusive prefix.
template <int KIND>
__global__ __launch_bounds__(kNumScanThreads) void k_num_scan_rows(NumArgs na)
{
    __shared__ int64_t s_red[kNumScanThreads / kWave + 1];
    const int64_t nblk = (na.M + kNumScanBlock - 1) / kNumScanBlock;
    SSP_GLOBAL int64_t* out = KIND == 0 ? na.slot_off : na.C_rpt;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t r0 = b * kNumScanBlock + (int64_t)threadIdx.x * kNumScanRows;
        int64_t v[kNumScanRows], sum = 0;
#pragma unroll
        for (int u = 0; u < kNumScanRows; ++u) {
            v[u] = r0 + u < na.M ? (KIND == 0 ? num_slot_size(na.cap[r0 + u], na.margin, na.N)
                                              : na.cnt[r0 + u])
                                 : 0;
            sum += v[u];
        }
        int64_t tot;
        int64_t run = na.part[b] + block_excl_scan<kNumScanThreads, int64_t>(sum, s_red, &tot);
#pragma unroll
        for (int u = 0; u < kNumScanRows; ++u) {
            if (r0 + u < na.M) out[r0 + u] = run;
            run += v[u];
        }
    }
}

// ----------------------------------------------------------- LDS hash bins

// Rows of at most kNumBin3Max products accumulate in an LDS hash table of
// (column, value) slots: 2^lg slots, at least twice the bound b on the
// distinct columns the pass must hold.  The first pass only has to keep the
// rows that fit their slot, so b = min(products, N, slot size); a row whose
// columns outnumber the table stops (every probe sequence ends after 2^lg
// steps) and is counted by the symbolic kernel instead.  With an overflow
// area, a row longer than its slot that completes with at most half its
// table goes to the area whole, and rows get b = min(products, N), so they
// all complete, unless that would move a row whose slot's table fits one
// wave to the workgroup kernel (a row of 125 distinct columns among 729
// products, as in the squared 27-point stencil, stays in the one-wave
// kernel: moving all such rows took that pass from 8.9 to 17.4 ms on the
// 128^3 grid).  The fallback pass knows each row's exact count and sizes b by
// it.
constexpr int kNumWaveSlots = 512;  // table of a row handled by one wave
constexpr int kNumUnroll = 4;       // products per lane whose loads are in flight together
constexpr int kNumWaveWaves = 4;    // such rows per workgroup

__device__ __forceinline__ uint32_t num_table_size(uint64_t b)
{
    uint32_t t = 32;
    while ((uint64_t)t < 2 * b) t <<= 1;
    return t;
}

// Bound on the distinct columns of a bin item's row that the pass must hold.
template <int PASS>
__device__ __forceinline__ uint64_t num_bound(const NumArgs& na, int64_t row, uint32_t rf)
{
    if (PASS == 2) return (uint64_t)na.cnt[row];
    const int64_t s = na.slot_off[row + 1] - na.slot_off[row];
    const int64_t b = (int64_t)rf < na.N ? (int64_t)rf : na.N;
    // (2 b <= kNumWaveSlots: the table for all the products fits one wave;
    // 2 s > kNumWaveSlots: the slot's table does not)
    const bool all = na.sp_cap > 0 && (2 * b <= kNumWaveSlots || 2 * s > kNumWaveSlots);
    return (uint64_t)(b <= s || all ? b : s);
}

// Adds v to column c's slot (open addressing, linear probing; columns are
// < 2^31, so the all-ones key marks a free slot).  False when all 2^lg slots
// hold other columns.
__device__ __forceinline__ bool num_hash_add(uint32_t* keys, double* vals, uint32_t c, double v,
                                             int lg)
{
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t h = (c * 0x9E3779B1u) >> (32 - lg);
    for (uint32_t n = 0; n <= mask; ++n) {
        // (one compare-and-swap per probe: its returned word tells an
        // insert, a repeat and an occupied slot apart)
        const uint32_t prev = atomicCAS(&keys[h], kEmpty, c);
        if (prev == kEmpty || prev == c) {
            __hip_atomic_fetch_add(&vals[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return true;
        }
        h = (h + 1u) & mask;
    }
    return false;
}

// Item k of the hash bins 1..3 taken as one list.
__device__ __forceinline__ BinItem num_hash_item(const BinLists& L, const uint32_t* cnt, uint32_t k)
{
    const uint32_t n1 = cnt[1], n2 = cnt[2];
    return k < n1 ? L.b1[k] : k < n1 + n2 ? L.b2[k - n1] : L.b3[k - n1 - n2];
}

// Records a row whose first-pass table filled up (the symbolic kernel counts it).
__device__ __forceinline__ void num_abort_row(int64_t row, uint32_t rf, Ctl* ctl, BinItem* list)
{
    const uint32_t i = atomicAdd(&ctl->num_abort, 1u);
    BinItem it;
    it.row = (int32_t)row;
    it.rf = rf;
    it.cs = 0;
    it.pad = 0;
    list[i] = it;
}

// Writes the c occupied slots of a table, columns increasing, at dst: each
// entry's place is its rank among the row's (distinct) keys.  The caller has
// compacted the entries to keys/vals[0, c) and set keys[c, c4) to kEmpty
// (c4 = c rounded up to 4).  EPT entries per lane (c <= EPT * NT); the rank
// loop costs c * EPT compares per lane, so the caller picks the smallest EPT.
template <int NT, int EPT>
__device__ __forceinline__ void num_write_ranked_n(const uint32_t* keys, const double* vals,
                                                   uint32_t c, int tid, SSP_GLOBAL int32_t* ocol,
                                                   SSP_GLOBAL double* oval, int64_t dst)
{
    const uint32_t c4 = (c + 3u) & ~3u;
    uint32_t key[EPT], rank[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const uint32_t e = (uint32_t)tid + (uint32_t)u * NT;
        key[u] = e < c ? keys[e] : kEmpty;
        rank[u] = 0;
    }
    for (uint32_t q = 0; q < c4; q += 4) {
        const uint4 k4 = *reinterpret_cast<const uint4*>(&keys[q]);
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            rank[u] += (k4.x < key[u]) + (k4.y < key[u]) + (k4.z < key[u]) + (k4.w < key[u]);
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const uint32_t e = (uint32_t)tid + (uint32_t)u * NT;
        if (e < c) {
            ocol[dst + rank[u]] = (int32_t)key[u];
            oval[dst + rank[u]] = vals[e];
        }
    }
}

// The same with the entries per lane chosen from c (uniform over the team):
// 1, 2, then EPT_MAX.
template <int NT, int EPT_MAX>
__device__ __forceinline__ void num_write_ranked(const uint32_t* keys, const double* vals,
                                                 uint32_t c, int tid, SSP_GLOBAL int32_t* ocol,
                                                 SSP_GLOBAL double* oval, int64_t dst)
{
    if (c <= (uint32_t)NT)
        num_write_ranked_n<NT, 1>(keys, vals, c, tid, ocol, oval, dst);
    else if (EPT_MAX > 2 && c <= 2u * NT)
        num_write_ranked_n<NT, (EPT_MAX > 2 ? 2 : EPT_MAX)>(keys, vals, c, tid, ocol, oval, dst);
    else
        num_write_ranked_n<NT, EPT_MAX>(keys, vals, c, tid, ocol, oval, dst);
}

// Rows whose table has at most kNumWaveSlots slots: one wave per row,
// kNumWaveWaves rows per workgroup, each wave with its own table.  The row's
// products are enumerated 64 entries of A at a time (a wave scan of the B row
// lengths gives each product's entry by a search over the lanes' offsets with
// cross-lane reads: no LDS beyond the tables, so six workgroups fit a CU
// instead of five; the squared 128^3 stencil's pass 6.8 -> 6.3 ms).
// PASS 1: count the row, write it to its slot when it fits.
// PASS 2: rows that did not fit, written to C at their final offset.
template <int PASS>
__global__ __launch_bounds__(kNumWaveWaves* kWave) void k_num_wave(const CaseDesc* __restrict__ cs,
                                                                   BinLists L, Ctl* ctl,
                                                                   BinItem* abort_list, NumArgs na)
{
    constexpr int SPT = kNumWaveSlots / kWave;  // table slots per lane
    constexpr int EPT = SPT / 2;                 // written entries per lane, at most
    __shared__ __align__(16) uint32_t s_keys[kNumWaveWaves][kNumWaveSlots];
    __shared__ double s_vals[kNumWaveWaves][kNumWaveSlots];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t* keys = s_keys[w];
    double* vals = s_vals[w];
    const uint32_t* cnt = ctl->bin_cnt;
    const uint32_t total = cnt[1] + cnt[2] + cnt[3];
    const Csr A = cs[0].A, B = cs[0].B;
    const uint64_t stride = (uint64_t)gridDim.x * kNumWaveWaves;
    // The wave's items are k0 + j * stride; 64 of them are looked at together,
    // one per lane, and the wave then takes the rows it owns (a table of at
    // most kNumWaveSlots slots, not yet done) in order, each from its lane.
    for (uint64_t k0 = (uint64_t)blockIdx.x * kNumWaveWaves + w; k0 < total;
         k0 += stride * kWave) {
        const uint64_t km = k0 + (uint64_t)lane * stride;
        uint32_t lgm = 0;
        BinItem x{};
        if (km < total) {
            x = num_hash_item(L, cnt, (uint32_t)km);
            if (!(PASS == 2 && (num_fits(na, x.row, na.cnt[x.row]) || na.sp_state[x.row]))) {
                const uint32_t Tm = num_table_size(num_bound<PASS>(na, x.row, x.rf));
                if (Tm <= (uint32_t)kNumWaveSlots) lgm = (uint32_t)__builtin_ctz(Tm);
            }
        }
        uint64_t todo = __ballot(lgm != 0);
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const BinItem item{__builtin_amdgcn_readlane(x.row, src),
                               (uint32_t)__builtin_amdgcn_readlane((int)x.rf, src), 0, 0};
            const int64_t row = item.row;
            const int lg = __builtin_amdgcn_readlane((int)lgm, src);
            const uint32_t T = 1u << lg;
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const uint32_t s = (uint32_t)lane + (uint32_t)u * kWave;
                if (s < T) {
                    keys[s] = kEmpty;
                    vals[s] = 0.0;
                }
            }
            wave_sync();
            bool ok = true;
            const int32_t a0 = A.rpt[row], a1 = A.rpt[row + 1];
            for (int32_t a = a0; a < a1; a += kWave) {
                const int32_t j = a + lane;
                uint32_t len = 0;
                int32_t b0 = 0;
                double av = 0.0;
                if (j < a1) {
                    const int32_t kk = A.col[j];
                    b0 = B.rpt[kk];
                    len = (uint32_t)(B.rpt[kk + 1] - b0);
                    av = na.Aval[j];
                }
                const uint32_t inc = wave_incl_scan(len);
                const uint32_t tot = lane63(inc);
                const uint32_t off = inc - len;  // (tot past the chunk's entries)
                // kNumUnroll products per lane at a time: their loads in flight together
                for (uint32_t p0 = 0; p0 < tot; p0 += kWave * kNumUnroll) {
                    uint32_t col[kNumUnroll];
                    double v[kNumUnroll];
#pragma unroll
                    for (int u = 0; u < kNumUnroll; ++u) {
                        const uint32_t pr = p0 + (uint32_t)(u * kWave + lane);
                        // (clamped: the loads are unconditional)
                        const uint32_t p = pr < tot ? pr : tot - 1;
                        // the product's entry: the last lane whose first product is
                        // <= p, by a fixed six-step search over the lanes' offsets
                        int lo = 0;
                        uint32_t olo = 0;
#pragma unroll
                        for (int st = kWave / 2; st > 0; st >>= 1) {
                            const uint32_t om = __shfl(off, lo + st, kWave);
                            if (om <= p) {
                                lo += st;
                                olo = om;
                            }
                        }
                        const int32_t q = __shfl(b0, lo, kWave) + (int32_t)(p - olo);
                        col[u] = (uint32_t)B.col[q];
                        v[u] = __shfl(av, lo, kWave) * na.Bval[q];
                    }
#pragma unroll
                    for (int u = 0; u < kNumUnroll; ++u)
                        if (p0 + (uint32_t)(u * kWave + lane) < tot)
                            ok = num_hash_add(keys, vals, col[u], v[u], lg) && ok;
                }
                wave_sync();
            }
            if (__ballot(!ok)) {  // (the first pass only: the fallback's tables hold every row)
                if (lane == 0) num_abort_row(row, item.rf, ctl, abort_list);
                continue;
            }
            // compaction of the occupied slots
            uint32_t kk[SPT];
            double vv[SPT];
            uint32_t mine = 0;
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const uint32_t s = (uint32_t)lane * SPT + u;
                kk[u] = s < T ? keys[s] : kEmpty;
                vv[u] = s < T ? vals[s] : 0.0;
                mine += kk[u] != kEmpty ? 1u : 0u;
            }
            const uint32_t inc = wave_incl_scan(mine);
            const uint32_t c = lane63(inc);
            uint32_t pos = inc - mine;
            wave_sync();
            int64_t dst;
            bool write, spill = false;
            if (PASS == 1) {
                if (lane == 0) na.cnt[row] = (int64_t)c;
                dst = na.slot_off[row];
                write = (int64_t)c <= na.slot_off[row + 1] - dst;
                if (!write && na.sp_cap > 0 && 2 * c <= T) {  // the whole row to the area
                    int64_t o = -1;
                    if (lane == 0 && spill_take_row(na, row, c, &o)) na.sp_state[row] = 2;
                    o = __shfl(o, 0, kWave);
                    spill = write = o >= 0;
                    dst = o;
                }
            } else {
                dst = na.C_rpt[row];
                write = dst + (int64_t)c <= na.capacity;
            }
            if (write) {  // (then c <= T / 2)
#pragma unroll
                for (int u = 0; u < SPT; ++u)
                    if (kk[u] != kEmpty) {
                        keys[pos] = kk[u];
                        vals[pos] = vv[u];
                        ++pos;
                    }
                const uint32_t c4 = (c + 3u) & ~3u;
                if ((uint32_t)lane < c4 - c) keys[c + lane] = kEmpty;
                wave_sync();
                num_write_ranked<kWave, EPT>(
                    keys, vals, c, lane, PASS == 2 ? na.C_col : spill ? na.sp_col : na.slot_col,
                    PASS == 2 ? na.C_val : spill ? na.sp_val : na.slot_val, dst);
            }
            wave_sync();  // the table is reset for the next row
        }
    }
}

// Rows whose table is larger: one workgroup of TEAM threads per row (bins 2
// and 3), the same steps with the whole workgroup.
template <int TEAM, int SLOTS, int PASS>
__global__ __launch_bounds__(TEAM) void k_num_hash(const CaseDesc* __restrict__ cs,
                                                   const BinItem* __restrict__ items,
                                                   const uint32_t* count, Ctl* ctl,
                                                   BinItem* abort_list, NumArgs na)
{
    constexpr int SPT = SLOTS / TEAM;
    static_assert(SPT >= 2 && SLOTS % TEAM == 0, "whole slots per thread");
    __shared__ __align__(16) uint32_t keys[SLOTS];
    __shared__ double vals[SLOTS];
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ double s_a[TEAM];
    __shared__ uint32_t s_red[TEAM / kWave + 1];
    __shared__ uint32_t s_fail;
    __shared__ int64_t s_spill;
    __shared__ int32_t s_row[TEAM];
    __shared__ uint32_t s_rf[TEAM];
    __shared__ uint8_t s_lg[TEAM];
    const uint32_t n = *count;
    const int t = threadIdx.x;
    const Csr A = cs[0].A, B = cs[0].B;
    const uint64_t G = gridDim.x;
    // The workgroup's items are blockIdx.x + k * gridDim.x.  TEAM of them are
    // looked at together, one per thread, and the rows this kernel owns (a
    // table of more than kNumWaveSlots slots, not yet done) are listed in LDS
    // in the same order: most items of a bin can belong to the one-wave kernel
    // (or, in the second pass, need nothing), and skipping them one at a time
    // costs a chain of dependent loads each.
    for (uint64_t r0 = blockIdx.x; r0 < n; r0 += G * TEAM) {
        const uint64_t mine_it = r0 + (uint64_t)t * G;
        uint32_t lgm = 0;
        BinItem x{};
        if (mine_it < n) {
            x = items[mine_it];
            if (!(PASS == 2 && (num_fits(na, x.row, na.cnt[x.row]) || na.sp_state[x.row]))) {
                const uint32_t Tm = num_table_size(num_bound<PASS>(na, x.row, x.rf));
                if (Tm > (uint32_t)kNumWaveSlots) lgm = (uint32_t)__builtin_ctz(Tm);
            }
        }
        uint32_t nsel;
        const uint32_t at = block_excl_scan<TEAM, uint32_t>(lgm ? 1u : 0u, s_red, &nsel);
        if (lgm) {
            s_row[at] = x.row;
            s_rf[at] = x.rf;
            s_lg[at] = (uint8_t)lgm;
        }
        __syncthreads();
        for (uint32_t q = 0; q < nsel; ++q) {
            const BinItem item{s_row[q], s_rf[q], 0, 0};
            const int64_t row = item.row;
            const int lg = s_lg[q];
            const uint32_t T = 1u << lg;
            for (uint32_t s = t; s < T; s += TEAM) {
                keys[s] = kEmpty;
                vals[s] = 0.0;
            }
            if (t == 0) s_fail = 0;
            __syncthreads();
            bool ok = true;
            const int32_t a0 = A.rpt[row], a1 = A.rpt[row + 1];
            for (int32_t a = a0; a < a1; a += TEAM) {
                const int32_t j = a + t;
                uint32_t len = 0;
                int32_t b0 = 0;
                double av = 0.0;
                if (j < a1) {
                    const int32_t k = A.col[j];
                    b0 = B.rpt[k];
                    len = (uint32_t)(B.rpt[k + 1] - b0);
                    av = na.Aval[j];
                }
                uint32_t tot;
                const uint32_t off = block_excl_scan<TEAM, uint32_t>(len, s_red, &tot);
                s_b0[t] = b0;
                s_off[t] = off;
                s_a[t] = av;
                __syncthreads();
                const int nent = (a1 - a) < TEAM ? (a1 - a) : TEAM;
                for (uint32_t p0 = 0; p0 < tot; p0 += TEAM * kNumUnroll) {
                    uint32_t col[kNumUnroll];
                    double v[kNumUnroll];
#pragma unroll
                    for (int u = 0; u < kNumUnroll; ++u) {
                        const uint32_t pr = p0 + (uint32_t)(u * TEAM + t);
                        const uint32_t p = pr < tot ? pr : tot - 1;
                        int lo = 0, hi = nent;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (s_off[mid] <= p) lo = mid;
                            else hi = mid;
                        }
                        const int32_t q = s_b0[lo] + (int32_t)(p - s_off[lo]);
                        col[u] = (uint32_t)B.col[q];
                        v[u] = s_a[lo] * na.Bval[q];
                    }
#pragma unroll
                    for (int u = 0; u < kNumUnroll; ++u)
                        if (p0 + (uint32_t)(u * TEAM + t) < tot)
                            ok = num_hash_add(keys, vals, col[u], v[u], lg) && ok;
                }
                __syncthreads();
            }
            if (!ok) s_fail = 1;
            __syncthreads();
            if (s_fail) {
                if (t == 0) num_abort_row(row, item.rf, ctl, abort_list);
                __syncthreads();
                continue;
            }
            // compaction of the occupied slots
            uint32_t kk[SPT];
            double vv[SPT];
            uint32_t mine = 0;
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const uint32_t s = (uint32_t)t * SPT + u;
                kk[u] = s < T ? keys[s] : kEmpty;
                vv[u] = s < T ? vals[s] : 0.0;
                mine += kk[u] != kEmpty ? 1u : 0u;
            }
            uint32_t c;
            uint32_t pos = block_excl_scan<TEAM, uint32_t>(mine, s_red, &c);
            int64_t dst;
            bool write, spill = false;
            if (PASS == 1) {
                if (t == 0) na.cnt[row] = (int64_t)c;
                dst = na.slot_off[row];
                write = (int64_t)c <= na.slot_off[row + 1] - dst;
                if (!write && na.sp_cap > 0 && 2 * c <= T) {  // the whole row to the area
                    if (t == 0) {
                        int64_t o = -1;
                        if (spill_take_row(na, row, c, &o)) na.sp_state[row] = 2;
                        s_spill = o;
                    }
                    __syncthreads();
                    spill = write = s_spill >= 0;
                    dst = s_spill;
                }
            } else {
                dst = na.C_rpt[row];
                write = dst + (int64_t)c <= na.capacity;
            }
            if (write) {  // (then c <= T / 2)
#pragma unroll
                for (int u = 0; u < SPT; ++u)
                    if (kk[u] != kEmpty) {
                        keys[pos] = kk[u];
                        vals[pos] = vv[u];
                        ++pos;
                    }
                const uint32_t c4 = (c + 3u) & ~3u;
                if ((uint32_t)t < c4 - c) keys[c + t] = kEmpty;
                __syncthreads();
                num_write_ranked<TEAM, SPT / 2>(
                    keys, vals, c, t, PASS == 2 ? na.C_col : spill ? na.sp_col : na.slot_col,
                    PASS == 2 ? na.C_val : spill ? na.sp_val : na.slot_val, dst);
            }
            __syncthreads();  // the table is reset for the next row
        }
    }
}

// ------------------------------------------------------ dense accumulators

// Global-memory OR of `bits` into word `word` for every lane of the wave (all
// 64 lanes call it; a lane with nothing passes kNoWord): neighbouring lanes
// naming one word (sorted B rows put consecutive products in one word) are
// combined first, one atomic per run.
__device__ __forceinline__ void wave_or_global(SSP_GLOBAL uint32_t* bm, uint32_t word,
                                               uint32_t bits)
{
    const int lane = lane_id();
    const uint64_t valid = __ballot(word != kNoWord);
    if (valid == 0) return;
    const uint32_t prev = __shfl_up(word, 1, kWave);
    const bool head = lane == 0 || prev != word;
    uint32_t acc = bits;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t ow = __shfl_down(word, off, kWave);
        const uint32_t ob = __shfl_down(acc, off, kWave);
        if (lane + off < kWave && ow == word) acc |= ob;
    }
    if (head && word != kNoWord)
        __hip_atomic_fetch_or(&bm[word], acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bin 4: rows of more than kNumBin3Max products.  A persistent grid of
// pool_slots workgroups takes the rows from a work queue; workgroup w owns
// accumulator w (N values in global memory, zero between rows).  Products
// are shared out as in the hash bins.  A product whose column is in the
// workgroup's LDS cache (an open-addressing table of kNumCacheSlots columns,
// filled up to half by the first columns met: the frequent ones) is added
// there; the others go to the accumulator with a global atomic, and the
// cache is added to the accumulator once at the end of the row (power-law
// rows meet a few columns very often: their atomics would otherwise
// serialise on one address).  The touched columns are marked in a bitmap, in
// LDS when N <= 2^19 (LDSMASK), else in the accumulator's global bitmap.  The
// row is then read back in column order over the bitmap words between its
// smallest and largest column: a scan of the words' popcounts ranks each set
// bit, the entry is written at its rank, and the value and the word are
// cleared again.
constexpr int kNumCacheLg = 11, kNumCacheSlots = 1 << kNumCacheLg;
constexpr int kNumCacheProbes = 8;
constexpr int64_t kNumLdsMaskWords = 16384;

template <int PASS, bool LDSMASK>
__global__ __launch_bounds__(kNumDenseTeam) void k_num_dense(const CaseDesc* __restrict__ cs,
                                                             const BigItem* __restrict__ items,
                                                             Ctl* ctl, uint32_t cap4, NumArgs na)
{
    constexpr int TEAM = kNumDenseTeam;
    extern __shared__ __align__(16) uint32_t s_mask[];  // LDSMASK: mask_words words
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ double s_a[TEAM];
    __shared__ uint64_t s_red[TEAM / kWave + 1];
    __shared__ uint32_t s_mm[2], s_k, s_fill;
    __shared__ uint32_t c_keys[kNumCacheSlots];
    __shared__ double c_vals[kNumCacheSlots];
    const int t = threadIdx.x;
    const uint32_t nheavy = ctl->bin_cnt[4], total = nheavy + ctl->bin_cnt[6];
    uint32_t* next = &ctl->num_next[PASS - 1];
    const Csr A = cs[0].A, B = cs[0].B;
    SSP_GLOBAL double* acc = na.pool + (int64_t)blockIdx.x * na.N;
    SSP_GLOBAL uint32_t* gmask = na.pool_mask + (int64_t)blockIdx.x * na.mask_words;
    if (LDSMASK)
        for (int64_t w = t; w < na.mask_words; w += TEAM) s_mask[w] = 0u;
    for (int s = t; s < kNumCacheSlots; s += TEAM) {
        c_keys[s] = kEmpty;
        c_vals[s] = 0.0;
    }
    for (;;) {
        if (t == 0) {
            s_k = atomicAdd(next, 1u);
            s_mm[0] = 0xFFFFFFFFu;
            s_mm[1] = 0u;
            s_fill = 0;
        }
        __syncthreads();
        const uint32_t k = s_k;
        if (k >= total) break;
        const BigItem item = items[big_index(k, nheavy, cap4)];
        const int64_t row = item.row;
        if (PASS == 2 && num_fits(na, row, na.cnt[row])) {
            __syncthreads();  // (s_k is rewritten)
            continue;
        }
        uint32_t wmin = 0xFFFFFFFFu, wmax = 0u;
        const int32_t a0 = item.e_lo, a1 = item.e_hi;
        for (int32_t a = a0; a < a1; a += TEAM) {
            const int32_t j = a + t;
            uint32_t len = 0;
            int32_t b0 = 0;
            double av = 0.0;
            if (j < a1) {
                const int32_t kk = A.col[j];
                b0 = B.rpt[kk];
                len = (uint32_t)(B.rpt[kk + 1] - b0);
                av = na.Aval[j];
            }
            uint32_t tot;
            const uint32_t off = block_excl_scan<TEAM, uint32_t>(len, (uint32_t*)s_red, &tot);
            s_b0[t] = b0;
            s_off[t] = off;
            s_a[t] = av;
            __syncthreads();
            const int nent = (a1 - a) < TEAM ? (a1 - a) : TEAM;
            // the LDS cache, else the accumulator
            auto add = [&](uint32_t col, double v) {
                uint32_t h = (col * 0x9E3779B1u) >> (32 - kNumCacheLg);
                for (int n = 0; n < kNumCacheProbes; ++n) {
                    uint32_t cur =
                        __hip_atomic_load(&c_keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (cur == kEmpty &&
                        __hip_atomic_load(&s_fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <
                            (uint32_t)(kNumCacheSlots / 2)) {
                        cur = atomicCAS(&c_keys[h], kEmpty, col);
                        if (cur == kEmpty) {
                            atomicAdd(&s_fill, 1u);
                            cur = col;
                        }
                    }
                    if (cur == col) {
                        __hip_atomic_fetch_add(&c_vals[h], v, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        return;
                    }
                    if (cur == kEmpty) break;  // (the cache is full enough)
                    h = (h + 1u) & (uint32_t)(kNumCacheSlots - 1);
                }
                __hip_atomic_fetch_add(&acc[col], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            // same trip count in every lane; kNumUnroll products per lane whose
            // loads are in flight together
            for (uint32_t p0 = 0; p0 < tot; p0 += TEAM * kNumUnroll) {
                uint32_t colv[kNumUnroll];
                double vv[kNumUnroll];
#pragma unroll
                for (int u = 0; u < kNumUnroll; ++u) {
                    const uint32_t pr = p0 + (uint32_t)(u * TEAM + t);
                    const uint32_t p = pr < tot ? pr : tot - 1;
                    int lo = 0, hi = nent;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_off[mid] <= p) lo = mid;
                        else hi = mid;
                    }
                    const int32_t q = s_b0[lo] + (int32_t)(p - s_off[lo]);
                    colv[u] = (uint32_t)B.col[q];
                    vv[u] = s_a[lo] * na.Bval[q];
                }
#pragma unroll
                for (int u = 0; u < kNumUnroll; ++u) {
                    uint32_t word = kNoWord, bit = 0;
                    if (p0 + (uint32_t)(u * TEAM + t) < tot) {
                        const uint32_t col = colv[u];
                        add(col, vv[u]);
                        word = col >> 5;
                        bit = 1u << (col & 31u);
                        wmin = word < wmin ? word : wmin;
                        wmax = word > wmax ? word : wmax;
                    }
                    if (LDSMASK)
                        lds_bitmap_or(s_mask, word, bit);
                    else
                        wave_or_global(gmask, word, bit);
                }
            }
            __syncthreads();
        }
        atomicMin(&s_mm[0], wmin);
        atomicMax(&s_mm[1], wmax);
        // the cache into the accumulator (and cleared)
        for (int s = t; s < kNumCacheSlots; s += TEAM) {
            const uint32_t key = c_keys[s];
            if (key != kEmpty) {
                __hip_atomic_fetch_add(&acc[key], c_vals[s], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                c_keys[s] = kEmpty;
                c_vals[s] = 0.0;
            }
        }
        // (workgroup scope: the accumulator is this workgroup's alone, and an
        //  agent-scope fence would write back and invalidate the whole L2)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const uint32_t w0 = s_mm[0], w1 = s_mm[1];
        auto mask_word = [&](uint32_t w) -> uint32_t {
            return LDSMASK ? s_mask[w]
                           : __hip_atomic_load(&gmask[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        // count
        uint64_t mine = 0;
        if (w0 <= w1)
            for (uint32_t w = w0 + t; w <= w1; w += TEAM) mine += (uint64_t)__popc(mask_word(w));
        const uint64_t c = block_sum<TEAM, uint64_t>(mine, s_red);
        int64_t dst;
        bool write;
        if (PASS == 1) {
            if (t == 0) na.cnt[row] = (int64_t)c;
            dst = na.slot_off[row];
            write = (int64_t)c <= na.slot_off[row + 1] - dst;
        } else {
            dst = na.C_rpt[row];
            write = dst + (int64_t)c <= na.capacity;
        }
        SSP_GLOBAL int32_t* ocol = PASS == 1 ? na.slot_col : na.C_col;
        SSP_GLOBAL double* oval = PASS == 1 ? na.slot_val : na.C_val;
        // read back in column order (or only clear, when the row does not fit)
        int64_t base = dst;
        if (w0 <= w1)
            for (uint32_t wb = w0; wb <= w1; wb += TEAM) {
                const uint32_t w = wb + t;
                uint32_t bits = w <= w1 ? mask_word(w) : 0u;
                uint64_t ctot;
                const uint64_t ex =
                    block_excl_scan<TEAM, uint64_t>((uint64_t)__popc(bits), s_red, &ctot);
                int64_t o = base + (int64_t)ex;
                while (bits) {
                    const uint32_t b = (uint32_t)__builtin_ctz(bits);
                    bits &= bits - 1u;
                    const uint32_t col = w * 32u + b;
                    if (write) {
                        ocol[o] = (int32_t)col;
                        oval[o] = __hip_atomic_load(&acc[col], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
                        ++o;
                    }
                    acc[col] = 0.0;
                }
                if (w <= w1) {
                    if (LDSMASK) s_mask[w] = 0u;
                    else gmask[w] = 0u;
                }
                base += (int64_t)ctot;
            }
        // the clears are seen by the next row's atomics
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// ------------------------------------------------------------- copy pass

// Rows that fitted their slot are copied to C at their final offsets, and so
// are the slot parts of longer rows whose other entries the overflow area
// holds.  Each workgroup copies a chunk of kNumCopyChunk entries of C (so a
// long row is shared by many workgroups): it finds the rows that overlap its
// chunk by binary search over C's row offsets and takes them kNumCopyRows at
// a time, their entries shared out over the threads (each finds its row by
// binary search in LDS).
constexpr int64_t kNumCopyChunk = 8192;

__global__ __launch_bounds__(kNumCopyRows) void k_num_copy(NumArgs na)
{
    __shared__ int64_t s_start[kNumCopyRows + 1];
    __shared__ int64_t s_src[kNumCopyRows], s_dst[kNumCopyRows];
    __shared__ int64_t s_red[kNumCopyRows / kWave + 1];
    __shared__ int64_t s_rows[2];
    const int t = threadIdx.x;
    const int64_t nnz = na.C_rpt[na.M];
    // last row whose offset is <= e (rows are [C_rpt[i], C_rpt[i+1]))
    auto row_of = [&](int64_t e) {
        int64_t lo = 0, hi = na.M;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (na.C_rpt[mid] <= e) lo = mid;
            else hi = mid;
        }
        return lo;
    };
    for (int64_t e0 = (int64_t)blockIdx.x * kNumCopyChunk; e0 < nnz;
         e0 += (int64_t)gridDim.x * kNumCopyChunk) {
        const int64_t e1 = (e0 + kNumCopyChunk) < nnz ? (e0 + kNumCopyChunk) : nnz;
        if (t == 0) {
            s_rows[0] = row_of(e0);
            s_rows[1] = row_of(e1 - 1);
        }
        __syncthreads();
        const int64_t r_first = s_rows[0], r_last = s_rows[1];
        for (int64_t r0 = r_first; r0 <= r_last; r0 += kNumCopyRows) {
            const int64_t i = r0 + t;
            int64_t n = 0, src = 0, dst = 0;
            if (i <= r_last) {
                const int64_t c = na.cnt[i], beg = na.C_rpt[i];
                const int64_t s = na.slot_off[i + 1] - na.slot_off[i];
                // entries of the row in its slot
                const int64_t m = c <= s ? c : (na.sp_state[i] == 1 ? s : 0);
                const int64_t lo = beg > e0 ? beg : e0;
                const int64_t hi = (beg + m) < e1 ? (beg + m) : e1;
                if (beg + c <= na.capacity && hi > lo) {
                    n = hi - lo;
                    src = na.slot_off[i] + (lo - beg);
                    dst = lo;
                }
            }
            int64_t tot;
            const int64_t ex = block_excl_scan<kNumCopyRows, int64_t>(n, s_red, &tot);
            s_start[t] = ex;
            s_src[t] = src;
            s_dst[t] = dst;
            if (t == 0) s_start[kNumCopyRows] = tot;
            __syncthreads();
            for (int64_t q = t; q < tot; q += kNumCopyRows) {
                int lo = 0, hi = kNumCopyRows;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_start[mid] <= q) lo = mid;
                    else hi = mid;
                }
                const int64_t d = q - s_start[lo];
                na.C_col[s_dst[lo] + d] = na.slot_col[s_src[lo] + d];
                na.C_val[s_dst[lo] + d] = na.slot_val[s_src[lo] + d];
            }
            __syncthreads();
        }
    }
}

// The runs the overflow area holds, to their place in C: one run per
// workgroup at a time (a run has at most kSpillChunk entries, or a window's).
// Empty records (row -1) and runs of rows that the area could not hold to the
// end are skipped (those rows are recomputed); so is a run outside its row or
// the area.
__global__ __launch_bounds__(256) void k_num_spill_copy(NumArgs na, int64_t nrec)
{
    for (int64_t r = blockIdx.x; r < nrec; r += gridDim.x) {
        const SpillRec x = na.sp_rec[r];
        if (x.row < 0 || (int64_t)x.row >= na.M || x.n <= 0 || !na.sp_state[x.row]) continue;
        const int64_t beg = na.C_rpt[x.row], c = na.cnt[x.row];
        if (beg + c > na.capacity || x.pos < 0 || (int64_t)x.pos + x.n > c || x.off < 0 ||
            x.off + x.n > na.sp_cap)
            continue;
        const int64_t d = beg + x.pos;
        for (int32_t q = threadIdx.x; q < x.n; q += 256) {
            na.C_col[d + q] = na.sp_col[x.off + q];
            na.C_val[d + q] = na.sp_val[x.off + q];
        }
    }
}

// ------------------------------------------- dense rows by column windows

// Rows of more than kNumBin3Max products when every row of B lists its
// columns in non-decreasing order (checked on the device per call): each row
// is accumulated one window of kNumWinCols columns at a time, entirely in LDS
// (a dense float64 window and its bitmap), with no global atomics.  A cursor
// per A entry of the row (its next position in the named B row, and that
// position's column) lives in LDS between windows, or in global scratch for
// rows of more entries than the workgroup has threads, so every product is
// read once: in a window an entry whose cursor column lies beyond the window
// is skipped, the others find their end in the window (a search by up to 64
// lanes per entry).  Window by window the set bits are ranked (popcount scan)
// and the row's entries written in column order, each wave's stores
// coalesced; the first pass writes
// what fits the row's slot to the slot and, with an overflow area, the rest
// to the area: thread 0 keeps the workgroup's current chunk of the area and
// the row's current run (positions and area offsets both consecutive), and
// records a run when the chunk changes or the row ends.  A row that the area
// cannot hold is redone by the fallback pass.  The exact count is recorded.
constexpr int kNumWinCols = 16384;
// Products per thread whose loads are in flight together in a window: two
// (and slots past the window's products skipped), since most windows hold
// far fewer products than the workgroup has threads (R-MAT 2^18: 46.5 ms
// with four, 44.1 with one, 42.9 with two; eight and sixteen were slower).
constexpr int kNumWinUnroll = 2;

// agg[5] != 0 when some row of B has a column smaller than its predecessor.
// Only the long rows' kernels depend on it: with no such row (bins 4 and 6
// empty, counted by the row-FLOP pass before this launch) nothing is read.
__global__ __launch_bounds__(256) void k_num_check_sorted(Csr B, const Ctl* ctl, NumArgs na)
{
    if (ctl->bin_cnt[4] + ctl->bin_cnt[6] == 0) return;
    // Flat over the entries (a thread per pair of neighbours, so a row of any
    // length is shared out): a descent is an error unless the second entry
    // starts a row, which a binary search over the row pointers tells (the
    // last row starting at or before the first entry ends right after it).
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q + 1 < B.nnz; q += stride) {
        if (B.col[q] <= B.col[q + 1]) continue;
        int64_t lo = 0, hi = B.nrows;  // (B.rpt[0] = 0 <= q < B.rpt[B.nrows] = B.nnz)
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)B.rpt[mid] <= q) lo = mid;
            else hi = mid;
        }
        bad = bad || (int64_t)B.rpt[lo + 1] != q + 1;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr((unsigned long long*)&na.agg[5], 1ull);
}

// agg[4] = the largest number of A entries of a bin-4 row.
__global__ __launch_bounds__(256) void k_num_maxlen(const BigItem* __restrict__ items, Ctl* ctl,
                                                    uint32_t cap4, NumArgs na)
{
    const uint32_t nheavy = ctl->bin_cnt[4], total = nheavy + ctl->bin_cnt[6];
    uint64_t m = 0;
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < total; k += gridDim.x * 256) {
        const BigItem it = items[big_index(k, nheavy, cap4)];
        const uint64_t len = (uint64_t)(it.e_hi - it.e_lo);
        m = len > m ? len : m;
    }
    // (a wave maximum, then one atomic per wave)
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_down(m, off, kWave);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && m) atomicMax((unsigned long long*)&na.agg[4], (unsigned long long)m);
}

template <int PASS>
__global__ __launch_bounds__(kNumDenseTeam) void k_num_dense_win(const CaseDesc* __restrict__ cs,
                                                                 const BigItem* __restrict__ items,
                                                                 Ctl* ctl, uint32_t cap4, NumArgs na,
                                                                 int2* __restrict__ cursors,
                                                                 int64_t cur_stride)
{
    constexpr int TEAM = kNumDenseTeam, WW = kNumWinCols / 32;
    extern __shared__ __align__(16) double s_acc[];  // kNumWinCols values
    __shared__ uint32_t s_flag[WW];
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ double s_a[TEAM];
    __shared__ int32_t s_cur[TEAM];   // per A entry: the cursor in its B row,
    __shared__ int32_t s_ccol[TEAM];  // the column there (INT32_MAX past the end),
    __shared__ int32_t s_pe[TEAM];    // the B row's end
    __shared__ uint64_t s_red[TEAM / kWave + 1];
    __shared__ uint32_t s_k;
    __shared__ int64_t s_spill;
    const int t = threadIdx.x;
    const uint32_t nheavy = ctl->bin_cnt[4], total = nheavy + ctl->bin_cnt[6];
    uint32_t* next = &ctl->num_next[PASS - 1];
    const Csr A = cs[0].A, B = cs[0].B;
    const int64_t N = B.ncols;
    int2* cur = cursors + (int64_t)blockIdx.x * cur_stride;  // (position, its column) per A entry
    // (thread 0) the workgroup's chunk of the overflow area [ck, ck_end); the
    // row's run: area offset, first position, entries; whether the area
    // holds the row so far
    int64_t ck = 0, ck_end = 0, run_off = 0, run_pos = 0, run_n = 0;
    bool held = true;
    for (int i = t; i < kNumWinCols; i += TEAM) s_acc[i] = 0.0;
    for (int i = t; i < WW; i += TEAM) s_flag[i] = 0u;
    for (;;) {
        if (t == 0) s_k = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t k = s_k;
        if (k >= total) break;
        const BigItem item = items[big_index(k, nheavy, cap4)];
        const int64_t row = item.row;
        if (PASS == 2 && (num_fits(na, row, na.cnt[row]) || na.sp_state[row])) {
            __syncthreads();  // (s_k is rewritten)
            continue;
        }
        const int32_t a0 = item.e_lo, a1 = item.e_hi;
        // Each A entry's state: its B row's cursor (the next position, and
        // that position's column) and end, and its A value.  A row of at most
        // TEAM entries keeps it in LDS for all the windows; a longer row keeps
        // the cursors in global scratch and loads TEAM entries' state per
        // window.
        const bool in_lds = a1 - a0 <= TEAM;  // (uniform)
        if (in_lds) {
            const int32_t e = a0 + t;
            if (e < a1) {
                const int32_t kk = A.col[e];
                const int32_t p = B.rpt[kk], pe = B.rpt[kk + 1];
                s_cur[t] = p;
                s_pe[t] = pe;
                s_ccol[t] = p < pe ? B.col[p] : INT32_MAX;
                s_a[t] = na.Aval[e];
            }
        } else {
            for (int32_t e = a0 + t; e < a1; e += TEAM) {
                const int32_t kk = A.col[e];
                const int32_t p = B.rpt[kk], pe = B.rpt[kk + 1];
                cur[e - a0] = make_int2(p, p < pe ? B.col[p] : INT32_MAX);
            }
            __threadfence_block();
        }
        __syncthreads();
        int64_t dst, cap;
        if (PASS == 1) {
            dst = na.slot_off[row];
            cap = na.slot_off[row + 1] - dst;
        } else {
            dst = na.C_rpt[row];
            cap = na.cnt[row];
        }
        SSP_GLOBAL int32_t* ocol = PASS == 1 ? na.slot_col : na.C_col;
        SSP_GLOBAL double* oval = PASS == 1 ? na.slot_val : na.C_val;
        int64_t c_total = 0;
        for (int64_t lo = 0; lo < N; lo += kNumWinCols) {
            const int64_t hi = (lo + kNumWinCols) < N ? (lo + kNumWinCols) : N;
            uint32_t any = 0;
            for (int32_t a = a0; a < a1; a += TEAM) {
                const int nent = (a1 - a) < TEAM ? (a1 - a) : TEAM;
                if (!in_lds) {
                    if (t < nent) {
                        const int32_t e = a + t;
                        const int2 c = cur[e - a0];
                        s_cur[t] = c.x;
                        s_ccol[t] = c.y;
                        if ((int64_t)c.y < hi) {  // (INT32_MAX: the B row is used up)
                            s_pe[t] = B.rpt[A.col[e] + 1];
                            s_a[t] = na.Aval[e];
                        }
                    }
                    __syncthreads();
                }
                // Each entry's products in the window are the positions from
                // its cursor to the first one whose column is >= hi (columns
                // non-decreasing).  G lanes search for that position together,
                // the most that still give every entry of the chunk a group:
                // each round probes G evenly spaced positions of the open
                // interval and keeps the gap where the columns cross hi, so a
                // span of m positions takes log_G(m) rounds of one load each.
                int G = kWave;
                while (G > 1 && TEAM / G < nent) G >>= 1;
                if (G > 1) {
                    const int lane = t & (kWave - 1);
                    const int gbase = lane & ~(G - 1);
                    const int j = lane - gbase;
                    const int ei = t / G;
                    const uint64_t gmask = G == kWave ? ~0ull : (((1ull << G) - 1ull) << gbase);
                    bool act = false;
                    int32_t L = 0, R = 0, Rc = INT32_MAX;
                    if (ei < nent) {
                        L = s_cur[ei];
                        act = (int64_t)s_ccol[ei] < hi;
                        R = act ? s_pe[ei] : L;
                    }
                    const int32_t p = L;
                    // (L: a position whose column is < hi; R: the end of the B
                    // row or a position whose column, Rc, is >= hi)
                    for (;;) {
                        const bool go = act && R - L > 1;
                        if (!__ballot(go)) break;  // (uniform over the wave)
                        const int32_t step = go ? (R - L - 1 + G - 1) / G : 1;
                        const int32_t pos = L + 1 + j * step;
                        const bool probe = go && pos < R;
                        int32_t cv = INT32_MAX;
                        if (probe) cv = B.col[pos];
                        const uint64_t okm = __ballot(probe && (int64_t)cv < hi) & gmask;
                        const int n = __popcll(okm);  // (the probes below hi: a prefix)
                        const int32_t fc = __shfl(cv, gbase + (n < G ? n : G - 1), kWave);
                        if (go) {
                            const int32_t fp = L + 1 + n * step;  // the first probe >= hi
                            if (n > 0) L += 1 + (n - 1) * step;
                            if (fp < R) {
                                R = fp;
                                Rc = fc;
                            }
                        }
                    }
                    if (ei < nent && j == 0) {
                        s_b0[ei] = p;
                        s_off[ei] = act ? (uint32_t)(R - p) : 0u;
                        if (act) {
                            s_cur[ei] = R;
                            s_ccol[ei] = Rc;
                        }
                    }
                } else if (t < nent) {
                    // one entry per thread: exponential then binary search
                    const int32_t p = s_cur[t];
                    uint32_t len = 0;
                    if ((int64_t)s_ccol[t] < hi) {
                        const int32_t pe = s_pe[t];
                        int32_t good = p, step = 1;
                        while (good + step < pe && (int64_t)B.col[good + step] < hi) {
                            good += step;
                            step <<= 1;
                        }
                        int32_t bad = (good + step) < pe ? (good + step) : pe;
                        while (bad - good > 1) {
                            const int32_t mid = (good + bad) >> 1;
                            if ((int64_t)B.col[mid] < hi) good = mid;
                            else bad = mid;
                        }
                        len = (uint32_t)(bad - p);
                        s_cur[t] = bad;
                        s_ccol[t] = bad < pe ? B.col[bad] : INT32_MAX;
                    }
                    s_b0[t] = p;
                    s_off[t] = len;
                }
                __syncthreads();
                uint32_t tot;
                const uint32_t len = t < nent ? s_off[t] : 0u;
                const uint32_t off = block_excl_scan<TEAM, uint32_t>(len, (uint32_t*)s_red, &tot);
                if (t < nent) {
                    s_off[t] = off;
                    if (!in_lds) cur[a + t - a0] = make_int2(s_cur[t], s_ccol[t]);
                }
                __syncthreads();
                any |= tot;
                for (uint32_t p0 = 0; p0 < tot; p0 += TEAM * kNumWinUnroll) {
                    uint32_t colv[kNumWinUnroll];
                    double vv[kNumWinUnroll];
#pragma unroll
                    for (int u = 0; u < kNumWinUnroll; ++u) {
                        colv[u] = 0;
                        vv[u] = 0.0;
                        if (p0 + (uint32_t)(u * TEAM) >= tot) continue;  // (uniform: no product)
                        const uint32_t pr = p0 + (uint32_t)(u * TEAM + t);
                        const uint32_t pp = pr < tot ? pr : tot - 1;
                        int lo2 = 0, hi2 = nent;
                        while (hi2 - lo2 > 1) {
                            const int mid = (lo2 + hi2) >> 1;
                            if (s_off[mid] <= pp) lo2 = mid;
                            else hi2 = mid;
                        }
                        const int32_t q = s_b0[lo2] + (int32_t)(pp - s_off[lo2]);
                        colv[u] = (uint32_t)B.col[q];
                        vv[u] = s_a[lo2] * na.Bval[q];
                    }
#pragma unroll
                    for (int u = 0; u < kNumWinUnroll; ++u) {
                        if (p0 + (uint32_t)(u * TEAM + t) >= tot) continue;
                        const uint32_t x = colv[u] - (uint32_t)lo;  // (in [0, kNumWinCols))
                        __hip_atomic_fetch_add(&s_acc[x], vv[u], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        atomicOr(&s_flag[x >> 5], 1u << (x & 31u));
                    }
                }
                __syncthreads();
            }
            if (!any) continue;  // (uniform: no product of the row in this window)
            // The window's entries in column order, then cleared.  Wave v
            // takes the bitmap words [32 v, 32 v + 32) and its lanes write
            // consecutive entries, so each store of a wave is coalesced (a
            // lane per word would scatter them 32 entries apart).
            static_assert(TEAM / kWave * 32 == WW, "32 bitmap words per wave");
            const int wv = t / kWave, ln = t % kWave;
            const int widx = wv * 32 + ln;
            const uint32_t bits = ln < 32 ? s_flag[widx] : 0u;
            uint64_t wtot;
            const uint64_t ex = block_excl_scan<TEAM, uint64_t>((uint64_t)__popc(bits), s_red, &wtot);
            // entries from position `from` on go to the overflow area at `sp`
            // (-1: nowhere)
            const int64_t wend = c_total + (int64_t)wtot;
            const int64_t from = cap > c_total ? cap : c_total;
            int64_t sp = -1;
            if (PASS == 1 && na.sp_cap > 0 && wend > cap) {  // (uniform)
                if (t == 0) {
                    const int64_t n = wend - from;  // (<= kNumWinCols)
                    if (held && ck + n > ck_end) {  // a new chunk: the run ends
                        if (run_n > 0) held = spill_record(na, row, run_pos, run_off, run_n);
                        run_n = 0;
                        // a chunk, else (the area nearly used up) just this window's entries
                        const int64_t want = n > na.sp_chunk ? n : na.sp_chunk;
                        int64_t o, r;
                        if (held && spill_take(na, want, false, &o, &r)) {
                            ck = o;
                            ck_end = o + want;
                        } else if (held && want > n && spill_take(na, n, false, &o, &r)) {
                            ck = o;
                            ck_end = o + n;
                        } else {
                            held = false;
                            ck = ck_end = 0;
                        }
                    }
                    if (held) {
                        if (run_n == 0) {
                            run_off = ck;
                            run_pos = from;
                        }
                        s_spill = ck;
                        ck += n;
                        run_n += n;
                    } else {
                        s_spill = -1;
                    }
                }
                __syncthreads();
                sp = s_spill;
            }
            // (the wave's first entry, its count, and each word's first entry
            // within the wave, in s_off: free until the next window)
            const uint64_t ex0 = __shfl(ex, 0, kWave);
            const uint32_t wn = (uint32_t)(__shfl(ex, 32, kWave) - ex0);
            if (ln < 32) s_off[widx] = (uint32_t)(ex - ex0);
            wave_sync();
            const uint32_t* wpre = &s_off[wv * 32];
            for (uint32_t k = (uint32_t)ln; k < wn; k += kWave) {
                // the word holding the wave's k-th entry (the last word whose
                // first entry is <= k: words without entries share the next
                // one's), then the rank of the entry's bit within it
                int w0 = 0, w1 = 32;
                while (w1 - w0 > 1) {
                    const int mid = (w0 + w1) >> 1;
                    if (wpre[mid] <= k) w0 = mid;
                    else w1 = mid;
                }
                uint32_t b = s_flag[wv * 32 + w0], r = k - wpre[w0], pos = 0, c;
                c = (uint32_t)__popc(b & 0xFFFFu);
                if (r >= c) { r -= c; b >>= 16; pos += 16; }
                c = (uint32_t)__popc(b & 0xFFu);
                if (r >= c) { r -= c; b >>= 8; pos += 8; }
                c = (uint32_t)__popc(b & 0xFu);
                if (r >= c) { r -= c; b >>= 4; pos += 4; }
                c = (uint32_t)__popc(b & 0x3u);
                if (r >= c) { r -= c; b >>= 2; pos += 2; }
                if (r >= (b & 1u)) pos += 1;
                const uint32_t x = (uint32_t)(wv * 32 + w0) * 32u + pos;
                const int64_t o = c_total + (int64_t)ex0 + (int64_t)k;
                const double v = s_acc[x];
                if (o < cap) {
                    ocol[dst + o] = (int32_t)(lo + x);
                    oval[dst + o] = v;
                } else if (sp >= 0) {
                    na.sp_col[sp + (o - from)] = (int32_t)(lo + x);
                    na.sp_val[sp + (o - from)] = v;
                }
                s_acc[x] = 0.0;
            }
            wave_sync();
            if (ln < 32) s_flag[widx] = 0u;
            c_total += (int64_t)wtot;
            __syncthreads();
        }
        if (PASS == 1 && t == 0) {
            na.cnt[row] = c_total;
            if (na.sp_cap > 0 && c_total > cap) {  // the row's last run
                if (held && run_n > 0) held = spill_record(na, row, run_pos, run_off, run_n);
                if (held) na.sp_state[row] = 1;
                run_n = 0;
                held = true;
            }
        }
        __syncthreads();
    }
}

// Sets n doubles (and the words after them) to zero: the dense accumulators
// when they are first allocated.
__global__ void k_num_zero(uint64_t* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

} // namespace ssp
