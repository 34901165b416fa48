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
    SSP_GLOBAL int64_t* part;       // per-block partials of the scans: 3 x blocks
    SSP_GLOBAL uint64_t* agg;       // [0] NNZ(C) [1] overflow rows [2] their nonzeros [3] slot entries
};

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
__device__ __forceinline__ int64_t num_scan_value(const NumArgs& na, int64_t i, int64_t* orow,
                                                  int64_t* onnz)
{
    if (KIND == 0) return num_slot_size(na.cap[i], na.margin, na.N);
    const int64_t c = na.cnt[i];
    if (!num_fits(na, i, c)) {
        *orow += 1;
        *onnz += c;
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
        int64_t sum = 0, orow = 0, onnz = 0;
        const int64_t r0 = b * kNumScanBlock + (int64_t)threadIdx.x * kNumScanRows;
#pragma unroll
        for (int u = 0; u < kNumScanRows; ++u)
            if (r0 + u < na.M) sum += num_scan_value<KIND>(na, r0 + u, &orow, &onnz);
        sum = block_sum<kNumScanThreads, int64_t>(sum, s_red);
        if (KIND == 1) {
            orow = block_sum<kNumScanThreads, int64_t>(orow, s_red);
            onnz = block_sum<kNumScanThreads, int64_t>(onnz, s_red);
        }
        if (threadIdx.x == 0) {
            na.part[b] = sum;
            if (KIND == 1) {
                na.part[nblk + b] = orow;
                na.part[2 * nblk + b] = onnz;
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
    int64_t run = 0, orow = 0, onnz = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += kNumScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nblk ? na.part[b] : 0;
        if (KIND == 1 && b < nblk) {
            orow += na.part[nblk + b];
            onnz += na.part[2 * nblk + b];
        }
        int64_t tot;
        const int64_t ex = block_excl_scan<kNumScanThreads, int64_t>(v, s_red, &tot);
        if (b < nblk) na.part[b] = run + ex;
        run += tot;
    }
    if (KIND == 1) {
        orow = block_sum<kNumScanThreads, int64_t>(orow, s_red);
        onnz = block_sum<kNumScanThreads, int64_t>(onnz, s_red);
    }
    if (threadIdx.x == 0) {
        out[na.M] = run;
        if (KIND == 0) {
            na.agg[3] = (uint64_t)run;
        } else {
            na.agg[0] = (uint64_t)run;
            na.agg[1] = (uint64_t)orow;
            na.agg[2] = (uint64_t)onnz;
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

// Adds v to column c's slot of an LDS table of 2^lg slots (open addressing,
// linear probing; columns are < 2^31, so the all-ones key marks a free slot).
__device__ __forceinline__ void num_hash_add(uint32_t* keys, double* vals, uint32_t c, double v,
                                             int lg)
{
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t h = (c * 0x9E3779B1u) >> (32 - lg);
    for (;;) {
        const uint32_t cur =
            __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == c) break;
        if (cur == kEmpty) {
            const uint32_t prev = atomicCAS(&keys[h], kEmpty, c);
            if (prev == kEmpty || prev == c) break;
        }
        h = (h + 1u) & mask;
    }
    __hip_atomic_fetch_add(&vals[h], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bins 1..3: one workgroup of TEAM threads per row.  The row's products are
// enumerated TEAM entries of A at a time (a scan of the B row lengths gives
// each product's A entry by binary search in LDS, so every thread handles an
// equal share whatever the B row lengths) and added into the hash table.
// The occupied slots are then compacted (a scan over the table, each thread
// holding SLOTS/TEAM slots in registers) and each entry's place in the
// sorted row is its rank among the keys.
// PASS 1: count the row, write it to its slot when it fits.
// PASS 2: rows that did not fit, written to C at their final offset.
template <int TEAM, int SLOTS, int PASS>
__global__ __launch_bounds__(TEAM) void k_num_hash(const CaseDesc* __restrict__ cs,
                                                   const BinItem* __restrict__ items,
                                                   const uint32_t* count, NumArgs na)
{
    constexpr int SPT = SLOTS / TEAM;
    static_assert(SPT >= 1 && SLOTS % TEAM == 0, "whole slots per thread");
    __shared__ __align__(16) uint32_t keys[SLOTS];
    __shared__ double vals[SLOTS];
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ double s_a[TEAM];
    __shared__ uint32_t s_red[TEAM / kWave + 1];
    const uint32_t n = *count;
    const int t = threadIdx.x;
    const Csr A = cs[0].A, B = cs[0].B;
    const int64_t N = B.ncols;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const BinItem item = items[it];
        const int64_t row = item.row;
        if (PASS == 2 && num_fits(na, row, na.cnt[row])) continue;  // (the same for the whole team)
        const uint32_t bound = (uint32_t)((int64_t)item.rf < N ? (int64_t)item.rf : N);
        uint32_t tsize = 32;
        while (tsize < 2u * bound) tsize <<= 1;
        const int lg = __builtin_ctz(tsize);
        for (uint32_t w = t; w < tsize; w += TEAM) {
            keys[w] = kEmpty;
            vals[w] = 0.0;
        }
        __syncthreads();
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
            for (uint32_t p = t; p < tot; p += TEAM) {
                int lo = 0, hi = nent;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const int32_t q = s_b0[lo] + (int32_t)(p - s_off[lo]);
                num_hash_add(keys, vals, (uint32_t)B.col[q], s_a[lo] * na.Bval[q], lg);
            }
            __syncthreads();
        }
        // compaction of the occupied slots
        uint32_t kk[SPT];
        double vv[SPT];
        uint32_t mine = 0;
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const uint32_t s = (uint32_t)t * SPT + u;
            kk[u] = s < tsize ? keys[s] : kEmpty;
            vv[u] = s < tsize ? vals[s] : 0.0;
            mine += kk[u] != kEmpty ? 1u : 0u;
        }
        uint32_t c;
        uint32_t pos = block_excl_scan<TEAM, uint32_t>(mine, s_red, &c);
        if (TEAM == kWave) __syncthreads();  // (one wave: no barrier inside the scan)
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
        if (write) {
#pragma unroll
            for (int u = 0; u < SPT; ++u)
                if (kk[u] != kEmpty) {
                    keys[pos] = kk[u];
                    vals[pos] = vv[u];
                    ++pos;
                }
            const uint32_t c4 = (c + 3u) & ~3u;  // (c4 <= tsize / 2: c <= bound)
            if ((uint32_t)t < c4 - c) keys[c + t] = kEmpty;
            __syncthreads();
            SSP_GLOBAL int32_t* ocol = PASS == 1 ? na.slot_col : na.C_col;
            SSP_GLOBAL double* oval = PASS == 1 ? na.slot_val : na.C_val;
            // rank of each entry among the row's keys (all keys distinct)
            constexpr int EPT = SPT;  // entries per thread (c <= tsize / 2 <= SLOTS / 2)
            uint32_t key[EPT], rank[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const uint32_t e = (uint32_t)t + (uint32_t)u * TEAM;
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
                const uint32_t e = (uint32_t)t + (uint32_t)u * TEAM;
                if (e < c) {
                    ocol[dst + rank[u]] = (int32_t)key[u];
                    oval[dst + rank[u]] = vals[e];
                }
            }
        }
        __syncthreads();  // the table is reset for the next row
    }
}

// ------------------------------------------------------ dense accumulators

// Bin 4: rows of more than kNumBin3Max products.  A persistent grid of
// pool_slots workgroups; workgroup w owns accumulator w (N values and an
// N-bit column bitmap in global memory, all zero between rows) and takes the
// bin's items w, w + G, ...  Products are shared out as in the hash bins and
// added with global atomics; the touched columns are marked in the bitmap.
// The row is then read back in column order over the bitmap words between
// its smallest and largest column: a scan of the words' popcounts ranks each
// set bit, the entry is written at its rank, and the value and the word are
// cleared again.
template <int PASS>
__global__ __launch_bounds__(kNumDenseTeam) void k_num_dense(const CaseDesc* __restrict__ cs,
                                                             const BigItem* __restrict__ items,
                                                             const uint32_t* cnt_heavy,
                                                             const uint32_t* cnt_light,
                                                             uint32_t cap4, NumArgs na)
{
    constexpr int TEAM = kNumDenseTeam;
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ double s_a[TEAM];
    __shared__ uint64_t s_red[TEAM / kWave + 1];
    __shared__ uint32_t s_mm[2];
    const int t = threadIdx.x;
    const uint32_t nheavy = *cnt_heavy, total = nheavy + *cnt_light;
    const Csr A = cs[0].A, B = cs[0].B;
    SSP_GLOBAL double* acc = na.pool + (int64_t)blockIdx.x * na.N;
    SSP_GLOBAL uint32_t* mask = na.pool_mask + (int64_t)blockIdx.x * na.mask_words;
    for (uint32_t k = blockIdx.x; k < total; k += gridDim.x) {
        const BigItem item = items[big_index(k, nheavy, cap4)];
        const int64_t row = item.row;
        if (PASS == 2 && num_fits(na, row, na.cnt[row])) continue;
        if (t == 0) {
            s_mm[0] = 0xFFFFFFFFu;
            s_mm[1] = 0u;
        }
        __syncthreads();
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
            for (uint32_t p = t; p < tot; p += TEAM) {
                int lo = 0, hi = nent;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const int32_t q = s_b0[lo] + (int32_t)(p - s_off[lo]);
                const uint32_t col = (uint32_t)B.col[q];
                __hip_atomic_fetch_add(&acc[col], s_a[lo] * na.Bval[q], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or(&mask[col >> 5], 1u << (col & 31u), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t w = col >> 5;
                wmin = w < wmin ? w : wmin;
                wmax = w > wmax ? w : wmax;
            }
            __syncthreads();
        }
        atomicMin(&s_mm[0], wmin);
        atomicMax(&s_mm[1], wmax);
        __threadfence();  // the global atomics have completed
        __syncthreads();
        const uint32_t w0 = s_mm[0], w1 = s_mm[1];
        // count
        uint64_t mine = 0;
        if (w0 <= w1)
            for (uint32_t w = w0 + t; w <= w1; w += TEAM)
                mine += (uint64_t)__popc(
                    __hip_atomic_load(&mask[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
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
                uint32_t bits = 0;
                if (w <= w1)
                    bits = __hip_atomic_load(&mask[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
                                                    __HIP_MEMORY_SCOPE_AGENT);
                        ++o;
                    }
                    acc[col] = 0.0;
                }
                if (w <= w1) mask[w] = 0u;
                base += (int64_t)ctot;
            }
        __threadfence();  // the clears are visible before the next row's atomics
        __syncthreads();
    }
}

// ------------------------------------------------------------- copy pass

// Rows that fitted their slot are copied to C at their final offsets:
// kNumCopyRows rows per workgroup, their entries shared out over the threads
// (each finds its row by binary search over the rows' starts in LDS).
__global__ __launch_bounds__(kNumCopyRows) void k_num_copy(NumArgs na)
{
    __shared__ int64_t s_start[kNumCopyRows + 1];
    __shared__ int64_t s_src[kNumCopyRows], s_dst[kNumCopyRows];
    __shared__ int64_t s_red[kNumCopyRows / kWave + 1];
    const int t = threadIdx.x;
    for (int64_t r0 = (int64_t)blockIdx.x * kNumCopyRows; r0 < na.M;
         r0 += (int64_t)gridDim.x * kNumCopyRows) {
        const int64_t i = r0 + t;
        int64_t n = 0, src = 0, dst = 0;
        if (i < na.M) {
            const int64_t c = na.cnt[i];
            src = na.slot_off[i];
            dst = na.C_rpt[i];
            if (num_fits(na, i, c) && dst + c <= na.capacity) n = c;
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

// Sets n doubles (and the words after them) to zero: the dense accumulators
// when they are first allocated.
__global__ void k_num_zero(uint64_t* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

} // namespace ssp
