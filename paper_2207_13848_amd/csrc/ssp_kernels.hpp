// HIP kernels of the prediction path for gfx950 (wave64).
//
// Order of one prediction (sample first, then one streaming pass):
//   k_init          clear the statistics and counters
//   k_sample_bin    pick the sampled rows (splitmix64), count each one's
//                   products with one wave, add them to f*, bin the row
//   k_sym / k_sym_big
//                   exact distinct-column count of every binned row (LDS hash
//                   table or LDS bitmap; long rows split over workgroups that
//                   merge bitmaps in a global slot), summed into z*
//   k_finalize_*    per-call constants (divisor of f*, reference fractions)
//   k_flop          one coalesced pass over A: products of every row as a
//                   pattern SpMV with the row lengths of B, then the per-row
//                   output (prediction, product count, or bin for the exact
//                   count), and the total F
#pragma once

#include "ssp_device.hpp"
#include "ssp_internal.hpp"

namespace ssp {

struct Csr {
    const int32_t* rpt;
    const int32_t* col;
    int64_t nrows, ncols, nnz;
};

struct BinLists {
    BinItem* b1;
    BinItem* b2;
    BinItem* b3;
    BigItem* b4;
    uint32_t* slots;
};

typedef unsigned long long ull;

__device__ __forceinline__ ull* as_ull(uint64_t* p) { return reinterpret_cast<ull*>(p); }

// ---------------------------------------------------------------- init

__global__ void k_init(Ctl* ctl, ssp_stats* st, uint64_t M)
{
    const int t = threadIdx.x;
    if (t < 8) ctl->bin_cnt[t] = 0;
    if (t == 0) {
        ctl->slot_ctr = 0;
        ctl->fallback = 0;
        st->total_flop = 0;
        st->n_sampled = 0;
        st->sample_flop = 0;
        st->sample_nnz = 0;
        st->out_sum = 0;
        st->nrows = M;
        st->flags = 0;
        st->a_sample_nnz = 0;
    }
}

// ------------------------------------------------------------- binning

// Bin-4 items of one long row: the row's products are cut into `nparts`
// near-equal ranges when a global merge slot is free.
__device__ inline void append_big(int32_t row, uint64_t rf, int64_t N, Ctl* ctl,
                                  const BinLists& L)
{
    const int64_t nwin = (N + kWinCols - 1) / kWinCols;
    int32_t nparts = 1, slot = -1;
    if (rf > kSplitTarget && nwin <= kSlotWindows) {
        const uint32_t s = atomicAdd(&ctl->slot_ctr, 1u);
        if (s < (uint32_t)kMaxSlots) {
            slot = (int32_t)s;
            const uint64_t want = (rf + kSplitTarget - 1) / kSplitTarget;
            nparts = (int32_t)(want < (uint64_t)kMaxParts ? want : (uint64_t)kMaxParts);
        }
    }
    const uint32_t base = atomicAdd(&ctl->bin_cnt[4], (uint32_t)nparts);
    for (int32_t p = 0; p < nparts; ++p) {
        BigItem it;
        it.row = row;
        it.slot = slot;
        it.part = p;
        it.nparts = nparts;
        it.rf = rf;
        L.b4[base + p] = it;
    }
}

__device__ __forceinline__ int bin_of(uint64_t rf)
{
    return rf == 0 ? 0 : rf <= kBin1Max ? 1 : rf <= kBin2Max ? 2 : rf <= kBin3Max ? 3 : 4;
}

// One row, appended by a single lane.
__device__ inline void append_row(int32_t row, uint64_t rf, int64_t N, Ctl* ctl,
                                  const BinLists& L)
{
    const int b = bin_of(rf);
    if (b == 0) return;
    if (b == 4) {
        append_big(row, rf, N, ctl, L);
        return;
    }
    BinItem it;
    it.row = row;
    it.rf = (uint32_t)rf;
    const uint32_t i = atomicAdd(&ctl->bin_cnt[b], 1u);
    (b == 1 ? L.b1 : b == 2 ? L.b2 : L.b3)[i] = it;
}

// ----------------------------------------------------- k_sample_bin

// One thread per candidate (a row of A in Bernoulli mode, a draw in paper
// mode); every wave then walks its sampled rows one by one, counting each
// row's products with all 64 lanes.
template <bool PAPER>
__global__ __launch_bounds__(256) void k_sample_bin(Csr A, Csr B, uint64_t seed, uint64_t thresh,
                                                   int64_t ndraws, Ctl* ctl, ssp_stats* st,
                                                   BinLists L)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = lane_id();
    int32_t row = -1;
    if (PAPER) {
        if (g < ndraws) {
            const u128 x = mul_64x64((uint64_t)A.nrows, splitmix64_at(seed, (uint64_t)g) >> 11);
            row = (int32_t)((x.lo >> 53) | (x.hi << 11));
        }
    } else {
        if (g < A.nrows && (splitmix64_at(seed, (uint64_t)g) >> 11) < thresh) row = (int32_t)g;
    }
    uint64_t mask = __ballot(row >= 0);
    if (mask == 0) return;
    if (lane == 0) atomicAdd(as_ull(&st->n_sampled), (ull)__popcll(mask));
    uint64_t fsum = 0, asum = 0;
    while (mask) {
        const int l = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const int32_t r = __shfl(row, l, kWave);
        const int32_t a0 = A.rpt[r], a1 = A.rpt[r + 1];
        uint64_t s = 0;
        for (int32_t j = a0 + lane; j < a1; j += kWave) s += csr_row_len(B.rpt, A.col[j]);
        const uint64_t rf = wave_sum(s);
        fsum += rf;
        asum += (uint64_t)(a1 - a0);
        if (lane == 0) append_row(r, rf, B.ncols, ctl, L);
    }
    if (lane == 0 && fsum) atomicAdd(as_ull(&st->sample_flop), (ull)fsum);
    if (lane == 0 && asum) atomicAdd(as_ull(&st->a_sample_nnz), (ull)asum);
}

// ------------------------------------------------- distinct counting

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// Open addressing with linear probing on an LDS table of 2^lg words;
// returns 1 when `c` was not yet present.  Columns are < 2^31, so the
// all-ones word marks an empty slot.
__device__ __forceinline__ uint32_t hash_insert(uint32_t* tab, uint32_t c, int lg)
{
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t h = (c * 0x9E3779B1u) >> (32 - lg);
    for (;;) {
        const uint32_t cur = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == c) return 0u;
        if (cur == kEmpty) {
            const uint32_t prev = atomicCAS(&tab[h], kEmpty, c);
            if (prev == kEmpty) return 1u;
            if (prev == c) return 0u;
        }
        h = (h + 1u) & mask;
    }
}

// Bins 1..3: one workgroup of TEAM threads per row.  The row's products are
// enumerated chunk by chunk of TEAM entries of A: a scan of the B row lengths
// gives each product's owner, found by binary search in LDS, so every thread
// handles an equal share of products whatever the B row lengths.  Counting
// uses an LDS bitmap of all N columns when that is no larger than the hash
// table, else the hash table (size >= 2 x the row's distinct bound).
// MODE 0: add the count to z*.  MODE 1: write it to out[row] (and out_sum).
template <int TEAM, int WORDS, int MODE>
__global__ __launch_bounds__(TEAM) void k_sym(Csr A, Csr B, const BinItem* __restrict__ items,
                                             const uint32_t* count, ssp_stats* st,
                                             int64_t* __restrict__ out)
{
    __shared__ uint32_t tab[WORDS];
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint32_t s_off[TEAM];
    __shared__ uint32_t s_red[TEAM / kWave + 1];
    const uint32_t n = *count;
    const int t = threadIdx.x;
    const int64_t N = B.ncols;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const BinItem item = items[it];
        const uint32_t bound = (uint32_t)((int64_t)item.rf < N ? (int64_t)item.rf : N);
        uint32_t tsize = 64;
        while (tsize < 2u * bound) tsize <<= 1;
        const bool bitmap = N <= 32 * (int64_t)tsize;
        const uint32_t words = bitmap ? (uint32_t)((N + 31) / 32) : tsize;
        const int lg = __builtin_ctz(tsize);
        const uint32_t fill = bitmap ? 0u : kEmpty;
        for (uint32_t w = t; w < words; w += TEAM) tab[w] = fill;
        __syncthreads();
        uint32_t cnt = 0;
        const int32_t a0 = A.rpt[item.row], a1 = A.rpt[item.row + 1];
        for (int32_t a = a0; a < a1; a += TEAM) {
            const int32_t j = a + t;
            uint32_t len = 0;
            int32_t b0 = 0;
            if (j < a1) {
                const int32_t k = A.col[j];
                b0 = B.rpt[k];
                len = (uint32_t)(B.rpt[k + 1] - b0);
            }
            uint32_t tot;
            const uint32_t off = block_excl_scan<TEAM, uint32_t>(len, s_red, &tot);
            s_b0[t] = b0;
            s_off[t] = off;
            __syncthreads();
            const int na = (a1 - a) < TEAM ? (a1 - a) : TEAM;
            for (uint32_t p = t; p < tot; p += TEAM) {
                int lo = 0, hi = na;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const uint32_t c = (uint32_t)B.col[s_b0[lo] + (int32_t)(p - s_off[lo])];
                if (bitmap) atomicOr(&tab[c >> 5], 1u << (c & 31));
                else cnt += hash_insert(tab, c, lg);
            }
            __syncthreads();
        }
        if (bitmap)
            for (uint32_t w = t; w < words; w += TEAM) cnt += (uint32_t)__popc(tab[w]);
        const uint32_t total = block_sum<TEAM, uint32_t>(cnt, s_red);
        if (t == 0) {
            if (MODE == 0) {
                atomicAdd(as_ull(&st->sample_nnz), (ull)total);
            } else {
                out[item.row] = (int64_t)total;
                atomicAdd(as_ull(&st->out_sum), (ull)total);
            }
        }
        __syncthreads();
    }
}

// Bin 4: long rows.  1024 threads per item, an LDS bitmap per window of
// 2^20 columns.  An item covers the product range [plo, phi) of its row; when
// a row is split (slot >= 0), every part ORs its window bitmap into the
// row's global slot, and the last part to finish a window counts the merged
// bits and clears the slot again (slots are all-zero between calls).
template <int MODE>
__global__ __launch_bounds__(kBin4Team) void k_sym_big(Csr A, Csr B,
                                                       const BigItem* __restrict__ items,
                                                       const uint32_t* count, uint32_t* slots,
                                                       ssp_stats* st, int64_t* __restrict__ out)
{
    constexpr int TEAM = kBin4Team;
    __shared__ uint32_t bm[kWinWords];
    __shared__ int32_t s_b0[TEAM];
    __shared__ uint64_t s_off[TEAM];
    __shared__ uint64_t s_red[TEAM / kWave + 1];
    __shared__ uint32_t s_last;
    const uint32_t n = *count;
    const int t = threadIdx.x;
    const int64_t N = B.ncols;
    const int64_t nwin = (N + kWinCols - 1) / kWinCols;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const BigItem item = items[it];
        const uint64_t np = (uint64_t)item.nparts, pp = (uint64_t)item.part;
        const uint64_t qq = item.rf / np, rr = item.rf % np;
        const uint64_t plo = qq * pp + (pp < rr ? pp : rr);
        const uint64_t phi = plo + qq + (pp < rr ? 1 : 0);
        const int32_t a0 = A.rpt[item.row], a1 = A.rpt[item.row + 1];
        uint64_t total = 0;
        for (int64_t w = 0; w < nwin; ++w) {
            const int64_t c_lo = w * kWinCols;
            const int64_t wcols = (N - c_lo) < kWinCols ? (N - c_lo) : kWinCols;
            const int words = (int)((wcols + 31) / 32);
            for (int i = t; i < words; i += TEAM) bm[i] = 0u;
            __syncthreads();
            uint64_t goff = 0;
            for (int32_t a = a0; a < a1 && goff < phi; a += TEAM) {
                const int32_t j = a + t;
                uint64_t len = 0;
                int32_t b0 = 0;
                if (j < a1) {
                    const int32_t k = A.col[j];
                    b0 = B.rpt[k];
                    len = (uint64_t)(uint32_t)(B.rpt[k + 1] - b0);
                }
                uint64_t tot;
                const uint64_t off = block_excl_scan<TEAM, uint64_t>(len, s_red, &tot);
                s_b0[t] = b0;
                s_off[t] = off;
                __syncthreads();
                const int na = (a1 - a) < TEAM ? (a1 - a) : TEAM;
                const uint64_t lo_p = plo > goff ? plo : goff;
                const uint64_t hi_p = (goff + tot) < phi ? (goff + tot) : phi;
                for (uint64_t p = lo_p + t; p < hi_p; p += TEAM) {
                    const uint64_t q = p - goff;
                    int lo = 0, hi = na;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_off[mid] <= q) lo = mid;
                        else hi = mid;
                    }
                    const uint64_t c =
                        (uint64_t)(uint32_t)B.col[(int64_t)s_b0[lo] + (int64_t)(q - s_off[lo])];
                    const uint64_t cw = c - (uint64_t)c_lo;
                    if (cw < (uint64_t)wcols) atomicOr(&bm[cw >> 5], 1u << (cw & 31));
                }
                goff += tot;
                __syncthreads();
            }
            if (item.slot < 0) {
                uint64_t cnt = 0;
                for (int i = t; i < words; i += TEAM) cnt += (uint64_t)__popc(bm[i]);
                total += block_sum<TEAM, uint64_t>(cnt, s_red);
            } else {
                uint32_t* g = slots + (int64_t)item.slot * kSlotWords + w * kWinWords;
                uint32_t* ctr = slots + (int64_t)item.slot * kSlotWords +
                                (int64_t)kSlotWindows * kWinWords + w;
                for (int i = t; i < words; i += TEAM) {
                    const uint32_t x = bm[i];
                    if (x) atomicOr(&g[i], x);
                }
                __threadfence();
                __syncthreads();
                if (t == 0) s_last = (atomicAdd(ctr, 1u) == (uint32_t)item.nparts - 1u);
                __syncthreads();
                if (s_last) {
                    __threadfence();
                    uint64_t cnt = 0;
                    for (int i = t; i < words; i += TEAM) {
                        const uint32_t x =
                            __hip_atomic_load(&g[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        cnt += (uint64_t)__popc(x);
                        if (x) __hip_atomic_store(&g[i], 0u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                    }
                    total += block_sum<TEAM, uint64_t>(cnt, s_red);
                    if (t == 0)
                        __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
        }
        if (t == 0 && total) {
            if (MODE == 0) {
                atomicAdd(as_ull(&st->sample_nnz), (ull)total);
            } else {
                atomicAdd(reinterpret_cast<ull*>(&out[item.row]), (ull)total);
                atomicAdd(as_ull(&st->out_sum), (ull)total);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- finalize

__global__ void k_finalize_predict(Ctl* ctl, ssp_stats* st)
{
    if (threadIdx.x != 0) return;
    const uint64_t fs = st->sample_flop;
    if (fs == 0) {
        ctl->fallback = 1;
        st->flags |= SSP_FLAG_EMPTY_SAMPLE;
        return;
    }
    ctl->fallback = 0;
    const Divisor D = make_divisor(fs);
    ctl->div_dn = D.dn;
    ctl->div_v = D.v;
    ctl->div_shift = D.shift;
}

__global__ void k_finalize_reference(Ctl* ctl, ssp_stats* st, uint64_t M)
{
    if (threadIdx.x != 0) return;
    if (st->sample_flop == 0) {
        ctl->fallback = 1;
        st->flags |= SSP_FLAG_EMPTY_SAMPLE;
        return;
    }
    ctl->fallback = 0;
    const u128 q = mul_64x64(st->sample_nnz, M);
    const u128 d = mul_64x64(st->n_sampled, st->total_flop);
    ctl->ref_q_lo = q.lo;
    ctl->ref_q_hi = q.hi;
    ctl->ref_d_lo = d.lo;
    ctl->ref_d_hi = d.hi;
}

// -------------------------------------------------------------- k_flop

enum { FLOP_PREDICT = 0, FLOP_ONLY = 1, FLOP_EXACT_BIN = 2 };

struct FlopArgs {
    Csr A, B;
    int64_t* out;      // PREDICT: nnz_pred; ONLY: row flop; EXACT_BIN: nnz_exact
    int64_t* out_flop; // PREDICT: optional row flop
    ssp_stats* st;
    Ctl* ctl;
    BinLists L;
};

// Tile = 256 * RPT consecutive rows.  The tile's entries of A are streamed in
// chunks of 2048 (two 16-byte loads per thread, each load instruction fully
// coalesced); each entry contributes the length of the B row it names.  An
// exclusive scan of these lengths over the chunk gives the running product
// count at every row boundary of the tile (kept in LDS), and a row's count is
// the difference of its two boundaries.  Rows longer than a chunk simply span
// several chunks.
template <int MODE, int RPT, bool VEC>
__global__ __launch_bounds__(kFlopThreads) void k_flop(FlopArgs a)
{
    constexpr int NT = kFlopThreads, RT = NT * RPT, CH = kFlopChunk, HALF = CH / 2;
    __shared__ int32_t s_bnd[RT + 1];
    __shared__ uint64_t s_rowP[RT + 1];
    __shared__ uint32_t s_x[CH];
    __shared__ uint64_t s_pre0[NT], s_pre1[NT];
    __shared__ uint64_t s_w[2 * (NT / kWave)];
    __shared__ uint64_t s_red[NT / kWave + 1];

    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
    const int64_t M = a.A.nrows;
    const int64_t r0 = (int64_t)blockIdx.x * RT;
    const int nr = (int)((M - r0) < RT ? (M - r0) : RT);
    const int32_t* __restrict__ Arpt = a.A.rpt;
    const int32_t* __restrict__ Acol = a.A.col;
    const int32_t* __restrict__ Brpt = a.B.rpt;
    const int64_t nnzA = a.A.nnz;

    for (int k = t; k <= nr; k += NT) s_bnd[k] = Arpt[r0 + k];
    __syncthreads();
    const int64_t e0 = s_bnd[0], e1 = s_bnd[nr];
    const int64_t a0 = e0 & ~(int64_t)3;
    uint64_t carry = 0;
    int64_t c0 = a0;
    for (; c0 < e1; c0 += CH) {
        uint64_t s[2] = {0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t p = c0 + q * HALF + 4 * t;
            uint32_t x[4] = {0, 0, 0, 0};
            if (p < e1 && p + 3 >= e0) {
                int32_t cc[4];
                if (VEC && p + 3 < nnzA) {
                    const int4 v = *reinterpret_cast<const int4*>(Acol + p);
                    cc[0] = v.x; cc[1] = v.y; cc[2] = v.z; cc[3] = v.w;
                } else {
#pragma unroll
                    for (int l = 0; l < 4; ++l) cc[l] = (p + l < e1) ? Acol[p + l] : 0;
                }
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const int64_t j = p + l;
                    x[l] = (j >= e0 && j < e1) ? csr_row_len(Brpt, cc[l]) : 0u;
                }
            }
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                s_x[q * HALF + 4 * t + l] = x[l];
                s[q] += x[l];
            }
        }
        // exclusive scans of the two halves, in lockstep
        uint64_t i0 = s[0], i1 = s[1];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint64_t u0 = __shfl_up(i0, o, kWave), u1 = __shfl_up(i1, o, kWave);
            if (lane >= o) {
                i0 += u0;
                i1 += u1;
            }
        }
        if (lane == kWave - 1) {
            s_w[wid] = i0;
            s_w[NT / kWave + wid] = i1;
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
        s_pre0[t] = w0 + i0 - s[0];
        s_pre1[t] = tot0 + w1 + i1 - s[1];
        __syncthreads();
        for (int k = t; k <= nr; k += NT) {
            const int64_t d = (int64_t)s_bnd[k] - c0;
            if (d >= 0 && d < CH) {
                const int q = (int)(d / HALF), tt = (int)((d % HALF) >> 2), l = (int)(d & 3);
                uint64_t v = carry + (q ? s_pre1[tt] : s_pre0[tt]);
                const int base = q * HALF + 4 * tt;
                for (int m = 0; m < l; ++m) v += s_x[base + m];
                s_rowP[k] = v;
            }
        }
        carry += tot0 + tot1;
        __syncthreads();
    }
    for (int k = t; k <= nr; k += NT)
        if ((int64_t)s_bnd[k] >= c0) s_rowP[k] = carry;
    __syncthreads();

    // ---- epilogue: one row per thread per pass
    uint64_t fsum = 0, osum = 0;
    Divisor D;
    uint64_t zs = 0;
    uint32_t fallback = 0;
    if (MODE == FLOP_PREDICT) {
        fallback = a.ctl->fallback;
        D.dn = a.ctl->div_dn;
        D.v = a.ctl->div_v;
        D.shift = a.ctl->div_shift;
        zs = a.st->sample_nnz;
    }
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int k = t + rr * NT;
        const bool valid = k < nr;
        const int64_t row = r0 + k;
        const uint64_t rf = valid ? s_rowP[k + 1] - s_rowP[k] : 0;
        fsum += rf;
        if (MODE == FLOP_PREDICT) {
            if (valid) {
                const uint64_t pred = fallback ? rf : (rf ? ceil_mul_div(rf, zs, D) : 0);
                a.out[row] = (int64_t)pred;
                if (a.out_flop) a.out_flop[row] = (int64_t)rf;
                osum += pred;
            }
        } else if (MODE == FLOP_ONLY) {
            if (valid) a.out[row] = (int64_t)rf;
        } else {
            const int b = valid ? bin_of(rf) : 0;
#pragma unroll
            for (int bb = 1; bb <= 3; ++bb) {
                const uint64_t m = __ballot(b == bb);
                if (m) {
                    const int leader = __ffsll((long long)m) - 1;
                    uint32_t base = 0;
                    if (lane == leader) base = atomicAdd(&a.ctl->bin_cnt[bb], (uint32_t)__popcll(m));
                    base = __shfl(base, leader, kWave);
                    if (b == bb) {
                        BinItem it;
                        it.row = (int32_t)row;
                        it.rf = (uint32_t)rf;
                        (bb == 1 ? a.L.b1 : bb == 2 ? a.L.b2 : a.L.b3)[base + rank_in(m)] = it;
                    }
                }
            }
            if (valid && (b == 0 || b == 4)) a.out[row] = 0;
            if (b == 4) append_big((int32_t)row, rf, a.B.ncols, a.ctl, a.L);
        }
    }
    const uint64_t F = block_sum<NT, uint64_t>(fsum, s_red);
    if (t == 0 && F) atomicAdd(as_ull(&a.st->total_flop), (ull)F);
    if (MODE == FLOP_PREDICT) {
        const uint64_t O = block_sum<NT, uint64_t>(osum, s_red);
        if (t == 0 && O) atomicAdd(as_ull(&a.st->out_sum), (ull)O);
    }
}

// --------------------------------------------------- reference rows

// nnz_ref[i] = ceil(rf_i * (z* M) / (n_s F)), saturating at INT64_MAX.
__global__ __launch_bounds__(256) void k_ref_rows(const int64_t* __restrict__ rf_in,
                                                  int64_t* __restrict__ out, int64_t M, Ctl* ctl,
                                                  ssp_stats* st)
{
    __shared__ uint64_t s_red[256 / kWave + 1];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t fallback = ctl->fallback;
    const u128 Q = {ctl->ref_q_lo, ctl->ref_q_hi};
    const u128 Dd = {ctl->ref_d_lo, ctl->ref_d_hi};
    uint64_t v = 0;
    bool sat = false;
    if (i < M) {
        const uint64_t rf = (uint64_t)rf_in[i];
        if (fallback || rf == 0) {
            v = rf;
        } else {
            const u128 p0 = mul_64x64(rf, Q.lo), p1 = mul_64x64(rf, Q.hi);
            const uint64_t l1 = p0.hi + p1.lo;
            const uint64_t l2 = p1.hi + (l1 < p0.hi);
            if (l2 != 0) {
                sat = true;
            } else {
                const u128 c = u128_ceil_div(u128{p0.lo, l1}, Dd);
                if (c.hi != 0 || c.lo > 0x7fffffffffffffffull) sat = true;
                else v = c.lo;
            }
            if (sat) v = 0x7fffffffffffffffull;
        }
        out[i] = (int64_t)v;
    }
    if (__ballot(sat) && lane_id() == 0) atomicOr(as_ull(&st->flags), (ull)SSP_FLAG_SATURATED);
    const uint64_t O = block_sum<256, uint64_t>(v, s_red);
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
