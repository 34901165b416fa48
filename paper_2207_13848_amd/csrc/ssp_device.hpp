// Device-side helpers shared by the HIP kernels: the row sampler's
// splitmix64, exact 128-bit arithmetic for the per-row ceilings, and
// wave64 / workgroup scans and reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssp {

constexpr int kWave = 64;

// ------------------------------------------------------------- sampler

// splitmix64 (Steele, Lea & Flood, OOPSLA 2014): the state starts at `seed`
// and advances by the golden-ratio increment; the (i+1)-th output is the
// state after i+1 steps passed through the finaliser.
__host__ __device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// --------------------------------------------------- 128-bit arithmetic

struct u128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ u128 mul_64x64(uint64_t a, uint64_t b)
{
    u128 r;
    r.lo = a * b;
    r.hi = __umul64hi(a, b);
    return r;
}

// Reciprocal of a normalised divisor d (top bit set):
//   v = floor((2^128 - 1) / d) - 2^64,
// i.e. the 64-bit quotient of the 128-bit number (~d, ~0) by d.  Plain
// restoring division; run only for rows of 2^48 or more products (the others
// take ceil_mul_div_est).
__device__ inline uint64_t reciprocal_of_normalised(uint64_t d)
{
    uint64_t rem = ~d, low = ~0ull, q = 0;
    for (int b = 0; b < 64; ++b) {
        const uint64_t top = rem >> 63;
        rem = (rem << 1) | (low >> 63);
        low <<= 1;
        q <<= 1;
        if (top || rem >= d) {
            rem -= d;
            q |= 1;
        }
    }
    return q;
}

// 2-by-1 division with a precomputed reciprocal (Moller & Granlund,
// "Improved division by invariant integers", IEEE TC 2011, Algorithm 4):
// divides (u1, u0) by normalised d, needs u1 < d; returns the quotient and
// stores the remainder.
__device__ __forceinline__ uint64_t div_2by1(uint64_t u1, uint64_t u0, uint64_t d, uint64_t v,
                                             uint64_t* rem)
{
    const u128 p = mul_64x64(v, u1);
    const uint64_t q0 = p.lo + u0;
    const uint64_t carry = q0 < u0;
    uint64_t q1 = p.hi + u1 + carry + 1;
    uint64_t r = u0 - q1 * d;
    if (r > q0) {
        q1 -= 1;
        r += d;
    }
    if (r >= d) {
        q1 += 1;
        r -= d;
    }
    *rem = r;
    return q1;
}

// Per-call constants to divide by the invariant f* (the sampled FLOP).
struct Divisor {
    uint64_t dn;    // f* << shift
    uint64_t v;     // reciprocal of dn
    uint32_t shift; // leading zeros of f*
    uint32_t pad;
};

__device__ inline Divisor make_divisor(uint64_t d)
{
    Divisor D;
    D.shift = (uint32_t)__clzll((long long)d);
    D.dn = d << D.shift;
    D.v = reciprocal_of_normalised(D.dn);
    D.pad = 0;
    return D;
}

// ceil(a * b / d) for a * b / d < 2^63 (true when b <= d and a < 2^63).
__device__ __forceinline__ uint64_t ceil_mul_div(uint64_t a, uint64_t b, const Divisor& D)
{
    const u128 x = mul_64x64(a, b);
    const uint32_t s = D.shift;
    const uint64_t u1 = s ? ((x.hi << s) | (x.lo >> (64 - s))) : x.hi;
    const uint64_t u0 = x.lo << s;
    uint64_t r;
    const uint64_t q = div_2by1(u1, u0, D.dn, D.v, &r);
    return q + (r != 0);
}

// The same ceiling from a double-precision estimate corrected in integers, for
// a < 2^48 and b <= d < 2^62, with r = (double)b / (double)d.  a is exact as a
// double, and the rounding of b, d, r and a r (each within 2^-53 relative)
// leaves the estimate within 2^48 * 2^-51 = 1/8 of a b / d, so q0 = floor of
// the estimate has a b - q0 d in [-d/8, 9d/8): that remainder, taken modulo
// 2^64, is exact as a signed 64-bit value and places a b / d in (q0 - 1, q0),
// [q0, q0 + 1) or [q0 + 1, q0 + 2).  Six 32-bit multiplies against fifteen.
constexpr uint64_t kEstMaxA = 1ull << 48;
constexpr uint64_t kEstMaxD = 1ull << 62;

__device__ __forceinline__ uint64_t ceil_mul_div_est(uint64_t a, uint64_t b, uint64_t d, double r)
{
    const uint64_t q0 = (uint64_t)((double)a * r);  // truncation = floor (non-negative)
    const int64_t R = (int64_t)(a * b - q0 * d);
    if (R < 0) return q0;
    if ((uint64_t)R < d) return q0 + (R != 0);
    return q0 + 1 + ((uint64_t)R != d);
}

// Part windows in the sampling scan's running sums, which carry them in the
// upper 32 bits of a packed 64-bit value: a group's count is clamped to
// budget + 1, and so is the carry between chunks of groups.  A prefix above
// the budget only has to stay above it (no later group is split then), and
// with these bounds the field cannot wrap, whatever the counts (a chunk adds
// at most 1024 (budget + 1) to a carry of at most budget + 1, budget <= 2^13).
__host__ __device__ __forceinline__ uint32_t clamp_windows(uint32_t wins, uint32_t budget)
{
    return wins <= budget ? wins : budget + 1u;
}

__host__ __device__ __forceinline__ uint64_t saturate_windows_hi(uint64_t packed, uint32_t budget)
{
    return (packed >> 32) <= (uint64_t)budget
               ? packed
               : (packed & 0xffffffffull) | ((uint64_t)(budget + 1u) << 32);
}

__host__ __device__ __forceinline__ bool u128_lt(u128 a, u128 b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

__host__ __device__ __forceinline__ u128 u128_sub(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo);
    return r;
}

__device__ __forceinline__ int u128_clz(u128 a)
{
    return a.hi ? __clzll((long long)a.hi) : 64 + (a.lo ? __clzll((long long)a.lo) : 64);
}

__device__ __forceinline__ u128 u128_shl(u128 a, int s)
{
    if (s == 0) return a;
    if (s >= 64) return u128{0, a.lo << (s - 64)};
    return u128{a.lo << s, (a.hi << s) | (a.lo >> (64 - s))};
}

// ceil(n / d) for 128-bit n and d > 0, by shift-and-subtract (the
// reference design only; not on the proposed method's path).
__device__ inline u128 u128_ceil_div(u128 n, u128 d)
{
    u128 q{0, 0};
    if (u128_lt(n, d)) {
        return (n.lo | n.hi) ? u128{1, 0} : u128{0, 0};
    }
    const int sh = u128_clz(d) - u128_clz(n);
    u128 dd = u128_shl(d, sh);
    u128 r = n;
    for (int b = sh; b >= 0; --b) {
        if (!u128_lt(r, dd)) {
            r = u128_sub(r, dd);
            if (b >= 64) q.hi |= 1ull << (b - 64);
            else q.lo |= 1ull << b;
        }
        dd = u128{(dd.lo >> 1) | (dd.hi << 63), dd.hi >> 1};
    }
    if (r.lo | r.hi) {
        q.lo += 1;
        q.hi += (q.lo == 0);
    }
    return q;
}

// ceil(n / d) for the 192-bit n = (n2, n1, n0) (n2 the top 64 bits) and
// 0 < d < 2^127 with (n2, n1) < d, i.e. a quotient below 2^64: the top 128
// bits are the first partial remainder and the 64 low bits are brought down
// one per step (restoring division; the partial remainder stays below d, so
// doubling it cannot overflow).  The reference design's rows whose numerator
// exceeds 128 bits.
__host__ __device__ inline uint64_t ceil_div_192_by_128(uint64_t n2, uint64_t n1, uint64_t n0,
                                                        u128 d)
{
    u128 r{n1, n2};
    uint64_t q = 0;
    for (int b = 63; b >= 0; --b) {
        r = u128{(r.lo << 1) | ((n0 >> b) & 1u), (r.hi << 1) | (r.lo >> 63)};
        q <<= 1;
        if (!u128_lt(r, d)) {
            r = u128_sub(r, d);
            q |= 1u;
        }
    }
    return q + ((r.lo | r.hi) != 0);
}

// ---------------------------------------------------- wave / block ops

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Lane shifts by DPP: VALU data movement, which (unlike __shfl_*, a
// ds_bpermute through the LDS crossbar) takes no LDS bandwidth from the other
// waves of the workgroup.  Lanes whose source lies outside the row read 0
// (bound_ctrl); lanes of rows left out by ROW_MASK get 0 (the `old` value).
// Every lane of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, true);
}

template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_shift(T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)u);
        const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(u >> 32));
        return (T)(((uint64_t)hi << 32) | lo);
    } else {
        return (T)dpp_u32<CTRL, ROW_MASK>((uint32_t)v);
    }
}

// Inclusive scan over the 64 lanes: shifts by 1, 2, 4, 8 within each row of
// 16 lanes (row_shr), then the last lane of rows 0 and 2 added to rows 1 and
// 3 (row_bcast:15), then lane 31 added to rows 2 and 3 (row_bcast:31).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x)
{
    x += dpp_shift<0x111, 0xf>(x);
    x += dpp_shift<0x112, 0xf>(x);
    x += dpp_shift<0x114, 0xf>(x);
    x += dpp_shift<0x118, 0xf>(x);
    x += dpp_shift<0x142, 0xa>(x);
    x += dpp_shift<0x143, 0xc>(x);
    return x;
}

// Value of lane 63, in every lane.
template <typename T>
__device__ __forceinline__ T lane63(T v)
{
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, kWave - 1);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), kWave - 1);
        return (T)(((uint64_t)hi << 32) | lo);
    } else {
        return (T)__builtin_amdgcn_readlane((uint32_t)v, kWave - 1);
    }
}

// Sum over the wave, returned to every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    return lane63(wave_incl_scan(v));
}

// Value of lane `l` (wave-uniform), in every lane.
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l)
{
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
        return (T)(((uint64_t)hi << 32) | lo);
    } else {
        return (T)__builtin_amdgcn_readlane((uint32_t)v, l);
    }
}

// Inclusive scan of the wave totals staged in sm[0..NW): lane w < NW holds
// the prefix through wave w (one row of 16 lanes, row_shr steps).
template <int NW, typename T>
__device__ __forceinline__ T scan_wave_totals(const T* sm)
{
    static_assert(NW >= 1 && NW <= 16, "wave totals within one row of 16 lanes");
    const int lane = lane_id();
    T x = lane < NW ? sm[lane] : T(0);
    x += dpp_shift<0x111, 0xf>(x);
    x += dpp_shift<0x112, 0xf>(x);
    x += dpp_shift<0x114, 0xf>(x);
    x += dpp_shift<0x118, 0xf>(x);
    return x;
}

// Exclusive scan over the workgroup (NT threads, a multiple of 64, at most
// 1024).  `sm` needs NT/64 entries.  Ends with a barrier so `sm` can be reused.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* sm, T* total)
{
    const T inc = wave_incl_scan(v);
    if constexpr (NT == kWave) {
        *total = lane63(inc);
        return inc - v;
    } else {
        constexpr int NW = NT / kWave;
        const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        if (lane_id() == kWave - 1) sm[wid] = inc;
        __syncthreads();
        const T x = scan_wave_totals<NW>(sm);
        const T pre = wid > 0 ? lane_value(x, wid - 1) : T(0);
        *total = lane_value(x, NW - 1);
        __syncthreads();
        return pre + inc - v;
    }
}

// Two exclusive scans over the workgroup in one pass (one pair of barriers).
// `sm` needs 2 NT/64 entries.  Ends with a barrier so `sm` can be reused.
template <int NT, typename T>
__device__ __forceinline__ void block_excl_scan2(T a, T b, T* sm, T* ea, T* eb, T* ta, T* tb)
{
    static_assert(NT > kWave, "workgroup of several waves");
    constexpr int NW = NT / kWave;
    const T ia = wave_incl_scan(a), ib = wave_incl_scan(b);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (lane_id() == kWave - 1) {
        sm[wid] = ia;
        sm[NW + wid] = ib;
    }
    __syncthreads();
    const T xa = scan_wave_totals<NW>(sm), xb = scan_wave_totals<NW>(sm + NW);
    *ea = (wid > 0 ? lane_value(xa, wid - 1) : T(0)) + ia - a;
    *eb = (wid > 0 ? lane_value(xb, wid - 1) : T(0)) + ib - b;
    *ta = lane_value(xa, NW - 1);
    *tb = lane_value(xb, NW - 1);
    __syncthreads();
}

// K exclusive scans over the workgroup at once, with one pair of barriers for
// all of them.  `sm` needs K * NT/64 entries.  Ends with a barrier.
template <int NT, int K, typename T>
__device__ __forceinline__ void block_excl_scan_n(const T (&v)[K], T* sm, T (&ex)[K], T (&total)[K])
{
    constexpr int NW = NT / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    T inc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) inc[k] = wave_incl_scan(v[k]);
    if (lane_id() == kWave - 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) sm[k * NW + wid] = inc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const T x = scan_wave_totals<NW>(sm + k * NW);
        const T pre = wid > 0 ? lane_value(x, wid - 1) : T(0);
        total[k] = lane_value(x, NW - 1);
        ex[k] = pre + inc[k] - v[k];
    }
    __syncthreads();
}

// Sum over the workgroup, returned to every thread.  `sm` needs NT/64 entries.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* sm)
{
    v = wave_sum(v);
    if constexpr (NT == kWave) {
        return v;
    } else {
        constexpr int NW = NT / kWave;
        const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        if (lane_id() == 0) sm[wid] = v;
        __syncthreads();
        const T tot = lane_value(scan_wave_totals<NW>(sm), NW - 1);
        __syncthreads();
        return tot;
    }
}

// Rank of this lane among the lanes whose bit is set in `mask`.
__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// OR `bits` into word `word` of an LDS bitmap (kNoWord: nothing), one LDS
// atomic per lane that returns nothing.  Neither reading the word first to
// skip bits already set nor combining neighbouring lanes that name one word
// by a segmented OR over the wave paid for itself: the read put an LDS round
// trip on every insert, the combining cost a dozen cross-lane shuffles to
// save a few atomics on one word (bins of R-MAT 2^16: 26.4 us with both, 25.4
// without the read, 18.9 without either).
constexpr uint32_t kNoWord = 0xFFFFFFFFu;

__device__ __forceinline__ void lds_bitmap_or(uint32_t* bm, uint32_t word, uint32_t bits)
{
    if (word != kNoWord) atomicOr(&bm[word], bits);
}

// Word w of a bitmap lives at w ^ ((w >> 6) & 63): its 64-word row keeps its
// place and the low six bits (the LDS bank) are scrambled by the row index,
// so lanes striding a sorted B row (word index advancing a few words per lane)
// spread over the banks instead of meeting every 64 words.  A bijection on
// every aligned run of 64 words; popcounts and ORs of whole bitmaps do not
// see it.
__device__ __forceinline__ uint32_t swz(uint32_t w) { return w ^ ((w >> 6) & 63u); }

// V columns per lane (kNoWord = none), normally neighbours in one B row:
// runs of them that fall in one bitmap word (sorted rows make such runs
// contiguous) are first combined inside the lane; then every remaining word
// goes to an LDS atomic OR, which returns nothing, so the wave does not wait
// on it.  (Reading each word first and ORing only the bits not yet set saved
// atomics on columns seen before, but put the read's latency on every insert:
// the long-row kernel on R-MAT 2^20 took 114 us that way, 98 us without.)
// Unsorted or repeated columns stay correct.  Columns outside the window
// [clo, clo + wc) are skipped.  No cross-lane traffic.
template <int V>
__device__ __forceinline__ void lane_bitmap_insert(uint32_t* bm, const uint32_t (&col)[V],
                                                   uint32_t clo, uint32_t wc)
{
    uint32_t word[V], bits[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const uint32_t cw = col[v] - clo;  // columns < 2^31: wraps above wc when col < clo
        const bool in = col[v] != kNoWord && cw < wc;
        word[v] = in ? (cw >> 5) : kNoWord;
        bits[v] = 1u << (cw & 31);
    }
#pragma unroll
    for (int v = 1; v < V; ++v) {
        const bool same = word[v] == word[v - 1];
        bits[v] = same ? (bits[v] | bits[v - 1]) : bits[v];
        word[v - 1] = same ? kNoWord : word[v - 1];
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (word[v] != kNoWord) atomicOr(&bm[swz(word[v])], bits[v]);
}

// The same for one window holding all N columns (columns are < N, so no
// window test): four neighbouring columns of one lane, as loaded.
__device__ __forceinline__ void lane_bitmap_insert4(uint32_t* bm, const int32_t __attribute__((ext_vector_type(4)))& v)
{
    const uint32_t c0 = (uint32_t)v.x, c1 = (uint32_t)v.y, c2 = (uint32_t)v.z, c3 = (uint32_t)v.w;
    const uint32_t w0 = c0 >> 5, w1 = c1 >> 5, w2 = c2 >> 5, w3 = c3 >> 5;
    uint32_t b0 = 1u << (c0 & 31), b1 = 1u << (c1 & 31), b2 = 1u << (c2 & 31),
             b3 = 1u << (c3 & 31);
    const bool s1 = w1 == w0, s2 = w2 == w1, s3 = w3 == w2;  // run continues
    b1 |= s1 ? b0 : 0u;
    b2 |= s2 ? b1 : 0u;
    b3 |= s3 ? b2 : 0u;
    const uint32_t p0 = swz(w0), p1 = swz(w1), p2 = swz(w2), p3 = swz(w3);
    // a word is ORed at the end of its run only
    if (!s1) atomicOr(&bm[p0], b0);
    if (!s2) atomicOr(&bm[p1], b1);
    if (!s3) atomicOr(&bm[p2], b2);
    atomicOr(&bm[p3], b3);
}

// V independent columns per lane (kNoWord = none), one window holding all
// N columns: an LDS OR per column, no merging.
template <int V>
__device__ __forceinline__ void lane_bitmap_insert_all(uint32_t* bm, const uint32_t (&col)[V])
{
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (col[v] != kNoWord) atomicOr(&bm[swz(col[v] >> 5)], 1u << (col[v] & 31));
}

// Global-memory pointers (device code): see ssp_internal.hpp.
#ifndef SSP_GLOBAL
#ifdef __HIP_DEVICE_COMPILE__
#define SSP_GLOBAL __attribute__((address_space(1)))
#else
#define SSP_GLOBAL
#endif
#endif

// 8- and 16-byte vectors of int32 at 4-byte alignment, for wide loads of
// CSR arrays at any entry
typedef int32_t i32x2u __attribute__((ext_vector_type(2), aligned(4)));
typedef int32_t i32x4u __attribute__((ext_vector_type(4), aligned(4)));

// A raw buffer resource over the `bytes` bytes at p (clamped to 2^32 - 1).
// Loads through it at a byte offset (register plus instruction offset) at or
// past the end return 0 and touch no memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const SSP_GLOBAL void* p,
                                                              uint64_t bytes)
{
    const uint32_t n = bytes < 0xFFFFFFFFull ? (uint32_t)bytes : 0xFFFFFFFFu;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>((const void*)p), (short)0, (int)n,
                                             0x00020000);
}

// Length of row k of a CSR matrix from its row pointers: one 8-byte read
// of rpt[k], rpt[k+1].
__device__ __forceinline__ uint32_t csr_row_len(const SSP_GLOBAL int32_t* __restrict__ rpt,
                                                int32_t k)
{
    const i32x2u v = *(const SSP_GLOBAL i32x2u*)(rpt + k);
    return (uint32_t)(v.y - v.x);
}

} // namespace ssp
