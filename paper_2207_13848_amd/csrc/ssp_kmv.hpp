// The existing sampling estimator the paper compares against (Sec. III):
// Amossen et al.'s k-minimum-values sketch over the intermediate products of
// C' = A'B', with BHash's sampling of rows of A and columns of B at the same
// probability, NNZ(C) = NNZ(C') / p^2.  C-ABI entry ssp_kmv_estimate
// (declared in include/ssp.h).  Included at the end of ssp_lib.hip.
//
//   row i of A kept     iff (splitmix64(seed,     i) >> 11) < floor(rate 2^53)
//   column j of B kept  iff (splitmix64(seed + 1, j) >> 11) < floor(rate 2^53)
//   hash of (i, j)      =   splitmix64(seed + 2, i N + j) >> 11   (53 bits)
//
// The k-th smallest distinct hash is found by keeping only the hashes below a
// threshold tau in a global hash set: tau starts where about 4k of the
// sample's products fall below it and is halved when the set would hold too
// many values, quadrupled when it holds fewer than k (up to all values).
// Every value below tau is in the set, so once it holds at least k values its
// k-th smallest is the sketch's exactly; a one-workgroup bitonic sort in LDS
// picks it.
#pragma once

namespace ssp {

constexpr int kKmvSetLg = 16;                         // set slots: 2^16 (512 KiB)
constexpr uint32_t kKmvMaxKept = 16384;               // values the selection sorts, at most
constexpr uint32_t kKmvStop = 2 * kKmvMaxKept;        // inserts stop here (tau is then halved)
constexpr uint32_t kKmvKMax = 4096;
constexpr int kKmvThreads = 256;
constexpr int kKmvUnroll = 8;  // products per thread whose loads are in flight together

struct KmvCounters {
    uint64_t rows, cols, products;
    uint32_t distinct, overflow;
    uint64_t kth;
    uint32_t nlight, nheavy;  // work items: kept rows of <= kKmvThreads entries; chunks of longer rows
    uint64_t pad[2];
};

__device__ __forceinline__ bool kmv_kept(uint64_t seed, uint64_t i, uint64_t T)
{
    return (splitmix64_at(seed, i) >> 11) < T;
}

// Inserts hash value hv into the set (0 marks a free slot, so hv + 1 is stored).
__device__ __forceinline__ void kmv_insert(uint64_t* set, uint64_t hv, KmvCounters* c)
{
    if (__hip_atomic_load(&c->distinct, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= kKmvStop) {
        c->overflow = 1u;
        return;
    }
    const uint64_t key = hv + 1u;
    const uint32_t mask = (1u << kKmvSetLg) - 1u;
    uint32_t h = (uint32_t)((hv * 0x9E3779B97F4A7C15ull) >> (64 - kKmvSetLg));
    for (uint32_t n = 0; n <= mask; ++n) {
        const uint64_t cur = __hip_atomic_load(&set[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) return;
        if (cur == 0) {
            const uint64_t prev = atomicCAS((unsigned long long*)&set[h], 0ull, (unsigned long long)key);
            if (prev == 0) {
                atomicAdd(&c->distinct, 1u);
                return;
            }
            if (prev == key) return;
        }
        h = (h + 1u) & mask;
    }
    c->overflow = 1u;
}

// Kept columns of B.
__global__ __launch_bounds__(kKmvThreads) void k_kmv_cols(int64_t N, uint64_t T, uint64_t seed,
                                                         KmvCounters* c)
{
    __shared__ uint64_t s_red[kKmvThreads / kWave + 1];
    uint64_t n = 0;
    for (int64_t j = (int64_t)blockIdx.x * kKmvThreads + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * kKmvThreads)
        n += kmv_kept(seed + 1u, (uint64_t)j, T) ? 1u : 0u;
    n = block_sum<kKmvThreads, uint64_t>(n, s_red);
    if (threadIdx.x == 0 && n) atomicAdd((unsigned long long*)&c->cols, (unsigned long long)n);
}

// The kept rows of A as work items: a row of at most kKmvThreads entries is
// one item (light list); a longer row is cut into chunks of kKmvThreads
// entries, one item each (heavy list), so hub rows are shared out over many
// workgroups.  Light rows are appended with one atomic per wave.
__global__ __launch_bounds__(kKmvThreads) void k_kmv_rows(Csr A, uint64_t T, uint64_t seed,
                                                         int32_t* light, int2* heavy,
                                                         KmvCounters* c)
{
    const int lane = lane_id();
    for (int64_t r0 = (int64_t)blockIdx.x * kKmvThreads; r0 < A.nrows;
         r0 += (int64_t)gridDim.x * kKmvThreads) {
        const int64_t r = r0 + threadIdx.x;
        const bool kept = r < A.nrows && kmv_kept(seed, (uint64_t)r, T);
        const int32_t len = kept ? A.rpt[r + 1] - A.rpt[r] : 0;
        const bool lt = kept && len <= kKmvThreads;
        const uint64_t m = __ballot(lt);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t pos = 0;
            if (lane == leader) pos = atomicAdd(&c->nlight, (uint32_t)__popcll(m));
            pos = __shfl(pos, leader, kWave);
            if (lt) light[pos + rank_in(m)] = (int32_t)r;
        }
        if (kept && !lt) {
            const int32_t nch = (len + kKmvThreads - 1) / kKmvThreads;
            const uint32_t base = atomicAdd(&c->nheavy, (uint32_t)nch);
            for (int32_t q = 0; q < nch; ++q) heavy[base + q] = make_int2((int32_t)r, q);
        }
        const uint64_t km = __ballot(kept);
        if (lane == 0 && km)
            atomicAdd((unsigned long long*)&c->rows, (unsigned long long)__popcll(km));
    }
}

// MODE 0: the products of C'.  MODE 1: every product's hash below tau into
// the set.  One work item (a light row or a chunk of a heavy one, at most
// kKmvThreads entries of A) per workgroup at a time; its products are
// enumerated over the workgroup (scan of the B row lengths, owner by binary
// search in LDS), kKmvUnroll per thread with their loads in flight together.
template <int MODE>
__global__ __launch_bounds__(kKmvThreads) void k_kmv_pass(Csr A, Csr B, uint64_t T, uint64_t seed,
                                                         uint64_t tau, uint64_t* set,
                                                         const int32_t* light, const int2* heavy,
                                                         KmvCounters* c)
{
    constexpr int NT = kKmvThreads;
    __shared__ int32_t s_b0[NT];
    __shared__ uint32_t s_off[NT];
    __shared__ uint32_t s_red[NT / kWave + 1];
    __shared__ uint64_t s_red64[NT / kWave + 1];
    const int t = threadIdx.x;
    const int64_t N = B.ncols;
    const uint32_t nl = c->nlight, nitems = nl + c->nheavy;
    uint64_t prods = 0;
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        int32_t i, a, a1;
        if (it < nl) {
            i = light[it];
            a = A.rpt[i];
            a1 = A.rpt[i + 1];
        } else {
            const int2 h = heavy[it - nl];
            i = h.x;
            a = A.rpt[i] + h.y * NT;
            const int32_t e = A.rpt[i + 1];
            a1 = (a + NT) < e ? (a + NT) : e;
        }
        const int32_t j = a + t;
        uint32_t len = 0;
        int32_t b0 = 0;
        if (j < a1) {
            const int32_t k = A.col[j];
            b0 = B.rpt[k];
            len = (uint32_t)(B.rpt[k + 1] - b0);
        }
        uint32_t tot;
        const uint32_t off = block_excl_scan<NT, uint32_t>(len, s_red, &tot);
        s_b0[t] = b0;
        s_off[t] = off;
        __syncthreads();
        const int nent = a1 - a;
        for (uint32_t p0 = 0; p0 < tot; p0 += NT * kKmvUnroll) {
            int32_t colv[kKmvUnroll];
#pragma unroll
            for (int u = 0; u < kKmvUnroll; ++u) {
                const uint32_t pr = p0 + (uint32_t)(u * NT + t);
                const uint32_t p = pr < tot ? pr : tot - 1;  // (clamped: loads unconditional)
                int lo = 0, hi = nent;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid;
                    else hi = mid;
                }
                colv[u] = B.col[s_b0[lo] + (int32_t)(p - s_off[lo])];
            }
#pragma unroll
            for (int u = 0; u < kKmvUnroll; ++u) {
                const uint64_t col = (uint64_t)colv[u];
                if (p0 + (uint32_t)(u * NT + t) >= tot || !kmv_kept(seed + 1u, col, T)) continue;
                if (MODE == 0) {
                    ++prods;
                } else {
                    const uint64_t hv = splitmix64_at(seed + 2u, (uint64_t)i * (uint64_t)N + col) >> 11;
                    if (hv < tau) kmv_insert(set, hv, c);
                }
            }
        }
        __syncthreads();
    }
    if (MODE == 0) {
        prods = block_sum<NT, uint64_t>(prods, s_red64);
        if (t == 0 && prods) atomicAdd((unsigned long long*)&c->products, (unsigned long long)prods);
    }
}

__global__ void k_kmv_reset(KmvCounters* c)
{
    if (threadIdx.x == 0) {
        c->distinct = 0;
        c->overflow = 0;
    }
}

// One workgroup: the set's values (at most kKmvMaxKept) into LDS, a bitonic
// sort, the k-th smallest out.
__global__ __launch_bounds__(1024) void k_kmv_select(const uint64_t* set, uint32_t k, KmvCounters* c)
{
    constexpr int NT = 1024, SPT = (1 << kKmvSetLg) / NT;
    extern __shared__ __align__(16) uint64_t s_v[];  // kKmvMaxKept values
    __shared__ uint32_t s_red[NT / kWave + 1];
    const int t = threadIdx.x;
    uint32_t mine = 0;  // (the slots are read twice: counted, then written)
    for (int u = 0; u < SPT; ++u) mine += set[t * SPT + u] != 0 ? 1u : 0u;
    uint32_t n;
    uint32_t pos = block_excl_scan<NT, uint32_t>(mine, s_red, &n);
    if (n > kKmvMaxKept || n < k) return;  // (the host calls with kKmvMaxKept >= n >= k)
    for (int u = 0; u < SPT; ++u) {
        const uint64_t v = set[t * SPT + u];
        if (v != 0) s_v[pos++] = v - 1u;
    }
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t i = n + t; i < P; i += NT) s_v[i] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = t; i < P / 2; i += NT) {
                // the lower element of the i-th compare-exchange pair
                const uint32_t lo = 2 * i - (i & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = s_v[lo], b = s_v[hi];
                if ((a > b) == up) {
                    s_v[lo] = b;
                    s_v[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    if (t == 0) c->kth = s_v[k - 1];
}

} // namespace ssp

namespace {

ssp_status kmv_estimate(ssp_handle h, const ssp_csr* A, const ssp_csr* B, double rate, uint32_t k,
                        uint64_t seed, ssp_kmv_result* out, hipStream_t s)
{
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kmv_select),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(kKmvMaxKept * sizeof(uint64_t)));
    });
    const int64_t M = A->nrows, N = B->ncols;
    const size_t set_bytes = ((size_t)1 << kKmvSetLg) * sizeof(uint64_t);
    const size_t o_light = set_bytes + align256(sizeof(KmvCounters));
    const size_t o_heavy = o_light + align256((size_t)std::max<int64_t>(M, 1) * sizeof(int32_t));
    // (chunks of the long rows: at most nnz(A) / kKmvThreads + rows)
    const size_t heavy_cap = (size_t)(A->nnz / kKmvThreads + M + 1);
    ssp_status st = ensure_workspace(h, o_heavy + heavy_cap * sizeof(int2));
    if (st != SSP_OK) return st;
    uint64_t* set = static_cast<uint64_t*>(h->ws);
    KmvCounters* cnt = reinterpret_cast<KmvCounters*>(static_cast<char*>(h->ws) + set_bytes);
    int32_t* light = reinterpret_cast<int32_t*>(static_cast<char*>(h->ws) + o_light);
    int2* heavy = reinterpret_cast<int2*>(static_cast<char*>(h->ws) + o_heavy);
    const Csr a = to_csr(A), b = to_csr(B);
    const uint64_t T = rate_threshold(rate);
    const int cus = h->num_cus;
    const unsigned grid_rows = (unsigned)std::max<int64_t>(1, std::min<int64_t>((M + kKmvThreads - 1) / kKmvThreads, 8LL * cus));
    const unsigned grid_cols = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + kKmvThreads - 1) / kKmvThreads, 4LL * cus));
    const unsigned grid_set = (unsigned)(((1u << kKmvSetLg) + 255) / 256);
    const unsigned grid_items = (unsigned)(8 * cus);  // (the items are counted on the device)
    const int64_t words = (int64_t)((set_bytes + sizeof(KmvCounters)) / sizeof(uint64_t));
    // kept rows and columns, products of C'
    hipLaunchKernelGGL(k_num_zero, dim3(grid_set), dim3(256), 0, s, (uint64_t*)h->ws, words);
    hipLaunchKernelGGL(k_kmv_cols, dim3(grid_cols), dim3(kKmvThreads), 0, s, N, T, seed, cnt);
    hipLaunchKernelGGL(k_kmv_rows, dim3(grid_rows), dim3(kKmvThreads), 0, s, a, T, seed, light,
                       heavy, cnt);
    hipLaunchKernelGGL(k_kmv_pass<0>, dim3(grid_items), dim3(kKmvThreads), 0, s, a, b, T, seed,
                       (uint64_t)0, set, (const int32_t*)light, (const int2*)heavy, cnt);
    SSP_LAUNCHED(h);
    KmvCounters hc;
    SSP_HIP(h, hipMemcpyAsync(&hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
    SSP_HIP(h, hipStreamSynchronize(s));
    ssp_kmv_result r;
    std::memset(&r, 0, sizeof(r));
    r.rows_kept = hc.rows;
    r.cols_kept = hc.cols;
    r.products = hc.products;
    r.k = k;
    const uint64_t all = 1ull << 53;
    uint64_t tau = 0;
    uint32_t d = 0;
    uint64_t kth = 0;
    if (hc.products > 0) {
        const unsigned __int128 want = ((unsigned __int128)4 * k) << 53;
        tau = (uint64_t)std::min<unsigned __int128>(all, (want + hc.products - 1) / hc.products);
        tau = std::max<uint64_t>(tau, 1);
        int iter = 0;
        for (;; ++iter) {
            if (iter == 64) {
                h->last_error = "sketch threshold did not settle";
                return SSP_ERR_HIP;
            }
            // (the set and the insert counters; the item lists and their sizes stay)
            hipLaunchKernelGGL(k_num_zero, dim3(grid_set), dim3(256), 0, s, (uint64_t*)h->ws,
                               (int64_t)(set_bytes / sizeof(uint64_t)));
            hipLaunchKernelGGL(k_kmv_reset, dim3(1), dim3(64), 0, s, cnt);
            hipLaunchKernelGGL(k_kmv_pass<1>, dim3(grid_items), dim3(kKmvThreads), 0, s, a, b, T, seed,
                               tau, set, (const int32_t*)light, (const int2*)heavy, cnt);
            SSP_LAUNCHED(h);
            SSP_HIP(h, hipMemcpyAsync(&hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
            SSP_HIP(h, hipStreamSynchronize(s));
            d = hc.distinct;
            if (hc.overflow || d > kKmvMaxKept) {
                tau = std::max<uint64_t>(1, tau / 2);
                continue;
            }
            if (d < k && tau < all) {
                tau = std::min<uint64_t>(all, tau * 4);
                continue;
            }
            break;
        }
        if (d >= k) {
            hipLaunchKernelGGL(k_kmv_select, dim3(1), dim3(1024), kKmvMaxKept * sizeof(uint64_t), s,
                               (const uint64_t*)set, k, cnt);
            SSP_LAUNCHED(h);
            SSP_HIP(h, hipMemcpyAsync(&hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
            SSP_HIP(h, hipStreamSynchronize(s));
            kth = hc.kth;
        }
    }
    r.distinct_kept = d;
    r.kth_hash = kth;
    r.threshold = tau;
    // the estimates (Sec. III): k / v, then / (p_r p_c) with the realised proportions
    const double zs = (d >= k && kth > 0) ? (double)k / ((double)kth / 9007199254740992.0) : (double)d;
    r.nnz_sample = zs;
    r.nnz_estimate = (r.rows_kept == 0 || r.cols_kept == 0)
                         ? -1.0
                         : zs / (((double)r.rows_kept / (double)M) * ((double)r.cols_kept / (double)N));
    *out = r;
    return SSP_OK;
}

} // namespace

extern "C" {

ssp_status ssp_kmv_estimate(ssp_handle h, const ssp_csr* A, const ssp_csr* B, double sample_rate,
                            uint32_t k, uint64_t seed, ssp_kmv_result* out, void* stream)
{
    if (!h || !out) return SSP_ERR_INVALID_ARG;
    const ssp_status st = check_pair(A, B);
    if (st != SSP_OK) return st;
    if (!(sample_rate >= 0.0 && sample_rate <= 1.0) || k == 0 || k > kKmvKMax)
        return SSP_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return kmv_estimate(h, A, B, sample_rate, k, seed, out, static_cast<hipStream_t>(stream));
}

} // extern "C"
