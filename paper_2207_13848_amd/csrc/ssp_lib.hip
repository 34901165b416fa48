// C-ABI of the structure-prediction library (declared in include/ssp.h):
// handle and workspace management, host-side argument checks and the launch
// sequences of the prediction, reference and exact paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "ssp_kernels.hpp"

using namespace ssp;

namespace {
enum Phase {
    PH_SAMPLE = 0,
    PH_SYM_BINS,
    PH_SYM_LONG,
    PH_SYM_MERGE,
    PH_FINALIZE,
    PH_TILES,
    PH_FLOP,
    PH_FLOP_FIXUP,
    PH_REF_ROWS,
    PH_PRED_ROWS,
    PH_COUNT
};
const char* const kPhaseNames[PH_COUNT] = {"sample_bin", "sym_bins",   "sym_long", "sym_merge",
                                           "finalize",   "tiles",      "flop",     "flop_fixup",
                                           "ref_rows",   "pred_rows"};
struct EventPair {
    int phase;
    hipEvent_t a, b;
};
} // namespace

struct ssp_context {
    int device = 0;
    size_t budget = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int num_cus = 256;
    std::string last_error;
    // per-phase timing (off unless enabled)
    bool timing = false;
    std::vector<EventPair> pending;
    std::vector<hipEvent_t> event_pool;
};

namespace {

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev_ >= 0) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = -1;
    bool ok_ = true;
};

ssp_status hip_fail(ssp_handle h, hipError_t e, const char* what)
{
    if (h) {
        h->last_error = std::string(what) + ": " + hipGetErrorString(e);
    }
    return SSP_ERR_HIP;
}

#define SSP_HIP(h, call)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call);                                 \
    } while (0)

#define SSP_LAUNCHED(h)                                                                        \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess) return hip_fail((h), e_, "kernel launch");                       \
    } while (0)

hipEvent_t take_event(ssp_handle h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches made while it lives with two events on `s`.
class PhaseTimer {
  public:
    PhaseTimer(ssp_handle h, int phase, hipStream_t s) : h_(h), s_(s)
    {
        if (!h->timing) return;
        p_.phase = phase;
        p_.a = take_event(h);
        p_.b = take_event(h);
        if (p_.a && p_.b) (void)hipEventRecord(p_.a, s);
    }
    ~PhaseTimer() { stop(); }
    void stop()
    {
        if (!h_->timing || !p_.a || !p_.b) return;
        (void)hipEventRecord(p_.b, s_);
        h_->pending.push_back(p_);
        p_.a = p_.b = nullptr;
    }

  private:
    ssp_handle h_;
    hipStream_t s_;
    EventPair p_{0, nullptr, nullptr};
};

ssp_status check_csr(const ssp_csr* m)
{
    if (!m) return SSP_ERR_INVALID_ARG;
    if (m->nrows < 0 || m->ncols < 0 || m->nnz < 0) return SSP_ERR_INVALID_ARG;
    if (m->nrows >= INT32_MAX || m->ncols > INT32_MAX || m->nnz > INT32_MAX) return SSP_ERR_OVERFLOW;
    if (!m->rpt) return SSP_ERR_INVALID_ARG;
    if (m->nnz > 0 && !m->col) return SSP_ERR_INVALID_ARG;
    return SSP_OK;
}

ssp_status check_pair(const ssp_csr* A, const ssp_csr* B)
{
    ssp_status s = check_csr(A);
    if (s != SSP_OK) return s;
    s = check_csr(B);
    if (s != SSP_OK) return s;
    if (A->ncols != B->nrows) return SSP_ERR_DIM_MISMATCH;
    return SSP_OK;
}

Csr to_csr(const ssp_csr* m)
{
    Csr c;
    c.rpt = m->rpt;
    c.col = m->col;
    c.nrows = m->nrows;
    c.ncols = m->ncols;
    c.nnz = m->nnz;
    return c;
}

uint64_t rate_threshold(double rate)
{
    if (!(rate > 0.0)) return 0;
    if (rate >= 1.0) return 1ull << 53;
    return (uint64_t)(rate * 9007199254740992.0);
}

int64_t paper_sample_num(int64_t M)
{
    const int64_t s = (int64_t)(0.003 * (double)M);
    return s < 300 ? s : 300;
}

// Grow the workspace to `bytes` (hipMalloc; freed buffers are released
// after the device is idle).
ssp_status ensure_workspace(ssp_handle h, size_t bytes)
{
    if (bytes <= h->ws_bytes) return SSP_OK;
    if (h->budget && bytes > h->budget) {
        h->last_error = "workspace of " + std::to_string(bytes) + " bytes exceeds the budget of " +
                        std::to_string(h->budget);
        return SSP_ERR_BUDGET;
    }
    size_t want = bytes + bytes / 4;
    if (h->budget && want > h->budget) want = bytes;
    if (h->ws) {
        SSP_HIP(h, hipDeviceSynchronize());
        SSP_HIP(h, hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->last_error = std::string("hipMalloc: ") + hipGetErrorString(e);
        return SSP_ERR_OOM;
    }
    h->ws = p;
    h->ws_bytes = want;
    return SSP_OK;
}

struct Bound {
    Ctl* ctl;
    BinLists L;
    int32_t* tile_row;
    TileMeta* meta;
    SampleCounts* samp;
    int64_t* rowtmp;
};

// Columns per bitmap window of the long-row kernel: all N columns when they
// fit the LDS window, else 2^20-column windows.
void window_shape(int64_t N, int32_t* words, int32_t* nwin)
{
    const int64_t need = (N + 31) / 32;
    if (need <= kWinWords) {
        *words = (int32_t)std::max<int64_t>((need + 3) / 4 * 4, 4);  // whole 16-byte groups
        *nwin = 1;
    } else {
        *words = kWinWords;
        *nwin = (int32_t)((N + (int64_t)kWinWords * 32 - 1) / ((int64_t)kWinWords * 32));
    }
}

Bound bind(ssp_handle h, const Layout& L, int64_t N)
{
    char* base = static_cast<char*>(h->ws);
    Bound b;
    b.ctl = reinterpret_cast<Ctl*>(base + L.ctl);
    b.L.b1 = reinterpret_cast<BinItem*>(base + L.bin1);
    b.L.b2 = reinterpret_cast<BinItem*>(base + L.bin2);
    b.L.b3 = reinterpret_cast<BinItem*>(base + L.bin3);
    b.L.b4 = reinterpret_cast<BigItem*>(base + L.bin4);
    b.L.merge = reinterpret_cast<MergeItem*>(base + L.merge);
    b.L.scratch = reinterpret_cast<uint32_t*>(base + L.scratch);
    window_shape(N, &b.L.win_words, &b.L.nwin);
    // bin 3 would hash (its table as a bitmap covers fewer than N columns) while
    // one bitmap window covers all N: those rows go to the long-row kernel
    b.L.big3 = (b.L.nwin == 1 && N > 32LL * kBin3Words) ? 1 : 0;
    int32_t mpr = 0;  // merge items of a split row: slices of every window
    for (int32_t w = 0; w < b.L.nwin; ++w) {
        const int64_t cols = std::min<int64_t>(N - (int64_t)w * b.L.win_words * 32,
                                               (int64_t)b.L.win_words * 32);
        mpr += (int32_t)(((cols + 31) / 32 + kMergeSlice - 1) / kMergeSlice);
    }
    b.L.merge_per_row = mpr;
    b.tile_row = reinterpret_cast<int32_t*>(base + L.tiles);
    b.meta = reinterpret_cast<TileMeta*>(base + L.meta);
    b.samp = reinterpret_cast<SampleCounts*>(base + L.samp);
    b.rowtmp = reinterpret_cast<int64_t*>(base + L.rowtmp);
    return b;
}

unsigned grid_for(int64_t items, int64_t cap)
{
    if (items < 1) items = 1;
    return (unsigned)std::min<int64_t>(items, cap);
}

// Workgroups of `kernel` that fit on the device at once (static LDS only),
// cached per kernel address.
template <typename K>
int64_t resident(K kernel, int threads, int cus)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    const void* key = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1)
            n = 1;
        it = cache.emplace(key, n).first;
    }
    return (int64_t)it->second * cus;
}

template <int MODE>
void launch_flop(ssp_handle h, const FlopArgs& fa, bool vec, hipStream_t s)
{
    const int cus = h->num_cus;
    // persistent: as many workgroups as can be resident at once, each walks
    // its tiles (grid-stride)
    static int resident[2] = {0, 0};
    int& r = resident[vec ? 1 : 0];
    if (r == 0) {
        int per_cu = 0;
        const hipError_t e =
            vec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_flop<MODE, true>,
                                                               kFlopThreads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_flop<MODE, false>,
                                                               kFlopThreads, 0);
        r = (e == hipSuccess && per_cu > 0) ? per_cu : 4;
    }
    const unsigned grid =
        (unsigned)std::max<int64_t>(std::min<int64_t>(fa.ntiles, (int64_t)r * cus), 1);
    if (fa.ntiles > 0) {
        PhaseTimer pt(h, PH_FLOP, s);
        if (vec) hipLaunchKernelGGL((k_flop<MODE, true>), dim3(grid), dim3(kFlopThreads), 0, s, fa);
        else hipLaunchKernelGGL((k_flop<MODE, false>), dim3(grid), dim3(kFlopThreads), 0, s, fa);
    }
    PhaseTimer pt(h, PH_FLOP_FIXUP, s);
    const unsigned fgrid = (unsigned)std::max<int64_t>((fa.ntiles + 255) / 256, 1);
    hipLaunchKernelGGL((k_flop_fixup<MODE>), dim3(fgrid), dim3(256), 0, s, fa);
}

// Symbolic kernels over the four bins and the merge of split rows (sizes of
// the lists are device-side; the grids are upper bounds and every kernel
// walks its list grid-stride).
template <int MODE>
ssp_status launch_symbolic(ssp_handle h, const Csr& A, const Csr& B, const Bound& b,
                           const Layout& L, ssp_stats* st, int64_t* out, hipStream_t s)
{
    const int cus = h->num_cus;
    const int64_t nitems = L.cap13;
    PhaseTimer pt_bins(h, PH_SYM_BINS, s);
    // bins 1..3: a grid of the resident capacity (rows are walked grid-stride;
    // more rows in flight hide the latency of each row's chain of loads)
    hipLaunchKernelGGL((k_sym<kBin1Team, kBin1Words, MODE>),
                       dim3(grid_for(nitems, resident(k_sym<kBin1Team, kBin1Words, MODE>, kBin1Team, cus))),
                       dim3(kBin1Team), 0, s, A, B, b.L.b1, &b.ctl->bin_cnt[1], b.ctl->zacc, out);
    hipLaunchKernelGGL((k_sym<kBin2Team, kBin2Words, MODE>),
                       dim3(grid_for(nitems, resident(k_sym<kBin2Team, kBin2Words, MODE>, kBin2Team, cus))),
                       dim3(kBin2Team), 0, s, A, B, b.L.b2, &b.ctl->bin_cnt[2], b.ctl->zacc, out);
    hipLaunchKernelGGL((k_sym<kBin3Team, kBin3Words, MODE>),
                       dim3(grid_for(nitems, resident(k_sym<kBin3Team, kBin3Words, MODE>, kBin3Team, cus))),
                       dim3(kBin3Team), 0, s, A, B, b.L.b3, &b.ctl->bin_cnt[3], b.ctl->zacc, out);
    pt_bins.stop();
    const size_t lds = (size_t)b.L.win_words * sizeof(uint32_t);
    // one window holding all N columns: the kernel skips the window tests
    const bool win1 = b.L.nwin == 1;
    static bool attr_set[2][2] = {{false, false}, {false, false}};
    static int big_resident[2][2] = {{0, 0}, {0, 0}};
    auto kfun = win1 ? k_sym_big<MODE, true> : k_sym_big<MODE, false>;
    if (!attr_set[MODE][win1]) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kfun),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(kWinWords * sizeof(uint32_t)));
        attr_set[MODE][win1] = true;
    }
    if (big_resident[MODE][win1] == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfun, kBin4Team,
                                                         kWinWords * sizeof(uint32_t)) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        big_resident[MODE][win1] = per_cu;
    }
    {
        PhaseTimer pt(h, PH_SYM_LONG, s);
        hipLaunchKernelGGL(kfun, dim3(grid_for(L.cap4, (int64_t)big_resident[MODE][win1] * cus)),
                           dim3(kBin4Team), lds, s, A, B, b.L.b4, &b.ctl->bin_cnt[4],
                           &b.ctl->big_next, b.L, b.ctl->zacc, out);
    }
    {
        PhaseTimer pt(h, PH_SYM_MERGE, s);
        hipLaunchKernelGGL((k_sym_merge<MODE>), dim3((unsigned)(2 * cus)), dim3(256), 0, s,
                           b.L.merge, &b.ctl->bin_cnt[5], b.L, B.ncols, b.ctl->zacc, out);
    }
    PhaseTimer pt_fin(h, PH_FINALIZE, s);
    hipLaunchKernelGGL((k_finalize<MODE>), dim3(1), dim3(kAccSlots), 0, s, b.ctl, st);
    SSP_LAUNCHED(h);
    return SSP_OK;
}

FlopArgs flop_args(const ssp_csr* A, const ssp_csr* B, const Bound& b, const Layout& L,
                   int64_t* out, ssp_stats* st)
{
    FlopArgs fa;
    fa.A = to_csr(A);
    fa.B = to_csr(B);
    fa.out = out;
    fa.st = st;
    fa.ctl = b.ctl;
    fa.L = b.L;
    fa.tile_row = b.tile_row;
    fa.meta = b.meta;
    fa.ntiles = L.ntiles;
    return fa;
}

// Merge-path tile starts and the streaming pass that leaves every row's
// product count in rf and F in st (mode FLOP_ONLY), or bins every row for the
// exact count (FLOP_EXACT_BIN).
template <int MODE>
ssp_status flop_pass(ssp_handle h, const ssp_csr* A, const ssp_csr* B, const Bound& b,
                     const Layout& L, int64_t* out, ssp_stats* st, hipStream_t s)
{
    const int64_t M = A->nrows;
    {
        PhaseTimer pt(h, PH_TILES, s);
        hipLaunchKernelGGL(k_tiles, dim3(grid_for((M + 255) / 256, 16LL * h->num_cus)), dim3(256),
                           0, s, to_csr(A), L.ntiles, b.tile_row);
    }
    const FlopArgs fa = flop_args(A, B, b, L, out, st);
    const bool vec = (reinterpret_cast<uintptr_t>(A->col) & 15u) == 0 && A->nnz >= 4;
    launch_flop<MODE>(h, fa, vec, s);
    SSP_LAUNCHED(h);
    return SSP_OK;
}

// The sampled part: row FLOP of every row into rf, sampling and binning,
// distinct counting of the sampled rows.  Leaves F, n_s, f*, z* in *st and
// the divisor of f* in ctl.
ssp_status sampled_part(ssp_handle h, const ssp_csr* A, const ssp_csr* B, ssp_sampler sampler,
                        double rate, uint64_t seed, const Bound& b, const Layout& L,
                        int64_t* rf, ssp_stats* st, hipStream_t s)
{
    ssp_status e = flop_pass<FLOP_ONLY>(h, A, B, b, L, rf, st, s);
    if (e != SSP_OK) return e;
    const Csr a = to_csr(A), bb = to_csr(B);
    const int64_t M = A->nrows;
    {
        PhaseTimer pt(h, PH_SAMPLE, s);
        const bool paper = sampler == SSP_SAMPLER_PAPER;
        const int64_t nc = paper ? paper_sample_num(M) : M;
        const uint64_t thr = paper ? 0 : rate_threshold(rate);
        // count, scan, write: per-group counters instead of device atomics
        const unsigned grid = grid_for((nc + 2047) / 2048, kSampleGroups);
        const int64_t* rfc = rf;
        if (paper)
            hipLaunchKernelGGL((k_sample_count<true>), dim3(grid), dim3(kSampleThreads), 0, s, a,
                               rfc, seed, thr, nc, b.L, b.samp);
        else
            hipLaunchKernelGGL((k_sample_count<false>), dim3(grid), dim3(kSampleThreads), 0, s, a,
                               rfc, seed, thr, nc, b.L, b.samp);
        hipLaunchKernelGGL(k_sample_scan, dim3(1), dim3(kScanThreads), 0, s, b.samp, (int)grid,
                           b.ctl, st);
        if (paper)
            hipLaunchKernelGGL((k_sample_write<true>), dim3(grid), dim3(kSampleThreads), 0, s, a,
                               rfc, seed, thr, nc, B->ncols, (const SampleCounts*)b.samp, b.L);
        else
            hipLaunchKernelGGL((k_sample_write<false>), dim3(grid), dim3(kSampleThreads), 0, s, a,
                               rfc, seed, thr, nc, B->ncols, (const SampleCounts*)b.samp, b.L);
    }
    SSP_LAUNCHED(h);
    return launch_symbolic<0>(h, a, bb, b, L, st, nullptr, s);
}

// Few large workgroups for the per-row outputs: each adds its part of the
// output total with one same-address atomic.
unsigned rows_grid(ssp_handle h, int64_t M)
{
    return grid_for((M + 4 * kRowsThreads - 1) / (4 * kRowsThreads), h->num_cus / 2);
}

ssp_status common_checks(ssp_handle h, const ssp_csr* A, const ssp_csr* B, ssp_sampler sampler,
                         double rate, const void* out)
{
    if (!h) return SSP_ERR_INVALID_ARG;
    const ssp_status s = check_pair(A, B);
    if (s != SSP_OK) return s;
    if (sampler != SSP_SAMPLER_BERNOULLI && sampler != SSP_SAMPLER_PAPER) return SSP_ERR_INVALID_ARG;
    if (sampler == SSP_SAMPLER_BERNOULLI && !(rate >= 0.0 && rate <= 1.0)) return SSP_ERR_INVALID_ARG;
    if (A->nrows > 0 && !out) return SSP_ERR_INVALID_ARG;
    return SSP_OK;
}

} // namespace

// ===================================================================== ABI

extern "C" {

const char* ssp_version(void) { return "ssp 0.1.0 (gfx950)"; }

const char* ssp_status_string(ssp_status s)
{
    switch (s) {
    case SSP_OK: return "ok";
    case SSP_ERR_INVALID_ARG: return "invalid argument";
    case SSP_ERR_DIM_MISMATCH: return "A.ncols != B.nrows";
    case SSP_ERR_OVERFLOW: return "size does not fit the int32 CSR format";
    case SSP_ERR_BUDGET: return "workspace exceeds the HBM budget";
    case SSP_ERR_OOM: return "device allocation failed";
    case SSP_ERR_HIP: return "HIP runtime error";
    case SSP_ERR_NO_DEVICE: return "no usable device";
    case SSP_ERR_INVALID_CSR: return "invalid CSR";
    case SSP_ERR_BUSY: return "resource busy";
    case SSP_ERR_NOT_READY: return "not ready";
    }
    return "unknown status";
}

const char* ssp_last_error(ssp_handle h) { return h ? h->last_error.c_str() : ""; }

ssp_status ssp_create(ssp_handle* out, int device, size_t hbm_budget_bytes)
{
    if (!out) return SSP_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return SSP_ERR_NO_DEVICE;
    }
    ssp_context* h = new (std::nothrow) ssp_context();
    if (!h) return SSP_ERR_OOM;
    h->device = device;
    h->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        h->num_cus = prop.multiProcessorCount;
    *out = h;
    return SSP_OK;
}

ssp_status ssp_destroy(ssp_handle h)
{
    if (!h) return SSP_ERR_INVALID_ARG;
    ssp_status st = SSP_OK;
    DeviceGuard g(h->device);
    if (h->ws) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(h->ws) != hipSuccess) st = SSP_ERR_HIP;
    }
    for (auto& p : h->pending) {
        h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    delete h;
    return st;
}

ssp_status ssp_timing_enable(ssp_handle h, int enable)
{
    if (!h) return SSP_ERR_INVALID_ARG;
    h->timing = enable != 0;
    return SSP_OK;
}

int ssp_timing_read(ssp_handle h, ssp_phase_time* out, int max)
{
    if (!h || (max > 0 && !out)) return -1;
    DeviceGuard g(h->device);
    uint64_t n[PH_COUNT] = {0};
    double ms[PH_COUNT] = {0};
    for (auto& p : h->pending) {
        float t = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            n[p.phase] += 1;
            ms[p.phase] += (double)t;
        }
        h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    h->pending.clear();
    int k = 0;
    for (int ph = 0; ph < PH_COUNT && k < max; ++ph) {
        if (!n[ph]) continue;
        std::memset(&out[k], 0, sizeof(out[k]));
        std::strncpy(out[k].name, kPhaseNames[ph], sizeof(out[k].name) - 1);
        out[k].launches = n[ph];
        out[k].total_ms = ms[ph];
        ++k;
    }
    return k;
}

size_t ssp_workspace_bytes(ssp_handle h) { return h ? h->ws_bytes : 0; }

ssp_status ssp_predict_structure_ex(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                    ssp_sampler sampler, double rate, uint64_t seed,
                                    int64_t* nnz_pred, int64_t* row_flop, ssp_stats* stats,
                                    void* stream)
{
    ssp_status s = common_checks(h, A, B, sampler, rate, nnz_pred);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    const int64_t M = A->nrows;
    const int64_t nitems = sampler == SSP_SAMPLER_PAPER ? paper_sample_num(M) : M;
    const Layout L = make_layout(nitems, M, A->nnz, row_flop == nullptr);
    if ((s = ensure_workspace(h, L.total)) != SSP_OK) return s;
    const Bound b = bind(h, L, B->ncols);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    ssp_stats* st = stats ? stats : &b.ctl->stats;
    int64_t* rf = row_flop ? row_flop : b.rowtmp;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, hs, b.ctl, st, (uint64_t)M);
    SSP_LAUNCHED(h);
    if (M == 0) return SSP_OK;
    if ((s = sampled_part(h, A, B, sampler, rate, seed, b, L, rf, st, hs)) != SSP_OK) return s;
    {
        PhaseTimer pt(h, PH_PRED_ROWS, hs);
        hipLaunchKernelGGL(k_pred_rows, dim3(rows_grid(h, M)), dim3(kRowsThreads), 0, hs,
                           (const int64_t*)rf, nnz_pred, M, b.ctl, st);
    }
    SSP_LAUNCHED(h);
    return SSP_OK;
}

ssp_status ssp_predict_structure(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                 double sample_rate, uint64_t seed, int64_t* nnz_pred,
                                 int64_t* row_flop, ssp_stats* stats, void* stream)
{
    return ssp_predict_structure_ex(h, A, B, SSP_SAMPLER_BERNOULLI, sample_rate, seed, nnz_pred,
                                    row_flop, stats, stream);
}

ssp_status ssp_reference_estimate(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                  ssp_sampler sampler, double rate, uint64_t seed,
                                  int64_t* nnz_ref, ssp_stats* stats, void* stream)
{
    ssp_status s = common_checks(h, A, B, sampler, rate, nnz_ref);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    const int64_t M = A->nrows;
    const int64_t nitems = sampler == SSP_SAMPLER_PAPER ? paper_sample_num(M) : M;
    const Layout L = make_layout(nitems, M, A->nnz, true);
    if ((s = ensure_workspace(h, L.total)) != SSP_OK) return s;
    const Bound b = bind(h, L, B->ncols);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    ssp_stats* st = stats ? stats : &b.ctl->stats;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, hs, b.ctl, st, (uint64_t)M);
    SSP_LAUNCHED(h);
    if (M == 0) return SSP_OK;
    if ((s = sampled_part(h, A, B, sampler, rate, seed, b, L, b.rowtmp, st, hs)) != SSP_OK)
        return s;
    {
        PhaseTimer pt(h, PH_FINALIZE, hs);
        hipLaunchKernelGGL(k_finalize_reference, dim3(1), dim3(64), 0, hs, b.ctl, st,
                           (uint64_t)M);
    }
    {
        PhaseTimer pt(h, PH_REF_ROWS, hs);
        hipLaunchKernelGGL(k_ref_rows, dim3(rows_grid(h, M)), dim3(kRowsThreads), 0, hs,
                           (const int64_t*)b.rowtmp, nnz_ref, M, b.ctl, st);
    }
    SSP_LAUNCHED(h);
    return SSP_OK;
}

ssp_status ssp_exact_structure(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                               int64_t* nnz_exact, ssp_stats* stats, void* stream)
{
    ssp_status s = common_checks(h, A, B, SSP_SAMPLER_BERNOULLI, 0.0, nnz_exact);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    const int64_t M = A->nrows;
    const Layout L = make_layout(M, M, A->nnz, false);
    if ((s = ensure_workspace(h, L.total)) != SSP_OK) return s;
    const Bound b = bind(h, L, B->ncols);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    ssp_stats* st = stats ? stats : &b.ctl->stats;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, hs, b.ctl, st, (uint64_t)M);
    SSP_LAUNCHED(h);
    if (M == 0) return SSP_OK;
    if ((s = flop_pass<FLOP_EXACT_BIN>(h, A, B, b, L, nnz_exact, st, hs)) != SSP_OK) return s;
    if ((s = launch_symbolic<1>(h, to_csr(A), to_csr(B), b, L, st, nnz_exact, hs)) != SSP_OK)
        return s;
    return SSP_OK;
}

ssp_status ssp_validate_csr(ssp_handle h, const ssp_csr* m, int64_t* n_bad, void* stream)
{
    if (!h || !n_bad) return SSP_ERR_INVALID_ARG;
    const ssp_status s = check_csr(m);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, hs, n_bad);
    const int64_t work = std::max<int64_t>(m->nrows + 1, m->nnz);
    const unsigned grid = (unsigned)std::min<int64_t>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(k_validate, dim3(std::max(grid, 1u)), dim3(256), 0, hs, to_csr(m), n_bad);
    SSP_LAUNCHED(h);
    return SSP_OK;
}

} // extern "C"
