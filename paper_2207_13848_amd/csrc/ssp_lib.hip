// C-ABI of the structure-prediction library (declared in include/ssp.h):
// handle and workspace management, host-side argument checks and the launch
// sequences of the prediction, reference and exact paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "ssp_numeric.hpp"

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
    PH_NUM_SCAN,
    PH_NUM_HASH,
    PH_NUM_DENSE,
    PH_NUM_COPY,
    PH_NUM_FALLBACK,
    PH_COUNT
};
const char* const kPhaseNames[PH_COUNT] = {"sample_bin", "sym_bins",   "sym_long",  "sym_merge",
                                           "finalize",   "tiles",      "flop",      "flop_fixup",
                                           "ref_rows",   "pred_rows",  "num_scan",  "num_hash",
                                           "num_dense",  "num_copy",   "num_fallback"};
struct EventPair {
    int phase;
    hipEvent_t a, b;
};
} // namespace

namespace {
ssp_tuning default_tuning()
{
    ssp_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.bin_max[0] = (uint32_t)ssp::kBin1Max;
    t.bin_max[1] = (uint32_t)ssp::kBin2Max;
    t.bin_max[2] = (uint32_t)ssp::kBin3Max;
    t.hash_mult = 2;
    t.long_len = ssp::kLongLenDefault;
    t.big3 = 1;
    t.split_target = ssp::kSplitTarget;
    t.est_max_rf = ssp::kEstMaxA;
    return t;
}

// The limits the kernels rely on: a bin's hash table holds hash_mult x its
// limit, a long B row has a whole 16-byte group, short products of a chunk
// fit a 20-bit field.
bool tuning_valid(const ssp_tuning& t)
{
    const uint32_t m = t.hash_mult;
    if (m != 2 && m != 4 && m != 8) return false;
    if (t.bin_max[0] < 1 || t.bin_max[0] > t.bin_max[1] || t.bin_max[1] > t.bin_max[2]) return false;
    if ((uint64_t)t.bin_max[0] * m > (uint64_t)ssp::kBin1Words ||
        (uint64_t)t.bin_max[1] * m > (uint64_t)ssp::kBin2Words ||
        (uint64_t)t.bin_max[2] * m > (uint64_t)ssp::kBin3Words)
        return false;
    if (t.long_len < 8 || t.long_len > 1024) return false;
    if (t.big3 != 0 && t.big3 != 1) return false;
    if (t.split_target < (1ull << 12) || t.split_target > (1ull << 40)) return false;
    if (t.est_max_rf > ssp::kEstMaxA) return false;
    return true;
}
} // namespace

struct ssp_context {
    ssp_tuning tuning = default_tuning();
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
    // pinned staging of batch case tables
    void* pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t pin_ev = nullptr;
    // numeric product: buffers of its own (other calls leave them alone
    // between ssp_spgemm_compute and ssp_spgemm_copy) and the state the copy
    // call reads; the dense accumulators are all zero between calls
    void* num_ws = nullptr;
    size_t num_ws_bytes = 0;
    void* num_slots = nullptr;
    size_t num_slots_bytes = 0;
    void* num_pool = nullptr;
    size_t num_pool_bytes = 0;
    bool num_pool_clean = false;
    hipEvent_t num_ev = nullptr;  // end of the last copy pass
    std::shared_ptr<void> num_state;
};

// A captured batch: its own workspace and case table, and the launch graph.
struct ssp_batch_graph_s {
    ssp_handle h = nullptr;
    int device = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int n = 0;
};

// Scratch of ssp_predict_structure_noalloc: its whole workspace, one copy per
// device, held from the library's load until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress gives for each
// device (noalloc_base); the array's name is not a device address on the
// host.
constexpr size_t kNoAllocBytes = 256ull << 20;
constexpr int64_t kNoAllocMinWindows = 16;  // part windows it may shrink to
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// The scratch array's device address per device, taken once per device with
// that device current (at ssp_create).
constexpr int kNoAllocDevices = 64;
struct NoAllocSlot {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
NoAllocSlot g_noalloc[kNoAllocDevices];

void noalloc_init(int device)
{
    if (device < 0 || device >= kNoAllocDevices) return;
    NoAllocSlot& s = g_noalloc[device];
    std::call_once(s.once, [&s] {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && p) {
            s.ptr = p;
        } else {
            (void)hipGetLastError();
            s.err = e == hipSuccess ? hipErrorInvalidSymbol : e;
        }
    });
}

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
    PhaseTimer(ssp_handle h, int phase, hipStream_t s, bool enabled = true) : h_(h), s_(s)
    {
        if (!h->timing || !enabled) return;
        p_.phase = phase;
        p_.a = take_event(h);
        p_.b = take_event(h);
        if (p_.a && p_.b) (void)hipEventRecord(p_.a, s);
    }
    ~PhaseTimer() { stop(); }
    void stop()
    {
        if (!p_.a || !p_.b) return;
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
    c.rpt = (decltype(c.rpt))m->rpt;
    c.col = (decltype(c.col))m->col;
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

// ------------------------------------------------------------- planning

// One case of a call as the host sees it.
struct CaseIn {
    Csr A, B;
    int sampler;     // ssp_sampler
    double rate;
    uint64_t seed;
    int64_t* out;
    int64_t* rf;     // the caller's row-FLOP array, or null (workspace)
    ssp_stats* st;   // the caller's stats, or null (workspace)
};

enum PlanKind { PLAN_PREDICT, PLAN_REFERENCE, PLAN_EXACT };

// Everything the launches of a call need: the case table (device pointers
// into the workspace resolved by bind_plan), grid sizes and the workspace
// layout.
struct Plan {
    PlanKind kind = PLAN_PREDICT;
    int n = 0;
    std::vector<CaseDesc> cs;
    std::vector<int64_t> rf_off;   // workspace row-FLOP offset per case, -1 = caller's
    std::vector<int64_t> blen_off; // workspace byte offset of B's row lengths per case (vec)
    std::vector<int> st_slot;      // workspace stats slot per case, -1 = caller's
    int64_t cap13 = 1, cap4 = 1, cap5 = 1, ngroups = 0, tiles = 0, rowtmp = 0;
    int64_t part_windows = kPartWindowsBase;  // scratch windows for the parts of split rows
    int32_t g_tiles = 0, g_flop = 0, g_fixup = 0, g_rows = 0;
    int32_t win_words_max = 4;
    bool win1 = true, vec = true;
    bool bin2_wave = false;  // bin 2 one wave per row (many sampled rows expected)
    size_t o_ctl = 0, o_scratch = 0, o_b1 = 0, o_b2 = 0, o_b3 = 0, o_b4 = 0, o_merge = 0,
           o_tiles = 0, o_tcase = 0, o_meta = 0, o_samp = 0, o_cases = 0, o_res = 0, o_stats = 0,
           o_rowtmp = 0, o_blen = 0, total = 0;
};

// Columns per bitmap window of the long-row kernel: all N columns when they
// fit the LDS window, else 2^20-column windows.
void window_shape(int64_t N, int32_t* words, int32_t* nwin)
{
    const int64_t need = bitmap_words(N);
    if (need <= kWinWords) {
        *words = (int32_t)std::max<int64_t>(need, 64);  // whole 64-word rows
        *nwin = 1;
    } else {
        *words = kWinWords;
        *nwin = (int32_t)((N + (int64_t)kWinWords * 32 - 1) / ((int64_t)kWinWords * 32));
    }
}

unsigned grid_for(int64_t items, int64_t cap)
{
    if (items < 1) items = 1;
    return (unsigned)std::min<int64_t>(items, cap);
}

// Workgroups of `kernel` that fit on the device at once (static LDS only),
// cached per kernel address.
template <typename K>
int64_t resident(K kernel, int threads, int cus, size_t dyn_lds = 0)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    const void* key = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        int k = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, kernel, threads, dyn_lds) != hipSuccess ||
            k < 1)
            k = 1;
        it = cache.emplace(key, k).first;
    }
    return (int64_t)it->second * cus;
}

// Per-case workgroup counts proportional to work, at least 1 for a case with
// work, at most `cap_c` (the case's useful maximum); returns the prefixes.
template <typename W, typename Cap>
int32_t share_wgs(int n, int64_t budget, W work, Cap cap_c, std::vector<int32_t>& first)
{
    int64_t total = 0;
    for (int c = 0; c < n; ++c) total += work(c);
    first.assign(n, 0);
    int64_t g = 0;
    for (int c = 0; c < n; ++c) {
        first[c] = (int32_t)g;
        const int64_t w = work(c);
        if (w <= 0) continue;
        int64_t k = total > 0 ? (int64_t)((double)budget * (double)w / (double)total + 0.5) : 1;
        k = std::max<int64_t>(1, std::min<int64_t>(k, cap_c(c)));
        g += k;
    }
    return (int32_t)g;
}

// Part windows of a plan: kPartWindowsBase per 32 cases, at most
// kPartWindowsMax (a call of one case holds 1024 windows, 128 MiB).
int64_t part_windows_for(int n)
{
    return std::min<int64_t>(kPartWindowsMax, (int64_t)kPartWindowsBase * ((n + 31) / 32));
}

Plan make_plan(ssp_handle h, const std::vector<CaseIn>& in, PlanKind kind,
               int64_t part_windows = -1)
{
    Plan P;
    P.kind = kind;
    P.n = (int)in.size();
    const int n = P.n, cus = h->num_cus;
    P.part_windows = part_windows > 0 ? part_windows : part_windows_for(std::max(n, 1));
    P.cs.assign(n, CaseDesc{});
    P.rf_off.assign(n, -1);
    P.st_slot.assign(n, -1);
    int64_t sumC = 0, exp_rows = 0;  // candidates; rows expected in the bins
    for (int c = 0; c < n; ++c) {
        CaseDesc& d = P.cs[c];
        const CaseIn& x = in[c];
        const int64_t M = x.A.nrows, nnz = x.A.nnz, N = x.B.ncols;
        d.A = x.A;
        d.B = x.B;
        d.out = (decltype(d.out))x.out;
        d.rf = (decltype(d.rf))x.rf;
        d.st = x.st;
        d.seed = x.seed;
        d.paper = x.sampler == SSP_SAMPLER_PAPER ? 1 : 0;
        d.thresh = d.paper ? 0 : rate_threshold(x.rate);
        d.ncand = (kind == PLAN_EXACT || M == 0) ? 0 : (d.paper ? paper_sample_num(M) : M);
        window_shape(N, &d.win_words, &d.nwin);
        // bin 3 would hash (its table as a bitmap covers fewer than N columns)
        // while one bitmap window covers all N: those rows go to the long-row kernel
        const ssp_tuning& tu = h->tuning;
        d.big3 = (tu.big3 && d.nwin == 1 && N > 32LL * kBin3Words) ? 1 : 0;
        d.bin_max[0] = tu.bin_max[0];
        d.bin_max[1] = tu.bin_max[1];
        d.bin_max[2] = tu.bin_max[2];
        d.hash_mult = tu.hash_mult;
        d.long_len = tu.long_len;
        // (a split part of a narrow window costs a smaller bitmap to clear, store
        // and merge: the target shrinks with the window, at least 2^12 products)
        d.split_target = std::max<uint64_t>(
            1ull << 12, tu.split_target / (uint64_t)(kWinWords / std::max<int32_t>(d.win_words, 64)));
        d.est_max_rf = tu.est_max_rf;
        int32_t mpr = 0;  // merge items of a split row: slices of every window
        for (int32_t w = 0; w < d.nwin; ++w) {
            const int64_t cols = std::min<int64_t>(N - (int64_t)w * d.win_words * 32,
                                                   (int64_t)d.win_words * 32);
            mpr += (int32_t)((bitmap_words(cols) + kMergeSlice - 1) / kMergeSlice);
        }
        d.merge_per_row = mpr;
        d.ntiles = M > 0 ? flop_tiles(M, nnz) : 0;
        d.tile_base = P.tiles;
        P.tiles += d.ntiles;
        if (!x.rf && kind != PLAN_EXACT) {
            P.rf_off[c] = P.rowtmp;
            P.rowtmp += M;
        }
        if (!x.st) P.st_slot[c] = c;
        sumC += d.ncand;
        P.win_words_max = std::max(P.win_words_max, d.win_words);
        if (d.nwin != 1) P.win1 = false;
        // (the streaming kernel's fast form reads through buffer resources:
        // B's row pointers at 32-bit byte offsets)
        if (M > 0 && (nnz < 1 || x.B.nrows >= ((int64_t)1 << 30))) P.vec = false;
        exp_rows += kind == PLAN_EXACT ? M : (d.paper ? d.ncand : (int64_t)(x.rate * (double)M));
    }
    P.bin2_wave = exp_rows >= kBin2WaveRows;
    // sampling groups: about kSampleTarget per call, at least 2048 candidates each
    int64_t gsize = (sumC + kSampleTarget - 1) / kSampleTarget;
    gsize = std::max<int64_t>(2048, (gsize + 255) / 256 * 256);
    for (int c = 0; c < n; ++c) {
        CaseDesc& d = P.cs[c];
        d.group_size = gsize;
        d.ngroups = (d.ncand + gsize - 1) / gsize;
        d.group_base = P.ngroups;
        P.ngroups += d.ngroups;
    }
    // workgroups per case, in proportion to the work
    std::vector<int32_t> f;
    auto Mof = [&](int c) { return P.cs[c].A.nrows; };
    auto T = [&](int c) { return P.cs[c].ntiles; };
    P.g_tiles = share_wgs(n, 16LL * cus, Mof, [&](int c) { return (Mof(c) + 255) / 256; }, f);
    for (int c = 0; c < n; ++c) P.cs[c].wg_tiles = f[c];
    (void)T;
    // the streaming pass walks all tiles, case after case, with one persistent grid
    const int64_t rflop = P.vec ? resident(k_flop<FLOP_ONLY, true>, kFlopThreads, cus)
                                : resident(k_flop<FLOP_ONLY, false>, kFlopThreads, cus);
    P.g_flop = (int32_t)std::min<int64_t>(rflop, P.tiles);
    P.g_fixup = (int32_t)((P.tiles + 255) / 256);
    // (every case gets a workgroup of the row kernels, rows or not: the
    // prediction kernel also finishes the case's statistics)
    auto rows_work = [&](int c) { return std::max<int64_t>(Mof(c), 1); };
    auto rows_cap = [&](int c) {  // (at least four rows per thread)
        return std::max<int64_t>(1, (Mof(c) + 4 * kRowsThreads - 1) / (4 * kRowsThreads));
    };
    // (about 32 rows per thread over the call, at least one workgroup per CU;
    // on 2^20 and 2^21 rows, 512 or 1024 workgroups took longer than 256:
    // each adds a same-address atomic and its own chain of dependent loads)
    int64_t rows_all = 0;
    for (int c = 0; c < n; ++c) rows_all += Mof(c);
    const int64_t rows_budget = std::max<int64_t>(cus, rows_all / (4 * 8 * kRowsThreads));
    P.g_rows = share_wgs(n, rows_budget, rows_work, rows_cap, f);
    for (int c = 0; c < n; ++c) P.cs[c].wg_rows = f[c];
    // list capacities
    int64_t sumM = 0;
    for (int c = 0; c < n; ++c) sumM += P.cs[c].A.nrows;
    P.cap13 = std::max<int64_t>(1, kind == PLAN_EXACT ? sumM : sumC);
    P.cap4 = P.cap13 + P.part_windows;
    P.cap5 = (int64_t)P.part_windows * (kWinWords / kMergeSlice) + 64;
    // workspace layout
    size_t o = 0;
    P.o_ctl = o;     o = align256(o + sizeof(Ctl));
    P.o_scratch = o; o = align256(o + (size_t)P.part_windows * kWinWords * sizeof(uint32_t));
    P.o_b1 = o;      o = align256(o + (size_t)P.cap13 * sizeof(BinItem));
    P.o_b2 = o;      o = align256(o + (size_t)P.cap13 * sizeof(BinItem));
    P.o_b3 = o;      o = align256(o + (size_t)P.cap13 * sizeof(BinItem));
    P.o_b4 = o;      o = align256(o + (size_t)P.cap4 * sizeof(BigItem));
    P.o_merge = o;   o = align256(o + (size_t)P.cap5 * sizeof(MergeItem));
    P.o_tiles = o;   o = align256(o + (size_t)std::max<int64_t>(P.tiles, 1) * sizeof(int32_t));
    P.o_tcase = o;   o = align256(o + (size_t)std::max<int64_t>(P.tiles, 1) * sizeof(int32_t));
    P.o_meta = o;    o = align256(o + (size_t)std::max<int64_t>(P.tiles, 1) * sizeof(TileMeta));
    P.o_samp = o;    o = align256(o + (size_t)std::max<int64_t>(P.ngroups, 1) * sizeof(SampleCounts));
    P.o_cases = o;   o = align256(o + (size_t)n * sizeof(CaseDesc));
    P.o_res = o;     o = align256(o + (size_t)n * sizeof(CaseRes));
    P.o_stats = o;   o = align256(o + (size_t)n * sizeof(ssp_stats));
    P.o_rowtmp = o;  o = align256(o + (size_t)std::max<int64_t>(P.rowtmp, 1) * sizeof(int64_t));
    // B's row lengths, two bytes each, for the streaming kernel's fast form
    P.o_blen = o;
    P.blen_off.assign(n, -1);
    if (P.vec) {
        // (one array per distinct B: cases of one B gather from one copy)
        size_t b = 0;
        std::unordered_map<const void*, int> first;
        for (int c = 0; c < n; ++c) {
            const void* key = (const void*)P.cs[c].B.rpt;
            auto it = first.find(key);
            if (it != first.end() && P.cs[it->second].B.nrows == P.cs[c].B.nrows) {
                P.blen_off[c] = P.blen_off[it->second];
                continue;
            }
            first[key] = c;
            P.cs[c].blen_own = 1;
            P.blen_off[c] = (int64_t)b;
            b = align256(b + (size_t)P.cs[c].B.nrows * sizeof(uint16_t));
        }
        o += b;
    }
    P.total = o;
    return P;
}

// The lists index their items with 32-bit offsets: a call whose rows (the
// sampled candidates, or every row for the exact structure) and part windows
// reach 2^31 is refused.
ssp_status plan_fits_lists(ssp_handle h, const Plan& P)
{
    if (P.cap4 < (int64_t)INT32_MAX) return SSP_OK;
    h->last_error = "the call's lists would hold " + std::to_string(P.cap4) +
                    " items, beyond 32-bit offsets";
    return SSP_ERR_OVERFLOW;
}

// Device pointers of a plan in a workspace at `base`; resolves the case
// table's workspace-backed row-FLOP arrays and statistics.
struct Bound {
    Ctl* ctl;
    BinLists L;
    int32_t* tile_row;
    int32_t* tile_case;
    TileMeta* meta;
    SampleCounts* samp;
    CaseDesc* cs;
    CaseRes* cr;
};

Bound bind_plan(Plan& P, void* ws)
{
    char* base = static_cast<char*>(ws);
    Bound b;
    b.ctl = reinterpret_cast<Ctl*>(base + P.o_ctl);
    b.L.b1 = reinterpret_cast<BinItem*>(base + P.o_b1);
    b.L.b2 = reinterpret_cast<BinItem*>(base + P.o_b2);
    b.L.b3 = reinterpret_cast<BinItem*>(base + P.o_b3);
    b.L.b4 = reinterpret_cast<BigItem*>(base + P.o_b4);
    b.L.merge = reinterpret_cast<MergeItem*>(base + P.o_merge);
    b.L.scratch = reinterpret_cast<uint32_t*>(base + P.o_scratch);
    b.L.cap4 = (uint32_t)P.cap4;
    b.L.part_windows = (uint32_t)P.part_windows;
    b.tile_row = reinterpret_cast<int32_t*>(base + P.o_tiles);
    b.tile_case = reinterpret_cast<int32_t*>(base + P.o_tcase);
    b.meta = reinterpret_cast<TileMeta*>(base + P.o_meta);
    b.samp = reinterpret_cast<SampleCounts*>(base + P.o_samp);
    b.cs = reinterpret_cast<CaseDesc*>(base + P.o_cases);
    b.cr = reinterpret_cast<CaseRes*>(base + P.o_res);
    ssp_stats* stats = reinterpret_cast<ssp_stats*>(base + P.o_stats);
    int64_t* rowtmp = reinterpret_cast<int64_t*>(base + P.o_rowtmp);
    for (int c = 0; c < P.n; ++c) {
        if (P.rf_off[c] >= 0) P.cs[c].rf = (decltype(P.cs[c].rf))(rowtmp + P.rf_off[c]);
        if (P.st_slot[c] >= 0) P.cs[c].st = stats + P.st_slot[c];
        P.cs[c].blen = P.blen_off[c] >= 0
                           ? (decltype(P.cs[c].blen))(base + P.o_blen + P.blen_off[c])
                           : nullptr;
    }
    return b;
}

// ------------------------------------------------------------- launches

template <int MODE>
void launch_flop(ssp_handle h, const Plan& P, const Bound& b, hipStream_t s, bool timed)
{
    if (P.g_flop > 0) {
        PhaseTimer pt(h, PH_FLOP, s, timed);
        if (P.vec)
            hipLaunchKernelGGL((k_flop<MODE, true>), dim3(P.g_flop), dim3(kFlopThreads), 0, s, b.cs,
                               (const int32_t*)b.tile_row, (const int32_t*)b.tile_case, P.tiles,
                               b.meta, b.ctl, b.L);
        else
            hipLaunchKernelGGL((k_flop<MODE, false>), dim3(P.g_flop), dim3(kFlopThreads), 0, s,
                               b.cs, (const int32_t*)b.tile_row, (const int32_t*)b.tile_case,
                               P.tiles, b.meta, b.ctl, b.L);
    }
    PhaseTimer pt(h, PH_FLOP_FIXUP, s, timed);
    if (P.g_fixup > 0)
        hipLaunchKernelGGL((k_flop_fixup<MODE>), dim3(P.g_fixup), dim3(256), 0, s, b.cs,
                           (const int32_t*)b.tile_row, (const int32_t*)b.tile_case, P.tiles,
                           (const TileMeta*)b.meta, b.ctl, b.L);
}

void launch_sampling(ssp_handle h, const Plan& P, const Bound& b, hipStream_t s, bool timed)
{
    PhaseTimer pt(h, PH_SAMPLE, s, timed);
    if (P.ngroups == 0) return;  // (the bin counters stay 0 from k_setup)
    // count, scan, write: per-group counters instead of device atomics
    hipLaunchKernelGGL(k_sample_count, dim3((unsigned)P.ngroups), dim3(kSampleThreads), 0, s, b.cs,
                       P.n, b.samp);
    if (P.ngroups <= kFusedScanGroups) {
        hipLaunchKernelGGL(k_sample_write<true>, dim3((unsigned)P.ngroups), dim3(kSampleThreads), 0,
                           s, b.cs, P.n, b.samp, b.ctl, b.L, P.ngroups, (uint32_t)P.part_windows);
    } else {
        hipLaunchKernelGGL(k_sample_scan, dim3(1), dim3(kScanThreads), 0, s, b.samp, P.ngroups,
                           b.cs, b.ctl, (uint32_t)P.part_windows);
        hipLaunchKernelGGL(k_sample_write<false>, dim3((unsigned)P.ngroups), dim3(kSampleThreads), 0,
                           s, b.cs, P.n, b.samp, b.ctl, b.L, P.ngroups, (uint32_t)P.part_windows);
    }
}

// Symbolic kernels over the four bins, the merge of split rows and the
// per-case finalize (sizes of the lists are device-side; the grids are upper
// bounds and every kernel walks its list grid-stride or by work queue).
template <int MODE>
void launch_symbolic(ssp_handle h, const Plan& P, const Bound& b, hipStream_t s, bool timed,
                     bool finalize)
{
    const int cus = h->num_cus;
    const int64_t nitems = P.cap13;
    {
        // bins 1..3: a grid of the resident capacity (more rows in flight hide
        // the latency of each row's chain of loads)
        PhaseTimer pt(h, PH_SYM_BINS, s, timed);
        if (P.bin2_wave) {
            hipLaunchKernelGGL((k_sym<kBin1Team, kBin1Words, MODE>),
                               dim3(grid_for(nitems, resident(k_sym<kBin1Team, kBin1Words, MODE>, kBin1Team, cus))),
                               dim3(kBin1Team), 0, s, b.cs, b.L.b1, &b.ctl->bin_cnt[1], b.cr);
            hipLaunchKernelGGL((k_sym<kWave, kBin2Words, MODE>),
                               dim3(grid_for(nitems, resident(k_sym<kWave, kBin2Words, MODE>, kWave, cus))),
                               dim3(kWave), 0, s, b.cs, b.L.b2, &b.ctl->bin_cnt[2], b.cr);
        } else {
            // bins 1 and 2 in one launch (few rows: the two latency chains
            // overlap), half the resident workgroups each
            const int64_t half =
                std::max<int64_t>(1, resident(k_sym_bins12<MODE>, kBins12Threads, cus) / 2);
            const int64_t nw = kBins12Threads / kWave;
            const int64_t g1 = std::max<int64_t>(1, std::min<int64_t>((nitems + nw - 1) / nw, half));
            const int64_t g2 = std::max<int64_t>(1, std::min<int64_t>(nitems, half));
            hipLaunchKernelGGL((k_sym_bins12<MODE>), dim3((unsigned)(g1 + g2)), dim3(kBins12Threads), 0,
                               s, b.cs, (const BinItem*)b.L.b1, (const uint32_t*)&b.ctl->bin_cnt[1],
                               (const BinItem*)b.L.b2, (const uint32_t*)&b.ctl->bin_cnt[2],
                               (uint32_t)g1, b.cr);
        }
        // (bin 3 stays empty when every case sends its rows to the long-row kernel)
        bool bin3 = false;
        for (int c = 0; c < P.n; ++c) bin3 = bin3 || !P.cs[c].big3;
        if (bin3)
            hipLaunchKernelGGL((k_sym<kBin3Team, kBin3Words, MODE>),
                               dim3(grid_for(nitems, resident(k_sym<kBin3Team, kBin3Words, MODE>, kBin3Team, cus))),
                               dim3(kBin3Team), 0, s, b.cs, b.L.b3, &b.ctl->bin_cnt[3], b.cr);
    }
    // one window holding all N columns in every case: no window tests
    auto kfun = P.win1 ? k_sym_big<MODE, true> : k_sym_big<MODE, false>;
    const size_t lds = (size_t)P.win_words_max * sizeof(uint32_t);
    {
        PhaseTimer pt(h, PH_SYM_LONG, s, timed);
        hipLaunchKernelGGL(kfun,
                           dim3(grid_for(P.cap4, resident(kfun, kBin4Team, cus, kWinWords * sizeof(uint32_t)))),
                           dim3(kBin4Team), lds, s, b.cs, b.L.b4, &b.ctl->bin_cnt[4],
                           &b.ctl->big_next, b.L, b.cr);
    }
    {
        PhaseTimer pt(h, PH_SYM_MERGE, s, timed);
        hipLaunchKernelGGL((k_sym_merge<MODE>), dim3((unsigned)(4 * cus)), dim3(256), 0, s, b.cs,
                           b.L.merge, &b.ctl->bin_cnt[5], b.L, b.cr);
    }
    if (!finalize) return;  // (the prediction kernel sums z* itself)
    PhaseTimer pt(h, PH_FINALIZE, s, timed);
    hipLaunchKernelGGL((k_finalize<MODE>), dim3(grid_for(P.n, 1024)), dim3(kAccSlots), 0, s, b.cs,
                       b.cr, P.n);
}

// Sets the long-row kernel's dynamic LDS limit once (before any capture).
void prepare_kernels()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const int bytes = (int)(kWinWords * sizeof(uint32_t));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sym_big<0, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sym_big<0, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sym_big<1, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sym_big<1, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    });
}

// The whole launch sequence of a call.  `table_on_device`: the case table is
// already in the workspace (batches, graphs); otherwise (at most kArgCases
// cases) k_setup writes it from its kernel arguments.
// Clears, the case table (from the kernel arguments for small calls) and the
// merge-path tile starts, in one launch.
void launch_setup(ssp_handle h, const Plan& P, const Bound& b, hipStream_t s,
                  bool table_on_device, bool timed)
{
    {
        PhaseTimer pt(h, PH_TILES, s, timed);
        CaseArgs args;
        std::memset(&args, 0, sizeof(args));
        const int ninit = table_on_device ? (int)grid_for(P.n, 1024) : P.n;
        const dim3 grid((unsigned)(ninit + P.g_tiles));
        if (table_on_device) {
            hipLaunchKernelGGL(k_setup<false>, grid, dim3(256), 0, s, b.ctl, b.cs, b.cr, P.n,
                               ninit, b.tile_row, b.tile_case, args);
        } else {
            for (int c = 0; c < P.n; ++c) args.d[c] = P.cs[c];
            hipLaunchKernelGGL(k_setup<true>, grid, dim3(256), 0, s, b.ctl, b.cs, b.cr, P.n,
                               ninit, b.tile_row, b.tile_case, args);
        }
    }
}

ssp_status launch_plan(ssp_handle h, const Plan& P, const Bound& b, hipStream_t s,
                       bool table_on_device, bool timed)
{
    launch_setup(h, P, b, s, table_on_device, timed);
    SSP_LAUNCHED(h);
    if (P.kind == PLAN_EXACT) {
        launch_flop<FLOP_EXACT_BIN>(h, P, b, s, timed);
        launch_symbolic<1>(h, P, b, s, timed, true);
        SSP_LAUNCHED(h);
        return SSP_OK;
    }
    launch_flop<FLOP_ONLY>(h, P, b, s, timed);
    launch_sampling(h, P, b, s, timed);
    launch_symbolic<0>(h, P, b, s, timed, P.kind != PLAN_PREDICT);
    if (P.kind == PLAN_PREDICT) {
        PhaseTimer pt(h, PH_PRED_ROWS, s, timed);
        if (P.g_rows > 0)
            hipLaunchKernelGGL(k_pred_rows, dim3(P.g_rows), dim3(kRowsThreads), 0, s, b.cs, P.n,
                               (const CaseRes*)b.cr);
    } else {
        {
            PhaseTimer pt(h, PH_FINALIZE, s, timed);
            hipLaunchKernelGGL(k_finalize_reference, dim3((unsigned)((P.n + 63) / 64)), dim3(64), 0,
                               s, (const CaseDesc*)b.cs, b.cr, P.n);
        }
        PhaseTimer pt(h, PH_REF_ROWS, s, timed);
        if (P.g_rows > 0)
            hipLaunchKernelGGL(k_ref_rows, dim3(P.g_rows), dim3(kRowsThreads), 0, s, b.cs, P.n,
                               (const CaseRes*)b.cr);
    }
    SSP_LAUNCHED(h);
    return SSP_OK;
}

// Copies a batch's case table to the workspace through the handle's pinned
// staging buffer (reused once the previous copy from it has completed).
ssp_status stage_table(ssp_handle h, const Plan& P, const Bound& b, hipStream_t s)
{
    const size_t bytes = (size_t)P.n * sizeof(CaseDesc);
    if (!h->pin_ev) SSP_HIP(h, hipEventCreateWithFlags(&h->pin_ev, hipEventDisableTiming));
    SSP_HIP(h, hipEventSynchronize(h->pin_ev));
    if (bytes > h->pin_bytes) {
        if (h->pin) SSP_HIP(h, hipHostFree(h->pin));
        h->pin = nullptr;
        h->pin_bytes = 0;
        SSP_HIP(h, hipHostMalloc(&h->pin, bytes, hipHostMallocDefault));
        h->pin_bytes = bytes;
    }
    std::memcpy(h->pin, P.cs.data(), bytes);
    SSP_HIP(h, hipMemcpyAsync(b.cs, h->pin, bytes, hipMemcpyHostToDevice, s));
    SSP_HIP(h, hipEventRecord(h->pin_ev, s));
    return SSP_OK;
}

// Plan, workspace, launches: the common body of every compute entry point.
ssp_status run_plan(ssp_handle h, const std::vector<CaseIn>& in, PlanKind kind, hipStream_t s)
{
    prepare_kernels();
    Plan P = make_plan(h, in, kind);
    ssp_status st = plan_fits_lists(h, P);
    if (st != SSP_OK) return st;
    st = ensure_workspace(h, P.total);
    if (st != SSP_OK) return st;
    const Bound b = bind_plan(P, h->ws);
    const bool small = P.n <= kArgCases;
    if (!small && (st = stage_table(h, P, b, s)) != SSP_OK) return st;
    return launch_plan(h, P, b, s, !small, true);
}

CaseIn case_in(const ssp_csr* A, const ssp_csr* B, ssp_sampler sampler, double rate,
               uint64_t seed, int64_t* out, int64_t* rf, ssp_stats* st)
{
    CaseIn x;
    x.A = to_csr(A);
    x.B = to_csr(B);
    x.sampler = sampler;
    x.rate = rate;
    x.seed = seed;
    x.out = out;
    x.rf = rf;
    x.st = st;
    return x;
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
    {
        DeviceGuard g(device);
        if (g.ok()) noalloc_init(device);
    }
    *out = h;
    return SSP_OK;
}

ssp_status ssp_destroy(ssp_handle h)
{
    if (!h) return SSP_ERR_INVALID_ARG;
    ssp_status st = SSP_OK;
    DeviceGuard g(h->device);
    if (h->ws || h->num_ws || h->num_slots || h->num_pool) {
        if (hipDeviceSynchronize() != hipSuccess) st = SSP_ERR_HIP;
        for (void* p : {h->ws, h->num_ws, h->num_slots, h->num_pool})
            if (p && hipFree(p) != hipSuccess) st = SSP_ERR_HIP;
    }
    h->num_state.reset();
    if (h->num_ev) (void)hipEventDestroy(h->num_ev);
    for (auto& p : h->pending) {
        h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    if (h->pin_ev) (void)hipEventSynchronize(h->pin_ev);
    if (h->pin) (void)hipHostFree(h->pin);
    if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
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
    const ssp_status s = common_checks(h, A, B, sampler, rate, nnz_pred);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return run_plan(h, {case_in(A, B, sampler, rate, seed, nnz_pred, row_flop, stats)},
                    PLAN_PREDICT, static_cast<hipStream_t>(stream));
}

ssp_status ssp_predict_structure(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                 double sample_rate, uint64_t seed, int64_t* nnz_pred,
                                 int64_t* row_flop, ssp_stats* stats, void* stream)
{
    return ssp_predict_structure_ex(h, A, B, SSP_SAMPLER_BERNOULLI, sample_rate, seed, nnz_pred,
                                    row_flop, stats, stream);
}

ssp_status ssp_predict_structure_noalloc(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                         ssp_sampler sampler, double rate, uint64_t seed,
                                         int64_t* nnz_pred, int64_t* row_flop, ssp_stats* stats,
                                         void* stream)
{
    const ssp_status s = common_checks(h, A, B, sampler, rate, nnz_pred);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    if (h->device >= kNoAllocDevices) {
        h->last_error = "no scratch array on device " + std::to_string(h->device);
        return SSP_ERR_NO_DEVICE;
    }
    const NoAllocSlot& slot = g_noalloc[h->device];
    if (!slot.ptr) return hip_fail(h, slot.err, "hipGetSymbolAddress(scratch)");
    prepare_kernels();
    // the plan of the allocating call; when it does not fit the array, fewer
    // part windows (rows split less, the counts are the same)
    const std::vector<CaseIn> in{case_in(A, B, sampler, rate, seed, nnz_pred, row_flop, stats)};
    Plan P;
    for (int64_t pw = kPartWindowsBase; pw >= kNoAllocMinWindows; pw /= 2) {
        P = make_plan(h, in, PLAN_PREDICT, pw);
        if (P.total <= kNoAllocBytes) break;
    }
    const ssp_status fit = plan_fits_lists(h, P);
    if (fit != SSP_OK) return fit;
    if (P.total > kNoAllocBytes) {
        h->last_error = "ssp_predict_structure_noalloc: needs " + std::to_string(P.total) +
                        " bytes of scratch, the fixed array holds " +
                        std::to_string(kNoAllocBytes);
        return SSP_ERR_BUDGET;
    }
    const Bound b = bind_plan(P, slot.ptr);
    return launch_plan(h, P, b, static_cast<hipStream_t>(stream), false, false);
}

ssp_status ssp_reference_estimate(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                  ssp_sampler sampler, double rate, uint64_t seed,
                                  int64_t* nnz_ref, ssp_stats* stats, void* stream)
{
    const ssp_status s = common_checks(h, A, B, sampler, rate, nnz_ref);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return run_plan(h, {case_in(A, B, sampler, rate, seed, nnz_ref, nullptr, stats)},
                    PLAN_REFERENCE, static_cast<hipStream_t>(stream));
}

ssp_status ssp_exact_structure(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                               int64_t* nnz_exact, ssp_stats* stats, void* stream)
{
    const ssp_status s = common_checks(h, A, B, SSP_SAMPLER_BERNOULLI, 0.0, nnz_exact);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return run_plan(h, {case_in(A, B, SSP_SAMPLER_BERNOULLI, 0.0, 0, nnz_exact, nullptr, stats)},
                    PLAN_EXACT, static_cast<hipStream_t>(stream));
}

namespace {
ssp_status batch_inputs(ssp_handle h, int n, const ssp_case* cases, std::vector<CaseIn>& in)
{
    if (!h || n < 0 || (n > 0 && !cases)) return SSP_ERR_INVALID_ARG;
    in.clear();
    in.reserve((size_t)n);
    for (int i = 0; i < n; ++i) {
        const ssp_case& c = cases[i];
        const ssp_sampler smp = (ssp_sampler)c.sampler;
        const ssp_status s = common_checks(h, &c.A, &c.B, smp, c.sample_rate, c.nnz_pred);
        if (s != SSP_OK) return s;
        in.push_back(case_in(&c.A, &c.B, smp, c.sample_rate, c.seed, c.nnz_pred, c.row_flop,
                             c.stats));
    }
    return SSP_OK;
}
} // namespace

ssp_status ssp_predict_batch(ssp_handle h, int n, const ssp_case* cases, void* stream)
{
    std::vector<CaseIn> in;
    const ssp_status s = batch_inputs(h, n, cases, in);
    if (s != SSP_OK) return s;
    if (n == 0) return SSP_OK;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return run_plan(h, in, PLAN_PREDICT, static_cast<hipStream_t>(stream));
}

ssp_status ssp_batch_graph_create(ssp_handle h, int n, const ssp_case* cases,
                                  ssp_batch_graph* out)
{
    if (!out) return SSP_ERR_INVALID_ARG;
    *out = nullptr;
    std::vector<CaseIn> in;
    ssp_status s = batch_inputs(h, n, cases, in);
    if (s != SSP_OK) return s;
    if (n == 0) return SSP_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    prepare_kernels();
    Plan P = make_plan(h, in, PLAN_PREDICT);
    if ((s = plan_fits_lists(h, P)) != SSP_OK) return s;
    if (h->budget && P.total > h->budget) {
        h->last_error = "graph workspace of " + std::to_string(P.total) +
                        " bytes exceeds the budget of " + std::to_string(h->budget);
        return SSP_ERR_BUDGET;
    }
    ssp_batch_graph_s* G = new (std::nothrow) ssp_batch_graph_s();
    if (!G) return SSP_ERR_OOM;
    G->h = h;
    G->device = h->device;
    G->n = n;
    auto fail = [&](ssp_status st) {
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        if (G->ws) (void)hipFree(G->ws);
        delete G;
        return st;
    };
    hipError_t e = hipMalloc(&G->ws, P.total);
    G->ws_bytes = P.total;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->last_error = std::string("hipMalloc: ") + hipGetErrorString(e);
        G->ws = nullptr;
        return fail(SSP_ERR_OOM);
    }
    const Bound b = bind_plan(P, G->ws);
    e = hipMemcpy(b.cs, P.cs.data(), (size_t)n * sizeof(CaseDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_fail(h, e, "hipMemcpy case table"));
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(h, e, "hipStreamCreate"));
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return fail(hip_fail(h, e, "hipStreamBeginCapture"));
    }
    s = launch_plan(h, P, b, cap, true, false);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    G->graph = graph;
    if (s != SSP_OK) return fail(s);
    if (e != hipSuccess) return fail(hip_fail(h, e, "hipStreamEndCapture"));
    e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(hip_fail(h, e, "hipGraphInstantiate"));
    *out = G;
    return SSP_OK;
}

ssp_status ssp_batch_graph_launch(ssp_batch_graph g, void* stream)
{
    if (!g || !g->exec) return SSP_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok()) return SSP_ERR_NO_DEVICE;
    const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(g->h, e, "hipGraphLaunch");
    return SSP_OK;
}

size_t ssp_batch_graph_workspace_bytes(ssp_batch_graph g) { return g ? g->ws_bytes : 0; }

ssp_status ssp_batch_graph_destroy(ssp_batch_graph g)
{
    if (!g) return SSP_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    ssp_status st = SSP_OK;
    if (hipDeviceSynchronize() != hipSuccess) st = SSP_ERR_HIP;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws && hipFree(g->ws) != hipSuccess) st = SSP_ERR_HIP;
    delete g;
    return st;
}

void ssp_default_tuning(ssp_tuning* t)
{
    if (t) *t = default_tuning();
}

ssp_status ssp_get_tuning(ssp_handle h, ssp_tuning* t)
{
    if (!h || !t) return SSP_ERR_INVALID_ARG;
    *t = h->tuning;
    return SSP_OK;
}

ssp_status ssp_set_tuning(ssp_handle h, const ssp_tuning* t)
{
    if (!h || !t || !tuning_valid(*t)) return SSP_ERR_INVALID_ARG;
    h->tuning = *t;
    return SSP_OK;
}

ssp_status ssp_autotune(ssp_handle h, int n, const ssp_case* cases, int reps,
                        ssp_tuning* chosen, double* best_ms, double* default_ms, void* stream)
{
    if (reps < 1 || n < 1) return SSP_ERR_INVALID_ARG;
    std::vector<CaseIn> in;
    ssp_status s = batch_inputs(h, n, cases, in);
    if (s != SSP_OK) return s;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SSP_HIP(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SSP_ERR_HIP;
    }
    const bool was_timing = h->timing;
    h->timing = false;
    const ssp_tuning start = h->tuning;
    auto measure = [&](const ssp_tuning& t, double* ms) -> ssp_status {
        h->tuning = t;
        ssp_status st = run_plan(h, in, PLAN_PREDICT, hs);  // warm-up (and workspace)
        if (st != SSP_OK) return st;
        if (hipEventRecord(e0, hs) != hipSuccess) return SSP_ERR_HIP;
        for (int r = 0; r < reps; ++r)
            if ((st = run_plan(h, in, PLAN_PREDICT, hs)) != SSP_OK) return st;
        if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return SSP_ERR_HIP;
        float t_ms = 0.f;
        if (hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess) return SSP_ERR_HIP;
        *ms = (double)t_ms / reps;
        return SSP_OK;
    };
    ssp_tuning best = start;
    double best_t = 0, def_t = 0;
    s = measure(default_tuning(), &def_t);
    if (s == SSP_OK) s = measure(best, &best_t);
    // coordinate descent over the parameters, a few values each
    const uint64_t splits[] = {1ull << 15, 1ull << 16, 1ull << 17, 1ull << 18, 1ull << 19};
    const uint32_t longs[] = {16, 32, 64, 128};
    const uint32_t bins[][4] = {{128, 1024, 8192, 2}, {64, 512, 4096, 4}, {64, 512, 8192, 2},
                                {32, 256, 4096, 2},  {128, 512, 4096, 2}};
    auto consider = [&](ssp_tuning t) {
        if (s != SSP_OK || !tuning_valid(t) || std::memcmp(&t, &best, sizeof(t)) == 0) return;
        double ms = 0;
        s = measure(t, &ms);
        if (s == SSP_OK && ms < 0.98 * best_t) {
            best = t;
            best_t = ms;
        }
    };
    for (uint64_t v : splits) {
        ssp_tuning t = best;
        t.split_target = v;
        consider(t);
    }
    for (uint32_t v : longs) {
        ssp_tuning t = best;
        t.long_len = v;
        consider(t);
    }
    for (int v = 0; v <= 1; ++v) {
        ssp_tuning t = best;
        t.big3 = v;
        consider(t);
    }
    for (const auto& b : bins) {
        ssp_tuning t = best;
        t.bin_max[0] = b[0];
        t.bin_max[1] = b[1];
        t.bin_max[2] = b[2];
        t.hash_mult = b[3];
        consider(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->timing = was_timing;
    if (s != SSP_OK) {
        h->tuning = start;
        return s;
    }
    h->tuning = best;
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = best_t;
    if (default_ms) *default_ms = def_t;
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

#include "ssp_server.hpp"
#include "ssp_spgemm.hpp"
#include "ssp_kmv.hpp"
