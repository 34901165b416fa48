// C-ABI of the structure-prediction library (declared in include/ssp.h):
// handle and workspace management, host-side argument checks and the launch
// sequences of the prediction, reference and exact paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ssp_kernels.hpp"

using namespace ssp;

namespace {
enum Phase { PH_SAMPLE = 0, PH_SYMBOLIC, PH_FINALIZE, PH_FLOP, PH_REF_ROWS, PH_COUNT };
const char* const kPhaseNames[PH_COUNT] = {"sample_bin", "symbolic", "finalize", "flop",
                                           "ref_rows"};
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
    ~PhaseTimer()
    {
        if (!h_->timing || !p_.a || !p_.b) return;
        (void)hipEventRecord(p_.b, s_);
        h_->pending.push_back(p_);
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

// Grow the workspace to `bytes`.  The slot region of a fresh buffer is
// cleared here (the kernels keep it clear afterwards).
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
    const Layout L0 = make_layout(0, 0, false);
    SSP_HIP(h, hipMemset(p, 0, L0.bin1));
    SSP_HIP(h, hipDeviceSynchronize());
    h->ws = p;
    h->ws_bytes = want;
    return SSP_OK;
}

struct Bound {
    Ctl* ctl;
    BinLists L;
    int64_t* rowtmp;
};

Bound bind(ssp_handle h, const Layout& L)
{
    char* base = static_cast<char*>(h->ws);
    Bound b;
    b.ctl = reinterpret_cast<Ctl*>(base + L.ctl);
    b.L.b1 = reinterpret_cast<BinItem*>(base + L.bin1);
    b.L.b2 = reinterpret_cast<BinItem*>(base + L.bin2);
    b.L.b3 = reinterpret_cast<BinItem*>(base + L.bin3);
    b.L.b4 = reinterpret_cast<BigItem*>(base + L.bin4);
    b.L.slots = reinterpret_cast<uint32_t*>(base + L.slots);
    b.rowtmp = reinterpret_cast<int64_t*>(base + L.rowtmp);
    return b;
}

unsigned grid_for(int64_t items, int64_t cap)
{
    if (items < 1) items = 1;
    return (unsigned)std::min<int64_t>(items, cap);
}

// Rows per thread of the streaming kernel: aim at ~4096 entries of A per tile.
int pick_rpt(const ssp_csr* A)
{
    const double d = A->nrows ? (double)A->nnz / (double)A->nrows : 0.0;
    const double want = 4096.0 / (kFlopThreads * std::max(d, 1e-9));
    if (want >= 8) return 8;
    if (want >= 4) return 4;
    if (want >= 2) return 2;
    return 1;
}

template <int MODE>
void launch_flop(const FlopArgs& fa, int rpt, bool vec, hipStream_t s)
{
    const int64_t M = fa.A.nrows;
    const unsigned grid = (unsigned)((M + (int64_t)kFlopThreads * rpt - 1) / ((int64_t)kFlopThreads * rpt));
    const dim3 blk(kFlopThreads);
#define SSP_FLOP_CASE(R)                                                                        \
    case R:                                                                                    \
        if (vec) hipLaunchKernelGGL((k_flop<MODE, R, true>), dim3(grid), blk, 0, s, fa);       \
        else hipLaunchKernelGGL((k_flop<MODE, R, false>), dim3(grid), blk, 0, s, fa);          \
        break;
    switch (rpt) {
        SSP_FLOP_CASE(1)
        SSP_FLOP_CASE(2)
        SSP_FLOP_CASE(4)
        SSP_FLOP_CASE(8)
    }
#undef SSP_FLOP_CASE
}

// Symbolic kernels over the four bins (sizes of the lists are device-side;
// the grids are upper bounds and every kernel walks its list grid-stride).
template <int MODE>
void launch_symbolic(ssp_handle h, const Csr& A, const Csr& B, const Bound& b, int64_t nitems,
                     int64_t nbig, ssp_stats* st, int64_t* out, hipStream_t s)
{
    const int cus = h->num_cus;
    hipLaunchKernelGGL((k_sym<kBin1Team, kBin1Words, MODE>), dim3(grid_for(nitems, 16LL * cus)),
                       dim3(kBin1Team), 0, s, A, B, b.L.b1, &b.ctl->bin_cnt[1], st, out);
    hipLaunchKernelGGL((k_sym<kBin2Team, kBin2Words, MODE>), dim3(grid_for(nitems, 4LL * cus)),
                       dim3(kBin2Team), 0, s, A, B, b.L.b2, &b.ctl->bin_cnt[2], st, out);
    hipLaunchKernelGGL((k_sym<kBin3Team, kBin3Words, MODE>), dim3(grid_for(nitems, 2LL * cus)),
                       dim3(kBin3Team), 0, s, A, B, b.L.b3, &b.ctl->bin_cnt[3], st, out);
    hipLaunchKernelGGL((k_sym_big<MODE>), dim3(grid_for(nbig, 1LL * cus)), dim3(kBin4Team), 0, s,
                       A, B, b.L.b4, &b.ctl->bin_cnt[4], b.L.slots, st, out);
}

// Sampling, per-row products of the sample, binning and distinct counting:
// leaves n_s, f* and z* in *st.
ssp_status sampled_part(ssp_handle h, const ssp_csr* A, const ssp_csr* B, ssp_sampler sampler,
                        double rate, uint64_t seed, const Bound& b, const Layout& L,
                        ssp_stats* st, hipStream_t s)
{
    const Csr a = to_csr(A), bb = to_csr(B);
    const int64_t M = A->nrows;
    {
    PhaseTimer pt(h, PH_SAMPLE, s);
    if (sampler == SSP_SAMPLER_PAPER) {
        const int64_t nd = paper_sample_num(M);
        const unsigned grid = (unsigned)std::max<int64_t>(1, (nd + 255) / 256);
        hipLaunchKernelGGL((k_sample_bin<true>), dim3(grid), dim3(256), 0, s, a, bb, seed,
                           (uint64_t)0, nd, b.ctl, st, b.L);
    } else {
        const unsigned grid = (unsigned)((M + 255) / 256);
        hipLaunchKernelGGL((k_sample_bin<false>), dim3(grid), dim3(256), 0, s, a, bb, seed,
                           rate_threshold(rate), (int64_t)0, b.ctl, st, b.L);
    }
    }
    SSP_LAUNCHED(h);
    {
        PhaseTimer pt(h, PH_SYMBOLIC, s);
        launch_symbolic<0>(h, a, bb, b, L.cap13, L.cap4, st, nullptr, s);
    }
    SSP_LAUNCHED(h);
    return SSP_OK;
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
    const Layout L = make_layout(nitems, M, false);
    if ((s = ensure_workspace(h, L.total)) != SSP_OK) return s;
    const Bound b = bind(h, L);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    ssp_stats* st = stats ? stats : &b.ctl->stats;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, hs, b.ctl, st, (uint64_t)M);
    SSP_LAUNCHED(h);
    if (M == 0) return SSP_OK;
    if ((s = sampled_part(h, A, B, sampler, rate, seed, b, L, st, hs)) != SSP_OK) return s;
    {
        PhaseTimer pt(h, PH_FINALIZE, hs);
        hipLaunchKernelGGL(k_finalize_predict, dim3(1), dim3(64), 0, hs, b.ctl, st);
    }
    FlopArgs fa;
    fa.A = to_csr(A);
    fa.B = to_csr(B);
    fa.out = nnz_pred;
    fa.out_flop = row_flop;
    fa.st = st;
    fa.ctl = b.ctl;
    fa.L = b.L;
    const bool vec = (reinterpret_cast<uintptr_t>(A->col) & 15u) == 0;
    {
        PhaseTimer pt(h, PH_FLOP, hs);
        launch_flop<FLOP_PREDICT>(fa, pick_rpt(A), vec, hs);
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
    const Layout L = make_layout(nitems, M, true);
    if ((s = ensure_workspace(h, L.total)) != SSP_OK) return s;
    const Bound b = bind(h, L);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    ssp_stats* st = stats ? stats : &b.ctl->stats;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, hs, b.ctl, st, (uint64_t)M);
    SSP_LAUNCHED(h);
    if (M == 0) return SSP_OK;
    if ((s = sampled_part(h, A, B, sampler, rate, seed, b, L, st, hs)) != SSP_OK) return s;
    FlopArgs fa;
    fa.A = to_csr(A);
    fa.B = to_csr(B);
    fa.out = b.rowtmp;
    fa.out_flop = nullptr;
    fa.st = st;
    fa.ctl = b.ctl;
    fa.L = b.L;
    const bool vec = (reinterpret_cast<uintptr_t>(A->col) & 15u) == 0;
    {
        PhaseTimer pt(h, PH_FLOP, hs);
        launch_flop<FLOP_ONLY>(fa, pick_rpt(A), vec, hs);
    }
    {
        PhaseTimer pt(h, PH_FINALIZE, hs);
        hipLaunchKernelGGL(k_finalize_reference, dim3(1), dim3(64), 0, hs, b.ctl, st,
                           (uint64_t)M);
    }
    {
        PhaseTimer pt(h, PH_REF_ROWS, hs);
        hipLaunchKernelGGL(k_ref_rows, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, hs,
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
    const Layout L = make_layout(M, M, false);
    if ((s = ensure_workspace(h, L.total)) != SSP_OK) return s;
    const Bound b = bind(h, L);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    ssp_stats* st = stats ? stats : &b.ctl->stats;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, hs, b.ctl, st, (uint64_t)M);
    SSP_LAUNCHED(h);
    if (M == 0) return SSP_OK;
    FlopArgs fa;
    fa.A = to_csr(A);
    fa.B = to_csr(B);
    fa.out = nnz_exact;
    fa.out_flop = nullptr;
    fa.st = st;
    fa.ctl = b.ctl;
    fa.L = b.L;
    const bool vec = (reinterpret_cast<uintptr_t>(A->col) & 15u) == 0;
    {
        PhaseTimer pt(h, PH_FLOP, hs);
        launch_flop<FLOP_EXACT_BIN>(fa, pick_rpt(A), vec, hs);
    }
    SSP_LAUNCHED(h);
    {
        PhaseTimer pt(h, PH_SYMBOLIC, hs);
        launch_symbolic<1>(h, fa.A, fa.B, b, L.cap13, L.cap4, st, nnz_exact, hs);
    }
    SSP_LAUNCHED(h);
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
