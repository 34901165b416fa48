// C-ABI of the numeric product that consumes a predicted structure
// (ssp_spgemm_compute, ssp_spgemm_copy; declared in include/ssp.h).  Included
// at the end of ssp_lib.hip, whose planning and launch helpers it uses: the
// row-FLOP pass of the precise method (Alg. 1 with binning) routes the rows,
// the kernels of ssp_numeric.hpp do the rest.
#pragma once

namespace {

// What ssp_spgemm_copy needs from the compute call.
struct NumState {
    Plan P;
    Bound b;
    NumArgs na;
    uint32_t bins[4] = {0, 0, 0, 0};  // items in bins 1..3 and bin 4
    int32_t dense_grid = 0;
    BinItem* abort_list = nullptr;    // rows whose first-pass table filled up
    bool win = false;                 // long rows by LDS column windows (B's rows sorted)
    int2* cursors = nullptr;          // their per-entry cursors (pool memory)
    int64_t cur_stride = 0;
    int64_t nrec = 0;                 // records of the overflow area
    int64_t recompute = 0;            // overflowing rows the area does not hold
    ssp_spgemm_info info{};
};

// Grows a device buffer of the handle (contents not kept), within the budget
// shared with the workspace.
ssp_status grow_buffer(ssp_handle h, void** p, size_t* have, size_t bytes, bool slack)
{
    if (bytes <= *have) return SSP_OK;
    const size_t others = h->ws_bytes + h->num_ws_bytes + h->num_slots_bytes + h->num_pool_bytes -
                          *have;
    if (h->budget && others + bytes > h->budget) {
        h->last_error = "numeric product buffers of " + std::to_string(bytes) +
                        " bytes exceed the budget of " + std::to_string(h->budget);
        return SSP_ERR_BUDGET;
    }
    size_t want = slack ? bytes + bytes / 4 : bytes;
    if (h->budget && others + want > h->budget) want = bytes;
    if (*p) {
        SSP_HIP(h, hipDeviceSynchronize());
        SSP_HIP(h, hipFree(*p));
        *p = nullptr;
        *have = 0;
    }
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->last_error = std::string("hipMalloc: ") + hipGetErrorString(e);
        return SSP_ERR_OOM;
    }
    *p = q;
    *have = want;
    return SSP_OK;
}

void launch_num_scan(const NumArgs& na, int kind, int cus, hipStream_t s)
{
    const int64_t nblk = (na.M + kNumScanBlock - 1) / kNumScanBlock;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nblk, 8LL * cus));
    if (kind == 0) {
        if (nblk > 0) hipLaunchKernelGGL(k_num_scan_part<0>, dim3(g), dim3(kNumScanThreads), 0, s, na);
        hipLaunchKernelGGL(k_num_scan_top<0>, dim3(1), dim3(kNumScanThreads), 0, s, na);
        if (nblk > 0) hipLaunchKernelGGL(k_num_scan_rows<0>, dim3(g), dim3(kNumScanThreads), 0, s, na);
    } else {
        if (nblk > 0) hipLaunchKernelGGL(k_num_scan_part<1>, dim3(g), dim3(kNumScanThreads), 0, s, na);
        hipLaunchKernelGGL(k_num_scan_top<1>, dim3(1), dim3(kNumScanThreads), 0, s, na);
        if (nblk > 0) hipLaunchKernelGGL(k_num_scan_rows<1>, dim3(g), dim3(kNumScanThreads), 0, s, na);
    }
}

// The dense kernel's LDS bitmap (up to 2^19 columns) needs more than the
// default dynamic LDS limit; set once.
void prepare_num_kernels()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const int wbytes = (int)(kNumWinCols * sizeof(double));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_num_dense_win<1>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, wbytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_num_dense_win<2>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, wbytes);
        const int bytes = (int)(kNumLdsMaskWords * sizeof(uint32_t));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_num_dense<1, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_num_dense<2, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    });
}

// The numeric kernels over the bins (pass 1 into the slots, pass 2 the rows
// that overflowed, into C); after pass 1 the symbolic kernel counts the rows
// whose first-pass table filled up.
template <int PASS>
void launch_num_rows(ssp_handle h, const NumState& S, hipStream_t s)
{
    const int cus = h->num_cus;
    const CaseDesc* cs = S.b.cs;
    Ctl* ctl = S.b.ctl;
    const uint32_t nhash = S.bins[0] + S.bins[1] + S.bins[2];
    {
        PhaseTimer pt(h, PASS == 1 ? PH_NUM_HASH : PH_NUM_FALLBACK, s);
        auto grid = [&](int64_t units, int64_t res) {
            return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(units, res)));
        };
        if (nhash)
            hipLaunchKernelGGL((k_num_wave<PASS>),
                               grid((nhash + kNumWaveWaves - 1) / kNumWaveWaves,
                                    resident(k_num_wave<PASS>, kNumWaveWaves * kWave, cus)),
                               dim3(kNumWaveWaves * kWave), 0, s, cs, S.b.L, ctl, S.abort_list, S.na);
        if (S.bins[1])
            hipLaunchKernelGGL((k_num_hash<kNumTeam2, kNumSlots2, PASS>),
                               grid(S.bins[1], resident(k_num_hash<kNumTeam2, kNumSlots2, PASS>, kNumTeam2, cus)),
                               dim3(kNumTeam2), 0, s, cs, (const BinItem*)S.b.L.b2,
                               (const uint32_t*)&ctl->bin_cnt[2], ctl, S.abort_list, S.na);
        if (S.bins[2])
            hipLaunchKernelGGL((k_num_hash<kNumTeam3, kNumSlots3, PASS>),
                               grid(S.bins[2], resident(k_num_hash<kNumTeam3, kNumSlots3, PASS>, kNumTeam3, cus)),
                               dim3(kNumTeam3), 0, s, cs, (const BinItem*)S.b.L.b3,
                               (const uint32_t*)&ctl->bin_cnt[3], ctl, S.abort_list, S.na);
        if (PASS == 1 && nhash)  // (the list is usually empty: the kernel then ends at once)
            hipLaunchKernelGGL((k_sym<kBin3Team, kBin3Words, 1>), dim3((unsigned)cus), dim3(kBin3Team),
                               0, s, cs, (const BinItem*)S.abort_list, (const uint32_t*)&ctl->num_abort,
                               S.b.cr);
    }
    if (S.bins[3] && S.dense_grid > 0) {
        PhaseTimer pt(h, PASS == 1 ? PH_NUM_DENSE : PH_NUM_FALLBACK, s);
        if (S.win)
            hipLaunchKernelGGL((k_num_dense_win<PASS>), dim3((unsigned)S.dense_grid), dim3(kNumDenseTeam),
                               (size_t)kNumWinCols * sizeof(double), s, cs, (const BigItem*)S.b.L.b4,
                               ctl, S.b.L.cap4, S.na, S.cursors, S.cur_stride);
        else if (S.na.mask_words <= kNumLdsMaskWords)
            hipLaunchKernelGGL((k_num_dense<PASS, true>), dim3((unsigned)S.dense_grid),
                               dim3(kNumDenseTeam), (size_t)S.na.mask_words * sizeof(uint32_t), s, cs,
                               (const BigItem*)S.b.L.b4, ctl, S.b.L.cap4, S.na);
        else
            hipLaunchKernelGGL((k_num_dense<PASS, false>), dim3((unsigned)S.dense_grid),
                               dim3(kNumDenseTeam), 0, s, cs, (const BigItem*)S.b.L.b4, ctl,
                               S.b.L.cap4, S.na);
    }
}

constexpr int64_t kNumPoolBytesMax = 1LL << 31;  // dense accumulators of a call, at most

ssp_status spgemm_compute(ssp_handle h, const ssp_csr* A, const double* A_val, const ssp_csr* B,
                          const double* B_val, const int64_t* row_cap, int32_t margin_pct,
                          int32_t spill_pct, int64_t* C_rpt, ssp_spgemm_info* info, hipStream_t s)
{
    // the previous call's copy pass may still read the slots and use the accumulators
    if (h->num_ev) SSP_HIP(h, hipEventSynchronize(h->num_ev));
    h->num_state.reset();
    prepare_num_kernels();
    const int cus = h->num_cus;
    const int64_t M = A->nrows, N = B->ncols;
    // the precise method's plan routes the rows; the numeric bins replace its limits
    std::vector<CaseIn> in(1, case_in(A, B, SSP_SAMPLER_BERNOULLI, 0.0, 0, nullptr, nullptr, nullptr));
    auto S = std::make_shared<NumState>();
    S->P = make_plan(h, in, PLAN_EXACT, 1);
    Plan& P = S->P;
    const int64_t nblk = (M + kNumScanBlock - 1) / kNumScanBlock;
    size_t o = align256(P.total);
    const size_t o_cnt = o;  o = align256(o + (size_t)std::max<int64_t>(M, 1) * sizeof(int64_t));
    const size_t o_slot = o; o = align256(o + (size_t)(M + 1) * sizeof(int64_t));
    const size_t o_part = o; o = align256(o + (size_t)std::max<int64_t>(5 * nblk, 1) * sizeof(int64_t));
    const size_t o_agg = o;  o = align256(o + kNumAgg * sizeof(uint64_t));
    const size_t o_abort = o; o = align256(o + (size_t)std::max<int64_t>(M, 1) * sizeof(BinItem));
    const size_t o_state = o; o = align256(o + (size_t)std::max<int64_t>(M, 1));
    ssp_status st = grow_buffer(h, &h->num_ws, &h->num_ws_bytes, o, true);
    if (st != SSP_OK) return st;
    char* base = static_cast<char*>(h->num_ws);
    S->b = bind_plan(P, h->num_ws);
    CaseDesc& d = P.cs[0];
    d.out = (decltype(d.out))(base + o_cnt);
    d.bin_max[0] = (uint32_t)kNumBin1Max;
    d.bin_max[1] = (uint32_t)kNumBin2Max;
    d.bin_max[2] = (uint32_t)kNumBin3Max;
    d.hash_mult = 2;
    d.big3 = 0;
    d.split_target = ~0ull;  // no row is split: one workgroup accumulates a whole row
    NumArgs& na = S->na;
    std::memset(&na, 0, sizeof(na));
    na.Aval = (decltype(na.Aval))A_val;
    na.Bval = (decltype(na.Bval))B_val;
    na.cap = (decltype(na.cap))row_cap;
    na.cnt = (decltype(na.cnt))(base + o_cnt);
    na.slot_off = (decltype(na.slot_off))(base + o_slot);
    na.part = (decltype(na.part))(base + o_part);
    na.agg = (decltype(na.agg))(base + o_agg);
    S->abort_list = reinterpret_cast<BinItem*>(base + o_abort);
    na.sp_state = (decltype(na.sp_state))(base + o_state);
    na.C_rpt = (decltype(na.C_rpt))C_rpt;
    na.M = M;
    na.N = N;
    na.margin = margin_pct;

    // 1. row FLOP and bins (Alg. 1), slot sizes and their offsets
    launch_setup(h, P, S->b, s, false, true);
    SSP_LAUNCHED(h);
    hipLaunchKernelGGL(k_num_zero, dim3(1), dim3(64), 0, s, (uint64_t*)na.agg, (int64_t)kNumAgg);
    {
        const int64_t words = (std::max<int64_t>(M, 1) + 7) / 8;
        hipLaunchKernelGGL(k_num_zero, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 4LL * cus)),
                           dim3(256), 0, s, (uint64_t*)na.sp_state, words);
    }
    launch_flop<FLOP_EXACT_BIN>(h, P, S->b, s, true);
    {
        PhaseTimer pt(h, PH_NUM_SCAN, s);
        launch_num_scan(na, 0, cus, s);
        // (for the long rows: whether B's rows are sorted, their longest A row)
        if (B->nrows > 0 && B->nnz > 0)
            hipLaunchKernelGGL(k_num_check_sorted, dim3((unsigned)std::min<int64_t>((B->nnz + 255) / 256, 8LL * cus)),
                               dim3(256), 0, s, P.cs[0].B, (const Ctl*)S->b.ctl, na);
        hipLaunchKernelGGL(k_num_maxlen, dim3((unsigned)(2 * cus)), dim3(256), 0, s,
                           (const BigItem*)S->b.L.b4, S->b.ctl, S->b.L.cap4, na);
    }
    SSP_LAUNCHED(h);
    SSP_HIP(h, hipStreamSynchronize(s));
    uint64_t agg[kNumAgg];
    Ctl ctl;
    SSP_HIP(h, hipMemcpy(agg, na.agg, sizeof(agg), hipMemcpyDeviceToHost));
    SSP_HIP(h, hipMemcpy(&ctl, S->b.ctl, sizeof(ctl), hipMemcpyDeviceToHost));
    const int64_t slots = (int64_t)agg[3];
    S->bins[0] = ctl.bin_cnt[1];
    S->bins[1] = ctl.bin_cnt[2];
    S->bins[2] = ctl.bin_cnt[3];
    S->bins[3] = ctl.bin_cnt[4] + ctl.bin_cnt[6];

    // 2. the slot area, the overflow area and its records, the dense accumulators
    const size_t slot_bytes = (size_t)std::max<int64_t>(slots, 1) * (sizeof(double) + sizeof(int32_t));
    const int64_t spc = std::min<int64_t>(kSpillCapMax, (int64_t)(((__int128)slots * spill_pct + 99) / 100));
    const int64_t rec_cap = spc > 0 ? std::min<int64_t>(kSpillRecMax, M + spc / kSpillChunk + 4096) : 0;
    size_t q = align256((size_t)std::max<int64_t>(slots, 1) * sizeof(double));
    const size_t q_col = q;   q = align256(q + (size_t)std::max<int64_t>(slots, 1) * sizeof(int32_t));
    const size_t q_spv = q;   q = align256(q + (size_t)spc * sizeof(double));
    const size_t q_spc = q;   q = align256(q + (size_t)spc * sizeof(int32_t));
    const size_t q_rec = q;   q = align256(q + (size_t)rec_cap * sizeof(SpillRec));
    if ((st = grow_buffer(h, &h->num_slots, &h->num_slots_bytes, q, true)) != SSP_OK) return st;
    char* sb = static_cast<char*>(h->num_slots);
    na.slot_val = (decltype(na.slot_val))sb;
    na.slot_col = (decltype(na.slot_col))(sb + q_col);
    na.sp_val = (decltype(na.sp_val))(sb + q_spv);
    na.sp_col = (decltype(na.sp_col))(sb + q_spc);
    na.sp_rec = (decltype(na.sp_rec))(sb + q_rec);
    na.sp_cap = spc;
    na.rec_cap = rec_cap;
    S->win = S->bins[3] > 0 && agg[5] == 0;
    if (S->win) {
        // LDS windows: no accumulators in global memory, a cursor per A entry
        S->cur_stride = std::max<int64_t>(1, (int64_t)agg[4]);
        const int64_t res = resident(k_num_dense_win<1>, kNumDenseTeam, cus, kNumWinCols * sizeof(double));
        const int64_t want = std::min<int64_t>((int64_t)S->bins[3], res);
        const size_t bytes = (size_t)(want * S->cur_stride) * sizeof(int2);
        if ((st = grow_buffer(h, &h->num_pool, &h->num_pool_bytes, bytes, false)) != SSP_OK) return st;
        h->num_pool_clean = false;  // (the cursors overwrite the accumulators' zeros)
        S->cursors = reinterpret_cast<int2*>(h->num_pool);
        S->dense_grid = (int32_t)want;
    } else if (S->bins[3] > 0) {
        na.mask_words = ((N + 31) / 32 + 1) / 2 * 2;  // (even: whole 8-byte words)
        const int64_t per_slot = N * (int64_t)sizeof(double) + na.mask_words * (int64_t)sizeof(uint32_t);
        const int64_t res = na.mask_words <= kNumLdsMaskWords
                                ? resident(k_num_dense<1, true>, kNumDenseTeam, cus, kNumLdsMaskWords * sizeof(uint32_t))
                                : resident(k_num_dense<1, false>, kNumDenseTeam, cus);
        const int64_t want = std::min<int64_t>({(int64_t)S->bins[3], res,
                                                std::max<int64_t>(1, kNumPoolBytesMax / per_slot)});
        const size_t bytes = (size_t)(want * per_slot);
        if (bytes > h->num_pool_bytes) h->num_pool_clean = false;
        if ((st = grow_buffer(h, &h->num_pool, &h->num_pool_bytes, bytes, false)) != SSP_OK) return st;
        na.pool_slots = (int32_t)want;
        na.pool = (decltype(na.pool))h->num_pool;
        na.pool_mask = (decltype(na.pool_mask))((char*)h->num_pool + (size_t)(want * N) * sizeof(double));
        S->dense_grid = (int32_t)want;
        if (!h->num_pool_clean) {
            const int64_t words = (int64_t)(h->num_pool_bytes / sizeof(uint64_t));
            hipLaunchKernelGGL(k_num_zero, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 16LL * cus)),
                               dim3(256), 0, s, (uint64_t*)h->num_pool, words);
            SSP_LAUNCHED(h);
        }
    }

    // chunks of the area for the long rows' workgroups: up to kSpillChunk
    // entries, the grid's chunks together at most an eighth of the area
    na.sp_chunk = std::max<int64_t>(1024, std::min<int64_t>(
                                              kSpillChunk, spc / (8 * std::max<int64_t>(1, S->dense_grid))));

    // 3. the numeric pass into the slots, then C's row offsets (a launched
    //    pass leaves the accumulators zero; one that failed to launch may not)
    const bool was_clean = h->num_pool_clean;
    h->num_pool_clean = false;
    launch_num_rows<1>(h, *S, s);
    SSP_LAUNCHED(h);
    h->num_pool_clean = S->win ? false : (S->bins[3] > 0 || was_clean);
    {
        PhaseTimer pt(h, PH_NUM_SCAN, s);
        launch_num_scan(na, 1, cus, s);
    }
    SSP_LAUNCHED(h);
    SSP_HIP(h, hipStreamSynchronize(s));
    ssp_stats stv;
    SSP_HIP(h, hipMemcpy(agg, na.agg, sizeof(agg), hipMemcpyDeviceToHost));
    SSP_HIP(h, hipMemcpy(&stv, P.cs[0].st, sizeof(stv), hipMemcpyDeviceToHost));
    ssp_spgemm_info& inf = S->info;
    inf.nnz = (int64_t)agg[0];
    inf.total_flop = (int64_t)stv.total_flop;
    inf.slot_entries = slots;
    inf.overflow_rows = (int64_t)agg[1];
    inf.overflow_nnz = (int64_t)agg[2];
    inf.slot_bytes = (int64_t)slot_bytes;
    inf.spill_rows = (int64_t)agg[8];
    inf.spill_nnz = (int64_t)agg[9];
    inf.spill_bytes = spc > 0 ? spc * (int64_t)(sizeof(double) + sizeof(int32_t)) +
                                    rec_cap * (int64_t)sizeof(SpillRec)
                              : 0;
    S->nrec = std::min<int64_t>((int64_t)(agg[6] >> kSpillShift), rec_cap);
    S->recompute = inf.overflow_rows - inf.spill_rows;
    *info = inf;
    h->num_state = S;
    return SSP_OK;
}

ssp_status spgemm_copy(ssp_handle h, int32_t* C_col, double* C_val, int64_t capacity, hipStream_t s)
{
    NumState* S = static_cast<NumState*>(h->num_state.get());
    if (!S) {
        h->last_error = "ssp_spgemm_copy without a preceding ssp_spgemm_compute";
        return SSP_ERR_INVALID_ARG;
    }
    if (capacity < S->info.nnz || (S->info.nnz > 0 && (!C_col || !C_val))) {
        h->last_error = "C needs " + std::to_string(S->info.nnz) + " entries";
        return SSP_ERR_INVALID_ARG;
    }
    NumArgs& na = S->na;
    na.C_col = (decltype(na.C_col))C_col;
    na.C_val = (decltype(na.C_val))C_val;
    na.capacity = capacity;
    const int cus = h->num_cus;
    if (S->info.nnz > S->info.overflow_nnz || S->info.spill_rows > 0) {
        PhaseTimer pt(h, PH_NUM_COPY, s);
        const int64_t blocks = (S->info.nnz + kNumCopyChunk - 1) / kNumCopyChunk;
        hipLaunchKernelGGL(k_num_copy, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 16LL * cus))),
                           dim3(kNumCopyRows), 0, s, na);
        if (S->info.spill_rows > 0 && S->nrec > 0)
            hipLaunchKernelGGL(k_num_spill_copy, dim3((unsigned)std::min<int64_t>(S->nrec, 16LL * cus)),
                               dim3(256), 0, s, na, S->nrec);
    }
    SSP_LAUNCHED(h);
    if (S->recompute > 0) {
        const bool was_clean = h->num_pool_clean;
        h->num_pool_clean = false;
        // (the dense fallback's work queue starts at 0 on every copy call)
        SSP_HIP(h, hipMemsetAsync(&S->b.ctl->num_next[1], 0, sizeof(uint32_t), s));
        launch_num_rows<2>(h, *S, s);
        SSP_LAUNCHED(h);
        // (the accumulators kernel leaves them zero; the windows kernel keeps cursors there)
        h->num_pool_clean = S->bins[3] > 0 ? !S->win : was_clean;
    }
    if (!h->num_ev) SSP_HIP(h, hipEventCreateWithFlags(&h->num_ev, hipEventDisableTiming));
    SSP_HIP(h, hipEventRecord(h->num_ev, s));
    return SSP_OK;
}

} // namespace

extern "C" {

ssp_status ssp_spgemm_compute(ssp_handle h, const ssp_csr* A, const double* A_val,
                              const ssp_csr* B, const double* B_val, const int64_t* row_cap,
                              int32_t margin_pct, int32_t spill_pct, int64_t* C_rpt,
                              ssp_spgemm_info* info, void* stream)
{
    if (!h || !info || !C_rpt) return SSP_ERR_INVALID_ARG;
    const ssp_status s = check_pair(A, B);
    if (s != SSP_OK) return s;
    if (margin_pct < 0 || margin_pct > kNumMarginMax) return SSP_ERR_INVALID_ARG;
    if (spill_pct < 0 || spill_pct > kNumMarginMax) return SSP_ERR_INVALID_ARG;
    if ((A->nnz > 0 && !A_val) || (B->nnz > 0 && !B_val) || (A->nrows > 0 && !row_cap))
        return SSP_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return spgemm_compute(h, A, A_val, B, B_val, row_cap, margin_pct, spill_pct, C_rpt, info,
                          static_cast<hipStream_t>(stream));
}

ssp_status ssp_spgemm_copy(ssp_handle h, int32_t* C_col, double* C_val, int64_t capacity,
                           void* stream)
{
    if (!h || capacity < 0) return SSP_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    return spgemm_copy(h, C_col, C_val, capacity, static_cast<hipStream_t>(stream));
}

} // extern "C"
