// Host build of the sampling scan's running sums of part windows (the field
// packed above each group's bin-3 count), for a CPU test.  Reads "budget
// ngroups" and then ngroups lines "n3 wins" (decimal), and prints per group
// "o3 wpre split", combining the groups as the one-workgroup scan does: 1024
// groups per chunk, an exclusive prefix inside the chunk, a carry between
// chunks, each group's window count clamped and the carry saturated by the
// library's own helpers.
#include <cinttypes>
#include <cstdio>
#include <vector>

#include "../../paper_2207_13848_amd/csrc/ssp_device.hpp"

int main()
{
    constexpr int NT = 1024;
    uint32_t budget = 0;
    long long ng = 0;
    if (std::scanf("%" SCNu32 " %lld", &budget, &ng) != 2) return 1;
    std::vector<uint32_t> n3(ng), wins(ng);
    for (long long g = 0; g < ng; ++g)
        if (std::scanf("%" SCNu32 " %" SCNu32, &n3[g], &wins[g]) != 2) return 1;
    uint64_t k2w = 0;
    for (long long g0 = 0; g0 < ng; g0 += NT) {
        uint64_t ex = 0;  // exclusive prefix inside the chunk
        for (long long g = g0; g < ng && g < g0 + NT; ++g) {
            const uint64_t p2w = k2w + ex;
            const uint32_t wpre = (uint32_t)(p2w >> 32);
            const bool split = wins[g] != 0 && (uint64_t)wpre + wins[g] <= (uint64_t)budget;
            std::printf("%" PRIu32 " %" PRIu32 " %d\n", (uint32_t)p2w, wpre, split ? 1 : 0);
            ex += (uint64_t)n3[g] | ((uint64_t)ssp::clamp_windows(wins[g], budget) << 32);
        }
        k2w = ssp::saturate_windows_hi(k2w + ex, budget);
    }
    return 0;
}
