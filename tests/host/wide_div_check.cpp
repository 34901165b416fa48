// Host build of the library's 192-by-128-bit ceiling division (the reference
// design's rows whose numerator exceeds 128 bits), for a CPU test: reads
// lines "a q_hi q_lo d_hi d_lo" (decimal u64) and prints ceil(a q / d),
// computed as k_ref_rows does (64x128-bit product, then the division).
#include <cinttypes>
#include <cstdio>

#include "../../paper_2207_13848_amd/csrc/ssp_device.hpp"

int main()
{
    uint64_t a, qh, ql, dh, dl;
    while (std::scanf("%" SCNu64 " %" SCNu64 " %" SCNu64 " %" SCNu64 " %" SCNu64, &a, &qh, &ql,
                      &dh, &dl) == 5) {
        const unsigned __int128 p0 = (unsigned __int128)a * ql, p1 = (unsigned __int128)a * qh;
        const uint64_t n0 = (uint64_t)p0;
        const unsigned __int128 top = (p0 >> 64) + p1;
        const uint64_t q = ssp::ceil_div_192_by_128((uint64_t)(top >> 64), (uint64_t)top, n0,
                                                    ssp::u128{dl, dh});
        std::printf("%" PRIu64 "\n", q);
    }
    return 0;
}
