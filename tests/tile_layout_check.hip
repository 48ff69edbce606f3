// Host-side checks of the fused kernel's tile layout (no GPU needed):
//  - ring_decode is a bijection from point indices onto the load region;
//  - region prefix property: index < |R_s| iff the point lies in R_s (the
//    tile grown by 4 - s sites), which the per-stage wave and lane tests use.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "../paper_1610_04914_amd/csrc/kern_fused.hpp"

using namespace lll;

template <int BX, int BY>
int check() {
    const int R[5] = {(BX + 8) * (BY + 8), (BX + 6) * (BY + 6), (BX + 4) * (BY + 4),
                      (BX + 2) * (BY + 2), BX * BY};
    std::vector<int> seen(R[0], 0);
    std::vector<int> LX(R[0]), LY(R[0]);
    int bad = 0;
    for (int idx = 0; idx < R[0]; ++idx) {
        int lx, ly;
        ring_decode<BX, BY>(idx, lx, ly);
        LX[idx] = lx;
        LY[idx] = ly;
        if (lx < -4 || lx >= BX + 4 || ly < -4 || ly >= BY + 4) {
            ++bad;
            continue;
        }
        seen[(ly + 4) * (BX + 8) + lx + 4]++;
        int d = 0;
        d = std::max(d, -lx);
        d = std::max(d, lx - (BX - 1));
        d = std::max(d, -ly);
        d = std::max(d, ly - (BY - 1));
        for (int s = 0; s <= 4; ++s)
            if ((d <= 4 - s) != (idx < R[s])) ++bad;
    }
    for (int v : seen)
        if (v != 1) ++bad;
    printf("%dx%d bad=%d\n", BX, BY, bad);
    return bad;
}

int main() {
    int b = 0;
    b += check<32, 16>() + check<16, 16>() + check<32, 8>() + check<64, 8>();
    b += check<16, 8>() + check<8, 8>() + check<24, 16>() + check<1, 1>();
    return b != 0;
}
