// Independent Philox4x32-10 used only to pin the oracle's generator: it calls
// the ten-round function of rocRAND's header-only engine (host side) for
// counters and keys read from stdin, one "c0 c1 c2 c3 k0 k1" line each.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Engine eng;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = eng.rounds(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
