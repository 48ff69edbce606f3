// Host-side checks of the fused kernel's tile order (paper_1610_04914_amd/csrc/
// tile_order.hpp), built with g++ by tests/test_tile_order.py.  Exit status 0
// when every check holds; a failing check prints its case and returns 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "tile_order.hpp"

struct T4 {
    int x, y, z, w;
};

static int fails = 0;
#define CHECK(c, ...)                                 \
    do {                                              \
        if (!(c)) {                                   \
            std::printf("FAIL %s: ", #c);             \
            std::printf(__VA_ARGS__);                 \
            std::printf("\n");                        \
            ++fails;                                  \
        }                                             \
    } while (0)

// tiles of replicas with cubic sizes L[r] and z-chunk min(bz, L) as the
// library builds them (replica-major, then z, y, x)
static std::vector<T4> make_tiles(const std::vector<int>& L, int bx, int by, int bz,
                                  std::vector<int>& Lz, std::vector<int>& bzr) {
    std::vector<T4> list;
    Lz = L;
    bzr.assign(L.size(), 0);
    for (size_t r = 0; r < L.size(); ++r) {
        const int b = std::min(bz, L[r]);
        bzr[r] = b;
        const int tx = (L[r] + bx - 1) / bx, ty = (L[r] + by - 1) / by, tz = (L[r] + b - 1) / b;
        for (int z = 0; z < tz; ++z)
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) list.push_back(T4{(int)r, x, y, z});
    }
    return list;
}

// completion time of each XCD: 32 CUs take the XCD's tiles in order, each
// onto the CU that frees first; returns the slowest XCD's time in planes
static int64_t makespan(const std::vector<T4>& list, const std::vector<int>& Lz,
                        const std::vector<int>& bz) {
    const int n = (int)list.size();
    const std::vector<int> slot = tileord::xcd_slots(n);
    std::vector<std::vector<int>> by_xcd(8);
    std::vector<std::pair<int, int>> ids;  // (workgroup id, position)
    for (int p = 0; p < n; ++p) ids.push_back({slot[p], p});
    std::sort(ids.begin(), ids.end());
    for (auto& [id, p] : ids) by_xcd[id % 8].push_back(tileord::tile_planes(list[p], Lz, bz));
    int64_t worst = 0;
    for (auto& v : by_xcd) {
        std::vector<int64_t> cu(32, 0);
        for (int len : v) {
            auto it = std::min_element(cu.begin(), cu.end());
            *it += len;
        }
        worst = std::max(worst, *std::max_element(cu.begin(), cu.end()));
    }
    return worst;
}

static void check_order(const char* name, const std::vector<T4>& in, const std::vector<T4>& out,
                        const std::vector<int>& Lz, const std::vector<int>& bz, bool whole) {
    const int n = (int)in.size();
    CHECK((int)out.size() == n, "%s: size %zu vs %d", name, out.size(), n);
    std::multiset<std::tuple<int, int, int, int>> a, b;
    for (auto& t : in) a.insert({t.x, t.y, t.z, t.w});
    for (auto& t : out) b.insert({t.x, t.y, t.z, t.w});
    CHECK(a == b, "%s: not a permutation of the tiles", name);
    if (!tileord::xcd_blocks_exact(n)) {
        for (int p = 1; p < n; ++p)
            CHECK(tileord::tile_planes(out[p - 1], Lz, bz) >= tileord::tile_planes(out[p], Lz, bz),
                  "%s: not longest first at %d", name, p);
        return;
    }
    const int per = (n + 7) / 8;
    std::map<int, int> rep_xcd;
    std::vector<int64_t> load(8, 0);
    for (int p = 0; p < n; ++p) {
        const int k = p / per;
        load[k] += tileord::tile_planes(out[p], Lz, bz);
        if (p % per)
            CHECK(tileord::tile_planes(out[p - 1], Lz, bz) >= tileord::tile_planes(out[p], Lz, bz),
                  "%s: XCD %d not longest first at %d", name, k, p);
        if (whole) {
            auto it = rep_xcd.find(out[p].x);
            if (it == rep_xcd.end())
                rep_xcd[out[p].x] = k;
            else
                CHECK(it->second == k, "%s: replica %d split over XCDs", name, out[p].x);
        }
    }
    // dealing whole replicas largest first onto the least-loaded XCD leaves
    // every XCD within the largest replica's work (plus a moved tile) of the mean
    int64_t tot = 0, big = 0, maxtile = 0;
    std::vector<int64_t> rw(Lz.size(), 0);
    for (auto& t : in) rw[t.x] += tileord::tile_planes(t, Lz, bz);
    for (auto& t : in) maxtile = std::max<int64_t>(maxtile, tileord::tile_planes(t, Lz, bz));
    for (int64_t w : rw) tot += w, big = std::max(big, w);
    for (int k = 0; k < 8; ++k)
        CHECK(load[k] * 8 <= tot + 8 * (big + maxtile), "%s: XCD %d load %lld of %lld", name, k,
              (long long)load[k], (long long)tot);
}

int main() {
    // the mapping: a permutation of the workgroup ids with XCD k = id % 8
    // receiving the k-th block of positions, or the identity
    for (int n = 1; n <= 300; ++n) {
        const std::vector<int> s = tileord::xcd_slots(n);
        std::set<int> ids(s.begin(), s.end());
        CHECK((int)ids.size() == n && *ids.begin() == 0 && *ids.rbegin() == n - 1,
              "slots of n = %d", n);
        const int per = (n + 7) / 8;
        for (int p = 0; p < n; ++p)
            CHECK(tileord::xcd_blocks_exact(n) ? s[p] % 8 == p / per : s[p] == p, "n %d p %d", n,
                  p);
    }
    // the uneven batch workload: 32 replicas each of 24^3, 48^3, 64^3, 32 x 16
    // tiles, z-chunk 64
    {
        std::vector<int> L;
        for (int s : {24, 48, 64})
            for (int i = 0; i < 32; ++i) L.push_back(s);
        std::vector<int> Lz, bz;
        const std::vector<T4> in = make_tiles(L, 32, 16, 64, Lz, bz);
        const std::vector<T4> out = tileord::balance_tiles(in, Lz, bz);
        check_order("batch96", in, out, Lz, bz, true);
        const int64_t before = makespan(in, Lz, bz), after = makespan(out, Lz, bz);
        int64_t tot = 0;
        for (auto& t : in) tot += tileord::tile_planes(t, Lz, bz);
        std::printf("batch96: %zu tiles, makespan %lld -> %lld planes (perfect split %.1f)\n",
                    in.size(), (long long)before, (long long)after, tot / 256.0);
        CHECK(before == 144, "replica-major makespan %lld", (long long)before);
        CHECK(after <= 128, "balanced makespan %lld", (long long)after);
    }
    // random uneven batches
    std::mt19937 g(12345);
    for (int trial = 0; trial < 300; ++trial) {
        const int nrep = 2 + (int)(g() % 60);
        std::vector<int> L(nrep);
        for (int& l : L) l = 4 + (int)(g() % 90);
        const int bzs[] = {4, 8, 16, 32, 64, 128};
        const int bxs[][2] = {{32, 16}, {16, 16}, {32, 8}, {64, 8}};
        const int bzv = bzs[g() % 6];
        const int* sh = bxs[g() % 4];
        std::vector<int> Lz, bz;
        const std::vector<T4> in = make_tiles(L, sh[0], sh[1], bzv, Lz, bz);
        const std::vector<T4> out = tileord::balance_tiles(in, Lz, bz);
        char name[64];
        std::snprintf(name, sizeof name, "trial %d (n %zu)", trial, in.size());
        check_order(name, in, out, Lz, bz, false);
    }
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
