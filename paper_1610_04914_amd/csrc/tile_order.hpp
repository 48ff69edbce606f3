// Order of the fused kernel's tiles over the eight XCDs (host code only, no
// HIP types: the tile type is any struct with int members x = replica,
// y = tile x, z = tile y, w = tile z).
//
// Workgroup w of a launch runs on XCD w % 8, and each XCD dispatches its
// workgroups in increasing order.  xcd_slots maps position p of a contiguous
// tile list to workgroup id (p % per) * 8 + p / per, per = ceil(n / 8), so
// that XCD k receives positions [k per, (k + 1) per) in order; where those
// blocks do not cover the ids 0 .. n-1 exactly, the list order is kept.
//
// balance_tiles orders the tiles of a batch of replicas before that mapping.
// Replicas of different sizes march z-chunks of different lengths, so a
// replica-major list leaves the XCDs that received the big replicas working
// long after the others.  Whole replicas are dealt instead, largest work
// first, each to the least-loaded XCD that still has room (work of a tile =
// planes it marches: its chunk plus 8 of pipeline fill); tiles are then moved,
// shortest first, from XCDs over their share to the least-loaded one under
// it; each XCD runs its longest tiles first.  A replica's tiles stay on one
// XCD where the counts allow, so their shared halo columns meet in its L2.
// Where the mapping keeps the list order, the longest tiles simply go first.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace tileord {

inline bool xcd_blocks_exact(int n) {
    const int per = (n + 7) / 8;
    for (int p = 0; p < n; ++p)
        if ((p % per) * 8 + p / per >= n) return false;
    return true;
}

inline std::vector<int> xcd_slots(int n) {
    std::vector<int> slot(n);
    const int per = n > 0 ? (n + 7) / 8 : 1;
    const bool exact = xcd_blocks_exact(n);
    for (int p = 0; p < n; ++p) slot[p] = exact ? (p % per) * 8 + p / per : p;
    return slot;
}

// Planes a tile marches: its z-chunk (the last one of a replica may be
// shorter) plus the eight planes of the pipeline fill.
template <class T4>
inline int tile_planes(const T4& t, const std::vector<int>& Lz, const std::vector<int>& bz) {
    return std::min(bz[t.x], Lz[t.x] - t.w * bz[t.x]) + 8;
}

template <class T4>
std::vector<T4> balance_tiles(const std::vector<T4>& list, const std::vector<int>& Lz,
                              const std::vector<int>& bz) {
    const int n = (int)list.size();
    const int nrep = (int)Lz.size();
    auto len = [&](const T4& t) { return tile_planes(t, Lz, bz); };
    auto longest_first = [&](std::vector<T4>& v) {
        std::stable_sort(v.begin(), v.end(),
                         [&](const T4& a, const T4& b) { return len(a) > len(b); });
    };
    if (n == 0 || !xcd_blocks_exact(n)) {
        std::vector<T4> v = list;
        longest_first(v);
        return v;
    }
    const int per = (n + 7) / 8;
    int cap[8];  // positions each XCD receives
    for (int k = 0; k < 8; ++k) cap[k] = std::max(0, std::min(per, n - k * per));
    std::vector<int64_t> work(nrep, 0);
    std::vector<std::vector<T4>> of_rep(nrep);
    for (const T4& t : list) {
        work[t.x] += len(t);
        of_rep[t.x].push_back(t);
    }
    std::vector<int> rord(nrep);
    for (int r = 0; r < nrep; ++r) rord[r] = r;
    std::stable_sort(rord.begin(), rord.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<T4> xl[8];
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r : rord) {
        if (of_rep[r].empty()) continue;
        int best = -1;
        for (int k = 0; k < 8; ++k) {
            if (cap[k] == 0) continue;
            const bool fits = (int)(xl[k].size() + of_rep[r].size()) <= cap[k];
            const bool bfits =
                best >= 0 && (int)(xl[best].size() + of_rep[r].size()) <= cap[best];
            if (best < 0 || (fits && !bfits) || (fits == bfits && load[k] < load[best])) best = k;
        }
        xl[best].insert(xl[best].end(), of_rep[r].begin(), of_rep[r].end());
        load[best] += work[r];
    }
    // even out the counts: shortest tiles move from full XCDs to the least
    // loaded one with room (one exists while any XCD is over its share)
    for (int k = 0; k < 8; ++k) {
        longest_first(xl[k]);
        while ((int)xl[k].size() > cap[k]) {
            int to = -1;
            for (int m = 0; m < 8; ++m)
                if ((int)xl[m].size() < cap[m] && (to < 0 || load[m] < load[to])) to = m;
            const T4 t = xl[k].back();
            xl[k].pop_back();
            load[k] -= len(t);
            xl[to].push_back(t);
            load[to] += len(t);
        }
    }
    std::vector<T4> out;
    out.reserve(n);
    for (int k = 0; k < 8; ++k) {
        longest_first(xl[k]);
        out.insert(out.end(), xl[k].begin(), xl[k].end());
    }
    return out;
}

}  // namespace tileord
