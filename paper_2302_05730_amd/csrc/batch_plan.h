// Host bookkeeping of the batched form, free of HIP so that the library and a
// sanitizer build on the CPU compile the same code: the split of a class's
// work into tiles, the per-integrand ranges of block partials, the number of
// shares of a class and the spread of the classes over streams.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

namespace mcubes {

// Work items [w_begin, w_end) of integrand `item`; its (sum S_c, sum var_c)
// go to partials[2 partial], [2 partial + 1].
struct BatchTile {
    uint32_t item, w_begin, w_end, partial;
};

// Splits the samples of the class's integrands (in the order of `items`;
// integrand i has m[i] cubes of p[i] samples) into `shares` equal contiguous
// shares, a share ending inside an integrand at a cube boundary, and appends
// one tile per (share, integrand) pair with work.  A tile's partial slot is
// its index in `tiles`, so the tiles of an integrand are consecutive.
inline void split_tiles(const std::vector<int> &items, const int64_t *m, const int64_t *p,
                        int shares, std::vector<BatchTile> &tiles) {
    const int k = (int)items.size();
    std::vector<int64_t> off(k + 1, 0);
    for (int q = 0; q < k; ++q) off[q + 1] = off[q] + m[items[q]] * p[items[q]];
    const int64_t S = off[k];
    // position of sample offset T: (item slot, first cube starting at or after T)
    auto position = [&](int64_t T) {
        const int q = (int)(std::upper_bound(off.begin(), off.end(), T) - off.begin()) - 1;
        if (q >= k) return std::make_pair(k, (int64_t)0);
        const int i = items[q];
        const int64_t w = (T - off[q] + p[i] - 1) / p[i];
        if (w >= m[i]) return std::make_pair(q + 1, (int64_t)0);
        return std::make_pair(q, w);
    };
    auto lo = position(0);
    for (int b = 0; b < shares; ++b) {
        const int64_t Tb = (int64_t)(((unsigned __int128)S * (uint64_t)(b + 1)) / (uint64_t)shares);
        const auto hi = position(Tb);
        for (int q = lo.first; q <= hi.first && q < k; ++q) {
            const int64_t wb = q == lo.first ? lo.second : 0;
            const int64_t we = q == hi.first ? hi.second : m[items[q]];
            if (we > wb) {
                BatchTile t;
                t.item = (uint32_t)items[q];
                t.w_begin = (uint32_t)wb;
                t.w_end = (uint32_t)we;
                t.partial = (uint32_t)tiles.size();
                tiles.push_back(t);
            }
        }
        lo = hi;
    }
}

// [begin[i], end[i]) = the partial slots of integrand i's tiles (0, 0 for an
// integrand without tiles).  Returns the index of the first tile whose
// integrand's tiles are not consecutive, or -1.
inline int64_t part_ranges(const std::vector<BatchTile> &tiles, int n, uint32_t *begin,
                           uint32_t *end) {
    for (int i = 0; i < n; ++i) begin[i] = end[i] = 0;
    std::vector<char> seen(n, 0);
    for (size_t t = 0; t < tiles.size(); ++t) {
        const uint32_t i = tiles[t].item;
        if (!seen[i]) {
            seen[i] = 1;
            begin[i] = tiles[t].partial;
        } else if (end[i] != tiles[t].partial) {
            return (int64_t)t;
        }
        end[i] = tiles[t].partial + 1;
    }
    return -1;
}

// Shares (workgroups before the split at integrand boundaries) of a class of
// `cubes` cubes: `want` if positive, else one per `block` cubes but at most
// `per_slot` per workgroup slot of the device (`resident` slots); never more
// than `max_shares` or the cubes, never fewer than one.  0 if no workgroup
// of the class fits (resident < 1).
inline int class_shares(int64_t cubes, int block, int resident, int want, int64_t per_slot,
                        int64_t max_shares) {
    if (resident < 1) return 0;
    int64_t shares = want;
    if (shares <= 0) {
        shares = (cubes + block - 1) / block;
        if (shares > per_slot * resident) shares = per_slot * resident;
    }
    if (shares > max_shares) shares = max_shares;
    if (shares > cubes) shares = cubes;
    if (shares < 1) shares = 1;
    return (int)shares;
}

// Spreads classes of the given costs over at most `streams` branches, longest
// first onto the least loaded branch.  branch[k] receives class k's branch;
// returns the number of branches, min(streams, classes) but at least 1 (a
// branch never goes without work).
inline int assign_branches(const std::vector<double> &cost, int streams,
                           std::vector<int> &branch) {
    std::vector<std::pair<double, int>> order;
    for (int k = 0; k < (int)cost.size(); ++k) order.push_back({cost[k], k});
    std::sort(order.begin(), order.end(), [](const std::pair<double, int> &a,
                                             const std::pair<double, int> &b) {
        return a.first > b.first || (a.first == b.first && a.second < b.second);
    });
    const int branches = std::max(1, std::min(streams, (int)cost.size()));
    std::vector<double> load(branches, 0.0);
    branch.assign(cost.size(), 0);
    for (const auto &ck : order) {
        const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        branch[ck.second] = br;
        load[br] += ck.first;
    }
    return branches;
}

}  // namespace mcubes
