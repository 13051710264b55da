// CPU driver of the batched form's host bookkeeping (batch_plan.h), built by
// tests/test_host_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer.  It replays a convergence schedule the way the
// batch runtime plans work -- classes of (family, dim, p == 2), shares per
// class, tiles, per-integrand partial ranges, branches over streams, and a
// new plan over the integrands still running whenever 2% of the planned
// samples have finished -- and checks every plan:
//   * the tiles of every running integrand cover its work items [0, m)
//     exactly once, in order, and no tile belongs to a finished integrand;
//   * partial slots are the tile indices, consecutive per integrand, and the
//     partial ranges agree with them;
//   * a class has between 1 and min(cubes, max) shares and at least as many
//     tiles as shares that carry work;
//   * every class has a branch in [0, branches), branches <= classes and
//     <= streams, and no branch is left without a class.
// Input (stdin): "schedule streams resident block" then n and n lines
// "family dim m p stop" (stop = iterations the integrand runs), or
// "fuzz seed rounds".  Prints "ok <plans> <tiles>" and exits 0, or prints
// the violated check and exits 1.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>
#include <string>
#include <tuple>
#include <vector>

#include "batch_plan.h"

using namespace mcubes;

namespace {

constexpr int64_t kPerSlot = 8;
constexpr int64_t kMaxShares = 1 << 20;

struct Item {
    int family, dim;
    int64_t m, p;
    int stop;
};

int64_t g_plans = 0, g_tiles = 0;

void require(bool ok, const std::string &what) {
    if (!ok) {
        printf("FAILED: %s\n", what.c_str());
        exit(1);
    }
}

// One plan over the active integrands, checked.  Returns the planned samples.
int64_t plan_and_check(const std::vector<Item> &items, const std::vector<char> &active,
                       int streams, int resident, int block) {
    const int n = (int)items.size();
    std::vector<int64_t> m(n), p(n);
    for (int i = 0; i < n; ++i) {
        m[i] = items[i].m;
        p[i] = items[i].p;
    }
    std::map<std::tuple<int, int, int>, std::vector<int>> groups;
    for (int i = 0; i < n; ++i)
        if (active[i]) groups[{items[i].family, items[i].dim, p[i] == 2 ? 1 : 0}].push_back(i);
    std::vector<BatchTile> tiles;
    std::vector<double> cost;
    int64_t samples = 0;
    for (auto &kv : groups) {
        int64_t cubes = 0, cls = 0;
        for (int i : kv.second) {
            cubes += m[i];
            cls += m[i] * p[i];
        }
        const int shares = class_shares(cubes, block, resident, 0, kPerSlot, kMaxShares);
        require(shares >= 1 && shares <= cubes && shares <= kPerSlot * resident,
                "share count of a class");
        const size_t t0 = tiles.size();
        split_tiles(kv.second, m.data(), p.data(), shares, tiles);
        require(tiles.size() - t0 >= 1, "a class with work has tiles");
        cost.push_back((double)cls * (std::get<1>(kv.first) + 4) * 1e-9);
        samples += cls;
    }
    // coverage: per integrand, its tiles in order cover [0, m) exactly once
    std::vector<int64_t> next(n, 0);
    for (size_t t = 0; t < tiles.size(); ++t) {
        const BatchTile &T = tiles[t];
        require(T.item < (uint32_t)n, "tile integrand in range");
        require(active[T.item], "no tile of a finished integrand");
        require(T.partial == (uint32_t)t, "partial slot = tile index");
        require(T.w_begin < T.w_end, "tile not empty");
        require((int64_t)T.w_begin == next[T.item], "tiles contiguous and in order");
        require((int64_t)T.w_end <= m[T.item], "tile inside the integrand");
        next[T.item] = T.w_end;
    }
    for (int i = 0; i < n; ++i)
        require(next[i] == (active[i] ? m[i] : 0), "every work item covered once");
    std::vector<uint32_t> pb(n), pe(n);
    require(part_ranges(tiles, n, pb.data(), pe.data()) < 0, "tiles of an integrand consecutive");
    std::vector<uint32_t> cnt(n, 0), first(n, 0);
    for (size_t t = 0; t < tiles.size(); ++t)
        if (cnt[tiles[t].item]++ == 0) first[tiles[t].item] = (uint32_t)t;
    for (int i = 0; i < n; ++i)
        require(pe[i] - pb[i] == cnt[i] && (cnt[i] == 0 || pb[i] == first[i]), "partial ranges");
    std::vector<int> branch;
    const int branches = assign_branches(cost, streams, branch);
    require(branches >= 1 && branches <= streams, "branch count within streams");
    require(cost.empty() || branches <= (int)cost.size(), "no more branches than classes");
    std::vector<int> used(branches, 0);
    for (int b : branch) {
        require(b >= 0 && b < branches, "branch in range");
        used[b] = 1;
    }
    if (!cost.empty())
        for (int b = 0; b < branches; ++b) require(used[b] == 1, "no branch without a class");
    ++g_plans;
    g_tiles += (int64_t)tiles.size();
    return samples;
}

// The batch runtime's loop with re-planning: iteration t runs the integrands
// with stop > t; after it, a new plan when 2% of the planned samples are done.
void schedule(const std::vector<Item> &items, int streams, int resident, int block) {
    const int n = (int)items.size();
    std::vector<char> active(n, 1);
    int itmax = 0;
    for (const Item &it : items) itmax = std::max(itmax, it.stop);
    int64_t planned = plan_and_check(items, active, streams, resident, block);
    for (int t = 0; t < itmax; ++t) {
        int64_t left = 0;
        int running = 0;
        for (int i = 0; i < n; ++i) {
            active[i] = items[i].stop > t + 1;
            if (active[i]) {
                left += items[i].m * items[i].p;
                ++running;
            }
        }
        if (running == 0) break;
        if (t + 1 < itmax && left < planned - planned / 50)
            planned = plan_and_check(items, active, streams, resident, block);
    }
}

void fuzz(uint64_t seed, int rounds) {
    std::mt19937_64 rng(seed);
    for (int r = 0; r < rounds; ++r) {
        const int n = 1 + (int)(rng() % 40);
        std::vector<Item> items(n);
        for (Item &it : items) {
            it.family = (int)(rng() % 6);
            it.dim = 2 + (int)(rng() % 9);
            const int kind = (int)(rng() % 4);
            it.m = kind == 0 ? 1 : (kind == 1 ? 1 + (int64_t)(rng() % 64)
                                              : 1 + (int64_t)(rng() % 3000000));
            it.p = 2 + (int64_t)(rng() % 3 == 0 ? rng() % 30 : 0);
            it.stop = 1 + (int)(rng() % 12);
        }
        const int streams = 1 + (int)(rng() % 4);
        const int resident = 1 + (int)(rng() % 300);
        const int block = 64 * (1 + (int)(rng() % 16));
        schedule(items, streams, resident, block);
    }
}

}  // namespace

int main() {
    char mode[32] = {0};
    if (scanf("%31s", mode) != 1) return 2;
    if (std::string(mode) == "schedule") {
        int streams, resident, block, n;
        if (scanf("%d %d %d %d", &streams, &resident, &block, &n) != 4) return 2;
        std::vector<Item> items(n);
        for (Item &it : items) {
            long long m, p;
            if (scanf("%d %d %lld %lld %d", &it.family, &it.dim, &m, &p, &it.stop) != 5) return 2;
            it.m = m;
            it.p = p;
        }
        schedule(items, streams, resident, block);
    } else if (std::string(mode) == "fuzz") {
        unsigned long long seed;
        int rounds;
        if (scanf("%llu %d", &seed, &rounds) != 2) return 2;
        fuzz(seed, rounds);
    } else {
        return 2;
    }
    printf("ok %lld %lld\n", (long long)g_plans, (long long)g_tiles);
    return 0;
}
