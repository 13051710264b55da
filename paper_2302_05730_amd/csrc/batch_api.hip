// Host runtime of the batched form (declared in include/mcubes.h): work
// split into per-class tile lists (batch_plan.h), graph capture and replay
// with per-integrand device done flags (the plan stays fixed during a call),
// and the autotuner.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "mcubes_internal.h"

using namespace mcubes;

namespace {

struct ClassKey {
    int family, dim, p2;
    bool operator<(const ClassKey &o) const {
        return std::tie(family, dim, p2) < std::tie(o.family, o.dim, o.p2);
    }
};

// Geometry chosen for a class (0 = library default).
struct ClassCfg {
    int block = 0, blocks = 0;
    double tuned_ms = 0.0, default_ms = 0.0;
};

struct ClassPlan {
    ClassKey key;
    std::vector<int> items;
    int block = 0, blocks = 0, max_block = 0;  // blocks = shares
    size_t lds = 0;
    const void *func = nullptr;      // kernel with bin sums (occupancy queries)
    VsTilesLaunchFn launch[2] = {};  // [nobins]
    uint32_t tile_off = 0;
    int ntiles = 0;
    int branch = 0;  // stream of the class's launch
    int64_t samples = 0, cubes = 0;
};

// Default split: kSharesPerSlot shares per workgroup slot of the device (the
// hardware dispatcher then balances the unequal tile times; one share per
// slot measured 1.6x slower on the 512-integrand workload), but at least one
// cube per thread.
constexpr int64_t kSharesPerSlot = 8;
constexpr int kMaxStreams = 4;
constexpr int64_t kMaxShares = 1 << 20;

}  // namespace

struct mcubes_batch {
    int n = 0, nb = 0, adapt_iters = -1, skip = 0, forced_block = 0;
    int prec = 0;  // 1: the FP32 map and integrand (MCUBES_FP32)
    double alpha = 1.5;
    int cus = 0;
    void *user_stream = nullptr;
    std::vector<BatchItem> items;
    std::vector<int> family, dim;
    std::vector<int64_t> g, m, p;
    std::vector<uint2> axes;
    std::map<ClassKey, ClassCfg> cfg;
    std::vector<ClassPlan> plan;
    std::vector<char> planned;  // items in the current plan
    int64_t planned_samples = 0;
    int ntiles = 0;
    bool tuned = false;
    int64_t grids_len = 0, bins_len = 0;
    size_t device_bytes = 0;

    BatchItem *d_items = nullptr;
    double *d_grids = nullptr, *d_bins = nullptr, *d_est = nullptr, *d_states = nullptr;
    uint32_t *d_done = nullptr;  // n flags, then the active count
    uint32_t *d_iter = nullptr;
    uint2 *d_axes = nullptr;
    BatchTile *d_tiles = nullptr;
    double *d_partials = nullptr;
    size_t cap_tiles = 0;
    uint32_t *h_done = nullptr;  // pinned, n + 1

    hipStream_t stream = nullptr;
    hipEvent_t ev[3] = {};
    hipGraphExec_t exec[2] = {};  // [frozen]
    // concurrent class launches: branch 0 runs on `stream`, branch k on side[k-1]
    int streams = kMaxStreams;
    int branches = 1;  // streams in use: min(streams, classes)
    hipStream_t side[kMaxStreams - 1] = {};
    hipEvent_t fork = nullptr, join[kMaxStreams - 1] = {};

    int last_iterations = 0, last_replans = 0;
    int64_t last_samples = 0;
    double last_ms = 0.0;
};

namespace {

void drop_graphs(mcubes_batch *B) {
    for (auto &e : B->exec) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
    }
}

void release(mcubes_batch *B) {
    if (!B) return;
    drop_graphs(B);
    for (auto &e : B->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : B->join)
        if (e) (void)hipEventDestroy(e);
    if (B->fork) (void)hipEventDestroy(B->fork);
    for (auto &q : B->side)
        if (q) (void)hipStreamDestroy(q);
    if (B->stream) (void)hipStreamDestroy(B->stream);
    (void)hipFree(B->d_items);
    (void)hipFree(B->d_grids);
    (void)hipFree(B->d_bins);
    (void)hipFree(B->d_est);
    (void)hipFree(B->d_states);
    (void)hipFree(B->d_done);
    (void)hipFree(B->d_iter);
    (void)hipFree(B->d_axes);
    (void)hipFree(B->d_tiles);
    (void)hipFree(B->d_partials);
    if (B->h_done) (void)hipHostFree(B->h_done);
    delete B;
}

template <typename T>
int device_alloc(mcubes_batch *B, T **ptr, size_t count) {
    const size_t bytes = (count ? count : 1) * sizeof(T);
    const hipError_t e = hipMalloc((void **)ptr, bytes);
    if (e != hipSuccess) return fail(MCUBES_E_ALLOC, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    B->device_bytes += bytes;
    return MCUBES_OK;
}

// Blocks of `block` threads of the class kernel resident on the whole device.
int resident_blocks(const mcubes_batch *B, const ClassPlan &c, int block) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c.func, block, 0) != hipSuccess)
        return 0;
    return per_cu * B->cus;
}

// Splits the class's samples into `shares` tiles (split_tiles).
void split_class(const mcubes_batch *B, const ClassPlan &c, int shares,
                 std::vector<BatchTile> &tiles) {
    mcubes::split_tiles(c.items, B->m.data(), B->p.data(), shares, tiles);
}

// Shares of a class for workgroups of `block` threads (class_shares).
int class_shares(const mcubes_batch *B, const ClassPlan &c, int block, int want) {
    return mcubes::class_shares(c.cubes, block, resident_blocks(B, c, block), want,
                                kSharesPerSlot, kMaxShares);
}

// Default workgroup size: small for low dimensions, where the LDS tables are
// small and finer tiles balance better (the autotuner's choice on the
// 512-integrand workload), the kernel's limit from 7-D on.
int default_block(const ClassPlan &c) {
    const int want = c.key.dim <= 3 ? 256 : (c.key.dim <= 6 ? 512 : 1024);
    return std::min(want, c.max_block / 64 * 64);
}

void set_item_step(mcubes_batch *B, int i, int block) {
    VsArgs tmp = B->items[i].args;
    set_step(tmp, B->dim[i], (uint64_t)block);
    B->items[i].step_block = tmp.step;
    memcpy(B->items[i].step_digit_block, tmp.step_digit, sizeof tmp.step_digit);
}

ClassPlan make_class(const mcubes_batch *B, const ClassKey &key) {
    ClassPlan c;
    c.key = key;
    const VsKernel &K = family_table(key.family)[key.dim];
    c.func = K.tiles_func[B->prec][0][key.p2];
    c.launch[0] = K.tiles_launch[B->prec][0][key.p2];
    c.launch[1] = K.tiles_launch[B->prec][1][key.p2];
    hipFuncAttributes fa;
    const bool ok = hipFuncGetAttributes(&fa, c.func) == hipSuccess;
    c.max_block = ok ? fa.maxThreadsPerBlock : 0;
    c.lds = ok ? fa.sharedSizeBytes : 0;  // static: tables for kMaxBins bins per axis
    return c;
}

// Spreads the classes over B->streams branches (assign_branches); the cost
// of a class is its tuned time, else its samples weighted by dimension.
void assign_branches(mcubes_batch *B) {
    std::vector<double> cost;
    for (const ClassPlan &c : B->plan) {
        auto it = B->cfg.find(c.key);
        cost.push_back((it != B->cfg.end() && it->second.tuned_ms > 0.0)
                           ? it->second.tuned_ms
                           : (double)c.samples * (c.key.dim + 4) * 1e-9);
    }
    std::vector<int> branch;
    B->branches = mcubes::assign_branches(cost, B->streams, branch);
    for (size_t k = 0; k < B->plan.size(); ++k) B->plan[k].branch = branch[k];
}

// (Re)builds the plan over the items not yet done: classes, geometry, tiles,
// and uploads the descriptors.  Invalidates the captured graphs.
int build_plan(mcubes_batch *B, const std::vector<char> &active) {
    // the descriptors are overwritten below: nothing may still read them
    if (B->stream) {
        hipError_t es = hipStreamSynchronize(B->stream);
        for (int q = 0; q < kMaxStreams - 1 && es == hipSuccess; ++q)
            if (B->side[q]) es = hipStreamSynchronize(B->side[q]);
        if (es != hipSuccess) return hip_fail(es, "hipStreamSynchronize");
    }
    drop_graphs(B);
    std::map<ClassKey, std::vector<int>> groups;
    for (int i = 0; i < B->n; ++i)
        if (active[i]) groups[ClassKey{B->family[i], B->dim[i], B->p[i] == 2 ? 1 : 0}].push_back(i);
    std::vector<ClassPlan> plan;
    std::vector<BatchTile> tiles;
    int64_t samples = 0;
    for (auto &kv : groups) {
        ClassPlan c = make_class(B, kv.first);
        c.items = kv.second;
        for (int i : c.items) {
            c.cubes += B->m[i];
            c.samples += B->m[i] * B->p[i];
        }
        if (c.max_block < 64) return fail(MCUBES_E_DEVICE, "V-Sample batch kernel unavailable");
        const ClassCfg &cf = B->cfg[kv.first];
        int block = B->forced_block ? B->forced_block : (cf.block ? cf.block : default_block(c));
        if (block > c.max_block) block = c.max_block / 64 * 64;
        c.block = block;
        c.blocks = class_shares(B, c, block, cf.blocks);
        if (c.blocks < 1)
            return fail(MCUBES_E_ARG, "V-Sample (family %d, dim %d) does not fit: block %d, LDS %zu",
                        c.key.family, c.key.dim, block, c.lds);
        for (int i : c.items) set_item_step(B, i, block);
        c.tile_off = (uint32_t)tiles.size();
        split_class(B, c, c.blocks, tiles);
        c.ntiles = (int)(tiles.size() - c.tile_off);
        samples += c.samples;
        plan.push_back(std::move(c));
    }
    // per-item partial ranges (the tiles of an item are consecutive)
    std::vector<uint32_t> pb(B->n), pe(B->n);
    const int64_t bad = part_ranges(tiles, B->n, pb.data(), pe.data());
    if (bad >= 0)
        return fail(MCUBES_E_DEVICE, "internal: tiles of item %u are not consecutive",
                    tiles[bad].item);
    for (int i = 0; i < B->n; ++i) {
        B->items[i].part_begin = pb[i];
        B->items[i].part_end = pe[i];
    }
    if (tiles.size() > B->cap_tiles) {
        (void)hipFree(B->d_tiles);
        (void)hipFree(B->d_partials);
        B->d_tiles = nullptr;
        B->d_partials = nullptr;
        const size_t cap = tiles.size() + tiles.size() / 4 + 64;
        int rc = device_alloc(B, &B->d_tiles, cap);
        if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_partials, 2 * cap);
        if (rc != MCUBES_OK) {
            B->cap_tiles = 0;
            return rc;
        }
        B->cap_tiles = cap;
    }
    hipError_t e = hipMemcpy(B->d_items, B->items.data(), B->items.size() * sizeof(BatchItem),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(B->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (batch plan)");
    B->plan = std::move(plan);
    B->planned = active;
    B->planned_samples = samples;
    B->ntiles = (int)tiles.size();
    assign_branches(B);
    return MCUBES_OK;
}

hipError_t launch_class(const mcubes_batch *B, const ClassPlan &c, bool frozen, hipStream_t s) {
    return c.launch[frozen ? 1 : 0](B->d_items, B->d_tiles + c.tile_off, c.ntiles, B->d_grids,
                                    B->d_bins, B->d_partials, B->d_iter, B->d_done, c.block, s);
}

// One iteration: [zero bins] -> V-Sample per class -> reduce -> combine ->
// [refine] -> advance the iteration counter.  `frozen` = no refinement.
// Every class's V-Sample, forked over the branches after the work already on
// s and joined back into s.
hipError_t enqueue_vsample(const mcubes_batch *B, bool frozen, hipStream_t s) {
    hipError_t e = hipSuccess;
    const int side = B->branches - 1;
    if (side > 0) e = hipEventRecord(B->fork, s);
    for (int k = 0; k < side && e == hipSuccess; ++k) e = hipStreamWaitEvent(B->side[k], B->fork, 0);
    for (const ClassPlan &c : B->plan)
        if (e == hipSuccess) e = launch_class(B, c, frozen, c.branch ? B->side[c.branch - 1] : s);
    for (int k = 0; k < side && e == hipSuccess; ++k) {
        e = hipEventRecord(B->join[k], B->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, B->join[k], 0);
    }
    return e;
}

hipError_t enqueue_iteration(const mcubes_batch *B, bool frozen, double rel_tol, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (!frozen) e = launch_fill(B->d_bins, B->bins_len, 0.0, s);
    if (e == hipSuccess) e = enqueue_vsample(B, frozen, s);
    if (e == hipSuccess) e = launch_batch_reduce(B->d_items, B->n, B->d_partials, B->d_done, B->d_est, s);
    if (e == hipSuccess)
        e = launch_batch_combine(B->n, B->d_est, B->d_states, B->d_done, B->d_done + B->n, B->d_iter,
                                 B->skip, rel_tol, s);
    if (e == hipSuccess && !frozen)
        e = launch_batch_refine(B->d_items, B->d_axes, (int)B->axes.size(), B->d_grids, B->d_bins,
                                B->d_states, B->d_iter, B->alpha, false, s);
    if (e == hipSuccess) e = launch_batch_advance(B->d_iter, s);
    return e;
}

int capture(mcubes_batch *B, bool frozen, double rel_tol) {
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const hipError_t el = enqueue_iteration(B, frozen, rel_tol, B->stream);
    e = hipStreamEndCapture(B->stream, &graph);
    if (el != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(el, "batch iteration launch (capture)");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&B->exec[frozen ? 1 : 0], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        B->exec[frozen ? 1 : 0] = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return MCUBES_OK;
}

// zero bins, one V-Sample per class, reduce, combine, refine, advance
int launches_per_iteration(const mcubes_batch *B) { return (int)B->plan.size() + 5; }

}  // namespace

extern "C" {

int mcubes_batch_create(const mcubes_batch_item *items, int n, uint64_t seed,
                        const mcubes_options *opt_in, mcubes_batch **out) {
    if (!out) return fail(MCUBES_E_ARG, "batch is NULL");
    if (!items) return fail(MCUBES_E_ARG, "items is NULL");
    if (n < 1 || n > 65536) return fail(MCUBES_E_ARG, "n must be in [1, 65536], got %d", n);
    mcubes_options opt;
    mcubes_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.nbins < 2 || opt.nbins > MCUBES_MAX_BINS)
        return fail(MCUBES_E_ARG, "nbins must be in [2, %d], got %d", MCUBES_MAX_BINS, opt.nbins);
    if (!(opt.alpha >= 0.0) || !isfinite(opt.alpha))
        return fail(MCUBES_E_ARG, "alpha must be finite and >= 0");
    if (opt.skip < 0) return fail(MCUBES_E_ARG, "skip must be >= 0");
    if (opt.block_size != 0 &&
        (opt.block_size < 64 || opt.block_size > kMaxBlock || opt.block_size % 64 != 0))
        return fail(MCUBES_E_ARG, "block_size must be 0 or a multiple of 64 in [64, %d]", kMaxBlock);
    if (opt.precision != MCUBES_FP64 && opt.precision != MCUBES_FP32)
        return fail(MCUBES_E_ARG, "precision must be MCUBES_FP64 or MCUBES_FP32");
    // validate every item before touching the device
    std::vector<int64_t> sizes(4 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const mcubes_batch_item &it = items[i];
        int rc = plan_sizes(it.dim, it.ncall, &sizes[4 * (size_t)i]);
        if (rc == MCUBES_OK) rc = validate_params(it.family, it.params, it.dim);
        if (rc == MCUBES_OK) rc = check_sizes(sizes[4 * (size_t)i + 1], sizes[4 * (size_t)i + 2], it.dim);
        if (rc != MCUBES_OK) {
            const std::string msg = mcubes_last_error();
            return fail(rc, "item %d: %s", i, msg.c_str());
        }
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    mcubes_batch *B = new (std::nothrow) mcubes_batch();
    if (!B) return fail(MCUBES_E_ALLOC, "out of host memory");
    e = hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        release(B);
        return hip_fail(e, "hipDeviceGetAttribute");
    }
    B->n = n;
    B->nb = opt.nbins;
    B->adapt_iters = opt.adapt_iters;
    B->skip = opt.skip;
    B->alpha = opt.alpha;
    B->forced_block = opt.block_size;
    B->prec = opt.precision == MCUBES_FP32 ? 1 : 0;
    B->user_stream = opt.stream;
    B->items.resize(n);
    B->family.resize(n);
    B->dim.resize(n);
    B->g.resize(n);
    B->m.resize(n);
    B->p.resize(n);
    int64_t goff = 0, boff = 0;
    for (int i = 0; i < n; ++i) {
        const mcubes_batch_item &it = items[i];
        const int64_t *sz = &sizes[4 * (size_t)i];
        B->family[i] = it.family;
        B->dim[i] = it.dim;
        B->g[i] = sz[0];
        B->m[i] = sz[1];
        B->p[i] = sz[2];
        BatchItem &bi = B->items[i];
        memset(&bi, 0, sizeof bi);
        make_args(it.family, it.params, it.dim, sz[0], sz[1], sz[2], B->nb, seed,
                  opt.stream_id + (uint32_t)i, bi.args);
        bi.grid_off = goff;
        bi.bins_off = boff;
        bi.dim = it.dim;
        bi.nb = B->nb;
        bi.n_samples = (double)sz[1] * (double)sz[2];
        bi.var_denom = (double)sz[2] * (double)sz[1] * (double)sz[1];
        goff += (int64_t)it.dim * (B->nb + 1);
        boff += (int64_t)it.dim * B->nb;
        for (int j = 0; j < it.dim; ++j) B->axes.push_back(make_uint2((unsigned)i, (unsigned)j));
    }
    B->grids_len = goff;
    B->bins_len = boff;
    int rc = device_alloc(B, &B->d_items, (size_t)n);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_grids, (size_t)B->grids_len);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_bins, (size_t)B->bins_len);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_est, 2 * (size_t)n);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_states, (size_t)n * MCUBES_STATE_LEN);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_done, (size_t)n + 1);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_iter, 1);
    if (rc == MCUBES_OK) rc = device_alloc(B, &B->d_axes, B->axes.size());
    if (rc != MCUBES_OK) {
        release(B);
        return rc;
    }
    e = hipHostMalloc((void **)&B->h_done, ((size_t)n + 1) * sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        B->h_done = nullptr;
        release(B);
        return fail(MCUBES_E_ALLOC, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
    for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipEventCreate(&B->ev[q]);
    for (int q = 0; q < kMaxStreams - 1 && e == hipSuccess; ++q) {
        e = hipStreamCreateWithFlags(&B->side[q], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->join[q], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpy(B->d_axes, B->axes.data(), B->axes.size() * sizeof(uint2),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(B);
        return hip_fail(e, "batch set-up");
    }
    rc = build_plan(B, std::vector<char>(n, 1));
    if (rc != MCUBES_OK) {
        release(B);
        return rc;
    }
    // uniform grids and a clean state, so that the autotuner can run at once
    e = launch_batch_init_grids(B->d_items, B->d_axes, (int)B->axes.size(), B->d_grids, B->stream);
    if (e == hipSuccess)
        e = launch_batch_reset(B->d_states, (int64_t)n * MCUBES_STATE_LEN, B->d_done, n, B->d_iter,
                               B->stream);
    if (e == hipSuccess) e = launch_fill(B->d_bins, B->bins_len, 0.0, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) {
        release(B);
        return hip_fail(e, "batch initialisation");
    }
    *out = B;
    return MCUBES_OK;
}

void mcubes_batch_destroy(mcubes_batch *B) {
    if (B) {
        // nothing of this batch may still run when its memory goes
        if (B->stream) (void)hipStreamSynchronize(B->stream);
        for (auto &q : B->side)
            if (q) (void)hipStreamSynchronize(q);
    }
    release(B);
}

int mcubes_batch_get_info(const mcubes_batch *B, mcubes_batch_info *info) {
    if (!B || !info) return fail(MCUBES_E_ARG, "NULL argument");
    info->items = B->n;
    info->classes = (int32_t)B->plan.size();
    info->tiles = B->ntiles;
    info->launches = launches_per_iteration(B);
    info->streams = B->streams;
    info->nbins = B->nb;
    info->tuned = B->tuned ? 1 : 0;
    info->precision = B->prec ? MCUBES_FP32 : MCUBES_FP64;
    info->grids_len = B->grids_len;
    info->samples_per_iter = B->planned_samples;
    info->device_bytes = (int64_t)B->device_bytes;
    info->last_iterations = B->last_iterations;
    info->last_replans = B->last_replans;
    info->last_samples = B->last_samples;
    info->last_ms = B->last_ms;
    return MCUBES_OK;
}

int mcubes_batch_get_class(const mcubes_batch *B, int k, mcubes_batch_class *out) {
    if (!B || !out) return fail(MCUBES_E_ARG, "NULL argument");
    if (k < 0 || k >= (int)B->plan.size())
        return fail(MCUBES_E_ARG, "class %d out of range [0, %zu)", k, B->plan.size());
    const ClassPlan &c = B->plan[k];
    out->family = c.key.family;
    out->dim = c.key.dim;
    out->p2 = c.key.p2;
    out->items = (int32_t)c.items.size();
    out->block_size = c.block;
    out->shares = c.blocks;
    out->tiles = c.ntiles;
    out->lds_bytes = (int32_t)c.lds;
    out->samples = c.samples;
    auto it = B->cfg.find(c.key);
    out->tuned_ms = it == B->cfg.end() ? 0.0 : it->second.tuned_ms;
    out->default_ms = it == B->cfg.end() ? 0.0 : it->second.default_ms;
    return MCUBES_OK;
}

int mcubes_batch_configure_class(mcubes_batch *B, int k, int block_size, int shares) {
    if (!B) return fail(MCUBES_E_ARG, "NULL argument");
    if (k < 0 || k >= (int)B->plan.size())
        return fail(MCUBES_E_ARG, "class %d out of range [0, %zu)", k, B->plan.size());
    const ClassPlan &c = B->plan[k];
    if (block_size < 64 || block_size > c.max_block || block_size % 64 != 0)
        return fail(MCUBES_E_ARG, "block_size must be a multiple of 64 in [64, %d]", c.max_block);
    if (shares < 1) return fail(MCUBES_E_ARG, "shares must be >= 1");
    ClassCfg &cf = B->cfg[c.key];
    cf.block = block_size;
    cf.blocks = shares;
    cf.tuned_ms = 0.0;
    cf.default_ms = 0.0;
    const int saved = B->forced_block;
    B->forced_block = 0;
    const std::vector<char> active = B->planned;
    const int rc = build_plan(B, active);
    B->forced_block = saved;
    return rc;
}

int mcubes_batch_set_streams(mcubes_batch *B, int streams) {
    if (!B) return fail(MCUBES_E_ARG, "NULL argument");
    if (streams < 1 || streams > kMaxStreams)
        return fail(MCUBES_E_ARG, "streams must be in [1, %d], got %d", kMaxStreams, streams);
    const hipError_t e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    B->streams = streams;
    assign_branches(B);
    drop_graphs(B);
    return MCUBES_OK;
}

int mcubes_batch_autotune(mcubes_batch *B) {
    if (!B) return fail(MCUBES_E_ARG, "NULL argument");
    hipError_t e = hipSuccess;
    if (B->user_stream) {
        e = hipEventRecord(B->ev[2], as_stream(B->user_stream));
        if (e == hipSuccess) e = hipStreamWaitEvent(B->stream, B->ev[2], 0);
        if (e != hipSuccess) return hip_fail(e, "stream ordering");
    }
    // tune every class, with no integrand marked done
    const std::vector<char> all(B->n, 1);
    if (B->planned != all) {
        const int prc = build_plan(B, all);
        if (prc != MCUBES_OK) return prc;
    }
    e = launch_batch_reset(B->d_states, (int64_t)B->n * MCUBES_STATE_LEN, B->d_done, B->n,
                           B->d_iter, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return hip_fail(e, "autotune set-up");
    static const int kBlocks[] = {256, 512, 768, 1024};
    static const int kCubesPerThread[] = {4, 16, 64};
    std::vector<BatchItem> items = B->items;  // step fields per candidate block size
    BatchItem *d_items = nullptr;
    BatchTile *d_tiles = nullptr;
    double *d_part = nullptr;
    size_t cap = 0;
    int rc = MCUBES_OK;
    if (hipMalloc((void **)&d_items, items.size() * sizeof(BatchItem)) != hipSuccess)
        return fail(MCUBES_E_ALLOC, "hipMalloc (autotune)");
    // times one candidate geometry of class c: warm-up, then the mean of two launches
    auto time_one = [&](const ClassPlan &c, int block, int shares, double *ms_out) -> int {
        for (int i : c.items) {
            VsArgs tmp = items[i].args;
            set_step(tmp, B->dim[i], (uint64_t)block);
            items[i].step_block = tmp.step;
            memcpy(items[i].step_digit_block, tmp.step_digit, sizeof tmp.step_digit);
        }
        std::vector<BatchTile> tiles;
        split_class(B, c, shares, tiles);
        if (tiles.size() > cap) {
            (void)hipFree(d_tiles);
            (void)hipFree(d_part);
            d_tiles = nullptr;
            d_part = nullptr;
            cap = tiles.size() + tiles.size() / 4 + 64;
            if (hipMalloc((void **)&d_tiles, cap * sizeof(BatchTile)) != hipSuccess ||
                hipMalloc((void **)&d_part, 2 * cap * sizeof(double)) != hipSuccess)
                return fail(MCUBES_E_ALLOC, "hipMalloc (autotune)");
        }
        hipError_t x = hipMemcpy(d_items, items.data(), items.size() * sizeof(BatchItem),
                                 hipMemcpyHostToDevice);
        if (x == hipSuccess)
            x = hipMemcpy(d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                          hipMemcpyHostToDevice);
        const int nt = (int)tiles.size();
        for (int r = 0; r < 3 && x == hipSuccess; ++r) {
            if (r == 1) x = hipEventRecord(B->ev[0], B->stream);
            if (x == hipSuccess)
                x = c.launch[0](d_items, d_tiles, nt, B->d_grids, B->d_bins, d_part, B->d_iter,
                                B->d_done, block, B->stream);
        }
        if (x == hipSuccess) x = hipEventRecord(B->ev[1], B->stream);
        if (x == hipSuccess) x = hipEventSynchronize(B->ev[1]);
        float ms = 0.0f;
        if (x == hipSuccess) x = hipEventElapsedTime(&ms, B->ev[0], B->ev[1]);
        if (x != hipSuccess) return hip_fail(x, "autotune launch");
        *ms_out = ms / 2.0;
        return MCUBES_OK;
    };
    for (const ClassPlan &c : B->plan) {
        double best_ms = -1.0, default_ms = 0.0;
        int best_block = 0, best_shares = 0;
        // the library's default geometry first
        const int dblock = B->forced_block ? std::min(B->forced_block, c.max_block / 64 * 64)
                                           : default_block(c);
        const int dshares = class_shares(B, c, dblock, 0);
        if (dshares >= 1) {
            rc = time_one(c, dblock, dshares, &default_ms);
            if (rc != MCUBES_OK) break;
            best_ms = default_ms;
            best_block = dblock;
            best_shares = dshares;
        }
        for (int bs : kBlocks) {
            if (bs > c.max_block || (B->forced_block && bs != B->forced_block)) continue;
            const int R = resident_blocks(B, c, bs);
            if (R < 1) continue;
            std::vector<int64_t> counts = {2 * (int64_t)R, 4 * (int64_t)R, 8 * (int64_t)R,
                                           16 * (int64_t)R};
            for (int cpt : kCubesPerThread) {
                const int64_t q = (c.cubes + (int64_t)bs * cpt - 1) / ((int64_t)bs * cpt);
                if (q < R) counts.push_back(q);
            }
            for (int64_t &q : counts) q = std::max<int64_t>(1, std::min<int64_t>(q, std::min<int64_t>(c.cubes, kMaxShares)));
            std::sort(counts.begin(), counts.end());
            counts.erase(std::unique(counts.begin(), counts.end()), counts.end());
            for (int64_t q : counts) {
                if (bs == dblock && q == dshares) continue;
                double ms = 0.0;
                rc = time_one(c, bs, (int)q, &ms);
                if (rc != MCUBES_OK) break;
                if (best_ms < 0.0 || ms < best_ms) {
                    best_ms = ms;
                    best_block = bs;
                    best_shares = (int)q;
                }
            }
            if (rc != MCUBES_OK) break;
        }
        if (rc != MCUBES_OK) break;
        if (best_ms < 0.0) {
            rc = fail(MCUBES_E_DEVICE, "no launch geometry fits class (family %d, dim %d)",
                      c.key.family, c.key.dim);
            break;
        }
        ClassCfg &cf = B->cfg[c.key];
        cf.block = best_block;
        cf.blocks = best_shares;
        cf.tuned_ms = best_ms;
        cf.default_ms = default_ms;
    }
    (void)hipFree(d_items);
    (void)hipFree(d_tiles);
    (void)hipFree(d_part);
    if (rc != MCUBES_OK) return rc;
    const int saved = B->forced_block;
    B->forced_block = 0;
    rc = build_plan(B, all);
    B->forced_block = saved;
    if (rc != MCUBES_OK) return rc;
    // number of concurrent streams for the class launches: the fastest of
    // 1, 2, 3, 4 over all classes (warm-up, then the mean of two)
    double best_ms = -1.0;
    int best_streams = 1;
    for (int ns = 1; ns <= kMaxStreams; ++ns) {
        B->streams = ns;
        assign_branches(B);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            if (r == 1) e = hipEventRecord(B->ev[0], B->stream);
            if (e == hipSuccess) e = enqueue_vsample(B, false, B->stream);
        }
        if (e == hipSuccess) e = hipEventRecord(B->ev[1], B->stream);
        if (e == hipSuccess) e = hipEventSynchronize(B->ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, B->ev[0], B->ev[1]);
        if (e != hipSuccess) return hip_fail(e, "autotune (streams)");
        if (best_ms < 0.0 || ms < best_ms) {
            best_ms = ms;
            best_streams = ns;
        }
    }
    B->streams = best_streams;
    assign_branches(B);
    drop_graphs(B);
    // the tuning launches added to the bin sums: start clean
    e = launch_fill(B->d_bins, B->bins_len, 0.0, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    B->tuned = true;
    return MCUBES_OK;
}

int mcubes_batch_step(mcubes_batch *B, uint32_t iteration, double *grids, double *est) {
    if (!B || !grids || !est) return fail(MCUBES_E_ARG, "NULL argument");
    if (iteration >= MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "iteration %u >= %d", iteration, MCUBES_MAX_ITERATIONS);
    // host-side check of the grids: the kernels assume monotone edges 0 .. 1
    const int64_t nb1 = B->nb + 1;
    for (int64_t r = 0; r < B->grids_len / nb1; ++r) {
        const double *row = grids + r * nb1;
        if (row[0] != 0.0 || row[B->nb] != 1.0)
            return fail(MCUBES_E_ARG, "grid row %lld must run from 0 to 1", (long long)r);
        for (int i = 0; i < B->nb; ++i)
            if (!(row[i + 1] >= row[i]))
                return fail(MCUBES_E_ARG, "grid row %lld is not monotone", (long long)r);
    }
    hipStream_t s = B->stream;
    hipError_t e = hipSuccess;
    if (B->user_stream) {
        e = hipEventRecord(B->ev[2], as_stream(B->user_stream));
        if (e == hipSuccess) e = hipStreamWaitEvent(s, B->ev[2], 0);
        if (e != hipSuccess) return hip_fail(e, "stream ordering");
    }
    const std::vector<char> all(B->n, 1);
    if (B->planned != all) {
        const int rc = build_plan(B, all);
        if (rc != MCUBES_OK) return rc;
    }
    e = launch_batch_reset(B->d_states, (int64_t)B->n * MCUBES_STATE_LEN, B->d_done, B->n,
                           B->d_iter, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->d_iter, &iteration, sizeof iteration, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->d_grids, grids, (size_t)B->grids_len * sizeof(double),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill(B->d_bins, B->bins_len, 0.0, s);
    if (e == hipSuccess) e = enqueue_vsample(B, false, s);
    if (e == hipSuccess) e = launch_batch_reduce(B->d_items, B->n, B->d_partials, B->d_done, B->d_est, s);
    if (e == hipSuccess)
        e = launch_batch_refine(B->d_items, B->d_axes, (int)B->axes.size(), B->d_grids, B->d_bins,
                                B->d_states, B->d_iter, B->alpha, true, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(est, B->d_est, 2 * (size_t)B->n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grids, B->d_grids, (size_t)B->grids_len * sizeof(double),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? MCUBES_OK : hip_fail(e, "batch step");
}

int mcubes_batch_integrate(mcubes_batch *B, int itmax, double rel_tol, int use_graph,
                           mcubes_result *results, double *grids_out, double *traces) {
    if (!B || !results) return fail(MCUBES_E_ARG, "NULL argument");
    if (itmax < 1 || itmax > MCUBES_MAX_ITERATIONS)
        return fail(MCUBES_E_ARG, "itmax must be in [1, %d]", MCUBES_MAX_ITERATIONS);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol))
        return fail(MCUBES_E_ARG, "rel_tol must be finite and >= 0");
    const int n = B->n;
    hipStream_t s = B->stream;
    hipError_t e = hipSuccess;
    int rc = MCUBES_OK;
    if (B->user_stream) {
        e = hipEventRecord(B->ev[2], as_stream(B->user_stream));
        if (e == hipSuccess) e = hipStreamWaitEvent(s, B->ev[2], 0);
        if (e != hipSuccess) return hip_fail(e, "stream ordering");
    }
    std::vector<char> active(n, 1);
    if (B->planned != active) {
        rc = build_plan(B, active);
        if (rc != MCUBES_OK) return rc;
    }
    // graphs bake rel_tol in: capture afresh for every call
    drop_graphs(B);
    e = launch_batch_init_grids(B->d_items, B->d_axes, (int)B->axes.size(), B->d_grids, s);
    if (e == hipSuccess)
        e = launch_batch_reset(B->d_states, (int64_t)n * MCUBES_STATE_LEN, B->d_done, n, B->d_iter, s);
    if (e != hipSuccess) return hip_fail(e, "batch reset");
    const int replans = 0;
    int iterations = 0;
    int64_t samples = 0, running = 0;
    for (int i = 0; i < n; ++i) running += B->m[i] * B->p[i];
    e = hipEventRecord(B->ev[0], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int t = 0; t < itmax; ++t) {
        const bool frozen = B->adapt_iters >= 0 && t >= B->adapt_iters;
        if (use_graph) {
            if (!B->exec[frozen ? 1 : 0]) {
                rc = capture(B, frozen, rel_tol);
                if (rc != MCUBES_OK) return rc;
            }
            e = hipGraphLaunch(B->exec[frozen ? 1 : 0], s);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        } else {
            e = enqueue_iteration(B, frozen, rel_tol, s);
            if (e != hipSuccess) return hip_fail(e, "batch iteration launch");
        }
        samples += running;  // integrands not done when iteration t starts
        iterations = t + 1;
        e = hipMemcpyAsync(B->h_done, B->d_done, ((size_t)n + 1) * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "batch flags");
        if (B->h_done[n] == 0u) break;
        // the tiles of finished integrands return at once; the plan (and the
        // captured graph) stays as it is for the whole call
        int64_t left = 0;
        for (int i = 0; i < n; ++i)
            if (B->h_done[i] == 0u) left += B->m[i] * B->p[i];
        running = left;
    }
    e = hipEventRecord(B->ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(B->ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, B->ev[0], B->ev[1]);
    if (e != hipSuccess) return hip_fail(e, "batch timing");
    std::vector<double> head((size_t)n * MCUBES_STATE_HEADER);
    e = hipMemcpy2D(head.data(), MCUBES_STATE_HEADER * sizeof(double), B->d_states,
                    MCUBES_STATE_LEN * sizeof(double), MCUBES_STATE_HEADER * sizeof(double), n,
                    hipMemcpyDeviceToHost);
    if (e == hipSuccess && traces)
        e = hipMemcpy2D(traces, 2 * (size_t)itmax * sizeof(double),
                        B->d_states + MCUBES_STATE_HEADER, MCUBES_STATE_LEN * sizeof(double),
                        2 * (size_t)itmax * sizeof(double), n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && grids_out)
        e = hipMemcpy(grids_out, B->d_grids, (size_t)B->grids_len * sizeof(double),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch results");
    int status = MCUBES_OK;
    for (int i = 0; i < n; ++i) {
        const double *h = &head[(size_t)i * MCUBES_STATE_HEADER];
        mcubes_result &r = results[i];
        r.estimate = h[0];
        r.error = h[1];
        r.chi2_dof = h[2];
        r.dof = (int32_t)h[3];
        r.iterations = (int32_t)h[4];
        r.converged = h[5] != 0.0;
        r.status = h[6] != 0.0 ? MCUBES_E_NONFINITE : (r.converged ? MCUBES_OK : MCUBES_NOT_CONVERGED);
        r.cube_side = B->g[i];
        r.ncubes = B->m[i];
        r.samples_per_cube = B->p[i];
        r.samples_per_iter = B->m[i] * B->p[i];
        r.kernel_ms = 0.0;
        if (r.status == MCUBES_E_NONFINITE)
            status = MCUBES_E_NONFINITE;
        else if (r.status == MCUBES_NOT_CONVERGED && status == MCUBES_OK)
            status = MCUBES_NOT_CONVERGED;
    }
    B->last_iterations = iterations;
    B->last_replans = replans;
    B->last_samples = samples;
    B->last_ms = ms;
    if (status == MCUBES_E_NONFINITE) fail(status, "some integrand produced a non-finite estimate");
    return status;
}

}  // extern "C"
