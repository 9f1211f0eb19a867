// Serving: weight-vector queries against registered formula structures, with
// continuous batching.
//
// Every registered structure is a plan whose descriptors (leaves,
// nodes, streaming tasks, matrix nodes and the lookup tables of the merged
// kernels) are uploaded once, at registration, into the server's buffer and
// stay there.  A request (structure, weights) is admitted when a slot is
// free and a region of the buffer large enough for its footprint (meta table
// + arena of its plan) is free: admission is by HBM footprint within a fixed
// budget.  The server advances in steps: one step runs, for every admitted
// request, the next launch of its plan (leaf fill for a newly admitted one).
// A step uploads only one small work entry per request (its region's arena
// and meta offsets and where its launch's descriptors live) plus the weights
// of newly admitted requests; one fused kernel runs every request's leaf
// fill, small nodes and streaming tasks, each workgroup finding its request
// by a search over the entries' first workgroups, and matrix nodes run as
// their own launches on the request's shifted arena.  A request that arrives
// while others are on the GPU joins at the next step; one that finishes
// frees its slot and region.  Each request's descriptors are its plan's, read
// relative to its region, so its arithmetic is the same alone or in any mix.
// A request can be cancelled, or given a deadline; either ends it with
// WMC_ERR_CANCELLED.  A request on a sliced structure runs as one part per
// slice (Algorithm 3), each admitted, stepped and released like a request
// of its own with the slice's bits in its leaf fill; the parts' values are
// summed in slice order with the finish kernel's arithmetic once the last
// one is done, so the request's value is wmc_contract's.
#include <chrono>
#include <deque>
#include <map>

#include "wmc_kernels.h"

namespace {

// Where one launch of a registered structure keeps its resident descriptors
// (byte offsets into the server buffer).
struct SLaunch {
    int32_t type = LAUNCH_NODES;
    int32_t gemm = -1;                 // LAUNCH_GEMM: index into gemms
    uint64_t nodes_off = 0;            // generic nodes
    int32_t nnodes = 0;
    long long node_work = 0;
    uint64_t tasks_off = 0, btask_off = 0;  // streaming tasks (by nk) and their workgroup -> task table
    long long gblock[5] = {0, 0, 0, 0, 0};
    int32_t gtask[5] = {0, 0, 0, 0, 0};
    unsigned sblocks = 0;
    // per wave of the generic nodes: descriptor offset and first output
    std::vector<std::pair<uint64_t, int32_t>> waves;
    // per streaming workgroup: task descriptor offset, summed-index bits and
    // workgroup number (counted from the task group's start)
    struct Blk {
        uint64_t off;
        int32_t nk, blk;
    };
    std::vector<Blk> blocks;
};

struct SStruct {
    int32_t n = 0;                // variables, auxiliary ones included
    int32_t n_user = 0;           // a request brings 2 * n_user weights
    std::vector<double> w_aux;    // (1, 1) per auxiliary variable
    std::vector<GemmDesc> gemms;  // host copies (launch shapes); the device reads the resident ones
    GemmShape gemm_shape;         // from the plan's tuning table
    std::vector<SLaunch> L;       // per launch of the plan; L[0] is the leaf fill
    uint64_t img_off = 0, img_bytes = 0;   // resident image (offset into the region pool)
    uint64_t leaves_off = 0, gemms_off = 0;
    std::vector<std::pair<uint64_t, int32_t>> leaf_waves;  // per wave of the leaf fill
    int32_t nleaves = 0;
    int32_t root = -1;
    long long root_off = 0;
    int64_t nt = 0;
    uint64_t meta_bytes = 0, arena_bytes = 0, footprint = 0;
    int64_t leaf_work = 0;
    uint64_t max_step_bytes = 0;  // largest staging contribution of one request in one step
    int64_t nslices = 1;          // slices of the plan: parts per request
};

struct SReq {
    uint64_t id = 0;
    int32_t s = 0;
    int32_t slot = -1;
    uint64_t region = 0;
    size_t k = 0;
    std::vector<double> w;
    double t_arrive = 0, t_admit = 0;
    double deadline = 0;          // server clock, 0 = none
    bool cancelled = false;
    uint64_t slice = 0;           // sliced structures: this part's slice bits
    int64_t agg = -1;             // sliced structures: key of the request's parts record
};

// The parts of a request on a sliced structure: their values by slice,
// and how many are still to complete.
struct SAgg {
    uint64_t id = 0;
    int32_t s = 0;
    double t_arrive = 0, t_admit = -1;
    int64_t left = 0;
    bool cancelled = false;
    std::vector<double> m;
    std::vector<long long> e;
};

struct FinishEntry {
    int root_meta;
    int slot;
    long long root_off;
};

struct ClearRange {
    long long first;
    long long count;
};

}  // namespace

// One request's share of a fused serving step: its streaming workgroups
// [sb0, sb0 + sn) of the step's streaming part, its region's arena and meta
// offsets, its weights (leaf fill) and its launch's resident streaming
// tasks.
struct ServeWork {
    unsigned sb0, sn;
    long long abase, mbase;
    unsigned long long eta;  // slice bits of the request's part (sliced structures)
    const double *w;
    const StreamTask *tasks;
    const int *block_task;
    long long gblock[5];
    int gtask[5];
    int pad;
};

// One streaming workgroup of a step: the task's resident descriptor, its
// summed-index bits, the request's work entry and the workgroup's number
// within the task's group.
struct ServeBlock {
    const StreamTask *task;
    int entry, nk, blk, pad;
};

// One wave of a step's small-node or leaf part: the node's (leaf's)
// resident descriptor, the request's work entry and the wave's first
// output.  Waves of different requests share workgroups.
struct ServeWave {
    const void *desc;
    int entry;
    int item;
};

static uint64_t sal(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

__global__ void k_clear_meta(const ClearRange *__restrict__ r, wmc_meta *meta) {
    const ClearRange c = r[blockIdx.x];
    for (long long i = threadIdx.x; i < c.count; i += blockDim.x) {
        meta[c.first + i].maxbits = 0ull;
        meta[c.first + i].exp = 0;
    }
}

// A descriptor the host wrote before the launch, addressed through the
// constant address space so that the wave reads it with scalar loads, as it
// reads descriptors whose pointers are kernel arguments.
template <typename D>
__device__ __forceinline__ const __attribute__((address_space(4))) D *const_desc(const void *p) {
    return (const __attribute__((address_space(4))) D *)(unsigned long long)p;
}

// A step: workgroups [0, sblocks) run the streaming tasks (blocks[]), then
// workgroups of four waves run the nwaves
// small-node waves and the leaf waves after them (waves[]); padding waves
// at the end exit at once.
template <typename T>
__global__ void __launch_bounds__(256) k_step_serve(const ServeWork *__restrict__ work, const ServeBlock *__restrict__ blocks,
                                                    const ServeWave *__restrict__ waves, unsigned sblocks,
                                                    unsigned nwaves, unsigned lwaves, T *__restrict__ arena,
                                                    wmc_meta *meta) {
    const unsigned bx = blockIdx.x;
    if (bx >= sblocks) {
        // wave-uniform index, so that the record, the work entry and the
        // descriptor are read with scalar loads
        const unsigned wv = __builtin_amdgcn_readfirstlane(((bx - sblocks) << 2) | (threadIdx.x >> 6));
        if (wv >= nwaves + lwaves) return;
        const ServeWave &rec = waves[wv];
        const ServeWork &w = work[rec.entry];
        const unsigned long long lane = threadIdx.x & (WMC_WAVE - 1);
        if (wv < nwaves)
            node_item<T>(const_desc<NodeDesc>(rec.desc), (unsigned long long)rec.item + lane, arena + w.abase,
                         meta + w.mbase);
        else
            leaf_item<T>(const_desc<LeafDesc>(rec.desc), (long long)rec.item + (long long)lane, w.w, arena + w.abase,
                         meta + w.mbase, w.eta);
        return;
    }
    const ServeBlock &b = blocks[bx];
    const ServeWork &w = work[b.entry];
    T *ar = arena + w.abase;
    wmc_meta *me = meta + w.mbase;
    // the task is found directly: a one-task list whose first workgroup
    // number is the task's own
    const auto t = const_desc<StreamTask>(b.task);
    switch (b.nk) {
    case 0: stream_multi_body<T, 0>(t, 1, ar, me, nullptr, b.blk); break;
    case 1: stream_multi_body<T, 1>(t, 1, ar, me, nullptr, b.blk); break;
    case 2: stream_multi_body<T, 2>(t, 1, ar, me, nullptr, b.blk); break;
    default: stream_multi_body<T, 3>(t, 1, ar, me, nullptr, b.blk); break;
    }
}

struct ServeRes {
    double m;
    long long e;
};

template <typename T>
__global__ void k_finish_serve(const FinishEntry *__restrict__ f, int n, const T *__restrict__ arena,
                               const wmc_meta *meta, ServeRes *res) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FinishEntry e = f[i];
    if (e.root_meta < 0) {  // no variables and no clauses: the empty product
        res[e.slot].m = 0.5;
        res[e.slot].e = 1;
        return;
    }
    double v = (double)arena[e.root_off];
    long long ex = meta[e.root_meta].exp;
    if (v != 0.0) {
        int k;
        v = frexp(v, &k);
        ex += k;
    } else {
        ex = 0;
    }
    res[e.slot].m = v;
    res[e.slot].e = ex;
}

struct wmc_server {
    wmc_serve_options opt{};
    int32_t elem = 8;
    char *dev = nullptr;
    uint64_t dev_bytes = 0;
    hipStream_t st = nullptr;
    uint64_t off_step = 0, step_cap = 0, off_res = 0, off_regions = 0, regions_bytes = 0;
    std::vector<SStruct> S;
    std::deque<SReq> queue;
    std::vector<SReq> active;
    std::vector<int32_t> free_slots;
    std::map<uint64_t, uint64_t> free_regions;  // offset -> size
    uint64_t used_bytes = 0, peak_used = 0, structure_bytes = 0;
    int64_t queued_deadlines = 0;                // queued requests with a deadline
    double next_deadline = 0;                    // no queued deadline before this
    int64_t peak_active = 0, steps = 0;
    uint8_t *stage[2] = {nullptr, nullptr};     // pinned staging, one per step parity
    ServeRes *res_host[2] = {nullptr, nullptr};  // pinned results, one per step parity
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool inflight = false;                       // a step was issued and not yet collected
    int parity = 0;                              // parity of the step in flight
    std::vector<SReq> finishing;                 // requests whose last launch is in flight
    std::vector<wmc_response> done;
    std::map<int64_t, SAgg> aggs;                // requests on sliced structures with parts left
    int64_t next_agg = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    ~wmc_server() {
        if (inflight && ev[parity]) (void)hipEventSynchronize(ev[parity]);
        for (int i = 0; i < 2; ++i) {
            if (stage[i]) (void)hipHostFree(stage[i]);
            if (res_host[i]) (void)hipHostFree(res_host[i]);
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    }
};

extern "C" wmc_status wmc_serve_create(const wmc_serve_options *opts, void *device_buffer, uint64_t bytes,
                                       void *stream, wmc_server **out) {
    if (!out || !opts) {
        wmc_set_error("wmc_serve_create: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    *out = nullptr;
    if (!device_buffer || ((uintptr_t)device_buffer & 255u)) {
        wmc_set_error("wmc_serve_create: device buffer is NULL or not 256-byte aligned");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (opts->max_slots <= 0 || opts->max_queue <= 0 ||
        (opts->precision != WMC_FP64 && opts->precision != WMC_FP32_SCALED)) {
        wmc_set_error("wmc_serve_create: invalid options");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    // default staging per step: 64 MiB, or an eighth of a smaller buffer
    const uint64_t dflt = std::min<uint64_t>(64ull << 20, std::max<uint64_t>(1ull << 20, bytes / 8));
    const uint64_t step_cap = sal(opts->step_bytes ? opts->step_bytes : dflt, 256);
    const uint64_t res_bytes = sal(sizeof(ServeRes) * (uint64_t)opts->max_slots, 256);
    if (bytes < 2 * step_cap + res_bytes + 4096) {
        wmc_set_error("wmc_serve_create: device buffer too small (%llu bytes)", (unsigned long long)bytes);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    try {
        wmc_server *V = new wmc_server();
        V->opt = *opts;
        V->elem = opts->precision == WMC_FP64 ? 8 : 4;
        V->dev = (char *)device_buffer;
        V->dev_bytes = bytes;
        V->st = (hipStream_t)stream;
        V->off_step = 0;  // two halves of step_cap, one per step parity
        V->step_cap = step_cap;
        V->off_res = 2 * step_cap;
        V->off_regions = 2 * step_cap + res_bytes;
        V->regions_bytes = (bytes - V->off_regions) / 256 * 256;
        if (opts->hbm_budget_bytes && opts->hbm_budget_bytes < V->regions_bytes)
            V->regions_bytes = sal(opts->hbm_budget_bytes, 256);
        V->free_regions[0] = V->regions_bytes;
        for (int32_t s = opts->max_slots - 1; s >= 0; --s) V->free_slots.push_back(s);
        for (int i = 0; i < 2; ++i)
            if (hipHostMalloc((void **)&V->stage[i], step_cap, 0) != hipSuccess ||
                hipHostMalloc((void **)&V->res_host[i], res_bytes, 0) != hipSuccess ||
                hipEventCreateWithFlags(&V->ev[i], hipEventDisableTiming) != hipSuccess) {
                delete V;
                wmc_set_error("wmc_serve_create: pinned host allocation or event creation failed");
                return WMC_ERR_OUT_OF_MEMORY;
            }
        *out = V;
    } catch (std::bad_alloc &) {
        wmc_set_error("wmc_serve_create: host allocation failed");
        return WMC_ERR_OUT_OF_MEMORY;
    }
    return WMC_OK;
}

extern "C" void wmc_serve_destroy(wmc_server *v) { delete v; }

static bool region_alloc(wmc_server *v, uint64_t size, uint64_t *off) {
    for (auto it = v->free_regions.begin(); it != v->free_regions.end(); ++it) {
        if (it->second < size) continue;
        *off = it->first;
        uint64_t rest = it->second - size, roff = it->first + size;
        v->free_regions.erase(it);
        if (rest) v->free_regions[roff] = rest;
        v->used_bytes += size;
        v->peak_used = std::max(v->peak_used, v->used_bytes);
        return true;
    }
    return false;
}

static void region_free(wmc_server *v, uint64_t off, uint64_t size) {
    v->used_bytes -= size;
    auto it = v->free_regions.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != v->free_regions.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        v->free_regions.erase(nx);
    }
    if (it != v->free_regions.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            v->free_regions.erase(it);
        }
    }
}

// Registration builds the structure's resident image -- leaves and their
// wave table, matrix-node descriptors, and per node launch its generic nodes
// with their wave table and its streaming tasks (grouped by summed-index
// size) with their workgroup table -- and uploads it once into the region
// pool, where it stays for the server's life.
extern "C" wmc_status wmc_serve_register(wmc_server *v, const wmc_plan_t *plan, int32_t *structure_id) {
    if (!v || !plan) {
        wmc_set_error("wmc_serve_register: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (plan->precision != v->opt.precision) {
        wmc_set_error("wmc_serve_register: plan precision differs from the server's");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (plan->sliced.size() > 16) {
        wmc_set_error("wmc_serve_register: %zu sliced variables (at most 16 are served)", plan->sliced.size());
        return WMC_ERR_UNSUPPORTED;
    }
    try {
        SStruct s;
        s.n = plan->n;
        s.n_user = plan->n_user;
        s.w_aux.assign(plan->w.begin() + 2 * (size_t)plan->n_user, plan->w.end());
        s.gemms = plan->gemms;
        s.gemm_shape = GemmShape{plan->tune.gemm_tpw_max_nt, plan->tune.gemm_orient};
        s.root = plan->root;
        s.root_off = plan->root >= 0 ? plan->T[(size_t)plan->root].off : 0;
        s.nt = (int64_t)std::max<size_t>(plan->T.size(), 1);
        s.meta_bytes = sal(sizeof(wmc_meta) * (uint64_t)s.nt, 256);
        s.arena_bytes = sal(std::max<uint64_t>(plan->arena_bytes, 256), 256);
        s.footprint = s.meta_bytes + s.arena_bytes;
        s.leaf_work = plan->leaf_work;
        s.nleaves = (int32_t)plan->leaves.size();
        s.nslices = (int64_t)1 << plan->sliced.size();
        // image, offsets relative to its start
        std::vector<uint8_t> img;
        auto put = [&](const void *src, size_t bytes) {
            const uint64_t at = sal(img.size(), 256);
            img.resize(at + bytes);
            if (bytes) std::memcpy(img.data() + at, src, bytes);
            return at;
        };
        s.leaves_off = put(plan->leaves.data(), sizeof(LeafDesc) * plan->leaves.size());
        for (size_t q = 0; q < plan->leaves.size(); ++q)
            for (uint64_t e = 0; e < (1ull << plan->leaves[q].rank); e += WMC_WAVE)
                s.leaf_waves.push_back({s.leaves_off + sizeof(LeafDesc) * q, (int32_t)e});
        std::vector<int> tab;
        s.gemms_off = put(plan->gemms.data(), sizeof(GemmDesc) * plan->gemms.size());
        s.L.resize(plan->launches.size());
        for (size_t k = 1; k < plan->launches.size(); ++k) {
            const Launch &Ln = plan->launches[k];
            SLaunch &sl = s.L[k];
            sl.type = Ln.type;
            if (Ln.type == LAUNCH_GEMM) {
                sl.gemm = Ln.pad;
                continue;
            }
            std::vector<NodeDesc> generic(plan->nodes.begin() + Ln.first, plan->nodes.begin() + Ln.first + Ln.count);
            std::vector<StreamTask> tasks;
            std::vector<int> nkf;
            int64_t work = 0;
            split_stream(generic, tasks, nkf, work, plan->tune.multi_min_rank);
            sl.nnodes = (int32_t)generic.size();
            sl.node_work = work;
            sl.nodes_off = put(generic.data(), sizeof(NodeDesc) * generic.size());
            for (size_t q = 0; q < generic.size(); ++q)
                for (uint64_t e = 0; e < (1ull << generic[q].rc); e += WMC_WAVE)
                    sl.waves.push_back({sl.nodes_off + sizeof(NodeDesc) * q, (int32_t)e});
            sl.tasks_off = put(tasks.data(), sizeof(StreamTask) * tasks.size());
            block_task_table(tasks, nkf, tab);
            sl.btask_off = put(tab.data(), sizeof(int) * tab.size());
            unsigned long long blocks = 0;
            for (int q = 0; q < 4; ++q) {
                sl.gblock[q] = (long long)blocks;
                sl.gtask[q] = nkf[(size_t)q];
                blocks += stream_multi_blocks(tasks.data(), nkf[(size_t)q], nkf[(size_t)q + 1]);
            }
            sl.gblock[4] = (long long)blocks;
            sl.gtask[4] = nkf[4];
            sl.sblocks = (unsigned)blocks;
            for (int q = 0; q < 4; ++q)
                for (int t = nkf[(size_t)q]; t < nkf[(size_t)q + 1]; ++t) {
                    const long long b0 = tasks[(size_t)t].block_begin;
                    const long long nb = (long long)stream_task_blocks(tasks[(size_t)t].a);
                    for (long long b = 0; b < nb; ++b)
                        sl.blocks.push_back({sl.tasks_off + sizeof(StreamTask) * (uint64_t)t, q, (int32_t)(b0 + b)});
                }
        }
        s.img_bytes = sal(std::max<uint64_t>(img.size(), 256), 256);
        // staging per request and step: its weights (first step), a work
        // entry, a clear range or a finish entry
        uint64_t units = sizeof(ServeWave) * s.leaf_waves.size();
        for (const SLaunch &sl : s.L)
            units = std::max<uint64_t>(units, sizeof(ServeBlock) * sl.sblocks + sizeof(ServeWave) * sl.waves.size());
        s.max_step_bytes = sal(sizeof(double) * 2 * (uint64_t)s.n, 256) + sizeof(ServeWork) + sizeof(ClearRange) +
                           sizeof(FinishEntry) + units + 6 * 256;
        if (s.footprint > v->regions_bytes || s.max_step_bytes > v->step_cap) {
            wmc_set_error("wmc_serve_register: structure needs %llu bytes of region and %llu of staging",
                          (unsigned long long)s.footprint, (unsigned long long)s.max_step_bytes);
            return WMC_ERR_CAP_UNREACHABLE;
        }
        const uint64_t peak = v->peak_used;
        if (!region_alloc(v, s.img_bytes, &s.img_off)) {
            wmc_set_error("wmc_serve_register: no room for the structure's %llu bytes of descriptors",
                          (unsigned long long)s.img_bytes);
            return WMC_ERR_OUT_OF_MEMORY;
        }
        // descriptors are resident: they leave the budget for requests
        v->used_bytes -= s.img_bytes;
        v->peak_used = peak;
        v->structure_bytes += s.img_bytes;
        if (v->inflight) HIP_TRY(hipEventSynchronize(v->ev[v->parity]));
        HIP_TRY(hipMemcpyAsync(v->dev + v->off_regions + s.img_off, img.data(), img.size(), hipMemcpyHostToDevice,
                               v->st));
        HIP_TRY(hipStreamSynchronize(v->st));
        v->S.push_back(std::move(s));
        if (structure_id) *structure_id = (int32_t)v->S.size() - 1;
    } catch (std::bad_alloc &) {
        wmc_set_error("wmc_serve_register: host allocation failed");
        return WMC_ERR_OUT_OF_MEMORY;
    }
    return WMC_OK;
}

static wmc_status serve_submit_at(wmc_server *v, int32_t structure, const double *weights, uint64_t request_id,
                                  double t_arrive, double deadline = 0.0) {
    if (structure < 0 || structure >= (int32_t)v->S.size()) {
        wmc_set_error("wmc_serve_submit: unknown structure %d", structure);
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const SStruct &s = v->S[(size_t)structure];
    if ((int64_t)v->queue.size() + s.nslices > v->opt.max_queue) {
        wmc_set_error("wmc_serve_submit: queue full (%d)", v->opt.max_queue);
        return WMC_ERR_BUSY;
    }
    SReq r;
    r.id = request_id;
    r.s = structure;
    r.t_arrive = t_arrive;
    r.deadline = deadline;
    if (s.n_user > 0) {
        if (!weights) {
            wmc_set_error("wmc_serve_submit: weights are NULL");
            return WMC_ERR_INVALID_ARGUMENT;
        }
        r.w.assign(weights, weights + 2 * (size_t)s.n_user);
        for (double x : r.w)
            if (!std::isfinite(x)) {
                wmc_set_error("wmc_serve_submit: non-finite weight");
                return WMC_ERR_INVALID_ARGUMENT;
            }
    }
    r.w.insert(r.w.end(), s.w_aux.begin(), s.w_aux.end());
    if (deadline > 0.0) {
        v->next_deadline = v->queued_deadlines ? std::min(v->next_deadline, deadline) : deadline;
        v->queued_deadlines += s.nslices;
    }
    if (s.nslices > 1) {
        SAgg a;
        a.id = request_id;
        a.s = structure;
        a.t_arrive = t_arrive;
        a.left = s.nslices;
        a.m.assign((size_t)s.nslices, 0.0);
        a.e.assign((size_t)s.nslices, 0);
        r.agg = v->next_agg++;
        v->aggs.emplace(r.agg, std::move(a));
        for (int64_t q = 0; q < s.nslices; ++q) {
            SReq part = r;
            part.slice = (uint64_t)q;
            v->queue.push_back(std::move(part));
        }
        return WMC_OK;
    }
    v->queue.push_back(std::move(r));
    return WMC_OK;
}

extern "C" wmc_status wmc_serve_submit(wmc_server *v, int32_t structure, const double *weights,
                                       uint64_t request_id) {
    if (!v) {
        wmc_set_error("wmc_serve_submit: server is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    return serve_submit_at(v, structure, weights, request_id, v->now());
}

extern "C" wmc_status wmc_serve_submit_deadline(wmc_server *v, int32_t structure, const double *weights,
                                                uint64_t request_id, double timeout_s) {
    if (!v) {
        wmc_set_error("wmc_serve_submit_deadline: server is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (!(timeout_s > 0.0) || !std::isfinite(timeout_s)) {
        wmc_set_error("wmc_serve_submit_deadline: timeout must be positive and finite");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const double t = v->now();
    return serve_submit_at(v, structure, weights, request_id, t, t + timeout_s);
}

// A request (or one part of a request on a sliced structure) is done:
// with its value (m * 2^e) or cancelled.  A request answers once: a sliced
// one when its last part is done, cancelled if any part was.
static void complete(wmc_server *v, const SReq &r, bool ok, double m, long long e) {
    wmc_response resp;
    std::memset(&resp, 0, sizeof resp);
    resp.request_id = r.id;
    resp.structure = r.s;
    resp.t_arrive = r.t_arrive;
    resp.t_admit = r.t_admit;
    resp.t_done = v->now();
    if (r.agg < 0) {
        resp.status = ok ? WMC_OK : WMC_ERR_CANCELLED;
        resp.value = ok ? make_value(m, e) : make_value(0.0, 0);
        v->done.push_back(resp);
        return;
    }
    auto it = v->aggs.find(r.agg);
    if (it == v->aggs.end()) return;
    SAgg &a = it->second;
    if (ok) {
        a.m[(size_t)r.slice] = m;
        a.e[(size_t)r.slice] = e;
    } else {
        a.cancelled = true;
    }
    if (r.t_admit > 0 && (a.t_admit < 0 || r.t_admit < a.t_admit)) a.t_admit = r.t_admit;
    if (--a.left > 0) return;
    resp.t_arrive = a.t_arrive;
    resp.t_admit = a.t_admit < 0 ? 0.0 : a.t_admit;
    if (a.cancelled) {
        resp.status = WMC_ERR_CANCELLED;
        resp.value = make_value(0.0, 0);
    } else {
        SliceSum acc;  // slice order, as the solo executor sums them
        for (size_t q = 0; q < a.m.size(); ++q) acc.add(a.m[q], a.e[q]);
        resp.status = WMC_OK;
        resp.value = (acc.s == 0.0 && acc.c == 0.0) ? make_value(0.0, 0) : make_value(acc.s + acc.c, acc.e);
    }
    v->done.push_back(resp);
    v->aggs.erase(it);
}

static void respond_cancelled(wmc_server *v, const SReq &r) { complete(v, r, false, 0.0, 0); }

extern "C" wmc_status wmc_serve_cancel(wmc_server *v, uint64_t request_id) {
    if (!v) {
        wmc_set_error("wmc_serve_cancel: server is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    // every part of the request (one unless its structure is sliced)
    bool found = false;
    for (auto it = v->queue.begin(); it != v->queue.end();) {
        if (it->id == request_id) {
            respond_cancelled(v, *it);
            if (it->deadline > 0.0) --v->queued_deadlines;
            it = v->queue.erase(it);
            found = true;
            continue;
        }
        ++it;
    }
    for (SReq &r : v->active)
        if (r.id == request_id && !r.cancelled) {
            r.cancelled = true;  // released once no step in flight can touch its region
            found = true;
        }
    if (found) return WMC_OK;
    wmc_set_error("wmc_serve_cancel: request %llu is not queued or running", (unsigned long long)request_id);
    return WMC_ERR_INVALID_ARGUMENT;
}

// Collect the step in flight: wait for it, publish its finished requests and
// release their slots and regions.
static wmc_status serve_collect(wmc_server *v) {
    if (!v->inflight) return WMC_OK;
    HIP_TRY(hipEventSynchronize(v->ev[v->parity]));
    v->inflight = false;
    const double t = v->now();
    const ServeRes *res = v->res_host[v->parity];
    for (SReq &r : v->finishing) {
        const SStruct &s = v->S[(size_t)r.s];
        if (r.cancelled) {
            respond_cancelled(v, r);
            region_free(v, r.region, s.footprint);
            v->free_slots.push_back(r.slot);
            continue;
        }
        (void)t;
        if (s.root < 0) complete(v, r, true, 0.5, 1);  // the empty product: 1
        else complete(v, r, true, res[r.slot].m, res[r.slot].e);
        region_free(v, r.region, s.footprint);
        v->free_slots.push_back(r.slot);
    }
    v->finishing.clear();
    return WMC_OK;
}

// Issue one step: admit what fits, run the next launch of every admitted
// request in shared kernels.  Requests issuing their last launch move to the
// finishing list; their slot and region are released when the step is
// collected (after the next step has been issued, so host preparation of step
// k+1 overlaps the GPU running step k).
template <typename T>
static wmc_status serve_issue_t(wmc_server *v, int h, std::vector<SReq> &finishing, bool *issued) {
    *issued = false;
    const uint64_t elem = (uint64_t)v->elem;
    const double tnow = v->now();
    // deadlines: queued requests past theirs end at once (the queue is
    // scanned only once the earliest queued deadline has passed), running
    // ones like a cancellation
    if (v->queued_deadlines > 0 && tnow > v->next_deadline) {
        v->queued_deadlines = 0;
        for (auto it = v->queue.begin(); it != v->queue.end();) {
            if (it->deadline > 0.0 && tnow > it->deadline) {
                respond_cancelled(v, *it);
                it = v->queue.erase(it);
                continue;
            }
            if (it->deadline > 0.0) {
                v->next_deadline = v->queued_deadlines ? std::min(v->next_deadline, it->deadline) : it->deadline;
                ++v->queued_deadlines;
            }
            ++it;
        }
    }
    for (SReq &r : v->active)
        if (r.deadline > 0.0 && tnow > r.deadline) r.cancelled = true;
    uint64_t stage_need = 0;
    for (const SReq &r : v->active) stage_need += v->S[(size_t)r.s].max_step_bytes;
    while (!v->queue.empty() && !v->free_slots.empty()) {
        SReq &r = v->queue.front();
        const SStruct &s = v->S[(size_t)r.s];
        if (stage_need + s.max_step_bytes > v->step_cap) break;
        uint64_t off;
        if (!region_alloc(v, s.footprint, &off)) break;
        r.region = off;
        r.slot = v->free_slots.back();
        v->free_slots.pop_back();
        r.k = 0;
        r.t_admit = v->now();
        stage_need += s.max_step_bytes;
        if (r.deadline > 0.0) --v->queued_deadlines;  // next_deadline stays a lower bound
        v->active.push_back(std::move(r));
        v->queue.pop_front();
    }
    if (v->active.empty()) return WMC_OK;
    v->peak_active = std::max<int64_t>(v->peak_active, (int64_t)v->active.size());

    // staging image: [weights][clears][work entries][finish entries]; the
    // work entries point into the staging half this step uploads to
    char *stp = v->dev + v->off_step + (uint64_t)h * v->step_cap;
    const char *img = v->dev + v->off_regions;
    std::vector<double> wts;
    std::vector<ClearRange> clears;
    std::vector<ServeWork> works;
    std::vector<long long> work_woff;  // weight offset (doubles) of each work entry's leaf fill, or -1
    struct GemmCall {
        const GemmDesc *host;
        const GemmDesc *dev;
        long long abase, mbase;
        GemmShape shape;
    };
    std::vector<GemmCall> gemms;
    std::vector<FinishEntry> fin;
    std::vector<ServeBlock> sblk;      // streaming workgroups
    std::vector<ServeWave> node_waves, leaf_waves;
    unsigned sblocks = 0;
    std::vector<SReq> keep;
    keep.reserve(v->active.size());
    for (size_t i = 0; i < v->active.size(); ++i) {
        SReq &r = v->active[i];
        const SStruct &s = v->S[(size_t)r.s];
        if (r.cancelled) {  // no further launches; released after the steps in flight
            finishing.push_back(std::move(r));
            continue;
        }
        const long long mbase = (long long)(r.region / sizeof(wmc_meta));
        const long long abase = (long long)((r.region + s.meta_bytes) / elem);
        const char *base = img + s.img_off;
        const int entry = (int)works.size();
        ServeWork w;
        std::memset(&w, 0, sizeof w);
        w.abase = abase;
        w.mbase = mbase;
        w.eta = r.slice;
        long long woff = -1;
        bool used = false;
        if (r.k == 0) {
            clears.push_back({mbase, s.nt});
            woff = (long long)wts.size();
            wts.insert(wts.end(), r.w.begin(), r.w.end());
            for (const auto &x : s.leaf_waves) leaf_waves.push_back({base + x.first, entry, x.second});
            used = !s.leaf_waves.empty();
        } else {
            const SLaunch &L = s.L[r.k];
            if (L.type == LAUNCH_GEMM) {
                gemms.push_back({&s.gemms[(size_t)L.gemm], (const GemmDesc *)(base + s.gemms_off) + L.gemm, abase, mbase,
                                 s.gemm_shape});
            } else {
                if (L.sblocks) {
                    w.tasks = (const StreamTask *)(base + L.tasks_off);
                    w.block_task = (const int *)(base + L.btask_off);
                    for (int q = 0; q < 5; ++q) {
                        w.gblock[q] = L.gblock[q];
                        w.gtask[q] = L.gtask[q];
                    }
                    w.sn = L.sblocks;
                    w.sb0 = sblocks;
                    sblocks += L.sblocks;
                    for (const SLaunch::Blk &x : L.blocks)
                        sblk.push_back({(const StreamTask *)(base + x.off), entry, x.nk, x.blk, 0});
                }
                for (const auto &x : L.waves) node_waves.push_back({base + x.first, entry, x.second});
                used = L.sblocks > 0 || !L.waves.empty();
            }
        }
        if (used) {
            works.push_back(w);
            work_woff.push_back(woff);
        }
        if (r.k + 1 >= s.L.size()) {
            fin.push_back({s.root < 0 ? -1 : s.root + (int)mbase, r.slot, s.root_off + abase});
            finishing.push_back(std::move(r));
        } else {
            r.k += 1;
            keep.push_back(std::move(r));
        }
    }
    v->active.swap(keep);
    const unsigned nwaves = (unsigned)node_waves.size(), lwaves = (unsigned)leaf_waves.size();
    node_waves.insert(node_waves.end(), leaf_waves.begin(), leaf_waves.end());
    uint64_t o = 0;
    auto place = [&](size_t bytes) {
        uint64_t at = o;
        o = sal(o + bytes, 256);
        return at;
    };
    const uint64_t o_w = place(sizeof(double) * wts.size());
    const uint64_t o_c = place(sizeof(ClearRange) * clears.size());
    const uint64_t o_k = place(sizeof(ServeWork) * works.size());
    const uint64_t o_b = place(sizeof(ServeBlock) * sblk.size());
    const uint64_t o_v = place(sizeof(ServeWave) * node_waves.size());
    const uint64_t o_f = place(sizeof(FinishEntry) * fin.size());
    if (o > v->step_cap) {
        wmc_set_error("wmc_serve: step staging overflow (%llu > %llu)", (unsigned long long)o,
                      (unsigned long long)v->step_cap);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    for (size_t q = 0; q < works.size(); ++q)
        if (work_woff[q] >= 0) works[q].w = (const double *)(stp + o_w) + work_woff[q];
    uint8_t *stage = v->stage[h];
    auto cp = [&](uint64_t at, const void *src, size_t bytes) {
        if (bytes) std::memcpy(stage + at, src, bytes);
    };
    cp(o_w, wts.data(), sizeof(double) * wts.size());
    cp(o_c, clears.data(), sizeof(ClearRange) * clears.size());
    cp(o_k, works.data(), sizeof(ServeWork) * works.size());
    cp(o_b, sblk.data(), sizeof(ServeBlock) * sblk.size());
    cp(o_v, node_waves.data(), sizeof(ServeWave) * node_waves.size());
    cp(o_f, fin.data(), sizeof(FinishEntry) * fin.size());
    hipStream_t st = v->st;
    if (o) HIP_TRY(hipMemcpyAsync(stp, stage, o, hipMemcpyHostToDevice, st));
    wmc_meta *meta = (wmc_meta *)(v->dev + v->off_regions);
    T *arena = (T *)(v->dev + v->off_regions);
    if (!clears.empty())
        hipLaunchKernelGGL(k_clear_meta, dim3((unsigned)clears.size()), dim3(256), 0, st,
                           (const ClearRange *)(stp + o_c), meta);
    const unsigned wblocks = (nwaves + lwaves + 3) / 4;
    if (sblocks + wblocks)
        hipLaunchKernelGGL(k_step_serve<T>, dim3(sblocks + wblocks), dim3(256), 0, st, (const ServeWork *)(stp + o_k),
                           (const ServeBlock *)(stp + o_b), (const ServeWave *)(stp + o_v), sblocks, nwaves, lwaves, arena,
                           meta);
    for (const GemmCall &g : gemms)
        launch_gemm<T>(*g.host, g.dev, arena + g.abase, meta + g.mbase, st, SliceGroup{0, 0, 0}, 1, g.shape);
    ServeRes *res = (ServeRes *)(v->dev + v->off_res);
    if (!fin.empty()) {
        hipLaunchKernelGGL(k_finish_serve<T>, dim3((unsigned)((fin.size() + 255) / 256)), dim3(256), 0, st,
                           (const FinishEntry *)(stp + o_f), (int)fin.size(), arena, meta, res);
        HIP_TRY(hipMemcpyAsync(v->res_host[h], res, sizeof(ServeRes) * (size_t)v->opt.max_slots,
                               hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(v->ev[h], st));
    ++v->steps;
    *issued = true;
    return WMC_OK;
}

// One call: issue the next step into the staging half not used by the step in
// flight, then collect the step in flight.
template <typename T>
static wmc_status serve_step_t(wmc_server *v) {
    std::vector<SReq> fin_now;
    const int h = v->parity ^ 1;
    bool issued = false;
    wmc_status st = serve_issue_t<T>(v, h, fin_now, &issued);
    if (st != WMC_OK) return st;
    st = serve_collect(v);
    if (st != WMC_OK) return st;
    if (issued) {
        v->parity = h;
        v->inflight = true;
        v->finishing.swap(fin_now);
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_serve_step(wmc_server *v, int32_t *n_active, int32_t *n_queued) {
    if (!v) {
        wmc_set_error("wmc_serve_step: server is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    wmc_status s = v->elem == 8 ? serve_step_t<double>(v) : serve_step_t<float>(v);
    // requests whose last launch is still in flight count as active
    if (n_active) *n_active = (int32_t)(v->active.size() + v->finishing.size());
    if (n_queued) *n_queued = (int32_t)v->queue.size();
    return s;
}

extern "C" wmc_status wmc_serve_poll(wmc_server *v, wmc_response *out, int32_t max, int32_t *n_out) {
    if (!v || (!out && max > 0)) {
        wmc_set_error("wmc_serve_poll: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    int32_t n = (int32_t)std::min<size_t>((size_t)std::max(max, 0), v->done.size());
    for (int32_t i = 0; i < n; ++i) out[i] = v->done[(size_t)i];
    v->done.erase(v->done.begin(), v->done.begin() + n);
    if (n_out) *n_out = n;
    return WMC_OK;
}

extern "C" wmc_status wmc_serve_wait(wmc_server *v, wmc_response *out, int32_t max, int32_t *n_out,
                                      int64_t timeout_us) {
    if (!v || (!out && max > 0)) {
        wmc_set_error("wmc_serve_wait: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const double t_end = v->now() + (double)std::max<int64_t>(timeout_us, 0) * 1e-6;
    while (v->done.empty() && (!v->active.empty() || !v->queue.empty() || v->inflight) && v->now() < t_end) {
        const wmc_status st = wmc_serve_step(v, nullptr, nullptr);
        if (st != WMC_OK) return st;
    }
    return wmc_serve_poll(v, out, max, n_out);
}

extern "C" wmc_status wmc_serve_stats(const wmc_server *v, wmc_serve_info *out) {
    if (!v || !out) {
        wmc_set_error("wmc_serve_stats: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    std::memset(out, 0, sizeof *out);
    out->region_bytes = v->regions_bytes;
    out->used_bytes = v->used_bytes;
    out->peak_used_bytes = v->peak_used;
    out->peak_active = v->peak_active;
    out->steps = v->steps;
    out->n_active = (int64_t)(v->active.size() + v->finishing.size());
    out->n_queued = (int64_t)v->queue.size();
    out->n_structures = (int64_t)v->S.size();
    return WMC_OK;
}

// Replay a trace of timed arrivals: requests are submitted when the wall
// clock passes their arrival offset, and the server steps while any work is
// admitted or queued.  Responses come back in completion order with arrival,
// admission and completion times (seconds from the start of the replay).
extern "C" wmc_status wmc_serve(wmc_server *v, const wmc_request *trace, int64_t n, wmc_response *out) {
    if (!v || (n > 0 && (!trace || !out))) {
        wmc_set_error("wmc_serve: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    for (int64_t i = 1; i < n; ++i)
        if (trace[i].t_arrive < trace[i - 1].t_arrive) {
            wmc_set_error("wmc_serve: trace not sorted by arrival time");
            return WMC_ERR_INVALID_ARGUMENT;
        }
    v->t0 = std::chrono::steady_clock::now();
    int64_t next = 0, got = 0;
    while (got < n) {
        const double t = v->now();
        while (next < n && trace[next].t_arrive <= t) {
            wmc_status s = serve_submit_at(v, trace[next].structure, trace[next].weights, trace[next].request_id,
                                           trace[next].t_arrive);
            if (s == WMC_ERR_BUSY) break;
            if (s != WMC_OK) return s;
            ++next;
        }
        if (v->active.empty() && v->queue.empty() && !v->inflight) {
            if (next < n) {
                // idle until the next arrival
                while (v->now() < trace[next].t_arrive) {
                }
            }
            continue;
        }
        int32_t na, nq;
        wmc_status s = wmc_serve_step(v, &na, &nq);
        if (s != WMC_OK) return s;
        int32_t k = 0;
        wmc_serve_poll(v, out + got, (int32_t)std::min<int64_t>(n - got, 1 << 30), &k);
        got += k;
    }
    return WMC_OK;
}
