// Serving: weight-vector queries against registered formula structures, with
// continuous batching.
//
// Every registered structure is an unsliced plan.  A request (structure,
// weights) is admitted when a slot is free and a region of the device buffer
// large enough for its footprint (meta table + arena of its plan) is free:
// admission is by HBM footprint within a fixed budget.  The server advances
// in steps: one step runs, for every admitted request, the next launch of its
// plan (leaf fill for a newly admitted one), all merged into shared kernels
// (one k_nodes launch for the generic/streaming nodes of every request, one
// MFMA launch per matrix node).  A request that arrives while others are on
// the GPU joins at the next step; one that finishes frees its slot and
// region at once.  Each request's descriptors are its plan's, shifted into
// its region, so its arithmetic is the same alone or in any mix.
#include <chrono>
#include <deque>
#include <map>

#include "wmc_kernels.h"

namespace {

struct SStruct {
    int32_t n = 0;                // variables, auxiliary ones included
    int32_t n_user = 0;           // a request brings 2 * n_user weights
    std::vector<double> w_aux;    // (1, 1) per auxiliary variable
    std::vector<int> task_of;     // per node: index into tasks if it streams in merged steps, else -1
    std::vector<StreamTask> tasks;  // streaming arguments of those nodes (region offsets not yet added)
    std::vector<LeafDesc> leaves;
    std::vector<NodeDesc> nodes;
    std::vector<GemmDesc> gemms;
    std::vector<Launch> launches;
    int32_t root = -1;
    long long root_off = 0;
    int64_t nt = 0;
    uint64_t meta_bytes = 0, arena_bytes = 0, footprint = 0;
    int64_t leaf_work = 0;
    uint64_t max_step_bytes = 0;  // largest staging contribution of one launch
};

struct SReq {
    uint64_t id = 0;
    int32_t s = 0;
    int32_t slot = -1;
    uint64_t region = 0;
    size_t k = 0;
    std::vector<double> w;
    double t_arrive = 0, t_admit = 0;
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

static uint64_t sal(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

__global__ void k_clear_meta(const ClearRange *__restrict__ r, wmc_meta *meta) {
    const ClearRange c = r[blockIdx.x];
    for (long long i = threadIdx.x; i < c.count; i += blockDim.x) {
        meta[c.first + i].maxbits = 0ull;
        meta[c.first + i].exp = 0;
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
    uint64_t used_bytes = 0, peak_used = 0;
    int64_t peak_active = 0, steps = 0;
    uint8_t *stage[2] = {nullptr, nullptr};     // pinned staging, one per step parity
    ServeRes *res_host[2] = {nullptr, nullptr};  // pinned results, one per step parity
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool inflight = false;                       // a step was issued and not yet collected
    int parity = 0;                              // parity of the step in flight
    std::vector<SReq> finishing;                 // requests whose last launch is in flight
    std::vector<wmc_response> done;
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

extern "C" wmc_status wmc_serve_register(wmc_server *v, const wmc_plan_t *plan, int32_t *structure_id) {
    if (!v || !plan) {
        wmc_set_error("wmc_serve_register: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (plan->precision != v->opt.precision) {
        wmc_set_error("wmc_serve_register: plan precision differs from the server's");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (!plan->sliced.empty()) {
        wmc_set_error("wmc_serve_register: sliced plans are not served");
        return WMC_ERR_UNSUPPORTED;
    }
    try {
        SStruct s;
        s.n = plan->n;
        s.n_user = plan->n_user;
        s.w_aux.assign(plan->w.begin() + 2 * (size_t)plan->n_user, plan->w.end());
        s.leaves = plan->leaves;
        s.task_of.assign(plan->nodes.size(), -1);
        for (size_t q = 0; q < plan->nodes.size(); ++q) {
            const NodeDesc &d = plan->nodes[q];
            StreamTask t;
            if (d.rc >= plan->tune.multi_min_rank && d.cls != WMC_CLASS_GEMM && stream_task(d, &t)) {
                s.task_of[q] = (int)s.tasks.size();
                s.tasks.push_back(t);
            }
        }
        s.nodes = plan->nodes;
        s.gemms = plan->gemms;
        s.launches = plan->launches;
        s.root = plan->root;
        s.root_off = plan->root >= 0 ? plan->T[(size_t)plan->root].off : 0;
        s.nt = (int64_t)std::max<size_t>(plan->T.size(), 1);
        s.meta_bytes = sal(sizeof(wmc_meta) * (uint64_t)s.nt, 256);
        s.arena_bytes = sal(std::max<uint64_t>(plan->arena_bytes, 256), 256);
        s.footprint = s.meta_bytes + s.arena_bytes;
        s.leaf_work = plan->leaf_work;
        uint64_t mx = sal(sizeof(double) * 2 * (uint64_t)s.n, 8) + sizeof(ClearRange) +
                      sizeof(LeafDesc) * s.leaves.size() + sizeof(int) * ((uint64_t)s.leaf_work / WMC_WAVE + 1) +
                      sizeof(FinishEntry);
        for (size_t k = 1; k < s.launches.size(); ++k) {
            const Launch &L = s.launches[k];
            // descriptors, plus the lookup tables of the merged kernels (one
            // int per wave of small nodes and per streaming workgroup)
            uint64_t b = L.type == LAUNCH_GEMM
                             ? sizeof(GemmDesc)
                             : sizeof(NodeDesc) * (uint64_t)L.count +
                                   sizeof(int) * ((uint64_t)L.work / WMC_WAVE + (uint64_t)L.work / 4096 +
                                                  (uint64_t)L.count + 2);
            mx = std::max(mx, b + sizeof(FinishEntry));
        }
        s.max_step_bytes = mx + 8 * 256;
        if (s.footprint > v->regions_bytes || s.max_step_bytes > v->step_cap) {
            wmc_set_error("wmc_serve_register: structure needs %llu bytes of region and %llu of staging",
                          (unsigned long long)s.footprint, (unsigned long long)s.max_step_bytes);
            return WMC_ERR_CAP_UNREACHABLE;
        }
        v->S.push_back(std::move(s));
        if (structure_id) *structure_id = (int32_t)v->S.size() - 1;
    } catch (std::bad_alloc &) {
        wmc_set_error("wmc_serve_register: host allocation failed");
        return WMC_ERR_OUT_OF_MEMORY;
    }
    return WMC_OK;
}

static wmc_status serve_submit_at(wmc_server *v, int32_t structure, const double *weights, uint64_t request_id,
                                  double t_arrive) {
    if (structure < 0 || structure >= (int32_t)v->S.size()) {
        wmc_set_error("wmc_serve_submit: unknown structure %d", structure);
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if ((int64_t)v->queue.size() >= v->opt.max_queue) {
        wmc_set_error("wmc_serve_submit: queue full (%d)", v->opt.max_queue);
        return WMC_ERR_BUSY;
    }
    const SStruct &s = v->S[(size_t)structure];
    SReq r;
    r.id = request_id;
    r.s = structure;
    r.t_arrive = t_arrive;
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
        wmc_response resp;
        std::memset(&resp, 0, sizeof resp);
        resp.request_id = r.id;
        resp.structure = r.s;
        resp.status = WMC_OK;
        resp.value = s.root < 0 ? make_value(1.0, 0) : make_value(res[r.slot].m, res[r.slot].e);
        resp.t_arrive = r.t_arrive;
        resp.t_admit = r.t_admit;
        resp.t_done = t;
        v->done.push_back(resp);
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
        v->active.push_back(std::move(r));
        v->queue.pop_front();
    }
    if (v->active.empty()) return WMC_OK;
    v->peak_active = std::max<int64_t>(v->peak_active, (int64_t)v->active.size());

    std::vector<double> wts;
    std::vector<ClearRange> clears;
    std::vector<LeafDesc> leaves;
    std::vector<NodeDesc> nodes;
    std::vector<GemmDesc> gemms;
    std::vector<FinishEntry> fin;
    std::vector<StreamTask> by_nk[4];
    int64_t leaf_work = 0, node_work = 0;
    std::vector<SReq> keep;
    keep.reserve(v->active.size());
    for (size_t i = 0; i < v->active.size(); ++i) {
        SReq &r = v->active[i];
        const SStruct &s = v->S[(size_t)r.s];
        const long long mbase = (long long)(r.region / sizeof(wmc_meta));
        const long long abase = (long long)((r.region + s.meta_bytes) / elem);
        if (r.k == 0) {
            clears.push_back({mbase, s.nt});
            const int woff = (int)(wts.size() / 2);
            wts.insert(wts.end(), r.w.begin(), r.w.end());
            for (LeafDesc d : s.leaves) {
                d.out += abase;
                d.tensor += (int)mbase;
                if (d.kind != WMC_LEAF_CLAUSE) d.var += woff;
                d.work_begin = leaf_work;
                leaf_work += (int64_t)sal((uint64_t)1 << d.rank, WMC_WAVE);
                leaves.push_back(d);
            }
        } else {
            const Launch &L = s.launches[r.k];
            if (L.type == LAUNCH_GEMM) {
                GemmDesc g = s.gemms[(size_t)L.pad];
                g.a += abase;
                g.b += abase;
                g.c += abase;
                g.ta += (int)mbase;
                g.tb += (int)mbase;
                g.tc += (int)mbase;
                gemms.push_back(g);
            } else {
                for (int32_t q = 0; q < L.count; ++q) {
                    const int ti = s.task_of[(size_t)(L.first + q)];
                    if (ti >= 0) {  // streams: arguments precomputed at registration
                        StreamTask t = s.tasks[(size_t)ti];
                        t.a.s += abase;
                        t.a.o += abase;
                        t.a.c += abase;
                        t.a.ts += (int)mbase;
                        t.a.to += (int)mbase;
                        t.a.tc += (int)mbase;
                        by_nk[s.nodes[(size_t)(L.first + q)].nk].push_back(t);
                        continue;
                    }
                    NodeDesc d = s.nodes[(size_t)(L.first + q)];
                    d.a += abase;
                    d.b += abase;
                    d.c += abase;
                    d.ta += (int)mbase;
                    d.tb += (int)mbase;
                    d.tc += (int)mbase;
                    d.work_begin = node_work;
                    node_work += (int64_t)sal((uint64_t)1 << d.rc, WMC_WAVE);
                    nodes.push_back(d);
                }
            }
        }
        if (r.k + 1 >= s.launches.size()) {
            fin.push_back({s.root < 0 ? -1 : s.root + (int)mbase, r.slot, s.root_off + abase});
            finishing.push_back(std::move(r));
        } else {
            r.k += 1;
            keep.push_back(std::move(r));
        }
    }
    v->active.swap(keep);
    // big streaming nodes of the merged step run in the multi-node streaming
    // kernel, one launch per summed-index size
    std::vector<StreamTask> tasks;
    std::vector<int> nkf(5, 0);
    for (int k = 0; k < 4; ++k) {
        nkf[(size_t)k] = (int)tasks.size();
        long long blocks = 0;
        for (StreamTask &t : by_nk[k]) {
            t.block_begin = blocks;
            blocks += (long long)stream_task_blocks(t.a);
            tasks.push_back(t);
        }
    }
    nkf[4] = (int)tasks.size();
    std::vector<int> wtab, btab, ltab;
    wave_leaf_table(leaves, leaf_work, ltab);
    wave_node_table(nodes, node_work, wtab);
    block_task_table(tasks, nkf, btab);
    // staging image: [weights][clears][leaves][nodes][gemms][finish][tasks][tables]
    uint64_t o = 0;
    auto place = [&](size_t bytes) {
        uint64_t at = o;
        o = sal(o + bytes, 256);
        return at;
    };
    const uint64_t o_w = place(sizeof(double) * wts.size());
    const uint64_t o_c = place(sizeof(ClearRange) * clears.size());
    const uint64_t o_l = place(sizeof(LeafDesc) * leaves.size());
    const uint64_t o_n = place(sizeof(NodeDesc) * nodes.size());
    const uint64_t o_g = place(sizeof(GemmDesc) * gemms.size());
    const uint64_t o_f = place(sizeof(FinishEntry) * fin.size());
    const uint64_t o_t = place(sizeof(StreamTask) * tasks.size());
    const uint64_t o_lt = place(sizeof(int) * ltab.size());
    const uint64_t o_wt = place(sizeof(int) * wtab.size());
    const uint64_t o_bt = place(sizeof(int) * btab.size());
    if (o > v->step_cap) {
        wmc_set_error("wmc_serve: step staging overflow (%llu > %llu)", (unsigned long long)o,
                      (unsigned long long)v->step_cap);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    uint8_t *stage = v->stage[h];
    auto cp = [&](uint64_t at, const void *src, size_t bytes) {
        if (bytes) std::memcpy(stage + at, src, bytes);
    };
    cp(o_w, wts.data(), sizeof(double) * wts.size());
    cp(o_c, clears.data(), sizeof(ClearRange) * clears.size());
    cp(o_l, leaves.data(), sizeof(LeafDesc) * leaves.size());
    cp(o_n, nodes.data(), sizeof(NodeDesc) * nodes.size());
    cp(o_g, gemms.data(), sizeof(GemmDesc) * gemms.size());
    cp(o_f, fin.data(), sizeof(FinishEntry) * fin.size());
    cp(o_t, tasks.data(), sizeof(StreamTask) * tasks.size());
    cp(o_lt, ltab.data(), sizeof(int) * ltab.size());
    cp(o_wt, wtab.data(), sizeof(int) * wtab.size());
    cp(o_bt, btab.data(), sizeof(int) * btab.size());
    hipStream_t st = v->st;
    char *stp = v->dev + v->off_step + (uint64_t)h * v->step_cap;
    HIP_TRY(hipMemcpyAsync(stp, stage, o, hipMemcpyHostToDevice, st));
    wmc_meta *meta = (wmc_meta *)(v->dev + v->off_regions);
    T *arena = (T *)(v->dev + v->off_regions);
    if (!clears.empty())
        hipLaunchKernelGGL(k_clear_meta, dim3((unsigned)clears.size()), dim3(256), 0, st,
                           (const ClearRange *)(stp + o_c), meta);
    // leaf fills of newly admitted requests, small nodes and streaming tasks
    // of the others: independent work, one launch
    StepArgs a{};
    if (!tasks.empty())
        step_stream_part(a, (const StreamTask *)(stp + o_t), tasks.data(), nkf.data(), (const int *)(stp + o_bt));
    if (!nodes.empty()) {
        a.nodes = (const NodeDesc *)(stp + o_n);
        a.nnodes = (int)nodes.size();
        a.node_work = (long long)node_work;
        a.wave_node = (const int *)(stp + o_wt);
        a.nblocks = grid_for(node_work);
    }
    if (!leaves.empty()) {
        a.leaves = (const LeafDesc *)(stp + o_l);
        a.nleaves = (int)leaves.size();
        a.leaf_work = (long long)leaf_work;
        a.w = (const double *)(stp + o_w);
        a.wave_leaf = (const int *)(stp + o_lt);
        a.lblocks = grid_for(leaf_work);
    }
    launch_step<T>(a, arena, meta, st);
    for (size_t q = 0; q < gemms.size(); ++q)
        launch_gemm<T>(gemms[q], (const GemmDesc *)(stp + o_g) + q, arena, meta, st);
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
