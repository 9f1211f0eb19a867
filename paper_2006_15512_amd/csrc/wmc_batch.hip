// Batched execution of many planned networks (many small formulas, or one
// structure with many weight vectors) in shared launches.
//
// A sliced plan (Algorithm 3) enters as one instance per slice: the slices
// share the plan's descriptors and weights, each has its own arena region
// and meta entries, and its leaves read the slice's bits from a per-leaf
// table.  The slices' roots are folded per plan on the host, in slice order,
// with the same compensated sum as the solo executor's finish kernel.
//
// Launch k of one plan depends only on that plan's launches < k, so launch k
// of every instance can run in the same kernel.  The batch concatenates the
// instances' leaf and node descriptors (offsets patched into one arena, one
// meta table and one weight vector), merges their launch lists by index,
// runs every generic or streaming node of a merged step in one k_nodes
// launch and every matrix node in its own MFMA launch, and finishes all
// roots with one kernel.  The whole sequence can be captured once as a HIP
// graph and replayed.
#include <array>
#include <mutex>

#include "wmc_kernels.h"

struct BatchRes {
    double m;
    long long e;
};


template <typename T>
__global__ void k_finish_batch(const T *__restrict__ arena, const long long *__restrict__ root_off,
                               const int *__restrict__ root, const wmc_meta *meta, int n, BatchRes *out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (root[i] < 0) {  // no variables and no clauses: the empty product
        out[i].m = 0.5;
        out[i].e = 1;
        return;
    }
    double v = (double)arena[root_off[i]];
    long long e = meta[root[i]].exp;
    if (v != 0.0) {
        int k;
        v = frexp(v, &k);
        e += k;
    } else {
        e = 0;
    }
    out[i].m = v;
    out[i].e = e;
}

struct wmc_batch {
    int32_t precision = WMC_FP64;
    int32_t elem = 8;
    int64_t n = 0;                     // plans (results)
    int64_t n_inst = 0;                // instances: one per slice of each plan
    std::vector<int64_t> inst_first;   // first instance of plan i (n + 1 entries)
    std::vector<unsigned long long> leaf_eta;  // slice of each leaf's instance
    uint64_t off_leaf_eta = 0;
    GemmShape gemm_shape;              // from the first plan's tuning table
    int64_t n_vars_total = 0;          // auxiliary variables included
    int64_t n_user_total = 0;          // caller weights: 2 * n_user of each plan, in plan order
    std::vector<int64_t> var_off;
    std::vector<int32_t> nvars, nuser;
    std::vector<double> w;
    std::vector<double> wstage;        // caller weights expanded with the auxiliary (1, 1)
    std::vector<LeafDesc> leaves;
    int64_t leaf_work = 0;
    std::vector<NodeDesc> nodes;
    std::vector<GemmDesc> gemms;
    std::vector<Launch> launches;  // [0] = leaves; then LAUNCH_NODES / LAUNCH_GEMM
    // streaming tasks of each NODES launch: tasks[task_first[k] ...], grouped by nk
    std::vector<StreamTask> tasks;
    std::vector<int> task_first;         // per launch
    std::vector<std::array<int, 5>> task_nk;  // per launch, relative to task_first
    uint64_t off_tasks = 0;
    // lookup tables replacing the kernels' searches (int32): per launch, the
    // offset of its wave -> node table and of its workgroup -> task table
    std::vector<int> tables;
    std::vector<int64_t> wave_off, btask_off;
    int64_t leaf_tab_off = 0;
    uint64_t off_tables = 0;
    std::vector<int32_t> roots;
    std::vector<long long> root_off;
    int64_t meta_total = 0;
    uint64_t off_res = 0, off_w = 0, off_meta = 0, off_leaf = 0, off_node = 0, off_gemm = 0, off_roots = 0,
             off_rootoff = 0, off_arena = 0;
    uint64_t arena_bytes = 0, workspace_bytes = 0, desc_bytes = 0;
    std::vector<uint8_t> image;  // [off_leaf, off_arena) of the workspace
    std::mutex mu;
    void *graph_ws = nullptr;
    void *image_ws = nullptr;  // workspace the descriptor image was last uploaded to
    // persistent form: the merged steps' arguments (absolute pointers into a
    // workspace, so kept after the arena and rebuilt for a new workspace)
    uint64_t off_steps = 0;
    std::vector<StepArgs> steps_host;
    void *steps_ws = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    ~wmc_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

static uint64_t bal(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

extern "C" wmc_status wmc_batch_create(const wmc_plan_t *const *plans, int64_t n, wmc_batch **out) {
    if (!out) {
        wmc_set_error("wmc_batch_create: out is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    *out = nullptr;
    if (n <= 0 || !plans) {
        wmc_set_error("wmc_batch_create: need at least one plan");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!plans[i]) {
            wmc_set_error("wmc_batch_create: plan %lld is NULL", (long long)i);
            return WMC_ERR_INVALID_ARGUMENT;
        }
        if (plans[i]->precision != plans[0]->precision) {
            wmc_set_error("wmc_batch_create: plans mix precisions");
            return WMC_ERR_INVALID_ARGUMENT;
        }
        if (plans[i]->sliced.size() > 20) {
            wmc_set_error("wmc_batch_create: plan %lld has 2^%zu slices; batches take at most 2^20 per plan",
                          (long long)i, plans[i]->sliced.size());
            return WMC_ERR_UNSUPPORTED;
        }
    }
    try {
        wmc_batch *B = new wmc_batch();
        B->precision = plans[0]->precision;
        B->gemm_shape = GemmShape{plans[0]->tune.gemm_tpw_max_nt, plans[0]->tune.gemm_orient};
        B->elem = plans[0]->elem;
        B->n = n;
        // instances: slice eta of plan i is instance inst_first[i] + eta
        B->inst_first.assign((size_t)n + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            B->inst_first[(size_t)i + 1] = B->inst_first[(size_t)i] + ((int64_t)1 << plans[i]->sliced.size());
        const int64_t ni = B->inst_first[(size_t)n];
        B->n_inst = ni;
        std::vector<int64_t> iplan((size_t)ni), ieta((size_t)ni);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = B->inst_first[(size_t)i]; j < B->inst_first[(size_t)i + 1]; ++j) {
                iplan[(size_t)j] = i;
                ieta[(size_t)j] = j - B->inst_first[(size_t)i];
            }
        std::vector<int64_t> abase((size_t)ni), mbase((size_t)ni);
        int64_t arena_elems = 0, meta = 0, vars = 0;
        size_t kmax = 0;
        for (int64_t i = 0; i < n; ++i) {
            const wmc_plan_t &P = *plans[i];
            B->var_off.push_back(vars);
            B->nvars.push_back(P.n);
            B->nuser.push_back(P.n_user);
            B->n_user_total += P.n_user;
            B->w.insert(B->w.end(), P.w.begin(), P.w.end());
            vars += P.n;
            kmax = std::max(kmax, P.launches.size());
        }
        for (int64_t j = 0; j < ni; ++j) {
            const wmc_plan_t &P = *plans[iplan[(size_t)j]];
            abase[(size_t)j] = arena_elems;
            mbase[(size_t)j] = meta;
            arena_elems += (int64_t)bal(P.arena_bytes / (uint64_t)P.elem, 64);
            meta += (int64_t)P.T.size();
        }
        B->n_vars_total = vars;
        B->meta_total = std::max<int64_t>(meta, 1);
        // leaves
        B->launches.push_back({LAUNCH_LEAF, 0, 0, 0, 0});
        for (int64_t j = 0; j < ni; ++j) {
            const int64_t i = iplan[(size_t)j];
            const wmc_plan_t &P = *plans[i];
            for (LeafDesc d : P.leaves) {
                d.out += abase[(size_t)j];
                d.tensor += (int)mbase[(size_t)j];
                if (d.kind != WMC_LEAF_CLAUSE) d.var += (int)B->var_off[(size_t)i];
                d.work_begin = B->leaf_work;
                B->leaf_work += (int64_t)bal((uint64_t)1 << d.rank, WMC_WAVE);
                B->leaves.push_back(d);
                B->leaf_eta.push_back((unsigned long long)ieta[(size_t)j]);
            }
        }
        B->launches[0].work = B->leaf_work;
        std::vector<int> ltab;
        wave_leaf_table(B->leaves, B->leaf_work, ltab);
        B->leaf_tab_off = (int64_t)B->tables.size();
        B->tables.insert(B->tables.end(), ltab.begin(), ltab.end());
        // node launches, merged by index; big streaming nodes become tasks
        B->task_first.push_back(0);
        B->task_nk.push_back({0, 0, 0, 0, 0});
        B->wave_off.push_back(0);
        B->btask_off.push_back(0);
        std::vector<int> tab;
        for (size_t k = 1; k < kmax; ++k) {
            Launch merged{LAUNCH_NODES, (int32_t)B->nodes.size(), 0, 0, 0};
            std::vector<Launch> gemm_launches;
            std::vector<NodeDesc> step_nodes;
            for (int64_t j = 0; j < ni; ++j) {
                const wmc_plan_t &P = *plans[iplan[(size_t)j]];
                const size_t i = (size_t)j;  // instance: arena and meta base
                if (k >= P.launches.size()) continue;
                const Launch &L = P.launches[k];
                if (L.type == LAUNCH_GEMM) {
                    GemmDesc g = P.gemms[(size_t)L.pad];
                    g.a += abase[(size_t)i];
                    g.b += abase[(size_t)i];
                    g.c += abase[(size_t)i];
                    g.ta += (int)mbase[(size_t)i];
                    g.tb += (int)mbase[(size_t)i];
                    g.tc += (int)mbase[(size_t)i];
                    gemm_launches.push_back({LAUNCH_GEMM, 0, 1, (int32_t)B->gemms.size(), 0});
                    B->gemms.push_back(g);
                    continue;
                }
                for (int32_t q = 0; q < L.count; ++q) {
                    NodeDesc d = P.nodes[(size_t)(L.first + q)];
                    d.a += abase[(size_t)i];
                    d.b += abase[(size_t)i];
                    d.c += abase[(size_t)i];
                    d.ta += (int)mbase[(size_t)i];
                    d.tb += (int)mbase[(size_t)i];
                    d.tc += (int)mbase[(size_t)i];
                    step_nodes.push_back(d);
                }
            }
            std::vector<StreamTask> tasks;
            std::vector<int> nkf;
            int64_t work = 0;
            split_stream(step_nodes, tasks, nkf, work, plans[0]->tune.multi_min_rank);
            merged.count = (int32_t)step_nodes.size();
            merged.work = work;
            B->nodes.insert(B->nodes.end(), step_nodes.begin(), step_nodes.end());
            if (merged.count || !tasks.empty()) {
                B->launches.push_back(merged);
                B->task_first.push_back((int)B->tasks.size());
                B->task_nk.push_back({nkf[0], nkf[1], nkf[2], nkf[3], nkf[4]});
                B->tasks.insert(B->tasks.end(), tasks.begin(), tasks.end());
                B->wave_off.push_back((int64_t)B->tables.size());
                wave_node_table(step_nodes, work, tab);
                B->tables.insert(B->tables.end(), tab.begin(), tab.end());
                B->btask_off.push_back((int64_t)B->tables.size());
                block_task_table(tasks, nkf, tab);
                B->tables.insert(B->tables.end(), tab.begin(), tab.end());
            }
            for (const Launch &g : gemm_launches) {
                B->launches.push_back(g);
                B->task_first.push_back((int)B->tasks.size());
                B->task_nk.push_back({0, 0, 0, 0, 0});
                B->wave_off.push_back(0);
                B->btask_off.push_back(0);
            }
        }
        for (int64_t j = 0; j < ni; ++j) {
            const wmc_plan_t &P = *plans[iplan[(size_t)j]];
            B->roots.push_back(P.root < 0 ? -1 : P.root + (int)mbase[(size_t)j]);
            B->root_off.push_back(P.root < 0 ? 0 : (long long)(P.T[(size_t)P.root].off + abase[(size_t)j]));
        }
        // workspace layout
        uint64_t off = 0;
        B->off_res = off;
        off += bal(sizeof(BatchRes) * (uint64_t)ni, 256);
        B->off_w = off;
        off += bal(sizeof(double) * 2 * (uint64_t)std::max<int64_t>(vars, 1), 256);
        B->off_meta = off;
        off += bal(sizeof(wmc_meta) * (uint64_t)B->meta_total, 256);
        B->off_leaf = off;
        off += bal(sizeof(LeafDesc) * std::max<size_t>(B->leaves.size(), 1), 256);
        B->off_node = off;
        off += bal(sizeof(NodeDesc) * std::max<size_t>(B->nodes.size(), 1), 256);
        B->off_gemm = off;
        off += bal(sizeof(GemmDesc) * std::max<size_t>(B->gemms.size(), 1), 256);
        B->off_tasks = off;
        off += bal(sizeof(StreamTask) * std::max<size_t>(B->tasks.size(), 1), 256);
        B->off_roots = off;
        off += bal(sizeof(int) * (uint64_t)ni, 256);
        B->off_rootoff = off;
        off += bal(sizeof(long long) * (uint64_t)ni, 256);
        B->off_leaf_eta = off;
        off += bal(sizeof(unsigned long long) * std::max<size_t>(B->leaf_eta.size(), 1), 256);
        B->off_tables = off;
        off += bal(sizeof(int) * std::max<size_t>(B->tables.size(), 1), 256);
        B->off_arena = off;
        B->arena_bytes = (uint64_t)arena_elems * (uint64_t)B->elem;
        B->off_steps = off + bal(B->arena_bytes, 256);
        // [barrier counter, flag][step arguments]
        B->workspace_bytes = B->off_steps + 256 + bal(sizeof(StepArgs) * B->launches.size(), 256);
        B->desc_bytes = B->off_arena - B->off_leaf;
        B->image.assign(B->desc_bytes, 0);
        uint8_t *img = B->image.data();
        auto put = [&](uint64_t o, const void *src, size_t bytes) {
            if (bytes) std::memcpy(img + (o - B->off_leaf), src, bytes);
        };
        put(B->off_leaf, B->leaves.data(), sizeof(LeafDesc) * B->leaves.size());
        put(B->off_node, B->nodes.data(), sizeof(NodeDesc) * B->nodes.size());
        put(B->off_gemm, B->gemms.data(), sizeof(GemmDesc) * B->gemms.size());
        put(B->off_tasks, B->tasks.data(), sizeof(StreamTask) * B->tasks.size());
        put(B->off_roots, B->roots.data(), sizeof(int) * B->roots.size());
        put(B->off_rootoff, B->root_off.data(), sizeof(long long) * B->root_off.size());
        put(B->off_tables, B->tables.data(), sizeof(int) * B->tables.size());
        put(B->off_leaf_eta, B->leaf_eta.data(), sizeof(unsigned long long) * B->leaf_eta.size());
        *out = B;
    } catch (std::bad_alloc &) {
        wmc_set_error("wmc_batch_create: host allocation failed");
        return WMC_ERR_OUT_OF_MEMORY;
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_batch_info(const wmc_batch *b, uint64_t *workspace_bytes, int64_t *n_launches,
                                     int64_t *n_instances) {
    if (!b) {
        wmc_set_error("wmc_batch_info: batch is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (workspace_bytes) *workspace_bytes = b->workspace_bytes;
    if (n_launches) *n_launches = (int64_t)b->launches.size() + 2;
    if (n_instances) *n_instances = b->n;
    return WMC_OK;
}

extern "C" void wmc_batch_destroy(wmc_batch *b) { delete b; }

// Arguments of merged step k (a node launch) on workspace ws.
static StepArgs step_args(const wmc_batch &B, char *ws, size_t k) {
    const Launch &Ln = B.launches[k];
    const int *tabs = (const int *)(ws + B.off_tables);
    StepArgs a{};
    const int tf = B.task_first[k];
    if (B.task_nk[k][4] > 0)
        step_stream_part(a, (const StreamTask *)(ws + B.off_tasks) + tf, B.tasks.data() + tf, B.task_nk[k].data(),
                         tabs + B.btask_off[k]);
    if (Ln.count) {
        a.nodes = (const NodeDesc *)(ws + B.off_node) + Ln.first;
        a.nnodes = Ln.count;
        a.node_work = Ln.work;
        a.wave_node = tabs + B.wave_off[k];
        a.nblocks = grid_for(Ln.work);
    }
    return a;
}

template <typename T>
static void batch_launches(const wmc_batch &B, char *ws, hipStream_t st) {
    wmc_meta *meta = (wmc_meta *)(ws + B.off_meta);
    const double *w = (const double *)(ws + B.off_w);
    const LeafDesc *L = (const LeafDesc *)(ws + B.off_leaf);
    const GemmDesc *G = (const GemmDesc *)(ws + B.off_gemm);
    T *arena = (T *)(ws + B.off_arena);
    const int nt = (int)B.meta_total;
    hipLaunchKernelGGL(k_begin, dim3((nt + WMC_BLOCK - 1) / WMC_BLOCK), dim3(WMC_BLOCK), 0, st, meta, nt,
                       (wmc_acc *)nullptr, 0);
    if (!B.leaves.empty())
        hipLaunchKernelGGL(k_leaves<T>, dim3(grid_for(B.leaf_work)), dim3(WMC_BLOCK), 0, st, L, (int)B.leaves.size(),
                           (long long)B.leaf_work, w, arena, meta, SliceGroup{0, 0, 0}, 0ull,
                           (const int *)(ws + B.off_tables) + B.leaf_tab_off,
                           (const unsigned long long *)(ws + B.off_leaf_eta));
    for (size_t k = 1; k < B.launches.size(); ++k) {
        const Launch &Ln = B.launches[k];
        if (Ln.type == LAUNCH_GEMM) {
            launch_gemm<T>(B.gemms[(size_t)Ln.pad], G + Ln.pad, arena, meta, st, SliceGroup{0, 0, 0}, 1, B.gemm_shape);
            continue;
        }
        // the merged step's small nodes and streaming tasks in one launch
        launch_step<T>(step_args(B, ws, k), arena, meta, st);
    }
    hipLaunchKernelGGL(k_finish_batch<T>, dim3((unsigned)((B.n_inst + 255) / 256)), dim3(256), 0, st, arena,
                       (const long long *)(ws + B.off_rootoff), (const int *)(ws + B.off_roots), meta, (int)B.n_inst,
                       (BatchRes *)(ws + B.off_res));
}

// Every merged step in one cooperative launch (batches without matrix
// nodes): begin, leaves, the persistent step kernel on a grid the device
// holds at once, finish.  Each step's work is k_step's, so the results are
// the fused launches' bit for bit.
template <typename T>
static wmc_status batch_persistent(wmc_batch &B, char *ws, hipStream_t st, bool resident) {
    // the step arguments go up with the descriptors (unless the caller says
    // they are resident and this batch put them into this workspace)
    if (B.steps_ws != (void *)ws) {
        B.steps_host.clear();
        for (size_t k = 1; k < B.launches.size(); ++k) B.steps_host.push_back(step_args(B, ws, k));
    }
    if ((B.steps_ws != (void *)ws || !resident) && !B.steps_host.empty())
        HIP_TRY(hipMemcpyAsync(ws + B.off_steps + 256, B.steps_host.data(), sizeof(StepArgs) * B.steps_host.size(),
                               hipMemcpyHostToDevice, st));
    B.steps_ws = ws;
    wmc_meta *meta = (wmc_meta *)(ws + B.off_meta);
    const double *w = (const double *)(ws + B.off_w);
    T *arena = (T *)(ws + B.off_arena);
    const int nt = (int)B.meta_total;
    hipLaunchKernelGGL(k_begin, dim3((nt + WMC_BLOCK - 1) / WMC_BLOCK), dim3(WMC_BLOCK), 0, st, meta, nt,
                       (wmc_acc *)nullptr, 0);
    if (!B.leaves.empty())
        hipLaunchKernelGGL(k_leaves<T>, dim3(grid_for(B.leaf_work)), dim3(WMC_BLOCK), 0, st,
                           (const LeafDesc *)(ws + B.off_leaf), (int)B.leaves.size(), (long long)B.leaf_work, w, arena,
                           meta, SliceGroup{0, 0, 0}, 0ull, (const int *)(ws + B.off_tables) + B.leaf_tab_off,
                           (const unsigned long long *)(ws + B.off_leaf_eta));
    // the barrier counter and the give-up flag start at zero (the host reads
    // the flag after every persistent call)
    unsigned *bar = (unsigned *)(ws + B.off_steps);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, bar, 2);
    if (!B.steps_host.empty()) {
        unsigned most = 1;
        for (const StepArgs &a : B.steps_host) most = std::max(most, a.sblocks + a.nblocks + a.lblocks);
        int dev = 0, ncu = 0, per = 0, coop = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (!coop) {
            wmc_set_error("wmc_batch_contract: the device has no cooperative launches (WMC_BATCH_PERSISTENT)");
            return WMC_ERR_UNSUPPORTED;
        }
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_steps_persistent<T>, 256, 0));
        if (per < 1 || ncu < 1) {
            wmc_set_error("wmc_batch_contract: the persistent step kernel cannot be resident");
            return WMC_ERR_DEVICE;
        }
        // one workgroup per compute unit: fewer workgroups starve the
        // gathers, more make every barrier dearer (measured 128 to 1024)
        const unsigned grid = std::min<unsigned>(most, (unsigned)ncu);
        const StepArgs *steps = (const StepArgs *)(ws + B.off_steps + 256);
        int nsteps = (int)B.steps_host.size();
        int khz = 0;
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        unsigned long long wait_ticks = (unsigned long long)std::max(khz, 1) * 1000ull * 20ull;  // 20 s
        void *args[] = {(void *)&steps, (void *)&nsteps, (void *)&arena, (void *)&meta, (void *)&bar,
                        (void *)&wait_ticks};
        HIP_TRY(hipLaunchCooperativeKernel((const void *)k_steps_persistent<T>, dim3(grid), dim3(256), args, 0, st));
    }
    hipLaunchKernelGGL(k_finish_batch<T>, dim3((unsigned)((B.n_inst + 255) / 256)), dim3(256), 0, st, arena,
                       (const long long *)(ws + B.off_rootoff), (const int *)(ws + B.off_roots), meta, (int)B.n_inst,
                       (BatchRes *)(ws + B.off_res));
    return WMC_OK;
}

extern "C" wmc_status wmc_batch_contract(wmc_batch *b, const double *weights, void *workspace,
                                         uint64_t workspace_bytes, void *stream, uint32_t flags, wmc_value *out) {
    if (!b || !out) {
        wmc_set_error("wmc_batch_contract: NULL batch or out");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    wmc_batch &B = *b;
    if (!workspace || ((uintptr_t)workspace & 255u)) {
        wmc_set_error("wmc_batch_contract: workspace is NULL or not 256-byte aligned");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (workspace_bytes < B.workspace_bytes) {
        wmc_set_error("wmc_batch_contract: workspace has %llu bytes, batch needs %llu",
                      (unsigned long long)workspace_bytes, (unsigned long long)B.workspace_bytes);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    if (weights)
        for (int64_t i = 0; i < 2 * B.n_user_total; ++i)
            if (!std::isfinite(weights[i])) {
                wmc_set_error("wmc_batch_contract: weight %lld is not finite", (long long)i);
                return WMC_ERR_INVALID_ARGUMENT;
            }
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    std::lock_guard<std::mutex> lock(B.mu);
    const double *w = B.w.data();
    if (weights) {
        // the caller's weights per instance, then each instance's auxiliary (1, 1)
        B.wstage = B.w;
        int64_t u = 0;
        for (size_t i = 0; i < B.nvars.size(); ++i) {
            std::copy(weights + 2 * u, weights + 2 * (u + B.nuser[i]), B.wstage.begin() + 2 * B.var_off[i]);
            u += B.nuser[i];
        }
        w = B.wstage.data();
    }
    if (B.n_vars_total > 0)
        HIP_TRY(hipMemcpyAsync(ws + B.off_w, w, sizeof(double) * 2 * (size_t)B.n_vars_total, hipMemcpyHostToDevice, st));
    // the image goes up unless the caller says it is there already and this
    // batch did put it into this workspace (a first call on a workspace
    // always uploads, whatever the flags say)
    if (!(flags & WMC_BATCH_RESIDENT) || B.image_ws != workspace) {
        HIP_TRY(hipMemcpyAsync(ws + B.off_leaf, B.image.data(), B.desc_bytes, hipMemcpyHostToDevice, st));
        B.image_ws = workspace;
    }
    const bool persistent = (flags & WMC_BATCH_PERSISTENT) && B.gemms.empty() && B.launches.size() > 1;
    if (persistent) {
        const bool resident = (flags & WMC_BATCH_RESIDENT) != 0;
        const wmc_status ps = B.precision == WMC_FP64 ? batch_persistent<double>(B, ws, st, resident)
                                                      : batch_persistent<float>(B, ws, st, resident);
        if (ps != WMC_OK) return ps;
    } else if (flags & WMC_BATCH_GRAPH) {
        if (B.exec && B.graph_ws != workspace) {
            HIP_TRY(hipGraphExecDestroy(B.exec));
            B.exec = nullptr;
        }
        if (!B.exec) {
            if (!B.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal));
            if (B.precision == WMC_FP64) batch_launches<double>(B, ws, B.cap_stream);
            else batch_launches<float>(B, ws, B.cap_stream);
            HIP_TRY(hipStreamEndCapture(B.cap_stream, &graph));
            hipError_t e = hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                B.exec = nullptr;
                wmc_set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
                return WMC_ERR_DEVICE;
            }
            B.graph_ws = workspace;
        }
        HIP_TRY(hipGraphLaunch(B.exec, st));
    } else {
        if (B.precision == WMC_FP64) batch_launches<double>(B, ws, st);
        else batch_launches<float>(B, ws, st);
    }
    HIP_TRY(hipGetLastError());
    std::vector<BatchRes> h((size_t)B.n_inst);
    HIP_TRY(hipMemcpyAsync(h.data(), ws + B.off_res, sizeof(BatchRes) * (size_t)B.n_inst, hipMemcpyDeviceToHost, st));
    unsigned gave_up = 0;
    if (persistent) HIP_TRY(hipMemcpyAsync(&gave_up, ws + B.off_steps + 4, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (gave_up) {
        wmc_set_error("wmc_batch_contract: a grid barrier of the persistent launch timed out");
        return WMC_ERR_DEVICE;
    }
    for (int64_t i = 0; i < B.n; ++i) {
        const int64_t j0 = B.inst_first[(size_t)i], j1 = B.inst_first[(size_t)i + 1];
        if (j1 - j0 == 1) {
            out[i] = make_value(h[(size_t)j0].m, h[(size_t)j0].e);
            continue;
        }
        // the slices of a sliced plan, in slice order
        SliceSum acc;
        for (int64_t j = j0; j < j1; ++j) acc.add(h[(size_t)j].m, h[(size_t)j].e);
        out[i] = (acc.s == 0.0 && acc.c == 0.0) ? make_value(0.0, 0) : make_value(acc.s + acc.c, acc.e);
    }
    return WMC_OK;
}

// Raw descriptor image of a batch, for tools and tests:
// [LeafDesc][NodeDesc][Launch][GemmDesc][root tensor int32][root offset int64]
// [StreamTask][per launch: task_first, nk group starts x5 (int32)];
// info[] = {n_leaves, n_nodes, n_launches, arena_elems, n_instances,
//           meta_total, elem_bytes, n_gemms, n_vars_total, n_tasks}.
extern "C" wmc_status wmc_batch_image(const wmc_batch *b, void *dst, uint64_t dst_bytes, uint64_t *needed,
                                      int64_t *info) {
    if (!b) {
        wmc_set_error("wmc_batch_image: batch is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const wmc_batch &B = *b;
    const uint64_t need = sizeof(LeafDesc) * B.leaves.size() + sizeof(NodeDesc) * B.nodes.size() +
                          sizeof(Launch) * B.launches.size() + sizeof(GemmDesc) * B.gemms.size() +
                          sizeof(int) * B.roots.size() + sizeof(long long) * B.root_off.size() +
                          sizeof(StreamTask) * B.tasks.size() + sizeof(int) * 6 * B.launches.size();
    if (needed) *needed = need;
    if (info) {
        info[0] = (int64_t)B.leaves.size();
        info[1] = (int64_t)B.nodes.size();
        info[2] = (int64_t)B.launches.size();
        info[3] = (int64_t)(B.arena_bytes / (uint64_t)B.elem);
        info[4] = B.n_inst;
        info[5] = B.meta_total;
        info[6] = B.elem;
        info[7] = (int64_t)B.gemms.size();
        info[8] = B.n_vars_total;
        info[9] = (int64_t)B.tasks.size();
    }
    if (!dst) return WMC_OK;
    if (dst_bytes < need) {
        wmc_set_error("wmc_batch_image: buffer too small");
        return WMC_ERR_OUT_OF_MEMORY;
    }
    char *p = (char *)dst;
    auto put = [&](const void *src, size_t bytes) {
        if (bytes) std::memcpy(p, src, bytes);
        p += bytes;
    };
    put(B.leaves.data(), sizeof(LeafDesc) * B.leaves.size());
    put(B.nodes.data(), sizeof(NodeDesc) * B.nodes.size());
    put(B.launches.data(), sizeof(Launch) * B.launches.size());
    put(B.gemms.data(), sizeof(GemmDesc) * B.gemms.size());
    put(B.roots.data(), sizeof(int) * B.roots.size());
    put(B.root_off.data(), sizeof(long long) * B.root_off.size());
    put(B.tasks.data(), sizeof(StreamTask) * B.tasks.size());
    for (size_t k = 0; k < B.launches.size(); ++k) {
        int row[6] = {B.task_first[k], B.task_nk[k][0], B.task_nk[k][1], B.task_nk[k][2], B.task_nk[k][3],
                      B.task_nk[k][4]};
        put(row, sizeof row);
    }
    return WMC_OK;
}
