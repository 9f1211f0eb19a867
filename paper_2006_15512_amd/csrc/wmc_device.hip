// Execution stage on gfx950 for one plan: the pairwise contractions of
// Algorithm 2 over the slices of Algorithm 3, all on the device.  Kernels
// and their numerics are in wmc_kernels.h.
#include <mutex>

#include "wmc_kernels.h"

// Optional per-launch timing: an event is recorded on the stream after every
// launch; ms[k] accumulates launch k's duration over the slices.
struct LaunchTimer {
    std::vector<hipEvent_t> ev;
    float *ms = nullptr;
    int64_t cap = 0;
    size_t k = 0;
    hipStream_t st = nullptr;
    void mark() {
        if (!ms) return;
        if (k < ev.size()) (void)hipEventRecord(ev[k], st);
        ++k;
    }
};

// Weights into the workspace: the caller's 2 * n_user (or the network's),
// then the constant (1, 1) of auxiliary variables from the plan.
static hipError_t upload_weights(const wmc_plan_t &P, const double *weights, char *ws, hipStream_t st) {
    const double *w = weights ? weights : P.w.data();
    hipError_t e = hipSuccess;
    if (P.n_user > 0) e = hipMemcpyAsync(ws + P.off_w, w, sizeof(double) * 2 * (size_t)P.n_user, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && P.n > P.n_user)
        e = hipMemcpyAsync(ws + P.off_w + sizeof(double) * 2 * (size_t)P.n_user, P.w.data() + 2 * (size_t)P.n_user,
                           sizeof(double) * 2 * (size_t)(P.n - P.n_user), hipMemcpyHostToDevice, st);
    return e;
}

// Lanes per summed-index group of a streaming node of the plan: the tuned
// split for FP64 nodes with K >= 16 (instances exist for K of 16 and 32).
template <typename T>
static inline int split_lanes_of(const wmc_plan_t &P, int nk) {
    return sizeof(T) == 8 && nk >= 4 && nk <= 5 ? P.tune.split_lanes : 0;
}

// Kernel family that runs node launch k (1 <= k < P.launches.size()) of a
// solo plan, with the streaming kernels' arguments filled in when one of
// them is chosen.  The executor and wmc_plan_kernels share this choice.
template <typename T>
static int solo_kernel(const wmc_plan_t &P, size_t k, Stream2Tab *tb, StreamMfmaArgs *ma) {
    const Launch &Ln = P.launches[k];
    if (Ln.type == LAUNCH_GEMM)
        return gemm_persistent<T>(P.gemms[(size_t)Ln.pad]) ? WMC_KERNEL_GEMM_P : WMC_KERNEL_GEMM;
    if (Ln.count == 1 && P.nodes[(size_t)Ln.first].cls == WMC_CLASS_STREAM) {
        const NodeDesc &d = P.nodes[(size_t)Ln.first];
        const wmc_tuning &tu = P.tune;
        if (tu.stream_mfma_min_bits > 0 && stream_mfma_args(d, ma, tu.stream_mfma_min_bits)) return WMC_KERNEL_STREAM_MFMA;
        if (stream2_args(d, &tb->a, tu.stream2_tile_bits, tu.stream2_min_thread_bits, tu.stream2_low_bits,
                         tu.stream2_vec != 0)) {
            const int lg = tb->a.vec ? 0 : split_lanes_of<T>(P, d.nk);
            // work items per workgroup: 256 threads, or 256 / lg lane groups
            if (stream2_tab(tb, lg > 0 ? 8 - (lg == 4 ? 2 : lg == 2 ? 1 : 3) : 8))
                return tb->a.vec ? WMC_KERNEL_STREAM2_VEC : lg > 0 ? WMC_KERNEL_STREAM2_SPLIT : WMC_KERNEL_STREAM2;
        }
    }
    return WMC_KERNEL_NODES;
}

template <typename T>
static wmc_status run_slices(const wmc_plan_t &P, char *ws, hipStream_t st, long long b, long long e,
                             wmc_value *per_slice, LaunchTimer *tm = nullptr, bool keep_sum = false) {
    wmc_meta *meta = (wmc_meta *)(ws + P.off_meta);
    wmc_acc *acc = (wmc_acc *)(ws + P.off_acc);
    const double *w = (const double *)(ws + P.off_w);
    const LeafDesc *L = (const LeafDesc *)(ws + P.off_leaf);
    const NodeDesc *D = (const NodeDesc *)(ws + P.off_node);
    const GemmDesc *Gd = (const GemmDesc *)(ws + P.off_gemm);
    const int *TB = (const int *)(ws + P.off_tab);
    T *arena = (T *)(ws + P.off_arena);
    const int nt = (int)P.T.size();
    // slices run in groups of up to P.group, side by side in every launch
    // (grid dimension z); per-slice results need one slice at a time
    const long long G = per_slice ? 1 : (long long)P.group;
    const SliceGroup sg{(long long)(P.arena_stride / sizeof(T)), (int)P.meta_stride, 0};
    for (long long eta = b; eta < e; eta += G) {
        const unsigned nz = (unsigned)std::min<long long>(G, e - eta);
        if (tm) {
            tm->k = 0;
            tm->mark();
        }
        const long long nmeta = (long long)(nz - 1) * P.meta_stride + nt;
        hipLaunchKernelGGL(k_begin, dim3((unsigned)((nmeta + WMC_BLOCK - 1) / WMC_BLOCK)), dim3(WMC_BLOCK), 0, st, meta,
                           (int)nmeta, acc, eta == b && !keep_sum ? 1 : 0);
        if (tm) tm->mark();
        if (!P.leaves.empty())
            hipLaunchKernelGGL(k_leaves<T>, dim3(grid_for(P.leaf_work), 1, nz), dim3(WMC_BLOCK), 0, st, L,
                               (int)P.leaves.size(), (long long)P.leaf_work, w, arena, meta, sg,
                               (unsigned long long)eta, P.leaf_tab >= 0 ? TB + P.leaf_tab : nullptr);
        if (tm) tm->mark();
        for (size_t k = 1; k < P.launches.size(); ++k) {
            const Launch &Ln = P.launches[k];
            Stream2Tab sa;
            StreamMfmaArgs ma;
            const int kern = solo_kernel<T>(P, k, &sa, &ma);
            if (kern == WMC_KERNEL_GEMM_P || kern == WMC_KERNEL_GEMM)
                launch_gemm<T>(P.gemms[(size_t)Ln.pad], Gd + Ln.pad, arena, meta, st, sg, nz,
                               GemmShape{P.tune.gemm_tpw_max_nt, P.tune.gemm_orient});
            else if (kern == WMC_KERNEL_STREAM_MFMA)
                launch_stream_mfma<T>(ma, P.nodes[(size_t)Ln.first].nk, arena, meta, st,
                                      (unsigned)P.tune.stream_mfma_grid_cap, sg, nz);
            else if ((kern == WMC_KERNEL_STREAM2 || kern == WMC_KERNEL_STREAM2_SPLIT || kern == WMC_KERNEL_STREAM2_VEC) &&
                     launch_stream2<T>(sa, P.nodes[(size_t)Ln.first].nk, arena, meta, st,
                                      kern == WMC_KERNEL_STREAM2_SPLIT ? split_lanes_of<T>(P, P.nodes[(size_t)Ln.first].nk) : 0,
                                      sg, nz, (unsigned)P.tune.stream2_grid_cap)) {
            } else
                hipLaunchKernelGGL(k_nodes<T>, dim3(grid_for(Ln.work), 1, nz), dim3(WMC_BLOCK), 0, st, D + Ln.first,
                                   Ln.count, (long long)Ln.work, arena, meta, sg,
                                   P.tab_off[k] >= 0 ? TB + P.tab_off[k] : nullptr);
            if (tm) tm->mark();
        }
        hipLaunchKernelGGL(k_finish<T>, dim3(1), dim3(1), 0, st, arena, (long long)P.T[(size_t)P.root].off, meta,
                           P.root, acc, (int)nz, sg.astride, sg.mstride);
        if (tm) tm->mark();
        HIP_TRY(hipGetLastError());
        if (tm) {
            HIP_TRY(hipEventSynchronize(tm->ev[tm->k - 1]));
            for (size_t q = 1; q < tm->k && (int64_t)(q - 1) < tm->cap; ++q) {
                float t = 0.f;
                HIP_TRY(hipEventElapsedTime(&t, tm->ev[q - 1], tm->ev[q]));
                tm->ms[q - 1] += t;
            }
        }
        if (per_slice) {
            wmc_acc h;
            HIP_TRY(hipMemcpyAsync(&h, acc, sizeof h, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            per_slice[eta - b] = make_value(h.last_m, h.last_e);
        }
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_contract_slices(const wmc_plan_t *plan, const double *weights, void *workspace,
                                          uint64_t workspace_bytes, void *stream, int64_t slice_begin,
                                          int64_t slice_end, wmc_value *out, wmc_value *per_slice) {
    if (!plan || !out) {
        wmc_set_error("wmc_contract: NULL plan or out");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const wmc_plan_t &P = *plan;
    const int64_t ns = (int64_t)1 << P.sliced.size();
    if (slice_begin < 0 || slice_end > ns || slice_begin > slice_end) {
        wmc_set_error("wmc_contract: slice range [%lld, %lld) outside [0, %lld)", (long long)slice_begin,
                      (long long)slice_end, (long long)ns);
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (weights)
        for (int64_t i = 0; i < 2 * (int64_t)P.n_user; ++i)
            if (!std::isfinite(weights[i])) {
                wmc_set_error("wmc_contract: weight %lld is not finite", (long long)i);
                return WMC_ERR_INVALID_ARGUMENT;
            }
    if (P.root < 0) {  // no variables and no clauses: the empty product
        *out = make_value(1.0, 0);
        if (per_slice)
            for (int64_t s = slice_begin; s < slice_end; ++s) per_slice[s - slice_begin] = *out;
        return WMC_OK;
    }
    if (!workspace || ((uintptr_t)workspace & 255u)) {
        wmc_set_error("wmc_contract: workspace is NULL or not 256-byte aligned");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (workspace_bytes < P.workspace_bytes) {
        wmc_set_error("wmc_contract: workspace has %llu bytes, plan needs %llu", (unsigned long long)workspace_bytes,
                      (unsigned long long)P.workspace_bytes);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    if (slice_begin == slice_end) {
        *out = make_value(0.0, 0);
        return WMC_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    HIP_TRY(upload_weights(P, weights, ws, st));
    HIP_TRY(hipMemcpyAsync(ws + P.off_leaf, P.desc_image.data(), P.desc_bytes, hipMemcpyHostToDevice, st));
    wmc_status s = P.precision == WMC_FP64 ? run_slices<double>(P, ws, st, slice_begin, slice_end, per_slice)
                                           : run_slices<float>(P, ws, st, slice_begin, slice_end, per_slice);
    if (s != WMC_OK) return s;
    wmc_acc h;
    HIP_TRY(hipMemcpyAsync(&h, ws + P.off_acc, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h.s == 0.0 && h.c == 0.0) {
        *out = make_value(0.0, 0);
    } else {
        *out = make_value(h.s + h.c, h.e);
    }
    return WMC_OK;
}

// Continue the running slice sum held in *state over the next `count`
// slices (Algorithm 3's loop over eta, split across calls).  The Neumaier
// pair and its exponent are restored into the device accumulator before the
// first slice and read back after the last, so a run split at any slice
// boundary gives the bits of one uninterrupted run.
extern "C" wmc_status wmc_contract_resume(const wmc_plan_t *plan, const double *weights, void *workspace,
                                          uint64_t workspace_bytes, void *stream, int64_t count,
                                          wmc_slice_state *state, wmc_value *out) {
    if (!plan || !state || !out) {
        wmc_set_error("wmc_contract_resume: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const wmc_plan_t &P = *plan;
    const int64_t ns = (int64_t)1 << P.sliced.size();
    if (state->next_slice == 0 && state->n_slices == 0) state->n_slices = ns;  // fresh state
    if (state->n_slices != ns || state->next_slice < 0 || state->next_slice > ns || count < 0 ||
        !std::isfinite(state->s) || !std::isfinite(state->c)) {
        wmc_set_error("wmc_contract_resume: state does not belong to this plan (next %lld of %lld slices, plan has %lld)",
                      (long long)state->next_slice, (long long)state->n_slices, (long long)ns);
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (weights)
        for (int64_t i = 0; i < 2 * (int64_t)P.n_user; ++i)
            if (!std::isfinite(weights[i])) {
                wmc_set_error("wmc_contract_resume: weight %lld is not finite", (long long)i);
                return WMC_ERR_INVALID_ARGUMENT;
            }
    if (!workspace || ((uintptr_t)workspace & 255u) || workspace_bytes < P.workspace_bytes) {
        wmc_set_error("wmc_contract_resume: workspace NULL, misaligned or below %llu bytes",
                      (unsigned long long)P.workspace_bytes);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    const int64_t b = state->next_slice, e = std::min<int64_t>(ns, b + count);
    if (P.root >= 0 && e > b) {
        hipStream_t st = (hipStream_t)stream;
        char *ws = (char *)workspace;
        wmc_acc h;
        std::memset(&h, 0, sizeof h);
        h.s = state->s;
        h.c = state->c;
        h.e = state->e;
        HIP_TRY(upload_weights(P, weights, ws, st));
        HIP_TRY(hipMemcpyAsync(ws + P.off_leaf, P.desc_image.data(), P.desc_bytes, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(ws + P.off_acc, &h, sizeof h, hipMemcpyHostToDevice, st));
        wmc_status s = P.precision == WMC_FP64 ? run_slices<double>(P, ws, st, b, e, nullptr, nullptr, true)
                                               : run_slices<float>(P, ws, st, b, e, nullptr, nullptr, true);
        if (s != WMC_OK) return s;
        HIP_TRY(hipMemcpyAsync(&h, ws + P.off_acc, sizeof h, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        state->s = h.s;
        state->c = h.c;
        state->e = h.e;
    }
    state->next_slice = e;
    if (P.root < 0) {
        *out = make_value(1.0, 0);  // no variables and no clauses
    } else {
        *out = (state->s == 0.0 && state->c == 0.0) ? make_value(0.0, 0) : make_value(state->s + state->c, state->e);
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_contract(const wmc_plan_t *plan, const double *weights, void *workspace,
                                   uint64_t workspace_bytes, void *stream, wmc_value *out) {
    if (!plan) {
        wmc_set_error("wmc_contract: NULL plan");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    return wmc_contract_slices(plan, weights, workspace, workspace_bytes, stream, 0,
                               (int64_t)1 << plan->sliced.size(), out, nullptr);
}

// wmc_contract with per-launch timing: ms[k] (k < n_launches of
// wmc_plan_launches) receives the summed duration of launch k over all
// slices, measured with HIP events recorded on `stream` between launches.
extern "C" wmc_status wmc_contract_profile(const wmc_plan_t *plan, const double *weights, void *workspace,
                                           uint64_t workspace_bytes, void *stream, float *ms, int64_t cap,
                                           wmc_value *out) {
    if (!plan || !out || !ms) {
        wmc_set_error("wmc_contract_profile: NULL argument");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const wmc_plan_t &P = *plan;
    const int64_t n = (int64_t)P.launches.size() + 2;
    if (cap < n - 1) {
        wmc_set_error("wmc_contract_profile: need %lld slots", (long long)(n - 1));
        return WMC_ERR_OUT_OF_MEMORY;
    }
    if (P.root < 0 || !workspace || workspace_bytes < P.workspace_bytes)
        return wmc_contract(plan, weights, workspace, workspace_bytes, stream, out);
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    LaunchTimer tm;
    tm.ms = ms;
    tm.cap = cap;
    tm.st = st;
    tm.ev.resize((size_t)n + 1);
    for (auto &e : tm.ev) HIP_TRY(hipEventCreate(&e));
    for (int64_t k = 0; k < cap; ++k) ms[k] = 0.f;
    wmc_status s = WMC_OK;
    if (upload_weights(P, weights, ws, st) != hipSuccess) s = WMC_ERR_DEVICE;
    if (s == WMC_OK && hipMemcpyAsync(ws + P.off_leaf, P.desc_image.data(), P.desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        s = WMC_ERR_DEVICE;
    const long long ns = 1ll << P.sliced.size();
    if (s == WMC_OK)
        s = P.precision == WMC_FP64 ? run_slices<double>(P, ws, st, 0, ns, nullptr, &tm)
                                    : run_slices<float>(P, ws, st, 0, ns, nullptr, &tm);
    wmc_acc h;
    if (s == WMC_OK && (hipMemcpyAsync(&h, ws + P.off_acc, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
        s = WMC_ERR_DEVICE;
    for (auto &e : tm.ev) (void)hipEventDestroy(e);
    if (s != WMC_OK) {
        if (s == WMC_ERR_DEVICE) wmc_set_error("wmc_contract_profile: HIP failure");
        return s;
    }
    *out = (h.s == 0.0 && h.c == 0.0) ? make_value(0.0, 0) : make_value(h.s + h.c, h.e);
    return WMC_OK;
}

// Kernel family of every launch wmc_contract issues for one slice, in the
// order of wmc_plan_launches (host only: the choice depends on the plan and,
// for the matrix kernel, on the current device's LDS size).
extern "C" wmc_status wmc_plan_kernels(const wmc_plan_t *plan, int32_t *kernel, int64_t cap, int64_t *n_out) {
    if (!plan) {
        wmc_set_error("wmc_plan_kernels: plan is NULL");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    const wmc_plan_t &P = *plan;
    const int64_t n = (int64_t)P.launches.size() + 2;
    if (n_out) *n_out = n;
    if (!kernel) return WMC_OK;
    if (cap < n) {
        wmc_set_error("wmc_plan_kernels: need %lld slots", (long long)n);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    kernel[0] = WMC_KERNEL_BEGIN;
    kernel[1] = WMC_KERNEL_LEAVES;
    for (size_t k = 1; k < P.launches.size(); ++k) {
        Stream2Tab sa;
        StreamMfmaArgs ma;
        kernel[k + 1] = P.precision == WMC_FP64 ? solo_kernel<double>(P, k, &sa, &ma) : solo_kernel<float>(P, k, &sa, &ma);
    }
    kernel[n - 1] = WMC_KERNEL_FINISH;
    return WMC_OK;
}

// Largest value a run list can deposit (every source bit set).
static unsigned long long deposit_all(const unsigned *runs, int n) {
    unsigned long long out = 0;
    for (int i = 0; i < n; ++i) out |= ((1ull << ((runs[i] >> 8) & 255u)) - 1ull) << (runs[i] >> 16);
    return out;
}

// Every index map of the kernels is a bit deposit, so the largest address a
// launch can form is the map of all ones: the OR of its table entries and
// tile bits.  Checked for every launch against the ranks of the tensors it
// reads and writes; every tensor against the arena.
template <typename T>
static bool validate_t(const wmc_plan_t &P, std::string *why) {
    char buf[160];
    auto fail = [&](size_t k, const char *what) {
        std::snprintf(buf, sizeof buf, "launch %zu: %s", k, what);
        *why = buf;
        return false;
    };
    auto rank = [&](int t) { return (int)P.T[(size_t)t].layout.size(); };
    auto fits = [](unsigned long long mx, int bits) { return bits >= 64 || (mx >> bits) == 0; };
    const uint64_t arena_elems = P.arena_bytes / (uint64_t)P.elem;
    for (size_t t = 0; t < P.T.size(); ++t)
        if (P.T[t].off < 0 || (uint64_t)P.T[t].off + (1ull << rank((int)t)) > arena_elems) {
            std::snprintf(buf, sizeof buf, "tensor %zu outside the arena", t);
            *why = buf;
            return false;
        }
    for (size_t k = 1; k < P.launches.size(); ++k) {
        const Launch &Ln = P.launches[k];
        Stream2Tab tb;
        StreamMfmaArgs ma;
        const int kern = solo_kernel<T>(P, k, &tb, &ma);
        if (kern == WMC_KERNEL_GEMM_P || kern == WMC_KERNEL_GEMM) {
            const GemmDesc &g = P.gemms[(size_t)Ln.pad];
            int top[GR_N] = {0};
            for (int q = 0; q < GR_N; ++q)
                for (int r = 0; r < g.nrun[q]; ++r) top[q] = std::max(top[q], (int)g.run[q][r][2] + (int)g.run[q][r][1]);
            const int ra = rank(g.ta), rb = rank(g.tb), rc = rank(g.tc);
            if (top[GR_MU_A] > ra - 4 - g.nk || top[GR_BETA_A] > ra - 4 - g.nk || top[GR_NU_B] > rb - g.nk ||
                top[GR_BETA_B] > rb - g.nk || top[GR_MU_C] > rc || top[GR_NU_C] > rc || top[GR_BETA_C] > rc ||
                ra != g.nk + g.nb + g.nm || rb != g.nk + g.nb + g.nn || rc != g.nb + g.nm + g.nn)
                return fail(k, "matrix node maps exceed its operands");
        } else if (kern == WMC_KERNEL_STREAM_MFMA) {
            unsigned long long c = 0, a = 0, b = 0;
            for (int q = 0; q < ma.nch; ++q)
                for (int v = 0; v < 16; ++v) {
                    c |= ma.tabc[q][v];
                    a |= ma.taba[q][v];
                    b |= ma.tabb[q][v];
                }
            for (int v = 0; v < 16; ++v) {
                a |= ma.lane_a[v] | ma.blk_a[v];
                b |= ma.lane_b[v] | ma.blk_b[v];
            }
            for (int t = 0; t < ma.nt; ++t) c |= 1ull << ma.tpos[t];
            const int nk = P.nodes[(size_t)Ln.first].nk;
            if (!fits(c, ma.rc) || ma.rc != rank(ma.tc) || !fits(a, rank(ma.ta) - nk) || !fits(b, rank(ma.tb) - nk))
                return fail(k, "matrix-core streaming tables exceed the node's tensors");
        } else if (kern == WMC_KERNEL_STREAM2 || kern == WMC_KERNEL_STREAM2_SPLIT || kern == WMC_KERNEL_STREAM2_VEC) {
            const Stream2Args &a = tb.a;
            unsigned long long c = 0, so = 0, oo = 0;
            for (int q = 0; q < tb.nch; ++q)
                for (int v = 0; v < 16; ++v) {
                    c |= tb.hr[q][v];
                    so |= tb.hs[q][v];
                    oo |= tb.ho[q][v];
                }
            for (int q = 0; q < 2; ++q)
                for (int v = 0; v < 16; ++v) {
                    c |= tb.lr[q][v];
                    so |= tb.ls[q][v];
                    oo |= tb.lo[q][v];
                }
            unsigned long long pq = 0;
            for (int t = 0; t < a.np; ++t) pq |= 1ull << a.pbit[t];
            for (int t = 0; t < a.nq; ++t) pq |= 1ull << a.qbit[t];
            c |= pq | (a.vec ? 1ull : 0ull);
            so |= deposit_all(a.srun, a.nsrun);
            oo |= deposit_all(a.orun, a.norun);
            const int nk = P.nodes[(size_t)Ln.first].nk;
            if (!fits(c, a.rc) || a.rc != rank(a.tc) || !fits(so, rank(a.ts) - nk) || !fits(oo, rank(a.to) - nk))
                return fail(k, "streaming tables exceed the node's tensors");
        } else {
            for (int32_t q = 0; q < Ln.count; ++q) {
                const NodeDesc &d = P.nodes[(size_t)(Ln.first + q)];
                if (d.rc != rank(d.tc) || !fits(deposit_all(d.ra, d.nra), rank(d.ta) - d.nk) ||
                    !fits(deposit_all(d.rb, d.nrb), rank(d.tb) - d.nk))
                    return fail(k, "node maps exceed the node's tensors");
            }
        }
    }
    return true;
}

bool wmc_validate_launches(const wmc_plan_t &P, std::string *why) {
    return P.precision == WMC_FP64 ? validate_t<double>(P, why) : validate_t<float>(P, why);
}

// ---------------------------------------------------------------------------
// Contraction without any device allocation: the workspace is a static
// device array of WMC_NOALLOC_SCRATCH_BYTES.  Host code never passes the
// array's name to a kernel or copy (on the host it is only a stand-in for
// the symbol); it passes the device address hipGetSymbolAddress returns,
// looked up once per device with that device current.  Every call on a
// device shares that device's array, so calls that overlap on one device
// race; k_begin clears the meta table and the accumulator at the start of
// every contraction, and nothing else in the workspace is read before it is
// written.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[WMC_NOALLOC_SCRATCH_BYTES];

#define WMC_NOALLOC_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[WMC_NOALLOC_MAX_DEVICES];

static wmc_status scratch_of_current_device(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= WMC_NOALLOC_MAX_DEVICES) {
        wmc_set_error("wmc_contract_noalloc: device %d beyond the %d supported", dev, WMC_NOALLOC_MAX_DEVICES);
        return WMC_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            wmc_set_error("wmc_contract_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return WMC_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return WMC_OK;
}

extern "C" wmc_status wmc_contract_noalloc(const wmc_plan_t *plan, const double *weights, void *stream,
                                           wmc_value *out) {
    if (!plan || !out) {
        wmc_set_error("wmc_contract_noalloc: NULL plan or out");
        return WMC_ERR_INVALID_ARGUMENT;
    }
    if (plan->workspace_bytes > WMC_NOALLOC_SCRATCH_BYTES) {
        wmc_set_error("wmc_contract_noalloc: plan needs a workspace of %llu bytes, the static scratch holds %llu",
                      (unsigned long long)plan->workspace_bytes, (unsigned long long)WMC_NOALLOC_SCRATCH_BYTES);
        return WMC_ERR_OUT_OF_MEMORY;
    }
    void *ws = nullptr;
    const wmc_status s = scratch_of_current_device(&ws);
    if (s != WMC_OK) return s;
    return wmc_contract(plan, weights, ws, WMC_NOALLOC_SCRATCH_BYTES, stream, out);
}
