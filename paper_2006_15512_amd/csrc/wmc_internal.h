// Host-side internals shared by the planner (wmc_host.cpp) and the executor
// (wmc_device.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

#include <cmath>

#include <string>
#include <vector>

#include "../../include/wmc.h"
#include "wmc_desc.h"

// A clause of the Theorem-2 reduction: its distinct variables (ascending,
// 1-based), the single assignment that falsifies it (bit i <-> vars[i]), and
// whether it is a tautology (x and not-x), in which case B_C is all ones.
struct WClause {
    std::vector<int32_t> vars;
    uint32_t falsify = 0;
    bool taut = false;
};

struct wmc_network {
    int32_t n = 0;                // variables, auxiliary ones included
    int32_t n_user = 0;           // variables of the caller's formula: 1..n_user
    std::vector<WClause> clauses;
    std::vector<double> w;        // 2n: {W(x,0), W(x,1)}; (1, 1) for auxiliary variables
    std::vector<int32_t> degree;  // clauses containing x (index x-1)
    int64_t n_indices = 0;
    // auxiliary variable n_user+1+i stands for the OR of the literals over
    // aux_prefix[i] (caller variables), the leading part of a long clause
    std::vector<std::vector<int32_t>> aux_prefix;
    // elimination order over all n variables carried by a network factored
    // along a tree decomposition (empty otherwise)
    std::vector<int32_t> order;
};

// A tensor of the contraction tree (leaf or internal node output).
struct TNode {
    int32_t kind = 0;   // 0 clause leaf, 1 weight leaf, 2 internal
    int32_t src = -1;   // clause index (kind 0) or variable 1..n (kind 1)
    int32_t a = -1, b = -1, parent = -1;
    std::vector<int32_t> vars;    // open variables (unsliced), ascending
    std::vector<int32_t> cnt;     // occurrences of vars[i] inside the subtree
    std::vector<uint8_t> has_w;   // whether A_x of vars[i] is inside the subtree
    std::vector<int32_t> kappa;   // internal: variables summed out here (unsliced)
    int32_t index_rank = 0;       // rank counting Theorem-2 indices
    // after slicing and layout
    std::vector<int32_t> layout;  // storage order, least-significant bit first
    int64_t off = 0;              // arena element offset
    int32_t birth = 0, death = 0; // launch indices
    int32_t cls = 0;              // internal: node class
};

enum { LAUNCH_LEAF = 0, LAUNCH_NODES = 1, LAUNCH_GEMM = 2 };

struct Launch {
    int32_t type;
    int32_t first, count;   // descriptor range (node launches); GEMM: first = GemmDesc index
    int32_t pad;
    int64_t work;           // padded work items
};
static_assert(sizeof(Launch) == 24, "Launch layout");

struct wmc_plan_t {
    int32_t n = 0;                    // variables, auxiliary ones included
    int32_t n_user = 0;               // weights a caller passes: 2 * n_user
    int64_t m = 0;
    int32_t precision = WMC_FP64;
    int32_t elem = 8;
    std::vector<double> w;            // the network's weights
    std::vector<TNode> T;
    int32_t root = -1;
    std::vector<int32_t> node_order;  // internal tensors in launch order
    std::vector<int32_t> sliced;      // sliced variables (bit i of eta <-> sliced[i])
    std::vector<Launch> launches;
    std::vector<LeafDesc> leaves;
    std::vector<NodeDesc> nodes;
    std::vector<GemmDesc> gemms;
    int64_t leaf_work = 0;
    // workspace layout (bytes)
    uint64_t off_acc = 0, off_w = 0, off_meta = 0, off_leaf = 0, off_node = 0, off_gemm = 0, off_tab = 0,
             off_arena = 0;
    // wave -> leaf / node lookup tables (ints at off_tab): entry offset of
    // the leaf table and of each launch's table, -1 where the kernel searches
    int64_t leaf_tab = -1;
    std::vector<int64_t> tab_off;
    uint64_t desc_bytes = 0;          // contiguous [off_leaf, off_arena) image
    std::vector<uint8_t> desc_image;
    uint64_t arena_bytes = 0, workspace_bytes = 0;
    // slices per launch: slice z of a group uses the arena at
    // off_arena + z * arena_stride bytes and the meta table at
    // off_meta + z * meta_stride entries
    wmc_tuning tune{};            // executor tuning copied at planning time
    int32_t group = 1;
    uint64_t arena_stride = 0;   // bytes, 256-aligned
    int64_t meta_stride = 0;     // wmc_meta entries
    wmc_plan_info info{};
};

void wmc_set_error(const char *fmt, ...);
// Bounds of every launch of a finished plan, proved on the host before
// anything runs (built with the device code, which owns the kernels'
// argument builders); false with a description at the first violation.
bool wmc_validate_launches(const wmc_plan_t &P, std::string *why);

// Running sum (s + c) * 2^e of normalised slice values m * 2^e, Neumaier
// compensated, renormalised after every add: the arithmetic of the solo
// executor's finish kernel, so a batch of slices gives the solo result.
struct SliceSum {
    double s = 0.0, c = 0.0;
    long long e = 0;
    void add(double v, long long ev) {
        if (v == 0.0) return;
        if (s == 0.0 && c == 0.0) {
            s = v;
            c = 0.0;
            e = ev;
            return;
        }
        if (ev > e) {
            const long long d = e - ev;
            const int di = d < -4000 ? -4000 : (int)d;
            s = std::ldexp(s, di);
            c = std::ldexp(c, di);
            e = ev;
        }
        const long long d = ev - e;
        const double t = std::ldexp(v, d < -4000 ? -4000 : (int)d);
        const double r = s + t;
        if (std::fabs(s) >= std::fabs(t)) c += (s - r) + t;
        else c += (t - r) + s;
        s = r;
        if (s != 0.0) {
            int k;
            s = std::frexp(s, &k);
            c = std::ldexp(c, -k);
            e += k;
        }
    }
};

