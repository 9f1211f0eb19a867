// Host side of the weighted model counter: the reduction of Theorem 2, the
// planning stage (contraction tree, index slicing of Algorithm 3, storage
// layouts, launch schedule, static arena) and the inspection entry points.
// Everything here is integer bookkeeping; all arithmetic on tensor entries
// runs in the HIP kernels (wmc_device.hip).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "wmc_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void wmc_set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

extern "C" const char *wmc_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *wmc_version(void) { return "wmc-mi355x 0.1 (gfx950)"; }

#define WMC_FAIL(code, ...)              \
    do {                                 \
        wmc_set_error(__VA_ARGS__);      \
        return code;                     \
    } while (0)

// ---------------------------------------------------------------------------
// Reduction (Theorem 2).  B_C is stored as (variables, falsifying assignment,
// tautology flag); A_x is symbolic: its degree and the two weights.
// ---------------------------------------------------------------------------
// The network of Theorem 2 over clause list cls (DIMACS literals over the
// caller's n_vars variables and the auxiliary ones after them, which weigh
// (1, 1); aux_prefix[i] lists the caller variables auxiliary variable
// n_vars + 1 + i depends on).
static wmc_network *make_network(int32_t n_vars, const double *weights, const std::vector<std::vector<int32_t>> &cls,
                                 std::vector<std::vector<int32_t>> aux_prefix) {
    const int32_t n_aux = (int32_t)aux_prefix.size();
    wmc_network *net = new wmc_network();
    net->n = n_vars + n_aux;
    net->n_user = n_vars;
    net->aux_prefix = std::move(aux_prefix);
    net->w.assign(weights, weights + 2 * (size_t)n_vars);
    net->w.resize(2 * (size_t)net->n, 1.0);
    net->degree.assign((size_t)net->n, 0);
    net->clauses.resize(cls.size());
    std::vector<int8_t> sign((size_t)net->n + 1, 0);  // bit0: positive seen, bit1: negative seen
    for (size_t c = 0; c < cls.size(); ++c) {
        WClause &cl = net->clauses[c];
        for (int32_t l : cls[c]) {
            int32_t v = l > 0 ? l : -l;
            if (!sign[v]) cl.vars.push_back(v);
            sign[v] |= (l > 0) ? 1 : 2;
        }
        std::sort(cl.vars.begin(), cl.vars.end());
        for (size_t i = 0; i < cl.vars.size(); ++i) {
            int32_t v = cl.vars[i];
            if (sign[v] == 3) cl.taut = true;
            // a positive literal is falsified by 0, a negative one by 1
            if (sign[v] == 2) cl.falsify |= 1u << i;
            sign[v] = 0;
            net->degree[(size_t)v - 1]++;
        }
        net->n_indices += (int64_t)cl.vars.size();
    }
    return net;
}

// Checks shared by the network builders: sizes, CSR offsets, literals in
// range, finite weights.
static wmc_status check_formula(const char *who, int32_t n_vars, int64_t n_clauses, const int64_t *clause_ptr,
                                const int32_t *lits, const double *weights) {
    if (n_vars < 0 || n_clauses < 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: negative size", who);
    if (n_clauses > 0 && !clause_ptr) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: clause_ptr is NULL", who);
    if (n_vars > 0 && !weights) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: weights is NULL", who);
    if (n_clauses > 0) {
        for (int64_t c = 0; c < n_clauses; ++c)
            if (clause_ptr[c + 1] < clause_ptr[c] || clause_ptr[c] < 0)
                WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: clause_ptr not non-decreasing at %lld", who, (long long)c);
        if (clause_ptr[n_clauses] > clause_ptr[0] && !lits) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: lits is NULL", who);
    }
    for (int64_t i = 0; i < 2 * (int64_t)n_vars; ++i)
        if (!std::isfinite(weights[i]))
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: weight %lld is not finite", who, (long long)i);
    for (int64_t j = n_clauses > 0 ? clause_ptr[0] : 0; n_clauses > 0 && j < clause_ptr[n_clauses]; ++j)
        if (lits[j] == 0 || lits[j] > n_vars || lits[j] < -n_vars)
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: literal %d out of range", who, (int)lits[j]);
    return WMC_OK;
}

extern "C" wmc_status wmc_build_network(int32_t n_vars, int64_t n_clauses, const int64_t *clause_ptr,
                                        const int32_t *lits, const double *weights,
                                        wmc_network **out) {
    if (!out) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_build_network: out is NULL");
    *out = nullptr;
    {
        const wmc_status st = check_formula("wmc_build_network", n_vars, n_clauses, clause_ptr, lits, weights);
        if (st != WMC_OK) return st;
    }
    try {
        // Clauses with more than WMC_FACTOR_ABOVE distinct variables are
        // factored into a chain of clauses of at most three literals over
        // auxiliary variables a_1..a_{k-2} (the clause is a COPY-like OR, and
        // an OR is tree-factorable, Def. 4): a_1 <-> l_1 v l_2,
        // a_i <-> a_{i-1} v l_{i+1}, and the clause a_{k-2} v l_k.  Each
        // assignment of the formula's variables extends to exactly one
        // assignment of the a_i, and the a_i weigh (1, 1), so W is unchanged.
        std::vector<std::vector<int32_t>> cls;
        std::vector<std::vector<int32_t>> aux_prefix;
        cls.reserve((size_t)n_clauses);
        {
            std::vector<int8_t> sign((size_t)n_vars + 1, 0);
            for (int64_t c = 0; c < n_clauses; ++c) {
                std::vector<int32_t> lv;  // distinct literals, first occurrence order
                bool taut = false;
                for (int64_t j = clause_ptr[c]; j < clause_ptr[c + 1]; ++j) {
                    const int32_t l = lits[j], v = l > 0 ? l : -l;
                    const int8_t bit = l > 0 ? 1 : 2;
                    if (!(sign[v] & bit)) {
                        if (sign[v]) taut = true;
                        else lv.push_back(l);
                        sign[v] |= bit;
                    }
                }
                for (int32_t l : lv) sign[(size_t)(l > 0 ? l : -l)] = 0;
                if (lv.size() <= WMC_FACTOR_ABOVE || taut) {
                    // short clauses (and tautologies, which weigh 1) keep their literals
                    std::vector<int32_t> raw(lits + clause_ptr[c], lits + clause_ptr[c + 1]);
                    if (taut && lv.size() > WMC_FACTOR_ABOVE) raw.clear(), raw.push_back(lv[0]), raw.push_back(-lv[0]);
                    cls.push_back(std::move(raw));
                    continue;
                }
                const int32_t k = (int32_t)lv.size();
                int32_t prev = 0;
                for (int32_t i = 1; i <= k - 2; ++i) {
                    const int32_t a = n_vars + (int32_t)aux_prefix.size() + 1;
                    aux_prefix.emplace_back();
                    for (int32_t t = 0; t <= i; ++t) aux_prefix.back().push_back(lv[(size_t)t] > 0 ? lv[(size_t)t] : -lv[(size_t)t]);
                    const int32_t x = i == 1 ? lv[0] : prev, y = lv[(size_t)i];
                    cls.push_back({-a, x, y});
                    cls.push_back({a, -x});
                    cls.push_back({a, -y});
                    prev = a;
                }
                cls.push_back({prev, lv[(size_t)k - 1]});
            }
        }
        if ((int64_t)n_vars + (int64_t)aux_prefix.size() > (int64_t)INT32_MAX / 2)
            WMC_FAIL(WMC_ERR_UNSUPPORTED, "wmc_build_network: too many variables after clause factoring");
        *out = make_network(n_vars, weights, cls, std::move(aux_prefix));
    } catch (std::bad_alloc &) {
        WMC_FAIL(WMC_ERR_OUT_OF_MEMORY, "wmc_build_network: host allocation failed");
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_network_info(const wmc_network *net, int64_t *n_tensors, int64_t *n_indices) {
    if (!net) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_network_info: net is NULL");
    if (n_tensors) *n_tensors = (int64_t)net->n + (int64_t)net->clauses.size();  // auxiliary tensors included
    if (n_indices) *n_indices = net->n_indices;
    return WMC_OK;
}

extern "C" void wmc_network_destroy(wmc_network *net) { delete net; }

// ---------------------------------------------------------------------------
// Seeded min-fill elimination order on the primal graph (variables adjacent
// when they share a clause).  Key: (fill-in edges, degree, seeded priority).
// ---------------------------------------------------------------------------
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static std::vector<int32_t> minfill_order(const wmc_network &net, uint64_t seed) {
    const int32_t n = net.n;
    const size_t W = ((size_t)n + 63) / 64;
    std::vector<uint64_t> adj((size_t)n * W, 0);
    auto row = [&](int32_t v) { return &adj[(size_t)v * W]; };
    for (const WClause &c : net.clauses)
        for (int32_t a : c.vars)
            for (int32_t b : c.vars)
                if (a != b) row(a - 1)[(size_t)(b - 1) / 64] |= 1ull << ((b - 1) % 64);
    std::vector<uint8_t> done((size_t)n, 0);
    std::vector<int64_t> fill((size_t)n, 0), deg((size_t)n, 0);
    std::vector<uint64_t> prio((size_t)n);
    for (int32_t v = 0; v < n; ++v) prio[(size_t)v] = splitmix64(seed * 0x100000001B3ull + (uint64_t)v);
    std::vector<int32_t> nb;
    auto neighbours = [&](int32_t v) {
        nb.clear();
        const uint64_t *r = row(v);
        for (size_t w = 0; w < W; ++w) {
            uint64_t bits = r[w];
            while (bits) {
                int t = __builtin_ctzll(bits);
                bits &= bits - 1;
                nb.push_back((int32_t)(w * 64 + t));
            }
        }
    };
    auto compute = [&](int32_t v) {
        neighbours(v);
        const uint64_t *rv = row(v);
        int64_t f = 0;
        for (int32_t u : nb) {
            const uint64_t *ru = row(u);
            int64_t c = 0;
            for (size_t w = 0; w < W; ++w) c += __builtin_popcountll(rv[w] & ~ru[w]);
            f += c - 1;  // u itself is in N(v) but not in N(u)
        }
        fill[(size_t)v] = f / 2;
        deg[(size_t)v] = (int64_t)nb.size();
    };
    for (int32_t v = 0; v < n; ++v) compute(v);
    std::vector<int32_t> order;
    order.reserve((size_t)n);
    std::vector<uint8_t> dirty((size_t)n, 0);
    std::vector<int32_t> nv;
    for (int32_t step = 0; step < n; ++step) {
        int32_t best = -1;
        for (int32_t v = 0; v < n; ++v) {
            if (done[(size_t)v]) continue;
            if (best < 0 || fill[(size_t)v] < fill[(size_t)best] ||
                (fill[(size_t)v] == fill[(size_t)best] &&
                 (deg[(size_t)v] < deg[(size_t)best] ||
                  (deg[(size_t)v] == deg[(size_t)best] && prio[(size_t)v] < prio[(size_t)best]))))
                best = v;
        }
        neighbours(best);
        nv = nb;
        // connect the neighbourhood, drop best from the graph
        uint64_t *rb = row(best);
        for (int32_t u : nv) {
            uint64_t *ru = row(u);
            for (size_t w = 0; w < W; ++w) ru[w] |= rb[w];
            ru[(size_t)u / 64] &= ~(1ull << (u % 64));
            ru[(size_t)best / 64] &= ~(1ull << (best % 64));
        }
        std::fill(rb, rb + W, 0);
        done[(size_t)best] = 1;
        order.push_back(best + 1);
        for (int32_t u : nv) {
            dirty[(size_t)u] = 1;
            neighbours(u);
            for (int32_t z : nb) dirty[(size_t)z] = 1;
        }
        for (int32_t u = 0; u < n; ++u)
            if (dirty[(size_t)u]) {
                dirty[(size_t)u] = 0;
                if (!done[(size_t)u]) compute(u);
            }
    }
    return order;
}

// ---------------------------------------------------------------------------
// Contraction-tree construction.  A tensor's open variables are those with
// some but not all of their occurrences (the clause leaves containing x and
// A_x) inside its subtree; a variable is summed out at the node whose subtree
// first holds all of them.  Keeping one storage mode per open variable is the
// tensor obtained by contracting A_x's COPY factors early, which partial
// contraction and tree-factorability (Definition 4) allow.
// ---------------------------------------------------------------------------
struct TreeBuilder {
    const wmc_network &net;
    std::vector<TNode> &T;
    std::vector<int32_t> total;  // occurrences: degree + 1 (A_x)

    TreeBuilder(const wmc_network &nt, std::vector<TNode> &t) : net(nt), T(t) {
        total.assign((size_t)net.n + 1, 0);
        for (int32_t x = 1; x <= net.n; ++x) total[(size_t)x] = net.degree[(size_t)x - 1] + 1;
    }

    int32_t leaf_clause(int32_t c) {
        TNode t;
        t.kind = 0;
        t.src = c;
        t.vars = net.clauses[(size_t)c].vars;
        t.cnt.assign(t.vars.size(), 1);
        t.has_w.assign(t.vars.size(), 0);
        t.index_rank = (int32_t)t.vars.size();
        T.push_back(std::move(t));
        return (int32_t)T.size() - 1;
    }

    int32_t leaf_weight(int32_t x) {
        TNode t;
        t.kind = 1;
        t.src = x;
        if (total[(size_t)x] > 1) {
            t.vars = {x};
            t.cnt = {1};
            t.has_w = {1};
        }
        t.index_rank = net.degree[(size_t)x - 1];
        T.push_back(std::move(t));
        return (int32_t)T.size() - 1;
    }

    // storage rank of the merge of a and b (ignoring slicing)
    int32_t merged_rank(int32_t a, int32_t b) const {
        const TNode &A = T[(size_t)a], &B = T[(size_t)b];
        size_t i = 0, j = 0;
        int32_t r = 0;
        while (i < A.vars.size() || j < B.vars.size()) {
            if (j == B.vars.size() || (i < A.vars.size() && A.vars[i] < B.vars[j])) {
                ++r;
                ++i;
            } else if (i == A.vars.size() || B.vars[j] < A.vars[i]) {
                ++r;
                ++j;
            } else {
                if (A.cnt[i] + B.cnt[j] < total[(size_t)A.vars[i]]) ++r;
                ++i;
                ++j;
            }
        }
        return r;
    }

    int32_t merge(int32_t a, int32_t b) {
        TNode t;
        t.kind = 2;
        t.a = a;
        t.b = b;
        const TNode &A = T[(size_t)a], &B = T[(size_t)b];
        size_t i = 0, j = 0;
        auto push = [&](int32_t v, int32_t c, uint8_t h) {
            if (c < total[(size_t)v]) {
                t.vars.push_back(v);
                t.cnt.push_back(c);
                t.has_w.push_back(h);
            } else {
                t.kappa.push_back(v);
            }
        };
        while (i < A.vars.size() || j < B.vars.size()) {
            if (j == B.vars.size() || (i < A.vars.size() && A.vars[i] < B.vars[j])) {
                push(A.vars[i], A.cnt[i], A.has_w[i]);
                ++i;
            } else if (i == A.vars.size() || B.vars[j] < A.vars[i]) {
                push(B.vars[j], B.cnt[j], B.has_w[j]);
                ++j;
            } else {
                push(A.vars[i], A.cnt[i] + B.cnt[j], (uint8_t)(A.has_w[i] | B.has_w[j]));
                ++i;
                ++j;
            }
        }
        int32_t ir = 0;
        for (size_t q = 0; q < t.vars.size(); ++q)
            ir += t.has_w[q] ? total[(size_t)t.vars[q]] - t.cnt[q] : t.cnt[q];
        t.index_rank = ir;
        T.push_back(std::move(t));
        int32_t id = (int32_t)T.size() - 1;
        T[(size_t)a].parent = id;
        T[(size_t)b].parent = id;
        return id;
    }

    // Merge a set of tensors pairwise, each step taking the pair whose result
    // has the smallest rank (ties: smaller operands, then creation order).
    int32_t merge_all(std::vector<int32_t> bucket) {
        while (bucket.size() > 1) {
            size_t bi = 0, bj = 1;
            int64_t best_key[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
            for (size_t i = 0; i < bucket.size(); ++i)
                for (size_t j = i + 1; j < bucket.size(); ++j) {
                    int64_t k0 = merged_rank(bucket[i], bucket[j]);
                    int64_t k1 = (int64_t)T[(size_t)bucket[i]].vars.size() + (int64_t)T[(size_t)bucket[j]].vars.size();
                    int64_t k2 = (int64_t)std::min(bucket[i], bucket[j]) * 1000003 + std::max(bucket[i], bucket[j]);
                    if (k0 < best_key[0] || (k0 == best_key[0] && (k1 < best_key[1] || (k1 == best_key[1] && k2 < best_key[2])))) {
                        best_key[0] = k0;
                        best_key[1] = k1;
                        best_key[2] = k2;
                        bi = i;
                        bj = j;
                    }
                }
            int32_t m = merge(bucket[bi], bucket[bj]);
            bucket.erase(bucket.begin() + (std::ptrdiff_t)bj);
            bucket[bi] = m;
        }
        return bucket.empty() ? -1 : bucket[0];
    }
};

// Rank bookkeeping of a bucket merge without building tensors: the same
// greedy pair choice as TreeBuilder::merge_all; returns the largest rank of
// any tensor it would create.
struct SimT {
    std::vector<int32_t> vars, cnt;
};

static int32_t sim_merge_all(std::vector<SimT> b, const std::vector<int32_t> &total) {
    int32_t mx = 0;
    auto merged = [&](const SimT &A, const SimT &B, SimT *out) {
        int32_t r = 0;
        size_t i = 0, j = 0;
        while (i < A.vars.size() || j < B.vars.size()) {
            int32_t v, c;
            if (j == B.vars.size() || (i < A.vars.size() && A.vars[i] < B.vars[j])) {
                v = A.vars[i];
                c = A.cnt[i++];
            } else if (i == A.vars.size() || B.vars[j] < A.vars[i]) {
                v = B.vars[j];
                c = B.cnt[j++];
            } else {
                v = A.vars[i];
                c = A.cnt[i++] + B.cnt[j++];
            }
            if (c < total[(size_t)v]) {
                ++r;
                if (out) {
                    out->vars.push_back(v);
                    out->cnt.push_back(c);
                }
            }
        }
        return r;
    };
    while (b.size() > 1) {
        size_t bi = 0, bj = 1;
        int64_t k0b = INT64_MAX, k1b = INT64_MAX;
        for (size_t i = 0; i < b.size(); ++i)
            for (size_t j = i + 1; j < b.size(); ++j) {
                int64_t k0 = merged(b[i], b[j], nullptr);
                int64_t k1 = (int64_t)b[i].vars.size() + (int64_t)b[j].vars.size();
                if (k0 < k0b || (k0 == k0b && k1 < k1b)) {
                    k0b = k0;
                    k1b = k1;
                    bi = i;
                    bj = j;
                }
            }
        SimT m;
        merged(b[bi], b[bj], &m);
        mx = std::max(mx, (int32_t)m.vars.size());
        b.erase(b.begin() + (std::ptrdiff_t)bj);
        b[bi] = std::move(m);
    }
    return mx;
}

static int32_t bucket_tree_fixed(const wmc_network &net, const std::vector<int32_t> &order, int32_t block,
                                 int32_t rank_limit, std::vector<TNode> &T);

// Bucket tree from an elimination order: each step gathers every live tensor
// that holds one of the step's variables plus their weight leaves A_x, and
// merges the bucket pairwise.  A step eliminates up to `block` consecutive
// variables; a variable joins the current step only if it already occurs in
// the step's tensors and the step's merges (simulated) create no tensor of
// rank above the one-variable-per-step tree's maximum.
static int32_t bucket_tree(const wmc_network &net, const std::vector<int32_t> &order, int32_t block,
                           std::vector<TNode> &T) {
    if (block <= 1) return bucket_tree_fixed(net, order, 1, 0, T);
    std::vector<TNode> probe;
    int32_t r = bucket_tree_fixed(net, order, 1, 0, probe);
    if (r < 0) return bucket_tree_fixed(net, order, 1, 0, T);
    int32_t limit = 0;
    for (const TNode &t : probe) limit = std::max(limit, (int32_t)t.vars.size());
    return bucket_tree_fixed(net, order, block, limit, T);
}

static int32_t bucket_tree_fixed(const wmc_network &net, const std::vector<int32_t> &order, int32_t block,
                                 int32_t rank_limit, std::vector<TNode> &T) {
    TreeBuilder tb(net, T);
    const int32_t n = net.n;
    std::vector<uint8_t> alive;
    std::vector<std::vector<int32_t>> holders((size_t)n + 1);
    std::vector<int32_t> scalars;
    auto add_alive = [&](int32_t id) {
        if ((size_t)id >= alive.size()) alive.resize((size_t)id + 1, 0);
        alive[(size_t)id] = 1;
        if (T[(size_t)id].vars.empty()) scalars.push_back(id);
        for (int32_t v : T[(size_t)id].vars) holders[(size_t)v].push_back(id);
    };
    for (int32_t c = 0; c < (int32_t)net.clauses.size(); ++c) add_alive(tb.leaf_clause(c));
    std::vector<int32_t> wleaf((size_t)n + 1, -1);
    for (int32_t x = 1; x <= n; ++x)
        if (net.degree[(size_t)x - 1] == 0) add_alive(tb.leaf_weight(x));
    if (block < 1) block = 1;
    // live tensors holding any of the variables order[s..e)
    std::vector<int32_t> seen_stamp;
    int32_t stamp = 0;
    auto members = [&](size_t s, size_t e, std::vector<int32_t> &out) {
        ++stamp;
        if (seen_stamp.size() < T.size()) seen_stamp.resize(T.size(), 0);
        out.clear();
        for (size_t q = s; q < e; ++q) {
            int32_t x = order[q];
            for (int32_t id : holders[(size_t)x]) {
                if (!alive[(size_t)id] || seen_stamp[(size_t)id] == stamp) continue;
                const std::vector<int32_t> &vs = T[(size_t)id].vars;
                if (!std::binary_search(vs.begin(), vs.end(), x)) continue;
                seen_stamp[(size_t)id] = stamp;
                out.push_back(id);
            }
        }
    };
    std::vector<int32_t> cand;
    for (size_t s = 0; s < order.size();) {
        size_t e = s + 1;
        while (block > 1 && e < order.size() && e < s + (size_t)block) {
            // the next variable must already occur in the step's tensors, so
            // the step's result is what eliminating it next would give anyway
            members(s, e, cand);
            bool adjacent = false;
            for (int32_t id : cand) {
                const std::vector<int32_t> &vs = T[(size_t)id].vars;
                if (std::binary_search(vs.begin(), vs.end(), order[e])) adjacent = true;
            }
            if (!adjacent) break;
            members(s, e + 1, cand);
            std::vector<SimT> sim;
            for (int32_t id : cand) sim.push_back({T[(size_t)id].vars, T[(size_t)id].cnt});
            for (size_t q = s; q <= e; ++q) {
                int32_t x = order[q];
                if (net.degree[(size_t)x - 1] > 0) sim.push_back({{x}, {1}});
            }
            if (sim_merge_all(sim, tb.total) > rank_limit) break;
            ++e;
        }
        std::vector<int32_t> bucket;
        for (size_t q = s; q < e; ++q) {
            int32_t x = order[q];
            if (net.degree[(size_t)x - 1] == 0) continue;
            for (int32_t id : holders[(size_t)x]) {
                if (!alive[(size_t)id]) continue;
                const std::vector<int32_t> &vs = T[(size_t)id].vars;
                if (!std::binary_search(vs.begin(), vs.end(), x)) continue;
                alive[(size_t)id] = 0;
                bucket.push_back(id);
            }
            holders[(size_t)x].clear();
            int32_t wl = tb.leaf_weight(x);
            if ((size_t)wl >= alive.size()) alive.resize((size_t)wl + 1, 0);
            bucket.push_back(wl);
        }
        s = e;
        if (bucket.empty()) continue;
        std::sort(bucket.begin(), bucket.end());
        int32_t r = tb.merge_all(bucket);
        add_alive(r);
    }
    std::vector<int32_t> rest;
    for (size_t id = 0; id < alive.size(); ++id)
        if (alive[id]) rest.push_back((int32_t)id);
    for (int32_t id : rest)
        if (!T[(size_t)id].vars.empty()) return -2;  // order did not cover every variable
    if (rest.empty()) return -1;
    int32_t root = rest[0];
    for (size_t i = 1; i < rest.size(); ++i) root = tb.merge(root, rest[i]);
    return root;
}

// Explicit tree: vertices 0..n-1 = A_x, n..n+m-1 = B_C, then internal vertices.
static wmc_status explicit_tree(const wmc_network &net, const int64_t *parent, int64_t n_nodes,
                                std::vector<TNode> &T, int32_t *root_out) {
    const int64_t L = (int64_t)net.n + (int64_t)net.clauses.size();
    if (L == 0) {
        if (n_nodes != 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: expected 0 vertices");
        *root_out = -1;
        return WMC_OK;
    }
    if (!parent || n_nodes != 2 * L - 1)
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: expected %lld vertices, got %lld",
                 (long long)(2 * L - 1), (long long)n_nodes);
    std::vector<std::vector<int64_t>> kids((size_t)n_nodes);
    int64_t root = -1;
    for (int64_t v = 0; v < n_nodes; ++v) {
        int64_t p = parent[v];
        if (p == -1) {
            if (root >= 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: two roots (%lld, %lld)",
                                    (long long)root, (long long)v);
            root = v;
            continue;
        }
        if (p < L || p >= n_nodes || p == v)
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: vertex %lld has invalid parent %lld",
                     (long long)v, (long long)p);
        kids[(size_t)p].push_back(v);
    }
    if (root < 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: no root");
    if (L == 1) {
        if (root != 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: single leaf must be the root");
    } else if (root < L) {
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: root is a leaf");
    }
    for (int64_t v = L; v < n_nodes; ++v)
        if (kids[(size_t)v].size() != 2)
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: internal vertex %lld has %zu children",
                     (long long)v, kids[(size_t)v].size());
    TreeBuilder tb(net, T);
    std::vector<int32_t> tid((size_t)n_nodes, -1);
    for (int32_t x = 1; x <= net.n; ++x) tid[(size_t)x - 1] = tb.leaf_weight(x);
    for (int64_t c = 0; c < (int64_t)net.clauses.size(); ++c) tid[(size_t)(net.n + c)] = tb.leaf_clause((int32_t)c);
    // post-order from the root (iterative), which also rejects cycles
    std::vector<std::pair<int64_t, int>> stack;
    stack.push_back({root, 0});
    int64_t visited = 0;
    std::vector<uint8_t> seen((size_t)n_nodes, 0);
    while (!stack.empty()) {
        auto &top = stack.back();
        int64_t v = top.first;
        if (v < L) {
            if (seen[(size_t)v]++) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: vertex reached twice");
            ++visited;
            stack.pop_back();
            continue;
        }
        if (top.second < 2) {
            int64_t c = kids[(size_t)v][(size_t)top.second++];
            if (seen[(size_t)c]) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: cycle");
            stack.push_back({c, 0});
            continue;
        }
        seen[(size_t)v] = 1;
        ++visited;
        tid[(size_t)v] = tb.merge(tid[(size_t)kids[(size_t)v][0]], tid[(size_t)kids[(size_t)v][1]]);
        stack.pop_back();
    }
    if (visited != n_nodes) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "explicit tree: not connected");
    *root_out = tid[(size_t)root];
    return WMC_OK;
}

// ---------------------------------------------------------------------------
// Lowered sizes under a slice set I
// ---------------------------------------------------------------------------
static inline bool is_sliced(const std::vector<uint8_t> &sl, int32_t v) { return sl[(size_t)v] != 0; }

static int32_t srank(const TNode &t, const std::vector<uint8_t> &sl) {
    int32_t r = 0;
    for (int32_t v : t.vars) r += !is_sliced(sl, v);
    return r;
}

static int32_t skappa(const TNode &t, const std::vector<uint8_t> &sl) {
    int32_t r = 0;
    for (int32_t v : t.kappa) r += !is_sliced(sl, v);
    return r;
}

// Node class from storage ranks: tiny nodes are batched many per launch;
// nodes with a real matrix shape (summed and column dimensions of at least
// 4, product at least 64, columns at most 128) run on MFMA; the rest
// (Hadamard, outer products, a single summed variable) stream.
static int32_t node_class(int32_t ra, int32_t rb, int32_t rc, int32_t nk) {
    int32_t mx = std::max(ra, std::max(rb, rc));
    if (mx <= 14 && rc + nk <= 18) return WMC_CLASS_SMALL;
    int32_t nb = ra + rb - rc - 2 * nk;
    int32_t nn = std::min(ra, rb) - nk - nb;  // columns: variables of the smaller operand only
    int32_t nm = std::max(ra, rb) - nk - nb;
    // matrix cores pay only with at least 16 summed entries (below that the
    // node is HBM-bound and streams) and for few batch bits: with many, each
    // workgroup owns a short matrix per batch index and the batch bits land
    // in the low address bits of the output, where the streaming kernel's
    // C-ordered stores do better (measured on banded formulas)
    if (nk >= 4 && nn >= 2 && nk + nn >= 6 && nn <= 7 && nm + nb >= 4 && nb <= 6) return WMC_CLASS_GEMM;
    return WMC_CLASS_STREAM;
}

// Compress (src, dst) bit pairs, src = 0, 1, 2, ... into runs where both advance together.
static bool make_runs(const std::vector<int32_t> &dst, unsigned char (*runs)[3], int *nrun, int cap) {
    int nr = 0;
    for (size_t t = 0; t < dst.size();) {
        size_t u = t + 1;
        while (u < dst.size() && dst[u] == dst[u - 1] + 1) ++u;
        if (nr >= cap) return false;
        runs[nr][0] = (unsigned char)t;
        runs[nr][1] = (unsigned char)(u - t);
        runs[nr][2] = (unsigned char)dst[t];
        ++nr;
        t = u;
    }
    *nrun = nr;
    return true;
}

// Matrix form of node id for the MFMA kernel, read off the layouts: the row
// operand A is stored [4 lowest mu variables | kappa | rest in C order] and
// the column operand B [kappa | rest in C order].  False if the shapes do not
// match that form or a run list overflows.
static bool make_gemm(const std::vector<TNode> &T, int32_t id, int32_t xa, const std::vector<uint8_t> &sl,
                      GemmDesc &g) {
    const TNode &C = T[(size_t)id];
    const int32_t xb = (xa == C.a) ? C.b : C.a;
    const TNode &A = T[(size_t)xa], &B = T[(size_t)xb];
    std::memset(&g, 0, sizeof g);
    g.a = A.off;
    g.b = B.off;
    g.c = C.off;
    g.ta = xa;
    g.tb = xb;
    g.tc = id;
    g.nk = skappa(C, sl);
    const int32_t nk = g.nk;
    auto pos_in = [](const std::vector<int32_t> &L, int32_t v, size_t from) -> int32_t {
        for (size_t q = from; q < L.size(); ++q)
            if (L[q] == v) return (int32_t)(q - from);
        return -1;
    };
    if ((int32_t)A.layout.size() < 4 + nk || (int32_t)B.layout.size() < nk) return false;
    for (int32_t q = 0; q < nk; ++q)
        if (A.layout[(size_t)(4 + q)] != B.layout[(size_t)q]) return false;
    std::vector<int32_t> mu_a, beta_a, nu_b, beta_b, mu_c, nu_c, beta_c;
    int32_t nmu = 0;
    for (size_t j = 0; j < C.layout.size(); ++j) {
        int32_t v = C.layout[j];
        int32_t pa = pos_in(A.layout, v, 0), pb = pos_in(B.layout, v, 0);
        if (pa >= 0 && pb >= 0) {
            if (pa < 4 + nk || pb < nk) return false;
            beta_a.push_back(pa - 4 - nk);
            beta_b.push_back(pb - nk);
            beta_c.push_back((int32_t)j);
        } else if (pa >= 0) {
            if (nmu < 4) {
                if (pa != nmu) return false;  // the 4 lowest mu variables sit at A's bits 0..3
            } else {
                if (pa < 4 + nk) return false;
                mu_a.push_back(pa - 4 - nk);
            }
            ++nmu;
            mu_c.push_back((int32_t)j);
        } else {
            if (pb < nk) return false;
            nu_b.push_back(pb - nk);
            nu_c.push_back((int32_t)j);
        }
    }
    g.nm = (int)mu_c.size();
    g.nn = (int)nu_c.size();
    g.nb = (int)beta_c.size();
    if (g.nm < 4) return false;
    const std::vector<int32_t> *lists[GR_N] = {&mu_a, &beta_a, &nu_b, &beta_b, &mu_c, &nu_c, &beta_c};
    for (int q = 0; q < GR_N; ++q)
        if (!make_runs(*lists[q], g.run[q], &g.nrun[q], WMC_GEMM_RUNS)) return false;
    return (int32_t)A.layout.size() == nk + g.nb + g.nm && (int32_t)B.layout.size() == nk + g.nb + g.nn;
}

// Post-order-compatible launch schedule: all ready small nodes go in one
// batched launch, big nodes one per launch.  Returns internal tensors in
// launch order and fills launch index per tensor (birth).
struct Schedule {
    std::vector<int32_t> order;            // internal tensors in launch order
    std::vector<std::pair<int32_t, int32_t>> launches;  // [first, count) into order
};

static Schedule make_schedule(const std::vector<TNode> &T, const std::vector<int32_t> &cls) {
    Schedule S;
    const size_t NT = T.size();
    std::vector<int32_t> pending(NT, 0);
    std::vector<int32_t> ready_small, ready_big;
    size_t n_internal = 0;
    for (size_t i = 0; i < NT; ++i)
        if (T[i].kind == 2) {
            ++n_internal;
            pending[i] = (T[(size_t)T[i].a].kind == 2) + (T[(size_t)T[i].b].kind == 2);
            if (pending[i] == 0) (cls[i] == WMC_CLASS_SMALL ? ready_small : ready_big).push_back((int32_t)i);
        }
    auto finish = [&](int32_t id) {
        int32_t p = T[(size_t)id].parent;
        if (p >= 0 && --pending[(size_t)p] == 0)
            (cls[(size_t)p] == WMC_CLASS_SMALL ? ready_small : ready_big).push_back(p);
    };
    while (S.order.size() < n_internal) {
        if (!ready_small.empty()) {
            std::vector<int32_t> batch;
            batch.swap(ready_small);
            std::sort(batch.begin(), batch.end());
            S.launches.push_back({(int32_t)S.order.size(), (int32_t)batch.size()});
            for (int32_t id : batch) S.order.push_back(id);
            for (int32_t id : batch) finish(id);
        } else {
            auto it = std::min_element(ready_big.begin(), ready_big.end());
            int32_t id = *it;
            ready_big.erase(it);
            S.launches.push_back({(int32_t)S.order.size(), 1});
            S.order.push_back(id);
            finish(id);
        }
    }
    return S;
}

// Peak of live tensor bytes over a schedule (MemCost of Algorithm 3).
static double peak_live(const std::vector<TNode> &T, const Schedule &S, const std::vector<uint8_t> &sl,
                        int32_t elem, int32_t root, bool aligned = false) {
    const size_t NL = S.launches.size();
    // launch 0 is the leaf fill; node launch k is index k+1
    std::vector<double> delta(NL + 3, 0.0);
    std::vector<int32_t> birth(T.size(), 0);
    for (size_t k = 0; k < NL; ++k)
        for (int32_t q = 0; q < S.launches[k].second; ++q)
            birth[(size_t)S.order[(size_t)(S.launches[k].first + q)]] = (int32_t)k + 1;
    for (size_t i = 0; i < T.size(); ++i) {
        double b = (double)elem * std::ldexp(1.0, srank(T[i], sl));
        if (aligned) b = std::max(b, 256.0);
        int32_t death = ((int32_t)i == root || T[i].parent < 0) ? (int32_t)NL + 1 : birth[(size_t)T[i].parent];
        delta[(size_t)birth[i]] += b;
        delta[(size_t)death + 1] -= b;
    }
    double cur = 0.0, peak = 0.0;
    for (size_t k = 0; k < delta.size(); ++k) {
        cur += delta[k];
        peak = std::max(peak, cur);
    }
    return peak;
}

static double flops_of(const std::vector<TNode> &T, const std::vector<uint8_t> &sl) {
    double f = 0.0;
    for (const TNode &t : T)
        if (t.kind == 2) f += 2.0 * std::ldexp(1.0, srank(t, sl) + skappa(t, sl));
    return f;
}

static int32_t max_rank_of(const std::vector<TNode> &T, const std::vector<uint8_t> &sl) {
    int32_t r = 0;
    for (const TNode &t : T) r = std::max(r, srank(t, sl));
    return r;
}

static std::vector<int32_t> classes_of(const std::vector<TNode> &T, const std::vector<uint8_t> &sl) {
    std::vector<int32_t> cls(T.size(), -1);
    for (size_t i = 0; i < T.size(); ++i)
        if (T[i].kind == 2)
            cls[i] = node_class(srank(T[(size_t)T[i].a], sl), srank(T[(size_t)T[i].b], sl), srank(T[i], sl),
                                skappa(T[i], sl));
    return cls;
}

// ---------------------------------------------------------------------------
// wmc_plan
// ---------------------------------------------------------------------------
static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Static arena of a schedule: each tensor lives from the launch that writes
// it (leaves: the leaf fill, launch 0) to the launch that reads it, and is
// placed first-fit over the tensors whose lifetimes overlap its own, largest
// first, each 256-byte aligned.  Returns the arena bytes; offs (optional)
// receives every tensor's element offset.  This is MemCost of Algorithm 3
// as the device sees it: the memory one slice's tensors occupy.
static uint64_t place_arena(const std::vector<TNode> &T, const Schedule &S, const std::vector<uint8_t> &sl,
                            int32_t elem, std::vector<int64_t> *offs) {
    const size_t NT = T.size();
    std::vector<int32_t> birth(NT, 0), death(NT, 0);
    for (size_t k = 0; k < S.launches.size(); ++k)
        for (int32_t q = 0; q < S.launches[k].second; ++q)
            birth[(size_t)S.order[(size_t)(S.launches[k].first + q)]] = (int32_t)k + 1;
    const int32_t NL = (int32_t)S.launches.size() + 1;
    for (size_t i = 0; i < NT; ++i) death[i] = (T[i].parent < 0) ? NL : birth[(size_t)T[i].parent];
    const uint64_t align_elems = 256 / (uint64_t)elem;
    std::vector<int32_t> by_size(NT);
    std::iota(by_size.begin(), by_size.end(), 0);
    std::vector<uint64_t> elems(NT);
    for (size_t i = 0; i < NT; ++i) elems[i] = align_up((uint64_t)1 << srank(T[i], sl), align_elems);
    std::stable_sort(by_size.begin(), by_size.end(), [&](int32_t a, int32_t b) {
        if (elems[(size_t)a] != elems[(size_t)b]) return elems[(size_t)a] > elems[(size_t)b];
        return birth[(size_t)a] < birth[(size_t)b];
    });
    std::vector<int64_t> off(NT, 0);
    std::vector<int32_t> placed;
    uint64_t arena_elems = 0;
    std::vector<std::pair<uint64_t, uint64_t>> busy;
    for (int32_t t : by_size) {
        busy.clear();
        for (int32_t p : placed) {
            if (death[(size_t)p] < birth[(size_t)t] || death[(size_t)t] < birth[(size_t)p]) continue;
            busy.push_back({(uint64_t)off[(size_t)p], (uint64_t)off[(size_t)p] + elems[(size_t)p]});
        }
        std::sort(busy.begin(), busy.end());
        uint64_t o = 0;
        for (auto &iv : busy) {
            if (iv.first >= o + elems[(size_t)t]) break;
            o = std::max(o, iv.second);
        }
        off[(size_t)t] = (int64_t)o;
        arena_elems = std::max(arena_elems, o + elems[(size_t)t]);
        placed.push_back(t);
    }
    if (offs) offs->swap(off);
    return arena_elems * (uint64_t)elem;
}

// Peak of live tensor bytes, sizes 256-byte aligned, over the schedule the
// slice set sl executes (its node classes decide which small nodes share a
// launch): the lower bound the arena placement reaches at best.
static double peak_live_aligned(const std::vector<TNode> &T, const std::vector<uint8_t> &sl, int32_t elem,
                                int32_t root) {
    const Schedule S = make_schedule(T, classes_of(T, sl));
    return peak_live(T, S, sl, elem, root, true);
}

// Excess over the rank cap: sum over tensors above it of 2^(rank - cap).
static double rank_excess(const std::vector<TNode> &T, const std::vector<uint8_t> &sl, int32_t cap) {
    double e = 0.0;
    for (const TNode &t : T) {
        const int32_t r = srank(t, sl);
        if (r > cap) e += std::ldexp(1.0, r - cap);
    }
    return e;
}

// Fewest sliced variables that bring every storage rank to the cap, sets of
// exactly k variables: the greedy growth of Algorithm 3 ranks candidates by
// MemCost, not by how many over-cap tensors they reach, and can end with
// more variables than the cap needs (every one doubles the slices).  Each
// sliced variable lowers a tensor's rank by at most one, so a set must hold
// at least (rank - cap) variables of every tensor; the search branches on
// the variables of the tensor furthest above the cap and drops a branch as
// soon as some tensor is further above it than the variables left.  The
// distinct sets found (at most max_sets) go to `accept`, which returns false
// to stop; every search step spends one unit of `budget` per over-cap
// tensor it checks, and the search ends when the budget is gone.
template <typename Accept>
static void slice_sets_of_size(const std::vector<const TNode *> &hot, int32_t n, int32_t cap, int32_t k,
                               long long &budget, size_t max_sets, Accept accept) {
    std::vector<uint8_t> s((size_t)n + 1, 0);
    std::vector<int32_t> chosen;
    std::vector<std::vector<int32_t>> seen;
    bool stop = false;
    auto dfs = [&](auto &&self, int32_t left) -> void {
        if (stop || budget <= 0) return;
        budget -= (long long)hot.size();
        int32_t worst = 0;
        const TNode *w = nullptr;
        for (const TNode *t : hot) {
            const int32_t e = srank(*t, s) - cap;
            if (e > worst) {
                worst = e;
                w = t;
            }
        }
        if (worst == 0) {
            std::vector<int32_t> I = chosen;
            std::sort(I.begin(), I.end());
            if (std::find(seen.begin(), seen.end(), I) != seen.end()) return;
            seen.push_back(I);
            if (!accept(I) || seen.size() >= max_sets) stop = true;
            return;
        }
        if (worst > left) return;
        for (int32_t v : w->vars) {
            if (s[(size_t)v]) continue;
            s[(size_t)v] = 1;
            chosen.push_back(v);
            self(self, left - 1);
            chosen.pop_back();
            s[(size_t)v] = 0;
            if (stop) return;
        }
    };
    dfs(dfs, k);
}

static wmc_status finalize_plan(const wmc_network &net, const wmc_plan_options &o, wmc_plan_t &P) {
    std::vector<TNode> &T = P.T;
    const size_t NT = T.size();
    const int32_t n = net.n;
    std::vector<uint8_t> sl((size_t)n + 1, 0);

    // ---- slicing (Algorithm 3): grow I greedily while the cap is exceeded.
    // The rank cap bounds the largest storage rank; the memory cap bounds
    // MemCost, the placed arena of the schedule this slice set executes
    // (node classes, and with them which small nodes share a launch, depend
    // on the slice set, so the schedule is rebuilt for every check).
    const int32_t rank0 = max_rank_of(T, sl);
    int32_t idx_rank = 0;
    for (const TNode &t : T) idx_rank = std::max(idx_rank, t.index_rank);
    const int32_t objective = o.slice_objective;  // WMC_SLICE_BY_MEMORY or WMC_SLICE_BY_FLOPS
    if (objective < 0 || objective > 1)
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: slice objective %d (0 = memory, 1 = flops)", objective);
    auto rank_over = [&](const std::vector<uint8_t> &s) { return o.rank_cap > 0 && max_rank_of(T, s) > o.rank_cap; };
    auto mem_over = [&](const std::vector<uint8_t> &s) {
        if (o.mem_cap_bytes == 0) return false;
        const Schedule S = make_schedule(T, classes_of(T, s));
        return place_arena(T, S, s, P.elem, nullptr) > o.mem_cap_bytes;
    };
    auto over = [&](const std::vector<uint8_t> &s) { return rank_over(s) || mem_over(s); };
    // how far a slice set is from the caps (0 once both hold): rank excess
    // first, then the aligned peak of live bytes above the memory cap
    auto excess = [&](const std::vector<uint8_t> &s) {
        double e = o.rank_cap > 0 ? 1e30 * rank_excess(T, s, o.rank_cap) : 0.0;
        if (o.mem_cap_bytes > 0) e += std::max(0.0, peak_live_aligned(T, s, P.elem, P.root) - (double)o.mem_cap_bytes);
        return e;
    };
    if (o.mem_cap_bytes > 0) {
        // every leaf is live during the leaf fill and takes at least 256
        // bytes, whatever is sliced: below that no slice set meets the cap
        uint64_t floor_bytes = 0;
        for (const TNode &t : T) floor_bytes += t.kind != 2 ? 256 : 0;
        if (floor_bytes > o.mem_cap_bytes)
            WMC_FAIL(WMC_ERR_CAP_UNREACHABLE, "wmc_plan: cap %llu below the %llu bytes the leaves occupy",
                     (unsigned long long)o.mem_cap_bytes, (unsigned long long)floor_bytes);
    }
    // greedy growth of I with one criterion (0: memory, 1: flops), then, for
    // the flops criterion, dropping the variables the caps no longer need
    auto grow = [&](int32_t crit, std::vector<int32_t> &I) -> wmc_status {
        std::vector<uint8_t> s2((size_t)n + 1, 0);
        for (int32_t v : I) s2[(size_t)v] = 1;
        while (over(s2)) {
            if ((int32_t)I.size() >= WMC_MAX_SLICED)
                WMC_FAIL(WMC_ERR_CAP_UNREACHABLE, "wmc_plan: cap not met after slicing %d variables", WMC_MAX_SLICED);
            // candidates: variables of the tensors within one of the maximum rank
            int32_t mr = max_rank_of(T, s2);
            if (mr == 0) WMC_FAIL(WMC_ERR_CAP_UNREACHABLE, "wmc_plan: cap below the arena of rank-0 tensors");
            std::vector<uint8_t> cand((size_t)n + 1, 0);
            for (const TNode &t : T)
                if (srank(t, s2) >= mr - 1)
                    for (int32_t v : t.vars)
                        if (!s2[(size_t)v]) cand[(size_t)v] = 1;
            const double ex0 = crit == 1 ? excess(s2) : 0.0;
            int32_t best = -1;
            double best_key = 0, best_tie = 0;
            for (int32_t v = 1; v <= n; ++v) {
                if (!cand[(size_t)v]) continue;
                s2[(size_t)v] = 1;
                double key, tie;
                if (crit == 0) {
                    // Algorithm 3's ChooseSliceIndex: least MemCost (aligned
                    // peak of live bytes on the executed schedule), ties by flops
                    key = peak_live_aligned(T, s2, P.elem, P.root);
                    if (o.rank_cap > 0) key += 1e30 * (double)std::max(0, max_rank_of(T, s2) - o.rank_cap);
                    tie = flops_of(T, s2);
                } else {
                    // least summed flops over all slices among the variables
                    // that bring the slice set closer to the caps
                    const double ex = excess(s2);
                    key = ex < ex0 ? std::ldexp(flops_of(T, s2), (int)I.size() + 1) : HUGE_VAL;
                    tie = ex;
                }
                s2[(size_t)v] = 0;
                if (best < 0 || key < best_key || (key == best_key && tie < best_tie)) {
                    best = v;
                    best_key = key;
                    best_tie = tie;
                }
            }
            if (best < 0) WMC_FAIL(WMC_ERR_CAP_UNREACHABLE, "wmc_plan: no variable left to slice");
            s2[(size_t)best] = 1;
            I.push_back(best);
        }
        if (objective == 1) {
            for (size_t q = I.size(); q-- > 0;) {
                const int32_t v = I[q];
                s2[(size_t)v] = 0;
                if (over(s2)) s2[(size_t)v] = 1;
                else I.erase(I.begin() + (long)q);
            }
        }
        return WMC_OK;
    };
    {
        std::vector<int32_t> I0;
        wmc_status st = grow(0, I0);
        if (st != WMC_OK) return st;
        if (objective == 1) {
            // the flops criterion keeps whichever of the two greedy slice
            // sets (both pruned) does less work over all its slices
            std::vector<int32_t> I1;
            if (grow(1, I1) == WMC_OK) {
                auto work = [&](const std::vector<int32_t> &I) {
                    std::vector<uint8_t> s2((size_t)n + 1, 0);
                    for (int32_t v : I) s2[(size_t)v] = 1;
                    return std::ldexp(flops_of(T, s2), (int)I.size());
                };
                if (work(I1) < work(I0)) I0.swap(I1);
            }
        }
        // (not past 24 variables: such plans run millions of slices either way)
        if (o.rank_cap > 0 && (int32_t)I0.size() > rank0 - o.rank_cap && I0.size() <= 24) {
            // fewer variables may meet the caps: sizes one below the current
            // set's, downwards, each size's sets ranked by the growth's own
            // criterion.  Slicing more never breaks a cap, so once a size has
            // no set (or the search budget is gone) no smaller one has.
            std::vector<const TNode *> hot;
            for (const TNode &t : T)
                if (srank(t, sl) > o.rank_cap) hot.push_back(&t);
            std::vector<uint8_t> s2((size_t)n + 1, 0);
            long long budget = 150000000;  // tensor checks over all sizes (about a second at most)
            for (int32_t k = (int32_t)I0.size() - 1; k >= rank0 - o.rank_cap && budget > 0; --k) {
                std::vector<int32_t> best;
                double best_key = 0, best_tie = 0;
                slice_sets_of_size(hot, n, o.rank_cap, k, budget, 64, [&](const std::vector<int32_t> &I) {
                    for (int32_t v : I) s2[(size_t)v] = 1;
                    if (!over(s2)) {
                        const double key = objective == 1 ? flops_of(T, s2) : peak_live_aligned(T, s2, P.elem, P.root);
                        const double tie = objective == 1 ? peak_live_aligned(T, s2, P.elem, P.root) : flops_of(T, s2);
                        if (best.empty() || key < best_key || (key == best_key && tie < best_tie)) {
                            best = I;
                            best_key = key;
                            best_tie = tie;
                        }
                    }
                    for (int32_t v : I) s2[(size_t)v] = 0;
                    return true;
                });
                if (best.empty()) break;
                I0 = best;
            }
        }
        P.sliced = I0;
        for (int32_t v : I0) sl[(size_t)v] = 1;
    }
    const int32_t rankS = max_rank_of(T, sl);
    if (rankS > WMC_MAX_RANK)
        WMC_FAIL(WMC_ERR_UNSUPPORTED, "wmc_plan: storage rank %d exceeds %d (set rank_cap or mem_cap)", rankS,
                 WMC_MAX_RANK);
    std::vector<int32_t> sbit((size_t)n + 1, -1);
    for (size_t i = 0; i < P.sliced.size(); ++i) sbit[(size_t)P.sliced[i]] = (int32_t)i;

    // ---- layouts, top-down.  An operand normally stores [kappa | its
    // variables in the order of the node's output]; the row operand of a
    // matrix-class node stores [its 4 lowest mu variables | kappa | rest], so
    // that 16 rows of one summed index are contiguous.  The root is a scalar.
    std::vector<int32_t> cls = classes_of(T, sl);
    std::vector<int32_t> gemm_a(NT, -1);
    if (P.root >= 0) {
        T[(size_t)P.root].layout.clear();
        for (int32_t v : T[(size_t)P.root].vars)
            if (!sl[(size_t)v]) T[(size_t)P.root].layout.push_back(v);
        std::vector<int32_t> stack = {P.root};
        std::vector<int32_t> mark((size_t)n + 1, 0);
        int32_t stamp = 0;
        while (!stack.empty()) {
            int32_t q = stack.back();
            stack.pop_back();
            TNode &C = T[(size_t)q];
            if (C.kind != 2) continue;
            std::vector<int32_t> kap;
            for (int32_t v : C.kappa)
                if (!sl[(size_t)v]) kap.push_back(v);
            auto plain = [&](int32_t child) {
                TNode &X = T[(size_t)child];
                ++stamp;
                for (int32_t v : X.vars) mark[(size_t)v] = stamp;
                X.layout = kap;
                for (int32_t v : C.layout)
                    if (mark[(size_t)v] == stamp) X.layout.push_back(v);
            };
            bool done = false;
            if (cls[(size_t)q] == WMC_CLASS_GEMM) {
                int32_t xa = C.a, xb = C.b;
                if (srank(T[(size_t)xb], sl) > srank(T[(size_t)xa], sl)) std::swap(xa, xb);
                plain(xb);
                TNode &A = T[(size_t)xa];
                ++stamp;
                for (int32_t v : A.vars) mark[(size_t)v] = stamp;
                const int32_t sB = stamp;
                (void)sB;
                std::vector<int32_t> lo, rest;
                std::vector<uint8_t> inB((size_t)n + 1, 0);
                for (int32_t v : T[(size_t)xb].vars) inB[(size_t)v] = 1;
                for (int32_t v : C.layout) {
                    if (mark[(size_t)v] != stamp) continue;
                    if (!inB[(size_t)v] && lo.size() < 4) lo.push_back(v);
                    else rest.push_back(v);
                }
                if (lo.size() == 4) {
                    A.layout = lo;
                    A.layout.insert(A.layout.end(), kap.begin(), kap.end());
                    A.layout.insert(A.layout.end(), rest.begin(), rest.end());
                    GemmDesc probe;
                    if (make_gemm(T, q, xa, sl, probe)) {
                        gemm_a[(size_t)q] = xa;
                        done = true;
                    }
                }
                if (!done) cls[(size_t)q] = WMC_CLASS_STREAM;
            }
            if (!done) {
                plain(C.a);
                plain(C.b);
            }
            for (int32_t child : {C.a, C.b}) {
                if ((int32_t)T[(size_t)child].layout.size() != srank(T[(size_t)child], sl))
                    WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: internal layout mismatch at tensor %d", child);
                stack.push_back(child);
            }
        }
    }

    // ---- schedule
    Schedule S = make_schedule(T, cls);
    P.node_order = S.order;
    P.launches.clear();
    P.launches.push_back({LAUNCH_LEAF, 0, 0, 0, 0});
    for (size_t k = 0; k < S.launches.size(); ++k)
        P.launches.push_back({LAUNCH_NODES, S.launches[k].first, S.launches[k].second, 0, 0});
    for (size_t i = 0; i < NT; ++i) T[i].birth = 0;
    for (size_t k = 0; k < S.launches.size(); ++k)
        for (int32_t q = 0; q < S.launches[k].second; ++q)
            T[(size_t)S.order[(size_t)(S.launches[k].first + q)]].birth = (int32_t)k + 1;
    const int32_t NL = (int32_t)P.launches.size();
    for (size_t i = 0; i < NT; ++i) {
        T[i].death = (T[i].parent < 0) ? NL : T[(size_t)T[i].parent].birth;
        if (T[i].kind == 2) T[i].cls = cls[i];
    }

    // ---- static arena: greedy placement by size over lifetime intervals
    std::vector<int64_t> offs;
    P.arena_bytes = place_arena(T, S, sl, P.elem, &offs);
    for (size_t i = 0; i < NT; ++i) T[i].off = offs[i];
    if (o.mem_cap_bytes > 0 && P.arena_bytes > o.mem_cap_bytes)
        WMC_FAIL(WMC_ERR_CAP_UNREACHABLE, "wmc_plan: internal arena %llu above the cap %llu",
                 (unsigned long long)P.arena_bytes, (unsigned long long)o.mem_cap_bytes);

    // ---- descriptors
    P.leaves.clear();
    P.nodes.clear();
    int64_t lw = 0;
    for (size_t i = 0; i < NT; ++i) {
        const TNode &X = T[i];
        if (X.kind == 2) continue;
        LeafDesc d;
        std::memset(&d, 0, sizeof d);
        d.out = X.off;
        d.work_begin = lw;
        d.tensor = (int32_t)i;
        d.rank = (int32_t)X.layout.size();
        for (int q = 0; q < WMC_LEAF_VARS; ++q) d.pos[q] = 0;
        auto pos_of = [&](int32_t v) -> int16_t {
            if (sl[(size_t)v]) return (int16_t)(-(1 + sbit[(size_t)v]));
            for (size_t q = 0; q < X.layout.size(); ++q)
                if (X.layout[q] == v) return (int16_t)q;
            return (int16_t)-1000;
        };
        if (X.kind == 0) {
            const WClause &c = net.clauses[(size_t)X.src];
            d.kind = WMC_LEAF_CLAUSE;
            d.k = (int32_t)c.vars.size();
            d.falsify = c.falsify;
            d.taut = c.taut ? 1 : 0;
            for (size_t q = 0; q < c.vars.size(); ++q) d.pos[q] = pos_of(c.vars[q]);
        } else {
            d.var = X.src - 1;
            if (X.vars.empty()) {
                d.kind = WMC_LEAF_WEIGHT_CLOSED;
            } else {
                d.kind = WMC_LEAF_WEIGHT;
                d.k = 1;
                d.pos[0] = pos_of(X.src);
            }
        }
        lw += (int64_t)align_up((uint64_t)1 << d.rank, WMC_WAVE);
        P.leaves.push_back(d);
    }
    P.leaf_work = lw;
    P.launches[0].work = lw;
    P.gemms.clear();
    for (size_t k = 1; k < P.launches.size(); ++k) {
        Launch &L = P.launches[k];
        if (L.count != 1) continue;
        int32_t id = P.node_order[(size_t)L.first];
        if (T[(size_t)id].cls != WMC_CLASS_GEMM) continue;
        GemmDesc g;
        if (!make_gemm(T, id, gemm_a[(size_t)id], sl, g))
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: internal matrix descriptor mismatch at node %d", id);
        L.type = LAUNCH_GEMM;
        L.pad = (int32_t)P.gemms.size();
        P.gemms.push_back(g);
    }
    std::vector<int32_t> mark((size_t)n + 1, 0);
    int32_t stamp = 0;
    for (size_t k = 1; k < P.launches.size(); ++k) {
        Launch &L = P.launches[k];
        int64_t work = 0;
        for (int32_t q = 0; q < L.count; ++q) {
            int32_t id = P.node_order[(size_t)(L.first + q)];
            const TNode &C = T[(size_t)id];
            NodeDesc d;
            std::memset(&d, 0, sizeof d);
            d.a = T[(size_t)C.a].off;
            d.b = T[(size_t)C.b].off;
            d.c = C.off;
            d.ta = C.a;
            d.tb = C.b;
            d.tc = id;
            d.rc = (int32_t)C.layout.size();
            d.nk = skappa(C, sl);
            d.cls = C.cls;
            d.work_begin = work;
            for (int which = 0; which < 2; ++which) {
                const TNode &X = T[(size_t)(which ? C.b : C.a)];
                ++stamp;
                for (int32_t v : X.vars) mark[(size_t)v] = stamp;
                unsigned *runs = which ? d.rb : d.ra;
                int nr = 0, dst = 0;
                for (int j = 0; j < d.rc;) {
                    if (mark[(size_t)C.layout[(size_t)j]] != stamp) {
                        ++j;
                        continue;
                    }
                    int s0 = j;
                    while (j < d.rc && mark[(size_t)C.layout[(size_t)j]] == stamp) ++j;
                    if (nr >= WMC_MAX_RUNS)
                        WMC_FAIL(WMC_ERR_UNSUPPORTED, "wmc_plan: node %d needs more than %d runs", id, WMC_MAX_RUNS);
                    runs[nr] = WMC_RUN(s0, j - s0, dst);
                    dst += j - s0;
                    ++nr;
                }
                if (which) d.nrb = nr; else d.nra = nr;
                if (dst + d.nk != (int32_t)X.layout.size())
                    WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: internal run mismatch at node %d", id);
            }
            work += (int64_t)align_up((uint64_t)1 << d.rc, WMC_WAVE);
            P.nodes.push_back(d);
        }
        L.work = work;
    }

    // ---- workspace layout
    uint64_t off = 0;
    P.off_acc = off;
    off += align_up(sizeof(wmc_acc), 256);
    P.off_w = off;
    off += align_up(sizeof(double) * 2 * (uint64_t)std::max(n, 1), 256);
    if (o.slice_group < 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: negative slice_group");
    P.group = (int32_t)std::min<int64_t>(std::max(o.slice_group, 1), (int64_t)1 << P.sliced.size());
    P.off_meta = off;
    P.meta_stride = (int64_t)(align_up(sizeof(wmc_meta) * (uint64_t)std::max<size_t>(NT, 1), 256) / sizeof(wmc_meta));
    off += (uint64_t)P.group * (uint64_t)P.meta_stride * sizeof(wmc_meta);
    P.off_leaf = off;
    off += align_up(sizeof(LeafDesc) * (uint64_t)std::max<size_t>(P.leaves.size(), 1), 256);
    P.off_node = off;
    off += align_up(sizeof(NodeDesc) * (uint64_t)std::max<size_t>(P.nodes.size(), 1), 256);
    P.off_gemm = off;
    off += align_up(sizeof(GemmDesc) * (uint64_t)std::max<size_t>(P.gemms.size(), 1), 256);
    // wave -> leaf and wave -> node tables, so the batched leaf and
    // small-node kernels find their item with one load instead of a
    // dependent binary search; only launches of several nodes need one
    std::vector<int32_t> tabs;
    if (P.leaves.size() > 1) {
        P.leaf_tab = 0;
        tabs.assign((size_t)(P.leaf_work / WMC_WAVE), 0);
        for (size_t q = 0; q < P.leaves.size(); ++q) {
            const int64_t b = P.leaves[q].work_begin / WMC_WAVE;
            const int64_t e = b + (int64_t)(((1ull << P.leaves[q].rank) + WMC_WAVE - 1) / WMC_WAVE);
            for (int64_t x = b; x < e; ++x) tabs[(size_t)x] = (int32_t)q;
        }
    }
    P.tab_off.assign(P.launches.size(), -1);
    for (size_t k = 1; k < P.launches.size(); ++k) {
        const Launch &Ln = P.launches[k];
        if (Ln.type == LAUNCH_GEMM || Ln.count < 2) continue;
        P.tab_off[k] = (int64_t)tabs.size();
        tabs.resize(tabs.size() + (size_t)(Ln.work / WMC_WAVE), 0);
        for (int32_t q = 0; q < Ln.count; ++q) {
            const NodeDesc &d = P.nodes[(size_t)(Ln.first + q)];
            const int64_t b = d.work_begin / WMC_WAVE;
            const int64_t e = b + (int64_t)(((1ull << d.rc) + WMC_WAVE - 1) / WMC_WAVE);
            for (int64_t x = b; x < e; ++x) tabs[(size_t)(P.tab_off[k] + x)] = q;
        }
    }
    P.off_tab = off;
    off += align_up(sizeof(int32_t) * (uint64_t)std::max<size_t>(tabs.size(), 1), 256);
    P.off_arena = off;
    P.desc_bytes = P.off_arena - P.off_leaf;
    P.desc_image.assign(P.desc_bytes, 0);
    if (!P.leaves.empty()) std::memcpy(P.desc_image.data(), P.leaves.data(), sizeof(LeafDesc) * P.leaves.size());
    if (!P.nodes.empty())
        std::memcpy(P.desc_image.data() + (P.off_node - P.off_leaf), P.nodes.data(), sizeof(NodeDesc) * P.nodes.size());
    if (!P.gemms.empty())
        std::memcpy(P.desc_image.data() + (P.off_gemm - P.off_leaf), P.gemms.data(), sizeof(GemmDesc) * P.gemms.size());
    if (!tabs.empty())
        std::memcpy(P.desc_image.data() + (P.off_tab - P.off_leaf), tabs.data(), sizeof(int32_t) * tabs.size());
    P.arena_stride = align_up(P.arena_bytes, 256);
    P.workspace_bytes = P.off_arena + (uint64_t)P.group * P.arena_stride;

    // ---- statistics
    wmc_plan_info &I = P.info;
    std::memset(&I, 0, sizeof I);
    I.n_vars = net.n_user;
    I.n_aux_vars = n - net.n_user;
    I.precision = P.precision;
    I.n_clauses = (int64_t)net.clauses.size();
    I.n_tensors = (int64_t)NT;
    I.n_nodes = (int64_t)P.nodes.size();
    I.max_rank = rankS;
    I.max_rank_unsliced = rank0;
    I.max_index_rank = idx_rank;
    I.n_sliced = (int32_t)P.sliced.size();
    I.n_slices = (int64_t)1 << P.sliced.size();
    for (size_t i = 0; i < P.sliced.size(); ++i) I.sliced_vars[i] = P.sliced[i];
    double fl = 0, by = 0, mx = 0;
    for (const NodeDesc &d : P.nodes) {
        double c = std::ldexp(1.0, d.rc);
        double a = std::ldexp(1.0, srank(T[(size_t)d.ta], sl));
        double b = std::ldexp(1.0, srank(T[(size_t)d.tb], sl));
        fl += 2.0 * c * std::ldexp(1.0, d.nk);
        double nb = (double)P.elem * (a + b + c);
        by += nb;
        mx = std::max(mx, nb);
        I.class_hist[d.cls]++;
    }
    I.flops_per_slice = fl;
    I.bytes_per_slice = by;
    I.max_node_bytes = mx;
    I.peak_live_bytes = peak_live(T, S, sl, P.elem, P.root, true);
    I.arena_bytes = P.arena_bytes;
    I.workspace_bytes = P.workspace_bytes;
    I.n_launches = (int64_t)P.launches.size() + 2;  // + begin and finish kernels
    I.slice_group = P.group;
    std::string why;
    if (!wmc_validate_launches(P, &why))
        WMC_FAIL(WMC_ERR_UNSUPPORTED, "wmc_plan: internal bounds check failed: %s", why.c_str());
    return WMC_OK;
}

// ---------------------------------------------------------------------------
// Executor tuning tables (one per precision), copied into every plan
// ---------------------------------------------------------------------------
// Built-in MI355X settings, measured on the sliced banded formula and the
// lattice: FP32 streaming launches run fastest with about one resident round
// of workgroups, FP64 ones with a few; K >= 16 FP64 nodes off the matrix
// cores split their summed index over groups of 4 lanes (with every K >= 16
// node on the register-tiled path: 7.04 -> 7.82 solves/s; groups of 8:
// 7.26), while FP32 (rows of 64 bytes) loses from the split.
static wmc_tuning default_tuning(int32_t precision) {
    wmc_tuning t;
    std::memset(&t, 0, sizeof t);
    t.stream2_grid_cap = precision == WMC_FP64 ? 4096 : 768;
    t.stream_mfma_grid_cap = 2048;
    t.stream_mfma_min_bits = 3;
    t.stream2_tile_bits = 2;
    t.stream2_min_thread_bits = 14;
    t.stream2_low_bits = 6;
    t.split_lanes = precision == WMC_FP64 ? 4 : 0;
    t.multi_min_rank = 12;
    t.gemm_tpw_max_nt = precision == WMC_FP64 ? 2 : 0;
    t.gemm_orient = 0;
    t.stream2_vec = precision == WMC_FP64 ? 1 : 0;  // FP64 pairs: 16-byte accesses; FP32 pairs measured slower
    return t;
}

static std::mutex g_tune_mu;
static wmc_tuning g_tune[2] = {default_tuning(WMC_FP64), default_tuning(WMC_FP32_SCALED)};

extern "C" wmc_status wmc_tuning_get(int32_t precision, wmc_tuning *out) {
    if (!out || (precision != WMC_FP64 && precision != WMC_FP32_SCALED))
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_tuning_get: bad precision or NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *out = g_tune[precision];
    return WMC_OK;
}

extern "C" wmc_status wmc_tuning_set(int32_t precision, const wmc_tuning *t) {
    if (precision != WMC_FP64 && precision != WMC_FP32_SCALED)
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_tuning_set: bad precision %d", precision);
    wmc_tuning v = t ? *t : default_tuning(precision);
    auto in = [](int32_t x, int32_t lo, int32_t hi) { return x >= lo && x <= hi; };
    if (!in(v.stream2_grid_cap, 8, 65536) || !in(v.stream_mfma_grid_cap, 8, 65536) ||
        !(v.stream_mfma_min_bits == 0 || in(v.stream_mfma_min_bits, 2, 8)) || !in(v.stream2_tile_bits, 0, 2) ||
        !in(v.stream2_min_thread_bits, 0, 30) || !in(v.stream2_low_bits, 0, 16) ||
        !(v.split_lanes == 0 || v.split_lanes == 4) || !in(v.multi_min_rank, 4, 30) ||
        !(v.gemm_tpw_max_nt == 0 || v.gemm_tpw_max_nt == 1 || v.gemm_tpw_max_nt == 2 || v.gemm_tpw_max_nt == 4) ||
        !in(v.gemm_orient, 0, 2) || !in(v.stream2_vec, 0, 1))
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_tuning_set: a field is outside its range");
    std::memset(v.reserved, 0, sizeof v.reserved);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[precision] = v;
    return WMC_OK;
}

extern "C" wmc_status wmc_plan(const wmc_network *net, const wmc_plan_options *opts, wmc_plan_t **out) {
    if (!out) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: out is NULL");
    *out = nullptr;
    if (!net || !opts) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: NULL argument");
    if (opts->precision != WMC_FP64 && opts->precision != WMC_FP32_SCALED)
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: unknown precision %d", opts->precision);
    if (opts->rank_cap < 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: negative rank_cap");
    try {
        wmc_plan_t *P = new wmc_plan_t();
        P->n = net->n;
        P->n_user = net->n_user;
        P->m = (int64_t)net->clauses.size();
        P->precision = opts->precision;
        P->elem = opts->precision == WMC_FP64 ? 8 : 4;
        P->w = net->w;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            P->tune = g_tune[opts->precision];
        }
        wmc_status st = WMC_OK;
        if (opts->kind == WMC_TREE_EXPLICIT) {
            if (net->n != net->n_user) {
                delete P;
                WMC_FAIL(WMC_ERR_UNSUPPORTED, "wmc_plan: a supplied tree cannot cover factored long clauses");
            }
            st = explicit_tree(*net, opts->parent, opts->n_tree_nodes, P->T, &P->root);
        } else if (opts->kind == WMC_TREE_ORDER || opts->kind == WMC_TREE_MINFILL || opts->kind == WMC_TREE_NETWORK) {
            std::vector<int32_t> order;
            if (opts->kind == WMC_TREE_NETWORK) {
                if (net->order.empty() && net->n > 0) {
                    delete P;
                    WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: the network carries no elimination order");
                }
                order = net->order;
            } else if (opts->kind == WMC_TREE_ORDER) {
                const int32_t nu = net->n_user;
                if (!opts->order || opts->order_len != nu) {
                    delete P;
                    WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: order must list all %d variables", nu);
                }
                std::vector<int32_t> pos((size_t)nu + 1, -1);
                for (int32_t i = 0; i < nu; ++i) {
                    int32_t v = opts->order[i];
                    if (v < 1 || v > nu || pos[(size_t)v] >= 0) {
                        delete P;
                        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: order is not a permutation (entry %d = %d)", i, v);
                    }
                    pos[(size_t)v] = i;
                }
                // an auxiliary variable of a factored clause is eliminated
                // right after the last of the caller's variables it depends on
                std::vector<std::vector<int32_t>> after((size_t)nu);
                for (size_t a = 0; a < net->aux_prefix.size(); ++a) {
                    int32_t last = 0;
                    for (int32_t v : net->aux_prefix[a]) last = std::max(last, pos[(size_t)v]);
                    after[(size_t)last].push_back(nu + 1 + (int32_t)a);
                }
                for (int32_t i = 0; i < nu; ++i) {
                    order.push_back(opts->order[i]);
                    for (int32_t a : after[(size_t)i]) order.push_back(a);
                }
            } else {
                order = minfill_order(*net, opts->seed);
            }
            P->root = bucket_tree(*net, order, opts->block, P->T);
            if (P->root == -2) st = WMC_ERR_INVALID_ARGUMENT;
        } else {
            delete P;
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan: unknown tree kind %d", opts->kind);
        }
        if (st == WMC_OK) st = finalize_plan(*net, *opts, *P);
        if (st != WMC_OK) {
            delete P;
            return st;
        }
        *out = P;
    } catch (std::bad_alloc &) {
        WMC_FAIL(WMC_ERR_OUT_OF_MEMORY, "wmc_plan: host allocation failed");
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_plan_stats(const wmc_plan_t *plan, wmc_plan_info *out) {
    if (!plan || !out) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_stats: NULL argument");
    *out = plan->info;
    return WMC_OK;
}

extern "C" void wmc_plan_destroy(wmc_plan_t *plan) { delete plan; }

extern "C" wmc_status wmc_plan_tensor(const wmc_plan_t *plan, int64_t t, int32_t *kind, int32_t *src,
                                      int32_t *rank, int32_t *vars) {
    if (!plan) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_tensor: plan is NULL");
    if (t < 0 || t >= (int64_t)plan->T.size())
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_tensor: tensor %lld out of range", (long long)t);
    const TNode &X = plan->T[(size_t)t];
    if (kind) *kind = X.kind;
    if (src) *src = X.src;
    if (rank) *rank = (int32_t)X.layout.size();
    if (vars)
        for (size_t q = 0; q < X.layout.size(); ++q) vars[q] = X.layout[q];
    return WMC_OK;
}

extern "C" wmc_status wmc_plan_node(const wmc_plan_t *plan, int64_t i, int64_t *a, int64_t *b, int64_t *c,
                                    int32_t *node_class) {
    if (!plan) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_node: plan is NULL");
    if (i < 0 || i >= (int64_t)plan->nodes.size())
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_node: node %lld out of range", (long long)i);
    const NodeDesc &d = plan->nodes[(size_t)i];
    if (a) *a = d.ta;
    if (b) *b = d.tb;
    if (c) *c = d.tc;
    if (node_class) *node_class = d.cls;
    return WMC_OK;
}

// Raw descriptor image, for tools and tests that replay the launch list:
// [LeafDesc x n_leaves][NodeDesc x n_nodes][Launch x n_launches][GemmDesc x n_gemms].
// info[] = {n_leaves, n_nodes, n_launches, arena_elems, root, root_off,
//           n_tensors, elem_bytes, sizeof LeafDesc, sizeof NodeDesc, sizeof Launch,
//           n_gemms, sizeof GemmDesc}.
extern "C" wmc_status wmc_plan_image(const wmc_plan_t *plan, void *dst, uint64_t dst_bytes, uint64_t *needed,
                                     int64_t *info) {
    if (!plan) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_image: plan is NULL");
    const wmc_plan_t &P = *plan;
    uint64_t need = sizeof(LeafDesc) * P.leaves.size() + sizeof(NodeDesc) * P.nodes.size() +
                    sizeof(Launch) * P.launches.size() + sizeof(GemmDesc) * P.gemms.size();
    if (needed) *needed = need;
    if (info) {
        info[0] = (int64_t)P.leaves.size();
        info[1] = (int64_t)P.nodes.size();
        info[2] = (int64_t)P.launches.size();
        info[3] = (int64_t)(P.arena_bytes / (uint64_t)P.elem);
        info[4] = P.root;
        info[5] = P.root >= 0 ? P.T[(size_t)P.root].off : -1;
        info[6] = (int64_t)P.T.size();
        info[7] = P.elem;
        info[8] = (int64_t)sizeof(LeafDesc);
        info[9] = (int64_t)sizeof(NodeDesc);
        info[10] = (int64_t)sizeof(Launch);
        info[11] = (int64_t)P.gemms.size();
        info[12] = (int64_t)sizeof(GemmDesc);
    }
    if (!dst) return WMC_OK;
    if (dst_bytes < need) WMC_FAIL(WMC_ERR_OUT_OF_MEMORY, "wmc_plan_image: buffer too small");
    char *p = (char *)dst;
    if (!P.leaves.empty()) std::memcpy(p, P.leaves.data(), sizeof(LeafDesc) * P.leaves.size());
    p += sizeof(LeafDesc) * P.leaves.size();
    if (!P.nodes.empty()) std::memcpy(p, P.nodes.data(), sizeof(NodeDesc) * P.nodes.size());
    p += sizeof(NodeDesc) * P.nodes.size();
    if (!P.launches.empty()) std::memcpy(p, P.launches.data(), sizeof(Launch) * P.launches.size());
    p += sizeof(Launch) * P.launches.size();
    if (!P.gemms.empty()) std::memcpy(p, P.gemms.data(), sizeof(GemmDesc) * P.gemms.size());
    return WMC_OK;
}

// Per-launch algorithmic traffic of one slice, in the order wmc_contract
// issues the kernels: [begin, leaf fill, node launches..., finish].
extern "C" wmc_status wmc_plan_launches(const wmc_plan_t *plan, double *bytes, double *flops, int32_t *cls,
                                        int64_t cap, int64_t *n_out) {
    if (!plan) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_plan_launches: plan is NULL");
    const wmc_plan_t &P = *plan;
    const int64_t n = (int64_t)P.launches.size() + 2;
    if (n_out) *n_out = n;
    if (!bytes && !flops && !cls) return WMC_OK;
    if (cap < n) WMC_FAIL(WMC_ERR_OUT_OF_MEMORY, "wmc_plan_launches: need %lld slots", (long long)n);
    std::vector<double> B((size_t)n, 0.0), F((size_t)n, 0.0);
    std::vector<int32_t> C((size_t)n, -1);
    B[0] = (double)(sizeof(wmc_meta) * P.T.size());
    for (const LeafDesc &d : P.leaves) B[1] += (double)P.elem * std::ldexp(1.0, d.rank);
    for (size_t k = 1; k < P.launches.size(); ++k) {
        const Launch &L = P.launches[k];
        for (int32_t q = 0; q < L.count; ++q) {
            const NodeDesc &d = P.nodes[(size_t)(L.first + q)];
            double a = std::ldexp(1.0, (int)P.T[(size_t)d.ta].layout.size());
            double b = std::ldexp(1.0, (int)P.T[(size_t)d.tb].layout.size());
            double c = std::ldexp(1.0, d.rc);
            B[k + 1] += (double)P.elem * (a + b + c);
            F[k + 1] += 2.0 * c * std::ldexp(1.0, d.nk);
            C[k + 1] = d.cls;
        }
    }
    B[(size_t)n - 1] = (double)(P.elem + sizeof(wmc_acc));
    for (int64_t k = 0; k < n; ++k) {
        if (bytes) bytes[k] = B[(size_t)k];
        if (flops) flops[k] = F[(size_t)k];
        if (cls) cls[k] = C[(size_t)k];
    }
    return WMC_OK;
}

// ---------------------------------------------------------------------------
// Elimination order from a tree decomposition of the primal graph (the
// decompositions of Section 2; the variable-elimination use of them that
// Section 3 contrasts with FactorTree).  Rooted at root_bag, every variable
// is eliminated at its top bag (the bag of least depth holding it), bags
// taken children first.  When x is eliminated, every variable that shares
// an original or fill edge with x and is still open lies in x's top bag:
// such a variable shares a bag with x, and its bags form a connected
// subtree that is not entirely below the top bag (else it would be gone
// already), so the subtree passes through the top bag.  The bucket of x
// therefore spans at most the top bag's size.
// A tree decomposition read from PACE ".td" text, rooted and checked: a
// tree over its bags, and every vertex's bags connected.
struct ParsedTD {
    long long nb = 0;
    std::vector<std::vector<int32_t>> bags;          // sorted vertex ids, 1-based
    std::vector<std::pair<long long, long long>> edges;
    std::vector<int64_t> bfs, par, depth;            // from the root: parents before children
    std::vector<int64_t> top;                        // per vertex: its bag of least depth, -1 if none
    std::vector<std::vector<int64_t>> bags_of;       // per vertex: its bags, in bfs order
    int32_t width = 0;
};

static wmc_status parse_td(const char *who, const char *td, long long nvert, int64_t root_bag, ParsedTD &T) {
    long long nb = -1, nv = -1;
    std::vector<std::vector<int32_t>> &bags = T.bags;
    std::vector<std::pair<long long, long long>> &edges = T.edges;
    const char *p = td;
    long long line = 0;
    while (*p) {
        const char *e = p;
        while (*e && *e != '\n') ++e;
        std::string s(p, (size_t)(e - p));
        p = *e ? e + 1 : e;
        ++line;
        size_t i = s.find_first_not_of(" \t\r");
        if (i == std::string::npos || s[i] == 'c') continue;
        if (s[i] == 's') {
            long long w = 0;
            if (nb >= 0 || std::sscanf(s.c_str() + i, "s td %lld %lld %lld", &nb, &w, &nv) != 3 || nb < 0 || nv < 0)
                WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: bad solution line %lld", who, line);
            if (nv != nvert)
                WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: %lld vertices, the graph has %lld", who, nv, nvert);
            // a tree of nb bags needs nb - 1 edge lines: more bags than
            // characters cannot be a well-formed file (and would only
            // allocate)
            if (nb > (long long)std::strlen(td))
                WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: %lld bags in a text of %zu bytes", who, nb, std::strlen(td));
            bags.assign((size_t)nb, {});
            continue;
        }
        if (nb < 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: line %lld before the 's td' line", who, line);
        const char *q = s.c_str() + i;
        char *end = nullptr;
        if (s[i] == 'b') {
            ++q;
            const long long id = std::strtoll(q, &end, 10);
            if (end == q || id < 1 || id > nb) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: bad bag id on line %lld", who, line);
            std::vector<int32_t> &B = bags[(size_t)(id - 1)];
            for (q = end;;) {
                const long long v = std::strtoll(q, &end, 10);
                if (end == q) break;
                if (v < 1 || v > nvert)
                    WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: vertex %lld out of range on line %lld", who, v, line);
                B.push_back((int32_t)v);
                q = end;
            }
            std::sort(B.begin(), B.end());
            B.erase(std::unique(B.begin(), B.end()), B.end());
        } else {
            const long long a = std::strtoll(q, &end, 10);
            const char *q2 = end;
            const long long b = std::strtoll(q2, &end, 10);
            if (end == q2 || a < 1 || a > nb || b < 1 || b > nb || a == b)
                WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: bad edge on line %lld", who, line);
            edges.push_back({a - 1, b - 1});
        }
    }
    if (nb < 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: no 's td' line", who);
    if (nb == 0 && nvert > 0) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: no bags", who);
    if ((long long)edges.size() != (nb > 0 ? nb - 1 : 0))
        WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: %zu edges for %lld bags (not a tree)", who, edges.size(), nb);
    T.nb = nb;
    // breadth-first order from the root: parents before children
    std::vector<std::vector<int64_t>> adj((size_t)nb);
    for (auto &e : edges) {
        adj[(size_t)e.first].push_back(e.second);
        adj[(size_t)e.second].push_back(e.first);
    }
    const int64_t root = root_bag > 0 ? root_bag - 1 : 0;
    if (nb > 0 && (root < 0 || root >= nb)) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: bad root bag", who);
    T.par.assign((size_t)nb, -2);
    T.depth.assign((size_t)nb, 0);
    if (nb > 0) {
        T.bfs.push_back(root);
        T.par[(size_t)root] = -1;
    }
    for (size_t h = 0; h < T.bfs.size(); ++h)
        for (int64_t c : adj[(size_t)T.bfs[h]])
            if (T.par[(size_t)c] == -2) {
                T.par[(size_t)c] = T.bfs[h];
                T.depth[(size_t)c] = T.depth[(size_t)T.bfs[h]] + 1;
                T.bfs.push_back(c);
            }
    if ((long long)T.bfs.size() != nb) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: bags not connected", who);
    // each vertex's bags must form a subtree (bags holding it minus tree
    // edges joining two of them = 1)
    T.top.assign((size_t)nvert + 1, -1);
    T.bags_of.assign((size_t)nvert + 1, {});
    std::vector<int64_t> nedges((size_t)nvert + 1, 0);
    for (int64_t b : T.bfs) {
        T.width = std::max(T.width, (int32_t)bags[(size_t)b].size() - 1);
        for (int32_t v : bags[(size_t)b]) {
            if (T.top[(size_t)v] < 0) T.top[(size_t)v] = b;
            T.bags_of[(size_t)v].push_back(b);
        }
    }
    for (auto &e : edges) {
        const std::vector<int32_t> &A = bags[(size_t)e.first], &B = bags[(size_t)e.second];
        std::vector<int32_t> both;
        std::set_intersection(A.begin(), A.end(), B.begin(), B.end(), std::back_inserter(both));
        for (int32_t v : both) ++nedges[(size_t)v];
    }
    for (long long v = 1; v <= nvert; ++v)
        if (!T.bags_of[(size_t)v].empty() && nedges[(size_t)v] != (int64_t)T.bags_of[(size_t)v].size() - 1)
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: bags of vertex %lld are not connected", who, v);
    return WMC_OK;
}

// FactorTree (Theorem 3; the FactorTree paragraph of Section 3.3): the
// network is factored along a tree decomposition of the formula's incidence
// graph (variables 1..n_vars, clause c as vertex n_vars + 1 + c), and the
// elimination order follows the decomposition.
//
// A clause C is an OR, which is tree-factorable (Def. 4).  Each literal of C
// is assigned to the bag nearest the root that holds both its variable and C
// (the edge of the incidence graph lies in some bag, and the bags of each
// vertex are connected).  Let T'_C be the smallest subtree spanning the
// assigned bags, L its top.  At every bag b of T'_C below L an auxiliary
// variable a_b = OR(literals assigned to b, a_c of b's children in T'_C) is
// introduced (clauses a_b -> OR(inputs) and input -> a_b); at L the clause
// OR(inputs) remains.  Every assignment of the formula's variables extends
// to exactly one assignment of the a_b, which weigh (1, 1), so W is
// unchanged (the network of Theorem 2 is a partial contraction of the
// factored one).  Gates wider than two inputs are chained through local
// auxiliary variables, so every factor has at most three variables.
//
// Elimination order, bags children first: at bag b the carries a_c of its
// children, then b's local chain variables, then the formula's variables
// whose bag of least depth is b.  When a bag's turn comes, every open
// variable is a variable of the bag or the carry of a clause in it, so
// intermediates stay near the width of the decomposition.
extern "C" wmc_status wmc_build_network_td(int32_t n_vars, int64_t n_clauses, const int64_t *clause_ptr,
                                           const int32_t *lits, const double *weights, const char *td,
                                           int64_t root_bag, wmc_network **out, int32_t *width) {
    const char *who = "wmc_build_network_td";
    if (!out || !td) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: NULL argument", who);
    *out = nullptr;
    {
        const wmc_status st = check_formula(who, n_vars, n_clauses, clause_ptr, lits, weights);
        if (st != WMC_OK) return st;
    }
    if ((long long)n_vars + n_clauses > (long long)INT32_MAX / 4)
        WMC_FAIL(WMC_ERR_UNSUPPORTED, "%s: incidence graph too large", who);
    ParsedTD T;
    {
        const wmc_status st = parse_td(who, td, (long long)n_vars + n_clauses, root_bag, T);
        if (st != WMC_OK) return st;
    }
    try {
        std::vector<std::vector<int32_t>> cls, aux_prefix;
        std::vector<int64_t> aux_node;     // bag at which each auxiliary variable is eliminated
        std::vector<uint8_t> aux_carry;    // a child's carry (eliminated before the bag's local chain)
        auto new_aux = [&](std::vector<int32_t> prefix, int64_t node, bool carry) {
            std::sort(prefix.begin(), prefix.end());
            prefix.erase(std::unique(prefix.begin(), prefix.end()), prefix.end());
            aux_prefix.push_back(std::move(prefix));
            aux_node.push_back(node);
            aux_carry.push_back(carry ? 1 : 0);
            return n_vars + (int32_t)aux_prefix.size();
        };
        // inputs of a gate or of the final clause: literal and the caller
        // variables it depends on
        struct In {
            int32_t lit;
            std::vector<int32_t> pre;
        };
        // out = 0: the clause OR(in); out = a: a <-> OR(in).  Inputs beyond
        // two are folded pairwise into local variables at `node` first.
        auto emit = [&](std::vector<In> in, int32_t out_lit, int64_t node) {
            const size_t keep = out_lit ? 2 : 3;
            while (in.size() > keep) {
                std::vector<int32_t> pre = in[0].pre;
                pre.insert(pre.end(), in[1].pre.begin(), in[1].pre.end());
                const int32_t t = new_aux(pre, node, false);
                cls.push_back({-t, in[0].lit, in[1].lit});
                cls.push_back({t, -in[0].lit});
                cls.push_back({t, -in[1].lit});
                In folded{t, aux_prefix.back()};
                in.erase(in.begin(), in.begin() + 2);
                in.insert(in.begin(), std::move(folded));
            }
            std::vector<int32_t> big;
            if (out_lit) big.push_back(-out_lit);
            for (const In &x : in) big.push_back(x.lit);
            cls.push_back(big);
            if (out_lit)
                for (const In &x : in) cls.push_back({out_lit, -x.lit});
        };
        std::vector<int8_t> sign((size_t)n_vars + 1, 0);
        std::vector<int64_t> cnt((size_t)T.nb, 0);
        std::vector<std::vector<In>> inputs((size_t)T.nb);
        for (int64_t c = 0; c < n_clauses; ++c) {
            std::vector<int32_t> lv;
            bool taut = false;
            for (int64_t j = clause_ptr[c]; j < clause_ptr[c + 1]; ++j) {
                const int32_t l = lits[j], v = l > 0 ? l : -l;
                const int8_t bit = l > 0 ? 1 : 2;
                if (!(sign[v] & bit)) {
                    if (sign[v]) taut = true;
                    else lv.push_back(l);
                    sign[v] |= bit;
                }
            }
            for (int32_t l : lv) sign[(size_t)(l > 0 ? l : -l)] = 0;
            if (taut) continue;  // an all-ones tensor: dropping it leaves W unchanged
            if (lv.empty()) {
                cls.push_back({});  // the empty clause: W = 0
                continue;
            }
            const int32_t cv = n_vars + 1 + (int32_t)c;
            if (T.bags_of[(size_t)cv].empty()) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: clause %lld in no bag", who, (long long)c);
            const int64_t topc = T.top[(size_t)cv];
            std::vector<int64_t> S;
            for (int32_t l : lv) {
                const int32_t x = l > 0 ? l : -l;
                int64_t at = -1;
                for (int64_t b : T.bags_of[(size_t)x])  // in bfs order: least depth first
                    if (std::binary_search(T.bags[(size_t)b].begin(), T.bags[(size_t)b].end(), cv)) {
                        at = b;
                        break;
                    }
                if (at < 0)
                    WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: no bag holds variable %d with clause %lld", who, (int)x,
                             (long long)c);
                if (inputs[(size_t)at].empty()) S.push_back(at);
                inputs[(size_t)at].push_back(In{l, {x}});
            }
            if (S.size() == 1 && lv.size() <= WMC_FACTOR_ABOVE) {
                cls.push_back(lv);  // the clause lies in one bag: kept whole
                inputs[(size_t)S[0]].clear();
                continue;
            }
            // smallest subtree spanning S: paths up to the clause's top bag,
            // cut at the deepest bag every path passes (their meeting point)
            std::vector<int64_t> touched;
            for (int64_t b0 : S)
                for (int64_t b = b0;; b = T.par[(size_t)b]) {
                    if (cnt[(size_t)b]++ == 0) touched.push_back(b);
                    if (b == topc || T.par[(size_t)b] < 0) break;
                }
            int64_t lca = -1;
            for (int64_t b : touched)
                if (cnt[(size_t)b] == (int64_t)S.size() && (lca < 0 || T.depth[(size_t)b] > T.depth[(size_t)lca])) lca = b;
            std::vector<int64_t> sub;
            for (int64_t b : touched)
                if (T.depth[(size_t)b] >= T.depth[(size_t)lca]) sub.push_back(b);
            std::sort(sub.begin(), sub.end(),
                      [&](int64_t a, int64_t b) { return T.depth[(size_t)a] > T.depth[(size_t)b]; });
            for (int64_t b : sub) {
                if (b == lca) {
                    emit(std::move(inputs[(size_t)b]), 0, b);
                } else {
                    std::vector<int32_t> pre;
                    for (const In &x : inputs[(size_t)b]) pre.insert(pre.end(), x.pre.begin(), x.pre.end());
                    const int64_t up = T.par[(size_t)b];
                    const int32_t a = new_aux(pre, up, true);
                    emit(std::move(inputs[(size_t)b]), a, b);
                    inputs[(size_t)up].push_back(In{a, aux_prefix.back()});
                }
                inputs[(size_t)b].clear();
            }
            for (int64_t b : touched) cnt[(size_t)b] = 0;
        }
        const int32_t n_aux = (int32_t)aux_prefix.size();
        if ((int64_t)n_vars + n_aux > (int64_t)INT32_MAX / 2)
            WMC_FAIL(WMC_ERR_UNSUPPORTED, "%s: too many variables after factoring", who);
        wmc_network *net = make_network(n_vars, weights, cls, aux_prefix);
        // elimination order: variables in no bag first, then bags children
        // first (carries into the bag, its local chain, its own variables)
        std::vector<std::vector<int32_t>> carry_at((size_t)T.nb), local_at((size_t)T.nb);
        for (int32_t i = 0; i < n_aux; ++i)
            (aux_carry[(size_t)i] ? carry_at : local_at)[(size_t)aux_node[(size_t)i]].push_back(n_vars + 1 + i);
        for (int32_t v = 1; v <= n_vars; ++v)
            if (T.top[(size_t)v] < 0) net->order.push_back(v);
        for (size_t h = T.bfs.size(); h-- > 0;) {
            const int64_t b = T.bfs[h];
            for (int32_t a : carry_at[(size_t)b]) net->order.push_back(a);
            for (int32_t a : local_at[(size_t)b]) net->order.push_back(a);
            for (int32_t v : T.bags[(size_t)b])
                if (v <= n_vars && T.top[(size_t)v] == b) net->order.push_back(v);
        }
        if ((int32_t)net->order.size() != net->n) {
            delete net;
            WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "%s: internal order of %zu variables, network has %d", who,
                     net->order.size(), (int)net->n);
        }
        if (width) *width = T.width;
        *out = net;
    } catch (std::bad_alloc &) {
        WMC_FAIL(WMC_ERR_OUT_OF_MEMORY, "%s: host allocation failed", who);
    }
    return WMC_OK;
}

extern "C" wmc_status wmc_order_from_td(const wmc_network *net, const char *td, int64_t root_bag,
                                        int32_t *order, int32_t *width) {
    if (!net || !td || !order) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_order_from_td: NULL argument");
    const int32_t n = net->n_user;
    ParsedTD T;
    {
        const wmc_status st = parse_td("wmc_order_from_td", td, n, root_bag, T);
        if (st != WMC_OK) return st;
    }
    const std::vector<std::vector<int32_t>> &bags = T.bags;
    const std::vector<int64_t> &bfs = T.bfs, &top = T.top;
    const std::vector<std::vector<int64_t>> &bags_of = T.bags_of;
    // every clause (its caller variables) inside one bag
    for (size_t c = 0; c < net->clauses.size(); ++c) {
        std::vector<int32_t> vs;
        for (int32_t v : net->clauses[c].vars)
            if (v <= n) vs.push_back(v);
        if (vs.empty()) continue;
        int32_t lead = vs[0];
        for (int32_t v : vs)
            if (bags_of[(size_t)v].size() < bags_of[(size_t)lead].size()) lead = v;
        bool ok = false;
        for (int64_t b : bags_of[(size_t)lead]) {
            const std::vector<int32_t> &B = bags[(size_t)b];
            ok = std::includes(B.begin(), B.end(), vs.begin(), vs.end());
            if (ok) break;
        }
        if (!ok) WMC_FAIL(WMC_ERR_INVALID_ARGUMENT, "wmc_order_from_td: no bag holds the variables of clause %zu", c);
    }
    // variables in no bag (in no clause) first, then bags children first
    size_t k = 0;
    for (int32_t v = 1; v <= n; ++v)
        if (top[(size_t)v] < 0) order[k++] = v;
    for (size_t h = bfs.size(); h-- > 0;) {
        const int64_t b = bfs[h];
        for (int32_t v : bags[(size_t)b])
            if (top[(size_t)v] == b) order[k++] = v;
    }
    if (width) *width = T.width;
    return WMC_OK;
}
