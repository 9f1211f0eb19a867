/*
 * wmc.h - C ABI of the MI355X tensor-network weighted model counter.
 *
 * The library computes the literal-weighted model count of a CNF formula
 * (Definition 1 of Dudek & Vardi, "Parallel Weighted Model Counting with
 * Tensor Networks"):
 *
 *     W(phi) = sum over tau in {0,1}^X of phi(tau) * prod_x W(x, tau(x))
 *
 * by the paper's three stages (Algorithm 1): the formula is reduced to a
 * tensor network (Theorem 2: one clause tensor B_C per clause, one
 * COPY/weight tensor A_x per variable, over binary indices), a contraction
 * tree is planned (Definition of a contraction tree; index slicing under a
 * memory bound, Algorithm 3), and the network is contracted pairwise along
 * the tree on the GPU (Algorithm 2), summing the slices (the slicing
 * theorem).
 *
 * Conventions
 *  - Every call returns wmc_status; nothing throws across the ABI.  On a
 *    non-OK status wmc_last_error() returns a thread-local message.
 *  - Inputs are copied at call time; the caller keeps ownership of every
 *    pointer it passes.  Handles are owned by the caller and released with
 *    the matching *_destroy (NULL is accepted and ignored).
 *  - Networks and plans are immutable after creation and may be shared
 *    between threads.  wmc_contract is reentrant given distinct workspaces.
 *  - Device memory belongs to the caller: wmc_contract runs entirely inside
 *    a caller-supplied device workspace of wmc_plan_info.workspace_bytes.
 *  - Streams are hipStream_t passed as void* (NULL = the default stream).
 *  - Variables are numbered 1..n_vars; literals are DIMACS signed integers.
 */
#ifndef WMC_H
#define WMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WMC_OK = 0,
    WMC_ERR_INVALID_ARGUMENT = 1, /* bad literal, NaN/Inf weight, malformed order/tree, NULL */
    WMC_ERR_OUT_OF_MEMORY = 2,    /* host allocation failed, or workspace too small */
    WMC_ERR_CAP_UNREACHABLE = 3,  /* slicing cannot meet the memory / rank cap */
    WMC_ERR_DEVICE = 4,           /* a HIP call failed; message in wmc_last_error() */
    WMC_ERR_BUSY = 5,             /* server queue full */
    WMC_ERR_UNSUPPORTED = 6,      /* rank too large, supplied tree over factored clauses,
                                     more than 16 sliced variables in a served plan */
    WMC_ERR_CANCELLED = 7         /* serving: the request was cancelled or passed its deadline */
} wmc_status;

typedef enum { WMC_FP64 = 0, WMC_FP32_SCALED = 1 } wmc_precision;

typedef enum {
    WMC_TREE_MINFILL = 0,  /* seeded min-fill elimination order -> bucket tree */
    WMC_TREE_ORDER = 1,    /* caller-supplied elimination order -> bucket tree */
    WMC_TREE_EXPLICIT = 2, /* caller-supplied contraction tree (parent array) */
    WMC_TREE_NETWORK = 3   /* the elimination order a network built by wmc_build_network_td
                              carries (FactorTree) -> bucket tree */
} wmc_tree_kind;

#define WMC_MAX_CLAUSE 24   /* distinct variables of a clause tensor */
#define WMC_FACTOR_ABOVE 8  /* longer clauses are factored into chains of 3-literal clauses */
#define WMC_MAX_RANK 34     /* largest storage rank of any intermediate */
#define WMC_MAX_SLICED 40   /* largest number of sliced variables */

/* A result: W = mantissa * 2^exp2 with |mantissa| in [0.5, 1), or exactly 0.
 * value = ldexp(mantissa, exp2) (may under- or overflow to 0 / inf);
 * log2_abs = log2|W| (-inf for 0). */
typedef struct {
    double mantissa;
    int64_t exp2;
    double value;
    double log2_abs;
} wmc_value;

typedef struct wmc_network wmc_network;
typedef struct wmc_plan_t wmc_plan_t;

/* ------------------------------------------------------------------ */
/* Reduction stage (Theorem 2)                                          */
/* ------------------------------------------------------------------ */

/* Build the tensor network of Theorem 2 from a CNF and literal weights.
 *   clause_ptr: n_clauses+1 offsets into lits (CSR), host memory
 *   lits:       DIMACS literals in 1..n_vars or -n_vars..-1, host memory
 *   weights:    2*n_vars doubles {W(x,0), W(x,1)} for x = 1..n_vars (finite)
 * Repeated literals collapse; a clause holding x and not-x is always true;
 * an empty clause makes W = 0; a variable in no clause contributes
 * W(x,0)+W(x,1).  A clause with more than WMC_FACTOR_ABOVE distinct
 * variables is factored into a chain of clauses of at most 3 literals over
 * k-2 auxiliary variables of weight (1, 1) that record the OR of a prefix of
 * the clause (exact: W is unchanged); the caller still passes 2*n_vars
 * weights everywhere, and auxiliary variables never appear in its orders.
 * The COPY tensors A_x are kept symbolically (degree, W(x,0), W(x,1)) and
 * never materialised. */
wmc_status wmc_build_network(int32_t n_vars, int64_t n_clauses, const int64_t *clause_ptr,
                             const int32_t *lits, const double *weights, wmc_network **out);

/* FactorTree (Theorem 3; the FactorTree paragraph of Section 3.3): the
 * network of Theorem 2 factored along a tree decomposition of the formula's
 * INCIDENCE graph, with the elimination order that follows the
 * decomposition (plan it with kind = WMC_TREE_NETWORK).
 *   td:       NUL-terminated PACE ".td" text, host memory: "s td <bags>
 *             <max bag size> <vertices>", "b <id> <v...>" lines and tree
 *             edges "<id> <id>"; 'c' lines are comments.  Vertices are
 *             1..n_vars for the variables and n_vars+1..n_vars+n_clauses for
 *             the clauses, in input order (vertices = n_vars + n_clauses).
 *   root_bag: bag to root the decomposition at (1-based; 0 = bag 1).
 *   width:    out (may be NULL): max |bag| - 1.
 * Every clause, an OR, is factored along the smallest subtree of bags that
 * covers its incidences: each bag below the subtree's top gets an auxiliary
 * variable (weight (1, 1)) holding the OR of the clause's literals in its
 * part of the subtree, and the top keeps the clause over its inputs (gates
 * of more than two inputs are chained, so no factor has more than three
 * variables).  W is unchanged.  Tautologies are dropped (all-ones tensors);
 * an empty clause gives W = 0.  Other arguments and the weights convention
 * as wmc_build_network (callers pass 2*n_vars weights everywhere).
 * WMC_ERR_INVALID_ARGUMENT for malformed text, a vertex count other than
 * n_vars + n_clauses, bags that are not a tree, a vertex whose bags are not
 * connected, or an incidence (variable, clause) that no bag covers. */
wmc_status wmc_build_network_td(int32_t n_vars, int64_t n_clauses, const int64_t *clause_ptr,
                                const int32_t *lits, const double *weights, const char *td, int64_t root_bag,
                                wmc_network **out, int32_t *width);

/* Size of the Theorem-2 network: n_tensors = n_vars + n_clauses tensors
 * (auxiliary variables and chain clauses of factored long clauses included),
 * n_indices = number of (variable, clause) incidences (distinct per clause). */
wmc_status wmc_network_info(const wmc_network *net, int64_t *n_tensors, int64_t *n_indices);

void wmc_network_destroy(wmc_network *net);

/* ------------------------------------------------------------------ */
/* Planning stage: contraction tree + index slicing (Algorithm 3)       */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t kind;            /* wmc_tree_kind */
    int32_t precision;       /* wmc_precision */
    uint64_t seed;           /* WMC_TREE_MINFILL tie-break seed */
    const int32_t *order;    /* WMC_TREE_ORDER: permutation of 1..n_vars (host) */
    int32_t order_len;
    int32_t block;           /* variables eliminated together per bucket step (>=1; 0 = 1) */
    const int64_t *parent;   /* WMC_TREE_EXPLICIT: parent of each tree vertex, -1 at the root.
                                Vertices 0..n-1 are A_x (x = i+1), n..n+m-1 are B_C (clause
                                i-n), n+m..2(n+m)-2 are internal; every internal vertex has
                                exactly two children. */
    int64_t n_tree_nodes;    /* = 2(n+m)-1 */
    uint64_t mem_cap_bytes;  /* Algorithm 3 bound m on MemCost, the bytes of the tensor arena
                                one slice occupies as placed (every tensor 256-byte aligned);
                                0 = none.  Met exactly: wmc_plan_info.arena_bytes <= m, or
                                WMC_ERR_CAP_UNREACHABLE. */
    int32_t rank_cap;        /* bound on the largest storage rank; 0 = none */
    int32_t slice_objective; /* wmc_slice_objective: how ChooseSliceIndex picks the next variable */
    int32_t slice_group;     /* slices run side by side in every launch (the slices of Algorithm 3
                                are independent): each has its own arena and meta table, so the
                                workspace holds this many arenas; 0 or 1 = one slice at a time;
                                capped at the slice count.  Results do not depend on it. */
    int32_t reserved[5];
} wmc_plan_options;

/* Choice of the next sliced variable (Algorithm 3's ChooseSliceIndex, over
 * the variables of the tensors within one of the largest rank):
 *  WMC_SLICE_BY_MEMORY: least MemCost after slicing it, ties by flops (the
 *    paper's greedy memory criterion);
 *  WMC_SLICE_BY_FLOPS: among the variables that bring the plan closer to the
 *    caps, least total flops over all slices (the alternative heuristics the
 *    slicing section leaves open); afterwards sliced variables the caps no
 *    longer need are dropped, last added first. */
typedef enum { WMC_SLICE_BY_MEMORY = 0, WMC_SLICE_BY_FLOPS = 1 } wmc_slice_objective;

/* Node classes of the histogram in wmc_plan_info. */
enum { WMC_CLASS_SMALL = 0, WMC_CLASS_STREAM = 1, WMC_CLASS_GEMM = 2, WMC_N_CLASSES = 4 };

typedef struct {
    int32_t n_vars;
    int32_t precision;
    int64_t n_clauses;
    int64_t n_tensors;          /* leaves + internal nodes of the tree */
    int64_t n_nodes;            /* internal nodes = pairwise contractions */
    int32_t max_rank;           /* largest storage rank (distinct variables) per slice */
    int32_t max_rank_unsliced;  /* the same before slicing */
    int32_t max_index_rank;     /* largest rank counting Theorem-2 indices (unsliced) */
    int32_t n_sliced;           /* |I| */
    int64_t n_slices;           /* 2^|I| */
    int32_t sliced_vars[WMC_MAX_SLICED];
    double flops_per_slice;     /* sum over nodes of 2*b*m*n*k */
    double bytes_per_slice;     /* sum over nodes of elem_size*(|A|+|B|+|C|) */
    double peak_live_bytes;     /* peak of live tensor bytes (256-byte aligned) over the executed
                                   schedule: a lower bound on arena_bytes */
    uint64_t arena_bytes;       /* static arena after placement (MemCost, what mem_cap bounds) */
    uint64_t workspace_bytes;   /* device workspace wmc_contract needs */
    int64_t class_hist[WMC_N_CLASSES];
    int64_t n_launches;         /* kernel launches per slice */
    double max_node_bytes;      /* largest single-node traffic */
    int32_t n_aux_vars;         /* auxiliary variables of factored long clauses */
    int32_t slice_group;        /* slices per launch (workspace holds this many arenas) */
} wmc_plan_info;

wmc_status wmc_plan(const wmc_network *net, const wmc_plan_options *opts, wmc_plan_t **out);

/* Elimination order from a tree decomposition of the formula's primal graph
 * (tree decompositions and their width as defined in Section 2; used the way
 * variable elimination uses them, which Section 3 sets beside FactorTree).
 *   td:       NUL-terminated text in the PACE ".td" format, host memory:
 *             "s td <bags> <max bag size> <vertices>", then "b <id> <v...>"
 *             lines (bag ids 1..bags, vertices = the caller's variables
 *             1..n_vars) and "<id> <id>" tree edges; lines starting with 'c'
 *             are comments.
 *   root_bag: bag to root the tree at (1-based; 0 = bag 1).
 *   order:    n_vars entries out (host), a permutation of 1..n_vars to pass
 *             as WMC_TREE_ORDER: variables in no bag first, then each
 *             variable at its bag nearest the root, bags children first.
 *   width:    out (may be NULL): the decomposition's width, max |bag| - 1.
 * With this order no bucket spans more variables than one bag holds, so a
 * plan built from it (block 1) has storage rank at most width + 1.
 * WMC_ERR_INVALID_ARGUMENT if the text is malformed, the vertex count is not
 * n_vars, the bags do not form a tree, a variable's bags are not connected,
 * or no bag holds all caller variables of some clause (message in
 * wmc_last_error()); nothing is written to order then. */
wmc_status wmc_order_from_td(const wmc_network *net, const char *td, int64_t root_bag, int32_t *order,
                             int32_t *width);
wmc_status wmc_plan_stats(const wmc_plan_t *plan, wmc_plan_info *out);
void wmc_plan_destroy(wmc_plan_t *plan);

/* Plan inspection, for tools and tests (host only, any pointer may be NULL).
 * Tensors are numbered 0..n_tensors-1 in creation order.
 *   wmc_plan_tensor: kind 0 = clause leaf (src = clause index), 1 = weight
 *     leaf A_x (src = variable), 2 = internal (src = -1); rank and vars give the
 *     storage layout after slicing, least-significant bit first (vars needs
 *     room for WMC_MAX_RANK entries).
 *   wmc_plan_node: node i (launch order) contracts tensors a and b into c.
 *   wmc_plan_image: the raw device descriptors as they are uploaded
 *     ([leaf descriptors][node descriptors][launch list][matrix-node
 *     descriptors]); with dst == NULL it only reports *needed and
 *     info[0..12] = {n_leaves, n_nodes, n_launches, arena_elems, root,
 *     root_offset, n_tensors, elem_bytes, leaf_desc_bytes, node_desc_bytes,
 *     launch_bytes, n_gemms, gemm_desc_bytes}. */
wmc_status wmc_plan_tensor(const wmc_plan_t *plan, int64_t t, int32_t *kind, int32_t *src,
                           int32_t *rank, int32_t *vars);
wmc_status wmc_plan_node(const wmc_plan_t *plan, int64_t i, int64_t *a, int64_t *b, int64_t *c,
                         int32_t *node_class);
wmc_status wmc_plan_image(const wmc_plan_t *plan, void *dst, uint64_t dst_bytes, uint64_t *needed,
                          int64_t *info /* 13 entries */);

/* ------------------------------------------------------------------ */
/* Execution stage (Algorithm 2 over the slices of Algorithm 3)         */
/* ------------------------------------------------------------------ */

/* Contract the planned network on the current HIP device.
 *   weights:   2*n_vars host doubles replacing the network's weights, or NULL
 *   workspace: device pointer of at least wmc_plan_info.workspace_bytes,
 *              256-byte aligned, owned by the caller; clobbered
 *   stream:    hipStream_t (void*), NULL for the default stream
 * Blocks until the result is on the host.  Errors: INVALID_ARGUMENT (NULL,
 * misaligned or non-finite weights), OUT_OF_MEMORY (workspace too small),
 * DEVICE (HIP failure). */
wmc_status wmc_contract(const wmc_plan_t *plan, const double *weights, void *workspace,
                        uint64_t workspace_bytes, void *stream, wmc_value *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * wmc_contract with its workspace taken from a static device array of
 * WMC_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends.  The call allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine).  Every call on a device shares
 * that device's array, so calls that overlap on one device (other threads,
 * other streams) race; successive calls on one stream are safe.  Blocks
 * until the result is on the host, as wmc_contract does.  Errors:
 * OUT_OF_MEMORY if wmc_plan_info.workspace_bytes exceeds
 * WMC_NOALLOC_SCRATCH_BYTES, INVALID_ARGUMENT (NULL, non-finite weights),
 * DEVICE (HIP failure, including the symbol lookup on first use). */
#define WMC_NOALLOC_SCRATCH_BYTES (64ull << 20)
wmc_status wmc_contract_noalloc(const wmc_plan_t *plan, const double *weights, void *stream, wmc_value *out);

/* Checkpoint of the slice loop (Algorithm 3): the running Neumaier sum
 * (s + c) * 2^e of the slices already run, the next slice to run and the
 * plan's slice count.  Zero-initialise to start; the struct is plain data and
 * can be saved to a file and restored in another process. */
typedef struct {
    double s, c;
    int64_t e;
    int64_t next_slice;
    int64_t n_slices;
    int64_t reserved;
} wmc_slice_state;

/* Run the next `count` slices after state->next_slice (fewer at the end),
 * continuing the running sum in *state, and update *state; *out receives the
 * sum so far (W itself once state->next_slice == n_slices).  Splitting the
 * slice loop across any number of calls gives the bits of one wmc_contract.
 * Errors: INVALID_ARGUMENT (state of another plan, non-finite weights),
 * OUT_OF_MEMORY (workspace), DEVICE. */
wmc_status wmc_contract_resume(const wmc_plan_t *plan, const double *weights, void *workspace,
                               uint64_t workspace_bytes, void *stream, int64_t count,
                               wmc_slice_state *state, wmc_value *out);

/* As wmc_contract, restricted to the slices eta in [slice_begin, slice_end)
 * (the slicing theorem: their sum is a partial sum of W).  If per_slice is
 * not NULL it receives one value per slice in that range. */
wmc_status wmc_contract_slices(const wmc_plan_t *plan, const double *weights, void *workspace,
                               uint64_t workspace_bytes, void *stream, int64_t slice_begin,
                               int64_t slice_end, wmc_value *out, wmc_value *per_slice);

/* Per-launch accounting for measurement.  Launch k of one slice, in the
 * order wmc_contract issues them: 0 = meta reset, 1 = leaf fill, then the
 * node launches, last = slice accumulation.  wmc_plan_launches gives each
 * launch's algorithmic bytes (elem_size * (|A|+|B|+|C|) summed over its
 * nodes), flops (2*b*m*n*k) and node class (-1 for non-node launches); with
 * all arrays NULL it only reports *n_out.  wmc_contract_profile is
 * wmc_contract with a HIP event recorded on `stream` around every launch;
 * ms (cap >= n_out entries) receives in ms[k] the duration of launch k in
 * that same order, summed over the slices. */
wmc_status wmc_plan_launches(const wmc_plan_t *plan, double *bytes, double *flops, int32_t *cls,
                             int64_t cap, int64_t *n_out);
wmc_status wmc_contract_profile(const wmc_plan_t *plan, const double *weights, void *workspace,
                                uint64_t workspace_bytes, void *stream, float *ms, int64_t cap,
                                wmc_value *out);

/* Kernel family of each launch of one slice, in the order of
 * wmc_plan_launches (for attributing measured time to kernels).  Host only;
 * the matrix-kernel choice reads the current device's LDS size.  With
 * kernel == NULL it only reports *n_out. */
enum {
    WMC_KERNEL_BEGIN = 0,         /* k_begin: meta reset */
    WMC_KERNEL_LEAVES = 1,        /* k_leaves: clause and weight tables of a slice */
    WMC_KERNEL_NODES = 2,         /* k_nodes: batched small nodes */
    WMC_KERNEL_GEMM_P = 3,        /* k_gemm_p: persistent MFMA matrix node */
    WMC_KERNEL_GEMM = 4,          /* k_gemm: chunked MFMA matrix node */
    WMC_KERNEL_STREAM_MFMA = 5,   /* k_stream_mfma: streaming node on 16x16 MFMA blocks */
    WMC_KERNEL_STREAM2 = 6,       /* k_stream2: register-tiled streaming node */
    WMC_KERNEL_STREAM2_SPLIT = 7, /* k_stream2_split: summed index split over lane groups */
    WMC_KERNEL_FINISH = 8,        /* k_finish: slice accumulation */
    WMC_KERNEL_STREAM2_VEC = 9    /* k_stream2_vec: K = 1 streaming node, output pairs per thread */
};
wmc_status wmc_plan_kernels(const wmc_plan_t *plan, int32_t *kernel, int64_t cap, int64_t *n_out);

/* ------------------------------------------------------------------ */
/* Batches: many planned networks contracted in shared launches         */
/* ------------------------------------------------------------------ */
/* Each instance is the paper's execution stage (Algorithm 2 over its plan's
 * tree); the paper runs formulas one at a time, this runs many together.
 * The plans' launch lists are merged by index (launch k of one plan depends
 * only on its own launches < k), their descriptors concatenated into one
 * arena, meta table and weight vector, and every root finished by one kernel.
 * Plans must share a precision.  A sliced plan enters as one instance per
 * slice (the slicing theorem: the slices are independent), each slice with
 * its own arena region and its leaves filled for its slice bits, and its
 * result is the FP64 compensated sum of its slices in slice order, as
 * wmc_contract forms it; at most 2^20 slices per plan (WMC_ERR_UNSUPPORTED
 * beyond).  The batch copies what it needs; the plans may be destroyed
 * afterwards.  A batch is used by one thread at a time (calls are
 * serialised internally). */
typedef struct wmc_batch wmc_batch;

#define WMC_BATCH_RESIDENT 1u /* descriptors already in this workspace from an earlier call (the
                                 first call of a batch on a workspace uploads them regardless; the
                                 caller must not overwrite them between calls) */
#define WMC_BATCH_GRAPH 2u    /* capture the launch sequence once per workspace as a HIP graph
                                 and replay it (captured on a private stream) */
#define WMC_BATCH_PERSISTENT 4u /* every merged step in one cooperative launch: one workgroup
                                   per compute unit walks the steps, a grid-wide barrier
                                   between them; results as without it, bit for bit. Batches
                                   with matrix nodes run as without it. Takes precedence over
                                   WMC_BATCH_GRAPH. Slower than graph replay on batches of
                                   small formulas (the barriers and the low occupancy cost
                                   more than the launches saved); WMC_ERR_UNSUPPORTED on a
                                   device without cooperative launches, WMC_ERR_DEVICE if a
                                   barrier wait times out (20 s) */

wmc_status wmc_batch_create(const wmc_plan_t *const *plans, int64_t n, wmc_batch **out);
wmc_status wmc_batch_info(const wmc_batch *b, uint64_t *workspace_bytes, int64_t *n_launches,
                          int64_t *n_instances);
/* weights: the instances' weight vectors concatenated (2 * sum of n_vars
 * doubles, host) or NULL for the networks' own; out: n_instances values. */
wmc_status wmc_batch_contract(wmc_batch *b, const double *weights, void *workspace,
                              uint64_t workspace_bytes, void *stream, uint32_t flags,
                              wmc_value *out);
void wmc_batch_destroy(wmc_batch *b);
/* Raw descriptor image of a batch (tools and tests): [leaf descriptors][node
 * descriptors][launch list][matrix-node descriptors][root tensor int32 x n]
 * [root offset int64 x n][streaming tasks][per launch: first task and the
 * start of each summed-rank group, 6 x int32], with n root entries, one per
 * slice of each plan; info[0..9] = {n_leaves, n_nodes, n_launches,
 * arena_elems, n (root entries), meta_total, elem_bytes, n_gemms,
 * n_vars_total, n_tasks}. */
wmc_status wmc_batch_image(const wmc_batch *b, void *dst, uint64_t dst_bytes, uint64_t *needed,
                           int64_t *info /* 10 entries */);

/* ------------------------------------------------------------------ */
/* Serving: weight queries on registered structures, continuous batching */
/* ------------------------------------------------------------------ */
/* Each request is the paper's execution stage (Algorithm 2) on a registered
 * plan with the request's weights W (Definition 1); requests share launches.
 * A registered structure's descriptors are uploaded once, into the request
 * region pool (they stay resident and count against it); a step uploads
 * only one small work entry per running request and the weights of newly
 * admitted ones.
 * A server owns a caller-supplied device buffer: two staging areas for step
 * descriptors (2 * step_bytes), a result table, and the request regions (at
 * most hbm_budget_bytes).  Registered structures are plans of the server's
 * precision.  A sliced plan (at most 16 sliced variables) serves each request
 * as one part per slice of Algorithm 3, every part queued, admitted and
 * stepped like a request of its own; the request answers once, with the
 * parts' values summed in slice order as wmc_contract sums them, or with
 * WMC_ERR_CANCELLED if any part was cancelled or passed its deadline (a
 * full queue is judged by the parts).  A request (structure, weight vector) waits in a FIFO
 * queue until a slot is free and a region of its footprint (its plan's meta
 * table + arena) fits in the budget: admission by HBM footprint.  Each step
 * runs the next launch of every admitted request's plan in shared kernels;
 * requests join and leave between steps (continuous batching).  A request's
 * descriptors are its plan's shifted into its region, so its value is the
 * same alone or in any mix.  A server is driven by one thread. */
typedef struct wmc_server wmc_server;

typedef struct {
    int32_t precision;          /* wmc_precision of every registered plan */
    int32_t max_slots;          /* requests in flight at once */
    int32_t max_queue;          /* waiting requests; WMC_ERR_BUSY beyond */
    int32_t reserved0;
    uint64_t hbm_budget_bytes;  /* request regions; 0 = all of the buffer left */
    uint64_t step_bytes;        /* staging per step (two are kept); 0 = min(64 MiB, bytes / 8) */
} wmc_serve_options;

typedef struct {
    uint64_t request_id;
    int32_t structure;
    int32_t status;             /* wmc_status */
    wmc_value value;
    double t_arrive, t_admit, t_done;  /* seconds from the server's clock origin */
} wmc_response;

typedef struct {
    double t_arrive;            /* seconds from the start of the replay */
    int32_t structure;
    int32_t reserved0;
    uint64_t request_id;
    const double *weights;      /* 2 * n_vars of the structure, host; copied at submission */
} wmc_request;

typedef struct {
    uint64_t region_bytes, used_bytes, peak_used_bytes;
    int64_t peak_active, steps, n_active, n_queued, n_structures;
} wmc_serve_info;

wmc_status wmc_serve_create(const wmc_serve_options *opts, void *device_buffer, uint64_t bytes,
                            void *stream, wmc_server **out);
wmc_status wmc_serve_register(wmc_server *s, const wmc_plan_t *plan, int32_t *structure_id);
/* Non-blocking: queue one request (WMC_ERR_BUSY if the queue is full). */
wmc_status wmc_serve_submit(wmc_server *s, int32_t structure, const double *weights,
                            uint64_t request_id);
/* As wmc_serve_submit, with a deadline timeout_s seconds from now: a request
 * not finished by then ends with status WMC_ERR_CANCELLED (checked at every
 * step; a running request stops issuing launches). */
wmc_status wmc_serve_submit_deadline(wmc_server *s, int32_t structure, const double *weights,
                                     uint64_t request_id, double timeout_s);
/* Cancel a queued or running request: its response carries status
 * WMC_ERR_CANCELLED (at once if queued; after the step in flight if
 * running, whose region is released only when no step can touch it).
 * INVALID_ARGUMENT if no such request is queued or running. */
wmc_status wmc_serve_cancel(wmc_server *s, uint64_t request_id);
/* Admit what fits and issue one step on the server's stream, then wait for
 * the step issued by the previous call and collect its completions, so the
 * host prepares step k+1 while the device runs step k.  *n_active counts
 * admitted requests, including those whose last launch is still in flight:
 * call until both counts are zero to drain. */
wmc_status wmc_serve_step(wmc_server *s, int32_t *n_active, int32_t *n_queued);
/* Move up to max completed responses into out. */
wmc_status wmc_serve_poll(wmc_server *s, wmc_response *out, int32_t max, int32_t *n_out);
/* Step the server until a response is ready, nothing is queued or running,
 * or timeout_us microseconds have passed; then poll as wmc_serve_poll. */
wmc_status wmc_serve_wait(wmc_server *s, wmc_response *out, int32_t max, int32_t *n_out, int64_t timeout_us);
/* Replay timed arrivals (sorted by t_arrive) until all n complete; out gets
 * the n responses in completion order. */
wmc_status wmc_serve(wmc_server *s, const wmc_request *trace, int64_t n, wmc_response *out);
wmc_status wmc_serve_stats(const wmc_server *s, wmc_serve_info *out);
void wmc_serve_destroy(wmc_server *s);

/* ------------------------------------------------------------------ */
/* Kernel tuning of the executor                                        */
/* ------------------------------------------------------------------ */
/* Launch shapes and kernel-family choices of wmc_contract's streaming
 * nodes, one table per precision.  wmc_plan copies the table current for
 * its precision into the plan, so a plan keeps the setting it was made
 * with.  Any valid setting gives results within the precision's
 * tolerance; the last bits can change where a node moves to another kernel
 * family or its summed index is split differently (split_lanes).  The
 * built-in defaults are measured MI355X settings; the autotuner replaces
 * them with a table measured on the device at hand. */
typedef struct {
    int32_t stream2_grid_cap;        /* workgroups of one register-tiled streaming launch, 8..65536 */
    int32_t stream_mfma_grid_cap;    /* workgroups of one matrix-core streaming launch, 8..65536 */
    int32_t stream_mfma_min_bits;    /* row and column output bits a K >= 16 node needs to run on the
                                        matrix cores, 2..8; 0 = never */
    int32_t stream2_tile_bits;       /* output bits per operand side looped inside a thread, 0..2 */
    int32_t stream2_min_thread_bits; /* looped bits are chosen so that 2^this threads remain, 0..30 */
    int32_t stream2_low_bits;        /* lowest output bits numbering lanes in output order, 0..16 */
    int32_t split_lanes;             /* FP64 nodes with K >= 16: lanes sharing one output's summed
                                        index, 0 (one lane) or 4; ignored for FP32 */
    int32_t multi_min_rank;          /* batches and servers: nodes of a merged step with at least
                                        2^this outputs run on the multi-node streaming kernel, the
                                        rest on the batched small-node kernel, 4..30 (taken from the
                                        first plan of a batch, each registered structure's plan) */
    int32_t gemm_tpw_max_nt;         /* matrix nodes: largest count of 16-column tiles (1, 2, 4) for
                                        which a wave computes two row tiles; 0 = never */
    int32_t gemm_orient;             /* matrix nodes: 0 = transposed tiles when the output's lowest
                                        address bit is a row bit, 1 = always, 2 = never */
    int32_t stream2_vec;             /* K = 1 streaming nodes: 1 = each thread owns output bit 0 and
                                        reads and writes entry pairs (k_stream2_vec), 0 = no */
    int32_t reserved[5];
} wmc_tuning;

/* The current table for a precision (a copy). */
wmc_status wmc_tuning_get(int32_t precision, wmc_tuning *out);
/* Replace the table for a precision for plans made afterwards (process-wide,
 * thread-safe); t == NULL restores the built-in defaults.
 * INVALID_ARGUMENT for a field outside its range. */
wmc_status wmc_tuning_set(int32_t precision, const wmc_tuning *t);

/* Thread-local description of the last non-OK status on this thread. */
const char *wmc_last_error(void);

/* Library version string. */
const char *wmc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WMC_H */
