// Device kernels and launch helpers of the execution stage, shared by the
// single-plan executor (wmc_device.hip) and the batch/serving engines
// (wmc_batch.hip).  Included by HIP translation units only.
//
// Numerics.  Every tensor t carries an exponent: its true entries are
// stored * 2^exp.  A node reads the largest magnitude of each operand (kept
// by the producer with an integer atomicMax on the IEEE bits), scales the
// operand by the power of two that brings that maximum into [0.5, 1) while
// it contracts (exact for normal numbers), and adds both shifts to the
// output's exponent.  Sums are formed in double for both storage
// precisions except on the FP32 matrix path (FP32 MFMA); the FP32 path rounds
// once when it stores.  Slices are summed in double as (s + c) * 2^e with
// Neumaier compensation, in slice order.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <utility>
#include <vector>

#include "wmc_internal.h"

#define WMC_BLOCK 256

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int scale_exp(unsigned long long maxbits) {
    double m = __longlong_as_double((long long)maxbits);
    if (!(m > 0.0)) return 0;
    int e;
    frexp(m, &e);
    return e;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WMC_WAVE));
    return v;
}

// Raise the running max of tensor t to v.  The max only grows, so a value
// read without the atomic is never above the true one: when v does not
// exceed it the atomic is skipped, and after the first few waves almost
// every wave skips it (many waves updating one address serialise there).
__device__ __forceinline__ void raise_max(wmc_meta *meta, int t, double v) {
    if (!(v > 0.0)) return;
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > __atomic_load_n(&meta[t].maxbits, __ATOMIC_RELAXED)) atomicMax(&meta[t].maxbits, b);
}

__device__ __forceinline__ void publish_max(wmc_meta *meta, int t, double v) {
    v = wave_max(v);
    if ((threadIdx.x & (WMC_WAVE - 1)) == 0) raise_max(meta, t, v);
}

// The same for a whole workgroup; every thread of the block must call it.
__device__ __forceinline__ void publish_max_block(wmc_meta *meta, int t, double v) {
    __shared__ double red[16];
    v = wave_max(v);
    const int nw = (int)((blockDim.x + WMC_WAVE - 1) / WMC_WAVE);
    if ((threadIdx.x & (WMC_WAVE - 1)) == 0) red[threadIdx.x / WMC_WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; ++i) v = fmax(v, red[i]);
        raise_max(meta, t, v);
    }
}

// Stores of a streaming node's output, marked non-temporal: a large output
// is read back only by a later node, after far more data than the caches
// hold has passed through them, so its lines need not be kept.  (The matrix
// kernel's scattered 4- and 8-byte stores are not: they need the cache to
// merge them into whole lines, and ran at half speed with the hint.)
template <typename T>
__device__ __forceinline__ void store_nt(T *p, T v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_pair_nt(double *p, double a, double b) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(v2{a, b}, (v2 *)p);
}
__device__ __forceinline__ void store_pair_nt(float *p, float a, float b) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(v2{a, b}, (v2 *)p);
}
__device__ __forceinline__ void store_quad_nt(float *p, float a, float b, float c, float d) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(v4{a, b, c, d}, (v4 *)p);
}

// bit extraction of r along runs (src bit, length, dst bit)
__device__ __forceinline__ unsigned long long pext_runs(unsigned long long r, const unsigned char (*runs)[3], int nr) {
    unsigned long long out = 0;
    for (int q = 0; q < nr; ++q) {
        unsigned s = runs[q][0], l = runs[q][1], d = runs[q][2];
        out |= ((r >> s) & ((1ull << l) - 1ull)) << d;
    }
    return out;
}

// the same for packed run words (src | len << 8 | dst << 16)
template <typename RP>
__device__ __forceinline__ unsigned long long pext_words(unsigned long long r, RP runs, int nr) {
    unsigned long long out = 0;
    for (int q = 0; q < nr; ++q) {
        const unsigned w = runs[q];
        const unsigned s = w & 255u, l = (w >> 8) & 255u, d = w >> 16;
        out |= ((r >> s) & ((1ull << l) - 1ull)) << d;
    }
    return out;
}

template <typename T>
__device__ __forceinline__ double ld(const T *p) { return (double)*p; }

// Slices run side by side in one launch (Algorithm 3's slices are
// independent): grid dimension z numbers the slice within the group, and
// slice z of the group owns its own arena (astride elements apart) and meta
// table (mstride entries apart).  A zero stride with one z leaves a kernel
// on the single arena of a batch or a server.
struct SliceGroup {
    long long astride;
    int mstride;
    int pad;
};

#define WMC_ENTER_SLICE(arena, meta, sg)                       \
    do {                                                       \
        (arena) += (long long)blockIdx.z * (sg).astride;       \
        (meta) += (long long)blockIdx.z * (long long)(sg).mstride; \
    } while (0)

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
static __global__ __attribute__((unused)) void k_begin(wmc_meta *meta, int nt, wmc_acc *acc, int reset) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nt) {
        meta[i].maxbits = 0ull;
        meta[i].exp = 0;
    }
    if (i == 0 && reset) {
        acc->s = 0.0;
        acc->c = 0.0;
        acc->e = 0;
        acc->n_added = 0;
        acc->last_m = 0.0;
        acc->last_e = 0;
    }
}

// Leaf fill (Theorem 2): clause tables B_C restricted to the slice, weight
// vectors [W(x,0), W(x,1)], or W(x,0)+W(x,1) for a variable in no clause.
// Entry e of leaf d filled for slice bits et (every lane of the wave calls
// it; e past the leaf's entries contributes nothing).
template <typename T, typename DP>
__device__ __forceinline__ void leaf_item(DP d, long long e, const double *__restrict__ w,
                                          T *__restrict__ arena, wmc_meta *meta, unsigned long long et) {
    const bool valid = e < (1ll << d->rank);
    double v = 0.0;
    if (valid) {
        if (d->kind == WMC_LEAF_CLAUSE) {
            unsigned a = 0;
            for (int q = 0; q < d->k; ++q) {
                int p = d->pos[q];
                unsigned bit = p >= 0 ? (unsigned)((e >> p) & 1) : (unsigned)((et >> (-p - 1)) & 1ull);
                a |= bit << q;
            }
            v = (d->taut || a != d->falsify) ? 1.0 : 0.0;
        } else {
            // a weight leaf carries its own power-of-two exponent, as every
            // intermediate does: stored entries have magnitude below 1, so
            // any finite weight fits the storage type (FP32 included)
            const double w0 = w[2 * d->var], w1 = w[2 * d->var + 1];
            if (d->kind == WMC_LEAF_WEIGHT) {
                int p = d->pos[0];
                unsigned bit = p >= 0 ? (unsigned)((e >> p) & 1) : (unsigned)((et >> (-p - 1)) & 1ull);
                v = bit ? w1 : w0;
            } else {
                v = w0 + w1;
            }
            const double mx = d->kind == WMC_LEAF_WEIGHT ? fmax(fabs(w0), fabs(w1)) : fabs(v);
            int ex = 0;
            if (mx > 0.0) frexp(mx, &ex);
            v = ldexp(v, -ex);
            if (e == 0) meta[d->tensor].exp = ex;
        }
        T s = (T)v;
        arena[d->out + e] = s;
        v = fabs((double)s);
    }
    publish_max(meta, d->tensor, v);
}

// The body takes its workgroup index and count, so that the fused step
// kernel can run it on a share of its workgroups.
template <typename T>
__device__ __forceinline__ void leaves_body(const LeafDesc *__restrict__ L, int nl, long long work,
                                            const double *__restrict__ w, T *__restrict__ arena, wmc_meta *meta,
                                            unsigned long long eta, const int *__restrict__ wave_leaf,
                                            const unsigned long long *__restrict__ leaf_eta, unsigned blk,
                                            unsigned nblk, unsigned width = 0, unsigned tid = 0) {
    // units of `width` threads (a workgroup by default, or one wave)
    const unsigned W = width ? width : blockDim.x, t = width ? tid : threadIdx.x;
    const long long stride = (long long)nblk * W;
    for (long long g = (long long)blk * W + t; g < work; g += stride) {
        // leaves start on wave boundaries: a wave's items belong to one leaf
        int lo = 0;
        if (wave_leaf) {
            lo = wave_leaf[g / WMC_WAVE];  // one load instead of a dependent search
        } else {
            int hi = nl - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (L[mid].work_begin <= g) lo = mid; else hi = mid - 1;
            }
        }
        // a batch of sliced plans gives every leaf the slice of its instance
        leaf_item<T>(L + lo, g - L[lo].work_begin, w, arena, meta, leaf_eta ? leaf_eta[lo] : eta);
    }
}

template <typename T>
__global__ void __launch_bounds__(WMC_BLOCK) k_leaves(const LeafDesc *__restrict__ L, int nl, long long work,
                                                      const double *__restrict__ w, T *__restrict__ arena,
                                                      wmc_meta *meta, const SliceGroup sg, unsigned long long eta,
                                                      const int *__restrict__ wave_leaf = nullptr,
                                                      const unsigned long long *__restrict__ leaf_eta = nullptr) {
    WMC_ENTER_SLICE(arena, meta, sg);
    leaves_body<T>(L, nl, work, w, arena, meta, eta + blockIdx.z, wave_leaf, leaf_eta, blockIdx.x, gridDim.x);
}

// Pairwise contraction, any shape: one output entry per thread,
// C[r] = 2^-(sA+sB) * sum_j A[(pext_A(r) << nk) | j] * B[(pext_B(r) << nk) | j].
// A launch covers a run of nodes; each node's outputs are padded to a wave
// multiple so that a wave never straddles two nodes.
// Output r of small node d (every lane of the wave calls it; r past the
// node's outputs contributes nothing): C[r] = 2^-(sA+sB) * sum_j
// A[(pext_A(r) << nk) | j] * B[(pext_B(r) << nk) | j].
// DP is a pointer to the descriptor: generic, or in the constant address
// space for descriptors read through the scalar path.
template <typename T, typename DP>
__device__ __forceinline__ void node_item(DP d, unsigned long long r, T *__restrict__ arena,
                                          wmc_meta *meta) {
    const bool valid = r < (1ull << d->rc);
    const int sA = scale_exp(meta[d->ta].maxbits);
    const int sB = scale_exp(meta[d->tb].maxbits);
    double v = 0.0;
    if (valid) {
        const T *A = arena + d->a + (pext_words(r, d->ra, d->nra) << d->nk);
        const T *B = arena + d->b + (pext_words(r, d->rb, d->nrb) << d->nk);
        const int K = 1 << d->nk;
        double acc = 0.0;
        for (int j = 0; j < K; ++j) acc = fma(ld(A + j), ld(B + j), acc);
        T s = (T)ldexp(acc, -(sA + sB));
        arena[d->c + (long long)r] = s;
        v = fabs((double)s);
    }
    publish_max(meta, d->tc, v);
    if (r == 0) meta[d->tc].exp = meta[d->ta].exp + meta[d->tb].exp + sA + sB;
}

template <typename T>
__device__ __forceinline__ void nodes_body(const NodeDesc *__restrict__ D, int nd, long long work,
                                           T *__restrict__ arena, wmc_meta *meta, const int *__restrict__ wave_node,
                                           unsigned blk, unsigned nblk, unsigned width = 0, unsigned tid = 0) {
    // units of `width` threads (a workgroup by default, or one wave)
    const unsigned W = width ? width : blockDim.x, t = width ? tid : threadIdx.x;
    const long long stride = (long long)nblk * W;
    for (long long g = (long long)blk * W + t; g < work; g += stride) {
        // a wave's 64 items belong to one node (outputs are padded to waves):
        // search with the wave's first item so the node index, and every
        // descriptor read, is wave-uniform (scalar loads)
        const long long g0 = ((long long)__builtin_amdgcn_readfirstlane((int)(g >> 6))) << 6;
        int lo = 0;
        if (wave_node) {
            lo = wave_node[g0 >> 6];  // one load instead of a dependent search
        } else {
            int hi = nd - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (D[mid].work_begin <= g0) lo = mid; else hi = mid - 1;
            }
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        node_item<T>(D + lo, (unsigned long long)(g - D[lo].work_begin), arena, meta);
    }
}

template <typename T>
__global__ void __launch_bounds__(WMC_BLOCK) k_nodes(const NodeDesc *__restrict__ D, int nd, long long work,
                                                     T *__restrict__ arena, wmc_meta *meta, const SliceGroup sg,
                                                     const int *__restrict__ wave_node = nullptr) {
    WMC_ENTER_SLICE(arena, meta, sg);
    nodes_body<T>(D, nd, work, arena, meta, wave_node, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Matrix-shaped contractions on MFMA (16x16x4, FP64 or FP32).
//
//   C[beta, mu, nu] = sum_k A[beta, mu, k] * B[beta, k, nu]
//
// The row operand A is stored [4 lowest mu bits | kappa | rest], so the 16
// rows of a row tile are contiguous for each summed index k.  For the
// 16x16x4 instruction lane l supplies row (or column) l%16 and reduction
// slot l/16; at step s lane group g = l/16 takes summed index k = 4s + g, so
// one load instruction of a wave reads A[tile][k = 4s..4s+3][16 rows]: 512
// contiguous bytes (FP64).  A and B use the same k for a given (s, g), so
// every (row, k, column) term is summed exactly once.  B, the small operand
// (columns contiguous in kappa), is staged per chunk of KC summed indices in
// LDS as [k][column].  A workgroup of 4 waves owns 8 row tiles (2 per wave)
// of one beta and all N <= 128 columns.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Output register v of lane l holds column l%16 and row out_row(l/16, v):
// rows g + 4v for the FP64 instruction, 4g + v for the FP32 one (measured).
template <> struct Mfma<double> {
    typedef dbl4 acc_t;
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int g, int v) { return g + 4 * v; }
};
template <> struct Mfma<float> {
    typedef flt4 acc_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int g, int v) { return 4 * g + v; }
};

#ifndef GEMM_TILES_PER_WAVE
#define GEMM_TILES_PER_WAVE 2
#endif
#define GEMM_TILES (4 * GEMM_TILES_PER_WAVE)
#define GEMM_LDS_BYTES (48 * 1024)

__host__ __device__ inline int gemm_ldn(int nn, int elem) { return (1 << nn) + (elem == 8 ? 2 : 4); }

__host__ __device__ inline int gemm_kc(int nk, int nn, int elem) {
    int K = 1 << nk;
    int kc = K < 64 ? K : 64;
    while (kc > 4 && (long long)kc * gemm_ldn(nn, elem) * elem > GEMM_LDS_BYTES) kc >>= 1;
    return kc;
}

template <typename T, int NT>
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc *__restrict__ G, T *__restrict__ arena, wmc_meta *meta,
                                              const SliceGroup sg) {
    WMC_ENTER_SLICE(arena, meta, sg);
    typedef typename Mfma<T>::acc_t acc_t;
    extern __shared__ char smem_raw[];
    T *Bs = (T *)smem_raw;
    const GemmDesc &d = *G;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, l16 = lane & 15;
    const int nk = d.nk;
    const int K = 1 << nk, N = 1 << d.nn;
    const int KC = gemm_kc(nk, d.nn, (int)sizeof(T));
    const int S = KC / 4;
    const int LDN = gemm_ldn(d.nn, (int)sizeof(T));
    const unsigned long long tiles = 1ull << (d.nm - 4);
    const unsigned long long beta = blockIdx.y;
    const int sA = scale_exp(meta[d.ta].maxbits);
    const int sB = scale_exp(meta[d.tb].maxbits);
    const unsigned long long rowBeta = pext_runs(beta, d.run[GR_BETA_A], d.nrun[GR_BETA_A]);
    const unsigned long long colBeta = pext_runs(beta, d.run[GR_BETA_B], d.nrun[GR_BETA_B]);
    const unsigned long long t0 = ((unsigned long long)blockIdx.x * 4 + wave) * GEMM_TILES_PER_WAVE;

    long long abase[GEMM_TILES_PER_WAVE];
    bool tv[GEMM_TILES_PER_WAVE];
#pragma unroll
    for (int rt = 0; rt < GEMM_TILES_PER_WAVE; ++rt) {
        unsigned long long t = t0 + rt;
        tv[rt] = t < tiles;
        abase[rt] = d.a + l16 +
                    (long long)((pext_runs(tv[rt] ? t : 0, d.run[GR_MU_A], d.nrun[GR_MU_A]) | rowBeta) << (4 + nk));
    }
    acc_t acc[GEMM_TILES_PER_WAVE][NT];
#pragma unroll
    for (int rt = 0; rt < GEMM_TILES_PER_WAVE; ++rt)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = acc_t{0, 0, 0, 0};

    for (int kc = 0; kc < K; kc += KC) {
        for (int idx = threadIdx.x; idx < N * KC; idx += 256) {
            int col = idx / KC, k = idx - col * KC;
            unsigned long long cb = pext_runs((unsigned long long)col, d.run[GR_NU_B], d.nrun[GR_NU_B]) | colBeta;
            Bs[k * LDN + col] = arena[d.b + (long long)(cb << nk) + kc + k];
        }
        T a[GEMM_TILES_PER_WAVE][16];
#pragma unroll
        for (int rt = 0; rt < GEMM_TILES_PER_WAVE; ++rt)
#pragma unroll
            for (int s = 0; s < 16; ++s)
                a[rt][s] = (s < S && tv[rt]) ? arena[abase[rt] + 16 * (long long)(kc + 4 * s + g)] : (T)0;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            if (s < S) {
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const int col = ct * 16 + l16;
                    T b = (col < N) ? Bs[(4 * s + g) * LDN + col] : (T)0;
#pragma unroll
                    for (int rt = 0; rt < GEMM_TILES_PER_WAVE; ++rt)
                        acc[rt][ct] = Mfma<T>::step(a[rt][s], b, acc[rt][ct]);
                }
            }
        }
        __syncthreads();
    }

    const double scale = ldexp(1.0, -(sA + sB));
    const unsigned long long cBeta = pext_runs(beta, d.run[GR_BETA_C], d.nrun[GR_BETA_C]);
    unsigned long long rowC[GEMM_TILES_PER_WAVE][4];
#pragma unroll
    for (int rt = 0; rt < GEMM_TILES_PER_WAVE; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            unsigned long long m = ((t0 + rt) << 4) + Mfma<T>::out_row(g, v);
            rowC[rt][v] = pext_runs(m, d.run[GR_MU_C], d.nrun[GR_MU_C]) | cBeta;
        }
    double vmax = 0.0;
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
        const int col = ct * 16 + l16;
        if (col >= N) continue;
        const unsigned long long cc = pext_runs((unsigned long long)col, d.run[GR_NU_C], d.nrun[GR_NU_C]);
#pragma unroll
        for (int rt = 0; rt < GEMM_TILES_PER_WAVE; ++rt) {
            if (!tv[rt]) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T sv = (T)((double)acc[rt][ct][v] * scale);
                arena[d.c + (long long)(rowC[rt][v] | cc)] = sv;
                vmax = fmax(vmax, fabs((double)sv));
            }
        }
    }
    publish_max_block(meta, d.tc, vmax);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        meta[d.tc].exp = meta[d.ta].exp + meta[d.tb].exp + sA + sB;
}

// Persistent form for the common case where all of B[beta] (K <= 64 summed
// indices x N columns) fits in LDS: each workgroup stages B once, then walks
// row-tile groups blockIdx.x, blockIdx.x + gridDim.x, ..., loading the next
// group's A fragments into registers while the MFMAs of the current group run.
// 64-bit value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ unsigned long long uniform64(unsigned long long x) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Row tiles per wave and tile group of the persistent kernel: two for FP64
// with at most 32 columns, else one (measured: the FP32 and the wide FP64
// variants run faster with more, smaller groups per workgroup).
template <typename T>
__host__ __device__ constexpr int gemm_tpw(int nt) { return (sizeof(T) == 8 && nt <= 2) ? 2 : 1; }

// SW selects the orientation of the matrix instruction.  SW = false: lane l
// of an output tile holds column l%16 and rows out_row(l/16, v).  SW = true
// computes the transposed tile (operands swapped: B^T A^T), so lane l holds
// row l%16 and columns out_row(l/16, v); used when C's lowest address bits
// belong to rows, so that 16 lanes store 16 consecutive elements.
template <typename T, int NT, int S, bool SW, int TPW>
__global__ void __launch_bounds__(256) k_gemm_p(const GemmDesc *__restrict__ G, T *__restrict__ arena,
                                                wmc_meta *meta, const SliceGroup sg) {
    WMC_ENTER_SLICE(arena, meta, sg);
    typedef typename Mfma<T>::acc_t acc_t;
    extern __shared__ char smem_raw[];
    __shared__ GemmDesc sd;
    T *Bs = (T *)smem_raw;
    // the descriptor lives in LDS so that run-list reads never wait on the
    // vector-memory counter that tracks the A prefetches
    for (int i = threadIdx.x; i < (int)(sizeof(GemmDesc) / sizeof(int)); i += 256)
        ((int *)&sd)[i] = ((const int *)G)[i];
    __syncthreads();
    const GemmDesc &d = sd;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, l16 = lane & 15;
    constexpr int K = 4 * S;
    const int nk = d.nk;
    const int N = 1 << d.nn;
    constexpr int LDN = NT * 16 + (sizeof(T) == 8 ? 2 : 4);
    const unsigned long long tiles = 1ull << (d.nm - 4);
    const unsigned long long groups = (tiles + 4 * TPW - 1) / (4 * TPW);
    const unsigned long long beta = blockIdx.y;
    const long long a0 = d.a, c0 = d.c;
    const int sA = scale_exp(meta[d.ta].maxbits);
    const int sB = scale_exp(meta[d.tb].maxbits);
    const unsigned long long rowBeta = pext_runs(beta, d.run[GR_BETA_A], d.nrun[GR_BETA_A]);
    const unsigned long long colBeta = pext_runs(beta, d.run[GR_BETA_B], d.nrun[GR_BETA_B]);
    const unsigned long long cBeta = pext_runs(beta, d.run[GR_BETA_C], d.nrun[GR_BETA_C]);
    const double scale = ldexp(1.0, -(sA + sB));

    // A fragments: loads are unconditional (a row tile past the end reads
    // tile 0 and is discarded) so the compiler can count them precisely
    T an[TPW][S];
    bool okn[TPW];
    auto load = [&](unsigned long long grp) {
#pragma unroll
        for (int rt = 0; rt < TPW; ++rt) {
            unsigned long long t = (grp * 4 + wave) * TPW + rt;
            okn[rt] = grp < groups && t < tiles;
            long long base =
                a0 + l16 + (long long)((pext_runs(okn[rt] ? t : 0, d.run[GR_MU_A], d.nrun[GR_MU_A]) | rowBeta) << (4 + nk));
#pragma unroll
            for (int s = 0; s < S; ++s) an[rt][s] = arena[base + 16 * (4 * s + g)];
        }
    };
    load(blockIdx.x);  // first A tile group in flight while B is staged

    // B[beta] as [k][column], columns N..16*NT-1 zero
    for (int idx = threadIdx.x; idx < NT * 16 * K; idx += 256) {
        int col = idx / K, k = idx - col * K;
        T v = (T)0;
        if (col < N) {
            unsigned long long cb = pext_runs((unsigned long long)col, d.run[GR_NU_B], d.nrun[GR_NU_B]) | colBeta;
            v = arena[d.b + (long long)(cb << nk) + k];
        }
        Bs[k * LDN + col] = v;
    }
    // Output addresses.  Bit extraction is an OR over disjoint source bits, so
    // the address of (row, col) splits into per-lane and wave-uniform parts:
    // out_row(g, v) = out_row(g, 0) | out_row(0, v), col = 16 ct | (col % 16).
    unsigned long long cols[SW ? 1 : NT];  // !SW: per-lane column part per column tile
    unsigned long long rlo[SW ? 1 : 4];    // !SW: per-lane row part per register
    unsigned long long lrow = 0, lcol = 0;  // SW: per-lane row and column parts
    unsigned long long ucol_v[SW ? 4 : 1], ucol_t[SW ? NT : 1];  // SW: uniform column parts
    if constexpr (!SW) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int col = ct * 16 + l16;
            cols[ct] = pext_runs((unsigned long long)(col < N ? col : 0), d.run[GR_NU_C], d.nrun[GR_NU_C]) | cBeta;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            rlo[v] = pext_runs((unsigned long long)Mfma<T>::out_row(g, v), d.run[GR_MU_C], d.nrun[GR_MU_C]);
    } else {
        lrow = pext_runs((unsigned long long)l16, d.run[GR_MU_C], d.nrun[GR_MU_C]);
        lcol = pext_runs((unsigned long long)Mfma<T>::out_row(g, 0), d.run[GR_NU_C], d.nrun[GR_NU_C]) | cBeta;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            ucol_v[v] = uniform64(pext_runs((unsigned long long)Mfma<T>::out_row(0, v), d.run[GR_NU_C], d.nrun[GR_NU_C]));
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
            ucol_t[ct] = uniform64(pext_runs((unsigned long long)(ct * 16), d.run[GR_NU_C], d.nrun[GR_NU_C]));
    }

    __syncthreads();
    double vmax = 0.0;
    for (unsigned long long grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        // B is the same in every group; keep the compiler from hoisting all
        // its LDS reads out of the loop when they would not fit beside the
        // accumulators (NT * S values per lane: 128 registers at K = N = 64,
        // which left one wave per SIMD)
        if constexpr (NT * S > 16) asm volatile("" ::: "memory");
        T a[TPW][S];
        bool ok[TPW];
#pragma unroll
        for (int rt = 0; rt < TPW; ++rt) {
            ok[rt] = okn[rt];
#pragma unroll
            for (int s = 0; s < S; ++s) a[rt][s] = an[rt][s];
        }
        unsigned long long thi[TPW];
#pragma unroll
        for (int rt = 0; rt < TPW; ++rt) {
            unsigned long long t = (grp * 4 + wave) * TPW + rt;
            thi[rt] = pext_runs(ok[rt] ? (t << 4) : 0, d.run[GR_MU_C], d.nrun[GR_MU_C]);
        }
        load(grp + gridDim.x);
        acc_t acc[TPW][NT];
#pragma unroll
        for (int rt = 0; rt < TPW; ++rt)
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                T b = Bs[(4 * s + g) * LDN + ct * 16 + l16];
#pragma unroll
                for (int rt = 0; rt < TPW; ++rt) {
                    if constexpr (SW)
                        acc[rt][ct] = Mfma<T>::step(b, a[rt][s], acc[rt][ct]);
                    else
                        acc[rt][ct] = Mfma<T>::step(a[rt][s], b, acc[rt][ct]);
                }
            }
        }
#pragma unroll
        for (int rt = 0; rt < TPW; ++rt) {
            if (!ok[rt]) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if constexpr (!SW) {
                    const unsigned long long rc = thi[rt] | rlo[v];
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) {
                        if (NT == 1 && l16 >= N) continue;
                        T sv = (T)((double)acc[rt][ct][v] * scale);
                        arena[c0 + (long long)(rc | cols[ct])] = sv;
                        vmax = fmax(vmax, fabs((double)sv));
                    }
                } else {
                    const unsigned long long rc = thi[rt] | lrow | lcol | ucol_v[v];
                    const bool live = NT > 1 || Mfma<T>::out_row(g, v) < N;
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) {
                        if (!live) continue;
                        T sv = (T)((double)acc[rt][ct][v] * scale);
                        arena[c0 + (long long)(rc | ucol_t[ct])] = sv;
                        vmax = fmax(vmax, fabs((double)sv));
                    }
                }
            }
        }
    }
    publish_max_block(meta, d.tc, vmax);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        meta[d.tc].exp = meta[d.ta].exp + meta[d.tb].exp + sA + sB;
}

// LDS a workgroup may use for B, from the device's per-block limit (kept to
// at most 96 KiB so that two workgroups share a CU).
static inline int lds_budget() {
    static int budget[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return GEMM_LDS_BYTES;
    if (!budget[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
        budget[dev] = v >= 96 * 1024 ? 96 * 1024 : GEMM_LDS_BYTES;
    }
    return budget[dev];
}

// LDS bytes of B[beta] in the persistent matrix kernel (rows padded against
// bank conflicts).
template <typename T>
static inline size_t gemm_p_lds(const GemmDesc &hd) {
    const int N = 1 << hd.nn, K = 1 << hd.nk;
    const int NT = (N + 15) / 16;
    return (size_t)K * (NT * 16 + (sizeof(T) == 8 ? 2 : 4)) * sizeof(T);
}

// True when a matrix node runs on the persistent kernel k_gemm_p (K of 4 to
// 64 and B[beta] fits the LDS budget); otherwise the chunked k_gemm runs.
template <typename T>
static inline bool gemm_persistent(const GemmDesc &hd) {
    const int K = 1 << hd.nk;
    return K >= 4 && K <= 64 && gemm_p_lds<T>(hd) <= (size_t)lds_budget();
}

// Launch shape of the persistent matrix kernel from the executor tuning
// table: the largest column-tile count that takes two row tiles per wave
// (-1: the built-in rule), and the orientation (0: transposed tiles when C's
// lowest address bit is a row bit, 1: always transposed, 2: never).
struct GemmShape {
    int tpw_max_nt = -1;
    int orient = 0;
};

template <typename T>
static void launch_gemm(const GemmDesc &hd, const GemmDesc *dd, T *arena, wmc_meta *meta, hipStream_t st,
                        const SliceGroup sg = SliceGroup{0, 0, 0}, unsigned nz = 1, GemmShape shape = GemmShape{}) {
    const int N = 1 << hd.nn, K = 1 << hd.nk;
    const int NT = (N + 15) / 16;
    const unsigned long long tiles = 1ull << (hd.nm - 4);
    const unsigned long long groups = (tiles + GEMM_TILES - 1) / GEMM_TILES;  // fallback kernel
    const size_t padded = gemm_p_lds<T>(hd);
    if (gemm_persistent<T>(hd)) {
        const int NTp = NT <= 1 ? 1 : NT <= 2 ? 2 : NT <= 4 ? 4 : 8;
        // two row tiles per wave up to 4 column tiles (8 would not fit the registers)
        const int tpw = NTp <= 4 && (shape.tpw_max_nt < 0 ? gemm_tpw<T>(NTp) == 2 : NTp <= shape.tpw_max_nt) ? 2 : 1;
        // persistent grid: as many workgroups as fit on the device at once
        auto grid_of = [&](const void *fn) {
            int dev = 0, cus = 256, per_cu = 2;
            if (hipGetDevice(&dev) == hipSuccess)
                (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, padded) != hipSuccess || per_cu < 1)
                per_cu = 2;
            // resident workgroups, shared by the nz slices of the launch
            unsigned long long total = (unsigned long long)cus * (unsigned long long)per_cu / nz;
            if (total < 1) total = 1;
            unsigned long long per_beta = (total + (1ull << hd.nb) - 1) >> hd.nb;
            if (per_beta < 1) per_beta = 1;
            const unsigned long long tg = 4ull * (unsigned long long)tpw;
            const unsigned long long pgroups = (tiles + tg - 1) / tg;
            return dim3((unsigned)(pgroups < per_beta ? pgroups : per_beta), 1u << hd.nb, nz);
        };
        // transposed tiles when C's lowest address bit is a row bit
        bool sw = false;
        for (int q = 0; q < hd.nrun[GR_MU_C]; ++q)
            if (hd.run[GR_MU_C][q][2] == 0) sw = true;
        if (shape.orient == 1) sw = true;
        if (shape.orient == 2) sw = false;
#define WMC_GP1(NTV, SV, SWV, TPWV)                                                                            \
    if (NTp == NTV && K / 4 == SV && sw == SWV && tpw == TPWV) {                                             \
        const void *fn = (const void *)&k_gemm_p<T, NTV, SV, SWV, TPWV>;                                     \
        hipLaunchKernelGGL((k_gemm_p<T, NTV, SV, SWV, TPWV>), grid_of(fn), dim3(256), padded, st, dd, arena, meta, \
                           sg);                                                                              \
        return;                                                                                              \
    }
#define WMC_GP(NTV, SV, TPWV) WMC_GP1(NTV, SV, false, TPWV) WMC_GP1(NTV, SV, true, TPWV)
#define WMC_GP_S(NTV, TPWV) \
    WMC_GP(NTV, 1, TPWV) WMC_GP(NTV, 2, TPWV) WMC_GP(NTV, 4, TPWV) WMC_GP(NTV, 8, TPWV) WMC_GP(NTV, 16, TPWV)
        WMC_GP_S(1, 1) WMC_GP_S(2, 1) WMC_GP_S(4, 1) WMC_GP_S(8, 1)
        WMC_GP_S(1, 2) WMC_GP_S(2, 2) WMC_GP_S(4, 2)
#undef WMC_GP_S
#undef WMC_GP
#undef WMC_GP1
    }
    const int KC = gemm_kc(hd.nk, hd.nn, (int)sizeof(T));
    const size_t smem = (size_t)KC * gemm_ldn(hd.nn, (int)sizeof(T)) * sizeof(T);
    dim3 grid((unsigned)groups, 1u << hd.nb, nz);
    if (NT <= 1) hipLaunchKernelGGL((k_gemm<T, 1>), grid, dim3(256), smem, st, dd, arena, meta, sg);
    else if (NT <= 2) hipLaunchKernelGGL((k_gemm<T, 2>), grid, dim3(256), smem, st, dd, arena, meta, sg);
    else if (NT <= 4) hipLaunchKernelGGL((k_gemm<T, 4>), grid, dim3(256), smem, st, dd, arena, meta, sg);
    else hipLaunchKernelGGL((k_gemm<T, 8>), grid, dim3(256), smem, st, dd, arena, meta, sg);
}

// ---------------------------------------------------------------------------
// Register-tiled streaming contraction for one big node,
//
//   C[beta, sigma, omega] = sum_kappa S[beta, sigma, kappa] * O[beta, omega, kappa]
//
// with S the larger operand, sigma the output bits only S has and omega the
// output bits only O has.  Each thread owns P = 2^np values of (up to two,
// high) sigma bits and Q = 2^nq values of (up to two, high) omega bits: it
// loads P rows of S and Q rows of O (2^nk contiguous summed entries each, in
// chunks of up to 8) and produces the P x Q outputs, so each S row is read
// once per Q outputs and each O row once per P.  The remaining output bits
// enumerate threads: the lowest ones in C order, so for a fixed (p, q) the
// lanes of a wave store consecutive outputs, then the other one-operand
// bits, so that threads sharing a row run at the same time.  The bits
// chosen for P and Q are the highest one-operand bits.  O is staged in LDS when it has at
// most 2^12 entries.  Every product is summed in the order of the summed
// index and scaled once at the end, exactly as the generic node kernel does.
#define STREAM2_RUNS 16
#define STREAM2_LRUNS 16
#define STREAM2_O_LDS 4096

struct Stream2Args {
    long long s, o, c;                 // element offsets in the arena
    int ts, to, tc;                    // meta entries of S, O, C
    int rc;                            // output rank
    int np, nq;                        // sigma bits and omega bits handled inside a thread
    int pbit[2], qbit[2];              // their positions in C
    int nlrun, nsrun, norun;
    unsigned lrun[STREAM2_LRUNS];      // thread index -> C address (runs src | len << 8 | dst << 16)
    unsigned srun[STREAM2_RUNS];       // C address -> S row
    unsigned orun[STREAM2_RUNS];       // C address -> O row
    int ro;                            // storage rank of O, summed bits included
    int o_lds;                         // O staged in LDS
    int vec;                           // K = 1: output bit 0 handled inside the thread (k_stream2_vec)
};

// The solo kernels' thread-index maps as tables.  A thread's work item u is
// (uh << lbits) | ul, uh uniform in the workgroup (its tile round) and ul
// the lane's part; the C address r0 = lmap(u) and the operand rows
// smap(r0), omap(r0) are bit deposits onto disjoint bits, hence linear in
// the bits of u: each is hi(uh) | lo(ul).  hi is an OR over 4-bit chunks of
// uh, looked up with scalar loads from the kernel arguments; lo is read once
// per thread.  This replaces three run expansions per work item (dozens of
// 64-bit shifts, and spills of the run words) with a few scalar loads.
#define STREAM2_NCH 7

struct Stream2Tab {
    Stream2Args a;
    int lbits, nch, pad0, pad1;
    unsigned long long hr[STREAM2_NCH][16], hs[STREAM2_NCH][16], ho[STREAM2_NCH][16];
    unsigned long long lr[2][16], ls[2][16], lo[2][16];
};

// Tables of t->a for lane parts of lbits bits; false if the uniform part
// needs more than STREAM2_NCH chunks.
static inline bool stream2_tab(Stream2Tab *t, int lbits) {
    const Stream2Args &a = t->a;
    auto runs = [](unsigned long long r, const unsigned *rn, int n) {
        unsigned long long out = 0;
        for (int i = 0; i < n; ++i)
            out |= ((r >> (rn[i] & 255u)) & ((1ull << ((rn[i] >> 8) & 255u)) - 1ull)) << (rn[i] >> 16);
        return out;
    };
    const int ubits = a.rc - a.np - a.nq - (a.vec ? 1 : 0);
    const int hbits = ubits > lbits ? ubits - lbits : 0;
    t->lbits = lbits;
    t->nch = (hbits + 3) / 4;
    if (t->nch > STREAM2_NCH || lbits > 8) return false;
    auto fill = [&](unsigned long long u, unsigned long long *r, unsigned long long *sr, unsigned long long *orow) {
        const unsigned long long c = runs(u, a.lrun, a.nlrun);
        *r = c;
        *sr = runs(c, a.srun, a.nsrun);
        *orow = runs(c, a.orun, a.norun);
    };
    for (unsigned v = 0; v < 16; ++v) {
        for (int c = 0; c < t->nch; ++c)
            fill((unsigned long long)v << (lbits + 4 * c), &t->hr[c][v], &t->hs[c][v], &t->ho[c][v]);
        for (int c = 0; c < 2; ++c) {
            const unsigned long long u = ((unsigned long long)v << (4 * c)) & ((1ull << lbits) - 1ull);
            fill(u, &t->lr[c][v], &t->ls[c][v], &t->lo[c][v]);
        }
    }
    return true;
}

// Bit extraction along at most MAX runs (unrolled with static indices, so
// run words passed in kernel arguments stay in scalar registers).
template <int MAX, typename RP>
__device__ __forceinline__ unsigned long long apply_runs(unsigned long long r, RP runs, int n) {
    unsigned long long out = 0;
#pragma unroll
    for (int i = 0; i < MAX; ++i)
        if (i < n) {
            const unsigned w = runs[i];
            out |= ((r >> (w & 255u)) & ((1ull << ((w >> 8) & 255u)) - 1ull)) << (w >> 16);
        }
    return out;
}

// KC consecutive entries of a row, widened to double.
template <typename T, int KC>
__device__ __forceinline__ void load_chunk(const T *__restrict__ p, double *v) {
    if constexpr (sizeof(T) == 8 && KC >= 2) {
#pragma unroll
        for (int h = 0; h < KC / 2; ++h) {
            const double2 x = ((const double2 *)p)[h];
            v[2 * h] = x.x;
            v[2 * h + 1] = x.y;
        }
    } else if constexpr (sizeof(T) == 4 && KC == 4) {
        const float4 x = *(const float4 *)p;
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    } else if constexpr (sizeof(T) == 4 && KC == 2) {
        const float2 x = *(const float2 *)p;
        v[0] = x.x;
        v[1] = x.y;
    } else {
#pragma unroll
        for (int k = 0; k < KC; ++k) v[k] = (double)p[k];
    }
}

// Two neighbouring outputs with one store (p is 2-element aligned).
__device__ __forceinline__ void store_pair(double *p, double a, double b) { *(double2 *)p = make_double2(a, b); }
__device__ __forceinline__ void store_pair(float *p, float a, float b) { *(float2 *)p = make_float2(a, b); }

// NP and NQ are compile-time so that the tile loops are straight-line code:
// all loads issue before the first wait and no store waits on another.
template <typename T, int NK, int NP, int NQ>
__global__ void __launch_bounds__(256) k_stream2(const Stream2Tab tab, T *__restrict__ arena, wmc_meta *meta,
                                                 const SliceGroup sg) {
    WMC_ENTER_SLICE(arena, meta, sg);
    const Stream2Args &args = tab.a;
    extern __shared__ char smem_raw[];
    double *Os = (double *)smem_raw;  // 2^ro entries when O is staged, else none
    constexpr int K = 1 << NK;
    // summed entries per register chunk: 8 for K >= 16 (fewer dependent
    // load rounds; measured 11-15% faster than 4 on the banded formula)
    constexpr int KC = K < 4 ? K : (NK >= 4 ? 8 : 4);
    constexpr int CHUNK_UNROLL = NK >= 4 ? 1 : 8;
    constexpr int P = 1 << NP, Q = 1 << NQ;
    const int sS = scale_exp(meta[args.ts].maxbits);
    const int sO = scale_exp(meta[args.to].maxbits);
    const T *__restrict__ S = arena + args.s;
    const T *__restrict__ O = arena + args.o;
    T *__restrict__ C = arena + args.c;
    if (args.o_lds) {
        for (int i = threadIdx.x; i < (1 << args.ro); i += 256) Os[i] = (double)O[i];
        __syncthreads();
    }
    unsigned long long cP[P], sP[P], cQ[Q], oQ[Q];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        unsigned long long c = 0;
#pragma unroll
        for (int t = 0; t < NP; ++t) c |= (unsigned long long)((i >> t) & 1) << args.pbit[t];
        cP[i] = uniform64(c);
        sP[i] = uniform64(apply_runs<STREAM2_RUNS>(c, args.srun, args.nsrun));
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        unsigned long long c = 0;
#pragma unroll
        for (int t = 0; t < NQ; ++t) c |= (unsigned long long)((j >> t) & 1) << args.qbit[t];
        cQ[j] = uniform64(c);
        oQ[j] = uniform64(apply_runs<STREAM2_RUNS>(c, args.orun, args.norun));
    }
    const int se = -(sS + sO);
    const unsigned long long threads = 1ull << (args.rc - NP - NQ);
    // workgroups are dealt to the 8 XCDs round-robin; renumber them so that
    // each XCD walks one contiguous slab of threads per sweep and rows shared
    // by nearby threads meet in that XCD's L2
    const unsigned G = gridDim.x;
    const unsigned lb = (G % 8u == 0u) ? (blockIdx.x % 8u) * (G / 8u) + blockIdx.x / 8u : blockIdx.x;
    double vmax = 0.0;
    const unsigned ul = threadIdx.x;
    const unsigned long long rl = tab.lr[0][ul & 15u] | tab.lr[1][(ul >> 4) & 15u];
    const unsigned long long sl = tab.ls[0][ul & 15u] | tab.ls[1][(ul >> 4) & 15u];
    const unsigned long long ol = tab.lo[0][ul & 15u] | tab.lo[1][(ul >> 4) & 15u];
    for (unsigned long long uh = lb; (uh << 8) < threads; uh += G) {
        if (((uh << 8) | ul) >= threads) continue;
        unsigned long long r0 = rl, s0 = sl, o0 = ol;
#pragma unroll
        for (int c = 0; c < STREAM2_NCH; ++c)
            if (c < tab.nch) {
                const unsigned v = (unsigned)(uh >> (4 * c)) & 15u;
                r0 |= tab.hr[c][v];
                s0 |= tab.hs[c][v];
                o0 |= tab.ho[c][v];
            }
        double acc[P][Q];
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < Q; ++j) acc[i][j] = 0.0;
        // K >= 16: the chunk loop stays rolled, so only one chunk's rows
        // are in registers (fully unrolled, the loads of every chunk were
        // hoisted: 256+ registers, one wave per SIMD)
#pragma unroll CHUNK_UNROLL
        for (int kc = 0; kc < K; kc += KC) {
            double sv[P][KC], ov[Q][KC];
#pragma unroll
            for (int i = 0; i < P; ++i) load_chunk<T, KC>(S + (((s0 | sP[i]) << NK) + kc), sv[i]);
            if (args.o_lds) {
#pragma unroll
                for (int j = 0; j < Q; ++j) {
                    const unsigned long long ob = ((o0 | oQ[j]) << NK) + kc;
#pragma unroll
                    for (int k = 0; k < KC; ++k) ov[j][k] = Os[ob + k];
                }
            } else {
#pragma unroll
                for (int j = 0; j < Q; ++j) load_chunk<T, KC>(O + (((o0 | oQ[j]) << NK) + kc), ov[j]);
            }
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
                for (int j = 0; j < Q; ++j)
#pragma unroll
                    for (int k = 0; k < KC; ++k) acc[i][j] = fma(sv[i][k], ov[j][k], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const T v = (T)ldexp(acc[i][j], se);
                store_nt(C + (r0 | cP[i] | cQ[j]), v);
                vmax = fmax(vmax, fabs((double)v));
            }
    }
    publish_max_block(meta, args.tc, vmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) meta[args.tc].exp = meta[args.ts].exp + meta[args.to].exp + sS + sO;
}

// Long summed index (K >= 8): the same register tile, but the K summed
// entries of every output are split over a group of LG lanes, lane p of a
// group holding entries [p K/LG, (p+1) K/LG) of each of its P + Q rows.  A
// load instruction then reads whole rows (LG lanes side by side in one
// row) instead of one 16-byte piece of 64 different rows, which is what
// bounds the unsplit kernel at K = 16.  After the partial products, a
// butterfly over the group (lane p and p ^ b, b = LG/2 ... 1) halves the
// P x Q partial sums per step: the lane with bit b set keeps the upper half
// and receives the partner's, the other the lower half, so each lane ends
// with PQ / LG complete outputs (or, when PQ < LG, the group's lanes agree
// on the single output and the lowest stores it).  The sum over the
// summed index is therefore a fixed tree over the lanes' sequential partial
// sums.
template <int V, int B>
__device__ __forceinline__ void group_reduce_scatter(double *v, int lane, int &fbase, int &dup) {
    if constexpr (B >= 1) {
        if constexpr (V > 1) {
            const bool up = (lane & B) != 0;
#pragma unroll
            for (int t = 0; t < V / 2; ++t) {
                const double send = up ? v[t] : v[t + V / 2];
                const double keep = up ? v[t + V / 2] : v[t];
                v[t] = keep + __shfl_xor(send, B, WMC_WAVE);
            }
            if (up) fbase += V / 2;
            group_reduce_scatter<V / 2, B / 2>(v, lane, fbase, dup);
        } else {
            v[0] += __shfl_xor(v[0], B, WMC_WAVE);
            dup |= B;
            group_reduce_scatter<1, B / 2>(v, lane, fbase, dup);
        }
    }
}

template <typename T, int NK, int NP, int NQ, int LG>
__global__ void __launch_bounds__(256) k_stream2_split(const Stream2Tab tab, T *__restrict__ arena,
                                                       wmc_meta *meta, const SliceGroup sg) {
    WMC_ENTER_SLICE(arena, meta, sg);
    const Stream2Args &args = tab.a;
    constexpr int K = 1 << NK;
    constexpr int KL = K / LG;  // summed entries per lane and row
    constexpr int P = 1 << NP, Q = 1 << NQ, PQ = P * Q;
    constexpr int GPB = 256 / LG;  // groups per workgroup
    constexpr int VF = PQ >= LG ? PQ / LG : 1;
    static_assert(KL >= 2 && LG <= 8, "split layout");
    const int sS = scale_exp(meta[args.ts].maxbits);
    const int sO = scale_exp(meta[args.to].maxbits);
    const T *__restrict__ S = arena + args.s;
    const T *__restrict__ O = arena + args.o;
    T *__restrict__ C = arena + args.c;
    const int lane = (int)(threadIdx.x & (LG - 1));
    unsigned long long sP[P], oQ[Q];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        unsigned long long c = 0;
#pragma unroll
        for (int t = 0; t < NP; ++t) c |= (unsigned long long)((i >> t) & 1) << args.pbit[t];
        sP[i] = uniform64(apply_runs<STREAM2_RUNS>(c, args.srun, args.nsrun));
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        unsigned long long c = 0;
#pragma unroll
        for (int t = 0; t < NQ; ++t) c |= (unsigned long long)((j >> t) & 1) << args.qbit[t];
        oQ[j] = uniform64(apply_runs<STREAM2_RUNS>(c, args.orun, args.norun));
    }
    const int se = -(sS + sO);
    const unsigned long long groups = 1ull << (args.rc - NP - NQ);
    const unsigned G = gridDim.x;
    const unsigned lb = (G % 8u == 0u) ? (blockIdx.x % 8u) * (G / 8u) + blockIdx.x / 8u : blockIdx.x;
    double vmax = 0.0;
    // a group's lanes share u, so every lane of a group runs the same
    // iterations and the exchanges below stay inside active groups
    // work item u = uh * GPB + ul (tables for lane parts of log2 GPB bits)
    const unsigned ul = threadIdx.x / LG;
    const unsigned long long rl = tab.lr[0][ul & 15u] | tab.lr[1][(ul >> 4) & 15u];
    const unsigned long long sl = tab.ls[0][ul & 15u] | tab.ls[1][(ul >> 4) & 15u];
    const unsigned long long ol = tab.lo[0][ul & 15u] | tab.lo[1][(ul >> 4) & 15u];
    for (unsigned long long uh = lb; uh * GPB < groups; uh += G) {
        if (uh * GPB + ul >= groups) continue;
        unsigned long long r0 = rl, s0 = sl, o0 = ol;
#pragma unroll
        for (int c = 0; c < STREAM2_NCH; ++c)
            if (c < tab.nch) {
                const unsigned v = (unsigned)(uh >> (4 * c)) & 15u;
                r0 |= tab.hr[c][v];
                s0 |= tab.hs[c][v];
                o0 |= tab.ho[c][v];
            }
        double sv[P][KL], ov[Q][KL];
#pragma unroll
        for (int i = 0; i < P; ++i) load_chunk<T, KL>(S + (((s0 | sP[i]) << NK) + lane * KL), sv[i]);
#pragma unroll
        for (int j = 0; j < Q; ++j) load_chunk<T, KL>(O + (((o0 | oQ[j]) << NK) + lane * KL), ov[j]);
        double acc[PQ];
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                double a = 0.0;
#pragma unroll
                for (int k = 0; k < KL; ++k) a = fma(sv[i][k], ov[j][k], a);
                acc[i * Q + j] = a;
            }
        int fbase = 0, dup = 0;
        group_reduce_scatter<PQ, LG / 2>(acc, lane, fbase, dup);
        if ((lane & dup) == 0) {
#pragma unroll
            for (int t = 0; t < VF; ++t) {
                const int f = fbase + t;  // output index i * Q + j
                unsigned long long c = r0;
#pragma unroll
                for (int b = 0; b < NQ; ++b)
                    if ((f >> b) & 1) c |= 1ull << args.qbit[b];
#pragma unroll
                for (int b = 0; b < NP; ++b)
                    if ((f >> (NQ + b)) & 1) c |= 1ull << args.pbit[b];
                const T v = (T)ldexp(acc[t], se);
                store_nt(C + c, v);
                vmax = fmax(vmax, fabs((double)v));
            }
        }
    }
    publish_max_block(meta, args.tc, vmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) meta[args.tc].exp = meta[args.ts].exp + meta[args.to].exp + sS + sO;
}

// Elementwise and outer products (K = 1) with output bit 0 inside the
// thread: each thread owns the two neighbouring outputs r and r | 1 of every
// (p, q) of its P x Q tile, so S and O are read two entries at a time where
// bit 0 is theirs (operands store their bits in C's order, so it is their
// bit 0 too) and the outputs are stored in pairs (8 bytes in FP32, 16 in
// FP64).  Products and rounding are those of k_stream2.
template <typename T, int NP, int NQ>
__global__ void __launch_bounds__(256) k_stream2_vec(const Stream2Tab tab, T *__restrict__ arena, wmc_meta *meta,
                                                     const SliceGroup sg) {
    WMC_ENTER_SLICE(arena, meta, sg);
    const Stream2Args &args = tab.a;
    constexpr int P = 1 << NP, Q = 1 << NQ;
    const int sS = scale_exp(meta[args.ts].maxbits);
    const int sO = scale_exp(meta[args.to].maxbits);
    const T *__restrict__ S = arena + args.s;
    const T *__restrict__ O = arena + args.o;
    T *__restrict__ C = arena + args.c;
    // does output bit 0 belong to S, to O (either or both)
    const bool s0b = apply_runs<STREAM2_RUNS>(1ull, args.srun, args.nsrun) != 0;
    const bool o0b = apply_runs<STREAM2_RUNS>(1ull, args.orun, args.norun) != 0;
    unsigned long long cP[P], sP[P], cQ[Q], oQ[Q];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        unsigned long long c = 0;
#pragma unroll
        for (int t = 0; t < NP; ++t) c |= (unsigned long long)((i >> t) & 1) << args.pbit[t];
        cP[i] = uniform64(c);
        sP[i] = uniform64(apply_runs<STREAM2_RUNS>(c, args.srun, args.nsrun));
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        unsigned long long c = 0;
#pragma unroll
        for (int t = 0; t < NQ; ++t) c |= (unsigned long long)((j >> t) & 1) << args.qbit[t];
        cQ[j] = uniform64(c);
        oQ[j] = uniform64(apply_runs<STREAM2_RUNS>(c, args.orun, args.norun));
    }
    const int se = -(sS + sO);
    const unsigned long long threads = 1ull << (args.rc - 1 - NP - NQ);
    const unsigned G = gridDim.x;
    const unsigned lb = (G % 8u == 0u) ? (blockIdx.x % 8u) * (G / 8u) + blockIdx.x / 8u : blockIdx.x;
    double vmax = 0.0;
    const unsigned ul = threadIdx.x;
    const unsigned long long rl = tab.lr[0][ul & 15u] | tab.lr[1][(ul >> 4) & 15u];
    const unsigned long long sl = tab.ls[0][ul & 15u] | tab.ls[1][(ul >> 4) & 15u];
    const unsigned long long ol = tab.lo[0][ul & 15u] | tab.lo[1][(ul >> 4) & 15u];
    for (unsigned long long uh = lb; (uh << 8) < threads; uh += G) {
        if (((uh << 8) | ul) >= threads) continue;
        unsigned long long r0 = rl, s0 = sl, o0 = ol;  // r0: bit 0 clear
#pragma unroll
        for (int c = 0; c < STREAM2_NCH; ++c)
            if (c < tab.nch) {
                const unsigned v = (unsigned)(uh >> (4 * c)) & 15u;
                r0 |= tab.hr[c][v];
                s0 |= tab.hs[c][v];
                o0 |= tab.ho[c][v];
            }
        double sv[P][2], ov[Q][2];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const T *p = S + (s0 | sP[i]);
            if (s0b) {
                load_chunk<T, 2>(p, sv[i]);
            } else {
                sv[i][0] = (double)p[0];
                sv[i][1] = sv[i][0];
            }
        }
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const T *p = O + (o0 | oQ[j]);
            if (o0b) {
                load_chunk<T, 2>(p, ov[j]);
            } else {
                ov[j][0] = (double)p[0];
                ov[j][1] = ov[j][0];
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const T v0 = (T)ldexp(fma(sv[i][0], ov[j][0], 0.0), se);
                const T v1 = (T)ldexp(fma(sv[i][1], ov[j][1], 0.0), se);
                store_pair_nt(C + (r0 | cP[i] | cQ[j]), v0, v1);
                vmax = fmax(vmax, fmax(fabs((double)v0), fabs((double)v1)));
            }
    }
    publish_max_block(meta, args.tc, vmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) meta[args.tc].exp = meta[args.ts].exp + meta[args.to].exp + sS + sO;
}

// Arguments of the register-tiled streaming kernel for a single-node launch,
// if the node fits it (at most 2^5 summed entries, run lists that fit).
static inline bool stream2_args(const NodeDesc &d, Stream2Args *a, int max_each = 2, int min_thread_bits = 14,
                                int low = -1, bool vec = false) {
    if (d.rc < 2 || d.nk > 5) return false;
    vec = vec && d.nk == 0 && d.rc >= 8;
    auto bits_of = [&](const unsigned *runs, int nr, std::vector<int> &in) {
        int n = 0;
        for (int q = 0; q < nr; ++q) {
            const unsigned src = runs[q] & 255u, len = (runs[q] >> 8) & 255u;
            for (unsigned j = 0; j < len; ++j) in[(size_t)(src + j)] = 1;
            n += (int)len;
        }
        return n;
    };
    std::vector<int> inA((size_t)d.rc + 1, 0), inB((size_t)d.rc + 1, 0);
    const int na = bits_of(d.ra, d.nra, inA), nb = bits_of(d.rb, d.nrb, inB);
    const bool a_is_s = na >= nb;
    const std::vector<int> &inS = a_is_s ? inA : inB, &inO = a_is_s ? inB : inA;
    const int nsr = a_is_s ? d.nra : d.nrb, nor = a_is_s ? d.nrb : d.nra;
    if (nsr > STREAM2_RUNS || nor > STREAM2_RUNS) return false;
    std::memset(a, 0, sizeof *a);
    a->s = a_is_s ? d.a : d.b;
    a->o = a_is_s ? d.b : d.a;
    a->c = d.c;
    a->ts = a_is_s ? d.ta : d.tb;
    a->to = a_is_s ? d.tb : d.ta;
    a->tc = d.tc;
    a->rc = d.rc;
    for (int q = 0; q < nsr; ++q) a->srun[q] = a_is_s ? d.ra[q] : d.rb[q];
    for (int q = 0; q < nor; ++q) a->orun[q] = a_is_s ? d.rb[q] : d.ra[q];
    a->nsrun = nsr;
    a->norun = nor;
    a->ro = (a_is_s ? nb : na) + d.nk;
    // bits looped inside a thread: the highest S-only and O-only bits at or
    // above bit 4 (lower ones are reused from cache between neighbouring
    // lanes), while keeping at least 2^14 threads
    const int budget = std::max(0, std::min(2 * max_each, d.rc - min_thread_bits));
    int taken = 0;
    for (int p = d.rc - 1; p >= 4 && taken < budget; --p) {
        if (inS[(size_t)p] && !inO[(size_t)p] && a->np < max_each) {
            a->pbit[a->np++] = p;
            ++taken;
        } else if (inO[(size_t)p] && !inS[(size_t)p] && a->nq < max_each) {
            a->qbit[a->nq++] = p;
            ++taken;
        }
    }
    // remaining C bits, numbered by the thread index: the lowest `low` of
    // them in C order (a wave's lanes store consecutive outputs), then the
    // bits that only one operand has, then the rest.  Threads that share an
    // operand row then run close together in time, so the row comes from
    // HBM once and from the L2 cache for its other readers.
    std::vector<int> rest;
    for (int p = vec ? 1 : 0; p < d.rc; ++p) {
        bool used = false;
        for (int t = 0; t < a->np; ++t) used |= a->pbit[t] == p;
        for (int t = 0; t < a->nq; ++t) used |= a->qbit[t] == p;
        if (!used) rest.push_back(p);
    }
    auto make_runs = [&](const std::vector<int> &order) {
        int nl = 0;
        for (size_t t = 0; t < order.size();) {
            size_t e = t + 1;
            while (e < order.size() && order[e] == order[e - 1] + 1) ++e;
            if (nl >= STREAM2_LRUNS) return -1;
            a->lrun[nl++] = WMC_RUN(t, e - t, order[t]);
            t = e;
        }
        return nl;
    };
    int nl = -1;
    if (low >= 0 && (int)rest.size() > low) {
        std::vector<int> order(rest.begin(), rest.begin() + low);
        for (size_t t = (size_t)low; t < rest.size(); ++t)
            if (inS[(size_t)rest[t]] != inO[(size_t)rest[t]]) order.push_back(rest[t]);
        for (size_t t = (size_t)low; t < rest.size(); ++t)
            if (inS[(size_t)rest[t]] == inO[(size_t)rest[t]]) order.push_back(rest[t]);
        nl = make_runs(order);
    }
    if (nl < 0) nl = make_runs(rest);
    if (nl < 0) return false;
    a->nlrun = nl;
    a->o_lds = (1 << a->ro) <= STREAM2_O_LDS && d.rc >= 16 && !vec;
    a->vec = vec ? 1 : 0;
    return true;
}

// Long summed index on the matrix cores.  For a node with K >= 16 the
// outputs sharing a batch value form a small matrix product
//   C[beta, mu, nu] = sum_k A[beta, mu, k] B[beta, nu, k],
// so a wave computes a 16 x 16 block of it (4 mu bits as rows, 4 nu bits
// as columns, fewer when the node has fewer: rows then repeat) with K/4
// MFMA steps, loading 16 rows of A and 16 of B once for 256 outputs, where
// the register-tiled kernels load P + Q rows for P x Q outputs.  Lane l
// holds summed entries [g K/4, (g+1) K/4) of its row and column (g = l/16)
// and step s multiplies entry g K/4 + s, so the steps together cover every
// k once.  A workgroup covers every combination of a set T of output bits:
// the row and column bits, and batch bits so that T holds C's four lowest
// bits (up to 16 blocks, one or more per wave).  The blocks go to LDS and
// are written out in C order, so every store covers whole 128-byte
// segments.  The remaining output bits number the workgroup tiles,
// one-operand bits first, so tiles sharing operand rows run together.
#define SMFMA_MAX_T 12
#define SMFMA_NCH 7  // 4-bit chunks of the tile index (tiles < 2^28)

struct StreamMfmaArgs {
    long long a, b, c;                 // element offsets: row operand, column operand, C
    int ta, tb, tc;                    // meta entries
    int rc;                            // output rank
    int nt;                            // |T|
    int nrb, ncb, nbt;                 // row, column and block (batch) bits in T
    int rbit[4], cbit[4], tbit[4];     // their C positions
    int tpos[SMFMA_MAX_T];             // T ascending by C position
    int tdst[SMFMA_MAX_T];             // bit of the LDS index (block << 8 | row << 4 | column) it feeds
    int nwrun, nwarun, nwbrun, nar, nbr;
    unsigned wrun[STREAM2_LRUNS];      // tile index -> C bits outside T
    unsigned warun[STREAM2_LRUNS];     // tile index -> A row bits
    unsigned wbrun[STREAM2_LRUNS];     // tile index -> B row bits
    unsigned arun[STREAM2_RUNS];       // C address -> A row
    unsigned brun[STREAM2_RUNS];       // C address -> B row
    // the three tile-index maps by 4-bit chunk: map(wt) = OR over chunks c of
    // tab[c][(wt >> 4c) & 15] (each map deposits disjoint bits, so it is
    // linear in the chunks); the tile index is uniform in a workgroup, so a
    // lookup is one scalar load from the kernel arguments
    int nch;
    unsigned long long tabc[SMFMA_NCH][16];  // C bits outside T
    unsigned long long taba[SMFMA_NCH][16];  // A row bits
    unsigned long long tabb[SMFMA_NCH][16];  // B row bits
    // a lane's row (column) inside a block and a block's batch value, as
    // operand row bits: A rows by lane l % 16, B rows by lane, and both by block
    unsigned long long lane_a[16], lane_b[16], blk_a[16], blk_b[16];
};

// N consecutive entries of a row in the storage type (N a multiple of 4).
template <typename T, int N>
__device__ __forceinline__ void load_row(const T *__restrict__ p, T *v) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int h = 0; h < N / 2; ++h) {
            const double2 x = ((const double2 *)p)[h];
            v[2 * h] = x.x;
            v[2 * h + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int h = 0; h < N / 4; ++h) {
            const float4 x = ((const float4 *)p)[h];
            v[4 * h] = x.x;
            v[4 * h + 1] = x.y;
            v[4 * h + 2] = x.z;
            v[4 * h + 3] = x.w;
        }
    }
}


template <typename T, int NK>
__global__ void __launch_bounds__(256) k_stream_mfma(const StreamMfmaArgs args, T *__restrict__ arena,
                                                     wmc_meta *meta, const SliceGroup sg) {
    WMC_ENTER_SLICE(arena, meta, sg);
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int K = 1 << NK, KG = K / 4;
    constexpr int NBW = NK == 4 ? 4 : 2;  // blocks per wave (at most 16 / 8 per tile)
    __shared__ T tile[16 * 256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, l16 = lane & 15;
    const int sA = scale_exp(meta[args.ta].maxbits);
    const int sB = scale_exp(meta[args.tb].maxbits);
    const int se = -(sA + sB);
    const T *__restrict__ A = arena + args.a;
    const T *__restrict__ B = arena + args.b;
    T *__restrict__ C = arena + args.c;
    // this lane's row and column inside a block, as operand row offsets
    const unsigned long long aR = args.lane_a[l16];
    const unsigned long long bC = args.lane_b[l16];
    // write-out: element e of the tile (T bits ascending) sits at LDS index
    // lds(e) and C offset off(e).  T's lowest bits are C bits 0 and 1, so
    // elements of one group of V (2 for FP64, 4 for FP32: 16 bytes either
    // way) are neighbours in C: a thread stores such a group with one
    // instruction; the next 8 bits of e are this thread's
    constexpr int VB = sizeof(T) == 8 ? 1 : 2;  // in-thread bits of e
    unsigned lds_lo = 0;
    unsigned long long off_lo = 0;
    for (int q = VB; q < args.nt && q < VB + 8; ++q)
        if ((threadIdx.x >> (q - VB)) & 1) {
            lds_lo |= 1u << args.tdst[q];
            off_lo |= 1ull << args.tpos[q];
        }
    const unsigned lds_pair = 1u << args.tdst[0];
    const unsigned lds_b1 = VB == 2 ? 1u << args.tdst[1] : 0u;
    const int nblk = 1 << args.nbt;
    const int mine = nblk > wave ? (nblk - wave + 3) / 4 : 0;  // blocks wave, wave + 4, ...
    // this wave's blocks: their C bits and operand row bits (uniform)
    unsigned long long ablk[NBW], bblk[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
        const int bt = (wave + 4 * i) & 15;
        ablk[i] = uniform64(args.blk_a[bt]);
        bblk[i] = uniform64(args.blk_b[bt]);
    }
    // T bits VB + 8 .. 11 of the write-out index (uniform per iteration)
    unsigned hdst[3];
    unsigned long long hoff[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        hdst[q] = VB + 8 + q < args.nt ? 1u << args.tdst[VB + 8 + q] : 0u;
        hoff[q] = VB + 8 + q < args.nt ? 1ull << args.tpos[VB + 8 + q] : 0ull;
    }
    // columns are stored XOR-ed with row and block (fewer bank conflicts
    // whichever of them the lanes walk): slot at(l).  at is linear over XOR
    // (shifts, XORs and a mask), and the write-out index bits are disjoint,
    // so at(x | y) = at(x) ^ at(y): the slots come from per-bit constants
    auto at = [](unsigned l) { return l ^ (((l >> 4) ^ (l >> 8)) & 15u); };
    const unsigned at_lo = at(lds_lo), at_pair = at(lds_pair), at_b1 = at(lds_b1);
    unsigned at_h[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) at_h[q] = at(hdst[q]);
    const unsigned npair = 1u << (args.nt - VB);  // groups of V elements
    const unsigned nit = npair > 256u ? npair >> 8 : 1u;
    const unsigned long long tiles = 1ull << (args.rc - args.nt);
    const unsigned G = gridDim.x;
    const unsigned lb = (G % 8u == 0u) ? (blockIdx.x % 8u) * (G / 8u) + blockIdx.x / 8u : blockIdx.x;
    T av[NBW][KG], bv[NBW][KG];
    // operands of tile wt, issued one tile ahead so that their latency
    // overlaps the previous tile's write-out
    auto tile_map = [&](unsigned long long wt, const unsigned long long (*tab)[16]) {
        unsigned long long r = 0;
#pragma unroll
        for (int c = 0; c < SMFMA_NCH; ++c)
            if (c < args.nch) r |= tab[c][(unsigned)(wt >> (4 * c)) & 15u];
        return r;
    };
    auto load_tile = [&](unsigned long long wt) {
        const unsigned long long ab = tile_map(wt, args.taba);
        const unsigned long long bb = tile_map(wt, args.tabb);
#pragma unroll
        for (int i = 0; i < NBW; ++i)
            if (i < mine) {
                load_row<T, KG>(A + ((((ab | ablk[i]) | aR) << NK) + g * KG), av[i]);
                load_row<T, KG>(B + ((((bb | bblk[i]) | bC) << NK) + g * KG), bv[i]);
            }
    };
    double vmax = 0.0;
    if (lb < tiles) load_tile(lb);
    for (unsigned long long wt = lb; wt < tiles; wt += G) {
        const unsigned long long base = tile_map(wt, args.tabc);
#pragma unroll
        for (int i = 0; i < NBW; ++i)
            if (i < mine) {
                const int bt = wave + 4 * i;
                acc_t acc = {};
#pragma unroll
                for (int st = 0; st < KG; ++st) acc = Mfma<T>::step(av[i][st], bv[i][st], acc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = Mfma<T>::out_row(g, v);
                    tile[(bt << 8) | (m << 4) | (l16 ^ m ^ bt)] = acc[v];
                }
            }
        if (wt + G < tiles) load_tile(wt + G);
        __syncthreads();
        for (unsigned it = 0; it < nit; ++it) {
            // LDS slot of the group's first element: at(lds_lo | bits of it),
            // one XOR per bit with the tile-invariant slots above
            unsigned a0 = at_lo;
            unsigned long long off = base | off_lo;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if ((it >> q) & 1u) {
                    a0 ^= at_h[q];
                    off |= hoff[q];
                }
            if (threadIdx.x < npair) {
                if constexpr (VB == 1) {
                    const T v0 = (T)ldexp((double)tile[a0], se);
                    const T v1 = (T)ldexp((double)tile[a0 ^ at_pair], se);
                    store_pair_nt(C + off, v0, v1);
                    vmax = fmax(vmax, fmax(fabs((double)v0), fabs((double)v1)));
                } else {
                    const T v0 = (T)ldexp((double)tile[a0], se);
                    const T v1 = (T)ldexp((double)tile[a0 ^ at_pair], se);
                    const T v2 = (T)ldexp((double)tile[a0 ^ at_b1], se);
                    const T v3 = (T)ldexp((double)tile[a0 ^ at_pair ^ at_b1], se);
                    store_quad_nt(C + off, v0, v1, v2, v3);
                    vmax = fmax(vmax, fmax(fmax(fabs((double)v0), fabs((double)v1)),
                                           fmax(fabs((double)v2), fabs((double)v3))));
                }
            }
        }
        __syncthreads();
    }
    publish_max_block(meta, args.tc, vmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) meta[args.tc].exp = meta[args.ta].exp + meta[args.tb].exp + sA + sB;
}

// Arguments of k_stream_mfma for a node, if it fits (K of 16 or 32, at
// least min_bits row and column bits, run lists that fit).  Measured on the
// sliced banded formula (FP64 / FP32 solves/s): min_bits 2: 9.27 / 14.0,
// 3: 9.41 / 14.2, 4: 9.25 / 14.1; the register-tiled kernels alone: 7.83 /
// 13.4.  Nodes with fewer row or column bits keep the register-tiled path.
static inline bool stream_mfma_args(const NodeDesc &d, StreamMfmaArgs *a, int min_bits = 3) {
    if (d.nk < 4 || d.nk > 5 || d.rc < 8 || d.rc > 62) return false;
    if (d.nra > STREAM2_RUNS || d.nrb > STREAM2_RUNS) return false;
    std::vector<int> inA((size_t)d.rc, 0), inB((size_t)d.rc, 0);
    for (int q = 0; q < d.nra; ++q)
        for (unsigned j = 0; j < ((d.ra[q] >> 8) & 255u); ++j) inA[(size_t)((d.ra[q] & 255u) + j)] = 1;
    for (int q = 0; q < d.nrb; ++q)
        for (unsigned j = 0; j < ((d.rb[q] >> 8) & 255u); ++j) inB[(size_t)((d.rb[q] & 255u) + j)] = 1;
    int nmu = 0, nnu = 0;
    for (int p = 0; p < d.rc; ++p) {
        nmu += inA[(size_t)p] && !inB[(size_t)p];
        nnu += inB[(size_t)p] && !inA[(size_t)p];
    }
    if (nmu < min_bits || nnu < min_bits) return false;
    std::memset(a, 0, sizeof *a);
    std::vector<int> inT((size_t)d.rc, 0);
    // rows and columns: the one-operand bits among C's four lowest first,
    // then the lowest others; block bits: the lowest batch bits, up to 16
    // blocks (8 for K = 32), so that a tile's fixed costs spread over up to
    // 4096 outputs
    for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < d.rc; ++p) {
            if (inT[(size_t)p] || (pass == 0) != (p < 4)) continue;
            if (inA[(size_t)p] && !inB[(size_t)p] && a->nrb < 4) {
                a->rbit[a->nrb++] = p;
                inT[(size_t)p] = 1;
            } else if (inB[(size_t)p] && !inA[(size_t)p] && a->ncb < 4) {
                a->cbit[a->ncb++] = p;
                inT[(size_t)p] = 1;
            } else if (inA[(size_t)p] && inB[(size_t)p] && a->nbt < (d.nk == 4 ? 4 : 3)) {
                a->tbit[a->nbt++] = p;
                inT[(size_t)p] = 1;
            }
        }
    for (int p = 0; p < 4 && p < d.rc; ++p)
        if (!inT[(size_t)p]) return false;
    for (int p = 0; p < d.rc; ++p)
        if (inT[(size_t)p]) {
            int dst = -1;
            for (int t = 0; t < a->nrb; ++t) if (a->rbit[t] == p) dst = 4 + t;
            for (int t = 0; t < a->ncb; ++t) if (a->cbit[t] == p) dst = t;
            for (int t = 0; t < a->nbt; ++t) if (a->tbit[t] == p) dst = 8 + t;
            a->tpos[a->nt] = p;
            a->tdst[a->nt] = dst;
            ++a->nt;
        }
    // tile index -> the other C bits: one-operand bits first, then batch
    std::vector<int> order;
    for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < d.rc; ++p)
            if (!inT[(size_t)p] && ((inA[(size_t)p] != inB[(size_t)p]) == (pass == 0))) order.push_back(p);
    int nw = 0;
    for (size_t t = 0; t < order.size();) {
        size_t e = t + 1;
        while (e < order.size() && order[e] == order[e - 1] + 1) ++e;
        if (nw >= STREAM2_LRUNS) return false;
        a->wrun[nw++] = WMC_RUN(t, e - t, order[t]);
        t = e;
    }
    a->nwrun = nw;
    // the same tile bits as operand row bits, through the operands' run lists
    auto compose = [&](const unsigned *oruns, int nor, unsigned *runs, int *nruns) {
        auto row_bit = [&](int p) {
            for (int q = 0; q < nor; ++q) {
                const int src = (int)(oruns[q] & 255u), len = (int)((oruns[q] >> 8) & 255u);
                if (p >= src && p < src + len) return (int)(oruns[q] >> 16) + (p - src);
            }
            return -1;
        };
        int n = 0;
        for (size_t t = 0; t < order.size();) {
            const int r0 = row_bit(order[t]);
            if (r0 < 0) {
                ++t;
                continue;
            }
            size_t e = t + 1;
            while (e < order.size() && row_bit(order[e]) == r0 + (int)(e - t)) ++e;
            if (n >= STREAM2_LRUNS) return false;
            runs[n++] = WMC_RUN(t, e - t, r0);
            t = e;
        }
        *nruns = n;
        return true;
    };
    if (!compose(d.ra, d.nra, a->warun, &a->nwarun) || !compose(d.rb, d.nrb, a->wbrun, &a->nwbrun)) return false;
    a->a = d.a;
    a->b = d.b;
    a->c = d.c;
    a->ta = d.ta;
    a->tb = d.tb;
    a->tc = d.tc;
    a->rc = d.rc;
    a->nar = d.nra;
    a->nbr = d.nrb;
    for (int q = 0; q < d.nra; ++q) a->arun[q] = d.ra[q];
    for (int q = 0; q < d.nrb; ++q) a->brun[q] = d.rb[q];
    // chunk tables of the tile-index maps
    const int nbits = d.rc - a->nt;
    a->nch = (nbits + 3) / 4;
    if (a->nch > SMFMA_NCH) return false;
    auto host_runs = [](unsigned long long r, const unsigned *runs, int n) {
        unsigned long long out = 0;
        for (int i = 0; i < n; ++i)
            out |= ((r >> (runs[i] & 255u)) & ((1ull << ((runs[i] >> 8) & 255u)) - 1ull)) << (runs[i] >> 16);
        return out;
    };
    for (int c = 0; c < a->nch; ++c)
        for (unsigned v = 0; v < 16; ++v) {
            const unsigned long long w = (unsigned long long)v << (4 * c);
            a->tabc[c][v] = host_runs(w, a->wrun, a->nwrun);
            a->taba[c][v] = host_runs(w, a->warun, a->nwarun);
            a->tabb[c][v] = host_runs(w, a->wbrun, a->nwbrun);
        }
    for (unsigned v = 0; v < 16; ++v) {
        unsigned long long rowc = 0, colc = 0, cb = 0;
        for (int t = 0; t < a->nrb; ++t)
            if ((v >> t) & 1) rowc |= 1ull << a->rbit[t];
        for (int t = 0; t < a->ncb; ++t)
            if ((v >> t) & 1) colc |= 1ull << a->cbit[t];
        for (int t = 0; t < a->nbt; ++t)
            if ((v >> t) & 1) cb |= 1ull << a->tbit[t];
        a->lane_a[v] = host_runs(rowc, a->arun, a->nar);
        a->lane_b[v] = host_runs(colc, a->brun, a->nbr);
        a->blk_a[v] = host_runs(cb, a->arun, a->nar);
        a->blk_b[v] = host_runs(cb, a->brun, a->nbr);
    }
    return true;
}

template <typename T>
static void launch_stream_mfma(const StreamMfmaArgs &a, int nk, T *arena, wmc_meta *meta, hipStream_t st,
                               unsigned cap = 2048, const SliceGroup sg = SliceGroup{0, 0, 0}, unsigned nz = 1) {
    const unsigned long long tiles = 1ull << (a.rc - a.nt);
    // the cap holds for the whole launch: nz slices share it
    const unsigned long long cz = cap / nz < 64 ? 64 : cap / nz;
    unsigned long long blocks = tiles < cz ? tiles : cz;
    if (blocks >= 64) blocks &= ~7ull;  // whole XCD rounds
    const dim3 g((unsigned)blocks, 1, nz), b(256);
    if (nk == 4) hipLaunchKernelGGL((k_stream_mfma<T, 4>), g, b, 0, st, a, arena, meta, sg);
    else hipLaunchKernelGGL((k_stream_mfma<T, 5>), g, b, 0, st, a, arena, meta, sg);
}

// Returns false (nothing launched) if no instance covers the arguments.
template <typename T>
static bool launch_stream2(const Stream2Tab &tb, int nk, T *arena, wmc_meta *meta, hipStream_t st, int lg = 0,
                           const SliceGroup sg = SliceGroup{0, 0, 0}, unsigned nz = 1, unsigned grid_cap = 0) {
    const Stream2Args &sa = tb.a;
    const unsigned long long threads =
        (1ull << (sa.rc - sa.np - sa.nq - (sa.vec ? 1 : 0))) * (unsigned long long)(lg > 0 ? lg : 1);
    unsigned long long blocks = (threads + 255) / 256;
    // grid cap (measured on the sliced banded formula): FP32 runs fastest
    // with about one resident round of workgroups looping over the outputs,
    // FP64 with a few rounds
    // (the cap holds for the whole launch: nz slices share it)
    unsigned long long cap = (grid_cap ? grid_cap : (sizeof(T) == 4 ? 768u : 4096u)) / nz;
    if (cap < 64) cap = 64;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (blocks >= 64) blocks = (blocks + 7) & ~7ull;  // whole XCD rounds; threads past the end idle
    // stage O in LDS only where each workgroup reuses it at least 16 times
    // over; smaller reuse is served by the caches without the staging pass
    Stream2Tab t = tb;
    Stream2Args &a = t.a;
    const unsigned long long outs_per_wg = (1ull << sa.rc) / blocks;
    if (a.o_lds && outs_per_wg < (16ull << sa.ro)) a.o_lds = 0;
    const size_t lds = a.o_lds ? sizeof(double) << a.ro : 0;
    const dim3 g((unsigned)blocks, 1, nz), b(256);
    if (a.vec) {
        if (nk != 0) return false;
#define WMC_S2V(NPV, NQV)                                                                     \
    if (a.np == NPV && a.nq == NQV) {                                                          \
        hipLaunchKernelGGL((k_stream2_vec<T, NPV, NQV>), g, b, 0, st, t, arena, meta, sg);    \
        return true;                                                                           \
    }
        WMC_S2V(0, 0) WMC_S2V(0, 1) WMC_S2V(0, 2) WMC_S2V(1, 0) WMC_S2V(1, 1) WMC_S2V(1, 2) WMC_S2V(2, 0)
        WMC_S2V(2, 1) WMC_S2V(2, 2)
#undef WMC_S2V
        return false;
    }
    if constexpr (sizeof(T) == 8) {
        if (lg > 0) {
#define WMC_S2X(NKV, LGV, NPV, NQV)                                                                    \
    if (nk == NKV && lg == LGV && a.np == NPV && a.nq == NQV) {                                        \
        hipLaunchKernelGGL((k_stream2_split<T, NKV, NPV, NQV, LGV>), g, b, 0, st, t, arena, meta, sg);  \
        return true;                                                                                   \
    }
#define WMC_S2X_PQ(NKV, LGV)                                                                          \
    WMC_S2X(NKV, LGV, 0, 0) WMC_S2X(NKV, LGV, 0, 1) WMC_S2X(NKV, LGV, 0, 2) WMC_S2X(NKV, LGV, 1, 0)   \
    WMC_S2X(NKV, LGV, 1, 1) WMC_S2X(NKV, LGV, 1, 2) WMC_S2X(NKV, LGV, 2, 0) WMC_S2X(NKV, LGV, 2, 1)   \
    WMC_S2X(NKV, LGV, 2, 2)
            WMC_S2X_PQ(4, 4) WMC_S2X_PQ(5, 4)
#undef WMC_S2X_PQ
#undef WMC_S2X
            return false;
        }
    }
#define WMC_S2(NKV, NPV, NQV)                                                                  \
    if (nk == NKV && a.np == NPV && a.nq == NQV) {                                             \
        hipLaunchKernelGGL((k_stream2<T, NKV, NPV, NQV>), g, b, lds, st, t, arena, meta, sg);  \
        return true;                                                                           \
    }
#define WMC_S2_PQ(NKV)                                                                         \
    WMC_S2(NKV, 0, 0) WMC_S2(NKV, 0, 1) WMC_S2(NKV, 0, 2) WMC_S2(NKV, 1, 0) WMC_S2(NKV, 1, 1) \
    WMC_S2(NKV, 1, 2) WMC_S2(NKV, 2, 0) WMC_S2(NKV, 2, 1) WMC_S2(NKV, 2, 2)
    WMC_S2_PQ(0) WMC_S2_PQ(1) WMC_S2_PQ(2) WMC_S2_PQ(3) WMC_S2_PQ(4) WMC_S2_PQ(5)
#undef WMC_S2_PQ
#undef WMC_S2
    return false;
}

// Many streaming nodes in one launch (the merged steps of batches and
// serving), on the register-tiled scheme of k_stream2 with a fixed 2 x 2
// tile: each thread loads two rows of S and two of O and writes the four
// outputs.  A node without an S-only (or O-only) looped bit repeats its one
// row, so the duplicate outputs are the same value stored at the same
// address.  Task t owns workgroups [block_begin_t, block_begin_{t+1}); each
// workgroup covers STREAM2_MULTI_THREADS consecutive threads of its node.
// Tasks of one launch share NK.
#define STREAM2_MULTI_THREADS 1024
#define STREAM2_MULTI_LRUNS 4  // thread-index runs a merged-step task may use

struct StreamTask {
    Stream2Args a;
    long long block_begin;
};
static_assert(sizeof(Stream2Args) == 280, "Stream2Args layout");
static_assert(offsetof(Stream2Args, lrun) == 76 && offsetof(Stream2Args, srun) == 140 &&
                  offsetof(Stream2Args, orun) == 204 && offsetof(Stream2Args, ro) == 268, "Stream2Args layout");
static_assert(sizeof(StreamTask) == 288, "StreamTask layout");

// Workgroups of one task.
static inline unsigned long long stream_task_blocks(const Stream2Args &a) {
    const unsigned long long threads = 1ull << (a.rc - a.np - a.nq);
    return (threads + STREAM2_MULTI_THREADS - 1) / STREAM2_MULTI_THREADS;
}

template <typename T, int NK, typename TP = const StreamTask *>
__device__ __forceinline__ void stream_multi_body(TP tasks, int ntasks,
                                                  T *__restrict__ arena, wmc_meta *meta,
                                                  const int *__restrict__ block_task, unsigned blk) {
    constexpr int K = 1 << NK;
    constexpr int KC = K < 4 ? K : 4;
    int lo = 0;
    if (block_task) {
        lo = block_task[blk];  // one load instead of a dependent search
    } else {
        int hi = ntasks - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].block_begin <= (long long)blk) lo = mid; else hi = mid - 1;
        }
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const auto &args = tasks[lo].a;
    const unsigned long long lb = (unsigned long long)((long long)blk - tasks[lo].block_begin);
    const int sS = scale_exp(meta[args.ts].maxbits);
    const int sO = scale_exp(meta[args.to].maxbits);
    const int se = -(sS + sO);
    const T *__restrict__ S = arena + args.s;
    const T *__restrict__ O = arena + args.o;
    T *__restrict__ C = arena + args.c;
    unsigned long long cP[2] = {0, 0}, sP[2] = {0, 0}, cQ[2] = {0, 0}, oQ[2] = {0, 0};
    if (args.np) {
        cP[1] = uniform64(1ull << args.pbit[0]);
        sP[1] = uniform64(apply_runs<STREAM2_RUNS>(cP[1], args.srun, args.nsrun));
    }
    if (args.nq) {
        cQ[1] = uniform64(1ull << args.qbit[0]);
        oQ[1] = uniform64(apply_runs<STREAM2_RUNS>(cQ[1], args.orun, args.norun));
    }
    const unsigned long long threads = 1ull << (args.rc - args.np - args.nq);
    const unsigned long long u0 = lb * STREAM2_MULTI_THREADS;
    const unsigned long long u1 = u0 + STREAM2_MULTI_THREADS < threads ? u0 + STREAM2_MULTI_THREADS : threads;
    double vmax = 0.0;
    for (unsigned long long u = u0 + threadIdx.x; u < u1; u += 256) {
        const unsigned long long r0 = apply_runs<STREAM2_MULTI_LRUNS>(u, args.lrun, args.nlrun);
        const unsigned long long s0 = apply_runs<STREAM2_RUNS>(r0, args.srun, args.nsrun);
        const unsigned long long o0 = apply_runs<STREAM2_RUNS>(r0, args.orun, args.norun);
        double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
        for (int kc = 0; kc < K; kc += KC) {
            double sv[2][KC], ov[2][KC];
#pragma unroll
            for (int i = 0; i < 2; ++i) load_chunk<T, KC>(S + (((s0 | sP[i]) << NK) + kc), sv[i]);
#pragma unroll
            for (int j = 0; j < 2; ++j) load_chunk<T, KC>(O + (((o0 | oQ[j]) << NK) + kc), ov[j]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int k = 0; k < KC; ++k) acc[i][j] = fma(sv[i][k], ov[j][k], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const T v = (T)ldexp(acc[i][j], se);
                C[r0 | cP[i] | cQ[j]] = v;
                vmax = fmax(vmax, fabs((double)v));
            }
    }
    publish_max_block(meta, args.tc, vmax);
    if (lb == 0 && threadIdx.x == 0) meta[args.tc].exp = meta[args.ts].exp + meta[args.to].exp + sS + sO;
}

// One merged step of a batch or a server in a single launch: workgroups
// [0, sblocks) run the streaming tasks (their summed-index groups
// concatenated in nk order, group k starting at workgroup gblock[k] and task
// gtask[k]), the next nblocks the batched small nodes, the last lblocks the
// leaf fills of the instances at their first launch.  The parts are
// independent (each belongs to a different instance, or to different nodes
// of one launch), so one launch replaces up to six.
struct StepArgs {
    const StreamTask *tasks;
    const int *block_task;
    long long gblock[5];
    int gtask[5];
    unsigned sblocks;
    const NodeDesc *nodes;
    const int *wave_node;
    long long node_work;
    int nnodes;
    unsigned nblocks;
    const LeafDesc *leaves;
    const int *wave_leaf;
    const unsigned long long *leaf_eta;
    const double *w;
    long long leaf_work;
    int nleaves;
    unsigned lblocks;
};

// Workgroup bx of merged step a (every thread of the workgroup runs it).  A
// macro rather than a function, so that both kernels keep the descriptor
// reads on the scalar path: the compiler proves them unclobbered only in a
// kernel's own body.
#define WMC_STEP_BLOCK(T, a, bx, arena, meta)                                                                 \
    do {                                                                                                      \
        if ((bx) < (a).sblocks) {                                                                             \
            int k_ = 0;                                                                                       \
            while (k_ < 3 && (long long)(bx) >= (a).gblock[k_ + 1]) ++k_;                                     \
            const StreamTask *t_ = (a).tasks + (a).gtask[k_];                                                 \
            const int nt_ = (a).gtask[k_ + 1] - (a).gtask[k_];                                                \
            const int *bt_ = (a).block_task ? (a).block_task + (a).gblock[k_] : nullptr;                      \
            const unsigned blk_ = (bx) - (unsigned)(a).gblock[k_];                                            \
            switch (k_) {                                                                                     \
            case 0: stream_multi_body<T, 0>(t_, nt_, arena, meta, bt_, blk_); break;                          \
            case 1: stream_multi_body<T, 1>(t_, nt_, arena, meta, bt_, blk_); break;                          \
            case 2: stream_multi_body<T, 2>(t_, nt_, arena, meta, bt_, blk_); break;                          \
            default: stream_multi_body<T, 3>(t_, nt_, arena, meta, bt_, blk_); break;                         \
            }                                                                                                 \
        } else if ((bx) < (a).sblocks + (a).nblocks) {                                                        \
            nodes_body<T>((a).nodes, (a).nnodes, (a).node_work, arena, meta, (a).wave_node, (bx) - (a).sblocks, \
                          (a).nblocks);                                                                       \
        } else {                                                                                              \
            leaves_body<T>((a).leaves, (a).nleaves, (a).leaf_work, (a).w, arena, meta, 0ull, (a).wave_leaf,   \
                           (a).leaf_eta, (bx) - (a).sblocks - (a).nblocks, (a).lblocks);                      \
        }                                                                                                     \
    } while (0)

template <typename T>
__global__ void __launch_bounds__(256) k_step(const StepArgs a, T *__restrict__ arena, wmc_meta *meta) {
    WMC_STEP_BLOCK(T, a, blockIdx.x, arena, meta);
}

// Grid-wide barrier number n (1, 2, ...) of a launch whose counter bar[0]
// starts at zero and whose workgroups are all resident: every thread
// releases its writes at agent scope (all XCDs), one thread per workgroup
// counts the arrival and waits for n * gridDim.x of them, and every thread
// acquires before going on.  A wait longer than wait_ticks of the constant
// wall clock gives up and sets bar[1] (the host reports it as an error), and
// later barriers then wait no more, so that a broken launch ends instead of
// hanging.
__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned n, unsigned long long wait_ticks) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = n * gridDim.x;
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > wait_ticks) {
                    __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Persistent form: one cooperative launch walks every merged step of a
// batch.  A step's workgroups are dealt to the resident grid (workgroup b
// takes b, b + gridDim.x, ...), and a grid-wide barrier separates the steps,
// so step k + 1 reads what step k wrote.  Every workgroup runs every step
// and reaches every barrier; the work of a workgroup index is k_step's.  A
// block barrier follows each index, since a workgroup may take several.
template <typename T>
__global__ void __launch_bounds__(256) k_steps_persistent(const StepArgs *__restrict__ steps, int nsteps,
                                                          T *__restrict__ arena, wmc_meta *meta, unsigned *bar,
                                                          unsigned long long wait_ticks) {
    for (int k = 0; k < nsteps; ++k) {
        const StepArgs &a = steps[k];
        const unsigned total = a.sblocks + a.nblocks + a.lblocks;
        for (unsigned bx = blockIdx.x; bx < total; bx += gridDim.x) {
            WMC_STEP_BLOCK(T, a, bx, arena, meta);
            __syncthreads();  // the block's max reduction reuses its LDS slots
        }
        grid_barrier(bar, (unsigned)k + 1, wait_ticks);
    }
}

// Zeroes n words (the persistent launch's barrier counter and flag).
static __global__ __attribute__((unused)) void k_zero_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

static inline bool stream_task(const NodeDesc &d, StreamTask *t) {
    std::memset(t, 0, sizeof *t);
    // threads in C order: at most three runs around the two looped bits
    if (d.nk > 3 || !stream2_args(d, &t->a, 1, 10) || t->a.nlrun > STREAM2_MULTI_LRUNS) return false;
    t->a.o_lds = 0;
    return true;
}

// Workgroups of the task group [f, l): the group's grid size.
static inline unsigned long long stream_multi_blocks(const StreamTask *host_tasks, int f, int l) {
    if (f == l) return 0;
    const StreamTask &last = host_tasks[l - 1];
    return (unsigned long long)last.block_begin + stream_task_blocks(last.a);
}

// Lookup tables that replace the kernels' searches: the node of every wave
// of a small-node launch, and the task (relative to its nk group) of every
// workgroup of the streaming groups, groups concatenated in nk order.
static inline void wave_node_table(const std::vector<NodeDesc> &nodes, int64_t work, std::vector<int> &out) {
    out.assign((size_t)(work / WMC_WAVE), 0);
    for (size_t q = 0; q < nodes.size(); ++q) {
        const int64_t b = nodes[q].work_begin / WMC_WAVE;
        const int64_t e = b + (int64_t)(((1ull << nodes[q].rc) + WMC_WAVE - 1) / WMC_WAVE);
        for (int64_t w = b; w < e; ++w) out[(size_t)w] = (int)q;
    }
}

static inline void wave_leaf_table(const std::vector<LeafDesc> &leaves, int64_t work, std::vector<int> &out) {
    out.assign((size_t)(work / WMC_WAVE), 0);
    for (size_t q = 0; q < leaves.size(); ++q) {
        const int64_t b = leaves[q].work_begin / WMC_WAVE;
        const int64_t e = b + (int64_t)(((1ull << leaves[q].rank) + WMC_WAVE - 1) / WMC_WAVE);
        for (int64_t x = b; x < e; ++x) out[(size_t)x] = (int)q;
    }
}

static inline void block_task_table(const std::vector<StreamTask> &tasks, const std::vector<int> &nk_first,
                                    std::vector<int> &out) {
    out.clear();
    for (int k = 0; k < 4; ++k) {
        const int f = nk_first[(size_t)k], l = nk_first[(size_t)k + 1];
        for (int t = f; t < l; ++t) {
            const unsigned long long e = stream_multi_blocks(tasks.data(), f, t + 1);  // end of task t
            const unsigned long long b = (unsigned long long)tasks[(size_t)t].block_begin;
            for (unsigned long long x = b; x < e; ++x) out.push_back(t - f);
        }
    }
}

// Fill the streaming part of a fused step from the nk groups of its tasks
// (nk_first[k] .. nk_first[k+1] have nk == k; host copies give the sizes).
static inline void step_stream_part(StepArgs &a, const StreamTask *dev_tasks, const StreamTask *host_tasks,
                                    const int *nk_first, const int *dev_block_task) {
    a.tasks = dev_tasks;
    a.block_task = dev_block_task;
    unsigned long long blocks = 0;
    for (int k = 0; k < 4; ++k) {
        a.gblock[k] = (long long)blocks;
        a.gtask[k] = nk_first[k];
        blocks += stream_multi_blocks(host_tasks, nk_first[k], nk_first[k + 1]);
    }
    a.gblock[4] = (long long)blocks;
    a.gtask[4] = nk_first[4];
    a.sblocks = (unsigned)blocks;
}

template <typename T>
static void launch_step(const StepArgs &a, T *arena, wmc_meta *meta, hipStream_t st) {
    const unsigned g = a.sblocks + a.nblocks + a.lblocks;
    if (g) hipLaunchKernelGGL(k_step<T>, dim3(g), dim3(256), 0, st, a, arena, meta);
}

// Split a merged node list into (generic nodes, streaming tasks grouped by
// nk).  Nodes with at least 2^min_rank outputs that the streaming kernel
// accepts become tasks; work_begin of the generic ones is recomputed.
static inline void split_stream(std::vector<NodeDesc> &generic, std::vector<StreamTask> &tasks,
                                std::vector<int> &nk_first, int64_t &generic_work, int min_rank) {
    std::vector<NodeDesc> keep;
    std::vector<StreamTask> by_nk[4];
    generic_work = 0;
    for (const NodeDesc &d : generic) {
        StreamTask t;
        if (d.rc >= min_rank && d.cls != WMC_CLASS_GEMM && stream_task(d, &t)) {
            by_nk[d.nk].push_back(t);
            continue;
        }
        NodeDesc e = d;
        e.work_begin = generic_work;
        generic_work += (int64_t)(((1ull << e.rc) + WMC_WAVE - 1) / WMC_WAVE * WMC_WAVE);
        keep.push_back(e);
    }
    generic.swap(keep);
    tasks.clear();
    nk_first.assign(5, 0);
    for (int k = 0; k < 4; ++k) {
        nk_first[(size_t)k] = (int)tasks.size();
        long long blocks = 0;
        for (StreamTask &t : by_nk[k]) {
            t.block_begin = blocks;
            blocks += (long long)stream_task_blocks(t.a);
            tasks.push_back(t);
        }
    }
    nk_first[4] = (int)tasks.size();
}

// Roots of nz consecutive slices (slice z's arena and meta table astride
// elements and mstride entries after slice z-1's): fold each value, in
// slice order, into the running sum (s + c) * 2^e.
template <typename T>
__device__ void finish_one(const T *__restrict__ arena, long long root_off, const wmc_meta *meta, int root,
                           wmc_acc *acc);

template <typename T>
__global__ void k_finish(const T *__restrict__ arena, long long root_off, const wmc_meta *meta, int root,
                         wmc_acc *acc, int nz, long long astride, int mstride) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int z = 0; z < nz; ++z)
        finish_one<T>(arena + (long long)z * astride, root_off, meta + (long long)z * mstride, root, acc);
}

template <typename T>
__device__ void finish_one(const T *__restrict__ arena, long long root_off, const wmc_meta *meta, int root,
                           wmc_acc *acc) {
    double v = (double)arena[root_off];
    long long e = meta[root].exp;
    if (v != 0.0) {
        int k;
        v = frexp(v, &k);
        e += k;
    } else {
        e = 0;
    }
    acc->last_m = v;
    acc->last_e = e;
    if (v == 0.0) return;
    if (acc->s == 0.0 && acc->c == 0.0) {
        acc->s = v;
        acc->c = 0.0;
        acc->e = e;
    } else {
        if (e > acc->e) {
            long long d = acc->e - e;
            int di = d < -4000 ? -4000 : (int)d;
            acc->s = ldexp(acc->s, di);
            acc->c = ldexp(acc->c, di);
            acc->e = e;
        }
        long long d = e - acc->e;
        double t = ldexp(v, d < -4000 ? -4000 : (int)d);
        double s = acc->s + t;
        if (fabs(acc->s) >= fabs(t)) acc->c += (acc->s - s) + t;
        else acc->c += (t - s) + acc->s;
        acc->s = s;
        if (acc->s != 0.0) {
            int k;
            acc->s = frexp(acc->s, &k);
            acc->c = ldexp(acc->c, -k);
            acc->e += k;
        }
    }
    acc->n_added += 1;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline wmc_value make_value(double m, long long e) {
    wmc_value v;
    if (m == 0.0 || !std::isfinite(m)) {
        v.mantissa = m == 0.0 ? 0.0 : m;
        v.exp2 = 0;
        v.value = m;
        v.log2_abs = m == 0.0 ? -INFINITY : NAN;
        return v;
    }
    int k;
    double mm = std::frexp(m, &k);
    v.mantissa = mm;
    v.exp2 = e + k;
    long long ee = v.exp2;
    v.value = std::ldexp(mm, ee > 5000 ? 5000 : (ee < -5000 ? -5000 : (int)ee));
    v.log2_abs = std::log2(std::fabs(mm)) + (double)v.exp2;
    return v;
}

static inline unsigned grid_for(long long work) {
    long long b = (work + WMC_BLOCK - 1) / WMC_BLOCK;
    if (b < 1) b = 1;
    if (b > (1ll << 20)) b = 1ll << 20;
    return (unsigned)b;
}

#define HIP_TRY(call)                                                                     \
    do {                                                                                  \
        hipError_t _e = (call);                                                           \
        if (_e != hipSuccess) {                                                           \
            wmc_set_error("%s failed: %s", #call, hipGetErrorString(_e));                 \
            return WMC_ERR_DEVICE;                                                        \
        }                                                                                 \
    } while (0)

