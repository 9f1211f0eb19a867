// Device-visible plan descriptors, written by the host planner and read by
// the HIP kernels.  Plain C structs, identical layout on host and device.
#pragma once
#include <stdint.h>

#define WMC_MAX_RUNS 20       // runs of a bit-extraction (pext) map
#define WMC_LEAF_VARS 24      // distinct variables of a clause leaf
#define WMC_WAVE 64

// Per-tensor bookkeeping in device memory.  The stored entries t of a tensor
// represent t * 2^exp; maxbits holds the IEEE bits of max |t| (non-negative
// doubles order like their bit patterns, so an integer atomicMax works).
struct wmc_meta {
    unsigned long long maxbits;
    long long exp;
};

// Running slice sum (s + c) * 2^e with Neumaier compensation c, plus the
// last slice's value (mantissa, exponent) for per-slice inspection.
struct wmc_acc {
    double s;
    double c;
    long long e;
    long long n_added;
    double last_m;
    long long last_e;
    long long pad[2];
};

// Leaf tensors: a clause indicator table B_C (restricted to the current
// slice) or the weight vector [W(x,0), W(x,1)] of a variable.
enum { WMC_LEAF_CLAUSE = 0, WMC_LEAF_WEIGHT = 1, WMC_LEAF_WEIGHT_CLOSED = 2 };

struct LeafDesc {
    long long out;        // element offset of the table in the arena
    long long work_begin; // first work item (entries padded to a wave multiple)
    int tensor;           // meta index
    int kind;             // WMC_LEAF_*
    int rank;             // storage rank after slicing
    int k;                // clause: distinct variables
    int var;              // weight leaves: variable index (0-based)
    unsigned falsify;     // clause: the one falsifying assignment over its variables
    int taut;             // clause holds x and not-x: all ones
    int pad;
    // clause variable i (weight leaf: slot 0): storage bit >= 0, or
    // -(1 + b) when the variable is sliced and takes bit b of the slice id
    short pos[WMC_LEAF_VARS];
};

// One pairwise contraction C[beta,mu,nu] = sum_kappa A[beta,mu,kappa] B[beta,kappa,nu].
// Every operand's storage layout is [kappa bits | its C-variables in C's
// storage order], so for an output address r:
//   addr_A(r, j) = (pext(r, maskA) << nk) | j,   j over the 2^nk kappa values,
// where pext is given as runs packed in one word each:
//   src bit in r | length << 8 | dst bit << 16.
#define WMC_RUN(src, len, dst) ((unsigned)(src) | ((unsigned)(len) << 8) | ((unsigned)(dst) << 16))
struct NodeDesc {
    long long a, b, c;        // element offsets in the arena
    long long work_begin;     // first work item of this node in its launch
    int ta, tb, tc;           // meta indices
    int rc;                   // storage rank of C
    int nk;                   // |kappa| (after slicing)
    int nra, nrb;             // number of runs in ra / rb
    int cls;                  // node class
    unsigned ra[WMC_MAX_RUNS];
    unsigned rb[WMC_MAX_RUNS];
};

// A contraction run as a batched matrix product on MFMA:
//   C[beta, mu, nu] = sum_kappa A[beta, mu, kappa] * B[beta, kappa, nu]
// with rows (beta, mu) of the larger operand A and columns (beta, nu) of B.
// Logical indices list their variables in C's storage order; each deposit
// run list maps a logical index onto storage bits (src bit, length, dst bit):
//   row of A = dep(mu, 0) | dep(beta, 1)   -> A + (row << nk) + kappa
//   col of B = dep(nu, 2) | dep(beta, 3)   -> B + (col << nk) + kappa
//   address in C = dep(mu, 4) | dep(nu, 5) | dep(beta, 6)
#define WMC_GEMM_RUNS 12
enum { GR_MU_A = 0, GR_BETA_A, GR_NU_B, GR_BETA_B, GR_MU_C, GR_NU_C, GR_BETA_C, GR_N };

struct GemmDesc {
    long long a, b, c;
    int ta, tb, tc;
    int nk, nm, nn, nb;
    int nrun[GR_N];
    unsigned char run[GR_N][WMC_GEMM_RUNS][3];
    int pad;
};

static_assert(sizeof(LeafDesc) == 96, "LeafDesc layout");
static_assert(sizeof(GemmDesc) == 336, "GemmDesc layout");
static_assert(sizeof(NodeDesc) == 224, "NodeDesc layout");
