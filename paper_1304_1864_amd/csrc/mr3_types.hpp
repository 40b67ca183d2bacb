// Data layout shared by the host driver and the kernels.
//
// Rows.  The inputs of all problems of one call are mapped to one internal
// "row space": problem p owns rows [row0, row0 + n).  Per-row arrays hold the
// scaled tridiagonal (binary64), the root representation of the block a row
// belongs to, and the off-diagonal products used to build eigenvectors.
//
// Blocks.  After splitting, every irreducible block is the root node of its
// own representation tree (Algorithm 1 runs per block).
//
// Slots.  One slot per eigenvalue index that the solve tracks: the requested
// indices of a block plus at most one neighbour on each side of the requested
// range ("helpers": their intervals give the gaps of the outermost requested
// eigenvalues; they are never written out).
//
// Nodes.  A node of a representation tree: a representation (its rows in the
// representation pool), the accumulated shift sigma, and a contiguous slot
// range.  Root nodes have the same index as their block.
#pragma once
#include <stdint.h>

namespace mr3 {

enum RangeKind { RANGE_ALL = 0, RANGE_VALUE = 1, RANGE_INDEX = 2 };

// slot classification results
enum SlotKind : int {
    KIND_NONE = 0,
    KIND_SINGLETON = 1,   // requested, well separated: RQI at this node
    KIND_HELPER = 2,      // helper singleton: nothing to compute
    KIND_CLUSTER_HEAD = 3,
    KIND_CLUSTER_MEMBER = 4,
    KIND_DROPPED = 5,     // run without requested members
};

struct ProbDesc {
    int64_t n;         // order of T
    const void* din;   // the caller's d and e (device, element type X)
    const void* ein;
    void* wout;        // the caller's W and Z (Z may be null: no vectors)
    void* zout;
    int64_t ldz;
    int64_t row0;      // first internal row
    int range;
    double vl, vu;
    int64_t il, iu;
};

struct ProbInfo {     // written by the preprocessing kernel
    int sexp;         // T_internal = 2^sexp * T_input
    int nblocks;
    int err;          // 1: non-finite entry
    int pad;
    double tnorm;     // ||T_internal||_1
};

struct BlockInfo {    // written by the preprocessing kernel, one per block
    int64_t start;    // first row within the problem
    int64_t n;
    int64_t il, iu;   // local requested index range (1-based); il > iu: none
    double gl, gu;    // Gerschgorin interval of the scaled block
};

struct Block {        // assembled by the host
    int prob;
    int64_t row0;     // internal row of the first row
    int64_t start;    // first row within the problem
    int64_t n;
    int64_t il, iu;
    double gl, gu;
    int64_t slot0;
    int64_t nslot;
};

struct Node {
    int block;
    int depth;
    int64_t rep;      // first row of its representation in the pool
    int64_t first, last;  // slot range
    double sigma_hi, sigma_lo;  // accumulated shift (y; lo = 0 for binary64 y)
    double spdiam;    // spectral diameter bound of the block (scaled)
};

struct Slot {
    int node;
    int kind;
    int64_t idx;      // local eigenvalue index within the block (1-based)
    int64_t out;      // output column within the problem; -1 helper
    double lo, hi;    // interval in the node frame (binary64)
    double lgap, rgap;  // absolute gaps to the neighbours (< 0: unknown)
    int64_t run_end;  // for cluster heads: last slot of the cluster
};

struct RqiResult {    // per singleton, consumed by the output kernel
    double lam_hi, lam_lo;  // eigenvalue of T_internal (y)
    double fT, fB;    // scale of the stored top / bottom parts
    double rowr;      // value at the twist row
    int64_t r;        // twist index (0-based row within the block)
    int64_t evT1, evT2;  // top storage rebasing events (see kernel)
    int64_t evB1, evB2;
    double evT2f, evB2f;  // factor for values between the last two events
    int iters;
    int status;       // 0 ok, 1 fallback used, 2 failure
};

struct Params {
    double gaptol;
    double gaptol_abs;
    double bisect_rel;
    double xi;
    double k_elg;
    double k_rs;
    double eps_x;
    double root_gap;      // mu stays root_gap * spdiam outside the spectrum
    int max_depth;
    int rqi_max_iter;
    int lanes_per_eig;
    int points_per_lane;
    int initial;          // MR3_INITIAL_*
    int force_rqi_fallback;
    int force_best_candidate;
    int profile;
    int refine_ends;      // cluster ends refined in y before the shift
    int force_resort;     // tests: outputs reversed before the order check
    int derive_lld;       // nodes keep d only; lld = e^2 / d formed where read
    long long debug_slot;  // development trace (MR3_DEBUG_SLOT), -1 = off
    unsigned long long seed;
};

}  // namespace mr3
