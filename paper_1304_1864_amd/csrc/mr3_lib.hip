// Host driver and C ABI of the mixed-precision MRRR library.
//
// One call runs Algorithm 1 of the paper for every irreducible block of every
// problem in the call, level by level over the representation trees:
//   preprocess -> root representations -> bisection -> [classify -> RQI on
//   singletons + output | child shifts -> child bisection]* -> order check
// The host only reads back counts (blocks, singletons, clusters, tile sizes)
// to size the next launches; all arithmetic runs in the kernels.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/mr3.h"
#include "mr3_internal.h"
#include "mr3_kernels.hip"

namespace mr3 {

// --------------------------------------------------------------------------
// small device utilities used only by the driver
// --------------------------------------------------------------------------
// slots of one kind whose node lies in [node_lo, node_hi): the nodes of one
// level of one group of the tree walk
struct SelectKind {
    const Slot* slots;
    int kind;
    int64_t node_lo, node_hi;
    __host__ __device__ bool operator()(const int64_t& s) const {
        const Slot& sl = slots[s];
        return sl.kind == kind && sl.node >= node_lo && sl.node < node_hi;
    }
};

// Block records of every problem from the preprocessing output (one thread
// per problem; boff[p] = first block index of problem p), with the number of
// slots each block needs: the requested indices plus one helper on each side
// that has a neighbour (the helpers carry the gaps to eigenvalues outside the
// range).
__global__ void k_blocks(const ProbDesc* __restrict__ probs, const ProbInfo* __restrict__ pinfo,
                         const BlockInfo* __restrict__ binfo, const int64_t* __restrict__ boff,
                         int64_t count, Block* __restrict__ blocks, int64_t* __restrict__ nslot) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const ProbDesc pd = probs[p];
    const int nb = pinfo[p].nblocks;
    for (int b = 0; b < nb; ++b) {
        const BlockInfo x = binfo[pd.row0 + b];
        Block bk{};
        bk.prob = (int)p;
        bk.row0 = pd.row0 + x.start;
        bk.start = x.start;
        bk.n = x.n;
        bk.il = max((int64_t)1, x.il);
        bk.iu = min(x.n, x.iu);
        bk.gl = x.gl;
        bk.gu = x.gu;
        const int64_t ns = (bk.il <= bk.iu) ? (bk.iu - bk.il + 1) + (bk.il > 1) + (bk.iu < bk.n) : 0;
        blocks[boff[p] + b] = bk;
        nslot[boff[p] + b] = ns;
    }
}

// slot ranges of the blocks (exclusive sum of nslot in slot0)
__global__ void k_blocks_slots(Block* __restrict__ blocks, const int64_t* __restrict__ nslot,
                               const int64_t* __restrict__ slot0, int64_t nb) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    blocks[b].slot0 = slot0[b];
    blocks[b].nslot = nslot[b];
}

// the slots of block blockIdx.x: local index, output column (-1 helper, -2
// decided later for split problems), gap markers
__global__ void k_slots(const Block* __restrict__ blocks, const ProbInfo* __restrict__ pinfo,
                        Slot* __restrict__ slots) {
    const Block bk = blocks[blockIdx.x];
    if (bk.nslot == 0) return;
    const bool multi = pinfo[bk.prob].nblocks > 1;
    const int64_t lo_i = bk.il > 1 ? bk.il - 1 : bk.il;
    const int64_t hi_i = bk.iu < bk.n ? bk.iu + 1 : bk.iu;
    for (int64_t i = lo_i + threadIdx.x; i <= hi_i; i += blockDim.x) {
        Slot sl{};
        sl.idx = i;
        const bool req = (i >= bk.il && i <= bk.iu);
        sl.out = req ? (multi ? -2 : i - bk.il) : -1;
        sl.lgap = (i == lo_i) ? (i == 1 ? MR3_BIG : -1.0) : 0.0;
        sl.rgap = (i == hi_i) ? (i == bk.n ? MR3_BIG : -1.0) : 0.0;
        sl.kind = KIND_NONE;
        slots[bk.slot0 + (i - lo_i)] = sl;
    }
}

// sort key of a singleton: its node, then its relative gap in steps of 2^-3
// (smaller gaps need more RQI iterations; a wave runs until its slowest pair
// is done, so pairs of similar gaps share chunks)
__global__ void k_gap_keys(const int64_t* __restrict__ list, int64_t count,
                           const Slot* __restrict__ slots, unsigned long long* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const Slot sl = slots[list[i]];
    double lg = sl.lgap, rg = sl.rgap;
    if (!(lg > 0.0)) lg = MR3_BIG;
    if (!(rg > 0.0)) rg = MR3_BIG;
    const double scale = fmax(fmax(fabs(sl.lo), fabs(sl.hi)), 1e-300);
    const double rel = fmin(fmin(lg, rg) / scale, 1.0);
    const int bucket = min(255, max(0, (int)(-log2(rel) / 3.0)));
    keys[i] = ((unsigned long long)(unsigned)sl.node << 8) | (unsigned long long)bucket;
}

__global__ void k_iota(int64_t* __restrict__ v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) v[i] = i;
}

// Node-pure chunks of at most 32 singletons.  The singleton list is ordered by
// slot and every node owns a contiguous slot range, so each node's singletons
// form one run of the list; chunks split the runs at every 32nd entry.
__global__ void k_seg_marks(const int64_t* __restrict__ list, int64_t count,
                            const Slot* __restrict__ slots, int64_t* __restrict__ seg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    seg[i] = (i == 0 || slots[list[i]].node != slots[list[i - 1]].node) ? i : 0;
}

// seg[i] = first position of i's run (after a max-scan): chunk starts
__global__ void k_chunk_marks(const int64_t* __restrict__ seg, int64_t count,
                              int64_t* __restrict__ mark) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    mark[i] = ((i - seg[i]) % 32 == 0) ? 1 : 0;
}

// cid[i] = chunk of position i + 1 (after an inclusive sum of the marks)
__global__ void k_chunk_table(const int64_t* __restrict__ list, int64_t count,
                              const Slot* __restrict__ slots, const Node* __restrict__ nodes,
                              const Block* __restrict__ blocks, const int64_t* __restrict__ seg,
                              const int64_t* __restrict__ cid, ChunkInfo* __restrict__ chunks,
                              int64_t* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || (i - seg[i]) % 32 != 0) return;
    int c = 1;
    while (c < 32 && i + c < count && seg[i + c] == seg[i]) ++c;
    const int64_t k = cid[i] - 1;
    ChunkInfo ci;
    ci.begin = i;
    ci.count = c;
    ci.pad = 0;
    chunks[k] = ci;
    rows[k] = blocks[nodes[slots[list[i]].node].block].n * 32;
}

struct MaxOp {
    __host__ __device__ int64_t operator()(const int64_t& a, const int64_t& b) const {
        return a > b ? a : b;
    }
};

struct ClusterRec {
    int64_t head, last;
    int parent;
    int pad;
};

__global__ void k_cluster_recs(const int64_t* __restrict__ heads, int64_t count,
                               const Slot* __restrict__ slots, ClusterRec* __restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    const Slot s = slots[heads[c]];
    ClusterRec r;
    r.head = heads[c];
    r.last = s.run_end;
    r.parent = s.node;
    r.pad = 0;
    out[c] = r;
}

template <class X>
__global__ void k_check_sorted(const ProbDesc* __restrict__ probs, const int64_t* __restrict__ m,
                               int* __restrict__ bad, int count) {
    // one workgroup per problem; bad[p] is cleared by the caller
    const int p = blockIdx.x;
    if (p >= count) return;
    const X* w = reinterpret_cast<const X*>(probs[p].wout);
    int b = 0;
    for (int64_t i = 1 + threadIdx.x; i < m[p]; i += blockDim.x) b |= !(w[i - 1] <= w[i]);
    if (b) atomicOr(&bad[p], 1);
}

// fault injection: reverse the order of problem blockIdx.x's eigenpairs
template <class X>
__global__ void k_reverse_outputs(const ProbDesc* __restrict__ probs, const int64_t* __restrict__ m) {
    const ProbDesc pd = probs[blockIdx.x];
    const int64_t mp = m[blockIdx.x];
    X* w = reinterpret_cast<X*>(pd.wout);
    X* z = reinterpret_cast<X*>(pd.zout);
    for (int64_t i = threadIdx.x; i < mp / 2; i += blockDim.x) {
        const X t = w[i];
        w[i] = w[mp - 1 - i];
        w[mp - 1 - i] = t;
    }
    if (!z) return;
    for (int64_t i = 0; i < mp / 2; ++i)
        for (int64_t k = threadIdx.x; k < pd.n; k += blockDim.x) {
            const X t = z[i * pd.ldz + k];
            z[i * pd.ldz + k] = z[(mp - 1 - i) * pd.ldz + k];
            z[(mp - 1 - i) * pd.ldz + k] = t;
        }
}

template <class X>
__global__ void k_zero_cols(X* __restrict__ Z, int64_t ldz, int64_t n, int64_t m) {
    const int64_t total = n * m;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = t / n, row = t % n;
        Z[col * ldz + row] = (X)0;
    }
}

// --------------------------------------------------------------------------
// device buffers
// --------------------------------------------------------------------------
constexpr int64_t GUARD = 64;

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
    bool fixed = false;  // carved from a caller's work region: never grown or freed
    hipError_t ensure(size_t bytes, bool keep = false, hipStream_t st = 0) {
        if (bytes <= cap) return hipSuccess;
        if (fixed) return hipErrorOutOfMemory;  // the plan covers every request
        size_t nc = std::max(bytes, cap + cap / 2);
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, nc);
        if (e != hipSuccess) return e;
        if (keep && p && cap) {
            e = hipMemcpyAsync(q, p, cap, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) { (void)hipFree(q); return e; }
        }
        if (p) (void)hipFree(p);
        p = q;
        cap = nc;
        return hipSuccess;
    }
    template <class T> T* as() const { return reinterpret_cast<T*>(p); }
    // per-row arrays carry GUARD rows (of `width` elements) before and after
    // the data, so that the kernels' software prefetch may read a few rows
    // past either end of a representation without bounds arithmetic
    template <class T> T* rows(int64_t width = 1) const { return as<T>() + GUARD * width; }
    void release() {
        if (p && !fixed) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        fixed = false;
    }
};

// A caller's work region, handed out front to back in 256-byte aligned pieces.
struct Region {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    bool carve(Buf& b, size_t bytes) {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off > cap || bytes > cap - off) return false;
        b.p = base + off;
        b.cap = bytes;
        b.fixed = true;
        used = off + bytes;
        return true;
    }
};

// Pinned host staging for the driver's small transfers: copies from pinned
// memory are asynchronous (a pageable copy would wait for the stream), and the
// space handed out during a solve is not reused before the next solve, which
// starts only after the previous one has synchronised.
struct Staging {
    struct Chunk {
        void* p;
        size_t cap, used;
    };
    std::vector<Chunk> chunks;
    bool grow = true;  // false: a solve on a caller's work region allocates nothing
    void* get(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto& c : chunks)
            if (c.cap - c.used >= bytes) {
                void* r = static_cast<char*>(c.p) + c.used;
                c.used += bytes;
                return r;
            }
        if (!grow) return nullptr;  // the caller copies from pageable memory
        size_t cap = std::max<size_t>(bytes, (size_t)4 << 20);
        if (!chunks.empty()) cap = std::max(cap, 2 * chunks.back().cap);
        void* p = nullptr;
        if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
        chunks.push_back(Chunk{p, cap, bytes});
        return p;
    }
    void reset() {
        for (auto& c : chunks) c.used = 0;
    }
    void release() {
        for (auto& c : chunks) (void)hipHostFree(c.p);
        chunks.clear();
    }
};

enum BufId {
    B_PROBS, B_PINFO, B_TD, B_TE, B_BINFO, B_BLOCKS, B_SLOTS, B_NODES, B_REPD, B_REPL, B_REPE,
    B_D64, B_L64, B_P, B_PE, B_Q, B_QE, B_LIST, B_LIST2, B_CNT, B_TILEOFF, B_TILES, B_RES,
    B_FLAGS, B_CUBTMP, B_JOBS, B_TMPC, B_TMPE, B_M, B_BAD, B_COUNTERS,
    B_BOFF, B_CREC, B_CHECK, B_NSLOT, B_SLOT0, B_GKEY, B_GVAL, B_BWG, B_VLIST, B_VWG, B_SLICE, B_SLB, B_SEG, B_CMARK, B_CID, B_CHUNK0, B_CHUNK1, B_SLIST0, B_SLIST1, B_TILEOFF1, B_TILES1, B_RES1, B_DQDS, B_DQB, B_P64, B_Q64, B_NBUF
};

// singleton work of tree level d runs on the handle's side stream with the
// buffers of parity d & 1, so that it overlaps the cluster work of the same
// level (which only depends on the classification)
constexpr int B_SIDE_LIST[2] = {B_SLIST0, B_SLIST1};
constexpr int B_SIDE_TOFF[2] = {B_TILEOFF, B_TILEOFF1};
constexpr int B_SIDE_TILES[2] = {B_TILES, B_TILES1};
constexpr int B_SIDE_RES[2] = {B_RES, B_RES1};
constexpr int B_SIDE_CHUNK[2] = {B_CHUNK0, B_CHUNK1};

// nodes of at least this many rows are bisected by the LDS-staged kernel with
// node-pure workgroups; shorter ones (which stay in cache) by the per-lane one
constexpr int64_t STAGE_MIN_N = 2048;

// counters: 8 x u64 (RQI iterations, fallbacks, failures), 8 x double
// (algorithmic row steps), 8 x int (status)
constexpr size_t COUNTER_BYTES = sizeof(unsigned long long) * 8 + sizeof(double) * 8 + sizeof(int) * 8;

// status of a solve on a caller's work region that is too small (mapped to
// the position of the work_bytes argument by the entry points)
constexpr int ERR_WORK_SMALL = -100000;

// --------------------------------------------------------------------------
// Workspace plan: the size of every buffer of one call, from the call's
// shape.  A solve on a caller's work region carves all of them up front, so
// it never allocates; the handle's pool grows the same buffers on demand.
// --------------------------------------------------------------------------
struct Shape {
    int64_t count = 0;     // problems
    int64_t R = 0;         // rows of all problems
    int64_t NB = 0;        // irreducible blocks
    int64_t K = 0;         // slots: wanted eigenvalues plus helpers
    int64_t nmax = 0;      // rows of the largest block with wanted eigenvalues
    int max_depth = 6;
    bool dd = false;       // y = double-double
    bool dqds = false;
    bool lld = true;       // nodes store lld in y (false: formed from e and d)
    size_t xsize = 8;
    int64_t rep_rows = 0;  // representation stack: root rows plus child rows
    int64_t tile_rows = 0; // eigenvector tile rows per side-stream parity
};

// hipcub temporary storage of the scans, selects and radix sorts over at most
// c items: the sort's key and value copies, plus a fixed allowance for
// histograms and look-back state
static size_t cub_bound(int64_t c) { return (size_t)40 * (size_t)(c + 1) + ((size_t)4 << 20); }

// at most NB roots plus, per level below the depth cap, disjoint clusters of
// at least two slots each
static int64_t node_bound(const Shape& s) {
    return s.NB + (int64_t)std::max(1, s.max_depth) * s.K / 2 + 1;
}

// buffers sized before the blocks are known (from count and R only)
static const int PREP_BUFS[] = {B_PROBS, B_PINFO, B_TD, B_TE, B_BINFO, B_BOFF,
                                B_BLOCKS, B_NSLOT, B_SLOT0, B_CUBTMP};
static bool is_prep_buf(int b) {
    for (int q : PREP_BUFS)
        if (q == b) return true;
    return false;
}

static void prep_sizes(const Shape& s, size_t* sz) {
    const int64_t G2 = 2 * GUARD;
    sz[B_PROBS] = sizeof(ProbDesc) * std::max<int64_t>(s.count, 1);
    sz[B_PINFO] = sizeof(ProbInfo) * std::max<int64_t>(s.count, 1);
    sz[B_TD] = sz[B_TE] = sizeof(double) * (s.R + G2);
    sz[B_BINFO] = sizeof(BlockInfo) * std::max<int64_t>(s.R, 1);
    sz[B_BOFF] = sizeof(int64_t) * (s.count + 1);
    sz[B_BLOCKS] = sizeof(Block) * std::max<int64_t>(s.R, 1);  // at most one block per row
    sz[B_NSLOT] = sz[B_SLOT0] = sizeof(int64_t) * (s.R + 1);
    sz[B_CUBTMP] = cub_bound(s.R + 1) + 256;  // every scan, select and sort covers <= R + 1 items
}

static void solve_sizes(const Shape& s, size_t* sz) {
    const int64_t G2 = 2 * GUARD, K = std::max<int64_t>(s.K, 1);
    const int64_t NB = std::max<int64_t>(s.NB, 1), KN = std::max(K, NB);
    const size_t ys = s.dd ? 16 : 8;
    const int64_t tmp_rows = std::max<int64_t>(s.rep_rows - s.R, 1);
    sz[B_SLOTS] = sizeof(Slot) * K;
    sz[B_NODES] = sizeof(Node) * node_bound(s);
    sz[B_REPD] = ys * (s.rep_rows + G2);
    sz[B_REPL] = s.lld ? ys * (s.rep_rows + G2) : 0;
    sz[B_D64] = sz[B_L64] = sizeof(double) * (s.rep_rows + G2);
    sz[B_REPE] = ys * std::max<int64_t>(s.R, 1);
    sz[B_P] = sz[B_Q] = ys * (s.R + G2);
    sz[B_PE] = sz[B_QE] = sizeof(int) * (s.R + G2);
    sz[B_P64] = sz[B_Q64] = s.dd ? sizeof(double) * (s.R + G2) : 0;  // binary64 mantissas of P, Q
    sz[B_LIST] = sizeof(int64_t) * KN;  // level nodes, identity and bisection lists
    sz[B_LIST2] = sizeof(int64_t) * K;
    sz[B_CNT] = sizeof(int64_t) * 4;
    sz[B_FLAGS] = sizeof(int64_t) * (K + 1);  // flags per slot, then tile rows per chunk
    sz[B_COUNTERS] = COUNTER_BYTES;
    sz[B_BWG] = sizeof(BisWG) * KN;
    // slice counts: at most max(1024, 6k) + 4 per root of >= STAGE_MIN_N rows
    sz[B_SLICE] = sizeof(int) * (6 * K + 1028 * (s.R / STAGE_MIN_N + 1));
    sz[B_SLB] = sz[B_DQB] = sizeof(int) * NB;
    sz[B_DQDS] = s.dqds ? sizeof(double) * 6 * s.R : 0;
    for (int q = 0; q < 2; ++q) {
        sz[B_SIDE_LIST[q]] = sizeof(int64_t) * K;
        sz[B_SIDE_TOFF[q]] = sizeof(int64_t) * (K + 1);
        sz[B_SIDE_TILES[q]] = sizeof(double) * (std::max<int64_t>(s.tile_rows, 1) + 2 * 32 * GUARD);
        sz[B_SIDE_RES[q]] = sizeof(RqiResult) * K;
        sz[B_SIDE_CHUNK[q]] = sizeof(ChunkInfo) * K;
    }
    sz[B_GKEY] = sizeof(unsigned long long) * 2 * K;
    sz[B_GVAL] = sz[B_SEG] = sz[B_CMARK] = sz[B_CID] = sizeof(int64_t) * K;
    sz[B_CREC] = sizeof(ClusterRec) * K;
    sz[B_JOBS] = sizeof(ChildJob) * K;
    sz[B_TMPC] = ys * tmp_rows;
    sz[B_TMPE] = sizeof(int) * tmp_rows;
    sz[B_VLIST] = sizeof(int64_t) * K;
    sz[B_VWG] = sizeof(BisWG) * K;
    sz[B_M] = sizeof(int64_t) * std::max<int64_t>(s.count, 1);
    sz[B_BAD] = sizeof(int) * std::max<int64_t>(s.count, 1);
    sz[B_CHECK] = s.xsize * std::max<int64_t>(s.nmax, 1);
}

// bytes the buffers of one phase take in a region, with their alignment
static size_t phase_bytes(const size_t* sz, bool prep) {
    size_t t = 256;
    for (int b = 0; b < B_NBUF; ++b)
        if (is_prep_buf(b) == prep) t += (sz[b] + 255) & ~(size_t)255;
    return t;
}

// The least the tree walk can run with: the roots plus one child of the
// largest block per level, and the tiles of one chunk of 32 eigenvectors.
static int64_t min_rep_rows(const Shape& s) { return s.R + (int64_t)std::max(1, s.max_depth) * s.nmax; }
static int64_t min_tile_rows(const Shape& s) { return 32 * std::max<int64_t>(s.nmax, 1); }
// Full speed: up to 512 clusters of the largest block on each of two levels
// at once, and the tiles of a whole level in one round (tile_full: the sum
// over blocks of n (wanted + 32)).
static int64_t full_rep_rows(const Shape& s) {
    return std::max(min_rep_rows(s), s.R + 2 * std::min<int64_t>(s.K / 2, 512) * s.nmax);
}

// Representation-stack and tile capacity for a region of `avail` bytes after
// the preprocessing buffers: the minimum first, then both towards full speed
// in proportion, and any rest to the stack.  False if the minimum does not fit.
static bool plan_region(Shape& s, size_t avail, int64_t tile_full) {
    s.rep_rows = min_rep_rows(s);
    s.tile_rows = min_tile_rows(s);
    size_t sz[B_NBUF] = {0};
    solve_sizes(s, sz);
    const size_t base = phase_bytes(sz, false) + 256 * (size_t)B_NBUF;  // rounding slack
    if (base > avail) return false;
    size_t left = avail - base;
    const size_t ys = s.dd ? 16 : 8;
    const size_t per_tile = 2 * sizeof(double);  // both side-stream parities
    // d, lld (unless formed on the fly), scratch; binary64 copies
    const size_t per_rep = (s.lld ? 3 : 2) * ys + 2 * sizeof(double) + sizeof(int);
    const double want_t = (double)std::max<int64_t>(tile_full - s.tile_rows, 0) * per_tile;
    const double want_r = (double)(full_rep_rows(s) - s.rep_rows) * per_rep;
    const double f = (want_t + want_r <= (double)left) ? 1.0 : (double)left / (want_t + want_r);
    const int64_t t = (int64_t)(f * want_t / per_tile);
    s.tile_rows += t;
    left -= (size_t)t * per_tile;
    s.rep_rows += (int64_t)(left / per_rep);
    return true;
}

// Bytes a call of this shape needs at full speed (the workspace query).
static size_t full_bytes(Shape s, int64_t tile_full) {
    size_t sz[B_NBUF] = {0};
    prep_sizes(s, sz);
    s.rep_rows = full_rep_rows(s);
    s.tile_rows = std::max(min_tile_rows(s), tile_full);
    solve_sizes(s, sz);
    return 256 + phase_bytes(sz, true) + phase_bytes(sz, false) + 256 * (size_t)B_NBUF;
}

}  // namespace mr3

struct mr3_handle_s {
    int device = 0;
    mr3_params user{};
    bool have_user = false;
    mr3::Buf buf[mr3::B_NBUF];
    mr3_stats stats{};
    // side streams (default priority) for singleton work, one per level
    // parity, and their events
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_jobs = nullptr;  // marks the copy of a level's shift-choice outcomes
    hipEvent_t ev_side[2] = {nullptr, nullptr};
    bool side_pending[2] = {false, false};
    mr3::Staging stage;      // pinned host staging
    bool clean_exit = true;  // the last solve synchronised its stream
    void* scratch = nullptr; // device address of this device's no-allocation scratch
    std::vector<mr3_tune_entry> tune;  // measured multisection shapes
};

namespace mr3 {

#define HIPCHK(x)                                              \
    do {                                                       \
        hipError_t _e = (x);                                   \
        if (_e != hipSuccess) {                                \
            last_hip_error = _e;                               \
            return MR3_ERR_HIP;                                \
        }                                                      \
    } while (0)

static thread_local hipError_t last_hip_error = hipSuccess;

// MR3_DEBUG=1 in the environment prints per-level counts and host-side phase
// times to stderr (development aid; off by default)
static bool debug_on() {
    static const bool on = [] {
        const char* v = std::getenv("MR3_DEBUG");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}
static double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Per-stage device time: with params.profile set, every launch is bracketed by
// two HIP events recorded on the launch stream; the elapsed times are summed
// per stage once the solve has synchronised.
struct Prof {
    bool on = false;
    struct Ev {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Ev> evs;
    void begin(int stage, hipStream_t st) {
        if (!on) return;
        Ev e{stage, nullptr, nullptr};
        (void)hipEventCreate(&e.a);
        (void)hipEventCreate(&e.b);
        (void)hipEventRecord(e.a, st);
        evs.push_back(e);
    }
    void end(hipStream_t st) {
        if (!on || evs.empty()) return;
        (void)hipEventRecord(evs.back().b, st);
    }
    void collect(mr3_stats& s) {
        for (auto& e : evs) {
            float ms = 0.f;
            if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
                s.stage_ms[e.stage] += ms;
                s.stage_launches[e.stage] += 1;
            }
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        evs.clear();
    }
    ~Prof() {
        for (auto& e : evs) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    }
};

static void defaults(mr3_params* p, int precision) {
    std::memset(p, 0, sizeof(*p));
    p->gaptol = (precision == 32) ? 1e-5 : 1e-10;
    p->bisect_rel = 1e-2 * p->gaptol;
    p->xi = (precision == 32) ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
    p->k_elg = 10.0;
    p->k_rs = 1.0;
    p->max_depth = 6;
    p->rqi_max_iter = 10;
    p->lanes_per_eig = 0;
    p->seed = 0x5eedull;
}

static Params effective(const mr3_handle_s* h, int precision) {
    mr3_params d;
    defaults(&d, precision);
    const mr3_params& u = h->user;
    Params p;
    p.gaptol = (h->have_user && u.gaptol > 0) ? u.gaptol : d.gaptol;
    p.gaptol_abs = (h->have_user && u.gaptol_abs > 0) ? u.gaptol_abs : 0.0;
    p.bisect_rel = (h->have_user && u.bisect_rel > 0) ? u.bisect_rel : 1e-2 * p.gaptol;
    p.xi = (h->have_user && u.xi > 0) ? u.xi : d.xi;
    p.k_elg = (h->have_user && u.k_elg > 0) ? u.k_elg : d.k_elg;
    p.k_rs = (h->have_user && u.k_rs > 0) ? u.k_rs : d.k_rs;
    p.eps_x = (precision == 32) ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
    p.root_gap = 1e-3;
    p.max_depth = (h->have_user && u.max_depth > 0) ? u.max_depth : d.max_depth;
    p.rqi_max_iter = (h->have_user && u.rqi_max_iter > 0) ? u.rqi_max_iter : d.rqi_max_iter;
    p.lanes_per_eig = h->have_user ? u.lanes_per_eig : 0;
    p.points_per_lane = h->have_user ? u.points_per_lane : 0;
    p.initial = h->have_user ? u.initial : MR3_INITIAL_BISECTION;
    p.refine_ends = h->have_user ? u.refine_ends : 0;
    p.derive_lld = h->have_user ? u.derive_lld : 0;
    p.force_resort = h->have_user ? u.force_resort : 0;
    p.force_rqi_fallback = h->have_user ? u.force_rqi_fallback : 0;
    p.force_best_candidate = h->have_user ? u.force_best_candidate : 0;
    p.seed = (h->have_user && u.seed) ? u.seed : d.seed;
    p.profile = h->have_user ? u.profile : 0;
    p.debug_slot = std::getenv("MR3_DEBUG_SLOT") ? std::atoll(std::getenv("MR3_DEBUG_SLOT")) : -1;
    return p;
}

// staging arena of the solve running on this thread (set by solve_impl)
static thread_local Staging* g_stage = nullptr;

template <class T>
static hipError_t upload(Buf& b, const std::vector<T>& v, hipStream_t st) {
    hipError_t e = b.ensure(std::max<size_t>(1, v.size()) * sizeof(T));
    if (e != hipSuccess || v.empty()) return e;
    const size_t bytes = v.size() * sizeof(T);
    void* pin = g_stage ? g_stage->get(bytes) : nullptr;
    if (!pin) return hipMemcpyAsync(b.p, v.data(), bytes, hipMemcpyHostToDevice, st);
    std::memcpy(pin, v.data(), bytes);
    return hipMemcpyAsync(b.p, pin, bytes, hipMemcpyHostToDevice, st);
}

template <class T>
static hipError_t download(std::vector<T>& v, const void* src, size_t count, hipStream_t st) {
    v.resize(count);
    if (count == 0) return hipSuccess;
    const size_t bytes = count * sizeof(T);
    void* pin = g_stage ? g_stage->get(bytes) : nullptr;
    hipError_t e = hipMemcpyAsync(pin ? pin : v.data(), src, bytes, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e == hipSuccess && pin) std::memcpy(v.data(), pin, bytes);
    return e;
}

// several downloads behind one stream synchronisation (each host round trip
// costs tens of microseconds, much of a small solve); the vectors must stay
// unresized until finish()
struct DownloadBatch {
    struct Item {
        void* dst;
        const void* pin;
        size_t bytes;
    };
    hipStream_t st;
    std::vector<Item> items;
    explicit DownloadBatch(hipStream_t s) : st(s) {}
    template <class T>
    hipError_t add(std::vector<T>& v, const void* src, size_t count) {
        v.resize(count);
        if (count == 0) return hipSuccess;
        const size_t bytes = count * sizeof(T);
        void* pin = g_stage ? g_stage->get(bytes) : nullptr;
        if (pin) items.push_back(Item{v.data(), pin, bytes});
        return hipMemcpyAsync(pin ? pin : v.data(), src, bytes, hipMemcpyDeviceToHost, st);
    }
    hipError_t finish() {
        const hipError_t e = hipStreamSynchronize(st);
        if (e == hipSuccess)
            for (const Item& it : items) std::memcpy(it.dst, it.pin, it.bytes);
        items.clear();
        return e;
    }
};

// LDS taken by a multi-wave RQI workgroup, windows included
constexpr size_t RQI_CU_LDS = 159u * 1024u;

// multisection shape: L lanes per eigenvalue, P points per lane and pass
struct BisectShape {
    int L, P;
};

static void launch_bisect(BisectShape sh, const int64_t* list, int64_t count, Slot* slots,
                          const Node* nodes, const Block* blocks, const double* d64,
                          const double* l64, double rtol, double widen, double* work,
                          int64_t skip_n, hipStream_t st) {
    if (count <= 0) return;
    const int G = 256 / sh.L;
    const dim3 grid((unsigned)((count + G - 1) / G));
#define MR3_BIS(LL, PP)                                                                        \
    if (sh.L == LL && sh.P == PP) {                                                            \
        hipLaunchKernelGGL((k_bisect<LL, PP>), grid, dim3(256), 0, st, list, count, slots,     \
                           nodes, blocks, d64, l64, rtol, widen, work, skip_n);                \
        return;                                                                                \
    }
    MR3_BIS(1, 1) MR3_BIS(1, 2) MR3_BIS(1, 4)
    MR3_BIS(2, 1) MR3_BIS(2, 2) MR3_BIS(2, 4)
    MR3_BIS(4, 1) MR3_BIS(4, 2) MR3_BIS(4, 4)
    MR3_BIS(8, 1) MR3_BIS(8, 2) MR3_BIS(8, 4)
    MR3_BIS(16, 1) MR3_BIS(16, 2) MR3_BIS(16, 4)
    MR3_BIS(32, 1) MR3_BIS(32, 2) MR3_BIS(32, 4)
    MR3_BIS(64, 1) MR3_BIS(64, 2) MR3_BIS(64, 4)
#undef MR3_BIS
    hipLaunchKernelGGL((k_bisect<1, 4>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       list, count, slots, nodes, blocks, d64, l64, rtol, widen, work, skip_n);
}

static void launch_bisect_staged(BisectShape sh, const BisWG* wgs, int64_t nwg, const int64_t* list,
                                 Slot* slots, const Node* nodes, const Block* blocks,
                                 const double* d64, const double* l64, double rtol, double widen,
                                 double* work, int check, hipStream_t st, int waves = 4) {
    if (nwg <= 0) return;
#define MR3_BST(LL, PP)                                                                        \
    if (sh.L == LL && sh.P == PP) {                                                            \
        hipLaunchKernelGGL((k_bisect_staged<LL, PP>), dim3((unsigned)nwg), dim3(64 * waves), 0, st, \
                           wgs, list, slots, nodes, blocks, d64, l64, rtol, widen, work, check); \
        return;                                                                                \
    }
    MR3_BST(1, 1) MR3_BST(1, 2) MR3_BST(1, 4)
    MR3_BST(2, 1) MR3_BST(2, 2) MR3_BST(2, 4)
    MR3_BST(3, 1) MR3_BST(6, 1) MR3_BST(12, 1) MR3_BST(24, 1)
    MR3_BST(4, 1) MR3_BST(4, 2) MR3_BST(4, 4)
    MR3_BST(8, 1) MR3_BST(8, 2) MR3_BST(8, 4)
    MR3_BST(16, 1) MR3_BST(16, 2) MR3_BST(16, 4)
    MR3_BST(32, 1) MR3_BST(32, 2) MR3_BST(32, 4)
    MR3_BST(64, 1) MR3_BST(64, 2) MR3_BST(64, 4)
#undef MR3_BST
}

// slice points for a root with k wanted eigenvalues: about 3k (each point
// costs one count, each eigenvalue gains log2(M + 1) halvings), a multiple of
// the workgroup size, between 1024 and 65536
static int64_t slice_points(int64_t k) {
    int64_t M = 1024;
    while (M < 3 * k && M < 65536) M *= 2;
    return M;
}

// development aid: MR3_NO_STAGE=1 sends every node to the per-lane kernel
static bool no_stage() {
    static const bool v = std::getenv("MR3_NO_STAGE") != nullptr;
    return v;
}

// slot list for a bisection launch: the slots of staged nodes first (with one
// workgroup per G of them), then the rest.  Every child node is staged: its
// eigenvalues share its rows, which a node of at most RESIDENT_ROWS rows keeps
// in LDS for all passes (the per-lane kernel, reading rows from memory per
// lane, took 7.5 ms for the clusters of a 4096-problem batch).
struct BisectPlan {
    std::vector<int64_t> list;
    std::vector<BisWG> wgs;
    int64_t n_staged = 0;
    void add(int node, int64_t n, int64_t first, int64_t count, int G, std::vector<int64_t>& rest) {
        if (n >= 1 && !no_stage()) {
            for (int64_t o = 0; o < count; o += G)
                wgs.push_back(BisWG{(int64_t)list.size() + o, (int)std::min<int64_t>(G, count - o), node});
            for (int64_t i = 0; i < count; ++i) list.push_back(first + i);
        } else {
            for (int64_t i = 0; i < count; ++i) rest.push_back(first + i);
        }
    }
    void finish(std::vector<int64_t>& rest) {
        n_staged = (int64_t)list.size();
        list.insert(list.end(), rest.begin(), rest.end());
    }
};

// lanes per eigenvalue and points per lane.  Measured on the device: with
// the rows staged through LDS the counts are issue bound, so one chain per
// lane (P = 1) is the least work, and L doubles until ~64K lanes are busy (at
// most 64 lanes, one wave, per eigenvalue).
static BisectShape pick_shape(int64_t count, int user_lanes, int user_points) {
    BisectShape sh{1, 1};
    if (user_lanes > 0) {
        while (sh.L * 2 <= user_lanes && sh.L < 64) sh.L *= 2;
    } else {
        while (sh.L < 64 && count * sh.L < 65536) sh.L *= 2;
    }
    if (user_points == 1 || user_points == 2 || user_points == 4) sh.P = user_points;
    return sh;
}

// lanes per eigenvalue of the LDS-staged kernels (its lane groups need not
// divide the wave)
static const int kLaneCands[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 64};
static bool lane_cand(int L) {
    for (int c : kLaneCands)
        if (c == L) return true;
    return false;
}
static int lanes_at_most(int L) {
    int r = 1;
    for (int c : kLaneCands)
        if (c <= L) r = c;
    return r;
}

// the table the library is built with: entries written by the package's
// tuner from timed solves on gfx950 (stage, precision, eigenvalue count range,
// mean node rows range, lanes)
static const mr3_tune_entry kBuiltinTuning[] = {
#define MR3_TUNE(st, pr, c0, c1, r0, r1, l) {st, pr, c0, c1, r0, r1, l, 0},
#include "tuning_gfx950.inc"
#undef MR3_TUNE
    {-1, 0, 0, 0, 0, 0, 0, 0}};

static std::vector<mr3_tune_entry> builtin_tuning() {
    std::vector<mr3_tune_entry> v;
    for (const mr3_tune_entry& t : kBuiltinTuning)
        if (t.stage >= 0) v.push_back(t);
    return v;
}

static bool tune_entry_ok(const mr3_tune_entry& t) {
    return (t.stage == MR3_TUNE_ROOT || t.stage == MR3_TUNE_CHILD) &&
           (t.precision == 32 || t.precision == 64) && t.count_lo < t.count_hi &&
           t.rows_lo < t.rows_hi && lane_cand(t.lanes);
}

// lanes of a staged launch from the override or the table; 0: the size rule
static int table_lanes(const std::vector<mr3_tune_entry>& tab, const Params& prm, int stage,
                       int precision, int64_t count, int64_t rows) {
    if (prm.lanes_per_eig > 0) return lanes_at_most(prm.lanes_per_eig);
    for (const mr3_tune_entry& t : tab)
        if (t.stage == stage && t.precision == precision && count >= t.count_lo &&
            count < t.count_hi && rows >= t.rows_lo && rows < t.rows_hi)
            return t.lanes;
    return 0;
}

// shape of the LDS-staged kernel for many small node-pure groups (the
// members of the clusters of a level): a pass costs about the same while the
// waves fit one per SIMD (1024) and proportionally more beyond, and gains
// log2(L + 1) bits, so L minimises max(1, waves(L) / 1024) / log2(L + 1), with
// waves(L) = sum over groups of ceil(size / (64 / L)) for one-wave workgroups
static BisectShape pick_shape_groups(const std::vector<int64_t>& sizes, int user_lanes) {
    if (user_lanes > 0) return BisectShape{lanes_at_most(user_lanes), 1};
    BisectShape best{64, 1};
    double best_cost = 1e300;
    for (int L : kLaneCands) {
        const int64_t gw = 64 / L;
        double waves = 0.0;
        for (int64_t m : sizes) waves += (double)((m + gw - 1) / gw);
        const double cost = std::max(1.0, waves / 1024.0) / std::log2((double)L + 1.0);
        if (cost < best_cost) {
            best_cost = cost;
            best.L = L;
        }
    }
    return best;
}

// shape of the LDS-staged kernel, whose lane groups need not divide the wave:
// the smallest L (one chain per lane) that fills about one wave per SIMD
// (1024 SIMDs), which spreads the waves evenly and keeps the redundant
// multisection work low
static BisectShape pick_shape_staged(int64_t count, int user_lanes) {
    if (user_lanes > 0) return BisectShape{lanes_at_most(user_lanes), 1};
    BisectShape sh{64, 1};
    for (int L : kLaneCands) {
        const int64_t gw = 64 / L;
        if ((count + gw - 1) / gw >= 900) {
            sh.L = L;
            break;
        }
    }
    return sh;
}

template <class X, class Y>
static int solve_impl(mr3_handle_s* h, int64_t count, const int64_t* n_h, const X* const* d_p,
                      const X* const* e_p, const mr3_range_desc* ranges, int64_t* m_out,
                      X* const* W_p, X* const* Z_p, const int64_t* ldz_h, hipStream_t st,
                      void* work_region, size_t work_bytes) {
    const int precision = sizeof(X) == 4 ? 32 : 64;
    const Params prm = effective(h, precision);
    const double t_start = now_ms();
    const bool is_dd = sizeof(Y) == 16;
    // a caller's work region: every buffer is carved from it up front and
    // nothing is allocated; otherwise the handle's pool grows on demand
    const bool fixed = work_region != nullptr;
    Buf Bf[B_NBUF];
    Buf* B = fixed ? Bf : h->buf;
    // lld of the nodes in y: stored, or formed from e and d where rows are read
    auto REPL = [&]() -> Y* { return prm.derive_lld ? nullptr : B[B_REPL].rows<Y>(); };
    Region reg;
    if (fixed) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(work_region);
        const uintptr_t al = (a + 255) & ~(uintptr_t)255;
        reg.base = reinterpret_cast<char*>(al);
        reg.cap = work_bytes > (size_t)(al - a) ? work_bytes - (size_t)(al - a) : 0;
    }
    int64_t rep_cap = INT64_MAX, tile_cap = INT64_MAX;  // bounded on a work region
    mr3_stats stats{};
    HIPCHK(hipSetDevice(h->device));
    // work a failed earlier call left on the side stream must end before
    // buffers are reused
    if (h->side_pending[0] || h->side_pending[1]) {
        HIPCHK(hipStreamSynchronize(h->side[0]));
        HIPCHK(hipStreamSynchronize(h->side[1]));
        h->side_pending[0] = h->side_pending[1] = false;
    }
    // pinned staging space is reused from the last solve, which has finished
    // unless it left with an error
    if (!h->clean_exit) HIPCHK(hipDeviceSynchronize());
    h->clean_exit = false;
    h->stage.reset();
    h->stage.grow = !fixed;
    struct StageScope {
        StageScope(Staging* s) { g_stage = s; }
        ~StageScope() { g_stage = nullptr; }
    } stage_scope(&h->stage);
    // every exit makes `st` wait for the side stream, so that synchronizing
    // the caller's stream covers all of this call's work
    struct SideJoin {
        mr3_handle_s* h;
        hipStream_t st;
        ~SideJoin() {
            for (int q = 0; q < 2; ++q)
                if (h->side_pending[q]) (void)hipStreamWaitEvent(st, h->ev_side[q], 0);
        }
    } side_join{h, st};
    // synchronizes the side stream before a buffer it may read is reallocated
    auto quiesce = [&]() -> hipError_t {
        if (!h->side_pending[0] && !h->side_pending[1]) return hipSuccess;
        hipError_t e = hipStreamSynchronize(h->side[0]);
        if (e == hipSuccess) e = hipStreamSynchronize(h->side[1]);
        h->side_pending[0] = h->side_pending[1] = false;
        return e;
    };
    // ---- problems ----
    std::vector<ProbDesc> probs((size_t)count);
    int64_t R = 0;
    for (int64_t p = 0; p < count; ++p) {
        ProbDesc& pd = probs[p];
        pd.n = n_h[p];
        pd.din = d_p[p];
        pd.ein = e_p[p] ? e_p[p] : d_p[p];  // never read for n <= 1
        pd.wout = W_p[p];
        pd.zout = Z_p ? Z_p[p] : nullptr;
        pd.ldz = (Z_p && Z_p[p]) ? ldz_h[p] : 1;
        pd.row0 = R;
        pd.range = ranges ? ranges[p].range : RANGE_ALL;
        pd.vl = ranges ? ranges[p].vl : 0.0;
        pd.vu = ranges ? ranges[p].vu : 0.0;
        pd.il = ranges ? ranges[p].il : 1;
        pd.iu = ranges ? ranges[p].iu : pd.n;
        if (pd.range == RANGE_ALL) { pd.il = 1; pd.iu = pd.n; }
        R += pd.n;
        m_out[p] = 0;
    }
    if (R == 0) { h->stats = stats; h->clean_exit = true; return MR3_OK; }
    if (fixed) {
        Shape sh;
        sh.count = count;
        sh.R = R;
        size_t sz[B_NBUF] = {0};
        prep_sizes(sh, sz);
        for (int b : PREP_BUFS)
            if (!reg.carve(B[b], sz[b])) { h->clean_exit = true; return ERR_WORK_SMALL; }
    }
    HIPCHK(upload(B[B_PROBS], probs, st));
    HIPCHK(B[B_PINFO].ensure(sizeof(ProbInfo) * count));
    HIPCHK(B[B_TD].ensure(sizeof(double) * (R + 2 * GUARD)));
    HIPCHK(B[B_TE].ensure(sizeof(double) * (R + 2 * GUARD)));
    HIPCHK(B[B_BINFO].ensure(sizeof(BlockInfo) * R));
    hipLaunchKernelGGL(k_prep<X>, dim3((unsigned)count), dim3(256), 0, st, B[B_PROBS].as<ProbDesc>(),
                       prm.eps_x, B[B_TD].rows<double>(), B[B_TE].rows<double>(),
                       B[B_PINFO].as<ProbInfo>(), B[B_BINFO].as<BlockInfo>());
    HIPCHK(hipGetLastError());
    std::vector<ProbInfo> pinfo;
    HIPCHK(download(pinfo, B[B_PINFO].p, (size_t)count, st));
    for (int64_t p = 0; p < count; ++p)
        if (pinfo[p].err) return -6;  // non-finite entry in d or e
    // ---- blocks and slots, assembled on the device ----
    std::vector<int> multi(count, 0);
    std::vector<int64_t> m_p(count, 0);
    std::vector<int64_t> boff((size_t)count + 1, 0);
    for (int64_t p = 0; p < count; ++p) {
        multi[p] = pinfo[p].nblocks > 1;
        boff[p + 1] = boff[p] + pinfo[p].nblocks;
    }
    const int64_t NB = boff[count];
    HIPCHK(upload(B[B_BOFF], boff, st));
    HIPCHK(B[B_BLOCKS].ensure(sizeof(Block) * (size_t)std::max<int64_t>(NB, 1)));
    HIPCHK(B[B_NSLOT].ensure(sizeof(int64_t) * (size_t)(NB + 1)));
    HIPCHK(B[B_SLOT0].ensure(sizeof(int64_t) * (size_t)(NB + 1)));
    int64_t* nslot_d = B[B_NSLOT].as<int64_t>();
    int64_t* slot0_d = B[B_SLOT0].as<int64_t>();
    std::vector<Block> blocks;
    if (NB > 0) {
        HIPCHK(hipMemsetAsync(nslot_d + NB, 0, sizeof(int64_t), st));
        hipLaunchKernelGGL(k_blocks, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                           B[B_PROBS].as<ProbDesc>(), B[B_PINFO].as<ProbInfo>(),
                           B[B_BINFO].as<BlockInfo>(), B[B_BOFF].as<int64_t>(), count,
                           B[B_BLOCKS].as<Block>(), nslot_d);
        size_t tb = 0;
        HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, nslot_d, slot0_d, NB + 1, st));
        HIPCHK(B[B_CUBTMP].ensure(tb + 256));
        tb = B[B_CUBTMP].cap;
        HIPCHK(hipcub::DeviceScan::ExclusiveSum(B[B_CUBTMP].p, tb, nslot_d, slot0_d, NB + 1, st));
        hipLaunchKernelGGL(k_blocks_slots, dim3((unsigned)((NB + 255) / 256)), dim3(256), 0, st,
                           B[B_BLOCKS].as<Block>(), nslot_d, slot0_d, NB);
        HIPCHK(download(blocks, B[B_BLOCKS].p, (size_t)NB, st));
    }
    int64_t K = 0;
    for (const Block& bk : blocks) {
        K += bk.nslot;
        if (bk.il <= bk.iu) m_p[bk.prob] += bk.iu - bk.il + 1;
    }
    stats.n_blocks = NB;
    for (int64_t p = 0; p < count; ++p) { m_out[p] = m_p[p]; stats.n_eigenpairs += m_p[p]; }
    if (K == 0) { h->stats = stats; h->clean_exit = true; return MR3_OK; }
    // Eigenvalues are approximated on binary64 copies, accurate to
    // (k_rr + k_bi) n eps_x relative (k_rr = k_bi = 10, Sec. 3.2 "Arithmetic
    // used to approximate eigenvalues").  On the double-double path a block
    // whose copy does not resolve gaptol has its brackets refined in y.
    // gaptol itself may go down to eps_y sqrt(n) / eps_x (eq. gaptolinterval);
    // brackets are held in binary64, so the refinement target 1e-2 gaptol also
    // stays above 4 ulp: smaller values are refused.
    std::vector<char> yref((size_t)NB, 0);
    {
        int64_t nmax = 0;
        for (int64_t b = 0; b < NB; ++b)
            if (blocks[b].nslot > 0) {
                nmax = std::max(nmax, blocks[b].n);
                yref[b] = is_dd && prm.gaptol < 20.0 * (double)blocks[b].n * prm.eps_x;
            }
        const double floor_ = std::max((double)YEps<Y>::v / prm.eps_x * std::sqrt((double)nmax),
                                       400.0 * 1.1102230246251565e-16);
        if (prm.gaptol < std::min(1e-3, floor_)) {
            h->clean_exit = true;
            return MR3_ERR_GAPTOL;
        }
    }
    const double rtol_y = std::max(prm.bisect_rel, 4.0 * 1.1102230246251565e-16);
    if (fixed) {
        // the rest of the plan, now that blocks and slots are known
        Shape sh;
        sh.count = count;
        sh.R = R;
        sh.NB = NB;
        sh.K = K;
        sh.max_depth = prm.max_depth;
        sh.dd = is_dd;
        sh.dqds = prm.initial == MR3_INITIAL_DQDS;
        sh.lld = !prm.derive_lld;
        sh.xsize = sizeof(X);
        int64_t tile_full = 0;
        for (const Block& bk : blocks)
            if (bk.nslot > 0) {
                sh.nmax = std::max(sh.nmax, bk.n);
                tile_full += bk.n * (bk.nslot + 32);
            }
        if (!plan_region(sh, reg.cap - std::min(reg.cap, reg.used), tile_full)) {
            h->clean_exit = true;
            return ERR_WORK_SMALL;
        }
        size_t sz[B_NBUF] = {0};
        solve_sizes(sh, sz);
        for (int b = 0; b < B_NBUF; ++b)
            if (!is_prep_buf(b) && !reg.carve(B[b], sz[b])) { h->clean_exit = true; return ERR_WORK_SMALL; }
        rep_cap = sh.rep_rows;
        tile_cap = sh.tile_rows;
        if (debug_on())
            std::fprintf(stderr, "[mr3] work region: %zu of %zu bytes, representation rows %lld (roots %lld), tile rows %lld of %lld\n",
                         reg.used, reg.cap, (long long)rep_cap, (long long)R, (long long)tile_cap, (long long)tile_full);
    }
    // inputs of the ascending-order check at the end, enqueued now (after a
    // caller's work region has been carved: B_M and B_BAD live there) so that
    // they are off the solve's tail
    {
        std::vector<int64_t> mv(m_p.begin(), m_p.end());
        HIPCHK(upload(B[B_M], mv, st));
        HIPCHK(B[B_BAD].ensure(sizeof(int) * count));
        HIPCHK(hipMemsetAsync(B[B_BAD].p, 0, sizeof(int) * count, st));
    }
    HIPCHK(B[B_SLOTS].ensure(sizeof(Slot) * (size_t)K));
    hipLaunchKernelGGL(k_slots, dim3((unsigned)NB), dim3(256), 0, st, B[B_BLOCKS].as<Block>(),
                       B[B_PINFO].as<ProbInfo>(), B[B_SLOTS].as<Slot>());
    // nodes: roots first (node index == block index), children appended
    int64_t node_cap = NB + K;  // grows with the tree on the handle's pool
    if (fixed) node_cap = (int64_t)(B[B_NODES].cap / sizeof(Node));
    HIPCHK(B[B_NODES].ensure(sizeof(Node) * (size_t)std::max<int64_t>(node_cap, 1)));
    // representation stack: root rows first
    HIPCHK(B[B_REPD].ensure(sizeof(Y) * (R + 2 * GUARD)));
    if (!prm.derive_lld) HIPCHK(B[B_REPL].ensure(sizeof(Y) * (R + 2 * GUARD)));
    HIPCHK(B[B_D64].ensure(sizeof(double) * (R + 2 * GUARD)));
    HIPCHK(B[B_L64].ensure(sizeof(double) * (R + 2 * GUARD)));
    HIPCHK(B[B_REPE].ensure(sizeof(Y) * R));
    HIPCHK(B[B_P].ensure(sizeof(Y) * (R + 2 * GUARD)));
    HIPCHK(B[B_Q].ensure(sizeof(Y) * (R + 2 * GUARD)));
    HIPCHK(B[B_PE].ensure(sizeof(int) * (R + 2 * GUARD)));
    HIPCHK(B[B_QE].ensure(sizeof(int) * (R + 2 * GUARD)));
    if (is_dd) {
        HIPCHK(B[B_P64].ensure(sizeof(double) * (R + 2 * GUARD)));
        HIPCHK(B[B_Q64].ensure(sizeof(double) * (R + 2 * GUARD)));
    }
    double* P64 = is_dd ? B[B_P64].rows<double>() : nullptr;
    double* Q64 = is_dd ? B[B_Q64].rows<double>() : nullptr;
    HIPCHK(B[B_COUNTERS].ensure(COUNTER_BYTES));
    HIPCHK(hipMemsetAsync(B[B_COUNTERS].p, 0, COUNTER_BYTES, st));
    unsigned long long* counters = B[B_COUNTERS].as<unsigned long long>();
    double* work = reinterpret_cast<double*>(counters + 8);
    int* status = reinterpret_cast<int*>(work + 8);
    Prof prof;
    prof.on = prm.profile != 0;
    // outputs: columns of split problems are zeroed outside their blocks
    bool any_z = false;
    for (int64_t p = 0; p < count; ++p) {
        X* Zp = reinterpret_cast<X*>(probs[p].zout);
        any_z |= Zp != nullptr;
        if (Zp && multi[p] && m_p[p] > 0) {
            const int64_t tot = probs[p].n * m_p[p];
            const unsigned g = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
            hipLaunchKernelGGL(k_zero_cols<X>, dim3(g), dim3(256), 0, st, Zp, probs[p].ldz,
                               probs[p].n, m_p[p]);
        }
    }
    Block* dblocks = B[B_BLOCKS].as<Block>();
    Slot* dslots = B[B_SLOTS].as<Slot>();
    Node* dnodes = B[B_NODES].as<Node>();
    // ---- a2: root representations ----
    prof.begin(MR3_STAGE_PREP, st);
    hipLaunchKernelGGL(k_root<Y>, dim3((unsigned)NB), dim3(256), 0, st, dblocks, B[B_TD].rows<double>(),
                       B[B_TE].rows<double>(), prm, B[B_REPD].rows<Y>(), REPL(),
                       B[B_REPE].as<Y>(), B[B_D64].rows<double>(), B[B_L64].rows<double>(), dnodes,
                       dslots, status);
    hipLaunchKernelGGL(k_pq<Y>, dim3((unsigned)NB), dim3(256), 0, st, dblocks, B[B_REPE].as<Y>(),
                       B[B_P].rows<Y>(), B[B_PE].rows<int>(), B[B_Q].rows<Y>(), B[B_QE].rows<int>(),
                       P64, Q64);
    prof.end(st);
    HIPCHK(hipGetLastError());
    // ---- a3: bisection of every slot on its root ----
    // the slot list is the identity; staged workgroups of a large block
    // serve its slot range directly, and the per-lane kernel skips those slots
    // every root is bisected by the staged kernel (a root's rows are shared by
    // all its eigenvalues; for small roots too this beats per-lane row reads);
    // only roots of at least STAGE_MIN_N rows are sliced first
    const int64_t root_stage_n = 1;
    int64_t k_staged = 0;
    for (int64_t b = 0; b < NB; ++b)
        if (blocks[b].n >= root_stage_n && !no_stage()) k_staged += blocks[b].nslot;
    // roots whose whole spectrum is wanted may start from dqds values instead
    // (one lane per root); their brackets are then checked by Sturm counts
    std::vector<int> dq_blocks;
    std::vector<char> is_dq((size_t)NB, 0);
    bool dq_staged = false;
    if (prm.initial == MR3_INITIAL_DQDS)
        for (int64_t b = 0; b < NB; ++b)
            if (blocks[b].nslot > 0 && blocks[b].nslot == blocks[b].n && blocks[b].n <= MR3_DQDS_MAX_N) {
                dq_blocks.push_back((int)b);
                is_dq[b] = 1;
                dq_staged |= blocks[b].n >= root_stage_n && !no_stage();
            }
    stats.n_dqds_roots = (int64_t)dq_blocks.size();
    BisectShape L = pick_shape(K - k_staged, prm.lanes_per_eig, prm.points_per_lane);
    // staged shape: the tuning table keyed by the eigenvalue count and the
    // mean rows of their roots, else the size rule
    BisectShape Ls = pick_shape_staged(k_staged, 0);
    if (k_staged > 0) {
        double rs = 0.0;
        for (int64_t b = 0; b < NB; ++b)
            if (blocks[b].n >= root_stage_n && !no_stage()) rs += (double)blocks[b].nslot * (double)blocks[b].n;
        const int64_t rows = (int64_t)(rs / (double)k_staged + 0.5);
        const int tl = table_lanes(h->tune, prm, MR3_TUNE_ROOT, precision, k_staged, rows);
        if (tl > 0) Ls = BisectShape{tl, 1};
        stats.bisect_count[MR3_TUNE_ROOT] = k_staged;
        stats.bisect_rows[MR3_TUNE_ROOT] = rows;
        stats.bisect_lanes[MR3_TUNE_ROOT] = Ls.L;
    }
    std::vector<BisWG> rwgs;
    int64_t k_small = 0;
    // one-wave workgroups when every root is resident in LDS (each then loads
    // its node once, and a small node leaves no idle waves behind its few
    // eigenvalues); four-wave ones share the staged windows of large roots
    int64_t nmax_root = 0;
    for (int64_t b = 0; b < NB; ++b) nmax_root = std::max(nmax_root, blocks[b].n);
    const int rwaves = nmax_root <= RESIDENT_ROWS ? 1 : 4;
    for (int64_t b = 0; b < NB; ++b) {
        if (blocks[b].n >= root_stage_n && !no_stage()) {
            const int G = rwaves * (64 / Ls.L);
            for (int64_t o = 0; o < blocks[b].nslot; o += G)
                rwgs.push_back(BisWG{blocks[b].slot0 + o,
                                     (int)std::min<int64_t>(G, blocks[b].nslot - o), (int)b});
        } else {
            k_small += blocks[b].nslot;
        }
    }
    HIPCHK(B[B_LIST].ensure(sizeof(int64_t) * (size_t)K));
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st,
                       B[B_LIST].as<int64_t>(), K);
    HIPCHK(upload(B[B_BWG], rwgs, st));
    // intervals from the binary64 copy are widened by k n eps_d |lambda| before
    // classification: k = 10 on the double-double path (relative robustness
    // constant of the copy, Sec. 3.2 "Arithmetic used to approximate
    // eigenvalues"), 4 when the copy is the representation itself
    const double widen_root = (is_dd ? 10.0 : 4.0) * 1.1102230246251565e-16;  // x n_block
    prof.begin(MR3_STAGE_BISECT, st);
    if (!dq_blocks.empty()) {
        HIPCHK(B[B_DQDS].ensure(sizeof(double) * 6 * (size_t)R));
        HIPCHK(upload(B[B_DQB], dq_blocks, st));
        const int nq = (int)dq_blocks.size();
        hipLaunchKernelGGL(k_dqds, dim3((unsigned)((nq + 63) / 64)), dim3(64), 0, st,
                           B[B_DQB].as<int>(), nq, dblocks, dnodes, B[B_D64].rows<double>(),
                           B[B_L64].rows<double>(), B[B_DQDS].as<double>(), dslots, counters + 4);
    }
    // staged (large) roots: spectrum slicing first; it proves every bracket,
    // and a bracket it cannot prove keeps the root interval, which holds by
    // construction (definite root, Gerschgorin bounds with slack)
    {
        std::vector<int64_t> soff;
        int64_t tot = 0;
        for (int64_t b = 0; b < NB; ++b) {
            soff.push_back(tot);
            if (blocks[b].n >= STAGE_MIN_N && blocks[b].nslot > 0 && !is_dq[b])
                tot += slice_points(blocks[b].nslot) + 4;  // counts, then the interval
        }
        if (tot > 0) {
            HIPCHK(B[B_SLICE].ensure(sizeof(int) * tot));
            for (int64_t b = 0; b < NB; ++b) {
                if (blocks[b].n < STAGE_MIN_N || blocks[b].nslot <= 0 || is_dq[b]) continue;
                const int64_t M = slice_points(blocks[b].nslot);
                stats.n_sliced_roots++;
                int* cnt = B[B_SLICE].as<int>() + soff[b];
                hipLaunchKernelGGL(k_slice, dim3((unsigned)(M / STAGE_ROWS)), dim3(STAGE_ROWS), 0, st,
                                   dblocks, (int)b, dnodes, dslots, B[B_D64].rows<double>(),
                                   B[B_L64].rows<double>(), M, cnt);
                hipLaunchKernelGGL(k_slice_assign, dim3((unsigned)((blocks[b].nslot + 255) / 256)),
                                   dim3(256), 0, st, dblocks, (int)b, dslots, M, cnt, work);
            }
        }
    }
    // small roots (resident in LDS) with enough wanted eigenvalues, when the
    // multisection is throughput bound (at most two lanes per eigenvalue, as
    // in a large batch): sliced by one workgroup each.  With more lanes per
    // eigenvalue a pass is cheap and the serial slicing workgroup would cost
    // more than the passes it saves.
    if (Ls.L <= 2) {
        std::vector<int> sb;
        for (int64_t b = 0; b < NB; ++b)
            if (blocks[b].n >= root_stage_n && blocks[b].n < STAGE_MIN_N && blocks[b].n <= RESIDENT_ROWS &&
                blocks[b].nslot >= 16 && !is_dq[b] && !no_stage())
                sb.push_back((int)b);
        if (!sb.empty()) {
            stats.n_sliced_roots += (int64_t)sb.size();
            HIPCHK(upload(B[B_SLB], sb, st));
            hipLaunchKernelGGL(k_slice_small, dim3((unsigned)sb.size()), dim3(256), 0, st,
                               B[B_SLB].as<int>(), dblocks, dnodes, dslots, B[B_D64].rows<double>(),
                               B[B_L64].rows<double>(), work);
        }
    }
    launch_bisect_staged(Ls, B[B_BWG].as<BisWG>(), (int64_t)rwgs.size(), B[B_LIST].as<int64_t>(),
                         dslots, dnodes, dblocks, B[B_D64].rows<double>(), B[B_L64].rows<double>(),
                         prm.bisect_rel, widen_root, work, dq_staged ? 1 : 0, st, rwaves);
    if (k_small > 0)
        launch_bisect(L, B[B_LIST].as<int64_t>(), K, dslots, dnodes, dblocks,
                      B[B_D64].rows<double>(), B[B_L64].rows<double>(), prm.bisect_rel, widen_root,
                      work, no_stage() ? INT64_MAX : root_stage_n, st);
    prof.end(st);
    HIPCHK(hipGetLastError());
    if (debug_on()) {
        std::vector<double> wk;
        HIPCHK(download(wk, work, 8, st));
        std::fprintf(stderr, "[mr3] root bisection: %lld intervals (%lld staged, lanes %d), passes max %.0f total %.0f\n",
                     (long long)K, (long long)k_staged, Ls.L, wk[6], wk[7]);
        HIPCHK(hipMemsetAsync(work + 6, 0, 2 * sizeof(double), st));
    }
    // brackets of roots whose binary64 copy does not resolve gaptol: checked
    // and refined in y (one workgroup per 32 slots of a root)
    {
        std::vector<int64_t> vlist;
        std::vector<BisWG> vwg;
        for (int64_t b = 0; b < NB; ++b) {
            if (!yref[b]) continue;
            const int64_t m = blocks[b].nslot;
            for (int64_t o = 0; o < m; o += 32)
                vwg.push_back(BisWG{(int64_t)vlist.size() + o, (int)std::min<int64_t>(32, m - o), (int)b});
            for (int64_t q = 0; q < m; ++q) vlist.push_back(blocks[b].slot0 + q);
        }
        if (!vwg.empty()) {
            stats.n_y_refined += (int64_t)vlist.size();
            HIPCHK(upload(B[B_VLIST], vlist, st));
            HIPCHK(upload(B[B_VWG], vwg, st));
            prof.begin(MR3_STAGE_VERIFY, st);
            hipLaunchKernelGGL(k_verify<Y>, dim3((unsigned)vwg.size()), dim3(64), 0, st,
                               B[B_VWG].as<BisWG>(), B[B_VLIST].as<int64_t>(), dslots, dnodes, dblocks,
                               B[B_REPD].rows<Y>(), REPL(), B[B_REPE].as<Y>(), rtol_y, counters + 3, 1);
            prof.end(st);
            HIPCHK(hipGetLastError());
        }
    }
    // ---- output columns of split problems: order by eigenvalue ----
    bool any_multi = false;
    for (int64_t p = 0; p < count; ++p) any_multi |= (multi[p] && m_p[p] > 0);
    if (any_multi) {
        // only the slots of split problems move: each problem's blocks hold a
        // contiguous slot range, which is read, ordered and written back
        std::vector<std::vector<int64_t>> pblocks((size_t)count);
        for (int64_t b = 0; b < NB; ++b)
            if (multi[blocks[b].prob]) pblocks[blocks[b].prob].push_back(b);
        std::vector<Node> roots;
        HIPCHK(download(roots, dnodes, (size_t)NB, st));
        for (int64_t p = 0; p < count; ++p) {
            if (!multi[p] || m_p[p] <= 0 || pblocks[p].empty()) continue;
            int64_t s0 = INT64_MAX, s1 = 0;
            for (int64_t b : pblocks[p]) {
                if (blocks[b].nslot <= 0) continue;
                s0 = std::min(s0, blocks[b].slot0);
                s1 = std::max(s1, blocks[b].slot0 + blocks[b].nslot);
            }
            if (s1 <= s0) continue;
            std::vector<Slot> cur;
            HIPCHK(download(cur, dslots + s0, (size_t)(s1 - s0), st));
            std::vector<std::pair<double, int64_t>> v;
            for (int64_t b : pblocks[p])
                for (int64_t s = blocks[b].slot0; s < blocks[b].slot0 + blocks[b].nslot; ++s)
                    if (cur[s - s0].out == -2)
                        v.push_back({roots[b].sigma_hi + 0.5 * (cur[s - s0].lo + cur[s - s0].hi), s});
            std::stable_sort(v.begin(), v.end(),
                             [](const std::pair<double, int64_t>& a, const std::pair<double, int64_t>& b) {
                                 return a.first < b.first;
                             });
            for (size_t i = 0; i < v.size(); ++i) cur[v[i].second - s0].out = (int64_t)i;
            HIPCHK(hipMemcpyAsync(dslots + s0, cur.data(), sizeof(Slot) * cur.size(),
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
    }
    int64_t nmax_blocks = 1;
    for (const Block& bk : blocks) nmax_blocks = std::max(nmax_blocks, bk.n);
    const int zsplit = (int)std::min<int64_t>(16, std::max<int64_t>(1, nmax_blocks / 2048));
    // ---- the representation trees ----
    // visit(lo, hi, depth) runs one level for the nodes [lo, hi): classify;
    // RQI and output of the singletons on a side stream; child representations
    // and child bisection of the clusters; then the children, recursively.
    // With the handle's pool every cluster of a level is expanded at once (one
    // group: the walk is breadth first).  On a caller's work region the
    // clusters are expanded in groups whose child rows fit the representation
    // stack, and each group's subtree is finished before the next group reuses
    // its rows (Sec. 3.2 / The representation tree: depth first bounds the
    // memory).
    int64_t n_nodes = NB;
    int64_t rep_top = R;  // first free row of the representation stack
    bool rows_recycled = false;
    HIPCHK(B[B_FLAGS].ensure(sizeof(int) * K));
    HIPCHK(B[B_LIST2].ensure(sizeof(int64_t) * K));
    HIPCHK(B[B_CNT].ensure(sizeof(int64_t) * 4));
    int64_t* dcnt = B[B_CNT].as<int64_t>();
    hipcub::CountingInputIterator<int64_t> iter(0);
    std::function<int(int64_t, int64_t, int)> visit = [&](int64_t node_lo, int64_t node_hi, int depth) -> int {
        stats.d_max = std::max(stats.d_max, depth);
        std::vector<int64_t> level_nodes((size_t)(node_hi - node_lo));
        std::iota(level_nodes.begin(), level_nodes.end(), node_lo);
        HIPCHK(upload(B[B_LIST], level_nodes, st));
        const int force_single = depth >= prm.max_depth;
        prof.begin(MR3_STAGE_CLASSIFY, st);
        hipLaunchKernelGGL(k_classify, dim3((unsigned)level_nodes.size()), dim3(256), 0, st,
                           B[B_LIST].as<int64_t>(), (int64_t)level_nodes.size(), dnodes, dslots,
                           B[B_FLAGS].as<int>(), prm.gaptol, prm.gaptol_abs, force_single);
        HIPCHK(hipGetLastError());
        // compact the singletons (into the side list of this level's parity)
        // and the cluster heads of these nodes
        const int par = depth & 1;
        if (h->side_pending[par]) {  // an earlier level still owns these buffers
            HIPCHK(hipEventSynchronize(h->ev_side[par]));
            h->side_pending[par] = false;
        }
        Buf& SL = B[B_SIDE_LIST[par]];
        Buf& STO = B[B_SIDE_TOFF[par]];
        Buf& STI = B[B_SIDE_TILES[par]];
        Buf& SRE = B[B_SIDE_RES[par]];
        Buf& SCK = B[B_SIDE_CHUNK[par]];
        HIPCHK(SL.ensure(sizeof(int64_t) * K));
        size_t tmp_bytes = 0, tb2 = 0;
        SelectKind sel_s{dslots, KIND_SINGLETON, node_lo, node_hi};
        SelectKind sel_c{dslots, KIND_CLUSTER_HEAD, node_lo, node_hi};
        HIPCHK(hipcub::DeviceSelect::If(nullptr, tmp_bytes, iter, SL.as<int64_t>(), dcnt, K,
                                        sel_s, st));
        HIPCHK(hipcub::DeviceSelect::If(nullptr, tb2, iter, B[B_LIST2].as<int64_t>(), dcnt + 1, K,
                                        sel_c, st));
        HIPCHK(B[B_CUBTMP].ensure(std::max(tmp_bytes, tb2) + 256));
        tmp_bytes = B[B_CUBTMP].cap;
        HIPCHK(hipcub::DeviceSelect::If(B[B_CUBTMP].p, tmp_bytes, iter, SL.as<int64_t>(),
                                        dcnt, K, sel_s, st));
        tmp_bytes = B[B_CUBTMP].cap;
        HIPCHK(hipcub::DeviceSelect::If(B[B_CUBTMP].p, tmp_bytes, iter, B[B_LIST2].as<int64_t>(),
                                        dcnt + 1, K, sel_c, st));
        prof.end(st);
        std::vector<int64_t> cnts;
        HIPCHK(download(cnts, dcnt, 2, st));
        const int64_t S = cnts[0], C = cnts[1];
        if (debug_on())
            std::fprintf(stderr, "[mr3] depth %d: nodes %zu singletons %lld clusters %lld  t=%.2f ms\n",
                         depth, level_nodes.size(), (long long)S, (long long)C, now_ms() - t_start);
        // ---- a6 + a7: singletons, on the side stream ----
        // With more chunks than SIMDs the singletons are put in node-major
        // order by gap bucket within a node, so that pairs needing the same
        // number of iterations share waves.  With fewer, every chunk has a
        // SIMD and the launch ends with its slowest wave either way; the list
        // stays in slot order, which is node-major already (every node owns
        // a contiguous slot range), and the sort's launches and their host
        // round trips are saved.
        if (S > 32 * 1024) {
            // node-major order, gap bucket within a node
            HIPCHK(B[B_GKEY].ensure(sizeof(unsigned long long) * 2 * S));
            HIPCHK(B[B_GVAL].ensure(sizeof(int64_t) * S));
            unsigned long long* k0 = B[B_GKEY].as<unsigned long long>();
            unsigned long long* k1 = k0 + S;
            int64_t* v1 = B[B_GVAL].as<int64_t>();
            hipLaunchKernelGGL(k_gap_keys, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st,
                               SL.as<int64_t>(), S, dslots, k0);
            int end_bit = 9;
            while (end_bit < 64 && ((int64_t)1 << (end_bit - 8)) <= n_nodes) ++end_bit;
            size_t tb = 0;
            HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k1, SL.as<int64_t>(), v1, (int)S,
                                                      0, end_bit, st));
            HIPCHK(B[B_CUBTMP].ensure(tb + 256));
            tb = B[B_CUBTMP].cap;
            HIPCHK(hipcub::DeviceRadixSort::SortPairs(B[B_CUBTMP].p, tb, k0, k1, SL.as<int64_t>(), v1,
                                                      (int)S, 0, end_bit, st));
            HIPCHK(hipMemcpyAsync(SL.p, v1, sizeof(int64_t) * S, hipMemcpyDeviceToDevice, st));
        }
        int64_t nchunk = 0;
        // host copy of the tile offsets when the tiles of the level take
        // several rounds (work region smaller than the level's tiles)
        std::vector<int64_t> toff_h;
        if (S > 0) {
            // node-pure chunks (at most S of them)
            HIPCHK(B[B_SEG].ensure(sizeof(int64_t) * S));
            HIPCHK(B[B_CMARK].ensure(sizeof(int64_t) * S));
            HIPCHK(B[B_CID].ensure(sizeof(int64_t) * S));
            int64_t* seg = B[B_SEG].as<int64_t>();
            int64_t* cmark = B[B_CMARK].as<int64_t>();
            int64_t* cid = B[B_CID].as<int64_t>();
            const unsigned gS = (unsigned)((S + 255) / 256);
            hipLaunchKernelGGL(k_seg_marks, dim3(gS), dim3(256), 0, st, SL.as<int64_t>(), S, dslots, seg);
            {
                size_t tb = 0;
                HIPCHK(hipcub::DeviceScan::InclusiveScan(nullptr, tb, seg, seg, MaxOp(), S, st));
                size_t tb3 = 0;
                HIPCHK(hipcub::DeviceScan::InclusiveSum(nullptr, tb3, cmark, cid, S, st));
                HIPCHK(B[B_CUBTMP].ensure(std::max(tb, tb3) + 256));
                tb = B[B_CUBTMP].cap;
                HIPCHK(hipcub::DeviceScan::InclusiveScan(B[B_CUBTMP].p, tb, seg, seg, MaxOp(), S, st));
                hipLaunchKernelGGL(k_chunk_marks, dim3(gS), dim3(256), 0, st, seg, S, cmark);
                tb3 = B[B_CUBTMP].cap;
                HIPCHK(hipcub::DeviceScan::InclusiveSum(B[B_CUBTMP].p, tb3, cmark, cid, S, st));
            }
            // the chunk table and its tile offsets are built for the bound of S
            // chunks (rows of absent chunks are 0), so that the chunk count and
            // the total tile rows come back behind one synchronisation
            HIPCHK(SCK.ensure(sizeof(ChunkInfo) * S));
            HIPCHK(STO.ensure(sizeof(int64_t) * (S + 1)));
            HIPCHK(B[B_FLAGS].ensure(sizeof(int64_t) * (S + 1)));
            int64_t* rows = reinterpret_cast<int64_t*>(B[B_FLAGS].p);
            HIPCHK(hipMemsetAsync(rows, 0, sizeof(int64_t) * (S + 1), st));
            hipLaunchKernelGGL(k_chunk_table, dim3(gS), dim3(256), 0, st, SL.as<int64_t>(), S, dslots,
                               dnodes, dblocks, seg, cid, SCK.as<ChunkInfo>(), rows);
            size_t sb = 0;
            HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, sb, rows, STO.as<int64_t>(), S + 1, st));
            HIPCHK(B[B_CUBTMP].ensure(sb + 256));
            sb = B[B_CUBTMP].cap;
            HIPCHK(hipcub::DeviceScan::ExclusiveSum(B[B_CUBTMP].p, sb, rows, STO.as<int64_t>(), S + 1,
                                                    st));
            std::vector<int64_t> nck, tot;
            {
                DownloadBatch db(st);
                HIPCHK(db.add(nck, cid + S - 1, 1));
                HIPCHK(db.add(tot, STO.as<int64_t>() + S, 1));
                HIPCHK(db.finish());
            }
            nchunk = nck[0];
            int64_t tile_need = tot[0];
            if (tile_need > tile_cap) {
                HIPCHK(download(toff_h, STO.p, (size_t)(nchunk + 1), st));
                tile_need = tile_cap;
            }
            HIPCHK(STI.ensure(sizeof(double) * (std::max<int64_t>(tile_need, 1) + 2 * 32 * GUARD)));
            HIPCHK(SRE.ensure(sizeof(RqiResult) * S));
        }
        // RQI and output of this level's singletons go to the side stream of
        // the level's parity once the level's cluster work up to the child
        // multisection has been issued: that chain leads the critical path, so
        // it gets the device first, and the singleton work then overlaps the
        // bracket check and the next level.
        auto fork_singletons = [&]() -> int {
            if (S == 0) return MR3_OK;
            hipStream_t side = h->side[par];
            HIPCHK(hipEventRecord(h->ev_fork, st));
            HIPCHK(hipStreamWaitEvent(side, h->ev_fork, 0));
            // several waves per workgroup when few chunks sweep large nodes
            // (they share rows through L1); one when many small problems'
            // chunks of unequal lengths would hold each other's CU slots
            const int wpg = nchunk <= 2048 ? RQI_WAVES : 1;
            // A multi-wave workgroup takes almost all of a CU's 160 KB of LDS, so
            // that its waves get a SIMD each and no other launch's waves share
            // them: the bracket check in y runs beside the depth-0 RQI on the
            // CUs the RQI leaves (at n = 20000 it went from 2.9 to 1.7 ms, the
            // solve from 33.1 to 32.4 ms, against workgroups of 82 KB).
            // One-wave workgroups take 20 KB of LDS with their windows, so that
            // a CU holds at most 8 of them (two waves per SIMD) even where the
            // kernel's registers would allow three: in the batch regime the
            // cluster chain runs beside this launch and needs the rest of each
            // SIMD (measured on the 4096-problem batch: 12 per CU 15.7 ms, 8 per
            // CU 14.0 ms, 6 per CU 15.6 ms).
            const unsigned pad = wpg > 1 ? (unsigned)(RQI_CU_LDS - RQI_WAVES * (sizeof(SweepWin<Y>) + sizeof(TwistWin)))
                                         : (unsigned)(20u * 1024u - sizeof(SweepWin<Y>) - sizeof(TwistWin));
            auto rqi = prm.derive_lld ? (wpg > 1 ? k_rqi<Y, RQI_WAVES, true> : k_rqi<Y, 1, true>)
                                      : (wpg > 1 ? k_rqi<Y, RQI_WAVES, false> : k_rqi<Y, 1, false>);
            // one round of consecutive chunks whose tiles fit the tile buffer
            // (all chunks unless the work region is smaller than the level's
            // tiles); the rounds reuse the buffer in stream order
            for (int64_t c0 = 0; c0 < nchunk;) {
                int64_t c1 = nchunk, base = 0;
                if (!toff_h.empty()) {
                    c1 = c0 + 1;
                    while (c1 < nchunk && toff_h[c1 + 1] - toff_h[c0] <= tile_cap) ++c1;
                    base = toff_h[c0];
                }
                const int64_t nc = c1 - c0;
                prof.begin(MR3_STAGE_RQI, side);
                hipLaunchKernelGGL(rqi, dim3((unsigned)((nc + wpg - 1) / wpg)), dim3(64 * wpg),
                                   pad, side, SCK.as<ChunkInfo>() + c0, nc,
                                   SL.as<int64_t>(), STO.as<int64_t>() + c0, base,
                                   STI.rows<double>(32), dslots,
                                   dnodes, dblocks, B[B_REPD].rows<Y>(), REPL(), B[B_REPE].as<Y>(),
                                   B[B_D64].rows<double>(), B[B_L64].rows<double>(), B[B_P].rows<Y>(),
                                   B[B_PE].rows<int>(), B[B_Q].rows<Y>(), B[B_QE].rows<int>(), P64, Q64,
                                   prm, (double)YEps<Y>::v, SRE.as<RqiResult>(), counters, work);
                prof.end(side);
                prof.begin(MR3_STAGE_ZOUT, side);
                // rows of a chunk are split over zsplit workgroups (blocks of
                // 64 rows), so that large nodes' output is not one serial loop
                hipLaunchKernelGGL((k_zout<X, Y>), dim3((unsigned)nc, (unsigned)zsplit), dim3(256), 0, side,
                                   SCK.as<ChunkInfo>() + c0, SL.as<int64_t>(), STO.as<int64_t>() + c0, base,
                                   STI.rows<double>(32), dslots,
                                   dnodes, dblocks, B[B_PINFO].as<ProbInfo>(), SRE.as<RqiResult>(),
                                   B[B_PROBS].as<ProbDesc>(), any_z);
                prof.end(side);
                HIPCHK(hipGetLastError());
                c0 = c1;
            }
            HIPCHK(hipEventRecord(h->ev_side[par], side));
            h->side_pending[par] = true;
            if (debug_on()) {
                HIPCHK(hipStreamSynchronize(side));
                std::vector<unsigned long long> c;
                HIPCHK(download(c, counters, 3, st));
                std::fprintf(stderr, "[mr3]   after RQI: iters %llu fallbacks %llu failures %llu t=%.2f ms\n",
                             c[0], c[1], c[2], now_ms() - t_start);
                if (std::getenv("MR3_DEBUG")[0] == '3') {
                    std::vector<RqiResult> rr;
                    HIPCHK(download(rr, SRE.p, (size_t)S, st));
                    int64_t hist[12] = {0};
                    for (int64_t i = 0; i < S; ++i) hist[std::min(std::max(rr[i].iters, 0), 11)]++;
                    std::fprintf(stderr, "[mr3]   iteration histogram:");
                    for (int k = 0; k < 12; ++k) std::fprintf(stderr, " %d:%lld", k, (long long)hist[k]);
                    std::fprintf(stderr, "\n");
                    // sweep lengths: per pair max(r+1, n-r), per chunk the max over its pairs
                    std::vector<ChunkInfo> cks;
                    HIPCHK(download(cks, SCK.p, (size_t)nchunk, st));
                    std::vector<Slot> sl;
                    std::vector<int64_t> ls;
                    std::vector<Node> nds;
                    HIPCHK(download(sl, dslots, (size_t)K, st));
                    HIPCHK(download(ls, SL.p, (size_t)S, st));
                    HIPCHK(download(nds, dnodes, (size_t)n_nodes, st));
                    double sp = 0, sc = 0, sn = 0, it_mean = 0, it_cmax = 0;
                    for (const ChunkInfo& ck : cks) {
                        const int64_t nn = blocks[nds[sl[ls[ck.begin]].node].block].n;
                        int64_t mx = 0;
                        int imx = 0;
                        for (int q = 0; q < ck.count; ++q) {
                            const int64_t r = rr[ck.begin + q].r;
                            const int64_t len = std::max(r + 1, nn - r);
                            sp += (double)len;
                            mx = std::max(mx, len);
                            imx = std::max(imx, rr[ck.begin + q].iters);
                            it_mean += rr[ck.begin + q].iters;
                        }
                        sc += (double)mx * ck.count;
                        sn += (double)nn * ck.count;
                        it_cmax += (double)imx * ck.count;
                    }
                    std::fprintf(stderr, "[mr3]   sweep length / n: pair mean %.3f, chunk max (pair-weighted) %.3f, chunks %lld; iterations: mean %.2f, chunk max %.2f\n",
                                 sp / sn, sc / sn, (long long)nchunk, it_mean / S, it_cmax / S);
                    // pairs by RQI iterations and by the log10 bucket of
                    // their relative gap
                    int64_t gh[6][12] = {{0}};
                    for (int64_t i = 0; i < S; ++i) {
                        const Slot& q = sl[ls[i]];
                        double g = 1e300;
                        if (q.lgap > 0.0) g = std::min(g, q.lgap);
                        if (q.rgap > 0.0) g = std::min(g, q.rgap);
                        const double lam = std::max(std::fabs(q.lo), std::fabs(q.hi));
                        const int bk = (int)std::min(11.0, std::max(0.0, -std::log10(std::max(g / lam, 1e-300))));
                        gh[std::min(std::max(rr[i].iters, 0), 5)][bk]++;
                    }
                    for (int it = 1; it < 6; ++it) {
                        std::fprintf(stderr, "[mr3]   iters %d by -log10(relgap):", it);
                        for (int bk = 0; bk < 12; ++bk) std::fprintf(stderr, " %lld", (long long)gh[it][bk]);
                        std::fprintf(stderr, "\n");
                    }
                }
                if (std::getenv("MR3_DEBUG")[0] == '2') {
                    std::vector<RqiResult> rr;
                    std::vector<int64_t> ls;
                    std::vector<Slot> sl;
                    HIPCHK(download(rr, SRE.p, (size_t)S, st));
                    HIPCHK(download(ls, SL.p, (size_t)S, st));
                    HIPCHK(download(sl, dslots, (size_t)K, st));
                    for (int64_t i = 0; i < S; ++i)
                        if (rr[i].status != 0 || rr[i].iters >= 6)
                            std::fprintf(stderr,
                                         "[mr3]   slot %lld idx %lld st %d it %d r %lld lam %.17g%+.3g "
                                         "[%.17g, %.17g] gaps %.3g %.3g fT %.3g fB %.3g rowr %.3g ev %lld %lld / %lld %lld\n",
                                         (long long)ls[i], (long long)sl[ls[i]].idx, rr[i].status, rr[i].iters,
                                         (long long)rr[i].r, rr[i].lam_hi, rr[i].lam_lo, sl[ls[i]].lo, sl[ls[i]].hi,
                                         sl[ls[i]].lgap, sl[ls[i]].rgap, rr[i].fT, rr[i].fB, rr[i].rowr,
                                         (long long)rr[i].evT1, (long long)rr[i].evT2, (long long)rr[i].evB1,
                                         (long long)rr[i].evB2);
                }
            }
            return MR3_OK;
        };
        if (C == 0) return fork_singletons();
        // With many more chunks than SIMDs (a large batch) the singleton work
        // is long and throughput bound while the cluster work is short: it
        // goes first, and the cluster work fills in beside it.  With few
        // chunks (one large problem) the cluster chain leads the critical path
        // and goes first (below).
        const bool fork_first = nchunk > 4096;
        bool forked = false;
        if (fork_first) {
            stats.n_singleton_first_levels++;
            const int rc = fork_singletons();
            if (rc) return rc;
            forked = true;
        }
        // ---- a5: clusters -> child representations ----
        HIPCHK(B[B_CREC].ensure(sizeof(ClusterRec) * C));
        hipLaunchKernelGGL(k_cluster_recs, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, st,
                           B[B_LIST2].as<int64_t>(), C, dslots, B[B_CREC].as<ClusterRec>());
        std::vector<ClusterRec> crec;
        std::vector<int64_t> cl_n((size_t)C);  // rows of each cluster's block
        std::vector<char> cl_y((size_t)C);     // ... and whether it is refined in y
        {
            std::vector<Node> allnodes;
            DownloadBatch db(st);
            HIPCHK(db.add(crec, B[B_CREC].p, (size_t)C));
            HIPCHK(db.add(allnodes, dnodes, (size_t)n_nodes));
            HIPCHK(db.finish());
            for (int64_t c = 0; c < C; ++c) {
                cl_n[c] = blocks[allnodes[crec[c].parent].block].n;
                cl_y[c] = yref[allnodes[crec[c].parent].block];
                stats.largest_cluster = std::max<int64_t>(stats.largest_cluster, crec[c].last - crec[c].head + 1);
            }
        }
        stats.n_clusters += C;
        // rows that groups below this level may need: one cluster of the
        // largest block per level down to the depth cap
        const int64_t reserve = (int64_t)std::max(0, prm.max_depth - 1 - depth) * nmax_blocks;
        for (int64_t g0 = 0; g0 < C;) {
            // ---- one group of clusters: [g0, g1) ----
            int64_t g1 = g0, new_rows = 0;
            while (g1 < C && (!fixed || rep_top + new_rows + cl_n[g1] + reserve <= rep_cap))
                new_rows += cl_n[g1++];
            if (g1 == g0) return MR3_ERR_HIP;  // cannot happen: the plan keeps room for one cluster
            const int64_t CG = g1 - g0;
            std::vector<ChildJob> jobs((size_t)CG);
            int64_t off = 0;
            for (int64_t c = 0; c < CG; ++c) {
                ChildJob j{};
                j.head = crec[g0 + c].head;
                j.last = crec[g0 + c].last;
                j.parent = crec[g0 + c].parent;
                j.child = (int)(n_nodes + c);
                j.rep = rep_top + off;
                j.tmp = off;
                off += cl_n[g0 + c];
                jobs[c] = j;
            }
            // the side stream reads nodes and representations: it must be idle
            // before any of these buffers is reallocated (handle's pool), and
            // before rows that an earlier group's subtree used are overwritten
            // (work region)
            const int64_t need = rep_top + new_rows;
            if (n_nodes + CG > node_cap || B[B_REPD].cap < sizeof(Y) * (need + 2 * GUARD) ||
                (!prm.derive_lld && B[B_REPL].cap < sizeof(Y) * (need + 2 * GUARD)) ||
                B[B_D64].cap < sizeof(double) * (need + 2 * GUARD) ||
                B[B_L64].cap < sizeof(double) * (need + 2 * GUARD))
                HIPCHK(quiesce());
            if (rows_recycled) {
                for (int q = 0; q < 2; ++q)
                    if (h->side_pending[q]) HIPCHK(hipStreamWaitEvent(st, h->ev_side[q], 0));
                rows_recycled = false;
            }
            if (n_nodes + CG > node_cap) {
                node_cap = n_nodes + CG + K;
                HIPCHK(B[B_NODES].ensure(sizeof(Node) * node_cap, true, st));
                dnodes = B[B_NODES].as<Node>();
            }
            HIPCHK(B[B_REPD].ensure(sizeof(Y) * (need + 2 * GUARD), true, st));
            if (!prm.derive_lld) HIPCHK(B[B_REPL].ensure(sizeof(Y) * (need + 2 * GUARD), true, st));
            HIPCHK(B[B_D64].ensure(sizeof(double) * (need + 2 * GUARD), true, st));
            HIPCHK(B[B_L64].ensure(sizeof(double) * (need + 2 * GUARD), true, st));
            HIPCHK(B[B_TMPC].ensure(sizeof(Y) * new_rows));
            HIPCHK(B[B_TMPE].ensure(sizeof(int) * new_rows));
            HIPCHK(upload(B[B_JOBS], jobs, st));
            if (prm.refine_ends) {
                // both extreme eigenvalues of each cluster, refined in y on
                // the parent (one workgroup of two slots per cluster)
                std::vector<int64_t> vlist;
                std::vector<BisWG> vwg;
                for (int64_t c = 0; c < CG; ++c) {
                    vwg.push_back(BisWG{(int64_t)vlist.size(), 2, jobs[c].parent});
                    vlist.push_back(jobs[c].head);
                    vlist.push_back(jobs[c].last);
                }
                HIPCHK(upload(B[B_VLIST], vlist, st));
                HIPCHK(upload(B[B_VWG], vwg, st));
                prof.begin(MR3_STAGE_VERIFY, st);
                hipLaunchKernelGGL(k_verify<Y>, dim3((unsigned)CG), dim3(64), 0, st, B[B_VWG].as<BisWG>(),
                                   B[B_VLIST].as<int64_t>(), dslots, dnodes, dblocks, B[B_REPD].rows<Y>(),
                                   REPL(), B[B_REPE].as<Y>(), 4.0 * 1.1102230246251565e-16, counters + 3, 1);
                prof.end(st);
            }
            prof.begin(MR3_STAGE_CHILD, st);
            hipLaunchKernelGGL(k_child_select, dim3((unsigned)CG), dim3(64), 0, st,
                               B[B_JOBS].as<ChildJob>(), CG, dslots, dnodes, dblocks,
                               B[B_D64].rows<double>(), B[B_L64].rows<double>(), prm,
                               prm.eps_x / (double)YEps<Y>::v);
            hipLaunchKernelGGL(k_child_rep<Y>, dim3((unsigned)CG), dim3(64), 0, st,
                               B[B_JOBS].as<ChildJob>(), CG, dslots, dnodes, dblocks, B[B_REPD].rows<Y>(),
                               REPL(), B[B_REPE].as<Y>(), B[B_D64].rows<double>(),
                               B[B_L64].rows<double>(), B[B_TMPC].as<Y>(), B[B_TMPE].as<int>(),
                               widen_root / prm.eps_x, prm.eps_x);
            prof.end(st);
            HIPCHK(hipGetLastError());
            // the outcomes of the shift choice (strict, least-growth candidate,
            // none) are copied now and read once the child multisection has
            // been enqueued, waiting on an event that marks the copy: the
            // multisection then follows the transform without a host round trip
            std::vector<ChildJob> done_jobs((size_t)CG);
            ChildJob* jpin = g_stage ? static_cast<ChildJob*>(g_stage->get(sizeof(ChildJob) * CG)) : nullptr;
            if (jpin) {
                HIPCHK(hipMemcpyAsync(jpin, B[B_JOBS].p, sizeof(ChildJob) * CG, hipMemcpyDeviceToHost, st));
                HIPCHK(hipEventRecord(h->ev_jobs, st));
            } else {
                HIPCHK(download(done_jobs, B[B_JOBS].p, (size_t)CG, st));
            }
            const int64_t child0 = n_nodes, top_saved = rep_top;
            rep_top += new_rows;
            n_nodes += CG;
            // ---- child bisection (Alg. 1, refine step): the members of every
            // new cluster, whose slots now belong to the child node ----
            int64_t KC = 0, KCs = 0;
            for (int64_t c = 0; c < CG; ++c) {
                const int64_t m = jobs[c].last - jobs[c].head + 1;
                KC += m;
                if (!no_stage()) KCs += m;
            }
            BisectShape L = pick_shape(KC - KCs, prm.lanes_per_eig, prm.points_per_lane);
            // one wave per workgroup: the clusters of a level are many and small
            const int cwaves = 1;
            BisectShape Lcs;
            {
                std::vector<int64_t> sizes;
                double rs = 0.0;
                for (int64_t c = 0; c < CG; ++c)
                    if (!no_stage()) {
                        sizes.push_back(jobs[c].last - jobs[c].head + 1);
                        rs += (double)sizes.back() * (double)cl_n[g0 + c];
                    }
                Lcs = pick_shape_groups(sizes, 0);
                if (KCs > 0) {
                    const int64_t rows = (int64_t)(rs / (double)KCs + 0.5);
                    const int tl = table_lanes(h->tune, prm, MR3_TUNE_CHILD, precision, KCs, rows);
                    if (tl > 0) Lcs = BisectShape{tl, 1};
                    if (KCs >= stats.bisect_count[MR3_TUNE_CHILD]) {
                        stats.bisect_count[MR3_TUNE_CHILD] = KCs;
                        stats.bisect_rows[MR3_TUNE_CHILD] = rows;
                        stats.bisect_lanes[MR3_TUNE_CHILD] = Lcs.L;
                    }
                }
            }
            BisectPlan cplan;
            {
                std::vector<int64_t> rest;
                for (int64_t c = 0; c < CG; ++c)
                    cplan.add(jobs[c].child, cl_n[g0 + c], jobs[c].head, jobs[c].last - jobs[c].head + 1,
                              cwaves * (64 / Lcs.L), rest);
                cplan.finish(rest);
            }
            HIPCHK(upload(B[B_LIST], cplan.list, st));
            HIPCHK(upload(B[B_BWG], cplan.wgs, st));
            if (debug_on()) HIPCHK(hipMemsetAsync(work + 6, 0, 2 * sizeof(double), st));
            prof.begin(MR3_STAGE_CBISECT, st);
            launch_bisect_staged(Lcs, B[B_BWG].as<BisWG>(), (int64_t)cplan.wgs.size(),
                                 B[B_LIST].as<int64_t>(), dslots, dnodes, dblocks,
                                 B[B_D64].rows<double>(), B[B_L64].rows<double>(), prm.bisect_rel,
                                 widen_root, work, 1, st, cwaves);
            launch_bisect(L, B[B_LIST].as<int64_t>() + cplan.n_staged, KC - cplan.n_staged, dslots,
                          dnodes, dblocks, B[B_D64].rows<double>(), B[B_L64].rows<double>(),
                          prm.bisect_rel, widen_root, work, INT64_MAX, st);
            prof.end(st);
            if (jpin) {
                HIPCHK(hipEventSynchronize(h->ev_jobs));
                std::memcpy(done_jobs.data(), jpin, sizeof(ChildJob) * CG);
            }
            for (auto& j : done_jobs) {
                if (j.best == 1) stats.n_best_candidate++;
                if (j.best == 2) return MR3_ERR_NUMERIC;
            }
            if (debug_on()) {
                std::vector<double> wk;
                HIPCHK(download(wk, work, 8, st));
                int nstrict = 0;
                for (int64_t c = 0; c < CG; ++c) nstrict += done_jobs[c].strict;
                std::fprintf(stderr, "[mr3]   child bisection: %lld intervals, staged lanes %d, passes max %.0f total %.0f; strict children %d of %lld\n",
                             (long long)KC, Lcs.L, wk[6], wk[7], nstrict, (long long)CG);
            }
            // the level's singleton work goes to the side stream now: the
            // bracket check (few waves) then shares the device with it, while
            // the shift choice, child transform and child multisection before
            // it (which fill the device and lead the critical path) do not
            if (!forked) {
                const int rc = fork_singletons();
                if (rc) return rc;
                forked = true;
            }
            prof.begin(MR3_STAGE_VERIFY, st);
            if (is_dd) {
                // A child accepted within the strict growth bound k_elg *
                // spdiam is relatively robust like the root (Sec. 2,
                // "Requirements on the representations"), so its binary64
                // copy brackets its eigenvalues after the widening.  A child
                // accepted under the relaxed bound or as least-growth
                // candidate may not be: check its brackets with counts in y.
                // Children of blocks whose binary64 copies do not resolve
                // gaptol have every bracket refined in y.  One workgroup per
                // 32 slots of one child node; the list holds the refined
                // children first.
                std::vector<int64_t> vlist;
                std::vector<BisWG> vwg;
                int64_t nwg_all = 0;
                for (int pass = 0; pass < 2; ++pass)
                    for (int64_t c = 0; c < CG; ++c) {
                        const bool all = cl_y[g0 + c];
                        if (pass == 0 ? !all : (all || done_jobs[c].strict)) continue;
                        const int64_t m = jobs[c].last - jobs[c].head + 1;
                        for (int64_t o = 0; o < m; o += 32)
                            vwg.push_back(BisWG{(int64_t)vlist.size() + o, (int)std::min<int64_t>(32, m - o),
                                                jobs[c].child});
                        for (int64_t sidx = jobs[c].head; sidx <= jobs[c].last; ++sidx) vlist.push_back(sidx);
                        if (pass == 0) {
                            nwg_all = (int64_t)vwg.size();
                            stats.n_y_refined += m;
                        }
                    }
                if (!vwg.empty()) {
                    HIPCHK(upload(B[B_VLIST], vlist, st));
                    HIPCHK(upload(B[B_VWG], vwg, st));
                    if (nwg_all > 0)
                        hipLaunchKernelGGL(k_verify<Y>, dim3((unsigned)nwg_all), dim3(64), 0, st,
                                           B[B_VWG].as<BisWG>(), B[B_VLIST].as<int64_t>(), dslots, dnodes,
                                           dblocks, B[B_REPD].rows<Y>(), REPL(), B[B_REPE].as<Y>(),
                                           rtol_y, counters + 3, 1);
                    if ((int64_t)vwg.size() > nwg_all)
                        hipLaunchKernelGGL(k_verify<Y>, dim3((unsigned)((int64_t)vwg.size() - nwg_all)),
                                           dim3(64), 0, st, B[B_VWG].as<BisWG>() + nwg_all,
                                           B[B_VLIST].as<int64_t>(), dslots, dnodes, dblocks,
                                           B[B_REPD].rows<Y>(), REPL(), B[B_REPE].as<Y>(),
                                           prm.bisect_rel, counters + 3, 0);
                }
            }
            prof.end(st);
            HIPCHK(hipGetLastError());
            // ---- the children of this group, recursively ----
            const int rc = visit(child0, child0 + CG, depth + 1);
            if (rc) return rc;
            if (fixed) {  // pop the group's rows; their readers finish first
                rep_top = top_saved;
                rows_recycled = true;
            }
            g0 = g1;
        }
        return MR3_OK;
    };
    {
        const int rc = visit(0, NB, 0);
        if (rc) return rc;
    }
    // ---- join the side stream; diagnostics and the ascending-order check ----
    for (int q = 0; q < 2; ++q)
        if (h->side_pending[q]) {
            HIPCHK(hipStreamWaitEvent(st, h->ev_side[q], 0));
            h->side_pending[q] = false;
        }
    // the ascending-order check is enqueued first, so that its flags come
    // back with the counters behind one synchronisation
    if (prm.force_resort)
        hipLaunchKernelGGL(k_reverse_outputs<X>, dim3((unsigned)count), dim3(256), 0, st,
                           B[B_PROBS].as<ProbDesc>(), B[B_M].as<int64_t>());
    hipLaunchKernelGGL(k_check_sorted<X>, dim3((unsigned)count), dim3(256), 0, st,
                       B[B_PROBS].as<ProbDesc>(), B[B_M].as<int64_t>(), B[B_BAD].as<int>(),
                       (int)count);
    std::vector<unsigned long long> ctr;
    std::vector<int> sts, bad;
    std::vector<double> wk;
    {
        DownloadBatch db(st);
        HIPCHK(db.add(ctr, counters, 8));
        HIPCHK(db.add(sts, status, 1));
        HIPCHK(db.add(wk, work, 4));
        HIPCHK(db.add(bad, B[B_BAD].p, (size_t)count));
        HIPCHK(db.finish());
    }
    stats.n_rqi_iters = (int64_t)ctr[0];
    stats.n_fallbacks = (int64_t)ctr[1];
    stats.dqds_transforms = (int64_t)ctr[4];
    stats.bisect_row_steps = wk[0];
    stats.rqi_row_steps = wk[1];
    stats.twist_row_steps = wk[2];
    prof.collect(stats);
    h->stats = stats;
    if (sts[0] != 0 || ctr[2] != 0) return MR3_ERR_NUMERIC;
    if (debug_on())
        std::fprintf(stderr, "[mr3] levels done t=%.2f ms (rqi iters %llu fallbacks %llu repaired brackets %llu)\n",
                     now_ms() - t_start, (unsigned long long)ctr[0], (unsigned long long)ctr[1],
                     (unsigned long long)ctr[3]);
    for (int64_t p = 0; p < count; ++p) {
        if (!bad[p]) continue;
        h->stats.n_resorted++;
        if (debug_on()) std::fprintf(stderr, "[mr3] problem %lld: eigenvalues reordered on the host\n", (long long)p);
        // rare: eigenvalues equal to working accuracy came out in the wrong
        // order; sort the pairs on the host
        const int64_t mp = m_p[p], np = probs[p].n;
        std::vector<X> w((size_t)mp);
        X* Wp = reinterpret_cast<X*>(probs[p].wout);
        X* Zp = reinterpret_cast<X*>(probs[p].zout);
        HIPCHK(hipMemcpy(w.data(), Wp, sizeof(X) * mp, hipMemcpyDeviceToHost));
        std::vector<int64_t> perm((size_t)mp);
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return w[a] < w[b]; });
        std::vector<X> w2((size_t)mp);
        for (int64_t i = 0; i < mp; ++i) w2[i] = w[perm[i]];
        HIPCHK(hipMemcpy(Wp, w2.data(), sizeof(X) * mp, hipMemcpyHostToDevice));
        if (Zp) {
            // apply the permutation to the columns on the device, cycle by
            // cycle through one scratch column (only misplaced columns move)
            HIPCHK(B[B_CHECK].ensure(sizeof(X) * (size_t)std::max<int64_t>(np, 1)));
            X* tmp = B[B_CHECK].as<X>();
            std::vector<char> seen((size_t)mp, 0);
            auto col = [&](int64_t c) { return Zp + c * probs[p].ldz; };
            for (int64_t s0 = 0; s0 < mp; ++s0) {
                if (seen[s0] || perm[s0] == s0) { seen[s0] = 1; continue; }
                // new column i takes old column perm[i]
                HIPCHK(hipMemcpyAsync(tmp, col(s0), sizeof(X) * np, hipMemcpyDeviceToDevice, st));
                int64_t i = s0;
                while (true) {
                    seen[i] = 1;
                    const int64_t src = perm[i];
                    if (src == s0) {
                        HIPCHK(hipMemcpyAsync(col(i), tmp, sizeof(X) * np, hipMemcpyDeviceToDevice, st));
                        break;
                    }
                    HIPCHK(hipMemcpyAsync(col(i), col(src), sizeof(X) * np, hipMemcpyDeviceToDevice, st));
                    i = src;
                }
            }
            HIPCHK(hipStreamSynchronize(st));
        }
    }
    h->clean_exit = true;
    return MR3_OK;
}

}  // namespace mr3

// --------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing (mr3_solve_noalloc): device
// memory of the library's code object, one copy per GPU, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress, once per device at handle set-up,
// and only that address is passed to kernels and copies.
// --------------------------------------------------------------------------
static __device__ __align__(256) char scratch[MR3_NOALLOC_SCRATCH_BYTES];

// device address of `scratch` on `device`, which must be current; nullptr if
// the runtime cannot resolve it
static void* scratch_address(int device) {
    static std::mutex mu;
    static std::vector<void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return nullptr;
    if ((int)addr.size() <= device) addr.resize((size_t)device + 1, nullptr);
    if (!addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        addr[device] = p;
    }
    return addr[device];
}

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
using namespace mr3;

static int check_single(int64_t n, const void* d, const void* e, int range, double vl, double vu,
                        int64_t il, int64_t iu, int64_t* m, const void* W, const void* Z,
                        int64_t ldz) {
    if (n < 0) return -2;
    if (n > 0 && !d) return -3;
    if (n > 1 && !e) return -4;
    if (range < 0 || range > 2) return -5;
    if (range == RANGE_VALUE && !(vl < vu)) return -7;
    if (range == RANGE_INDEX && (il < 1 || iu > n || il > iu + 1)) return (il < 1) ? -8 : -9;
    if (!m) return -10;
    if (n > 0 && !W) return -11;
    if (Z && ldz < std::max<int64_t>(1, n)) return -13;
    return 0;
}

// After a failed solve on a caller's work region, device work of the call may
// still read or write the region: it ends before the caller gets it back.
static int finish_on_region(mr3_handle h, int rc, void* work, void* stream) {
    if (rc != MR3_OK && work) {
        (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize((hipStream_t)stream);
    }
    return rc;
}

template <class X, class Y>
static int solve_single(mr3_handle h, int64_t n, const X* d, const X* e, int range, double vl,
                        double vu, int64_t il, int64_t iu, int64_t* m, X* W, X* Z, int64_t ldz,
                        void* work, size_t work_bytes, void* stream, int work_small_rc) {
    if (!h) return -1;
    int rc = check_single(n, d, e, range, vl, vu, il, iu, m, W, Z, ldz);
    if (rc) return rc;
    if (range == RANGE_INDEX && il > iu) { *m = 0; return MR3_OK; }
    mr3_range_desc rd;
    rd.range = range;
    rd.vl = vl;
    rd.vu = vu;
    rd.il = il;
    rd.iu = iu;
    const int64_t nn = n, lz = ldz;
    rc = solve_impl<X, Y>(h, 1, &nn, &d, &e, &rd, m, &W, &Z, &lz, (hipStream_t)stream, work,
                          work_bytes);
    if (rc == ERR_WORK_SMALL) rc = work_small_rc;
    return finish_on_region(h, rc, work, stream);
}

// base pointers + element offsets -> per-problem pointers
template <class X, class Y>
static int batched_ptrs(mr3_handle h, int64_t count, const int64_t* n, const int64_t* de_off,
                        const X* d, const X* e, const mr3_range_desc* ranges, int64_t* m, X* W,
                        const int64_t* w_off, X* Z, const int64_t* z_off, const int64_t* ldz,
                        void* work, size_t work_bytes, hipStream_t st) {
    std::vector<const X*> dp((size_t)count), ep((size_t)count);
    std::vector<X*> wp((size_t)count), zp((size_t)count, nullptr);
    for (int64_t p = 0; p < count; ++p) {
        dp[p] = d + de_off[p];
        ep[p] = e + de_off[p];
        wp[p] = W + w_off[p];
        if (Z) zp[p] = Z + z_off[p];
    }
    int rc = solve_impl<X, Y>(h, count, n, dp.data(), ep.data(), ranges, m, wp.data(),
                              Z ? zp.data() : nullptr, ldz, st, work, work_bytes);
    if (rc == ERR_WORK_SMALL) rc = -16;
    return finish_on_region(h, rc, work, st);
}

template <class X, class Y>
static int solve_ptrs_typed(mr3_handle h, int64_t count, const int64_t* n, const void* const* d,
                            const void* const* e, const mr3_range_desc* ranges, int64_t* m,
                            void* const* W, void* const* Z, const int64_t* ldz, void* work,
                            size_t work_bytes, hipStream_t st) {
    std::vector<const X*> dp((size_t)count), ep((size_t)count);
    std::vector<X*> wp((size_t)count), zp((size_t)count, nullptr);
    for (int64_t p = 0; p < count; ++p) {
        dp[p] = static_cast<const X*>(d[p]);
        ep[p] = static_cast<const X*>(e[p]);
        wp[p] = static_cast<X*>(W[p]);
        if (Z) zp[p] = static_cast<X*>(Z[p]);
    }
    const int rc = solve_impl<X, Y>(h, count, n, dp.data(), ep.data(), ranges, m, wp.data(),
                                    Z ? zp.data() : nullptr, ldz, st, work, work_bytes);
    return finish_on_region(h, rc, work, st);
}

int mr3_solve_ptrs(mr3_handle h, int precision, int64_t count, const int64_t* n,
                   const void* const* d, const void* const* e, const mr3_range_desc* ranges,
                   int64_t* m, void* const* W, void* const* Z, const int64_t* ldz, void* work,
                   size_t work_bytes, void* stream) {
    if (!h) return -1;
    if (count <= 0) return MR3_OK;
    if (precision == 32)
        return solve_ptrs_typed<float, double>(h, count, n, d, e, ranges, m, W, Z, ldz, work,
                                               work_bytes, (hipStream_t)stream);
    return solve_ptrs_typed<double, dd>(h, count, n, d, e, ranges, m, W, Z, ldz, work, work_bytes,
                                        (hipStream_t)stream);
}

void mr3_handle_copy_params(mr3_handle dst, mr3_handle src) {
    if (!dst || !src) return;
    dst->user = src->user;
    dst->have_user = src->have_user;
    dst->tune = src->tune;
}

int mr3_handle_device(mr3_handle h) { return h ? h->device : -1; }

extern "C" {

const char* mr3_version(void) { return "mr3-mi355x 0.1"; }

int mr3_create(mr3_handle* h, int device) {
    if (!h) return -1;
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd <= 0) return MR3_ERR_NO_DEVICE;
    if (device < 0 || device >= nd) return -2;
    mr3_handle_s* x = new mr3_handle_s();
    x->device = device;
    x->tune = mr3::builtin_tuning();
    // set-up on the device: the side streams and their events, the device
    // address of the no-allocation scratch array, and a first pinned staging
    // chunk (a solve on a caller's work region does not grow it)
    bool ok = hipSetDevice(device) == hipSuccess &&
              hipStreamCreateWithFlags(&x->side[0], hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&x->side[1], hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&x->ev_fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&x->ev_jobs, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&x->ev_side[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&x->ev_side[1], hipEventDisableTiming) == hipSuccess;
    if (ok) {
        x->scratch = scratch_address(device);
        ok = x->scratch != nullptr;
    }
    if (ok) {
        x->stage.reset();
        ok = x->stage.get(1) != nullptr;
        x->stage.reset();
    }
    if (!ok) {
        (void)mr3_destroy(x);
        return MR3_ERR_HIP;
    }
    *h = x;
    return MR3_OK;
}

int mr3_destroy(mr3_handle h) {
    if (!h) return -1;
    (void)hipSetDevice(h->device);
    mr3_dense_release(h);
    for (auto& sd : h->side)
        if (sd) (void)hipStreamSynchronize(sd);
    for (auto& b : h->buf) b.release();
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_jobs) (void)hipEventDestroy(h->ev_jobs);
    for (auto& ev : h->ev_side)
        if (ev) (void)hipEventDestroy(ev);
    for (auto& sd : h->side)
        if (sd) (void)hipStreamDestroy(sd);
    h->stage.release();
    delete h;
    return MR3_OK;
}

int mr3_default_params(mr3_params* p, int precision) {
    if (!p) return -1;
    if (precision != 32 && precision != 64) return -2;
    defaults(p, precision);
    return MR3_OK;
}

int mr3_set_params(mr3_handle h, const mr3_params* p) {
    if (!h) return -1;
    if (p) {
        if (p->initial != MR3_INITIAL_BISECTION && p->initial != MR3_INITIAL_DQDS) return -2;
        h->user = *p;
        h->have_user = true;
    } else {
        h->have_user = false;
    }
    return MR3_OK;
}

int mr3_set_tuning(mr3_handle h, const mr3_tune_entry* t, int count) {
    if (!h) return -1;
    if (!t && count < 0) {
        h->tune = mr3::builtin_tuning();
        return MR3_OK;
    }
    if (count < 0 || (count > 0 && !t)) return -2;
    for (int i = 0; i < count; ++i)
        if (!mr3::tune_entry_ok(t[i])) return -2;
    h->tune.assign(t, t + count);
    return MR3_OK;
}

int mr3_get_tuning(mr3_handle h, mr3_tune_entry* t, int cap) {
    if (!h) return -1;
    const int nt = (int)h->tune.size();
    for (int i = 0; i < nt && i < cap && t; ++i) t[i] = h->tune[i];
    return nt;
}

int mr3_bisect_lanes(mr3_handle h, int stage, int precision, int64_t count, int64_t rows) {
    if (!h) return -1;
    if ((stage != MR3_TUNE_ROOT && stage != MR3_TUNE_CHILD) || (precision != 32 && precision != 64))
        return -2;
    return mr3::table_lanes(h->tune, mr3::effective(h, precision), stage, precision, count, rows);
}

int mr3_get_stats(mr3_handle h, mr3_stats* s) {
    if (!h) return -1;
    if (!s) return -2;
    *s = h->stats;
    return MR3_OK;
}

int mr3_solve_f32(mr3_handle h, int64_t n, const float* d, const float* e, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t* m, float* W, float* Z, int64_t ldz,
                  void* work, size_t work_bytes, void* stream) {
    return solve_single<float, double>(h, n, d, e, range, vl, vu, il, iu, m, W, Z, ldz, work,
                                       work_bytes, stream, -15);
}

int mr3_solve_f64(mr3_handle h, int64_t n, const double* d, const double* e, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t* m, double* W, double* Z, int64_t ldz,
                  void* work, size_t work_bytes, void* stream) {
    return solve_single<double, dd>(h, n, d, e, range, vl, vu, il, iu, m, W, Z, ldz, work,
                                    work_bytes, stream, -15);
}

int mr3_solve_noalloc(mr3_handle h, int precision, int64_t n, const void* d, const void* e,
                      int range, double vl, double vu, int64_t il, int64_t iu, int64_t* m, void* W,
                      void* Z, int64_t ldz, void* stream) {
    if (!h) return -1;
    if (precision != 32 && precision != 64) return -2;
    if (n > MR3_NOALLOC_MAX_N) return -3;
    const int rc = check_single(n, d, e, range, vl, vu, il, iu, m, W, Z, ldz);
    if (rc) return rc - 1;  // positions after the extra `precision` argument
    if (!h->scratch) return MR3_ERR_HIP;
    // the scratch is the work region of an ordinary solve; one that does not
    // fit it (n above the limit) is refused as a size error
    if (precision == 32)
        return solve_single<float, double>(h, n, (const float*)d, (const float*)e, range, vl, vu, il,
                                           iu, m, (float*)W, (float*)Z, ldz, h->scratch,
                                           MR3_NOALLOC_SCRATCH_BYTES, stream, -3);
    return solve_single<double, dd>(h, n, (const double*)d, (const double*)e, range, vl, vu, il, iu,
                                    m, (double*)W, (double*)Z, ldz, h->scratch,
                                    MR3_NOALLOC_SCRATCH_BYTES, stream, -3);
}

// Shape of a single problem for the workspace query: every row its own block
// at worst; k wanted eigenvalues plus at most two helpers per block that has
// wanted eigenvalues (no more slots than rows).
static Shape query_shape(mr3_handle h, int64_t n, int range, int64_t k_max, int precision) {
    const Params prm = h ? effective(h, precision) : Params{};
    Shape s;
    s.count = 1;
    s.R = n;
    s.NB = n;
    const int64_t k = (range == RANGE_ALL || k_max <= 0) ? n : std::min(n, k_max);
    s.K = (range == RANGE_ALL || k == n) ? n : std::min(n, 3 * k);
    s.nmax = n;
    s.max_depth = h ? prm.max_depth : 6;
    s.dd = precision == 64;
    s.dqds = h && prm.initial == MR3_INITIAL_DQDS;
    s.lld = !(h && prm.derive_lld);
    s.xsize = precision == 64 ? 8 : 4;
    return s;
}

size_t mr3_workspace_bytes(mr3_handle h, int64_t n, int range, int64_t k_max, int precision) {
    if (n <= 0 || range < 0 || range > 2 || (precision != 32 && precision != 64)) return 0;
    const Shape s = query_shape(h, n, range, k_max, precision);
    return full_bytes(s, n * (s.K + 32));
}

size_t mr3_workspace_min_bytes(mr3_handle h, int64_t n, int range, int64_t k_max, int precision) {
    if (n <= 0 || range < 0 || range > 2 || (precision != 32 && precision != 64)) return 0;
    Shape s = query_shape(h, n, range, k_max, precision);
    size_t sz[B_NBUF] = {0};
    prep_sizes(s, sz);
    s.rep_rows = min_rep_rows(s);
    s.tile_rows = min_tile_rows(s);
    solve_sizes(s, sz);
    return 256 + phase_bytes(sz, true) + phase_bytes(sz, false) + 256 * (size_t)B_NBUF;
}

size_t mr3_workspace_bytes_batched(mr3_handle h, int64_t count, int precision, const int64_t* n,
                                   const mr3_range_desc* ranges) {
    if (count <= 0 || !n || (precision != 32 && precision != 64)) return 0;
    Shape s;
    int64_t tile_full = 0;
    for (int64_t p = 0; p < count; ++p) {
        if (n[p] < 0) return 0;
        const int r = ranges ? ranges[p].range : RANGE_ALL;
        const int64_t k = (r == RANGE_INDEX) ? std::max<int64_t>(ranges[p].iu - ranges[p].il + 1, 0) : n[p];
        const Shape q = query_shape(h, n[p], r, k, precision);
        s.R += q.R;
        s.NB += q.NB;
        s.K += q.K;
        s.nmax = std::max(s.nmax, q.nmax);
        s.max_depth = q.max_depth;
        s.dd = q.dd;
        s.dqds = q.dqds;
        s.lld = q.lld;
        s.xsize = q.xsize;
        tile_full += q.R * (q.K + 32);
    }
    s.count = count;
    if (s.R == 0) return 0;
    return full_bytes(s, tile_full);
}

int mr3_solve_batched(mr3_handle h, int64_t count, int precision, const int64_t* n,
                      const int64_t* de_off, const void* d, const void* e,
                      const mr3_range_desc* ranges, int64_t* m, void* W, const int64_t* w_off,
                      void* Z, const int64_t* z_off, const int64_t* ldz, void* work,
                      size_t work_bytes, void* stream) {
    if (!h) return -1;
    if (count < 0) return -2;
    if (precision != 32 && precision != 64) return -3;
    if (count == 0) return MR3_OK;
    if (!n) return -4;
    if (!de_off) return -5;
    int64_t tot = 0;
    for (int64_t p = 0; p < count; ++p) {
        if (n[p] < 0) return -4;
        tot += n[p];
        if (ranges) {
            const mr3_range_desc& r = ranges[p];
            if (r.range < 0 || r.range > 2) return -8;
            if (r.range == RANGE_VALUE && !(r.vl < r.vu)) return -8;
            if (r.range == RANGE_INDEX && (r.il < 1 || r.iu > n[p] || r.il > r.iu)) return -8;
        }
        if (Z && (!z_off || !ldz || ldz[p] < std::max<int64_t>(1, n[p]))) return -14;
    }
    if (tot > 0 && (!d || !e)) return -6;
    if (!m) return -9;
    if (!W || !w_off) return -10;
    if (precision == 32)
        return batched_ptrs<float, double>(h, count, n, de_off, (const float*)d, (const float*)e,
                                           ranges, m, (float*)W, w_off, (float*)Z, z_off, ldz,
                                           work, work_bytes, (hipStream_t)stream);
    return batched_ptrs<double, dd>(h, count, n, de_off, (const double*)d, (const double*)e, ranges,
                                    m, (double*)W, w_off, (double*)Z, z_off, ldz, work, work_bytes,
                                    (hipStream_t)stream);
}

}  // extern "C"
