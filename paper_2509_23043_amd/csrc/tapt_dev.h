// Device-side descriptors shared by the HIP kernels and the host runtime of
// libtapt. Everything the kernels read about a problem instance lives in one
// InstDev struct in device memory; a persistent launch is a list of WorkItems,
// one per workgroup.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tapt {

enum : int32_t { KIND_LATTICE = 0, KIND_CSR = 1 };
enum : uint32_t {
    TAG_INIT = 1, TAG_SWEEP = 2, TAG_REFINE = 3, TAG_PROPOSE = 4, TAG_SWAP = 5, TAG_BANK = 6,
    TAG_CONTEXT = 7, TAG_CTXSWEEP = 8
};
constexpr uint32_t ALWAYS = 0xFFFFFFFFu;   // threshold meaning "accept unconditionally"
constexpr int MAX_COLORS = 64;
// sparse-graph sweepers of the workgroup-synchronous kernel
enum : int32_t { SPARSE_CSR = 0, SPARSE_WIDE = 1, SPARSE_QUAD = 2, SPARSE_ROW = 3, SPARSE_ROW4 = 4 };
// packed-row sparse sweeper: bonds per lane, lanes per (site, storage) item
// for a largest degree, limits, and the LDS bytes of its rows
constexpr int CSR_ROW_BPL = 16, CSR_ROW_MAXN = 4095, CSR_ROW_MAXJ = 7;
__host__ __device__ inline int csr_row_lanes(int maxdeg) { return maxdeg <= CSR_ROW_BPL ? 1 : 2; }
__host__ __device__ inline size_t csr_row_graph_bytes(int ncolors, int maxcnt, int lanes)
{
    return (size_t)ncolors * maxcnt * lanes * 36 + 32;
}
// the same for the four-storages-per-lane variant (16 bonds of 32 bits per record)
constexpr int CSR_ROW4_BPL = 16;
__host__ __device__ inline int csr_row4_lanes(int maxdeg) { return maxdeg <= CSR_ROW4_BPL ? 1 : 2; }
__host__ __device__ inline size_t csr_row4_graph_bytes(int ncolors, int maxcnt, int lanes)
{
    return (size_t)ncolors * maxcnt * lanes * 68 + 64;
}

// The one-slot-per-wavefront sparse kernel packs a site's bonds in chunks of
// CSRW_CHUNK 16-bit words; a rank group of 64 sites takes as many chunks as
// its largest degree needs. Graphs with larger degrees or more rank groups
// run in the other kernels.
constexpr int CSRW_CHUNK = 8, CSRW_MAXDEG = 64, CSRW_MAXGROUPS = 64;

struct BestRec {          // best min_r E_r seen; ordered by (E, t, slot)
    int32_t E;
    int32_t slot;
    int64_t t;
    int64_t first_hit;    // -1: target not reached
    int64_t pad;
};

struct InstDev {
    int32_t n, L, R, kind;
    int32_t rule, M, D, tflip_stride;       // flip table: index d + D, d = m_i I_i in [-D, D]
    int32_t has_target, target, ncolors, nfree;
    int32_t nnz, ctx_sweeps;                // ctx_sweeps: completion sweeps of a contextual proposal
    uint32_t seed_lo, seed_hi;
    uint32_t epoch;                         // bumps when the state is replaced
    int32_t ctx_K;                          // context sites of a contextual proposal
    int32_t ctx_on;                         // 1: proposals are contextual
    int32_t maxdeg;                         // largest degree of a free site
    int32_t maxcnt, maxabsj;                // largest colour class (free sites); largest |J|
    int32_t csrw_chunks;                    // bond chunks of the packed rows of the one-slot-per-
                                            // wavefront sparse kernel (0: the graph does not fit it)
    int32_t stop_at_hit;                    // 1: chunk launches sweep no more once the target is
                                            // reached (serving requests)
    int64_t prop_start, prop_period, prop_stop;
    uint64_t sweep_cap;                     // batched runs stop at this sweep count

    // problem
    const int8_t *J3;          // lattice: [3][n] +x,+y,+z bond couplings
    const int32_t *row_ptr;    // CSR [n+1]
    const int16_t *col;        // CSR [nnz]
    const int8_t *Jc;          // CSR [nnz]
    const int16_t *h;          // [n]
    const int8_t *clamp;       // [n]
    const int16_t *color_sites;// CSR: free sites by color, within a color by degree (largest
                               // first), then index [nfree]
    const int32_t *color_off;  // [ncolors + 1]
    const int32_t *csrw_groups;// CSR: rank group (c, k) of the one-slot-per-wavefront sparse
                               // kernel (sites 64k .. 64k + 63 of class c): first chunk << 8 |
                               // chunks, over ceil(largest degree in the group / CSRW_CHUNK)

    // acceptance tables (uint32 thresholds, built on the host in FP64)
    const uint32_t *tflip;     // [R][tflip_stride]
    const uint32_t *tprop;     // row r: entries for d = 1..tprop_len[r] at tprop_off[r]
    const int32_t *tprop_off, *tprop_len;
    const uint32_t *tswap;     // pair r: entries for d = 1..tswap_len[r] at tswap_off[r]
    const int32_t *tswap_off, *tswap_len;

    // state (slot order)
    int8_t *spins;             // [R][n]
    int32_t *E;                // [R]
    unsigned long long *t;     // completed sweeps
    int32_t *cursor;           // [R]

    // proposal banks
    const int8_t *const *bank; // [R] device pointers, null = slot not proposal-enabled
    const int32_t *const *bankE;
    const int32_t *bank_n;     // [R]

    // counters
    unsigned long long *swap_att, *swap_acc;   // [R-1]
    unsigned long long *prop_att, *prop_acc;   // [R]
    unsigned long long *flips;                 // [R]

    BestRec *best;             // canonical record
    int8_t *best_spins;        // [n]
};

// The sweep count a chunk launch may take an instance to: its cap, or where it
// stands if it stops at its target and has reached it (the canonical record
// changes only in the finish kernel, so every launch of a round sees the same).
__device__ inline uint64_t chunk_cap(const InstDev &I, uint64_t t0)
{
    return (I.stop_at_hit && I.best->first_hit >= 0) ? t0 : I.sweep_cap;
}

// The record of a workgroup that sweeps nothing in a launch: it merges as
// nothing in the finish kernel (its buffer may hold another layout's record).
__device__ inline void idle_best(BestRec *b)
{
    b->E = 0x7FFFFFFF;
    b->slot = -1;
    b->t = -1;
    b->first_hit = -1;
    b->pad = 0;
}

struct WorkItem {              // one workgroup of a persistent chunk launch
    const InstDev *inst;
    int32_t s0, G;             // beta slots [s0, s0 + G) held by this workgroup
    int32_t w, W;              // index of this workgroup in the instance's ladder split
    BestRec *best;             // this workgroup's record for the chunk
    int8_t *best_spins;        // [n]
    unsigned long long *xbuf;  // instance exchange area: [W][2 sides][2 buffers][xwords]
    int32_t xwords;            // 64-bit words per buffer: ceil(n/32) spin words + energy, padded
    int32_t variant;           // sweeper of the item in a mixed launch (chunk_kernel_mixed)
};

struct InstStatus {            // per-instance progress written after every chunk
    int64_t t;                 // completed sweeps
    int64_t best_t;
    int64_t first_hit;
    int32_t best_E;
    int32_t best_slot;
};

struct ChunkArgs {
    const WorkItem *items;
    const int32_t *order;      // blockIdx -> item index (XCD-aware placement)
    int32_t n_items;
    uint32_t K;                // sweeps per launch
    int32_t *err;              // [8]: err[0] = 1 when a cross-workgroup wait timed out,
                               // err[1..7] = item, w, side, cycle, seen tag lo/hi, epoch
    uint32_t spin_limit;       // polls before a wait gives up
    int32_t tsw_entries;       // LDS swap-table capacity (entries) of every workgroup
};

} // namespace tapt
