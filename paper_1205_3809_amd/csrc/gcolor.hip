// Speculative iterative distance-1 colouring for gfx950 (MI355X).
//
// Method: the iterative parallel colouring of Catalyurek et al. (Algorithm 2:
// rounds of tentative first-fit colouring of a worklist, then conflict
// detection that re-queues the later vertex of each conflicting edge), run
// round-synchronously: phase 1 reads only colours committed in earlier rounds,
// so the result is a pure function of (graph, priority).
//
// Two engines compute that same function:
//
//  * plain: each round rescans every worklist row in both phases, exactly as
//    the two parallel loops of Algorithm 2 do.  Kernels k_phase1 (tentative
//    first-fit against committed neighbour colours) and k_phase2 (conflict
//    detection, commit of winners, compaction of losers into the next
//    worklist).
//
//  * incremental (default): keeps per uncoloured vertex its tentative colour
//    and conf[v] = number of preceding worklist neighbours holding the same
//    tentative colour; a vertex loses a round exactly when conf[v] > 0.  Only
//    events change this state.  A commit of colour t marks "dirty" each
//    uncoloured neighbour whose tentative colour is t (its tentative colour
//    must move); a dirty vertex re-takes first-fit over its row and has its
//    counter recounted, and its later neighbours adjust their counters by +-1.
//    Tentative colours of other vertices cannot change (their forbidden sets
//    only grew by colours they do not hold), so rounds are the plain engine's,
//    vertex for vertex.  Kernels per round: k_inc_a (first-fit of dirty
//    vertices, counter recount and updates, candidate list, and for a dirty
//    vertex with dirty preceding neighbours the list of those neighbours) and
//    k_inc_c (counters completed for dirty vertices with dirty preceding
//    neighbours, from those lists or by rescanning the row, commit of
//    candidates whose counter is 0, dirty marks to neighbours).
//    A vertex's state word holds its tentative colour while it is uncoloured
//    and minus its colour once committed, so one gather of a neighbour's word
//    answers both "committed, with which colour" and "same tentative colour".
//
// A third engine computes a different function: the dataflow algorithm
// (Algorithm 3) in rounds (GCOLOR_DATAFLOW; k_flow_seed, k_flow), whose result
// is the serial first-fit in (priority, id) order.
//
// Degree bins (the vertex-to-lane mapping of every row-scanning kernel):
//   bin 0: one lane per vertex         bin 1: 4 lanes per vertex
//   bin 2: 16 lanes per vertex         bin 3: one wavefront (64 lanes)
//   bin 4: one workgroup (256 lanes)
// Lanes of a group stride over the row (coalesced CSR reads); first-fit builds
// a 64-colour window bitset per lane, ORs it across the group with shuffles
// (LDS across the waves of bin 4) and takes ctz(~mask); a full window moves
// on to the next 64 colours.
//
// List appends go through a per-workgroup LDS stage (wave ballot + LDS
// atomic), flushed to the global lists with one global atomic per bin; global
// atomics on a shared counter are ~300x slower than LDS ones on this chip.
//
// Each kernel is one launch of a fixed grid; blocks walk a chunk space that
// concatenates the bins (heaviest first), so hubs spread across the chip.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <vector>

#include "gcolor.h"

namespace {

// Load the next chunks' vertex data ahead in the dirty-vertex kernel.
#ifndef GC_PREFETCH_A
#define GC_PREFETCH_A 1
#endif

constexpr int kBlock = 256;
constexpr int kWave = 64;
// Rows longer than this (the register cache of a wave) keep an active copy in
// the wave and workgroup tiers of the incremental engine.
constexpr int kHeavyDeg = 512;
// Words per heavy row of the dropped-colour bitmap: colours 1..64, then
// 65..4160, then padding.
constexpr int kFW = 132;
constexpr int kBins = 5;
constexpr int kSets = 6;          // list sets (plain: 0,1 worklist ping-pong; incremental: see below)
constexpr int kMaxLog = 1 << 16;  // rounds recorded in the device log
constexpr int kLogW = 5;          // int64 words per logged round
constexpr int kSeedBlocksPerCu = 16;  // workgroups per CU of the seed kernels
constexpr int kSumShift = 9;      // dirty-bitmap summary: one flag per 512 words (16384 vertices)
// Pair lists: a start below 2^kPairShift and a count below 2^(31 - kPairShift)
// packed into one non-negative int.
constexpr int kPairShift = 24;
constexpr int kPairMaxCap = 1 << kPairShift;
constexpr int kPairMaxCount = (1 << (31 - kPairShift)) - 1;

// Vertices covered by one block-sized chunk of each bin.
__host__ __device__ constexpr int chunk_vertices(int b) {
    return b == 0 ? 256 : b == 1 ? 64 : b == 2 ? 16 : b == 3 ? 4 : 1;
}

// LDS stage capacity per bin and offsets into the stage array.
__host__ __device__ constexpr int stage_cap(int b) {
    return b == 0 ? 1024 : b == 1 ? 512 : b == 2 ? 256 : b == 3 ? 128 : 64;
}
__host__ __device__ constexpr int stage_off(int b) {
    return b == 0 ? 0 : b == 1 ? 1024 : b == 2 ? 1536 : b == 3 ? 1792 : 1920;
}
constexpr int kStageTotal = 1984;

struct BinCfg {
    int dmax[4];  // bin b (b < 4) holds degrees <= dmax[b]; bin 4 the rest
};

struct Ctl {
    int32_t cnt[8][8];      // [list set][bin] list lengths
    int32_t rounds;         // last round that committed a vertex
    int32_t err;            // validation error bits
    int32_t maxcolor;
    int32_t maxdeg;
    unsigned long long committed;  // vertices committed so far
    int32_t nheavy;                // (incremental) rows with an active copy
    int32_t binpop[kBins];         // vertices whose degree falls in each bin
    int32_t widened;               // (stream-ordered) the state words moved to 32 bits
    int32_t pad[3];
};
static_assert(sizeof(Ctl) == 320, "ctl layout");

struct Args {
    int n;
    const int* __restrict__ row_ptr;
    const int* __restrict__ colp;  // original col_idx, or the reordered copy
    int* __restrict__ split;       // entries at the front of each row that precede the vertex (the
                                   // incremental engine copies them into its vertex records)
    int* __restrict__ color;       // the caller's colors_out (incremental engine: written after the rounds)
    int* __restrict__ tent;        // (plain) tentative colour
    void* st;                      // (incremental) state words, int8_t, int16_t or int32_t
    int* __restrict__ conf;        // (dataflow) preceding entries still uncoloured; the incremental
                                   // engine keeps its counters in the vertex records
    int* __restrict__ cflag;       // (incremental) round of last candidate mark
    int* __restrict__ lists;       // [kSets][n], bins at the offsets of their populations
    unsigned* __restrict__ dbits;  // (incremental) 3 dirty bitmaps of nwords words
    unsigned* __restrict__ bplane; // (incremental) each vertex's degree bin as 3 bit planes of nwords words
    int nwords;
    Ctl* ctl;
    long long* __restrict__ log;   // [kMaxLog][kLogW]
    BinCfg cfg;
    // (incremental) heavy rows: id per vertex of degree > kHeavyDeg, per id
    // (preceding active, later active, buffer, -) and the dropped-colour
    // bitmap; two active-row buffers indexed like col_idx
    int* __restrict__ hid;
    int4* __restrict__ hrow;
    unsigned* __restrict__ hF;
    int* __restrict__ act;
    long long nnz;
    // sequential finish: rounds stop once at most `tail` vertices are
    // uncoloured (0: rounds to the end)
    int tail;
    const uint32_t* __restrict__ key;  // the priority array (NULL: natural)
    int* __restrict__ bcnt;            // (incremental) per-block bin counts of the dirty-list build
    unsigned char* __restrict__ dsum;  // (incremental) per dirty bitmap: a flag per kSumWords-word region with a mark
    int nregions;                      // regions per bitmap
    // (incremental) dirty preceding neighbours of the dirty vertices whose
    // counter the commit kernel completes: pref[w] = start in pbuf | count
    // << kPairShift, or -1 (the commit kernel then rescans w's preceding
    // entries); pbuf holds pcap ids, an equal region per wavefront
    int* __restrict__ pref;
    int* __restrict__ pbuf;
    int pcap;
    // (incremental) per vertex (row start, row end, split point, counter):
    // the row bounds and split point of a vertex come in one 16-byte load
    int* __restrict__ vrec;
};

struct Stage {
    int cnt[kBins];
    int base[kBins];
    int off[kBins];  // bin offsets inside a list set (from the bin populations)
    int q[kStageTotal];
};

__device__ __forceinline__ int bin_of(int deg, const BinCfg& c) {
    return deg <= c.dmax[0] ? 0 : deg <= c.dmax[1] ? 1 : deg <= c.dmax[2] ? 2 : deg <= c.dmax[3] ? 3 : 4;
}

// Each list set is one n-entry array: bin b starts after the populations of
// bins 0..b-1 (a vertex only ever enters the bin of its degree, and no set
// holds a vertex twice, so a bin never outgrows its population).
__device__ __forceinline__ int bin_offset(const Ctl* ctl, int b) {
    int off = 0;
#pragma unroll
    for (int i = 0; i < kBins - 1; ++i) off += i < b ? ctl->binpop[i] : 0;
    return off;
}

__device__ __forceinline__ int* list_ptr(const Args& a, int set, int b) {
    return a.lists + (size_t)set * (size_t)a.n + bin_offset(a.ctl, b);
}

// All bin offsets at once (four independent loads, issued together).
__device__ __forceinline__ void bin_offsets(const Ctl* ctl, int* off) {
    const int p0 = ctl->binpop[0], p1 = ctl->binpop[1], p2 = ctl->binpop[2], p3 = ctl->binpop[3];
    off[0] = 0;
    off[1] = p0;
    off[2] = p0 + p1;
    off[3] = p0 + p1 + p2;
    off[4] = p0 + p1 + p2 + p3;
}

template <int GS>
__device__ __forceinline__ uint64_t group_or(uint64_t m) {
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) m |= __shfl_xor(m, o, GS);
    return m;
}

template <int GS>
__device__ __forceinline__ int group_sum(int x) {
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, GS);
    return x;
}

// Bits of `ballot` belonging to this lane's group of GS lanes.
template <int GS>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int lane) {
    if constexpr (GS == 64) {
        return ballot;
    } else {
        const int gbase = lane & ~(GS - 1);
        return (ballot >> gbase) & ((1ull << GS) - 1ull);
    }
}

// Per-wavefront list stage of the incremental round kernels: each wavefront
// walks its own chunks and flushes its own stage, with no workgroup barrier.
constexpr int kWaves = kBlock / kWave;
__host__ __device__ constexpr int wstage_cap(int b) {
    return b == 0 ? 512 : b == 1 ? 256 : b == 2 ? 128 : b == 3 ? 64 : 32;
}
__host__ __device__ constexpr int wstage_off(int b) {
    return b == 0 ? 0 : b == 1 ? 512 : b == 2 ? 768 : b == 3 ? 896 : 960;
}
constexpr int kWStageTotal = 992;

struct WaveStage {
    int cnt[kBins];
    int base[kBins];
    int off[kBins];  // bin offsets inside a list set (from the bin populations)
    int pbase, pfill, plen;  // (dirty-vertex kernel) this wavefront's pair region: start, used, size
    int q[kWStageTotal];
};

__device__ __forceinline__ int scap(const Stage*, int b) { return stage_cap(b); }
__device__ __forceinline__ int soff(const Stage*, int b) { return stage_off(b); }
__device__ __forceinline__ int scap(const WaveStage*, int b) { return wstage_cap(b); }
__device__ __forceinline__ int soff(const WaveStage*, int b) { return wstage_off(b); }

// Lanes of one wavefront see each other's LDS writes after this.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void stage_init(const Args& a, Stage* st) {
    if (threadIdx.x < kBins) {
        st->cnt[threadIdx.x] = 0;
        st->off[threadIdx.x] = bin_offset(a.ctl, threadIdx.x);
    }
    __syncthreads();
}

// Staged append of the active lanes with pred set into bin b of list set
// `set`: one LDS atomic per wavefront and bin; entries beyond the stage
// capacity go straight to the global list.  Safe in divergent code: every
// active lane must call it, the leader of each ballot is an active lane.
template <class ST>
__device__ __forceinline__ void stage_append(const Args& a, ST* st, bool pred, int v, int deg, int set) {
    const uint64_t any = __ballot(pred);
    if (any == 0) return;
    const int b = pred ? bin_of(deg, a.cfg) : -1;
    const int lane = __lane_id();
#pragma unroll
    for (int k = 0; k < kBins; ++k) {
        const uint64_t m = __ballot(b == k);
        if (m == 0) continue;
        const int leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&st->cnt[k], __popcll(m));
        base = __shfl(base, leader);
        if (b == k) {
            const int slot = base + __popcll(m & __lanemask_lt());
            if (slot < scap(st, k)) {
                st->q[soff(st, k) + slot] = v;
            } else {
                const int g = atomicAdd(&a.ctl->cnt[set][k], 1);
                a.lists[(size_t)set * (size_t)a.n + st->off[k] + g] = v;
            }
        }
    }
}

// Staged append of one vertex by one lane (sparse appends from inside row
// loops): a per-lane LDS atomic, no wavefront-wide ballots.
template <class ST>
__device__ __forceinline__ void stage_push(const Args& a, ST* st, int v, int deg, int set) {
    const int k = bin_of(deg, a.cfg);
    const int slot = atomicAdd(&st->cnt[k], 1);
    if (slot < scap(st, k)) {
        st->q[soff(st, k) + slot] = v;
    } else {
        const int g = atomicAdd(&a.ctl->cnt[set][k], 1);
        a.lists[(size_t)set * (size_t)a.n + st->off[k] + g] = v;
    }
}

// Staged append where the degree must still be looked up.
template <class ST>
__device__ __forceinline__ void stage_append_lookup(const Args& a, ST* st, bool pred, int v, int set) {
    if (pred) stage_push(a, st, v, a.row_ptr[v + 1] - a.row_ptr[v], set);
}

// Per-wavefront stage: clear (wave-uniform call).
__device__ __forceinline__ void wstage_init(const Args& a, WaveStage* st) {
    if (__lane_id() < kBins) {
        st->cnt[__lane_id()] = 0;
        st->off[__lane_id()] = bin_offset(a.ctl, __lane_id());
    }
    wave_sync();
}

// Move a wavefront's staged entries to the global lists (wave-uniform call).
__device__ __forceinline__ void wstage_flush(const Args& a, WaveStage* st, int set) {
    wave_sync();
    const int lane = __lane_id();
    if (lane < kBins) {
        const int c = min(st->cnt[lane], wstage_cap(lane));
        st->base[lane] = c ? atomicAdd(&a.ctl->cnt[set][lane], c) : 0;
        st->cnt[lane] = c;
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        int* dst = a.lists + (size_t)set * (size_t)a.n + st->off[b] + st->base[b];
        for (int i = lane; i < st->cnt[b]; i += kWave) dst[i] = st->q[wstage_off(b) + i];
    }
    wave_sync();
    if (lane < kBins) st->cnt[lane] = 0;
    wave_sync();
}

// Flush when any bin of the wavefront's stage is at least half full.
__device__ __forceinline__ void wstage_maybe_flush(const Args& a, WaveStage* st, int set) {
    wave_sync();
    bool full = false;
#pragma unroll
    for (int b = 0; b < kBins; ++b) full |= st->cnt[b] * 2 >= wstage_cap(b);
    if (full) wstage_flush(a, st, set);
}

// Move the staged entries to the global lists (block-uniform call).
__device__ __forceinline__ void stage_flush(const Args& a, Stage* st, int set) {
    __syncthreads();
    if (threadIdx.x < kBins) {
        const int b = threadIdx.x;
        const int c = min(st->cnt[b], stage_cap(b));
        st->base[b] = c ? atomicAdd(&a.ctl->cnt[set][b], c) : 0;
        st->cnt[b] = c;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        int* dst = a.lists + (size_t)set * (size_t)a.n + st->off[b] + st->base[b];
        for (int i = threadIdx.x; i < st->cnt[b]; i += blockDim.x) dst[i] = st->q[stage_off(b) + i];
    }
    __syncthreads();
    if (threadIdx.x < kBins) st->cnt[threadIdx.x] = 0;
    __syncthreads();
}

// Flush when any bin is at least half full (block-uniform call).
__device__ __forceinline__ void stage_maybe_flush(const Args& a, Stage* st, int set) {
    __syncthreads();
    bool full = false;
#pragma unroll
    for (int b = 0; b < kBins; ++b) full |= st->cnt[b] * 2 >= stage_cap(b);
    if (full) stage_flush(a, st, set);
}

struct ChunkMap {
    int cnt[kBins];
    int start[kBins];  // chunk-space start of each bin; bins ordered 4,3,2,1,0
    int off[kBins];    // bin offsets inside the set's array
    int total;
};

__device__ __forceinline__ ChunkMap make_map(const Ctl* ctl, int set) {
    ChunkMap m;
    int tot = 0;
    for (int b = kBins - 1; b >= 0; --b) {
        m.cnt[b] = ctl->cnt[set][b];
        m.start[b] = tot;
        tot += (m.cnt[b] + chunk_vertices(b) - 1) / chunk_vertices(b);
    }
    int off = 0;
    for (int b = 0; b < kBins; ++b) {
        m.off[b] = off;
        off += ctl->binpop[b];
    }
    m.total = tot;
    return m;
}

__device__ __forceinline__ int chunk_bin(const ChunkMap& m, int c) {
    // bins occupy [start[4], start[3]), [start[3], start[2]), ... in that order
    return 4 - (c >= m.start[3]) - (c >= m.start[2]) - (c >= m.start[1]) - (c >= m.start[0]);
}

// m.start[b] / m.cnt[b] without dynamic register indexing.
__device__ __forceinline__ int pick5(const int* x, int b) {
    return b == 0 ? x[0] : b == 1 ? x[1] : b == 2 ? x[2] : b == 3 ? x[3] : x[4];
}

// Smallest colour >= base not held by a committed neighbour in the row
// [s, e).  Uncommitted neighbours hold 0, which no window contains.
template <int GS>
__device__ __forceinline__ int first_fit_group(int s, int e, int lig, int base, const int* __restrict__ colp,
                                               const int* __restrict__ color) {
    for (;;) {
        uint64_t m = 0;
        int p = s + lig;
        for (; p + 3 * GS < e; p += 4 * GS) {
            const int w0 = colp[p], w1 = colp[p + GS], w2 = colp[p + 2 * GS], w3 = colp[p + 3 * GS];
            const unsigned c0 = (unsigned)(color[w0] - base);
            const unsigned c1 = (unsigned)(color[w1] - base);
            const unsigned c2 = (unsigned)(color[w2] - base);
            const unsigned c3 = (unsigned)(color[w3] - base);
            if (c0 < 64u) m |= 1ull << c0;
            if (c1 < 64u) m |= 1ull << c1;
            if (c2 < 64u) m |= 1ull << c2;
            if (c3 < 64u) m |= 1ull << c3;
        }
        for (; p < e; p += GS) {
            const unsigned c = (unsigned)(color[colp[p]] - base);
            if (c < 64u) m |= 1ull << c;
        }
        m = group_or<GS>(m);
        if (~m) return base + __builtin_ctzll(~m);
        base += 64;
    }
}

// Block-wide version for bin 4 (red: 4 words of LDS).
__device__ __forceinline__ int first_fit_block(int s, int e, int base, const int* __restrict__ colp,
                                               const int* __restrict__ color, uint64_t* red) {
    const int wid = threadIdx.x / kWave;
    for (;;) {
        uint64_t m = 0;
        for (int p = s + (int)threadIdx.x; p < e; p += kBlock) {
            const unsigned c = (unsigned)(color[colp[p]] - base);
            if (c < 64u) m |= 1ull << c;
        }
        m = group_or<kWave>(m);
        if (__lane_id() == 0) red[wid] = m;
        __syncthreads();
        const uint64_t all = red[0] | red[1] | red[2] | red[3];
        __syncthreads();
        if (~all) return base + __builtin_ctzll(~all);
        base += 64;
    }
}

// Walk the chunk space of list set SET: each chunk runs BODY_GS(GS, list,
// count, local chunk index) for the group bins or BODY_BLOCK(vertex) for
// the workgroup bin, then AFTER() (block-uniform).
#define GC_FOR_CHUNKS(A, SET, BODY_GS, BODY_BLOCK, AFTER)                              \
    {                                                                                  \
        const ChunkMap m_ = make_map((A).ctl, (SET));                                  \
        for (int c_ = blockIdx.x; c_ < m_.total; c_ += gridDim.x) {                     \
            const int b_ = chunk_bin(m_, c_);                                          \
            const int local_ = c_ - pick5(m_.start, b_);                                      \
            const int* list_ = (A).lists + (size_t)(SET) * (size_t)(A).n + pick5(m_.off, b_); \
            const int cnt_ = pick5(m_.cnt, b_);                                               \
            switch (b_) {                                                              \
                case 0: BODY_GS(1, list_, cnt_, local_); break;                        \
                case 1: BODY_GS(4, list_, cnt_, local_); break;                        \
                case 2: BODY_GS(16, list_, cnt_, local_); break;                       \
                case 3: BODY_GS(64, list_, cnt_, local_); break;                       \
                default: BODY_BLOCK(list_[local_]); break;                             \
            }                                                                          \
            AFTER();                                                                   \
        }                                                                              \
    }

// Same walk over a chunk map computed beforehand.
#define GC_WALK_CHUNKS(A, M, SET, BODY_GS, BODY_BLOCK, AFTER)                          \
    {                                                                                  \
        for (int c_ = blockIdx.x; c_ < (M).total; c_ += gridDim.x) {                    \
            const int b_ = chunk_bin((M), c_);                                         \
            const int local_ = c_ - pick5((M).start, b_);                                     \
            const int* list_ = (A).lists + (size_t)(SET) * (size_t)(A).n + pick5((M).off, b_); \
            const int cnt_ = pick5((M).cnt, b_);                                              \
            switch (b_) {                                                              \
                case 0: BODY_GS(1, list_, cnt_, local_); break;                        \
                case 1: BODY_GS(4, list_, cnt_, local_); break;                        \
                case 2: BODY_GS(16, list_, cnt_, local_); break;                       \
                case 3: BODY_GS(64, list_, cnt_, local_); break;                       \
                default: BODY_BLOCK(list_[local_]); break;                             \
            }                                                                          \
            AFTER();                                                                   \
        }                                                                              \
    }

#define GC_NOTHING() \
    do {             \
    } while (0)

__device__ __forceinline__ void block_add_log(long long x, long long* slot) {
    __shared__ long long part[kBlock / kWave];
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    __syncthreads();
    if (__lane_id() == 0) part[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd((unsigned long long*)slot, (unsigned long long)t);
    }
}

// ===========================================================================
// Plain engine (rounds k = 0, 1, ... on worklist sets k & 1)
// ===========================================================================

template <int GS>
__device__ __forceinline__ void phase1_chunk(const Args& a, const int* list, int cnt, int local) {
    constexpr int CV = kBlock / GS;
    const int lig = threadIdx.x & (GS - 1);
    const int idx = local * CV + (int)threadIdx.x / GS;
    if (idx < cnt) {
        const int v = list[idx];
        const int t = first_fit_group<GS>(a.row_ptr[v], a.row_ptr[v + 1], lig, 1, a.colp, a.color);
        if (lig == 0) a.tent[v] = t;
    }
}

// Phase 1 of round k over worklist set `side`: tentative first-fit.
__global__ __launch_bounds__(kBlock) void k_phase1(Args a, int side, int k) {
    __shared__ uint64_t red[kBlock / kWave];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int usize = 0;
        for (int b = 0; b < kBins; ++b) usize += a.ctl->cnt[side][b];
        for (int b = 0; b < 8; ++b) a.ctl->cnt[side ^ 1][b] = 0;
        if (usize > 0) {
            a.ctl->rounds = k + 1;
            if (k < kMaxLog) {
                a.log[kLogW * k] = usize;
                a.log[kLogW * k + 1] = 0;
            }
        }
    }
    const ChunkMap m = make_map(a.ctl, side);
    if ((int)blockIdx.x >= m.total) return;
#define P1_GS(GS, L, C, LOC) phase1_chunk<GS>(a, L, C, LOC)
#define P1_BLOCK(V)                                                                                \
    {                                                                                              \
        const int v_ = (V);                                                                        \
        const int t_ = first_fit_block(a.row_ptr[v_], a.row_ptr[v_ + 1], 1, a.colp, a.color, red); \
        if (threadIdx.x == 0) a.tent[v_] = t_;                                                     \
    }
    GC_WALK_CHUNKS(a, m, side, P1_GS, P1_BLOCK, GC_NOTHING)
#undef P1_GS
#undef P1_BLOCK
}

// Does some entry of the preceding prefix [s, lim) hold tentative colour t?
// Neighbours committed in earlier rounds cannot: phase 1 avoided their colours.
template <int GS>
__device__ __forceinline__ bool loses_group(int s, int lim, int t, int lig, int lane,
                                            const int* __restrict__ colp, const int* __restrict__ tent) {
    for (int p0 = s; p0 < lim; p0 += GS) {
        const int p = p0 + lig;
        const bool hit = (p < lim) && (tent[colp[p]] == t);
        if constexpr (GS == 1) {
            if (hit) return true;
        } else {
            if (group_bits<GS>(__ballot(hit), lane)) return true;
        }
    }
    return false;
}

template <int GS>
__device__ __forceinline__ void phase2_chunk(const Args& a, Stage* st, const int* list, int cnt, int local,
                                             int nside, long long* ework) {
    constexpr int CV = kBlock / GS;
    const int lane = __lane_id();
    const int lig = threadIdx.x & (GS - 1);
    const int idx = local * CV + (int)threadIdx.x / GS;
    bool lose = false;
    int v = 0, deg = 0;
    if (idx < cnt) {
        v = list[idx];
        const int s = a.row_ptr[v];
        deg = a.row_ptr[v + 1] - s;
        if (lig == 0) *ework += deg;
        const int t = a.tent[v];
        lose = loses_group<GS>(s, s + a.split[v], t, lig, lane, a.colp, a.tent);
        if (!lose && lig == 0) a.color[v] = t;
    }
    stage_append(a, st, lose && lig == 0, v, deg, nside);
}

__device__ __forceinline__ void phase2_block(const Args& a, Stage* st, int v, int nside, long long* ework) {
    const int s = a.row_ptr[v];
    const int lim = s + a.split[v];
    const int t = a.tent[v];
    bool lose = false;
    for (int p0 = s; p0 < lim; p0 += kBlock) {
        const int p = p0 + (int)threadIdx.x;
        const int hit = (p < lim) && (a.tent[a.colp[p]] == t);
        if (__syncthreads_or(hit)) {
            lose = true;
            break;
        }
    }
    const int deg = a.row_ptr[v + 1] - s;
    if (threadIdx.x == 0) {
        *ework += deg;
        if (!lose) a.color[v] = t;
    }
    if (threadIdx.x < kWave) stage_append(a, st, lose && threadIdx.x == 0, v, deg, nside);
}

// Phase 2 of round k: conflict detection, commit, compaction into side^1.
__global__ __launch_bounds__(kBlock) void k_phase2(Args a, int side, int k) {
    __shared__ Stage st;
    const ChunkMap m = make_map(a.ctl, side);
    if ((int)blockIdx.x >= m.total) return;
    stage_init(a, &st);
    const int nside = side ^ 1;
    long long ework = 0;
#define P2_GS(GS, L, C, LOC) phase2_chunk<GS>(a, &st, L, C, LOC, nside, &ework)
#define P2_BLOCK(V) phase2_block(a, &st, (V), nside, &ework)
#define P2_AFTER() stage_maybe_flush(a, &st, nside)
    GC_WALK_CHUNKS(a, m, side, P2_GS, P2_BLOCK, P2_AFTER)
#undef P2_GS
#undef P2_BLOCK
#undef P2_AFTER
    stage_flush(a, &st, nside);
    if (k < kMaxLog) block_add_log(ework, &a.log[kLogW * k + 1]);
}

// ===========================================================================
// Incremental engine (rounds k = 1, 2, ...; round 1 needs only k_inc_c)
//
// One signed state word per vertex: S = int8_t for rounds 1..127 (no
// colour can exceed the round number), then int16_t, or int32_t when max
// degree + 1 exceeds 32767:
//   st[v] > 0   v is uncoloured, st[v] is its tentative colour
//   st[v] < 0   v is committed with colour -st[v]
// so a single gather of a neighbour's word answers every question a kernel
// asks about it.  colors_out is written once, from the state words, after
// the last round (k_inc_colors): the commits write only state words.
//
// Round k:
//   k_inc_a  for each dirty vertex w (tentative colour must move): one scan
//            of its row gives the new tentative colour (first-fit over the
//            committed words) and, from the same gathered words, the count
//            of preceding clean neighbours holding the new colour; later
//            clean neighbours holding the old or the new colour get their
//            counters adjusted by -1 / +1.  Dirty neighbours are recognised
//            in a one-bit-per-vertex bitmap (L2 resident).  A dirty vertex
//            with a preceding dirty neighbour joins the candidate list as ~w.
//   k_inc_c  completes, for each ~w, the counter with the preceding dirty
//            neighbours holding w's new colour (final since k_inc_a; one
//            committed in this kernel shows -t, so the count takes |word|);
//            then commits every candidate whose counter is 0 and marks
//            dirty each later neighbour holding the same tentative colour
//            (a preceding one cannot: it would have kept the counter above
//            0).
// List sets: dirty lists rotate over 3 sets (k % 3) with their bitmaps, so
// the bits of round k-1 can be cleared during round k; candidate lists
// alternate over 2 sets.
// ===========================================================================

constexpr int kSetCand = 3;  // + (k & 1)

__host__ __device__ inline int dlist(int k) { return k % 3; }
__host__ __device__ inline int cset(int k) { return kSetCand + (k & 1); }

__device__ __forceinline__ unsigned* dbits(const Args& a, int k) {
    return a.dbits + (size_t)dlist(k) * (size_t)a.nwords;
}

__device__ __forceinline__ unsigned char* dsum(const Args& a, int k) {
    return a.dsum + (size_t)dlist(k) * (size_t)a.nregions;
}

__device__ __forceinline__ bool is_dirty(const unsigned* __restrict__ bits, int x) {
    return (bits[x >> 5] >> (x & 31)) & 1u;
}

// Vertex record of the incremental engine: x = row start, y = row end,
// z = split point, w = counter (conf).
__device__ __forceinline__ int4 vrec_load(const Args& a, int v) {
    return reinterpret_cast<const int4*>(a.vrec)[v];
}
__device__ __forceinline__ int* vconf(const Args& a, int v) { return a.vrec + 4 * (size_t)v + 3; }

// Round-1 state: every tentative colour is 1, so conf[v] is the number of
// preceding neighbours; vertices with none are the round-1 candidates.
// Natural order (rows sorted): split[v] = lower_bound(row, v) - row start.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_inc_seed(Args a, int natural) {
    __shared__ Stage stg;
    if (a.ctl->err) return;  // the CSR failed validation: nothing is read
    stage_init(a, &stg);
    S* st = static_cast<S*>(a.st);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int t = 0; t < kSets; ++t)
            if (t != cset(1))
                for (int b = 0; b < 8; ++b) a.ctl->cnt[t][b] = 0;
        for (int i = 0; i < kLogW; ++i) a.log[i] = 0;
    }
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < 3 * a.nwords; i += stride) a.dbits[i] = 0u;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < 3 * a.nregions; i += stride) a.dsum[i] = 0;
    for (int base = blockIdx.x * kBlock; base < a.n; base += stride) {
        const int v = base + (int)threadIdx.x;
        const bool ok = v < a.n;
        int deg = 0, sp = -1;
        if (ok) {
            const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
            deg = e - s;
            if (natural) {
                int lo = s, hi = e;
                while (lo < hi) {
                    const int mid = lo + ((hi - lo) >> 1);
                    if (a.colp[mid] < v) lo = mid + 1;
                    else hi = mid;
                }
                sp = lo - s;
            } else {
                sp = a.split[v];
            }
            st[v] = 1;
            reinterpret_cast<int4*>(a.vrec)[v] = make_int4(s, e, sp, sp);
            a.cflag[v] = 0;
        }
        // heavy rows: an id each (wave-aggregated) and the whole row as the
        // initial active view in the original buffer; the bitmap is written
        // at the first compaction
        const bool heavy = ok && deg > kHeavyDeg;
        const unsigned long long hm = __ballot(heavy);
        if (hm) {
            const int leader = __ffsll((long long)hm) - 1;
            int hb = 0;
            if (__lane_id() == leader) hb = atomicAdd(&a.ctl->nheavy, __popcll(hm));
            hb = __shfl(hb, leader);
            if (heavy) {
                const int h = hb + __popcll(hm & __lanemask_lt());
                a.hid[v] = h;
                a.hrow[h] = make_int4(sp, deg - sp, 0, 0);
            }
        }
        // the degree bin as three bit planes, 32 vertices a word (a
        // wavefront holds 64 consecutive vertices: two words)
        {
            const int bn = ok ? bin_of(deg, a.cfg) : 0;
            const int lane = __lane_id();
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const unsigned long long m = __ballot((bn >> q) & 1);
                const int word = v >> 5;
                if ((lane & 31) == 0 && word < a.nwords)
                    a.bplane[(size_t)q * a.nwords + word] = (unsigned)(lane ? (m >> 32) : m);
            }
        }
        stage_append(a, &stg, ok && sp == 0, v, deg, cset(1));
        stage_maybe_flush(a, &stg, cset(1));
    }
    stage_flush(a, &stg, cset(1));
}

// Colours base..base+63 held by committed neighbours among the entries
// start, start + STRIDE, ... < e of a row, read from the state words
// (committed = negative); four independent gathers in flight per lane.
template <int STRIDE, typename S>
__device__ __forceinline__ uint64_t state_window(int start, int e, int base, const int* __restrict__ colp,
                                                 const S* __restrict__ st) {
    uint64_t m = 0;
    int p = start;
    for (; p + 3 * STRIDE < e; p += 4 * STRIDE) {
        const int w0 = colp[p], w1 = colp[p + STRIDE], w2 = colp[p + 2 * STRIDE], w3 = colp[p + 3 * STRIDE];
        const int x0 = st[w0], x1 = st[w1], x2 = st[w2], x3 = st[w3];
        const unsigned c0 = (unsigned)(-x0 - base), c1 = (unsigned)(-x1 - base);
        const unsigned c2 = (unsigned)(-x2 - base), c3 = (unsigned)(-x3 - base);
        if (c0 < 64u) m |= 1ull << c0;
        if (c1 < 64u) m |= 1ull << c1;
        if (c2 < 64u) m |= 1ull << c2;
        if (c3 < 64u) m |= 1ull << c3;
    }
    for (; p < e; p += STRIDE) {
        const unsigned c = (unsigned)(-(int)st[colp[p]] - base);
        if (c < 64u) m |= 1ull << c;
    }
    return m;
}

// Row entries kept in registers: up to kCache per lane.
constexpr int kCache = 8;

// Long rows (beyond the register cache) of the wave and workgroup tiers:
// first-fit in one pass over the row.  Colours 1..64 collect in a per-lane
// mask, colours 65..64 + kFFBits in an LDS bitmap (one per wave for the wave
// tier).  Returns the first free colour, or 0 when all of 1..64 + kFFBits are
// taken (the caller continues with 64-colour windows above that range).
constexpr int kFFWords = 128;
constexpr int kFFBits = kFFWords * 32;

template <int GS>
__device__ __forceinline__ void group_sync() {
    if constexpr (GS == kBlock) {
        __syncthreads();
    } else {
        static_assert(GS == kWave, "wave or workgroup groups only");
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int GS, typename S>
__device__ __forceinline__ int first_fit_long(const int* __restrict__ colp, const S* __restrict__ st, int start,
                                              int e, unsigned* bm, uint64_t* red, int* shc) {
    const int lig = threadIdx.x & (GS - 1);
    for (int i = lig; i < kFFWords; i += GS) bm[i] = 0u;
    group_sync<GS>();
    uint64_t m = 0;
    for (int p0 = start; p0 < e; p0 += 4 * GS) {
        int x[4], c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * GS;
            x[j] = p < e ? colp[p] : -1;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = x[j] >= 0 ? -(int)st[x[j]] : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned lo = (unsigned)(c[j] - 1), hi = (unsigned)(c[j] - 65);
            if (lo < 64u) m |= 1ull << lo;
            else if (hi < (unsigned)kFFBits) atomicOr(&bm[hi >> 5], 1u << (hi & 31));
        }
    }
    if constexpr (GS == kBlock) {
        m = group_or<kWave>(m);
        if (__lane_id() == 0) red[threadIdx.x / kWave] = m;
        __syncthreads();  // also completes the bitmap
        m = red[0] | red[1] | red[2] | red[3];
    } else {
        m = group_or<GS>(m);
        group_sync<GS>();
    }
    int pos = 0x7fffffff;
    if (~m) {
        pos = __builtin_ctzll(~m) - 64;
    } else {
        for (int i = lig; i < kFFWords; i += GS) {
            const unsigned z = ~bm[i];
            if (z) {
                pos = min(pos, i * 32 + __builtin_ctz(z));
                break;
            }
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) pos = min(pos, __shfl_xor(pos, o));
        if constexpr (GS == kBlock) {
            if (__lane_id() == 0) shc[threadIdx.x / kWave] = pos;
            __syncthreads();
            pos = min(min(shc[0], shc[1]), min(shc[2], shc[3]));
        }
    }
    group_sync<GS>();  // red / shc / bitmap free for reuse
    return pos == 0x7fffffff ? 0 : 65 + pos;
}

// Evaluation of one entry (x with word sx at row position p) of dirty vertex
// w after its new colour `now` is known.  Preceding clean neighbours count
// toward w's counter; later clean neighbours holding old / now get -1 / +1
// (returns true when such a counter just reached 0 for the first time in
// this round: x becomes a candidate).  Dirty neighbours are skipped; a
// preceding one sets *dlow (k_inc_c finishes w's count).
__device__ __forceinline__ bool inc_a_eval(const Args& a, const unsigned* __restrict__ bits, int k, int w, int p,
                                           int lim, int now, int old, int x, int sx, int* cnt, bool* dlow) {
    if (p < lim) {
        // committed words are negative and a dirty vertex's word stays
        // positive while this kernel rewrites it, so the bitmap is read only
        // for uncommitted neighbours
        if (sx > 0 && is_dirty(bits, x)) *dlow = true;
        else *cnt += (sx == now);
        return false;
    }
    if (x == w || (sx != now && sx != old)) return false;
    if (is_dirty(bits, x)) return false;
    if (sx == now) {
        atomicAdd(vconf(a, x), 1);
        return false;
    }
    if (atomicSub(vconf(a, x), 1) != 1) return false;
    return atomicExch(&a.cflag[x], k) != k;
}


// Pair list of a dirty vertex w with dirty preceding neighbours (wavefront
// tier, row in registers: ids xs, the dirty preceding ones in the slots of
// dpm): its group's lanes write those neighbours into the wavefront's region
// of the pair buffer, at offsets from a wavefront-wide prefix over the active
// lanes (counts up to kCache: four ballots), and lane 0 of the group stores
// the list's start and length in pref[w].  A list that does not fit the
// region (or is longer than kPairMaxCount) is stored as -1: the commit kernel
// then rescans w's preceding entries.  Every active lane of the wavefront
// calls this.
template <int GS>
__device__ __forceinline__ void pair_list(const Args& a, WaveStage* stg, int w, const int* xs, unsigned dpm) {
    static_assert(kCache < 16, "counts fit four ballots");
    const int mine = __popc(dpm);
    int pre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t m = __ballot((mine >> q) & 1);
        pre += __popcll(m & __lanemask_lt()) << q;
        tot += __popcll(m) << q;
    }
    if (tot == 0) return;  // wavefront-uniform
    const int fill = stg->pfill;
    const bool fits = fill + tot <= stg->plen;
    const int at = stg->pbase + fill + pre;
    if (fits && mine) {
        int i = 0;
#pragma unroll
        for (int j = 0; j < kCache; ++j)
            if (dpm >> j & 1u) a.pbuf[at + i++] = xs[j];
    }
    const int gtot = group_sum<GS>(mine);
    const int gat = __shfl(at, __lane_id() & ~(GS - 1));
    if (gtot > 0 && (__lane_id() & (GS - 1)) == 0)
        a.pref[w] = fits && gtot <= kPairMaxCount ? gat | (gtot << kPairShift) : -1;
    wave_sync();  // every lane has read pfill
    if (fits && __lane_id() == __ffsll((unsigned long long)__ballot(true)) - 1) stg->pfill = fill + tot;
    wave_sync();
}

// inc_a_eval over N entries of dirty vertex w held in registers (ids xs,
// words sv, at positions start, start + GS, ...; preceding below lim), in
// stages over all of them: every bitmap read, then every counter atomic,
// then the rare flag exchanges, so that a lane keeps its reads and atomics
// in flight together instead of waiting on each entry in turn.  Positions
// from e on hold w itself and are skipped.  *dpm collects the slots j that
// hold a dirty preceding neighbour; with LIST they also form w's pair list.
template <int GS, int N, bool LIST = false>
__device__ __forceinline__ void inc_a_eval_staged(const Args& a, WaveStage* stg, const unsigned* __restrict__ bits, int k,
                                                  int w, int start, int e, int lim, int now, int old, const int* xs,
                                                  const int* sv, int* cnt, bool* dlow, unsigned* dpm) {
    // which entries need their dirty bit: uncommitted preceding neighbours,
    // and later ones (not w) holding now or old
    unsigned need = 0u;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int p = start + j * GS;
        const int sx = sv[j];
        const bool nd = p < e && (p < lim ? sx > 0 : (xs[j] != w && (sx == now || sx == old)));
        need |= (nd ? 1u : 0u) << j;
    }
    unsigned word[N];
#pragma unroll
    for (int j = 0; j < N; ++j) word[j] = (need >> j & 1u) ? bits[xs[j] >> 5] : 0u;
    unsigned addm = 0u, subm = 0u;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int p = start + j * GS;
        if (p >= e) continue;
        const int sx = sv[j];
        const bool dirty = (word[j] >> (xs[j] & 31)) & 1u;
        if (p < lim) {
            if (sx > 0 && dirty) {
                *dlow = true;
                *dpm |= 1u << j;
            } else {
                *cnt += (sx == now);
            }
        } else if ((need >> j & 1u) && !dirty) {
            if (sx == now) addm |= 1u << j;
            else subm |= 1u << j;
        }
    }
    if constexpr (LIST) pair_list<GS>(a, stg, w, xs, *dpm);
    int r[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        r[j] = 0;
        if (addm >> j & 1u) atomicAdd(vconf(a, xs[j]), 1);
        else if (subm >> j & 1u) r[j] = atomicSub(vconf(a, xs[j]), 1);
    }
    unsigned zm = 0u;
#pragma unroll
    for (int j = 0; j < N; ++j) zm |= ((subm >> j & 1u) && r[j] == 1 ? 1u : 0u) << j;
    if (zm == 0u) return;
    int f[N];
#pragma unroll
    for (int j = 0; j < N; ++j) f[j] = (zm >> j & 1u) ? atomicExch(&a.cflag[xs[j]], k) : k;
#pragma unroll
    for (int j = 0; j < N; ++j) stage_append_lookup(a, stg, f[j] != k, xs[j], cset(k));
}

// Heavy rows (degree > kHeavyDeg) in the wave and workgroup tiers keep an
// active copy: the neighbours not committed yet, plus committed ones whose
// colour lies above the bitmap range, in two segments at the row's offsets
// (preceding neighbours at s, later ones at s + split) of one of two buffers;
// the colours of the committed neighbours dropped from it are kept in a
// per-row bitmap (colours 1..64 + kFFBits).  Buffer 0 is the original row.
// The set of uncommitted neighbours is all that the counters and the dirty
// marks look at, and the committed colours only grow, so each dirty visit
// scans the active row instead of the full row; the visit rewrites the
// active row into the other buffer once a quarter of it has committed.
struct HeavyView {
    const int* row;
    int s0, s1;   // segment starts
    int pa, la;   // segment lengths
    int buf, h;
};

__device__ __forceinline__ HeavyView heavy_view(const Args& a, int v, int s, int sp) {
    HeavyView hv;
    hv.h = a.hid[v];
    const int4 r = a.hrow[hv.h];
    hv.pa = r.x;
    hv.la = r.y;
    hv.buf = r.z;
    hv.row = r.z == 0 ? a.colp : a.act + (size_t)(r.z - 1) * (size_t)a.nnz;
    hv.s0 = s;
    hv.s1 = s + sp;
    return hv;
}

// Entry q of the active row (segment 0 first).
__device__ __forceinline__ int hv_at(const HeavyView& hv, int q) {
    return hv.row[q < hv.pa ? hv.s0 + q : hv.s1 + (q - hv.pa)];
}

// Committed colour c (c = minus the state word) of an entry that stays in the
// active row: not committed (c < 0) or beyond the bitmap.
__device__ __forceinline__ bool hv_keep(int c) { return c < 0 || c > 64 + kFFBits; }

// Dirty heavy vertex w: new tentative colour, the per-lane part of its
// counter and of the preceding-dirty flag, the later neighbours' counter
// updates (as inc_a_eval), and the compaction of its active row.
template <int GS, typename S>
__device__ __forceinline__ void inc_a_heavy(const Args& a, WaveStage* stg, int k, int w, int s, int sp, int old, int lig,
                                            uint64_t* red, int* shc, unsigned* bm, int* cc, int* now_out,
                                            int* cnt_out, bool* dlow_out, int* len_out) {
    S* st = static_cast<S*>(a.st);
    const unsigned* bits = dbits(a, k);
    const HeavyView hv = heavy_view(a, w, s, sp);
    const int len = hv.pa + hv.la;
    unsigned* F = a.hF + (size_t)hv.h * kFW;

    // pass 1: forbidden colours (starting from the dropped ones) and the
    // number of entries that stay
    for (int i = lig; i < kFFWords; i += GS) bm[i] = hv.buf ? F[2 + i] : 0u;
    uint64_t m = 0;
    if (hv.buf && lig == 0) m = (uint64_t)F[0] | ((uint64_t)F[1] << 32);
    group_sync<GS>();
    int keep = 0;
    for (int q0 = lig; q0 < len; q0 += 4 * GS) {
        int x[4], c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = q0 + j * GS;
            x[j] = q < len ? hv_at(hv, q) : -1;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = x[j] >= 0 ? -(int)st[x[j]] : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned lo = (unsigned)(c[j] - 1), hi = (unsigned)(c[j] - 65);
            if (lo < 64u) m |= 1ull << lo;
            else if (hi < (unsigned)kFFBits) atomicOr(&bm[hi >> 5], 1u << (hi & 31));
            keep += x[j] >= 0 && hv_keep(c[j]);
        }
    }
    if constexpr (GS == kBlock) {
        m = group_or<kWave>(m);
        keep = group_sum<kWave>(keep);
        if (__lane_id() == 0) {
            red[threadIdx.x / kWave] = m;
            shc[threadIdx.x / kWave] = keep;
        }
        __syncthreads();  // also completes the bitmap
        m = red[0] | red[1] | red[2] | red[3];
        keep = shc[0] + shc[1] + shc[2] + shc[3];
        __syncthreads();
    } else {
        m = group_or<GS>(m);
        keep = group_sum<GS>(keep);
        group_sync<GS>();
    }
    int pos = 0x7fffffff;
    if (~m) {
        pos = __builtin_ctzll(~m) - 64;
    } else {
        for (int i = lig; i < kFFWords; i += GS) {
            const unsigned z = ~bm[i];
            if (z) {
                pos = min(pos, i * 32 + __builtin_ctz(z));
                break;
            }
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) pos = min(pos, __shfl_xor(pos, o));
        if constexpr (GS == kBlock) {
            if (__lane_id() == 0) shc[threadIdx.x / kWave] = pos;
            __syncthreads();
            pos = min(min(shc[0], shc[1]), min(shc[2], shc[3]));
        }
    }
    const bool compact = keep * 4 <= len * 3;
    if (compact) {
        if (lig == 0) {
            F[0] = (unsigned)m;
            F[1] = (unsigned)(m >> 32);
        }
        for (int i = lig; i < kFFWords; i += GS) F[2 + i] = bm[i];
    }
    group_sync<GS>();  // bitmap, red and shc free again
    int now = pos == 0x7fffffff ? 0 : 65 + pos;
    // every colour up to 64 + kFFBits taken: 64-colour windows above, over
    // the active row (colours there are never dropped)
    for (int base = 65 + kFFBits; now == 0; base += 64) {
        uint64_t wm = 0;
        for (int q = lig; q < len; q += GS) {
            const unsigned c = (unsigned)(-(int)st[hv_at(hv, q)] - base);
            if (c < 64u) wm |= 1ull << c;
        }
        if constexpr (GS == kBlock) {
            wm = group_or<kWave>(wm);
            if (__lane_id() == 0) red[threadIdx.x / kWave] = wm;
            __syncthreads();
            wm = red[0] | red[1] | red[2] | red[3];
            __syncthreads();
        } else {
            wm = group_or<GS>(wm);
        }
        if (~wm) now = base + __builtin_ctzll(~wm);
    }

    // pass 2: counters, and the kept entries into the other buffer (any
    // order within a segment: positions from ballots)
    const int dbuf = hv.buf == 1 ? 2 : 1;
    int* dst = a.act + (size_t)(dbuf - 1) * (size_t)a.nnz;
    int n0 = 0, n1 = 0;
    if constexpr (GS == kBlock) {
        if (compact) {
            if (threadIdx.x == 0) {
                cc[0] = 0;
                cc[1] = 0;
            }
            __syncthreads();
        }
    }
    int cnt = 0;
    bool dlow = false;
    for (int qb = 0; qb < len; qb += 4 * GS) {
        int x[4], sx[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = qb + lig + j * GS;
            x[j] = q < len ? hv_at(hv, q) : w;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) sx[j] = st[x[j]];
        unsigned dpm = 0u;
        inc_a_eval_staged<GS, 4>(a, stg, bits, k, w, qb + lig, len, hv.pa, now, old, x, sx, &cnt, &dlow, &dpm);
        if (compact) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = qb + lig + j * GS;
                const bool ok = q < len;
                const bool kp = ok && hv_keep(-sx[j]);
                const bool pre = q < hv.pa;
                const unsigned long long m0 = __ballot(kp && pre), m1 = __ballot(kp && !pre);
                int b0, b1;
                if constexpr (GS == kBlock) {
                    int t0 = 0, t1 = 0;
                    if (__lane_id() == 0) {
                        if (m0) t0 = atomicAdd(&cc[0], __popcll(m0));
                        if (m1) t1 = atomicAdd(&cc[1], __popcll(m1));
                    }
                    b0 = __shfl(t0, 0);
                    b1 = __shfl(t1, 0);
                } else {
                    b0 = n0;
                    b1 = n1;
                    n0 += __popcll(m0);
                    n1 += __popcll(m1);
                }
                const unsigned long long lt = __lanemask_lt();
                if (kp) dst[pre ? hv.s0 + b0 + __popcll(m0 & lt) : hv.s1 + b1 + __popcll(m1 & lt)] = x[j];
            }
        }
    }
    if (compact) {
        if constexpr (GS == kBlock) {
            __syncthreads();
            if (threadIdx.x == 0) a.hrow[hv.h] = make_int4(cc[0], cc[1], dbuf, 0);
        } else {
            if (lig == 0) a.hrow[hv.h] = make_int4(n0, n1, dbuf, 0);
        }
    }
    *now_out = now;
    *cnt_out = cnt;
    *dlow_out = dlow;
    *len_out = len;
}

// Second pass over a row too long for the register cache: re-gather.
template <int STRIDE, typename S>
__device__ __forceinline__ void inc_a_pass2_gather(const Args& a, WaveStage* stg, const S* __restrict__ st,
                                                   const unsigned* __restrict__ bits, int k, int w, int start, int e,
                                                   int lim, int now, int old, int* cnt, bool* dlow) {
    const int cs = cset(k);
    for (int p0 = start; p0 < e; p0 += 4 * STRIDE) {
        int x[4], sx[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * STRIDE;
            x[j] = p < e ? a.colp[p] : w;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) sx[j] = st[x[j]];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * STRIDE;
            const bool cand = (p < e) && inc_a_eval(a, bits, k, w, p, lim, now, old, x[j], sx[j], cnt, dlow);
            stage_append_lookup(a, stg, cand, x[j], cs);
        }
    }
}

// Dirty vertex w handled by a group of GS lanes (GS = kBlock: the whole
// workgroup, with LDS for the reductions).  Returns via the stage: w itself
// to the candidate list, as ~w while preceding dirty neighbours leave its
// count open, as w when the count is final and 0.  A ~w of the wavefront
// tier whose row did not sit in registers (listed false) gets no pair list.
template <int GS, typename S>
__device__ __forceinline__ void inc_a_finish(const Args& a, WaveStage* stg, int k, int w, int deg,
                                             int scanned, int lig, int now, int cnt, bool dlow, int* shc,
                                             long long* dedges, bool listed = false);

// What a dirty vertex's processing reads first: its id, row bounds, split
// point and state word.  The wavefront walk loads it one chunk ahead (no
// other group writes these words of w during the kernel).
struct VInfo {
    int w, s, e, sp, old;
};

template <typename S>
__device__ __forceinline__ VInfo load_vinfo(const Args& a, int w) {
    VInfo r;
    r.w = w;
    if (w >= 0) {
        const int4 q = vrec_load(a, w);
        r.s = q.x;
        r.e = q.y;
        r.sp = q.z;
        r.old = static_cast<const S*>(a.st)[w];
    } else {
        r.s = r.e = r.sp = r.old = 0;
    }
    return r;
}

template <int GS, typename S>
__device__ __forceinline__ void inc_a_vertex_pre(const Args& a, WaveStage* stg, int k, const VInfo& vi, int lig,
                                                 uint64_t* red, int* shc, unsigned* ffbm, int* cc,
                                                 long long* dedges);

template <int GS, typename S>
__device__ __forceinline__ void inc_a_vertex(const Args& a, WaveStage* stg, int k, int w, int lig,
                                             uint64_t* red, int* shc, unsigned* ffbm, int* cc, long long* dedges) {
    inc_a_vertex_pre<GS, S>(a, stg, k, load_vinfo<S>(a, w), lig, red, shc, ffbm, cc, dedges);
}

template <int GS, typename S>
__device__ __forceinline__ void inc_a_vertex_pre(const Args& a, WaveStage* stg, int k, const VInfo& vi, int lig,
                                                 uint64_t* red, int* shc, unsigned* ffbm, int* cc,
                                                 long long* dedges) {
    S* st = static_cast<S*>(a.st);
    const unsigned* bits = dbits(a, k);
    const int w = vi.w, s = vi.s, e = vi.e;
    const int old = vi.old;
    if constexpr (GS == kBlock || GS == kWave) {
        if (e - s > kHeavyDeg) {
            unsigned* bm = GS == kBlock ? ffbm : ffbm + (threadIdx.x / kWave) * kFFWords;
            int now, cnt;
            bool dlow;
            int len;
            inc_a_heavy<GS, S>(a, stg, k, w, s, vi.sp, old, lig, red, shc, bm, cc, &now, &cnt, &dlow, &len);
            inc_a_finish<GS, S>(a, stg, k, w, e - s, len, lig, now, cnt, dlow, shc, dedges);
            return;
        }
    }
    const int lim = s + vi.sp;
    const bool cached = (e - s) <= kCache * GS;
    int xs[kCache], sv[kCache];
    if (cached) {
#pragma unroll
        for (int j = 0; j < kCache; ++j) {
            const int p = s + lig + j * GS;
            xs[j] = p < e ? a.colp[p] : w;
        }
#pragma unroll
        for (int j = 0; j < kCache; ++j) sv[j] = st[xs[j]];  // p >= e reads w's own (positive) word
    }
    // new tentative colour: first window of 64 colours with a free slot
    int now = 0, base0 = 1;
    if constexpr (GS == kBlock || GS == kWave) {
        if (!cached) {
            unsigned* bm = GS == kBlock ? ffbm : ffbm + (threadIdx.x / kWave) * kFFWords;
            now = first_fit_long<GS, S>(a.colp, st, s + lig, e, bm, red, shc);
            base0 = 65 + kFFBits;
        }
    }
    for (int base = base0; now == 0; base += 64) {
        uint64_t m = 0;
        if (cached) {
#pragma unroll
            for (int j = 0; j < kCache; ++j) {
                const unsigned c = (unsigned)(-sv[j] - base);
                if (c < 64u) m |= 1ull << c;
            }
        } else {
            m = state_window<GS, S>(s + lig, e, base, a.colp, st);
        }
        if constexpr (GS == kBlock) {
            m = group_or<kWave>(m);
            if (__lane_id() == 0) red[threadIdx.x / kWave] = m;
            __syncthreads();
            m = red[0] | red[1] | red[2] | red[3];
            __syncthreads();
        } else {
            m = group_or<GS>(m);
        }
        if (~m) now = base + __builtin_ctzll(~m);
    }
    // counters
    int cnt = 0;
    bool dlow = false;
    unsigned dpm = 0u;
    if (cached) {
        inc_a_eval_staged<GS, kCache, GS <= kWave>(a, stg, bits, k, w, s + lig, e, lim, now, old, xs, sv, &cnt,
                                                   &dlow, &dpm);
    } else {
        inc_a_pass2_gather<GS, S>(a, stg, st, bits, k, w, s + lig, e, lim, now, old, &cnt, &dlow);
    }
    inc_a_finish<GS, S>(a, stg, k, w, e - s, e - s, lig, now, cnt, dlow, shc, dedges, cached);
}


// Group totals of the counter and the preceding-dirty flag; state, counter
// and list appends of dirty vertex w.
template <int GS, typename S>
__device__ __forceinline__ void inc_a_finish(const Args& a, WaveStage* stg, int k, int w, int deg,
                                             int scanned, int lig, int now, int cnt, bool dlow, int* shc,
                                             long long* dedges, bool listed) {
    S* st = static_cast<S*>(a.st);
    const int cs = cset(k);
    int dl = dlow ? 1 : 0;
    if constexpr (GS == kBlock) {
        cnt = group_sum<kWave>(cnt);
        dl = group_sum<kWave>(dl);
        if (__lane_id() == 0) {
            shc[threadIdx.x / kWave] = cnt;
            shc[4 + threadIdx.x / kWave] = dl;
        }
        __syncthreads();
        cnt = shc[0] + shc[1] + shc[2] + shc[3];
        dl = shc[4] + shc[5] + shc[6] + shc[7];
        __syncthreads();
    } else {
        cnt = group_sum<GS>(cnt);
        dl = group_sum<GS>(dl);
        // the commit kernel reads pref[w] of every ~w of bins 0..3 (a row
        // in registers had its list stored by the staged evaluation)
        if (!listed && dl > 0 && lig == 0) a.pref[w] = -1;
    }
    bool to_b = false, cand = false;
    if (lig == 0) {
        st[w] = (S)now;
        *vconf(a, w) = cnt;
        dedges[0] += deg;
        dedges[1] += scanned;
        to_b = dl > 0;
        cand = !to_b && cnt == 0 && (atomicExch(&a.cflag[w], k) != k);
    }
    if (GS == kBlock && threadIdx.x >= kWave) return;
    stage_append(a, stg, to_b || cand, to_b ? ~w : w, deg, cs);
}

// Chunk space of the group tiers (bins 0..3) for wavefront walks: a chunk
// is what one wavefront takes at once, 64 / 16 / 4 / 1 vertices for bins
// 0 / 1 / 2 / 3 (64 / 4 / 1 lanes per vertex ... one wavefront per
// vertex); bins ordered 3, 2, 1, 0 (heaviest first).
__host__ __device__ constexpr int wchunk(int b) { return b == 0 ? 64 : b == 1 ? 16 : b == 2 ? 4 : 1; }

struct WaveMap {
    int cnt[4];
    int start[4];
    int off[4];  // bin offsets inside the set's array
    int total;
};

__device__ __forceinline__ WaveMap make_wave_map(const Ctl* ctl, int set) {
    WaveMap m;
    int tot = 0;
    for (int b = 3; b >= 0; --b) {
        m.cnt[b] = ctl->cnt[set][b];
        m.start[b] = tot;
        tot += (m.cnt[b] + wchunk(b) - 1) / wchunk(b);
    }
    int off = 0;
    for (int b = 0; b < 4; ++b) {
        m.off[b] = off;
        off += ctl->binpop[b];
    }
    m.total = tot;
    return m;
}

__device__ __forceinline__ int wave_chunk_bin(const WaveMap& m, int c) {
    return 3 - (c >= m.start[2]) - (c >= m.start[1]) - (c >= m.start[0]);
}

__device__ __forceinline__ int pick4(const int* x, int b) {
    return b == 0 ? x[0] : b == 1 ? x[1] : b == 2 ? x[2] : x[3];
}

// List entry that lane `lane` takes in wavefront chunk c of list set `set`
// (its group's vertex), or INT_MIN when the chunk or the group is past the
// end.
__device__ __forceinline__ int wave_chunk_entry(const Args& a, const WaveMap& m, int set, int c, int lane) {
    if (c >= m.total) return INT_MIN;
    const int b = wave_chunk_bin(m, c);
    const int idx = (c - pick4(m.start, b)) * wchunk(b) + lane / (kWave / wchunk(b));
    return idx < pick4(m.cnt, b) ? a.lists[(size_t)set * (size_t)a.n + pick4(m.off, b) + idx] : INT_MIN;
}

// Round k, kernel A.  Also clears the bitmap of round k-1's dirty vertices
// (its list is still intact), so that round k+1 can reuse it.  The
// workgroup tier runs first, one vertex per workgroup; then every wavefront
// walks its own chunks of the group tiers with no workgroup barrier, with
// the list entry of the chunk after next and the row bounds, split point
// and state word of the next chunk loaded before the current one is
// processed.
template <typename S>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_inc_a(Args a, int k) {
    __shared__ uint64_t red[kWaves];
    __shared__ int shc[8];
    __shared__ WaveStage wstg[kWaves];
    __shared__ unsigned ffbm[kWaves * kFFWords];
    __shared__ int cc[2];
    // sequential finish requested and at most `tail` vertices left: this
    // round and every later one do nothing (the finish colours the rest)
    if (a.tail > 0 && (long long)a.n - (long long)a.ctl->committed <= a.tail) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the list that this round's commits fill (round k-2's dirty list,
        // whose bitmap words k_inc_a of round k-1 cleared)
        for (int b = 0; b < 8; ++b) a.ctl->cnt[dlist(k + 1)][b] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && k - 1 < kMaxLog) {
        long long nd = 0;
        for (int b = 0; b < kBins; ++b) nd += a.ctl->cnt[dlist(k)][b];
        a.log[kLogW * (k - 1) + 0] = 0;
        a.log[kLogW * (k - 1) + 1] = 0;
        a.log[kLogW * (k - 1) + 2] = nd;
        // fields 3 and 4 (dirty degree sum, entries scanned) collect this
        // kernel's blocks: the previous kernel cleared them, not block 0 here,
        // so that no block adds before they are cleared
    }
    {
        // this round's lists are built: its bitmap's summary flags start
        // over for round k+3 (marked by the commit kernel of round k+2)
        unsigned char* sm = dsum(a, k);
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.nregions; i += gridDim.x * kBlock) sm[i] = 0;
    }
    const int set = dlist(k);
    const int n4 = a.ctl->cnt[set][4];
    const WaveMap m = make_wave_map(a.ctl, set);
    int nprev = 0;
    for (int b = 0; b < kBins; ++b) nprev += a.ctl->cnt[dlist(k - 1)][b];
    const int clear_blocks = (nprev + kBlock - 1) / kBlock;
    if ((int)blockIdx.x >= max(max(n4, (m.total + kWaves - 1) / kWaves), clear_blocks)) return;
    {
        // every bit of that bitmap belongs to a previous dirty vertex, so the
        // words holding them can be zeroed whole
        unsigned* pbits = dbits(a, k - 1);
        int off[kBins];
        bin_offsets(a.ctl, off);
        for (int b = 0; b < kBins; ++b) {
            const int c = a.ctl->cnt[dlist(k - 1)][b];
            const int* l = a.lists + (size_t)dlist(k - 1) * (size_t)a.n + off[b];
            for (int i = blockIdx.x * kBlock + threadIdx.x; i < c; i += gridDim.x * kBlock) pbits[l[i] >> 5] = 0u;
        }
    }
    const int cs = cset(k);
    WaveStage* stg = &wstg[threadIdx.x / kWave];
    wstage_init(a, stg);
    if (__lane_id() == 0) {  // this wavefront's region of the pair buffer
        const int waves = gridDim.x * kWaves;
        stg->plen = a.pcap / waves;
        stg->pbase = (blockIdx.x * kWaves + (int)threadIdx.x / kWave) * stg->plen;
        stg->pfill = 0;
    }
    wave_sync();
    long long dedges[2] = {0, 0};  // degree sum and scanned entries of the dirty rows
    const int* l4 = list_ptr(a, set, 4);
    for (int c = blockIdx.x; c < n4; c += gridDim.x) {
        inc_a_vertex<kBlock, S>(a, stg, k, l4[c], (int)threadIdx.x, red, shc, ffbm, cc, dedges);
        wstage_maybe_flush(a, stg, cs);
    }
    const int lane = __lane_id();
    const int W = gridDim.x * kWaves;
    int c = blockIdx.x * kWaves + (int)threadIdx.x / kWave;
#if GC_PREFETCH_A
    int e2 = wave_chunk_entry(a, m, set, c + W, lane);
    VInfo nxt = load_vinfo<S>(a, max(wave_chunk_entry(a, m, set, c, lane), -1));
#endif
    for (; c < m.total; c += W) {
#if GC_PREFETCH_A
        const VInfo cur = nxt;
        nxt = load_vinfo<S>(a, max(e2, -1));
        e2 = wave_chunk_entry(a, m, set, c + 2 * W, lane);
#else
        const VInfo cur = load_vinfo<S>(a, max(wave_chunk_entry(a, m, set, c, lane), -1));
#endif
        if (cur.w >= 0) {
            switch (wave_chunk_bin(m, c)) {
                case 0: inc_a_vertex_pre<1, S>(a, stg, k, cur, 0, nullptr, nullptr, ffbm, nullptr, dedges); break;
                case 1: inc_a_vertex_pre<4, S>(a, stg, k, cur, lane & 3, nullptr, nullptr, ffbm, nullptr, dedges); break;
                case 2:
                    inc_a_vertex_pre<16, S>(a, stg, k, cur, lane & 15, nullptr, nullptr, ffbm, nullptr, dedges);
                    break;
                default:
                    inc_a_vertex_pre<kWave, S>(a, stg, k, cur, lane, nullptr, nullptr, ffbm, nullptr, dedges);
                    break;
            }
        }
        wstage_maybe_flush(a, stg, cs);
    }
    wstage_flush(a, stg, cs);
    if (k - 1 < kMaxLog) {
        block_add_log(dedges[0], &a.log[kLogW * (k - 1) + 3]);
        block_add_log(dedges[1], &a.log[kLogW * (k - 1) + 4]);
    }
}

// Preceding dirty neighbours of w (entries start, start + STRIDE, ... < lim
// of row) holding colour now: dirty vertices are uncoloured at the start of
// the round, and one committed during the commit kernel shows -now, so the
// count compares |word| (both ways the neighbour keeps w from committing
// with now).
template <int STRIDE, typename S>
__device__ __forceinline__ int inc_b_count(const int* __restrict__ row, const S* __restrict__ st,
                                           const unsigned* __restrict__ bits, int w, int start, int lim, int now) {
    int c = 0;
    for (int p0 = start; p0 < lim; p0 += 4 * STRIDE) {
        int x[4];
        bool d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * STRIDE;
            x[j] = p < lim ? row[p] : w;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = (p0 + j * STRIDE < lim) && is_dirty(bits, x[j]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (d[j]) {
                const int sx = st[x[j]];
                c += ((sx < 0 ? -sx : sx) == now);
            }
    }
    return c;
}

// Dirty marks from committed vertex v (colour t) over its later entries
// start, start + STRIDE, ... < e: an entry u whose word is t is uncoloured
// with tentative colour t, so its tentative colour must move in round k+1;
// its bit is set in round k+1's bitmap (the round's dirty lists are built
// from the bitmap after this kernel, in ascending vertex order).  A neighbour
// committed in this same kernel holds a colour different from t (two
// adjacent vertices with equal tentative colours cannot both have counter
// 0), so reading its word before or after its commit gives no match.  Eight
// entries per step, in stages (state reads, bitmap reads, then the atomics),
// so that each stage's memory operations of a lane are in flight together.
template <int STRIDE, typename S>
__device__ __forceinline__ void inc_c_row(const Args& a, const int* __restrict__ row, const S* __restrict__ st,
                                          int k, int v, int t, int start, int e) {
    constexpr int U = 8;
    unsigned* nbits = dbits(a, k + 1);
    unsigned char* nsum = dsum(a, k + 1);
    for (int p0 = start; p0 < e; p0 += U * STRIDE) {
        int u[U], su[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int p = p0 + j * STRIDE;
            u[j] = p < e ? row[p] : v;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) su[j] = st[u[j]];
        // a plain read of the bitmap first skips most repeated marks
        unsigned need = 0u;
#pragma unroll
        for (int j = 0; j < U; ++j) need |= (u[j] != v && su[j] == t ? 1u : 0u) << j;
        if (need == 0u) continue;
        unsigned word[U];
#pragma unroll
        for (int j = 0; j < U; ++j) word[j] = (need >> j & 1u) ? nbits[u[j] >> 5] : ~0u;
        unsigned setm = 0u;
#pragma unroll
        for (int j = 0; j < U; ++j) setm |= ((word[j] >> (u[j] & 31)) & 1u ? 0u : 1u) << j;
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (setm >> j & 1u) {
                atomicOr(&nbits[u[j] >> 5], 1u << (u[j] & 31));
                nsum[u[j] >> (5 + kSumShift)] = 1;
            }
    }
}

// One entry of the candidate list: a candidate v (>= 0) commits if its
// counter is 0; ~w (a dirty vertex with preceding dirty neighbours) first
// has its counter completed (inc_b_count) and commits if the total is 0.
// What the entry's processing reads first (entry, state word, row bounds,
// split point, counter) comes preloaded: only the entry's own group writes
// those words of v in this kernel.
struct CInfo {
    int ent, t, s, e, sp, conf, pref;
};

template <typename S>
__device__ __forceinline__ CInfo load_cinfo(const Args& a, int ent) {
    CInfo r;
    r.ent = ent;
    if (ent != INT_MIN) {
        const int v = ent < 0 ? ~ent : ent;
        r.t = static_cast<const S*>(a.st)[v];
        const int4 q = vrec_load(a, v);
        r.s = q.x;
        r.e = q.y;
        r.sp = q.z;
        r.conf = q.w;
        r.pref = ent < 0 ? a.pref[v] : -1;
    } else {
        r.t = r.s = r.e = r.sp = r.conf = 0;
        r.pref = -1;
    }
    return r;
}

// Preceding dirty neighbours of w holding colour now, from w's pair list
// (start and length packed in pr): the same neighbours, compared the same
// way, as inc_b_count over the row.
template <int STRIDE, typename S>
__device__ __forceinline__ int pair_count(const Args& a, const S* __restrict__ st, int pr, int lig, int now) {
    const int* __restrict__ q = a.pbuf + (pr & (kPairMaxCap - 1));
    const int len = pr >> kPairShift;
    int c = 0;
    for (int i0 = lig; i0 < len; i0 += 4 * STRIDE) {
        int x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = i0 + j * STRIDE < len ? q[i0 + j * STRIDE] : -1;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (x[j] >= 0) {
                const int sx = st[x[j]];
                c += ((sx < 0 ? -sx : sx) == now);
            }
    }
    return c;
}

template <int GS, typename S>
__device__ __forceinline__ void inc_c_entry(const Args& a, int k, const CInfo& ci, int lig,
                                            long long* ncom, long long* ndeg) {
    S* st = static_cast<S*>(a.st);
    const int ent = ci.ent;
    const int v = ent < 0 ? ~ent : ent;
    const int t = ci.t;
    const int s = ci.s, e = ci.e;
    bool commit;
    if (ent < 0) {
        int c;
        if (ci.pref >= 0) {  // group-uniform
            c = group_sum<GS>(pair_count<GS, S>(a, st, ci.pref, lig, t));
        } else {
            const int* row = a.colp;
            int lim = s + ci.sp;
            if constexpr (GS == kWave) {
                if (e - s > kHeavyDeg) {  // preceding segment of the active row
                    const HeavyView hv = heavy_view(a, v, s, ci.sp);
                    row = hv.row;
                    lim = s + hv.pa;
                }
            }
            c = group_sum<GS>(inc_b_count<GS, S>(row, st, dbits(a, k), v, s + lig, lim, t));
        }
        const int tot = ci.conf + c;
        if (lig == 0) *vconf(a, v) = tot;
        commit = tot == 0;
    } else {
        commit = ci.conf == 0 && t > 0;
    }
    if (commit) {
        const int* row = a.colp;
        int start = s + ci.sp, end = e;
        if constexpr (GS == kWave) {
            if (e - s > kHeavyDeg) {  // later segment of the active row
                const HeavyView hv = heavy_view(a, v, s, ci.sp);
                row = hv.row;
                start = hv.s1;
                end = hv.s1 + hv.la;
            }
        }
        inc_c_row<GS, S>(a, row, st, k, v, t, start + lig, end);
        if (lig == 0) {
            st[v] = (S)(-t);
            *ncom += 1;
            *ndeg += e - s;
            a.ctl->rounds = k;
        }
    }
}

template <typename S>
__device__ __forceinline__ void inc_c_block(const Args& a, int k, int ent, int* sh, long long* ncom,
                                            long long* ndeg) {
    S* st = static_cast<S*>(a.st);
    const int v = ent < 0 ? ~ent : ent;
    const int t = st[v];
    const int4 q = vrec_load(a, v);
    const int s = q.x, e = q.y, sp = q.z;
    if (ent < 0) {
        const int* row = a.colp;
        int lim = s + sp;
        if (e - s > kHeavyDeg) {  // preceding segment of the active row
            const HeavyView hv = heavy_view(a, v, s, sp);
            row = hv.row;
            lim = s + hv.pa;
        }
        const int c = group_sum<kWave>(inc_b_count<kBlock, S>(row, st, dbits(a, k), v, s + (int)threadIdx.x, lim, t));
        if (__lane_id() == 0) sh[threadIdx.x / kWave] = c;
        __syncthreads();
        const int tot = q.w + sh[0] + sh[1] + sh[2] + sh[3];
        __syncthreads();  // every thread has read sh
        if (threadIdx.x == 0) *vconf(a, v) = tot;
        if (tot != 0) return;  // block-uniform
    } else if (q.w != 0 || t <= 0) {
        return;  // block-uniform: only this block writes them in this kernel
    }
    const int* row = a.colp;
    int start = s + sp, end = e;
    if (e - s > kHeavyDeg) {  // later segment of the active row
        const HeavyView hv = heavy_view(a, v, s, sp);
        row = hv.row;
        start = hv.s1;
        end = hv.s1 + hv.la;
    }
    inc_c_row<kBlock, S>(a, row, st, k, v, t, start + (int)threadIdx.x, end);
    __syncthreads();  // every thread has read st[v] before it is overwritten
    if (threadIdx.x == 0) {
        st[v] = (S)(-t);
        *ncom += 1;
        *ndeg += e - s;
        a.ctl->rounds = k;
    }
}

// Round k, kernel C: commit every candidate whose counter is 0, mark its
// dirty neighbours for round k+1 in that round's bitmap.  Clears the
// candidate list of round k+1.  Same walk as k_inc_a: the workgroup tier
// first, then per-wavefront chunks with the next chunk's entries preloaded.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_inc_c(Args a, int k) {
    __shared__ int sh[kWaves];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int b = 0; b < 8; ++b) a.ctl->cnt[cset(k + 1)][b] = 0;
        if (k < kMaxLog) {  // round k+1's dirty degree sum and scanned entries
            a.log[kLogW * k + 3] = 0;
            a.log[kLogW * k + 4] = 0;
        }
    }
    const int set = cset(k);
    const int n4 = a.ctl->cnt[set][4];
    const WaveMap m = make_wave_map(a.ctl, set);
    if ((int)blockIdx.x >= max(n4, (m.total + kWaves - 1) / kWaves)) return;
    long long ncom = 0, ndeg = 0;
    const int* l4 = list_ptr(a, set, 4);
    for (int c = blockIdx.x; c < n4; c += gridDim.x) inc_c_block<S>(a, k, l4[c], sh, &ncom, &ndeg);
    const int lane = __lane_id();
    const int W = gridDim.x * kWaves;
    int c = blockIdx.x * kWaves + (int)threadIdx.x / kWave;
    int e2 = wave_chunk_entry(a, m, set, c + W, lane);
    CInfo nxt = load_cinfo<S>(a, wave_chunk_entry(a, m, set, c, lane));
    for (; c < m.total; c += W) {
        const CInfo cur = nxt;
        nxt = load_cinfo<S>(a, e2);
        e2 = wave_chunk_entry(a, m, set, c + 2 * W, lane);
        if (cur.ent != INT_MIN) {
            switch (wave_chunk_bin(m, c)) {
                case 0: inc_c_entry<1, S>(a, k, cur, 0, &ncom, &ndeg); break;
                case 1: inc_c_entry<4, S>(a, k, cur, lane & 3, &ncom, &ndeg); break;
                case 2: inc_c_entry<16, S>(a, k, cur, lane & 15, &ncom, &ndeg); break;
                default: inc_c_entry<kWave, S>(a, k, cur, lane, &ncom, &ndeg); break;
            }
        }
    }
    block_add_log(ncom, (long long*)&a.ctl->committed);
    if (k - 1 < kMaxLog) {
        block_add_log(ncom, &a.log[kLogW * (k - 1)]);
        block_add_log(ndeg, &a.log[kLogW * (k - 1) + 1]);
    }
}

// ---------------------------------------------------------------------------
// Dirty lists of round kk in ascending vertex order, built from the round's
// bitmap after the commit kernel of round kk-1 has set it: a count pass
// (per workgroup and bin) and a write pass (each workgroup's offsets from
// the counts of the workgroups before it).  Processing dirty rows in vertex
// order keeps the neighbour gathers of nearby rows close in time, which the
// L2 caches serve better than a random order (on R-MAT, neighbour ids share
// high bits with the row's id).  Workgroup b owns the bitmap words
// [b W, (b+1) W), its threads consecutive slices of them, so the lists come
// out sorted.  (A single count pass whose last workgroup computed the
// offsets needed device-scope fences in every workgroup, which write the
// L2s back on this multi-XCD chip: 81 us per pass instead of a few.)
// ---------------------------------------------------------------------------
#ifndef GC_COMPACT_WORDS
#define GC_COMPACT_WORDS 512
#endif
constexpr int kCompactWordsPerBlock = GC_COMPACT_WORDS;
constexpr int kCompactMaxBlocks = 8192;

__host__ __device__ inline int compact_blocks(int nwords) {
    const int b = (nwords + kCompactWordsPerBlock - 1) / kCompactWordsPerBlock;
    return b < 1 ? 1 : (b > kCompactMaxBlocks ? kCompactMaxBlocks : b);
}

// Whether the workgroup's bitmap words hold any mark (the summary flags of
// the regions they overlap; a flag is set with every new mark).
__device__ __forceinline__ bool block_has_marks(const Args& a, int kk) {
    const int G = gridDim.x;
    const int per_block = (a.nwords + G - 1) / G;
    const int b0 = blockIdx.x * per_block, b1 = min(a.nwords, b0 + per_block);
    if (b0 >= b1) return false;
    const unsigned char* sm = dsum(a, kk);
    bool any = false;
    for (int r = b0 >> kSumShift; r <= (b1 - 1) >> kSumShift; ++r) any |= sm[r] != 0;
    return any;
}

// This thread's slice of bitmap words.
__device__ __forceinline__ void compact_slice(int nwords, int* w0, int* w1) {
    const int G = gridDim.x;
    const int per_block = (nwords + G - 1) / G;
    const int b0 = blockIdx.x * per_block, b1 = min(nwords, b0 + per_block);
    const int per_thread = (per_block + kBlock - 1) / kBlock;
    *w0 = min(b1, b0 + (int)threadIdx.x * per_thread);
    *w1 = min(b1, *w0 + per_thread);
}

// Bin counts of the dirty vertices in this thread's slice.
// Set bits of bitmap word w whose vertex lies in degree bin b (the bit
// planes hold each vertex's bin).
__device__ __forceinline__ unsigned bin_mask(const Args& a, int w, int b) {
    const unsigned p0 = a.bplane[w], p1 = a.bplane[a.nwords + w], p2 = a.bplane[2 * (size_t)a.nwords + w];
    return ((b & 1) ? p0 : ~p0) & ((b & 2) ? p1 : ~p1) & ((b & 4) ? p2 : ~p2);
}

// Bin counts of the dirty vertices in this thread's slice.
__device__ __forceinline__ void compact_count(const Args& a, const unsigned* __restrict__ bits, int w0, int w1,
                                              int* c) {
#pragma unroll
    for (int b = 0; b < kBins; ++b) c[b] = 0;
    for (int w = w0; w < w1; ++w) {
        const unsigned x = bits[w];
        if (x == 0u) continue;
#pragma unroll
        for (int b = 0; b < kBins; ++b) c[b] += __popc(x & bin_mask(a, w, b));
    }
}

__global__ __launch_bounds__(kBlock) void k_dcount(Args a, int kk) {
    __shared__ int part[kWaves][kBins];
    const long long left = (long long)a.n - (long long)a.ctl->committed;
    if (left == 0 || (a.tail > 0 && left <= a.tail)) return;  // nothing to list
    if (!block_has_marks(a, kk)) {  // block-uniform: no mark in these words
        if (threadIdx.x < kBins) a.bcnt[blockIdx.x * 8 + threadIdx.x] = 0;
        return;
    }
    const unsigned* bits = dbits(a, kk);
    int w0, w1;
    compact_slice(a.nwords, &w0, &w1);
    int c[kBins];
    compact_count(a, bits, w0, w1, c);
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        const int t = group_sum<kWave>(c[b]);
        if (__lane_id() == 0) part[threadIdx.x / kWave][b] = t;
    }
    __syncthreads();
    if (threadIdx.x < kBins) {
        int t = 0;
        for (int q = 0; q < kWaves; ++q) t += part[q][threadIdx.x];
        a.bcnt[blockIdx.x * 8 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_dwrite(Args a, int kk) {
    __shared__ int base[kBins];
    __shared__ int wsum[kWaves][kBins];
    const long long left = (long long)a.n - (long long)a.ctl->committed;
    if (left == 0 || (a.tail > 0 && left <= a.tail)) return;  // the list stays empty
    const int set = dlist(kk);
    // no mark in these words: nothing to write (the last workgroup still
    // writes the list totals)
    if (blockIdx.x != gridDim.x - 1 && !block_has_marks(a, kk)) return;
    const unsigned* bits = dbits(a, kk);
    // offsets: the counts of the workgroups before this one (and, for the
    // last workgroup, the list totals)
    int pre[kBins];
#pragma unroll
    for (int b = 0; b < kBins; ++b) pre[b] = 0;
    for (int q = threadIdx.x; q < (int)blockIdx.x; q += kBlock)
#pragma unroll
        for (int b = 0; b < kBins; ++b) pre[b] += a.bcnt[q * 8 + b];
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        const int t = group_sum<kWave>(pre[b]);
        if (__lane_id() == 0) wsum[threadIdx.x / kWave][b] = t;
    }
    __syncthreads();
    if (threadIdx.x < kBins) {
        int t = 0;
        for (int q = 0; q < kWaves; ++q) t += wsum[q][threadIdx.x];
        base[threadIdx.x] = t;
        if (blockIdx.x == gridDim.x - 1) a.ctl->cnt[set][threadIdx.x] = t + a.bcnt[blockIdx.x * 8 + threadIdx.x];
    }
    __syncthreads();
    // this thread's offsets inside the workgroup: exclusive scan of the
    // slices' counts (waves in order, lanes in order)
    int w0, w1;
    compact_slice(a.nwords, &w0, &w1);
    int c[kBins];
    compact_count(a, bits, w0, w1, c);
    int off[kBins];
    const int lane = __lane_id();
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        int x = c[b];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        off[b] = x - c[b];
        if (lane == kWave - 1) wsum[threadIdx.x / kWave][b] = x;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        int before = base[b];
        for (int q = 0; q < (int)threadIdx.x / kWave; ++q) before += wsum[q][b];
        off[b] += before;
    }
    int* dsts[kBins];
    {
        int off[kBins];
        bin_offsets(a.ctl, off);
#pragma unroll
        for (int b = 0; b < kBins; ++b) dsts[b] = a.lists + (size_t)set * (size_t)a.n + off[b];
    }
    for (int w = w0; w < w1; ++w) {
        const unsigned x = bits[w];
        if (x == 0u) continue;
#pragma unroll
        for (int b = 0; b < kBins; ++b) {
            unsigned y = x & bin_mask(a, w, b);
            int* dst = dsts[b];
            int o = off[b];
            while (y) {
                dst[o++] = w * 32 + __builtin_ctz(y);
                y &= y - 1;
            }
            off[b] = o;
        }
    }
}

// ===========================================================================
// Dataflow engine (section "A dataflow algorithm", Algorithm 3), in rounds.
//
// conf[v] counts the entries of v's preceding segment whose vertex is not
// coloured yet.  Round k colours every vertex on its ready list (count 0)
// with the smallest colour none of its preceding neighbours holds -- all of
// them are final by then -- and takes one off the count of each later
// neighbour; a count reaching 0 puts that neighbour on round k+1's list.
// The colouring is the serial first-fit in (priority, id) order
// (Algorithm 1), and round k holds the vertices whose longest chain of
// preceding neighbours has k vertices.  One kernel per round.
// Colours are gathered from a byte copy, min(colour, 255), where 255 sends
// the reader to colors_out: a quarter of the gathered working set.
// Lists rotate over sets 0..2: round k reads set k % 3, appends to
// (k + 1) % 3 and clears the counts of (k + 2) % 3 (read in round k - 1,
// filled in round k + 1).
// ===========================================================================

__host__ __device__ inline int fset(int k) { return k % 3; }

__device__ __forceinline__ int flow_colour(const uint8_t* __restrict__ cb, const int* __restrict__ color, int w) {
    const int c = cb[w];
    return c == 255 ? color[w] : c;
}

// Colours base..base+63 held by the vertices of entries start, start +
// STRIDE, ... < lim (all coloured); four gathers in flight per lane.
template <int STRIDE>
__device__ __forceinline__ uint64_t flow_window(const int* __restrict__ colp, const uint8_t* __restrict__ cb,
                                                const int* __restrict__ color, int start, int lim, int base) {
    uint64_t m = 0;
    int p = start;
    for (; p + 3 * STRIDE < lim; p += 4 * STRIDE) {
        const int w0 = colp[p], w1 = colp[p + STRIDE], w2 = colp[p + 2 * STRIDE], w3 = colp[p + 3 * STRIDE];
        const unsigned c0 = (unsigned)(flow_colour(cb, color, w0) - base);
        const unsigned c1 = (unsigned)(flow_colour(cb, color, w1) - base);
        const unsigned c2 = (unsigned)(flow_colour(cb, color, w2) - base);
        const unsigned c3 = (unsigned)(flow_colour(cb, color, w3) - base);
        if (c0 < 64u) m |= 1ull << c0;
        if (c1 < 64u) m |= 1ull << c1;
        if (c2 < 64u) m |= 1ull << c2;
        if (c3 < 64u) m |= 1ull << c3;
    }
    for (; p < lim; p += STRIDE) {
        const unsigned c = (unsigned)(flow_colour(cb, color, colp[p]) - base);
        if (c < 64u) m |= 1ull << c;
    }
    return m;
}

__device__ __forceinline__ void flow_store(const Args& a, int v, int c) {
    a.color[v] = c;
    static_cast<uint8_t*>(a.st)[v] = (uint8_t)min(c, 255);
}

// One pass over the whole row of v, entries start, start + STRIDE, ... < e:
// preceding entries (below lim) add their colours in 1..64 to the mask,
// later ones are released at once -- the released vertices read v's colour
// only in the next round, so nothing here waits for the first-fit.  Four
// entries per step, in stages: every colour byte and every release atomic
// of the step are issued before any is used, then the rare full colours
// (byte 255).
template <int STRIDE>
__device__ __forceinline__ uint64_t flow_row(const Args& a, Stage* stg, const uint8_t* __restrict__ cb, int v,
                                             int start, int lim, int e, int set) {
    uint64_t m = 0;
    for (int p0 = start; p0 < e; p0 += 4 * STRIDE) {
        int x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * STRIDE;
            x[j] = p < e ? a.colp[p] : v;
        }
        unsigned pre = 0u, rel = 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * STRIDE;
            pre |= (p < lim ? 1u : 0u) << j;
            rel |= (p >= lim && x[j] != v ? 1u : 0u) << j;
        }
        int c[4], left[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c[j] = (pre >> j & 1u) ? (int)cb[x[j]] : 0;
            left[j] = (rel >> j & 1u) ? atomicSub(&a.conf[x[j]], 1) : 0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (c[j] == 255) c[j] = a.color[x[j]];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned b = (unsigned)(c[j] - 1);
            if (b < 64u) m |= 1ull << b;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) stage_append_lookup(a, stg, left[j] == 1, x[j], set);
    }
    return m;
}

template <int GS>
__device__ __forceinline__ void flow_chunk(const Args& a, Stage* stg, int k, const int* list, int cnt, int local,
                                           long long* ncol, long long* work) {
    constexpr int CV = kBlock / GS;
    const uint8_t* cb = static_cast<const uint8_t*>(a.st);
    const int lig = threadIdx.x & (GS - 1);
    const int idx = local * CV + (int)threadIdx.x / GS;
    if (idx < cnt) {
        const int v = list[idx];
        const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
        const int lim = s + a.split[v];
        uint64_t m = group_or<GS>(flow_row<GS>(a, stg, cb, v, s + lig, lim, e, fset(k + 1)));
        int c = ~m ? 1 + __builtin_ctzll(~m) : 0;
        for (int base = 65; c == 0; base += 64) {  // colours 1..64 all taken
            m = group_or<GS>(flow_window<GS>(a.colp, cb, a.color, s + lig, lim, base));
            if (~m) c = base + __builtin_ctzll(~m);
        }
        if (lig == 0) {
            flow_store(a, v, c);
            *ncol += 1;
            *work += e - s;
        }
    }
}

__device__ __forceinline__ void flow_block(const Args& a, Stage* stg, int k, int v, uint64_t* red, long long* ncol,
                                           long long* work) {
    const uint8_t* cb = static_cast<const uint8_t*>(a.st);
    const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
    const int lim = s + a.split[v];
    uint64_t m = flow_row<kBlock>(a, stg, cb, v, s + (int)threadIdx.x, lim, e, fset(k + 1));
    int c = 0;
    for (int base = 1; c == 0; base += 64) {
        if (base > 1) m = flow_window<kBlock>(a.colp, cb, a.color, s + (int)threadIdx.x, lim, base);
        m = group_or<kWave>(m);
        if (__lane_id() == 0) red[threadIdx.x / kWave] = m;
        __syncthreads();
        m = red[0] | red[1] | red[2] | red[3];
        __syncthreads();
        if (~m) c = base + __builtin_ctzll(~m);
    }
    if (threadIdx.x == 0) {
        flow_store(a, v, c);
        *ncol += 1;
        *work += e - s;
    }
}

// Round 1's list and the counts: conf[v] = split[v] (natural order: the
// split is found here by binary search in the sorted row).
__global__ __launch_bounds__(kBlock) void k_flow_seed(Args a, int natural) {
    __shared__ Stage stg;
    stage_init(a, &stg);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int i = 0; i < kLogW; ++i) a.log[i] = 0;
    const int stride = gridDim.x * kBlock;
    for (int base = blockIdx.x * kBlock; base < a.n; base += stride) {
        const int v = base + (int)threadIdx.x;
        const bool ok = v < a.n;
        int deg = 0, sp = -1;
        if (ok) {
            const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
            deg = e - s;
            if (natural) {
                int lo = s, hi = e;
                while (lo < hi) {
                    const int mid = lo + ((hi - lo) >> 1);
                    if (a.colp[mid] < v) lo = mid + 1;
                    else hi = mid;
                }
                sp = lo - s;
                a.split[v] = sp;
            } else {
                sp = a.split[v];
            }
            a.conf[v] = sp;
            a.color[v] = 0;
        }
        stage_append(a, &stg, ok && sp == 0, v, deg, fset(1));
        stage_maybe_flush(a, &stg, fset(1));
    }
    stage_flush(a, &stg, fset(1));
}

// Round k: colour the ready list, release later neighbours into round k+1's.
// Log row k-1: vertices coloured and their degree sum; row k is cleared for
// the next round.
__global__ __launch_bounds__(kBlock) void k_flow(Args a, int k) {
    __shared__ uint64_t red[kBlock / kWave];
    __shared__ Stage stg;
    const ChunkMap m = make_map(a.ctl, fset(k));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int usize = 0;
        for (int b = 0; b < kBins; ++b) usize += m.cnt[b];
        for (int b = 0; b < 8; ++b) a.ctl->cnt[fset(k + 2)][b] = 0;
        if (usize > 0) {
            a.ctl->rounds = k;
            if (k - 1 < kMaxLog) a.log[kLogW * (k - 1)] = usize;
            if (k < kMaxLog)
                for (int i = 0; i < kLogW; ++i) a.log[kLogW * k + i] = 0;
        }
    }
    if ((int)blockIdx.x >= m.total) return;
    stage_init(a, &stg);
    long long ncol = 0, work = 0;
    const int ns = fset(k + 1);
#define F_GS(GS, L, C, LOC) flow_chunk<GS>(a, &stg, k, L, C, LOC, &ncol, &work)
#define F_BLOCK(V) flow_block(a, &stg, k, (V), red, &ncol, &work)
#define F_AFTER() stage_maybe_flush(a, &stg, ns)
    GC_WALK_CHUNKS(a, m, fset(k), F_GS, F_BLOCK, F_AFTER)
#undef F_GS
#undef F_BLOCK
#undef F_AFTER
    stage_flush(a, &stg, ns);
    block_add_log(ncol, (long long*)&a.ctl->committed);
    if (k - 1 < kMaxLog) block_add_log(work, &a.log[kLogW * (k - 1) + 1]);
}

// Largest row length (the colour bound Delta + 1 picks the state width).
__global__ __launch_bounds__(kBlock) void k_maxdeg(int n, const int* __restrict__ row_ptr, Ctl* ctl) {
    int mx = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
        mx = max(mx, row_ptr[v + 1] - row_ptr[v]);
    for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    if (__lane_id() == 0 && mx) atomicMax(&ctl->maxdeg, mx);
}

// ---------------------------------------------------------------------------
// Set-up: clear colours, split points, initial binned worklist.
// ---------------------------------------------------------------------------

// Natural order (no priority): rows are sorted, so the neighbours preceding v
// are the prefix below v; split[v] = lower_bound(row, v) - row start.
__global__ __launch_bounds__(kBlock) void k_setup_natural(Args a, int* split) {
    __shared__ Stage st;
    stage_init(a, &st);
    const int stride = gridDim.x * kBlock;
    for (int base = blockIdx.x * kBlock; base < a.n; base += stride) {
        const int v = base + (int)threadIdx.x;
        const bool ok = v < a.n;
        int deg = 0;
        if (ok) {
            const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
            deg = e - s;
            int lo = s, hi = e;
            while (lo < hi) {
                const int mid = lo + ((hi - lo) >> 1);
                if (a.colp[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            split[v] = lo - s;
            a.color[v] = 0;
        }
        stage_append(a, &st, ok, v, deg, 0);
        stage_maybe_flush(a, &st, 0);
    }
    stage_flush(a, &st, 0);
}

// Priority order, step 1: clear colours and bin every vertex.
// Vertices per degree bin (the list sets place bin b after bins 0..b-1).
__global__ __launch_bounds__(kBlock) void k_bin_pop(Args a) {
    __shared__ int h[kBins];
    if (a.ctl->err) return;  // the CSR failed validation: nothing is read
    if (threadIdx.x < kBins) h[threadIdx.x] = 0;
    __syncthreads();
    int c[kBins] = {0, 0, 0, 0, 0};
    for (int v = blockIdx.x * kBlock + (int)threadIdx.x; v < a.n; v += gridDim.x * kBlock) {
        const int b = bin_of(a.row_ptr[v + 1] - a.row_ptr[v], a.cfg);
#pragma unroll
        for (int i = 0; i < kBins; ++i) c[i] += b == i;
    }
#pragma unroll
    for (int i = 0; i < kBins; ++i) {
        const int x = group_sum<kWave>(c[i]);
        if (__lane_id() == 0 && x) atomicAdd(&h[i], x);
    }
    __syncthreads();
    if (threadIdx.x < kBins && h[threadIdx.x]) atomicAdd(&a.ctl->binpop[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(kBlock) void k_setup_bins(Args a) {
    __shared__ Stage st;
    if (a.ctl->err) return;  // the CSR failed validation: nothing is read
    stage_init(a, &st);
    const int stride = gridDim.x * kBlock;
    for (int base = blockIdx.x * kBlock; base < a.n; base += stride) {
        const int v = base + (int)threadIdx.x;
        const bool ok = v < a.n;
        int deg = 0;
        if (ok) {
            deg = a.row_ptr[v + 1] - a.row_ptr[v];
            a.color[v] = 0;
        }
        stage_append(a, &st, ok, v, deg, 0);
        stage_maybe_flush(a, &st, 0);
    }
    stage_flush(a, &st, 0);
}

__device__ __forceinline__ bool precedes(const uint32_t* __restrict__ key, int w, uint32_t kv, int v) {
    const uint32_t kw = key[w];
    return kw < kv || (kw == kv && w < v);
}

// Priority order, step 2: copy each row with the preceding neighbours first,
// in one pass: preceding entries fill the row from its start upwards, later
// ones from its end downwards (the order inside each segment is irrelevant
// to every engine), so each neighbour's key is gathered once.
template <int GS>
__device__ __forceinline__ void reorder_group(const int* __restrict__ col, int* __restrict__ out,
                                              int* __restrict__ split, const uint32_t* __restrict__ key,
                                              int v, int s, int e, int lig, int lane) {
    const uint32_t kv = key[v];
    int plo = s, phi = e;
    const uint64_t below = (lig == 0) ? 0ull : ((1ull << lig) - 1ull);
    for (int p0 = s; p0 < e; p0 += 4 * GS) {
        int w[4];
        bool in[4], lo[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j * GS + lig;
            in[j] = p < e;
            w[j] = in[j] ? col[p] : v;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) lo[j] = in[j] && precedes(key, w[j], kv, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t blo = group_bits<GS>(__ballot(lo[j]), lane);
            const uint64_t bhi = group_bits<GS>(__ballot(in[j] && !lo[j]), lane);
            if (lo[j]) out[plo + __popcll(blo & below)] = w[j];
            else if (in[j]) out[phi - 1 - __popcll(bhi & below)] = w[j];
            plo += __popcll(blo);
            phi -= __popcll(bhi);
        }
    }
    if (lig == 0) split[v] = plo - s;
}

template <int GS>
__device__ __forceinline__ void reorder_chunk(const Args& a, const int* col, int* out, int* split,
                                              const uint32_t* key, const int* list, int cnt, int local) {
    constexpr int CV = kBlock / GS;
    const int lane = __lane_id();
    const int lig = threadIdx.x & (GS - 1);
    const int idx = local * CV + (int)threadIdx.x / GS;
    if (idx < cnt) {
        const int v = list[idx];
        reorder_group<GS>(col, out, split, key, v, a.row_ptr[v], a.row_ptr[v + 1], lig, lane);
    }
}

// One workgroup per hub row: one pass of 256-entry tiles with block-wide
// offsets, preceding entries upwards from the start, later ones downwards
// from the end.
__device__ void reorder_hub(const Args& a, const int* __restrict__ col, int* __restrict__ out,
                            int* __restrict__ split, const uint32_t* __restrict__ key, int v, int* sh) {
    const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
    const int lane = __lane_id();
    const int wid = threadIdx.x / kWave;
    const uint32_t kv = key[v];
    const uint64_t below = __lanemask_lt();
    int plo = s, phi = e;
    for (int p0 = s; p0 < e; p0 += kBlock) {
        const int p = p0 + (int)threadIdx.x;
        int w = 0;
        bool lo = false;
        if (p < e) {
            w = col[p];
            lo = precedes(key, w, kv, v);
        }
        const uint64_t blo = __ballot(p < e && lo);
        const uint64_t bhi = __ballot(p < e && !lo);
        if (lane == 0) {
            sh[wid] = __popcll(blo);
            sh[4 + wid] = __popcll(bhi);
        }
        __syncthreads();
        int olo = 0, ohi = 0, tlo = 0, thi = 0;
        for (int k = 0; k < kBlock / kWave; ++k) {
            if (k < wid) {
                olo += sh[k];
                ohi += sh[4 + k];
            }
            tlo += sh[k];
            thi += sh[4 + k];
        }
        __syncthreads();
        if (p < e) {
            if (lo) out[plo + olo + __popcll(blo & below)] = w;
            else out[phi - 1 - ohi - __popcll(bhi & below)] = w;
        }
        plo += tlo;
        phi -= thi;
    }
    if (threadIdx.x == 0) split[v] = plo - s;
}

__global__ __launch_bounds__(kBlock) void k_reorder(Args a, const int* __restrict__ col, int* __restrict__ out,
                                                    int* __restrict__ split, const uint32_t* __restrict__ key) {
    __shared__ int sh[16];
    const ChunkMap m = make_map(a.ctl, 0);
    for (int c = blockIdx.x; c < m.total; c += gridDim.x) {
        const int b = chunk_bin(m, c);
        const int local = c - m.start[b];
        const int* list = a.lists + pick5(m.off, b);
        switch (b) {
            case 0: reorder_chunk<1>(a, col, out, split, key, list, m.cnt[0], local); break;
            case 1: reorder_chunk<4>(a, col, out, split, key, list, m.cnt[1], local); break;
            case 2: reorder_chunk<16>(a, col, out, split, key, list, m.cnt[2], local); break;
            case 3: reorder_chunk<64>(a, col, out, split, key, list, m.cnt[3], local); break;
            default: reorder_hub(a, col, out, split, key, list[local], sh); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Validation (opt-in) and statistics.
// ---------------------------------------------------------------------------

enum : int { kErrRowPtr = 1, kErrColRange = 2, kErrUnsorted = 4, kErrAsym = 8 };

__global__ __launch_bounds__(kBlock) void k_validate_rows(int n, int nnz, const int* __restrict__ row_ptr,
                                                          Ctl* ctl) {
    int bad = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v <= n; v += gridDim.x * kBlock) {
        const int r = row_ptr[v];
        if (r < 0 || r > nnz) bad |= kErrRowPtr;
        if (v == 0 && r != 0) bad |= kErrRowPtr;
        if (v < n && row_ptr[v + 1] < r) bad |= kErrRowPtr;
    }
    if (bad) atomicOr(&ctl->err, bad);
}

__global__ __launch_bounds__(kBlock) void k_validate_cols(int n, const int* __restrict__ row_ptr,
                                                          const int* __restrict__ col, int need_sorted,
                                                          Ctl* ctl) {
    if (ctl->err) return;  // row offsets already failed: rows cannot be walked
    int bad = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int s = row_ptr[v], e = row_ptr[v + 1];
        for (int p = s; p < e; ++p) {
            const int w = col[p];
            if (w < 0 || w >= n) {
                bad |= kErrColRange;
                continue;
            }
            if (p > s && col[p - 1] > w) bad |= kErrUnsorted;
        }
    }
    if (bad) atomicOr(&ctl->err, bad);
    (void)need_sorted;
}

// Symmetry: every entry (v, w) needs v in row w.  Rows are sorted (checked
// first), so a binary search decides it.
__global__ __launch_bounds__(kBlock) void k_validate_sym(int n, const int* __restrict__ row_ptr,
                                                         const int* __restrict__ col, Ctl* ctl) {
    if (ctl->err) return;  // ids out of range or rows unsorted: no search
    int bad = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int s = row_ptr[v], e = row_ptr[v + 1];
        for (int p = s; p < e; ++p) {
            const int w = col[p];
            int lo = row_ptr[w], hi = row_ptr[w + 1];
            while (lo < hi) {
                const int mid = lo + ((hi - lo) >> 1);
                if (col[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            if (lo >= row_ptr[w + 1] || col[lo] != v) bad |= kErrAsym;
        }
    }
    if (bad) atomicOr(&ctl->err, bad);
}

__global__ __launch_bounds__(kBlock) void k_maxcolor(int n, const int* __restrict__ color, Ctl* ctl) {
    int mx = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) mx = max(mx, color[v]);
    for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    if (__lane_id() == 0 && mx) atomicMax(&ctl->maxcolor, mx);
}

__global__ void k_zero_ctl(Ctl* ctl) {
    int* p = reinterpret_cast<int*>(ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / 4); i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t ctl, log, tent, told, conf, cflag, split, lists, dbits, bplane, bcnt, dsum, colp, hid, hrow, hF, act, pref,
        pbuf, vrec, total;
};

// Entries of the pair buffer: one per vertex, at most kPairMaxCap.
int pair_capacity(int32_t n) { return n < kPairMaxCap ? n : kPairMaxCap; }

// Summary regions of a dirty bitmap of n bits (one flag per 2^kSumShift words).
int sum_regions(int32_t n) {
    const int64_t words = ((int64_t)n + 31) / 32;
    return (int)((words + (1 << kSumShift) - 1) >> kSumShift) + 1;
}

Layout layout(int32_t n, int64_t nnz) {
    Layout L;
    const size_t vn = sizeof(int32_t) * (size_t)n;
    size_t off = 0;
    L.ctl = off;   off += align_up(sizeof(Ctl));
    L.log = off;   off += align_up(sizeof(int64_t) * kLogW * (size_t)kMaxLog);
    L.tent = off;  off += align_up(vn);
    L.told = off;  off += align_up(vn);
    L.conf = off;  off += align_up(vn);
    L.cflag = off; off += align_up(vn);
    L.split = off; off += align_up(vn);
    L.lists = off; off += align_up(vn * kSets);
    L.dbits = off; off += align_up(sizeof(uint32_t) * 3 * (((size_t)n + 31) / 32));
    L.bplane = off; off += align_up(sizeof(uint32_t) * 3 * (((size_t)n + 31) / 32));
    L.bcnt = off;  off += align_up(sizeof(int32_t) * 8 * (size_t)kCompactMaxBlocks);
    L.dsum = off;  off += align_up(3 * (size_t)sum_regions(n));
    L.colp = off;  off += align_up(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    // rows of degree > kHeavyDeg: at most nnz / (kHeavyDeg + 1) of them
    const size_t nh = (size_t)(nnz > 0 ? nnz : 0) / (kHeavyDeg + 1) + 1;
    L.hid = off;   off += align_up(vn);
    L.hrow = off;  off += align_up(sizeof(int4) * nh);
    L.hF = off;    off += align_up(sizeof(uint32_t) * kFW * nh);
    L.act = off;   off += align_up(sizeof(int32_t) * 2 * (size_t)(nnz > 0 ? nnz : 1));
    L.pref = off;  off += align_up(vn);
    L.vrec = off;  off += align_up(4 * vn);
    L.pbuf = off;  off += align_up(sizeof(int32_t) * (size_t)pair_capacity(n));
    L.total = off;
    return L;
}

struct DeviceCache {
    void* ws = nullptr;
    size_t bytes = 0;
    int cus = 0;
};

std::mutex g_mu;
std::vector<DeviceCache> g_dev;
// Calls on the library's workspace hold their device's lock from the
// workspace lookup to their return, so that concurrent host threads take
// turns instead of sharing (or freeing) one buffer.
constexpr int kMaxDevices = 64;
std::mutex g_call_mu[kMaxDevices];

// Process-wide tuning: degree-bin limits and blocks per CU of the grids.
int g_bins[4] = {8, 32, 128, 2048};
int g_blocks_per_cu = 4;
// blocks per CU of k_inc_a and k_inc_c (0: g_blocks_per_cu)
int g_kernel_blocks[2] = {0, 0};
// Most rounds a call may take (0: n + 64).  Every engine ends within n
// rounds on valid input, so the default is never reached; a smaller cap
// exercises the GCOLOR_EROUNDS path.
int g_round_cap = 0;
// Vertices left to the sequential finish (GCOLOR_SERIAL_TAIL).
int g_serial_tail = 1024;

int64_t round_limit(int64_t n) {
    std::lock_guard<std::mutex> g(g_mu);
    return g_round_cap > 0 ? g_round_cap : n + 64;
}

// Optional per-kernel timing with HIP events recorded around each launch.
enum { kProfPhase1 = 0, kProfPhase2 = 1, kProfIncA = 2, kProfLists = 3, kProfIncC = 4, kProfFlow = 5, kProfKinds = 6 };
bool g_prof = false;
double g_prof_ms[kProfKinds] = {};
int64_t g_prof_launches[kProfKinds] = {};

struct EventPairs {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t used = 0;
    hipError_t next(hipEvent_t* a, hipEvent_t* b, int k) {
        while (ev.size() < 2 * (used + 1)) {
            hipEvent_t e;
            hipError_t rc = hipEventCreate(&e);
            if (rc != hipSuccess) return rc;
            ev.push_back(e);
        }
        if (kind.size() < used + 1) kind.resize(used + 1);
        kind[used] = k;
        *a = ev[2 * used];
        *b = ev[2 * used + 1];
        ++used;
        return hipSuccess;
    }
};

int32_t* pinned_buffer() {
    thread_local int32_t* buf = nullptr;
    if (!buf) {
        if (hipHostMalloc((void**)&buf, 256, hipHostMallocDefault) != hipSuccess) buf = nullptr;
    }
    return buf;
}

#define GC_CHECK(x)                                \
    do {                                           \
        if ((x) != hipSuccess) return GCOLOR_EHIP; \
    } while (0)

BinCfg current_bins() {
    std::lock_guard<std::mutex> g(g_mu);
    BinCfg c;
    for (int i = 0; i < 4; ++i) c.dmax[i] = g_bins[i];
    return c;
}

int device_cus(int dev) {
    std::lock_guard<std::mutex> g(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    if (!g_dev[dev].cus) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        g_dev[dev].cus = cus;
    }
    return g_dev[dev].cus;
}

int library_workspace(int dev, size_t need, void** out) {
    std::lock_guard<std::mutex> g(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    DeviceCache& d = g_dev[dev];
    if (d.bytes < need) {
        if (d.ws) {
            if (hipFree(d.ws) != hipSuccess) return GCOLOR_EHIP;
            d.ws = nullptr;
            d.bytes = 0;
        }
        if (hipMalloc(&d.ws, need) != hipSuccess) {
            d.ws = nullptr;
            return GCOLOR_EHIP;
        }
        d.bytes = need;
    }
    *out = d.ws;
    return GCOLOR_OK;
}

// Launch with optional HIP events around it.
struct Launcher {
    hipStream_t st;
    bool prof;
    EventPairs* evp;
    template <typename F>
    hipError_t operator()(int kind, F&& launch) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            hipError_t rc = evp->next(&e0, &e1, kind);
            if (rc != hipSuccess) return rc;
            rc = hipEventRecord(e0, st);
            if (rc != hipSuccess) return rc;
        }
        launch();
        hipError_t rc = hipGetLastError();
        if (rc != hipSuccess) return rc;
        if (prof) return hipEventRecord(e1, st);
        return hipSuccess;
    }
};

int validate(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx, Ctl* ctl, int grid,
             int32_t* host, hipStream_t st) {
    k_validate_rows<<<grid, kBlock, 0, st>>>(n, (int)nnz, row_ptr, ctl);
    GC_CHECK(hipGetLastError());
    GC_CHECK(hipMemcpyAsync(host, &ctl->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GC_CHECK(hipStreamSynchronize(st));
    if (host[0]) return GCOLOR_ECSR;
    k_validate_cols<<<grid, kBlock, 0, st>>>(n, row_ptr, col_idx, 1, ctl);
    GC_CHECK(hipGetLastError());
    GC_CHECK(hipMemcpyAsync(host, &ctl->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GC_CHECK(hipStreamSynchronize(st));
    if (host[0]) return GCOLOR_ECSR;
    k_validate_sym<<<grid, kBlock, 0, st>>>(n, row_ptr, col_idx, ctl);
    GC_CHECK(hipGetLastError());
    GC_CHECK(hipMemcpyAsync(host, &ctl->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GC_CHECK(hipStreamSynchronize(st));
    if (host[0]) return GCOLOR_ECSR;
    return GCOLOR_OK;
}

int sum_counts(const int32_t* h) {
    int t = 0;
    for (int b = 0; b < kBins; ++b) t += h[b];
    return t;
}

// Batches end at the round cap, so a colouring returns GCOLOR_EROUNDS
// exactly when it needs more rounds than the cap.
int run_plain(const Args& a, int64_t limit, int grid, Launcher& L, int32_t* host, hipStream_t st) {
    int64_t k = 0;
    int batch = 4;
    for (;;) {
        const int64_t nb = std::min<int64_t>(batch, limit - k);
        for (int64_t j = 0; j < nb; ++j, ++k) {
            const int side = (int)(k & 1), kk = (int)k;
            GC_CHECK(L(kProfPhase1, [&] { k_phase1<<<grid, kBlock, 0, st>>>(a, side, kk); }));
            GC_CHECK(L(kProfPhase2, [&] { k_phase2<<<grid, kBlock, 0, st>>>(a, side, kk); }));
        }
        // worklist of round k (0-based), the next to run
        GC_CHECK(hipMemcpyAsync(host, &a.ctl->cnt[k & 1][0], sizeof(int32_t) * kBins, hipMemcpyDeviceToHost, st));
        GC_CHECK(hipStreamSynchronize(st));
        if (sum_counts(host) == 0) return GCOLOR_OK;
        if (k >= limit) return GCOLOR_EROUNDS;
        batch = std::min(batch * 2, 16);
    }
}

// Round kk's dirty lists, in vertex order, from its bitmap.
hipError_t launch_dirty_lists(const Args& a, int kk, hipStream_t st) {
    const int G = compact_blocks(a.nwords);
    k_dcount<<<G, kBlock, 0, st>>>(a, kk);
    k_dwrite<<<G, kBlock, 0, st>>>(a, kk);
    return hipGetLastError();
}

// Rounds *k, *k + 1, ... up to round `last` (inclusive, at most `limit`)
// or the end, in batches between host checks; *done when the next round's
// dirty list is empty (every vertex committed).  GCOLOR_EROUNDS when rounds
// 1..limit have run and a vertex is left.
template <typename S>
int inc_rounds(const Args& a, int64_t limit, const int* grid, Launcher& L, int32_t* host, hipStream_t st, int* kio,
               int last, int* batch, bool* done) {
    int k = *kio;
    *done = false;
    last = (int)std::min<int64_t>(last, limit);
    for (;;) {
        const int nb = std::max(0, std::min(*batch, last - k + 1));
        for (int j = 0; j < nb; ++j, ++k) {
            GC_CHECK(L(kProfIncA, [&] { k_inc_a<S><<<grid[0], kBlock, 0, st>>>(a, k); }));
            GC_CHECK(L(kProfIncC, [&] { k_inc_c<S><<<grid[1], kBlock, 0, st>>>(a, k); }));
            GC_CHECK(L(kProfLists, [&] { (void)launch_dirty_lists(a, k + 1, st); }));
        }
        // dirty list of the next round k: empty exactly when every vertex is committed
        GC_CHECK(hipMemcpyAsync(host, &a.ctl->cnt[dlist(k)][0], sizeof(int32_t) * kBins, hipMemcpyDeviceToHost, st));
        if (a.tail > 0)  // with a sequential finish: the vertices left
            GC_CHECK(hipMemcpyAsync(host + 8, &a.ctl->committed, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                    st));
        GC_CHECK(hipStreamSynchronize(st));
        *kio = k;
        if (sum_counts(host) == 0) {
            *done = true;
            return GCOLOR_OK;
        }
        if (a.tail > 0 &&
            (long long)a.n - (long long)*reinterpret_cast<const unsigned long long*>(host + 8) <= a.tail) {
            *done = true;  // the rounds since the switch did nothing
            return GCOLOR_OK;
        }
        if (k > limit) return GCOLOR_EROUNDS;
        if (k > last) return GCOLOR_OK;
        *batch = std::min(*batch * 2, 16);
    }
}

// Dataflow rounds in batches between host checks (the batch grows to 256
// rounds: a natural-order graph can need tens of thousands).
int run_dataflow(const Args& a, int64_t n, int64_t limit, int vgrid, int sgrid, int grid, bool natural, Launcher& L,
                 int32_t* host, hipStream_t st) {
    k_flow_seed<<<sgrid, kBlock, 0, st>>>(a, natural ? 1 : 0);
    GC_CHECK(hipGetLastError());
    int64_t k = 1;
    int batch = 4;
    for (;;) {
        const int64_t nb = std::min<int64_t>(batch, limit - k + 1);
        for (int64_t j = 0; j < nb; ++j, ++k) {
            const int kk = (int)k;
            GC_CHECK(L(kProfFlow, [&] { k_flow<<<grid, kBlock, 0, st>>>(a, kk); }));
        }
        // round k's list (the next to run): empty once nothing is left to release
        GC_CHECK(hipMemcpyAsync(host, &a.ctl->cnt[fset((int)k)][0], sizeof(int32_t) * kBins, hipMemcpyDeviceToHost,
                                st));
        GC_CHECK(hipStreamSynchronize(st));
        if (sum_counts(host) == 0) break;
        if (k > limit) return GCOLOR_EROUNDS;
        batch = std::min(batch * 2, 256);
    }
    unsigned long long coloured = 0;
    GC_CHECK(hipMemcpyAsync(&coloured, &a.ctl->committed, sizeof(coloured), hipMemcpyDeviceToHost, st));
    GC_CHECK(hipStreamSynchronize(st));
    return coloured == (unsigned long long)n ? GCOLOR_OK : GCOLOR_EINTERNAL;
}

// Widen the state words into another slot (int8 -> int16 / int32).
template <typename D>
__global__ __launch_bounds__(kBlock) void k_widen(int n, const int8_t* __restrict__ src, D* __restrict__ dst) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) dst[v] = (D)src[v];
}

// ---------------------------------------------------------------------------
// Sequential finish (section "Iterative and degree of concurrency": once
// conflicts are few, the remaining vertices can be coloured sequentially).
// The rounds stop when at most `tail` vertices are uncoloured; those are
// listed, then one workgroup colours them one at a time in ascending
// (priority, id) order, each with the smallest colour none of its neighbours
// holds (committed colours, and colours given earlier in the finish).
// ---------------------------------------------------------------------------
constexpr int kTailMax = 8192;   // largest tail (LDS sort keys: 64 KiB)
constexpr int kTailSet = 5;      // list set holding the tail (unused by the rounds)
constexpr int kTailThreads = 1024;

template <typename S>
__global__ __launch_bounds__(kBlock) void k_tail_collect(Args a) {
    const S* st = static_cast<const S*>(a.st);
    int* list = list_ptr(a, kTailSet, 0);
    for (int base = blockIdx.x * kBlock; base < a.n; base += gridDim.x * kBlock) {
        const int v = base + (int)threadIdx.x;
        const bool left = v < a.n && st[v] > 0;
        const uint64_t m = __ballot(left);
        if (m == 0) continue;
        const int leader = __ffsll((unsigned long long)m) - 1;
        int b = 0;
        if (__lane_id() == leader) b = atomicAdd(&a.ctl->cnt[kTailSet][0], __popcll(m));
        b = __shfl(b, leader);
        if (left) {
            list[b + __popcll(m & __lanemask_lt())] = v;
            a.color[v] = 0;  // uncoloured until the finish reaches it
        }
    }
}

__global__ __launch_bounds__(kTailThreads) void k_tail_finish(Args a) {
    __shared__ unsigned long long keys[kTailMax];
    __shared__ uint64_t red[kTailThreads / kWave];
    const int m = min(a.ctl->cnt[kTailSet][0], kTailMax);
    const int* list = list_ptr(a, kTailSet, 0);
    int P = 1;
    while (P < m) P <<= 1;
    for (int i = threadIdx.x; i < P; i += kTailThreads) {
        if (i < m) {
            const int v = list[i];
            const uint32_t kv = a.key ? a.key[v] : (uint32_t)v;
            keys[i] = ((unsigned long long)kv << 32) | (unsigned)v;
        } else {
            keys[i] = ~0ull;
        }
    }
    __syncthreads();
    // bitonic sort of (priority, id) ascending
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += kTailThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long x = keys[i], y = keys[l];
                    if (((i & k) == 0) == (x > y)) {
                        keys[i] = y;
                        keys[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    constexpr int nw = kTailThreads / kWave;
    for (int i = 0; i < m; ++i) {
        const int v = (int)(unsigned)(keys[i] & 0xffffffffull);
        const int s = a.row_ptr[v], e = a.row_ptr[v + 1];
        int c = 0;
        for (int base = 1; c == 0; base += 64) {
            uint64_t mask = 0;
            for (int p = s + (int)threadIdx.x; p < e; p += kTailThreads) {
                const int w = a.colp[p];
                const unsigned x = (unsigned)(a.color[w] - base);
                if (w != v && x < 64u) mask |= 1ull << x;
            }
            mask = group_or<kWave>(mask);
            if (__lane_id() == 0) red[threadIdx.x / kWave] = mask;
            __syncthreads();
            uint64_t all = 0;
#pragma unroll
            for (int q = 0; q < nw; ++q) all |= red[q];
            __syncthreads();
            if (~all) c = base + __builtin_ctzll(~all);
        }
        if (threadIdx.x == 0) a.color[v] = c;
        __syncthreads();  // the colour is seen by the next vertices' scans
    }
    if (threadIdx.x == 0 && m > 0) atomicAdd((unsigned long long*)&a.ctl->committed, (unsigned long long)m);
}

// Output colours of the incremental engine, written once after the rounds
// (the commits only write state words): minus the word of a committed vertex,
// 0 for a vertex still uncoloured (left to the sequential finish).
template <typename S>
__global__ __launch_bounds__(kBlock) void k_inc_colors(int n, const S* __restrict__ st, int* __restrict__ color) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int x = st[v];
        color[v] = x < 0 ? -x : 0;
    }
}

// The same for the stream-ordered colouring, whose state words are 32-bit
// from round 128 on only when round 128 had work (ctl->widened).
__global__ __launch_bounds__(kBlock) void k_inc_colors_async(int n, const int8_t* __restrict__ narrow,
                                                             const int32_t* __restrict__ wide, const Ctl* ctl,
                                                             int* __restrict__ color) {
    const bool w = ctl->widened != 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int x = w ? wide[v] : (int)narrow[v];
        color[v] = x < 0 ? -x : 0;
    }
}

// Stream-ordered colouring: the round count is not known to the host, so the
// engine enqueues a fixed budget of rounds; a round whose dirty list is empty
// finds no work and its blocks return at once.  The state widens (to int32)
// before round 128 only when round 128 has work.
__global__ __launch_bounds__(kBlock) void k_widen_if_busy(int n, const int8_t* __restrict__ src,
                                                          int32_t* __restrict__ dst, Ctl* ctl, int set) {
    int busy = 0;
    for (int b = 0; b < kBins; ++b) busy += ctl->cnt[set][b];
    if (busy == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->widened = 1;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) dst[v] = (int32_t)src[v];
}

// Device-side end of a stream-ordered colouring: the statistics of the call
// and its status (GCOLOR_ECSR after failed validation, GCOLOR_EROUNDS when
// the round budget ended with vertices left, GCOLOR_EINTERNAL when the
// worklist emptied early).  One thread; the edge work sums the per-round
// worklist degree sums, nnz minus the degrees committed in earlier rounds.
__global__ void k_async_empty(gcolor_stats_t* out) {
    if (threadIdx.x == 0) *out = gcolor_stats_t{0, 0, 0, GCOLOR_OK, 0};
}

__global__ void k_async_finish(const Ctl* ctl, const long long* __restrict__ log, int n, long long nnz,
                               int next_set, gcolor_stats_t* out) {
    if (threadIdx.x != 0) return;
    int status = GCOLOR_OK;
    int left = 0;
    for (int b = 0; b < kBins; ++b) left += ctl->cnt[next_set][b];
    if (ctl->err) status = GCOLOR_ECSR;
    else if (ctl->committed != (unsigned long long)n) status = left ? GCOLOR_EROUNDS : GCOLOR_EINTERNAL;
    const int rounds = ctl->rounds;
    long long ew = 0, e = nnz;
    const int nl = min(rounds, kMaxLog);
    for (int r = 0; r < nl; ++r) {
        ew += e;
        e -= log[kLogW * r + 1];
    }
    gcolor_stats_t st;
    st.rounds = status == GCOLOR_OK ? rounds : 0;
    st.num_colors = status == GCOLOR_OK ? ctl->maxcolor : 0;
    st.edge_work = status == GCOLOR_OK ? ew : 0;
    st.status = status;
    st.serial_tail = 0;
    *out = st;
}

// A tentative colour is at most one above the largest committed colour, and
// that grows by at most one per round, so every colour of rounds 1..127 fits
// a signed byte: the engine starts with 8-bit state words (half the bytes of
// the gathers that dominate every kernel) and, if round 128 is reached,
// widens them to 16 bits (32 when max degree + 1 exceeds 32767).
int run_incremental(Args a, int64_t n, int64_t limit, int vgrid, int sgrid, const int* grid, bool natural, void* wide_slot,
                    Launcher& L, int32_t* host, hipStream_t st) {
    constexpr int kLast8 = 127;
    k_inc_seed<int8_t><<<sgrid, kBlock, 0, st>>>(a, natural ? 1 : 0);
    GC_CHECK(hipGetLastError());
    int width = 1;  // bytes of the state words when the rounds end
    if (a.tail < n) {  // with a sequential finish of every vertex there is no round
        GC_CHECK(L(kProfIncC, [&] { k_inc_c<int8_t><<<grid[1], kBlock, 0, st>>>(a, 1); }));
        GC_CHECK(L(kProfLists, [&] { (void)launch_dirty_lists(a, 2, st); }));
        int k = 2, batch = 4;
        bool done = false;
        int rc = inc_rounds<int8_t>(a, limit, grid, L, host, st, &k, kLast8, &batch, &done);
        if (rc) return rc;
        if (!done) {
            k_maxdeg<<<vgrid, kBlock, 0, st>>>((int)n, a.row_ptr, a.ctl);
            GC_CHECK(hipGetLastError());
            GC_CHECK(hipMemcpyAsync(host, &a.ctl->maxdeg, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            GC_CHECK(hipStreamSynchronize(st));
            const int8_t* narrow = static_cast<const int8_t*>(a.st);
            a.st = wide_slot;
            if (host[0] + 1 <= 32767) {
                k_widen<int16_t><<<vgrid, kBlock, 0, st>>>((int)n, narrow, static_cast<int16_t*>(wide_slot));
                GC_CHECK(hipGetLastError());
                rc = inc_rounds<int16_t>(a, limit, grid, L, host, st, &k, INT_MAX - 16, &batch, &done);
                width = 2;
            } else {
                k_widen<int32_t><<<vgrid, kBlock, 0, st>>>((int)n, narrow, static_cast<int32_t*>(wide_slot));
                GC_CHECK(hipGetLastError());
                rc = inc_rounds<int32_t>(a, limit, grid, L, host, st, &k, INT_MAX - 16, &batch, &done);
                width = 4;
            }
            if (rc) return rc;
        }
    }
    if (width == 1) k_inc_colors<int8_t><<<vgrid, kBlock, 0, st>>>((int)n, static_cast<const int8_t*>(a.st), a.color);
    else if (width == 2) k_inc_colors<int16_t><<<vgrid, kBlock, 0, st>>>((int)n, static_cast<const int16_t*>(a.st), a.color);
    else k_inc_colors<int32_t><<<vgrid, kBlock, 0, st>>>((int)n, static_cast<const int32_t*>(a.st), a.color);
    GC_CHECK(hipGetLastError());
    if (a.tail > 0) {
        // the vertices the rounds left (at most `tail`), one at a time
        if (width == 1) k_tail_collect<int8_t><<<vgrid, kBlock, 0, st>>>(a);
        else if (width == 2) k_tail_collect<int16_t><<<vgrid, kBlock, 0, st>>>(a);
        else k_tail_collect<int32_t><<<vgrid, kBlock, 0, st>>>(a);
        k_tail_finish<<<1, kTailThreads, 0, st>>>(a);
        GC_CHECK(hipGetLastError());
    }
    unsigned long long committed = 0;
    GC_CHECK(hipMemcpyAsync(&committed, &a.ctl->committed, sizeof(committed), hipMemcpyDeviceToHost, st));
    GC_CHECK(hipStreamSynchronize(st));
    return committed == (unsigned long long)n ? GCOLOR_OK : GCOLOR_EINTERNAL;
}

// Device arguments of one colouring: the caller's arrays and the workspace
// carved up by its layout.
Args make_args(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t* colors, char* base,
               const Layout& Lw, Ctl* ctl, long long* log) {
    Args a;
    a.n = n;
    a.row_ptr = row_ptr;
    a.colp = col_idx;
    a.split = reinterpret_cast<int*>(base + Lw.split);
    a.color = colors;
    a.tent = reinterpret_cast<int*>(base + Lw.tent);
    // the incremental engine's state words share the plain engine's slots
    a.st = base + Lw.tent;
    a.conf = reinterpret_cast<int*>(base + Lw.conf);
    a.cflag = reinterpret_cast<int*>(base + Lw.cflag);
    a.lists = reinterpret_cast<int*>(base + Lw.lists);
    a.dbits = reinterpret_cast<unsigned*>(base + Lw.dbits);
    a.bplane = reinterpret_cast<unsigned*>(base + Lw.bplane);
    a.nwords = (int)(((int64_t)n + 31) / 32);
    a.ctl = ctl;
    a.log = log;
    a.cfg = current_bins();
    a.hid = reinterpret_cast<int*>(base + Lw.hid);
    a.hrow = reinterpret_cast<int4*>(base + Lw.hrow);
    a.hF = reinterpret_cast<unsigned*>(base + Lw.hF);
    a.act = reinterpret_cast<int*>(base + Lw.act);
    a.nnz = nnz;
    a.tail = 0;
    a.key = nullptr;
    a.bcnt = reinterpret_cast<int*>(base + Lw.bcnt);
    a.dsum = reinterpret_cast<unsigned char*>(base + Lw.dsum);
    a.nregions = sum_regions(n);
    a.pref = reinterpret_cast<int*>(base + Lw.pref);
    a.pbuf = reinterpret_cast<int*>(base + Lw.pbuf);
    a.pcap = pair_capacity(n);
    a.vrec = reinterpret_cast<int*>(base + Lw.vrec);

    return a;
}

int run_coloring(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                 const uint32_t* priority, int32_t* colors, void* ws, uint32_t flags,
                 gcolor_stats_t* stats, gcolor_round_t* round_log, int32_t max_log, hipStream_t st) {
    int dev = 0;
    GC_CHECK(hipGetDevice(&dev));
    const int cus = device_cus(dev);
    const Layout Lw = layout(n, nnz);
    char* base = static_cast<char*>(ws);
    Ctl* ctl = reinterpret_cast<Ctl*>(base + Lw.ctl);
    long long* log = reinterpret_cast<long long*>(base + Lw.log);
    int32_t* host = pinned_buffer();
    if (!host) return GCOLOR_EHIP;
    const bool plain = (flags & GCOLOR_PLAIN) != 0;
    const bool flow = (flags & GCOLOR_DATAFLOW) != 0;
    const bool natural = priority == nullptr;
    int grid, kgrid[2];
    {
        std::lock_guard<std::mutex> g(g_mu);
        grid = cus * g_blocks_per_cu;
        for (int i = 0; i < 2; ++i) kgrid[i] = cus * (g_kernel_blocks[i] > 0 ? g_kernel_blocks[i] : g_blocks_per_cu);
    }

    k_zero_ctl<<<1, 64, 0, st>>>(ctl);
    GC_CHECK(hipGetLastError());
    if (flags & GCOLOR_VALIDATE) {
        const int rc = validate(n, nnz, row_ptr, col_idx, ctl, grid, host, st);
        if (rc) return rc;
    }

    Args a = make_args(n, nnz, row_ptr, col_idx, colors, base, Lw, ctl, log);
    a.key = priority;
    if (flags & GCOLOR_SERIAL_TAIL) {
        std::lock_guard<std::mutex> g(g_mu);
        a.tail = g_serial_tail;
    }

    const int vgrid = std::max(1, std::min(grid, (n + kBlock - 1) / kBlock));
    // the seed kernels wait on binary searches of the rows: more workgroups
    // in flight than the round kernels use
    const int sgrid = std::max(1, std::min(cus * kSeedBlocksPerCu, (n + kBlock - 1) / kBlock));
    k_bin_pop<<<sgrid, kBlock, 0, st>>>(a);
    if (!natural) {
        // rows reordered so that the neighbours preceding v come first
        int* colp = reinterpret_cast<int*>(base + Lw.colp);
        k_setup_bins<<<vgrid, kBlock, 0, st>>>(a);
        GC_CHECK(hipGetLastError());
        k_reorder<<<grid, kBlock, 0, st>>>(a, col_idx, colp, a.split, priority);
        GC_CHECK(hipGetLastError());
        a.colp = colp;
    }

    thread_local EventPairs evp;
    evp.used = 0;
    Launcher L{st, g_prof, &evp};
    const int64_t limit = round_limit(n);
    int rc;
    if (plain) {
        if (natural) {
            k_setup_natural<<<vgrid, kBlock, 0, st>>>(a, a.split);
            GC_CHECK(hipGetLastError());
        }
        rc = run_plain(a, limit, grid, L, host, st);
    } else if (flow) {
        rc = run_dataflow(a, n, limit, vgrid, sgrid, grid, natural, L, host, st);
    } else {
        rc = run_incremental(a, n, limit, vgrid, sgrid, kgrid, natural, base + Lw.told, L, host, st);
    }
    if (rc) return rc;

    if (L.prof) {
        GC_CHECK(hipStreamSynchronize(st));
        std::lock_guard<std::mutex> g(g_mu);
        for (size_t i = 0; i < evp.used; ++i) {
            float ms = 0.f;
            GC_CHECK(hipEventElapsedTime(&ms, evp.ev[2 * i], evp.ev[2 * i + 1]));
            g_prof_ms[evp.kind[i]] += ms;
            g_prof_launches[evp.kind[i]] += 1;
        }
    }

    if (stats || round_log) {
        k_maxcolor<<<grid, kBlock, 0, st>>>(n, colors, ctl);
        GC_CHECK(hipGetLastError());
        Ctl hc;
        GC_CHECK(hipMemcpyAsync(&hc, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        GC_CHECK(hipStreamSynchronize(st));
        const int rounds = hc.rounds;
        const int nl = std::min(rounds, kMaxLog);
        std::vector<long long> hl(kLogW * (size_t)std::max(nl, 1), 0);
        if (nl > 0)
            GC_CHECK(hipMemcpyAsync(hl.data(), log, sizeof(long long) * kLogW * (size_t)nl, hipMemcpyDeviceToHost,
                                    st));
        GC_CHECK(hipStreamSynchronize(st));
        // per round: worklist size and its degree sum
        std::vector<long long> U(nl), E(nl), C(nl, 0), D(nl, 0), DE(nl, 0), SC(nl, 0);
        if (plain) {
            for (int r = 0; r < nl; ++r) {
                U[r] = hl[kLogW * r];
                E[r] = hl[kLogW * r + 1];
                C[r] = U[r] - (r + 1 < nl ? hl[kLogW * (r + 1)] : 0);
            }
        } else if (flow) {
            // the round's list is coloured whole
            for (int r = 0; r < nl; ++r) {
                U[r] = hl[kLogW * r];
                E[r] = hl[kLogW * r + 1];
                C[r] = U[r];
            }
        } else {
            long long u = n, e = nnz;
            for (int r = 0; r < nl; ++r) {
                U[r] = u;
                E[r] = e;
                C[r] = hl[kLogW * r];
                D[r] = hl[kLogW * r + 2];
                DE[r] = hl[kLogW * r + 3];
                SC[r] = hl[kLogW * r + 4];
                u -= hl[kLogW * r];
                e -= hl[kLogW * r + 1];
            }
        }
        if (stats) {
            stats->rounds = rounds;
            stats->num_colors = hc.maxcolor;
            long long ew = 0;
            for (int r = 0; r < nl; ++r) ew += E[r];
            stats->edge_work = ew;
            stats->status = 0;
            stats->serial_tail = a.tail > 0 ? hc.cnt[kTailSet][0] : 0;
        }
        if (round_log) {
            for (int r = 0; r < std::min(nl, max_log); ++r) {
                round_log[r].round = r + 1;
                round_log[r].worklist = U[r];
                round_log[r].edge_work = E[r];
                round_log[r].committed = C[r];
                round_log[r].dirty = D[r];
                round_log[r].dirty_edges = DE[r];
                round_log[r].scanned = SC[r];
            }
        }
    }
    return GCOLOR_OK;
}

// Stream-ordered incremental colouring with a round budget (no host
// synchronisation, no allocation).
int run_async(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* priority,
              int32_t* colors, void* ws, int32_t budget, bool validate, gcolor_stats_t* stats_dev, hipStream_t st) {
    int dev = 0;
    GC_CHECK(hipGetDevice(&dev));
    const int cus = device_cus(dev);
    const Layout Lw = layout(n, nnz);
    char* base = static_cast<char*>(ws);
    Ctl* ctl = reinterpret_cast<Ctl*>(base + Lw.ctl);
    long long* log = reinterpret_cast<long long*>(base + Lw.log);
    int grid, kgrid[2];
    {
        std::lock_guard<std::mutex> g(g_mu);
        grid = cus * g_blocks_per_cu;
        for (int i = 0; i < 2; ++i) kgrid[i] = cus * (g_kernel_blocks[i] > 0 ? g_kernel_blocks[i] : g_blocks_per_cu);
    }
    k_zero_ctl<<<1, 64, 0, st>>>(ctl);
    GC_CHECK(hipGetLastError());
    if (validate) {
        // each stage returns at once when an earlier one found an error
        k_validate_rows<<<grid, kBlock, 0, st>>>(n, (int)nnz, row_ptr, ctl);
        k_validate_cols<<<grid, kBlock, 0, st>>>(n, row_ptr, col_idx, 1, ctl);
        k_validate_sym<<<grid, kBlock, 0, st>>>(n, row_ptr, col_idx, ctl);
        GC_CHECK(hipGetLastError());
    }
    Args a = make_args(n, nnz, row_ptr, col_idx, colors, base, Lw, ctl, log);
    const bool natural = priority == nullptr;
    const int vgrid = std::max(1, std::min(grid, (n + kBlock - 1) / kBlock));
    // the seed kernels wait on binary searches of the rows: more workgroups
    // in flight than the round kernels use
    const int sgrid = std::max(1, std::min(cus * kSeedBlocksPerCu, (n + kBlock - 1) / kBlock));
    k_bin_pop<<<sgrid, kBlock, 0, st>>>(a);
    if (!natural) {
        int* colp = reinterpret_cast<int*>(base + Lw.colp);
        k_setup_bins<<<vgrid, kBlock, 0, st>>>(a);
        k_reorder<<<grid, kBlock, 0, st>>>(a, col_idx, colp, a.split, priority);
        GC_CHECK(hipGetLastError());
        a.colp = colp;
    }
    constexpr int kLast8 = 127;
    k_inc_seed<int8_t><<<sgrid, kBlock, 0, st>>>(a, natural ? 1 : 0);
    k_inc_c<int8_t><<<kgrid[1], kBlock, 0, st>>>(a, 1);
    GC_CHECK(launch_dirty_lists(a, 2, st));
    int k = 2;
    for (; k <= std::min(budget, kLast8); ++k) {
        k_inc_a<int8_t><<<kgrid[0], kBlock, 0, st>>>(a, k);
        k_inc_c<int8_t><<<kgrid[1], kBlock, 0, st>>>(a, k);
        GC_CHECK(launch_dirty_lists(a, k + 1, st));
    }
    GC_CHECK(hipGetLastError());
    if (budget > kLast8) {
        void* wide = base + Lw.told;
        k_widen_if_busy<<<vgrid, kBlock, 0, st>>>(n, static_cast<const int8_t*>(a.st), static_cast<int32_t*>(wide),
                                                 ctl, dlist(kLast8 + 1));
        a.st = wide;
        for (; k <= budget; ++k) {
            k_inc_a<int32_t><<<kgrid[0], kBlock, 0, st>>>(a, k);
            k_inc_c<int32_t><<<kgrid[1], kBlock, 0, st>>>(a, k);
            GC_CHECK(launch_dirty_lists(a, k + 1, st));
        }
        GC_CHECK(hipGetLastError());
    }
    k_inc_colors_async<<<vgrid, kBlock, 0, st>>>(n, reinterpret_cast<const int8_t*>(base + Lw.tent),
                                                 reinterpret_cast<const int32_t*>(base + Lw.told), ctl, colors);
    k_maxcolor<<<grid, kBlock, 0, st>>>(n, colors, ctl);
    k_async_finish<<<1, 64, 0, st>>>(ctl, log, n, (long long)nnz, dlist(budget + 1), stats_dev);
    GC_CHECK(hipGetLastError());
    return GCOLOR_OK;
}

int read_nnz(int32_t n, const int32_t* row_ptr, hipStream_t st, int64_t* nnz) {
    int32_t* host = pinned_buffer();
    if (!host) return GCOLOR_EHIP;
    GC_CHECK(hipMemcpyAsync(host, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GC_CHECK(hipStreamSynchronize(st));
    *nnz = host[0];
    return GCOLOR_OK;
}

// Workspace of the allocation-free entry point: one array per device, part
// of the code object (so it exists on every device the library runs on and
// is held until the process ends).  Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, looked
// up once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;

struct ScratchAddr {
    void* p = nullptr;
};
std::vector<ScratchAddr> g_scratch;  // per device, under g_mu

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GCOLOR_EHIP;
    std::lock_guard<std::mutex> g(g_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1);
    if (!g_scratch[dev].p) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GCOLOR_EHIP;
        g_scratch[dev].p = p;
    }
    *out = g_scratch[dev].p;
    return GCOLOR_OK;
}

}  // namespace

extern "C" {

size_t gcolor_workspace_bytes(int32_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    return layout(n, nnz).total;
}

int color_graph_ex(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* priority,
                   int32_t* colors_out, void* workspace, size_t ws_bytes, uint32_t flags,
                   gcolor_stats_t* stats, gcolor_round_t* round_log, int32_t max_log, gcolor_stream_t stream) {
    if (n < 0) return GCOLOR_EINVAL;
    if (flags & ~(uint32_t)(GCOLOR_VALIDATE | GCOLOR_STATS | GCOLOR_PLAIN | GCOLOR_DATAFLOW | GCOLOR_SERIAL_TAIL))
        return GCOLOR_EINVAL;
    if ((flags & GCOLOR_PLAIN) && (flags & GCOLOR_DATAFLOW)) return GCOLOR_EINVAL;
    if ((flags & GCOLOR_SERIAL_TAIL) && (flags & (GCOLOR_PLAIN | GCOLOR_DATAFLOW))) return GCOLOR_EINVAL;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (n == 0) return GCOLOR_OK;
    if (!row_ptr || !colors_out) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int64_t nnz = 0;
    int rc = read_nnz(n, row_ptr, st, &nnz);
    if (rc) return rc;
    if (nnz < 0) return GCOLOR_ECSR;
    if (nnz > 0 && !col_idx) return GCOLOR_EINVAL;
    const size_t need = gcolor_workspace_bytes(n, nnz);
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < need) return GCOLOR_EWORKSPACE;
    }
    std::unique_lock<std::mutex> call;
    if (!ws) {
        int dev = 0;
        GC_CHECK(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices) return GCOLOR_ENOTSUP;
        call = std::unique_lock<std::mutex>(g_call_mu[dev]);
        rc = library_workspace(dev, need, &ws);
        if (rc) return rc;
    }
    rc = run_coloring(n, nnz, row_ptr, col_idx, priority, colors_out, ws, flags, stats, round_log, max_log, st);
    if (stats) stats->status = rc;
    return rc;
}

int color_graph(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* priority,
                int32_t* colors_out, gcolor_stream_t stream) {
    return color_graph_ex(n, row_ptr, col_idx, priority, colors_out, nullptr, 0, 0, nullptr, nullptr, 0, stream);
}

int color_graph_async(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      const uint32_t* priority, int32_t* colors_out, void* workspace, size_t ws_bytes,
                      int32_t max_rounds, uint32_t flags, gcolor_stats_t* stats_dev, gcolor_stream_t stream) {
    if (n < 0 || nnz < 0 || nnz > INT_MAX || max_rounds < 1 || !stats_dev) return GCOLOR_EINVAL;
    if (flags & ~(uint32_t)GCOLOR_VALIDATE) return GCOLOR_EINVAL;
    if (n > 0 && (!row_ptr || !colors_out || !workspace)) return GCOLOR_EINVAL;
    if (nnz > 0 && !col_idx) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n == 0) {
        k_async_empty<<<1, 64, 0, st>>>(stats_dev);
        return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
    }
    if (ws_bytes < gcolor_workspace_bytes(n, nnz)) return GCOLOR_EWORKSPACE;
    return run_async(n, nnz, row_ptr, col_idx, priority, colors_out, workspace, max_rounds,
                     (flags & GCOLOR_VALIDATE) != 0, stats_dev, st);
}

size_t gcolor_noalloc_max_bytes(void) { return kScratchBytes; }

int color_graph_async_noalloc(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              const uint32_t* priority, int32_t* colors_out, int32_t max_rounds, uint32_t flags,
                              gcolor_stats_t* stats_dev, gcolor_stream_t stream) {
    if (n < 0 || nnz < 0 || nnz > INT_MAX || max_rounds < 1 || !stats_dev) return GCOLOR_EINVAL;
    if (flags & ~(uint32_t)GCOLOR_VALIDATE) return GCOLOR_EINVAL;
    if (n > 0 && (!row_ptr || !colors_out)) return GCOLOR_EINVAL;
    if (nnz > 0 && !col_idx) return GCOLOR_EINVAL;
    if (gcolor_workspace_bytes(n, nnz) > kScratchBytes) return GCOLOR_ENOTSUP;
    void* ws = nullptr;
    if (n > 0) {
        const int rc = scratch_address(&ws);
        if (rc) return rc;
    }
    return color_graph_async(n, nnz, row_ptr, col_idx, priority, colors_out, ws, kScratchBytes, max_rounds, flags,
                             stats_dev, stream);
}

const char* gcolor_strerror(int code) {
    switch (code) {
        case GCOLOR_OK: return "ok";
        case GCOLOR_EINVAL: return "invalid argument";
        case GCOLOR_ECSR: return "malformed CSR";
        case GCOLOR_EWORKSPACE: return "workspace too small";
        case GCOLOR_EHIP: return "HIP runtime error";
        case GCOLOR_EROUNDS: return "round cap exceeded";
        case GCOLOR_ENOTSUP: return "unsupported size";
        case GCOLOR_EINTERNAL: return "internal consistency check failed";
        default: return "unknown error";
    }
}

const char* gcolor_version(void) { return "gcolor 0.2 (gfx950)"; }

int gcolor_set_tuning(const int32_t* bin_limits, int32_t blocks_per_cu) {
    if (bin_limits) {
        for (int i = 0; i < 4; ++i)
            if (bin_limits[i] < 0 || (i > 0 && bin_limits[i] < bin_limits[i - 1])) return GCOLOR_EINVAL;
    }
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return GCOLOR_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    if (bin_limits)
        for (int i = 0; i < 4; ++i) g_bins[i] = bin_limits[i];
    if (blocks_per_cu > 0) g_blocks_per_cu = blocks_per_cu;
    return GCOLOR_OK;
}

int gcolor_set_kernel_blocks(int32_t blocks_a, int32_t blocks_c) {
    if (blocks_a < 0 || blocks_a > 64 || blocks_c < 0 || blocks_c > 64) return GCOLOR_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    g_kernel_blocks[0] = blocks_a;
    g_kernel_blocks[1] = blocks_c;
    return GCOLOR_OK;
}

int gcolor_get_kernel_blocks(int32_t* blocks_a, int32_t* blocks_c) {
    std::lock_guard<std::mutex> g(g_mu);
    if (blocks_a) *blocks_a = g_kernel_blocks[0];
    if (blocks_c) *blocks_c = g_kernel_blocks[1];
    return GCOLOR_OK;
}

int gcolor_set_serial_tail(int32_t max_vertices) {
    if (max_vertices < 1 || max_vertices > kTailMax) return GCOLOR_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    g_serial_tail = max_vertices;
    return GCOLOR_OK;
}

int gcolor_get_serial_tail(int32_t* max_vertices) {
    if (!max_vertices) return GCOLOR_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    *max_vertices = g_serial_tail;
    return GCOLOR_OK;
}

int gcolor_set_round_cap(int32_t max_rounds) {
    if (max_rounds < 0) return GCOLOR_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    g_round_cap = max_rounds;
    return GCOLOR_OK;
}

int gcolor_get_round_cap(int32_t* max_rounds) {
    std::lock_guard<std::mutex> g(g_mu);
    if (max_rounds) *max_rounds = g_round_cap;
    return GCOLOR_OK;
}

int gcolor_get_tuning(int32_t* bin_limits, int32_t* blocks_per_cu) {
    std::lock_guard<std::mutex> g(g_mu);
    if (bin_limits)
        for (int i = 0; i < 4; ++i) bin_limits[i] = g_bins[i];
    if (blocks_per_cu) *blocks_per_cu = g_blocks_per_cu;
    return GCOLOR_OK;
}

int gcolor_profile(int32_t enable) {
    std::lock_guard<std::mutex> g(g_mu);
    g_prof = enable != 0;
    for (int i = 0; i < kProfKinds; ++i) {
        g_prof_ms[i] = 0;
        g_prof_launches[i] = 0;
    }
    return GCOLOR_OK;
}

int gcolor_profile_read(int32_t kernel, double* total_ms, int64_t* launches) {
    if (kernel < 0 || kernel >= kProfKinds) return GCOLOR_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    if (total_ms) *total_ms = g_prof_ms[kernel];
    if (launches) *launches = g_prof_launches[kernel];
    return GCOLOR_OK;
}

}  // extern "C"
