// Block Gauss-Seidel variant of the speculative colouring (Algorithm 2 with
// the static schedule of the section "Scalability Results": each thread owns
// a fixed contiguous range of vertices, visits it in index order and sees
// its own colours of the current round at once).
//
// Blocks are the id ranges [b*B, (b+1)*B).  Round k, U = uncoloured vertices:
//   phase 1 (k_blk_first, one wavefront per block): the block's vertices of
//     U in ascending id take the smallest colour held neither by a coloured
//     neighbour nor by a neighbour of the same block chosen earlier in this
//     round (kept in LDS while the block is coloured, and written to tent);
//   phase 2 (k_blk_check, one wavefront per 64 vertices): v in U loses when a
//     neighbour holds its colour (tent for vertices of U, the committed
//     colour otherwise) and precedes it in (key, id) order; winners commit
//     at once (this pass reads the committed colours of its own vertices
//     only) and OR their colour into their neighbours' masks of committed
//     colours; losers form U for round k+1.
// The kernel boundaries order the phases, so the result is a function of the
// input and B.  B = 1 is Algorithm 2 itself; one block holding every vertex
// is the serial greedy in index order, done in one round.  Every round
// commits the uncoloured vertex first in (key, id) order, so a graph of n
// vertices needs at most n rounds.
//
// Memory: colors_out holds the committed colours (0 = uncoloured); the
// workspace holds the round counters (64 slots of 128 bytes), tent
// (int32[n]), byte copies of the committed and current colours, clamped at
// 255 (c8, t8: uint8[n]), per vertex whether it may have a neighbour
// earlier in its block (hp: uint8[n], decided by the first walk of its row)
// and the mask of its neighbours' committed colours 1..64 (fm: uint64[n]).
// Phase 1 takes the committed colours from fm and walks a row only for the
// neighbours inside the block, and only while hp is set; a vertex with 1..64
// all taken scans its row with the int32 colours.  Phase 2 gathers the
// bytes: equal bytes are equal colours unless both sides are 255 or more
// (then tent decides).  Block sizes run from 1 to kMaxBlock (LDS per
// wavefront of phase 1: 4 bytes and 1 bit per vertex of its block plus the
// state of one 64-vertex chunk).
//
// Both row passes work on chunks of 64 consecutive vertices: a wavefront
// compacts the chunk's vertices of U, prefix-sums their degrees and walks
// their rows as one concatenated range, 256 entries per step (four
// consecutive ones per lane), so a hub row is spread over every lane and
// light rows share a step.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "gcolor.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlock = 2048;

// Round counters, spread over kSlots cache lines: workgroup b adds to slot
// b % kSlots, so the one-wavefront-per-chunk grid (tens of thousands of
// workgroups) does not queue its device-scope atomics on one address; the
// host sums the slots.
constexpr int kSlots = 64;
struct BlkSlot {
    unsigned long long committed;  // vertices committed so far
    long long work;                // sum over rounds of the degrees of U
    int32_t rounds;                // last round that committed a vertex
    int32_t maxcolor;
    int32_t pad[26];
};
static_assert(sizeof(BlkSlot) == 128, "counter slot");
struct BlkCtl {
    BlkSlot slot[kSlots];
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct BlkLayout {
    size_t tent, c8, t8, hp, fm, total;
};

BlkLayout blk_layout(int32_t n) {
    BlkLayout L;
    const size_t vn = sizeof(int32_t) * (size_t)(n > 0 ? n : 1);
    L.tent = align_up(sizeof(BlkCtl));
    const size_t bn = (size_t)(n > 0 ? n : 1);
    L.c8 = L.tent + align_up(vn);
    L.t8 = L.c8 + align_up(bn);
    L.hp = L.t8 + align_up(bn);
    L.fm = L.hp + align_up(bn);
    L.total = L.fm + align_up(sizeof(unsigned long long) * bn);
    return L;
}

__device__ __forceinline__ bool blk_before(const uint32_t* __restrict__ key, int w, int v) {
    if (!key) return w < v;
    const uint32_t kw = key[w], kv = key[v];
    return kw < kv || (kw == kv && w < v);
}

__device__ __forceinline__ uint8_t blk_byte(int c) { return (uint8_t)min(c, 255); }

__global__ void k_blk_init(int n, int* __restrict__ color, uint8_t* __restrict__ c8, uint8_t* __restrict__ hp,
                           unsigned long long* __restrict__ fm, BlkCtl* ctl) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    int* c = reinterpret_cast<int*>(ctl);
    for (int j = i; j < (int)(sizeof(BlkCtl) / sizeof(int)); j += gridDim.x * kThreads) c[j] = 0;
    for (int v = i; v < n; v += gridDim.x * kThreads) {
        color[v] = 0;
        c8[v] = 0;
        hp[v] = 1;  // not known yet: the first walk of the row decides
        fm[v] = 0;
    }
}

// Colour of neighbour w as vertex v (block starting at v0) sees it in
// phase 1: the committed colour, or this round's choice of an earlier
// vertex of the same block (LDS), else 0 (no constraint).
__device__ __forceinline__ int blk_seen(const int* __restrict__ color, const int* lt, int w, int v, int v0) {
    if (w == v) return 0;
    const int c = color[w];
    return (c == 0 && w >= v0 && w < v) ? lt[w - v0] : c;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront LDS for a chunk of 64 consecutive vertices.  For the k-th
// uncoloured vertex of the chunk (ascending id): its row start, its position
// in the chunk, the sum of the degrees of the uncoloured vertices before it
// (pre[nU] = the chunk's total) and, in phase 2, its tentative colour.  m and
// d collect per vertex what the chunk's row walk finds.
struct ChunkLds {
    unsigned long long m[64];  // phase 1: colours 1..64 taken; phase 2: nonzero = loses
    unsigned long long d[64];  // phase 1: uncoloured earlier vertices of the chunk adjacent
    int pre[65];
    int rs[64];
    int qp[64];
    int tv[64];
    int hpf[64];  // phase 1: a neighbour earlier in the same block was seen
    int pad[3];
};
static_assert(sizeof(ChunkLds) % 8 == 0, "chunk LDS alignment");

// LDS of one wavefront of k_blk_first: its chunk state, one int per vertex
// of its block (the choices), then one bit per vertex of its block (still
// uncoloured at the start of the round).
__host__ __device__ constexpr size_t blk_lt_bytes(int B) { return ((size_t)B * sizeof(int) + 7) & ~(size_t)7; }
__host__ __device__ constexpr size_t blk_wave_lds(int B) {
    return sizeof(ChunkLds) + blk_lt_bytes(B) + sizeof(unsigned long long) * (((size_t)B + 63) / 64);
}

// Sets up the chunk [c0, c1): returns the mask of its uncoloured vertices
// (bit q = vertex c0 + q); for them fills pre/rs/qp (and tv from tent when
// tent is given), clears d and hpf and sets m to fm (0 without fm); with hp,
// the rows of vertices whose hp is 0 are left out of the walk.  total = the sum of their degrees, k =
// the calling lane's rank among them.  Uniform over the wavefront.
__device__ __forceinline__ uint64_t chunk_setup(int c0, int c1, const int* __restrict__ row_ptr,
                                                const int* __restrict__ color, const int* __restrict__ tent,
                                                const unsigned long long* __restrict__ fm,
                                                const uint8_t* __restrict__ hp, ChunkLds* L, int lane, int& total,
                                                int& k) {
    const int u = c0 + (lane < c1 - c0 ? lane : 0);
    int s = 0, e = 0;
    bool unc = false;
    if (lane < c1 - c0) {
        s = row_ptr[u];
        e = row_ptr[u + 1];
        unc = color[u] == 0;
    }
    const uint64_t mask = __ballot(unc);
    if (mask == 0) return 0;
    // with hp, a row is walked only while it may hold a neighbour earlier in
    // the block (rows of the others count as empty)
    const int deg = unc && (!hp || hp[u]) ? e - s : 0;
    int x = deg;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    total = __shfl(x, 63);
    k = __popcll(mask & ((1ull << lane) - 1));
    if (unc) {
        L->pre[k] = x - deg;
        L->rs[k] = s;
        L->qp[k] = lane;
        L->m[k] = fm ? fm[u] : 0;
        L->d[k] = 0;
        L->hpf[k] = 0;
        if (tent) L->tv[k] = tent[u];
    }
    if (lane == 0) L->pre[__popcll(mask)] = total;
    wave_sync();
    return mask;
}

// The uncoloured vertex of the chunk whose row holds entry j of the
// concatenated rows: the largest k < nU with pre[k] <= j.
__device__ __forceinline__ int chunk_owner(const ChunkLds* L, int nU, int j) {
    int lo = 0, hi = nU;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L->pre[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Entries i0 .. i0+3 of the chunk's concatenated rows: their owners (-1 past
// the end) and column ids.  One search, then the owner only moves forward.
__device__ __forceinline__ void chunk_entries(const ChunkLds* L, int nU, int total, int i0,
                                              const int* __restrict__ col_idx, int (&o)[4], int (&w)[4]) {
    int oc = i0 < total ? chunk_owner(L, nU, i0) : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int idx = i0 + j;
        o[j] = -1;
        w[j] = 0;
        if (idx < total) {
            while (L->pre[oc + 1] <= idx) ++oc;  // pre[nU] = total > idx bounds the walk
            o[j] = oc;
            w[j] = col_idx[L->rs[oc] + (idx - L->pre[oc])];
        }
    }
}

// First fit for vertex v from colour `base` on, the whole wavefront striding
// its row (four entries per lane per step) and OR-ing masks of the colours
// base..base+63 it sees.  lt must hold the choices of every uncoloured vertex
// of the block before v.
__device__ int blk_first_fit(int v, int v0, int base, const int* __restrict__ row_ptr,
                             const int* __restrict__ col_idx, const int* __restrict__ color, const int* lt,
                             int lane) {
    const int s = row_ptr[v], e = row_ptr[v + 1];
    for (;; base += 64) {
        uint64_t m = 0;
        for (int p0 = s + lane; p0 < e; p0 += 4 * 64) {
            int w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = p0 + j * 64 < e ? col_idx[p0 + j * 64] : v;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const unsigned c = (unsigned)(blk_seen(color, lt, w[j], v, v0) - base);
                if (c < 64u) m |= 1ull << c;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m |= __shfl_xor(m, o);
        if (~m) return base + __builtin_ctzll(~m);
    }
}

// Phase 1: one wavefront per block, in chunks of 64 vertices.  The lanes walk
// the concatenated rows of the chunk's uncoloured vertices and record, per
// vertex, the colours 1..64 that coloured neighbours and uncoloured
// neighbours of earlier chunks of the block hold (the latter from LDS), and
// which earlier uncoloured vertices of the chunk are adjacent.  Then the
// chunk's vertices are settled in ascending id: each takes the first colour
// free of both; a vertex with all of 1..64 taken is settled by a full
// first-fit scan of its row (blk_first_fit).
__global__ __launch_bounds__(kThreads) void k_blk_first(int n, int B, long long nblocks,
                                                        const int* __restrict__ row_ptr,
                                                        const int* __restrict__ col_idx,
                                                        const int* __restrict__ color,
                                                        const uint8_t* __restrict__ c8,
                                                        const unsigned long long* __restrict__ fm,
                                                        uint8_t* __restrict__ hp, int* __restrict__ tent,
                                                        uint8_t* __restrict__ t8) {
    extern __shared__ unsigned long long lds64[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    char* wbase = reinterpret_cast<char*>(lds64) + (size_t)wid * blk_wave_lds(B);
    ChunkLds* L = reinterpret_cast<ChunkLds*>(wbase);
    int* lt = reinterpret_cast<int*>(wbase + sizeof(ChunkLds));
    unsigned long long* ub = reinterpret_cast<unsigned long long*>(wbase + sizeof(ChunkLds) + blk_lt_bytes(B));
    for (long long b = (long long)blockIdx.x * kWaves + wid; b < nblocks; b += (long long)gridDim.x * kWaves) {
        const int v0 = (int)(b * B);
        const int v1 = (int)std::min<long long>(n, (long long)v0 + B);
        for (int i0 = 0; i0 < v1 - v0; i0 += 64) {  // which of the block's vertices are uncoloured
            const unsigned long long bits = __ballot(i0 + lane < v1 - v0 && c8[v0 + i0 + lane] == 0);
            if (lane == 0) ub[i0 >> 6] = bits;
        }
        wave_sync();
        for (long long cc0 = v0; cc0 < v1; cc0 += 64) {
            const int c0 = (int)cc0, c1 = (int)std::min<long long>(v1, cc0 + 64);
            int total = 0, k = 0;
            const uint64_t mask = chunk_setup(c0, c1, row_ptr, color, nullptr, fm, hp, L, lane, total, k);
            if (mask == 0) continue;  // uniform
            const int nU = __popcll(mask);
            int acck = -1;
            uint64_t am = 0, ad = 0;
            bool ahp = false;
            for (int jb = 0; jb < total; jb += 4 * 64) {
                int o[4], w[4];
                chunk_entries(L, nU, total, jb + 4 * lane, col_idx, o, w);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (o[j] < 0) continue;
                    if (o[j] != acck) {
                        if (acck >= 0) {
                            if (am) atomicOr(&L->m[acck], am);
                            if (ad) atomicOr(&L->d[acck], ad);
                            if (ahp) L->hpf[acck] = 1;
                        }
                        am = ad = 0;
                        ahp = false;
                        acck = o[j];
                    }
                    // committed neighbours are in fm already; what is left
                    // is the block's uncoloured vertices before v
                    const int v = c0 + L->qp[o[j]], x = w[j];
                    if (x == v || x < v0 || x >= v) continue;
                    ahp = true;
                    const int i = x - v0;
                    if (!((ub[i >> 6] >> (i & 63)) & 1)) continue;
                    if (x >= c0) {
                        ad |= 1ull << (x - c0);
                        continue;
                    }
                    const int cc = lt[i];
                    if ((unsigned)(cc - 1) < 64u) am |= 1ull << (cc - 1);
                }
            }
            if (acck >= 0) {
                if (am) atomicOr(&L->m[acck], am);
                if (ad) atomicOr(&L->d[acck], ad);
                if (ahp) L->hpf[acck] = 1;
            }
            wave_sync();
            const bool unc = (mask >> lane) & 1;
            uint64_t F = unc ? L->m[k] : 0, dep = unc ? L->d[k] : 0;
            int t = 0;
            for (uint64_t rem = mask; rem; rem &= rem - 1) {
                const int q = __builtin_ctzll(rem);
                int tq = __shfl(~F ? __builtin_ctzll(~F) + 1 : 0, q);
                if (tq == 0) {  // colours 1..64 all taken around vertex c0 + q
                    if (unc && lane < q) lt[c0 - v0 + lane] = t;
                    wave_sync();
                    tq = blk_first_fit(c0 + q, v0, 65, row_ptr, col_idx, color, lt, lane);
                }
                if (lane == q) t = tq;
                if (((dep >> q) & 1) && tq <= 64) F |= 1ull << (tq - 1);
            }
            if (unc) {
                if (hp[c0 + lane] && !L->hpf[k]) hp[c0 + lane] = 0;  // walked: none earlier in the block
                lt[c0 - v0 + lane] = t;
                tent[c0 + lane] = t;
                t8[c0 + lane] = blk_byte(t);
            }
            wave_sync();  // the chunk state and lt are read by the next chunk
        }
    }
}

__device__ __forceinline__ long long blk_block_sum(long long x, long long* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) t += red[i];
    return t;  // valid in thread 0
}

// Phase 2: verdict of every uncoloured vertex against this round's colours,
// one wavefront per chunk of 64 vertices walking the concatenated rows of
// its uncoloured vertices.  tent holds every vertex's current colour: phase
// 1 writes it for the uncoloured vertices only, and a vertex commits the
// value it holds there, so one gather serves both kinds of neighbour.
__global__ __launch_bounds__(kThreads) void k_blk_check(int n, int round, const int* __restrict__ row_ptr,
                                                        const int* __restrict__ col_idx,
                                                        const uint32_t* __restrict__ key, int* __restrict__ color,
                                                        const int* __restrict__ tent,
                                                        const uint8_t* __restrict__ t8, uint8_t* __restrict__ c8,
                                                        unsigned long long* __restrict__ fm, BlkCtl* ctl) {
    __shared__ ChunkLds chunks[kWaves];
    __shared__ long long red[kWaves];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    ChunkLds* L = &chunks[wid];
    long long work = 0, ncom = 0;
    int mx = 0;
    const long long nchunks = ((long long)n + 63) / 64;
    for (long long ch = (long long)blockIdx.x * kWaves + wid; ch < nchunks; ch += (long long)gridDim.x * kWaves) {
        const int c0 = (int)(ch * 64);
        const int c1 = (int)std::min<long long>(n, (long long)c0 + 64);
        int total = 0, k = 0;
        const uint64_t mask = chunk_setup(c0, c1, row_ptr, color, tent, nullptr, nullptr, L, lane, total, k);
        if (mask == 0) continue;  // uniform
        const int nU = __popcll(mask);
        for (int jb = 0; jb < total; jb += 4 * 64) {
            int o[4], w[4], c[4], vv[4];
            bool need[4];
            chunk_entries(L, nU, total, jb + 4 * lane, col_idx, o, w);
#pragma unroll
            for (int j = 0; j < 4; ++j) vv[j] = o[j] >= 0 ? c0 + L->qp[o[j]] : 0;
            // without priorities only a smaller id can precede; a vertex that
            // has lost already needs no more gathers
#pragma unroll
            for (int j = 0; j < 4; ++j) need[j] = o[j] >= 0 && (key || w[j] < vv[j]) && L->m[o[j]] == 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = need[j] ? t8[w[j]] : 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!need[j]) continue;
                const int v = vv[j];
                const int tv = L->tv[o[j]];
                if (w[j] != v && c[j] == (int)blk_byte(tv) && (tv < 255 || tent[w[j]] == tv) &&
                    blk_before(key, w[j], v))
                    atomicOr(&L->m[o[j]], 1ull);
            }
        }
        wave_sync();
        const bool won = ((mask >> lane) & 1) && L->m[k] == 0;
        int t = 0;
        if (won) {  // a winner commits its choice
            t = L->tv[k];
            color[c0 + lane] = t;
            c8[c0 + lane] = blk_byte(t);
            mx = max(mx, t);
            ++ncom;
        }
        if (lane == 0) work += total;
        // the winners put their colour (when at most 64) into the masks of
        // their neighbours, walking their rows as one concatenated range
        const uint64_t wmask = __ballot(won && t <= 64);
        wave_sync();  // the chunk state is rewritten below
        if (wmask) {
            int s = 0, e = 0;
            if ((wmask >> lane) & 1) {
                s = row_ptr[c0 + lane];
                e = row_ptr[c0 + lane + 1];
            }
            const int deg = e - s;
            int x = deg;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            const int wtotal = __shfl(x, 63), nW = __popcll(wmask);
            if ((wmask >> lane) & 1) {
                const int r = __popcll(wmask & ((1ull << lane) - 1));
                L->pre[r] = x - deg;
                L->rs[r] = s;
                L->qp[r] = lane;
                L->tv[r] = t;
            }
            if (lane == 0) L->pre[nW] = wtotal;
            wave_sync();
            for (int jb = 0; jb < wtotal; jb += 4 * 64) {
                int o[4], w[4];
                chunk_entries(L, nW, wtotal, jb + 4 * lane, col_idx, o, w);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (o[j] >= 0 && w[j] != c0 + L->qp[o[j]])
                        atomicOr(&fm[w[j]], 1ull << (L->tv[o[j]] - 1));
            }
        }
        wave_sync();  // the chunk state is rewritten by the next chunk
    }
    // one update of this workgroup's slot: the work and commit sums share a
    // word per wavefront (commits < 2^20 per workgroup), the largest colour
    // its own
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    __shared__ int rmx[kWaves];
    if (lane == 0) rmx[wid] = mx;
    const long long t = blk_block_sum((work << 20) | ncom, red);
    if (threadIdx.x == 0 && t) {
        BlkSlot* sl = &ctl->slot[blockIdx.x % kSlots];
        int m = 0;
        for (int i = 0; i < kWaves; ++i) m = max(m, rmx[i]);
        const long long c = t & ((1 << 20) - 1);
        atomicAdd((unsigned long long*)&sl->work, (unsigned long long)(t >> 20));
        if (c) {
            atomicAdd(&sl->committed, (unsigned long long)c);
            atomicMax(&sl->rounds, round);
            atomicMax(&sl->maxcolor, m);
        }
    }
}

struct DevWs {
    void* p = nullptr;
    size_t bytes = 0;
};
std::mutex g_mu;
std::vector<DevWs> g_ws;
// Calls on the library's workspace hold their device's lock until they
// return (concurrent host threads take turns on the one buffer).
constexpr int kMaxDevices = 64;
std::mutex g_call_mu[kMaxDevices];

int blk_workspace(int dev, size_t need, void** out) {
    std::lock_guard<std::mutex> g(g_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    DevWs& d = g_ws[dev];
    if (d.bytes < need) {
        if (d.p && hipFree(d.p) != hipSuccess) return GCOLOR_EHIP;
        d.p = nullptr;
        d.bytes = 0;
        if (hipMalloc(&d.p, need) != hipSuccess) {
            d.p = nullptr;
            return GCOLOR_EHIP;
        }
        d.bytes = need;
    }
    *out = d.p;
    return GCOLOR_OK;
}

// Per-thread pinned staging for the counters and the entry count.
struct BlkHost {
    BlkCtl ctl;
    int32_t nnz;
};
BlkHost* blk_host() {
    thread_local BlkHost* h = nullptr;
    if (!h && hipHostMalloc((void**)&h, sizeof(BlkHost), hipHostMallocDefault) != hipSuccess) h = nullptr;
    return h;
}

// Sums of the round counters over the slots.
struct BlkTotals {
    unsigned long long committed = 0;
    long long work = 0;
    int32_t rounds = 0, maxcolor = 0;
};
BlkTotals blk_totals(const BlkCtl& c) {
    BlkTotals t;
    for (int i = 0; i < kSlots; ++i) {
        t.committed += c.slot[i].committed;
        t.work += c.slot[i].work;
        t.rounds = std::max(t.rounds, c.slot[i].rounds);
        t.maxcolor = std::max(t.maxcolor, c.slot[i].maxcolor);
    }
    return t;
}

#define BLK_CHECK(x)                               \
    do {                                           \
        if ((x) != hipSuccess) return GCOLOR_EHIP; \
    } while (0)

int grid_for(int dev, long long items) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    const long long want = (items + kThreads - 1) / kThreads;
    return (int)std::max<long long>(1, std::min<long long>(want, (long long)cus * 8));
}

// Workgroups for one wavefront per item (the kernels stride past the cap).
int wave_grid(long long items) {
    return (int)std::max<long long>(1, std::min<long long>((items + kWaves - 1) / kWaves, 1 << 22));
}

}  // namespace

extern "C" {

size_t gcolor_blocks_workspace_bytes(int32_t n) {
    if (n < 0) return 0;
    return blk_layout(n).total;
}

int color_graph_blocks(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* priority,
                       int32_t block_size, int32_t* colors_out, void* workspace, size_t ws_bytes,
                       gcolor_stats_t* stats, gcolor_stream_t stream) {
    if (stats) memset(stats, 0, sizeof(*stats));
    if (n < 0 || block_size < 1 || block_size > kMaxBlock) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    if (!row_ptr || !colors_out) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    BlkHost* h = blk_host();
    if (!h) return GCOLOR_EHIP;
    BLK_CHECK(hipMemcpyAsync(&h->nnz, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BLK_CHECK(hipStreamSynchronize(st));
    const int64_t nnz = h->nnz;
    if (nnz < 0) return GCOLOR_ECSR;
    if (nnz > 0 && !col_idx) return GCOLOR_EINVAL;
    int dev = 0;
    BLK_CHECK(hipGetDevice(&dev));
    const BlkLayout L = blk_layout(n);
    void* ws = workspace;
    std::unique_lock<std::mutex> call;
    if (ws) {
        if (ws_bytes < L.total) return GCOLOR_EWORKSPACE;
    } else {
        if (dev < 0 || dev >= kMaxDevices) return GCOLOR_ENOTSUP;
        call = std::unique_lock<std::mutex>(g_call_mu[dev]);
        const int rc = blk_workspace(dev, L.total, &ws);
        if (rc) return rc;
    }
    char* base = static_cast<char*>(ws);
    BlkCtl* ctl = reinterpret_cast<BlkCtl*>(base);
    int* tent = reinterpret_cast<int*>(base + L.tent);
    uint8_t* c8 = reinterpret_cast<uint8_t*>(base + L.c8);
    uint8_t* t8 = reinterpret_cast<uint8_t*>(base + L.t8);
    unsigned long long* fm = reinterpret_cast<unsigned long long*>(base + L.fm);
    uint8_t* hp = reinterpret_cast<uint8_t*>(base + L.hp);
    int32_t cap = 0;
    gcolor_get_round_cap(&cap);
    const long long limit = cap > 0 ? cap : (long long)n + 64;
    const long long nblocks = ((long long)n + block_size - 1) / block_size;
    const int vgrid = grid_for(dev, n);
    // One wavefront per block (phase 1) and per 64-vertex chunk (phase 2): the
    // dispatcher hands out workgroups as others finish, which evens out the
    // degree skew of neighbouring id ranges that a fixed stride would gather
    // onto the same wavefronts.
    const int bgrid = wave_grid(nblocks), cgrid = wave_grid(((long long)n + 63) / 64);
    const size_t lds_bytes = (size_t)kWaves * blk_wave_lds(block_size);

    k_blk_init<<<vgrid, kThreads, 0, st>>>(n, colors_out, c8, hp, fm, ctl);
    BLK_CHECK(hipGetLastError());
    long long k = 0;
    int batch = 4;
    int rc = GCOLOR_OK;
    BlkTotals tot;
    for (;;) {
        const long long nb = std::min<long long>(batch, limit - k);
        for (long long j = 0; j < nb; ++j) {
            ++k;
            k_blk_first<<<bgrid, kThreads, lds_bytes, st>>>(n, block_size, nblocks, row_ptr, col_idx, colors_out,
                                                            c8, fm, hp, tent, t8);
            k_blk_check<<<cgrid, kThreads, 0, st>>>(n, (int)k, row_ptr, col_idx, priority, colors_out, tent, t8, c8,
                                                  fm, ctl);
            BLK_CHECK(hipGetLastError());
        }
        BLK_CHECK(hipMemcpyAsync(&h->ctl, ctl, sizeof(BlkCtl), hipMemcpyDeviceToHost, st));
        BLK_CHECK(hipStreamSynchronize(st));
        tot = blk_totals(h->ctl);
        if (tot.committed >= (unsigned long long)n) break;
        if (k >= limit) {
            rc = GCOLOR_EROUNDS;
            break;
        }
        batch = std::min(batch * 2, 16);
    }
    if (rc == GCOLOR_OK && tot.committed != (unsigned long long)n) rc = GCOLOR_EINTERNAL;
    if (stats) {
        if (rc == GCOLOR_OK) {
            stats->rounds = tot.rounds;
            stats->num_colors = tot.maxcolor;
            stats->edge_work = tot.work;
        }
        stats->status = rc;
    }
    return rc;
}

}  // extern "C"
