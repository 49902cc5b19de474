// Batched colouring: many independent graphs in one persistent launch.
//
// Each graph is coloured exactly as color_graph colours it alone (the
// round-synchronous reading of Algorithm 2 with its precedence rule), so a
// batch is the same function as a loop of single calls; only the execution
// differs.  A work-queue kernel hands graphs to workgroups, largest first
// (edge count); one workgroup runs every round of its graph with workgroup
// barriers instead of kernel boundaries, keeping list lengths in LDS.  The
// rounds are those of the incremental engine of the single-graph path: a
// commit marks "dirty" the later neighbours holding its colour, a dirty
// vertex re-takes first-fit and recounts its conflict counter (preceding
// neighbours with the same tentative colour) while adjusting its later
// neighbours' counters, and candidates whose counter is 0 commit.
//
// Lanes: groups of 8 lanes per vertex (the stencil and geometric graphs of a
// batch have degrees of a few to a few tens; 4 in the LDS path for lists
// longer than one pass), row entries kept in registers between the
// first-fit and the counter pass; longer rows are re-gathered.
//
// Graphs of at most nl vertices (nl is set per launch from the batch's mean
// graph size, at most 65536) and maximum degree at most 126 keep their
// per-vertex state in LDS (see color_one_lds); the others use global memory.
// Per-graph start/end times come from the constant-rate wall clock.  No host
// synchronisation and no allocation happen inside the call, so it can be
// captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>

#include "gcolor.h"

namespace {

constexpr int kG = 8;         // lanes per vertex
constexpr int kCache = 8;     // row entries per lane kept in registers
constexpr int kSortMax = 8192;

struct BCtl {
    int queue;      // next position in the processing order
    int pad[63];
};

struct BArgs {
    int G;
    int64_t V;
    const int64_t* __restrict__ vtx_off;
    const int64_t* __restrict__ edge_off;
    const int* __restrict__ row_ptr;   // concatenated local row pointers, graph g at vtx_off[g] + g
    const int* __restrict__ col_idx;   // concatenated local neighbour ids
    const uint32_t* __restrict__ key;  // priority or null
    int* __restrict__ colors;
    int* __restrict__ colp;            // reordered rows (priority runs)
    int* __restrict__ st;              // state word: > 0 tentative colour, < 0 committed colour
    int* __restrict__ conf;
    int* __restrict__ stamp;
    int* __restrict__ cflag;
    int* __restrict__ split;
    int* __restrict__ lists;           // [6][V]: dirty x3, candidates x2, second-pass
    unsigned* __restrict__ bits;       // 3 bitmaps of (V/32 + G) words
    int64_t nbw;                       // words per bitmap
    int* __restrict__ order;
    BCtl* ctl;
    long long* __restrict__ ticks;     // [2G] start, end (wall clock) or null
    int* __restrict__ rounds;          // [G] or null
    int nl;                            // vertex capacity of the LDS path (0: off)
};

struct GView {
    int n;
    const int* rp;
    const int* col;  // row entries (reordered copy with a priority)
    int* st;
    int* conf;
    int* stamp;
    int* cflag;
    int* split;
    int* color;
    int* lbase;       // list i starts at lbase + i * lstride
    int64_t lstride;
    unsigned* bbase;  // bitmap i starts at bbase + i * bstride
    int64_t bstride;
    __device__ __forceinline__ int* L(int i) const { return lbase + (int64_t)i * lstride; }
    __device__ __forceinline__ unsigned* bits(int i) const { return bbase + (int64_t)i * bstride; }
};

template <int GS>
__device__ __forceinline__ uint64_t gor(uint64_t m) {
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) m |= __shfl_xor(m, o, GS);
    return m;
}

template <int GS>
__device__ __forceinline__ int gsum(int x) {
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, GS);
    return x;
}

__device__ __forceinline__ bool dirty_bit(const unsigned* b, int x) { return (b[x >> 5] >> (x & 31)) & 1u; }

// One workgroup owns all of a graph's working data, so its atomics need only
// workgroup scope (shorter round trips than device-scope ones).
__device__ __forceinline__ int wg_add(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int wg_exch(int* p, int v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned wg_or(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Per-workgroup list lengths live in LDS: cnt[0..2] dirty, [3..4] candidates, [5] second pass.
__device__ __forceinline__ void push(const GView& g, int* cnt, int list, int v) {
    const int slot = atomicAdd(&cnt[list], 1);
    g.L(list)[slot] = v;
}

__device__ __forceinline__ int dl(int k) { return k % 3; }
__device__ __forceinline__ int cl(int k) { return 3 + (k & 1); }

// Later-entry evaluation of dirty vertex w (see the single-graph engine).
__device__ __forceinline__ bool eval_dirty(const GView& g, const unsigned* bits, int k, int w, int p, int lim,
                                           int now, int old, int x, int sx, int* cnt, bool* dlow) {
    if (p < lim) {
        if (dirty_bit(bits, x)) *dlow = true;
        else *cnt += (sx == now);
        return false;
    }
    if (x == w || (sx != now && sx != old)) return false;
    if (dirty_bit(bits, x)) return false;
    if (sx == now) {
        wg_add(&g.conf[x], 1);
        return false;
    }
    if (wg_add(&g.conf[x], -1) != 1) return false;
    return wg_exch(&g.cflag[x], k) != k;
}

// Phase A of round k for dirty vertex w (group of kG lanes).
__device__ void phase_a(const GView& g, int* cnt, int k, int w, int lig) {
    const unsigned* bits = g.bits(dl(k));
    const int s = g.rp[w], e = g.rp[w + 1];
    const int lim = s + g.split[w];
    const int old = g.st[w];
    const bool cached = (e - s) <= kCache * kG;
    int xs[kCache], sv[kCache];
    if (cached) {
#pragma unroll
        for (int j = 0; j < kCache; ++j) {
            const int p = s + lig + j * kG;
            xs[j] = p < e ? g.col[p] : w;
        }
#pragma unroll
        for (int j = 0; j < kCache; ++j) sv[j] = g.st[xs[j]];
    }
    int now = 0;
    for (int base = 1;; base += 64) {
        uint64_t m = 0;
        if (cached) {
#pragma unroll
            for (int j = 0; j < kCache; ++j) {
                const unsigned c = (unsigned)(-sv[j] - base);
                if (c < 64u) m |= 1ull << c;
            }
        } else {
            for (int p = s + lig; p < e; p += kG) {
                const unsigned c = (unsigned)(-g.st[g.col[p]] - base);
                if (c < 64u) m |= 1ull << c;
            }
        }
        m = gor<kG>(m);
        if (~m) {
            now = base + __builtin_ctzll(~m);
            break;
        }
    }
    int c = 0;
    bool dlow = false;
    if (cached) {
#pragma unroll
        for (int j = 0; j < kCache; ++j) {
            const int p = s + lig + j * kG;
            if (p < e && eval_dirty(g, bits, k, w, p, lim, now, old, xs[j], sv[j], &c, &dlow))
                push(g, cnt, cl(k), xs[j]);
        }
    } else {
        for (int p = s + lig; p < e; p += kG) {
            const int x = g.col[p];
            if (eval_dirty(g, bits, k, w, p, lim, now, old, x, g.st[x], &c, &dlow)) push(g, cnt, cl(k), x);
        }
    }
    c = gsum<kG>(c);
    const int d = gsum<kG>(dlow ? 1 : 0);
    if (lig == 0) {
        g.st[w] = now;
        g.conf[w] = c;
        if (d > 0) push(g, cnt, 5, w);
        else if (c == 0 && wg_exch(&g.cflag[w], k) != k) push(g, cnt, cl(k), w);
    }
}

// Phase B: dirty vertices with preceding dirty neighbours add those holding
// the same final new colour.
__device__ void phase_b(const GView& g, int* cnt, int k, int w, int lig) {
    const unsigned* bits = g.bits(dl(k));
    const int s = g.rp[w];
    const int lim = s + g.split[w];
    const int now = g.st[w];
    int c = 0;
    for (int p = s + lig; p < lim; p += kG) {
        const int x = g.col[p];
        if (dirty_bit(bits, x)) c += (g.st[x] == now);
    }
    c = gsum<kG>(c);
    if (lig == 0) {
        const int t = g.conf[w] + c;
        g.conf[w] = t;
        if (t == 0 && wg_exch(&g.cflag[w], k) != k) push(g, cnt, cl(k), w);
    }
}

// Phase C: commit a candidate whose counter is 0; mark its later
// neighbours holding the same tentative colour dirty for round k+1.
__device__ void phase_c(const GView& g, int* cnt, int k, int v, int lig) {
    const int t = g.st[v];
    if (g.conf[v] != 0 || t <= 0) return;  // uniform over the group
    unsigned* nbits = g.bits(dl(k + 1));
    const int s = g.rp[v], e = g.rp[v + 1];
    for (int p = s + g.split[v] + lig; p < e; p += kG) {
        const int u = g.col[p];
        if (u == v || g.st[u] != t) continue;
        if (g.stamp[u] == k + 1) continue;
        if (wg_exch(&g.stamp[u], k + 1) == k + 1) continue;
        wg_or(&nbits[u >> 5], 1u << (u & 31));
        push(g, cnt, dl(k + 1), u);
    }
    if (lig == 0) {
        g.color[v] = t;
        g.st[v] = -t;
    }
}


// ---------------------------------------------------------------------------
// LDS-resident rounds.  A graph of at most nl vertices whose maximum degree is
// at most kLdsMaxDeg keeps its per-vertex state in LDS: signed-byte state
// words (colours are at most max degree + 1 <= 127), byte counters packed
// four to a word and changed with 32-bit atomics (a counter never exceeds the
// degree, so +1 never carries into the next byte, and -1 is only applied to a
// positive counter), two dirty bitmaps alternating by round (the first mark
// of a vertex is the one that sets its bit) and a bitmap of this round's
// candidates.  Row data, split points, colours and lists stay in global
// memory.  A round's chain of dependent accesses then reaches global memory a
// few times instead of about twenty, and it is that chain, slowed by the load
// the rest of the batch puts on the memory system, which paces the long runs
// of small rounds (natural-order grids: ~1250 rounds of ~50 vertices).
constexpr int kLdsMaxDeg = 126;

struct LView {
    int n, nw;
    const int* rp;
    const int* col;
    const int* split;
    int* color;
    int* lbase;
    int64_t lstride;
    int8_t* st;    // LDS: state words
    unsigned* cf;  // LDS: byte counters, four per word
    unsigned* db;  // LDS: dirty bitmaps of rounds with even / odd index
    unsigned* cb;  // LDS: candidates pushed in this round
    __device__ __forceinline__ int* L(int i) const { return lbase + (int64_t)i * lstride; }
    __device__ __forceinline__ unsigned* dbits(int k) const { return db + (k & 1) * nw; }
};

__device__ __forceinline__ unsigned vbit(int v) { return 1u << (v & 31); }

__device__ __forceinline__ int lconf(const LView& g, int v) { return (g.cf[v >> 2] >> ((v & 3) * 8)) & 0xff; }

// Adds d to v's byte counter; returns the byte before.
__device__ __forceinline__ int lconf_add(const LView& g, int v, int d) {
    const unsigned sh = (unsigned)(v & 3) * 8u;
    const unsigned old = atomicAdd(&g.cf[v >> 2], (unsigned)d << sh);
    return (int)((old >> sh) & 0xffu);
}

// First push of candidate x in this round.
__device__ __forceinline__ bool lcand(const LView& g, int x) { return !(atomicOr(&g.cb[x >> 5], vbit(x)) & vbit(x)); }

__device__ __forceinline__ void lpush(const LView& g, int* cnt, int list, int v) {
    const int slot = atomicAdd(&cnt[list], 1);
    g.L(list)[slot] = v;
}

// Entry x (word sx) of dirty vertex w, as eval_dirty with LDS state.
__device__ __forceinline__ void eval_l(const LView& g, int* cnt, const unsigned* bits, int k, int w, bool pre, int now,
                                       int old, int x, int sx, int* c, bool* dlow) {
    if (pre) {
        if (dirty_bit(bits, x)) *dlow = true;
        else *c += (sx == now);
    } else if (x != w && (sx == now || sx == old) && !dirty_bit(bits, x)) {
        if (sx == now) lconf_add(g, x, 1);
        else if (lconf_add(g, x, -1) == 1 && lcand(g, x)) lpush(g, cnt, cl(k), x);
    }
}

template <int GS>
__device__ void phase_a_l(const LView& g, int* cnt, int k, int w, int s, int e, int sp, int lig) {
    const unsigned* bits = g.dbits(k);
    const int lim = s + sp;
    const int old = g.st[w];
    constexpr int KC = GS == 4 ? 2 * kCache : kCache;  // rows up to 64 entries stay in registers
    const bool cached = (e - s) <= KC * GS;
    int xs[KC], sv[KC];
    if (cached) {
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int p = s + lig + j * GS;
            xs[j] = p < e ? g.col[p] : w;
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) sv[j] = g.st[xs[j]];
    }
    int now = 0;
    for (int base = 1;; base += 64) {
        uint64_t m = 0;
        if (cached) {
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                const unsigned c = (unsigned)(-sv[j] - base);
                if (c < 64u) m |= 1ull << c;
            }
        } else {
            for (int p = s + lig; p < e; p += GS) {
                const unsigned c = (unsigned)(-(int)g.st[g.col[p]] - base);
                if (c < 64u) m |= 1ull << c;
            }
        }
        m = gor<GS>(m);
        if (~m) {
            now = base + __builtin_ctzll(~m);
            break;
        }
    }
    int c = 0;
    bool dlow = false;
    if (cached) {
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int p = s + lig + j * GS;
            if (p < e) eval_l(g, cnt, bits, k, w, p < lim, now, old, xs[j], sv[j], &c, &dlow);
        }
    } else {
        for (int p = s + lig; p < e; p += GS) {
            const int x = g.col[p];
            eval_l(g, cnt, bits, k, w, p < lim, now, old, x, g.st[x], &c, &dlow);
        }
    }
    c = gsum<GS>(c);
    const int d = gsum<GS>(dlow ? 1 : 0);
    if (lig == 0) {
        g.st[w] = (int8_t)now;
        // w is dirty, so no other group changes its counter in this phase
        lconf_add(g, w, c - lconf(g, w));
        if (d > 0) lpush(g, cnt, 5, w);
        else if (c == 0 && lcand(g, w)) lpush(g, cnt, cl(k), w);
    }
}

template <int GS>
__device__ void phase_b_l(const LView& g, int* cnt, int k, int w, int s, int e, int sp, int lig) {
    const unsigned* bits = g.dbits(k);
    const int lim = s + sp;
    const int now = g.st[w];
    int c = 0;
    for (int p = s + lig; p < lim; p += GS) {
        const int x = g.col[p];
        if (dirty_bit(bits, x)) c += ((int)g.st[x] == now);
    }
    c = gsum<GS>(c);
    if (lig == 0) {
        const int t = lconf_add(g, w, c) + c;
        if (t == 0 && lcand(g, w)) lpush(g, cnt, cl(k), w);
    }
}

template <int GS>
__device__ void phase_c_l(const LView& g, int* cnt, int k, int v, int s, int e, int sp, int lig) {
    if (lig == 0) atomicAnd(&g.cb[v >> 5], ~vbit(v));  // the candidate bit is free for the next round
    const int t = g.st[v];
    if (lconf(g, v) != 0 || t <= 0) return;  // uniform over the group
    unsigned* nbits = g.dbits(k + 1);
    for (int p = s + sp + lig; p < e; p += GS) {
        const int u = g.col[p];
        if (u == v || (int)g.st[u] != t) continue;
        if (atomicOr(&nbits[u >> 5], vbit(u)) & vbit(u)) continue;  // marked already
        lpush(g, cnt, dl(k + 1), u);
    }
    if (lig == 0) g.st[v] = (int8_t)(-t);  // colors_out is written after the last round
}

// Walk list l[0..m) with groups of GS lanes (vertex i to group tid / GS,
// then i + B / GS, ...), calling body(w, row start, row end, split).  Each
// group loads the row offsets and split of its next vertex, and the list
// entry of the one after, before it processes the current one, so that a
// vertex waits for one global access (its row) instead of three in a chain.
template <int B, int GS, typename F>
__device__ __forceinline__ void lds_walk(const LView& g, const int* l, int m, int tid, F&& body) {
    constexpr int STEP = B / GS;
    int i = tid / GS;
    if (i >= m) return;
    int w = l[i];
    int s = g.rp[w], e = g.rp[w + 1], sp = g.split[w];
    int wn = i + STEP < m ? l[i + STEP] : 0;
    for (;;) {
        const int in = i + STEP;
        int sn = 0, en = 0, spn = 0, wnn = 0;
        if (in < m) {
            sn = g.rp[wn];
            en = g.rp[wn + 1];
            spn = g.split[wn];
        }
        if (in + STEP < m) wnn = l[in + STEP];
        body(w, s, e, sp);
        if (in >= m) break;
        i = in;
        w = wn;
        s = sn;
        e = en;
        sp = spn;
        wn = wnn;
    }
}

// Rounds of graph gi (n vertices, split points set) with LDS state; the
// caller has cleared cnt[].
// Phase P over the m vertices of list l: 8 lanes per vertex while the list
// fits one pass of the workgroup, else 4 (twice the vertices in flight per
// pass for the large rounds; phase A keeps rows up to 64 entries in
// registers either way).
#define LDS_PHASE(P, m, l)                                                                            \
    do {                                                                                              \
        const int m_ = (m);                                                                           \
        const int* l_ = (l);                                                                          \
        if (m_ <= B / 8) {                                                                            \
            lds_walk<B, 8>(g, l_, m_, tid,                                                            \
                           [&](int w_, int s_, int e_, int p_) { P<8>(g, cnt, k, w_, s_, e_, p_, tid & 7); }); \
        } else {                                                                                      \
            lds_walk<B, 4>(g, l_, m_, tid,                                                            \
                           [&](int w_, int s_, int e_, int p_) { P<4>(g, cnt, k, w_, s_, e_, p_, tid & 3); }); \
        }                                                                                             \
    } while (0)

template <int B>
__device__ void color_one_lds(const BArgs& a, const GView& gg, int gi, int* cnt, unsigned char* lds, int& kout) {
    const int tid = threadIdx.x;
    LView g;
    g.n = gg.n;
    g.nw = (a.nl + 31) >> 5;
    g.rp = gg.rp;
    g.col = gg.col;
    g.split = gg.split;
    g.color = gg.color;
    g.lbase = gg.lbase;
    g.lstride = gg.lstride;
    g.st = reinterpret_cast<int8_t*>(lds);
    g.cf = reinterpret_cast<unsigned*>(lds + a.nl);
    g.db = reinterpret_cast<unsigned*>(lds + 2 * (size_t)a.nl);
    g.cb = g.db + 2 * g.nw;
    const int nw = (g.n + 31) >> 5;
    for (int i = tid; i < nw; i += B) {
        g.db[i] = 0u;
        g.db[g.nw + i] = 0u;
        g.cb[i] = 0u;
    }
    unsigned char* cfb = reinterpret_cast<unsigned char*>(g.cf);
    for (int v = tid; v < g.n; v += B) {
        const int sp = g.split[v];
        g.st[v] = 1;
        cfb[v] = (unsigned char)sp;
        if (sp == 0) lpush(g, cnt, cl(1), v);
    }
    if (tid == 0) cnt[dl(2)] = 0;
    __syncthreads();
    int k = 1;
    for (;; ++k) {
        if (k > 1) {
            const int nd = cnt[dl(k)];
            if (nd == 0) break;
            // round k-1's bitmap becomes round k+1's: clear the words of its
            // dirty vertices (every bit set in it belongs to one of them)
            const int np = cnt[dl(k - 1)];
            for (int i = tid; i < np; i += B) g.dbits(k - 1)[g.L(dl(k - 1))[i] >> 5] = 0u;
            if (tid == 0) {
                cnt[cl(k)] = 0;
                cnt[5] = 0;
                cnt[dl(k + 1)] = 0;
            }
            __syncthreads();
            LDS_PHASE(phase_a_l, nd, g.L(dl(k)));
            __syncthreads();
            const int nb = cnt[5];
            if (nb > 0) {
                LDS_PHASE(phase_b_l, nb, g.L(5));
                __syncthreads();
            }
        }
        const int nc = cnt[cl(k)];
        LDS_PHASE(phase_c_l, nc, g.L(cl(k)));
        __syncthreads();
    }
    // the rounds end when no vertex is dirty, which happens only once every
    // vertex has committed (while any is left, the first of a chain of
    // equal tentative colours commits and its successor becomes dirty): the
    // colours go out in one coalesced pass from the state words
    for (int v = tid; v < g.n; v += B) g.color[v] = -(int)g.st[v];
    kout = k;
}

__device__ __forceinline__ bool precedes(const uint32_t* key, int w, uint32_t kv, int v) {
    const uint32_t kw = key[w];
    return kw < kv || (kw == kv && w < v);
}

// Colour graph gi with the whole workgroup (B threads).
template <int B>
__device__ void color_one(const BArgs& a, int gi, int* cnt, unsigned char* lds, int* shmax) {
    constexpr int kPerIt = B / kG;
    const int tid = threadIdx.x;
    const int64_t vo = a.vtx_off[gi], eo = a.edge_off[gi];
    const int n = (int)(a.vtx_off[gi + 1] - vo);
    if (a.ticks && tid == 0) a.ticks[2 * gi] = wall_clock64();
    if (n == 0) {
        if (tid == 0) {
            if (a.rounds) a.rounds[gi] = 0;
            if (a.ticks) a.ticks[2 * gi + 1] = wall_clock64();
        }
        __syncthreads();
        return;
    }
    GView g;
    g.n = n;
    g.rp = a.row_ptr + vo + gi;
    g.col = a.key ? a.colp + eo : a.col_idx + eo;
    g.st = a.st + vo;
    g.conf = a.conf + vo;
    g.stamp = a.stamp + vo;
    g.cflag = a.cflag + vo;
    g.split = a.split + vo;
    g.color = a.colors + vo;
    g.lbase = a.lists + vo;
    g.lstride = a.V;
    const int64_t wbase = (vo >> 5) + gi;
    const int nw = (n + 31) >> 5;
    g.bbase = a.bits + wbase;
    g.bstride = a.nbw;
    const uint32_t* key = a.key ? a.key + vo : nullptr;
    const int* raw = a.col_idx + eo;

    // LDS path when the graph fits and every colour and counter fits a byte
    bool use_lds = false;
    if (a.nl > 0 && n <= a.nl) {
        int md = 0;
        for (int v = tid; v < n; v += B) md = max(md, g.rp[v + 1] - g.rp[v]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) md = max(md, __shfl_xor(md, o));
        if ((tid & 63) == 0) shmax[tid >> 6] = md;
        __syncthreads();
        md = 0;
        for (int i = 0; i < B / 64; ++i) md = max(md, shmax[i]);
        use_lds = md <= kLdsMaxDeg;
        __syncthreads();
    }
    if (tid < 8) cnt[tid] = 0;
    if (!use_lds)
        for (int i = tid; i < 3 * nw; i += B) g.bits(i / nw)[i % nw] = 0u;
    __syncthreads();
    // set-up: split points (reordered rows with a priority), round-1 state
    for (int v = tid; v < n; v += B) {
        const int s = g.rp[v], e = g.rp[v + 1];
        int sp;
        if (!key) {
            int lo = s, hi = e;
            while (lo < hi) {
                const int mid = lo + ((hi - lo) >> 1);
                if (raw[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            sp = lo - s;
        } else {
            const uint32_t kv = key[v];
            int* out = a.colp + eo;
            int nlo = 0;
            for (int p = s; p < e; ++p) nlo += precedes(key, raw[p], kv, v);
            int pl = s, ph = s + nlo;
            for (int p = s; p < e; ++p) {
                const int w = raw[p];
                if (precedes(key, w, kv, v)) out[pl++] = w;
                else out[ph++] = w;
            }
            sp = nlo;
        }
        g.split[v] = sp;
        if (use_lds) continue;
        g.st[v] = 1;
        g.conf[v] = sp;
        g.stamp[v] = 0;
        g.cflag[v] = 0;
        if (sp == 0) push(g, cnt, cl(1), v);
    }
    __syncthreads();
    if (use_lds) {
        int k = 1;
        color_one_lds<B>(a, g, gi, cnt, lds, k);
        if (tid == 0) {
            if (a.rounds) a.rounds[gi] = k - 1;
            if (a.ticks) a.ticks[2 * gi + 1] = wall_clock64();
        }
        __syncthreads();
        return;
    }
    const int grp = tid / kG, lig = tid & (kG - 1);
    int k = 1;
    for (;; ++k) {
        if (k > 1) {
            // round k: dirty list dl(k); clear round k-1's bits; reset lists
            const int nd = cnt[dl(k)];
            if (nd == 0) break;
            const int np = cnt[dl(k - 1)];
            for (int i = tid; i < np; i += B) g.bits(dl(k - 1))[g.L(dl(k - 1))[i] >> 5] = 0u;
            __syncthreads();
            if (tid == 0) {
                cnt[cl(k)] = 0;
                cnt[5] = 0;
            }
            __syncthreads();
            for (int i = grp; i < nd; i += kPerIt) phase_a(g, cnt, k, g.L(dl(k))[i], lig);
            __syncthreads();
            const int nb = cnt[5];
            for (int i = grp; i < nb; i += kPerIt) phase_b(g, cnt, k, g.L(5)[i], lig);
            __syncthreads();
        }
        // commits of round k fill dl(k+1)
        if (tid == 0) cnt[dl(k + 1)] = 0;
        __syncthreads();
        const int nc = cnt[cl(k)];
        for (int i = grp; i < nc; i += kPerIt) phase_c(g, cnt, k, g.L(cl(k))[i], lig);
        __syncthreads();
    }
    if (tid == 0) {
        if (a.rounds) a.rounds[gi] = k - 1;
        if (a.ticks) a.ticks[2 * gi + 1] = wall_clock64();
    }
    __syncthreads();
}

// B threads per workgroup: 1024 when the LDS path's capacity leaves one
// workgroup per CU anyway (more vertex groups in flight for the large rounds
// of big graphs), else 256 (several workgroups, graphs, per CU).
template <int B>
__global__ __launch_bounds__(B) void k_batch(BArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];  // 19 nl / 8 bytes for the LDS path
    __shared__ int cnt[8];
    __shared__ int shmax[B / 64];
    __shared__ int slot;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(&a.ctl->queue, 1);
        __syncthreads();
        const int q = slot;
        __syncthreads();
        if (q >= a.G) return;  // every wave of the workgroup leaves here once the queue is drained
        color_one<B>(a, a.order[q], cnt, lds, shmax);
    }
}

// Processing order: graphs by edge count, largest first (bitonic sort in
// LDS for up to kSortMax graphs; index order beyond).
__global__ __launch_bounds__(1024) void k_batch_order(int G, const int64_t* __restrict__ edge_off,
                                                      int* __restrict__ order, BCtl* ctl) {
    __shared__ long long keyv[kSortMax];
    if (threadIdx.x == 0) ctl->queue = 0;
    if (G > kSortMax) {
        for (int i = threadIdx.x; i < G; i += blockDim.x) order[i] = i;
        return;
    }
    int P = 1;
    while (P < G) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        // key: -(edges) in the high bits, index in the low bits (ties by index)
        keyv[i] = i < G ? ((-(long long)(edge_off[i + 1] - edge_off[i])) << 20) | i : LLONG_MAX;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const long long x = keyv[i], y = keyv[j];
                    if ((x > y) == up) {
                        keyv[i] = y;
                        keyv[j] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < G; i += blockDim.x) order[i] = (int)(keyv[i] & ((1 << 20) - 1));
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Process-wide batch tuning (gcolor_set_batch_tuning).
std::atomic<int> g_block_threads{0};
std::atomic<int> g_lds_factor{8};
std::atomic<int> g_lds_max{65536};

struct BLayout {
    size_t ctl, order, st, conf, stamp, cflag, split, lists, bits, colp, total;
    int64_t nbw;
};

BLayout blayout(int32_t G, int64_t V, int64_t nnz) {
    BLayout L;
    size_t off = 0;
    const size_t vb = sizeof(int32_t) * (size_t)(V > 0 ? V : 1);
    L.nbw = (V >> 5) + G + 1;
    L.ctl = off;   off += al(sizeof(BCtl));
    L.order = off; off += al(sizeof(int32_t) * (size_t)(G > 0 ? G : 1));
    L.st = off;    off += al(vb);
    L.conf = off;  off += al(vb);
    L.stamp = off; off += al(vb);
    L.cflag = off; off += al(vb);
    L.split = off; off += al(vb);
    L.lists = off; off += al(6 * vb);
    L.bits = off;  off += al(sizeof(uint32_t) * 3 * (size_t)L.nbw);
    L.colp = off;  off += al(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

size_t gcolor_batch_workspace_bytes(int32_t num_graphs, int64_t total_vertices, int64_t total_nnz) {
    if (num_graphs < 0 || total_vertices < 0 || total_nnz < 0) return 0;
    return blayout(num_graphs, total_vertices, total_nnz).total;
}

int color_graph_batch(int32_t num_graphs, int64_t total_vertices, int64_t total_nnz, const int64_t* vtx_off,
                      const int64_t* edge_off, const int32_t* row_ptr, const int32_t* col_idx,
                      const uint32_t* priority, int32_t* colors_out, void* workspace, size_t ws_bytes,
                      int64_t* ticks, int32_t* rounds, gcolor_stream_t stream) {
    if (num_graphs < 0 || total_vertices < 0 || total_nnz < 0) return GCOLOR_EINVAL;
    if (num_graphs == 0) return GCOLOR_OK;
    if (total_vertices >= (int64_t)1 << 40 || total_nnz >= (int64_t)1 << 40) return GCOLOR_ENOTSUP;
    if (!vtx_off || !edge_off || !row_ptr || !workspace || (total_vertices > 0 && !colors_out) ||
        (total_nnz > 0 && !col_idx))
        return GCOLOR_EINVAL;
    const BLayout L = blayout(num_graphs, total_vertices, total_nnz);
    if (ws_bytes < L.total) return GCOLOR_EWORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(workspace);
    BArgs a;
    a.G = num_graphs;
    a.V = total_vertices;
    a.vtx_off = vtx_off;
    a.edge_off = edge_off;
    a.row_ptr = row_ptr;
    a.col_idx = col_idx;
    a.key = priority;
    a.colors = colors_out;
    a.colp = reinterpret_cast<int*>(base + L.colp);
    a.st = reinterpret_cast<int*>(base + L.st);
    a.conf = reinterpret_cast<int*>(base + L.conf);
    a.stamp = reinterpret_cast<int*>(base + L.stamp);
    a.cflag = reinterpret_cast<int*>(base + L.cflag);
    a.split = reinterpret_cast<int*>(base + L.split);
    a.lists = reinterpret_cast<int*>(base + L.lists);
    a.bits = reinterpret_cast<unsigned*>(base + L.bits);
    a.nbw = L.nbw;
    a.order = reinterpret_cast<int*>(base + L.order);
    a.ctl = reinterpret_cast<BCtl*>(base + L.ctl);
    a.ticks = reinterpret_cast<long long*>(ticks);
    a.rounds = rounds;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GCOLOR_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    k_batch_order<<<1, 1024, 0, st>>>(num_graphs, edge_off, a.order, a.ctl);
    if (hipGetLastError() != hipSuccess) return GCOLOR_EHIP;
    // LDS path capacity: lds_factor (default 8) times the mean graph size, at
    // least 1024 and at most lds_max (default 65536) vertices (19/8 bytes per
    // vertex: 152 KiB at the top); the largest graphs of a batch of small ones
    // then take the global path rather than lowering every workgroup's
    // occupancy.
    const int lds_max = g_lds_max.load(), lds_factor = g_lds_factor.load();
    int64_t nl = 0;
    if (lds_max > 0) {
        nl = total_vertices > 0 ? (lds_factor * total_vertices + num_graphs - 1) / num_graphs : 0;
        nl = std::max<int64_t>(nl, 1024);
        nl = std::min<int64_t>(nl, lds_max);
        nl = (nl + 31) & ~(int64_t)31;
    }
    a.nl = (int)nl;
    const size_t lds_bytes = (size_t)19 * (size_t)nl / 8;
    const int grid = std::min(num_graphs, cus * 8);
    const int bt = g_block_threads.load();
    if (bt == 1024 || (bt == 0 && nl >= 16384)) {
        if (hipFuncSetAttribute((const void*)k_batch<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_bytes) != hipSuccess)
            return GCOLOR_EHIP;
        k_batch<1024><<<grid, 1024, lds_bytes, st>>>(a);
    } else {
        if (hipFuncSetAttribute((const void*)k_batch<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_bytes) != hipSuccess)
            return GCOLOR_EHIP;
        k_batch<256><<<grid, 256, lds_bytes, st>>>(a);
    }
    if (hipGetLastError() != hipSuccess) return GCOLOR_EHIP;
    return GCOLOR_OK;
}

int gcolor_set_batch_tuning(int32_t block_threads, int32_t lds_factor, int32_t lds_max_vertices) {
    if (block_threads != 0 && block_threads != 256 && block_threads != 1024) return GCOLOR_EINVAL;
    if (lds_factor < 1 || lds_factor > 64 || lds_max_vertices < 0 || lds_max_vertices > 65536) return GCOLOR_EINVAL;
    g_block_threads.store(block_threads);
    g_lds_factor.store(lds_factor);
    g_lds_max.store(lds_max_vertices);
    return GCOLOR_OK;
}

int gcolor_get_batch_tuning(int32_t* block_threads, int32_t* lds_factor, int32_t* lds_max_vertices) {
    if (block_threads) *block_threads = g_block_threads.load();
    if (lds_factor) *lds_factor = g_lds_factor.load();
    if (lds_max_vertices) *lds_max_vertices = g_lds_max.load();
    return GCOLOR_OK;
}

int gcolor_wall_clock_khz(int32_t* khz) {
    if (!khz) return GCOLOR_EINVAL;
    int dev = 0, rate = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GCOLOR_EHIP;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return GCOLOR_EHIP;
    *khz = rate;
    return GCOLOR_OK;
}

}  // extern "C"
