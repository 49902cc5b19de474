// Exact smallest-last order on the device.
//
// The order of Matula and Beck ("Smallest-last ordering and clustering and
// graph coloring algorithms", JACM 1983), which the paper's section "Number
// of colors" names among the orderings that bound the colours of the greedy
// scheme: repeatedly remove a vertex of least remaining degree (ties to the
// smallest id); colour in the reverse of the removal order.  rank[v] is v's
// position in the colouring order (n - 1 - its removal step), the same
// contract as gcolor_smallest_last_host.
//
// The removal sequence is inherently sequential, so one workgroup walks it,
// many removals per step.  A step takes the m smallest ids of the least
// degree delta (the candidates c_0 < c_1 < ...) and finds the longest prefix
// that the one-at-a-time process would remove in that same order: c_{q+1}
// follows c_q unless removing c_0..c_q
//   * drops a remaining vertex below delta (it would go next), other than
//     c_{q+1} itself, or
//   * brings a vertex y down to delta with y < c_{q+1} (it would go first by
//     id); if y > c_{q+1} it goes before the first later candidate above y.
// A vertex y with degree d_y and h_y of its neighbours among the candidates
// reaches delta at its (d_y - delta)-th candidate neighbour and drops below
// at the next one, so the test needs, per y, the order statistics of its
// candidate neighbours' positions: pairs (candidate, remaining neighbour) are
// staged in LDS, hashed by neighbour, and each pair finds its rank in its
// neighbour's list.  The prefix is removed, the neighbours' degrees are
// decremented, and the next step starts.  The first candidate is always the
// true next removal, so every step removes at least one vertex.
//
// Degree buckets: for each degree d up to a bound of the degeneracy, a
// three-level bitmap over vertex ids (level 0: one bit per vertex, exact;
// levels 1 and 2: one bit per word of the level below, set whenever the word
// below is non-zero, cleared lazily when a scan finds the word empty).  The
// smallest ids of a bucket come from one read of the top level, one of up to
// 16 level-1 words and one of up to 1024 level-0 words.  Per-degree counts
// give the least non-empty degree, which moves down by at most one per step.
// The bound: a k-core has at least k + 1 vertices of degree >= k, so the
// degeneracy is at most the largest k with that many; with int32 row offsets
// it is below 46341 (a k-core holds at least k (k + 1) entries).
//
// The workgroup keeps shared arrays coherent through device-scope atomics and
// device-scope loads (the vector L1 does not see atomics performed in L2).

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <vector>

#include "gcolor.h"

namespace {

typedef unsigned long long u64;

constexpr int kT = 1024;        // threads of the peel workgroup
constexpr int kChunk = 1024;    // candidates per step, at most
constexpr int kPairs = 2048;    // staged (candidate, neighbour) pairs
constexpr int kHashBits = 12;
constexpr int kHash = 1 << kHashBits;  // >= 2 kPairs slots
constexpr int kDegCap = 46341;  // histogram cap: every degeneracy is below it
constexpr int kMaxN = 1 << 28;  // the top bitmap level fits one read by kT threads
constexpr int kLdsHist = 2048;  // per-workgroup counts in the bucket set-up
constexpr int kCntLds = 4096;   // bucket counts kept in LDS when the bound is below this
constexpr int kScanBudget = 32768;  // row entries scanned per step (the first candidate's row in full)

struct PeelCtl {
    int err;         // 0 ok; 1 no non-empty bucket left; 2 step cap; 3 bucket bits inconsistent
    int degeneracy;  // largest least degree of a step
    int steps;
    int pad;
};

__device__ __forceinline__ int ald(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ u64 ald64(u64* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ast(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Buckets {
    u64* bm;           // (dcap + 1) x stride words
    int* cnt;          // vertices of each degree 0..dcap
    int dcap;
    long long w0, w1, w2;  // words per level
    __device__ u64* l0(int d) const { return bm + (long long)d * (w0 + w1 + w2); }
    // add v to bucket d, setting the parent bits unconditionally (no
    // dependent round trips; a parent bit over an empty word is harmless)
    __device__ void set_all(int d, int v) const {
        u64* a = l0(d);
        const long long w = v >> 6;
        atomicOr(&a[w], 1ull << (v & 63));
        atomicOr(&a[w0 + (w >> 6)], 1ull << (w & 63));
        atomicOr(&a[w0 + w1 + (w >> 12)], 1ull << ((w >> 6) & 63));
    }
    // add v to bucket d (parents first seen empty get their bit)
    __device__ void set(int d, int v) const {
        u64* a = l0(d);
        const long long w = v >> 6;
        if (atomicOr(&a[w], 1ull << (v & 63)) == 0ull)
            if (atomicOr(&a[w0 + (w >> 6)], 1ull << (w & 63)) == 0ull)
                atomicOr(&a[w0 + w1 + (w >> 12)], 1ull << ((w >> 6) & 63));
    }
    __device__ void clear(int d, int v) const { atomicAnd(&l0(d)[v >> 6], ~(1ull << (v & 63))); }
};

// Exclusive prefix sum over the kT threads; total gets the sum.  Two barriers.
__device__ int wg_scan(int x, int* ws, int& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kT / 64; ++i) {
        const int s = ws[i];
        base += i < w ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return base + inc - x;
}

// Degrees without self-loops, ranks unset, and the histogram of degrees
// (capped at kDegCap) that bounds the degeneracy; *bad is set when a row's
// offsets decrease, an entry lies outside [0, n), or col is NULL under a
// non-empty row.  Rows longer than kLongRow are listed for k_peel_long
// (a workgroup each) instead of one thread walking them.
constexpr int kLongRow = 64;

__device__ __forceinline__ void hist_add(int* h, int* hist, int d) {
    if (d < kLdsHist) atomicAdd(&h[d], 1);
    else atomicAdd(&hist[min(d, kDegCap)], 1);
}

__global__ __launch_bounds__(256) void k_peel_init(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                   int* __restrict__ deg, int* __restrict__ rank,
                                                   int* __restrict__ hist, int* __restrict__ bad,
                                                   int* __restrict__ longs, int* __restrict__ nlong) {
    __shared__ int h[kLdsHist];
    for (int i = threadIdx.x; i < kLdsHist; i += 256) h[i] = 0;
    __syncthreads();
    for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const int s = row_ptr[v], e = row_ptr[v + 1];
        rank[v] = -1;
        if (e < s || (v == 0 && s != 0) || (e > s && col == nullptr)) {
            atomicOr(bad, 1);
            deg[v] = 0;
            continue;
        }
        if (e - s > kLongRow) {
            longs[atomicAdd(nlong, 1)] = v;
            continue;
        }
        int d = 0;
        for (int p = s; p < e; ++p) {
            const int w = col[p];
            if (w < 0 || w >= n) atomicOr(bad, 1);
            d += w != v;
        }
        deg[v] = d;
        hist_add(h, hist, d);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLdsHist; i += 256)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ __launch_bounds__(256) void k_peel_long(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                   int* __restrict__ deg, int* __restrict__ hist,
                                                   int* __restrict__ bad, const int* __restrict__ longs,
                                                   const int* __restrict__ nlong) {
    __shared__ int part[4];
    const int total = *nlong;
    for (int i = blockIdx.x; i < total; i += gridDim.x) {
        const int v = longs[i];
        const int s = row_ptr[v], e = row_ptr[v + 1];
        int loops = 0;
        for (int p = s + (int)threadIdx.x; p < e; p += 256) {
            const int w = col[p];
            if (w < 0 || w >= n) atomicOr(bad, 1);
            loops += w == v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) loops += __shfl_xor(loops, o);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = loops;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int d = (e - s) - (part[0] + part[1] + part[2] + part[3]);
            deg[v] = d;
            atomicAdd(&hist[min(d, kDegCap)], 1);
        }
        __syncthreads();  // part is reused by the next row
    }
}

// Every vertex into the bucket of its degree (degrees above the bound stay
// out until they come down to it).
__global__ __launch_bounds__(256) void k_peel_buckets(int n, const int* __restrict__ deg, Buckets b) {
    __shared__ int h[kLdsHist];
    for (int i = threadIdx.x; i < kLdsHist; i += 256) h[i] = 0;
    __syncthreads();
    for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const int d = deg[v];
        if (d > b.dcap) continue;
        b.set(d, v);
        if (d < kLdsHist) atomicAdd(&h[d], 1);
        else atomicAdd(&b.cnt[d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLdsHist && i <= b.dcap; i += 256)
        if (h[i]) atomicAdd(&b.cnt[i], h[i]);
}

struct PeelLds {
    int cand[kChunk];      // candidate ids, ascending
    int rstart[kChunk];    // their row starts
    int roff[kChunk + 1];  // exclusive prefix of their row lengths
    int py[kPairs];        // remaining neighbour of the pair
    int pd[kPairs];        // its degree at the start of the step
    short pq[kPairs];      // the pair's candidate position
    short pp[kPairs];      // the neighbour's own candidate position, -1 if none
    short pnext[kPairs];   // next pair with the same neighbour
    short pslot[kPairs];   // hash slot of the neighbour (-1: pair not used)
    int hkey[kHash];
    int hhead[kHash];
    int hcount[kHash];
    int hmin[kHash];
    int htk[kHash];        // hits by the removed candidates
    int cnt[kCntLds];      // bucket counts (when the bound is below kCntLds)
    int nxt[kChunk];       // the next step's candidates, when known without a scan
    int lj[kChunk];        // neighbours left at delta - 1 (from the front) or delta (from the back)
    int l1idx[16];
    u64 l1w[16];
    int ws[kT / 64];
    int found, np, cut, istar;
    int removed, delta, chunk, degen, err;
    int nlow, njoin, njp, nnext, ndelta;
};

// A neighbour whose new degree is delta - 1 or delta may be a candidate of
// the next step: listed from the front and the back of lj (an overflow is
// seen from the two counts).
__device__ __forceinline__ void note_level(PeelLds& L, int y, int d1, int delta) {
    if (d1 == delta - 1) {
        const int k = atomicAdd(&L.nlow, 1);
        if (k < kChunk) L.lj[k] = y;
    } else if (d1 == delta) {
        const int k = atomicAdd(&L.njoin, 1);
        if (k < kChunk) L.lj[kChunk - 1 - k] = y;
    }
}

__global__ __launch_bounds__(kT) void k_peel(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                             int* deg, int* rank, Buckets b, PeelCtl* ctl) {
    __shared__ PeelLds L;
    const int tid = threadIdx.x;
    // bucket counts: LDS when they fit (only this workgroup changes them)
    const bool lds_cnt = b.dcap < kCntLds;
    if (lds_cnt)
        for (int d = tid; d <= b.dcap; d += kT) L.cnt[d] = b.cnt[d];
    auto cnt_get = [&](int d) { return lds_cnt ? L.cnt[d] : ald(&b.cnt[d]); };
    auto cnt_add = [&](int d, int x) {
        if (lds_cnt) atomicAdd(&L.cnt[d], x);
        else atomicAdd(&b.cnt[d], x);
    };
    if (tid == 0) {
        L.nnext = 0;
        L.removed = 0;
        L.delta = 0;
        L.chunk = 64;
        L.degen = 0;
        L.err = 0;
    }
    __syncthreads();
    long long step = 0;
    for (;;) {
        const int removed = L.removed;
        if (removed >= n) break;
        if (++step > (long long)n + 1) {
            if (tid == 0) L.err = 2;
            break;
        }
        const int K = L.chunk;
        const int carried = L.nnext;
        int delta, m;
        if (carried > 0) {
            // candidates carried over from the previous step
            delta = L.ndelta;
            m = min(carried, K);
            if (tid < m) L.cand[tid] = L.nxt[tid];
        } else {
            // least non-empty degree, from one below the last one up
            if (tid == 0) L.found = INT_MAX;
            __syncthreads();
            for (int base = max(L.delta - 1, 0); base <= b.dcap; base += kT) {
                const int d = base + tid;
                if (d <= b.dcap && cnt_get(d) > 0) atomicMin(&L.found, d);
                __syncthreads();
                const int f = L.found;
                __syncthreads();
                if (f != INT_MAX) break;
            }
            delta = L.found;
            if (delta == INT_MAX) {
                if (tid == 0) L.err = 1;
                break;
            }
            u64* B0 = b.l0(delta);
            u64* B1 = B0 + b.w0;
            u64* B2 = B1 + b.w1;

            // the K smallest ids of degree delta (a pass that meets only stale
            // upper-level bits clears them and looks again)
            m = 0;
            bool bad = false;
            for (long long pass = 0;; ++pass) {
                const u64 w2 = tid < b.w2 ? ald64(&B2[tid]) : 0ull;
                int tot2;
                const int o2 = wg_scan(__popcll(w2), L.ws, tot2);
                u64 x = w2;
                for (int k = o2; x && k < 16; ++k) {
                    L.l1idx[k] = tid * 64 + __builtin_ctzll(x);
                    x &= x - 1;
                }
                __syncthreads();
                const int nl1 = min(tot2, 16);
                if (nl1 == 0 || pass > b.w1 + b.w2 + 2) {
                    bad = true;
                    break;
                }
                if (tid < nl1) {
                    const int i1 = L.l1idx[tid];
                    const u64 w1 = ald64(&B1[i1]);
                    L.l1w[tid] = w1;
                    if (w1 == 0ull) atomicAnd(&B2[i1 >> 6], ~(1ull << (i1 & 63)));
                }
                __syncthreads();
                // thread t: level-1 word t / 64, bit t % 64 (ascending word order)
                const int j = tid >> 6, bit = tid & 63;
                u64 w0 = 0;
                long long i0 = 0;
                if (j < nl1 && (L.l1w[j] >> bit & 1ull)) {
                    i0 = (long long)L.l1idx[j] * 64 + bit;
                    w0 = ald64(&B0[i0]);
                    if (w0 == 0ull) atomicAnd(&B1[L.l1idx[j]], ~(1ull << bit));
                }
                int tot0;
                const int o0 = wg_scan(__popcll(w0), L.ws, tot0);
                x = w0;
                for (int k = o0; x && k < K; ++k) {
                    L.cand[k] = (int)(i0 * 64 + __builtin_ctzll(x));
                    x &= x - 1;
                }
                __syncthreads();
                m = min(tot0, K);
                if (m > 0) break;
            }
            if (bad) {
                if (tid == 0) L.err = 3;
                break;
            }
        }
        // rows of the candidates
        int rlen = 0;
        if (tid < m) {
            const int v = L.cand[tid];
            const int s = row_ptr[v];
            L.rstart[tid] = s;
            rlen = row_ptr[v + 1] - s;
        }
        int T;
        const int ro = wg_scan(rlen, L.ws, T);
        if (tid < m) L.roff[tid] = ro;
        if (tid == 0) {
            L.roff[m] = T;
            L.np = 0;
            L.cut = m;
            L.istar = INT_MAX;
            L.nlow = 0;
            L.njoin = 0;
            L.njp = 0;
        }
        __syncthreads();
        // candidates whose rows end past the scan budget wait for a later step
        if (tid > 0 && tid < m && ro + rlen > kScanBudget) atomicMin(&L.cut, tid);
        __syncthreads();
        const int Tscan = L.roff[L.cut];

        // pairs (candidate q, remaining neighbour y), y not a candidate at or
        // before q; an overflow cuts the candidates at the first position
        // that lost a pair
        for (int i = tid; i < Tscan; i += kT) {
            int a = 0, hi = m - 1;
            while (a < hi) {
                const int mid = (a + hi + 1) >> 1;
                if (L.roff[mid] <= i) a = mid;
                else hi = mid - 1;
            }
            const int q = a;
            if (q >= L.cut) continue;
            const int v = L.cand[q];
            const int y = col[L.rstart[q] + (i - L.roff[q])];
            if (y == v) continue;
            const int dy = ald(&deg[y]);
            if (dy < 0) continue;  // removed
            int lo2 = 0, hi2 = m;
            while (lo2 < hi2) {
                const int mid = (lo2 + hi2) >> 1;
                if (L.cand[mid] < y) lo2 = mid + 1;
                else hi2 = mid;
            }
            const int pos = (lo2 < m && L.cand[lo2] == y) ? lo2 : -1;
            if (pos >= 0 && pos <= q) continue;
            const int slot = atomicAdd(&L.np, 1);
            if (slot < kPairs) {
                L.py[slot] = y;
                L.pd[slot] = dy;
                L.pq[slot] = (short)q;
                L.pp[slot] = (short)pos;
            } else {
                atomicMin(&L.cut, q);
            }
        }
        for (int s = tid; s < kHash; s += kT) {
            L.hkey[s] = -1;
            L.hhead[s] = -1;
            L.hcount[s] = 0;
            L.hmin[s] = INT_MAX;
            L.htk[s] = 0;
        }
        __syncthreads();
        const int meff = min(m, L.cut);
        const int np = min(L.np, kPairs);

        // group the pairs by neighbour
        for (int i = tid; i < np; i += kT) {
            if (L.pq[i] >= meff) {
                L.pslot[i] = -1;
                continue;
            }
            const int y = L.py[i];
            unsigned h = ((unsigned)y * 2654435761u) >> (32 - kHashBits);
            for (;;) {
                const int prev = atomicCAS(&L.hkey[h], -1, y);
                if (prev == -1 || prev == y) break;
                h = (h + 1) & (kHash - 1);
            }
            L.pslot[i] = (int)h;
            atomicAdd(&L.hcount[h], 1);
            atomicMin(&L.hmin[h], (int)L.pq[i]);
            L.pnext[i] = atomicExch(&L.hhead[h], i);
        }
        __syncthreads();

        // the first candidate position that the one-at-a-time process would
        // not take next (1-based: istar - 1 candidates are taken)
        for (int i = tid; i < np; i += kT) {
            const int h = L.pslot[i];
            if (h < 0) continue;
            const int q = L.pq[i], y = L.py[i], pos = L.pp[i];
            int viol = INT_MAX;
            if (pos >= 0) {
                // a later candidate drops below delta at its first hit: it
                // goes next, which is fine only if it is next anyway
                if (L.hmin[h] == q && q + 1 != pos) viol = q + 2;
            } else {
                const int t0 = L.pd[i] - delta;  // hits that bring y to delta
                if (t0 <= 0) {
                    if (L.hmin[h] == q) viol = q + 2;
                } else if (L.hcount[h] >= t0) {
                    int r = 0;  // hits of y before this one
                    for (int k = L.hhead[h]; k >= 0; k = L.pnext[k]) r += L.pq[k] < q;
                    if (r + 1 == t0) {
                        // y now ties delta: it precedes the first later
                        // candidate with a larger id
                        int a = q + 1, hi = meff;
                        while (a < hi) {
                            const int mid = (a + hi) >> 1;
                            if (L.cand[mid] > y) hi = mid;
                            else a = mid + 1;
                        }
                        if (a < meff) viol = a + 1;
                    } else if (r == t0) {
                        viol = q + 2;  // y drops below delta
                    }
                }
            }
            if (viol != INT_MAX) atomicMin(&L.istar, viol);
        }
        __syncthreads();
        const int take = meff == 0 ? 1 : max(1, min(meff, L.istar == INT_MAX ? meff : L.istar - 1));

        // remove the prefix; count each remaining neighbour's hits by it
        if (tid < take) {
            const int v = L.cand[tid];
            ast(&rank[v], n - 1 - (removed + tid));
            ast(&deg[v], -1);
            b.clear(delta, v);
        }
        if (tid == 0) {
            cnt_add(delta, -take);
            L.degen = max(L.degen, delta);
        }
        if (meff > 0)
            for (int i = tid; i < np; i += kT) {
                const int h = L.pslot[i], pos = L.pp[i];
                if (h >= 0 && L.pq[i] < take && !(pos >= 0 && pos < take)) atomicAdd(&L.htk[h], 1);
            }
        __syncthreads();
        // each remaining neighbour once (at its pair with the first candidate
        // position): its new degree and buckets; or, for a first candidate
        // with more remaining neighbours than the stage holds, its row (one
        // hit each)
        if (meff > 0) {
            for (int i = tid; i < np; i += kT) {
                const int h = L.pslot[i], q = L.pq[i], pos = L.pp[i];
                if (h < 0 || q != L.hmin[h] || q >= take || (pos >= 0 && pos < take)) continue;
                const int y = L.py[i], d0 = L.pd[i], d1 = d0 - L.htk[h];
                ast(&deg[y], d1);
                note_level(L, y, d1, delta);
                if (d0 <= b.dcap) {
                    b.clear(d0, y);
                    cnt_add(d0, -1);
                }
                if (d1 >= 0 && d1 <= b.dcap) {
                    b.set_all(d1, y);
                    cnt_add(d1, 1);
                }
            }
        } else {
            const int v = L.cand[0];
            const int s0 = L.rstart[0], e0 = L.rstart[0] + (L.roff[1] - L.roff[0]);
            for (int p = s0 + tid; p < e0; p += kT) {
                const int y = col[p];
                if (y == v) continue;
                const int d0 = ald(&deg[y]);
                if (d0 < 0) continue;
                const int d1 = d0 - 1;
                ast(&deg[y], d1);
                note_level(L, y, d1, delta);
                if (d0 <= b.dcap) {
                    b.clear(d0, y);
                    cnt_add(d0, -1);
                }
                if (d1 >= 0 && d1 <= b.dcap) {
                    b.set_all(d1, y);
                    cnt_add(d1, 1);
                }
            }
        }
        __syncthreads();
        // the next step's candidates when they are known here: every vertex
        // left at delta - 1 (none was below delta, so these are all of that
        // degree); otherwise, with no candidate hit, the candidates not taken
        // and the vertices that came down to delta, either all of degree
        // delta or those below the last candidate (so still a prefix of the
        // bucket in id order).  Else the next step scans the buckets.
        {
            const int nlow = L.nlow, njoin = L.njoin;
            const bool ovf = nlow + njoin > kChunk;
            const int cd = cnt_get(delta);
            if (!ovf && nlow > 0) {
                for (int i = tid; i < nlow; i += kT) {
                    const int y = L.lj[i];
                    int r = 0;
                    for (int j = 0; j < nlow; ++j) r += L.lj[j] < y;
                    L.nxt[r] = y;
                }
                if (tid == 0) {
                    L.nnext = nlow;
                    L.ndelta = delta - 1;
                }
            } else if (!ovf && cd > 0) {
                const int rc = m - take;
                const int* J = &L.lj[kChunk - njoin];
                const int limit = rc + njoin == cd ? INT_MAX : L.cand[m - 1];
                for (int i = tid; i < rc; i += kT) {
                    const int r = L.cand[take + i];
                    int c = 0;
                    for (int j = 0; j < njoin; ++j) c += J[j] < limit && J[j] < r;
                    if (i + c < kChunk) L.nxt[i + c] = r;
                }
                for (int i = tid; i < njoin; i += kT) {
                    const int y = J[i];
                    if (y >= limit) continue;
                    int a = take, hi = m;
                    while (a < hi) {
                        const int mid = (a + hi) >> 1;
                        if (L.cand[mid] < y) a = mid + 1;
                        else hi = mid;
                    }
                    int c = a - take;
                    for (int j = 0; j < njoin; ++j) c += J[j] < limit && J[j] < y;
                    if (c < kChunk) L.nxt[c] = y;
                    atomicAdd(&L.njp, 1);
                }
                __syncthreads();
                if (tid == 0) {
                    L.nnext = min(rc + L.njp, kChunk);
                    L.ndelta = delta;
                }
            } else if (tid == 0) {
                L.nnext = 0;
            }
        }
        if (tid == 0) {
            L.removed = removed + take;
            L.delta = delta;
            L.chunk = min(kChunk, max(16, 2 * take));
        }
        __syncthreads();
    }
    if (tid == 0) {
        ctl->err = L.err;
        ctl->degeneracy = L.degen;
        ctl->steps = (int)min(step, (long long)INT_MAX);
    }
}

int grid_for(long long n) {
    long long g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

extern "C" {

int gcolor_smallest_last(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* rank,
                         int32_t* degeneracy, gcolor_stream_t stream) {
    if (n < 0) return GCOLOR_EINVAL;
    if (n == 0) {
        if (degeneracy) *degeneracy = 0;
        return GCOLOR_OK;
    }
    if (!row_ptr || !rank) return GCOLOR_EINVAL;  // col_idx may be NULL when no row has entries
    if (n > kMaxN) return GCOLOR_ENOTSUP;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int* deg = nullptr;
    int* hist = nullptr;
    int* longs = nullptr;
    PeelCtl* ctl = nullptr;
    u64* bm = nullptr;
    int* cnt = nullptr;
    int rc = GCOLOR_OK;
    std::vector<int> h(kDegCap + 2);
    PeelCtl hc{};
    Buckets b{};
    long long words = 0;
    int dcap = 0;
    // hist[0..kDegCap]: degree counts; hist[kDegCap + 1]: the malformed-CSR
    // flag; hist[kDegCap + 2]: the number of long rows listed in longs
    if (hipMalloc(&deg, sizeof(int) * (size_t)n) != hipSuccess || hipMalloc(&hist, sizeof(int) * (kDegCap + 3)) != hipSuccess ||
        hipMalloc(&longs, sizeof(int) * (size_t)n) != hipSuccess ||
        hipMalloc(&ctl, sizeof(PeelCtl)) != hipSuccess) {
        rc = GCOLOR_EHIP;
        goto done;
    }
    if (hipMemsetAsync(hist, 0, sizeof(int) * (kDegCap + 3), st) != hipSuccess) {
        rc = GCOLOR_EHIP;
        goto done;
    }
    k_peel_init<<<grid_for(n), 256, 0, st>>>(n, row_ptr, col_idx, deg, rank, hist, hist + kDegCap + 1, longs,
                                             hist + kDegCap + 2);
    k_peel_long<<<grid_for((long long)n * 4), 256, 0, st>>>(n, row_ptr, col_idx, deg, hist, hist + kDegCap + 1, longs,
                                                            hist + kDegCap + 2);
    if (hipMemcpyAsync(h.data(), hist, sizeof(int) * (kDegCap + 2), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        rc = GCOLOR_EHIP;
        goto done;
    }
    if (h[kDegCap + 1]) {
        rc = GCOLOR_ECSR;
        goto done;
    }
    {
        // largest k with at least k + 1 vertices of degree >= k
        long long ge = 0;
        for (int k = kDegCap; k >= 0; --k) {
            ge += h[k];
            if (ge >= (long long)k + 1) {
                dcap = k;
                break;
            }
        }
    }
    b.dcap = dcap;
    b.w0 = ((long long)n + 63) / 64;
    b.w1 = (b.w0 + 63) / 64;
    b.w2 = (b.w1 + 63) / 64;
    words = (long long)(dcap + 1) * (b.w0 + b.w1 + b.w2);
    if (hipMalloc(&bm, sizeof(u64) * (size_t)words) != hipSuccess ||
        hipMalloc(&cnt, sizeof(int) * (size_t)(dcap + 1)) != hipSuccess) {
        rc = GCOLOR_EHIP;
        goto done;
    }
    b.bm = bm;
    b.cnt = cnt;
    if (hipMemsetAsync(bm, 0, sizeof(u64) * (size_t)words, st) != hipSuccess ||
        hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)(dcap + 1), st) != hipSuccess ||
        hipMemsetAsync(ctl, 0, sizeof(PeelCtl), st) != hipSuccess) {
        rc = GCOLOR_EHIP;
        goto done;
    }
    k_peel_buckets<<<grid_for(n), 256, 0, st>>>(n, deg, b);
    k_peel<<<1, kT, 0, st>>>(n, row_ptr, col_idx, deg, rank, b, ctl);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&hc, ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        rc = GCOLOR_EHIP;
        goto done;
    }
    if (hc.err) rc = GCOLOR_EINTERNAL;
    else if (degeneracy) *degeneracy = hc.degeneracy;
done:
    if (bm) (void)hipFree(bm);
    if (cnt) (void)hipFree(cnt);
    if (deg) (void)hipFree(deg);
    if (longs) (void)hipFree(longs);
    if (hist) (void)hipFree(hist);
    if (ctl) (void)hipFree(ctl);
    return rc;
}

}  // extern "C"
