/*
 * CPU oracle for distance-1 graph colouring (test infrastructure only).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * call this file.  It shares no code with the GPU library.  Every function
 * is written for obviousness, not speed: the two phases of a round are the
 * paper's two parallel loops over the worklist, nothing is fused or reordered.
 *
 * Paper: Catalyurek, Feo, Gebremedhin, Halappanavar, Pothen, "Graph colouring
 * algorithms for multi-core and massively multithreaded architectures".
 *
 * Conventions (the readings the whole project uses):
 *  - colours are positive integers, 0 means "not coloured" (section "The
 *    problem" and the description of the greedy algorithm);
 *  - precedence: vertex w beats v when (key[w], w) < (key[v], v); with no key
 *    array the key is the index, so the smaller index wins (conflict rule of
 *    Algorithm 2);
 *  - w == v entries (self-loops) are ignored in both phases.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static inline int or_before(const uint32_t* key, int32_t w, int32_t v) {
    const uint32_t kw = key ? key[w] : (uint32_t)w;
    const uint32_t kv = key ? key[v] : (uint32_t)v;
    return kw < kv || (kw == kv && w < v);
}

static int32_t or_max_degree(int32_t n, const int32_t* row_ptr) {
    int32_t d = 0;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] > d) d = row_ptr[v + 1] - row_ptr[v];
    return d;
}

/* Visit order of the serial greedy: ascending (key, id). */
static const uint32_t* or_sort_key;
static int or_cmp_vertex(const void* a, const void* b) {
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    if (or_before(or_sort_key, x, y)) return -1;
    if (or_before(or_sort_key, y, x)) return 1;
    return 0;
}

/*
 * Serial greedy first-fit (Algorithm 1).  For each vertex in ascending
 * (key, id) order: stamp the colours of its neighbours as forbidden with a
 * per-visit label, then take the smallest positive colour not stamped.
 * The forbidden array is indexed by colour and sized max degree + 2, the
 * bound the paper gives for the colour count.
 * Returns the number of colours used (the largest colour).
 */
int32_t or_greedy(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                  const uint32_t* key, int32_t* color) {
    const int32_t dmax = or_max_degree(n, row_ptr);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* forbidden = (int64_t*)malloc(sizeof(int64_t) * (size_t)(dmax + 2));
    for (int32_t v = 0; v < n; ++v) order[v] = v;
    if (key) {
        or_sort_key = key;
        qsort(order, (size_t)n, sizeof(int32_t), or_cmp_vertex);
    }
    for (int32_t c = 0; c < dmax + 2; ++c) forbidden[c] = -1;
    for (int32_t v = 0; v < n; ++v) color[v] = 0;
    int32_t ncol = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t v = order[i];
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col_idx[e];
            if (w == v) continue;
            forbidden[color[w]] = v; /* colour 0 (uncoloured) is never chosen */
        }
        int32_t c = 1;
        while (forbidden[c] == v) ++c;
        color[v] = c;
        if (c > ncol) ncol = c;
    }
    free(order);
    free(forbidden);
    return ncol;
}

/*
 * Round-synchronous simulation of the iterative speculative colouring
 * (Algorithm 2), with the two readings that make it a function of the input:
 *  (a) phase 1 reads the colours as they stood at the end of the previous
 *      round (an explicit snapshot);
 *  (b) the losers of phase 2 have their tentative colour revoked (set to 0)
 *      before the next round.
 *
 * Round k:
 *   S = copy(color)                      (every worklist vertex has S = 0)
 *   phase 1, for v in U: tent[v] = min{c >= 1 : c not in {S[w] : w in adj(v)}}
 *   for v in U: color[v] = tent[v]
 *   phase 2, for v in U: v loses if some neighbour w has color[w] == color[v]
 *            and (key[w], w) < (key[v], v)
 *   losers: color[v] = 0, they form the next worklist (ascending id order).
 *
 * fixed_round[v] receives the round in which v kept its colour (may be NULL).
 * log (may be NULL) receives 4 int64 per round: k, |U_k|, sum of degrees over
 * U_k, |R_k|; at most max_log rounds are logged.
 * Returns the number of rounds, or -5 when max_rounds is exceeded.
 * nthreads <= 0 means OpenMP's default; the result never depends on it.
 */
int32_t or_spec_sim(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                    const uint32_t* key, int32_t* color, int32_t* fixed_round,
                    int64_t* log, int32_t max_log, int32_t max_rounds, int32_t nthreads) {
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    const int32_t dmax = or_max_degree(n, row_ptr);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* tent = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* U = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* R = (int32_t*)malloc(sizeof(int32_t) * nn);
    unsigned char* lose = (unsigned char*)malloc(nn);
    int64_t nU = n;
    for (int32_t v = 0; v < n; ++v) {
        color[v] = 0;
        U[v] = v;
        if (fixed_round) fixed_round[v] = 0;
    }
    int32_t k = 0;
    while (nU > 0) {
        if (k >= max_rounds) { k = -5; break; }
        ++k;
        memcpy(S, color, sizeof(int32_t) * (size_t)n);

        /* Phase 1: tentative colouring against the snapshot.  Each thread
         * owns a forbidden array stamped with a label unique to the visit. */
#pragma omp parallel num_threads(nthreads)
        {
            int64_t* forbidden = (int64_t*)malloc(sizeof(int64_t) * (size_t)(dmax + 2));
            for (int32_t c = 0; c < dmax + 2; ++c) forbidden[c] = -1;
#pragma omp for schedule(dynamic, 1024)
            for (int64_t i = 0; i < nU; ++i) {
                const int32_t v = U[i];
                const int64_t label = i;
                for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                    const int32_t w = col_idx[e];
                    if (w == v) continue;
                    forbidden[S[w]] = label;
                }
                int32_t c = 1;
                while (forbidden[c] == label) ++c;
                tent[v] = c;
            }
            free(forbidden);
        }
        for (int64_t i = 0; i < nU; ++i) color[U[i]] = tent[U[i]];

        /* Phase 2: conflict detection; the later vertex in (key, id) order
         * of a conflicting pair is re-queued. */
        int64_t edge_work = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1024) reduction(+ : edge_work)
        for (int64_t i = 0; i < nU; ++i) {
            const int32_t v = U[i];
            unsigned char l = 0;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t w = col_idx[e];
                if (w == v) continue;
                if (color[w] == color[v] && or_before(key, w, v)) l = 1;
            }
            lose[v] = l;
            edge_work += row_ptr[v + 1] - row_ptr[v];
        }
        int64_t nR = 0;
        for (int64_t i = 0; i < nU; ++i) {
            const int32_t v = U[i];
            if (lose[v]) R[nR++] = v;
            else if (fixed_round) fixed_round[v] = k;
        }
        for (int64_t i = 0; i < nR; ++i) color[R[i]] = 0;
        if (log && k <= max_log) {
            log[4 * (k - 1) + 0] = k;
            log[4 * (k - 1) + 1] = nU;
            log[4 * (k - 1) + 2] = edge_work;
            log[4 * (k - 1) + 3] = nR;
        }
        int32_t* t = U; U = R; R = t;
        nU = nR;
    }
    free(S);
    free(tent);
    free(U);
    free(R);
    free(lose);
    return k;
}

/*
 * Iterative colouring with a sequential finish (the closing remark of section
 * "Iterative and degree of concurrency": once conflicts are few, switch to a
 * sequential computation).  Rounds of Algorithm 2 exactly as in or_spec_sim
 * run while more than `tail` vertices are uncoloured; the vertices left are
 * then coloured one at a time in ascending (key, id) order, each with the
 * smallest positive colour held by none of its neighbours (those committed
 * by the rounds and those coloured earlier in the finish).  tail = 0 is
 * or_spec_sim; tail >= n is the serial greedy or_greedy.
 * *tail_count receives the number of vertices the finish coloured.
 * Returns the number of rounds run (the finish is not a round), or -5 when
 * max_rounds is exceeded.
 */
int32_t or_spec_tail(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* key,
                     int64_t tail, int32_t* color, int64_t* tail_count, int32_t max_rounds) {
    const int32_t dmax = or_max_degree(n, row_ptr);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* tent = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* U = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* R = (int32_t*)malloc(sizeof(int32_t) * nn);
    int64_t* forbidden = (int64_t*)malloc(sizeof(int64_t) * (size_t)(dmax + 2));
    int64_t nU = n;
    int64_t label = 0;
    for (int32_t c = 0; c < dmax + 2; ++c) forbidden[c] = -1;
    for (int32_t v = 0; v < n; ++v) {
        color[v] = 0;
        U[v] = v;
    }
    int32_t k = 0;
    while (nU > tail) {
        if (k >= max_rounds) { k = -5; break; }
        ++k;
        memcpy(S, color, sizeof(int32_t) * (size_t)n);
        /* phase 1 against the snapshot (one stamp label per visit) */
        for (int64_t i = 0; i < nU; ++i) {
            const int32_t v = U[i];
            ++label;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t w = col_idx[e];
                if (w != v) forbidden[S[w]] = label;
            }
            int32_t c = 1;
            while (forbidden[c] == label) ++c;
            tent[v] = c;
        }
        for (int64_t i = 0; i < nU; ++i) color[U[i]] = tent[U[i]];
        /* phase 2: the later vertex of a conflicting pair is re-queued */
        int64_t nR = 0;
        for (int64_t i = 0; i < nU; ++i) {
            const int32_t v = U[i];
            int lose = 0;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t w = col_idx[e];
                if (w != v && color[w] == color[v] && or_before(key, w, v)) lose = 1;
            }
            if (lose) R[nR++] = v;
        }
        for (int64_t i = 0; i < nR; ++i) color[R[i]] = 0;
        int32_t* t = U; U = R; R = t;
        nU = nR;
    }
    if (k >= 0) {
        /* sequential finish in ascending (key, id) order */
        or_sort_key = key;
        qsort(U, (size_t)nU, sizeof(int32_t), or_cmp_vertex);
        for (int64_t i = 0; i < nU; ++i) {
            const int32_t v = U[i];
            ++label;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t w = col_idx[e];
                if (w != v) forbidden[color[w]] = label;
            }
            int32_t c = 1;
            while (forbidden[c] == label) ++c;
            color[v] = c;
        }
        if (tail_count) *tail_count = nU;
    }
    free(S);
    free(tent);
    free(U);
    free(R);
    free(forbidden);
    return k;
}

/*
 * Smallest-last ordering (Matula and Beck): repeatedly remove a vertex of
 * minimum degree in the remaining graph, ties to the smallest id; the
 * colouring order is the reverse of the removal order.  Implemented with a
 * binary heap of (current degree, id) entries and lazy deletion.
 * rank[v] receives v's position in the colouring order (0 = coloured first).
 * Returns the degeneracy (the largest degree seen at removal).
 */
static void or_heap_push(int64_t* h, int64_t* sz, int64_t x) {
    int64_t i = (*sz)++;
    h[i] = x;
    while (i > 0) {
        const int64_t p = (i - 1) / 2;
        if (h[p] <= h[i]) break;
        const int64_t t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static int64_t or_heap_pop(int64_t* h, int64_t* sz) {
    const int64_t top = h[0];
    h[0] = h[--(*sz)];
    int64_t i = 0;
    for (;;) {
        const int64_t l = 2 * i + 1, r = l + 1;
        int64_t m = i;
        if (l < *sz && h[l] < h[m]) m = l;
        if (r < *sz && h[r] < h[m]) m = r;
        if (m == i) break;
        const int64_t t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

int32_t or_smallest_last(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* rank) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * nn);
    unsigned char* gone = (unsigned char*)calloc(nn, 1);
    const int64_t cap = (int64_t)n + (int64_t)row_ptr[n] + 1;
    int64_t* heap = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    int64_t sz = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = 0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) d += (col_idx[e] != v);
        deg[v] = d;
        or_heap_push(heap, &sz, ((int64_t)d << 32) | (int64_t)v);
    }
    int32_t removed = 0, degeneracy = 0;
    while (removed < n) {
        const int64_t top = or_heap_pop(heap, &sz);
        const int32_t v = (int32_t)(top & 0xFFFFFFFF);
        const int32_t d = (int32_t)(top >> 32);
        if (gone[v] || d != deg[v]) continue; /* stale entry */
        gone[v] = 1;
        if (d > degeneracy) degeneracy = d;
        rank[v] = n - 1 - removed;
        ++removed;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col_idx[e];
            if (w == v || gone[w]) continue;
            deg[w] -= 1;
            or_heap_push(heap, &sz, ((int64_t)deg[w] << 32) | (int64_t)w);
        }
    }
    free(deg);
    free(gone);
    free(heap);
    return degeneracy;
}

/*
 * Dataflow colouring (Algorithm 3, section "A dataflow algorithm"), read in
 * rounds: a vertex is coloured in the round after the last of its preceding
 * neighbours ((key, id) precedence) is coloured -- in round 1 when it has
 * none -- with the smallest positive colour none of those neighbours holds.
 * So
 *   round[v] = 1 + max{round[w] : w in adj(v), w precedes v}   (1 if none),
 *   color[v] = min{c >= 1 : c not in {color[w] : w in adj(v), w precedes v}}.
 * Both refer only to preceding vertices, so one visit of the vertices in
 * ascending (key, id) order fills them.  The forbidden array is stamped with
 * the preceding neighbours' colours only (the later ones are not read).
 * Returns the number of rounds (the largest round; 0 for n == 0).
 */
int32_t or_dataflow(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* key,
                    int32_t* color, int32_t* round) {
    const int32_t dmax = or_max_degree(n, row_ptr);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* forbidden = (int64_t*)malloc(sizeof(int64_t) * (size_t)(dmax + 2));
    for (int32_t v = 0; v < n; ++v) order[v] = v;
    if (key) {
        or_sort_key = key;
        qsort(order, (size_t)n, sizeof(int32_t), or_cmp_vertex);
    }
    for (int32_t c = 0; c < dmax + 2; ++c) forbidden[c] = -1;
    int32_t rounds = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t v = order[i];
        int32_t r = 0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col_idx[e];
            if (w == v || !or_before(key, w, v)) continue;
            forbidden[color[w]] = v;
            if (round[w] > r) r = round[w];
        }
        int32_t c = 1;
        while (forbidden[c] == v) ++c;
        color[v] = c;
        round[v] = r + 1;
        if (r + 1 > rounds) rounds = r + 1;
    }
    free(order);
    free(forbidden);
    return rounds;
}

int or_num_threads(void) { return omp_get_max_threads(); }

/*
 * Block Gauss-Seidel variant of the speculative colouring (Algorithm 2 with
 * the static schedule of section "Scalability Results": each thread owns a
 * fixed contiguous range of vertices and visits it in index order, seeing its
 * own colours of the current round at once).  Blocks are the id ranges
 * [b*B, (b+1)*B).  Round k, with U the uncoloured vertices:
 *   S = copy(color)
 *   phase 1, for each block, for v in U in the block in ascending id:
 *     tent[v] = min{c >= 1 : c not in {S[w] : w in adj(v)}
 *                                  and not in {tent[w] : w in adj(v), w in U,
 *                                              w in v's block, w < v}}
 *   phase 2, for v in U: v loses if some neighbour w holds its colour
 *     (tent[w] for w in U, S[w] otherwise) and (key[w], w) < (key[v], v)
 *   winners keep tent[v]; losers stay uncoloured (next worklist).
 * B = 1 is the round-synchronous simulation above; B >= n (one block) is the
 * serial greedy in index order, finished in one round.  The blocks are
 * independent within phase 1, so their order of visit does not matter.
 * log (may be NULL) receives per round: k, |U_k|, sum of degrees over U_k,
 * number of losers; at most max_log rounds.
 * nthreads <= 0 means OpenMP's default; the result never depends on it.
 * Returns the number of rounds, or -5 when max_rounds is exceeded.
 */
int32_t or_block_gs(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* key,
                    int32_t block, int32_t* color, int64_t* log, int32_t max_log, int32_t max_rounds,
                    int32_t nthreads) {
    if (block < 1) return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    const int32_t dmax = or_max_degree(n, row_ptr);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * nn);
    int32_t* tent = (int32_t*)malloc(sizeof(int32_t) * nn);
    unsigned char* inU = (unsigned char*)malloc(nn);
    unsigned char* lose = (unsigned char*)malloc(nn);
    for (int32_t v = 0; v < n; ++v) color[v] = 0;
    const int64_t nblocks = ((int64_t)n + block - 1) / block;
    int64_t nU = n;
    int32_t k = 0;
    while (nU > 0) {
        if (k >= max_rounds) { k = -5; break; }
        ++k;
        memcpy(S, color, sizeof(int32_t) * (size_t)n);
        for (int32_t v = 0; v < n; ++v) inU[v] = color[v] == 0;

        /* Phase 1: each block's worklist vertices in id order.  Blocks read
         * only S and their own tent entries, so they are independent and run
         * on the threads in any order; each thread stamps a forbidden array
         * of its own, fresh every round, with the visited vertex. */
#pragma omp parallel num_threads(nthreads)
        {
            int64_t* forbidden = (int64_t*)malloc(sizeof(int64_t) * (size_t)(dmax + 2));
            for (int32_t c = 0; c < dmax + 2; ++c) forbidden[c] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t b = 0; b < nblocks; ++b) {
                const int64_t b0 = b * block;
                const int64_t b1 = b0 + block < n ? b0 + block : n;
                for (int64_t vv = b0; vv < b1; ++vv) {
                    const int32_t v = (int32_t)vv;
                    if (!inU[v]) continue;
                    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                        const int32_t w = col_idx[e];
                        if (w == v) continue;
                        forbidden[S[w]] = v;
                        if (inU[w] && w >= b0 && w < v) forbidden[tent[w]] = v;
                    }
                    int32_t c = 1;
                    while (forbidden[c] == v) ++c;
                    tent[v] = c;
                }
            }
            free(forbidden);
        }

        /* Phase 2: conflicts against every neighbour's colour of this round. */
        int64_t work = 0, nR = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1024) reduction(+ : work)
        for (int32_t v = 0; v < n; ++v) {
            if (!inU[v]) continue;
            unsigned char l = 0;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t w = col_idx[e];
                if (w == v) continue;
                const int32_t cw = inU[w] ? tent[w] : S[w];
                if (cw == tent[v] && or_before(key, w, v)) l = 1;
            }
            lose[v] = l;
            work += row_ptr[v + 1] - row_ptr[v];
        }
        for (int32_t v = 0; v < n; ++v) {
            if (!inU[v]) continue;
            if (lose[v]) ++nR;
            else color[v] = tent[v];
        }
        if (log && k <= max_log) {
            log[4 * (k - 1) + 0] = k;
            log[4 * (k - 1) + 1] = nU;
            log[4 * (k - 1) + 2] = work;
            log[4 * (k - 1) + 3] = nR;
        }
        nU = nR;
    }
    free(S);
    free(tent);
    free(inU);
    free(lose);
    return k;
}

