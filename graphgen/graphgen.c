/*
 * Seeded synthetic graph generators (host C, OpenMP).
 *
 * This module only produces inputs: edge samples and symmetric CSR.  It holds
 * none of the colouring arithmetic, and both the CPU oracle and the GPU path
 * consume what it writes.
 *
 * Random numbers come from a counter-based use of splitmix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
 * k-th draw of a stream with state s is mix(s + (k+1) * GAMMA), where mix is
 * splitmix64's output finaliser.  Every draw is a pure function of
 * (seed, purpose tag, counter), so results do not depend on thread count.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004; the generator of the paper's
 * test-graph section): each sample descends `scale` levels, picking quadrant
 * (0,0), (0,1), (1,0), (1,1) with probabilities a, b, c, d; the row bit and
 * the column bit of each level are appended most-significant first.  No noise
 * is added.  Self-loops are dropped and duplicates merged when the CSR is
 * built, as the paper's section on the generator states.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* State of the stream for (seed, tag). */
static inline uint64_t gg_stream(uint64_t seed, uint64_t tag) {
    return gg_mix(seed * GG_GAMMA + gg_mix(tag + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t gg_draw(uint64_t stream, uint64_t ctr) {
    return gg_mix(stream + (ctr + 1) * GG_GAMMA);
}

/* Uniform integer in [0, n) from the high 32 bits (multiply-shift). */
static inline uint32_t gg_below(uint64_t h, uint32_t n) {
    return (uint32_t)(((h >> 32) * (uint64_t)n) >> 32);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double gg_unit(uint64_t h) {
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

enum { TAG_UNIFORM = 1, TAG_RMAT = 2, TAG_HASH = 3, TAG_EXTRA = 4, TAG_POINTS = 5 };

void gg_hash_u64(uint64_t seed, uint64_t tag, int64_t count, uint64_t* out) {
    const uint64_t s = gg_stream(seed, TAG_HASH ^ (tag << 8));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) out[i] = gg_draw(s, (uint64_t)i);
}

/* m endpoint pairs, each endpoint uniform on [0, n). */
void gg_uniform_pairs(uint64_t seed, int32_t n, int64_t m, int32_t* src, int32_t* dst) {
    const uint64_t s = gg_stream(seed, TAG_UNIFORM);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        src[i] = (int32_t)gg_below(gg_draw(s, 2 * (uint64_t)i), (uint32_t)n);
        dst[i] = (int32_t)gg_below(gg_draw(s, 2 * (uint64_t)i + 1), (uint32_t)n);
    }
}

/* m R-MAT samples on 2^scale vertices; one 53-bit draw per level. */
void gg_rmat_pairs(uint64_t seed, int32_t scale, int64_t m, double a, double b, double c,
                   int32_t* src, int32_t* dst) {
    const uint64_t s = gg_stream(seed, TAG_RMAT);
    const uint64_t ta = (uint64_t)(a * 9007199254740992.0);
    const uint64_t tab = (uint64_t)((a + b) * 9007199254740992.0);
    const uint64_t tabc = (uint64_t)((a + b + c) * 9007199254740992.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            const uint64_t r = gg_draw(s, (uint64_t)i * (uint64_t)scale + (uint64_t)l) >> 11;
            uint32_t rb, cb;
            if (r < ta) { rb = 0; cb = 0; }
            else if (r < tab) { rb = 0; cb = 1; }
            else if (r < tabc) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            u = (u << 1) | rb;
            v = (v << 1) | cb;
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
}

/* m extra pairs uniform on [0, n) drawn from a separate stream (used to add
 * random long edges to stencil grids). */
void gg_extra_pairs(uint64_t seed, int32_t n, int64_t m, int32_t* src, int32_t* dst) {
    const uint64_t s = gg_stream(seed, TAG_EXTRA);
    for (int64_t i = 0; i < m; ++i) {
        src[i] = (int32_t)gg_below(gg_draw(s, 2 * (uint64_t)i), (uint32_t)n);
        dst[i] = (int32_t)gg_below(gg_draw(s, 2 * (uint64_t)i + 1), (uint32_t)n);
    }
}

/* n points uniform in the unit square. */
void gg_unit_points(uint64_t seed, int32_t n, double* x, double* y) {
    const uint64_t s = gg_stream(seed, TAG_POINTS);
    for (int32_t i = 0; i < n; ++i) {
        x[i] = gg_unit(gg_draw(s, 2 * (uint64_t)i));
        y[i] = gg_unit(gg_draw(s, 2 * (uint64_t)i + 1));
    }
}

/* Pairs (i, j), i < j, with squared distance <= r2; cell-list search.
 * Returns the number of pairs written, or -1 if `cap` is too small. */
int64_t gg_rgg_pairs(int32_t n, const double* x, const double* y, double r,
                     int32_t* src, int32_t* dst, int64_t cap) {
    int32_t g = (int32_t)floor(1.0 / r);
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    const int64_t cells = (int64_t)g * g;
    int32_t* head = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cells + 1));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    memset(head, 0, sizeof(int32_t) * (size_t)(cells + 1));
    for (int32_t i = 0; i < n; ++i) {
        int32_t cx = (int32_t)(x[i] * g), cy = (int32_t)(y[i] * g);
        if (cx >= g) cx = g - 1;
        if (cy >= g) cy = g - 1;
        cell[i] = cy * g + cx;
        head[cell[i] + 1]++;
    }
    for (int64_t k = 0; k < cells; ++k) head[k + 1] += head[k];
    {
        int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)cells);
        memcpy(cur, head, sizeof(int32_t) * (size_t)cells);
        for (int32_t i = 0; i < n; ++i) order[cur[cell[i]]++] = i;
        free(cur);
    }
    const double r2 = r * r;
    int64_t cnt = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t cx = cell[i] % g, cy = cell[i] / g;
        for (int32_t dy = -1; dy <= 1; ++dy) {
            const int32_t yy = cy + dy;
            if (yy < 0 || yy >= g) continue;
            for (int32_t dx = -1; dx <= 1; ++dx) {
                const int32_t xx = cx + dx;
                if (xx < 0 || xx >= g) continue;
                const int32_t k = yy * g + xx;
                for (int32_t p = head[k]; p < head[k + 1]; ++p) {
                    const int32_t j = order[p];
                    if (j <= i) continue;
                    const double ddx = x[i] - x[j], ddy = y[i] - y[j];
                    if (ddx * ddx + ddy * ddy <= r2) {
                        if (cnt >= cap) { free(head); free(order); free(cell); return -1; }
                        src[cnt] = i;
                        dst[cnt] = j;
                        ++cnt;
                    }
                }
            }
        }
    }
    free(head);
    free(order);
    free(cell);
    return cnt;
}

static int gg_cmp_i32(const void* a, const void* b) {
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static void gg_sort_row(int32_t* a, int64_t len) {
    if (len <= 48) {
        for (int64_t i = 1; i < len; ++i) {
            const int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
        return;
    }
    qsort(a, (size_t)len, sizeof(int32_t), gg_cmp_i32);
}

/*
 * Symmetric CSR from m sample pairs: drop self-loops, add both directions,
 * sort each row ascending and merge duplicates.  row_ptr has n+1 entries;
 * col_idx must hold 2*m entries.  Returns nnz, or -1 if nnz >= 2^31 or
 * memory runs out.
 */
int64_t gg_build_csr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                     int32_t* row_ptr, int32_t* col_idx) {
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!off) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        if (src[i] == dst[i]) continue;
#pragma omp atomic
        off[src[i] + 1]++;
#pragma omp atomic
        off[dst[i] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    const int64_t total = off[n];
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!tmp || !cur) { free(off); free(tmp); free(cur); return -1; }
    memcpy(cur, off, sizeof(int64_t) * (size_t)n);
    /* Fill order inside a row depends on thread timing; rows are sorted
     * below, so the result does not. */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        const int32_t u = src[i], v = dst[i];
        if (u == v) continue;
        int64_t pu, pv;
#pragma omp atomic capture
        pu = cur[u]++;
#pragma omp atomic capture
        pv = cur[v]++;
        tmp[pu] = v;
        tmp[pv] = u;
    }
    free(cur);
    int32_t* newdeg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) {
        int32_t* row = tmp + off[v];
        const int64_t len = off[v + 1] - off[v];
        gg_sort_row(row, len);
        int64_t k = 0;
        for (int64_t i = 0; i < len; ++i)
            if (k == 0 || row[i] != row[k - 1]) row[k++] = row[i];
        newdeg[v] = (int32_t)k;
    }
    int64_t nnz = 0;
    for (int32_t v = 0; v < n; ++v) nnz += newdeg[v];
    if (nnz >= 2147483647LL) { free(off); free(tmp); free(newdeg); return -1; }
    row_ptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) row_ptr[v + 1] = row_ptr[v] + newdeg[v];
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v)
        memcpy(col_idx + row_ptr[v], tmp + off[v], sizeof(int32_t) * (size_t)newdeg[v]);
    free(off);
    free(tmp);
    free(newdeg);
    return nnz;
}

int gg_num_threads(void) { return omp_get_max_threads(); }
