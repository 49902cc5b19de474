/*
 * Host-side memory and undefined-behaviour check of the oracle and the
 * input generator: this file includes both C sources, generates a few
 * seeded graphs and runs every oracle routine on them.  The CPU test suite
 * compiles it with gcc -fsanitize=address,undefined and runs it; any
 * sanitizer report or failed check fails the test.
 */
#include "../../graphgen/graphgen.c"
#include "../../oracle/oracle.c"

#include <stdio.h>

static int check_proper(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* col) {
    for (int32_t v = 0; v < n; ++v) {
        if (col[v] < 1 || col[v] > rp[v + 1] - rp[v] + 1) return 0;
        for (int32_t p = rp[v]; p < rp[v + 1]; ++p)
            if (ci[p] != v && col[ci[p]] == col[v]) return 0;
    }
    return 1;
}

static int run_graph(const char* name, int32_t n, const int32_t* rp, const int32_t* ci) {
    int32_t* col = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* fixed = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* rank = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* rnd = malloc(sizeof(int32_t) * (size_t)(n + 1));
    uint32_t* key = malloc(sizeof(uint32_t) * (size_t)(n + 1));
    int64_t* log = malloc(sizeof(int64_t) * 4 * (size_t)(n + 64));
    uint64_t* h = malloc(sizeof(uint64_t) * (size_t)(n + 1));
    int ok = 1;
    gg_hash_u64(7, 3, n, h);
    for (int32_t v = 0; v < n; ++v) key[v] = (uint32_t)(h[v] & 15u);  /* keys with ties */
    or_greedy(n, rp, ci, key, col);
    ok &= check_proper(n, rp, ci, col);
    for (int th = 1; th <= 4; th += 3) {
        ok &= or_spec_sim(n, rp, ci, NULL, col, fixed, log, n + 64, n + 1, th) >= 0;
        ok &= check_proper(n, rp, ci, col);
        ok &= or_block_gs(n, rp, ci, key, 7, col, log, n + 64, n + 1, th) >= 0;
        ok &= check_proper(n, rp, ci, col);
    }
    int64_t tail = 0;
    ok &= or_spec_tail(n, rp, ci, key, 33, col, &tail, n + 1) >= 0;
    ok &= check_proper(n, rp, ci, col);
    or_smallest_last(n, rp, ci, rank);
    ok &= or_dataflow(n, rp, ci, (const uint32_t*)rank, col, rnd) >= 0;
    ok &= check_proper(n, rp, ci, col);
    printf("%s: n=%d nnz=%d %s\n", name, n, rp[n], ok ? "ok" : "FAILED");
    free(col); free(fixed); free(rank); free(rnd); free(key); free(log); free(h);
    return ok;
}

static int build_and_run(const char* name, int32_t n, int64_t m, int32_t* src, int32_t* dst) {
    int32_t* rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* ci = malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    const int64_t nnz = gg_build_csr(n, m, src, dst, rp, ci);
    int ok = nnz >= 0 && run_graph(name, n, rp, ci);
    free(rp);
    free(ci);
    return ok;
}

int main(void) {
    int ok = 1;
    {
        const int32_t scale = 11;
        const int64_t m = 8 << scale;
        const int64_t cap = 20000;  /* the largest pair count below */
        int32_t* s = malloc(sizeof(int32_t) * (size_t)cap);
        int32_t* d = malloc(sizeof(int32_t) * (size_t)cap);
        gg_rmat_pairs(5, scale, m, 0.55, 0.1, 0.1, s, d);
        ok &= build_and_run("rmat11", 1 << scale, m, s, d);
        gg_uniform_pairs(6, 3000, 20000, s, d);
        ok &= build_and_run("uniform3000", 3000, 20000, s, d);
        gg_extra_pairs(8, 500, 100, s, d);
        ok &= build_and_run("extra500", 500, 100, s, d);
        free(s);
        free(d);
    }
    {
        const int32_t n = 2000;
        double* x = malloc(sizeof(double) * n);
        double* y = malloc(sizeof(double) * n);
        gg_unit_points(9, n, x, y);
        const int64_t cap = 200000;
        int32_t* s = malloc(sizeof(int32_t) * (size_t)cap);
        int32_t* d = malloc(sizeof(int32_t) * (size_t)cap);
        const int64_t m = gg_rgg_pairs(n, x, y, 0.04, s, d, cap);
        ok &= m >= 0 && build_and_run("rgg2000", n, m, s, d);
        free(x); free(y); free(s); free(d);
    }
    {
        int32_t rp[1] = {0};
        ok &= run_graph("empty", 0, rp, NULL);
    }
    return ok ? 0 : 1;
}
