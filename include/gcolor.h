/*
 * gcolor -- speculative iterative distance-1 graph colouring on MI355X (gfx950).
 *
 * C ABI of libgcolor.so.  Method: Catalyurek, Feo, Gebremedhin, Halappanavar,
 * Pothen, "Graph colouring algorithms for multi-core and massively
 * multithreaded architectures", section "Iterative parallel coloring
 * algorithm" (Algorithm 2), built on the serial first-fit of Algorithm 1.
 *
 * What is computed (the round-synchronous reading of Algorithm 2):
 *   colour = 0 everywhere; U = all vertices
 *   repeat until U is empty:
 *     phase 1 (tentative colouring), for each v in U:
 *       tent[v] = smallest c >= 1 not held by a neighbour, where the neighbours'
 *       colours are those committed at the end of the previous round (vertices
 *       still in U count as uncoloured);
 *     phase 2 (conflict detection), for each v in U:
 *       v is re-queued if a neighbour w in U has tent[w] == tent[v] and w
 *       precedes v; otherwise v keeps tent[v] for good.
 *   "w precedes v" means (priority[w], w) < (priority[v], v); with no priority
 *   array the vertex index alone decides, as in the paper (the smaller index
 *   keeps its colour).
 * The result is a deterministic function of (graph, priority): it does not
 * depend on launch shapes, thread timing or the order of the worklist.
 *
 * Graph format (all arrays in device memory, owned by the caller):
 *   row_ptr  int32[n+1], row_ptr[0] == 0, non-decreasing, nnz = row_ptr[n] < 2^31;
 *   col_idx  int32[nnz] (may be NULL when nnz == 0), neighbour ids in [0, n); the adjacency must be
 *            symmetric (w in adj(v) iff v in adj(w)).  Without a priority array
 *            every row must be sorted ascending.  Self-loops are ignored.  A
 *            neighbour may be listed more than once provided each pair is
 *            listed equally often in both rows (as in a CSR built by
 *            symmetrising an edge list with repeated edges); the result is
 *            that of the graph without the repeats.
 *   priority uint32[n] or NULL.
 *   colors_out int32[n]: receives colours in [1, max degree + 1].
 * Nothing is read or written outside these extents; the library never frees
 * caller memory.
 *
 * Errors: every entry point returns 0 on success or a negative code
 * (GCOLOR_E*); nothing aborts or throws across the ABI.  gcolor_strerror()
 * names a code.  A HIP error raised by an earlier, unrelated call on the same
 * device may surface here as GCOLOR_EHIP.
 *
 * Streams: all device work is enqueued on `stream` (0 = the null stream).
 * color_graph, color_graph_ex and color_graph_blocks read small counters back
 * to the host to decide when the worklist is empty, so they return only after
 * the colouring is complete; color_graph_async (a round budget instead) and
 * color_graph_batch never wait on the host.
 */
#ifndef GCOLOR_H
#define GCOLOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gcolor_stream_t; /* same object as hipStream_t */

enum {
    GCOLOR_OK = 0,
    GCOLOR_EINVAL = -1,     /* bad argument: negative n, NULL array, bad flags */
    GCOLOR_ECSR = -2,       /* malformed CSR (reported only with GCOLOR_VALIDATE) */
    GCOLOR_EWORKSPACE = -3, /* caller workspace smaller than gcolor_workspace_bytes */
    GCOLOR_EHIP = -4,       /* a HIP runtime call failed */
    GCOLOR_EROUNDS = -5,    /* round cap exceeded (only with a cap below the default) */
    GCOLOR_ENOTSUP = -6,    /* sizes beyond what the library supports */
    GCOLOR_EINTERNAL = -7   /* an internal consistency check failed (a bug; report it) */
};

/* Flags for color_graph_ex. */
enum {
    GCOLOR_VALIDATE = 1u << 0, /* check the CSR on the device first (costs a pass) */
    GCOLOR_STATS = 1u << 1,    /* fill *stats (rounds, colours, edge work) */
    GCOLOR_PLAIN = 1u << 2,    /* use the plain engine: every round rescans every worklist row
                                  (same result as the default incremental engine) */
    GCOLOR_DATAFLOW = 1u << 3, /* a different colouring: the dataflow algorithm (section "A
                                  dataflow algorithm", Algorithm 3) in rounds.  A vertex is
                                  coloured once all of its preceding neighbours are, with the
                                  smallest colour none of them holds; the result is the serial
                                  first-fit (Algorithm 1) visiting vertices in ascending
                                  (priority, id) order, and the number of rounds is the number of
                                  vertices on the longest path along which each vertex precedes
                                  the next (n on a path in natural order).  Not combinable with
                                  GCOLOR_PLAIN. */
    GCOLOR_SERIAL_TAIL = 1u << 4 /* a different colouring: the rounds run while more than
                                    gcolor_get_serial_tail() vertices are uncoloured, then the
                                    rest are coloured one at a time in ascending (priority, id)
                                    order, each with the smallest colour none of its neighbours
                                    holds (the switch to a sequential computation that section
                                    "Iterative and degree of concurrency" suggests once
                                    conflicts are few).  Default engine only. */
};

typedef struct gcolor_stats {
    int32_t rounds;     /* number of rounds (a round = phase 1 + phase 2) */
    int32_t num_colors; /* largest colour assigned */
    int64_t edge_work;  /* sum over rounds of the degrees of the worklist (the first 65536
                           rounds: the device keeps per-round records for those) */
    int32_t status;     /* 0, or the code the call returned */
    int32_t serial_tail; /* vertices coloured by the sequential finish (GCOLOR_SERIAL_TAIL) */
} gcolor_stats_t;

/* Per-round record written to round_log (host memory) by color_graph_ex:
 * round index (1-based), |U_k| (worklist size), E_k (sum of degrees over
 * U_k), vertices committed in the round, and for the incremental engine the
 * number of dirty vertices (tentative colour changed), their degree sum, and
 * the row entries its dirty pass read for them (equal to the degree sum
 * except for rows longer than 512 entries, which are read without the
 * neighbours already committed).  With GCOLOR_DATAFLOW the worklist of round
 * k is the set of vertices coloured in it (committed == worklist), the
 * dirty fields are 0, and edge_work over all rounds is nnz. */
typedef struct gcolor_round {
    int64_t round;
    int64_t worklist;
    int64_t edge_work;
    int64_t committed;
    int64_t dirty;
    int64_t dirty_edges;
    int64_t scanned;
} gcolor_round_t;

/* Bytes of device workspace color_graph_ex needs for a graph of this size. */
size_t gcolor_workspace_bytes(int32_t n, int64_t nnz);

/*
 * Colour the graph.  Uses a workspace the library allocates on first use and
 * keeps per device (grown when a larger graph arrives); calls on that
 * workspace from several host threads take turns (each holds its device's
 * lock until it returns).  Returns 0 or a negative GCOLOR_E* code.  Every colouring call also keeps a 256-byte pinned
 * host buffer per calling host thread for its small read-backs (held until
 * the process ends).
 */
int color_graph(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                const uint32_t* priority, int32_t* colors_out, gcolor_stream_t stream);

/*
 * As color_graph, with a caller-provided device workspace of ws_bytes bytes
 * (>= gcolor_workspace_bytes(n, nnz); NULL selects the library's own), flags
 * (GCOLOR_*), optional host pointers: stats (filled when GCOLOR_STATS is set)
 * and round_log (capacity max_log records; the first min(rounds, max_log,
 * 65536) rounds are written).
 */
int color_graph_ex(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                   const uint32_t* priority, int32_t* colors_out, void* workspace,
                   size_t ws_bytes, uint32_t flags, gcolor_stats_t* stats,
                   gcolor_round_t* round_log, int32_t max_log, gcolor_stream_t stream);

/*
 * Stream-ordered colouring (Algorithm 2's loop "while U is not empty" run
 * for a fixed budget of rounds, so that the host never waits): every kernel
 * is enqueued on `stream` and the call returns at once, with no host
 * synchronisation and no allocation, so it may be captured into a HIP graph
 * and replayed.  The colouring is color_graph's, vertex for vertex (the
 * default incremental engine).
 *   n, row_ptr, col_idx, priority, colors_out: as color_graph;
 *   nnz        row_ptr[n] (the caller knows it; nothing is read back);
 *   workspace  device memory of gcolor_workspace_bytes(n, nnz) bytes, owned
 *              by the caller (required);
 *   max_rounds the round budget (>= 1): exactly this many rounds are
 *              enqueued; rounds after the worklist has emptied find no work
 *              and return at once (a few microseconds each);
 *   flags      0 or GCOLOR_VALIDATE (the CSR checks run on the device: a
 *              malformed CSR stops the colouring before any row is walked);
 *   stats_dev  device gcolor_stats_t, written when the stream reaches the
 *              end of the call: rounds, colours and edge work as
 *              color_graph_ex reports them, and status = GCOLOR_OK,
 *              GCOLOR_ECSR (validation failed), GCOLOR_EROUNDS (the budget
 *              ended with vertices uncoloured; colors_out is then
 *              incomplete) or GCOLOR_EINTERNAL.  The other fields are 0
 *              unless status is GCOLOR_OK.
 * The return value reports only what the host can see: GCOLOR_EINVAL
 * (negative n or nnz, nnz >= 2^31, max_rounds < 1, NULL pointers, other
 * flags), GCOLOR_EWORKSPACE, GCOLOR_EHIP (a launch failed).  The process-wide
 * round cap does not apply (the budget replaces it).  Calls sharing one
 * workspace must not overlap.
 */
int color_graph_async(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      const uint32_t* priority, int32_t* colors_out, void* workspace, size_t ws_bytes,
                      int32_t max_rounds, uint32_t flags, gcolor_stats_t* stats_dev, gcolor_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * color_graph_async with the library's own fixed workspace, a device array
 * of gcolor_noalloc_max_bytes() bytes (64 MiB) that is part of the code
 * object, one per device, held until the process ends.  The call allocates
 * nothing (the array's device address is looked up once per device, on the
 * first call there); the caller still passes inputs and outputs as for
 * color_graph_async.  Graphs whose gcolor_workspace_bytes(n, nnz) exceeds the
 * array are refused with GCOLOR_ENOTSUP before any device work (about
 * 315,000 vertices at 10 entries per vertex).  Every call on a device shares
 * that device's array, which keeps the last call's contents: calls that
 * overlap on one device (other streams or threads) race and must be
 * serialised by the caller.  Other errors and stats_dev: as
 * color_graph_async.
 */
size_t gcolor_noalloc_max_bytes(void);
int color_graph_async_noalloc(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              const uint32_t* priority, int32_t* colors_out, int32_t max_rounds, uint32_t flags,
                              gcolor_stats_t* stats_dev, gcolor_stream_t stream);

/*
 * Tuning (process-wide, applies to later calls): bin_limits[4] are the
 * largest degrees of bins 0..3 (one lane, 4 lanes, 16 lanes and one
 * wavefront per vertex); larger degrees take a workgroup per vertex.  Must be
 * non-decreasing.  blocks_per_cu (1..64, 0 = keep) sizes the phase grids.
 * NULL bin_limits keeps the current limits.  Defaults: {8, 32, 128, 2048}
 * and 4.  Results never depend on tuning.  The autotuner (Python package,
 * autotune.py) searches these per configuration.
 */
int gcolor_set_tuning(const int32_t* bin_limits, int32_t blocks_per_cu);
int gcolor_get_tuning(int32_t* bin_limits, int32_t* blocks_per_cu);

/*
 * Blocks per CU of the incremental engine's two round kernels: blocks_a for
 * the dirty-vertex kernel, blocks_c for the commit kernel (which also
 * completes the counters of dirty vertices with dirty preceding
 * neighbours).  1..64 each, 0 = the common blocks_per_cu above (the
 * default).  Errors: GCOLOR_EINVAL outside 0..64.  Results never depend on
 * it.
 */
int gcolor_set_kernel_blocks(int32_t blocks_a, int32_t blocks_c);
int gcolor_get_kernel_blocks(int32_t* blocks_a, int32_t* blocks_c);

/*
 * Round cap (process-wide, applies to later color_graph / color_graph_ex
 * calls of every engine): a call that needs more than max_rounds rounds
 * stops launching after round max_rounds and returns GCOLOR_EROUNDS, with
 * colors_out and *stats undefined.  A call that needs at most max_rounds
 * rounds is unaffected.  0 restores the default, n + 64 for a graph of n
 * vertices: every engine ends within n rounds on valid input (the vertex
 * with the smallest key among those left is committed in every round of
 * Algorithm 2; the dataflow rounds follow increasing paths of the order), so
 * the default is never reached and GCOLOR_EROUNDS then signals a bug.
 * Errors: GCOLOR_EINVAL for max_rounds < 0.
 */
int gcolor_set_round_cap(int32_t max_rounds);
int gcolor_get_round_cap(int32_t* max_rounds);

/*
 * Size of the sequential finish of GCOLOR_SERIAL_TAIL (process-wide, applies
 * to later calls): the rounds stop once at most max_vertices vertices are
 * uncoloured.  1..8192 (one workgroup sorts and colours them); default 1024.
 * Errors: GCOLOR_EINVAL outside 1..8192 or a NULL pointer.
 */
int gcolor_set_serial_tail(int32_t max_vertices);
int gcolor_get_serial_tail(int32_t* max_vertices);

/*
 * Block Gauss-Seidel variant of the speculative colouring (Algorithm 2 run
 * with the static schedule of the section "Scalability Results": a thread
 * owns a fixed contiguous range of vertices, visits it in index order and
 * sees its own colours of the round at once).  A different colouring from
 * color_graph's, deterministic for a given block_size:
 *   blocks are the id ranges [b*block_size, (b+1)*block_size); in each round
 *   every block gives its uncoloured vertices, in ascending id, the smallest
 *   colour held neither by a coloured neighbour nor by a neighbour of the
 *   same block chosen earlier in the round; then an uncoloured vertex whose
 *   choice equals that of a neighbour preceding it in (priority, id) order
 *   gives its choice back, and the others keep theirs.
 * block_size 1 gives exactly color_graph's colouring; one block holding every
 * vertex gives the serial greedy in index order in one round.
 *   n, row_ptr, col_idx, priority, colors_out, stream: as color_graph (rows
 *                 need not be sorted; priority may be NULL);
 *   block_size    1 .. 2048;
 *   workspace     device memory of gcolor_blocks_workspace_bytes(n) bytes, or
 *                 NULL for the library's cached per-device allocation (calls
 *                 on it from several host threads take turns);
 *   stats         optional (host): rounds, largest colour, and the sum over
 *                 rounds of the degrees of the uncoloured vertices.
 * The CSR is not validated.  The process-wide round cap of
 * gcolor_set_round_cap applies.  Errors: GCOLOR_EINVAL (negative n,
 * block_size outside 1..2048, NULL arrays), GCOLOR_EWORKSPACE,
 * GCOLOR_EHIP, GCOLOR_EROUNDS.  Blocking: returns after the colouring is
 * complete on `stream`.
 */
size_t gcolor_blocks_workspace_bytes(int32_t n);
int color_graph_blocks(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* priority,
                       int32_t block_size, int32_t* colors_out, void* workspace, size_t ws_bytes,
                       gcolor_stats_t* stats, gcolor_stream_t stream);

/*
 * Batch tuning (process-wide, applies to later color_graph_batch calls).
 * block_threads: threads per workgroup, 256 or 1024, or 0 for the default
 * (1024 when the LDS capacity below is at least 16384 vertices, else 256).
 * lds_factor (1..64): the LDS path's vertex capacity is lds_factor times the
 * batch's mean graph size, at least 1024 and at most lds_max_vertices
 * (0..65536; 0 disables the LDS path, every graph then keeps its state in
 * global memory).  Errors: GCOLOR_EINVAL for values out of range.  Results
 * never depend on tuning.
 */
int gcolor_set_batch_tuning(int32_t block_threads, int32_t lds_factor, int32_t lds_max_vertices);
int gcolor_get_batch_tuning(int32_t* block_threads, int32_t* lds_factor, int32_t* lds_max_vertices);

/*
 * Kernel timing with HIP events recorded around every phase launch.
 * gcolor_profile(1) enables it and clears the totals, gcolor_profile(0)
 * disables it.  gcolor_profile_read(kernel, ...) returns the summed
 * milliseconds and launch count of a kernel: 0 = plain phase 1 (tentative
 * colouring), 1 = plain phase 2 (conflict detection and worklist
 * compaction), 2 = incremental tentative colours of dirty vertices,
 * 3 = incremental dirty lists built from the round's bitmap (two kernels
 * per round, timed together), 4 = incremental counter completion, commit
 * and dirty marks, 5 = dataflow round.
 */
int gcolor_profile(int32_t enable);
int gcolor_profile_read(int32_t kernel, double* total_ms, int64_t* launches);

/*
 * Batched colouring of many independent graphs in one persistent launch
 * (each graph is coloured exactly as color_graph colours it alone).
 *   vtx_off  int64[G+1]  vertex offsets: graph g owns vertices
 *                        [vtx_off[g], vtx_off[g+1]) of colors_out / priority;
 *   edge_off int64[G+1]  entry offsets of each graph in col_idx;
 *   row_ptr  int32[V+G]  each graph's own n_g+1 row offsets (local, starting
 *                        at 0), concatenated: graph g's at vtx_off[g] + g;
 *   col_idx  int32[nnz]  local neighbour ids (0 .. n_g-1), symmetric per graph;
 *                        rows sorted ascending unless priority is given;
 *   priority uint32[V] or NULL (precedence within each graph, ties by id);
 *   total_vertices = V = vtx_off[G], total_nnz = edge_off[G] (the caller knows
 *   them; they size the workspace, no device value is read back).
 * workspace: device memory of gcolor_batch_workspace_bytes(G, V, nnz) bytes.
 * ticks (int64[2G], optional): per graph, wall-clock ticks (rate from
 * gcolor_wall_clock_khz) when its workgroup started and finished it.
 * rounds (int32[G], optional): rounds each graph took.
 * Fully asynchronous on `stream`: no host synchronisation, no allocation, so
 * the call may be captured into a HIP graph.  Malformed input is not
 * detected (validate with color_graph_ex per graph when in doubt).
 */
size_t gcolor_batch_workspace_bytes(int32_t num_graphs, int64_t total_vertices, int64_t total_nnz);
int color_graph_batch(int32_t num_graphs, int64_t total_vertices, int64_t total_nnz, const int64_t* vtx_off,
                      const int64_t* edge_off, const int32_t* row_ptr, const int32_t* col_idx,
                      const uint32_t* priority, int32_t* colors_out, void* workspace, size_t ws_bytes,
                      int64_t* ticks, int32_t* rounds, gcolor_stream_t stream);

/* Rate of the device wall clock used by the batch ticks, in kHz. */
int gcolor_wall_clock_khz(int32_t* khz);

/*
 * Learned ordering (a small MLP predicts each vertex's normalised position in
 * the smallest-last order; its scores become priority keys).
 *
 * Model: 8 features -> 64 -> 64 -> 1, ReLU.  Parameters live in one FP32
 * array `master` of GCOLOR_MLP_NPARAM floats laid out as below (W row-major,
 * row = output unit); the forward pass uses BF16 copies `wbf` (uint16 bits,
 * same layout; only the W entries are read) and accumulates in FP32.
 * `norm` holds 16 floats: per-feature mean and standard deviation of
 * log1p(feature) over the training vertices; x = (log1p(f) - mean) / std.
 */
#define GCOLOR_MLP_FEATURES 8
#define GCOLOR_MLP_HIDDEN 64
#define GCOLOR_MLP_W1 0     /* [64][8] */
#define GCOLOR_MLP_B1 512   /* [64] */
#define GCOLOR_MLP_W2 576   /* [64][64] */
#define GCOLOR_MLP_B2 4672  /* [64] */
#define GCOLOR_MLP_W3 4736  /* [64] */
#define GCOLOR_MLP_B3 4800  /* [1] */
#define GCOLOR_MLP_NPARAM 4801

/*
 * Raw features, float[n][8] (device): degree, log2(1 + degree), min / mean /
 * max neighbour degree, two-hop paths (sum of neighbour degree - 1), a
 * triangle estimate from 8 hashed wedges (closed fraction times
 * degree (degree - 1) / 2; wedge choices are splitmix64 of (seed, vertex,
 * sample)), and the h-index of the neighbour degrees (a core-number
 * estimate).  Rows must be sorted ascending.  workspace: device memory of
 * gcolor_features_workspace_bytes(n) bytes owned by the caller (vertices of
 * degree >= 128 are listed there and processed one workgroup each); calls
 * on different streams need workspaces of their own.  Asynchronous on
 * `stream`.  Errors: GCOLOR_EINVAL (n < 0, NULL pointers with n > 0),
 * GCOLOR_EWORKSPACE, GCOLOR_EHIP.
 */
size_t gcolor_features_workspace_bytes(int32_t n);
int gcolor_features(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint64_t seed, float* feat_out,
                    void* workspace, size_t ws_bytes, gcolor_stream_t stream);

/* Adds sum and sum of squares of log1p(feature) per feature (double[16],
 * device, caller zeroes it) over n vertices. */
int gcolor_feature_stats(int64_t n, const float* feat, double* acc, gcolor_stream_t stream);

/* norm (float[16], device) from the sums of gcolor_feature_stats over count
 * vertices: per feature the mean and the population standard deviation of
 * log1p(feature), the variance floored at 1e-12.  Errors: GCOLOR_EINVAL for
 * count <= 0 or NULL pointers. */
int gcolor_feature_norm(int64_t count, const double* acc, float* norm, gcolor_stream_t stream);

/* Training targets (device): target[v] = log(1 + rank[v]) / log(max(n, 2))
 * for smallest-last positions rank[v] in [0, n). */
int gcolor_rank_targets(int32_t n, const int32_t* rank, float* target, gcolor_stream_t stream);

/* score[v] for n vertices (all pointers device). */
int gcolor_mlp_forward(int64_t n, const float* feat, const float* master, const uint16_t* wbf, const float* norm,
                       float* score, gcolor_stream_t stream);

/*
 * Gradient of the mean squared error over a minibatch: vertices idx[0..batch)
 * of feat, targets target[v].  grad (float[NPARAM + 1], device) receives the
 * gradient and, last, the loss; partial is device scratch of
 * gcolor_mlp_partial_floats(batch) floats.
 */
size_t gcolor_mlp_partial_floats(int32_t batch);
int gcolor_mlp_grad(int32_t batch, const int32_t* idx, const float* feat, const float* target, const float* master,
                    const uint16_t* wbf, const float* norm, float* partial, float* grad, gcolor_stream_t stream);

/* Adam step (step >= 1) on master, refreshing wbf; mom/vel are NPARAM floats. */
int gcolor_mlp_adam(float* master, uint16_t* wbf, float* mom, float* vel, const float* grad, float lr, float beta1,
                    float beta2, float eps, int32_t step, gcolor_stream_t stream);

/* wbf = BF16(master), round to nearest even. */
int gcolor_mlp_refresh_bf16(const float* master, uint16_t* wbf, gcolor_stream_t stream);

/* Order-preserving float -> uint32 keys; *bad (device int) is set to 1 when
 * a score is NaN (caller zeroes it). */
int gcolor_scores_to_keys(int64_t n, const float* score, uint32_t* keys, int32_t* bad, gcolor_stream_t stream);

/*
 * Learned priority keys in one call: features (seed as gcolor_features) ->
 * MLP scores -> order-preserving keys, all on `stream`, for color_graph's
 * priority argument (ties between equal keys go to the smaller id).
 *   master, wbf, norm: the model as above (device);
 *   keys_out  uint32[n] (device);
 *   nan_flag  device int32 the caller zeroes; set to 1 when a score is NaN
 *             (the keys are then unusable);
 *   workspace device memory of gcolor_order_learned_workspace_bytes(n) bytes
 *             (features, scores, the features' vertex list).
 * Asynchronous: no host synchronisation, no allocation.  Errors:
 * GCOLOR_EINVAL, GCOLOR_EWORKSPACE, GCOLOR_EHIP.
 */
size_t gcolor_order_learned_workspace_bytes(int32_t n);
int gcolor_order_learned(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint64_t seed,
                         const float* master, const uint16_t* wbf, const float* norm, uint32_t* keys_out,
                         int32_t* nan_flag, void* workspace, size_t ws_bytes, gcolor_stream_t stream);

/* Exact smallest-last order on the host (host pointers): rank[v] = position
 * in the colouring order (the reverse of the removal order; each removal
 * takes a minimum-degree vertex, the smallest id among them). */
int gcolor_smallest_last_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* rank,
                              int32_t* degeneracy);

/* Exact smallest-last order on the device (Matula and Beck 1983; the paper's
 * section "Number of colors" cites it among the orderings that bound the
 * colours of the greedy scheme).  The same order as
 * gcolor_smallest_last_host: each removal takes a vertex of least remaining
 * degree, the smallest id among them; rank[v] (device, int32[n], written) is
 * v's position in the colouring order, n - 1 minus its removal step, so
 * rank works directly as a colour_graph priority.  row_ptr / col_idx: device
 * CSR, symmetric, no duplicate entries (self-loops are ignored); col_idx may
 * be NULL when no row has entries.
 * *degeneracy (host, may be NULL) receives the largest least degree met.
 * One workgroup walks the removals, many per step: the longest run of the
 * smallest ids of the least degree that the one-at-a-time process removes in
 * id order.  Synchronous on `stream`: allocates its own device memory (degree
 * buckets as bitmaps: about n/8 bytes per degree up to a bound of the
 * degeneracy) and returns when the ranks are written.
 * Errors: GCOLOR_EINVAL (n < 0, NULL row_ptr or rank), GCOLOR_ECSR
 * (decreasing row offsets, an entry outside [0, n), or entries with a NULL
 * col_idx), GCOLOR_ENOTSUP (n > 2^28),
 * GCOLOR_EHIP, GCOLOR_EINTERNAL. */
int gcolor_smallest_last(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* rank,
                         int32_t* degeneracy, gcolor_stream_t stream);

/* Human-readable name of a return code. */
const char* gcolor_strerror(int code);

/* Library version string. */
const char* gcolor_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GCOLOR_H */
